/*
 * wandqs oracle -- TEST INFRASTRUCTURE ONLY, NOT THE PRODUCT.
 *
 * A plain, slow FP64 CPU implementation of one quasi-static
 * xi-slice step of plasma electrons driven by a frozen luminal beam, after
 * T. Wang, V. Khudik, J. Kim, G. Shvets, "WAND-PIC: an accelerated
 * three-dimensional quasi-static particle-in-cell code" (arXiv 2012.00881).
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header or constant with the GPU library.
 *
 * Units: time 1/omega_p, length 1/k_p, momenta mc, fields mc omega_p/e,
 * density n0, current -e n0 c (paper Sec. III, opening paragraph).
 *
 * Discretisation (the paper is silent on these; the readings are listed in the
 * design notes of the repository):
 *  - vertex-centred transverse grid x_a = -L + a h, a = 0..N (same in y),
 *    all five fields zero on the boundary nodes;
 *  - cloud-in-cell (bilinear) deposit and gather;
 *  - central differences at interior nodes, one-sided at boundary nodes only
 *    for the gradient of psi used by the particle gather;
 *  - 5-point Laplacian of Sec. VII.B, eq. (33);
 *  - geometric multigrid: V(nu1,nu2) cycles of plain red-black Gauss-Seidel
 *    (the paper names only "iterative relaxation" on a hierarchy of grids),
 *    full weighting, bilinear prolongation, rediscretised coarse operators,
 *    exact solve on the 2x2-cell grid (Sec. II item 4 and Sec. VII.A).
 *
 * Array layout: node (a, b) of an (N+1)x(N+1) array is element b*(N+1)+a
 * (x index fastest).  Field order: psi, Ez, Bz, Bx, By.
 *
 * The forward slice is written once for a scalar type: double is the oracle;
 * a dual number (value plus directional derivatives) gives its tangent-linear
 * model (oracle_run_tangent).  The reverse sweep (oracle_slice_adjoint,
 * oracle_run_loss) is written by hand from the same formulas.
 *
 * Threads (OpenMP): loops whose iterations write disjoint elements run in
 * parallel (colour sweeps, transfers, per-particle gathers and pushes, node
 * formulas); the deposit splits the node rows among the threads, each of which
 * adds the particles in index order; norms are summed serially.  Every result
 * is therefore bitwise the same for any thread count, and equal to the serial
 * program's.
 *
 * Parity status of each function is recorded in the design notes; every
 * function here is pinned by a test in tests/test_oracle_*.py.
 */
#include <limits>
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#include <omp.h>

extern "C" {

typedef struct {
    int kind;             /* 0: Gaussian, 1: piecewise-constant radial bins */
    double amp, sigma_r, sigma_z, xi_c, x0, y0;
    int n_bins;           /* kind 1 only */
    double r_max;         /* kind 1 only: bins of width r_max/n_bins on [0, r_max) */
    const double* bin_amp;/* kind 1 only */
} oracle_beam;

typedef struct {
    int n_cells;          /* N */
    double half_width;    /* L: box [-L, L]^2 */
    int ppc;              /* macroparticles per cell (weight n0 h^2 / ppc) */
    double n0;            /* plasma (and ion background) density */
    double dxi0;          /* initial step of Algorithm 1 */
    int adaptive;         /* Step_Size_Refinement on/off */
    int refine_k;         /* floor dxi >= dxi0/k (0: no floor) */
    double mg_rtol, mg_atol;
    int mg_max_cycles, nu_pre, nu_post;
    int n_beams;
    const oracle_beam* beams;
    int pusher;           /* 0: Boris-like; 1, 2, 4: Runge-Kutta of that order */
    /* longitudinal current of driver macroparticles (oracle_driver_deposit) on
     * drv_nz planes xi = drv_xi0 + m drv_dz, [drv_nz][nn]; NULL: none */
    const double* drv_planes;
    int drv_nz;
    double drv_xi0, drv_dz;
    /* laser envelope A-hat of eq. (20) on las_nz planes xi_m = m dxi0, complex
     * [las_nz][nn] stored as (re, im) pairs; NULL: no laser.  las_k0 is the
     * carrier wavenumber k0 = omega0/omega_p. */
    const double* las_env;
    int las_nz;
    double las_k0;
    /* sub-steps of the driver push per time step (0 or 1: one) */
    int drv_nsub;
} oracle_cfg;

typedef struct {
    double xi, dxi, dxi_next, vmax;
    int cycles[5];
    double rel_resid[5];
    double invariant_err;  /* max |gamma - p_z - (1+psi)| when p_z is carried */
    int status;            /* 0 ok, -4 multigrid did not converge, -5 1+psi <= 0 */
} oracle_info;

enum { ORC_OK = 0, ORC_INVALID = -1, ORC_NOCONV = -4, ORC_NONPHYS = -5 };
enum { PUSH_BORIS = 0, PUSH_RK1 = 1, PUSH_RK2 = 2, PUSH_RK4 = 4 };

} /* extern "C" */

namespace {

/* ------------------------------------------------------------- scalars -- */
/* The forward code below is written once for a scalar type T: double (the
 * oracle) or Dual<K>, a value with K directional derivatives (forward-mode,
 * the tangent-linear model of the same discrete map).  Every value part of a
 * Dual follows exactly the double arithmetic; the discrete decisions (the CIC
 * cell, wall reflections, the multigrid stop) are taken on values. */
template <int K>
struct Dual {
    double v;
    double d[K];
    Dual(double x = 0.0) : v(x) {
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
};
template <int K> Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v + b.v);
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <int K> Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v - b.v);
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <int K> Dual<K> operator-(const Dual<K>& a) {
    Dual<K> r(-a.v);
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
    return r;
}
template <int K> Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v * b.v);
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int K> Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
    Dual<K> r(a.v / b.v);
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
template <int K> Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K> Dual<K> operator*(const Dual<K>& a, double b) { return a * Dual<K>(b); }
template <int K> Dual<K> operator*(double a, const Dual<K>& b) { return Dual<K>(a) * b; }
template <int K> Dual<K> operator/(const Dual<K>& a, double b) { return a / Dual<K>(b); }
template <int K> Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { return a = a + b; }
template <int K> Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { return a = a - b; }
template <int K> Dual<K> sqrt(const Dual<K>& a) {
    Dual<K> r(std::sqrt(a.v));
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
template <int K> Dual<K> exp(const Dual<K>& a) {
    Dual<K> r(std::exp(a.v));
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * r.v;
    return r;
}
using std::exp;
using std::sqrt;

inline double val(double x) { return x; }
template <int K> double val(const Dual<K>& x) { return x.v; }
/* components for the multigrid stop rule: the value and every derivative */
inline int ncomp(double) { return 1; }
template <int K> int ncomp(const Dual<K>&) { return K + 1; }
inline double comp(double x, int) { return x; }
template <int K> double comp(const Dual<K>& x, int c) { return c == 0 ? x.v : x.d[c - 1]; }
/* complex values (the laser envelope): the real and imaginary parts are the
 * two components the multigrid's stop rule checks */
using cplx = std::complex<double>;
inline int ncomp(const cplx&) { return 2; }
inline double comp(const cplx& x, int c) { return c == 0 ? x.real() : x.imag(); }

/* ------------------------------------------------------------------ grid -- */

struct Grid {
    int N;
    double L, h;
    Grid(int n, double l) : N(n), L(l), h(2.0 * l / n) {}
    int nn() const { return (N + 1) * (N + 1); }
    int id(int a, int b) const { return b * (N + 1) + a; }
    double xa(int a) const { return -L + a * h; }
};

/* Cloud-in-cell shape: cell index c in [0, N-1] and offset d in [0, 1] so that
 * the particle weights node c by (1 - d) and node c+1 by d. */
template <class T>
void cic(const Grid& g, const T& x, int& c, T& d) {
    T t = (x + g.L) / g.h;
    int k = (int)std::floor(val(t));
    if (k < 0) k = 0;
    if (k > g.N - 1) k = g.N - 1;
    c = k;
    d = t - (double)k;
}

/* deposit(q)[a,b] = sum_i w q_i W_a(x_i) W_b(y_i) / h^2 with w = n0 h^2 / ppc.
 * With q = 1 this is the surface density n* of Sec. III.B (n* = int f* dP).
 * Each thread owns a band of node rows b and adds, in particle order, the
 * contributions of the particles whose cell touches its rows, so every node
 * sums its particles in index order whatever the number of threads. */
template <class T>
void deposit(const Grid& g, const oracle_cfg& c, int P, const T* x, const T* y, const T* q,
             T* out) {
    const double w = c.n0 * g.h * g.h / c.ppc;
    std::fill(out, out + g.nn(), T(0.0));
#pragma omp parallel
    {
        const int nt = omp_get_num_threads(), t = omp_get_thread_num();
        const int rows = g.N + 1;
        const int r0 = (int)((long)rows * t / nt), r1 = (int)((long)rows * (t + 1) / nt);
        for (int i = 0; i < P; ++i) {
            int a, b;
            T dx, dy;
            cic(g, y[i], b, dy);
            if (b + 1 < r0 || b >= r1) continue;
            cic(g, x[i], a, dx);
            T s = w * (q ? q[i] : T(1.0)) / (g.h * g.h);
            if (b >= r0) {
                out[g.id(a, b)] += s * (1.0 - dx) * (1.0 - dy);
                out[g.id(a + 1, b)] += s * dx * (1.0 - dy);
            }
            if (b + 1 < r1) {
                out[g.id(a, b + 1)] += s * (1.0 - dx) * dy;
                out[g.id(a + 1, b + 1)] += s * dx * dy;
            }
        }
    }
}

/* gather(F)_i = sum over the four cell corners of F W_a W_b. */
template <class T>
T gather1(const Grid& g, const T* F, const T& x, const T& y) {
    int a, b;
    T dx, dy;
    cic(g, x, a, dx);
    cic(g, y, b, dy);
    return F[g.id(a, b)] * (1.0 - dx) * (1.0 - dy) + F[g.id(a + 1, b)] * dx * (1.0 - dy) +
           F[g.id(a, b + 1)] * (1.0 - dx) * dy + F[g.id(a + 1, b + 1)] * dx * dy;
}

/* Central differences D_x u, D_y u at interior nodes. */
template <class T>
T Dx(const Grid& g, const T* u, int a, int b) {
    return (u[g.id(a + 1, b)] - u[g.id(a - 1, b)]) / (2.0 * g.h);
}
template <class T>
T Dy(const Grid& g, const T* u, int a, int b) {
    return (u[g.id(a, b + 1)] - u[g.id(a, b - 1)]) / (2.0 * g.h);
}

/* ------------------------------------------------------------- multigrid -- */

/* One level of the hierarchy for  L_h u - k2 u = f  on the interior nodes,
 * u = 0 on the boundary.  k2 == empty means the Poisson operator. */
template <class T>
struct Level {
    int N;
    double h;
    std::vector<T> u, f, k2;
    int id(int a, int b) const { return b * (N + 1) + a; }
};

/* (L_h u - k2 u) at interior node (a, b); 5-point Laplacian, Sec. VII.B eq. (33). */
template <class T>
T apply_at(const Level<T>& lv, const T* u, int a, int b) {
    T lap = (u[lv.id(a - 1, b)] + u[lv.id(a + 1, b)] + u[lv.id(a, b - 1)] +
             u[lv.id(a, b + 1)] - 4.0 * u[lv.id(a, b)]) / (lv.h * lv.h);
    T k2 = lv.k2.empty() ? T(0.0) : lv.k2[lv.id(a, b)];
    return lap - k2 * u[lv.id(a, b)];
}

/* Red-black Gauss-Seidel half sweep: each node with (a+b) % 2 == color takes
 * the value that zeroes its own equation given its four neighbours,
 * u = (sum of the neighbours - h^2 f) / (4 + h^2 k2).  The nodes of one colour
 * depend only on the other colour, so the rows can be swept in any order. */
template <class T>
void relax_color(Level<T>& lv, int color) {
    const double h2 = lv.h * lv.h;
#pragma omp parallel for schedule(static)
    for (int b = 1; b < lv.N; ++b)
        for (int a = 1; a < lv.N; ++a) {
            if (((a + b) & 1) != color) continue;
            T nb = lv.u[lv.id(a - 1, b)] + lv.u[lv.id(a + 1, b)] + lv.u[lv.id(a, b - 1)] +
                   lv.u[lv.id(a, b + 1)];
            T k2 = lv.k2.empty() ? T(0.0) : lv.k2[lv.id(a, b)];
            lv.u[lv.id(a, b)] = (nb - h2 * lv.f[lv.id(a, b)]) / (4.0 + h2 * k2);
        }
}

template <class T>
void smooth(Level<T>& lv, int nu) {
    for (int s = 0; s < nu; ++s) {
        relax_color(lv, 0);
        relax_color(lv, 1);
    }
}

/* Residual r = f - A u at the interior nodes (zero on the boundary). */
template <class T>
void residual(const Level<T>& lv, std::vector<T>& r) {
    r.assign((lv.N + 1) * (lv.N + 1), T(0.0));
#pragma omp parallel for schedule(static)
    for (int b = 1; b < lv.N; ++b)
        for (int a = 1; a < lv.N; ++a)
            r[lv.id(a, b)] = lv.f[lv.id(a, b)] - apply_at(lv, lv.u.data(), a, b);
}

/* 2-norm over the interior nodes of component c (0: the value). */
template <class T>
double norm2_interior(const Level<T>& lv, const std::vector<T>& v, int c = 0) {
    double s = 0.0;
    for (int b = 1; b < lv.N; ++b)
        for (int a = 1; a < lv.N; ++a) s += comp(v[lv.id(a, b)], c) * comp(v[lv.id(a, b)], c);
    return std::sqrt(s);
}

/* Full weighting of a fine-grid node array onto the interior coarse nodes. */
template <class T>
void full_weighting(const Level<T>& fine, const std::vector<T>& r, Level<T>& coarse,
                    std::vector<T>& out) {
    out.assign((coarse.N + 1) * (coarse.N + 1), T(0.0));
#pragma omp parallel for schedule(static)
    for (int J = 1; J < coarse.N; ++J)
        for (int I = 1; I < coarse.N; ++I) {
            int a = 2 * I, b = 2 * J;
            T s = 4.0 * r[fine.id(a, b)] +
                  2.0 * (r[fine.id(a - 1, b)] + r[fine.id(a + 1, b)] + r[fine.id(a, b - 1)] +
                         r[fine.id(a, b + 1)]) +
                  (r[fine.id(a - 1, b - 1)] + r[fine.id(a + 1, b - 1)] +
                   r[fine.id(a - 1, b + 1)] + r[fine.id(a + 1, b + 1)]);
            out[coarse.id(I, J)] = s / 16.0;
        }
}

/* u_fine += bilinear interpolation of u_coarse. */
template <class T>
void prolong_add(const Level<T>& coarse, Level<T>& fine) {
#pragma omp parallel for schedule(static)
    for (int b = 1; b < fine.N; ++b)
        for (int a = 1; a < fine.N; ++a) {
            int I = a / 2, J = b / 2;
            bool ox = a & 1, oy = b & 1;
            const std::vector<T>& e = coarse.u;
            T v;
            if (!ox && !oy) v = e[coarse.id(I, J)];
            else if (ox && !oy) v = 0.5 * (e[coarse.id(I, J)] + e[coarse.id(I + 1, J)]);
            else if (!ox && oy) v = 0.5 * (e[coarse.id(I, J)] + e[coarse.id(I, J + 1)]);
            else
                v = 0.25 * (e[coarse.id(I, J)] + e[coarse.id(I + 1, J)] + e[coarse.id(I, J + 1)] +
                            e[coarse.id(I + 1, J + 1)]);
            fine.u[fine.id(a, b)] += v;
        }
}

template <class T>
void vcycle(std::vector<Level<T>>& lv, size_t l, int nu1, int nu2) {
    Level<T>& L = lv[l];
    if (L.N == 2) { /* one interior node, four zero boundary neighbours: exact */
        T k2 = L.k2.empty() ? T(0.0) : L.k2[L.id(1, 1)];
        L.u[L.id(1, 1)] = -L.f[L.id(1, 1)] / (4.0 / (L.h * L.h) + k2);
        return;
    }
    smooth(L, nu1);
    std::vector<T> r;
    residual(L, r);
    Level<T>& C = lv[l + 1];
    full_weighting(L, r, C, C.f);
    std::fill(C.u.begin(), C.u.end(), T(0.0));
    vcycle(lv, l + 1, nu1, nu2);
    prolong_add(C, L);
    smooth(L, nu2);
}

/* Solve (L_h - k2) u = f for the interior nodes with u = 0 on the boundary,
 * starting from the guess held in u.  Stops when ||r|| <= rtol ||f|| + atol sqrt(n)
 * (n interior nodes; ||r_0|| in place of ||f|| when f = 0), or at the rounding
 * floor: ||r|| <= 0.35 eps (8/h^2 ||u|| + ||f||), the size of the rounding
 * error in forming r (a backward-error test; 8/h^2 bounds ||L_h||), or a cycle
 * after the second that reduces ||r|| by less than 2x while
 * ||r|| <= 1e-9 max(||f||, ||r_0||) (the guard keeps a slowly converging solve
 * from being taken for a converged one).  Otherwise returns ORC_NOCONV after
 * max_cycles.  For a Dual scalar every component (value and each derivative)
 * must meet the rule: the derivative solves converge along with the value. */
template <class T>
int mg_solve(int N, double h, const T* k2, const T* f, T* u, double rtol, double atol,
             int max_cycles, int nu1, int nu2, int* cycles_out, double* rel_out) {
    std::vector<Level<T>> lv;
    for (int n = N; n >= 2; n /= 2) {
        Level<T> l;
        l.N = n;
        l.h = h * (N / n);
        l.u.assign((n + 1) * (n + 1), T(0.0));
        l.f.assign((n + 1) * (n + 1), T(0.0));
        lv.push_back(l);
    }
    Level<T>& top = lv[0];
    std::copy(f, f + top.u.size(), top.f.begin());
    std::copy(u, u + top.u.size(), top.u.begin());
    for (int b = 0; b <= N; ++b)  /* Dirichlet: boundary values are zero */
        for (int a = 0; a <= N; ++a)
            if (a == 0 || b == 0 || a == N || b == N) {
                top.u[top.id(a, b)] = T(0.0);
                top.f[top.id(a, b)] = T(0.0);
            }
    if (k2) {  /* coarse k2 by full weighting of the finer level */
        top.k2.assign(k2, k2 + top.u.size());
        for (size_t l = 1; l < lv.size(); ++l) full_weighting(lv[l - 1], lv[l - 1].k2, lv[l], lv[l].k2);
    }
    const int nc = ncomp(T(0.0));
    std::vector<T> r;
    residual(top, r);
    std::vector<double> fnorm(nc), rn(nc), rprev(nc), tol(nc), scale(nc), un(nc);
    const double floor_be = 0.35 * std::numeric_limits<double>::epsilon();
    const double a_norm = 8.0 / (h * h);
    for (int c = 0; c < nc; ++c) {
        fnorm[c] = norm2_interior(top, top.f, c);
        rn[c] = rprev[c] = norm2_interior(top, r, c);
        /* relative to ||f||; for f = 0 (solution 0) relative to the initial residual */
        tol[c] = rtol * (fnorm[c] > 0 ? fnorm[c] : rn[c]) + atol * std::sqrt((double)(N - 1) * (N - 1));
        scale[c] = std::max(fnorm[c], rn[c]);
    }
    std::vector<bool> done(nc);
    for (int c = 0; c < nc; ++c) done[c] = rn[c] <= tol[c];
    auto all_done = [&]() {
        for (int c = 0; c < nc; ++c)
            if (!done[c]) return false;
        return true;
    };
    int cyc = 0;
    while (!all_done() && cyc < max_cycles) {
        vcycle(lv, 0, nu1, nu2);
        ++cyc;
        residual(top, r);
        for (int c = 0; c < nc; ++c) {
            rprev[c] = rn[c];
            rn[c] = norm2_interior(top, r, c);
            un[c] = norm2_interior(top, top.u, c);
            if (rn[c] <= tol[c] || rn[c] <= floor_be * (a_norm * un[c] + fnorm[c])) done[c] = true;
            else if (cyc >= 2 && rn[c] > 0.5 * rprev[c] && rn[c] <= 1e-9 * scale[c])
                done[c] = true; /* floor */
            else done[c] = false;
        }
    }
    std::copy(top.u.begin(), top.u.end(), u);
    if (cycles_out) *cycles_out = cyc;
    if (rel_out) *rel_out = fnorm[0] > 0 ? rn[0] / fnorm[0] : rn[0];
    bool finite = true;
    for (int c = 0; c < nc; ++c) finite = finite && std::isfinite(rn[c]);
    return (finite && all_done()) ? ORC_OK : ORC_NOCONV;
}

/* --------------------------------------------------------------- drivers -- */

/* Frozen luminal driver density n_b(x, y, xi); zero for xi < 0 (the xi axis
 * starts at 0, Table 1 footnote).  Gaussian: amp exp(-r^2/sr^2 - (xi-xc)^2/sz^2)
 * as in Sec. V.A; radial bins: bin_amp[floor(r/dr)] exp(-(xi-xc)^2/sz^2).
 * theta (or NULL: the configuration's values) lists the amplitudes beam by
 * beam: amp (Gaussian) or the bin amplitudes (radial bins). */
template <class T>
T beam_density(const oracle_cfg& c, const T* theta, double x, double y, double xi) {
    if (xi < 0.0) return T(0.0);
    T s(0.0);
    int t = 0;
    for (int k = 0; k < c.n_beams; ++k) {
        const oracle_beam& B = c.beams[k];
        double rx = x - B.x0, ry = y - B.y0;
        double r2 = rx * rx + ry * ry;
        double lz = (xi - B.xi_c) * (xi - B.xi_c) / (B.sigma_z * B.sigma_z);
        if (B.kind == 0) {
            const T amp = theta ? theta[t] : T(B.amp);
            s += amp * std::exp(-r2 / (B.sigma_r * B.sigma_r) - lz);
            t += 1;
        } else {
            double r = std::sqrt(r2);
            double dr = B.r_max / B.n_bins;
            int k2 = (int)std::floor(r / dr);
            if (r < B.r_max && k2 < B.n_bins) s += (theta ? theta[t + k2] : T(B.bin_amp[k2])) * std::exp(-lz);
            t += B.n_bins;
        }
    }
    return s;
}
double beam_density(const oracle_cfg& c, double x, double y, double xi) {
    return beam_density<double>(c, nullptr, x, y, xi);
}

/* Driver macroparticles' longitudinal current at node i and slice position
 * xi: linear interpolation between the two deposit planes around xi, zero
 * outside the planes. */
double driver_current(const oracle_cfg& c, int i, int nn, double xi) {
    if (!c.drv_planes || c.drv_nz < 2) return 0.0;
    const double t = (xi - c.drv_xi0) / c.drv_dz;
    const int m = (int)std::floor(t);
    if (m < 0 || m > c.drv_nz - 2) return 0.0;
    const double a = t - m;
    return (1.0 - a) * c.drv_planes[(size_t)m * nn + i] + a * c.drv_planes[(size_t)(m + 1) * nn + i];
}

/* |A-hat|^2 of the laser envelope on the nodes at slice position xi: the
 * planes xi_m = m dxi0 around xi interpolated linearly in xi, planes outside
 * [0, las_nz) taken as zero.  Empty without a laser. */
std::vector<double> laser_a2(const Grid& g, const oracle_cfg& c, double xi) {
    if (!c.las_env || c.las_nz < 1) return {};
    const int nn = g.nn();
    std::vector<double> out(nn, 0.0);
    const double t = xi / c.dxi0;
    const double mf = std::floor(t);
    const double a = t - mf;
    const double w[2] = {1.0 - a, a};
    for (int k = 0; k < 2; ++k) {
        const double q = mf + k;
        if (q < 0.0 || q >= c.las_nz) continue;
        const double* e = c.las_env + 2 * (size_t)q * nn;
        for (int i = 0; i < nn; ++i) out[i] += w[k] * (e[2 * i] * e[2 * i] + e[2 * i + 1] * e[2 * i + 1]);
    }
    return out;
}

/* ------------------------------------------------------ laser envelope -- */

/* One time step dt of the envelope equation (eq. (20)) at one xi-plane.
 * With a0 = A-hat(t, xi_j), a1 = A-hat(t + dt, xi_j) and p0, p1 the same on
 * the plane ahead, xi_{j-1} = xi_j - dxi (zero ahead of the first plane),
 * eq. (20) is taken centred in t,
 *   2 i k0 (a1 - a0)/dt - 2 [(a1 - a0) - (p1 - p0)]/(dt dxi)
 *       + L_h (a1 + a0)/2 = chi (a1 + a0)/2,
 * the xi-derivative backward (the plane ahead is already at t + dt when the
 * sweep reaches plane j).  For a1 it is the complex Helmholtz problem
 *   L_h a1 - (chi + beta - i gam) a1 = (chi - beta + i gam) a0 - L_h a0 - beta (p1 - p0),
 * beta = 4/(dt dxi), gam = 4 k0/dt, with a1 = 0 on the boundary, solved by the
 * multigrid above from the guess a0.  chi (the plasma susceptibility n* / (1+psi)
 * at the nodes) may be NULL (vacuum). */
int laser_plane_advance(const Grid& g, const oracle_cfg& c, double dt, const double* chi,
                        const cplx* a0, const cplx* p0, const cplx* p1, cplx* a1, int* cycles,
                        double* rel) {
    const int nn = g.nn();
    const double beta = 4.0 / (dt * c.dxi0), gam = 4.0 * c.las_k0 / dt;
    const cplx ig(0.0, gam);
    std::vector<cplx> k2(nn, cplx(0.0)), f(nn, cplx(0.0));
    const double h2 = g.h * g.h;
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a) {
            const int i = g.id(a, b);
            const double x = chi ? chi[i] : 0.0;
            k2[i] = x + beta - ig;
            if (a == 0 || b == 0 || a == g.N || b == g.N) continue;
            const cplx lap = (a0[g.id(a - 1, b)] + a0[g.id(a + 1, b)] + a0[g.id(a, b - 1)] +
                              a0[g.id(a, b + 1)] - 4.0 * a0[i]) / h2;
            const cplx dp = (p1 ? p1[i] : cplx(0.0)) - (p0 ? p0[i] : cplx(0.0));
            f[i] = (x - beta + ig) * a0[i] - lap - beta * dp;
        }
    std::copy(a0, a0 + nn, a1);
    return mg_solve<cplx>(g.N, g.h, k2.data(), f.data(), a1, c.mg_rtol, c.mg_atol, c.mg_max_cycles,
                          c.nu_pre, c.nu_post, cycles, rel);
}

/* ----------------------------------------------------------- slice step -- */

template <class T>
struct MomentsT { /* node arrays deposited from the particles of one slice */
    std::vector<T> n, jx, jy, txx, txy, tyy;
};
using Moments = MomentsT<double>;

/* Assembly of the B-perp system (Sec. III.B eqs. (18)-(19), i.e. rows 4-5 of
 * eq. (30)):  G = n*<gamma> (eq. (9) and the gamma of Sec. III.A, with
 * a2 = |A-hat|^2 of a laser envelope, zero without one), plasma
 * j_z = n*<p_z>/(1+psi) = G/g - n*, total j_z adds the beam and the driver
 * particles, k2 = n* / g, and the right-hand sides
 *   f_Bx =  S_y,  f_By = -S_x   (from -e_z x S),
 *   S = grad j_z - div T + (e_z x j) Bz/g + (G grad psi - n* grad(a2/4))/g^2
 *       - j Ez/g - T.grad psi/g.
 * Returns ORC_NONPHYS if g <= 0 at a node that holds plasma. */
template <class T>
int assemble(const Grid& g, const oracle_cfg& c, double xi, const MomentsT<T>& m,
             const T* psi, const T* Ez, const T* Bz, std::vector<T>& k2,
             std::vector<T>& fBx, std::vector<T>& fBy, std::vector<T>* jz_out,
             const T* theta = nullptr) {
    const int nn = g.nn();
    std::vector<T> G(nn, T(0.0)), jz(nn, T(0.0));
    const std::vector<double> A2 = laser_a2(g, c, xi);
    const bool las = !A2.empty();
    int nonphys = 0;
#pragma omp parallel for schedule(static) reduction(| : nonphys)
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a) {
            int i = g.id(a, b);
            T gg = 1.0 + psi[i];
            T plasma_jz(0.0);
            if (val(m.n[i]) > 0.0) {
                if (val(gg) <= 0.0) nonphys = 1;
                /* <gamma> = (1 + <p_perp^2> + g^2 + a2/2)/(2g) with <p_perp^2> = g^2 <V^2> */
                const double a2 = las ? A2[i] : 0.0;
                G[i] = (m.n[i] * (1.0 + gg * gg + 0.5 * a2) + gg * gg * (m.txx[i] + m.tyy[i])) /
                       (2.0 * gg);
                plasma_jz = G[i] / gg - m.n[i];
            }
            jz[i] = plasma_jz + beam_density(c, theta, g.xa(a), g.xa(b), xi) +
                    driver_current(c, i, nn, xi);
        }
    const int status = nonphys ? ORC_NONPHYS : ORC_OK;
    k2.assign(nn, T(0.0));
    fBx.assign(nn, T(0.0));
    fBy.assign(nn, T(0.0));
#pragma omp parallel for schedule(static)
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) {
            int i = g.id(a, b);
            T gg = 1.0 + psi[i];
            T px = Dx(g, psi, a, b), py = Dy(g, psi, a, b);
            /* grad j_z - div T, written as the D-terms of rows 4-5 of eq. (30) */
            T d_jz_tyy = (jz[g.id(a, b + 1)] - m.tyy[g.id(a, b + 1)] -
                          (jz[g.id(a, b - 1)] - m.tyy[g.id(a, b - 1)])) / (2.0 * g.h);
            T d_txx_jz = (m.txx[g.id(a + 1, b)] - jz[g.id(a + 1, b)] -
                          (m.txx[g.id(a - 1, b)] - jz[g.id(a - 1, b)])) / (2.0 * g.h);
            T fx = d_jz_tyy - Dx(g, m.txy.data(), a, b);
            T fy = d_txx_jz + Dy(g, m.txy.data(), a, b);
            if (val(m.n[i]) > 0.0) {
                k2[i] = m.n[i] / gg;
                fx += (m.jx[i] * Bz[i] - m.jy[i] * Ez[i]) / gg +
                      (G[i] / (gg * gg) - m.tyy[i] / gg) * py - (m.txy[i] / gg) * px;
                fy += (m.jy[i] * Bz[i] + m.jx[i] * Ez[i]) / gg -
                      (G[i] / (gg * gg) - m.txx[i] / gg) * px + (m.txy[i] / gg) * py;
                if (las) { /* the ponderomotive term -n* grad(a2/4)/g^2 of S */
                    fx -= m.n[i] * (0.25 * Dy(g, A2.data(), a, b)) / (gg * gg);
                    fy += m.n[i] * (0.25 * Dx(g, A2.data(), a, b)) / (gg * gg);
                }
            }
            fBx[i] = fx;
            fBy[i] = fy;
        }
    if (jz_out) *jz_out = jz;
    return status;
}

/* Node gradient of psi for the particle gather: central at interior nodes,
 * one-sided on the boundary rows/columns. */
template <class T>
void psi_gradient(const Grid& g, const T* psi, std::vector<T>& gx, std::vector<T>& gy) {
    gx.assign(g.nn(), T(0.0));
    gy.assign(g.nn(), T(0.0));
#pragma omp parallel for schedule(static)
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a) {
            int i = g.id(a, b);
            if (a == 0) gx[i] = (psi[g.id(1, b)] - psi[g.id(0, b)]) / g.h;
            else if (a == g.N) gx[i] = (psi[g.id(g.N, b)] - psi[g.id(g.N - 1, b)]) / g.h;
            else gx[i] = (psi[g.id(a + 1, b)] - psi[g.id(a - 1, b)]) / (2.0 * g.h);
            if (b == 0) gy[i] = (psi[g.id(a, 1)] - psi[g.id(a, 0)]) / g.h;
            else if (b == g.N) gy[i] = (psi[g.id(a, g.N)] - psi[g.id(a, g.N - 1)]) / g.h;
            else gy[i] = (psi[g.id(a, b + 1)] - psi[g.id(a, b - 1)]) / (2.0 * g.h);
        }
}

/* Boris-like advance of one plasma electron over dxi with the fields frozen at
 * the current slice (Sec. III.A eqs. (6)-(7)):
 *   dr/dxi = V = p/g,
 *   dp/dxi = (gamma grad psi - grad(a2/4))/g + (e_z x V) Bz + e_z x B_perp,
 *   gamma = (1 + p^2 + g^2 + a2/2)/(2g)  taken at the old momentum,
 * a2 = |A-hat|^2 of a laser envelope and (ax, ay) its gradient, gathered at the
 * particle (zero without a laser).
 * Half kick with F = (gamma grad psi - grad(a2/4))/g + e_z x B_perp, rotation
 * by the (e_z x V) Bz term (angle 2 atan(Bz dxi / 2g)), half kick, drift with
 * the new momentum, specular reflection at the walls x, y = +-L. */
template <class T>
void push_one(double L, double dxi, const T& g_i, const T& gx, const T& gy, const T& Bx,
              const T& By, const T& Bz, T& x, T& y, T& px, T& py, double a2 = 0.0,
              double ax = 0.0, double ay = 0.0) {
    T gamma = (1.0 + px * px + py * py + g_i * g_i + 0.5 * a2) / (2.0 * g_i);
    T Fx = (gamma * gx - 0.25 * ax) / g_i - By;
    T Fy = (gamma * gy - 0.25 * ay) / g_i + Bx;
    T mx = px + 0.5 * dxi * Fx;
    T my = py + 0.5 * dxi * Fy;
    T t = Bz * dxi / (2.0 * g_i);
    T s = 2.0 * t / (1.0 + t * t);
    T qx = mx - t * my;
    T qy = my + t * mx;
    T rx = mx - s * qy;
    T ry = my + s * qx;
    px = rx + 0.5 * dxi * Fx;
    py = ry + 0.5 * dxi * Fy;
    x = x + dxi * px / g_i;
    y = y + dxi * py / g_i;
    if (val(x) > L) { x = 2.0 * L - x; px = -px; }
    if (val(x) < -L) { x = -2.0 * L - x; px = -px; }
    if (val(y) > L) { y = 2.0 * L - y; py = -py; }
    if (val(y) < -L) { y = -2.0 * L - y; py = -py; }
}

/* A laser envelope's |A-hat|^2 on the nodes of a slice and its node gradient
 * (the same differences as psi's); all empty without a laser. */
struct LaserNodes {
    std::vector<double> a2, ax, ay;
    bool on() const { return !a2.empty(); }
};

/* Right-hand side of the plasma electron's equations of motion in xi with the
 * fields frozen at the slice (Sec. III.A eqs. (6)-(7)), at the position and
 * momentum s = (x, y, p_x, p_y):
 *   dr/dxi = V = p/g,
 *   dp/dxi = (gamma grad psi - grad(a2/4))/g + (e_z x V) B_z + e_z x B_perp,
 *   g = 1 + psi and gamma = (1 + p^2 + g^2 + a2/2)/(2g),
 * every field gathered (CIC) at the position itself.  Returns false when
 * g <= 0 there. */
template <class T>
bool eom_rhs(const Grid& g, const T* psi, const T* gx, const T* gy, const T* Bx, const T* By,
             const T* Bz, const LaserNodes& las, const T (&s)[4], T (&d)[4]) {
    const T gg = 1.0 + gather1(g, psi, s[0], s[1]);
    if (!(val(gg) > 0.0)) return false;
    const T Gx = gather1(g, gx, s[0], s[1]), Gy = gather1(g, gy, s[0], s[1]);
    const T bx = gather1(g, Bx, s[0], s[1]), by = gather1(g, By, s[0], s[1]);
    const T bz = gather1(g, Bz, s[0], s[1]);
    T a2(0.0), ax(0.0), ay(0.0);
    if (las.on()) {
        a2 = gather1(g, las.a2.data(), val(s[0]), val(s[1]));
        ax = gather1(g, las.ax.data(), val(s[0]), val(s[1]));
        ay = gather1(g, las.ay.data(), val(s[0]), val(s[1]));
    }
    const T gamma = (1.0 + s[2] * s[2] + s[3] * s[3] + gg * gg + 0.5 * a2) / (2.0 * gg);
    const T vx = s[2] / gg, vy = s[3] / gg;
    d[0] = vx;
    d[1] = vy;
    d[2] = (gamma * Gx - 0.25 * ax) / gg - vy * bz - by;
    d[3] = (gamma * Gy - 0.25 * ay) / gg + vx * bz + bx;
    return true;
}

/* Runge-Kutta advance over dxi of the same equations (the alternative pushers
 * the paper lists beside the Boris-like one, Sec. VII.A): order 1 (forward
 * Euler), 2 (the midpoint rule) or 4 (the classical four-stage scheme).
 * Every stage gathers the frozen fields at its own position (a stage position
 * outside the box uses its edge cell's bilinear form); the walls reflect the
 * end position as in push_one.  Returns false when a stage meets g <= 0. */
template <class T>
bool push_rk(const Grid& g, int order, double dxi, const T* psi, const T* gx, const T* gy,
             const T* Bx, const T* By, const T* Bz, const LaserNodes& las, T& x, T& y, T& px,
             T& py) {
    const T s0[4] = {x, y, px, py};
    T k1[4], k2[4], k3[4], k4[4], s[4];
    bool ok = eom_rhs(g, psi, gx, gy, Bx, By, Bz, las, s0, k1);
    T out[4];
    if (order == PUSH_RK1) {
        for (int q = 0; q < 4; ++q) out[q] = s0[q] + dxi * k1[q];
    } else if (order == PUSH_RK2) {
        for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k1[q];
        ok = eom_rhs(g, psi, gx, gy, Bx, By, Bz, las, s, k2) && ok;
        for (int q = 0; q < 4; ++q) out[q] = s0[q] + dxi * k2[q];
    } else {
        for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k1[q];
        ok = eom_rhs(g, psi, gx, gy, Bx, By, Bz, las, s, k2) && ok;
        for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k2[q];
        ok = eom_rhs(g, psi, gx, gy, Bx, By, Bz, las, s, k3) && ok;
        for (int q = 0; q < 4; ++q) s[q] = s0[q] + dxi * k3[q];
        ok = eom_rhs(g, psi, gx, gy, Bx, By, Bz, las, s, k4) && ok;
        for (int q = 0; q < 4; ++q)
            out[q] = s0[q] + (dxi / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    }
    x = out[0];
    y = out[1];
    px = out[2];
    py = out[3];
    const double L = g.L;
    if (val(x) > L) { x = 2.0 * L - x; px = -px; }
    if (val(x) < -L) { x = -2.0 * L - x; px = -px; }
    if (val(y) > L) { y = 2.0 * L - y; py = -py; }
    if (val(y) < -L) { y = -2.0 * L - y; py = -py; }
    return ok;
}

/* Step_Size_Refinement (Algorithm 1): the step is the largest that keeps the
 * fastest particle within one cell, h / Vmax, but never above the initial
 * step dxi0 (the paper's V0 = h / dxi0 marks where the refinement starts) and,
 * with refinement level k, never below dxi0 / k (Sec. V.A). */
double next_dxi(const oracle_cfg& c, double h, double vmax) {
    double d = c.dxi0;
    if (c.adaptive && vmax > 0.0) {
        d = std::min(c.dxi0, h / vmax);
        if (c.refine_k > 0) d = std::max(d, c.dxi0 / c.refine_k);
    }
    return d;
}


/* One xi-slice (Algorithm 1 inner loop: Collect_Source, Solve_Wakefield,
 * Push_Trajectory, Step_Size_Refinement).
 *   in:  particles (x, y, px, py) at xi, fields[5][nn] = previous slice's fields
 *        (multigrid initial guesses), *xi, *dxi (the step to take now);
 *   out: fields at xi, particles at xi + dxi, *xi += dxi, *dxi = next step.
 * moments_out ([6][nn], may be NULL) receives n*, jx, jy, Txx, Txy, Tyy and
 * extra_out ([4][nn], may be NULL) receives k2, f_Bx, f_By, j_z.
 * pz (may be NULL) carries p_z for the dynamic check of gamma - p_z = 1 + psi. */
template <class T>
int slice_step_t(const oracle_cfg* c, int P, T* x, T* y, T* px, T* py, T* pz, T* fields,
                 double* xi, double* dxi, oracle_info* info, T* moments_out, T* extra_out,
                 const T* theta) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    T* psi = fields;
    T* Ez = fields + nn;
    T* Bz = fields + 2 * nn;
    T* Bx = fields + 3 * nn;
    T* By = fields + 4 * nn;
    oracle_info inf;
    std::memset(&inf, 0, sizeof(inf));
    inf.xi = *xi;
    inf.dxi = *dxi;
    int status = ORC_OK;
    auto solve = [&](int k, const std::vector<T>* k2, const std::vector<T>& f, T* u) {
        int st = mg_solve<T>(g.N, g.h, k2 ? k2->data() : nullptr, f.data(), u, c->mg_rtol, c->mg_atol,
                          c->mg_max_cycles, c->nu_pre, c->nu_post, &inf.cycles[k], &inf.rel_resid[k]);
        if (st != ORC_OK && status == ORC_OK) status = st;
    };

    /* 1. surface density n* (Collect_Source). */
    MomentsT<T> m;
    m.n.assign(nn, T(0.0));
    deposit<T>(g, *c, P, x, y, nullptr, m.n.data());

    /* 2. psi: L_h psi = n* - n0 (Sec. III.B eq. (12)). */
    std::vector<T> f(nn, T(0.0));
    for (int i = 0; i < nn; ++i) f[i] = m.n[i] - c->n0;
    solve(0, nullptr, f, psi);

    /* 3. per-particle g_i = 1 + psi(r_i) and V_i = p_i/g_i (eq. (6)); currents
     *    j = n*<V> (eq. (9)) and pressure tensor T = n*<V V> (below eq. (16)). */
    std::vector<T> gi(P), vx(P), vy(P), vxx(P), vxy(P), vyy(P);
    double inv_err = 0.0;
    int nonphys = 0;
#pragma omp parallel for schedule(static) reduction(max : inv_err) reduction(| : nonphys)
    for (int i = 0; i < P; ++i) {
        gi[i] = 1.0 + gather1(g, psi, x[i], y[i]);
        if (!(val(gi[i]) > 0.0)) nonphys = 1;
        vx[i] = px[i] / gi[i];
        vy[i] = py[i] / gi[i];
        vxx[i] = vx[i] * vx[i];
        vxy[i] = vx[i] * vy[i];
        vyy[i] = vy[i] * vy[i];
        if (pz) {
            T gam = (1.0 + px[i] * px[i] + py[i] * py[i] + gi[i] * gi[i]) / (2.0 * gi[i]);
            inv_err = std::max(inv_err, std::fabs(val(gam - pz[i] - gi[i])));
        }
    }
    if (nonphys) status = ORC_NONPHYS;
    inf.invariant_err = inv_err;
    m.jx.assign(nn, T(0.0));
    m.jy.assign(nn, T(0.0));
    m.txx.assign(nn, T(0.0));
    m.txy.assign(nn, T(0.0));
    m.tyy.assign(nn, T(0.0));
    deposit<T>(g, *c, P, x, y, vx.data(), m.jx.data());
    deposit<T>(g, *c, P, x, y, vy.data(), m.jy.data());
    deposit<T>(g, *c, P, x, y, vxx.data(), m.txx.data());
    deposit<T>(g, *c, P, x, y, vxy.data(), m.txy.data());
    deposit<T>(g, *c, P, x, y, vyy.data(), m.tyy.data());

    /* 4. Ez and Bz: L_h Ez = -div j (eq. (13)), L_h Bz = e_z.(curl j) (eq. (14)). */
    std::vector<T> fE(nn, T(0.0)), fB(nn, T(0.0));
#pragma omp parallel for schedule(static)
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) {
            int i = g.id(a, b);
            fE[i] = -(Dx(g, m.jx.data(), a, b) + Dy(g, m.jy.data(), a, b));
            fB[i] = Dx(g, m.jy.data(), a, b) - Dy(g, m.jx.data(), a, b);
        }
    solve(1, nullptr, fE, Ez);
    solve(2, nullptr, fB, Bz);

    /* 5-6. B_perp: (L_h - n* / g) B_perp = -e_z x S (eqs. (18)-(19)). */
    std::vector<T> k2, fBx, fBy, jz;
    int st = assemble<T>(g, *c, *xi, m, psi, Ez, Bz, k2, fBx, fBy, &jz, theta);
    if (st != ORC_OK && status == ORC_OK) status = st;
    solve(3, &k2, fBx, Bx);
    solve(4, &k2, fBy, By);

    if (moments_out) {
        const std::vector<T>* arr[6] = {&m.n, &m.jx, &m.jy, &m.txx, &m.txy, &m.tyy};
        for (int k = 0; k < 6; ++k) std::copy(arr[k]->begin(), arr[k]->end(), moments_out + k * nn);
    }
    if (extra_out) {
        const std::vector<T>* arr[4] = {&k2, &fBx, &fBy, &jz};
        for (int k = 0; k < 4; ++k) std::copy(arr[k]->begin(), arr[k]->end(), extra_out + k * nn);
    }

    /* 7-8. gather grad psi, B (and a laser's a2 = |A-hat|^2 with its gradient)
     *      and push (Push_Trajectory), Vmax after the push. */
    std::vector<T> gx, gy;
    psi_gradient<T>(g, psi, gx, gy);
    LaserNodes las;
    las.a2 = laser_a2(g, *c, *xi);
    if (las.on()) psi_gradient<double>(g, las.a2.data(), las.ax, las.ay);
    double vmax = 0.0;
    if (c->pusher != PUSH_BORIS) {
        int rk_nonphys = 0;
#pragma omp parallel for schedule(static) reduction(max : vmax) reduction(| : rk_nonphys)
        for (int i = 0; i < P; ++i) {
            if (!push_rk(g, c->pusher, *dxi, psi, gx.data(), gy.data(), Bx, By, Bz, las, x[i], y[i],
                         px[i], py[i]))
                rk_nonphys = 1;
            double v = val(sqrt(px[i] * px[i] + py[i] * py[i]) / gi[i]);
            if (v > vmax) vmax = v;
        }
        if (rk_nonphys) status = ORC_NONPHYS;
    } else {
#pragma omp parallel for schedule(static) reduction(max : vmax)
        for (int i = 0; i < P; ++i) {
            T Gx = gather1(g, gx.data(), x[i], y[i]);
            T Gy = gather1(g, gy.data(), x[i], y[i]);
            T bx = gather1(g, Bx, x[i], y[i]);
            T by = gather1(g, By, x[i], y[i]);
            T bz = gather1(g, Bz, x[i], y[i]);
            T ez = pz ? gather1(g, Ez, x[i], y[i]) : T(0.0);
            T p0x = px[i], p0y = py[i];
            double a2 = 0.0, ax = 0.0, ay = 0.0;
            if (las.on()) {
                const double xv = val(x[i]), yv = val(y[i]);
                a2 = gather1(g, las.a2.data(), xv, yv);
                ax = gather1(g, las.ax.data(), xv, yv);
                ay = gather1(g, las.ay.data(), xv, yv);
            }
            push_one(g.L, *dxi, gi[i], Gx, Gy, bx, by, bz, x[i], y[i], px[i], py[i], a2, ax, ay);
            if (pz) { /* dp_z/dxi = -gamma Ez/g - Vx By + Vy Bx at the mean momentum */
                T mx = 0.5 * (p0x + px[i]), my = 0.5 * (p0y + py[i]);
                T gam = (1.0 + mx * mx + my * my + gi[i] * gi[i]) / (2.0 * gi[i]);
                pz[i] += *dxi * (-gam * ez / gi[i] - (mx / gi[i]) * by + (my / gi[i]) * bx);
            }
            double v = val(sqrt(px[i] * px[i] + py[i] * py[i]) / gi[i]);
            if (v > vmax) vmax = v;
        }
    }

    /* 9. Step_Size_Refinement for the next slice. */
    inf.vmax = vmax;
    inf.dxi_next = next_dxi(*c, g.h, vmax);
    *xi = *xi + *dxi;
    *dxi = inf.dxi_next;
    inf.status = status;
    if (info) *info = inf;
    return status;
}


} /* namespace */

/* ================================================================ C API == */
extern "C" {

int oracle_deposit(const oracle_cfg* c, int P, const double* x, const double* y,
                   const double* q, double* out) {
    Grid g(c->n_cells, c->half_width);
    deposit(g, *c, P, x, y, q, out);
    return ORC_OK;
}

int oracle_gather(const oracle_cfg* c, int P, const double* x, const double* y,
                  const double* F, double* out) {
    Grid g(c->n_cells, c->half_width);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P; ++i) out[i] = gather1(g, F, x[i], y[i]);
    return ORC_OK;
}

/* out = L_h u - k2 u at interior nodes, 0 on the boundary (k2 may be NULL). */
int oracle_apply(int N, double h, const double* k2, const double* u, double* out) {
    Level<double> lv;
    lv.N = N;
    lv.h = h;
    if (k2) lv.k2.assign(k2, k2 + (N + 1) * (N + 1));
    std::fill(out, out + (N + 1) * (N + 1), 0.0);
    for (int b = 1; b < N; ++b)
        for (int a = 1; a < N; ++a) out[lv.id(a, b)] = apply_at(lv, u, a, b);
    return ORC_OK;
}

int oracle_mg_solve(int N, double h, const double* k2, const double* f, double* u, double rtol,
                    double atol, int max_cycles, int nu1, int nu2, int* cycles, double* rel) {
    if (N < 2 || (N & (N - 1))) return ORC_INVALID;
    return mg_solve(N, h, k2, f, u, rtol, atol, max_cycles, nu1, nu2, cycles, rel);
}

/* Node gradient of psi as the particle gather uses it (see psi_gradient):
 * out [2][nn] = d/dx, d/dy. */
int oracle_psi_gradient(int N, double L, const double* psi, double* out) {
    Grid g(N, L);
    std::vector<double> gx, gy;
    psi_gradient(g, psi, gx, gy);
    std::copy(gx.begin(), gx.end(), out);
    std::copy(gy.begin(), gy.end(), out + g.nn());
    return ORC_OK;
}

/* Threads used by the parallel loops (n <= 0: the OpenMP default). */
void oracle_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}
int oracle_get_threads(void) { return omp_get_max_threads(); }

int oracle_beam_density(const oracle_cfg* c, double xi, double* out) {
    Grid g(c->n_cells, c->half_width);
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a) out[g.id(a, b)] = beam_density(*c, g.xa(a), g.xa(b), xi);
    return ORC_OK;
}

int oracle_push(double L, double dxi, int P, const double* g_i, const double* gx,
                const double* gy, const double* Bx, const double* By, const double* Bz,
                double* x, double* y, double* px, double* py) {
    for (int i = 0; i < P; ++i)
        push_one(L, dxi, g_i[i], gx[i], gy[i], Bx[i], By[i], Bz[i], x[i], y[i], px[i], py[i]);
    return ORC_OK;
}

/* The particle advance of a slice at xi given its solved fields [5][nn] (psi,
 * Ez, Bz, Bx, By): node gradient of psi, g_i = 1 + psi(r_i), then the pusher
 * of the configuration (Boris-like or Runge-Kutta), walls included, with the
 * laser envelope's ponderomotive terms at xi when the configuration has one.
 * vmax (may be NULL) receives max |p_new|/g_i. */
int oracle_push_fields(const oracle_cfg* c, double xi, double dxi, int P, const double* fields,
                       double* x, double* y, double* px, double* py, double* vmax) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    const double *psi = fields, *Bz = fields + 2 * nn, *Bx = fields + 3 * nn, *By = fields + 4 * nn;
    std::vector<double> gx, gy;
    psi_gradient(g, psi, gx, gy);
    LaserNodes las;
    las.a2 = laser_a2(g, *c, xi);
    if (las.on()) psi_gradient<double>(g, las.a2.data(), las.ax, las.ay);
    double vm = 0.0;
    int nonphys = 0;
#pragma omp parallel for schedule(static) reduction(max : vm) reduction(| : nonphys)
    for (int i = 0; i < P; ++i) {
        const double gi = 1.0 + gather1(g, psi, x[i], y[i]);
        if (!(gi > 0.0)) nonphys = 1;
        if (c->pusher == PUSH_BORIS) {
            double a2 = 0.0, ax = 0.0, ay = 0.0;
            if (las.on()) {
                a2 = gather1(g, las.a2.data(), x[i], y[i]);
                ax = gather1(g, las.ax.data(), x[i], y[i]);
                ay = gather1(g, las.ay.data(), x[i], y[i]);
            }
            push_one(g.L, dxi, gi, gather1(g, gx.data(), x[i], y[i]), gather1(g, gy.data(), x[i], y[i]),
                     gather1(g, Bx, x[i], y[i]), gather1(g, By, x[i], y[i]), gather1(g, Bz, x[i], y[i]),
                     x[i], y[i], px[i], py[i], a2, ax, ay);
        } else if (!push_rk(g, c->pusher, dxi, psi, gx.data(), gy.data(), Bx, By, Bz, las, x[i], y[i],
                            px[i], py[i])) {
            nonphys = 1;
        }
        vm = std::max(vm, std::sqrt(px[i] * px[i] + py[i] * py[i]) / gi);
    }
    if (vmax) *vmax = vm;
    return nonphys ? ORC_NONPHYS : ORC_OK;
}

double oracle_next_dxi(const oracle_cfg* c, double vmax) {
    return next_dxi(*c, 2.0 * c->half_width / c->n_cells, vmax);
}

/* Assembly given the node moments (layout [6][nn]: n*, jx, jy, Txx, Txy, Tyy)
 * and the solved psi, Ez, Bz.  Output [4][nn]: k2, f_Bx, f_By, j_z. */
int oracle_assemble(const oracle_cfg* c, double xi, const double* mom, const double* psi,
                    const double* Ez, const double* Bz, double* out) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    Moments m;
    m.n.assign(mom, mom + nn);
    m.jx.assign(mom + nn, mom + 2 * nn);
    m.jy.assign(mom + 2 * nn, mom + 3 * nn);
    m.txx.assign(mom + 3 * nn, mom + 4 * nn);
    m.txy.assign(mom + 4 * nn, mom + 5 * nn);
    m.tyy.assign(mom + 5 * nn, mom + 6 * nn);
    std::vector<double> k2, fBx, fBy, jz;
    int st = assemble(g, *c, xi, m, psi, Ez, Bz, k2, fBx, fBy, &jz);
    std::copy(k2.begin(), k2.end(), out);
    std::copy(fBx.begin(), fBx.end(), out + nn);
    std::copy(fBy.begin(), fBy.end(), out + 2 * nn);
    std::copy(jz.begin(), jz.end(), out + 3 * nn);
    return st;
}

int oracle_slice_step(const oracle_cfg* c, int P, double* x, double* y, double* px, double* py,
                      double* pz, double* fields, double* xi, double* dxi, oracle_info* info,
                      double* moments_out, double* extra_out) {
    if (!(c->pusher == PUSH_BORIS || c->pusher == PUSH_RK1 || c->pusher == PUSH_RK2 ||
          c->pusher == PUSH_RK4) || (pz && c->pusher != PUSH_BORIS))
        return ORC_INVALID;
    return slice_step_t<double>(c, P, x, y, px, py, pz, fields, xi, dxi, info, moments_out,
                                extra_out, nullptr);
}

/* Tangent-linear model (forward mode) of n_slices slices with up to 8
 * directions at once: the slice step above instantiated with Dual numbers.
 * Seeds (each may be NULL = 0): dP [K][4][P] tangents of the input particles
 * (x, y, px, py), dtheta [K][n_theta] tangents of the driver parameters (beam
 * by beam: amp, or the bin amplitudes).  The fields given are the multigrid
 * initial guesses only and carry no tangent.  The dxi sequence is that of the
 * forward run (held, not differentiated).  Outputs (each may be NULL):
 * dout [K][4][P] tangents of the final particles, dF [K][5][nn] tangents of the
 * last slice's fields, loss / dloss[K] the probe loss of oracle_run_loss and
 * its tangents.  The values (particles, fields, xi, dxi) advance exactly as in
 * oracle_run. */
int oracle_run_tangent(const oracle_cfg* c, int P, double* x, double* y, double* px, double* py,
                       double* fields, double* xi, double* dxi, int n_slices, int K,
                       const double* dP, const double* dtheta, int n_probes, const double* probes,
                       const double* weights, double* loss, double* dloss, double* dout,
                       double* dF) {
    constexpr int KD = 8;
    using D = Dual<KD>;
    if (K < 1 || K > KD || P < 0) return ORC_INVALID;
    if (c->pusher != PUSH_BORIS || c->las_env) return ORC_INVALID;
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    int nth = 0;
    for (int k = 0; k < c->n_beams; ++k) nth += c->beams[k].kind == 0 ? 1 : c->beams[k].n_bins;
    std::vector<D> X(P), Y(P), PX(P), PY(P), F(5 * (size_t)nn), TH(nth);
    for (int i = 0; i < P; ++i) {
        X[i] = D(x[i]);
        Y[i] = D(y[i]);
        PX[i] = D(px[i]);
        PY[i] = D(py[i]);
        if (dP)
            for (int k = 0; k < K; ++k) {
                const double* s = dP + (size_t)k * 4 * P;
                X[i].d[k] = s[i];
                Y[i].d[k] = s[P + i];
                PX[i].d[k] = s[2 * P + i];
                PY[i].d[k] = s[3 * P + i];
            }
    }
    for (size_t i = 0; i < F.size(); ++i) F[i] = D(fields[i]);
    int t = 0;
    for (int k = 0; k < c->n_beams; ++k) {
        const oracle_beam& B = c->beams[k];
        if (B.kind == 0) TH[t++] = D(B.amp);
        else
            for (int m = 0; m < B.n_bins; ++m) TH[t++] = D(B.bin_amp[m]);
    }
    if (dtheta)
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < nth; ++q) TH[q].d[k] = dtheta[(size_t)k * nth + q];
    D Ls(0.0);
    int status = ORC_OK;
    std::vector<int> nodes;
    for (int j = 0; j < n_slices; ++j) {
        oracle_info inf;
        int st = slice_step_t<D>(c, P, X.data(), Y.data(), PX.data(), PY.data(), nullptr,
                                 F.data(), xi, dxi, &inf, nullptr, nullptr, TH.data());
        if (st != ORC_OK) status = st;
        for (int k = 0; k < n_probes; ++k) {
            const double* p = probes + 6 * k;
            if (j < (int)p[1] || j >= (int)p[2]) continue;
            nodes.clear();
            for (int b = 0; b <= g.N; ++b)
                for (int a = 0; a <= g.N; ++a) {
                    double rx = g.xa(a) - p[4], ry = g.xa(b) - p[5];
                    if (rx * rx + ry * ry <= p[3] * p[3]) nodes.push_back(g.id(a, b));
                }
            D sum(0.0);
            for (int i : nodes) sum += F[(int)p[0] * nn + i];
            if (!nodes.empty()) Ls += weights[k] * sum / (double)nodes.size() / (p[2] - p[1]);
        }
    }
    for (int i = 0; i < P; ++i) {
        x[i] = X[i].v;
        y[i] = Y[i].v;
        px[i] = PX[i].v;
        py[i] = PY[i].v;
    }
    for (size_t i = 0; i < F.size(); ++i) fields[i] = F[i].v;
    if (loss) *loss = Ls.v;
    for (int k = 0; k < K; ++k) {
        if (dloss) dloss[k] = Ls.d[k];
        if (dout)
            for (int i = 0; i < P; ++i) {
                double* o = dout + (size_t)k * 4 * P;
                o[i] = X[i].d[k];
                o[P + i] = Y[i].d[k];
                o[2 * P + i] = PX[i].d[k];
                o[3 * P + i] = PY[i].d[k];
            }
        if (dF)
            for (size_t i = 0; i < F.size(); ++i) dF[(size_t)k * F.size() + i] = F[i].d[k];
    }
    return status;
}

/* n_slices consecutive slices from the given state.  fields_hist (may be NULL)
 * receives [n_slices][5][nn]; infos (may be NULL) receives one record per slice. */
int oracle_run(const oracle_cfg* c, int P, double* x, double* y, double* px, double* py,
               double* pz, double* fields, double* xi, double* dxi, int n_slices,
               double* fields_hist, oracle_info* infos) {
    const int nn = (c->n_cells + 1) * (c->n_cells + 1);
    for (int j = 0; j < n_slices; ++j) {
        oracle_info inf;
        int st = oracle_slice_step(c, P, x, y, px, py, pz, fields, xi, dxi, &inf, nullptr, nullptr);
        if (infos) infos[j] = inf;
        if (fields_hist) std::copy(fields, fields + 5 * nn, fields_hist + (size_t)j * 5 * nn);
        if (st != ORC_OK) return st;
    }
    return ORC_OK;
}

} /* extern "C" */

/* ============================================================ driver == */
/*
 * The time loop of Algorithm 1 around the xi-sweep: driver macroparticles
 * (positions x, y, xi = t - z, momenta p_x, p_y, p_z, charge-to-mass ratio
 * q/m in units of e/m_e, and weight w = their number in units of n0 k_p^-3)
 * deposit their longitudinal current onto planes in xi, the plasma is swept
 * through the slices with that current in j_z, the wakefields are gathered at
 * the driver particles and the driver is advanced in t by eqs. (25)-(26).
 * Driver state layout [8][n]: x, y, xi, px, py, pz, qm, w.
 */
namespace {

enum { DX = 0, DY, DXI, DPX, DPY, DPZ, DQM, DW, DNV };

/* The wakefields at one point from a stack of solved slices: psi's node
 * gradient, Ez, Bz, B_perp gathered (CIC) in the two slices that bracket xi
 * (xi_j <= xi < xi_{j+1}) and interpolated linearly in xi; zero ahead of the
 * first slice, at or behind the last and outside the transverse box.  E_perp = -grad psi - e_z x B_perp (the
 * field whose force on a luminal particle is -grad psi, as in the plasma
 * electrons' equations of motion), so E = (-d_x psi + B_y, -d_y psi - B_x, Ez). */
struct SliceStack {
    const Grid* g;
    int ns;
    const double* xi;                  /* [ns] */
    const double* F;                   /* [ns][5][nn] */
    const std::vector<double>* gx;     /* [ns] node gradients of psi */
    const std::vector<double>* gy;
};

void wake_at(const SliceStack& S, double x, double y, double xi, double (&E)[3], double (&B)[3]) {
    for (int q = 0; q < 3; ++q) E[q] = B[q] = 0.0;
    const Grid& g = *S.g;
    if (S.ns < 2 || xi < S.xi[0] || xi >= S.xi[S.ns - 1] || std::fabs(x) > g.L || std::fabs(y) > g.L)
        return;
    int j = 0;  /* xi_j <= xi < xi_{j+1} */
    while (S.xi[j + 1] <= xi) ++j;
    const int j1 = j + 1;
    const double a = (xi - S.xi[j]) / (S.xi[j1] - S.xi[j]);
    const int nn = g.nn();
    const int js[2] = {j, j1};
    const double ws[2] = {1.0 - a, a};
    for (int k = 0; k < 2; ++k) {
        const double* F = S.F + (size_t)js[k] * 5 * nn;
        const double Gx = gather1(g, S.gx[js[k]].data(), x, y), Gy = gather1(g, S.gy[js[k]].data(), x, y);
        const double ez = gather1(g, F + nn, x, y), bz = gather1(g, F + 2 * nn, x, y);
        const double bx = gather1(g, F + 3 * nn, x, y), by = gather1(g, F + 4 * nn, x, y);
        E[0] += ws[k] * (-Gx + by);
        E[1] += ws[k] * (-Gy - bx);
        E[2] += ws[k] * ez;
        B[0] += ws[k] * bx;
        B[1] += ws[k] * by;
        B[2] += ws[k] * bz;
    }
}

/* The high-frequency fields of the laser (Sec. IV, eqs. (21)-(24)) at (x, y,
 * xi) and time t + tau dt, from the envelope planes at t (A0) and t + dt (A1)
 * (x-polarised: A-hat is A-hat_x).  The envelope there is the interpolant
 * linear in t between A0 and A1, linear in xi between the planes xi_m = m
 * dxi0 around xi (planes outside [0, las_nz) are zero) and bilinear (CIC) in
 * x, y; its derivatives are those of the interpolant.  With the phase
 * e = exp(-i k0 xi):
 *   E_x = Re[-(d_t A + d_xi A - i k0 A) e],  B_y = Re[(-d_xi A + i k0 A) e],
 *   E_z = Re[-d_x A e],                      B_z = Re[-d_y A e],
 * E_y = B_x = 0; zero outside the transverse box. */
void laser_fields_at(const Grid& g, const oracle_cfg& c, const cplx* A0, const cplx* A1, double dt,
                     double tau, double x, double y, double xi, double (&E)[3], double (&B)[3]) {
    for (int q = 0; q < 3; ++q) E[q] = B[q] = 0.0;
    if (std::fabs(x) > g.L || std::fabs(y) > g.L) return;
    const int nn = g.nn();
    int a, b;
    double dx, dy;
    cic(g, x, a, dx);
    cic(g, y, b, dy);
    const double t = xi / c.dxi0;
    const double mf = std::floor(t);
    const double wz = t - mf;
    /* value, d/dx, d/dy of the bilinear interpolant of one plane */
    auto plane = [&](const cplx* A, double q, cplx& v, cplx& vx, cplx& vy) {
        v = vx = vy = cplx(0.0);
        if (q < 0.0 || q >= c.las_nz) return;
        const cplx* P = A + (size_t)q * nn;
        const cplx f00 = P[g.id(a, b)], f10 = P[g.id(a + 1, b)];
        const cplx f01 = P[g.id(a, b + 1)], f11 = P[g.id(a + 1, b + 1)];
        v = f00 * ((1.0 - dx) * (1.0 - dy)) + f10 * (dx * (1.0 - dy)) + f01 * ((1.0 - dx) * dy) +
            f11 * (dx * dy);
        vx = ((f10 - f00) * (1.0 - dy) + (f11 - f01) * dy) / g.h;
        vy = ((f01 - f00) * (1.0 - dx) + (f11 - f10) * dx) / g.h;
    };
    cplx v[2][2], vx[2][2], vy[2][2];  /* [time level][plane m, m + 1] */
    const cplx* As[2] = {A0, A1};
    for (int l = 0; l < 2; ++l)
        for (int k = 0; k < 2; ++k) plane(As[l], mf + k, v[l][k], vx[l][k], vy[l][k]);
    const double wt[2] = {1.0 - tau, tau}, wq[2] = {1.0 - wz, wz};
    cplx A(0.0), At(0.0), Axi(0.0), Ax(0.0), Ay(0.0);
    for (int l = 0; l < 2; ++l)
        for (int k = 0; k < 2; ++k) {
            A += (wt[l] * wq[k]) * v[l][k];
            Ax += (wt[l] * wq[k]) * vx[l][k];
            Ay += (wt[l] * wq[k]) * vy[l][k];
        }
    for (int k = 0; k < 2; ++k) At += wq[k] * (v[1][k] - v[0][k]) / dt;
    for (int l = 0; l < 2; ++l) Axi += wt[l] * (v[l][1] - v[l][0]) / c.dxi0;
    const cplx e(std::cos(c.las_k0 * xi), -std::sin(c.las_k0 * xi));
    const cplx ik0A = cplx(0.0, c.las_k0) * A;
    E[0] = std::real(-(At + Axi - ik0A) * e);
    E[2] = std::real(-Ax * e);
    B[1] = std::real((ik0A - Axi) * e);
    B[2] = std::real(-Ay * e);
}

/* The laser's planes at t and t + dt seen by the driver push (both NULL: no
 * laser fields). */
struct LaserPair {
    const cplx* A0;
    const cplx* A1;
};

/* One sub-step of length d of the driver push below, at the fraction tau of
 * the time step dt: a drift of d/2, a kick of d/2 by qm E, the rotation of a
 * Boris push about qm B/gamma, a kick of d/2 and a drift of d/2 with the new
 * momentum (a volume-preserving splitting of the relativistic Lorentz-force
 * flow), with E, B = the wake (Ew, Bw) plus the laser's fields at the mid
 * position.  In (x, y, xi): dx/dt = p_x/gamma, dy/dt = p_y/gamma,
 * dxi/dt = 1 - p_z/gamma. */
void sub_step(const SliceStack& S, const LaserPair& las, const oracle_cfg& c, double d, double tau,
              double dt, const double (&Ew)[3], const double (&Bw)[3], double* st) {
    const double g0 = std::sqrt(1.0 + st[DPX] * st[DPX] + st[DPY] * st[DPY] + st[DPZ] * st[DPZ]);
    const double xh = st[DX] + 0.5 * d * st[DPX] / g0;
    const double yh = st[DY] + 0.5 * d * st[DPY] / g0;
    const double xih = st[DXI] + 0.5 * d * (1.0 - st[DPZ] / g0);
    double E[3] = {Ew[0], Ew[1], Ew[2]}, B[3] = {Bw[0], Bw[1], Bw[2]};
    if (las.A0) {
        double El[3], Bl[3];
        laser_fields_at(*S.g, c, las.A0, las.A1, dt, tau, xh, yh, xih, El, Bl);
        for (int q = 0; q < 3; ++q) {
            E[q] += El[q];
            B[q] += Bl[q];
        }
    }
    const double k = 0.5 * d * st[DQM];
    double m[3] = {st[DPX] + k * E[0], st[DPY] + k * E[1], st[DPZ] + k * E[2]};
    const double gm = std::sqrt(1.0 + m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    const double t[3] = {k * B[0] / gm, k * B[1] / gm, k * B[2] / gm};
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    const double sv[3] = {2.0 * t[0] / (1.0 + tt), 2.0 * t[1] / (1.0 + tt), 2.0 * t[2] / (1.0 + tt)};
    const double pr[3] = {m[0] + (m[1] * t[2] - m[2] * t[1]), m[1] + (m[2] * t[0] - m[0] * t[2]),
                          m[2] + (m[0] * t[1] - m[1] * t[0])};
    const double pp[3] = {m[0] + (pr[1] * sv[2] - pr[2] * sv[1]), m[1] + (pr[2] * sv[0] - pr[0] * sv[2]),
                          m[2] + (pr[0] * sv[1] - pr[1] * sv[0])};
    st[DPX] = pp[0] + k * E[0];
    st[DPY] = pp[1] + k * E[1];
    st[DPZ] = pp[2] + k * E[2];
    const double g1 = std::sqrt(1.0 + st[DPX] * st[DPX] + st[DPY] * st[DPY] + st[DPZ] * st[DPZ]);
    st[DX] = xh + 0.5 * d * st[DPX] / g1;
    st[DY] = yh + 0.5 * d * st[DPY] / g1;
    st[DXI] = xih + 0.5 * d * (1.0 - st[DPZ] / g1);
}

/* One step dt of eqs. (25)-(26) for one driver particle in c.drv_nsub
 * sub-steps (the sub-cycling of Sec. IV that resolves the laser's
 * oscillation).  The wake is gathered once, at the mid-step position of the
 * whole step (it changes over the step only as the particle moves through
 * it), the laser's fields (laser_fields_at) at every sub-step's mid position
 * and time. */
void drive_one(const SliceStack& S, const LaserPair& las, const oracle_cfg& c, double dt,
               double* st) {
    const int nsub = c.drv_nsub > 1 ? c.drv_nsub : 1;
    const double g0 = std::sqrt(1.0 + st[DPX] * st[DPX] + st[DPY] * st[DPY] + st[DPZ] * st[DPZ]);
    double Ew[3], Bw[3];
    wake_at(S, st[DX] + 0.5 * dt * st[DPX] / g0, st[DY] + 0.5 * dt * st[DPY] / g0,
            st[DXI] + 0.5 * dt * (1.0 - st[DPZ] / g0), Ew, Bw);
    const double d = dt / nsub;
    for (int sub = 0; sub < nsub; ++sub) sub_step(S, las, c, d, (sub + 0.5) / nsub, dt, Ew, Bw, st);
}

}  // namespace

extern "C" {

/* Longitudinal current of the driver particles on nz planes xi_m = xi0 +
 * m dz (out [nz][nn]): each particle adds -qm w v_z (its charge -qm in units
 * of -e times its number, times v_z = p_z/gamma) with CIC weights in x and y
 * and linear (hat) weights in xi, divided by h^2 dz.  Particles outside the
 * transverse box or the plane range add nothing.  (A luminal driver,
 * v_z -> 1, has rho_b = J_bz: it enters the slice only through j_z.) */
int oracle_driver_deposit(const oracle_cfg* c, int n, const double* st, int nz, double xi0,
                          double dz, double* out) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    std::fill(out, out + (size_t)nz * nn, 0.0);
    for (int p = 0; p < n; ++p) {
        const double x = st[DX * n + p], y = st[DY * n + p], xi = st[DXI * n + p];
        if (std::fabs(x) > g.L || std::fabs(y) > g.L) continue;
        const double t = (xi - xi0) / dz;
        const int m = (int)std::floor(t);
        if (m < 0 || m > nz - 2) continue;
        const double az = t - m;
        const double px = st[DPX * n + p], py = st[DPY * n + p], pz = st[DPZ * n + p];
        const double vz = pz / std::sqrt(1.0 + px * px + py * py + pz * pz);
        const double q = -st[DQM * n + p] * st[DW * n + p] * vz / (g.h * g.h * dz);
        int a, b;
        double dx, dy;
        cic(g, x, a, dx);
        cic(g, y, b, dy);
        for (int k = 0; k < 2; ++k) {
            double* P = out + (size_t)(m + k) * nn;
            const double wz = k ? az : 1.0 - az;
            P[g.id(a, b)] += q * wz * (1.0 - dx) * (1.0 - dy);
            P[g.id(a + 1, b)] += q * wz * dx * (1.0 - dy);
            P[g.id(a, b + 1)] += q * wz * (1.0 - dx) * dy;
            P[g.id(a + 1, b + 1)] += q * wz * dx * dy;
        }
    }
    return ORC_OK;
}

/* Advance n driver particles (state [8][n], updated) by dt through the wake
 * of ns solved slices at positions xi_s[ns] with fields F_s [ns][5][nn] and,
 * when env0 and env1 are given (the laser's planes at t and t + dt, complex
 * [las_nz][nn]), the laser's fields, in c->drv_nsub sub-steps. */
int oracle_driver_push(const oracle_cfg* c, double dt, int n, double* st, int ns,
                       const double* xi_s, const double* F_s, const double* env0,
                       const double* env1) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    if ((env0 == nullptr) != (env1 == nullptr)) return ORC_INVALID;
    std::vector<std::vector<double>> gx(ns), gy(ns);
    for (int j = 0; j < ns; ++j) psi_gradient(g, F_s + (size_t)j * 5 * nn, gx[j], gy[j]);
    const SliceStack S{&g, ns, xi_s, F_s, gx.data(), gy.data()};
    const LaserPair las{reinterpret_cast<const cplx*>(env0), reinterpret_cast<const cplx*>(env1)};
#pragma omp parallel for schedule(static)
    for (int p = 0; p < n; ++p) {
        double v[DNV];
        for (int q = 0; q < DNV; ++q) v[q] = st[(size_t)q * n + p];
        drive_one(S, las, *c, dt, v);
        for (int q = 0; q < DNV; ++q) st[(size_t)q * n + p] = v[q];
    }
    return ORC_OK;
}

/* Envelope planes env_in [nz][nn] (complex, (re, im) pairs) at time t
 * advanced by dt into env_out (same layout), plane after plane from the front
 * (laser_plane_advance), with the susceptibility chi [nz][nn] (NULL: vacuum).
 * The configuration gives k0, the plane spacing dxi0 and the multigrid's stop
 * rule; cycles [nz] (may be NULL) receives each plane's cycle count. */
int oracle_laser_advance(const oracle_cfg* c, double dt, int nz, const double* env_in,
                         const double* chi, double* env_out, int* cycles) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    const cplx* A0 = reinterpret_cast<const cplx*>(env_in);
    cplx* A1 = reinterpret_cast<cplx*>(env_out);
    for (int j = 0; j < nz; ++j) {
        int cyc = 0;
        double rel = 0.0;
        const int st = laser_plane_advance(
            g, *c, dt, chi ? chi + (size_t)j * nn : nullptr, A0 + (size_t)j * nn,
            j ? A0 + (size_t)(j - 1) * nn : nullptr, j ? A1 + (size_t)(j - 1) * nn : nullptr,
            A1 + (size_t)j * nn, &cyc, &rel);
        if (cycles) cycles[j] = cyc;
        if (st != ORC_OK) return st;
    }
    return ORC_OK;
}

/* The laser's fields (laser_fields_at) at n points pts [3][n] (x, y, xi) and
 * time t + tau dt from the planes env0 (t) and env1 (t + dt): out [6][n] =
 * E_x, E_y, E_z, B_x, B_y, B_z. */
int oracle_laser_fields(const oracle_cfg* c, double dt, double tau, int n, const double* pts,
                        const double* env0, const double* env1, double* out) {
    Grid g(c->n_cells, c->half_width);
    const cplx* A0 = reinterpret_cast<const cplx*>(env0);
    const cplx* A1 = reinterpret_cast<const cplx*>(env1);
    for (int p = 0; p < n; ++p) {
        double E[3], B[3];
        laser_fields_at(g, *c, A0, A1, dt, tau, pts[p], pts[n + p], pts[2 * n + p], E, B);
        for (int q = 0; q < 3; ++q) {
            out[(size_t)q * n + p] = E[q];
            out[(size_t)(3 + q) * n + p] = B[q];
        }
    }
    return ORC_OK;
}

/* One step of the time loop (Algorithm 1, outer loop): the driver's current
 * on nz planes (xi0, dz), a sweep of n_slices slices through the plasma given
 * (normally the cold plasma at xi = 0 with zero fields, advanced in place)
 * with that current in j_z, then the driver advanced by dt through the wake
 * of those slices.  xi_hist [n_slices] and fields_hist [n_slices][5][nn] (may
 * be NULL) receive the slices.
 * With a laser envelope in the configuration (c->las_env, the planes at t)
 * the plasma sees it, and env_next (non-NULL, [las_nz][nn] complex) receives
 * the planes at t + dt: each plane j is advanced (laser_plane_advance) right
 * after slice j, with that slice's susceptibility chi = n* / (1+psi) (the k2 of
 * its B-perp system); the driver push then adds the laser's fields from both
 * sets of planes.  This needs fixed steps (adaptive = 0, so that slice j lies
 * on plane j) and n_slices >= las_nz. */
int oracle_time_step(const oracle_cfg* c, int P, double* x, double* y, double* px, double* py,
                     double* fields, double* xi, double* dxi, int n_slices, int n_drv,
                     double* drv, int nz, double xi0, double dz, double dt, double* xi_hist,
                     double* fields_hist, oracle_info* infos, double* env_next) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    const bool las = c->las_env && env_next;
    if (las && (c->adaptive || n_slices < c->las_nz)) return ORC_INVALID;
    std::vector<double> planes((size_t)nz * nn), hx(n_slices), hF((size_t)n_slices * 5 * nn);
    std::vector<double> extra(las ? 4 * (size_t)nn : 0);
    const cplx* A0 = reinterpret_cast<const cplx*>(c->las_env);
    cplx* A1 = reinterpret_cast<cplx*>(env_next);
    oracle_driver_deposit(c, n_drv, drv, nz, xi0, dz, planes.data());
    oracle_cfg cc = *c;
    cc.drv_planes = planes.data();
    cc.drv_nz = nz;
    cc.drv_xi0 = xi0;
    cc.drv_dz = dz;
    int status = ORC_OK;
    for (int j = 0; j < n_slices && status == ORC_OK; ++j) {
        hx[j] = *xi;
        oracle_info inf;
        status = oracle_slice_step(&cc, P, x, y, px, py, nullptr, fields, xi, dxi, &inf, nullptr,
                                   las ? extra.data() : nullptr);
        if (infos) infos[j] = inf;
        std::copy(fields, fields + 5 * nn, hF.begin() + (size_t)j * 5 * nn);
        if (las && status == ORC_OK && j < c->las_nz)
            status = laser_plane_advance(g, *c, dt, extra.data(), A0 + (size_t)j * nn,
                                         j ? A0 + (size_t)(j - 1) * nn : nullptr,
                                         j ? A1 + (size_t)(j - 1) * nn : nullptr,
                                         A1 + (size_t)j * nn, nullptr, nullptr);
    }
    if (status != ORC_OK) return status;
    oracle_driver_push(c, dt, n_drv, drv, n_slices, hx.data(), hF.data(), las ? c->las_env : nullptr,
                       las ? env_next : nullptr);
    if (xi_hist) std::copy(hx.begin(), hx.end(), xi_hist);
    if (fields_hist) std::copy(hF.begin(), hF.end(), fields_hist);
    return ORC_OK;
}

} /* extern "C" */

/* =========================================================== adjoint == */
/*
 * Reverse mode of the discrete slice map above (discretise, then
 * differentiate): given the adjoints of a slice's outputs (the particles at
 * xi + dxi and the five fields at xi) it returns the adjoints of its inputs
 * (the particles at xi) and adds the adjoint of the driver parameters theta.
 * theta lists, beam by beam, the Gaussian amplitude or the radial-bin
 * amplitudes.  The step dxi is treated as a constant; at the kinks of the
 * map (cell crossings, wall reflections) the branch actually taken is
 * differentiated.  The elliptic operators are symmetric, so every adjoint
 * solve uses the same multigrid as the forward solves.
 */
namespace {

struct CicW {
    int a, b;
    double dx, dy;
};

CicW cicw(const Grid& g, double x, double y) {
    CicW w;
    cic(g, x, w.a, w.dx);
    cic(g, y, w.b, w.dy);
    return w;
}

/* Value and x/y derivatives of the bilinear interpolant of F in the particle's cell. */
void interp_grad(const Grid& g, const double* F, const CicW& w, double& v, double& vx, double& vy) {
    const double f00 = F[g.id(w.a, w.b)], f10 = F[g.id(w.a + 1, w.b)];
    const double f01 = F[g.id(w.a, w.b + 1)], f11 = F[g.id(w.a + 1, w.b + 1)];
    v = f00 * (1 - w.dx) * (1 - w.dy) + f10 * w.dx * (1 - w.dy) + f01 * (1 - w.dx) * w.dy +
        f11 * w.dx * w.dy;
    vx = ((f10 - f00) * (1 - w.dy) + (f11 - f01) * w.dy) / g.h;
    vy = ((f01 - f00) * (1 - w.dx) + (f11 - f10) * w.dx) / g.h;
}

/* Adjoint of gather: Fbar[corners] += s * weights. */
void scatter(const Grid& g, double* Fbar, const CicW& w, double s) {
    Fbar[g.id(w.a, w.b)] += s * (1 - w.dx) * (1 - w.dy);
    Fbar[g.id(w.a + 1, w.b)] += s * w.dx * (1 - w.dy);
    Fbar[g.id(w.a, w.b + 1)] += s * (1 - w.dx) * w.dy;
    Fbar[g.id(w.a + 1, w.b + 1)] += s * w.dx * w.dy;
}

/* d(beam density)/d(theta_k) at one node and slice position, k over all params. */
void beam_dtheta(const oracle_cfg& c, double x, double y, double xi, std::vector<double>& out) {
    out.clear();
    for (int k = 0; k < c.n_beams; ++k) {
        const oracle_beam& B = c.beams[k];
        double rx = x - B.x0, ry = y - B.y0;
        double r2 = rx * rx + ry * ry;
        double lz = (xi - B.xi_c) * (xi - B.xi_c) / (B.sigma_z * B.sigma_z);
        if (B.kind == 0) {
            out.push_back(xi < 0.0 ? 0.0 : std::exp(-r2 / (B.sigma_r * B.sigma_r) - lz));
        } else {
            double r = std::sqrt(r2);
            double dr = B.r_max / B.n_bins;
            int kb = (int)std::floor(r / dr);
            for (int m = 0; m < B.n_bins; ++m)
                out.push_back((xi >= 0.0 && r < B.r_max && kb == m) ? std::exp(-lz) : 0.0);
        }
    }
}

int theta_count(const oracle_cfg& c) {
    int n = 0;
    for (int k = 0; k < c.n_beams; ++k) n += c.beams[k].kind == 0 ? 1 : c.beams[k].n_bins;
    return n;
}

/* Zero the boundary entries of a node adjoint (the boundary values are fixed). */
void zero_boundary(const Grid& g, std::vector<double>& v) {
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a)
            if (a == 0 || b == 0 || a == g.N || b == g.N) v[g.id(a, b)] = 0.0;
}

/* ubar of an interior node array from the adjoint of D_x u (or D_y u) given at
 * interior nodes: D^T. */
void add_Dx_T(const Grid& g, const std::vector<double>& dbar, std::vector<double>& ubar) {
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) {
            double s = dbar[g.id(a, b)] / (2.0 * g.h);
            ubar[g.id(a + 1, b)] += s;
            ubar[g.id(a - 1, b)] -= s;
        }
}
void add_Dy_T(const Grid& g, const std::vector<double>& dbar, std::vector<double>& ubar) {
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) {
            double s = dbar[g.id(a, b)] / (2.0 * g.h);
            ubar[g.id(a, b + 1)] += s;
            ubar[g.id(a, b - 1)] -= s;
        }
}

int adjoint_solve(const Grid& g, const oracle_cfg& c, const std::vector<double>* k2,
                  std::vector<double> rhs, std::vector<double>& lam) {
    zero_boundary(g, rhs);
    lam.assign(g.nn(), 0.0);
    int cyc;
    double rel;
    return mg_solve(g.N, g.h, k2 ? k2->data() : nullptr, rhs.data(), lam.data(), c.mg_rtol, c.mg_atol,
                    c.mg_max_cycles, c.nu_pre, c.nu_post, &cyc, &rel);
}

} /* namespace */

extern "C" {

int oracle_theta_count(const oracle_cfg* c) { return theta_count(*c); }

/* Reverse of one slice.  Inputs: the slice's input particles (x, y, px, py),
 * its solved fields [5][nn], xi and dxi; xb, yb, pxb, pyb: adjoints of the
 * output particles (overwritten with the adjoints of the input particles);
 * Fbar [5][nn] (may be NULL): adjoints of the fields; theta_bar: accumulated. */
int oracle_slice_adjoint(const oracle_cfg* c, int P, const double* x, const double* y,
                         const double* px, const double* py, const double* fields, double xi,
                         double dxi, double* xb, double* yb, double* pxb, double* pyb,
                         const double* Fbar, double* theta_bar) {
    /* the reverse sweep is the Boris-like push's, without a laser */
    if (c->pusher != PUSH_BORIS || c->las_env) return ORC_INVALID;
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    const double* psi = fields;
    const double* Ez = fields + nn;
    const double* Bz = fields + 2 * nn;
    const double* Bx = fields + 3 * nn;
    const double* By = fields + 4 * nn;
    const double wd = c->n0 * g.h * g.h / c->ppc / (g.h * g.h);  /* deposit weight per particle */
    int status = ORC_OK;

    /* forward quantities recomputed from the slice input */
    std::vector<CicW> W(P);
    std::vector<double> gi(P), vx(P), vy(P);
    Moments m;
    m.n.assign(nn, 0.0);
    deposit<double>(g, *c, P, x, y, nullptr, m.n.data());
    for (int i = 0; i < P; ++i) {
        W[i] = cicw(g, x[i], y[i]);
        gi[i] = 1.0 + gather1(g, psi, x[i], y[i]);
        vx[i] = px[i] / gi[i];
        vy[i] = py[i] / gi[i];
    }
    {
        std::vector<double> q(P);
        m.jx.assign(nn, 0.0); deposit(g, *c, P, x, y, vx.data(), m.jx.data());
        m.jy.assign(nn, 0.0); deposit(g, *c, P, x, y, vy.data(), m.jy.data());
        for (int i = 0; i < P; ++i) q[i] = vx[i] * vx[i];
        m.txx.assign(nn, 0.0); deposit(g, *c, P, x, y, q.data(), m.txx.data());
        for (int i = 0; i < P; ++i) q[i] = vx[i] * vy[i];
        m.txy.assign(nn, 0.0); deposit(g, *c, P, x, y, q.data(), m.txy.data());
        for (int i = 0; i < P; ++i) q[i] = vy[i] * vy[i];
        m.tyy.assign(nn, 0.0); deposit(g, *c, P, x, y, q.data(), m.tyy.data());
    }
    std::vector<double> k2, fBx, fBy, jz;
    assemble(g, *c, xi, m, psi, Ez, Bz, k2, fBx, fBy, &jz);
    std::vector<double> gxn, gyn;
    psi_gradient(g, psi, gxn, gyn);

    /* node adjoints */
    std::vector<double> psib(nn, 0.0), Ezb(nn, 0.0), Bzb(nn, 0.0), Bxb(nn, 0.0), Byb(nn, 0.0);
    std::vector<double> gxb(nn, 0.0), gyb(nn, 0.0), gib(P, 0.0);
    if (Fbar) {
        for (int i = 0; i < nn; ++i) {
            psib[i] += Fbar[i];
            Ezb[i] += Fbar[nn + i];
            Bzb[i] += Fbar[2 * nn + i];
            Bxb[i] += Fbar[3 * nn + i];
            Byb[i] += Fbar[4 * nn + i];
        }
    }

    /* --- 7. push, reversed per particle (fields frozen, dxi constant) */
    for (int i = 0; i < P; ++i) {
        const CicW& w = W[i];
        double Gx, Gxx, Gxy, Gy, Gyx, Gyy, bx, bxx, bxy, by, byx, byy, bz, bzx, bzy;
        interp_grad(g, gxn.data(), w, Gx, Gxx, Gxy);
        interp_grad(g, gyn.data(), w, Gy, Gyx, Gyy);
        interp_grad(g, Bx, w, bx, bxx, bxy);
        interp_grad(g, By, w, by, byx, byy);
        interp_grad(g, Bz, w, bz, bzx, bzy);
        const double G_ = gi[i], p0x = px[i], p0y = py[i], d = dxi, L = g.L;
        /* forward replay */
        const double gam = (1.0 + p0x * p0x + p0y * p0y + G_ * G_) / (2.0 * G_);
        const double Fx = gam * Gx / G_ - by, Fy = gam * Gy / G_ + bx;
        const double mx = p0x + 0.5 * d * Fx, my = p0y + 0.5 * d * Fy;
        const double t = bz * d / (2.0 * G_), s = 2.0 * t / (1.0 + t * t);
        const double qx = mx - t * my, qy = my + t * mx;
        const double rx = mx - s * qy, ry = my + s * qx;
        const double p1x = rx + 0.5 * d * Fx, p1y = ry + 0.5 * d * Fy;
        const double x1 = x[i] + d * p1x / G_, y1 = y[i] + d * p1y / G_;
        /* reverse */
        double x1b = xb[i], y1b = yb[i], p1xb = pxb[i], p1yb = pyb[i];
        if (x1 > L || x1 < -L) { x1b = -x1b; p1xb = -p1xb; }
        if (y1 > L || y1 < -L) { y1b = -y1b; p1yb = -p1yb; }
        double xbar = x1b, ybar = y1b, gb = 0.0;
        p1xb += x1b * d / G_;
        p1yb += y1b * d / G_;
        gb += -(x1b * d * p1x + y1b * d * p1y) / (G_ * G_);
        double rxb = p1xb, ryb = p1yb, Fxb = 0.5 * d * p1xb, Fyb = 0.5 * d * p1yb;
        double mxb = rxb, myb = ryb, sb = -rxb * qy + ryb * qx;
        double qyb = -rxb * s, qxb = ryb * s;
        mxb += qxb + qyb * t;
        myb += -qxb * t + qyb;
        double tb = -qxb * my + qyb * mx;
        tb += sb * 2.0 * (1.0 - t * t) / ((1.0 + t * t) * (1.0 + t * t));
        double bzb = tb * d / (2.0 * G_);
        gb += -tb * bz * d / (2.0 * G_ * G_);
        double p0xb = mxb, p0yb = myb;
        Fxb += 0.5 * d * mxb;
        Fyb += 0.5 * d * myb;
        double gamb = Fxb * Gx / G_ + Fyb * Gy / G_;
        double Gxb = Fxb * gam / G_, Gyb = Fyb * gam / G_;
        gb += -(Fxb * gam * Gx + Fyb * gam * Gy) / (G_ * G_);
        double byb = -Fxb, bxb = Fyb;
        p0xb += gamb * p0x / G_;
        p0yb += gamb * p0y / G_;
        gb += gamb * (G_ * G_ - 1.0 - p0x * p0x - p0y * p0y) / (2.0 * G_ * G_);
        /* gathers of grad psi and B: node adjoints and position derivatives */
        scatter(g, gxb.data(), w, Gxb);
        scatter(g, gyb.data(), w, Gyb);
        scatter(g, Bxb.data(), w, bxb);
        scatter(g, Byb.data(), w, byb);
        scatter(g, Bzb.data(), w, bzb);
        xbar += Gxb * Gxx + Gyb * Gyx + bxb * bxx + byb * byx + bzb * bzx;
        ybar += Gxb * Gxy + Gyb * Gyy + bxb * bxy + byb * byy + bzb * bzy;
        xb[i] = xbar;
        yb[i] = ybar;
        pxb[i] = p0xb;
        pyb[i] = p0yb;
        gib[i] = gb;
    }
    /* node gradient of psi (central inside, one-sided on the boundary), reversed */
    for (int b = 0; b <= g.N; ++b)
        for (int a = 0; a <= g.N; ++a) {
            double sx = gxb[g.id(a, b)], sy = gyb[g.id(a, b)];
            if (a == 0) { psib[g.id(1, b)] += sx / g.h; psib[g.id(0, b)] -= sx / g.h; }
            else if (a == g.N) { psib[g.id(g.N, b)] += sx / g.h; psib[g.id(g.N - 1, b)] -= sx / g.h; }
            else { psib[g.id(a + 1, b)] += sx / (2 * g.h); psib[g.id(a - 1, b)] -= sx / (2 * g.h); }
            if (b == 0) { psib[g.id(a, 1)] += sy / g.h; psib[g.id(a, 0)] -= sy / g.h; }
            else if (b == g.N) { psib[g.id(a, g.N)] += sy / g.h; psib[g.id(a, g.N - 1)] -= sy / g.h; }
            else { psib[g.id(a, b + 1)] += sy / (2 * g.h); psib[g.id(a, b - 1)] -= sy / (2 * g.h); }
        }

    /* --- 6. B_perp Helmholtz solves: lambda = (L_h - k2)^-1 Bbar, k2bar = lambda B */
    std::vector<double> lx, ly;
    if (adjoint_solve(g, *c, &k2, Bxb, lx) != ORC_OK) status = ORC_NOCONV;
    if (adjoint_solve(g, *c, &k2, Byb, ly) != ORC_OK) status = ORC_NOCONV;

    /* --- 5. assembly reversed (f_Bx = lx, f_By = ly, k2bar) */
    std::vector<double> nb(nn, 0.0), jxb(nn, 0.0), jyb(nn, 0.0), txxb(nn, 0.0), txyb(nn, 0.0),
        tyyb(nn, 0.0), jzb(nn, 0.0), psxb(nn, 0.0), psyb(nn, 0.0);
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) {
            const int i = g.id(a, b);
            const double Lxb = lx[i], Lyb = ly[i];
            const double s = 1.0 / (2.0 * g.h);
            /* D_y(j_z - Tyy) - D_x Txy  and  D_x(Txx - j_z) + D_y Txy */
            jzb[g.id(a, b + 1)] += Lxb * s; jzb[g.id(a, b - 1)] -= Lxb * s;
            tyyb[g.id(a, b + 1)] -= Lxb * s; tyyb[g.id(a, b - 1)] += Lxb * s;
            txyb[g.id(a + 1, b)] -= Lxb * s; txyb[g.id(a - 1, b)] += Lxb * s;
            txxb[g.id(a + 1, b)] += Lyb * s; txxb[g.id(a - 1, b)] -= Lyb * s;
            jzb[g.id(a + 1, b)] -= Lyb * s; jzb[g.id(a - 1, b)] += Lyb * s;
            txyb[g.id(a, b + 1)] += Lyb * s; txyb[g.id(a, b - 1)] -= Lyb * s;
            if (!(m.n[i] > 0.0)) continue;
            const double gg = 1.0 + psi[i], n = m.n[i];
            const double G = (n * (1.0 + gg * gg) + gg * gg * (m.txx[i] + m.tyy[i])) / (2.0 * gg);
            const double psx = Dx(g, psi, a, b), psy = Dy(g, psi, a, b);
            const double jx_ = m.jx[i], jy_ = m.jy[i], Txx = m.txx[i], Txy = m.txy[i], Tyy = m.tyy[i];
            jxb[i] += (Lxb * Bz[i] + Lyb * Ez[i]) / gg;
            jyb[i] += (-Lxb * Ez[i] + Lyb * Bz[i]) / gg;
            Bzb[i] += (Lxb * jx_ + Lyb * jy_) / gg;
            Ezb[i] += (-Lxb * jy_ + Lyb * jx_) / gg;
            double Gb = (Lxb * psy - Lyb * psx) / (gg * gg);
            tyyb[i] += -Lxb * psy / gg;
            txxb[i] += Lyb * psx / gg;
            txyb[i] += (-Lxb * psx + Lyb * psy) / gg;
            psxb[i] += -Lxb * Txy / gg - Lyb * (G / (gg * gg) - Txx / gg);
            psyb[i] += Lxb * (G / (gg * gg) - Tyy / gg) + Lyb * Txy / gg;
            double ggb = Lxb * (-(jx_ * Bz[i] - jy_ * Ez[i]) / (gg * gg) +
                                (-2.0 * G / (gg * gg * gg) + Tyy / (gg * gg)) * psy +
                                (Txy / (gg * gg)) * psx) +
                         Lyb * (-(jy_ * Bz[i] + jx_ * Ez[i]) / (gg * gg) -
                                (-2.0 * G / (gg * gg * gg) + Txx / (gg * gg)) * psx -
                                (Txy / (gg * gg)) * psy);
            /* k2 = n / g with k2bar = lx Bx + ly By */
            const double k2b = lx[i] * Bx[i] + ly[i] * By[i];
            nb[i] += k2b / gg;
            ggb += -k2b * n / (gg * gg);
            /* G = [n (1 + g^2) + g^2 (Txx + Tyy)] / (2g) */
            nb[i] += Gb * (1.0 + gg * gg) / (2.0 * gg);
            txxb[i] += Gb * gg / 2.0;
            tyyb[i] += Gb * gg / 2.0;
            ggb += Gb * (n * (gg * gg - 1.0) / (2.0 * gg * gg) + (Txx + Tyy) / 2.0);
            psib[i] += ggb;
        }
    add_Dx_T(g, psxb, psib);
    add_Dy_T(g, psyb, psib);
    /* j_z = G/g - n* + n_b(theta) on every node (plasma part where n* > 0) */
    {
        std::vector<double> dth;
        const int nth = theta_count(*c);
        for (int b = 0; b <= g.N; ++b)
            for (int a = 0; a <= g.N; ++a) {
                const int i = g.id(a, b);
                const double s = jzb[i];
                if (s == 0.0) continue;
                if (m.n[i] > 0.0) {
                    const double gg = 1.0 + psi[i], n = m.n[i];
                    nb[i] += s * (1.0 - gg * gg) / (2.0 * gg * gg);
                    txxb[i] += s * 0.5;
                    tyyb[i] += s * 0.5;
                    psib[i] += -s * n / (gg * gg * gg);
                }
                beam_dtheta(*c, g.xa(a), g.xa(b), xi, dth);
                for (int k = 0; k < nth; ++k) theta_bar[k] += s * dth[k];
            }
    }

    /* --- 4. Ez, Bz Poisson solves reversed */
    std::vector<double> lE, lB;
    if (adjoint_solve(g, *c, nullptr, Ezb, lE) != ORC_OK) status = ORC_NOCONV;
    if (adjoint_solve(g, *c, nullptr, Bzb, lB) != ORC_OK) status = ORC_NOCONV;
    {   /* f_Ez = -(Dx jx + Dy jy), f_Bz = Dx jy - Dy jx */
        std::vector<double> t(nn);
        for (int i = 0; i < nn; ++i) t[i] = -lE[i];
        add_Dx_T(g, t, jxb);
        add_Dy_T(g, t, jyb);
        add_Dx_T(g, lB, jyb);
        for (int i = 0; i < nn; ++i) t[i] = -lB[i];
        add_Dy_T(g, t, jxb);
    }

    /* --- 3. deposits of j and T reversed, then g_i = 1 + gather(psi) */
    for (int i = 0; i < P; ++i) {
        const CicW& w = W[i];
        double v, dvx, dvy;
        const double q[5] = {vx[i], vy[i], vx[i] * vx[i], vx[i] * vy[i], vy[i] * vy[i]};
        const std::vector<double>* A[5] = {&jxb, &jyb, &txxb, &txyb, &tyyb};
        double qb[5];
        double xbar = 0.0, ybar = 0.0;
        for (int k = 0; k < 5; ++k) {
            interp_grad(g, A[k]->data(), w, v, dvx, dvy);
            qb[k] = wd * v;
            xbar += wd * q[k] * dvx;
            ybar += wd * q[k] * dvy;
        }
        const double vxb = qb[0] + 2.0 * vx[i] * qb[2] + vy[i] * qb[3];
        const double vyb = qb[1] + vx[i] * qb[3] + 2.0 * vy[i] * qb[4];
        pxb[i] += vxb / gi[i];
        pyb[i] += vyb / gi[i];
        const double gb = gib[i] - (vxb * vx[i] + vyb * vy[i]) / gi[i];
        double pv, pvx, pvy;
        interp_grad(g, psi, w, pv, pvx, pvy);
        scatter(g, psib.data(), w, gb);
        xbar += gb * pvx;
        ybar += gb * pvy;
        xb[i] += xbar;
        yb[i] += ybar;
    }

    /* --- 2. psi solve reversed: f_psi = n* - n0 on interior nodes */
    std::vector<double> lpsi;
    if (adjoint_solve(g, *c, nullptr, psib, lpsi) != ORC_OK) status = ORC_NOCONV;
    for (int b = 1; b < g.N; ++b)
        for (int a = 1; a < g.N; ++a) nb[g.id(a, b)] += lpsi[g.id(a, b)];

    /* --- 1. deposit of n* reversed (positions only) */
    for (int i = 0; i < P; ++i) {
        double v, dvx, dvy;
        interp_grad(g, nb.data(), W[i], v, dvx, dvy);
        xb[i] += wd * dvx;
        yb[i] += wd * dvy;
    }
    return status;
}

/* Loss of a run: L = sum_k w_k * probe_k, probe_k = mean over the slices
 * [s0_k, s1_k) of the mean of field f_k over the nodes within r_k of (x0_k, y0_k).
 * probes: [n_probes][6] = field, s0, s1, r, x0, y0 (as doubles).  With
 * theta_bar non-NULL the reverse sweep runs too (all slice states are kept). */
int oracle_run_loss(const oracle_cfg* c, int P, double* x, double* y, double* px, double* py,
                    double* fields, double* xi, double* dxi, int n_slices, int n_probes,
                    const double* probes, const double* weights, double* loss,
                    double* theta_bar) {
    Grid g(c->n_cells, c->half_width);
    const int nn = g.nn();
    struct Rec { std::vector<double> x, y, px, py, F; double xi, dxi; };
    std::vector<Rec> tape;
    double Ls = 0.0;
    int status = ORC_OK;
    auto disc = [&](int k, std::vector<int>& nodes) {
        const double* p = probes + 6 * k;
        nodes.clear();
        for (int b = 0; b <= g.N; ++b)
            for (int a = 0; a <= g.N; ++a) {
                double rx = g.xa(a) - p[4], ry = g.xa(b) - p[5];
                if (rx * rx + ry * ry <= p[3] * p[3]) nodes.push_back(g.id(a, b));
            }
    };
    std::vector<int> nodes;
    for (int j = 0; j < n_slices; ++j) {
        if (theta_bar)
            tape.push_back(Rec{std::vector<double>(x, x + P), std::vector<double>(y, y + P),
                               std::vector<double>(px, px + P), std::vector<double>(py, py + P),
                               {}, *xi, *dxi});
        oracle_info inf;
        int st = oracle_slice_step(c, P, x, y, px, py, nullptr, fields, xi, dxi, &inf, nullptr, nullptr);
        if (st != ORC_OK) status = st;
        if (theta_bar) tape.back().F.assign(fields, fields + 5 * nn);
        for (int k = 0; k < n_probes; ++k) {
            const double* p = probes + 6 * k;
            if (j < (int)p[1] || j >= (int)p[2]) continue;
            disc(k, nodes);
            double s = 0.0;
            for (int i : nodes) s += fields[(int)p[0] * nn + i];
            if (!nodes.empty()) Ls += weights[k] * s / nodes.size() / (p[2] - p[1]);
        }
    }
    *loss = Ls;
    if (!theta_bar || status != ORC_OK) return status;
    std::vector<double> xb(P, 0.0), yb(P, 0.0), pxb(P, 0.0), pyb(P, 0.0), Fb(5 * nn);
    for (int j = n_slices - 1; j >= 0; --j) {
        std::fill(Fb.begin(), Fb.end(), 0.0);
        for (int k = 0; k < n_probes; ++k) {
            const double* p = probes + 6 * k;
            if (j < (int)p[1] || j >= (int)p[2]) continue;
            disc(k, nodes);
            for (int i : nodes) Fb[(int)p[0] * nn + i] += weights[k] / nodes.size() / (p[2] - p[1]);
        }
        const Rec& r = tape[j];
        int st = oracle_slice_adjoint(c, P, r.x.data(), r.y.data(), r.px.data(), r.py.data(),
                                      r.F.data(), r.xi, r.dxi, xb.data(), yb.data(), pxb.data(),
                                      pyb.data(), Fb.data(), theta_bar);
        if (st != ORC_OK) status = st;
    }
    return status;
}

} /* extern "C" */

/* ============================================== non-uniform grids == */
/*
 * Sec. VII.B: the transverse operator on a non-uniform tensor grid x_0 < x_1
 * < ... < x_N (and y_0 < ... < y_N), the general wakefield equation
 * lap u + M u = J with u = 0 on the boundary nodes.
 *
 * Along x at an interior node i, with h- = x_i - x_{i-1}, h+ = x_{i+1} - x_i,
 * ha = h+ + h-, hb = h+ - h-:
 *   Dxx u = 2 (h+ u_{i-1} - ha u_i + h- u_{i+1}) / (h- h+ ha),
 *   dx u  = h-/(ha h+) (u_{i+1} - u_i) + h+/(ha h-) (u_i - u_{i-1})
 * (the second-order three-point derivative of Sec. VII.B).  A Taylor expansion
 * gives Dxx u = u_xx + (hb/3) u_xxx + O(h^2), so u_xx = Dxx u - (hb/3) u_xxx
 * (the printed eq. (34) has the opposite sign; the expansion decides).  The
 * third derivatives follow eq. (36): hb_x u_xxx + hb_y u_yyy =
 * (hb_x dx + hb_y dy)(lap u) - hb_x dx(u_yy) - hb_y dy(u_xx) with lap u =
 * J - M u, u_yy ~ Dyy u and u_xx ~ Dxx u, so the discrete equation is
 *   L u = R J,
 *   L u = Dxx u + Dyy u + (1/3)[hb_x dx(Dyy u) + hb_y dy(Dxx u)]
 *         + (1/3)(hb_x dx + hb_y dy)(M u) + M u,
 *   R J = J + (1/3)(hb_x dx + hb_y dy) J,
 * a nine-point operator (dx(Dyy u) reaches the diagonal neighbours), not
 * symmetric.  On a uniform grid hb = 0 and L is the 5-point Laplacian plus M.
 *
 * Multigrid: the coarse grid keeps every other node, L is rediscretised on it;
 * prolongation is linear interpolation in the coordinates, restriction its
 * transpose weighted by the control volumes V_i = (x_{i+1} - x_{i-1})/2 (the
 * transfers weighted by the neighbouring cells' sizes, Sec. VII.B), in each
 * direction; M is restricted the same way.  Smoothing: Gauss-Seidel in four
 * colours (i mod 2, j mod 2), each node of a colour taking u += (F - L u)/d
 * with d the coefficient of u_ij in its own equation (the nine-point stencil
 * couples no two nodes of one colour); exact on the single interior node of
 * the 2-cell grid.
 */
namespace {

/* The 1-D coefficients of one interior index: Dxx weights (i-1, i, i+1),
 * first-derivative weights (i-1, i, i+1) and hb. */
struct AxisCoef {
    double d2[3], d1[3], hb;
};

AxisCoef axis_coef(const std::vector<double>& X, int i) {
    AxisCoef c;
    const double hm = X[i] - X[i - 1], hp = X[i + 1] - X[i], ha = hm + hp;
    c.d2[0] = 2.0 * hp / (hm * hp * ha);
    c.d2[1] = -2.0 * ha / (hm * hp * ha);
    c.d2[2] = 2.0 * hm / (hm * hp * ha);
    c.d1[0] = -hp / (ha * hm);
    c.d1[1] = -hm / (ha * hp) + hp / (ha * hm);
    c.d1[2] = hm / (ha * hp);
    c.hb = hp - hm;
    return c;
}

struct NuLevel {
    int N;
    std::vector<double> X, Y;
    std::vector<AxisCoef> cx, cy;  /* [N+1], interior entries used */
    std::vector<double> u, F, M;   /* (N+1)^2, node (i, j) at j (N+1) + i */
    int id(int i, int j) const { return j * (N + 1) + i; }
    void build(int n, std::vector<double> x, std::vector<double> y) {
        N = n;
        X = std::move(x);
        Y = std::move(y);
        cx.assign(N + 1, AxisCoef{});
        cy.assign(N + 1, AxisCoef{});
        for (int i = 1; i < N; ++i) {
            cx[i] = axis_coef(X, i);
            cy[i] = axis_coef(Y, i);
        }
        u.assign((size_t)(N + 1) * (N + 1), 0.0);
        F = u;
        M = u;
    }
};

/* Dxx u at (i, j) and Dyy u at (i, j) for i, j interior in that direction;
 * zero on a boundary line (u = 0 there). */
double nu_dxx(const NuLevel& l, const std::vector<double>& u, int i, int j) {
    if (i <= 0 || i >= l.N) return 0.0;
    const AxisCoef& c = l.cx[i];
    return c.d2[0] * u[l.id(i - 1, j)] + c.d2[1] * u[l.id(i, j)] + c.d2[2] * u[l.id(i + 1, j)];
}
double nu_dyy(const NuLevel& l, const std::vector<double>& u, int i, int j) {
    if (j <= 0 || j >= l.N) return 0.0;
    const AxisCoef& c = l.cy[j];
    return c.d2[0] * u[l.id(i, j - 1)] + c.d2[1] * u[l.id(i, j)] + c.d2[2] * u[l.id(i, j + 1)];
}

/* (L u) at the interior node (i, j). */
double nu_apply_at(const NuLevel& l, const std::vector<double>& u, int i, int j) {
    const AxisCoef &a = l.cx[i], &b = l.cy[j];
    auto Mu = [&](int p, int q) { return l.M[l.id(p, q)] * u[l.id(p, q)]; };
    double s = nu_dxx(l, u, i, j) + nu_dyy(l, u, i, j);
    s += (a.hb * (a.d1[0] * nu_dyy(l, u, i - 1, j) + a.d1[1] * nu_dyy(l, u, i, j) +
                  a.d1[2] * nu_dyy(l, u, i + 1, j)) +
          b.hb * (b.d1[0] * nu_dxx(l, u, i, j - 1) + b.d1[1] * nu_dxx(l, u, i, j) +
                  b.d1[2] * nu_dxx(l, u, i, j + 1))) / 3.0;
    s += (a.hb * (a.d1[0] * Mu(i - 1, j) + a.d1[1] * Mu(i, j) + a.d1[2] * Mu(i + 1, j)) +
          b.hb * (b.d1[0] * Mu(i, j - 1) + b.d1[1] * Mu(i, j) + b.d1[2] * Mu(i, j + 1))) / 3.0;
    return s + Mu(i, j);
}

/* The coefficient of u_ij in its own equation. */
double nu_diag(const NuLevel& l, int i, int j) {
    const AxisCoef &a = l.cx[i], &b = l.cy[j];
    const double m = l.M[l.id(i, j)];
    return a.d2[1] + b.d2[1] + (a.hb * a.d1[1] * b.d2[1] + b.hb * b.d1[1] * a.d2[1]) / 3.0 +
           (a.hb * a.d1[1] + b.hb * b.d1[1]) * m / 3.0 + m;
}

void nu_relax(NuLevel& l, int nu) {
    for (int s = 0; s < nu; ++s)
        for (int color = 0; color < 4; ++color) {
            const int pi = color & 1, pj = color >> 1;
#pragma omp parallel for schedule(static)
            for (int j = 1; j < l.N; ++j) {
                if ((j & 1) != pj) continue;
                for (int i = 1; i < l.N; ++i) {
                    if ((i & 1) != pi) continue;
                    const double r = l.F[l.id(i, j)] - nu_apply_at(l, l.u, i, j);
                    l.u[l.id(i, j)] += r / nu_diag(l, i, j);
                }
            }
        }
}

void nu_residual(const NuLevel& l, std::vector<double>& r) {
    r.assign(l.u.size(), 0.0);
#pragma omp parallel for schedule(static)
    for (int j = 1; j < l.N; ++j)
        for (int i = 1; i < l.N; ++i) r[l.id(i, j)] = l.F[l.id(i, j)] - nu_apply_at(l, l.u, i, j);
}

/* 1-D transfer weights between fine node 2I + s (s = -1, 0, 1) and coarse
 * node I: prolongation P (linear interpolation in the coordinate) and the
 * volume-weighted restriction V_f P / V_c. */
double prol_w(const std::vector<double>& X, int I, int s) {
    if (s == 0) return 1.0;
    const int f = 2 * I + s;  /* odd fine node between coarse I and I + s */
    const double lo = X[f - 1], hi = X[f + 1];
    return s > 0 ? (hi - X[f]) / (hi - lo) : (X[f] - lo) / (hi - lo);
}
double rest_w(const std::vector<double>& X, int I, int s) {
    const int f = 2 * I + s;
    const double Vf = 0.5 * (X[f + 1] - X[f - 1]);
    const double Vc = 0.5 * (X[2 * I + 2] - X[2 * I - 2]);
    return prol_w(X, I, s) * Vf / Vc;
}

/* out (coarse, interior nodes) = restriction of the fine node array in. */
void nu_restrict(const NuLevel& f, const std::vector<double>& in, const NuLevel& c,
                 std::vector<double>& out) {
    out.assign((size_t)(c.N + 1) * (c.N + 1), 0.0);
#pragma omp parallel for schedule(static)
    for (int J = 1; J < c.N; ++J)
        for (int I = 1; I < c.N; ++I) {
            double s = 0.0;
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx)
                    s += rest_w(f.X, I, sx) * rest_w(f.Y, J, sy) * in[f.id(2 * I + sx, 2 * J + sy)];
            out[c.id(I, J)] = s;
        }
}

/* fine u += prolongation of the coarse array e (interior fine nodes). */
void nu_prolong_add(const NuLevel& c, const std::vector<double>& e, NuLevel& f) {
#pragma omp parallel for schedule(static)
    for (int j = 1; j < f.N; ++j)
        for (int i = 1; i < f.N; ++i) {
            /* the coarse nodes around fine node i: I = i/2 (and I+1 when i is odd) */
            const int I = i / 2, J = j / 2;
            const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1;
            double v = 0.0;
            for (int q = 0; q < nj; ++q)
                for (int p = 0; p < ni; ++p) {
                    /* weight of coarse node I + p seen from fine node i = 2(I+p) + s */
                    const double wx = (i & 1) ? prol_w(f.X, I + p, p ? -1 : 1) : 1.0;
                    const double wy = (j & 1) ? prol_w(f.Y, J + q, q ? -1 : 1) : 1.0;
                    v += wx * wy * e[c.id(I + p, J + q)];
                }
            f.u[f.id(i, j)] += v;
        }
}

double nu_norm(const NuLevel& l, const std::vector<double>& v) {
    double s = 0.0;
    for (int j = 1; j < l.N; ++j)
        for (int i = 1; i < l.N; ++i) s += v[l.id(i, j)] * v[l.id(i, j)];
    return std::sqrt(s);
}

void nu_vcycle(std::vector<NuLevel>& lv, size_t k, int nu1, int nu2) {
    NuLevel& L = lv[k];
    if (L.N == 2) {
        L.u[L.id(1, 1)] = L.F[L.id(1, 1)] / nu_diag(L, 1, 1);
        return;
    }
    nu_relax(L, nu1);
    std::vector<double> r;
    nu_residual(L, r);
    NuLevel& C = lv[k + 1];
    nu_restrict(L, r, C, C.F);
    std::fill(C.u.begin(), C.u.end(), 0.0);
    nu_vcycle(lv, k + 1, nu1, nu2);
    nu_prolong_add(C, C.u, L);
    nu_relax(L, nu2);
}

std::vector<NuLevel> nu_levels(int N, const double* X, const double* Y, const double* M) {
    std::vector<NuLevel> lv;
    std::vector<double> x(X, X + N + 1), y(Y, Y + N + 1);
    for (int n = N; n >= 2; n /= 2) {
        NuLevel l;
        l.build(n, x, y);
        lv.push_back(std::move(l));
        std::vector<double> xc, yc;
        for (int i = 0; i <= n; i += 2) {
            xc.push_back(x[i]);
            yc.push_back(y[i]);
        }
        x.swap(xc);
        y.swap(yc);
    }
    if (M) {
        for (int j = 1; j < N; ++j)
            for (int i = 1; i < N; ++i) lv[0].M[lv[0].id(i, j)] = M[(size_t)j * (N + 1) + i];
        for (size_t k = 1; k < lv.size(); ++k) nu_restrict(lv[k - 1], lv[k - 1].M, lv[k], lv[k].M);
    }
    return lv;
}

/* R J at the interior nodes (zero on the boundary). */
void nu_rhs(const NuLevel& l, const double* J, std::vector<double>& F) {
    F.assign(l.u.size(), 0.0);
    for (int j = 1; j < l.N; ++j)
        for (int i = 1; i < l.N; ++i) {
            const AxisCoef &a = l.cx[i], &b = l.cy[j];
            auto Jv = [&](int p, int q) { return J[(size_t)q * (l.N + 1) + p]; };
            F[l.id(i, j)] = Jv(i, j) + (a.hb * (a.d1[0] * Jv(i - 1, j) + a.d1[1] * Jv(i, j) +
                                               a.d1[2] * Jv(i + 1, j)) +
                                        b.hb * (b.d1[0] * Jv(i, j - 1) + b.d1[1] * Jv(i, j) +
                                               b.d1[2] * Jv(i, j + 1))) / 3.0;
        }
}

bool increasing(const double* X, int N) {
    for (int i = 0; i < N; ++i)
        if (!(X[i + 1] > X[i])) return false;
    return true;
}

}  // namespace

extern "C" {

/* out [nn] = L u at the interior nodes (zero on the boundary) for the grid
 * X, Y ([N+1] each, increasing) and M ([nn] or NULL: 0). */
int oracle_nu_apply(int N, const double* X, const double* Y, const double* M, const double* u,
                    double* out) {
    if (N < 2 || (N & (N - 1)) || !increasing(X, N) || !increasing(Y, N)) return ORC_INVALID;
    std::vector<NuLevel> lv = nu_levels(N, X, Y, M);
    NuLevel& l = lv[0];
    std::vector<double> uu(u, u + l.u.size());
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i)
            if (i == 0 || j == 0 || i == N || j == N) uu[l.id(i, j)] = 0.0;
    std::fill(out, out + l.u.size(), 0.0);
    for (int j = 1; j < N; ++j)
        for (int i = 1; i < N; ++i) out[l.id(i, j)] = nu_apply_at(l, uu, i, j);
    return ORC_OK;
}

/* out [nn] = R J (interior nodes). */
int oracle_nu_rhs(int N, const double* X, const double* Y, const double* J, double* out) {
    if (N < 2 || (N & (N - 1)) || !increasing(X, N) || !increasing(Y, N)) return ORC_INVALID;
    std::vector<NuLevel> lv = nu_levels(N, X, Y, nullptr);
    std::vector<double> F;
    nu_rhs(lv[0], J, F);
    std::copy(F.begin(), F.end(), out);
    return ORC_OK;
}

/* The transfers between the grid (X, Y) and its coarse grid: mode 0 restricts
 * a fine array in [(N+1)^2] to out [(N/2+1)^2]; mode 1 prolongs a coarse array
 * in to out (fine, interior nodes; boundary 0). */
int oracle_nu_transfer(int N, const double* X, const double* Y, int mode, const double* in,
                       double* out) {
    if (N < 4 || (N & (N - 1)) || !increasing(X, N) || !increasing(Y, N)) return ORC_INVALID;
    std::vector<NuLevel> lv = nu_levels(N, X, Y, nullptr);
    if (mode == 0) {
        std::vector<double> v(in, in + lv[0].u.size()), o;
        nu_restrict(lv[0], v, lv[1], o);
        std::copy(o.begin(), o.end(), out);
    } else {
        std::vector<double> e(in, in + lv[1].u.size());
        nu_prolong_add(lv[1], e, lv[0]);
        std::copy(lv[0].u.begin(), lv[0].u.end(), out);
    }
    return ORC_OK;
}

/* Solve L u = R J (u = 0 on the boundary) from the guess in u, with the stop
 * rule of oracle_mg_solve: ||r|| <= rtol ||F|| + atol sqrt(n), or the
 * rounding floor ||r|| <= 0.35 eps (a ||u|| + ||F||) with a = 2 max |d| (a
 * bound on the operator's size), or stagnation -- a cycle after the second
 * that reduces ||r|| by less than 10% once ||r|| <= 1e-9 ||F|| (||r_0|| when
 * F = 0): the point smoother converges at 0.3 to 0.75 per cycle on cells of
 * aspect ratio up to 3, so slow progress alone is not the floor. */
int oracle_nu_mg_solve(int N, const double* X, const double* Y, const double* M, const double* J,
                       double* u, double rtol, double atol, int max_cycles, int nu1, int nu2,
                       int* cycles, double* rel) {
    if (N < 2 || (N & (N - 1)) || !increasing(X, N) || !increasing(Y, N)) return ORC_INVALID;
    std::vector<NuLevel> lv = nu_levels(N, X, Y, M);
    NuLevel& top = lv[0];
    nu_rhs(top, J, top.F);
    for (int j = 1; j < N; ++j)
        for (int i = 1; i < N; ++i) top.u[top.id(i, j)] = u[(size_t)j * (N + 1) + i];
    double amax = 0.0;
    for (int j = 1; j < N; ++j)
        for (int i = 1; i < N; ++i) amax = std::max(amax, std::fabs(nu_diag(top, i, j)));
    std::vector<double> r;
    nu_residual(top, r);
    const double fn = nu_norm(top, top.F);
    double rn = nu_norm(top, r), rprev = rn;
    const double tol = rtol * (fn > 0 ? fn : rn) + atol * std::sqrt((double)(N - 1) * (N - 1));
    const double scale = fn > 0 ? fn : rn;
    const double floor_be = 0.35 * std::numeric_limits<double>::epsilon();
    bool done = rn <= tol;
    int cyc = 0;
    while (!done && cyc < max_cycles) {
        nu_vcycle(lv, 0, nu1, nu2);
        ++cyc;
        nu_residual(top, r);
        rprev = rn;
        rn = nu_norm(top, r);
        const double un = nu_norm(top, top.u);
        done = rn <= tol || rn <= floor_be * (2.0 * amax * un + fn) ||
               (cyc >= 2 && rn > 0.9 * rprev && rn <= 1e-9 * scale);
    }
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) u[(size_t)j * (N + 1) + i] = top.u[top.id(i, j)];
    if (cycles) *cycles = cyc;
    if (rel) *rel = fn > 0 ? rn / fn : rn;
    return (done && std::isfinite(rn)) ? ORC_OK : ORC_NOCONV;
}

}  /* extern "C" */
