// Multigrid on a non-uniform transverse grid (Sec. VII.B): lap u + M u = J on
// a tensor grid x_0 < ... < x_N, y_0 < ... < y_N with u = 0 on the boundary.
//
// Along x at an interior node i (h- = x_i - x_{i-1}, h+ = x_{i+1} - x_i,
// ha = h+ + h-, hb = h+ - h-): Dxx u = 2 (h+ u_{i-1} - ha u_i + h- u_{i+1}) /
// (h- h+ ha) and the three-point derivative dx u = h-/(ha h+) (u_{i+1} - u_i)
// + h+/(ha h-) (u_i - u_{i-1}).  Since Dxx u = u_xx + (hb/3) u_xxx + O(h^2),
// the third-order terms are removed with eq. (36), which gives the discrete
// equation L u = R J with
//   L u = Dxx u + Dyy u + (1/3)[hb_x dx(Dyy u) + hb_y dy(Dxx u)]
//         + (1/3)(hb_x dx + hb_y dy)(M u) + M u,
//   R J = J + (1/3)(hb_x dx + hb_y dy) J,
// a nine-point, non-symmetric operator (the 5-point Laplacian plus M on a
// uniform grid).
//
// The solver: V-cycles smoothing by alternating zebra line relaxation on the
// levels above 64^2 (x-lines of odd then even rows, y-lines of odd then even
// columns, once before and once after the coarse correction: cells of aspect
// ratio up to 3 defeat point smoothers) and by Gauss-Seidel in four colours
// (i mod 2, j mod 2; the nine-point stencil couples no two nodes of one
// colour; nu_pre / nu_post sweeps) on the levels <= 64^2, u += (R J - L u) / d
// with d the coefficient of u_ij in its own equation; coarse grids keep every
// other node and rediscretise L; the
// prolongation interpolates linearly in the coordinates and the restriction
// is its transpose weighted by the control volumes (x_{i+1} - x_{i-1})/2 per
// direction, for the residual and for M.  Levels of N <= 64 run in one
// workgroup in LDS down to the single interior node of the 2-cell grid.  The
// stop rule is the context's (mg_rtol, mg_atol, the rounding floor with
// 2 max |d| as the size of L), except that a cycle counts as stagnating only
// when it reduces ||r|| by less than 10% (this smoother converges at 0.3 to
// 0.75 per cycle on cells of aspect ratio up to 3) once ||r|| <= 1e-9 ||R J||.
//
// Per-level 1-D tables (host-made, one copy per call): for every index the
// Dxx weights, the dx weights and hb (7 doubles); for the restriction to the
// next level, three weights per coarse index; for the prolongation from it,
// two per fine index.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "wq_common.h"

namespace wq {
namespace {

constexpr int kNuCoarse = 64;
static_assert(kCoarseMax <= kNuCoarse, "the coarse workgroup's LDS holds levels up to 64 cells");
constexpr int kNuThreads = 1024;
constexpr int kNuLdsNodes = 65 * 65 + 33 * 33 + 17 * 17 + 9 * 9 + 5 * 5 + 3 * 3;
constexpr int kNormT = 256;

// the tables of one level: cx, cy [7 (N+1)]; rx, ry [3 (N/2+1)] (restriction to
// the next level); px, py [2 (N+1)] (prolongation from the next level)
struct NuTabs {
    const double *cx, *cy, *rx, *ry, *px, *py;
};

template <class A>
__device__ __forceinline__ double nu_Lu(const A& u, const A& M, int i, int j, const double* cx,
                                        const double* cy) {
    const double* a = cx + 7 * i;
    const double* b = cy + 7 * j;
    auto dyy = [&](int p) { return b[0] * u(p, j - 1) + b[1] * u(p, j) + b[2] * u(p, j + 1); };
    auto dxx = [&](int q) { return a[0] * u(i - 1, q) + a[1] * u(i, q) + a[2] * u(i + 1, q); };
    auto mu = [&](int p, int q) { return M(p, q) * u(p, q); };
    double s = dxx(j) + dyy(i);
    s += (a[6] * (a[3] * dyy(i - 1) + a[4] * dyy(i) + a[5] * dyy(i + 1)) +
          b[6] * (b[3] * dxx(j - 1) + b[4] * dxx(j) + b[5] * dxx(j + 1))) / 3.0;
    s += (a[6] * (a[3] * mu(i - 1, j) + a[4] * mu(i, j) + a[5] * mu(i + 1, j)) +
          b[6] * (b[3] * mu(i, j - 1) + b[4] * mu(i, j) + b[5] * mu(i, j + 1))) / 3.0;
    return s + mu(i, j);
}

__device__ __forceinline__ double nu_diag(double m, int i, int j, const double* cx, const double* cy) {
    const double* a = cx + 7 * i;
    const double* b = cy + 7 * j;
    return a[1] + b[1] + (a[6] * a[4] * b[1] + b[6] * b[4] * a[1]) / 3.0 +
           (a[6] * a[4] + b[6] * b[4]) * m / 3.0 + m;
}

// a pitched node array (global memory or LDS)
struct Arr {
    double* p;
    int pitch;
    __device__ __forceinline__ double& operator()(int i, int j) const { return p[(size_t)j * pitch + i]; }
};

// Dense [N+1][N+1] to the padded layout, boundary nodes included (J's
// boundary values enter R J at the nodes next to it).
__global__ void k_nu_copy_in(int N, int pitch, const double* __restrict__ src, double* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i > N) return;
    dst[(size_t)j * pitch + i] = src[(size_t)j * (N + 1) + i];
}

// R J on the interior nodes (boundary 0) and u = 0 on the boundary.
__global__ void k_nu_rhs(int N, int pitch, const double* __restrict__ J, const double* cx,
                         const double* cy, double* __restrict__ F, double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i > N) return;
    const size_t g = (size_t)j * pitch + i;
    if (i == 0 || j == 0 || i == N || j == N) {
        F[g] = 0.0;
        u[g] = 0.0;
        return;
    }
    const double* a = cx + 7 * i;
    const double* b = cy + 7 * j;
    F[g] = J[g] + (a[6] * (a[3] * J[g - 1] + a[4] * J[g] + a[5] * J[g + 1]) +
                   b[6] * (b[3] * J[g - pitch] + b[4] * J[g] + b[5] * J[g + pitch])) / 3.0;
}

// One colour (pi, pj) of the four-colour Gauss-Seidel sweep.
__global__ void k_nu_smooth(int N, int pitch, int pi, int pj, double* u, const double* __restrict__ F,
                            double* M, const double* cx, const double* cy) {
    const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + pi;
    const int j = 2 * blockIdx.y + pj;
    if (i < 1 || i > N - 1 || j < 1 || j > N - 1) return;
    const Arr U{u, pitch}, Mm{M, pitch};
    const size_t g = (size_t)j * pitch + i;
    const double r = F[g] - nu_Lu(U, Mm, i, j, cx, cy);
    u[g] += r / nu_diag(M[g], i, j, cx, cy);
}

// Line relaxation: the unknowns of one grid line solved together with the
// neighbouring lines held fixed.  DIR 0: the x-line of row `line` (unknowns
// u(1..n-1, line)); DIR 1: the y-line of column `line`.  Holding the other
// lines, L restricted to the line is tridiagonal: for an x-line the
// coefficients of u(i-1, j), u(i, j), u(i+1, j) are
//   Dxx weights x (1 + hb_y dy_0/3) + (hb_x dx_k/3)(Dyy_0 + M(i+k-1, j)) and,
//   on the diagonal, the coefficient d of the point smoother
// (dy_0, Dyy_0: the y-stencils' central weights), mirrored for a y-line.  The
// line takes u += T^-1 (R J - L u), T solved by parallel cyclic reduction in
// LDS.  Lines of one parity do not couple (the stencil reaches one line
// over), so each launch relaxes every other line.
constexpr int kLineThreads = 512;
constexpr int kLineMax = 4095;
constexpr int kLinePer = (kLineMax + kLineThreads - 1) / kLineThreads;

template <int DIR>
__global__ __launch_bounds__(kLineThreads) void k_nu_line(int n, int pitch, int par, double* u,
                                                          const double* __restrict__ F, double* M,
                                                          const double* cx, const double* cy) {
    extern __shared__ double sh[];
    const int m = n - 1;
    double* A = sh;
    double* B = sh + m;
    double* C = sh + 2 * m;
    double* D = sh + 3 * m;
    const int line = 2 * blockIdx.x + par;
    if (line < 1 || line > n - 1) return;  // the whole workgroup
    const Arr U{u, pitch}, Mm{M, pitch};
    for (int t = threadIdx.x; t < m; t += kLineThreads) {
        const int i = DIR == 0 ? t + 1 : line, j = DIR == 0 ? line : t + 1;
        const double* a = cx + 7 * i;
        const double* b = cy + 7 * j;
        const double r = F[(size_t)j * pitch + i] - nu_Lu(U, Mm, i, j, cx, cy);
        double sub, sup;
        if (DIR == 0) {
            const double fy = 1.0 + b[6] * b[4] / 3.0, gx = a[6] / 3.0;
            sub = a[0] * fy + gx * a[3] * (b[1] + Mm(i - 1, j));
            sup = a[2] * fy + gx * a[5] * (b[1] + Mm(i + 1, j));
        } else {
            const double fx = 1.0 + a[6] * a[4] / 3.0, gy = b[6] / 3.0;
            sub = b[0] * fx + gy * b[3] * (a[1] + Mm(i, j - 1));
            sup = b[2] * fx + gy * b[5] * (a[1] + Mm(i, j + 1));
        }
        A[t] = t == 0 ? 0.0 : sub;
        C[t] = t == m - 1 ? 0.0 : sup;
        B[t] = nu_diag(Mm(i, j), i, j, cx, cy);
        D[t] = r;
    }
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        double na[kLinePer], nb[kLinePer], nc[kLinePer], nd[kLinePer];
#pragma unroll
        for (int q = 0; q < kLinePer; ++q) {
            const int t = threadIdx.x + q * kLineThreads;
            if (t >= m) break;
            double xa = 0.0, xc = 0.0, xb = B[t], xd = D[t];
            if (t - s >= 0) {
                const double al = -A[t] / B[t - s];
                xa = al * A[t - s];
                xb += al * C[t - s];
                xd += al * D[t - s];
            }
            if (t + s < m) {
                const double ga = -C[t] / B[t + s];
                xc = ga * C[t + s];
                xb += ga * A[t + s];
                xd += ga * D[t + s];
            }
            na[q] = xa;
            nb[q] = xb;
            nc[q] = xc;
            nd[q] = xd;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kLinePer; ++q) {
            const int t = threadIdx.x + q * kLineThreads;
            if (t >= m) break;
            A[t] = na[q];
            B[t] = nb[q];
            C[t] = nc[q];
            D[t] = nd[q];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < m; t += kLineThreads) {
        const int i = DIR == 0 ? t + 1 : line, j = DIR == 0 ? line : t + 1;
        u[(size_t)j * pitch + i] += D[t] / B[t];
    }
}

// Coarse right-hand side = weighted restriction of the fine residual; the
// coarse correction starts at zero.
__global__ void k_nu_restrict(int nc, int pf, double* uf, const double* __restrict__ Ff, double* Mf,
                              const double* cx, const double* cy, const double* rx,
                              const double* ry, int pc, double* __restrict__ Fc,
                              double* __restrict__ uc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
    if (I > nc) return;
    const size_t ic = (size_t)J * pc + I;
    uc[ic] = 0.0;
    double s = 0.0;
    if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1) {
        const Arr U{uf, pf}, Mm{Mf, pf};
        for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx) {
                const int i = 2 * I + sx, j = 2 * J + sy;
                const double r = Ff[(size_t)j * pf + i] - nu_Lu(U, Mm, i, j, cx, cy);
                s += rx[3 * I + sx + 1] * ry[3 * J + sy + 1] * r;
            }
    }
    Fc[ic] = s;
}

// The same weighted restriction of a node array (M), interior coarse nodes.
__global__ void k_nu_restrict_plain(int nc, int pf, const double* __restrict__ vf, const double* rx,
                                    const double* ry, int pc, double* __restrict__ vc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
    if (I > nc) return;
    double s = 0.0;
    if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1)
        for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx)
                s += rx[3 * I + sx + 1] * ry[3 * J + sy + 1] * vf[(size_t)(2 * J + sy) * pf + 2 * I + sx];
    vc[(size_t)J * pc + I] = s;
}

// u_fine += prolongation of the coarse correction (interior fine nodes): at
// an odd fine index the weights of coarse I = i/2 and I + 1 are px[2i], px[2i+1].
__device__ __forceinline__ double prolong_at(const Arr& e, int i, int j, const double* px,
                                             const double* py) {
    const int I = i >> 1, J = j >> 1;
    const bool ox = i & 1, oy = j & 1;
    const double wx0 = ox ? px[2 * i] : 1.0, wx1 = ox ? px[2 * i + 1] : 0.0;
    const double wy0 = oy ? py[2 * j] : 1.0, wy1 = oy ? py[2 * j + 1] : 0.0;
    double v = wy0 * (wx0 * e(I, J) + (ox ? wx1 * e(I + 1, J) : 0.0));
    if (oy) v += wy1 * (wx0 * e(I, J + 1) + (ox ? wx1 * e(I + 1, J + 1) : 0.0));
    return v;
}

__global__ void k_nu_prolong(int nf, int pf, double* __restrict__ uf, int pc, double* uc,
                             const double* px, const double* py) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i < 1 || i > nf - 1 || j < 1 || j > nf - 1) return;
    uf[(size_t)j * pf + i] += prolong_at(Arr{uc, pc}, i, j, px, py);
}

// The V-cycle from level n0 (<= kNuCoarse) down to 2 cells in one workgroup,
// in LDS: u (the initial iterate), F and M of level n0 come from global memory
// (pitch), u goes back.  tabs[q] are the tables of chain level q.
struct NuChain {
    NuTabs t[8];
};
__global__ __launch_bounds__(kNuThreads) void k_nu_coarse(int n0, int pitch, int nu1, int nu2,
                                                          double* ug, const double* __restrict__ Fg,
                                                          const double* __restrict__ Mg, NuChain ch) {
    __shared__ double U[kNuLdsNodes], F[kNuLdsNodes], M[kNuLdsNodes];
    int off[8], nq[8];
    int Q = 0;
    {
        int o = 0;
        for (int n = n0; n >= 2; n >>= 1, ++Q) {
            off[Q] = o;
            nq[Q] = n;
            o += (n + 1) * (n + 1);
        }
    }
    const int tid = threadIdx.x;
    {
        const int m = n0 + 1;
        for (int k = tid; k < m * m; k += kNuThreads) {
            const size_t g = (size_t)(k / m) * pitch + k % m;
            U[k] = ug[g];
            F[k] = Fg[g];
            M[k] = Mg[g];
        }
    }
    __syncthreads();
    for (int q = 1; q < Q; ++q) {  // M of the coarser levels
        const int n = nq[q], m = n + 1, mf = nq[q - 1] + 1;
        const double *rx = ch.t[q - 1].rx, *ry = ch.t[q - 1].ry;
        for (int k = tid; k < m * m; k += kNuThreads) {
            const int I = k % m, J = k / m;
            double s = 0.0;
            if (I >= 1 && J >= 1 && I <= n - 1 && J <= n - 1)
                for (int sy = -1; sy <= 1; ++sy)
                    for (int sx = -1; sx <= 1; ++sx)
                        s += rx[3 * I + sx + 1] * ry[3 * J + sy + 1] * M[off[q - 1] + (2 * J + sy) * mf + 2 * I + sx];
            M[off[q] + k] = s;
        }
        __syncthreads();
    }
    auto smooth = [&](int q, int nu) {
        const int n = nq[q], m = n + 1;
        const Arr Uq{U + off[q], m}, Mq{M + off[q], m};
        const double *cx = ch.t[q].cx, *cy = ch.t[q].cy;
        for (int s = 0; s < nu; ++s)
            for (int color = 0; color < 4; ++color) {
                const int pi = color & 1, pj = color >> 1;
                const int h = n / 2;  // nodes of one parity per line: <= h
                for (int k = tid; k < h * h; k += kNuThreads) {
                    const int i = 2 * (k % h) + pi, j = 2 * (k / h) + pj;
                    if (i < 1 || j < 1 || i > n - 1 || j > n - 1) continue;
                    const double r = F[off[q] + j * m + i] - nu_Lu(Uq, Mq, i, j, cx, cy);
                    U[off[q] + j * m + i] += r / nu_diag(M[off[q] + j * m + i], i, j, cx, cy);
                }
                __syncthreads();
            }
    };
    for (int q = 0; q + 1 < Q; ++q) {
        smooth(q, nu1);
        const int nf = nq[q], mf = nf + 1, n = nq[q + 1], m = n + 1;
        const Arr Uq{U + off[q], mf}, Mq{M + off[q], mf};
        const double *cx = ch.t[q].cx, *cy = ch.t[q].cy, *rx = ch.t[q].rx, *ry = ch.t[q].ry;
        for (int k = tid; k < m * m; k += kNuThreads) {
            const int I = k % m, J = k / m;
            double s = 0.0;
            if (I >= 1 && J >= 1 && I <= n - 1 && J <= n - 1)
                for (int sy = -1; sy <= 1; ++sy)
                    for (int sx = -1; sx <= 1; ++sx) {
                        const int i = 2 * I + sx, j = 2 * J + sy;
                        const double r = F[off[q] + j * mf + i] - nu_Lu(Uq, Mq, i, j, cx, cy);
                        s += rx[3 * I + sx + 1] * ry[3 * J + sy + 1] * r;
                    }
            F[off[q + 1] + k] = s;
            U[off[q + 1] + k] = 0.0;
        }
        __syncthreads();
    }
    if (tid == 0) {  // the 2-cell level: one interior node (1, 1)
        const int k = off[Q - 1] + 4;
        U[k] = F[k] / nu_diag(M[k], 1, 1, ch.t[Q - 1].cx, ch.t[Q - 1].cy);
    }
    __syncthreads();
    for (int q = Q - 2; q >= 0; --q) {
        const int nf = nq[q], mf = nf + 1;
        const Arr E{U + off[q + 1], nq[q + 1] + 1};
        for (int k = tid; k < mf * mf; k += kNuThreads) {
            const int i = k % mf, j = k / mf;
            if (i < 1 || j < 1 || i > nf - 1 || j > nf - 1) continue;
            U[off[q] + k] += prolong_at(E, i, j, ch.t[q].px, ch.t[q].py);
        }
        __syncthreads();
        smooth(q, nu2);
    }
    {
        const int m = n0 + 1;
        for (int k = tid; k < m * m; k += kNuThreads) ug[(size_t)(k / m) * pitch + k % m] = U[k];
    }
}

// Per interior row: sum of F^2 (mode 0) or of r^2 (mode 1), sum of u^2, max |d|.
__global__ __launch_bounds__(kNormT) void k_nu_norm(int N, int pitch, int mode, double* u,
                                                    const double* __restrict__ F, double* M,
                                                    const double* cx, const double* cy,
                                                    double* __restrict__ part) {
    __shared__ double red[3][kNormT];
    const int j = blockIdx.x + 1;
    const Arr U{u, pitch}, Mm{M, pitch};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = 1 + threadIdx.x; i <= N - 1; i += kNormT) {
        const size_t g = (size_t)j * pitch + i;
        const double v = mode == 0 ? F[g] : F[g] - nu_Lu(U, Mm, i, j, cx, cy);
        s0 += v * v;
        s1 += u[g] * u[g];
        s2 = fmax(s2, fabs(nu_diag(M[g], i, j, cx, cy)));
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = kNormT / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) part[(size_t)3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kNormT) void k_nu_norm_fin(int rows, const double* __restrict__ part,
                                                        double* __restrict__ out) {
    __shared__ double red[3][kNormT];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int r = threadIdx.x; r < rows; r += kNormT) {
        s0 += part[3 * (size_t)r];
        s1 += part[3 * (size_t)r + 1];
        s2 = fmax(s2, part[3 * (size_t)r + 2]);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = kNormT / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
            red[2][threadIdx.x] = fmax(red[2][threadIdx.x], red[2][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

dim3 rows(int n, int t) { return dim3((n + 1 + t - 1) / t, n + 1); }

// The tables of every level into host vectors (offsets per level and kind).
struct HostTabs {
    std::vector<double> buf;
    std::vector<size_t> cx, cy, rx, ry, px, py;
};

void axis_tabs(const std::vector<double>& X, std::vector<double>& c) {
    const int N = (int)X.size() - 1;
    c.assign(7 * (size_t)(N + 1), 0.0);
    for (int i = 1; i < N; ++i) {
        const double hm = X[i] - X[i - 1], hp = X[i + 1] - X[i], ha = hm + hp;
        double* t = &c[7 * (size_t)i];
        t[0] = 2.0 * hp / (hm * hp * ha);
        t[1] = -2.0 * ha / (hm * hp * ha);
        t[2] = 2.0 * hm / (hm * hp * ha);
        t[3] = -hp / (ha * hm);
        t[4] = -hm / (ha * hp) + hp / (ha * hm);
        t[5] = hm / (ha * hp);
        t[6] = hp - hm;
    }
}

// restriction weights of coarse index I (fine 2I - 1, 2I, 2I + 1) and
// prolongation weights of fine index i (coarse i/2 and i/2 + 1)
void transfer_tabs(const std::vector<double>& X, std::vector<double>& r, std::vector<double>& p) {
    const int N = (int)X.size() - 1, Nc = N / 2;
    auto pw = [&](int f, bool right) {  // odd fine f: weight of its left / right coarse node
        const double lo = X[f - 1], hi = X[f + 1];
        return right ? (X[f] - lo) / (hi - lo) : (hi - X[f]) / (hi - lo);
    };
    r.assign(3 * (size_t)(Nc + 1), 0.0);
    for (int I = 1; I < Nc; ++I) {
        const double Vc = 0.5 * (X[2 * I + 2] - X[2 * I - 2]);
        for (int s = -1; s <= 1; ++s) {
            const int f = 2 * I + s;
            const double Vf = 0.5 * (X[f + 1] - X[f - 1]);
            const double P = s == 0 ? 1.0 : pw(f, s < 0);
            r[3 * (size_t)I + s + 1] = P * Vf / Vc;
        }
    }
    p.assign(2 * (size_t)(N + 1), 0.0);
    for (int f = 1; f < N; f += 2) {
        p[2 * (size_t)f] = pw(f, false);
        p[2 * (size_t)f + 1] = pw(f, true);
    }
}

}  // namespace

size_t nu_table_doubles(int N) {
    size_t s = 0;
    for (int n = N; n >= 2; n /= 2) s += 2 * (7 * (size_t)(n + 1) + 3 * (size_t)(n / 2 + 1) + 2 * (size_t)(n + 1));
    return s;
}

}  // namespace wq

using namespace wq;

extern "C" wandqs_status wandqs_nu_mg_solve(wandqs_ctx* c, const double* h_x, const double* h_y,
                                            const double* d_M, const double* d_J, double* d_u,
                                            int32_t* h_cycles, double* h_rel) {
    if (!c || !h_x || !h_y || !d_J || !d_u) return WANDQS_E_INVALID;
    const int N = c->N;
    for (int i = 0; i < N; ++i)
        if (!(h_x[i + 1] > h_x[i]) || !(h_y[i + 1] > h_y[i])) {
            c->err = "grid coordinates must increase";
            return WANDQS_E_INVALID;
        }
    hipStream_t s = c->stream;
    // tables of every level
    const int nlev = c->nlev;
    std::vector<std::vector<double>> X(nlev), Y(nlev);
    X[0].assign(h_x, h_x + N + 1);
    Y[0].assign(h_y, h_y + N + 1);
    for (int l = 1; l < nlev; ++l)
        for (size_t i = 0; i < X[l - 1].size(); i += 2) {
            X[l].push_back(X[l - 1][i]);
            Y[l].push_back(Y[l - 1][i]);
        }
    std::vector<double> host;
    host.reserve(nu_table_doubles(N));
    std::vector<NuTabs> tabs(nlev);
    std::vector<size_t> offs(nlev * 6);
    for (int l = 0; l < nlev; ++l) {
        std::vector<double> cx, cy, rx, ry, px, py;
        axis_tabs(X[l], cx);
        axis_tabs(Y[l], cy);
        if (l + 1 < nlev) {
            transfer_tabs(X[l], rx, px);
            transfer_tabs(Y[l], ry, py);
        }
        const std::vector<double>* parts[6] = {&cx, &cy, &rx, &ry, &px, &py};
        for (int k = 0; k < 6; ++k) {
            offs[6 * l + k] = host.size();
            host.insert(host.end(), parts[k]->begin(), parts[k]->end());
        }
    }
    if (host.size() > nu_table_doubles(N)) {
        c->err = "internal: non-uniform tables overflow";
        return WANDQS_E_INVALID;
    }
    for (int l = 0; l < nlev; ++l) {
        const double* b = c->nu_tab;
        tabs[l] = NuTabs{b + offs[6 * l], b + offs[6 * l + 1], b + offs[6 * l + 2],
                         b + offs[6 * l + 3], b + offs[6 * l + 4], b + offs[6 * l + 5]};
    }
    WQ_HIP(hipMemcpyAsync(c->nu_tab, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice, s));
    // level arrays: u, F, M (level 0: the field, f and k2 scratch; J in the
    // j_z scratch, which every slice rewrites whole: the multigrid's own
    // scratch arrays keep zero boundary values that its passes rely on)
    const int lc = c->lc;
    auto U = [&](int l) { return l == 0 ? c->fields[0] : c->lev[l].u[0]; };
    auto Fa = [&](int l) { return c->lev[l].f[0]; };
    auto Ma = [&](int l) { return c->lev[l].k2; };
    Level& L0 = c->lev[0];
    double* Jp = c->jz;
    wandqs_status st;
    {
        {
            ProfScope ps(c, "k_nu_copy_in", (double)(N + 1) * (N + 1) * 16.0);
            WQ_KLAUNCH(ps, k_nu_copy_in, rows(N, 128), dim3(128), 0, s, N, L0.pitch, d_J, Jp);
        }
        WQ_LAUNCH_CHECK();
        double* du[1] = {U(0)};
        if ((st = unpack_fields(c, d_u, 1, du)) != WANDQS_OK) return st;
        double* dm[1] = {Ma(0)};
        if (d_M) {
            if ((st = unpack_fields(c, d_M, 1, dm)) != WANDQS_OK) return st;
        } else if ((st = fill_f64(c, Ma(0), (size_t)(N + 1) * L0.pitch, 0.0)) != WANDQS_OK) {
            return st;
        }
    }
    c->tape_ok = false;  // the level arrays are the slice's scratch
    {
        ProfScope ps(c, "k_nu_rhs", (double)(N + 1) * (N + 1) * 24.0);
        WQ_KLAUNCH(ps, k_nu_rhs, rows(N, 128), dim3(128), 0, s, N, L0.pitch, Jp, tabs[0].cx,
                   tabs[0].cy, Fa(0), U(0));
    }
    for (int l = 1; l <= lc; ++l) {
        const Level &Fl = c->lev[l - 1], &Cl = c->lev[l];
        ProfScope ps(c, "k_nu_restrict_plain", (double)(Fl.N + 1) * (Fl.N + 1) * 8.0 + (double)(Cl.N + 1) * (Cl.N + 1) * 8.0);
        WQ_KLAUNCH(ps, k_nu_restrict_plain, rows(Cl.N, 128), dim3(128), 0, s, Cl.N, Fl.pitch, Ma(l - 1),
                   tabs[l - 1].rx, tabs[l - 1].ry, Cl.pitch, Ma(l));
    }
    NuChain ch{};
    for (int q = 0; lc + q < nlev && q < 8; ++q) ch.t[q] = tabs[lc + q];
    const int nu1 = c->cfg.nu_pre, nu2 = c->cfg.nu_post;
    double* hn = c->h_pin + kMaxSlots * kNormVec + 16;  // [F^2, u^2, max d, -, r^2, u^2, max d]
    auto norms = [&](int mode, double* out) -> wandqs_status {
        {
            ProfScope ps(c, "k_nu_norm", (double)(N + 1) * (N + 1) * (mode ? 32.0 : 24.0));
            WQ_KLAUNCH(ps, k_nu_norm, dim3(N - 1), dim3(kNormT), 0, s, N, L0.pitch, mode, U(0), Fa(0),
                       Ma(0), tabs[0].cx, tabs[0].cy, c->nu_part);
        }
        {
            ProfScope ps(c, "k_nu_norm_fin", 24.0 * (N - 1));
            WQ_KLAUNCH(ps, k_nu_norm_fin, dim3(1), dim3(kNormT), 0, s, N - 1, c->nu_part, c->nu_red);
        }
        WQ_LAUNCH_CHECK();
        WQ_HIP(hipMemcpyAsync(out, c->nu_red, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        return WANDQS_OK;
    };
    // one smoothing step on a tile level: x-lines of odd and even rows, then
    // y-lines of odd and even columns (alternating zebra line relaxation)
    auto line_step = [&](int l) {
        const Level& Fl = c->lev[l];
        const size_t lds = 4 * sizeof(double) * (size_t)(Fl.N - 1);
        for (int dir = 0; dir < 2; ++dir)
            for (int par = 1; par >= 0; --par) {
                ProfScope ps(c, dir ? "k_nu_line<1>" : "k_nu_line<0>", (double)(Fl.N + 1) * (Fl.N + 1) * 24.0);
                if (dir == 0)
                    WQ_KLAUNCH(ps, k_nu_line<0>, dim3(Fl.N / 2), dim3(kLineThreads), lds, s, Fl.N, Fl.pitch,
                               par, U(l), Fa(l), Ma(l), tabs[l].cx, tabs[l].cy);
                else
                    WQ_KLAUNCH(ps, k_nu_line<1>, dim3(Fl.N / 2), dim3(kLineThreads), lds, s, Fl.N, Fl.pitch,
                               par, U(l), Fa(l), Ma(l), tabs[l].cx, tabs[l].cy);
            }
    };
    auto vcycle = [&]() -> wandqs_status {
        for (int l = 0; l < lc; ++l) {
            const Level &Fl = c->lev[l], &Cl = c->lev[l + 1];
            line_step(l);  // one alternating line step smooths like several point sweeps
            ProfScope ps(c, "k_nu_restrict", (double)(Fl.N + 1) * (Fl.N + 1) * 24.0 + (double)(Cl.N + 1) * (Cl.N + 1) * 16.0);
            WQ_KLAUNCH(ps, k_nu_restrict, rows(Cl.N, 128), dim3(128), 0, s, Cl.N, Fl.pitch, U(l), Fa(l),
                       Ma(l), tabs[l].cx, tabs[l].cy, tabs[l].rx, tabs[l].ry, Cl.pitch, Fa(l + 1), U(l + 1));
        }
        {
            const Level& Cl = c->lev[lc];
            ProfScope ps(c, "k_nu_coarse", (double)(Cl.N + 1) * (Cl.N + 1) * 32.0);
            WQ_KLAUNCH(ps, k_nu_coarse, dim3(1), dim3(kNuThreads), 0, s, Cl.N, Cl.pitch, nu1, nu2, U(lc),
                       Fa(lc), Ma(lc), ch);
        }
        for (int l = lc - 1; l >= 0; --l) {
            const Level &Fl = c->lev[l], &Cl = c->lev[l + 1];
            {
                ProfScope ps(c, "k_nu_prolong", (double)(Fl.N + 1) * (Fl.N + 1) * 16.0 + (double)(Cl.N + 1) * (Cl.N + 1) * 8.0);
                WQ_KLAUNCH(ps, k_nu_prolong, rows(Fl.N, 128), dim3(128), 0, s, Fl.N, Fl.pitch, U(l), Cl.pitch,
                           U(l + 1), tabs[l].px, tabs[l].py);
            }
            line_step(l);
        }
        WQ_LAUNCH_CHECK();
        return WANDQS_OK;
    };
    {
        // line solves of up to 4095 unknowns keep four arrays of them in LDS
        const int bytes = (int)(4 * sizeof(double) * (size_t)(N - 1));
        WQ_HIP(hipFuncSetAttribute((const void*)k_nu_line<0>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
        WQ_HIP(hipFuncSetAttribute((const void*)k_nu_line<1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    }
    if ((st = norms(0, hn)) != WANDQS_OK || (st = norms(1, hn + 4)) != WANDQS_OK) return st;
    WQ_HIP(hipStreamSynchronize(s));
    const double fn = std::sqrt(hn[0]), amax = hn[2];
    double rn = std::sqrt(hn[4]), rprev = rn;
    const double tol = c->cfg.mg_rtol * (fn > 0 ? fn : rn) + c->cfg.mg_atol * std::sqrt((double)(N - 1) * (N - 1));
    const double scale = fn > 0 ? fn : rn;
    const double floor_be = kFloorBE * std::numeric_limits<double>::epsilon();
    bool done = rn <= tol;
    int cyc = 0;
    while (!done && cyc < c->cfg.mg_max_cycles) {
        if ((st = vcycle()) != WANDQS_OK) return st;
        ++cyc;
        if ((st = norms(1, hn + 4)) != WANDQS_OK) return st;
        WQ_HIP(hipStreamSynchronize(s));
        rprev = rn;
        rn = std::sqrt(hn[4]);
        const double un = std::sqrt(hn[5]);
        done = rn <= tol || rn <= floor_be * (2.0 * amax * un + fn) ||
               (cyc >= 2 && rn > 0.9 * rprev && rn <= 1e-9 * scale);
    }
    if ((st = pack_fields(c, c->fields, 1, d_u)) != WANDQS_OK) return st;
    WQ_HIP(hipStreamSynchronize(s));
    if (h_cycles) *h_cycles = cyc;
    if (h_rel) *h_rel = fn > 0 ? rn / fn : rn;
    if (!(done && std::isfinite(rn))) {
        c->err = "non-uniform multigrid did not converge";
        return WANDQS_E_NOCONV;
    }
    return WANDQS_OK;
}
