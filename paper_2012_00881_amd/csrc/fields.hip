// Node-array kernels of one slice: the right-hand sides of the Ez and Bz
// Poisson equations (WAND-PIC Sec. III.B eqs. (13)-(14)), the longitudinal
// current with the frozen driver, the B_perp Helmholtz system (eqs. (18)-(19),
// rows 4-5 of eq. (30) with the laser envelope absent), probes and layout
// conversion between the padded internal arrays and the dense interface arrays.
#include "wq_common.h"

namespace wq {
namespace {

// f_Ez = -(D_x jx + D_y jy), f_Bz = D_x jy - D_y jx on the interior nodes.
__global__ void k_rhs_EB(int N, double h, int pitch, const double* __restrict__ jx,
                         const double* __restrict__ jy, double* __restrict__ fE,
                         double* __restrict__ fB) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t g = (size_t)b * pitch + a;
    double e = 0.0, m = 0.0;
    if (a >= 1 && b >= 1 && a <= N - 1 && b <= N - 1) {
        const double i2h = 1.0 / (2.0 * h);
        const double dxjx = (jx[g + 1] - jx[g - 1]) * i2h;
        const double dyjy = (jy[g + pitch] - jy[g - pitch]) * i2h;
        const double dxjy = (jy[g + 1] - jy[g - 1]) * i2h;
        const double dyjx = (jx[g + pitch] - jx[g - pitch]) * i2h;
        e = -(dxjx + dyjy);
        m = dxjy - dyjx;
    }
    fE[g] = e;
    fB[g] = m;
}

// Driver density at node (a, b) = (x, y).  Radial-bin membership comes from the
// node map built on the host, so bin edges are decided exactly once.
__device__ double beam_density(const BeamSet& B, double x, double y, size_t node, double xi) {
    if (xi < 0.0) return 0.0;
    double s = 0.0;
    for (int k = 0; k < B.n; ++k) {
        const double lz = (xi - B.xc[k]) * (xi - B.xc[k]) / (B.sz[k] * B.sz[k]);
        if (B.kind[k] == 0) {
            const double rx = x - B.x0[k], ry = y - B.y0[k];
            const double r2 = rx * rx + ry * ry;
            s += B.amp[k] * exp(-r2 / (B.sr[k] * B.sr[k]) - lz);
        } else {
            const int kb = B.bmap[k][node];
            if (kb >= 0) s += B.bins[k][kb] * exp(-lz);
        }
    }
    return s;
}

// Node (a, b) inside the disc of radius r around (x0, y0); every operation
// rounded separately so that host and device agree on the edge.
__device__ bool in_disc(double L, double h, int a, int b, double x0, double y0, double r) {
#pragma clang fp contract(off)
    const double rx = (-L + a * h) - x0, ry = (-L + b * h) - y0;
    return rx * rx + ry * ry <= r * r;
}

// Current of the driver macroparticles (time loop) at a node and slice
// position xi: the fixed-point deposit planes interpolated linearly in xi
// (zero outside them).
struct DriverPlanes {
    const unsigned long long* p;  // nullptr: no driver particles in this sweep
    int nz;
    double xi0, dz;
    size_t plane;  // words per plane
};

__device__ __forceinline__ double driver_current(const DriverPlanes& D, size_t i, double xi) {
    if (!D.p) return 0.0;
    const double t = (xi - D.xi0) / D.dz;
    const int m = (int)floor(t);
    if (m < 0 || m > D.nz - 2) return 0.0;
    const double a = t - m;
    constexpr double kUnfix = 1.0 / 1099511627776.0;  // one unit of the planes: 2^-40
    const double v0 = (double)(long long)D.p[(size_t)m * D.plane + i] * kUnfix;
    const double v1 = (double)(long long)D.p[(size_t)(m + 1) * D.plane + i] * kUnfix;
    return (1.0 - a) * v0 + a * v1;
}

// Total j_z on every node: plasma n*<p_z>/g = G/g - n* with G = n*<gamma> =
// [n*(1 + g^2 + a2/2) + g^2 (Txx + Tyy)]/(2g) (eq. (9) and the gamma of Sec.
// III.A, <p_perp^2> = g^2 <V^2>, a2 = |A-hat|^2 of a laser envelope or 0 when
// a2 is null), plus the frozen drivers' density at xi (luminal beam current)
// and the driver macroparticles' current (time loop).
__global__ void k_jz(int N, double L, double h, int pitch, const double* __restrict__ n,
                     const double* __restrict__ txx, const double* __restrict__ tyy,
                     const double* __restrict__ psi, const double* __restrict__ a2,
                     const double* __restrict__ st, BeamSet beams, DriverPlanes drv,
                     double* __restrict__ jz, double* __restrict__ k2,
                     int32_t* __restrict__ flags) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t i = (size_t)b * pitch + a;
    // every load unconditional and the plasma term selected after (a load
    // behind the n* > 0 branch would be waited for inside it)
    const double ni = n[i], g = 1.0 + psi[i], tt = txx[i] + tyy[i];
    const double q = a2 ? 0.5 * a2[i] : 0.0;
    if (ni > 0.0 && !(g > 0.0)) atomicOr(flags, 1);
    const double G = (ni * (1.0 + g * g + q) + g * g * tt) / (2.0 * g);
    const double v = ni > 0.0 ? G / g - ni : 0.0;
    jz[i] = v + beam_density(beams, -L + a * h, -L + b * h, (size_t)b * (N + 1) + a, st[0]) +
            driver_current(drv, i, st[0]);
    // k2 = n* / g of the B_perp Helmholtz system (eqs. (18)-(19)) on the
    // interior nodes (it reads neither E_z nor B_z)
    const bool interior = a >= 1 && b >= 1 && a <= N - 1 && b <= N - 1;
    k2[i] = interior && ni > 0.0 ? ni / g : 0.0;
}

// The B_perp right-hand sides on the interior nodes (k_jz writes k2 = n* / g):
//   f_Bx = D_y(j_z - Tyy) - D_x Txy + (jx Bz - jy Ez)/g + (G/g^2 - Tyy/g) psi_y - (Txy/g) psi_x
//          - n* D_y(a2/4)/g^2
//   f_By = D_x(Txx - j_z) + D_y Txy + (jy Bz + jx Ez)/g - (G/g^2 - Txx/g) psi_x + (Txy/g) psi_y
//          + n* D_x(a2/4)/g^2
// (G as in k_jz; the a2 terms are the ponderomotive part of S, present when a2
// is not null).
__global__ void k_assemble(int N, double h, int pitch, const double* __restrict__ n,
                           const double* __restrict__ jx, const double* __restrict__ jy,
                           const double* __restrict__ txx, const double* __restrict__ txy,
                           const double* __restrict__ tyy, const double* __restrict__ psi,
                           const double* __restrict__ Ez, const double* __restrict__ Bz,
                           const double* __restrict__ jz, const double* __restrict__ a2,
                           double* __restrict__ fBx, double* __restrict__ fBy) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t i = (size_t)b * pitch + a;
    double fx = 0.0, fy = 0.0;
    if (a >= 1 && b >= 1 && a <= N - 1 && b <= N - 1) {
        const double i2h = 1.0 / (2.0 * h);
        const size_t e = i + 1, w = i - 1, nn = i + pitch, s = i - pitch;
        const double g = 1.0 + psi[i];
        const double psx = (psi[e] - psi[w]) * i2h, psy = (psi[nn] - psi[s]) * i2h;
        fx = ((jz[nn] - tyy[nn]) - (jz[s] - tyy[s])) * i2h - (txy[e] - txy[w]) * i2h;
        fy = ((txx[e] - jz[e]) - (txx[w] - jz[w])) * i2h + (txy[nn] - txy[s]) * i2h;
        if (n[i] > 0.0) {
            const double q = a2 ? 0.5 * a2[i] : 0.0;
            const double G = (n[i] * (1.0 + g * g + q) + g * g * (txx[i] + tyy[i])) / (2.0 * g);
            fx += (jx[i] * Bz[i] - jy[i] * Ez[i]) / g + (G / (g * g) - tyy[i] / g) * psy -
                  (txy[i] / g) * psx;
            fy += (jy[i] * Bz[i] + jx[i] * Ez[i]) / g - (G / (g * g) - txx[i] / g) * psx +
                  (txy[i] / g) * psy;
            if (a2) {
                fx -= n[i] * (0.25 * ((a2[nn] - a2[s]) * i2h)) / (g * g);
                fy += n[i] * (0.25 * ((a2[e] - a2[w]) * i2h)) / (g * g);
            }
        }
    }
    fBx[i] = fx;
    fBy[i] = fy;
}

// Probe k adds the mean of its field over its disc (fixed summation order, one block).
__global__ __launch_bounds__(256) void k_probe(int N, double L, double h, int pitch,
                                               const double* __restrict__ F, double x0, double y0,
                                               double rmax, double scale,
                                               double* __restrict__ acc) {
    __shared__ double red[2][4];
    double s = 0.0, cnt = 0.0;
    for (int i = threadIdx.x; i < (N + 1) * (N + 1); i += 256) {
        const int b = i / (N + 1), a = i - b * (N + 1);
        if (in_disc(L, h, a, b, x0, y0, rmax)) {
            s += F[(size_t)b * pitch + a];
            cnt += 1.0;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        cnt += __shfl_xor(cnt, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s;
        red[1][threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double S = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        const double C = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
        if (C > 0) *acc += scale * S / C;
    }
}

// Adjoint seed of a probe: Fb += w on the interior nodes of its disc (the
// boundary values are fixed, their adjoints never propagate).
__global__ void k_probe_seed(int N, double L, double h, int pitch, double x0, double y0,
                             double rmax, double w, double* __restrict__ Fb) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a < 1 || a > N - 1 || b < 1 || b > N - 1) return;
    if (in_disc(L, h, a, b, x0, y0, rmax)) Fb[(size_t)b * pitch + a] += w;
}

__global__ void k_pack(int N, int pitch, const double* __restrict__ src, double* __restrict__ dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    dst[(size_t)b * (N + 1) + a] = src[(size_t)b * pitch + a];
}

__global__ void k_unpack(int N, int pitch, const double* __restrict__ src, double* __restrict__ dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const bool bnd = a == 0 || b == 0 || a == N || b == N;
    dst[(size_t)b * pitch + a] = bnd ? 0.0 : src[(size_t)b * (N + 1) + a];
}

// Initial guesses for the five solves of this slice: the fields u of the last
// slice (at xi_0), extrapolated to xi through the slices before (p1 at xi_1,
// p2 at xi_2, p3 at xi_3) -- order 0: u; order m: the Lagrange polynomial of
// degree m through u, p1, ..., pm.  The guess goes to `out` (the oldest
// array, which the host then rotates into the field's place).
struct FieldPtrs {
    const double* u[5];
    const double* p1[5];
    const double* p2[5];
    const double* p3[5];
    double* out[5];
};

// Lagrange weights of the guess through the stored slices (one thread): the
// order drops while two of the points coincide; wts = [order, w1, w2, w3].
__global__ void k_guess_weights(const double* __restrict__ st, int order, double* __restrict__ wts) {
    if (threadIdx.x != 0) return;
    const double xi = st[0];
    const double x[4] = {st[2], st[3], st[4], st[5]};
    for (bool ok = false; !ok && order > 0;) {
        ok = true;
        for (int i = 0; i <= order && ok; ++i)
            for (int j = 0; j < i; ++j)
                if (x[i] == x[j]) ok = false;
        if (!ok) --order;
    }
    double w[4] = {1.0, 0.0, 0.0, 0.0};  // weights of p1..p3 relative to u (w[0] unused)
    for (int i = 1; i <= order; ++i) {
        double l = 1.0;
        for (int j = 0; j <= order; ++j)
            if (j != i) l *= (xi - x[j]) / (x[i] - x[j]);
        w[i] = l;
    }
    wts[0] = (double)order;
    wts[1] = w[1];
    wts[2] = w[2];
    wts[3] = w[3];
}

__global__ void k_extrapolate(int N, int pitch, const double* __restrict__ wts, FieldPtrs f) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t g = (size_t)b * pitch + a;
    const int order = (int)wts[0];
    const double w1 = wts[1], w2 = wts[2], w3 = wts[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double u = f.u[k][g];
        double v = u;
        if (order == 1) v = u + w1 * (f.p1[k][g] - u);
        if (order == 2) v = u + (w1 * (f.p1[k][g] - u) + w2 * (f.p2[k][g] - u));
        if (order == 3)
            v = u + (w1 * (f.p1[k][g] - u) + w2 * (f.p2[k][g] - u) + w3 * (f.p3[k][g] - u));
        f.out[k][g] = v;
    }
}

__global__ void k_fill(double* p, size_t n, double v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

dim3 node_grid(int N) { return dim3((N + 1 + 127) / 128, N + 1); }

}  // namespace

wandqs_status rhs_EB(wandqs_ctx* c) {
    const Level& L0 = c->lev[0];
    {
        ProfScope ps(c, "k_rhs_EB", (double)(c->N + 1) * (c->N + 1) * 32.0);
        WQ_KLAUNCH(ps, k_rhs_EB, node_grid(c->N), dim3(128), 0, c->stream, c->N, c->h, L0.pitch,
                           c->mom[1], c->mom[2], L0.f[0], L0.f[1]);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status plasma_jz(wandqs_ctx* c) {
    const Level& L0 = c->lev[0];
    {
        const DriverPlanes drv{c->drv_active ? c->drv_planes : nullptr, c->drv_nz, c->cfg.driver_xi0,
                               c->cfg.driver_dz, (size_t)(c->N + 1) * L0.pitch};
        ProfScope ps(c, "k_jz", (double)(c->N + 1) * (c->N + 1) * 48.0);
        WQ_KLAUNCH(ps, k_jz, node_grid(c->N), dim3(128), 0, c->stream, c->N, c->L, c->h, L0.pitch,
                           c->mom[0], c->mom[3], c->mom[5], c->fields[0],
                           c->las_on ? c->las_a2 : nullptr, c->st, c->beamset, drv, c->jz, L0.k2,
                           c->flags);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

// jz_ready: plasma_jz has run already (it does not read E_z or B_z).
wandqs_status assemble(wandqs_ctx* c, bool jz_ready) {
    const Level& L0 = c->lev[0];
    if (!jz_ready) {
        const wandqs_status s = plasma_jz(c);
        if (s != WANDQS_OK) return s;
    }
    {
        ProfScope ps(c, "k_assemble", (double)(c->N + 1) * (c->N + 1) * 96.0);
        WQ_KLAUNCH(ps, k_assemble, node_grid(c->N), dim3(128), 0, c->stream, c->N, c->h, L0.pitch,
                           c->mom[0], c->mom[1], c->mom[2], c->mom[3], c->mom[4], c->mom[5],
                           c->fields[0], c->fields[1], c->fields[2], c->jz,
                           c->las_on ? c->las_a2 : nullptr, L0.f[0], L0.f[1]);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status probes_accumulate(wandqs_ctx* c, int64_t slice) {
    for (size_t k = 0; k < c->probes.size(); ++k) {
        const wandqs_probe& p = c->probes[k];
        if (slice < p.slice_begin || slice >= p.slice_end) continue;
        const double scale = 1.0 / (double)(p.slice_end - p.slice_begin);
        {
            ProfScope ps(c, "k_probe", (double)(c->N + 1) * (c->N + 1) * 8.0);
            WQ_KLAUNCH(ps, k_probe, dim3(1), dim3(256), 0, c->stream, c->N, c->L, c->h,
                               c->lev[0].pitch, c->fields[p.field], p.x0, p.y0, p.r_max, scale,
                               c->probe_acc + k);
        }
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status probe_seed(wandqs_ctx* c, int k, double w, double* const* Fb) {
    const wandqs_probe& p = c->probes[k];
    {
        ProfScope ps(c, "k_probe_seed", (double)(c->N + 1) * (c->N + 1) * 16.0);
        WQ_KLAUNCH(ps, k_probe_seed, node_grid(c->N), dim3(128), 0, c->stream, c->N, c->L, c->h,
                           c->lev[0].pitch, p.x0, p.y0, p.r_max, w, Fb[p.field]);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status pack_fields(wandqs_ctx* c, double* const* src, int n, double* dst) {
    const size_t nn = (size_t)(c->N + 1) * (c->N + 1);
    for (int k = 0; k < n; ++k)
        {
            ProfScope ps(c, "k_pack", (double)(c->N + 1) * (c->N + 1) * 16.0);
            WQ_KLAUNCH(ps, k_pack, node_grid(c->N), dim3(128), 0, c->stream, c->N,
                               c->lev[0].pitch, src[k], dst + k * nn);
        }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status unpack_fields(wandqs_ctx* c, const double* src, int n, double* const* dst) {
    const size_t nn = (size_t)(c->N + 1) * (c->N + 1);
    for (int k = 0; k < n; ++k)
        {
            ProfScope ps(c, "k_unpack", (double)(c->N + 1) * (c->N + 1) * 16.0);
            WQ_KLAUNCH(ps, k_unpack, node_grid(c->N), dim3(128), 0, c->stream, c->N,
                               c->lev[0].pitch, src + k * nn, dst[k]);
        }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status extrapolate_guess(wandqs_ctx* c, int order) {
    FieldPtrs f;
    double* const* oldest = kGuessMax > 3 ? c->fields_prev3 : c->fields_prev2;
    for (int k = 0; k < 5; ++k) {
        f.u[k] = c->fields[k];
        f.p1[k] = c->fields_prev[k];
        f.p2[k] = c->fields_prev2[k];
        f.p3[k] = kGuessMax > 3 ? c->fields_prev3[k] : c->fields_prev2[k];
        f.out[k] = oldest[k];
    }
    order = order < 0 ? 0 : (order > kGuessMax - 1 ? kGuessMax - 1 : order);
    double* wts = c->st + 8;
    {
        ProfScope ps(c, "k_guess_weights", 80.0);
        WQ_KLAUNCH(ps, k_guess_weights, dim3(1), dim3(64), 0, c->stream, c->st, order, wts);
    }
    {
        ProfScope ps(c, "k_extrapolate", (double)(c->N + 1) * (c->N + 1) * 5 * 8.0 * (order + 2));
        WQ_KLAUNCH(ps, k_extrapolate, node_grid(c->N), dim3(128), 0, c->stream, c->N,
                   c->lev[0].pitch, wts, f);
    }
    WQ_LAUNCH_CHECK();
    for (int k = 0; k < 5; ++k) {  // oldest <- ... <- prev <- u <- guess
        double* g = oldest[k];
        if (kGuessMax > 3) c->fields_prev3[k] = c->fields_prev2[k];
        c->fields_prev2[k] = c->fields_prev[k];
        c->fields_prev[k] = c->fields[k];
        c->fields[k] = g;
    }
    return WANDQS_OK;
}

wandqs_status copy_d2d(wandqs_ctx* c, void* dst, const void* src, size_t bytes) {
    WQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    return WANDQS_OK;
}

wandqs_status fill_f64(wandqs_ctx* c, double* p, size_t n, double v) {
    if (n == 0) return WANDQS_OK;
    {
        ProfScope ps(c, "k_fill", 8.0 * n);
        WQ_KLAUNCH(ps, k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n, v);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace wq
