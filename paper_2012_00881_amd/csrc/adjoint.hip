// Reverse mode of one xi-slice (discretise, then differentiate) for gradients
// of probe losses with respect to the driver parameters theta (the Gaussian
// amplitudes and the radial-bin amplitudes of the frozen driver, Sec. V.A).
//
// The reverse of a slice visits the forward steps last to first:
//   push (per particle; the gathers of grad psi, B_perp and Bz transposed into
//   node adjoints, with the CIC position derivatives), the B_perp Helmholtz
//   solves (lambda = (L_h - k2)^-1 Bbar, then k2bar = lambda . B), the B_perp
//   assembly (j, T, n*, psi, Ez, Bz and the driver through j_z), the Ez / Bz
//   Poisson solves, the deposits of j and T and the gather g = 1 + psi, the psi
//   solve, the deposit of n*.  The discrete operators are symmetric, so each
//   adjoint solve is a forward multigrid solve.  Particle-to-node transposes
//   run in the cell tiles of the deposits (fixed summation order, no atomics);
//   node-to-node transposes are written in gather form; dL/dtheta is a fixed-
//   order segmented sum.  Adjoints of the particles travel between slices in
//   particle-ID order.
#include <cmath>

#include "wq_common.h"

namespace wq {
namespace {

constexpr int TN = kDepTile;
constexpr int TC = TN + 1;

__device__ __forceinline__ void cic(double x, double L, double h, int N, int& c, double& d) {
    const double t = (x + L) / h;
    int k = (int)floor(t);
    k = k < 0 ? 0 : (k > N - 1 ? N - 1 : k);
    c = k;
    d = t - k;
}

// Bilinear interpolant of four cell corners: value and its x / y derivatives.
struct Interp {
    double v, dx, dy;
};
__device__ __forceinline__ Interp interp(double f00, double f10, double f01, double f11,
                                         double ddx, double ddy, double h) {
    Interp r;
    r.v = f00 * (1.0 - ddx) * (1.0 - ddy) + f10 * ddx * (1.0 - ddy) + f01 * (1.0 - ddx) * ddy +
          f11 * ddx * ddy;
    r.dx = ((f10 - f00) * (1.0 - ddy) + (f11 - f01) * ddy) / h;
    r.dy = ((f01 - f00) * (1.0 - ddx) + (f11 - f10) * ddx) / h;
    return r;
}

// Node gradient of psi: central inside, one-sided on the boundary lines (the
// three values loaded from clamped indices and the formula selected after, so
// that no load waits behind a branch).
__device__ __forceinline__ double gradx(const double* psi, int pitch, int N, double h, int a, int b) {
    const double* r = psi + (size_t)b * pitch;
    const double pl = r[a > 0 ? a - 1 : 0], pc = r[a], pr = r[a < N ? a + 1 : N];
    return a == 0 ? (pr - pc) / h : (a == N ? (pc - pl) / h : (pr - pl) / (2.0 * h));
}
__device__ __forceinline__ double grady(const double* psi, int pitch, int N, double h, int a, int b) {
    const double pl = psi[(size_t)(b > 0 ? b - 1 : 0) * pitch + a], pc = psi[(size_t)b * pitch + a],
                 pr = psi[(size_t)(b < N ? b + 1 : N) * pitch + a];
    return b == 0 ? (pr - pc) / h : (b == N ? (pc - pl) / h : (pr - pl) / (2.0 * h));
}

// Particles per batch of loads in the reverse push and deposits: a batch's
// loads (and then its adjoint loads by ID) are all in flight together, the
// particles then taken in order as before.  Measured over the C5 reverse
// sweep: 386 / 268 us for k_push_adj / k_dep_adj with 2, 566 / 279 with 4
// (k_push_adj's registers then allow one wavefront per SIMD), 446 / 450 with
// the particles loaded one at a time.
#ifndef WQ_ADJ_BATCH
#define WQ_ADJ_BATCH 2
#endif
constexpr int kAdjBatch = WQ_ADJ_BATCH;

__device__ __forceinline__ bool interior(int N, int a, int b) {
    return a >= 1 && b >= 1 && a <= N - 1 && b <= N - 1;
}

// Node sums of a tile from the per-cell corner accumulators: node (a, b) is
// corner 11 of cell (a-1, b-1), 01 of (a, b-1), 10 of (a-1, b) and 00 of (a, b).
template <int M>
__device__ __forceinline__ void tile_node_sums(const double (*corner)[4 * M], int a0, int b0,
                                               int N, int pitch, double* const* out) {
    for (int i = threadIdx.x; i < TN * TN; i += blockDim.x) {
        const int ny = i / TN, nx = i - ny * TN;
        const int ga = a0 + nx, gb = b0 + ny;
        if (ga > N || gb > N) continue;
        const size_t g = (size_t)gb * pitch + ga;
#pragma unroll
        for (int m = 0; m < M; ++m)
            out[m][g] = corner[ny * TC + nx][3 * M + m] + corner[ny * TC + nx + 1][2 * M + m] +
                        corner[(ny + 1) * TC + nx][1 * M + m] +
                        corner[(ny + 1) * TC + nx + 1][0 * M + m];
    }
}

struct PushAdjArgs {
    int N;
    double L, h;
    int pitch;
    int64_t P;
    const double *x, *y, *px, *py;  // slice input, cell order
    const int32_t *id, *start;
    const double *psi, *Bx, *By, *Bz;  // solved fields of the slice
    const double* st;                  // [xi, dxi]
    const double* adj_in;              // [4][P] ID order: adjoints of the pushed particles
    double *xb, *yb, *pxb, *pyb, *gb;  // out (cell order): partial input adjoints, adjoint of g_i
    double *Gxb, *Gyb, *Bxb, *Byb, *Bzb;  // out: node adjoints of the gathered fields
};

// Push reversed (kick, rotation, kick, drift, specular walls; the branch the
// forward took is differentiated).  A workgroup owns the cells of its tile and
// writes their particles; the rim cells below and left of the tile only add to
// the corner sums of the tile's nodes.
__global__ __launch_bounds__(256) void k_push_adj(PushAdjArgs a) {
    constexpr int M = 5;
    __shared__ double corner[TC * TC][4 * M];
    int tbx, tby;
    tile_of_block(tbx, tby);
    const int a0 = tbx * TN, b0 = tby * TN;
    const int N = a.N, pitch = a.pitch;
    const double h = a.h, L = a.L, d = a.st[1];
    const int64_t P = a.P;
    for (int c = threadIdx.x; c < TC * TC; c += blockDim.x) {
        const int cy = c / TC, cx = c - cy * TC;
        const int ga = a0 - 1 + cx, gb = b0 - 1 + cy;
        double s[4][M];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) s[q][m] = 0.0;
        {
            // the cell clamped into the grid, its particle range emptied when
            // it lies outside (no load behind a lane-dependent branch)
            const bool valid = ga >= 0 && ga < N && gb >= 0 && gb < N;
            const int gac = min(max(ga, 0), N - 1), gbc = min(max(gb, 0), N - 1);
            const bool own = cx >= 1 && cy >= 1;
            const int cell = gbc * N + gac;
            const size_t g = (size_t)gbc * pitch + gac;
            const double p00 = a.psi[g], p10 = a.psi[g + 1], p01 = a.psi[g + pitch],
                         p11 = a.psi[g + pitch + 1];
            const double gx00 = gradx(a.psi, pitch, N, h, gac, gbc),
                         gx10 = gradx(a.psi, pitch, N, h, gac + 1, gbc),
                         gx01 = gradx(a.psi, pitch, N, h, gac, gbc + 1),
                         gx11 = gradx(a.psi, pitch, N, h, gac + 1, gbc + 1);
            const double gy00 = grady(a.psi, pitch, N, h, gac, gbc),
                         gy10 = grady(a.psi, pitch, N, h, gac + 1, gbc),
                         gy01 = grady(a.psi, pitch, N, h, gac, gbc + 1),
                         gy11 = grady(a.psi, pitch, N, h, gac + 1, gbc + 1);
            const double bx00 = a.Bx[g], bx10 = a.Bx[g + 1], bx01 = a.Bx[g + pitch],
                         bx11 = a.Bx[g + pitch + 1];
            const double by00 = a.By[g], by10 = a.By[g + 1], by01 = a.By[g + pitch],
                         by11 = a.By[g + pitch + 1];
            const double bz00 = a.Bz[g], bz10 = a.Bz[g + 1], bz01 = a.Bz[g + pitch],
                         bz11 = a.Bz[g + pitch + 1];
            const int k0 = a.start[cell], k1 = k0 + (a.start[cell + 1] - k0) * (valid ? 1 : 0);
            for (int kb = k0; kb < k1; kb += kAdjBatch) {
            const int cnt = min(kAdjBatch, k1 - kb);
            double xv[kAdjBatch], yv[kAdjBatch], pxv[kAdjBatch], pyv[kAdjBatch];
            int64_t idv[kAdjBatch];
#pragma unroll
            for (int ib = 0; ib < kAdjBatch; ++ib) {
                const int kk = kb + min(ib, cnt - 1);
                xv[ib] = a.x[kk];
                yv[ib] = a.y[kk];
                pxv[ib] = a.px[kk];
                pyv[ib] = a.py[kk];
                idv[ib] = a.id[kk];
            }
            double av[kAdjBatch][4];
#pragma unroll
            for (int ib = 0; ib < kAdjBatch; ++ib)
#pragma unroll
                for (int q = 0; q < 4; ++q) av[ib][q] = a.adj_in[q * P + idv[ib]];
#pragma unroll
            for (int ib = 0; ib < kAdjBatch; ++ib) {
                if (ib >= cnt) break;
                const int k = kb + ib;
                const double ddx = (xv[ib] + L) / h - ga, ddy = (yv[ib] + L) / h - gb;
                const Interp gp = interp(p00, p10, p01, p11, ddx, ddy, h);
                const Interp Gxi = interp(gx00, gx10, gx01, gx11, ddx, ddy, h);
                const Interp Gyi = interp(gy00, gy10, gy01, gy11, ddx, ddy, h);
                const Interp bxi = interp(bx00, bx10, bx01, bx11, ddx, ddy, h);
                const Interp byi = interp(by00, by10, by01, by11, ddx, ddy, h);
                const Interp bzi = interp(bz00, bz10, bz01, bz11, ddx, ddy, h);
                const double G_ = 1.0 + gp.v, p0x = pxv[ib], p0y = pyv[ib];
                const double Gx = Gxi.v, Gy = Gyi.v, bx = bxi.v, by = byi.v, bz = bzi.v;
                // forward replay
                const double gam = (1.0 + p0x * p0x + p0y * p0y + G_ * G_) / (2.0 * G_);
                const double Fx = gam * Gx / G_ - by, Fy = gam * Gy / G_ + bx;
                const double mx = p0x + 0.5 * d * Fx, my = p0y + 0.5 * d * Fy;
                const double t = bz * d / (2.0 * G_), sr = 2.0 * t / (1.0 + t * t);
                const double qx = mx - t * my, qy = my + t * mx;
                const double rx = mx - sr * qy, ry = my + sr * qx;
                const double p1x = rx + 0.5 * d * Fx, p1y = ry + 0.5 * d * Fy;
                const double x1 = xv[ib] + d * p1x / G_, y1 = yv[ib] + d * p1y / G_;
                // reverse
                double x1b = av[ib][0], y1b = av[ib][1];
                double p1xb = av[ib][2], p1yb = av[ib][3];
                if (x1 > L || x1 < -L) {
                    x1b = -x1b;
                    p1xb = -p1xb;
                }
                if (y1 > L || y1 < -L) {
                    y1b = -y1b;
                    p1yb = -p1yb;
                }
                double xbar = x1b, ybar = y1b;
                p1xb += x1b * d / G_;
                p1yb += y1b * d / G_;
                double gbar = -(x1b * d * p1x + y1b * d * p1y) / (G_ * G_);
                double Fxb = 0.5 * d * p1xb, Fyb = 0.5 * d * p1yb;
                double mxb = p1xb, myb = p1yb;
                const double sb = -p1xb * qy + p1yb * qx;
                const double qyb = -p1xb * sr, qxb = p1yb * sr;
                mxb += qxb + qyb * t;
                myb += -qxb * t + qyb;
                double tb = -qxb * my + qyb * mx;
                tb += sb * 2.0 * (1.0 - t * t) / ((1.0 + t * t) * (1.0 + t * t));
                const double bzb = tb * d / (2.0 * G_);
                gbar += -tb * bz * d / (2.0 * G_ * G_);
                double p0xb = mxb, p0yb = myb;
                Fxb += 0.5 * d * mxb;
                Fyb += 0.5 * d * myb;
                const double gamb = Fxb * Gx / G_ + Fyb * Gy / G_;
                const double Gxb = Fxb * gam / G_, Gyb = Fyb * gam / G_;
                gbar += -(Fxb * gam * Gx + Fyb * gam * Gy) / (G_ * G_);
                const double byb = -Fxb, bxb = Fyb;
                p0xb += gamb * p0x / G_;
                p0yb += gamb * p0y / G_;
                gbar += gamb * (G_ * G_ - 1.0 - p0x * p0x - p0y * p0y) / (2.0 * G_ * G_);
                xbar += Gxb * Gxi.dx + Gyb * Gyi.dx + bxb * bxi.dx + byb * byi.dx + bzb * bzi.dx;
                ybar += Gxb * Gxi.dy + Gyb * Gyi.dy + bxb * bxi.dy + byb * byi.dy + bzb * bzi.dy;
                if (own) {
                    a.xb[k] = xbar;
                    a.yb[k] = ybar;
                    a.pxb[k] = p0xb;
                    a.pyb[k] = p0yb;
                    a.gb[k] = gbar;
                }
                const double w[4] = {(1.0 - ddx) * (1.0 - ddy), ddx * (1.0 - ddy),
                                     (1.0 - ddx) * ddy, ddx * ddy};
                const double q[M] = {Gxb, Gyb, bxb, byb, bzb};
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int m = 0; m < M; ++m) s[r][m] += w[r] * q[m];
            }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int m = 0; m < M; ++m) corner[c][r * M + m] = s[r][m];
    }
    __syncthreads();
    double* out[M] = {a.Gxb, a.Gyb, a.Bxb, a.Byb, a.Bzb};
    tile_node_sums<M>(corner, a0, b0, N, pitch, out);
}

// psib = transposed node gradient applied to (Gxb, Gyb) (interior nodes; the
// boundary entries are never used); clears the boundary entries of Bxb, Byb,
// Bzb (fixed values) and all of Ezb.
__global__ void k_grad_adj(int N, double h, int pitch, const double* __restrict__ Gxb,
                           const double* __restrict__ Gyb, double* __restrict__ psib,
                           double* __restrict__ Bxb, double* __restrict__ Byb,
                           double* __restrict__ Bzb, double* __restrict__ Ezb) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t g = (size_t)b * pitch + a;
    const bool in = interior(N, a, b);
    double v = 0.0;
    if (in) {
        const double i2h = 1.0 / (2.0 * h), ih = 1.0 / h;
        // gx(a') reads psi(a) with +1/2h for a' = a - 1 and -1/2h for a' = a + 1
        // (1/h where a' lies on the boundary line)
        v += Gxb[g - 1] * (a - 1 == 0 ? ih : i2h);
        v -= Gxb[g + 1] * (a + 1 == N ? ih : i2h);
        v += Gyb[g - pitch] * (b - 1 == 0 ? ih : i2h);
        v -= Gyb[g + pitch] * (b + 1 == N ? ih : i2h);
    }
    psib[g] = v;
    Ezb[g] = 0.0;
    if (!in) {
        Bxb[g] = 0.0;
        Byb[g] = 0.0;
        Bzb[g] = 0.0;
    }
}

// Adds dense field adjoints [5][N+1][N+1] on the interior nodes.
struct FieldBar {
    double* f[5];
};
__global__ void k_field_seed(int N, int pitch, const double* __restrict__ src, FieldBar dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (!interior(N, a, b)) return;
    const size_t nn = (size_t)(N + 1) * (N + 1);
    const size_t g = (size_t)b * pitch + a, d = (size_t)b * (N + 1) + a;
#pragma unroll
    for (int k = 0; k < 5; ++k) dst.f[k][g] += src[k * nn + d];
}

struct AsmAdjArgs {
    int N;
    double L, h;
    int pitch;
    const double *n, *jx, *jy, *txx, *txy, *tyy;  // moments of the slice
    const double *psi, *Ez, *Bz, *Bx, *By;        // fields of the slice
    const double *lx, *ly;                        // B_perp adjoint solutions
    double *nb, *jxb, *jyb, *txxb, *txyb, *tyyb;  // set by the local part
    double *psxb, *psyb, *gnb;                    // adjoints of psi_x, psi_y, g at the node
    double *Ezb, *Bzb;                            // added to
    double *psib, *jzb;                           // diff part: psib added to, jzb set
};

// Assembly reversed, the node-local terms at each interior node with plasma:
// the (e_z x j) Bz / g, j Ez / g, G grad psi / g^2 and T . grad psi / g terms of
// f_B and k2 = n* / g with k2bar = lx Bx + ly By.
__global__ void k_asm_adj_local(AsmAdjArgs a) {
    const int ia = blockIdx.x * blockDim.x + threadIdx.x;
    const int ib = blockIdx.y;
    const int N = a.N;
    if (ia > N) return;
    const size_t i = (size_t)ib * a.pitch + ia;
    double nb = 0, jxb = 0, jyb = 0, txxb = 0, txyb = 0, tyyb = 0, psxb = 0, psyb = 0, ggb = 0;
    if (interior(N, ia, ib) && a.n[i] > 0.0) {
        const double i2h = 1.0 / (2.0 * a.h);
        const double Lxb = a.lx[i], Lyb = a.ly[i];
        const double gg = 1.0 + a.psi[i], n = a.n[i];
        const double Txx = a.txx[i], Txy = a.txy[i], Tyy = a.tyy[i], jx_ = a.jx[i], jy_ = a.jy[i];
        const double Ez = a.Ez[i], Bz = a.Bz[i];
        const double G = (n * (1.0 + gg * gg) + gg * gg * (Txx + Tyy)) / (2.0 * gg);
        const double psx = (a.psi[i + 1] - a.psi[i - 1]) * i2h;
        const double psy = (a.psi[i + a.pitch] - a.psi[i - a.pitch]) * i2h;
        jxb = (Lxb * Bz + Lyb * Ez) / gg;
        jyb = (-Lxb * Ez + Lyb * Bz) / gg;
        a.Bzb[i] += (Lxb * jx_ + Lyb * jy_) / gg;
        a.Ezb[i] += (-Lxb * jy_ + Lyb * jx_) / gg;
        const double Gb = (Lxb * psy - Lyb * psx) / (gg * gg);
        tyyb = -Lxb * psy / gg;
        txxb = Lyb * psx / gg;
        txyb = (-Lxb * psx + Lyb * psy) / gg;
        psxb = -Lxb * Txy / gg - Lyb * (G / (gg * gg) - Txx / gg);
        psyb = Lxb * (G / (gg * gg) - Tyy / gg) + Lyb * Txy / gg;
        ggb = Lxb * (-(jx_ * Bz - jy_ * Ez) / (gg * gg) +
                     (-2.0 * G / (gg * gg * gg) + Tyy / (gg * gg)) * psy + (Txy / (gg * gg)) * psx) +
              Lyb * (-(jy_ * Bz + jx_ * Ez) / (gg * gg) -
                     (-2.0 * G / (gg * gg * gg) + Txx / (gg * gg)) * psx - (Txy / (gg * gg)) * psy);
        const double k2b = Lxb * a.Bx[i] + Lyb * a.By[i];
        nb = k2b / gg;
        ggb += -k2b * n / (gg * gg);
        nb += Gb * (1.0 + gg * gg) / (2.0 * gg);
        txxb += Gb * gg / 2.0;
        tyyb += Gb * gg / 2.0;
        ggb += Gb * (n * (gg * gg - 1.0) / (2.0 * gg * gg) + (Txx + Tyy) / 2.0);
    }
    a.nb[i] = nb;
    a.jxb[i] = jxb;
    a.jyb[i] = jyb;
    a.txxb[i] = txxb;
    a.txyb[i] = txyb;
    a.tyyb[i] = tyyb;
    a.psxb[i] = psxb;
    a.psyb[i] = psyb;
    a.gnb[i] = ggb;
}

__device__ __forceinline__ double at_interior(const double* v, int N, int pitch, int a, int b) {
    return interior(N, a, b) ? v[(size_t)b * pitch + a] : 0.0;
}
// (D_x^T v) and (D_y^T v) at node (a, b) for v given on the interior nodes
// (D_x u = (u(a+1) - u(a-1)) / 2h).
__device__ __forceinline__ double DxT(const double* v, int N, int pitch, double i2h, int a, int b) {
    return (at_interior(v, N, pitch, a - 1, b) - at_interior(v, N, pitch, a + 1, b)) * i2h;
}
__device__ __forceinline__ double DyT(const double* v, int N, int pitch, double i2h, int a, int b) {
    return (at_interior(v, N, pitch, a, b - 1) - at_interior(v, N, pitch, a, b + 1)) * i2h;
}

// Assembly reversed, the difference terms in gather form on every node:
// D_y(j_z - Tyy) - D_x Txy and D_x(Txx - j_z) + D_y Txy, the psi_x / psi_y
// adjoints onto psi, and j_z = G/g - n* + n_b (plasma part where n* > 0).
// jzb (the adjoint of the total j_z) is kept for dL/dtheta.
__global__ void k_asm_adj_diff(AsmAdjArgs a) {
    const int ia = blockIdx.x * blockDim.x + threadIdx.x;
    const int ib = blockIdx.y;
    const int N = a.N, pitch = a.pitch;
    if (ia > N) return;
    const size_t i = (size_t)ib * pitch + ia;
    const double i2h = 1.0 / (2.0 * a.h);
    const double Lx_y = DyT(a.lx, N, pitch, i2h, ia, ib);
    const double Lx_x = DxT(a.lx, N, pitch, i2h, ia, ib);
    const double Ly_x = DxT(a.ly, N, pitch, i2h, ia, ib);
    const double Ly_y = DyT(a.ly, N, pitch, i2h, ia, ib);
    const double jzb = Lx_y - Ly_x;
    double nb = a.nb[i], txxb = a.txxb[i] + Ly_x, tyyb = a.tyyb[i] - Lx_y;
    const double txyb = a.txyb[i] - Lx_x + Ly_y;
    double pb = 0.0;
    const bool in = interior(N, ia, ib);
    if (in) pb = a.gnb[i] + DxT(a.psxb, N, pitch, i2h, ia, ib) + DyT(a.psyb, N, pitch, i2h, ia, ib);
    if (jzb != 0.0 && a.n[i] > 0.0) {
        const double gg = 1.0 + a.psi[i], n = a.n[i];
        nb += jzb * (1.0 - gg * gg) / (2.0 * gg * gg);
        txxb += jzb * 0.5;
        tyyb += jzb * 0.5;
        pb += -jzb * n / (gg * gg * gg);
    }
    a.nb[i] = nb;
    a.txxb[i] = txxb;
    a.tyyb[i] = tyyb;
    a.txyb[i] = txyb;
    if (in) a.psib[i] += pb;
    a.jzb[i] = jzb;
}

// One partial sum per segment: sum over its nodes of jzb * d n_b / d theta
// without the xi factor exp(-(xi - xi_c)^2 / sigma_z^2) (applied per theta).
// seg = [beam, theta, begin, end]; Gaussian segments index the dense node
// numbering, radial-bin segments the node list grouped by bin.
__global__ __launch_bounds__(256) void k_theta_seg(int N, double L, double h, int pitch,
                                                   const int32_t* __restrict__ seg,
                                                   const int32_t* __restrict__ bin_nodes,
                                                   const double* __restrict__ jzb, BeamSet B,
                                                   double* __restrict__ part) {
    __shared__ double red[4];
    const int beam = seg[4 * blockIdx.x], i0 = seg[4 * blockIdx.x + 2], i1 = seg[4 * blockIdx.x + 3];
    const bool gauss = B.kind[beam] == 0;
    const double x0 = B.x0[beam], y0 = B.y0[beam], sr2 = B.sr[beam] * B.sr[beam];
    double s = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        const int node = gauss ? i : bin_nodes[i];
        const int b = node / (N + 1), a = node - b * (N + 1);
        double v = jzb[(size_t)b * pitch + a];
        if (gauss) {
            const double rx = -L + a * h - x0, ry = -L + b * h - y0;
            v *= exp(-(rx * rx + ry * ry) / sr2);
        }
        s += v;
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// theta_bar[t] += exp(-(xi - xi_c)^2 / sigma_z^2) * (its segments' partials in
// order), nothing for xi < 0 (no driver before the xi axis starts).
__global__ void k_theta_reduce(int n_theta, const int32_t* __restrict__ seg,
                               const int32_t* __restrict__ seg_first,
                               const double* __restrict__ part, const double* __restrict__ st,
                               BeamSet B, double* __restrict__ theta_bar) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_theta) return;
    const int s0 = seg_first[t], s1 = seg_first[t + 1];
    const double xi = st[0];
    if (s1 <= s0 || xi < 0.0) return;
    double s = 0.0;
    for (int k = s0; k < s1; ++k) s += part[k];
    const int beam = seg[4 * s0];
    const double lz = (xi - B.xc[beam]) * (xi - B.xc[beam]) / (B.sz[beam] * B.sz[beam]);
    theta_bar[t] += s * exp(-lz);
}

// jxb, jyb += adjoints of f_Ez = -(D_x jx + D_y jy) and f_Bz = D_x jy - D_y jx.
__global__ void k_EB_adj(int N, double h, int pitch, const double* __restrict__ lE,
                         const double* __restrict__ lB, double* __restrict__ jxb,
                         double* __restrict__ jyb) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const double i2h = 1.0 / (2.0 * h);
    const size_t g = (size_t)b * pitch + a;
    jxb[g] += -DxT(lE, N, pitch, i2h, a, b) - DyT(lB, N, pitch, i2h, a, b);
    jyb[g] += -DyT(lE, N, pitch, i2h, a, b) + DxT(lB, N, pitch, i2h, a, b);
}

struct DepAdjArgs {
    int N;
    double L, h, wd;
    int pitch;
    const double *x, *y, *px, *py;
    const int32_t* start;
    const double* psi;
    const double *jxb, *jyb, *txxb, *txyb, *tyyb;  // node adjoints of the moments
    const double* gb;                              // adjoint of g_i from the push
    double *xb, *yb, *pxb, *pyb;                   // added to (cell order)
    double* psib_dep;                              // out: node adjoint of psi through g_i
};

// Deposits of j and T reversed (gathers of the node adjoints with the CIC
// position derivatives; V = p / g), then the gather g = 1 + psi reversed.
__global__ __launch_bounds__(256) void k_dep_adj(DepAdjArgs a) {
    __shared__ double corner[TC * TC][4];
    int tbx, tby;
    tile_of_block(tbx, tby);
    const int a0 = tbx * TN, b0 = tby * TN;
    const int N = a.N, pitch = a.pitch;
    const double h = a.h, L = a.L, wd = a.wd;
    for (int c = threadIdx.x; c < TC * TC; c += blockDim.x) {
        const int cy = c / TC, cx = c - cy * TC;
        const int ga = a0 - 1 + cx, gb = b0 - 1 + cy;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        {
            // the cell clamped into the grid, its particle range emptied when
            // it lies outside (no load behind a lane-dependent branch)
            const bool valid = ga >= 0 && ga < N && gb >= 0 && gb < N;
            const int gac = min(max(ga, 0), N - 1), gbc = min(max(gb, 0), N - 1);
            const bool own = cx >= 1 && cy >= 1;
            const int cell = gbc * N + gac;
            const size_t g = (size_t)gbc * pitch + gac;
            const double* A[5] = {a.jxb, a.jyb, a.txxb, a.txyb, a.tyyb};
            double A00[5], A10[5], A01[5], A11[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                A00[m] = A[m][g];
                A10[m] = A[m][g + 1];
                A01[m] = A[m][g + pitch];
                A11[m] = A[m][g + pitch + 1];
            }
            const double p00 = a.psi[g], p10 = a.psi[g + 1], p01 = a.psi[g + pitch],
                         p11 = a.psi[g + pitch + 1];
            const int k0 = a.start[cell], k1 = k0 + (a.start[cell + 1] - k0) * (valid ? 1 : 0);
            for (int kb = k0; kb < k1; kb += kAdjBatch) {
            const int cnt = min(kAdjBatch, k1 - kb);
            // the batch's particles, the push's adjoint of g and the current
            // sums of the particle adjoints, all loads issued together
            double xv[kAdjBatch], yv[kAdjBatch], pxv[kAdjBatch], pyv[kAdjBatch], gv[kAdjBatch];
            double xo[kAdjBatch], yo[kAdjBatch], pxo[kAdjBatch], pyo[kAdjBatch];
#pragma unroll
            for (int ib = 0; ib < kAdjBatch; ++ib) {
                const int kk = kb + min(ib, cnt - 1);
                xv[ib] = a.x[kk];
                yv[ib] = a.y[kk];
                pxv[ib] = a.px[kk];
                pyv[ib] = a.py[kk];
                gv[ib] = a.gb[kk];
                xo[ib] = a.xb[kk];
                yo[ib] = a.yb[kk];
                pxo[ib] = a.pxb[kk];
                pyo[ib] = a.pyb[kk];
            }
#pragma unroll
            for (int ib = 0; ib < kAdjBatch; ++ib) {
                if (ib >= cnt) break;
                const int k = kb + ib;
                const double ddx = (xv[ib] + L) / h - ga, ddy = (yv[ib] + L) / h - gb;
                const Interp gp = interp(p00, p10, p01, p11, ddx, ddy, h);
                const double gi = 1.0 + gp.v;
                const double vx = pxv[ib] / gi, vy = pyv[ib] / gi;
                const double q[5] = {vx, vy, vx * vx, vx * vy, vy * vy};
                double qb[5], xbar = 0.0, ybar = 0.0;
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    const Interp t = interp(A00[m], A10[m], A01[m], A11[m], ddx, ddy, h);
                    qb[m] = wd * t.v;
                    xbar += wd * q[m] * t.dx;
                    ybar += wd * q[m] * t.dy;
                }
                const double vxb = qb[0] + 2.0 * vx * qb[2] + vy * qb[3];
                const double vyb = qb[1] + vx * qb[3] + 2.0 * vy * qb[4];
                const double gtot = gv[ib] - (vxb * vx + vyb * vy) / gi;
                xbar += gtot * gp.dx;
                ybar += gtot * gp.dy;
                if (own) {
                    a.pxb[k] = pxo[ib] + vxb / gi;
                    a.pyb[k] = pyo[ib] + vyb / gi;
                    a.xb[k] = xo[ib] + xbar;
                    a.yb[k] = yo[ib] + ybar;
                }
                s[0] += gtot * (1.0 - ddx) * (1.0 - ddy);
                s[1] += gtot * ddx * (1.0 - ddy);
                s[2] += gtot * (1.0 - ddx) * ddy;
                s[3] += gtot * ddx * ddy;
            }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) corner[c][r] = s[r];
    }
    __syncthreads();
    double* out[1] = {a.psib_dep};
    tile_node_sums<1>(corner, a0, b0, N, pitch, out);
}

// psib = psib + psib_dep on the interior nodes, 0 on the boundary (the psi
// adjoint solve's right-hand side).
__global__ void k_add_interior(int N, int pitch, double* __restrict__ dst,
                               const double* __restrict__ add) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a > N) return;
    const size_t g = (size_t)b * pitch + a;
    dst[g] = interior(N, a, b) ? dst[g] + add[g] : 0.0;
}

// Deposit of n* reversed (f_psi = n* - n0 on the interior nodes, so the node
// adjoint of n* is nb + lambda_psi there), then the particle adjoints are
// written back in particle-ID order.
__global__ void k_n_adj_out(int64_t P, int N, double L, double h, double wd, int pitch,
                            const double* __restrict__ x, const double* __restrict__ y,
                            const int32_t* __restrict__ id, const double* __restrict__ nb,
                            const double* __restrict__ lpsi, const double* __restrict__ xb,
                            const double* __restrict__ yb, const double* __restrict__ pxb,
                            const double* __restrict__ pyb, double* __restrict__ adj_out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    int a, b;
    double ddx, ddy;
    cic(x[j], L, h, N, a, ddx);
    cic(y[j], L, h, N, b, ddy);
    const size_t g = (size_t)b * pitch + a;
    auto tot = [&](size_t q, int qa, int qb) {
        return nb[q] + (interior(N, qa, qb) ? lpsi[q] : 0.0);
    };
    const Interp t = interp(tot(g, a, b), tot(g + 1, a + 1, b), tot(g + pitch, a, b + 1),
                            tot(g + pitch + 1, a + 1, b + 1), ddx, ddy, h);
    const int64_t k = id[j];
    adj_out[k] = xb[j] + wd * t.dx;
    adj_out[P + k] = yb[j] + wd * t.dy;
    adj_out[2 * P + k] = pxb[j];
    adj_out[3 * P + k] = pyb[j];
}

__global__ void k_zero(double* p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

dim3 node_grid(int N) { return dim3((N + 1 + 127) / 128, N + 1); }

}  // namespace

wandqs_status adj_zero_solutions(wandqs_ctx* c) {
    const size_t nn = (size_t)(c->N + 1) * c->lev[0].pitch;
    AdjBuffers& A = c->adj;
    double* arr[5] = {A.lx, A.ly, A.lE, A.lB, A.lpsi};
    for (double* p : arr) {
        ProfScope ps(c, "k_zero", 8.0 * nn);
        WQ_KLAUNCH(ps, k_zero, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream, p, nn);
    }
    if (c->n_theta > 0) {
        ProfScope ps(c, "k_zero", 8.0 * c->n_theta);
        WQ_KLAUNCH(ps, k_zero, dim3((unsigned)((c->n_theta + 255) / 256)), dim3(256), 0, c->stream,
                           A.theta_bar, (size_t)c->n_theta);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status slice_adjoint(wandqs_ctx* c, const TapeSlot& ts, const double* d_field_bar,
                            const double* probe_w) {
    hipStream_t s = c->stream;
    const int N = c->N, pitch = c->lev[0].pitch;
    const double nnd = (double)(N + 1) * (N + 1);
    const double P = (double)c->P;
    const double wd = c->cfg.n0 / c->ppc;
    const dim3 ng = node_grid(N);
    const int nt = (N + 1 + TN - 1) / TN;
    AdjBuffers& A = c->adj;
    wandqs_status st;

    {  // push
        PushAdjArgs a{N, c->L, c->h, pitch, c->P, ts.pa[0], ts.pa[1], ts.pa[2], ts.pa[3], ts.pid,
                      ts.start, ts.fields[0], ts.fields[3], ts.fields[4], ts.fields[2], ts.st,
                      A.adj_id, A.xb, A.yb, A.pxb, A.pyb, A.gb, A.Gxb, A.Gyb, A.Bxb, A.Byb, A.Bzb};
        ProfScope ps(c, "k_push_adj<16>", P * 108.0 + nnd * 76.0);
        WQ_KLAUNCH(ps, k_push_adj, dim3(nt, nt), dim3(256), 0, s, a);
    }
    {
        ProfScope ps(c, "k_grad_adj", nnd * 64.0);
        WQ_KLAUNCH(ps, k_grad_adj, ng, dim3(128), 0, s, N, c->h, pitch, A.Gxb, A.Gyb, A.psib,
                           A.Bxb, A.Byb, A.Bzb, A.Ezb);
    }
    double* Fb[5] = {A.psib, A.Ezb, A.Bzb, A.Bxb, A.Byb};
    if (d_field_bar) {
        FieldBar fb{{Fb[0], Fb[1], Fb[2], Fb[3], Fb[4]}};
        ProfScope ps(c, "k_field_seed", nnd * 120.0);
        WQ_KLAUNCH(ps, k_field_seed, ng, dim3(128), 0, s, N, pitch, d_field_bar, fb);
    }
    for (size_t k = 0; k < c->probes.size(); ++k)
        if (probe_w && probe_w[k] != 0.0 && (st = probe_seed(c, (int)k, probe_w[k], Fb)) != WANDQS_OK)
            return st;
    WQ_LAUNCH_CHECK();

    // B_perp: lambda = (L_h - k2)^-1 Bbar (warm start: the previous slice's lambda)
    SolveResult res;
    double* ul[2] = {A.lx, A.ly};
    double* fl[2] = {A.Bxb, A.Byb};
    if ((st = mg_solve(c, kSolveBperpAdj, 2, true, ul, fl, ts.k2, &res)) != WANDQS_OK) return st;

    AsmAdjArgs aa{N, c->L, c->h, pitch, ts.mom[0], ts.mom[1], ts.mom[2], ts.mom[3], ts.mom[4],
                  ts.mom[5], ts.fields[0], ts.fields[1], ts.fields[2], ts.fields[3], ts.fields[4],
                  A.lx, A.ly, A.nb, A.jxb, A.jyb, A.txxb, A.txyb, A.tyyb, A.psxb, A.psyb, A.gnb,
                  A.Ezb, A.Bzb, A.psib, A.jzb};
    {
        ProfScope ps(c, "k_asm_adj_local", nnd * 200.0);
        WQ_KLAUNCH(ps, k_asm_adj_local, ng, dim3(128), 0, s, aa);
    }
    {
        ProfScope ps(c, "k_asm_adj_diff", nnd * 152.0);
        WQ_KLAUNCH(ps, k_asm_adj_diff, ng, dim3(128), 0, s, aa);
    }
    if (c->n_seg > 0) {
        {
            ProfScope ps(c, "k_theta_seg", nnd * 8.0);
            WQ_KLAUNCH(ps, k_theta_seg, dim3(c->n_seg), dim3(256), 0, s, N, c->L, c->h, pitch,
                               A.seg, A.bin_nodes, A.jzb, c->beamset, A.theta_part);
        }
        {
            ProfScope ps(c, "k_theta_reduce", 8.0 * c->n_seg + 16.0 * c->n_theta);
            WQ_KLAUNCH(ps, k_theta_reduce, dim3((c->n_theta + 255) / 256), dim3(256), 0, s,
                               c->n_theta, A.seg, A.seg_first, A.theta_part, ts.st, c->beamset,
                               A.theta_bar);
        }
    }
    WQ_LAUNCH_CHECK();

    // Ez, Bz Poisson solves reversed
    double* ue[2] = {A.lE, A.lB};
    double* fe[2] = {A.Ezb, A.Bzb};
    if ((st = mg_solve(c, kSolveEBAdj, 2, false, ue, fe, nullptr, &res)) != WANDQS_OK) return st;
    {
        ProfScope ps(c, "k_EB_adj", nnd * 48.0);
        WQ_KLAUNCH(ps, k_EB_adj, ng, dim3(128), 0, s, N, c->h, pitch, A.lE, A.lB, A.jxb, A.jyb);
    }
    {
        DepAdjArgs d{N, c->L, c->h, wd, pitch, ts.pa[0], ts.pa[1], ts.pa[2], ts.pa[3], ts.start,
                     ts.fields[0], A.jxb, A.jyb, A.txxb, A.txyb, A.tyyb, A.gb, A.xb, A.yb, A.pxb,
                     A.pyb, A.psib_dep};
        ProfScope ps(c, "k_dep_adj<16>", P * 104.0 + nnd * 60.0);
        WQ_KLAUNCH(ps, k_dep_adj, dim3(nt, nt), dim3(256), 0, s, d);
    }
    {
        ProfScope ps(c, "k_add_interior", nnd * 24.0);
        WQ_KLAUNCH(ps, k_add_interior, ng, dim3(128), 0, s, N, pitch, A.psib, A.psib_dep);
    }
    WQ_LAUNCH_CHECK();

    // psi Poisson solve reversed, then the n* deposit
    double* up[2] = {A.lpsi, nullptr};
    double* fp[2] = {A.psib, nullptr};
    if ((st = mg_solve(c, kSolvePsiAdj, 1, false, up, fp, nullptr, &res)) != WANDQS_OK) return st;
    {
        ProfScope ps(c, "k_n_adj_out", P * 84.0 + nnd * 16.0);
        WQ_KLAUNCH(ps, k_n_adj_out, dim3((unsigned)((c->P + 255) / 256)), dim3(256), 0, s, c->P,
                           N, c->L, c->h, wd, pitch, ts.pa[0], ts.pa[1], ts.pid, A.nb, A.lpsi, A.xb,
                           A.yb, A.pxb, A.pyb, A.adj_id);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace wq
