// Laser envelope driver: the paraxial envelope equation (eq. (20)) advanced in
// t plane by plane, and the node arrays through which the plasma feels the
// envelope (|A-hat|^2 and its gradient for the ponderomotive terms of eqs.
// (7), (9) and (19)).
//
// Envelope planes: A-hat at xi_m = m dxi0 (m = 0 .. laser_nz - 1), complex
// (double2: re, im) in the padded node layout, [laser_nz][(N+1) * pitch].  Two
// sets: las_env[las_cur] holds the planes at t (the plasma sees them), the
// other one receives the planes at t + dt.
//
// One time step of a plane j, with a0 = A-hat(t, xi_j), a1 = A-hat(t + dt,
// xi_j) and p0, p1 the same on the plane ahead (zero ahead of plane 0), is eq.
// (20) centred in t with the xi-derivative taken backward (the plane ahead is
// already at t + dt when the sweep reaches plane j):
//   L_h a1 - (chi + beta - i gam) a1 = (chi - beta + i gam) a0 - L_h a0 - beta (p1 - p0),
//   beta = 4/(dt dxi0), gam = 4 k0/dt,  a1 = 0 on the boundary,
// chi = n* / (1 + psi) at the nodes.  It is solved by a complex multigrid:
// V(nu_pre, nu_post) cycles of red-black Gauss-Seidel on the levels above
// kLasCoarse (per level one fused down pass -- the pre-sweeps, the residual
// and its full weighting, on LDS tiles with halos -- and one fused up pass --
// bilinear prolongation and the post-sweeps) and one workgroup that runs the rest of
// the V-cycle (levels kLasCoarse^2 .. 2^2, exact on the single interior node of
// 2^2) in LDS; the context's stop rule (mg_rtol, mg_atol, the rounding floor)
// on the real and imaginary parts, from the guess a0.
#include <algorithm>
#include <cmath>
#include <limits>

#include "wq_common.h"

namespace wq {
namespace {

constexpr int kLasCoarse = 32;      // levels at or below this run in one workgroup
constexpr int kLasThreads = 1024;   // that workgroup
constexpr int kLasLdsNodes = 33 * 33 + 17 * 17 + 9 * 9 + 5 * 5 + 3 * 3;
constexpr int kNormThreads = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscl(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = 1.0 / (b.x * b.x + b.y * b.y);
    return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// |A-hat|^2 at slice position xi = st[0] on every node: the planes around xi
// interpolated linearly, planes outside [0, nz) taken as zero.
__global__ void k_las_a2(int N, int pitch, size_t plane, int nz, double dxi0,
                         const double* __restrict__ st, const double2* __restrict__ env,
                         double* __restrict__ a2) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (a > N) return;
    const size_t i = (size_t)b * pitch + a;
    const double t = st[0] / dxi0;
    const double mf = floor(t);
    const double w = t - mf;
    double v = 0.0;
    if (mf >= 0.0 && mf < nz) {
        const double2 e = env[(size_t)mf * plane + i];
        v += (1.0 - w) * (e.x * e.x + e.y * e.y);
    }
    if (mf + 1.0 >= 0.0 && mf + 1.0 < nz) {
        const double2 e = env[(size_t)(mf + 1.0) * plane + i];
        v += w * (e.x * e.x + e.y * e.y);
    }
    a2[i] = v;
}

// Level-0 problem of one plane: the shift k = chi + beta - i gam, the
// right-hand side f (interior nodes) and the initial iterate (zero on the
// boundary): a0 plus the plane ahead's change over the step, p1 - p0 (the
// envelope changes smoothly from plane to plane), or a0 on the first plane.
// chi, p0 and p1 may be null (vacuum, first plane).
__global__ void k_las_rhs(int N, double h, int pitch, double beta, double gam,
                          const double* __restrict__ chi, const double2* __restrict__ a0,
                          const double2* __restrict__ p0, const double2* __restrict__ p1,
                          double2* __restrict__ f, double2* __restrict__ k, double2* __restrict__ u) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (a > N) return;
    const size_t i = (size_t)b * pitch + a;
    const double x = chi ? chi[i] : 0.0;
    k[i] = make_double2(x + beta, -gam);
    if (a == 0 || b == 0 || a == N || b == N) {
        f[i] = make_double2(0.0, 0.0);
        u[i] = make_double2(0.0, 0.0);
        return;
    }
    const double ih2 = 1.0 / (h * h);
    const double2 c = a0[i];
    const double2 lap = cscl(ih2, csub(cadd(cadd(a0[i - 1], a0[i + 1]), cadd(a0[i - pitch], a0[i + pitch])),
                                       cscl(4.0, c)));
    double2 d = make_double2(0.0, 0.0);
    if (p1) d = p1[i];
    if (p0) d = csub(d, p0[i]);
    f[i] = csub(csub(cmul(make_double2(x - beta, gam), c), lap), cscl(beta, d));
    u[i] = cadd(c, d);
}

__device__ __forceinline__ double2 resid_at(const double2* u, const double2* f, const double2* k,
                                            size_t i, int pitch, double ih2) {
    const double2 c = u[i];
    const double2 lap = cscl(ih2, csub(cadd(cadd(u[i - 1], u[i + 1]), cadd(u[i - pitch], u[i + pitch])),
                                       cscl(4.0, c)));
    return csub(f[i], csub(lap, cmul(k[i], c)));
}

// Tiles of the fused passes: kLTX x kLTY owned nodes, loaded with a halo of
// up to kLH nodes into LDS (u, f and the shift k: 16 B each per node).
constexpr int kLTX = 32, kLTY = 16, kLH = 8;
constexpr int kLRX = kLTX + 2 * kLH, kLRY = kLTY + 2 * kLH;
constexpr int kLTThreads = 512;
constexpr int kLIt = (kLRX * kLRY + kLTThreads - 1) / kLTThreads;  // tile nodes per thread

// Node q of this thread in a tile of RW x RH nodes at (ax0, by0): its LDS
// slot, its grid node and its index clamped into the grid (threads past the
// tile redo its last node).  The tile loads read every node unconditionally
// and mask the values (every value loaded is finite): a load the compiler
// moves behind a lane-dependent branch is waited for before the branch ends,
// which would serialize the tile's loads.
struct LasTileNode {
    int lx, ly, a, b;
    size_t g;
    bool in, inner;  // inside [0, n]^2; interior
};
__device__ __forceinline__ LasTileNode las_node(int q, int RW, int RH, int ax0, int by0, int n,
                                                int pitch) {
    LasTileNode nd;
    const int t = min((int)threadIdx.x + q * kLTThreads, RW * RH - 1);
    nd.lx = t % RW;
    nd.ly = t / RW;
    nd.a = ax0 + nd.lx;
    nd.b = by0 + nd.ly;
    nd.in = nd.a >= 0 && nd.b >= 0 && nd.a <= n && nd.b <= n;
    nd.inner = nd.a > 0 && nd.b > 0 && nd.a < n && nd.b < n;
    nd.g = (size_t)min(max(nd.b, 0), n) * pitch + min(max(nd.a, 0), n);
    return nd;
}

// Red-black Gauss-Seidel sweeps on the tile's region in LDS: a node with its
// four neighbours in the region and inside the domain takes (sum of the
// neighbours - h^2 f) / (4 + h^2 k); the region's edge keeps its loaded values,
// so each half sweep leaves one more layer inside it exact.
__device__ void tile_sweeps(double2 (*U)[kLRX], const double2 (*F)[kLRX], const double2 (*K)[kLRX],
                            int RW, int RH, int ax0, int by0, int n, double h2, int nu) {
    // a thread visits the same nodes in every half sweep: their 1 / (4 + h^2 k)
    // formed once, in registers
    double2 idg[kLIt];
#pragma unroll
    for (int q = 0; q < kLIt; ++q) {
        const int t = min((int)threadIdx.x + q * kLTThreads, RW * RH - 1);
        const double2 kk = K[t / RW][t % RW];
        idg[q] = cdiv(make_double2(1.0, 0.0), make_double2(4.0 + h2 * kk.x, h2 * kk.y));
    }
    for (int s = 0; s < nu; ++s)
        for (int color = 0; color < 2; ++color) {
#pragma unroll
            for (int q = 0; q < kLIt; ++q) {
                const int t = threadIdx.x + q * kLTThreads;
                if (t >= RW * RH) break;
                const int lx = t % RW, ly = t / RW;
                const int a = ax0 + lx, b = by0 + ly;
                if (lx < 1 || ly < 1 || lx > RW - 2 || ly > RH - 2) continue;
                if (a < 1 || b < 1 || a > n - 1 || b > n - 1 || ((a + b) & 1) != color) continue;
                const double2 nb = cadd(cadd(U[ly][lx - 1], U[ly][lx + 1]), cadd(U[ly - 1][lx], U[ly + 1][lx]));
                U[ly][lx] = cmul(csub(nb, cscl(h2, F[ly][lx])), idg[q]);
            }
            __syncthreads();
        }
}

// Down pass of one level: nu red-black sweeps of (L_h - k) u = f on the tile
// (halo 2 nu + 2), the smoothed owned nodes into um, and, for the coarse nodes
// the tile owns, the full weighting of the residual into the coarse f and a
// zero coarse correction.  u_in is read only (tiles never see each other's
// writes within a pass).
__global__ __launch_bounds__(kLTThreads) void k_las_down(int n, double h, int pitch, int nu,
                                                         const double2* __restrict__ u_in,
                                                         const double2* __restrict__ f,
                                                         const double2* __restrict__ k,
                                                         double2* __restrict__ um, int pc,
                                                         double2* __restrict__ fc,
                                                         double2* __restrict__ uc) {
    __shared__ double2 U[kLRY][kLRX], F[kLRY][kLRX], K[kLRY][kLRX];
    const int H = 2 * nu + 2;
    const int x0 = blockIdx.x * kLTX, y0 = blockIdx.y * kLTY;
    const int ax0 = x0 - H, by0 = y0 - H, RW = kLTX + 2 * H, RH = kLTY + 2 * H;
    const double2 z = make_double2(0.0, 0.0);
    {
        double2 uu[kLIt], ff[kLIt], kk[kLIt];
#pragma unroll
        for (int q = 0; q < kLIt; ++q) {
            const LasTileNode nd = las_node(q, RW, RH, ax0, by0, n, pitch);
            const double2 uv = u_in[nd.g], fv = f[nd.g], kv = k[nd.g];
            uu[q] = cscl(nd.inner ? 1.0 : 0.0, uv);
            ff[q] = cscl(nd.in ? 1.0 : 0.0, fv);
            kk[q] = cscl(nd.in ? 1.0 : 0.0, kv);
        }
#pragma unroll
        for (int q = 0; q < kLIt; ++q) {
            const LasTileNode nd = las_node(q, RW, RH, ax0, by0, n, pitch);
            U[nd.ly][nd.lx] = uu[q];
            F[nd.ly][nd.lx] = ff[q];
            K[nd.ly][nd.lx] = kk[q];
        }
    }
    __syncthreads();
    const double h2 = h * h;
    tile_sweeps(U, F, K, RW, RH, ax0, by0, n, h2, nu);
    for (int t = threadIdx.x; t < kLTX * kLTY; t += kLTThreads) {
        const int a = x0 + t % kLTX, b = y0 + t / kLTX;
        if (a <= n && b <= n) um[(size_t)b * pitch + a] = U[b - by0][a - ax0];
    }
    const int nc = n / 2;
    const double ih2 = 1.0 / h2;
    for (int t = threadIdx.x; t < (kLTX / 2) * (kLTY / 2); t += kLTThreads) {
        const int I = x0 / 2 + t % (kLTX / 2), J = y0 / 2 + t / (kLTX / 2);
        if (I > nc || J > nc) continue;
        double2 acc = z;
        if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1) {
            const double w[3] = {1.0, 2.0, 1.0};
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx) {
                    const int lx = 2 * I + sx - ax0, ly = 2 * J + sy - by0;
                    const double2 c = U[ly][lx];
                    const double2 lap = cscl(ih2, csub(cadd(cadd(U[ly][lx - 1], U[ly][lx + 1]),
                                                            cadd(U[ly - 1][lx], U[ly + 1][lx])),
                                                       cscl(4.0, c)));
                    const double2 r = csub(F[ly][lx], csub(lap, cmul(K[ly][lx], c)));
                    acc = cadd(acc, cscl(w[sx + 1] * w[sy + 1], r));
                }
            acc = cscl(1.0 / 16.0, acc);
        }
        fc[(size_t)J * pc + I] = acc;
        uc[(size_t)J * pc + I] = z;
    }
}

// Up pass of one level: um plus the bilinear interpolation of the coarse
// correction on the tile (halo 2 nu), nu red-black sweeps, the owned nodes
// into u_out.
__global__ __launch_bounds__(kLTThreads) void k_las_up(int n, double h, int pitch, int nu,
                                                       const double2* __restrict__ um,
                                                       const double2* __restrict__ f,
                                                       const double2* __restrict__ k, int pc,
                                                       const double2* __restrict__ uc,
                                                       double2* __restrict__ u_out) {
    __shared__ double2 U[kLRY][kLRX], F[kLRY][kLRX], K[kLRY][kLRX];
    const int H = 2 * nu;
    const int x0 = blockIdx.x * kLTX, y0 = blockIdx.y * kLTY;
    const int ax0 = x0 - H, by0 = y0 - H, RW = kLTX + 2 * H, RH = kLTY + 2 * H;
    {
        const int nc = n / 2;
        double2 uu[kLIt], ff[kLIt], kk[kLIt];
#pragma unroll
        for (int q = 0; q < kLIt; ++q) {
            const LasTileNode nd = las_node(q, RW, RH, ax0, by0, n, pitch);
            const double2 fv = f[nd.g], kv = k[nd.g], mv = um[nd.g];
            // the coarse cell's four corners (indices clamped into the coarse
            // grid; a node outside the interior is masked below)
            const int I = min(max(nd.a >> 1, 0), nc - 1), J = min(max(nd.b >> 1, 0), nc - 1);
            const size_t cc = (size_t)J * pc + I;
            const double2 c00 = uc[cc], c10 = uc[cc + 1], c01 = uc[cc + pc], c11 = uc[cc + pc + 1];
            // the four bilinear forms, one selected by the node's parity (no
            // branch, so the next node's loads are not held back)
            const bool ox = nd.a & 1, oy = nd.b & 1;
            const double2 e_oe = cscl(0.5, cadd(c00, c10)), e_eo = cscl(0.5, cadd(c00, c01));
            const double2 e_oo = cscl(0.25, cadd(cadd(c00, c10), cadd(c01, c11)));
            const double2 e_o = oy ? e_oo : e_oe, e_e = oy ? e_eo : c00;
            const double2 e = ox ? e_o : e_e;
            uu[q] = cscl(nd.inner ? 1.0 : 0.0, cadd(mv, e));
            ff[q] = cscl(nd.in ? 1.0 : 0.0, fv);
            kk[q] = cscl(nd.in ? 1.0 : 0.0, kv);
        }
#pragma unroll
        for (int q = 0; q < kLIt; ++q) {
            const LasTileNode nd = las_node(q, RW, RH, ax0, by0, n, pitch);
            U[nd.ly][nd.lx] = uu[q];
            F[nd.ly][nd.lx] = ff[q];
            K[nd.ly][nd.lx] = kk[q];
        }
    }
    __syncthreads();
    tile_sweeps(U, F, K, RW, RH, ax0, by0, n, h * h, nu);
    for (int t = threadIdx.x; t < kLTX * kLTY; t += kLTThreads) {
        const int a = x0 + t % kLTX, b = y0 + t / kLTX;
        if (a <= n && b <= n) u_out[(size_t)b * pitch + a] = U[b - by0][a - ax0];
    }
}

// Full weighting of the shift k onto the interior coarse nodes.
__global__ void k_las_krestrict(int nc, int pf, const double2* __restrict__ kf, int pc,
                                double2* __restrict__ kc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
    if (I > nc) return;
    double2 s = make_double2(0.0, 0.0);
    if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1) {
        const size_t c = (size_t)(2 * J) * pf + 2 * I;
        s = cadd(cscl(4.0, kf[c]), cadd(cscl(2.0, cadd(cadd(kf[c - 1], kf[c + 1]), cadd(kf[c - pf], kf[c + pf]))),
                                        cadd(cadd(kf[c - pf - 1], kf[c - pf + 1]), cadd(kf[c + pf - 1], kf[c + pf + 1]))));
        s = cscl(1.0 / 16.0, s);
    }
    kc[(size_t)J * pc + I] = s;
}

// The V-cycle from level n0 (<= kLasCoarse) down to 2^2 in one workgroup, in
// LDS: u (the initial iterate), f and k of level n0 are read from global
// memory, u is written back.  Level q of the chain is dense (n+1)^2 at offset
// off[q].
__global__ __launch_bounds__(kLasThreads) void k_las_coarse(int n0, double h0, int pitch, int nu1,
                                                            int nu2, double2* __restrict__ ug,
                                                            const double2* __restrict__ fg,
                                                            const double2* __restrict__ kg) {
    __shared__ double2 U[kLasLdsNodes], F[kLasLdsNodes], K[kLasLdsNodes];
    int off[6], nq[6];
    double hq[6];
    int Q = 0;
    {
        int o = 0;
        for (int n = n0; n >= 2; n >>= 1, ++Q) {
            off[Q] = o;
            nq[Q] = n;
            hq[Q] = h0 * (double)(n0 / n);
            o += (n + 1) * (n + 1);
        }
    }
    const int tid = threadIdx.x;
    {
        const int m = n0 + 1;
        for (int i = tid; i < m * m; i += kLasThreads) {
            const size_t g = (size_t)(i / m) * pitch + i % m;
            U[i] = ug[g];
            F[i] = fg[g];
            K[i] = kg[g];
        }
    }
    __syncthreads();
    // shifts of the coarser levels: full weighting
    for (int q = 1; q < Q; ++q) {
        const int n = nq[q], m = n + 1, mf = nq[q - 1] + 1;
        double2* Kc = K + off[q];
        const double2* Kf = K + off[q - 1];
        for (int i = tid; i < m * m; i += kLasThreads) {
            const int I = i % m, J = i / m;
            double2 s = make_double2(0.0, 0.0);
            if (I >= 1 && J >= 1 && I <= n - 1 && J <= n - 1) {
                const int c = (2 * J) * mf + 2 * I;
                s = cadd(cscl(4.0, Kf[c]), cadd(cscl(2.0, cadd(cadd(Kf[c - 1], Kf[c + 1]), cadd(Kf[c - mf], Kf[c + mf]))),
                                                cadd(cadd(Kf[c - mf - 1], Kf[c - mf + 1]), cadd(Kf[c + mf - 1], Kf[c + mf + 1]))));
                s = cscl(1.0 / 16.0, s);
            }
            Kc[i] = s;
        }
        __syncthreads();
    }
    auto smooth = [&](int q, int nu) {
        const int n = nq[q], m = n + 1;
        const double h2 = hq[q] * hq[q];
        double2* u = U + off[q];
        const double2* f = F + off[q];
        const double2* k = K + off[q];
        for (int s = 0; s < nu; ++s)
            for (int color = 0; color < 2; ++color) {
                for (int i = tid; i < m * m; i += kLasThreads) {
                    const int a = i % m, b = i / m;
                    if (a < 1 || b < 1 || a > n - 1 || b > n - 1 || ((a + b) & 1) != color) continue;
                    const double2 nb = cadd(cadd(u[i - 1], u[i + 1]), cadd(u[i - m], u[i + m]));
                    u[i] = cdiv(csub(nb, cscl(h2, f[i])), make_double2(4.0 + h2 * k[i].x, h2 * k[i].y));
                }
                __syncthreads();
            }
    };
    // down
    for (int q = 0; q + 1 < Q; ++q) {
        smooth(q, nu1);
        const int nf = nq[q], mf = nf + 1, n = nq[q + 1], m = n + 1;
        const double ih2 = 1.0 / (hq[q] * hq[q]);
        const double2 *u = U + off[q], *f = F + off[q], *k = K + off[q];
        for (int i = tid; i < m * m; i += kLasThreads) {
            const int I = i % m, J = i / m;
            double2 s = make_double2(0.0, 0.0);
            if (I >= 1 && J >= 1 && I <= n - 1 && J <= n - 1) {
                const int c = (2 * J) * mf + 2 * I;
                const double w[3] = {1.0, 2.0, 1.0};
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx)
                        s = cadd(s, cscl(w[dx + 1] * w[dy + 1], resid_at(u, f, k, c + dy * mf + dx, mf, ih2)));
                s = cscl(1.0 / 16.0, s);
            }
            F[off[q + 1] + i] = s;
            U[off[q + 1] + i] = make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
    // the 2^2 level: one interior node with four zero neighbours
    if (tid == 0) {
        const int i = off[Q - 1] + 4;  // node (1, 1) of a 3 x 3 array
        const double h2 = hq[Q - 1] * hq[Q - 1];
        const double2 k = K[i];
        U[i] = cdiv(cscl(-h2, F[i]), make_double2(4.0 + h2 * k.x, h2 * k.y));
    }
    __syncthreads();
    // up
    for (int q = Q - 2; q >= 0; --q) {
        const int nf = nq[q], mf = nf + 1, mc = nq[q + 1] + 1;
        double2* u = U + off[q];
        const double2* e = U + off[q + 1];
        for (int i = tid; i < mf * mf; i += kLasThreads) {
            const int a = i % mf, b = i / mf;
            if (a < 1 || b < 1 || a > nf - 1 || b > nf - 1) continue;
            const int I = a >> 1, J = b >> 1, c = J * mc + I;
            double2 v;
            if (!(a & 1) && !(b & 1)) v = e[c];
            else if (a & 1 && !(b & 1)) v = cscl(0.5, cadd(e[c], e[c + 1]));
            else if (!(a & 1)) v = cscl(0.5, cadd(e[c], e[c + mc]));
            else v = cscl(0.25, cadd(cadd(e[c], e[c + 1]), cadd(e[c + mc], e[c + mc + 1])));
            u[i] = cadd(u[i], v);
        }
        __syncthreads();
        smooth(q, nu2);
    }
    {
        const int m = n0 + 1;
        for (int i = tid; i < m * m; i += kLasThreads) ug[(size_t)(i / m) * pitch + i % m] = U[i];
    }
}

// Per node row b: sums over the interior nodes of (f_re^2, f_im^2) (mode 0) or
// of (r_re^2, r_im^2, u_re^2, u_im^2), r = f - (L_h u - k u) (mode 1).
__global__ __launch_bounds__(kNormThreads) void k_las_norm(int n, int pitch, double ih2, int mode,
                                                           const double2* __restrict__ u,
                                                           const double2* __restrict__ f,
                                                           const double2* __restrict__ k,
                                                           double* __restrict__ part) {
    __shared__ double red[4][kNormThreads];
    const int b = blockIdx.x + 1;  // rows 1 .. n-1
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 1 + threadIdx.x; a <= n - 1; a += kNormThreads) {
        const size_t i = (size_t)b * pitch + a;
        if (mode == 0) {
            const double2 v = f[i];
            s[0] += v.x * v.x;
            s[1] += v.y * v.y;
        } else {
            const double2 r = resid_at(u, f, k, i, pitch, ih2);
            const double2 w = u[i];
            s[0] += r.x * r.x;
            s[1] += r.y * r.y;
            s[2] += w.x * w.x;
            s[3] += w.y * w.y;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = kNormThreads / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[(size_t)4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the row partials (rows in order within each thread, then a fixed
// tree): out[q] for q = 0..3.
__global__ __launch_bounds__(kNormThreads) void k_las_norm_fin(int rows, const double* __restrict__ part,
                                                               double* __restrict__ out) {
    __shared__ double red[4][kNormThreads];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < rows; r += kNormThreads)
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += part[(size_t)4 * r + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = kNormThreads / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = red[threadIdx.x][0];
}

// Dense [N+1][N+1] complex <-> padded plane.
__global__ void k_las_unpack(int N, int pitch, const double2* __restrict__ src, double2* __restrict__ dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (a > N) return;
    dst[(size_t)b * pitch + a] = src[(size_t)b * (N + 1) + a];
}
__global__ void k_las_pack(int N, int pitch, const double2* __restrict__ src, double2* __restrict__ dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (a > N) return;
    dst[(size_t)b * (N + 1) + a] = src[(size_t)b * pitch + a];
}

dim3 rows_grid(int n, int t) { return dim3((n + 1 + t - 1) / t, n + 1); }

// Residual norms of the level-0 problem: out = {||.||^2 ...} as k_las_norm.
wandqs_status las_norms(wandqs_ctx* c, int mode, const double2* u, const double2* f,
                        const double2* k, double* out4) {
    const Level& L0 = c->lev[0];
    const int rows = L0.N - 1;
    {
        ProfScope ps(c, "k_las_norm", (double)(L0.N + 1) * (L0.N + 1) * (mode ? 48.0 : 16.0));
        WQ_KLAUNCH(ps, k_las_norm, dim3(rows), dim3(kNormThreads), 0, c->stream, L0.N, L0.pitch,
                   1.0 / (L0.h * L0.h), mode, u, f, k, c->las_part);
    }
    {
        ProfScope ps(c, "k_las_norm_fin", 32.0 * rows);
        WQ_KLAUNCH(ps, k_las_norm_fin, dim3(1), dim3(kNormThreads), 0, c->stream, rows, c->las_part,
                   c->las_red);
    }
    WQ_LAUNCH_CHECK();
    WQ_HIP(hipMemcpyAsync(out4, c->las_red, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return WANDQS_OK;
}

wandqs_status las_vcycle(wandqs_ctx* c, double2* u0) {
    const int ll = c->las_ll, nu1 = c->cfg.nu_pre, nu2 = c->cfg.nu_post;
    hipStream_t s = c->stream;
    auto U = [&](int l) { return l == 0 ? u0 : c->las_u[l]; };
    auto tiles = [](int n) { return dim3((n + 1 + kLTX - 1) / kLTX, (n + 1 + kLTY - 1) / kLTY); };
    for (int l = 0; l < ll; ++l) {
        const Level& F = c->lev[l];
        const Level& C = c->lev[l + 1];
        ProfScope ps(c, "k_las_down", (double)(F.N + 1) * (F.N + 1) * 64.0 + (double)(C.N + 1) * (C.N + 1) * 32.0);
        WQ_KLAUNCH(ps, k_las_down, tiles(F.N), dim3(kLTThreads), 0, s, F.N, F.h, F.pitch, nu1, U(l),
                   c->las_f[l], c->las_k[l], c->las_um[l], C.pitch, c->las_f[l + 1], U(l + 1));
    }
    {
        const Level& Cl = c->lev[ll];
        ProfScope ps(c, "k_las_coarse", (double)(Cl.N + 1) * (Cl.N + 1) * 64.0);
        WQ_KLAUNCH(ps, k_las_coarse, dim3(1), dim3(kLasThreads), 0, s, Cl.N, Cl.h, Cl.pitch, nu1, nu2,
                   U(ll), c->las_f[ll], c->las_k[ll]);
    }
    for (int l = ll - 1; l >= 0; --l) {
        const Level& F = c->lev[l];
        const Level& C = c->lev[l + 1];
        ProfScope ps(c, "k_las_up", (double)(F.N + 1) * (F.N + 1) * 64.0 + (double)(C.N + 1) * (C.N + 1) * 16.0);
        WQ_KLAUNCH(ps, k_las_up, tiles(F.N), dim3(kLTThreads), 0, s, F.N, F.h, F.pitch, nu2,
                   c->las_um[l], c->las_f[l], c->las_k[l], C.pitch, U(l + 1), U(l));
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace

wandqs_status laser_nodes(wandqs_ctx* c) {
    const Level& L0 = c->lev[0];
    {
        ProfScope ps(c, "k_las_a2", (double)(L0.N + 1) * (L0.N + 1) * 40.0);
        WQ_KLAUNCH(ps, k_las_a2, rows_grid(L0.N, 128), dim3(128), 0, c->stream, L0.N, L0.pitch,
                   (size_t)(L0.N + 1) * L0.pitch, c->cfg.laser_nz, c->cfg.dxi0, c->st,
                   c->las_env[c->las_cur], c->las_a2);
    }
    WQ_LAUNCH_CHECK();
    return node_gradient(c, c->las_a2, c->las_g[0], c->las_g[1]);
}

wandqs_status laser_plane_advance(wandqs_ctx* c, double dt, const double* chi, int j, int* cycles) {
    const Level& L0 = c->lev[0];
    const size_t plane = (size_t)(L0.N + 1) * L0.pitch;
    const double2* A0 = c->las_env[c->las_cur];
    double2* A1 = c->las_env[1 - c->las_cur];
    const double2* a0 = A0 + (size_t)j * plane;
    const double2* p0 = j ? A0 + (size_t)(j - 1) * plane : nullptr;
    const double2* p1 = j ? A1 + (size_t)(j - 1) * plane : nullptr;
    double2* u = A1 + (size_t)j * plane;
    const double beta = 4.0 / (dt * c->cfg.dxi0), gam = 4.0 * c->cfg.laser_k0 / dt;
    {
        ProfScope ps(c, "k_las_rhs", (double)(L0.N + 1) * (L0.N + 1) * 104.0);
        WQ_KLAUNCH(ps, k_las_rhs, rows_grid(L0.N, 128), dim3(128), 0, c->stream, L0.N, L0.h, L0.pitch,
                   beta, gam, chi, a0, p0, p1, c->las_f[0], c->las_k[0], u);
    }
    for (int l = 1; l <= c->las_ll; ++l) {
        const Level& F = c->lev[l - 1];
        const Level& C = c->lev[l];
        ProfScope ps(c, "k_las_krestrict", (double)(F.N + 1) * (F.N + 1) * 16.0 + (double)(C.N + 1) * (C.N + 1) * 16.0);
        WQ_KLAUNCH(ps, k_las_krestrict, rows_grid(C.N, 128), dim3(128), 0, c->stream, C.N, F.pitch,
                   c->las_k[l - 1], C.pitch, c->las_k[l]);
    }
    WQ_LAUNCH_CHECK();
    // the stop rule of the multigrid solves, on the real and imaginary parts
    double* hn = c->h_pin + kMaxSlots * kNormVec + 8;  // [fn re, fn im, -, -, r re, r im, u re, u im]
    wandqs_status s;
    if ((s = las_norms(c, 0, u, c->las_f[0], c->las_k[0], hn)) != WANDQS_OK) return s;
    if ((s = las_norms(c, 1, u, c->las_f[0], c->las_k[0], hn + 4)) != WANDQS_OK) return s;
    WQ_HIP(hipStreamSynchronize(c->stream));
    const double eps = std::numeric_limits<double>::epsilon();
    const double a_norm = 8.0 / (L0.h * L0.h);
    const double nint = (double)(L0.N - 1) * (L0.N - 1);
    double fn[2], rn[2], rprev[2], tol[2], scale[2];
    bool done[2];
    for (int q = 0; q < 2; ++q) {
        fn[q] = std::sqrt(hn[q]);
        rn[q] = rprev[q] = std::sqrt(hn[4 + q]);
        tol[q] = c->cfg.mg_rtol * (fn[q] > 0 ? fn[q] : rn[q]) + c->cfg.mg_atol * std::sqrt(nint);
        scale[q] = std::max(fn[q], rn[q]);
        done[q] = rn[q] <= tol[q];
    }
    int cyc = 0;
    // the first batch runs one cycle fewer than the last plane needed (planes
    // next to each other converge alike), then one cycle per norm check
    int batch = std::max(1, c->las_pred - 1);
    while (!(done[0] && done[1]) && cyc < c->cfg.mg_max_cycles) {
        const int b = std::min(batch, c->cfg.mg_max_cycles - cyc);
        for (int q = 0; q < b; ++q)
            if ((s = las_vcycle(c, u)) != WANDQS_OK) return s;
        cyc += b;
        batch = 1;
        if ((s = las_norms(c, 1, u, c->las_f[0], c->las_k[0], hn + 4)) != WANDQS_OK) return s;
        WQ_HIP(hipStreamSynchronize(c->stream));
        for (int q = 0; q < 2; ++q) {
            rprev[q] = rn[q];
            rn[q] = std::sqrt(hn[4 + q]);
            const double un = std::sqrt(hn[6 + q]);
            if (rn[q] <= tol[q] || rn[q] <= kFloorBE * eps * (a_norm * un + fn[q])) done[q] = true;
            else if (cyc >= 2 && rn[q] > 0.5 * rprev[q] && rn[q] <= 1e-9 * scale[q]) done[q] = true;
            else done[q] = false;
        }
    }
    if (cycles) *cycles = cyc;
    c->las_pred = cyc;
    if (!(std::isfinite(rn[0]) && std::isfinite(rn[1]) && done[0] && done[1])) {
        c->err = "laser envelope: multigrid did not converge";
        return WANDQS_E_NOCONV;
    }
    return WANDQS_OK;
}

wandqs_status laser_unpack(wandqs_ctx* c, const double* src, int set) {
    const Level& L0 = c->lev[0];
    const size_t plane = (size_t)(L0.N + 1) * L0.pitch, dense = (size_t)(L0.N + 1) * (L0.N + 1);
    for (int j = 0; j < c->cfg.laser_nz; ++j) {
        ProfScope ps(c, "k_las_unpack", 32.0 * dense);
        WQ_KLAUNCH(ps, k_las_unpack, rows_grid(L0.N, 128), dim3(128), 0, c->stream, L0.N, L0.pitch,
                   (const double2*)src + j * dense, c->las_env[set] + j * plane);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status laser_pack(wandqs_ctx* c, double* dst) {
    const Level& L0 = c->lev[0];
    const size_t plane = (size_t)(L0.N + 1) * L0.pitch, dense = (size_t)(L0.N + 1) * (L0.N + 1);
    for (int j = 0; j < c->cfg.laser_nz; ++j) {
        ProfScope ps(c, "k_las_pack", 32.0 * dense);
        WQ_KLAUNCH(ps, k_las_pack, rows_grid(L0.N, 128), dim3(128), 0, c->stream, L0.N, L0.pitch,
                   c->las_env[c->las_cur] + j * plane, (double2*)dst + j * dense);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace wq
