// Geometric multigrid for (L_h - k2) u = f with u = 0 on the boundary, the
// solver behind Solve_Wakefield (WAND-PIC, Sec. II item 4 and Sec. VII.A).
// L_h is the 5-point Laplacian of Sec. VII.B eq. (33); psi, Ez and Bz use
// k2 = 0 (eqs. (12)-(14)), B_perp uses k2 = n* / (1+psi) (eq. (18)).
//
// One V(nu1, nu2) cycle over levels N, N/2, ..., 2:
//   * levels with N > 64 run two fused tile kernels per level:
//       down: load a tile plus halo into LDS, nu1 red-black Gauss-Seidel sweeps,
//             write the smoothed tile, residual, full-weighting restriction;
//       up:   load a tile plus halo, add the bilinear prolongation of the coarse
//             correction, nu2 sweeps, write the tile;
//     the halo (2 nu + 2 nodes) makes the tile result identical to a global
//     red-black sweep, so every node array is read and written once per pass;
//   * the levels N <= 64 run inside one workgroup in LDS (one workgroup per
//     right-hand side), the 2x2-cell grid solved exactly.
// Two right-hand sides with one operator (Ez, Bz and Bx, By) share each pass.
// All reductions (residual norms) have a fixed order: results are bitwise
// reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <type_traits>

#include "wq_common.h"

namespace wq {
namespace {

// Kernel names for the per-kernel timing; formatted only when it is on.
template <class... A>
void prof_name(const wandqs_ctx* c, char* nm, size_t n, const char* fmt, A... a) {
    if (c->prof.on) std::snprintf(nm, n, fmt, a...);
    else nm[0] = 0;
}

#ifndef WQ_COARSE_CYCLES
#define WQ_COARSE_CYCLES 1
#endif
#ifndef WQ_COARSE_F32
#define WQ_COARSE_F32 1
#endif
#ifndef WQ_SMALL_TILE_MAX
#define WQ_SMALL_TILE_MAX 256
#endif
constexpr int kThreads = 256;  // norm and reduction kernels
// Helmholtz levels with h^2 n0 > kOmegaH2N0 smooth with plain Gauss-Seidel:
// where the diagonal shift h^2 k2 (k2 ~ n0 in the plasma) is no longer small,
// over-relaxation slows the cycle (measured).
constexpr double kOmegaH2N0 = 0.125;
// Pre-smoothing on the levels kFullPreLevels and more below the finest (the
// coarse kernel's levels included when it lies that deep) is one sweep: a
// second sweep there cost more time than the extra V-cycles it saved
// (measured).  The finer levels and every post-smoothing keep nu_pre, nu_post.
constexpr int kFullPreLevels = 2;
#ifndef WQ_COARSE_THREADS
#define WQ_COARSE_THREADS 1024
#endif
constexpr int kCoarseThreads = WQ_COARSE_THREADS;
// Tile kernels: 32 x 32 owned nodes with 512 threads, or 16 x 16 with 256
// threads on the levels N <= WQ_SMALL_TILE_MAX (more workgroups and a shorter
// chain of dependent LDS phases per workgroup where the grid is small).
// 64 x 64 with 1024 threads on the levels N >= WQ_BIG_TILE_MIN (the finest
// level of the large grids: a quarter of the halo re-reads of 32 x 32 tiles).
#ifndef WQ_BIG_TILE_MIN
#define WQ_BIG_TILE_MIN 1024
#endif
template <int T>
constexpr int tile_threads() { return T >= 64 ? 1024 : (T >= 32 ? 512 : 256); }
int tile_for(const wandqs_ctx* c, int N) {
    return N <= c->small_tile_max ? 16 : (N >= (WQ_BIG_TILE_MIN) ? 64 : 32);
}

// Deterministic block sum of NV values; the result is valid in thread 0.
template <int NV, int NT>
__device__ void block_sum(double (&v)[NV], double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += red[w * NV + k];
            v[k] = s;
        }
    }
}

// ------------------------------------------------------------ tile engine --
//
// A tile kernel holds an EX x EY block of nodes whose node (0, 0) is global
// node (ex0, ey0), ex0 even.  The iterate u lives in LDS; each thread owns
// KP horizontal node pairs (x = 2p, 2p+1 of a row) and keeps their f and the
// Gauss-Seidel diagonal D = 4 + h^2 k2 (and 1/D) in registers.  In a pair the
// two nodes have opposite colours, so every thread updates exactly one node of
// each of its pairs in every half sweep.
// Fused multiply-add, written out so that every tile kernel rounds the same
// way whatever the compiler shares between sweeps.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Value select (not an address select, so register arrays stay in registers).
template <typename T>
__device__ __forceinline__ T pick(int j, T a, T b) { return j ? b : a; }

template <int R, bool HELM, int EX, int EY, int NT>
struct TileShape {
    static constexpr int PW = EX / 2;
    static constexpr int NP = PW * EY;
    static constexpr int KP = (NP + NT - 1) / NT;
    static constexpr int EN = EX * EY;
    static_assert(EX % 2 == 0, "tile width must be even");
};

// E is the element type of the iterate, f and the sweep arithmetic (double, or
// float for the inner cycles of the mixed form); k2 is always read as double
// and D = 4 + h^2 k2, 1/D are formed in double before rounding to E.
template <typename E, int R, bool HELM, int EX, int EY, int KP, int NT>
__device__ __forceinline__ void tile_load(E (*su)[EX * EY], E (&fr)[R][KP][2], E (&Dr)[KP][2],
                                          E (&iDr)[KP][2], const E* const* u, const E* const* f,
                                          const double* k2, int pitch, int ex0, int ey0, int N,
                                          double h2) {
    constexpr int PW = EX / 2, NP = PW * EY;
    // Every load and LDS store is unconditional, so that the loads are all in
    // flight at once (the compiler waits for a load moved behind a
    // lane-dependent branch before the branch ends): the threads past the
    // tile redo the last pair (the same values to the same slots), the
    // indices are clamped into the grid and the values outside it masked by a
    // product with 0 (every value loaded is finite).
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int p = min((int)threadIdx.x + k * NT, NP - 1);
        const int ly = p / PW, px = p - ly * PW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * px + j;
            const int gx = ex0 + lx, gy = ey0 + ly;
            const bool in = gx >= 0 && gx <= N && gy >= 0 && gy <= N;
            const size_t g = (size_t)min(max(gy, 0), N) * pitch + min(max(gx, 0), N);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const E* ur = u[r] ? u[r] : f[r];
                const E uv = ur[g] * E(in && u[r] ? 1 : 0);
                su[r][ly * EX + lx] = uv;
                fr[r][k][j] = f[r][g] * E(in ? 1 : 0);
            }
            const double D = fmad(h2, HELM ? k2[g] * (in ? 1.0 : 0.0) : 0.0, 4.0);
            Dr[k][j] = (E)D;
            iDr[k][j] = HELM ? (E)(1.0 / D) : E(0.25);
        }
    }
}

// Over-relaxed red-black update of one node: with g = (sum of the 4
// neighbours - h^2 f) / D, the node's own equation solved for it,
// u <- u + om (g - u).  Every smoothing kernel forms it with these three
// fused operations, so they all give the same bits.
template <typename E>
__device__ __forceinline__ E sor_update(E u, E nb, E fv, E iD, E h2, E om) {
    return fmad(om, fmad(fmad(-h2, fv, nb), iD, -u), u);
}

// One red-black half sweep (sor_update) on the nodes of colour `color`
// ((gx + gy) % 2) that have all four neighbours in the tile and lie inside the
// domain.
template <typename E, int R, bool HELM, int EX, int EY, int KP, int NT>
__device__ __forceinline__ void tile_sweep(E (*su)[EX * EY], const E (&fr)[R][KP][2],
                                           const E (&iDr)[KP][2], int ex0, int ey0, int N, E h2,
                                           E om, int color) {
    constexpr int PW = EX / 2, NP = PW * EY;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int p = threadIdx.x + k * NT;
        const int ly = p / PW, px = p - ly * PW;
        const int gy = ey0 + ly;
        const int j = (gy + color) & 1;  // ex0 is even
        const int lx = 2 * px + j;
        const int gx = ex0 + lx;
        if (p < NP && lx >= 1 && lx <= EX - 2 && ly >= 1 && ly <= EY - 2 && gx >= 1 &&
            gx <= N - 1 && gy >= 1 && gy <= N - 1) {
            const int l = ly * EX + lx;
            const E id = pick(j, iDr[k][0], iDr[k][1]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const E fv = pick(j, fr[r][k][0], fr[r][k][1]);
                const E nb = su[r][l - 1] + su[r][l + 1] + su[r][l - EX] + su[r][l + EX];
                su[r][l] = sor_update(su[r][l], nb, fv, id, h2, om);
            }
        }
    }
}

template <typename E>
struct DownArgs {
    int N;
    double h;
    int pitch, pitch_c;
    const E* u_in[2];  // nullptr: zero initial guess
    const E* f[2];
    const double* k2;
    E* u_out[2];
    E* f_c[2];
    double* norm_part;  // (double only) nullptr or [3R][nblk]: sums r^2, f^2, u^2 of the incoming u
    int nblk;
    double omega;  // relaxation factor of the smoothing sweeps
};

// Down pass of one level: nu1 sweeps on the tile, write the smoothed tile,
// residual, full-weighting restriction onto the coarse tile.  Halo: 2 nu + 2
// nodes on the low side (the residual at x0 - 1 needs the smoothed u at x0 - 2),
// 2 nu + 2 on the high side (one more than needed, to keep the width even).
template <typename E, int R, bool HELM, int NU, int T>
__global__ __launch_bounds__(tile_threads<T>()) void k_mg_down(DownArgs<E> a) {
    constexpr int NT = tile_threads<T>();
    constexpr int HL = 2 * NU + 2, HH = 2 * NU + 2;
    constexpr int EX = T + HL + HH, EY = EX;
    using S = TileShape<R, HELM, EX, EY, NT>;
    constexpr int PW = S::PW, NP = S::NP, KP = S::KP, EN = S::EN;
    __shared__ E su[R][EN];
    __shared__ double red[(NT / 64) * 3 * R];

    const int tid = threadIdx.x;
    const int N = a.N;
    int bx, by, z;  // z: right-hand side of a split launch (R = 1, one per z)
    tile_rhs_of_block(bx, by, z);
    const int x0 = bx * T, y0 = by * T;
    const int ex0 = x0 - HL, ey0 = y0 - HL;
    const E h2 = (E)(a.h * a.h), ih2 = (E)(1.0 / (a.h * a.h));
    const E om = (E)a.omega;

    E fr[R][KP][2], Dr[KP][2], iDr[KP][2];
    tile_load<E, R, HELM, EX, EY, KP, NT>(su, fr, Dr, iDr, a.u_in + z, a.f + z, a.k2, a.pitch, ex0, ey0, N,
                                      a.h * a.h);
    __syncthreads();

    auto residual = [&](int r, int k, int j, int l) {
        const E u0 = su[r][l];
        const E nb = su[r][l - 1] + su[r][l + 1] + su[r][l - EX] + su[r][l + EX];
        const E D = pick(j, Dr[k][0], Dr[k][1]);
        const E fv = pick(j, fr[r][k][0], fr[r][k][1]);
        return fmad(-fmad(-D, u0, nb), ih2, fv);
    };

    if (a.norm_part) {  // residual of the incoming iterate on the owned interior nodes
        double acc[3 * R];
#pragma unroll
        for (int q = 0; q < 3 * R; ++q) acc[q] = 0.0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int p = tid + k * NT;
            const int ly = p / PW, px = p - ly * PW;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int lx = 2 * px + j;
                const int gx = ex0 + lx, gy = ey0 + ly;
                if (p < NP && lx >= HL && lx < HL + T && ly >= HL && ly < HL + T && gx >= 1 &&
                    gx <= N - 1 && gy >= 1 && gy <= N - 1) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double rr = residual(r, k, j, ly * EX + lx);
                        const double fv = pick(j, fr[r][k][0], fr[r][k][1]);
                        const double uv = su[r][ly * EX + lx];
                        acc[3 * r] += rr * rr;
                        acc[3 * r + 1] += fv * fv;
                        acc[3 * r + 2] += uv * uv;
                    }
                }
            }
        }
        block_sum<3 * R, NT>(acc, red);
        if (tid == 0) {
            const int b = by * gridDim.x + bx;
#pragma unroll
            for (int q = 0; q < 3 * R; ++q) a.norm_part[(3 * z + q) * a.nblk + b] = acc[q];
        }
    }

    for (int s = 0; s < NU; ++s)
        for (int color = 0; color < 2; ++color) {
            tile_sweep<E, R, HELM, EX, EY, KP, NT>(su, fr, iDr, ex0, ey0, N, h2, om, color);
            __syncthreads();
        }

    // write the owned nodes; residual on [x0-1, x0+T-1]^2 into registers
    E rr[R][KP][2];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int p = tid + k * NT;
        const int ly = p / PW, px = p - ly * PW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * px + j;
            const int gx = ex0 + lx, gy = ey0 + ly;
            const int l = ly * EX + lx;
            if (p < NP && lx >= HL && lx < HL + T && ly >= HL && ly < HL + T && gx <= N - 1 &&
                gy <= N - 1)
#pragma unroll
                for (int r = 0; r < R; ++r) a.u_out[r + z][(size_t)gy * a.pitch + gx] = su[r][l];
            const bool interior = p < NP && lx >= HL - 1 && lx <= HL + T - 1 && ly >= HL - 1 &&
                                  ly <= HL + T - 1 && gx >= 1 && gx <= N - 1 && gy >= 1 &&
                                  gy <= N - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) rr[r][k][j] = interior ? residual(r, k, j, l) : E(0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP; ++k) {  // the residual replaces u in LDS
        const int p = tid + k * NT;
        const int ly = p / PW, px = p - ly * PW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * px + j;
            if (p < NP && lx >= HL - 1 && lx <= HL + T - 1 && ly >= HL - 1 && ly <= HL + T - 1)
#pragma unroll
                for (int r = 0; r < R; ++r) su[r][ly * EX + lx] = rr[r][k][j];
        }
    }
    __syncthreads();

    // full weighting onto coarse nodes x0/2 .. x0/2 + T/2 - 1 (< N/2)
    const int Nc = N / 2;
    for (int i = tid; i < (T / 2) * (T / 2); i += NT) {
        const int oy = i / (T / 2), ox = i - oy * (T / 2);
        const int I = x0 / 2 + ox, J = y0 / 2 + oy;
        if (I > Nc - 1 || J > Nc - 1) continue;
        const bool interior = I >= 1 && J >= 1;
        const int l = (2 * J - ey0) * EX + (2 * I - ex0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            E v = E(0);
            if (interior) {
                const E* q = su[r];
                v = (E(4) * q[l] + E(2) * (q[l - 1] + q[l + 1] + q[l - EX] + q[l + EX]) +
                     (q[l - EX - 1] + q[l - EX + 1] + q[l + EX - 1] + q[l + EX + 1])) *
                    E(1.0 / 16.0);
            }
            a.f_c[r + z][(size_t)J * a.pitch_c + I] = v;
        }
    }
}

template <typename E>
struct UpArgs {
    int N;
    double h;
    int pitch, pitch_c;
    const E* u_mid[2];
    const E* e_c[2];
    const E* f[2];
    const double* k2;
    E* u_out[2];
    double omega;
    // (register tiles, double only) nullptr or [3R][nblk]: sums r^2, f^2, u^2
    // of the corrected, smoothed u on the owned nodes (halo 2 nu + 2)
    double* norm_part;
    int nblk;
    // (float, finest level of the mixed form) nullptr, or the FP64 iterates
    // that the result corrects in place (u += e) instead of being stored
    double* corr[2];
};

// Up pass of one level: u += bilinear prolongation of the coarse correction on
// the whole tile (halo 2 nu), nu2 sweeps, write the owned nodes.
template <typename E, int R, bool HELM, int NU, int T>
__global__ __launch_bounds__(tile_threads<T>()) void k_mg_up(UpArgs<E> a) {
    constexpr int NT = tile_threads<T>();
    constexpr int H = 2 * NU;
    constexpr int EX = T + 2 * H, EY = EX;
    using S = TileShape<R, HELM, EX, EY, NT>;
    constexpr int PW = S::PW, NP = S::NP, KP = S::KP, EN = S::EN;
    constexpr int CX = EX / 2 + 1, CY = EY / 2 + 1;
    __shared__ E su[R][EN];
    __shared__ E se[R][CX * CY];

    const int tid = threadIdx.x;
    const int N = a.N, Nc = N / 2;
    int bx, by, z;  // z: right-hand side of a split launch (R = 1, one per z)
    tile_rhs_of_block(bx, by, z);
    const int x0 = bx * T, y0 = by * T;
    const int ex0 = x0 - H, ey0 = y0 - H;  // even
    const int cx0 = ex0 / 2, cy0 = ey0 / 2;
    const E h2 = (E)(a.h * a.h);
    const E om = (E)a.omega;

    E fr[R][KP][2], Dr[KP][2], iDr[KP][2];
    tile_load<E, R, HELM, EX, EY, KP, NT>(su, fr, Dr, iDr, a.u_mid + z, a.f + z, a.k2, a.pitch, ex0, ey0, N,
                                      a.h * a.h);
    // the coarse correction, loaded as the tile (threads past the end redo
    // the last node)
#pragma unroll
    for (int q = 0; q < (CX * CY + NT - 1) / NT; ++q) {
        const int i = min(tid + q * NT, CX * CY - 1);
        const int cy = i / CX, cx = i - cy * CX;
        const int I = cx0 + cx, J = cy0 + cy;
        const bool in = I >= 0 && I <= Nc && J >= 0 && J <= Nc;
        const size_t g = (size_t)min(max(J, 0), Nc) * a.pitch_c + min(max(I, 0), Nc);
#pragma unroll
        for (int r = 0; r < R; ++r) se[r][i] = a.e_c[r + z][g] * E(in ? 1 : 0);
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < KP; ++k) {  // each thread corrects the nodes of its own pairs
        const int p = tid + k * NT;
        const int ly = p / PW, px = p - ly * PW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * px + j;
            const int gx = ex0 + lx, gy = ey0 + ly;
            if (p >= NP || gx < 1 || gx > N - 1 || gy < 1 || gy > N - 1) continue;
            const int c = ((gy >> 1) - cy0) * CX + (gx >> 1) - cx0;
            const bool ox = gx & 1, oy = gy & 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const E* e = se[r];
                E v;
                if (!ox && !oy) v = e[c];
                else if (ox && !oy) v = E(0.5) * (e[c] + e[c + 1]);
                else if (!ox && oy) v = E(0.5) * (e[c] + e[c + CX]);
                else v = E(0.25) * (e[c] + e[c + 1] + e[c + CX] + e[c + CX + 1]);
                su[r][ly * EX + lx] += v;
            }
        }
    }
    __syncthreads();

    for (int s = 0; s < NU; ++s)
        for (int color = 0; color < 2; ++color) {
            tile_sweep<E, R, HELM, EX, EY, KP, NT>(su, fr, iDr, ex0, ey0, N, h2, om, color);
            __syncthreads();
        }

#pragma unroll
    for (int k = 0; k < KP; ++k) {
        const int p = tid + k * NT;
        const int ly = p / PW, px = p - ly * PW;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int lx = 2 * px + j;
            const int gx = ex0 + lx, gy = ey0 + ly;
            if (p < NP && lx >= H && lx < H + T && ly >= H && ly < H + T && gx <= N - 1 &&
                gy <= N - 1)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const size_t g = (size_t)gy * a.pitch + gx;
                    if (a.corr[0]) a.corr[r + z][g] += (double)su[r][ly * EX + lx];
                    else a.u_out[r + z][g] = su[r][ly * EX + lx];
                }
        }
    }
}

// ------------------------------------------------------- register tiles --
//
// Tile kernels for the large levels with the iterate held in registers.  A
// workgroup of NW wavefronts holds a 128-column x 4 NW-row block of nodes
// whose node (0, 0) is global node (ex0, ey0), both even: lane l of wavefront
// w holds the node pair (2l, 2l + 1) of the rows 4w .. 4w + 3.  The colour of
// element j of row k is (j + k) % 2, so in a half sweep every lane updates one
// node per row, with no divergence.  Horizontal neighbours come from the next
// lane by DPP wave shifts, vertical ones from the lane's own rows; the rows at
// wavefront boundaries go through LDS once per half sweep.  The arithmetic and
// its order are those of the LDS tile kernels above: both give the same bits.
#ifndef WQ_REG_ROWS
#define WQ_REG_ROWS 4
#endif
constexpr int kRegRows = WQ_REG_ROWS;  // rows per wavefront (even)
#ifndef WQ_REG_WAVES
#define WQ_REG_WAVES 8
#endif
#ifndef WQ_REG_TILE_MIN
#define WQ_REG_TILE_MIN 512
#endif
constexpr int kRegWaves = WQ_REG_WAVES;
static_assert(kRegWaves * kRegRows >= 32, "register tiles need at least 32 rows");

// DPP wave shifts by one lane: lane i reads lane i - 1 (wave_shr:1) or lane
// i + 1 (wave_shl:1); the lane past the end of the wavefront reads 0.
constexpr int kFromLeft = 0x138, kFromRight = 0x130;
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <typename E> struct Pair2;
template <> struct Pair2<double> { using T = double2; };
template <> struct Pair2<float> { using T = float2; };

// Geometry of a register tile with halo HL: owned TX x TY nodes (K rows per
// wavefront).
template <int HL, int NW, int K = kRegRows>
struct RegShape {
    static constexpr int ROWS = K * NW;
    static constexpr int TX = 128 - 2 * HL, TY = ROWS - 2 * HL;
    static_assert(TY > 0 && HL % 2 == 0, "register tile shape");
};

// Loads the lane's pairs of u (nullptr: 0), f and the Gauss-Seidel diagonal:
// D = 4 + h^2 k2 and 1/D formed in double, rounded to E.  Nodes outside
// [0, N]^2 read 0 (D = 4).
template <typename E, int R, bool HELM, int K>
__device__ __forceinline__ void reg_load(E (&u)[R][K][2], E (&f)[R][K][2], E (&D)[K][2],
                                         E (&iD)[K][2], const E* const* uin, const E* const* fin,
                                         const double* k2, int pitch, int gx, int gy0, int N,
                                         double h2) {
    using V2 = typename Pair2<E>::T;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int gy = gy0 + k;
        const bool in = gy >= 0 && gy <= N && gx >= 0 && gx <= N;
        const bool in1 = in && gx + 1 <= N;  // gx + 1 <= pitch - 1: the load stays in the row
        // every row's loads issued without a lane-dependent branch (a node
        // past the grid loads node 0 and is masked by a product with 0: the
        // values are finite), so that the rows' loads are in flight together
        const size_t g = in ? (size_t)gy * pitch + gx : 0;
        const E m0 = in ? E(1) : E(0), m1 = in1 ? E(1) : E(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            V2 uv{E(0), E(0)};
            if (uin[r]) uv = *reinterpret_cast<const V2*>(uin[r] + g);  // uniform
            const V2 fv = *reinterpret_cast<const V2*>(fin[r] + g);
            u[r][k][0] = uv.x * m0;
            u[r][k][1] = uv.y * m1;
            f[r][k][0] = fv.x * m0;
            f[r][k][1] = fv.y * m1;
        }
        double q0 = 0.0, q1 = 0.0;
        if (HELM) {
            const double2 kv = *reinterpret_cast<const double2*>(k2 + g);
            q0 = kv.x * (double)m0;
            q1 = kv.y * (double)m1;
        }
        const double D0 = fmad(h2, q0, 4.0), D1 = fmad(h2, q1, 4.0);
        D[k][0] = (E)D0;
        D[k][1] = (E)D1;
        iD[k][0] = HELM ? (E)(1.0 / D0) : E(0.25);
        iD[k][1] = HELM ? (E)(1.0 / D1) : E(0.25);
    }
}

// Rows 0 and K-1 of every wavefront into buffer b; after a barrier each
// wavefront reads the row above its row 0 and the row below its row K-1
// (0 past the tile).
template <typename E, int R, int K, int NW>
struct RegExchange {
    using V2 = typename Pair2<E>::T;
    V2 (*xb)[R][NW][2][64];
    __device__ __forceinline__ void put(int b, const E (&v)[R][K][2], int w, int lane) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xb[b][r][w][0][lane] = V2{v[r][0][0], v[r][0][1]};
            xb[b][r][w][1][lane] = V2{v[r][K - 1][0], v[r][K - 1][1]};
        }
    }
    __device__ __forceinline__ void get(int b, V2 (&up)[R], V2 (&dn)[R], int w, int lane) const {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            up[r] = w > 0 ? xb[b][r][w - 1][1][lane] : V2{E(0), E(0)};
            dn[r] = w < NW - 1 ? xb[b][r][w + 1][0][lane] : V2{E(0), E(0)};
        }
    }
};

template <typename V2>
__device__ __forceinline__ auto el(const V2& v, int j) { return j ? v.y : v.x; }

// One red-black half sweep of colour c over the lane's rows; upd[k][j] marks
// the nodes inside the tile's update region and the domain interior.
template <typename E, int R, bool HELM, int K>
__device__ __forceinline__ void reg_half_sweep(E (&u)[R][K][2], const E (&f)[R][K][2],
                                               const E (&iD)[K][2], const bool (&upd)[K][2],
                                               const typename Pair2<E>::T (&up)[R],
                                               const typename Pair2<E>::T (&dn)[R], E h2, E om,
                                               int c) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            if (((c + k) & 1) != jj) continue;  // element jj of row k has colour c
            const int j = jj;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                E left, right;
                if (j == 0) {
                    left = lane_shift<kFromLeft>(u[r][k][1]);
                    right = u[r][k][1];
                } else {
                    left = u[r][k][0];
                    right = lane_shift<kFromRight>(u[r][k][0]);
                }
                const E upv = k == 0 ? el(up[r], j) : u[r][k - 1][j];
                const E dnv = k == K - 1 ? el(dn[r], j) : u[r][k + 1][j];
                const E nb = left + right + upv + dnv;
                const E nv = sor_update(u[r][k][j], nb, f[r][k][j], iD[k][j], h2, om);
                u[r][k][j] = upd[k][j] ? nv : u[r][k][j];
            }
        }
    }
}

// Residual f - A u of every node of the lane's rows (0 outside the domain
// interior); up/dn are the rows across the wavefront boundaries.
template <typename E, int R, int K>
__device__ __forceinline__ void reg_residual(E (&rr)[R][K][2], const E (&u)[R][K][2],
                                             const E (&f)[R][K][2], const E (&D)[K][2],
                                             const bool (&dom)[K][2],
                                             const typename Pair2<E>::T (&up)[R],
                                             const typename Pair2<E>::T (&dn)[R], E ih2) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const E l0 = lane_shift<kFromLeft>(u[r][k][1]);
            const E r1 = lane_shift<kFromRight>(u[r][k][0]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const E left = j == 0 ? l0 : u[r][k][0];
                const E right = j == 0 ? u[r][k][1] : r1;
                const E upv = k == 0 ? el(up[r], j) : u[r][k - 1][j];
                const E dnv = k == K - 1 ? el(dn[r], j) : u[r][k + 1][j];
                const E nb = left + right + upv + dnv;
                const E v = fmad(-fmad(-D[k][j], u[r][k][j], nb), ih2, f[r][k][j]);
                rr[r][k][j] = dom[k][j] ? v : E(0);
            }
        }
}

// Down pass with register tiles: the same steps as k_mg_down.
template <typename E, int R, bool HELM, int NU, int NW>
__global__ __launch_bounds__(64 * NW) void k_mg_down_reg(DownArgs<E> a) {
    constexpr int K = kRegRows;
    constexpr int HL = 2 * NU + 2;
    using S = RegShape<HL, NW>;
    constexpr int TX = S::TX, TY = S::TY, ROWS = S::ROWS;
    using V2 = typename Pair2<E>::T;
    __shared__ V2 xb[2][R][NW][2][64];
    __shared__ double red[NW * 3 * R];
    const RegExchange<E, R, K, NW> xc{xb};

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int N = a.N;
    int bx, by, z;  // z: right-hand side of a split launch (R = 1, one per z)
    tile_rhs_of_block(bx, by, z);
    const int x0 = bx * TX, y0 = by * TY;
    const int ex0 = x0 - HL, ey0 = y0 - HL;
    const int gx = ex0 + 2 * lane, gy0 = ey0 + w * K;
    const E h2 = (E)(a.h * a.h), ih2 = (E)(1.0 / (a.h * a.h));
    const E om = (E)a.omega;

    E u[R][K][2], f[R][K][2], D[K][2], iD[K][2];
    reg_load<E, R, HELM, K>(u, f, D, iD, a.u_in + z, a.f + z, a.k2, a.pitch, gx, gy0, N, a.h * a.h);

    bool upd[K][2], dom[K][2], own[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int Y = w * K + k, gy = gy0 + k;
        own[k] = Y >= HL && Y < HL + TY;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int X = 2 * lane + j;
            dom[k][j] = gx + j >= 1 && gx + j <= N - 1 && gy >= 1 && gy <= N - 1;
            upd[k][j] = dom[k][j] && X >= 1 && X <= 126 && Y >= 1 && Y <= ROWS - 2;
        }
    }
    const bool own_x = 2 * lane >= HL && 2 * lane < HL + TX;

    V2 up[R], dn[R];
    int buf = 0;
    xc.put(buf, u, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);

    if (a.norm_part) {  // residual of the incoming iterate on the owned interior nodes
        E rr[R][K][2];
        reg_residual<E, R, K>(rr, u, f, D, dom, up, dn, ih2);
        double acc[3 * R];
#pragma unroll
        for (int q = 0; q < 3 * R; ++q) acc[q] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (own[k] && own_x && dom[k][j])
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double rv = rr[r][k][j];
                        const double fv = f[r][k][j];
                        const double uv = u[r][k][j];
                        acc[3 * r] += rv * rv;
                        acc[3 * r + 1] += fv * fv;
                        acc[3 * r + 2] += uv * uv;
                    }
        block_sum<3 * R, 64 * NW>(acc, red);
        if (threadIdx.x == 0) {
            const int b = by * gridDim.x + bx;
#pragma unroll
            for (int q = 0; q < 3 * R; ++q) a.norm_part[(3 * z + q) * a.nblk + b] = acc[q];
        }
    }

#pragma unroll
    for (int q = 0; q < 2 * NU; ++q) {
        if (q > 0) {
            buf ^= 1;
            xc.put(buf, u, w, lane);
            __syncthreads();
            xc.get(buf, up, dn, w, lane);
        }
        reg_half_sweep<E, R, HELM, K>(u, f, iD, upd, up, dn, h2, om, q & 1);
    }

    // the smoothed owned nodes
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int gy = gy0 + k;
        if (own[k] && own_x && gx <= N - 1 && gy <= N - 1)
#pragma unroll
            for (int r = 0; r < R; ++r)
                *reinterpret_cast<V2*>(a.u_out[r + z] + (size_t)gy * a.pitch + gx) =
                    V2{u[r][k][0], u[r][k][1]};
    }

    // residual of the smoothed iterate, then full weighting onto the coarse
    // nodes (x0/2 + i, y0/2 + m) owned by this tile
    buf ^= 1;
    xc.put(buf, u, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);
    E rr[R][K][2];
    reg_residual<E, R, K>(rr, u, f, D, dom, up, dn, ih2);
    buf ^= 1;
    xc.put(buf, rr, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);

    const int Nc = N / 2;
    const int I = ex0 / 2 + lane;
#pragma unroll
    for (int k = 0; k < K; k += 2) {
        const int J = (gy0 + k) / 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const E am = k == 0 ? up[r].y : rr[r][k - 1][1];  // row k-1, odd column
            const E a0 = k == 0 ? up[r].x : rr[r][k - 1][0];
            const E sl = lane_shift<kFromLeft>(rr[r][k][1]);
            const E sm = lane_shift<kFromLeft>(am);
            const E sp = lane_shift<kFromLeft>(rr[r][k + 1][1]);
            if (own[k] && own_x && I <= Nc - 1 && J <= Nc - 1) {
                E v = E(0);
                if (I >= 1 && J >= 1)
                    v = (E(4) * rr[r][k][0] +
                         E(2) * (sl + rr[r][k][1] + a0 + rr[r][k + 1][0]) +
                         (sm + am + sp + rr[r][k + 1][1])) *
                        E(1.0 / 16.0);
                a.f_c[r + z][(size_t)J * a.pitch_c + I] = v;
            }
        }
    }
}

// Up pass with register tiles: the same steps as k_mg_up.  NORM: the tiles
// carry a halo of 2 nu + 2, so that the residual of the result is exact on the
// owned nodes, and its norms go to a.norm_part (the last cycle of a batch).
template <typename E, int R, bool HELM, int NU, int NW, bool NORM>
__global__ __launch_bounds__(64 * NW) void k_mg_up_reg(UpArgs<E> a) {
    constexpr int K = kRegRows;
    constexpr int H = NORM ? 2 * NU + 2 : 2 * NU;
    using S = RegShape<H, NW>;
    constexpr int TX = S::TX, TY = S::TY, ROWS = S::ROWS;
    using V2 = typename Pair2<E>::T;
    __shared__ V2 xb[2][R][NW][2][64];
    const RegExchange<E, R, K, NW> xc{xb};

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int N = a.N, Nc = N / 2;
    int bx, by, z;  // z: right-hand side of a split launch (R = 1, one per z)
    tile_rhs_of_block(bx, by, z);
    const int x0 = bx * TX, y0 = by * TY;
    const int ex0 = x0 - H, ey0 = y0 - H;
    const int gx = ex0 + 2 * lane, gy0 = ey0 + w * K;
    const E h2 = (E)(a.h * a.h);
    const E om = (E)a.omega;

    E u[R][K][2], f[R][K][2], D[K][2], iD[K][2];
    reg_load<E, R, HELM, K>(u, f, D, iD, a.u_mid + z, a.f + z, a.k2, a.pitch, gx, gy0, N, a.h * a.h);

    // coarse correction at (I, J0 + m) and (I + 1, J0 + m), m = 0 .. K/2
    constexpr int KC = K / 2 + 1;
    const int I = ex0 / 2 + lane, J0 = gy0 / 2;
    E eL[R][KC], eR[R][KC];
#pragma unroll
    for (int m = 0; m < KC; ++m) {
        const int J = J0 + m;
        const bool inJ = J >= 0 && J <= Nc;
        const bool inL = inJ && I >= 0 && I <= Nc, inR = inJ && I + 1 >= 0 && I + 1 <= Nc;
        // indices clamped into the coarse grid, values masked after (no load
        // behind a lane-dependent branch)
        const size_t row = (size_t)min(max(J, 0), Nc) * a.pitch_c;
        const int iL = min(max(I, 0), Nc), iR = min(max(I + 1, 0), Nc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            eL[r][m] = a.e_c[r + z][row + iL] * (inL ? E(1) : E(0));
            eR[r][m] = a.e_c[r + z][row + iR] * (inR ? E(1) : E(0));
        }
    }

    bool upd[K][2], own[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int Y = w * K + k, gy = gy0 + k;
        own[k] = Y >= H && Y < H + TY;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int X = 2 * lane + j;
            const bool dom = gx + j >= 1 && gx + j <= N - 1 && gy >= 1 && gy <= N - 1;
            upd[k][j] = dom && X >= 1 && X <= 126 && Y >= 1 && Y <= ROWS - 2;
            // u += bilinear prolongation (gy even: row J0 + k/2; odd: between it and the next)
            const int m = k / 2;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                E v;
                if (!(k & 1)) v = j == 0 ? eL[r][m] : E(0.5) * (eL[r][m] + eR[r][m]);
                else if (j == 0) v = E(0.5) * (eL[r][m] + eL[r][m + 1]);
                else v = E(0.25) * (eL[r][m] + eR[r][m] + eL[r][m + 1] + eR[r][m + 1]);
                if (dom) u[r][k][j] += v;
            }
        }
    }
    const bool own_x = 2 * lane >= H && 2 * lane < H + TX;

    V2 up[R], dn[R];
#pragma unroll
    for (int q = 0; q < 2 * NU; ++q) {
        xc.put(q & 1, u, w, lane);
        __syncthreads();
        xc.get(q & 1, up, dn, w, lane);
        reg_half_sweep<E, R, HELM, K>(u, f, iD, upd, up, dn, h2, om, q & 1);
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int gy = gy0 + k;
        if (own[k] && own_x && gx <= N - 1 && gy <= N - 1)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const size_t g = (size_t)gy * a.pitch + gx;
                if (a.corr[0]) {
                    double2* p = reinterpret_cast<double2*>(a.corr[r + z] + g);
                    double2 o = *p;
                    o.x += (double)u[r][k][0];
                    o.y += (double)u[r][k][1];
                    *p = o;
                } else {
                    *reinterpret_cast<V2*>(a.u_out[r + z] + g) = V2{u[r][k][0], u[r][k][1]};
                }
            }
    }

    if (NORM) {  // residual norms of the result on the owned interior nodes
        __shared__ double red[NW * 3 * R];
        bool dom[K][2];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                dom[k][j] = gx + j >= 1 && gx + j <= N - 1 && gy0 + k >= 1 && gy0 + k <= N - 1;
        const int qb = 2 * NU;  // exchange buffer not used by the last sweep
        xc.put(qb & 1, u, w, lane);
        __syncthreads();
        xc.get(qb & 1, up, dn, w, lane);
        E rr[R][K][2];
        reg_residual<E, R, K>(rr, u, f, D, dom, up, dn, (E)(1.0 / (a.h * a.h)));
        double acc[3 * R];
#pragma unroll
        for (int q = 0; q < 3 * R; ++q) acc[q] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (own[k] && own_x && dom[k][j])
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double rv = rr[r][k][j];
                        const double fv = f[r][k][j];
                        const double uv = u[r][k][j];
                        acc[3 * r] += rv * rv;
                        acc[3 * r + 1] += fv * fv;
                        acc[3 * r + 2] += uv * uv;
                    }
        block_sum<3 * R, 64 * NW>(acc, red);
        if (threadIdx.x == 0) {
            const int b = by * gridDim.x + bx;
#pragma unroll
            for (int q = 0; q < 3 * R; ++q) a.norm_part[(3 * z + q) * a.nblk + b] = acc[q];
        }
    }
}

// Up pass of one V-cycle fused with the down pass of the next, on the finest
// level (register tiles, FP64, one right-hand side per workgroup): the tile of
// the smoothed iterate of the last down pass is corrected by the prolonged
// coarse correction and post-smoothed (the up pass), the residual norms of that
// iterate are recorded (those the next down pass would record), then it is
// pre-smoothed, written, and its residual restricted (the down pass).  The
// arithmetic and its order are those of the two passes, so the result has the
// same bits; the iterate between them never goes to memory.  Halo: 2 NU2 + 2
// NU1 + 2 nodes.
template <typename E>
struct FuseArgs {
    int N;
    double h;
    int pitch, pitch_c;
    const E* u_mid[2];  // smoothed iterate of the previous down pass
    const E* e_c[2];    // coarse correction
    const E* f[2];
    const double* k2;
    E* u_out[2];        // smoothed iterate of this pass's down part
    E* f_c[2];          // restricted residual
    double omega;
    double* norm_part;  // [3R][nblk]: sums r^2, f^2, u^2 of the up part's result
    int nblk;
};

template <typename E, int R, bool HELM, int NU1, int NU2, int NW, int K>
__global__ __launch_bounds__(64 * NW) void k_mg_updown_reg(FuseArgs<E> a) {
    constexpr int HL = 2 * NU2 + 2 * NU1 + 2;
    using S = RegShape<HL, NW, K>;
    constexpr int TX = S::TX, TY = S::TY, ROWS = S::ROWS;
    using V2 = typename Pair2<E>::T;
    __shared__ V2 xb[2][R][NW][2][64];
    __shared__ double red[NW * 3 * R];
    const RegExchange<E, R, K, NW> xc{xb};

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int N = a.N, Nc = N / 2;
    int bx, by, z;  // z: right-hand side of a split launch (R = 1, one per z)
    tile_rhs_of_block(bx, by, z);
    const int x0 = bx * TX, y0 = by * TY;
    const int ex0 = x0 - HL, ey0 = y0 - HL;
    const int gx = ex0 + 2 * lane, gy0 = ey0 + w * K;
    const E h2 = (E)(a.h * a.h), ih2 = (E)(1.0 / (a.h * a.h));
    const E om = (E)a.omega;

    E u[R][K][2], f[R][K][2], D[K][2], iD[K][2];
    reg_load<E, R, HELM, K>(u, f, D, iD, a.u_mid + z, a.f + z, a.k2, a.pitch, gx, gy0, N, a.h * a.h);

    // up part: coarse correction at (I, J0 + m) and (I + 1, J0 + m)
    constexpr int KC = K / 2 + 1;
    const int I = ex0 / 2 + lane, J0 = gy0 / 2;
    E eL[R][KC], eR[R][KC];
#pragma unroll
    for (int m = 0; m < KC; ++m) {
        const int J = J0 + m;
        const bool inJ = J >= 0 && J <= Nc;
        const bool inL = inJ && I >= 0 && I <= Nc, inR = inJ && I + 1 >= 0 && I + 1 <= Nc;
        // indices clamped into the coarse grid, values masked after (no load
        // behind a lane-dependent branch)
        const size_t row = (size_t)min(max(J, 0), Nc) * a.pitch_c;
        const int iL = min(max(I, 0), Nc), iR = min(max(I + 1, 0), Nc);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            eL[r][m] = a.e_c[r + z][row + iL] * (inL ? E(1) : E(0));
            eR[r][m] = a.e_c[r + z][row + iR] * (inR ? E(1) : E(0));
        }
    }
    bool upd[K][2], dom[K][2], own[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int Y = w * K + k, gy = gy0 + k;
        own[k] = Y >= HL && Y < HL + TY;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int X = 2 * lane + j;
            dom[k][j] = gx + j >= 1 && gx + j <= N - 1 && gy >= 1 && gy <= N - 1;
            upd[k][j] = dom[k][j] && X >= 1 && X <= 126 && Y >= 1 && Y <= ROWS - 2;
            const int m = k / 2;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                E v;
                if (!(k & 1)) v = j == 0 ? eL[r][m] : E(0.5) * (eL[r][m] + eR[r][m]);
                else if (j == 0) v = E(0.5) * (eL[r][m] + eL[r][m + 1]);
                else v = E(0.25) * (eL[r][m] + eR[r][m] + eL[r][m + 1] + eR[r][m + 1]);
                if (dom[k][j]) u[r][k][j] += v;
            }
        }
    }
    const bool own_x = 2 * lane >= HL && 2 * lane < HL + TX;

    V2 up[R], dn[R];
    int buf = 0;
#pragma unroll
    for (int q = 0; q < 2 * NU2; ++q) {
        xc.put(buf, u, w, lane);
        __syncthreads();
        xc.get(buf, up, dn, w, lane);
        buf ^= 1;
        reg_half_sweep<E, R, HELM, K>(u, f, iD, upd, up, dn, h2, om, q & 1);
    }

    // the norms of the up part's result (the next cycle's incoming iterate)
    xc.put(buf, u, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);
    buf ^= 1;
    {
        E rr[R][K][2];
        reg_residual<E, R, K>(rr, u, f, D, dom, up, dn, ih2);
        double acc[3 * R];
#pragma unroll
        for (int q = 0; q < 3 * R; ++q) acc[q] = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (own[k] && own_x && dom[k][j])
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const double rv = rr[r][k][j];
                        const double fv = f[r][k][j];
                        const double uv = u[r][k][j];
                        acc[3 * r] += rv * rv;
                        acc[3 * r + 1] += fv * fv;
                        acc[3 * r + 2] += uv * uv;
                    }
        block_sum<3 * R, 64 * NW>(acc, red);
        if (threadIdx.x == 0) {
            const int b = by * gridDim.x + bx;
#pragma unroll
            for (int q = 0; q < 3 * R; ++q) a.norm_part[(3 * z + q) * a.nblk + b] = acc[q];
        }
    }

    // down part: pre-smoothing (the first half sweep uses the exchange above)
#pragma unroll
    for (int q = 0; q < 2 * NU1; ++q) {
        if (q > 0) {
            xc.put(buf, u, w, lane);
            __syncthreads();
            xc.get(buf, up, dn, w, lane);
            buf ^= 1;
        }
        reg_half_sweep<E, R, HELM, K>(u, f, iD, upd, up, dn, h2, om, q & 1);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int gy = gy0 + k;
        if (own[k] && own_x && gx <= N - 1 && gy <= N - 1)
#pragma unroll
            for (int r = 0; r < R; ++r)
                *reinterpret_cast<V2*>(a.u_out[r + z] + (size_t)gy * a.pitch + gx) =
                    V2{u[r][k][0], u[r][k][1]};
    }
    xc.put(buf, u, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);
    buf ^= 1;
    E rr[R][K][2];
    reg_residual<E, R, K>(rr, u, f, D, dom, up, dn, ih2);
    xc.put(buf, rr, w, lane);
    __syncthreads();
    xc.get(buf, up, dn, w, lane);
    const int Ic = ex0 / 2 + lane;
#pragma unroll
    for (int k = 0; k < K; k += 2) {
        const int J = (gy0 + k) / 2;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const E am = k == 0 ? up[r].y : rr[r][k - 1][1];  // row k-1, odd column
            const E a0 = k == 0 ? up[r].x : rr[r][k - 1][0];
            const E sl = lane_shift<kFromLeft>(rr[r][k][1]);
            const E sm = lane_shift<kFromLeft>(am);
            const E sp = lane_shift<kFromLeft>(rr[r][k + 1][1]);
            if (own[k] && own_x && Ic <= Nc - 1 && J <= Nc - 1) {
                E v = E(0);
                if (Ic >= 1 && J >= 1)
                    v = (E(4) * rr[r][k][0] +
                         E(2) * (sl + rr[r][k][1] + a0 + rr[r][k + 1][0]) +
                         (sm + am + sp + rr[r][k + 1][1])) *
                        E(1.0 / 16.0);
                a.f_c[r + z][(size_t)J * a.pitch_c + Ic] = v;
            }
        }
    }
}


// ---------------------------------------------------------------- coarse --

template <typename E>
struct CoarseArgs {
    int N;  // <= kCoarseMax
    double h;
    int pitch;
    const E* f[2];
    const E* u_init[2];   // nullptr: zero initial guess
    const double* k2lev;  // Helmholtz: k2 of every level N..2, dense, concatenated
    const float* k2levf;  // the same in float, and 1 / (4 + h_l^2 k2) in float
    const float* idlevf;
    E* u_out[2];
    int ncycles, nu1, nu2;
    double omega;   // relaxation factor of the levels with h^2 <= h2max (Helmholtz)
    double h2max;   // coarser Helmholtz levels relax with factor 1
};

constexpr int coarse_nodes() {
    int t = 0;
    for (int n = kCoarseMax; n >= 2; n /= 2) t += (n + 1) * (n + 1);
    return t;
}

// Levels of at most WQ_COARSE_WAVE_N cells a side run in the first wavefront
// alone: a phase there has a few dozen nodes, and ordering its LDS traffic
// inside one wavefront (whose LDS operations complete in order) costs no
// workgroup barrier.  0: every level uses the whole workgroup.  The results
// are the same bits for any value (the nodes of one colour are independent);
// the Helmholtz coarse kernel measured 22.9 / 23.5 / 24.6 / 31.3 us with 8 /
// 0 / 16 / 32: the phases are LDS latency chains more than barrier waits.
#ifndef WQ_COARSE_WAVE_N
#define WQ_COARSE_WAVE_N 8
#endif
constexpr int kCoarseWaveN = WQ_COARSE_WAVE_N;

// Level operations with the level size as a compile-time constant, run by NT
// threads (the workgroup, or the first wavefront when NT = 64).  FAST (float
// LDS copies, which leave room in LDS): the restriction computes each fine
// residual once into a buffer, and the Helmholtz sweeps multiply by a stored
// 1/D instead of dividing.
template <typename E, bool HELM, int n, bool FAST, int NT>
struct LdsLevel {
    static constexpr int W = n + 1;
    static constexpr int HALF = n / 2;                // node slots of one colour per interior row
    static constexpr int ITEMS = (n - 1) * HALF;
    static constexpr int NTH = NT;
    static constexpr int PER = (ITEMS + NTH - 1) / NTH;

    static __device__ __forceinline__ void sync() {
        if constexpr (NT == 64) wave_sync();
        else __syncthreads();
    }

    // nu over-relaxed red-black sweeps (sor_update); iD (FAST and HELM) =
    // 1 / (4 + h2 k2); iDf (HELM, not FAST) = the same in float, refined by one
    // Newton step to the precision of E instead of dividing
    static __device__ void smooth(E* u, const E* f, const E* k2, const E* iD, const float* iDf, E h2,
                                  E om, int nu) {
        // slot i: row b, first node a0 = 1 + 2 (i mod HALF); colour c updates a0 + ((1 + b + c) % 2)
        int lb[PER], pb[PER];
        bool ok[PER], last[PER];
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int i = threadIdx.x + m * NTH;
            const int b = 1 + i / HALF;
            const int a0 = 1 + 2 * (i - (b - 1) * HALF);
            ok[m] = i < ITEMS;
            last[m] = a0 == n - 1;  // a0 + 1 lies on the boundary
            lb[m] = b * W + a0;
            pb[m] = (1 + b) & 1;
        }
        for (int s = 0; s < nu; ++s)
            for (int color = 0; color < 2; ++color) {
#pragma unroll
                for (int m = 0; m < PER; ++m) {
                    const int d = (pb[m] + color) & 1;
                    if (!ok[m] || (d && last[m])) continue;
                    const int l = lb[m] + d;
                    const E nb = u[l - 1] + u[l + 1] + u[l - W] + u[l + W];
                    if (HELM && !FAST) {
                        const E D = fmad(h2, k2[l], E(4));
                        E q = (E)iDf[l];
                        q = q * fmad(-D, q, E(2));
                        const E g = fmad(-h2, f[l], nb) * q;
                        u[l] = fmad(om, g - u[l], u[l]);
                    } else {
                        u[l] = sor_update(u[l], nb, f[l], HELM ? iD[l] : E(0.25), h2, om);
                    }
                }
                sync();
            }
    }

    static __device__ E resid(const E* u, const E* f, const E* k2, E ih2, int l) {
        E au = (u[l - 1] + u[l + 1] + u[l - W] + u[l + W] - E(4) * u[l]) * ih2;
        if (HELM) au -= k2[l] * u[l];
        return f[l] - au;
    }

    // f_c = full weighting of the residual; u_c = 0.  sr (FAST): residual
    // buffer of the level's size.
    static __device__ void restrict_to(const E* u, const E* f, const E* k2, E ih2, E* uc, E* fc,
                                       E* sr) {
        constexpr int nc = n / 2, Wc = nc + 1;
        if (FAST) {
            for (int i = threadIdx.x; i < (n - 1) * (n - 1); i += NTH) {
                const int y = 1 + i / (n - 1), x = 1 + i - (y - 1) * (n - 1);
                sr[y * W + x] = resid(u, f, k2, ih2, y * W + x);
            }
            sync();
        }
        for (int i = threadIdx.x; i < Wc * Wc; i += NTH) {
            const int J = i / Wc, I = i - J * Wc;
            E v = E(0);
            if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1) {
                const int c = (2 * J) * W + 2 * I;
                if (FAST)
                    v = (E(4) * sr[c] + E(2) * (sr[c - 1] + sr[c + 1] + sr[c - W] + sr[c + W]) +
                         (sr[c - W - 1] + sr[c - W + 1] + sr[c + W - 1] + sr[c + W + 1])) *
                        E(1.0 / 16.0);
                else
                    v = (E(4) * resid(u, f, k2, ih2, c) +
                         E(2) * (resid(u, f, k2, ih2, c - 1) + resid(u, f, k2, ih2, c + 1) +
                                 resid(u, f, k2, ih2, c - W) + resid(u, f, k2, ih2, c + W)) +
                         (resid(u, f, k2, ih2, c - W - 1) + resid(u, f, k2, ih2, c - W + 1) +
                          resid(u, f, k2, ih2, c + W - 1) + resid(u, f, k2, ih2, c + W + 1))) *
                        E(1.0 / 16.0);
            }
            fc[i] = v;
            uc[i] = E(0);
        }
        sync();
    }

    // u += bilinear interpolation of the coarse correction uc, one coarse cell
    // (its four fine nodes 2I..2I+1 x 2J..2J+1, interior ones only) per item
    static __device__ void prolong_add(E* u, const E* uc) {
        constexpr int nc = n / 2, Wc = nc + 1;
        for (int i = threadIdx.x; i < nc * nc; i += NTH) {
            const int J = i / nc, I = i - J * nc;
            const int c = J * Wc + I, l = (2 * J) * W + 2 * I;
            const E e00 = uc[c], e10 = uc[c + 1], e01 = uc[c + Wc], e11 = uc[c + Wc + 1];
            if (I >= 1 && J >= 1) u[l] += e00;
            if (J >= 1) u[l + 1] += E(0.5) * (e00 + e10);
            if (I >= 1) u[l + W] += E(0.5) * (e00 + e01);
            u[l + W + 1] += E(0.25) * (e00 + e10 + e01 + e11);
        }
        sync();
    }
};

// Level dispatch: runtime level size -> compile-time specialisation (for the
// first wavefront alone only the sizes it runs).
template <typename E, bool HELM, bool FAST, int NT, typename Fn>
__device__ __forceinline__ void with_level(int n, Fn&& fn) {
    constexpr int NMAX = NT == 64 ? kCoarseWaveN : 64;
    switch (n) {
        case 64:
            if constexpr (NMAX >= 64) fn(LdsLevel<E, HELM, 64, FAST, NT>{});
            break;
        case 32:
            if constexpr (NMAX >= 32) fn(LdsLevel<E, HELM, 32, FAST, NT>{});
            break;
        case 16:
            if constexpr (NMAX >= 16) fn(LdsLevel<E, HELM, 16, FAST, NT>{});
            break;
        case 8:
            if constexpr (NMAX >= 8) fn(LdsLevel<E, HELM, 8, FAST, NT>{});
            break;
        default:
            if constexpr (NMAX >= 4) fn(LdsLevel<E, HELM, 4, FAST, NT>{});
            break;
    }
}

// All levels N <= 64 in one workgroup per right-hand side; the 2x2-cell grid
// is solved exactly in double.  E is the type of the arrays in memory, C the
// type of the LDS copy and of the sweep arithmetic: below a finer level the
// result is only a coarse-grid correction, whose rounding never reaches the
// fixed point (the finer levels' FP64 residual and smoothing set it), so it
// runs in float there; when the coarse kernel is the whole solve, C = E.
template <typename E, typename C, bool HELM>
__global__ __launch_bounds__(kCoarseThreads) void k_mg_coarse(CoarseArgs<E> a) {
    constexpr int TOT = coarse_nodes();
    constexpr bool FAST = sizeof(C) == 4;
    // (slot TOT of each array takes the stores of the threads past the end,
    // so that no branch guards a store of loaded data)
    __shared__ C su[TOT + 1];
    __shared__ C sf[TOT + 1];
    __shared__ C sk[HELM ? TOT + 1 : 1];
    __shared__ C siD[(HELM && FAST) ? TOT + 1 : 1];
    __shared__ float siDf[(HELM && !FAST) ? TOT + 1 : 1];  // float 1/D for the double sweeps
    __shared__ C sr[FAST ? (kCoarseMax + 1) * (kCoarseMax + 1) : 1];
    const int r = blockIdx.x;
    const int tid = threadIdx.x;

    int Ns[8], off[8], nl = 0, tot = 0;
    for (int n = a.N; n >= 2; n /= 2) {
        Ns[nl] = n;
        off[nl] = tot;
        tot += (n + 1) * (n + 1);
        ++nl;
    }
    const int N = a.N;
    // loads in batches of kB per thread so that their latencies overlap; every
    // load and every LDS store of its value is unconditional (an index clamped
    // into its array, the value selected after it, the store of a thread past
    // the end going to slot TOT): a load that the compiler can move behind a
    // lane-dependent branch is waited for before the branch ends, which would
    // serialize the batch
    constexpr int kB = 8;
    const int nt = (N + 1) * (N + 1);
    const bool has_u = a.u_init[r] != nullptr;
    const E* ui = has_u ? a.u_init[r] : a.f[r];
    const E* fi = a.f[r];
    // (the values are masked by a product with 0 or 1, not a select: the
    // compiler turns a select between a loaded value and a constant into a
    // branch around the load; every value loaded here is finite)
    const auto load_uf = [&](int i, E& uo, E& fo) {
        const int ic = min(i, nt - 1);
        const int y = ic / (N + 1), x = ic - y * (N + 1);
        const size_t g = (size_t)y * a.pitch + x;
        const E ut = ui[g], ft = fi[g];
        const bool ok = i < nt && x != 0 && y != 0 && x != N && y != N;
        uo = ut * E(ok && has_u ? 1 : 0);
        fo = ft * E(ok ? 1 : 0);
    };
    if (HELM && tot <= kB * kCoarseThreads) {
        // one batch: u, f, k2 and 1/D all issued before the first LDS store
        // (k2 in the type of the sweeps; 1/D always from the float table)
        E uv[kB], fv[kB];
        C kv[kB];
        float dv[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int i = b * kCoarseThreads + tid, ic = min(i, tot - 1);
            load_uf(i, uv[b], fv[b]);
            kv[b] = FAST ? (C)a.k2levf[ic] : (C)a.k2lev[ic];
            dv[b] = a.idlevf[ic];
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int i = b * kCoarseThreads + tid;
            const int iu = i < nt ? i : TOT, ik = i < tot ? i : TOT;
            su[iu] = (C)uv[b];
            sf[iu] = (C)fv[b];
            sk[ik] = kv[b];
            if (FAST) siD[ik] = (C)dv[b];
            else siDf[ik] = dv[b];
        }
    } else {
        for (int base = 0; base < nt; base += kB * kCoarseThreads) {
            E uv[kB], fv[kB];
#pragma unroll
            for (int b = 0; b < kB; ++b) load_uf(base + b * kCoarseThreads + tid, uv[b], fv[b]);
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const int i = base + b * kCoarseThreads + tid, iu = i < nt ? i : TOT;
                su[iu] = (C)uv[b];
                sf[iu] = (C)fv[b];
            }
        }
        if (HELM)  // k2 and 1/D of every level, made once per solve by k_coarse_k2
            for (int base = 0; base < tot; base += kB * kCoarseThreads) {
                C kv[kB];
                float dv[kB];
#pragma unroll
                for (int b = 0; b < kB; ++b) {
                    const int i = base + b * kCoarseThreads + tid, ic = min(i, tot - 1);
                    kv[b] = FAST ? (C)a.k2levf[ic] : (C)a.k2lev[ic];
                    dv[b] = a.idlevf[ic];
                }
#pragma unroll
                for (int b = 0; b < kB; ++b) {
                    const int i = base + b * kCoarseThreads + tid, ik = i < tot ? i : TOT;
                    sk[ik] = kv[b];
                    if (FAST) siD[ik] = (C)dv[b];
                    else siDf[ik] = dv[b];
                }
            }
    }
    __syncthreads();

    auto down = [&](int l, auto nt) {
        constexpr int NT = decltype(nt)::value;
        const double hl = a.h * (double)(1 << l);
        C* u = su + off[l];
        C* f = sf + off[l];
        const C* k2 = sk + (HELM ? off[l] : 0);
        const C* iD = siD + ((HELM && FAST) ? off[l] : 0);
        const float* iDf = siDf + ((HELM && !FAST) ? off[l] : 0);
        with_level<C, HELM, FAST, NT>(Ns[l], [&](auto L) {
            L.smooth(u, f, k2, iD, iDf, (C)(hl * hl), (C)(HELM && hl * hl > a.h2max ? 1.0 : a.omega), a.nu1);
            L.restrict_to(u, f, k2, (C)(1.0 / (hl * hl)), su + off[l + 1], sf + off[l + 1], sr);
        });
    };
    auto up = [&](int l, auto nt) {
        constexpr int NT = decltype(nt)::value;
        const double hl = a.h * (double)(1 << l);
        C* u = su + off[l];
        with_level<C, HELM, FAST, NT>(Ns[l], [&](auto L) {
            L.prolong_add(u, su + off[l + 1]);
            L.smooth(u, sf + off[l], sk + (HELM ? off[l] : 0), siD + ((HELM && FAST) ? off[l] : 0),
                     siDf + ((HELM && !FAST) ? off[l] : 0), (C)(hl * hl),
                     (C)(HELM && hl * hl > a.h2max ? 1.0 : a.omega), a.nu2);
        });
    };
    const std::integral_constant<int, kCoarseThreads> all{};
    const std::integral_constant<int, 64> wave{};
    // levels lw and below (at most kCoarseWaveN cells a side) in the first
    // wavefront; the workgroup's barriers before and after hand the LDS over
    int lw = 0;
    while (lw < nl - 1 && Ns[lw] > kCoarseWaveN) ++lw;
    for (int cyc = 0; cyc < a.ncycles; ++cyc) {
        for (int l = 0; l < lw; ++l) down(l, all);
        if (tid < 64) {
            for (int l = lw; l < nl - 1; ++l) down(l, wave);
            if (tid == 0) {  // 2x2 cells: one unknown, four zero neighbours
                const int l = nl - 1;
                const double hl = a.h * (double)(1 << l);
                const int c = 1 * 3 + 1;
                const double k2c = HELM ? (double)sk[off[l] + c] : 0.0;
                su[off[l] + c] = (C)(-(double)sf[off[l] + c] / (4.0 / (hl * hl) + k2c));
            }
            wave_sync();
            for (int l = nl - 2; l >= lw; --l) up(l, wave);
        }
        __syncthreads();
        for (int l = lw - 1; l >= 0; --l) up(l, all);
    }
    for (int i = tid; i < (N + 1) * (N + 1); i += kCoarseThreads) {
        const int y = i / (N + 1), x = i - y * (N + 1);
        a.u_out[r][(size_t)y * a.pitch + x] = (E)su[i];
    }
}

// Exact solve of the Poisson problem on the 64^2 coarse level (u = 0 on the
// boundary).  The 2-D sine transform diagonalises the 5-point operator of
// eq. (33): with S_jk = sin(pi (j+1)(k+1) / 64) (S S = 32 I) and the
// eigenvalues lambda_kl = -(4/H^2) (sin^2(pi (k+1)/128) + sin^2(pi (l+1)/128)),
// u = S (M o (S f S)) S with M = 1 / (32^2 lambda).  The four products run on
// fp32 MFMA (v_mfma_f32_16x16x4_f32), 16 wavefronts with one 16 x 16 output
// tile each; the 63 interior rows and columns are padded to 64 with zeros.
// Like the V-cycle coarse kernel below a finer level, the coarse correction
// is computed in float.
constexpr int kDstN = 64;
constexpr int kDstLd = 68;  // LDS row stride of the 64 x 64 matrices
typedef float dst_v4f __attribute__((ext_vector_type(4)));

template <typename E>
struct DstArgs {
    int pitch;
    const E* f[2];
    E* u_out[2];
    const float* S;
    const float* M;
};

// D = A B for 64 x 64 matrices in LDS: A row-major, B given transposed (Bt[j][k]
// = B[k][j]).  Wavefront w computes the tile rows 16 (w / 4) .., columns
// 16 (w % 4) ..; lane l feeds A[i0 + l % 16][4 s + l / 16] and
// Bt[j0 + l % 16][4 s + l / 16] at step s and holds D[i0 + 4 (l / 16) + q][j0 + l % 16].
__device__ __forceinline__ dst_v4f dst_tile(const float* A, const float* Bt) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = 16 * (w >> 2), j0 = 16 * (w & 3);
    const float* a = A + (i0 + (lane & 15)) * kDstLd + (lane >> 4);
    const float* b = Bt + (j0 + (lane & 15)) * kDstLd + (lane >> 4);
    dst_v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < kDstN / 4; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * s], b[4 * s], acc, 0, 0, 0);
    return acc;
}

template <typename E>
__global__ __launch_bounds__(1024) void k_coarse_dst(DstArgs<E> a) {
    __shared__ float sS[kDstN * kDstLd];
    __shared__ float sX[kDstN * kDstLd];
    __shared__ float sY[kDstN * kDstLd];
    const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i0 = 16 * (w >> 2), j0 = 16 * (w & 3);
    const int ti = i0 + 4 * (lane >> 4), tj = j0 + (lane & 15);  // this lane's outputs: rows ti + q, column tj
    float mv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) mv[q] = a.M[(ti + q) * kDstN + tj];
    // S (symmetric, so also S^T) and f^T: sX[x][y] = f(node y + 1, x + 1); every
    // load is issued before the first store, so their latencies overlap
    {
        constexpr int kIt = kDstN * kDstN / 1024;
        float sv[kIt], fv[kIt];
#pragma unroll
        for (int t = 0; t < kIt; ++t) {
            const int i = tid + t * 1024, y = i >> 6, x = i & 63;
            sv[t] = a.S[i];
            fv[t] = (x < kDstN - 1 && y < kDstN - 1) ? (float)a.f[r][(size_t)(y + 1) * a.pitch + x + 1]
                                                     : 0.f;
        }
#pragma unroll
        for (int t = 0; t < kIt; ++t) {
            const int i = tid + t * 1024, y = i >> 6, x = i & 63;
            sS[y * kDstLd + x] = sv[t];
            sX[x * kDstLd + y] = fv[t];
        }
    }
    __syncthreads();
    dst_v4f d = dst_tile(sS, sX);  // Y = S F
#pragma unroll
    for (int q = 0; q < 4; ++q) sY[(ti + q) * kDstLd + tj] = d[q];
    __syncthreads();
    d = dst_tile(sY, sS);  // X = M o (Y S), stored transposed for the next product
    __syncthreads();       // every read of the operands is done before sX is rewritten
#pragma unroll
    for (int q = 0; q < 4; ++q) sX[tj * kDstLd + ti + q] = mv[q] * d[q];
    __syncthreads();
    d = dst_tile(sS, sX);  // Y = S X
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) sY[(ti + q) * kDstLd + tj] = d[q];
    __syncthreads();
    d = dst_tile(sY, sS);  // U = Y S
#pragma unroll
    for (int q = 0; q < 4; ++q) sX[(ti + q) * kDstLd + tj] = d[q];
    __syncthreads();
    for (int i = tid; i < (kDstN + 1) * (kDstN + 1); i += 1024) {
        const int y = i / (kDstN + 1), x = i - y * (kDstN + 1);
        const bool in = x >= 1 && x <= kDstN - 1 && y >= 1 && y <= kDstN - 1;
        a.u_out[r][(size_t)y * a.pitch + x] = (E)(in ? sX[(y - 1) * kDstLd + x - 1] : 0.f);
    }
}

// FP64 form of the exact 64^2 coarse Poisson solve, for the mixed form, whose
// coarsest-grid solve stays in FP64 while its V-cycle levels run in FP32.
// The products run on FP64 MFMA (v_mfma_f64_16x16x4_f64: one 16 x 16 output
// tile per wavefront, lane l feeding A[i0 + l % 16][4 s + l / 16] and
// Bt[j0 + l % 16][4 s + l / 16] and holding D[i0 + 4 (l / 16) + q][j0 + l % 16],
// the layout of the FP32 instruction).  Plain FP64 fused multiply-adds from LDS
// were LDS-bound here: a wavefront's read of one shared row element costs a
// full LDS pass.
typedef double dst_v4d __attribute__((ext_vector_type(4)));
constexpr int kDstLd64 = kDstN + 4;  // LDS row stride (doubles) of the 64 x 64 operands

// 16 x 16 tile (rows 0..15 of A, columns j0.. of B) of A B for an inner
// dimension n: A row-major with stride LDA, B given transposed (Bt[j][k] =
// B[k][j]) with stride LDB.
template <int n, int LDA, int LDB>
__device__ __forceinline__ dst_v4d tile64(const double* A, const double* Bt, int j0) {
    const int lane = threadIdx.x & 63;
    const double* pa = A + (lane & 15) * LDA + (lane >> 4);
    const double* pb = Bt + (j0 + (lane & 15)) * LDB + (lane >> 4);
    dst_v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int s = 0; s < n / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s], pb[4 * s], acc, 0, 0, 0);
    return acc;
}

// The 64^2 exact solve in FP64 (grids of 128^2): one workgroup of 16
// wavefronts per right-hand side, u = S (M o (S F S)) S as four products in
// LDS, as in k_coarse_dst.
template <typename E>
struct DstArgs64 {
    int pitch;
    const E* f[2];
    E* u_out[2];
    const double* S;
    const double* M;
};

template <typename E>
__global__ __launch_bounds__(1024) void k_coarse_dst64(DstArgs64<E> a) {
    __shared__ double sS[kDstN * kDstLd64];
    __shared__ double sX[kDstN * kDstLd64];
    __shared__ double sY[kDstN * kDstLd64];
    const int r = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i0 = 16 * (w >> 2), j0 = 16 * (w & 3);
    const int ti = i0 + 4 * (lane >> 4), tj = j0 + (lane & 15);
    double mv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) mv[q] = a.M[(ti + q) * kDstN + tj];
    constexpr int kIt = kDstN * kDstN / 1024;
    {   // S and F^T: sX[x][y] = f(node y + 1, x + 1); unconditional loads first
        double sv[kIt], fv[kIt];
#pragma unroll
        for (int t = 0; t < kIt; ++t) {
            const int i = tid + t * 1024, y = i >> 6, x = i & (kDstN - 1);
            const bool in = x < kDstN - 1 && y < kDstN - 1;
            sv[t] = a.S[i];
            const double v = (double)a.f[r][in ? (size_t)(y + 1) * a.pitch + x + 1 : 0];
            fv[t] = in ? v : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kIt; ++t) {
            const int i = tid + t * 1024, y = i >> 6, x = i & (kDstN - 1);
            sS[y * kDstLd64 + x] = sv[t];
            sX[x * kDstLd64 + y] = fv[t];
        }
    }
    __syncthreads();
    dst_v4d d = tile64<kDstN, kDstLd64, kDstLd64>(sS + i0 * kDstLd64, sX, j0);  // Y = S F
#pragma unroll
    for (int q = 0; q < 4; ++q) sY[(ti + q) * kDstLd64 + tj] = d[q];
    __syncthreads();
    d = tile64<kDstN, kDstLd64, kDstLd64>(sY + i0 * kDstLd64, sS, j0);  // X = M o (Y S), stored transposed
    __syncthreads();  // every read of the operands is done before sX is rewritten
#pragma unroll
    for (int q = 0; q < 4; ++q) sX[tj * kDstLd64 + ti + q] = mv[q] * d[q];
    __syncthreads();
    d = tile64<kDstN, kDstLd64, kDstLd64>(sS + i0 * kDstLd64, sX, j0);  // Y = S X
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) sY[(ti + q) * kDstLd64 + tj] = d[q];
    __syncthreads();
    d = tile64<kDstN, kDstLd64, kDstLd64>(sY + i0 * kDstLd64, sS, j0);  // U = Y S
#pragma unroll
    for (int q = 0; q < 4; ++q) sX[(ti + q) * kDstLd64 + tj] = d[q];
    __syncthreads();
    for (int i = tid; i < (kDstN + 1) * (kDstN + 1); i += 1024) {
        const int y = i / (kDstN + 1), x = i - y * (kDstN + 1);
        const bool in = x >= 1 && x <= kDstN - 1 && y >= 1 && y <= kDstN - 1;
        a.u_out[r][(size_t)y * a.pitch + x] = (E)(in ? sX[(y - 1) * kDstLd64 + x - 1] : 0.0);
    }
}

// Tables of the exact coarse Poisson solve on an n^2 level of spacing H:
// S_jk = sin(pi (j+1)(k+1) / n) (the argument reduced exactly modulo 2 pi),
// M_jk = 1 / ((n/2)^2 lambda_jk), lambda_jk = -(4/H^2)(sin^2(pi (j+1)/2n) +
// sin^2(pi (k+1)/2n)), the eigenvalue of the 5-point operator for the sine
// mode (j+1, k+1); row and column n-1 are zero.  Float and (when S64 is set)
// double copies.
__global__ void k_dst_tables(int n, double H, float* S, float* M, double* S64, double* M64) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int jj = i / n, kk = i - jj * n;
    const bool in = jj < n - 1 && kk < n - 1;
    const double pi = 3.14159265358979323846;
    double sv = 0.0, mv = 0.0;
    if (in) {
        const int m = ((jj + 1) * (kk + 1)) % (2 * n);
        sv = sin(pi * (double)m / (double)n);
        const double sj = sin(pi * (jj + 1) / (2.0 * n));
        const double sk = sin(pi * (kk + 1) / (2.0 * n));
        const double lambda = -(4.0 / (H * H)) * (sj * sj + sk * sk);
        mv = 1.0 / ((n / 2.0) * (n / 2.0) * lambda);
    }
    S[i] = (float)sv;
    M[i] = (float)mv;
    if (S64) {
        S64[i] = sv;
        M64[i] = mv;
    }
}

// k2 of the coarse-kernel levels: the top level (N <= 64, pitched) copied
// densely, then full weighting level by level.  One block.
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_k2(int N, int pitch, double h,
                                                              const double* __restrict__ k2top,
                                                              double* __restrict__ out,
                                                              float* __restrict__ outf,
                                                              float* __restrict__ idf) {
    // every level in LDS: the top level's loads in batches of kB per thread,
    // the restrictions from LDS, the three outputs written once
    __shared__ double sk[coarse_nodes()];
    constexpr int kB = 8;
    const int tid = threadIdx.x;
    const int nt = (N + 1) * (N + 1);
    for (int base = 0; base < nt; base += kB * kCoarseThreads) {
        double v[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int i = base + b * kCoarseThreads + tid;
            const int y = i / (N + 1), x = i - y * (N + 1);
            const bool ok = i < nt && x != 0 && y != 0 && x != N && y != N;
            v[b] = ok ? k2top[(size_t)y * pitch + x] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const int i = base + b * kCoarseThreads + tid;
            if (i < nt) sk[i] = v[b];
        }
    }
    __syncthreads();
    int off = 0;
    for (int nf = N; nf > 2; nf /= 2) {
        const int nc = nf / 2, w = nf + 1;
        const double* kf = sk + off;
        double* kc = sk + off + (nf + 1) * (nf + 1);
        for (int i = tid; i < (nc + 1) * (nc + 1); i += kCoarseThreads) {
            const int J = i / (nc + 1), I = i - J * (nc + 1);
            double v = 0.0;
            if (I >= 1 && J >= 1 && I <= nc - 1 && J <= nc - 1) {
                const int c = (2 * J) * w + 2 * I;
                v = (4.0 * kf[c] + 2.0 * (kf[c - 1] + kf[c + 1] + kf[c - w] + kf[c + w]) +
                     (kf[c - w - 1] + kf[c - w + 1] + kf[c + w - 1] + kf[c + w + 1])) *
                    (1.0 / 16.0);
            }
            kc[i] = v;
        }
        __syncthreads();
        off += (nf + 1) * (nf + 1);
    }
    // double and float copies and 1 / (4 + h_l^2 k2) for the coarse kernel's
    // FP32 sweeps
    off = 0;
    for (int n = N, l = 0; n >= 2; n /= 2, ++l) {
        const double hl = h * (double)(1 << l);
        const float h2 = (float)(hl * hl);
        for (int i = tid; i < (n + 1) * (n + 1); i += kCoarseThreads) {
            const double kd = sk[off + i];
            const float kf = (float)kd;
            out[off + i] = kd;
            outf[off + i] = kf;
            idf[off + i] = 1.f / (4.f + h2 * kf);
        }
        off += (n + 1) * (n + 1);
    }
}

// Residual norms of the current iterate over the same tiles as the down pass.
// With r_out set (mixed form), the FP64 residual is also stored, rounded to
// float, as the right-hand side of the FP32 error equation (boundary 0).
template <int R, bool HELM>
__global__ __launch_bounds__(kThreads) void k_resnorm(int N, double h, int pitch,
                                                      const double* u0, const double* u1,
                                                      const double* f0, const double* f1,
                                                      const double* k2, double* part, int nblk,
                                                      float* r0, float* r1, int pitch32, int TX,
                                                      int TY) {
    __shared__ double red[(kThreads / 64) * 3 * R];
    const double ih2 = 1.0 / (h * h);
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const double* u[2] = {u0, u1};
    const double* f[2] = {f0, f1};
    float* ro[2] = {r0, r1};
    double acc[3 * R];
#pragma unroll
    for (int k = 0; k < 3 * R; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < TX * TY; i += kThreads) {
        const int oy = i / TX, ox = i - oy * TX;
        const int gx = x0 + ox, gy = y0 + oy;
        if (gx > N - 1 || gy > N - 1) continue;
        const bool interior = gx >= 1 && gy >= 1;
        const size_t g = (size_t)gy * pitch + gx;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double rr = 0.0;
            if (interior) {
                const double* q = u[r];
                double au = (q[g - 1] + q[g + 1] + q[g - pitch] + q[g + pitch] - 4.0 * q[g]) * ih2;
                if (HELM) au -= k2[g] * q[g];
                rr = f[r][g] - au;
                acc[3 * r] += rr * rr;
                acc[3 * r + 1] += f[r][g] * f[r][g];
                acc[3 * r + 2] += q[g] * q[g];
            }
            if (ro[0]) ro[r][(size_t)gy * pitch32 + gx] = (float)rr;
        }
    }
    block_sum<3 * R, kThreads>(acc, red);
    if (threadIdx.x == 0) {
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
        for (int k = 0; k < 3 * R; ++k) part[k * nblk + b] = acc[k];
    }
}

// Mixed form: u += e on the interior nodes (the FP32 correction added in FP64).
__global__ void k_correct(int N, int pitch, int pitch32, double* __restrict__ u0,
                          double* __restrict__ u1, const float* __restrict__ e0,
                          const float* __restrict__ e1) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (a < 1 || a > N - 1 || b < 1 || b > N - 1) return;
    u0[(size_t)b * pitch + a] += (double)e0[(size_t)b * pitch32 + a];
    if (u1) u1[(size_t)b * pitch + a] += (double)e1[(size_t)b * pitch32 + a];
}

// The norms of a batch of V-cycles to the host: one workgroup per slot and
// sum adds the slot's per-tile partials (in a fixed order) and writes the sum
// into the host's coherent pinned array dst; the last workgroup to finish
// (device-scope counter, which it resets) then copies the flags word and
// publishes the sequence number with a system-scope release, after which the
// host reads the sums.  Slot up_slot has nblk_up tiles, the slots in
// [fuse_lo, fuse_hi) nblk_fuse (fused passes), the others nblk.
__global__ __launch_bounds__(kThreads) void k_reduce_publish(
    const double* part, int stride, int nblk, int s0, int nvec, int up_slot, int nblk_up,
    int fuse_lo, int fuse_hi, int nblk_fuse, double* dst, const int32_t* __restrict__ flags,
    int32_t* dst_flags, uint32_t* dst_seq, uint32_t seq, uint32_t* count) {
    __shared__ double red[kThreads / 64];
    const int s = s0 + blockIdx.x / nvec, k = blockIdx.x % nvec;
    if (s == up_slot) nblk = nblk_up;
    if (s >= fuse_lo && s < fuse_hi) nblk = nblk_fuse;  // written by fused up-and-down passes
    const double* p = part + (size_t)s * stride + (size_t)k * nblk;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += kThreads) acc[0] += p[b];
    block_sum<1, kThreads>(acc, red);
    if (threadIdx.x == 0) {
        dst[s * kNormVec + k] = acc[0];
        __threadfence_system();
        if (atomicAdd(count, 1u) == gridDim.x - 1) {
            *count = 0;
            *dst_flags = *flags;
            __threadfence_system();
            __hip_atomic_store(dst_seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Full weighting of a fine node array onto the interior coarse nodes (boundary 0).
__global__ void k_restrict_fw(const double* fine, int pf, double* coarse, int pc, int Nc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y;
    if (I > Nc) return;
    double v = 0.0;
    if (I >= 1 && J >= 1 && I <= Nc - 1 && J <= Nc - 1) {
        const size_t c = (size_t)(2 * J) * pf + 2 * I;
        v = (4.0 * fine[c] + 2.0 * (fine[c - 1] + fine[c + 1] + fine[c - pf] + fine[c + pf]) +
             (fine[c - pf - 1] + fine[c - pf + 1] + fine[c + pf - 1] + fine[c + pf + 1])) *
            (1.0 / 16.0);
    }
    coarse[(size_t)J * pc + I] = v;
}

// ------------------------------------------------------------- dispatch --

template <typename E, int R, bool HELM, int T>
void launch_down_t(const DownArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps) {
    constexpr int NT = tile_threads<T>();
    switch (nu) {
        case 1: WQ_KLAUNCH(ps, (k_mg_down<E, R, HELM, 1, T>), grid, dim3(NT), 0, s, a); break;
        case 2: WQ_KLAUNCH(ps, (k_mg_down<E, R, HELM, 2, T>), grid, dim3(NT), 0, s, a); break;
        default: WQ_KLAUNCH(ps, (k_mg_down<E, R, HELM, 3, T>), grid, dim3(NT), 0, s, a); break;
    }
}

template <typename E, int R, bool HELM, int T>
void launch_up_t(const UpArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps) {
    constexpr int NT = tile_threads<T>();
    switch (nu) {
        case 1: WQ_KLAUNCH(ps, (k_mg_up<E, R, HELM, 1, T>), grid, dim3(NT), 0, s, a); break;
        case 2: WQ_KLAUNCH(ps, (k_mg_up<E, R, HELM, 2, T>), grid, dim3(NT), 0, s, a); break;
        default: WQ_KLAUNCH(ps, (k_mg_up<E, R, HELM, 3, T>), grid, dim3(NT), 0, s, a); break;
    }
}

template <typename E, int R, bool HELM>
void launch_down(const DownArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps, int T) {
    if (T == 16) launch_down_t<E, R, HELM, 16>(a, nu, grid, s, ps);
    else if (T == 64) launch_down_t<E, R, HELM, 64>(a, nu, grid, s, ps);
    else launch_down_t<E, R, HELM, 32>(a, nu, grid, s, ps);
}

template <typename E, int R, bool HELM>
void launch_up(const UpArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps, int T) {
    if (T == 16) launch_up_t<E, R, HELM, 16>(a, nu, grid, s, ps);
    else if (T == 64) launch_up_t<E, R, HELM, 64>(a, nu, grid, s, ps);
    else launch_up_t<E, R, HELM, 32>(a, nu, grid, s, ps);
}

template <typename E>
void down(int R, bool helm, const DownArgs<E>& a, int nu, dim3 g, hipStream_t s, const ProfScope& ps, int T) {
    if (R == 1) helm ? launch_down<E, 1, true>(a, nu, g, s, ps, T) : launch_down<E, 1, false>(a, nu, g, s, ps, T);
    else helm ? launch_down<E, 2, true>(a, nu, g, s, ps, T) : launch_down<E, 2, false>(a, nu, g, s, ps, T);
}

template <typename E>
void up(int R, bool helm, const UpArgs<E>& a, int nu, dim3 g, hipStream_t s, const ProfScope& ps, int T) {
    if (R == 1) helm ? launch_up<E, 1, true>(a, nu, g, s, ps, T) : launch_up<E, 1, false>(a, nu, g, s, ps, T);
    else helm ? launch_up<E, 2, true>(a, nu, g, s, ps, T) : launch_up<E, 2, false>(a, nu, g, s, ps, T);
}

dim3 tiles(int N, int T = kTile) { return dim3((N + T - 1) / T, (N + T - 1) / T); }

// Tiles of a level's down or up pass: register tiles on the levels
// N >= c->reg_tile_min, LDS tiles of edge tile_for(N) below.  TX x TY owned
// nodes per workgroup.  split (register tiles) and split_lds (LDS tiles): two
// right-hand sides run as separate workgroups of one launch (grid z), not both
// in each workgroup.
struct PassGeom {
    bool reg, split, split_lds;
    int TX, TY;
    dim3 grid;
};
PassGeom pass_geom(const wandqs_ctx* c, int N, int nu, bool down, bool norm = false) {
    PassGeom g{};
    g.reg = N >= c->reg_tile_min;
    g.split = c->reg_split;
    g.split_lds = c->lds_split;
    if (g.reg) {
        const int halo = down || norm ? 2 * nu + 2 : 2 * nu;
        g.TX = 128 - 2 * halo;
        g.TY = kRegRows * kRegWaves - 2 * halo;
    } else {
        g.TX = g.TY = tile_for(c, N);
    }
    g.grid = dim3((N + g.TX - 1) / g.TX, (N + g.TY - 1) / g.TY);
    return g;
}

template <typename E, int R, bool HELM>
void launch_down_reg(const DownArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps) {
    constexpr int NW = kRegWaves;
    switch (nu) {
        case 1: WQ_KLAUNCH(ps, (k_mg_down_reg<E, R, HELM, 1, NW>), grid, dim3(64 * NW), 0, s, a); break;
        case 2: WQ_KLAUNCH(ps, (k_mg_down_reg<E, R, HELM, 2, NW>), grid, dim3(64 * NW), 0, s, a); break;
        default: WQ_KLAUNCH(ps, (k_mg_down_reg<E, R, HELM, 3, NW>), grid, dim3(64 * NW), 0, s, a); break;
    }
}

template <typename E, int R, bool HELM>
void launch_up_reg(const UpArgs<E>& a, int nu, dim3 grid, hipStream_t s, const ProfScope& ps) {
    constexpr int NW = kRegWaves;
    if (a.norm_part) {
        switch (nu) {
            case 1: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 1, NW, true>), grid, dim3(64 * NW), 0, s, a); break;
            case 2: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 2, NW, true>), grid, dim3(64 * NW), 0, s, a); break;
            default: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 3, NW, true>), grid, dim3(64 * NW), 0, s, a); break;
        }
        return;
    }
    switch (nu) {
        case 1: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 1, NW, false>), grid, dim3(64 * NW), 0, s, a); break;
        case 2: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 2, NW, false>), grid, dim3(64 * NW), 0, s, a); break;
        default: WQ_KLAUNCH(ps, (k_mg_up_reg<E, R, HELM, 3, NW, false>), grid, dim3(64 * NW), 0, s, a); break;
    }
}

template <typename E>
void down_pass(int R, bool helm, const DownArgs<E>& a, int nu, const PassGeom& g, hipStream_t s,
               const ProfScope& ps) {
    if (!g.reg) {
        if (g.split_lds) return down<E>(1, helm, a, nu, dim3(g.grid.x, g.grid.y, R), s, ps, g.TX);
        return down<E>(R, helm, a, nu, g.grid, s, ps, g.TX);
    }
    if (R == 1 || g.split) {
        const dim3 gz(g.grid.x, g.grid.y, R);
        helm ? launch_down_reg<E, 1, true>(a, nu, gz, s, ps) : launch_down_reg<E, 1, false>(a, nu, gz, s, ps);
    } else {
        helm ? launch_down_reg<E, 2, true>(a, nu, g.grid, s, ps) : launch_down_reg<E, 2, false>(a, nu, g.grid, s, ps);
    }
}

template <typename E>
void up_pass(int R, bool helm, const UpArgs<E>& a, int nu, const PassGeom& g, hipStream_t s,
             const ProfScope& ps) {
    if (!g.reg) {
        if (g.split_lds) return up<E>(1, helm, a, nu, dim3(g.grid.x, g.grid.y, R), s, ps, g.TX);
        return up<E>(R, helm, a, nu, g.grid, s, ps, g.TX);
    }
    if (R == 1 || g.split) {
        const dim3 gz(g.grid.x, g.grid.y, R);
        helm ? launch_up_reg<E, 1, true>(a, nu, gz, s, ps) : launch_up_reg<E, 1, false>(a, nu, gz, s, ps);
    } else {
        helm ? launch_up_reg<E, 2, true>(a, nu, g.grid, s, ps) : launch_up_reg<E, 2, false>(a, nu, g.grid, s, ps);
    }
}

const char* type_name(double) { return "double"; }
const char* type_name(float) { return "float"; }

// Arrays of one solve: level 0 (u, f, k2) and the per-level buffers of type E.
// Geometry of the fused level-0 up-and-down launch (halo 2 nu_post + 2 nu_pre
// + 2), and whether a solve can use it: FP64 register tiles with one
// right-hand side per workgroup, equal pre- and post-sweep counts of 1 or 2.
bool fuse_possible(const wandqs_ctx* c) {
    const int nu = c->cfg.nu_pre;
    return c->mg_fuse && c->lc > 0 && c->N >= c->reg_tile_min && c->reg_split &&
           nu == c->cfg.nu_post && nu >= 1 && nu <= 2 && c->lev[0].um2[0] != nullptr;
}
#ifndef WQ_FUSE_ROWS
#define WQ_FUSE_ROWS 8
#endif
constexpr int kFuseRows = WQ_FUSE_ROWS;  // rows per wavefront of the fused tiles
#ifndef WQ_FUSE_WAVES
#define WQ_FUSE_WAVES 8
#endif
constexpr int kFuseWaves = WQ_FUSE_WAVES;  // wavefronts of a fused tile
dim3 fuse_grid(const wandqs_ctx* c, int R) {
    const int hl = 4 * c->cfg.nu_pre + 2;
    const int TX = 128 - 2 * hl, TY = kFuseRows * kFuseWaves - 2 * hl, N = c->N;
    return dim3((N + TX - 1) / TX, (N + TY - 1) / TY, R);
}
void launch_updown_reg(const FuseArgs<double>& a, bool helm, int nu, dim3 grid, hipStream_t s,
                       const ProfScope& ps) {
    constexpr int NW = kFuseWaves;
    const dim3 blk(64 * NW);
    if (helm) {
        if (nu == 1) WQ_KLAUNCH(ps, (k_mg_updown_reg<double, 1, true, 1, 1, NW, kFuseRows>), grid, blk, 0, s, a);
        else WQ_KLAUNCH(ps, (k_mg_updown_reg<double, 1, true, 2, 2, NW, kFuseRows>), grid, blk, 0, s, a);
    } else {
        if (nu == 1) WQ_KLAUNCH(ps, (k_mg_updown_reg<double, 1, false, 1, 1, NW, kFuseRows>), grid, blk, 0, s, a);
        else WQ_KLAUNCH(ps, (k_mg_updown_reg<double, 1, false, 2, 2, NW, kFuseRows>), grid, blk, 0, s, a);
    }
}

// Level-0 fusion state of one cycle inside a batch (FP64 only).
struct FuseCtl {
    bool skip_down0 = false;  // the level-0 down pass ran fused into the previous cycle
    bool fuse_up0 = false;    // the level-0 up pass fuses with the next cycle's down pass
    int next_slot = -1;       // norm slot of the next cycle's incoming iterate
    int cur = 0;              // level-0 pre-smoothed iterate in um (0) or um2 (1)
};

template <typename E>
struct Hier {
    E* u0[2];
    E* f0[2];
    const double* k2;
};

template <typename E> E* lev_u(wq::Level& L, int r);
template <> double* lev_u<double>(wq::Level& L, int r) { return L.u[r]; }
template <> float* lev_u<float>(wq::Level& L, int r) { return L.u32[r]; }
template <typename E> E* lev_um(wq::Level& L, int r);
template <> double* lev_um<double>(wq::Level& L, int r) { return L.um[r]; }
template <> float* lev_um<float>(wq::Level& L, int r) { return L.um32[r]; }
template <typename E> E* lev_f(wq::Level& L, int r);
template <> double* lev_f<double>(wq::Level& L, int r) { return L.f[r]; }
template <> float* lev_f<float>(wq::Level& L, int r) { return L.f32[r]; }

int nu_pre_at(const wandqs_ctx* c, int l) { return l >= kFullPreLevels ? 1 : c->cfg.nu_pre; }

// One V-cycle on levels 0..L.  zero_guess: the level-0 iterate starts from 0.
// norm_slot >= 0 (double only) records the residual of the incoming iterate.
template <typename E>
void vcycle(wandqs_ctx* c, int R, bool helm, const Hier<E>& hz, bool zero_guess, int norm_slot,
            int up_norm_slot = -1, double* const* corr = nullptr, const FuseCtl* fz = nullptr) {
    hipStream_t s = c->stream;
    const int lc = c->lc;
    const double eb = sizeof(E);
    auto U = [&](int l, int r) { return l == 0 ? hz.u0[r] : lev_u<E>(c->lev[l], r); };
    auto F = [&](int l, int r) { return l == 0 ? hz.f0[r] : lev_f<E>(c->lev[l], r); };
    auto K = [&](int l) { return l == 0 ? hz.k2 : (const double*)c->lev[l].k2; };
    // Poisson: the V-cycle ends with the exact fast-sine-transform solve on
    // level 1 when that is 128^2 .. 2048^2
    const bool fst = !helm && fst_used(c);
    const int lb = fst ? 1 : lc;
    // relaxation factor of the smoothing sweeps: the Helmholtz levels whose
    // diagonal shift is no longer small (h^2 n0 > 1/8) relax with factor 1
    const double om = helm ? c->cfg.mg_omega_helm : c->cfg.mg_omega;
    const double h2max = helm ? kOmegaH2N0 / c->cfg.n0 : std::numeric_limits<double>::infinity();
    auto omega_of = [&](double h) { return h * h > h2max ? 1.0 : om; };
    // the level-0 pre-smoothed iterate (the fused passes alternate two buffers)
    auto um0 = [&](int r) -> E* {
        if (fz && fz->cur) return reinterpret_cast<E*>(c->lev[0].um2[r]);
        return lev_um<E>(c->lev[0], r);
    };
    for (int l = 0; l < lb; ++l) {
        if (l == 0 && fz && fz->skip_down0) continue;
        wq::Level& L = c->lev[l];
        DownArgs<E> a{};
        a.omega = omega_of(L.h);
        a.N = L.N;
        a.h = L.h;
        a.pitch = L.pitch;
        a.pitch_c = c->lev[l + 1].pitch;
        for (int r = 0; r < R; ++r) {
            a.u_in[r] = (l == 0 && !zero_guess) ? hz.u0[r] : nullptr;
            a.f[r] = F(l, r);
            a.u_out[r] = l == 0 ? um0(r) : lev_um<E>(L, r);
            a.f_c[r] = F(l + 1, r);
        }
        a.k2 = helm ? K(l) : nullptr;
        const int nu = nu_pre_at(c, l);
        const PassGeom g = pass_geom(c, L.N, nu, true);
        a.nblk = g.grid.x * g.grid.y;
        a.norm_part = (l == 0 && norm_slot >= 0)
                          ? c->norm_part + (size_t)norm_slot * kNormVec * c->max_tiles
                          : nullptr;
        // algorithmic bytes per owned node: u (when read), f, k2, smoothed u, coarse f
        const double nodes = (double)L.N * L.N;
        char nm[64];
        if (g.reg)
            prof_name(c, nm, sizeof nm, "k_mg_down_reg<%s, %d, %s, %d, %d>@%d", type_name(E()), g.split ? 1 : R,
                          helm ? "true" : "false", nu, kRegWaves, L.N);
        else
            prof_name(c, nm, sizeof nm, "k_mg_down<%s, %d, %s, %d, %d>@%d", type_name(E()), g.split_lds ? 1 : R,
                          helm ? "true" : "false", nu, g.TX, L.N);
        ProfScope ps(c, nm, nodes * ((a.u_in[0] ? eb * R : 0.0) + eb * R + (helm ? 8.0 : 0.0) +
                                     eb * R + eb * R / 4));
        down_pass<E>(R, helm, a, nu, g, s, ps);
    }
    // the mixed form's inner cycles (E = float) solve their coarsest grid in FP64
    constexpr bool coarse64 = std::is_same<E, float>::value;
    if (fst) {
        const E* fo[2] = {F(1, 0), R > 1 ? F(1, 1) : nullptr};
        E* uo[2] = {U(1, 0), R > 1 ? U(1, 1) : nullptr};
        fst_solve<E>(c, R, fo, uo);
    } else {
        wq::Level& L = c->lev[lc];
        CoarseArgs<E> a{};
        a.omega = om;
        a.h2max = h2max;
        a.N = L.N;
        a.h = L.h;
        a.pitch = L.pitch;
        for (int r = 0; r < R; ++r) {
            a.f[r] = F(lc, r);
            a.u_init[r] = (lc == 0 && !zero_guess) ? hz.u0[r] : nullptr;
            a.u_out[r] = U(lc, r);
        }
        a.k2lev = helm ? c->k2lev : nullptr;
        a.k2levf = helm ? c->k2levf : nullptr;
        a.idlevf = helm ? c->idlevf : nullptr;
        a.ncycles = WQ_COARSE_CYCLES;
        a.nu1 = nu_pre_at(c, lc);
        a.nu2 = c->cfg.nu_post;
        const double nodes = (double)(L.N + 1) * (L.N + 1);
        char nm[64];
        if (!helm && lc > 0 && L.N == kDstN && coarse64) {  // exact Poisson coarse solve, FP64
            DstArgs64<E> d{};
            d.pitch = L.pitch;
            for (int r = 0; r < R; ++r) {
                d.f[r] = F(lc, r);
                d.u_out[r] = U(lc, r);
            }
            d.S = c->dst_S64;
            d.M = c->dst_M64;
            ProfScope ps(c, "k_coarse_dst64<float>", nodes * 2.0 * eb * R + 2.0 * 8.0 * kDstN * kDstN);
            WQ_KLAUNCH(ps, k_coarse_dst64<E>, dim3(R), dim3(1024), 0, s, d);
        } else if (!helm && lc > 0 && L.N == kDstN) {  // exact Poisson coarse solve
            DstArgs<E> d{};
            d.pitch = L.pitch;
            for (int r = 0; r < R; ++r) {
                d.f[r] = F(lc, r);
                d.u_out[r] = U(lc, r);
            }
            d.S = c->dst_S;
            d.M = c->dst_M;
            prof_name(c, nm, sizeof nm, "k_coarse_dst<%s>", type_name(E()));
            ProfScope ps(c, nm, nodes * 2.0 * eb * R + 2.0 * 4.0 * kDstN * kDstN);
            WQ_KLAUNCH(ps, k_coarse_dst<E>, dim3(R), dim3(1024), 0, s, d);
        } else {
            // float sweeps when the coarse levels only correct a finer FP64
            // level; the mixed form's inner cycles run them in double
            const bool f32 = WQ_COARSE_F32 && lc > 0 && !coarse64;
            prof_name(c, nm, sizeof nm, "k_mg_coarse<%s, %s, %s>", type_name(E()),
                          f32 ? "float" : (coarse64 ? "double" : type_name(E())), helm ? "true" : "false");
            ProfScope ps(c, nm, nodes * (eb * R + (a.u_init[0] ? eb * R : 0.0) + (helm ? 8.0 : 0.0) + eb * R));
            if (coarse64) {
                if (helm) WQ_KLAUNCH(ps, (k_mg_coarse<E, double, true>), dim3(R), dim3(kCoarseThreads), 0, s, a);
                else WQ_KLAUNCH(ps, (k_mg_coarse<E, double, false>), dim3(R), dim3(kCoarseThreads), 0, s, a);
            } else if (f32) {
                if (helm) WQ_KLAUNCH(ps, (k_mg_coarse<E, float, true>), dim3(R), dim3(kCoarseThreads), 0, s, a);
                else WQ_KLAUNCH(ps, (k_mg_coarse<E, float, false>), dim3(R), dim3(kCoarseThreads), 0, s, a);
            } else {
                if (helm) WQ_KLAUNCH(ps, (k_mg_coarse<E, E, true>), dim3(R), dim3(kCoarseThreads), 0, s, a);
                else WQ_KLAUNCH(ps, (k_mg_coarse<E, E, false>), dim3(R), dim3(kCoarseThreads), 0, s, a);
            }
        }
    }
    for (int l = lb - 1; l >= 0; --l) {
        wq::Level& L = c->lev[l];
        if constexpr (std::is_same<E, double>::value) {
            if (l == 0 && fz && fz->fuse_up0) {
                // up pass fused with the next cycle's down pass: into the other
                // buffer, recording the norms of the next cycle's incoming iterate
                FuseArgs<double> a{};
                a.N = L.N;
                a.h = L.h;
                a.pitch = L.pitch;
                a.pitch_c = c->lev[1].pitch;
                a.omega = omega_of(L.h);
                for (int r = 0; r < R; ++r) {
                    a.u_mid[r] = um0(r);
                    a.e_c[r] = U(1, r);
                    a.f[r] = F(0, r);
                    a.u_out[r] = fz->cur ? L.um[r] : L.um2[r];
                    a.f_c[r] = F(1, r);
                }
                a.k2 = helm ? K(0) : nullptr;
                const dim3 g = fuse_grid(c, R);
                a.nblk = g.x * g.y;
                a.norm_part = c->norm_part + (size_t)fz->next_slot * kNormVec * c->max_tiles;
                const double nodes = (double)L.N * L.N;
                char nm[64];
                prof_name(c, nm, sizeof nm, "k_mg_updown_reg<double, 1, %s, %d, %d, %d, %d>@%d",
                          helm ? "true" : "false", c->cfg.nu_pre, c->cfg.nu_post, kFuseWaves,
                          kFuseRows, L.N);
                // per owned node and right-hand side: smoothed u, 1/4 coarse e,
                // f, new smoothed u, 1/4 coarse f; k2 once
                ProfScope ps(c, nm, nodes * (R * (8.0 + 2.0 + 8.0 + 8.0 + 2.0) + (helm ? 8.0 : 0.0)));
                launch_updown_reg(a, helm, c->cfg.nu_pre, g, s, ps);
                continue;
            }
        }
        UpArgs<E> a{};
        a.omega = omega_of(L.h);
        a.N = L.N;
        a.h = L.h;
        a.pitch = L.pitch;
        a.pitch_c = c->lev[l + 1].pitch;
        for (int r = 0; r < R; ++r) {
            a.u_mid[r] = l == 0 ? um0(r) : lev_um<E>(L, r);
            a.e_c[r] = U(l + 1, r);
            a.f[r] = F(l, r);
            a.u_out[r] = U(l, r);
        }
        a.k2 = helm ? K(l) : nullptr;
        // per owned node: smoothed u, coarse correction (1/4), f, k2, corrected u
        const double nodes = (double)L.N * L.N;
        char nm[64];
        // the finest up pass of a batch's last cycle records the result's norms
        const bool unorm = l == 0 && up_norm_slot >= 0;
        if (l == 0 && corr)
            for (int r = 0; r < R; ++r) a.corr[r] = corr[r];
        const PassGeom g = pass_geom(c, L.N, c->cfg.nu_post, false, unorm);
        if (unorm) {
            a.norm_part = c->norm_part + (size_t)up_norm_slot * kNormVec * c->max_tiles;
            a.nblk = g.grid.x * g.grid.y;
        }
        if (g.reg)
            prof_name(c, nm, sizeof nm, "k_mg_up_reg<%s, %d, %s, %d, %d, %s>@%d", type_name(E()),
                      g.split ? 1 : R, helm ? "true" : "false", c->cfg.nu_post, kRegWaves,
                      unorm ? "true" : "false", L.N);
        else
            prof_name(c, nm, sizeof nm, "k_mg_up<%s, %d, %s, %d, %d>@%d", type_name(E()), g.split_lds ? 1 : R,
                          helm ? "true" : "false", c->cfg.nu_post, g.TX, L.N);
        ProfScope ps(c, nm, nodes * (eb * R + eb * R / 4 + eb * R + (helm ? 8.0 : 0.0) + eb * R));
        up_pass<E>(R, helm, a, c->cfg.nu_post, g, s, ps);
    }
}

// FP64 residual norms of the level-0 iterate into `slot`; with r32 set the
// residual is also stored in float (the mixed form's defect).
void resnorm(wandqs_ctx* c, int R, bool helm, const Hier<double>& hz, int slot,
             float* const* r32) {
    const wq::Level& L = c->lev[0];
    // the same tiles as the level-0 down pass: every norm slot of a solve has
    // one partial-sum layout
    const PassGeom pg = pass_geom(c, L.N, nu_pre_at(c, 0), true);
    const dim3 g = pg.grid;
    const int TX = pg.TX, TY = pg.TY;
    double* part = c->norm_part + (size_t)slot * kNormVec * c->max_tiles;
    const int nblk = g.x * g.y;
    const double* u1 = R > 1 ? hz.u0[1] : nullptr;
    const double* f1 = R > 1 ? hz.f0[1] : nullptr;
    float* o0 = r32 ? r32[0] : nullptr;
    float* o1 = (r32 && R > 1) ? r32[1] : nullptr;
    char nm[56];
    prof_name(c, nm, sizeof nm, "k_resnorm<%d, %s>%s", R, helm ? "true" : "false",
                  r32 ? "+defect" : "");
    ProfScope ps(c, nm, (double)L.N * L.N * (16.0 * R + (helm ? 8.0 : 0.0) + (r32 ? 4.0 * R : 0.0)));
    if (R == 1) {
        if (helm) WQ_KLAUNCH(ps, (k_resnorm<1, true>), g, dim3(kThreads), 0, c->stream, L.N, L.h, L.pitch, hz.u0[0], u1, hz.f0[0], f1, hz.k2, part, nblk, o0, o1, L.pitch, TX, TY);
        else WQ_KLAUNCH(ps, (k_resnorm<1, false>), g, dim3(kThreads), 0, c->stream, L.N, L.h, L.pitch, hz.u0[0], u1, hz.f0[0], f1, hz.k2, part, nblk, o0, o1, L.pitch, TX, TY);
    } else {
        if (helm) WQ_KLAUNCH(ps, (k_resnorm<2, true>), g, dim3(kThreads), 0, c->stream, L.N, L.h, L.pitch, hz.u0[0], u1, hz.f0[0], f1, hz.k2, part, nblk, o0, o1, L.pitch, TX, TY);
        else WQ_KLAUNCH(ps, (k_resnorm<2, false>), g, dim3(kThreads), 0, c->stream, L.N, L.h, L.pitch, hz.u0[0], u1, hz.f0[0], f1, hz.k2, part, nblk, o0, o1, L.pitch, TX, TY);
    }
}

// One outer iteration of the mixed form: defect r = f - A u in FP64 (stored in
// float, norms recorded in `slot`), `inner` FP32 V-cycles on A e = r from e = 0,
// then u += e in FP64.
void mixed_iteration(wandqs_ctx* c, int R, bool helm, const Hier<double>& hz, int slot) {
    wq::Level& L0 = c->lev[0];
    Hier<float> hf{{L0.u32[0], L0.u32[1]}, {L0.f32[0], L0.f32[1]}, hz.k2};
    resnorm(c, R, helm, hz, slot, hf.f0);
    const int inner = c->cfg.mg_inner_cycles > 0 ? c->cfg.mg_inner_cycles : 1;
    // the last inner cycle's finest up pass adds its result to the FP64
    // iterate (u += e) itself, unless level 0 is the coarse kernel's
    double* const corr[2] = {hz.u0[0], R > 1 ? hz.u0[1] : nullptr};
    const bool fused = c->lc > 0;
    for (int i = 0; i < inner; ++i)
        vcycle<float>(c, R, helm, hf, i == 0, -1, -1, fused && i == inner - 1 ? corr : nullptr);
    if (fused) return;
    ProfScope ps(c, "k_correct", (double)L0.N * L0.N * 20.0 * R);
    WQ_KLAUNCH(ps, k_correct, dim3((L0.N + 1 + 127) / 128, L0.N + 1), dim3(128), 0, c->stream,
                       L0.N, L0.pitch, L0.pitch, hz.u0[0], R > 1 ? hz.u0[1] : nullptr, L0.u32[0],
                       R > 1 ? L0.u32[1] : nullptr);
}

}  // namespace

int reg_tile_min_default() { return WQ_REG_TILE_MIN; }
int small_tile_max_default() { return WQ_SMALL_TILE_MAX; }

wandqs_status make_dst_tables(wandqs_ctx* c) {
    const int n1 = kDstN;
    hipLaunchKernelGGL(k_dst_tables, dim3((n1 * n1 + 255) / 256), dim3(256), 0, c->stream, n1,
                       c->lev[c->lc].h, c->dst_S, c->dst_M, c->dst_S64, c->dst_M64);
    WQ_LAUNCH_CHECK();
    return make_fst_tables(c);
}


// Launches one cycle, body() on c->stream, as a HIP graph: the graph of `key`
// is captured on c->cap_stream and instantiated at its first use and replayed
// after.  With graphs off, with the per-kernel timing on (its events belong to
// direct launches), or when a capture fails (graphs then stay off for the
// context), body() launches directly.
template <class F>
hipError_t run_cycle(wandqs_ctx* c, const CycleKey& key, F&& body) {
    if (c->graphs_on && !c->prof.on && hipPeekAtLastError() == hipSuccess) {
        for (const CycleGraph& g : c->graphs)
            if (g.key == key) return hipGraphLaunch(g.exec, c->stream);
        if ((int)c->graphs.size() < kMaxGraphs) {
            hipGraphExec_t ex = nullptr;
            bool ok = c->cap_stream ||
                      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
            if (!ok) c->cap_stream = nullptr;
            ok = ok && hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
            if (ok) {
                const hipStream_t s0 = c->stream;
                c->stream = c->cap_stream;
                body();
                c->stream = s0;
                const bool launched = hipGetLastError() == hipSuccess;
                hipGraph_t g = nullptr;
                ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && launched && g &&
                     hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
                if (g) (void)hipGraphDestroy(g);
            }
            if (ok) {
                c->graphs.push_back(CycleGraph{key, ex});
                return hipGraphLaunch(ex, c->stream);
            }
            if (ex) (void)hipGraphExecDestroy(ex);
            (void)hipGetLastError();
            c->graphs_on = false;
        }
    }
    body();
    return hipSuccess;
}

// Waits until the device has published sequence number seq (k_reduce_publish): a
// bounded spin on the coherent host word, then a stream synchronisation,
// which also reports a failed kernel.
wandqs_status wait_published(wandqs_ctx* c, const uint32_t* h_seq, uint32_t seq) {
    const auto t0 = std::chrono::steady_clock::now();
    for (long it = 0;; ++it) {
        if (__atomic_load_n(h_seq, __ATOMIC_ACQUIRE) == seq) return WANDQS_OK;
        if ((it & 1023) == 1023 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200))
            break;
        __builtin_ia32_pause();
    }
    WQ_HIP(hipStreamSynchronize(c->stream));
    if (__atomic_load_n(h_seq, __ATOMIC_ACQUIRE) == seq) return WANDQS_OK;
    c->err = "residual norms were not published by the device";
    return WANDQS_E_HIP;
}

// Solve with the context's stop rule.  Tolerance mode (mg_rtol > 0) runs a batch
// of V-cycles sized by the previous slice's count for this solve, reads the
// residual norms back once per batch and adds single cycles until every
// right-hand side meets ||r|| <= rtol ||f|| + atol sqrt(n) or reaches the
// rounding floor: either ||r|| <= kFloorBE eps (8/h^2 ||u|| + ||f||) (the
// residual is at the size that rounding in forming it leaves), or a cycle no
// longer halves ||r|| once ||r|| <= 1e-9 max(||f||, ||r_0||), r_0 the initial
// residual.
// Fixed mode runs mg_max_cycles cycles without any host synchronisation.
wandqs_status helm_levels(wandqs_ctx* c, const double* k2) {
    hipStream_t s = c->stream;
    {  // k2 on the tile levels 1..lc
        for (int l = 1; l <= c->lc; ++l) {
            const wq::Level& F = c->lev[l - 1];
            const wq::Level& C = c->lev[l];
            const double* src = l == 1 ? k2 : F.k2;
            ProfScope ps(c, "k_restrict_fw", 8.0 * ((double)(F.N + 1) * (F.N + 1) + (double)(C.N + 1) * (C.N + 1)));
            WQ_KLAUNCH(ps, k_restrict_fw, dim3((C.N + 1 + 127) / 128, C.N + 1), dim3(128), 0, s,
                               src, F.pitch, C.k2, C.pitch, C.N);
        }
        // k2 of the coarse-kernel levels, once per solve
        const wq::Level& T = c->lev[c->lc];
        const double* top = c->lc == 0 ? k2 : T.k2;
        int tot = 0;
        for (int n = T.N; n >= 2; n /= 2) tot += (n + 1) * (n + 1);
        ProfScope ps(c, "k_coarse_k2", 24.0 * tot);
        WQ_KLAUNCH(ps, k_coarse_k2, dim3(1), dim3(kCoarseThreads), 0, s, T.N, T.pitch, T.h, top,
                           c->k2lev, c->k2levf, c->idlevf);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status mg_solve(wandqs_ctx* c, int kind, int R, bool helm, double* const u[2],
                       double* const f[2], const double* k2, SolveResult* res,
                       const std::function<wandqs_status()>& ahead, bool k2_levels_ready) {
    hipStream_t s = c->stream;
    Hier<double> hz{{u[0], R > 1 ? u[1] : nullptr}, {f[0], R > 1 ? f[1] : nullptr}, k2};
    const bool mixed = c->cfg.precision == WANDQS_MIXED;
    if (helm && !k2_levels_ready) {
        const wandqs_status st = helm_levels(c, k2);
        if (st != WANDQS_OK) return st;
    }
    // one "cycle" is a V-cycle (FP64) or an outer defect-correction iteration
    // (mixed) that records its residual norms in `slot` (FP64: -1, none)
    hipError_t gerr = hipSuccess;
    // upslot >= 0 (FP64, register tiles on level 0): the cycle's finest up pass
    // records the norms of its result in slot upslot
    auto cycle = [&](int slot, int upslot, const FuseCtl& fz) {
        const int fk = (fz.skip_down0 ? 1 : 0) | (fz.fuse_up0 ? 2 : 0) | (fz.cur ? 4 : 0);
        const CycleKey key{{hz.u0[0], hz.u0[1], hz.f0[0], hz.f0[1], hz.k2}, R, helm, mixed, slot,
                           upslot, fk};
        const hipError_t e = run_cycle(c, key, [&] {
            if (mixed) mixed_iteration(c, R, helm, hz, slot);
            else vcycle<double>(c, R, helm, hz, false, slot, upslot, nullptr, &fz);
        });
        if (gerr == hipSuccess) gerr = e;
    };
    auto graph_check = [&]() -> wandqs_status {
        if (gerr == hipSuccess) return WANDQS_OK;
        c->err = std::string("hipGraphLaunch: ") + hipGetErrorString(gerr);
        return WANDQS_E_HIP;
    };
    // the down pass records the incoming residual itself unless the top level is
    // the coarse kernel (FP64) ; the mixed defect kernel always records it
    const bool separate_norm = !mixed && c->lc == 0;
    const int maxc = c->cfg.mg_max_cycles;
    if (!(c->cfg.mg_rtol > 0.0)) {
        for (int k = 0; k < maxc; ++k) cycle(mixed ? 0 : -1, -1, FuseCtl{});
        if (graph_check() != WANDQS_OK) return WANDQS_E_HIP;
        WQ_LAUNCH_CHECK();
        if (res) *res = SolveResult{maxc, {-1.0, -1.0}};
        return ahead ? ahead() : WANDQS_OK;
    }
    const int N = c->N;
    const double atol = c->cfg.mg_atol * std::sqrt((double)(N - 1) * (N - 1));
    // partial sums per tile (the level-0 tiles, for both the down pass and the
    // residual-norm kernel)
    const dim3 g = pass_geom(c, N, nu_pre_at(c, 0), true).grid;
    const int nblk = g.x * g.y;
    // the batch's last cycle records the final norms in its finest up pass
    // (register tiles, FP64) instead of a separate residual pass
    const PassGeom gu = pass_geom(c, N, c->cfg.nu_post, false, true);
    const bool up_norms = !mixed && !separate_norm && gu.reg;
    const int nblk_up = gu.grid.x * gu.grid.y;
    // inside a batch, each cycle's level-0 up pass but the last fuses with the
    // next cycle's down pass; their norm slots have the fused launch's tiles
    const bool fuse = !mixed && up_norms && fuse_possible(c);
    const dim3 fg = fuse_grid(c, R);
    const int nblk_fuse = fg.x * fg.y;
    int cur = 0;
    int done = 0;
    int pred = c->pred[kind] < 1 ? 1 : c->pred[kind];
    double* hr = c->h_pin;  // [kMaxSlots][kNormVec] + flags
    constexpr int V = kNormVec;
    const double a_norm = 8.0 / (c->lev[0].h * c->lev[0].h);  // ||L_h||_2 bound
    const double eps = std::numeric_limits<double>::epsilon();
    if (separate_norm) resnorm(c, R, helm, hz, 0, nullptr);
    while (true) {
        int b = done == 0 ? pred : 1;
        if (done + b > maxc) b = maxc - done;
        for (int k = 0; k < b; ++k) {
            const int cyc = done + k;
            FuseCtl fz;
            fz.skip_down0 = fuse && k > 0;
            fz.fuse_up0 = fuse && k < b - 1;
            fz.next_slot = cyc + 1;
            fz.cur = cur;
            cycle(mixed || c->lc > 0 ? cyc : -1, up_norms && k == b - 1 ? cyc + 1 : -1, fz);
            if (fz.fuse_up0) cur ^= 1;
            if (separate_norm) resnorm(c, R, helm, hz, cyc + 1, nullptr);
        }
        if (!separate_norm && !up_norms) resnorm(c, R, helm, hz, done + b, nullptr);
        const int s0 = done == 0 ? 0 : done + 1;
        const int ns = done + b + 1 - s0;
        if (graph_check() != WANDQS_OK) return WANDQS_E_HIP;
        WQ_LAUNCH_CHECK();
        int32_t* h_flags = reinterpret_cast<int32_t*>(hr + V * kMaxSlots);
        uint32_t* h_seq = reinterpret_cast<uint32_t*>(hr + V * kMaxSlots + 1);
        const uint32_t seq = ++c->pub_seq;
        {
            ProfScope ps(c, "k_reduce_publish", 8.0 * ns * 3 * R * (nblk + 1));
            WQ_KLAUNCH(ps, k_reduce_publish, dim3(ns * 3 * R), dim3(kThreads), 0, s,
                       c->norm_part, V * c->max_tiles, nblk, s0, 3 * R, up_norms ? done + b : -1,
                       nblk_up, fuse ? done + 1 : 0, fuse ? done + b : 0, nblk_fuse, hr, c->flags,
                       h_flags, h_seq, seq, c->pub_count);
        }
        WQ_LAUNCH_CHECK();
        // behind the first batch: the caller's follow-up work, on the device
        // while the host waits for the norms
        const bool first = done == 0;
        if (first && ahead) {
            const wandqs_status st = ahead();
            if (st != WANDQS_OK) return st;
        }
        if (wait_published(c, h_seq, seq) != WANDQS_OK) return WANDQS_E_HIP;
        done += b;
        const int32_t fl = __atomic_load_n(h_flags, __ATOMIC_ACQUIRE);
        // first cycle count at which every rhs satisfies the stop rule
        int need = -1;
        for (int k = 0; k <= done && need < 0; ++k) {
            bool all = true;
            for (int r = 0; r < R; ++r) {
                const double rr = std::sqrt(hr[V * k + 3 * r]);
                const double ff = std::sqrt(hr[V * k + 3 * r + 1]);
                const double uu = std::sqrt(hr[V * k + 3 * r + 2]);
                // relative to ||f||; for f = 0 (solution 0) relative to ||r_0||
                const double ref = ff > 0 ? ff : std::sqrt(hr[3 * r]);
                bool ok = std::isfinite(rr) && (rr <= c->cfg.mg_rtol * ref + atol ||
                                                rr <= kFloorBE * eps * (a_norm * uu + ff));
                if (!ok && k >= 2) {
                    const double rp = std::sqrt(hr[V * (k - 1) + 3 * r]);
                    const double scale = std::max(ff, std::sqrt(hr[3 * r]));
                    ok = std::isfinite(rr) && rr > 0.5 * rp && rr <= 1e-9 * scale;
                }
                all = all && ok;
            }
            if (all) need = k;
        }
        if (need >= 0 || done >= maxc || (fl & 1)) {
            if (res) {
                res->cycles = done;
                for (int r = 0; r < R; ++r) {
                    const double rr = std::sqrt(hr[V * done + 3 * r]);
                    const double ff = std::sqrt(hr[V * done + 3 * r + 1]);
                    res->rel[r] = ff > 0 ? rr / ff : rr;
                }
            }
            if (fl & 1) {
                c->err = "1 + psi <= 0 where plasma is present";
                return WANDQS_E_NONPHYS;
            }
            if (need < 0) {
                static const char* names[kPredKinds] = {"psi", "Ez/Bz", "B_perp", "user",
                                                        "psi adjoint", "Ez/Bz adjoint",
                                                        "B_perp adjoint", "?"};
                c->err = std::string("multigrid did not converge within mg_max_cycles (") +
                         names[kind & (kPredKinds - 1)] + " solve, ||r||/||f|| = " +
                         std::to_string(res ? res->rel[0] : -1.0) + ")";
                return WANDQS_E_NOCONV;
            }
            c->pred[kind] = need < 1 ? 1 : need;
            // further cycles ran after the follow-up work: it reads the final
            // iterate only when enqueued again
            if (!first && ahead) return ahead();
            return WANDQS_OK;
        }
    }
}

}  // namespace wq

