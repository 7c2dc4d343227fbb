// Plasma macroparticles: cell sort, deposits (Collect_Source), gather and push
// (Push_Trajectory), adaptive step (Step_Size_Refinement) -- WAND-PIC Sec. III.A,
// Sec. III.B and Algorithm 1.
//
// Particles are a structure of arrays x, y, px, py (float64) plus a permanent
// int32 ID.  Every slice starts with a stable-by-ID counting sort by CIC cell:
// histogram (integer atomics), exclusive scan, scatter, then each cell's
// particles are ordered by ID, so the storage order -- and every floating-point
// sum that follows -- is independent of thread timing.  Deposits are
// atomics-free: a workgroup owns a tile of nodes, one thread per cell of the
// tile (plus the one-cell rim shared with the neighbouring tiles) sums its
// particles' corner weights in registers, and each node adds its four cells'
// corners from LDS in a fixed order.
#include <algorithm>

#include "wq_common.h"

namespace wq {
namespace {

constexpr int kPushThreads = 256;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

// Cloud-in-cell cell and offset, clamped so that x = L falls in the last cell.
__device__ __forceinline__ void cic(double x, double L, double h, int N, int& c, double& d) {
    const double t = (x + L) / h;
    int k = (int)floor(t);
    k = k < 0 ? 0 : (k > N - 1 ? N - 1 : k);
    c = k;
    d = t - k;
}

// Bilinear interpolation from the four corners of a cell.
__device__ __forceinline__ double cic_gather(double f00, double f10, double f01, double f11,
                                             double dx, double dy) {
    return f00 * (1.0 - dx) * (1.0 - dy) + f10 * dx * (1.0 - dy) + f01 * (1.0 - dx) * dy +
           f11 * dx * dy;
}

// Lanes of a wave holding the same key in consecutive lanes form a run (the
// particles are stored in cell order from the previous slice, so most keys
// repeat).  Returns the run's first lane and length; one atomic per run.
__device__ __forceinline__ void key_run(int key, bool valid, int& head, int& len) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool is_head = valid && (lane == 0 || prev != key);
    const unsigned long long heads = __ballot(is_head);
    const unsigned long long live = __ballot(valid);
    // head: highest head lane <= lane; next head: lowest head lane > lane
    const unsigned long long below = heads & (lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1));
    head = 63 - __clzll(below);
    const unsigned long long above = heads & ~(lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1));
    const int end_live = 64 - __clzll(live);  // one past the last valid lane
    const int next = above ? __ffsll(above) - 1 : end_live;
    len = next - head;
}

__global__ void k_cell_key(int64_t P, const double* __restrict__ x, const double* __restrict__ y,
                           double L, double h, int N, int32_t* __restrict__ key,
                           int32_t* __restrict__ count, int32_t* __restrict__ big_n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *big_n = 0;  // list of crowded cells for k_cell_sort_big
    const bool valid = i < P;
    int k = -1;
    if (valid) {
        int a, b;
        double d;
        cic(x[i], L, h, N, a, d);
        cic(y[i], L, h, N, b, d);
        k = b * N + a;
        key[i] = k;
    }
    int head, len;
    key_run(k, valid, head, len);
    if (valid && (threadIdx.x & 63) == head) atomicAdd(&count[k], len);
}

// Exclusive scan, phase 1: each block scans kScanBlock items and emits its total.
__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int32_t* __restrict__ in,
                                                              int n, int32_t* __restrict__ out,
                                                              int32_t* __restrict__ blk) {
    __shared__ int32_t tot[kScanThreads];
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {  // inclusive Hillis-Steele over totals
        int32_t t = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = tot[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) blk[blockIdx.x] = tot[kScanThreads - 1];
}

// Phase 2: one block scans the block totals (serial chunks per thread) and
// writes the grand total to out[n].
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t* __restrict__ blk, int nb,
                                                           int32_t* __restrict__ out, int n) {
    __shared__ int32_t tot[kScanThreads];
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = threadIdx.x * per;
    int32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) s += blk[b0 + k];
    tot[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int32_t t = threadIdx.x >= off ? tot[threadIdx.x - off] : 0;
        __syncthreads();
        tot[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = tot[threadIdx.x] - s;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) {
            const int32_t t = blk[b0 + k];
            blk[b0 + k] = run;
            run += t;
        }
    if (threadIdx.x == kScanThreads - 1) out[n] = tot[kScanThreads - 1];
}

__global__ void k_scan_add(int32_t* __restrict__ out, int n, const int32_t* __restrict__ blk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += blk[i / kScanBlock];
}

// Scatter: count[] is consumed back to zero, ready for the next slice.  One
// atomic per run of equal keys; the run's lanes take consecutive slots.
__global__ void k_scatter(int64_t P, const int32_t* __restrict__ key,
                          const int32_t* __restrict__ start, int32_t* __restrict__ count,
                          int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < P;
    const int k = valid ? key[i] : -1;
    int head, len;
    key_run(k, valid, head, len);
    const int lane = threadIdx.x & 63;
    int top = 0;
    if (valid && lane == head) top = atomicSub(&count[k], len);
    top = __shfl(top, head, 64);
    if (valid) perm[start[k] + top - len + (lane - head)] = (int32_t)i;
}

// Place each particle in the new order, by cell and within a cell by
// permanent ID: the particle in slot i of the scatter's order (perm) moves to
// slot s + r of its cell, r the number of the cell's particles with a smaller
// ID (IDs are unique), and its x, y, px, py and ID are copied there.  One
// thread per slot; its cell's IDs are loaded in batches of kRankBatch so that
// their latencies overlap.  Cells of more than kSmallCell particles (blowout)
// go on a list for k_cell_sort_big.
constexpr int kSmallCell = 16;
constexpr int kRankBatch = 8;
constexpr int kBigCellLds = 4096;

struct PartArrays {
    const double *x, *y, *px, *py;
    const int32_t* id;
    double *x2, *y2, *px2, *py2;
    int32_t* id2;
    __device__ __forceinline__ void move(int32_t from, int to) const {
        x2[to] = x[from];
        y2[to] = y[from];
        px2[to] = px[from];
        py2[to] = py[from];
        id2[to] = id[from];
    }
};

__global__ void k_cell_rank(int64_t P, const int32_t* __restrict__ start,
                            const int32_t* __restrict__ perm, const int32_t* __restrict__ key,
                            PartArrays pa, int32_t* __restrict__ big,
                            int32_t* __restrict__ big_n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int32_t p = perm[i];
    const int c = key[p];
    const int s = start[c], e = start[c + 1];
    if (e - s > kSmallCell) {
        if (i == s) big[atomicAdd(big_n, 1)] = c;
        return;
    }
    const int32_t* __restrict__ id = pa.id;
    const int32_t mine = id[p];
    int r = 0;
    for (int j0 = s; j0 < e; j0 += kRankBatch) {
        int32_t q[kRankBatch];
#pragma unroll
        for (int t = 0; t < kRankBatch; ++t) q[t] = j0 + t < e ? perm[j0 + t] : p;
#pragma unroll
        for (int t = 0; t < kRankBatch; ++t) r += id[q[t]] < mine;
    }
    pa.move(p, s + r);
}

// Crowded cells, one workgroup each: the same ranks and moves.
__global__ __launch_bounds__(256) void k_cell_sort_big(const int32_t* __restrict__ start,
                                                       const int32_t* __restrict__ perm,
                                                       PartArrays pa,
                                                       const int32_t* __restrict__ big,
                                                       const int32_t* __restrict__ big_n) {
    __shared__ int32_t sid[kBigCellLds];
    const int32_t* __restrict__ id = pa.id;
    const int nbig = *big_n;
    for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
        const int c = big[b];
        const int s = start[c], n = start[c + 1] - s;
        const bool lds = n <= kBigCellLds;
        if (lds)
            for (int i = threadIdx.x; i < n; i += blockDim.x) sid[i] = id[perm[s + i]];
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const int32_t v = lds ? sid[i] : id[perm[s + i]];
            int r = 0;
            if (lds)
                for (int j = 0; j < n; ++j) r += sid[j] < v;
            else
                for (int j = 0; j < n; ++j) r += id[perm[s + j]] < v;
            pa.move(perm[s + i], s + r);
        }
        __syncthreads();
    }
}

// particles per batch of loads in the deposits (latencies overlap; the sums
// keep the cell's particle order), one thread per cell of a tile's
// (tile + 1)^2 cells.  The density deposit uses kDepTile = 16 (five
// wavefronts); the current and stress deposit, whose LDS sets the occupancy,
// 15 x 15 node tiles (16 x 16 cells, four wavefronts: the fastest measured of
// 8..16).
constexpr int kDepBatch = 8, kDepBatchJ = 4;
#ifndef WQ_DEP_TILE_J
#define WQ_DEP_TILE_J 15
#endif
#ifndef WQ_DEP_THREADS_J
#define WQ_DEP_THREADS_J 256
#endif
constexpr int kDepThreads = 320, kDepTileJ = WQ_DEP_TILE_J, kDepThreadsJ = WQ_DEP_THREADS_J;
static_assert((kDepTile + 1) * (kDepTile + 1) <= kDepThreads, "one cell per deposit thread");

// n* = deposit(1) (Sec. III.B: surface density) and the psi right-hand side
// n* - n0 (eq. (12)) on the interior nodes.
template <int TN>
__global__ __launch_bounds__(kDepThreads) void k_deposit_n(int N, double L, double h, double wdep,
                                                   double n0, int pitch,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const int32_t* __restrict__ start,
                                                   double* __restrict__ nstar,
                                                   double* __restrict__ fpsi) {
    constexpr int TC = TN + 1;
    __shared__ double corner[TC * TC][4];
    int tbx, tby;
    tile_of_block(tbx, tby);
    const int a0 = tbx * TN, b0 = tby * TN;
    for (int c = threadIdx.x; c < TC * TC; c += blockDim.x) {
        const int cy = c / TC, cx = c - cy * TC;
        const int ga = a0 - 1 + cx, gb = b0 - 1 + cy;
        double s00 = 0.0, s10 = 0.0, s01 = 0.0, s11 = 0.0;
        if (ga >= 0 && ga < N && gb >= 0 && gb < N) {
            const int cell = gb * N + ga;
            const int k1 = start[cell + 1];
            // the cell's particles in order, loaded kDepBatch at a time
            for (int k0 = start[cell]; k0 < k1; k0 += kDepBatch) {
                double xv[kDepBatch], yv[kDepBatch];
#pragma unroll
                for (int t = 0; t < kDepBatch; ++t) {
                    xv[t] = k0 + t < k1 ? x[k0 + t] : 0.0;
                    yv[t] = k0 + t < k1 ? y[k0 + t] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < kDepBatch; ++t) {
                    if (k0 + t >= k1) break;
                    const double dx = (xv[t] + L) / h - ga;
                    const double dy = (yv[t] + L) / h - gb;
                    s00 += (1.0 - dx) * (1.0 - dy);
                    s10 += dx * (1.0 - dy);
                    s01 += (1.0 - dx) * dy;
                    s11 += dx * dy;
                }
            }
        }
        corner[c][0] = s00;
        corner[c][1] = s10;
        corner[c][2] = s01;
        corner[c][3] = s11;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TN * TN; i += blockDim.x) {
        const int ny = i / TN, nx = i - ny * TN;
        const int ga = a0 + nx, gb = b0 + ny;
        if (ga > N || gb > N) continue;
        // node (ga, gb) is corner 11 of cell (ga-1, gb-1), 01 of (ga, gb-1),
        // 10 of (ga-1, gb) and 00 of (ga, gb)
        const double v = (corner[ny * TC + nx][3] + corner[ny * TC + nx + 1][2] +
                          corner[(ny + 1) * TC + nx][1] + corner[(ny + 1) * TC + nx + 1][0]) *
                         wdep;
        const size_t g = (size_t)gb * pitch + ga;
        nstar[g] = v;
        const bool interior = ga >= 1 && gb >= 1 && ga <= N - 1 && gb <= N - 1;
        fpsi[g] = interior ? v - n0 : 0.0;
    }
}

// Gather psi to each particle: g_i = 1 + psi_i (> 0 or the NONPHYS flag),
// V_i = p_i / g_i (eq. (6)); deposit j = n*<V> (eq. (9)) and T = n*<V V>
// (below eq. (16)).  Output order: jx, jy, Txx, Txy, Tyy.
template <int TN>
__global__ __launch_bounds__(kDepThreadsJ) void k_deposit_jT(int N, double L, double h, double wdep,
                                                    int pitch, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ px,
                                                    const double* __restrict__ py,
                                                    const int32_t* __restrict__ start,
                                                    const double* __restrict__ psi,
                                                    double* __restrict__ jx,
                                                    double* __restrict__ jy,
                                                    double* __restrict__ txx,
                                                    double* __restrict__ txy,
                                                    double* __restrict__ tyy,
                                                    int32_t* __restrict__ flags) {
    constexpr int TC = TN + 1;
    constexpr int M = 5;
    __shared__ double corner[TC * TC][4 * M];
    int tbx, tby;
    tile_of_block(tbx, tby);
    const int a0 = tbx * TN, b0 = tby * TN;
    bool bad = false;
    for (int c = threadIdx.x; c < TC * TC; c += blockDim.x) {
        const int cy = c / TC, cx = c - cy * TC;
        const int ga = a0 - 1 + cx, gb = b0 - 1 + cy;
        double s[4][M];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) s[q][m] = 0.0;
        if (ga >= 0 && ga < N && gb >= 0 && gb < N) {
            const int cell = gb * N + ga;
            const size_t g = (size_t)gb * pitch + ga;
            const double p00 = psi[g], p10 = psi[g + 1], p01 = psi[g + pitch],
                         p11 = psi[g + pitch + 1];
            const int k1 = start[cell + 1];
            // the cell's particles in order, loaded kDepBatchJ at a time
            for (int k0 = start[cell]; k0 < k1; k0 += kDepBatchJ) {
                double xv[kDepBatchJ], yv[kDepBatchJ], pxv[kDepBatchJ], pyv[kDepBatchJ];
#pragma unroll
                for (int t = 0; t < kDepBatchJ; ++t) {
                    const bool in = k0 + t < k1;
                    xv[t] = in ? x[k0 + t] : 0.0;
                    yv[t] = in ? y[k0 + t] : 0.0;
                    pxv[t] = in ? px[k0 + t] : 0.0;
                    pyv[t] = in ? py[k0 + t] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < kDepBatchJ; ++t) {
                    if (k0 + t >= k1) break;
                    const double dx = (xv[t] + L) / h - ga;
                    const double dy = (yv[t] + L) / h - gb;
                    const double gi = 1.0 + cic_gather(p00, p10, p01, p11, dx, dy);
                    bad |= !(gi > 0.0);
                    const double ig = 1.0 / gi;
                    const double vx = pxv[t] * ig, vy = pyv[t] * ig;
                    const double q[M] = {vx, vy, vx * vx, vx * vy, vy * vy};
                    const double w[4] = {(1.0 - dx) * (1.0 - dy), dx * (1.0 - dy),
                                         (1.0 - dx) * dy, dx * dy};
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
    if (bad) atomicOr(flags, 1);
    __syncthreads();
    double* out[M] = {jx, jy, txx, txy, tyy};
    for (int i = threadIdx.x; i < TN * TN; i += blockDim.x) {
        const int ny = i / TN, nx = i - ny * TN;
        const int ga = a0 + nx, gb = b0 + ny;
        if (ga > N || gb > N) continue;
        const size_t g = (size_t)gb * pitch + ga;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const double v = (corner[ny * TC + nx][3 * M + m] + corner[ny * TC + nx + 1][2 * M + m] +
                              corner[(ny + 1) * TC + nx][1 * M + m] +
                              corner[(ny + 1) * TC + nx + 1][0 * M + m]) *
                             wdep;
            out[m][g] = v;
        }
    }
}

// d psi / dx at node (a, b): central inside, one-sided on the boundary columns
// (ih = 1/h, ih2 = 1/(2h)).  The three values are loaded unconditionally
// (indices clamped into the row) and the formula selected after, so that no
// load waits behind a branch.
__device__ __forceinline__ double grad_x(const double* psi, int pitch, int N, double ih,
                                         double ih2, int a, int b) {
    const double* r = psi + (size_t)b * pitch;
    const double pl = r[a > 0 ? a - 1 : 0], pc = r[a], pr = r[a < N ? a + 1 : N];
    return a == 0 ? (pr - pc) * ih : (a == N ? (pc - pl) * ih : (pr - pl) * ih2);
}

__device__ __forceinline__ double grad_y(const double* psi, int pitch, int N, double ih,
                                         double ih2, int a, int b) {
    const double pl = psi[(size_t)(b > 0 ? b - 1 : 0) * pitch + a];
    const double pc = psi[(size_t)b * pitch + a];
    const double pr = psi[(size_t)(b < N ? b + 1 : N) * pitch + a];
    return b == 0 ? (pr - pc) * ih : (b == N ? (pc - pl) * ih : (pr - pl) * ih2);
}

// grad psi at every node (grad_x, grad_y above) into two node arrays, once per
// slice, so that the push gathers it like the other fields.
__global__ void k_grad_psi(int N, double h, int pitch, const double* __restrict__ psi,
                           double* __restrict__ gx, double* __restrict__ gy) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (a > N) return;
    const double ih = 1.0 / h, ih2 = 0.5 * ih;
    const size_t g = (size_t)b * pitch + a;
    gx[g] = grad_x(psi, pitch, N, ih, ih2, a, b);
    gy[g] = grad_y(psi, pitch, N, ih, ih2, a, b);
}

// Nodes a and a + 1 of a row in one 16-byte load (8-byte aligned).
__device__ __forceinline__ double2 ld_pair(const double* p) {
    double2 v;
    __builtin_memcpy(&v, p, sizeof(v));
    return v;
}

// Boris-like push over dxi with the fields frozen at this slice (eqs. (6)-(7)):
// half kick by F = (gamma grad psi - grad(a2/4)) / g + e_z x B_perp with
// gamma = (1 + p^2 + g^2 + a2/2)/(2g) from the old momentum, rotation by the
// (e_z x V) Bz term through angle 2 atan(Bz dxi / 2g), half kick, drift with
// the new momentum, specular walls.  LAS: a laser envelope's a2 = |A-hat|^2
// and its node gradient (ax, ay) are gathered too (else a2 = 0).  Emits the
// block maximum of |p_new| / g_i for Algorithm 1.
template <bool LAS>
__global__ __launch_bounds__(kPushThreads) void k_push(
    int64_t P, int N, double L, double h, int pitch, const double* __restrict__ st,
    const double* __restrict__ psi, const double* __restrict__ gpx, const double* __restrict__ gpy,
    const double* __restrict__ Bx, const double* __restrict__ By,
    const double* __restrict__ Bz, const double* __restrict__ la2, const double* __restrict__ lax,
    const double* __restrict__ lay, double* __restrict__ x, double* __restrict__ y,
    double* __restrict__ px, double* __restrict__ py, double* __restrict__ vmax_part) {
    __shared__ double red[kPushThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < P) {
        const double dxi = st[1];
        double xi_ = x[i], yi = y[i], pxi = px[i], pyi = py[i];
        int a, b;
        double dx, dy;
        cic(xi_, L, h, N, a, dx);
        cic(yi, L, h, N, b, dy);
        // the cell's four nodes: (a, a + 1) of rows b and b + 1 (a + 1 <= N < pitch)
        const size_t g = (size_t)b * pitch + a;
        const double2 p0 = ld_pair(psi + g), p1 = ld_pair(psi + g + pitch);
        const double2 x0 = ld_pair(gpx + g), x1 = ld_pair(gpx + g + pitch);
        const double2 y0 = ld_pair(gpy + g), y1 = ld_pair(gpy + g + pitch);
        const double2 bx0 = ld_pair(Bx + g), bx1 = ld_pair(Bx + g + pitch);
        const double2 by0 = ld_pair(By + g), by1 = ld_pair(By + g + pitch);
        const double2 bz0 = ld_pair(Bz + g), bz1 = ld_pair(Bz + g + pitch);
        const double g_i = 1.0 + cic_gather(p0.x, p0.y, p1.x, p1.y, dx, dy);
        const double Gx = cic_gather(x0.x, x0.y, x1.x, x1.y, dx, dy);
        const double Gy = cic_gather(y0.x, y0.y, y1.x, y1.y, dx, dy);
        const double bx = cic_gather(bx0.x, bx0.y, bx1.x, bx1.y, dx, dy);
        const double by = cic_gather(by0.x, by0.y, by1.x, by1.y, dx, dy);
        const double bz = cic_gather(bz0.x, bz0.y, bz1.x, bz1.y, dx, dy);
        double a2 = 0.0, ax = 0.0, ay = 0.0;
        if (LAS) {
            const double2 q0 = ld_pair(la2 + g), q1 = ld_pair(la2 + g + pitch);
            const double2 u0 = ld_pair(lax + g), u1 = ld_pair(lax + g + pitch);
            const double2 v0 = ld_pair(lay + g), v1 = ld_pair(lay + g + pitch);
            a2 = cic_gather(q0.x, q0.y, q1.x, q1.y, dx, dy);
            ax = cic_gather(u0.x, u0.y, u1.x, u1.y, dx, dy);
            ay = cic_gather(v0.x, v0.y, v1.x, v1.y, dx, dy);
        }

        const double ig = 1.0 / g_i;
        const double gamma = (1.0 + pxi * pxi + pyi * pyi + g_i * g_i + 0.5 * a2) * (0.5 * ig);
        const double Fx = (gamma * Gx - 0.25 * ax) * ig - by;
        const double Fy = (gamma * Gy - 0.25 * ay) * ig + bx;
        const double mx = pxi + 0.5 * dxi * Fx;
        const double my = pyi + 0.5 * dxi * Fy;
        const double t = bz * dxi * (0.5 * ig);
        const double s = 2.0 * t / (1.0 + t * t);
        const double qx = mx - t * my;
        const double qy = my + t * mx;
        const double rx = mx - s * qy;
        const double ry = my + s * qx;
        pxi = rx + 0.5 * dxi * Fx;
        pyi = ry + 0.5 * dxi * Fy;
        xi_ = xi_ + dxi * pxi * ig;
        yi = yi + dxi * pyi * ig;
        if (xi_ > L) { xi_ = 2.0 * L - xi_; pxi = -pxi; }
        if (xi_ < -L) { xi_ = -2.0 * L - xi_; pxi = -pxi; }
        if (yi > L) { yi = 2.0 * L - yi; pyi = -pyi; }
        if (yi < -L) { yi = -2.0 * L - yi; pyi = -pyi; }
        x[i] = xi_;
        y[i] = yi;
        px[i] = pxi;
        py[i] = pyi;
        v = sqrt(pxi * pxi + pyi * pyi) / g_i;  // decides the step: same arithmetic as Algorithm 1
    }
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kPushThreads / 64; ++w) m = fmax(m, red[w]);
        vmax_part[blockIdx.x] = m;
    }
}

// Frozen slice fields for the Runge-Kutta pushers: psi, its node gradient,
// B_perp and B_z, and a laser envelope's |A-hat|^2 with its node gradient
// (null without a laser), gathered (CIC) at any position.
struct PushFields {
    int N, pitch;
    double L, h;
    const double *psi, *gx, *gy, *Bx, *By, *Bz;
    const double *a2, *ax, *ay;
};

// Right-hand side of the equations of motion at s = (x, y, p_x, p_y) (Sec.
// III.A eqs. (6)-(7)): dr/dxi = p/g, dp/dxi = (gamma grad psi - grad(a2/4))/g
// + (e_z x V) B_z + e_z x B_perp with g = 1 + psi and gamma = (1 + p^2 + g^2 +
// a2/2)/(2g), every field gathered at s.  Returns g.
__device__ __forceinline__ double eom_rhs(const PushFields& F, const double (&s)[4],
                                          double (&d)[4]) {
    int a, b;
    double dx, dy;
    cic(s[0], F.L, F.h, F.N, a, dx);
    cic(s[1], F.L, F.h, F.N, b, dy);
    const size_t g = (size_t)b * F.pitch + a;
    const double2 p0 = ld_pair(F.psi + g), p1 = ld_pair(F.psi + g + F.pitch);
    const double2 x0 = ld_pair(F.gx + g), x1 = ld_pair(F.gx + g + F.pitch);
    const double2 y0 = ld_pair(F.gy + g), y1 = ld_pair(F.gy + g + F.pitch);
    const double2 bx0 = ld_pair(F.Bx + g), bx1 = ld_pair(F.Bx + g + F.pitch);
    const double2 by0 = ld_pair(F.By + g), by1 = ld_pair(F.By + g + F.pitch);
    const double2 bz0 = ld_pair(F.Bz + g), bz1 = ld_pair(F.Bz + g + F.pitch);
    const double gg = 1.0 + cic_gather(p0.x, p0.y, p1.x, p1.y, dx, dy);
    const double Gx = cic_gather(x0.x, x0.y, x1.x, x1.y, dx, dy);
    const double Gy = cic_gather(y0.x, y0.y, y1.x, y1.y, dx, dy);
    const double bx = cic_gather(bx0.x, bx0.y, bx1.x, bx1.y, dx, dy);
    const double by = cic_gather(by0.x, by0.y, by1.x, by1.y, dx, dy);
    const double bz = cic_gather(bz0.x, bz0.y, bz1.x, bz1.y, dx, dy);
    double a2 = 0.0, ax = 0.0, ay = 0.0;
    if (F.a2) {
        const double2 q0 = ld_pair(F.a2 + g), q1 = ld_pair(F.a2 + g + F.pitch);
        const double2 u0 = ld_pair(F.ax + g), u1 = ld_pair(F.ax + g + F.pitch);
        const double2 v0 = ld_pair(F.ay + g), v1 = ld_pair(F.ay + g + F.pitch);
        a2 = cic_gather(q0.x, q0.y, q1.x, q1.y, dx, dy);
        ax = cic_gather(u0.x, u0.y, u1.x, u1.y, dx, dy);
        ay = cic_gather(v0.x, v0.y, v1.x, v1.y, dx, dy);
    }
    const double ig = 1.0 / gg;
    const double gamma = (1.0 + s[2] * s[2] + s[3] * s[3] + gg * gg + 0.5 * a2) * (0.5 * ig);
    const double vx = s[2] * ig, vy = s[3] * ig;
    d[0] = vx;
    d[1] = vy;
    d[2] = (gamma * Gx - 0.25 * ax) * ig - vy * bz - by;
    d[3] = (gamma * Gy - 0.25 * ay) * ig + vx * bz + bx;
    return gg;
}

// Runge-Kutta push over dxi with the fields frozen at this slice, the
// alternative to the Boris-like push (Sec. VII.A): ORDER 1 (forward Euler), 2
// (midpoint rule) or 4 (classical four stages); each stage gathers at its own
// position.  Walls, V_max (with g at the start position) and the block maxima
// as in k_push; a stage with g <= 0 raises flags bit 0.
template <int ORDER>
__global__ __launch_bounds__(kPushThreads) void k_push_rk(int64_t P, PushFields F,
                                                          const double* __restrict__ st,
                                                          double* __restrict__ x, double* __restrict__ y,
                                                          double* __restrict__ px, double* __restrict__ py,
                                                          double* __restrict__ vmax_part,
                                                          int32_t* __restrict__ flags) {
    __shared__ double red[kPushThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < P) {
        const double dxi = st[1], L = F.L;
        const double s0[4] = {x[i], y[i], px[i], py[i]};
        double k1[4], k2[4], k3[4], k4[4], s[4], o[4];
        const double g_i = eom_rhs(F, s0, k1);
        bool bad = !(g_i > 0.0);
        if (ORDER == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = s0[q] + dxi * k1[q];
        } else if (ORDER == 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k1[q];
            bad = !(eom_rhs(F, s, k2) > 0.0) || bad;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = s0[q] + dxi * k2[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k1[q];
            bad = !(eom_rhs(F, s, k2) > 0.0) || bad;
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = s0[q] + (0.5 * dxi) * k2[q];
            bad = !(eom_rhs(F, s, k3) > 0.0) || bad;
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = s0[q] + dxi * k3[q];
            bad = !(eom_rhs(F, s, k4) > 0.0) || bad;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                o[q] = s0[q] + (dxi / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
        }
        if (o[0] > L) { o[0] = 2.0 * L - o[0]; o[2] = -o[2]; }
        if (o[0] < -L) { o[0] = -2.0 * L - o[0]; o[2] = -o[2]; }
        if (o[1] > L) { o[1] = 2.0 * L - o[1]; o[3] = -o[3]; }
        if (o[1] < -L) { o[1] = -2.0 * L - o[1]; o[3] = -o[3]; }
        x[i] = o[0];
        y[i] = o[1];
        px[i] = o[2];
        py[i] = o[3];
        v = sqrt(o[2] * o[2] + o[3] * o[3]) / g_i;
        if (bad) atomicOr(flags, 1);
    }
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kPushThreads / 64; ++w) m = fmax(m, red[w]);
        vmax_part[blockIdx.x] = m;
    }
}

// Step_Size_Refinement (Algorithm 1) with the floor dxi0/k (Sec. V.A); writes
// the slice record (xi, dxi, vmax, flags) and advances xi.  One block; each
// thread issues its loads of the push-block maxima in batches of kDxiBatch so
// that their latencies overlap (max is exact in any order).
constexpr int kDxiThreads = 1024, kDxiBatch = 8;
__global__ __launch_bounds__(kDxiThreads) void k_dxi(int nparts,
                                                     const double* __restrict__ vmax_part,
                                                     double* __restrict__ st, double dxi0,
                                                     double h, int adaptive, int refine_k,
                                                     const int32_t* __restrict__ flags,
                                                     double* __restrict__ rec) {
    __shared__ double red[kDxiThreads / 64];
    double v = 0.0;
    for (int b0 = threadIdx.x; b0 < nparts; b0 += kDxiBatch * kDxiThreads) {
        double w[kDxiBatch];
#pragma unroll
        for (int q = 0; q < kDxiBatch; ++q) {
            const int b = b0 + q * kDxiThreads;
            w[q] = b < nparts ? vmax_part[b] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kDxiBatch; ++q) v = fmax(v, w[q]);
    }
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double vmax = red[0];
    for (int q = 1; q < kDxiThreads / 64; ++q) vmax = fmax(vmax, red[q]);
    // Step_Size_Refinement: the step that keeps the fastest particle within one
    // cell, capped at dxi0 and floored at dxi0 / k
    double d = dxi0;
    if (adaptive && vmax > 0.0) {
        d = fmin(dxi0, h / vmax);
        if (refine_k > 0) d = fmax(d, dxi0 / refine_k);
    }
    if (rec) {
        rec[0] = st[0];
        rec[1] = st[1];
        rec[2] = vmax;
        rec[3] = (double)flags[0];
    }
    st[5] = st[4];  // the fields now stored belong to this slice
    st[4] = st[3];
    st[3] = st[2];
    st[2] = st[0];
    st[0] = st[0] + st[1];
    st[1] = d;
}

__global__ void k_to_id_order(int64_t P, const int32_t* __restrict__ id,
                              const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ px, const double* __restrict__ py,
                              double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    const int64_t k = id[j];
    out[k] = x[j];
    out[P + k] = y[j];
    out[2 * P + k] = px[j];
    out[3 * P + k] = py[j];
}

__global__ void k_from_id_order(int64_t P, const double* __restrict__ in, double* __restrict__ x,
                                double* __restrict__ y, double* __restrict__ px,
                                double* __restrict__ py, int32_t* __restrict__ id) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    x[k] = in[k];
    y[k] = in[P + k];
    px[k] = in[2 * P + k];
    py[k] = in[3 * P + k];
    id[k] = (int32_t)k;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

wandqs_status slice_sort(wandqs_ctx* c) {
    hipStream_t s = c->stream;
    const int a = c->cur, b = 1 - c->cur;
    const int ncell = c->N * c->N;
    {
        ProfScope ps(c, "k_cell_key", (double)c->P * 20.0 + (double)ncell * 8.0);
        WQ_KLAUNCH(ps, k_cell_key, dim3(blocks_for(c->P, 256)), dim3(256), 0, s, c->P,
                           c->pa[a][0], c->pa[a][1], c->L, c->h, c->N, c->key, c->cell_count,
                           c->big_count);
    }
    const int nb = (ncell + kScanBlock - 1) / kScanBlock;
    {
        ProfScope ps(c, "k_scan_blocks", (double)ncell * 8.0);
        WQ_KLAUNCH(ps, k_scan_blocks, dim3(nb), dim3(kScanThreads), 0, s, c->cell_count, ncell,
                           c->cell_start, c->scan_blk);
    }
    {
        ProfScope ps(c, "k_scan_top", 8.0 * nb);
        WQ_KLAUNCH(ps, k_scan_top, dim3(1), dim3(kScanThreads), 0, s, c->scan_blk, nb,
                           c->cell_start, ncell);
    }
    {
        ProfScope ps(c, "k_scan_add", (double)ncell * 8.0);
        WQ_KLAUNCH(ps, k_scan_add, dim3(blocks_for(ncell, 256)), dim3(256), 0, s, c->cell_start,
                           ncell, c->scan_blk);
    }
    {
        ProfScope ps(c, "k_scatter", (double)c->P * 12.0 + (double)ncell * 8.0);
        WQ_KLAUNCH(ps, k_scatter, dim3(blocks_for(c->P, 256)), dim3(256), 0, s, c->P, c->key,
                           c->cell_start, c->cell_count, c->perm);
    }
    const PartArrays pa{c->pa[a][0], c->pa[a][1], c->pa[a][2], c->pa[a][3], c->pid[a],
                        c->pa[b][0], c->pa[b][1], c->pa[b][2], c->pa[b][3], c->pid[b]};
    {
        ProfScope ps(c, "k_cell_rank", (double)c->P * 88.0 + (double)ncell * 4.0);
        WQ_KLAUNCH(ps, k_cell_rank, dim3(blocks_for(c->P, 256)), dim3(256), 0, s, c->P,
                           c->cell_start, c->perm, c->key, pa, c->big_cells, c->big_count);
    }
    {
        ProfScope ps(c, "k_cell_sort_big", 0.0);
        WQ_KLAUNCH(ps, k_cell_sort_big, dim3(std::min(ncell, 512)), dim3(256), 0, s,
                           c->cell_start, c->perm, pa, c->big_cells, c->big_count);
    }
    WQ_LAUNCH_CHECK();
    c->cur = b;
    return WANDQS_OK;
}

wandqs_status deposit_n(wandqs_ctx* c) {
    const int nt = (c->N + 1 + kDepTile - 1) / kDepTile;
    const double wdep = c->cfg.n0 / c->ppc;
    {
        ProfScope ps(c, "k_deposit_n<16>", (double)c->P * 16.0 + (double)c->N * c->N * 4.0 + (double)(c->N + 1) * (c->N + 1) * 16.0);
        WQ_KLAUNCH(ps, (k_deposit_n<kDepTile>), dim3(nt, nt), dim3(kDepThreads), 0, c->stream, c->N, c->L,
                           c->h, wdep, c->cfg.n0, c->lev[0].pitch, c->pa[c->cur][0], c->pa[c->cur][1],
                           c->cell_start, c->mom[0], c->lev[0].f[0]);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status deposit_jT(wandqs_ctx* c) {
    const int nt = (c->N + 1 + kDepTileJ - 1) / kDepTileJ;
    const double wdep = c->cfg.n0 / c->ppc;
    const int k = c->cur;
    {
        ProfScope ps(c, "k_deposit_jT<15>", (double)c->P * 32.0 + (double)c->N * c->N * 4.0 + (double)(c->N + 1) * (c->N + 1) * 48.0);
        WQ_KLAUNCH(ps, (k_deposit_jT<kDepTileJ>), dim3(nt, nt), dim3(kDepThreadsJ), 0, c->stream, c->N, c->L,
                           c->h, wdep, c->lev[0].pitch, c->pa[k][0], c->pa[k][1], c->pa[k][2],
                           c->pa[k][3], c->cell_start, c->fields[0], c->mom[1], c->mom[2], c->mom[3],
                           c->mom[4], c->mom[5], c->flags);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

// grad_ready: grad psi (gpsi) is made already (node_gradient of fields[0]).
wandqs_status push_and_step(wandqs_ctx* c, int rec_slot, bool grad_ready) {
    const int k = c->cur;
    if (!grad_ready) {
        ProfScope pg(c, "k_grad_psi", (double)(c->N + 1) * (c->N + 1) * 24.0);
        WQ_KLAUNCH(pg, k_grad_psi, dim3((c->N + 1 + 127) / 128, c->N + 1), dim3(128), 0, c->stream,
                           c->N, c->h, c->lev[0].pitch, c->fields[0], c->gpsi[0], c->gpsi[1]);
    }
    const int pusher = c->cfg.pusher;
    const bool las = c->las_on;
    if (pusher == WANDQS_PUSH_BORIS && !las) {
        ProfScope ps(c, "k_push", (double)c->P * 64.0 + (double)(c->N + 1) * (c->N + 1) * 48.0);
        WQ_KLAUNCH(ps, k_push<false>, dim3(c->n_push_blocks), dim3(kPushThreads), 0, c->stream, c->P,
                           c->N, c->L, c->h, c->lev[0].pitch, c->st, c->fields[0], c->gpsi[0],
                           c->gpsi[1], c->fields[3], c->fields[4], c->fields[2], nullptr, nullptr,
                           nullptr, c->pa[k][0], c->pa[k][1], c->pa[k][2], c->pa[k][3], c->vmax_part);
    } else if (pusher == WANDQS_PUSH_BORIS) {
        ProfScope ps(c, "k_push<laser>", (double)c->P * 64.0 + (double)(c->N + 1) * (c->N + 1) * 72.0);
        WQ_KLAUNCH(ps, k_push<true>, dim3(c->n_push_blocks), dim3(kPushThreads), 0, c->stream, c->P,
                           c->N, c->L, c->h, c->lev[0].pitch, c->st, c->fields[0], c->gpsi[0],
                           c->gpsi[1], c->fields[3], c->fields[4], c->fields[2], c->las_a2,
                           c->las_g[0], c->las_g[1], c->pa[k][0], c->pa[k][1], c->pa[k][2],
                           c->pa[k][3], c->vmax_part);
    } else {
        const PushFields F{c->N, c->lev[0].pitch, c->L, c->h, c->fields[0], c->gpsi[0], c->gpsi[1],
                           c->fields[3], c->fields[4], c->fields[2], las ? c->las_a2 : nullptr,
                           las ? c->las_g[0] : nullptr, las ? c->las_g[1] : nullptr};
        // per particle: its state read and written; per node (read once): six fields
        const double bytes = (double)c->P * 64.0 + (double)(c->N + 1) * (c->N + 1) * 48.0;
        const dim3 g(c->n_push_blocks), b(kPushThreads);
        if (pusher == WANDQS_PUSH_RK1) {
            ProfScope ps(c, "k_push_rk<1>", bytes);
            WQ_KLAUNCH(ps, k_push_rk<1>, g, b, 0, c->stream, c->P, F, c->st, c->pa[k][0], c->pa[k][1],
                       c->pa[k][2], c->pa[k][3], c->vmax_part, c->flags);
        } else if (pusher == WANDQS_PUSH_RK2) {
            ProfScope ps(c, "k_push_rk<2>", bytes);
            WQ_KLAUNCH(ps, k_push_rk<2>, g, b, 0, c->stream, c->P, F, c->st, c->pa[k][0], c->pa[k][1],
                       c->pa[k][2], c->pa[k][3], c->vmax_part, c->flags);
        } else {
            ProfScope ps(c, "k_push_rk<4>", bytes);
            WQ_KLAUNCH(ps, k_push_rk<4>, g, b, 0, c->stream, c->P, F, c->st, c->pa[k][0], c->pa[k][1],
                       c->pa[k][2], c->pa[k][3], c->vmax_part, c->flags);
        }
    }
    double* rec = rec_slot >= 0 ? c->rec + 4 * (size_t)rec_slot : nullptr;
    {
        ProfScope ps(c, "k_dxi", 8.0 * c->n_push_blocks);
        WQ_KLAUNCH(ps, k_dxi, dim3(1), dim3(kDxiThreads), 0, c->stream, c->n_push_blocks, c->vmax_part,
                           c->st, c->cfg.dxi0, c->h, c->cfg.adaptive, c->cfg.refine_k, c->flags, rec);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status node_gradient(wandqs_ctx* c, const double* u, double* gx, double* gy) {
    {
        ProfScope pg(c, "k_grad_psi", (double)(c->N + 1) * (c->N + 1) * 24.0);
        WQ_KLAUNCH(pg, k_grad_psi, dim3((c->N + 1 + 127) / 128, c->N + 1), dim3(128), 0, c->stream,
                           c->N, c->h, c->lev[0].pitch, u, gx, gy);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status particles_to_id_order(wandqs_ctx* c, double* dst) {
    const int k = c->cur;
    {
        ProfScope ps(c, "k_to_id_order", (double)c->P * 68.0);
        WQ_KLAUNCH(ps, k_to_id_order, dim3(blocks_for(c->P, 256)), dim3(256), 0, c->stream, c->P,
                           c->pid[k], c->pa[k][0], c->pa[k][1], c->pa[k][2], c->pa[k][3], dst);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

wandqs_status particles_from_id_order(wandqs_ctx* c, const double* src) {
    const int k = c->cur;
    {
        ProfScope ps(c, "k_from_id_order", (double)c->P * 68.0);
        WQ_KLAUNCH(ps, k_from_id_order, dim3(blocks_for(c->P, 256)), dim3(256), 0, c->stream, c->P,
                           src, c->pa[k][0], c->pa[k][1], c->pa[k][2], c->pa[k][3], c->pid[k]);
    }
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

}  // namespace wq
