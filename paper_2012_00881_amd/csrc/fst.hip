// Exact Poisson solve on the level just below the finest by fast sine
// transforms, FP64 (the coarse-grid correction of the Poisson V-cycles of
// eqs. (12)-(15), Sec. III.B; the five-point operator of Sec. VII.B on a
// uniform grid).
//
// With zero Dirichlet values the five-point Laplacian of an n x n-cell level
// of spacing H has the eigenvectors sin(pi i k / n) sin(pi j l / n) (1 <= k, l
// <= n - 1) and the eigenvalues -(4 / H^2) (sin^2(pi k / 2n) + sin^2(pi l / 2n)),
// so u = (2/n)^2 S (S f S ./ lambda) S with the sine matrix S.
//
// The sine transform X_k = sum_{j=1}^{n-1} x_j sin(pi j k / n) of one real row
// comes from the real DFT Y of length n of
//     y_j = sin(pi j / n) (x_j + x_{n-j}) + (x_j - x_{n-j}) / 2   (x_0 = x_n = 0):
// the symmetric part x_j + x_{n-j}, weighted by sin(pi j / n), turns
// cos(2 pi j k / n) into a difference of odd-frequency sines and the
// antisymmetric part gives the even-frequency ones, so
//     X_2k = -Im Y_k,   X_2k+1 = X_2k-1 + Re Y_k   (X_1 = Re Y_0 / 2),
// the odd coefficients a prefix sum.  Y comes from one complex FFT of length
// n/2 of z_m = y_2m + i y_2m+1 (Y_k = E_k + W_n^k O_k, E and O the transforms
// of the even and odd samples, from Z_k and conj(Z_{n/2-k})).
//
// One wavefront transforms one row: a Stockham (self-sorting) radix-4 FFT
// (one radix-2 stage last for an odd power of two) whose stages exchange
// through LDS (one pad slot per 16 doubles) with no workgroup barrier, since a
// wavefront's LDS operations complete in order.  Three launches; T1 and T2 are
// stored transposed, so that every pass reads whole rows and only the writes
// of the first two are scattered (two rows per workgroup, written in pairs):
//   x: row g of f -> column g of T1 (T1[k-1][g-1] = coefficient k);
//   y: row k-1 of T1 -> transform, divide by lambda, transform back ->
//      column k-1 of T2 (T2[j-1][k-1], j the y-node);
//   x inverse: row j-1 of T2 -> row j of u.
// A first form with two rows packed into one complex FFT of length 2n (the
// odd extensions; 256 threads and a barrier per stage) measured 9.7 / 6.6 /
// 5.3 us for the y / x inverse / x passes at n = 512, this one 7.5 / 5.4 /
// 5.4.
#include <cstdio>

#include "wq_common.h"

namespace wq {
namespace {

template <typename E>
struct FstArgs {
    int pitch;  // row stride of f and u
    int ld;     // row stride of T1 and T2
    const E* f[2];
    double* t1[2];
    double* t2[2];
    E* u[2];
    const double2* tw;  // exp(-2 pi i m / 2n), m < 2n
    const double* s2;   // sin^2(pi k / (2n)), k <= n
    double lam;         // -4 / H^2
    double scale;       // (2 / n)^2
};

// In-register DFT of length R (2 or 4), natural order in and out.
template <int R>
__device__ __forceinline__ void dft(double (&re)[R], double (&im)[R]) {
    static_assert(R == 2 || R == 4, "radix");
    if constexpr (R == 2) {
        const double ar = re[0], ai = im[0];
        re[0] = ar + re[1];
        im[0] = ai + im[1];
        re[1] = ar - re[1];
        im[1] = ai - im[1];
    } else {
        // X_q = sum_s x_s (-i)^(s q)
        const double s0r = re[0] + re[2], s0i = im[0] + im[2];
        const double d0r = re[0] - re[2], d0i = im[0] - im[2];
        const double s1r = re[1] + re[3], s1i = im[1] + im[3];
        const double d1r = re[1] - re[3], d1i = im[1] - im[3];
        re[0] = s0r + s1r;
        im[0] = s0i + s1i;
        re[2] = s0r - s1r;
        im[2] = s0i - s1i;
        re[1] = d0r + d1i;  // d0 - i d1
        im[1] = d0i - d1r;
        re[3] = d0r - d1i;  // d0 + i d1
        im[3] = d0i + d1r;
    }
}

// LDS slot of element i of a padded buffer
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

// Twiddle W_L^m (m < L) from the table of W_L^m, m < L / 2 (W_L^(m + L/2) = -W_L^m).
template <int L>
__device__ __forceinline__ double2 twiddle(const double2* tw, int m) {
    if (m < L / 2) return tw[m];
    const double2 v = tw[m - L / 2];
    return double2{-v.x, -v.y};
}

template <int LOGN>
struct FstSize {
    static constexpr int n = 1 << LOGN;
    static constexpr int H = n / 2;                 // complex FFT length
    static constexpr int PER = H / 64;              // Y coefficients per lane (chunk)
    static constexpr int NB = (H / 4 + 63) / 64;    // first-stage butterflies per lane
    static constexpr int LP = H + H / 16;           // padded FFT buffer
    static_assert(PER >= 1, "n >= 128");
};

// One radix-R Stockham stage of the length-H FFT run by one wavefront:
// butterfly j (lane + 64 b) takes X[j + s H / R] (s < R; src(t, b, s) gives
// input t) times W_(NS R)^(k s), k = j mod NS, and puts its DFT at
// (j - k) R + k + q NS.  The twiddles W_(NS R)^(k s) = W_n^(2 k s H / (NS R))
// come from the LDS table T of W_n^m, m < H.
template <int H, int R, int NS, class Src>
__device__ __forceinline__ void wstage(const Src& src, double* yr, double* yi, const double2* T) {
    constexpr int NBF = H / R, NBL = (NBF + 63) / 64;
#pragma unroll
    for (int b = 0; b < NBL; ++b) {
        const int j = (threadIdx.x & 63) + 64 * b;
        if (NBF % 64 != 0 && j >= NBF) break;
        const int k = j & (NS - 1);
        double vr[R], vi[R];
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const double2 x = src(j + s * (H / R), b, s);
            if (NS > 1 && s > 0) {
                const double2 w = twiddle<2 * H>(T, 2 * (k * s * (H / (NS * R))));
                vr[s] = x.x * w.x - x.y * w.y;
                vi[s] = x.x * w.y + x.y * w.x;
            } else {
                vr[s] = x.x;
                vi[s] = x.y;
            }
        }
        dft<R>(vr, vi);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            yr[pidx(base + q * NS)] = vr[q];
            yi[pidx(base + q * NS)] = vi[q];
        }
    }
}

template <int H, int NS, class Src>
__device__ __forceinline__ void wfft(const Src& src, double* xr, double* xi, double* yr, double* yi,
                                     const double2* T, double*& out_r, double*& out_i) {
    constexpr int R = H / NS >= 4 ? 4 : H / NS;
    wstage<H, R, NS>(src, yr, yi, T);
    wave_sync();
    if constexpr (NS * R < H) {
        const auto lds = [yr, yi](int t, int, int) { return double2{yr[pidx(t)], yi[pidx(t)]}; };
        wfft<H, NS * R>(lds, yr, yi, xr, xi, T, out_r, out_i);
    } else {
        out_r = yr;
        out_i = yi;
    }
}

// Sine transform of the row x (get(j) = x_j for j in 1 .. n-1, called with
// clamped indices only) by the lane: xe[q] = X_2k, xo[q] = X_2k+1 for
// k = lane PER + q.  sn[b][s][e] = sin(pi j / n) of the lane's sample
// j = 2m + e (m = the first-stage input of butterfly b, leg s), loaded by the
// caller.  buf: 4 LP doubles of LDS (get may read it: its loads come first).
// STORE: the lane's entries tv of the LDS table T (T[lane + 64 q] = tv[q]) are
// stored once the row's loads are issued, so that both sets of loads overlap.
template <int LOGN, bool STORE, class Get>
__device__ __forceinline__ void wdst(const Get& get, const double (&sn)[FstSize<LOGN>::NB][4][2],
                                     double* buf, double2* T, const double2 (&tv)[FstSize<LOGN>::PER],
                                     double (&xe)[FstSize<LOGN>::PER], double (&xo)[FstSize<LOGN>::PER]) {
    using F = FstSize<LOGN>;
    constexpr int n = F::n, H = F::H, NB = F::NB, PER = F::PER, LP = F::LP;
    const int lane = threadIdx.x & 63;
    // first-stage inputs z_m, m = min(lane + 64 b, H/4 - 1) + s H/4; every load
    // issued before any is used (indices clamped, zero ends masked after)
    double xa[NB][4][2], xb[NB][4][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int m = min(lane + 64 * b, H / 4 - 1) + s * (H / 4);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int j = 2 * m + e;  // 0 .. n-1; n - j in 1 .. n
                xa[b][s][e] = get(max(j, 1)) * (j >= 1 ? 1.0 : 0.0);
                xb[b][s][e] = get(min(n - j, n - 1)) * (j >= 1 ? 1.0 : 0.0);
            }
        }
    if (STORE)
#pragma unroll
        for (int q = 0; q < PER; ++q) T[lane + 64 * q] = tv[q];
    wave_sync();
    double2 z[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double y[2];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                y[e] = sn[b][s][e] * (xa[b][s][e] + xb[b][s][e]) + 0.5 * (xa[b][s][e] - xb[b][s][e]);
            z[b][s] = double2{y[0], y[1]};
        }
    double* Ar = buf;
    double* Ai = Ar + LP;
    double* Br = Ai + LP;
    double* Bi = Br + LP;
    double *zr, *zi;
    wfft<H, 1>([&](int, int b, int s) { return z[b][s]; }, Ar, Ai, Br, Bi, T, zr, zi);
    // Y_k over the lane's chunk, then the prefix sum of Re Y (Re Y_0 halved)
    double rs[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = lane * PER + q, km = (H - k) & (H - 1);
        const double ar = zr[pidx(k)], ai = zi[pidx(k)], br = zr[pidx(km)], bi = zi[pidx(km)];
        const double er = 0.5 * (ar + br), ei = 0.5 * (ai - bi);
        const double orr = 0.5 * (ai + bi), oi = -0.5 * (ar - br);
        const double2 w = T[k];
        const double yr = er + w.x * orr - w.y * oi, yi = ei + w.x * oi + w.y * orr;
        xe[q] = -yi;
        rs[q] = (k == 0 ? 0.5 : 1.0) * yr;
    }
    double run = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        run += rs[q];
        rs[q] = run;
    }
    double incl = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(incl, d, 64);
        incl += lane >= d ? t : 0.0;
    }
    const double excl = incl - run;
#pragma unroll
    for (int q = 0; q < PER; ++q) xo[q] = excl + rs[q];
    wave_sync();  // the caller may overwrite buf next
}

// MODE 0: x pass; MODE 1: y pass; MODE 2: x inverse (see above).  A
// workgroup holds RW wavefronts, wavefront w transforming row RW b + w
// (0-based interior; b the block) of right-hand side r; a wavefront past the
// last row transforms the last row again and writes nothing.  With RW > 1 the
// transposed writes of MODE 0 and 1 go through LDS, RW consecutive rows'
// values of one coefficient written together.
template <typename E, int LOGN, int MODE, int RW>
__global__ __launch_bounds__(64 * RW) void k_fst(FstArgs<E> a) {
    using F = FstSize<LOGN>;
    constexpr int n = F::n, H = F::H, NB = F::NB, PER = F::PER, LP = F::LP;
    __shared__ double bufs[RW][4 * LP];
    __shared__ double2 T[H];
    int pb, r;
    tile_of_block(pb, r);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool live = pb * RW + w < n - 1;
    const int p = live ? pb * RW + w : n - 2;
    double* buf = bufs[w];
    // tables: W_n^m (m < H) = W_2n^2m into LDS; the lane's sin(pi j / n) =
    // -Im W_2n^j; for MODE 1 its sin^2(pi l / 2n) and that of k = p + 1
    double2 tv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) tv[q] = a.tw[2 * (lane + 64 * q)];
    double sn[NB][4][2];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int m = min(lane + 64 * b, H / 4 - 1) + s * (H / 4);
                sn[b][s][e] = -a.tw[2 * m + e].y;
            }
    double s2e[MODE == 1 ? PER : 1], s2o[MODE == 1 ? PER : 1], s2k = 0.0;
    if (MODE == 1) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = lane * PER + q;
            s2e[q] = a.s2[2 * k];
            s2o[q] = a.s2[2 * k + 1];
        }
        s2k = a.s2[p + 1];
    }
    const size_t ld = a.ld;
    double xe[PER], xo[PER];
    if (MODE == 0) {
        const E* row = a.f[r] + (size_t)(p + 1) * a.pitch;
        const auto get = [=](int j) { return (double)row[j]; };
        wdst<LOGN, true>(get, sn, buf, T, tv, xe, xo);
    } else {
        const double* row = (MODE == 1 ? a.t1 : a.t2)[r] + (size_t)p * ld - 1;
        const auto get = [=](int j) { return row[j]; };
        wdst<LOGN, true>(get, sn, buf, T, tv, xe, xo);
    }
    if (MODE == 1) {
        // coefficient (k, l) over its eigenvalue, into LDS by l (V[0] = 0),
        // then transformed back along y
        double* V = buf;
        const double lam = a.lam, lk = lam * s2k;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = lane * PER + q;
            V[2 * k] = k == 0 ? 0.0 : xe[q] / (lk + lam * s2e[q]);
            V[2 * k + 1] = xo[q] / (lk + lam * s2o[q]);
        }
        wave_sync();
        const auto get = [=](int j) { return V[j]; };
        wdst<LOGN, false>(get, sn, buf, T, tv, xe, xo);
    }
    if (MODE < 2 && RW == 1) {
        // coefficient c (1 .. n-1) of this row to T[c - 1][p]
        double* Tt = (MODE == 0 ? a.t1 : a.t2)[r] + p;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = 2 * (lane * PER + q);
            if (c >= 1) Tt[(size_t)(c - 1) * ld] = xe[q];
            Tt[(size_t)c * ld] = xo[q];
        }
    } else if (MODE < 2) {
        // the RW rows' coefficients through LDS: T[c - 1][RW b .. RW b + RW - 1]
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = lane * PER + q;
            buf[2 * k] = xe[q];
            buf[2 * k + 1] = xo[q];
        }
        __syncthreads();
        double* Tt = (MODE == 0 ? a.t1 : a.t2)[r] + pb * RW;
        for (int i = threadIdx.x; i < (n - 1) * RW; i += 64 * RW) {
            const int c = 1 + i / RW, ww = i % RW;
            if (pb * RW + ww < n - 1) Tt[(size_t)(c - 1) * ld + ww] = bufs[ww][c];
        }
    } else {
        E* u = a.u[r];
        E* row = u + (size_t)(p + 1) * a.pitch;
        const double sc = a.scale;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = 2 * (lane * PER + q);
            row[c] = c == 0 ? E(0) : (E)(sc * xe[q]);
            row[c + 1] = (E)(sc * xo[q]);
        }
        if (lane == 63) row[n] = E(0);
        if (p == 0)
            for (int x = lane; x <= n; x += 64) {
                u[x] = E(0);
                u[(size_t)n * a.pitch + x] = E(0);
            }
    }
}

// Rows per workgroup of the x and y passes, whose transposed writes then go
// out in 16-byte pieces: at n = 512 they measured 5.4 / 7.5 us with 2 rows,
// 6.1 / 8.0 with 1 and 5.7 / 8.0 with 4 (the same bits in every case)
#ifndef WQ_FST_ROWS
#define WQ_FST_ROWS 2
#endif

template <typename E, int LOGN>
void launch_fst(wandqs_ctx* c, const FstArgs<E>& a, int R, const char* tname) {
    constexpr int n = 1 << LOGN;
    constexpr int RW = LOGN <= 10 ? WQ_FST_ROWS : 1;
    const dim3 g(n - 1, R), gw((n - 1 + RW - 1) / RW, R);
    const double nodes = (double)(n - 1) * (n - 1) * R;
    const double eb = sizeof(E);
    char nm[64];
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, x>@%d", tname, n);
        ProfScope ps(c, nm, nodes * (eb + 8.0));
        WQ_KLAUNCH(ps, (k_fst<E, LOGN, 0, RW>), gw, dim3(64 * RW), 0, c->stream, a);
    }
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, y>@%d", tname, n);
        ProfScope ps(c, nm, nodes * 16.0);
        WQ_KLAUNCH(ps, (k_fst<E, LOGN, 1, RW>), gw, dim3(64 * RW), 0, c->stream, a);
    }
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, xinv>@%d", tname, n);
        ProfScope ps(c, nm, nodes * (8.0 + eb));
        WQ_KLAUNCH(ps, (k_fst<E, LOGN, 2, 1>), g, dim3(64), 0, c->stream, a);
    }
}

__global__ void k_fst_tables(int L, double2* tw, double* s2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) {
        double sv, cv;
        sincospi(-2.0 * i / L, &sv, &cv);
        tw[i] = double2{cv, sv};
    }
    if (i <= L / 2) {
        const double s = sinpi((double)i / L);  // sin(pi k / (2n)), L = 2n
        s2[i] = s * s;
    }
}

}  // namespace

bool fst_used(const wandqs_ctx* c) {
    return c->lc >= 2 && c->lev[1].N >= kFstMinN && c->lev[1].N <= kFstMaxN;
}

size_t fst_ld(const wandqs_ctx* c) { return (size_t)c->lev[1].N + 8; }

wandqs_status make_fst_tables(wandqs_ctx* c) {
    if (!fst_used(c)) return WANDQS_OK;
    const int L = 2 * c->lev[1].N;
    hipLaunchKernelGGL(k_fst_tables, dim3(L / 256 + 1), dim3(256), 0, c->stream, L, c->fst_tw,
                       c->fst_s2);
    WQ_LAUNCH_CHECK();
    return WANDQS_OK;
}

template <typename E>
void fst_solve(wandqs_ctx* c, int R, const E* const* f, E* const* u) {
    const Level& L1 = c->lev[1];
    FstArgs<E> a{};
    a.pitch = L1.pitch;
    a.ld = (int)fst_ld(c);
    for (int r = 0; r < R; ++r) {
        a.f[r] = f[r];
        a.u[r] = u[r];
        a.t1[r] = c->fst_t1[r];
        a.t2[r] = c->fst_t2[r];
    }
    a.tw = c->fst_tw;
    a.s2 = c->fst_s2;
    a.lam = -4.0 / (L1.h * L1.h);
    a.scale = (2.0 / L1.N) * (2.0 / L1.N);
    const char* tn = sizeof(E) == 8 ? "double" : "float";
    switch (L1.N) {
        case 128: launch_fst<E, 7>(c, a, R, tn); break;
        case 256: launch_fst<E, 8>(c, a, R, tn); break;
        case 512: launch_fst<E, 9>(c, a, R, tn); break;
        case 1024: launch_fst<E, 10>(c, a, R, tn); break;
        default: launch_fst<E, 11>(c, a, R, tn); break;
    }
}

template void fst_solve<double>(wandqs_ctx*, int, const double* const*, double* const*);
template void fst_solve<float>(wandqs_ctx*, int, const float* const*, float* const*);

}  // namespace wq
