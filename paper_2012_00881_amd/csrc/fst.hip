// Exact Poisson solve on the level just below the finest by fast sine
// transforms, FP64 (the coarse-grid correction of the Poisson V-cycles of
// eqs. (12)-(15), Sec. III.B; the five-point operator of Sec. VII.B on a
// uniform grid).
//
// With zero Dirichlet values the five-point Laplacian of an n x n-cell level
// of spacing H has the eigenvectors sin(pi i k / n) sin(pi j l / n) (1 <= k, l
// <= n - 1) and the eigenvalues -(4 / H^2) (sin^2(pi k / 2n) + sin^2(pi l / 2n)),
// so u = (2/n)^2 S (S f S ./ lambda) S with the sine matrix S.  The sine
// transform of a row is taken from a complex FFT of length L = 2n of the row's
// odd extension; two real rows share one FFT as its real and imaginary parts
// (the transform of an odd real sequence is imaginary, so the two separate).
//
// Three launches, each over rows or columns that a workgroup transforms in
// LDS:
//   x: rows of f, transform along x, to the rows of T1 (FP64);
//   y: columns of T1, transform along y, divide by lambda, inverse transform
//      along y, to the rows of T2;
//   x inverse: columns of T2, inverse transform along x, scaled into the rows
//      of u (boundary nodes 0).
// One workgroup computes one FFT (two rows) as a Stockham (self-sorting)
// decimation in time: radix-4 stages (and one radix-2 stage last for an odd
// power of two), each thread taking one butterfly of the stage in registers
// (up to 256 threads; more per thread above L = 1024), with the stages
// ping-ponging between two LDS buffers (one pad slot per 16 doubles, which spreads the strided writes of
// the first stages over the banks).  The first stage reads its inputs
// straight from memory.
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
    const double2* tw;  // exp(-2 pi i m / L), m < L
    const double* s2;   // sin^2(pi k / (2n)), k <= n
    double lam;         // -4 / H^2
    double scale;       // (2 / n)^2
};

// cos and sin of 2 pi m / 16 (m < 8)
__device__ __forceinline__ constexpr double cos16(int m) {
    return m == 0   ? 1.0
           : m == 1 ? 0.9238795325112867561281831893967883
           : m == 2 ? 0.7071067811865475244008443621048490
           : m == 3 ? 0.3826834323650897717284599840303988
           : m == 4 ? 0.0
           : m == 5 ? -0.3826834323650897717284599840303988
           : m == 6 ? -0.7071067811865475244008443621048490
                    : -0.9238795325112867561281831893967883;
}
__device__ __forceinline__ constexpr double sin16(int m) { return m <= 4 ? cos16(4 - m) : cos16(m - 4); }

// In-register DFT of length R (2, 4, 8 or 16), natural order in and out:
// radix 2 and 4 written out, 8 and 16 by one radix-2 decimation-in-time step
// over two half-length DFTs.
template <int R>
__device__ __forceinline__ void dft(double (&re)[R], double (&im)[R]) {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
    if constexpr (R >= 8) {
        constexpr int H = R / 2;
        double er[H], ei[H], orr[H], oi[H];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            er[q] = re[2 * q];
            ei[q] = im[2 * q];
            orr[q] = re[2 * q + 1];
            oi[q] = im[2 * q + 1];
        }
        dft<H>(er, ei);
        dft<H>(orr, oi);
#pragma unroll
        for (int q = 0; q < H; ++q) {
            // W_R^q = cos(2 pi q / R) - i sin(2 pi q / R)
            const double wr = cos16(q * (16 / R)), wi = -sin16(q * (16 / R));
            const double tr = wr * orr[q] - wi * oi[q], ti = wr * oi[q] + wi * orr[q];
            re[q] = er[q] + tr;
            im[q] = ei[q] + ti;
            re[q + H] = er[q] - tr;
            im[q + H] = ei[q] - ti;
        }
    } else if constexpr (R == 2) {
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

// Radix of the full stages: WQ_FST_RADIX, at most L / 64 (so that one
// butterfly per thread takes a whole wavefront at least).  Radix 16 (one
// wavefront per FFT of 1024, three stages) measured slower than radix 4 (256
// threads, five stages): 12.5 / 7.8 / 7.1 against 9.5 / 6.5 / 5.2 us for the
// y / x inverse / x passes at 512^2.
#ifndef WQ_FST_RADIX
#define WQ_FST_RADIX 4
#endif
template <int L>
constexpr int fst_radix() { return L / 64 < WQ_FST_RADIX ? L / 64 : WQ_FST_RADIX; }

// Radix of the stage whose input span is NS: the full radix, and what is left
// for the last stage.
template <int L, int NS>
constexpr int stage_radix() {
    return L / NS >= fst_radix<L>() ? fst_radix<L>() : L / NS;
}

// LDS slot of element i of a padded buffer
__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

template <int L>
constexpr int padded_len() { return L + L / 16; }

// Threads of the workgroup that computes one FFT of length L: one butterfly
// of a full stage each, at most 256.
template <int L>
constexpr int fst_threads() { return L / fst_radix<L>() < 256 ? L / fst_radix<L>() : 256; }

// Twiddle W_L^m (m < L) from the table of W_L^m, m < L / 2 (TW2) or of all m.
template <int L, bool TW2>
__device__ __forceinline__ double2 twiddle(const double2* tw, int m) {
    if constexpr (TW2) {
        if (m < L / 2) return tw[m];
        const double2 v = tw[m - L / 2];
        return double2{-v.x, -v.y};
    } else {
        return tw[m];
    }
}

// One Stockham stage: butterfly j takes X[j + s L / R] (s < R) times
// W_(NS R)^(k s), k = j mod NS, and puts its DFT at (j - k) R + k + q NS.
template <int L, int R, int NS, bool TW2, class Src>
__device__ __forceinline__ void stockham_stage(const Src& src, double* yr, double* yi,
                                               const double2* tw) {
    constexpr int NT = fst_threads<L>();
    static_assert((L / R) % NT == 0, "every thread takes a butterfly");
#pragma unroll
    for (int b = 0; b < L / R / NT; ++b) {
        const int j = threadIdx.x + NT * b, k = j & (NS - 1);
        double vr[R], vi[R];
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const double2 x = src(j + s * (L / R));
            if (NS > 1 && s > 0) {
                const double2 w = twiddle<L, TW2>(tw, k * s * (L / (NS * R)));
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

// The stages from span NS on: the first reads src and writes (yr, yi), the
// next ones alternate between the two buffers; the result's buffer is
// returned in (out_r, out_i).  hook() runs after the first stage's LDS writes,
// before its barrier (the kernel stores its LDS tables there, so that their
// loads overlap the first stage's).  Ends with a barrier.
template <int L, int NS, bool TW2, class Src, class Hook>
__device__ __forceinline__ void fft_run(const Src& src, double* xr, double* xi, double* yr,
                                        double* yi, const double2* tw, double*& out_r,
                                        double*& out_i, const Hook& hook) {
    constexpr int R = stage_radix<L, NS>();
    stockham_stage<L, R, NS, TW2>(src, yr, yi, tw);
    hook();
    __syncthreads();
    if constexpr (NS * R < L) {
        const auto lds = [yr, yi](int t) { return double2{yr[pidx(t)], yi[pidx(t)]}; };
        fft_run<L, NS * R, TW2>(lds, yr, yi, xr, xi, tw, out_r, out_i, [] {});
    } else {
        out_r = yr;
        out_i = yi;
    }
}

// Element t of the odd extension (length L = 2n) of the packed row pair
// (row a in the real part, row b in the imaginary part), from get(tt) for the
// row element tt in 1 .. n-1.  get is called for every t (with an index
// clamped into 1 .. n-1) and the zero slots t = 0, n are selected after it:
// no load sits behind a branch, so a stage's loads are all in flight at once.
template <int L, class Get>
__device__ __forceinline__ double2 odd_ext(int t, const Get& get) {
    constexpr int n = L / 2;
    const bool lo = t < n;
    int tt = lo ? t : L - t;
    tt = tt < 1 ? 1 : (tt > n - 1 ? n - 1 : tt);
    const double2 v = get(tt);
    const bool zero = t == 0 || t == n;
    return double2{zero ? 0.0 : (lo ? v.x : -v.x), zero ? 0.0 : (lo ? v.y : -v.y)};
}

// Sine transform of real row e at index k, from the FFT Z of the packed odd
// extensions (padded buffers): row 0 gives -Im Z_k / 2, row 1 Re Z_k / 2.
__device__ __forceinline__ double sine_coef(const double* re, const double* im, int k, int e) {
    return e ? 0.5 * re[pidx(k)] : -0.5 * im[pidx(k)];
}

// MODE 0: transform along x (rows g of f) -> rows g of T1 (T1[j][k]);
// MODE 1: along y (columns k of T1), divide, inverse along y -> rows k of T2
// (T2[k][j]); MODE 2: inverse along x (columns j of T2) -> rows j of u.  Every
// write is a whole row; the column reads of MODE 1 and 2 take 16 bytes of each
// line, so the workgroups are dealt to the XCDs in contiguous ranges (the
// eight workgroups reading one line share an L2).  A workgroup transforms the
// rows (or columns) ga = 2 p and gb = ga + 1, 0-based interior indices (node
// index one higher), of right-hand side r.  ga <= n - 2 always; gb = n - 1
// (past the interior) only in the last workgroup, whose loads of it stay in
// bounds (the boundary row of f, the padding column of T) and are replaced by
// zeros.
template <typename E, int LOG, int MODE>
__global__ __launch_bounds__(fst_threads<1 << LOG>()) void k_fst(FstArgs<E> a) {
    constexpr int L = 1 << LOG, n = L / 2, LP = padded_len<L>(), NT = fst_threads<L>();
    // the twiddles W_L^m (m < L / 2) and, for MODE 1, sin^2(pi k / L) (k < n)
    // in LDS, except at L = 4096, whose buffers leave no room; each thread
    // loads the same number of entries (L / 2 is a multiple of NT), with no
    // branch, so that the loads stay in flight through the first stage
    constexpr bool TWL = L <= 2048;
    static_assert((L / 2) % NT == 0, "table share");
    constexpr int NTW = TWL ? L / 2 / NT : 0;
    constexpr int NS2 = TWL && MODE == 1 ? n / NT : 0;
    __shared__ double smem[4 * LP];
    __shared__ double2 stw[TWL ? L / 2 : 1];
    __shared__ double ss2[NS2 ? n : 1];
    int p, r;
    tile_of_block(p, r);
    const int ga = 2 * p, gb = ga + 1;
    const bool vb = gb < n - 1;
    double* Ar = smem;
    double* Ai = Ar + LP;
    double* Br = Ai + LP;
    double* Bi = Br + LP;

    double2 twv[NTW > 0 ? NTW : 1];
    double s2v[NS2 > 0 ? NS2 : 1];
#pragma unroll
    for (int q = 0; q < NTW; ++q) twv[q] = a.tw[threadIdx.x + q * NT];
#pragma unroll
    for (int q = 0; q < NS2; ++q) s2v[q] = a.s2[threadIdx.x + q * NT];
    const auto store_tables = [&] {
#pragma unroll
        for (int q = 0; q < NTW; ++q) stw[threadIdx.x + q * NT] = twv[q];
#pragma unroll
        for (int q = 0; q < NS2; ++q) ss2[threadIdx.x + q * NT] = s2v[q];
    };
    const double2* tw = TWL ? stw : a.tw;

    double *zr, *zi;
    if (MODE == 0) {
        const E* pa = a.f[r] + (size_t)(ga + 1) * a.pitch;
        const E* pb = a.f[r] + (size_t)(gb + 1) * a.pitch;
        const auto get = [=](int tt) {
            const double b = (double)pb[tt];
            return double2{(double)pa[tt], vb ? b : 0.0};
        };
        fft_run<L, 1, TWL>([&](int t) { return odd_ext<L>(t, get); }, Ar, Ai, Br, Bi, tw, zr, zi,
                           store_tables);
    } else {
        // columns ga and gb: element tt at T[(tt - 1) ld + ga], one 16-byte load
        const double* T = (MODE == 1 ? a.t1 : a.t2)[r] + ga;
        const size_t ld = a.ld;
        const auto get = [=](int tt) {
            const double2 v = *reinterpret_cast<const double2*>(T + (size_t)(tt - 1) * ld);
            return double2{v.x, vb ? v.y : 0.0};
        };
        fft_run<L, 1, TWL>([&](int t) { return odd_ext<L>(t, get); }, Ar, Ai, Br, Bi, tw, zr, zi,
                           store_tables);
    }

    if (MODE == 1) {
        // coefficient (k, l) over its eigenvalue (k = this workgroup's
        // columns, 1-based), transformed back along y from the other buffer
        const int ka = ga + 1, kb = gb + 1;
        const double* s2 = NS2 ? ss2 : a.s2;
        const double lam = a.lam;
        const double la = lam * s2[ka < n ? ka : 0], lb = lam * s2[kb < n ? kb : 0];
        const double* fr = zr;
        const double* fi = zi;
        const auto get = [=](int l) {
            const double sl = lam * s2[l];
            return double2{sine_coef(fr, fi, l, 0) / (la + sl),
                           vb ? sine_coef(fr, fi, l, 1) / (lb + sl) : 0.0};
        };
        double* xr = zr;
        double* xi = zi;
        double* yr = zr == Ar ? Br : Ar;
        double* yi = zr == Ar ? Bi : Ai;
        fft_run<L, 1, TWL>([&](int t) { return odd_ext<L>(t, get); }, xr, xi, yr, yi, tw, zr, zi,
                           [] {});
    }

    if (MODE < 2) {
        // coefficient k of the two rows to T[ga or gb][k - 1]
        double* T = (MODE == 0 ? a.t1 : a.t2)[r];
        double* ta = T + (size_t)ga * a.ld - 1;
        double* tb = T + (size_t)gb * a.ld - 1;
        for (int k = 1 + threadIdx.x; k <= n - 1; k += NT) {
            ta[k] = sine_coef(zr, zi, k, 0);
            if (vb) tb[k] = sine_coef(zr, zi, k, 1);
        }
    } else {
        E* u = a.u[r];
        E* ua = u + (size_t)(ga + 1) * a.pitch;
        E* ub = u + (size_t)(gb + 1) * a.pitch;
        for (int t = threadIdx.x; t < n; t += NT) {
            if (t == 0) {
                ua[0] = ua[n] = E(0);
                if (vb) ub[0] = ub[n] = E(0);
            } else {
                ua[t] = (E)(a.scale * sine_coef(zr, zi, t, 0));
                if (vb) ub[t] = (E)(a.scale * sine_coef(zr, zi, t, 1));
            }
        }
        if (p == 0)
            for (int x = threadIdx.x; x <= n; x += NT) {
                u[x] = E(0);
                u[(size_t)n * a.pitch + x] = E(0);
            }
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

template <typename E, int LOG>
void launch_fst(wandqs_ctx* c, const FstArgs<E>& a, int R, const char* tname) {
    constexpr int n = (1 << LOG) / 2, NT = fst_threads<1 << LOG>();
    const dim3 g(n / 2, R);  // ceil((n - 1) / 2) row pairs
    const double nodes = (double)(n - 1) * (n - 1) * R;
    const double eb = sizeof(E);
    char nm[64];
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, x>@%d", tname, n);
        ProfScope ps(c, nm, nodes * (eb + 8.0));
        WQ_KLAUNCH(ps, (k_fst<E, LOG, 0>), g, dim3(NT), 0, c->stream, a);
    }
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, y>@%d", tname, n);
        ProfScope ps(c, nm, nodes * 16.0);
        WQ_KLAUNCH(ps, (k_fst<E, LOG, 1>), g, dim3(NT), 0, c->stream, a);
    }
    {
        std::snprintf(nm, sizeof nm, "k_fst<%s, xinv>@%d", tname, n);
        ProfScope ps(c, nm, nodes * (8.0 + eb));
        WQ_KLAUNCH(ps, (k_fst<E, LOG, 2>), g, dim3(NT), 0, c->stream, a);
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
    const int L = 2 * L1.N;
    const char* tn = sizeof(E) == 8 ? "double" : "float";
    switch (L) {
        case 256: launch_fst<E, 8>(c, a, R, tn); break;
        case 512: launch_fst<E, 9>(c, a, R, tn); break;
        case 1024: launch_fst<E, 10>(c, a, R, tn); break;
        case 2048: launch_fst<E, 11>(c, a, R, tn); break;
        default: launch_fst<E, 12>(c, a, R, tn); break;
    }
}

template void fst_solve<double>(wandqs_ctx*, int, const double* const*, double* const*);
template void fst_solve<float>(wandqs_ctx*, int, const float* const*, float* const*);

}  // namespace wq
