// wandqs_mg_solve_noalloc: the multigrid solve of wandqs_mg_solve for callers
// that cannot allocate device memory.  Its level hierarchy, coarse-level k2
// arrays, sine-transform tables and norm partials live in one static device
// array of the library (`scratch`) instead of a context's workspace; the
// kernels are those of wandqs_mg_solve in its fixed-cycle mode.
#include <cstdio>
#include <mutex>

#include "wq_common.h"

namespace {

// Largest grid the static array holds: every array of a 256^2 solve in the
// mixed form (the larger of the two forms) takes about 8 MiB.
constexpr size_t kScratchBytes = size_t(12) << 20;
constexpr int kScratchMaxN = 256;

// One copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel: it uses the device address that hipGetSymbolAddress
// returns for the current device (scratch_base).
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
char* g_scratch_base[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
wandqs_status scratch_base(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        wq::set_call_error("wandqs_mg_solve_noalloc: no usable current HIP device");
        return WANDQS_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_base[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            wq::set_call_error("wandqs_mg_solve_noalloc: hipGetSymbolAddress of the static "
                               "scratch array failed");
            return WANDQS_E_HIP;
        }
        g_scratch_base[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_base[dev];
    return WANDQS_OK;
}

wandqs_status invalid(const char* m) {
    wq::set_call_error(m);
    return WANDQS_E_INVALID;
}

}  // namespace

extern "C" wandqs_status wandqs_mg_solve_noalloc(const wandqs_config* cfg, int32_t nrhs,
                                                 const double* d_k2, const double* d_f,
                                                 double* d_u, void* hip_stream) {
    if (!cfg || (nrhs != 1 && nrhs != 2) || !d_f || !d_u)
        return invalid("wandqs_mg_solve_noalloc: needs cfg, nrhs = 1 or 2, d_f and d_u");
    if (cfg->n_cells > kScratchMaxN)
        return invalid("wandqs_mg_solve_noalloc: n_cells above 256 does not fit the static scratch "
                       "array (12 MiB); use wandqs_mg_solve");
    if (cfg->mg_rtol > 0.0)
        return invalid("wandqs_mg_solve_noalloc runs exactly mg_max_cycles V-cycles with no host "
                       "synchronisation: set mg_rtol <= 0");
    wandqs_ctx c;  // host bookkeeping only; no member allocates on this path
    if (const char* e = wq::setup_solver_ctx(&c, cfg)) return invalid(e);
    const size_t need = wq::carve_solver(&c, nullptr);
    if (need > kScratchBytes)
        return invalid("wandqs_mg_solve_noalloc: the solve's arrays exceed the static scratch array");
    char* base = nullptr;
    wandqs_status s = scratch_base(&base);
    if (s != WANDQS_OK) return s;
    wq::carve_solver(&c, base);
    c.stream = static_cast<hipStream_t>(hip_stream);
    // the array keeps the previous call's contents: clear every array of this
    // layout (boundary nodes and the unused padding of each row included) with
    // a fill kernel, then build the tables the solve reads
    wq::Level& L0 = c.lev[0];
    if ((s = wq::fill_f64(&c, reinterpret_cast<double*>(base), need / sizeof(double), 0.0)) != WANDQS_OK ||
        (s = wq::make_dst_tables(&c)) != WANDQS_OK ||
        (s = wq::unpack_fields(&c, d_f, nrhs, L0.f)) != WANDQS_OK ||
        (s = wq::unpack_fields(&c, d_u, nrhs, c.fields)) != WANDQS_OK ||
        (d_k2 && (s = wq::unpack_fields(&c, d_k2, 1, &L0.k2)) != WANDQS_OK)) {
        wq::set_call_error(c.err.c_str());
        return s;
    }
    double* u[2] = {c.fields[0], nrhs > 1 ? c.fields[1] : nullptr};
    double* f[2] = {L0.f[0], nrhs > 1 ? L0.f[1] : nullptr};
    if ((s = wq::mg_solve(&c, wq::kSolveUser, nrhs, d_k2 != nullptr, u, f, d_k2 ? L0.k2 : nullptr,
                          nullptr)) != WANDQS_OK ||
        (s = wq::pack_fields(&c, c.fields, nrhs, d_u)) != WANDQS_OK) {
        wq::set_call_error(c.err.c_str());
        return s;
    }
    return WANDQS_OK;
}
