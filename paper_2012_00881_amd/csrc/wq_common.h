// Internal declarations of the wandqs library (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "wandqs.h"

namespace wq {

constexpr int kMaxBeams = 8;
constexpr int kMaxProbes = 16;
constexpr int kMaxLevels = 13;
#ifndef WQ_COARSE_MAX
#define WQ_COARSE_MAX 64
#endif
constexpr int kCoarseMax = WQ_COARSE_MAX;  // levels with N <= kCoarseMax are solved inside one workgroup
constexpr int kMaxSlots = 208;  // residual-norm records per solve (mg_max_cycles + batches)
constexpr int kNormVec = 6;     // per record and right-hand side r: sums of r^2, f^2, u^2 at 3r .. 3r+2
// Rounding-floor test of the stop rule: ||r|| <= kFloorBE eps (||L_h|| ||u|| + ||f||).
// Residuals formed in FP64 from an iterate at the floor measure about 0.2-0.25
// of eps (8/h^2 ||u|| + ||f||); one cycle before the floor, 0.5 or more.
constexpr double kFloorBE = 0.35;
constexpr int kTile = 32;       // multigrid tile edge (fine nodes owned by one workgroup)
constexpr int kDepTile = 16;    // deposit tile edge (nodes owned by one workgroup)
constexpr int kPredKinds = 8;   // solve kinds with their own V-cycle batch prediction
constexpr int kThetaSeg = 4096; // nodes per partial sum of the driver-parameter adjoint
#ifndef WQ_EXTRAP_ORDER
#define WQ_EXTRAP_ORDER 3
#endif
constexpr int kGuessMax = WQ_EXTRAP_ORDER + 1;  // solved slices the guesses use

// Driver beams as a by-value kernel argument.
struct BeamSet {
    int n;
    int kind[kMaxBeams];
    double amp[kMaxBeams], sr[kMaxBeams], sz[kMaxBeams], xc[kMaxBeams], x0[kMaxBeams],
        y0[kMaxBeams], rmax[kMaxBeams];
    int nbins[kMaxBeams];
    const double* bins[kMaxBeams];
    const int32_t* bmap[kMaxBeams];  // radial bins: bin of each node (dense [N+1]^2), -1 outside
};

// One multigrid level.  Node arrays are row-major with a padded row pitch.
struct Level {
    int N = 0;
    double h = 0;
    int pitch = 0;
    double* u[2] = {nullptr, nullptr};   // solution (level 0) or coarse correction
    double* um[2] = {nullptr, nullptr};  // pre-smoothed iterate written by the down pass
    // level 0 on register tiles: the second buffer of the pre-smoothed iterate,
    // which the fused up-and-down passes write alternately with um
    double* um2[2] = {nullptr, nullptr};
    double* f[2] = {nullptr, nullptr};   // right-hand side
    double* k2 = nullptr;                // Helmholtz coefficient (restricted)
    // float buffers of the mixed form's inner cycles (level 0: error e, its
    // pre-smoothed copy and the defect r)
    float* u32[2] = {nullptr, nullptr};
    float* um32[2] = {nullptr, nullptr};
    float* f32[2] = {nullptr, nullptr};
};

// Tile of this workgroup in a 2-D grid of tiles.  Workgroups are dealt to the
// 8 XCDs round-robin in dispatch order; the mapping gives each XCD a contiguous
// band of tiles (row-major), so the halo a tile shares with its neighbours is
// mostly fetched once into that XCD's L2 instead of once per tile.
__device__ __forceinline__ void tile_of_block(int& bx, int& by) {
    const int gx = gridDim.x, n = gx * gridDim.y;
    const int b = blockIdx.y * gx + blockIdx.x;
    const int k = b & 7, q = n >> 3, r = n & 7;
    const int t = k * q + (k < r ? k : r) + (b >> 3);
    by = t / gx;
    bx = t - by * gx;
}

// The same over a 3-D grid whose z indexes the right-hand sides of a split
// launch: a tile's right-hand sides follow each other in its XCD's range, so
// the operator's array that both read (k2) is fetched into that XCD's L2 once.
__device__ __forceinline__ void tile_rhs_of_block(int& bx, int& by, int& z) {
    const int gx = gridDim.x, gz = gridDim.z, n = gx * gridDim.y * gz;
    const int b = (blockIdx.z * gridDim.y + blockIdx.y) * gx + blockIdx.x;
    const int k = b & 7, q = n >> 3, r = n & 7;
    const int t = k * q + (k < r ? k : r) + (b >> 3);
    z = t % gz;
    const int tile = t / gz;
    by = tile / gx;
    bx = tile - by * gx;
}

// Orders the LDS accesses of one wavefront around this point: the compiler
// keeps them in program order and the hardware completes them in order.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

enum SolveKind {
    kSolvePsi = 0,
    kSolveEB = 1,
    kSolveBperp = 2,
    kSolveUser = 3,
    kSolvePsiAdj = 4,
    kSolveEBAdj = 5,
    kSolveBperpAdj = 6
};

// Checkpoint of the slice loop state (the adjoint recomputes from it).
struct Checkpoint {
    double* pa[4] = {};
    int32_t* pid = nullptr;
    double* fields[5] = {};
    double* fields_prev[5] = {};
    double* fields_prev2[5] = {};
    double* fields_prev3[5] = {};
    double* st = nullptr;
    int pred[kPredKinds] = {};
    int n_guess = 0;
};

// What the reverse of one slice reads: its particles in cell order, the cell
// offsets, the solved fields, the deposited moments, k2 and [xi, dxi].
struct TapeSlot {
    double* pa[4] = {};
    int32_t* pid = nullptr;
    int32_t* start = nullptr;
    double* fields[5] = {};
    double* mom[6] = {};
    double* k2 = nullptr;
    double* st = nullptr;
};

// Work arrays of the reverse sweep.  Node arrays use the padded level-0 layout.
struct AdjBuffers {
    double *Gxb = nullptr, *Gyb = nullptr, *Bxb = nullptr, *Byb = nullptr, *Bzb = nullptr,
           *Ezb = nullptr, *psib = nullptr;
    double *lx = nullptr, *ly = nullptr, *lE = nullptr, *lB = nullptr, *lpsi = nullptr;
    double *nb = nullptr, *jxb = nullptr, *jyb = nullptr, *txxb = nullptr, *txyb = nullptr,
           *tyyb = nullptr, *psxb = nullptr, *psyb = nullptr, *gnb = nullptr, *psib_dep = nullptr,
           *jzb = nullptr;
    double *xb = nullptr, *yb = nullptr, *pxb = nullptr, *pyb = nullptr, *gb = nullptr;  // slice order
    double* adj_id = nullptr;      // [4][P] particle-ID order
    double* theta_bar = nullptr;   // [n_theta]
    double* theta_part = nullptr;  // [n_seg]
    int32_t* seg = nullptr;        // [n_seg][4]: beam, theta, begin, end
    int32_t* seg_first = nullptr;  // [n_theta + 1]
    int32_t* bin_nodes = nullptr;  // radial-bin nodes grouped by bin
};

struct SolveResult {
    int cycles = -1;
    double rel[2] = {-1.0, -1.0};
};

// One multigrid cycle of a solve as an instantiated HIP graph, keyed by every
// launch argument that varies between cycles: the solve's arrays, the number
// of right-hand sides, the operator, the precision form and the norm slot.
struct CycleKey {
    const void* p[5];
    int R, helm, mixed, slot, upslot;
    int fuse;  // 1: the level-0 down pass was fused into the last cycle; 2: the
               // level-0 up pass fuses with the next down pass; 4: um2 is current
    bool operator==(const CycleKey& o) const {
        for (int i = 0; i < 5; ++i)
            if (p[i] != o.p[i]) return false;
        return R == o.R && helm == o.helm && mixed == o.mixed && slot == o.slot &&
               upslot == o.upslot && fuse == o.fuse;
    }
};
struct CycleGraph {
    CycleKey key;
    hipGraphExec_t exec;
};
constexpr int kMaxGraphs = 1024;

// Optional per-kernel timing with HIP events (see wandqs_profile).
struct ProfPending {
    int cls;
    hipEvent_t a, b;
    double bytes;
};

struct Prof {
    bool on = false;
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> ms, bytes;
    std::vector<hipEvent_t> free_ev, all_ev;
    std::vector<ProfPending> pending;
};

}  // namespace wq

struct wandqs_ctx {
    // configuration (deep copy)
    wandqs_config cfg{};
    std::vector<wandqs_beam> beams;
    std::vector<std::vector<double>> bin_amp;
    std::vector<wandqs_probe> probes;

    int N = 0, ppc = 0, nlev = 0, lc = 0;
    // levels N >= reg_tile_min run the register-tile pass kernels (environment
    // WANDQS_MG_TILES=lds at init: never; the LDS tiles give the same bits)
    int reg_tile_min = 0;
    // the tile kernels run the two right-hand sides of a solve as separate
    // workgroups of one launch (environment WANDQS_MG_SPLIT at init: 0, both in
    // every workgroup; reg, split on the register-tile levels only; lds, on the
    // LDS-tile levels only; the same bits in every case)
    bool reg_split = true, lds_split = true;
    // inside a batch of V-cycles the level-0 up pass of one cycle and the down
    // pass of the next run as one fused launch (environment WANDQS_MG_FUSE=0 at
    // init: never; the same bits either way)
    bool mg_fuse = true;
    // LDS tiles of 16 x 16 owned nodes on the levels N <= small_tile_max
    // (environment WANDQS_MG_SMALL at init), 32 x 32 or 64 x 64 above
    int small_tile_max = 0;
    // environment WANDQS_GRAPHS=1 at init: multigrid cycles replay as HIP
    // graphs, captured on cap_stream at their first use (the kernels and their
    // arguments are those of the direct launches; on the 1024^2 job the
    // replays run 5-6% slower than direct launches, so they are off by default)
    bool graphs_on = false;
    hipStream_t cap_stream = nullptr;
    std::vector<wq::CycleGraph> graphs;
    double L = 0, h = 0;
    int64_t P = 0;
    int rec_cap = 0;
    int n_bins_total = 0;  // radial-bin amplitudes over all beams
    int n_bin_beams = 0;   // beams of kind RADIAL_BINS
    int n_theta = 0;       // driver parameters: one per Gaussian beam, n_bins per radial-bin beam
    hipStream_t stream = nullptr;

    // device memory carved from the caller's workspace
    wq::Level lev[wq::kMaxLevels];
    double* fields[5] = {};
    // fields of the slices before (initial-guess extrapolation); the arrays of
    // each field rotate by pointer
    double* fields_prev[5] = {};
    double* fields_prev2[5] = {};
    double* fields_prev3[5] = {};
    double* mom[6] = {};
    double* jz = nullptr;
    double* gpsi[2] = {};  // grad psi at the nodes (x, y), for the push
    // time loop (driver_max > 0): driver state [8][driver_max], the wake at its
    // mid-step positions [6][driver_max], the current planes (fixed point,
    // [driver_nz][N+1][pitch]), the previous slice's grad psi, and the cold
    // lattice the plasma restarts from at every time step
    double* drv = nullptr;
    double* drv_eb = nullptr;
    unsigned long long* drv_planes = nullptr;
    int64_t drv_n = 0;
    int drv_nz = 0;
    bool drv_active = false;  // inside wandqs_time_step's sweep
    double drv_dt = 0.0;
    double* gpsi_prev[2] = {};
    double* lat[2] = {};
    int32_t* lat_id = nullptr;
    // laser envelope (laser_nz > 0): two sets of planes [laser_nz][N+1][pitch]
    // (complex), las_env[las_cur] at the current time; |A-hat|^2 of the slice
    // and its node gradient; the complex multigrid's levels 1 .. las_ll (level
    // 0's iterate is the plane being advanced) and its norm partials
    double2* las_env[2] = {};
    int las_cur = 0;
    bool las_on = false;      // an envelope has been set: the plasma feels it
    bool las_adv = false;     // inside wandqs_time_step: each slice advances its plane
    double las_dt = 0.0;
    int las_j = 0;            // plane of the next slice in the time step's sweep
    int las_cycles = 0;       // multigrid cycles of the last plane advanced
    int las_pred = 1;         // cycles the last solved plane needed (first batch size)
    double* las_a2 = nullptr;
    double* las_g[2] = {};
    double2* las_u[wq::kMaxLevels] = {};
    double2* las_um[wq::kMaxLevels] = {};  // smoothed iterate of each down pass
    double2* las_f[wq::kMaxLevels] = {};
    double2* las_k[wq::kMaxLevels] = {};
    int las_ll = 0;           // level solved (with those below) by one workgroup
    double* las_part = nullptr;
    double* las_red = nullptr;
    // non-uniform grid solver (wandqs_nu_mg_solve): the per-level 1-D tables,
    // the norm partials [3][N-1] and their sums [3]
    double* nu_tab = nullptr;
    double* nu_part = nullptr;
    double* nu_red = nullptr;
    double* k2lev = nullptr;  // k2 of the coarse-kernel levels (dense, concatenated)
    float* k2levf = nullptr;  // the same in float, and 1 / (4 + h_l^2 k2) in float
    float* idlevf = nullptr;
    // exact Poisson solve on the 64^2 coarse level: sine-transform matrix S and
    // the scaled inverse eigenvalues M, [64][64] float each (zero row/column 63)
    float* dst_S = nullptr;
    float* dst_M = nullptr;
    // double copies of the tables for the mixed form, whose coarsest-grid
    // solve runs in FP64 (null in the FP64 form)
    double* dst_S64 = nullptr;
    double* dst_M64 = nullptr;
    // exact Poisson solve on level 1 by fast sine transforms (levels of 128^2
    // to 2048^2 below a finer one): the FP64 intermediates T1, T2 of each
    // right-hand side, [N1 - 1][N1 + 8]; the FFT twiddles exp(-2 pi i m / 2 N1),
    // m < 2 N1; and sin^2(pi k / 2 N1), k <= N1
    double* fst_t1[2] = {};
    double* fst_t2[2] = {};
    double2* fst_tw = nullptr;
    double* fst_s2 = nullptr;
    double* pa[2][4] = {};
    int32_t* pid[2] = {};
    int cur = 0;
    int32_t *key = nullptr, *perm = nullptr, *cell_count = nullptr, *cell_start = nullptr,
            *scan_blk = nullptr;
    int32_t* big_cells = nullptr;  // [N*N] cells too crowded for one thread's sort
    int32_t* big_count = nullptr;  // their number
    int n_scan_blocks = 0;
    double* st = nullptr;  // [xi, dxi, xi of fields, of fields_prev, of fields_prev2, of fields_prev3]
    double* vmax_part = nullptr;  // per push block
    int n_push_blocks = 0;
    int32_t* flags = nullptr;
    double* norm_part = nullptr;  // [kMaxSlots][kNormVec][max_tiles]
    uint32_t* pub_count = nullptr;  // workgroups of k_reduce_publish done (0 between batches)
    int max_tiles = 0;
    double* rec = nullptr;        // [rec_cap][4] : xi, dxi, vmax, flags
    double* probe_acc = nullptr;  // [kMaxProbes]
    double* bins_dev = nullptr;
    int32_t* bin_map = nullptr;  // [n_bin_beams][N+1]^2
    wq::BeamSet beamset{};

    // adjoint tape (checkpoint_every = K > 0): a checkpoint before every K-th
    // slice since init / set_state, one extra for the state at the start of a
    // backward sweep, and K slots for the slices of one recomputed segment
    int tape_K = 0;
    int n_ckpt = 0;
    int n_seg = 0, n_seg_cap = 0;
    int64_t tape_n = 0;     // slices since the tape start
    bool tape_ok = true;    // false after wandqs_mg_solve or past the capacity
    int64_t run_begin = 0;  // tape index of the first slice of the last wandqs_run
    int64_t run_len = -1;   // its slice count (-1: no completed run)
    std::vector<wq::Checkpoint> ckpt;
    std::vector<wq::TapeSlot> slot;
    wq::AdjBuffers adj;
    std::vector<double> probe_count;  // nodes in each probe disc

    // host side
    double* h_pin = nullptr;  // pinned coherent readback buffer
    uint32_t pub_seq = 0;     // last sequence number published into h_pin
    int pred[wq::kPredKinds] = {1, 1, 1, 1, 1, 1, 1, 1};  // V-cycles of the last solve per kind (batch size)
    bool failed = false;
    int n_guess = 0;  // slices since init/set_state, up to kGuessMax (extrapolation order + 1)
    std::string err;
    wq::SolveResult last[3];
    wq::Prof prof;
};

namespace wq {

// layout of the workspace (offsets from the base, computed for any base)
size_t carve(wandqs_ctx* c, char* base);
// layout of the arrays of a solve alone (the same rules; base may be NULL)
size_t carve_solver(wandqs_ctx* c, char* base);
// a context for solves only on cfg's grid; returns NULL or the reason cfg is invalid
const char* setup_solver_ctx(wandqs_ctx* c, const wandqs_config* cfg);
// message for wandqs_last_error(NULL) (copied into a fixed buffer)
void set_call_error(const char* m);
// smallest level that runs the register-tile pass kernels by default
int reg_tile_min_default();
// largest level with 16 x 16 LDS tiles by default
int small_tile_max_default();
// tables of the exact coarse-level Poisson solves (the 64^2 level and, when
// used, the fast sine transform solve on level 1), made on the device on the
// context's stream
wandqs_status make_dst_tables(wandqs_ctx* c);
// fast sine transform solve (fst.hip): whether the Poisson V-cycles end with
// it on level 1, the row stride of its intermediates, its tables, and the
// solve itself (R right-hand sides f of level 1 into u of level 1)
constexpr int kFstMinN = 128;
constexpr int kFstMaxN = 2048;
bool fst_used(const wandqs_ctx* c);
size_t fst_ld(const wandqs_ctx* c);
wandqs_status make_fst_tables(wandqs_ctx* c);
template <typename E>
void fst_solve(wandqs_ctx* c, int R, const E* const* f, E* const* u);

// multigrid (mg.hip)
// ahead (optional): work that reads the solution but does not change what the
// solve reads, enqueued behind the first batch of cycles while the host waits
// for its residual norms (so that the device does not idle), and enqueued once
// more behind the last cycle when further cycles follow.
// k2_levels_ready: helm_levels(c, k2) has run already for this k2.
wandqs_status mg_solve(wandqs_ctx* c, int kind, int R, bool helm, double* const u[2],
                       double* const f[2], const double* k2, SolveResult* res,
                       const std::function<wandqs_status()>& ahead = {},
                       bool k2_levels_ready = false);
// The Helmholtz operator's k2 on the coarser levels (full weighting level by
// level, then the coarse kernel's dense levels), from the finest level's k2.
wandqs_status helm_levels(wandqs_ctx* c, const double* k2);

// particles and fields (particles.hip, fields.hip)
wandqs_status slice_sort(wandqs_ctx* c);
wandqs_status deposit_n(wandqs_ctx* c);
wandqs_status deposit_jT(wandqs_ctx* c);
wandqs_status rhs_EB(wandqs_ctx* c);
wandqs_status plasma_jz(wandqs_ctx* c);
wandqs_status assemble(wandqs_ctx* c, bool jz_ready = false);
wandqs_status push_and_step(wandqs_ctx* c, int rec_slot, bool grad_ready = false);
wandqs_status probes_accumulate(wandqs_ctx* c, int64_t slice);
wandqs_status pack_fields(wandqs_ctx* c, double* const* src, int n, double* dst);
wandqs_status unpack_fields(wandqs_ctx* c, const double* src, int n, double* const* dst);
wandqs_status particles_to_id_order(wandqs_ctx* c, double* dst);
wandqs_status particles_from_id_order(wandqs_ctx* c, const double* src);
wandqs_status fill_f64(wandqs_ctx* c, double* p, size_t n, double v);
wandqs_status extrapolate_guess(wandqs_ctx* c, int order);
wandqs_status copy_d2d(wandqs_ctx* c, void* dst, const void* src, size_t bytes);
wandqs_status probe_seed(wandqs_ctx* c, int k, double w, double* const* Fb);

// laser envelope (laser.hip): |A-hat|^2 of the slice at st[0] and its node
// gradient; one plane's time step (chi: n* / (1+psi) at the nodes, may be
// null); dense <-> padded copies of the planes
wandqs_status laser_nodes(wandqs_ctx* c);
wandqs_status laser_plane_advance(wandqs_ctx* c, double dt, const double* chi, int j, int* cycles);
wandqs_status laser_unpack(wandqs_ctx* c, const double* src, int set);
wandqs_status laser_pack(wandqs_ctx* c, double* dst);
// doubles of the non-uniform solver's 1-D tables for an N-cell grid (nonuniform.hip)
size_t nu_table_doubles(int N);
// node gradient (central inside, one-sided on the boundary lines), as the
// push's grad psi (particles.hip)
wandqs_status node_gradient(wandqs_ctx* c, const double* u, double* gx, double* gy);

// time loop (driver.hip)
wandqs_status driver_deposit(wandqs_ctx* c);
wandqs_status driver_gather(wandqs_ctx* c, double dt);
wandqs_status driver_push(wandqs_ctx* c, double dt);

// adjoint (adjoint.hip); tape slot t holds the slice, tape index j its place
// in the slice sequence (for probe seeds)
wandqs_status slice_adjoint(wandqs_ctx* c, const TapeSlot& ts, const double* d_field_bar,
                            const double* probe_w);
wandqs_status adj_zero_solutions(wandqs_ctx* c);
wandqs_status adj_reduce_theta_init(wandqs_ctx* c);

// node inside the disc |x - x0| <= r of a probe, in IEEE double without
// contraction (the host and the device take the same decision)
bool node_in_disc_host(double L, double h, int a, int b, double x0, double y0, double r);

const char* hip_err(hipError_t e);

// Timing of one kernel launch when profiling is on: a pair of events that the
// launch itself records (WQ_KLAUNCH), so the interval is the kernel's dispatch,
// with no event packets in between.
class ProfScope {
  public:
    ProfScope(wandqs_ctx* c, const char* name, double bytes);
    ~ProfScope();
    hipEvent_t start() const { return a_; }
    hipEvent_t stop() const { return b_; }

  private:
    wandqs_ctx* c_;
    int cls_ = -1;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    double bytes_ = 0;
};
void prof_harvest(wandqs_ctx* c);
void prof_reset(wandqs_ctx* c, bool on);

}  // namespace wq

// Kernel launch under a ProfScope: with profiling on, the dispatch records the
// scope's start and stop events.
#define WQ_KLAUNCH(ps, kernel, grid, block, shmem, stream, ...)                          \
    do {                                                                                \
        if ((ps).start())                                                               \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, (ps).start(),     \
                                  (ps).stop(), 0, __VA_ARGS__);                         \
        else                                                                            \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);        \
    } while (0)

#define WQ_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            c->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
            return WANDQS_E_HIP;                                                      \
        }                                                                             \
    } while (0)

#define WQ_LAUNCH_CHECK()                                                             \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) {                                                       \
            c->err = std::string("kernel launch: ") + hipGetErrorString(e_);          \
            return WANDQS_E_HIP;                                                      \
        }                                                                             \
    } while (0)
