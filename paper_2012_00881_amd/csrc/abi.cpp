// C ABI of the wandqs library: configuration checks, workspace layout, plasma
// initialisation and the slice loop (WAND-PIC Algorithm 1, inner xi loop).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <vector>
#include <new>
#include <string>

#include "wq_common.h"

namespace {

// message of the last failed call made without a context (copied into a fixed
// buffer: no allocation on the paths that must not allocate)
thread_local char g_init_err[256];

void set_init_err(const char* m) {
    std::snprintf(g_init_err, sizeof g_init_err, "%s", m ? m : "");
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Returns NULL when the configuration is valid, else the reason.
const char* check_config(const wandqs_config* c, int32_t n_slices) {
    if (!c) return "config is NULL";
    if (n_slices < 1) return "n_slices must be >= 1";
    if (!is_pow2(c->n_cells) || c->n_cells < 8 || c->n_cells > 4096)
        return "n_cells must be a power of two in [8, 4096]";
    if (!(c->half_width > 0.0) || !std::isfinite(c->half_width)) return "half_width must be > 0";
    if (c->ppc_side < 1 || c->ppc_side > 4) return "ppc_side must be in [1, 4]";
    if (!(c->jitter >= 0.0) || c->jitter > 0.5 / c->ppc_side)
        return "jitter must be in [0, 0.5/ppc_side]";
    if (!(c->n0 > 0.0) || !std::isfinite(c->n0)) return "n0 must be > 0";
    if (!(c->dxi0 > 0.0) || !std::isfinite(c->dxi0)) return "dxi0 must be > 0";
    if (c->adaptive != 0 && c->adaptive != 1) return "adaptive must be 0 or 1";
    if (c->refine_k < 0) return "refine_k must be >= 0";
    if (c->precision != WANDQS_FP64 && c->precision != WANDQS_MIXED) return "unknown precision";
    if (c->mg_inner_cycles < 0 || c->mg_inner_cycles > 8) return "mg_inner_cycles must be in [0, 8]";
    if (!std::isfinite(c->mg_rtol) || !(c->mg_atol >= 0.0)) return "bad mg_rtol / mg_atol";
    if (c->mg_max_cycles < 1 || c->mg_max_cycles > 200) return "mg_max_cycles must be in [1, 200]";
    if (c->nu_pre < 1 || c->nu_pre > 3 || c->nu_post < 1 || c->nu_post > 3)
        return "nu_pre and nu_post must be in [1, 3]";
    for (double om : {c->mg_omega, c->mg_omega_helm})
        if (!(om == 0.0 || (om > 0.0 && om < 2.0))) return "mg_omega and mg_omega_helm must be in (0, 2) or 0";
    if (c->n_beams < 0 || c->n_beams > wq::kMaxBeams) return "n_beams must be in [0, 8]";
    if (c->n_beams > 0 && !c->beams) return "beams is NULL";
    for (int k = 0; k < c->n_beams; ++k) {
        const wandqs_beam& b = c->beams[k];
        if (!(b.sigma_z > 0.0)) return "beam sigma_z must be > 0";
        if (b.kind == WANDQS_BEAM_GAUSS) {
            if (!(b.sigma_r > 0.0)) return "beam sigma_r must be > 0";
        } else if (b.kind == WANDQS_BEAM_RADIAL_BINS) {
            if (b.n_bins < 1 || b.n_bins > 4096 || !(b.r_max > 0.0) || !b.bin_amp)
                return "radial-bin beam needs 1..4096 bins, r_max > 0 and bin_amp";
        } else {
            return "unknown beam kind";
        }
    }
    if (c->n_probes < 0 || c->n_probes > wq::kMaxProbes) return "n_probes must be in [0, 16]";
    if (c->n_probes > 0 && !c->probes) return "probes is NULL";
    for (int k = 0; k < c->n_probes; ++k) {
        const wandqs_probe& p = c->probes[k];
        if (p.field < 0 || p.field > 4 || p.slice_begin < 0 || p.slice_end <= p.slice_begin ||
            !(p.r_max >= 0.0))
            return "bad probe";
    }
    if (c->checkpoint_every < 0) return "checkpoint_every must be >= 0";
    if (c->adjoint_hold_dxi != 0 && c->adjoint_hold_dxi != 1) return "adjoint_hold_dxi must be 0 or 1";
    if (c->pusher != WANDQS_PUSH_BORIS && c->pusher != WANDQS_PUSH_RK1 &&
        c->pusher != WANDQS_PUSH_RK2 && c->pusher != WANDQS_PUSH_RK4)
        return "pusher must be WANDQS_PUSH_BORIS, _RK1, _RK2 or _RK4";
    if (c->checkpoint_every > 0 && c->pusher != WANDQS_PUSH_BORIS)
        return "the adjoint tape needs the Boris-like pusher (the reverse sweep is its adjoint)";
    if (c->driver_max < 0) return "driver_max must be >= 0";
    if (c->driver_max > 0) {
        if (c->driver_nz < 2 || c->driver_nz > 65536 || !(c->driver_dz > 0.0) ||
            !std::isfinite(c->driver_xi0))
            return "a time loop needs driver_nz in [2, 65536], driver_dz > 0 and a finite driver_xi0";
        if (c->checkpoint_every > 0) return "the time loop (driver_max > 0) has no adjoint tape";
    }
    if (c->laser_nz < 0 || c->laser_nz > 65536) return "laser_nz must be in [0, 65536]";
    if (c->driver_nsub < 0 || c->driver_nsub > 4096) return "driver_nsub must be in [0, 4096]";
    if (c->laser_nz > 0) {
        if (!(c->laser_k0 > 0.0) || !std::isfinite(c->laser_k0)) return "a laser needs laser_k0 > 0";
        if (c->checkpoint_every > 0) return "a laser envelope (laser_nz > 0) has no adjoint tape";
    }
    if (c->checkpoint_every > 0 && c->adaptive && !c->adjoint_hold_dxi)
        return "a tape with adaptive steps differentiates with the forward's steps held fixed "
               "(they depend on the state through Vmax): set adjoint_hold_dxi = 1 to accept that";
    return nullptr;
}

// SplitMix64 (Steele, Lea & Flood 2014), counter form: draw k of stream `seed`.
uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double unit(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

int total_bins(const wandqs_config* cfg) {
    int t = 0;
    for (int k = 0; k < cfg->n_beams; ++k)
        if (cfg->beams[k].kind == WANDQS_BEAM_RADIAL_BINS) t += cfg->beams[k].n_bins;
    return t;
}

void set_sizes(wandqs_ctx* c, const wandqs_config* cfg, int32_t n_slices) {
    c->N = cfg->n_cells;
    c->L = cfg->half_width;
    c->h = 2.0 * c->L / c->N;
    c->ppc = cfg->ppc_side * cfg->ppc_side;
    c->P = (int64_t)c->N * c->N * c->ppc;
    c->nlev = 0;
    for (int n = c->N; n >= 2; n /= 2) {
        wq::Level& L = c->lev[c->nlev];
        L.N = n;
        L.h = c->h * (double)(c->N / n);
        L.pitch = ((n + 1) + 7) & ~7;
        ++c->nlev;
    }
    // lc: first level with N <= kCoarseMax
    c->lc = 0;
    while (c->lev[c->lc].N > wq::kCoarseMax) ++c->lc;
    {
        const char* e = std::getenv("WANDQS_MG_TILES");
        c->reg_tile_min = (e && std::strcmp(e, "lds") == 0) ? INT_MAX : wq::reg_tile_min_default();
        if (e && std::atoi(e) >= 8) c->reg_tile_min = std::atoi(e);  // smallest register-tile level
        const char* st = std::getenv("WANDQS_MG_SMALL");
        c->small_tile_max = st && std::atoi(st) >= 8 ? std::atoi(st) : wq::small_tile_max_default();
        const char* sp = std::getenv("WANDQS_MG_SPLIT");
        const std::string spm = sp ? sp : "";
        c->reg_split = !(spm == "0" || spm == "lds");
        c->lds_split = !(spm == "0" || spm == "reg");
        const char* fu = std::getenv("WANDQS_MG_FUSE");
        c->mg_fuse = !(fu && std::strcmp(fu, "0") == 0);
        const char* g = std::getenv("WANDQS_GRAPHS");
        c->graphs_on = g && std::strcmp(g, "1") == 0;
    }
    const int t = (c->N + 15) / 16;  // norm partials: one per tile of the smallest tile size
    c->max_tiles = t * t;
    c->n_push_blocks = (int)((c->P + 255) / 256);
    c->n_scan_blocks = (c->N * c->N + 2047) / 2048;
    c->rec_cap = n_slices;
    c->n_bins_total = total_bins(cfg);
    c->n_bin_beams = 0;
    c->n_theta = 0;
    c->n_seg_cap = 0;
    const int nn = (c->N + 1) * (c->N + 1);
    const int segs_all = (nn + wq::kThetaSeg - 1) / wq::kThetaSeg;
    for (int k = 0; k < cfg->n_beams; ++k) {
        if (cfg->beams[k].kind == WANDQS_BEAM_RADIAL_BINS) {
            ++c->n_bin_beams;
            c->n_theta += cfg->beams[k].n_bins;
            c->n_seg_cap += cfg->beams[k].n_bins + segs_all;
        } else {
            ++c->n_theta;
            c->n_seg_cap += segs_all;
        }
    }
    c->drv_nz = cfg->driver_max > 0 ? cfg->driver_nz : 0;
    c->las_ll = 0;  // the laser's workgroup levels: N <= 32
    while (c->lev[c->las_ll].N > 32) ++c->las_ll;
    c->tape_K = cfg->checkpoint_every;
    c->n_ckpt = c->tape_K > 0 ? (n_slices + c->tape_K - 1) / c->tape_K + 1 : 0;
}

// relaxation factors measured to minimise the V-cycles per solve on the
// blowout workloads (the Helmholtz one on its levels with h^2 n0 <= 1/8)
void apply_defaults(wandqs_ctx* c) {
    if (c->cfg.mg_omega == 0.0) c->cfg.mg_omega = 1.175;
    if (c->cfg.mg_omega_helm == 0.0) c->cfg.mg_omega_helm = 1.175;
}

wandqs_status fail(wandqs_ctx* c, wandqs_status s) {
    if (s != WANDQS_OK && s != WANDQS_E_INVALID) c->failed = true;
    return s;
}

size_t node_bytes(const wandqs_ctx* c) {
    return sizeof(double) * (size_t)(c->N + 1) * c->lev[0].pitch;
}

// Checkpoint of the slice-loop state: particles (storage order), the fields
// and the two previous slices' fields (initial guesses), the xi state,
// the batch predictions and the extrapolation count.  A recompute from it
// repeats the same arithmetic, bit for bit.
wandqs_status save_checkpoint(wandqs_ctx* c, wq::Checkpoint& k) {
    using namespace wq;
    wandqs_status s;
    const size_t pb = sizeof(double) * (size_t)c->P, nb = node_bytes(c);
    for (int q = 0; q < 4; ++q)
        if ((s = copy_d2d(c, k.pa[q], c->pa[c->cur][q], pb)) != WANDQS_OK) return s;
    if ((s = copy_d2d(c, k.pid, c->pid[c->cur], sizeof(int32_t) * (size_t)c->P)) != WANDQS_OK) return s;
    for (int q = 0; q < 5; ++q) {
        if ((s = copy_d2d(c, k.fields[q], c->fields[q], nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, k.fields_prev[q], c->fields_prev[q], nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, k.fields_prev2[q], c->fields_prev2[q], nb)) != WANDQS_OK) return s;
        if (kGuessMax > 3 && (s = copy_d2d(c, k.fields_prev3[q], c->fields_prev3[q], nb)) != WANDQS_OK)
            return s;
    }
    if ((s = copy_d2d(c, k.st, c->st, 6 * sizeof(double))) != WANDQS_OK) return s;
    std::memcpy(k.pred, c->pred, sizeof(k.pred));
    k.n_guess = c->n_guess;
    return WANDQS_OK;
}

wandqs_status restore_checkpoint(wandqs_ctx* c, const wq::Checkpoint& k) {
    using namespace wq;
    wandqs_status s;
    const size_t pb = sizeof(double) * (size_t)c->P, nb = node_bytes(c);
    for (int q = 0; q < 4; ++q)
        if ((s = copy_d2d(c, c->pa[c->cur][q], k.pa[q], pb)) != WANDQS_OK) return s;
    if ((s = copy_d2d(c, c->pid[c->cur], k.pid, sizeof(int32_t) * (size_t)c->P)) != WANDQS_OK) return s;
    for (int q = 0; q < 5; ++q) {
        if ((s = copy_d2d(c, c->fields[q], k.fields[q], nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, c->fields_prev[q], k.fields_prev[q], nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, c->fields_prev2[q], k.fields_prev2[q], nb)) != WANDQS_OK) return s;
        if (kGuessMax > 3 && (s = copy_d2d(c, c->fields_prev3[q], k.fields_prev3[q], nb)) != WANDQS_OK)
            return s;
    }
    if ((s = copy_d2d(c, c->st, k.st, 6 * sizeof(double))) != WANDQS_OK) return s;
    std::memcpy(c->pred, k.pred, sizeof(k.pred));
    c->n_guess = k.n_guess;
    return WANDQS_OK;
}

// One slice (Algorithm 1 inner loop body).  taping: the slice belongs to the
// sequence the adjoint can reverse (a checkpoint is taken before every K-th);
// rec (or NULL) receives what the reverse of this slice reads.
wandqs_status do_slice(wandqs_ctx* c, int rec_slot, int64_t probe_slice, bool taping,
                       const wq::TapeSlot* rec) {
    using namespace wq;
    wandqs_status s;
    Level& L0 = c->lev[0];
    if (taping && c->tape_K > 0 && c->tape_n >= c->rec_cap) c->tape_ok = false;  // capacity
    if (taping && c->tape_K > 0 && c->tape_ok && c->tape_n % c->tape_K == 0) {
        const int64_t k = c->tape_n / c->tape_K;
        if (k >= c->n_ckpt - 1) c->tape_ok = false;  // past the capacity given at init
        else if ((s = save_checkpoint(c, c->ckpt[k])) != WANDQS_OK) return s;
    }
    // initial guesses: the previous slice's fields (Sec. VII.A), extrapolated in
    // xi through the last slices once they are known
    if ((s = extrapolate_guess(c, c->n_guess - 1)) != WANDQS_OK) return s;
    // a laser envelope's |A-hat|^2 at this slice and its gradient (ponderomotive terms)
    c->las_cycles = 0;
    if (c->las_on && (s = laser_nodes(c)) != WANDQS_OK) return s;
    if ((s = slice_sort(c)) != WANDQS_OK) return s;
    if (rec) {
        const size_t pb = sizeof(double) * (size_t)c->P;
        for (int q = 0; q < 4; ++q)
            if ((s = copy_d2d(c, rec->pa[q], c->pa[c->cur][q], pb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, rec->pid, c->pid[c->cur], sizeof(int32_t) * (size_t)c->P)) != WANDQS_OK)
            return s;
        if ((s = copy_d2d(c, rec->start, c->cell_start, sizeof(int32_t) * ((size_t)c->N * c->N + 1))) !=
            WANDQS_OK)
            return s;
    }
    if ((s = deposit_n(c)) != WANDQS_OK) return s;  // Collect_Source: n*
    double* u1[2] = {c->fields[0], nullptr};
    double* f1[2] = {L0.f[0], nullptr};
    // the j, T deposit (Collect_Source) reads psi only: it runs behind the psi
    // solve's first batch while the host waits for that batch's norms (and
    // again after any further cycle; its 1 + psi <= 0 flag on the first
    // batch's iterate, which differs from the solution by the last cycles'
    // corrections, marks a state at breakdown either way)
    if ((s = mg_solve(c, kSolvePsi, 1, false, u1, f1, nullptr, &c->last[0],
                      [c] { return deposit_jT(c); })) != WANDQS_OK)
        return s;
    if ((s = rhs_EB(c)) != WANDQS_OK) return s;
    double* u2[2] = {c->fields[1], c->fields[2]};
    double* f2[2] = {L0.f[0], L0.f[1]};
    // j_z and k2 = n*/g (with its coarser levels for the B_perp multigrid) do
    // not read E_z or B_z: they run behind the E_z / B_z solve's first batch
    if ((s = mg_solve(c, kSolveEB, 2, false, u2, f2, nullptr, &c->last[1], [c, &L0] {
             const wandqs_status st = plasma_jz(c);
             return st != WANDQS_OK ? st : helm_levels(c, L0.k2);
         })) != WANDQS_OK)
        return s;
    if ((s = assemble(c, true)) != WANDQS_OK) return s;
    double* u3[2] = {c->fields[3], c->fields[4]};
    // grad psi for the push does not read B_perp: it runs behind the B_perp
    // solve's first batch
    if ((s = mg_solve(c, kSolveBperp, 2, true, u3, f2, L0.k2, &c->last[2],
                      [c] { return node_gradient(c, c->fields[0], c->gpsi[0], c->gpsi[1]); },
                      true)) != WANDQS_OK)
        return s;
    if (rec) {
        const size_t nb = node_bytes(c);
        for (int q = 0; q < 5; ++q)
            if ((s = copy_d2d(c, rec->fields[q], c->fields[q], nb)) != WANDQS_OK) return s;
        for (int q = 0; q < 6; ++q)
            if ((s = copy_d2d(c, rec->mom[q], c->mom[q], nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, rec->k2, L0.k2, nb)) != WANDQS_OK) return s;
        if ((s = copy_d2d(c, rec->st, c->st, 2 * sizeof(double))) != WANDQS_OK) return s;
    }
    if (!c->probes.empty() && (s = probes_accumulate(c, probe_slice)) != WANDQS_OK) return s;
    if ((s = push_and_step(c, rec_slot, true)) != WANDQS_OK) return s;  // Push_Trajectory + Step_Size_Refinement
    if (c->drv_active) {
        // the driver particles whose mid-step xi lies between the previous
        // slice and this one take their wake from the two; this slice's
        // grad psi becomes the previous one
        if (c->n_guess >= 1 && (s = driver_gather(c, c->drv_dt)) != WANDQS_OK) return s;
        std::swap(c->gpsi[0], c->gpsi_prev[0]);
        std::swap(c->gpsi[1], c->gpsi_prev[1]);
    }
    if (c->las_adv) {
        // time loop: this slice's plane of the envelope advances by dt with the
        // slice's susceptibility chi = n* / (1+psi), the k2 of its B_perp system
        if (c->las_j < c->cfg.laser_nz &&
            (s = laser_plane_advance(c, c->las_dt, L0.k2, c->las_j, &c->las_cycles)) != WANDQS_OK)
            return s;
        ++c->las_j;
    }
    if (c->n_guess < kGuessMax) ++c->n_guess;
    if (taping) ++c->tape_n;
    return WANDQS_OK;
}

void fill_info_host(const wandqs_ctx* c, wandqs_slice_info* info) {
    const wq::SolveResult* r = c->last;
    const int idx[5][2] = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}};
    for (int k = 0; k < 5; ++k) {
        info->vcycles[k] = r[idx[k][0]].cycles;
        info->rel_resid[k] = r[idx[k][0]].rel[idx[k][1]];
    }
    info->laser_vcycles = c->las_cycles;
}

wandqs_status check_flags(wandqs_ctx* c) {
    int32_t fl = 0;
    WQ_HIP(hipMemcpyAsync(&fl, c->flags, sizeof(fl), hipMemcpyDeviceToHost, c->stream));
    WQ_HIP(hipStreamSynchronize(c->stream));
    if (fl & 1) {
        c->err = "1 + psi <= 0 where plasma is present";
        return WANDQS_E_NONPHYS;
    }
    return WANDQS_OK;
}

// Tables of the exact coarse Poisson solves (the 64^2 sine matrices in float,
// with double copies for the mixed form's FP64 coarsest-grid solve) and the
// arrays of the fast sine transform solve on level 1.
template <class Take>
void carve_dst(wandqs_ctx* c, Take&& take) {
    const bool mixed = c->cfg.precision == WANDQS_MIXED;
    c->dst_S = (float*)take(sizeof(float) * 64 * 64);
    c->dst_M = (float*)take(sizeof(float) * 64 * 64);
    c->dst_S64 = mixed ? (double*)take(sizeof(double) * 64 * 64) : nullptr;
    c->dst_M64 = mixed ? (double*)take(sizeof(double) * 64 * 64) : nullptr;
    if (wq::fst_used(c)) {
        const size_t n1 = c->lev[1].N;
        for (int r = 0; r < 2; ++r) {
            c->fst_t1[r] = (double*)take(sizeof(double) * (n1 - 1) * wq::fst_ld(c));
            c->fst_t2[r] = (double*)take(sizeof(double) * (n1 - 1) * wq::fst_ld(c));
        }
        c->fst_tw = (double2*)take(sizeof(double2) * 2 * n1);
        c->fst_s2 = (double*)take(sizeof(double) * (n1 + 1));
    }
}

}  // namespace

size_t wq::carve(wandqs_ctx* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~(size_t)255;
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    auto arr = [&](int l) {
        return (double*)take(sizeof(double) * (size_t)(c->lev[l].N + 1) * c->lev[l].pitch);
    };
    Level& L0 = c->lev[0];
    for (int k = 0; k < 5; ++k) c->fields[k] = arr(0);
    for (int k = 0; k < 5; ++k) c->fields_prev[k] = arr(0);
    for (int k = 0; k < 5; ++k) c->fields_prev2[k] = arr(0);
    if (kGuessMax > 3)
        for (int k = 0; k < 5; ++k) c->fields_prev3[k] = arr(0);
    for (int r = 0; r < 2; ++r) {
        L0.um[r] = arr(0);
        L0.um2[r] = c->N >= c->reg_tile_min ? arr(0) : nullptr;
        L0.f[r] = arr(0);
    }
    L0.k2 = arr(0);
    for (int k = 0; k < 6; ++k) c->mom[k] = arr(0);
    c->jz = arr(0);
    {
        int tot = 0;
        for (int n = c->lev[c->lc].N; n >= 2; n /= 2) tot += (n + 1) * (n + 1);
        c->k2lev = (double*)take(sizeof(double) * (size_t)tot);
        c->k2levf = (float*)take(sizeof(float) * (size_t)tot);
        c->idlevf = (float*)take(sizeof(float) * (size_t)tot);
    }
    carve_dst(c, take);
    for (int l = 1; l <= c->lc; ++l) {
        Level& L = c->lev[l];
        for (int r = 0; r < 2; ++r) {
            L.u[r] = arr(l);
            L.um[r] = l < c->lc ? arr(l) : nullptr;
            L.f[r] = arr(l);
        }
        L.k2 = arr(l);
    }
    if (c->cfg.precision == WANDQS_MIXED) {
        auto arr32 = [&](int l) {
            return (float*)take(sizeof(float) * (size_t)(c->lev[l].N + 1) * c->lev[l].pitch);
        };
        for (int l = 0; l <= c->lc; ++l)
            for (int r = 0; r < 2; ++r) {
                Level& L = c->lev[l];
                L.u32[r] = arr32(l);
                L.um32[r] = l < c->lc ? arr32(l) : nullptr;
                L.f32[r] = arr32(l);
            }
    }
    const size_t P = (size_t)c->P;
    const size_t ncell = (size_t)c->N * c->N;
    for (int s = 0; s < 2; ++s) {
        for (int k = 0; k < 4; ++k) c->pa[s][k] = (double*)take(sizeof(double) * P);
        c->pid[s] = (int32_t*)take(sizeof(int32_t) * P);
    }
    c->key = (int32_t*)take(sizeof(int32_t) * P);
    c->perm = (int32_t*)take(sizeof(int32_t) * P);
    for (int q = 0; q < 2; ++q) c->gpsi[q] = arr(0);
    if (c->cfg.driver_max > 0) {
        const size_t D = (size_t)c->cfg.driver_max;
        c->drv = (double*)take(sizeof(double) * 8 * D);
        c->drv_eb = (double*)take(sizeof(double) * 6 * D);
        c->drv_planes = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)c->drv_nz *
                                                  (c->N + 1) * L0.pitch);
        for (int q = 0; q < 2; ++q) c->gpsi_prev[q] = arr(0);
    }
    if (c->cfg.driver_max > 0 || c->cfg.laser_nz > 0) {  // the time loop's cold lattice
        for (int q = 0; q < 2; ++q) c->lat[q] = (double*)take(sizeof(double) * P);
        c->lat_id = (int32_t*)take(sizeof(int32_t) * P);
    }
    if (c->cfg.laser_nz > 0) {
        auto carr = [&](int l) {
            return (double2*)take(sizeof(double2) * (size_t)(c->lev[l].N + 1) * c->lev[l].pitch);
        };
        const size_t plane = (size_t)(c->N + 1) * L0.pitch;
        for (int q = 0; q < 2; ++q)
            c->las_env[q] = (double2*)take(sizeof(double2) * plane * (size_t)c->cfg.laser_nz);
        c->las_a2 = arr(0);
        for (int q = 0; q < 2; ++q) c->las_g[q] = arr(0);
        for (int l = 0; l <= c->las_ll; ++l) {
            c->las_u[l] = l ? carr(l) : nullptr;
            c->las_um[l] = l < c->las_ll ? carr(l) : nullptr;
            c->las_f[l] = carr(l);
            c->las_k[l] = carr(l);
        }
        c->las_part = (double*)take(sizeof(double) * 4 * (size_t)(c->N + 1));
        c->las_red = (double*)take(sizeof(double) * 4);
    }
    c->nu_tab = (double*)take(sizeof(double) * nu_table_doubles(c->N));
    c->nu_part = (double*)take(sizeof(double) * 3 * (size_t)(c->N + 1));
    c->nu_red = (double*)take(sizeof(double) * 4);
    c->cell_count = (int32_t*)take(sizeof(int32_t) * ncell);
    c->cell_start = (int32_t*)take(sizeof(int32_t) * (ncell + 1));
    c->big_cells = (int32_t*)take(sizeof(int32_t) * ncell);
    c->big_count = (int32_t*)take(sizeof(int32_t));
    c->scan_blk = (int32_t*)take(sizeof(int32_t) * c->n_scan_blocks);
    c->st = (double*)take(sizeof(double) * 16);  // [xi, dxi, 4 slice positions, -, -, guess weights]
    c->vmax_part = (double*)take(sizeof(double) * c->n_push_blocks);
    c->flags = (int32_t*)take(sizeof(int32_t) * 4);
    c->norm_part = (double*)take(sizeof(double) * kMaxSlots * kNormVec * (size_t)c->max_tiles);
    c->pub_count = (uint32_t*)take(sizeof(uint32_t));
    c->rec = (double*)take(sizeof(double) * 4 * (size_t)c->rec_cap);
    c->probe_acc = (double*)take(sizeof(double) * kMaxProbes);
    c->bins_dev = (double*)take(sizeof(double) * (size_t)(c->n_bins_total + 1));
    const size_t nnd = (size_t)(c->N + 1) * (c->N + 1);
    c->bin_map = (int32_t*)take(sizeof(int32_t) * nnd * (size_t)c->n_bin_beams);
    if (c->tape_K > 0) {
        c->ckpt.assign(c->n_ckpt, Checkpoint{});
        for (auto& k : c->ckpt) {
            for (int q = 0; q < 4; ++q) k.pa[q] = (double*)take(sizeof(double) * P);
            k.pid = (int32_t*)take(sizeof(int32_t) * P);
            for (int q = 0; q < 5; ++q) {
                k.fields[q] = arr(0);
                k.fields_prev[q] = arr(0);
                k.fields_prev2[q] = arr(0);
                k.fields_prev3[q] = kGuessMax > 3 ? arr(0) : nullptr;
            }
            k.st = (double*)take(sizeof(double) * 8);
        }
        c->slot.assign(std::min(c->tape_K, c->rec_cap), TapeSlot{});
        for (auto& t : c->slot) {
            for (int q = 0; q < 4; ++q) t.pa[q] = (double*)take(sizeof(double) * P);
            t.pid = (int32_t*)take(sizeof(int32_t) * P);
            t.start = (int32_t*)take(sizeof(int32_t) * (ncell + 1));
            for (int q = 0; q < 5; ++q) t.fields[q] = arr(0);
            for (int q = 0; q < 6; ++q) t.mom[q] = arr(0);
            t.k2 = arr(0);
            t.st = (double*)take(sizeof(double) * 2);
        }
        AdjBuffers& A = c->adj;
        double** node[] = {&A.Gxb, &A.Gyb, &A.Bxb, &A.Byb, &A.Bzb, &A.Ezb, &A.psib, &A.lx, &A.ly,
                           &A.lE, &A.lB, &A.lpsi, &A.nb, &A.jxb, &A.jyb, &A.txxb, &A.txyb, &A.tyyb,
                           &A.psxb, &A.psyb, &A.gnb, &A.psib_dep, &A.jzb};
        for (double** p : node) *p = arr(0);
        double** part[] = {&A.xb, &A.yb, &A.pxb, &A.pyb, &A.gb};
        for (double** p : part) *p = (double*)take(sizeof(double) * P);
        A.adj_id = (double*)take(sizeof(double) * 4 * P);
        A.theta_bar = (double*)take(sizeof(double) * (size_t)(c->n_theta + 1));
        A.theta_part = (double*)take(sizeof(double) * (size_t)(c->n_seg_cap + 1));
        A.seg = (int32_t*)take(sizeof(int32_t) * 4 * (size_t)(c->n_seg_cap + 1));
        A.seg_first = (int32_t*)take(sizeof(int32_t) * (size_t)(c->n_theta + 1));
        A.bin_nodes = (int32_t*)take(sizeof(int32_t) * nnd * (size_t)(c->n_bin_beams + 1));
    }
    return (off + 255) & ~(size_t)255;
}

// The arrays of a solve alone (wandqs_mg_solve_noalloc): the two level-0
// iterates, the level hierarchy, the coarse-level k2 arrays, the sine-transform
// tables and one residual-norm slot, in the layout carve() gives them inside a
// context's workspace.
size_t wq::carve_solver(wandqs_ctx* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~(size_t)255;
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    auto arr = [&](int l) {
        return (double*)take(sizeof(double) * (size_t)(c->lev[l].N + 1) * c->lev[l].pitch);
    };
    Level& L0 = c->lev[0];
    for (int k = 0; k < 2; ++k) c->fields[k] = arr(0);
    for (int r = 0; r < 2; ++r) {
        L0.um[r] = arr(0);
        L0.um2[r] = c->N >= c->reg_tile_min ? arr(0) : nullptr;
        L0.f[r] = arr(0);
    }
    L0.k2 = arr(0);
    {
        int tot = 0;
        for (int n = c->lev[c->lc].N; n >= 2; n /= 2) tot += (n + 1) * (n + 1);
        c->k2lev = (double*)take(sizeof(double) * (size_t)tot);
        c->k2levf = (float*)take(sizeof(float) * (size_t)tot);
        c->idlevf = (float*)take(sizeof(float) * (size_t)tot);
    }
    carve_dst(c, take);
    for (int l = 1; l <= c->lc; ++l) {
        Level& L = c->lev[l];
        for (int r = 0; r < 2; ++r) {
            L.u[r] = arr(l);
            L.um[r] = l < c->lc ? arr(l) : nullptr;
            L.f[r] = arr(l);
        }
        L.k2 = arr(l);
    }
    if (c->cfg.precision == WANDQS_MIXED) {
        auto arr32 = [&](int l) {
            return (float*)take(sizeof(float) * (size_t)(c->lev[l].N + 1) * c->lev[l].pitch);
        };
        for (int l = 0; l <= c->lc; ++l)
            for (int r = 0; r < 2; ++r) {
                Level& L = c->lev[l];
                L.u32[r] = arr32(l);
                L.um32[r] = l < c->lc ? arr32(l) : nullptr;
                L.f32[r] = arr32(l);
            }
    }
    c->norm_part = (double*)take(sizeof(double) * kNormVec * (size_t)c->max_tiles);
    c->pub_count = (uint32_t*)take(sizeof(uint32_t));
    return (off + 255) & ~(size_t)255;
}

// A context for solves on cfg's grid only: its sizes and settings, no beams,
// probes, tape or HIP graphs.  Returns the reason when cfg is not valid.
const char* wq::setup_solver_ctx(wandqs_ctx* c, const wandqs_config* cfg) {
    if (!cfg) return "config is NULL";
    c->cfg = *cfg;
    c->cfg.n_beams = 0;
    c->cfg.beams = nullptr;
    c->cfg.n_probes = 0;
    c->cfg.probes = nullptr;
    c->cfg.checkpoint_every = 0;
    if (const char* e = check_config(&c->cfg, 1)) return e;
    apply_defaults(c);
    set_sizes(c, &c->cfg, 1);
    c->graphs_on = false;
    return nullptr;
}

const char* wq::hip_err(hipError_t e) { return hipGetErrorString(e); }

void wq::set_call_error(const char* m) { set_init_err(m); }

// (this file is compiled without floating-point contraction)
bool wq::node_in_disc_host(double L, double h, int a, int b, double x0, double y0, double r) {
    const double rx = (-L + a * h) - x0, ry = (-L + b * h) - y0;
    return rx * rx + ry * ry <= r * r;
}

extern "C" {

wandqs_status wandqs_workspace_bytes(const wandqs_config* cfg, int32_t n_slices, size_t* bytes) {
    const char* e = check_config(cfg, n_slices);
    if (e || !bytes) {
        set_init_err(e ? e : "bytes is NULL");
        return WANDQS_E_INVALID;
    }
    wandqs_ctx tmp;
    tmp.cfg = *cfg;
    set_sizes(&tmp, cfg, n_slices);
    *bytes = wq::carve(&tmp, nullptr);
    return WANDQS_OK;
}

wandqs_status wandqs_init(const wandqs_config* cfg, int32_t n_slices, void* d_workspace,
                          size_t bytes, void* hip_stream, wandqs_ctx** out) {
    if (!out) {
        set_init_err("out is NULL");
        return WANDQS_E_INVALID;
    }
    *out = nullptr;
    const char* e = check_config(cfg, n_slices);
    if (e) {
        set_init_err(e);
        return WANDQS_E_INVALID;
    }
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) {
        set_init_err("workspace must be a 256-byte aligned device pointer");
        return WANDQS_E_INVALID;
    }
    wandqs_ctx* c = new (std::nothrow) wandqs_ctx();
    if (!c) {
        set_init_err("out of host memory");
        return WANDQS_E_NOMEM;
    }
    c->cfg = *cfg;
    apply_defaults(c);
    c->beams.assign(cfg->beams, cfg->beams + cfg->n_beams);
    c->probes.assign(cfg->probes, cfg->probes + cfg->n_probes);
    c->cfg.beams = nullptr;
    c->cfg.probes = nullptr;
    for (auto& b : c->beams) {
        if (b.kind == WANDQS_BEAM_RADIAL_BINS) c->bin_amp.emplace_back(b.bin_amp, b.bin_amp + b.n_bins);
        else c->bin_amp.emplace_back();
        b.bin_amp = nullptr;
    }
    c->stream = (hipStream_t)hip_stream;
    set_sizes(c, cfg, n_slices);
    const size_t need = wq::carve(c, nullptr);
    if (bytes < need) {
        set_init_err(("workspace too small: need " + std::to_string(need) + " bytes").c_str());
        delete c;
        return WANDQS_E_NOMEM;
    }
    wq::carve(c, (char*)d_workspace);

    auto bail = [&](const std::string& msg) {
        set_init_err(msg.c_str());
        if (c->h_pin) (void)hipHostFree(c->h_pin);
        delete c;
        return WANDQS_E_HIP;
    };
    // coherent: the kernels publish residual norms into it (mg_solve)
    // (+ 8: flags and sequence word; + 8: the laser solve's norms; + 8: the
    // non-uniform solve's)
    if (hipHostMalloc((void**)&c->h_pin, sizeof(double) * (wq::kMaxSlots * wq::kNormVec + 24),
                      hipHostMallocCoherent) != hipSuccess)
        return bail("hipHostMalloc failed");
    std::memset(c->h_pin, 0, sizeof(double) * (wq::kMaxSlots * wq::kNormVec + 24));
    if (hipMemsetAsync(d_workspace, 0, need, c->stream) != hipSuccess)
        return bail("hipMemsetAsync of the workspace failed");

    // beams: device copy of the bin amplitudes and the by-value descriptor
    wq::BeamSet& B = c->beamset;
    B.n = (int)c->beams.size();
    size_t boff = 0;
    std::vector<double> bins_host;
    for (int k = 0; k < B.n; ++k) {
        const wandqs_beam& b = c->beams[k];
        B.kind[k] = b.kind;
        B.amp[k] = b.amp;
        B.sr[k] = b.sigma_r;
        B.sz[k] = b.sigma_z;
        B.xc[k] = b.xi_c;
        B.x0[k] = b.x0;
        B.y0[k] = b.y0;
        B.rmax[k] = b.r_max;
        B.nbins[k] = b.n_bins;
        B.bins[k] = nullptr;
        if (b.kind == WANDQS_BEAM_RADIAL_BINS) {
            B.bins[k] = c->bins_dev + boff;
            bins_host.insert(bins_host.end(), c->bin_amp[k].begin(), c->bin_amp[k].end());
            boff += b.n_bins;
        }
    }

    // radial-bin node maps: the bin of node (x_a, y_b) is floor(r / (r_max / n_bins))
    // for r = |(x_a, y_b) - (x0, y0)| < r_max, decided once here for the forward
    // density and for the adjoint's sums over bins
    const size_t nnd = (size_t)(c->N + 1) * (c->N + 1);
    std::vector<int32_t> bmap(nnd * (size_t)c->n_bin_beams, -1);
    {
        int q = 0;
        for (int k = 0; k < B.n; ++k) {
            B.bmap[k] = nullptr;
            const wandqs_beam& b = c->beams[k];
            if (b.kind != WANDQS_BEAM_RADIAL_BINS) continue;
            int32_t* m = bmap.data() + (size_t)q * nnd;
            const double dr = b.r_max / b.n_bins;
            for (int jb = 0; jb <= c->N; ++jb)
                for (int ja = 0; ja <= c->N; ++ja) {
                    const double rx = (-c->L + ja * c->h) - b.x0, ry = (-c->L + jb * c->h) - b.y0;
                    const double r = std::sqrt(rx * rx + ry * ry);
                    const int kb = (int)std::floor(r / dr);
                    m[(size_t)jb * (c->N + 1) + ja] = (r < b.r_max && kb < b.n_bins) ? kb : -1;
                }
            B.bmap[k] = c->bin_map + (size_t)q * nnd;
            ++q;
        }
    }
    // adjoint: segments of the sums over nodes behind dL/dtheta (theta in beam
    // order; a Gaussian beam's amplitude sums over all nodes, a bin's amplitude
    // over the nodes of its bin)
    std::vector<int32_t> seg, seg_first, bin_nodes;
    if (c->tape_K > 0) {
        int t = 0, q = 0;
        auto add = [&](int k, int i0, int i1) {
            for (int i = i0; i < i1; i += wq::kThetaSeg) {
                const int e = std::min(i1, i + wq::kThetaSeg);
                seg.insert(seg.end(), {k, t, i, e});
            }
        };
        for (int k = 0; k < B.n; ++k) {
            const wandqs_beam& b = c->beams[k];
            if (b.kind == WANDQS_BEAM_GAUSS) {
                seg_first.push_back((int32_t)(seg.size() / 4));
                add(k, 0, (int)nnd);
                ++t;
                continue;
            }
            const int32_t* m = bmap.data() + (size_t)q * nnd;
            std::vector<std::vector<int32_t>> by(b.n_bins);
            for (size_t i = 0; i < nnd; ++i)
                if (m[i] >= 0) by[m[i]].push_back((int32_t)i);
            for (int j = 0; j < b.n_bins; ++j) {
                seg_first.push_back((int32_t)(seg.size() / 4));
                const int off = (int)bin_nodes.size();
                bin_nodes.insert(bin_nodes.end(), by[j].begin(), by[j].end());
                add(k, off, (int)bin_nodes.size());
                ++t;
            }
            ++q;
        }
        seg_first.push_back((int32_t)(seg.size() / 4));
        c->n_seg = (int)(seg.size() / 4);
        if (c->n_seg > c->n_seg_cap) return bail("internal: theta segment table overflow");
    }
    c->probe_count.clear();
    for (const auto& p : c->probes) {
        double n = 0.0;
        for (int jb = 0; jb <= c->N; ++jb)
            for (int ja = 0; ja <= c->N; ++ja)
                n += wq::node_in_disc_host(c->L, c->h, ja, jb, p.x0, p.y0, p.r_max) ? 1.0 : 0.0;
        c->probe_count.push_back(n);
    }

    // cold plasma at rest on the jittered lattice (same generator and draw order
    // as the test-side input module)
    const int N = c->N, s = cfg->ppc_side;
    const double L = c->L, h = c->h, J = cfg->jitter;
    std::vector<double> host((size_t)c->P * 2);
    std::vector<int32_t> ids((size_t)c->P);
    size_t i = 0;
    for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a)
            for (int sy = 0; sy < s; ++sy)
                for (int sx = 0; sx < s; ++sx, ++i) {
                    const double ux = unit(splitmix64(cfg->seed, 2 * i));
                    const double uy = unit(splitmix64(cfg->seed, 2 * i + 1));
                    host[i] = -L + h * (((double)a + ((double)sx + 0.5) / s) + J * (2.0 * ux - 1.0));
                    host[c->P + i] = -L + h * (((double)b + ((double)sy + 0.5) / s) + J * (2.0 * uy - 1.0));
                    ids[i] = (int32_t)i;
                }
    const double st0[6] = {0.0, cfg->dxi0, 0.0, 0.0, 0.0, 0.0};
    bool ok = wq::make_dst_tables(c) == WANDQS_OK &&
              hipMemcpyAsync(c->pa[0][0], host.data(), sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
              hipMemcpyAsync(c->pa[0][1], host.data() + c->P, sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
              hipMemcpyAsync(c->pid[0], ids.data(), sizeof(int32_t) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
              (!c->lat[0] || (hipMemcpyAsync(c->lat[0], host.data(), sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                              hipMemcpyAsync(c->lat[1], host.data() + c->P, sizeof(double) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess &&
                              hipMemcpyAsync(c->lat_id, ids.data(), sizeof(int32_t) * c->P, hipMemcpyHostToDevice, c->stream) == hipSuccess)) &&
              hipMemcpyAsync(c->st, st0, sizeof(st0), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
              (bins_host.empty() || hipMemcpyAsync(c->bins_dev, bins_host.data(), sizeof(double) * bins_host.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
              (bmap.empty() || hipMemcpyAsync(c->bin_map, bmap.data(), sizeof(int32_t) * bmap.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
              (seg.empty() || hipMemcpyAsync(c->adj.seg, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
              (seg_first.empty() || hipMemcpyAsync(c->adj.seg_first, seg_first.data(), sizeof(int32_t) * seg_first.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
              (bin_nodes.empty() || hipMemcpyAsync(c->adj.bin_nodes, bin_nodes.data(), sizeof(int32_t) * bin_nodes.size(), hipMemcpyHostToDevice, c->stream) == hipSuccess) &&
              hipStreamSynchronize(c->stream) == hipSuccess;
    if (!ok) return bail("copying the initial state failed");
    c->cur = 0;
    *out = c;
    return WANDQS_OK;
}

wandqs_status wandqs_slice_step(wandqs_ctx* c, double* d_fields_out, wandqs_slice_info* h_info) {
    if (!c) return WANDQS_E_INVALID;
    if (c->failed) {
        c->err = "context failed earlier; call wandqs_set_state";
        return WANDQS_E_STATE;
    }
    wandqs_status s = do_slice(c, 0, -1, true, nullptr);
    if (s != WANDQS_OK) return fail(c, s);
    if (d_fields_out && (s = wq::pack_fields(c, c->fields, 5, d_fields_out)) != WANDQS_OK)
        return fail(c, s);
    if (h_info) {
        double r[4];
        if (hipMemcpyAsync(r, c->rec, sizeof(r), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            c->err = "reading the slice record failed";
            return fail(c, WANDQS_E_HIP);
        }
        h_info->xi = r[0];
        h_info->dxi = r[1];
        h_info->vmax = r[2];
        h_info->flags = (int32_t)r[3];
        fill_info_host(c, h_info);
        if (h_info->flags & 1) {
            c->err = "1 + psi <= 0 where plasma is present";
            return fail(c, WANDQS_E_NONPHYS);
        }
    }
    return WANDQS_OK;
}

wandqs_status wandqs_run(wandqs_ctx* c, int32_t n_slices, double* d_probe_out,
                         wandqs_slice_info* h_infos) {
    if (!c || n_slices < 0) return WANDQS_E_INVALID;
    if (c->failed) {
        c->err = "context failed earlier; call wandqs_set_state";
        return WANDQS_E_STATE;
    }
    wandqs_status s;
    if (!c->probes.empty() && (s = wq::fill_f64(c, c->probe_acc, wq::kMaxProbes, 0.0)) != WANDQS_OK)
        return fail(c, s);
    c->run_begin = c->tape_n;
    c->run_len = -1;
    std::vector<double> rec;
    int32_t chunk0 = 0;
    auto flush = [&](int32_t upto) -> wandqs_status {
        const int32_t n = upto - chunk0;
        if (!h_infos || n <= 0) return WANDQS_OK;
        rec.resize((size_t)4 * n);
        WQ_HIP(hipMemcpyAsync(rec.data(), c->rec, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
        WQ_HIP(hipStreamSynchronize(c->stream));
        for (int32_t j = 0; j < n; ++j) {
            h_infos[chunk0 + j].xi = rec[4 * j];
            h_infos[chunk0 + j].dxi = rec[4 * j + 1];
            h_infos[chunk0 + j].vmax = rec[4 * j + 2];
            h_infos[chunk0 + j].flags = (int32_t)rec[4 * j + 3];
        }
        chunk0 = upto;
        return WANDQS_OK;
    };
    for (int32_t j = 0; j < n_slices; ++j) {
        if (j - chunk0 == c->rec_cap && (s = flush(j)) != WANDQS_OK) return fail(c, s);
        if ((s = do_slice(c, j - chunk0, j, true, nullptr)) != WANDQS_OK) {
            flush(j);
            return fail(c, s);
        }
        if (h_infos) fill_info_host(c, &h_infos[j]);
    }
    if ((s = flush(n_slices)) != WANDQS_OK) return fail(c, s);
    if (d_probe_out && !c->probes.empty()) {
        if (hipMemcpyAsync(d_probe_out, c->probe_acc, sizeof(double) * c->probes.size(),
                           hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
            c->err = "copying the probes failed";
            return fail(c, WANDQS_E_HIP);
        }
    }
    if ((s = check_flags(c)) != WANDQS_OK) return fail(c, s);
    c->run_len = n_slices;
    return WANDQS_OK;
}

wandqs_status wandqs_get_state(wandqs_ctx* c, double* d_particles, double* d_fields,
                               double* h_xi_dxi) {
    if (!c) return WANDQS_E_INVALID;
    wandqs_status s;
    if (d_particles && (s = wq::particles_to_id_order(c, d_particles)) != WANDQS_OK) return fail(c, s);
    if (d_fields && (s = wq::pack_fields(c, c->fields, 5, d_fields)) != WANDQS_OK) return fail(c, s);
    if (h_xi_dxi) {
        WQ_HIP(hipMemcpyAsync(h_xi_dxi, c->st, sizeof(double) * 2, hipMemcpyDeviceToHost, c->stream));
        WQ_HIP(hipStreamSynchronize(c->stream));
    }
    return WANDQS_OK;
}

wandqs_status wandqs_set_state(wandqs_ctx* c, const double* d_particles, const double* d_fields,
                               const double* h_xi_dxi) {
    if (!c) return WANDQS_E_INVALID;
    if (h_xi_dxi && (!std::isfinite(h_xi_dxi[0]) || !(h_xi_dxi[1] > 0.0))) {
        c->err = "xi must be finite and dxi > 0";
        return WANDQS_E_INVALID;
    }
    wandqs_status s;
    if (d_particles && (s = wq::particles_from_id_order(c, d_particles)) != WANDQS_OK) return fail(c, s);
    if (d_fields && (s = wq::unpack_fields(c, d_fields, 5, c->fields)) != WANDQS_OK) return fail(c, s);
    if (h_xi_dxi) WQ_HIP(hipMemcpyAsync(c->st, h_xi_dxi, sizeof(double) * 2, hipMemcpyHostToDevice, c->stream));
    WQ_HIP(hipMemsetAsync(c->flags, 0, sizeof(int32_t), c->stream));
    WQ_HIP(hipStreamSynchronize(c->stream));
    c->failed = false;
    c->n_guess = 0;
    c->tape_n = 0;  // the tape restarts from this state
    c->tape_ok = true;
    c->run_len = -1;
    return WANDQS_OK;
}

wandqs_status wandqs_driver_set(wandqs_ctx* c, int64_t n, const double* d_state) {
    if (!c) return WANDQS_E_INVALID;
    if (c->cfg.driver_max <= 0) {
        c->err = "no room for driver particles: initialise with driver_max > 0";
        return WANDQS_E_INVALID;
    }
    if (n < 0 || n > c->cfg.driver_max || (n > 0 && !d_state)) {
        c->err = "driver particle count must be in [0, driver_max] with a state array";
        return WANDQS_E_INVALID;
    }
    const size_t D = (size_t)c->cfg.driver_max;
    wandqs_status s;
    for (int q = 0; q < 8 && n > 0; ++q)
        if ((s = wq::copy_d2d(c, c->drv + q * D, d_state + (size_t)q * n, sizeof(double) * n)) != WANDQS_OK)
            return fail(c, s);
    c->drv_n = n;
    return WANDQS_OK;
}

wandqs_status wandqs_driver_get(wandqs_ctx* c, double* d_state) {
    if (!c || (c->drv_n > 0 && !d_state)) return WANDQS_E_INVALID;
    const size_t D = (size_t)c->cfg.driver_max, n = (size_t)c->drv_n;
    wandqs_status s;
    for (int q = 0; q < 8 && n > 0; ++q)
        if ((s = wq::copy_d2d(c, d_state + q * n, c->drv + q * D, sizeof(double) * n)) != WANDQS_OK)
            return fail(c, s);
    return WANDQS_OK;
}

wandqs_status wandqs_time_step(wandqs_ctx* c, double dt, int32_t n_slices, wandqs_slice_info* h_infos) {
    using namespace wq;
    if (!c || n_slices < 1 || !std::isfinite(dt)) return WANDQS_E_INVALID;
    if (c->cfg.driver_max <= 0 && c->cfg.laser_nz <= 0) {
        c->err = "no time loop: initialise with driver_max > 0 or laser_nz > 0";
        return WANDQS_E_INVALID;
    }
    if (c->las_on && (c->cfg.adaptive || n_slices < c->cfg.laser_nz || !(dt > 0.0))) {
        c->err = "a time step with a laser envelope needs fixed steps (adaptive = 0, so that "
                 "slice j lies on plane j), n_slices >= laser_nz and dt > 0";
        return WANDQS_E_INVALID;
    }
    if (c->failed) {
        c->err = "context failed earlier; call wandqs_set_state";
        return WANDQS_E_STATE;
    }
    // the plasma ahead of the drivers is the cold plasma at rest: every time
    // step sweeps it from xi = 0 with zero fields
    wandqs_status s;
    const size_t P = (size_t)c->P, nb = (size_t)(c->N + 1) * c->lev[0].pitch;
    const int k = c->cur;
    if ((s = copy_d2d(c, c->pa[k][0], c->lat[0], sizeof(double) * P)) != WANDQS_OK ||
        (s = copy_d2d(c, c->pa[k][1], c->lat[1], sizeof(double) * P)) != WANDQS_OK ||
        (s = copy_d2d(c, c->pid[k], c->lat_id, sizeof(int32_t) * P)) != WANDQS_OK ||
        (s = fill_f64(c, c->pa[k][2], P, 0.0)) != WANDQS_OK ||
        (s = fill_f64(c, c->pa[k][3], P, 0.0)) != WANDQS_OK)
        return fail(c, s);
    for (int q = 0; q < 5; ++q) {
        double* arrs[4] = {c->fields[q], c->fields_prev[q], c->fields_prev2[q], c->fields_prev3[q]};
        for (double* a : arrs)
            if (a && (s = fill_f64(c, a, nb, 0.0)) != WANDQS_OK) return fail(c, s);
    }
    const bool drv = c->cfg.driver_max > 0;
    if ((s = fill_f64(c, c->st, 16, 0.0)) != WANDQS_OK || (s = fill_f64(c, c->st + 1, 1, c->cfg.dxi0)) != WANDQS_OK ||
        (drv && (s = driver_deposit(c)) != WANDQS_OK) ||
        (drv && (s = fill_f64(c, c->drv_eb, 6 * (size_t)c->cfg.driver_max, 0.0)) != WANDQS_OK))
        return fail(c, s);
    WQ_HIP(hipMemsetAsync(c->flags, 0, sizeof(int32_t), c->stream));
    c->n_guess = 0;
    c->tape_n = 0;
    c->drv_active = drv;
    c->drv_dt = dt;
    c->las_adv = c->las_on;
    c->las_dt = dt;
    c->las_j = 0;
    s = wandqs_run(c, n_slices, nullptr, h_infos);
    c->drv_active = false;
    c->las_adv = false;
    if (s != WANDQS_OK) return s;
    // the driver push takes the laser's fields from the planes at t and t + dt
    if (drv && (s = driver_push(c, dt)) != WANDQS_OK) return fail(c, s);
    if (c->las_on) c->las_cur = 1 - c->las_cur;  // the planes at t + dt
    return WANDQS_OK;
}

wandqs_status wandqs_laser_set(wandqs_ctx* c, const double* d_env) {
    if (!c) return WANDQS_E_INVALID;
    if (c->cfg.laser_nz <= 0) {
        c->err = "no room for a laser envelope: initialise with laser_nz > 0";
        return WANDQS_E_INVALID;
    }
    if (!d_env) {
        c->las_on = false;
        return WANDQS_OK;
    }
    wandqs_status s;
    if ((s = wq::laser_unpack(c, d_env, c->las_cur)) != WANDQS_OK) return fail(c, s);
    c->las_on = true;
    return WANDQS_OK;
}

wandqs_status wandqs_laser_get(wandqs_ctx* c, double* d_env) {
    if (!c || !d_env) return WANDQS_E_INVALID;
    if (!c->las_on) {
        c->err = "no laser envelope set";
        return WANDQS_E_STATE;
    }
    wandqs_status s;
    if ((s = wq::laser_pack(c, d_env)) != WANDQS_OK) return fail(c, s);
    return WANDQS_OK;
}

wandqs_status wandqs_laser_advance(wandqs_ctx* c, double dt, const double* d_chi, int32_t* h_cycles) {
    if (!c || !(dt > 0.0) || !std::isfinite(dt)) return WANDQS_E_INVALID;
    if (!c->las_on) {
        c->err = "no laser envelope set";
        return WANDQS_E_STATE;
    }
    const size_t dense = (size_t)(c->N + 1) * (c->N + 1);
    wandqs_status s;
    for (int j = 0; j < c->cfg.laser_nz; ++j) {
        double* k2 = c->lev[0].k2;
        if (d_chi && (s = wq::unpack_fields(c, d_chi + j * dense, 1, &k2)) != WANDQS_OK) return fail(c, s);
        int cyc = 0;
        s = wq::laser_plane_advance(c, dt, d_chi ? k2 : nullptr, j, &cyc);
        if (h_cycles) h_cycles[j] = cyc;
        if (s != WANDQS_OK) return s;
    }
    c->las_cur = 1 - c->las_cur;
    return WANDQS_OK;
}

wandqs_status wandqs_mg_solve(wandqs_ctx* c, int32_t nrhs, const double* d_k2, const double* d_f,
                              double* d_u, int32_t* h_cycles, double* h_rel) {
    if (!c || (nrhs != 1 && nrhs != 2) || !d_f || !d_u) return WANDQS_E_INVALID;
    wandqs_status s;
    wq::Level& L0 = c->lev[0];
    if ((s = wq::unpack_fields(c, d_f, nrhs, L0.f)) != WANDQS_OK) return fail(c, s);
    if ((s = wq::unpack_fields(c, d_u, nrhs, c->fields)) != WANDQS_OK) return fail(c, s);
    if (d_k2 && (s = wq::unpack_fields(c, d_k2, 1, &L0.k2)) != WANDQS_OK) return fail(c, s);
    wq::SolveResult res;
    double* u[2] = {c->fields[0], nrhs > 1 ? c->fields[1] : nullptr};
    double* f[2] = {L0.f[0], nrhs > 1 ? L0.f[1] : nullptr};
    c->n_guess = 0;  // the stored fields no longer belong to the slice sequence
    c->tape_ok = false;
    s = wq::mg_solve(c, 3, nrhs, d_k2 != nullptr, u, f, d_k2 ? L0.k2 : nullptr, &res);
    if (s != WANDQS_OK && s != WANDQS_E_NOCONV) return fail(c, s);
    wandqs_status s2 = wq::pack_fields(c, c->fields, nrhs, d_u);
    if (s2 != WANDQS_OK) return fail(c, s2);
    WQ_HIP(hipStreamSynchronize(c->stream));
    if (h_cycles) *h_cycles = res.cycles;
    if (h_rel)
        for (int r = 0; r < nrhs; ++r) h_rel[r] = res.rel[r];
    return s;
}

wandqs_status wandqs_get_moments(wandqs_ctx* c, double* d_out) {
    if (!c || !d_out) return WANDQS_E_INVALID;
    double* src[9] = {c->mom[0], c->mom[1], c->mom[2], c->mom[3], c->mom[4], c->mom[5],
                      c->lev[0].k2, c->lev[0].f[0], c->lev[0].f[1]};
    wandqs_status s = wq::pack_fields(c, src, 9, d_out);
    return s == WANDQS_OK ? s : fail(c, s);
}

int64_t wandqs_num_particles(const wandqs_ctx* c) { return c ? c->P : 0; }

int32_t wandqs_num_theta(const wandqs_ctx* c) { return c ? c->n_theta : 0; }

int64_t wandqs_tape_slices(const wandqs_ctx* c) {
    return c && c->tape_K > 0 && c->tape_ok ? c->tape_n : -1;
}

wandqs_status wandqs_backward(wandqs_ctx* c, const double* h_dL_dprobe, const double* d_dL_dfields,
                              const double* d_dL_dparticles, double* h_dL_dtheta,
                              double* d_dL_dparticles0) {
    using namespace wq;
    if (!c) return WANDQS_E_INVALID;
    if (c->tape_K <= 0) {
        c->err = "no adjoint tape: initialise with checkpoint_every > 0";
        return WANDQS_E_STATE;
    }
    if (c->failed) {
        c->err = "context failed earlier; call wandqs_set_state";
        return WANDQS_E_STATE;
    }
    if (!c->tape_ok) {
        c->err = "the tape is incomplete (more slices than given at init, or wandqs_mg_solve "
                 "replaced the fields); call wandqs_set_state";
        return WANDQS_E_STATE;
    }
    if (h_dL_dprobe && !c->probes.empty() && c->run_len < 0) {
        c->err = "probe adjoints given but no wandqs_run completed since the tape start";
        return WANDQS_E_STATE;
    }
    const int64_t S = c->tape_n, K = c->tape_K;
    const size_t P = (size_t)c->P, nnd = (size_t)(c->N + 1) * (c->N + 1);
    if (S > c->rec_cap || (S > 0 && (S - 1) / K >= c->n_ckpt - 1) ||
        (int64_t)c->slot.size() < std::min(S, K)) {
        c->err = "internal: tape larger than its buffers";
        return WANDQS_E_STATE;
    }
    wandqs_status s;
    Checkpoint& fin = c->ckpt[c->n_ckpt - 1];
    if ((s = save_checkpoint(c, fin)) != WANDQS_OK) return fail(c, s);
    if ((s = adj_zero_solutions(c)) != WANDQS_OK) return fail(c, s);
    if (d_dL_dparticles)
        s = copy_d2d(c, c->adj.adj_id, d_dL_dparticles, sizeof(double) * 4 * P);
    else
        s = fill_f64(c, c->adj.adj_id, 4 * P, 0.0);
    if (s != WANDQS_OK) return fail(c, s);

    std::vector<double> w(c->probes.size());
    for (int64_t seg = (S + K - 1) / K - 1; seg >= 0; --seg) {
        const int64_t j0 = seg * K, j1 = std::min(S, j0 + K);
        if ((s = restore_checkpoint(c, c->ckpt[seg])) != WANDQS_OK) return fail(c, s);
        for (int64_t j = j0; j < j1; ++j)
            if ((s = do_slice(c, -1, -1, false, &c->slot[j - j0])) != WANDQS_OK) return fail(c, s);
        for (int64_t j = j1 - 1; j >= j0; --j) {
            // probe seeds: d(probe k)/d(field node) = 1 / (nodes in the disc * slices in the window)
            bool any = false;
            for (size_t k = 0; k < c->probes.size(); ++k) {
                const wandqs_probe& p = c->probes[k];
                const int64_t r = j - c->run_begin;
                w[k] = 0.0;
                if (h_dL_dprobe && c->run_len >= 0 && r >= 0 && r < c->run_len && r >= p.slice_begin &&
                    r < p.slice_end && c->probe_count[k] > 0) {
                    w[k] = h_dL_dprobe[k] / c->probe_count[k] / (double)(p.slice_end - p.slice_begin);
                    any = true;
                }
            }
            const double* fb = d_dL_dfields ? d_dL_dfields + (size_t)j * 5 * nnd : nullptr;
            if ((s = slice_adjoint(c, c->slot[j - j0], fb, any ? w.data() : nullptr)) != WANDQS_OK)
                return fail(c, s);
        }
    }
    if (d_dL_dparticles0 &&
        (s = copy_d2d(c, d_dL_dparticles0, c->adj.adj_id, sizeof(double) * 4 * P)) != WANDQS_OK)
        return fail(c, s);
    if ((s = restore_checkpoint(c, fin)) != WANDQS_OK) return fail(c, s);
    if (h_dL_dtheta && c->n_theta > 0)
        WQ_HIP(hipMemcpyAsync(h_dL_dtheta, c->adj.theta_bar, sizeof(double) * c->n_theta,
                              hipMemcpyDeviceToHost, c->stream));
    WQ_HIP(hipStreamSynchronize(c->stream));
    return WANDQS_OK;
}

void wandqs_destroy(wandqs_ctx* c) {
    if (!c) return;
    wq::prof_reset(c, false);
    for (const wq::CycleGraph& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    delete c;
}

const char* wandqs_last_error(const wandqs_ctx* c) {
    return c ? c->err.c_str() : g_init_err;
}

}  // extern "C"
