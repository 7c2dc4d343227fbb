/*
 * wandqs -- quasi-static xi-slice step of plasma electrons on one MI355X (gfx950).
 *
 * The library advances the plasma electrons of a quasi-static particle-in-cell
 * model through xi-slices behind a frozen, luminal driver beam, following
 * T. Wang et al., "WAND-PIC: an accelerated three-dimensional quasi-static
 * particle-in-cell code" (arXiv 2012.00881):
 *   Collect_Source   deposit n*, j_perp = n*<V> and T = n*<V V>     (Sec. III.B, eqs. (8)-(9), (16))
 *   Solve_Wakefield  psi, Ez, Bz by Poisson solves (eqs. (12)-(14)) and B_perp by the
 *                    explicit Helmholtz system (eqs. (18)-(19)), geometric multigrid
 *   Push_Trajectory  gather and Boris-like push of (r_perp, p_perp) (Sec. III.A, eqs. (6)-(7))
 *   Step_Size_Refinement  adaptive dxi (Algorithm 1, with the floor dxi0/k of Sec. V.A)
 *
 * Units are the paper's (Sec. III): lengths 1/k_p, densities n0, momenta mc,
 * fields mc omega_p/e, currents -e n0 c.  Transverse grid: N cells per side on
 * [-L, L]^2, vertex centred, nodes x_a = -L + a h, h = 2L/N, a = 0..N; all five
 * fields vanish on the boundary nodes.  Node arrays passed across this
 * interface are dense row-major [N+1][N+1] float64 with x fastest
 * (element b*(N+1)+a is node (x_a, y_b)); field order is psi, Ez, Bz, Bx, By.
 *
 * Conventions
 *  - Ownership: the caller owns all device memory (the workspace, inputs and
 *    outputs) and the HIP stream.  The library never allocates device memory;
 *    it allocates a few hundred bytes of pinned host memory per context.
 *    "d_" pointers are device pointers, "h_" pointers host pointers.
 *  - Streams: every call enqueues its work on the stream given to wandqs_init
 *    and returns when that work is enqueued, except where noted (calls that
 *    fill a host output synchronise the stream).
 *  - Errors: every call returns a status; on any error other than
 *    WANDQS_E_INVALID raised by argument checks, the context is marked failed
 *    and further steps return WANDQS_E_STATE until wandqs_set_state.
 *    wandqs_last_error gives a text message.
 *  - Threads: a context is used by one host thread at a time.
 */
#ifndef WANDQS_H
#define WANDQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wandqs_ctx wandqs_ctx;

typedef enum {
    WANDQS_OK = 0,
    WANDQS_E_INVALID = -1, /* bad argument or configuration (context unchanged) */
    WANDQS_E_NOMEM = -2,   /* workspace smaller than wandqs_workspace_bytes */
    WANDQS_E_HIP = -3,     /* a HIP runtime call failed */
    WANDQS_E_NOCONV = -4,  /* a multigrid solve did not converge in mg_max_cycles */
    WANDQS_E_NONPHYS = -5, /* 1 + psi <= 0 where plasma is present (never clamped) */
    WANDQS_E_STATE = -6    /* context failed earlier, or no state for the request */
} wandqs_status;

typedef enum { WANDQS_FP64 = 0, WANDQS_MIXED = 1 } wandqs_precision;
typedef enum { WANDQS_BEAM_GAUSS = 0, WANDQS_BEAM_RADIAL_BINS = 1 } wandqs_beam_kind;

/* Plasma pushers (Sec. VII.A: a Boris-like pusher, with first-, second- and
 * fourth-order Runge-Kutta as alternatives).  All advance (r_perp, p_perp) over
 * dxi with the fields frozen at the slice (eqs. (6)-(7)).  BORIS: half kick by
 * gamma grad psi/g + e_z x B_perp with gamma from the old momentum, rotation for
 * (e_z x V) B_z through angle 2 atan(B_z dxi / 2g), half kick, drift with the new
 * momentum and g at the start.  RK1 / RK2 / RK4: forward Euler, the midpoint
 * rule and the classical four-stage scheme on dr/dxi = p/g, dp/dxi = the force
 * above, each stage gathering psi (hence g), grad psi and B at its own
 * position.  Every pusher reflects the end position at the walls x, y = +-L.
 * The adjoint (wandqs_backward) is that of BORIS only. */
typedef enum {
    WANDQS_PUSH_BORIS = 0,
    WANDQS_PUSH_RK1 = 1,
    WANDQS_PUSH_RK2 = 2,
    WANDQS_PUSH_RK4 = 4
} wandqs_pusher;

/* Frozen luminal driver (Sec. V.A).  It enters only through the longitudinal
 * current j_z of the B_perp source (a luminal beam has rho_b = J_bz, so it drops
 * out of the psi equation).  Density for xi >= 0, zero for xi < 0:
 *   GAUSS:        amp * exp(-r^2/sigma_r^2 - (xi - xi_c)^2/sigma_z^2)
 *   RADIAL_BINS:  bin_amp[floor(r / (r_max/n_bins))] * exp(-(xi - xi_c)^2/sigma_z^2), r < r_max
 * with r measured from (x0, y0).  bin_amp is a host array copied at init. */
typedef struct {
    int32_t kind;
    double amp, sigma_r, sigma_z, xi_c, x0, y0;
    int32_t n_bins;
    double r_max;
    const double* bin_amp;
} wandqs_beam;

/* A probe is the mean of one field over the nodes within r_max of (x0, y0)
 * and over the slices slice_begin <= j < slice_end of a wandqs_run call. */
typedef struct {
    int32_t field; /* 0 psi, 1 Ez, 2 Bz, 3 Bx, 4 By */
    int32_t slice_begin, slice_end;
    double r_max, x0, y0;
} wandqs_probe;

typedef struct {
    int32_t n_cells;     /* N: power of two, 8 .. 4096 */
    double half_width;   /* L > 0 */
    int32_t ppc_side;    /* s = 1..4: s*s macroparticles per cell, weight n0 h^2 / s^2 */
    double jitter;       /* J in cells, 0 <= J <= 0.5/s: uniform displacement of each lattice point */
    uint64_t seed;       /* SplitMix64 seed of the jitter */
    double n0;           /* plasma density and ion background (1 in the paper's units) */
    double dxi0;         /* initial step of Algorithm 1 (> 0) */
    int32_t adaptive;    /* 1: Step_Size_Refinement, 0: fixed dxi0 */
    int32_t refine_k;    /* floor dxi >= dxi0 / k; 0 = no floor */
    int32_t precision;   /* wandqs_precision */
    double mg_rtol;      /* stop when ||r|| <= rtol ||f|| + atol sqrt(n) (n interior nodes;
                            ||r_0|| in place of ||f|| when f = 0) or
                            at the rounding floor: a cycle that no longer halves ||r|| once
                            ||r|| <= 1e-9 max(||f||, ||r_0||); rtol <= 0: exactly
                            mg_max_cycles V-cycles, no host syncs */
    double mg_atol;      /* >= 0; 0 recommended (an absolute floor loosens small fields) */
    int32_t mg_max_cycles; /* 1 .. 200 */
    int32_t nu_pre, nu_post; /* over-relaxed red-black Gauss-Seidel sweeps per V-cycle,
                                each 1 .. 3; the levels two or more below the
                                finest pre-smooth with one sweep */
    int32_t n_beams;       /* 0 .. 8 */
    const wandqs_beam* beams;
    int32_t n_probes;      /* 0 .. 16 */
    const wandqs_probe* probes;
    int32_t checkpoint_every; /* K > 0: keep the adjoint tape (a checkpoint of the
                                 state before every K-th slice since init or
                                 set_state, up to the n_slices given at init, plus
                                 K recompute slots); 0 = no tape */
    int32_t mg_inner_cycles;  /* WANDQS_MIXED: FP32 V-cycles per FP64 defect correction
                                 (0: 1, the fastest measured at C5).  The mixed form keeps the residual, the
                                 correction sum u += e and the coarsest-grid solve (the
                                 exact sine-transform solve of the Poisson V-cycle's last
                                 level; the Helmholtz levels <= 64^2) in FP64 and
                                 smooths/transfers the error equation on the levels
                                 above in FP32; particles stay FP64.  Each "V-cycle" counted in
                                 wandqs_slice_info.vcycles is then one outer iteration. */
    double mg_omega;          /* relaxation factor om of the smoothing sweeps of the
                                 Poisson solves (psi, Ez, Bz): each node of a
                                 half sweep moves to u + om (g - u), g the value that
                                 solves its own equation; 0 < om < 2, 0 selects
                                 1.175.  om = 1 is plain Gauss-Seidel. */
    double mg_omega_helm;     /* the same for the Helmholtz solve (B_perp) on its
                                 levels with h^2 n0 <= 1/8; the coarser ones,
                                 whose diagonal shift h^2 k2 is no longer small,
                                 relax with om = 1; 0 selects 1.175 */
    int32_t adjoint_hold_dxi; /* 1: with adaptive = 1 and a tape (checkpoint_every > 0),
                                 wandqs_backward differentiates the slice map with
                                 the step sequence dxi_j the forward took held
                                 fixed (Step_Size_Refinement is not differentiated:
                                 the gradient is exact only while each step is
                                 dxi0 or its floor dxi0/k, where Vmax does not
                                 enter); 0: such a configuration is rejected
                                 (WANDQS_E_INVALID), since the step then depends on
                                 the state through Vmax.  Ignored without adaptive
                                 steps or without a tape. */
    int32_t pusher;           /* a wandqs_pusher value, 0 = Boris-like; a tape needs BORIS */
    int32_t driver_max;       /* > 0: room for that many driver macroparticles and the
                                 time loop (wandqs_driver_set, wandqs_time_step); 0: none.
                                 Not with a tape. */
    int32_t driver_nz;        /* driver current planes xi_m = driver_xi0 + m driver_dz,   */
    double driver_xi0, driver_dz; /* m = 0 .. driver_nz - 1 (>= 2 planes, dz > 0)          */
    int32_t laser_nz;         /* > 0: room for a laser envelope on laser_nz planes
                                 xi_m = m dxi0 (wandqs_laser_set) and the time loop
                                 that advances it; 0: none.  Not with a tape. */
    double laser_k0;          /* carrier wavenumber k0 = omega0/omega_p (> 0 with a laser) */
    int32_t driver_nsub;      /* sub-steps of the driver push per time step, 0 .. 4096
                                 (0 or 1: one); see wandqs_time_step */
} wandqs_config;

typedef struct {
    double xi;            /* slice position */
    double dxi;           /* step taken from this slice to the next */
    double vmax;          /* max |V_perp| after the push (Algorithm 1) */
    int32_t vcycles[5];   /* V-cycles per field solve (psi, Ez, Bz, Bx, By); -1 if not tracked */
    double rel_resid[5];  /* final ||r||/||f|| per field; -1 if not tracked */
    int32_t flags;        /* bit 0: 1+psi <= 0 met */
    int32_t laser_vcycles; /* multigrid cycles of the envelope plane this slice advanced
                              (time loop with a laser), else 0 */
} wandqs_slice_info;

/* Bytes of device workspace needed for cfg and runs of up to n_slices slices
 * per wandqs_run call (n_slices >= 1; it sizes the per-slice record buffer and,
 * with checkpoint_every = K > 0, the adjoint tape: ceil(n_slices/K) + 1
 * checkpoints of the particles and two field sets, K slots of one slice's
 * particles, fields and moments, and the adjoint work arrays). */
wandqs_status wandqs_workspace_bytes(const wandqs_config* cfg, int32_t n_slices, size_t* bytes);

/* Validate cfg, bind the caller's workspace (d_workspace, >= 256-byte aligned,
 * at least wandqs_workspace_bytes), build the cold plasma at rest on the lattice
 * (Sec. III.A: H = 1, P = 0 before the driver), zero the fields, xi = 0,
 * dxi = dxi0.  hip_stream is a hipStream_t (NULL: the null stream).  Synchronises
 * the stream once.  *out is NULL on error.  Diagnostic: with the environment
 * variable WANDQS_MG_TILES=lds at init, every multigrid level runs the LDS tile
 * kernels instead of the register tiles of the large levels (same results,
 * bit for bit); with WANDQS_GRAPHS=1 at init, each multigrid cycle is captured
 * once as a HIP graph per set of launch arguments and replayed (same kernels,
 * same results; the graphs are freed by wandqs_destroy). */
wandqs_status wandqs_init(const wandqs_config* cfg, int32_t n_slices, void* d_workspace,
                          size_t bytes, void* hip_stream, wandqs_ctx** out);

/* One xi-slice: sort, deposit, five solves, push, step update.  d_fields_out
 * (device [5][N+1][N+1] or NULL) receives the fields of this slice; h_info
 * (host, or NULL) its record (synchronises the stream). */
wandqs_status wandqs_slice_step(wandqs_ctx* ctx, double* d_fields_out, wandqs_slice_info* h_info);

/* n_slices consecutive slices.  d_probe_out (device [n_probes] or NULL)
 * receives the probe means; h_infos (host [n_slices] or NULL) one record per
 * slice.  Records are gathered on the device and copied once per call. */
wandqs_status wandqs_run(wandqs_ctx* ctx, int32_t n_slices, double* d_probe_out,
                         wandqs_slice_info* h_infos);

/* Current state.  d_particles (device [4][P], rows x, y, px, py in particle-ID
 * order, P = N^2 s^2), d_fields (device [5][N+1][N+1]: the last solved fields,
 * used as the next slice's multigrid initial guesses) and h_xi_dxi (host [2])
 * may each be NULL.  h_xi_dxi synchronises the stream. */
wandqs_status wandqs_get_state(wandqs_ctx* ctx, double* d_particles, double* d_fields,
                               double* h_xi_dxi);

/* Replace the state (same layouts; NULL leaves that part unchanged).  Field
 * boundary nodes are set to zero.  Clears a failed context. */
wandqs_status wandqs_set_state(wandqs_ctx* ctx, const double* d_particles,
                               const double* d_fields, const double* h_xi_dxi);

/* The time loop of Algorithm 1 (outer loop over t, Push_Driver; Sec. VII.A,
 * eqs. (25)-(26)), for contexts made with driver_max > 0.
 *
 * wandqs_driver_set copies n (<= driver_max) driver macroparticles, device
 * [8][n] rows x, y, xi (= t - z), p_x, p_y, p_z (momenta in m_e c), q/m (in
 * units of e/m_e: -1 for electrons) and w (the number of particles each
 * stands for, in units of n0 k_p^-3); wandqs_driver_get copies the current
 * ones back (device [8][n]).
 *
 * wandqs_time_step(dt, n_slices): the driver particles deposit their
 * longitudinal current -q/m w v_z (CIC in x, y; linear in xi onto the planes
 * xi_m = driver_xi0 + m driver_dz; particles outside the box or the planes add
 * nothing; a fixed-point sum, so the deposit is deterministic); the plasma
 * restarts as the cold plasma at rest at xi = 0 with zero fields and is swept
 * through n_slices slices (as wandqs_run, the records in h_infos) with that
 * current added to j_z, the planes interpolated linearly in xi at each slice
 * (a near-luminal driver has rho_b = J_bz, so it enters only j_z); each
 * driver particle takes the wake at its mid-step position x + (dt/2) v,
 * xi + (dt/2)(1 - v_z) from the two slices that bracket it (CIC in each,
 * linear in xi; zero ahead of the first slice, at or behind the last and
 * outside the box), with E = (-d_x psi + B_y, -d_y psi - B_x, Ez) and B =
 * (Bx, By, Bz); finally every driver particle advances by dt in driver_nsub
 * sub-steps d = dt / driver_nsub (the sub-cycling of Sec. IV), each a drift of
 * d/2, a kick d/2, the rotation of a Boris push about (q/m) B / gamma, a kick
 * d/2 and a drift d/2, with E, B = that wake plus, with a laser set (see
 * wandqs_laser_set), the laser's fields of eqs. (21)-(24) at the sub-step's mid
 * position and time: x-polarised, from the envelope interpolated linearly in t
 * between the planes at t and t + dt, linearly in xi between planes and
 * bilinearly in x, y, with e = exp(-i k0 xi),
 *   E_x = Re[-(d_t A + d_xi A - i k0 A) e],  B_y = Re[(-d_xi A + i k0 A) e],
 *   E_z = Re[-d_x A e],  B_z = Re[-d_y A e],  E_y = B_x = 0
 * (derivatives of that interpolant; zero outside the box).  The fields and
 * plasma state after the call are those of the last slice.  WANDQS_E_INVALID
 * without driver_max or laser_nz. */
wandqs_status wandqs_driver_set(wandqs_ctx* ctx, int64_t n, const double* d_state);

/* Laser driver (Sec. IV, eq. (20); contexts made with laser_nz > 0).  The
 * complex envelope A-hat of the laser's vector potential (A = A-hat
 * exp(-i k0 xi), normalised to m c / e) lives on the planes xi_m = m dxi0,
 * m = 0 .. laser_nz - 1.
 *
 * wandqs_laser_set copies the planes from device memory, [laser_nz][N+1][N+1]
 * complex numbers as (re, im) pairs of doubles (NULL: the context forgets its
 * laser); wandqs_laser_get copies the current planes back (same layout).
 *
 * With a laser set, every slice takes a2 = |A-hat|^2 at its position (the two
 * planes around xi interpolated linearly; zero outside the planes) and the
 * plasma feels it through the ponderomotive terms of eqs. (6)-(7) (the push:
 * gamma = (1 + p^2 + g^2 + a2/2)/(2g), force -grad(a2/4)/g), eq. (9) (<gamma>
 * and j_z) and eq. (19) (the term -n* grad(a2/4)/g^2 of S).
 *
 * The envelope advances in t by eq. (20) taken centred in t with a backward
 * xi-difference between neighbouring planes, plane after plane from the
 * front: with a0, a1 a plane at t and t + dt and p0, p1 the plane ahead
 * (zero ahead of plane 0), a1 solves the complex Helmholtz problem
 *   L_h a1 - (chi + beta - i gam) a1 = (chi - beta + i gam) a0 - L_h a0 - beta (p1 - p0),
 * beta = 4/(dt dxi0), gam = 4 k0/dt, a1 = 0 on the boundary, by multigrid
 * with the context's mg_* stop rule, from the guess a0; chi = n* / (1 + psi)
 * is the plasma's susceptibility.
 *
 * wandqs_laser_advance(dt, d_chi, h_cycles) advances every plane by dt > 0
 * with chi given on the device as [laser_nz][N+1][N+1] doubles (NULL:
 * vacuum); h_cycles (host [laser_nz] or NULL) receives each plane's V-cycles.
 * In wandqs_time_step (which a laser alone also enables) the plasma sees the
 * planes at t, and each slice j (< laser_nz) advances plane j right after it
 * with its own chi (the k2 of its B_perp system); this needs adaptive = 0 (so
 * that slice j lies on plane j), n_slices >= laser_nz and dt > 0, else
 * WANDQS_E_INVALID.  WANDQS_E_NOCONV if a plane's solve does not converge in
 * mg_max_cycles; WANDQS_E_STATE if no envelope is set. */
wandqs_status wandqs_laser_set(wandqs_ctx* ctx, const double* d_env);
wandqs_status wandqs_laser_get(wandqs_ctx* ctx, double* d_env);
wandqs_status wandqs_laser_advance(wandqs_ctx* ctx, double dt, const double* d_chi,
                                   int32_t* h_cycles);
wandqs_status wandqs_driver_get(wandqs_ctx* ctx, double* d_state);
wandqs_status wandqs_time_step(wandqs_ctx* ctx, double dt, int32_t n_slices,
                               wandqs_slice_info* h_infos);

/* Multigrid solve on the context's grid, the solver of Solve_Wakefield
 * (Sec. II item 4, Sec. VII.A): (L_h - k2) u = f on the interior nodes with
 * u = 0 on the boundary, L_h the 5-point Laplacian of eq. (33).  nrhs = 1 or 2
 * right-hand sides share the operator.  d_k2 (device [N+1][N+1], k2 >= 0) or
 * NULL for Poisson; d_f (device [nrhs][N+1][N+1]); d_u (device, same shape)
 * holds the initial guess and receives the solution.  Uses the context's
 * mg_* settings; h_cycles / h_rel (host, may be NULL) receive the V-cycle count
 * and ||r||/||f|| per rhs.  Clobbers the context's multigrid scratch arrays and
 * the stored fields used as initial guesses. */
wandqs_status wandqs_mg_solve(wandqs_ctx* ctx, int32_t nrhs, const double* d_k2,
                              const double* d_f, double* d_u, int32_t* h_cycles, double* h_rel);

/* Multigrid solve on a non-uniform transverse grid (Sec. VII.B): lap u + M u =
 * J on the tensor grid of nodes (x_i, y_j), i, j = 0 .. N (N = the context's
 * n_cells), u = 0 on the boundary.  Along x at an interior node, with h- =
 * x_i - x_{i-1}, h+ = x_{i+1} - x_i, ha = h+ + h-, hb = h+ - h-:
 *   Dxx u = 2 (h+ u_{i-1} - ha u_i + h- u_{i+1}) / (h- h+ ha),
 *   dx u  = h-/(ha h+) (u_{i+1} - u_i) + h+/(ha h-) (u_i - u_{i-1}),
 * and the same along y; the discrete equation is L u = R J with the
 * third-order correction of eqs. (34)-(36) (sign from the Taylor expansion,
 * Dxx u = u_xx + (hb/3) u_xxx + O(h^2)):
 *   L u = Dxx u + Dyy u + (1/3)[hb_x dx(Dyy u) + hb_y dy(Dxx u)]
 *         + (1/3)(hb_x dx + hb_y dy)(M u) + M u,
 *   R J = J + (1/3)(hb_x dx + hb_y dy) J,
 * nine-point and not symmetric; on a uniform grid the 5-point Laplacian + M.
 * V-cycles with alternating zebra line relaxation on the levels above 64^2
 * (one step before and one after the coarse correction) and nu_pre / nu_post
 * sweeps of four-colour Gauss-Seidel below, coarse grids with
 * every other node, linear interpolation in the coordinates as prolongation
 * and its control-volume weighted transpose as restriction (for M too);
 * the context's stop rule (mg_rtol, mg_atol, the rounding floor with
 * 2 max |diagonal| as the operator's size; a cycle stagnates only when it
 * gains less than 10% once ||r|| <= 1e-9 ||R J||).
 *   h_x, h_y  host [N+1] each, strictly increasing
 *   d_M       device [N+1][N+1] (row j, column i) or NULL (M = 0)
 *   d_J       device [N+1][N+1]
 *   d_u       device [N+1][N+1]: the initial guess in, the solution out
 *             (its boundary values are taken as zero)
 *   h_cycles, h_rel  host or NULL: V-cycles, final ||r|| / ||R J||
 * Clobbers the context's multigrid scratch arrays and the stored fields used
 * as initial guesses.  WANDQS_E_INVALID for coordinates that do not
 * increase, WANDQS_E_NOCONV after mg_max_cycles. */
wandqs_status wandqs_nu_mg_solve(wandqs_ctx* ctx, const double* h_x, const double* h_y,
                                 const double* d_M, const double* d_J, double* d_u,
                                 int32_t* h_cycles, double* h_rel);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * multigrid solve of wandqs_mg_solve without a context or workspace.  The level
 * hierarchy and every other work array live in one static device array of the
 * library (12 MiB, one copy per GPU, held until the process ends); on its
 * success path the call allocates no device or host memory.
 *   cfg       the grid (n_cells a power of two in [8, 256], half_width), n0,
 *             precision, nu_pre / nu_post, mg_omega / mg_omega_helm, and
 *             mg_max_cycles = the number of V-cycles (FP64) or outer
 *             iterations (mixed) run; mg_rtol must be <= 0 (no tolerance mode:
 *             it would need the host to read norms); beams, probes and the tape
 *             are ignored
 *   nrhs, d_k2, d_f, d_u  as in wandqs_mg_solve (device, dense [N+1][N+1]
 *             per array; d_u holds the guess and receives the result)
 *   hip_stream the hipStream_t the work is enqueued on (NULL: null stream),
 *             on the current device; the call returns once it is enqueued
 * The result equals wandqs_mg_solve's on a context made with the same cfg.
 * Calls on one GPU share its static array: calls that overlap in time on one
 * GPU (on different streams or from different threads) race and give wrong
 * results; each call clears the array before use.  WANDQS_E_INVALID (no work
 * enqueued) for a bad argument, a grid above 256 or mg_rtol > 0; WANDQS_E_HIP
 * if a launch fails.  wandqs_last_error(NULL) gives the message. */
wandqs_status wandqs_mg_solve_noalloc(const wandqs_config* cfg, int32_t nrhs, const double* d_k2,
                                      const double* d_f, double* d_u, void* hip_stream);

/* Diagnostic copy of the node arrays of the last slice (device [9][N+1][N+1]):
 * n*, jx, jy, Txx, Txy, Tyy, k2 = n* / (1+psi), f_Bx, f_By. */
wandqs_status wandqs_get_moments(wandqs_ctx* ctx, double* d_out);

/* Kernel timing for benchmarks and roofline reports.  While enabled, every
 * kernel launch of the context is bracketed by a pair of HIP events on the
 * context's stream; launches are grouped by kernel instantiation (multigrid
 * tile kernels also by grid level, as "name@N").  alg_bytes
 * is the algorithmic DRAM traffic of those launches (each array element the
 * kernel must read or write, counted once). */
typedef struct {
    char name[56];
    int64_t launches;
    double total_ms;
    double alg_bytes;
} wandqs_kernel_stat;

/* enable != 0 starts (and resets) the per-kernel timing; 0 stops it. */
wandqs_status wandqs_profile(wandqs_ctx* ctx, int32_t enable);

/* Copies up to max records (host array) and sets *h_n to the number of
 * kernel groups; synchronises the stream. */
wandqs_status wandqs_profile_stats(wandqs_ctx* ctx, wandqs_kernel_stat* h_out, int32_t max,
                                   int32_t* h_n);

/* Reverse-mode gradient of a loss through every slice run since init or the
 * last wandqs_set_state (discretise-then-differentiate adjoint of the slice map
 * of Sec. III and Algorithm 1; the step dxi is held at its forward values and at
 * cell crossings and wall reflections the branch taken is differentiated).
 * Needs checkpoint_every = K > 0 at init.  Each K-slice segment, last first, is
 * recomputed from its checkpoint (bit-identical to the forward) and then
 * reversed slice by slice; every adjoint elliptic solve is a multigrid solve
 * with the context's mg_* settings.
 *   h_dL_dprobe      host [n_probes] or NULL: dL/d(probe value) of the last
 *                    wandqs_run call (its probes' slice windows are relative to
 *                    that call's first slice)
 *   d_dL_dfields     device [S][5][N+1][N+1] or NULL: dL/d(fields of tape slice
 *                    j) for the S = wandqs_tape_slices slices (boundary entries
 *                    are ignored: the boundary values are fixed)
 *   d_dL_dparticles  device [4][P] or NULL: dL/d(final particles x, y, px, py),
 *                    particle-ID order
 *   h_dL_dtheta      host [wandqs_num_theta] or NULL (out): dL/dtheta, theta =
 *                    for each beam in order its amp (GAUSS) or its bin_amp[]
 *                    (RADIAL_BINS)
 *   d_dL_dparticles0 device [4][P] or NULL (out): dL/d(particles at the tape
 *                    start), particle-ID order
 * The state (particles, fields, xi) is the same after the call as before.
 * Synchronises the stream.  WANDQS_E_STATE without a tape, after
 * wandqs_mg_solve, past the tape capacity (more slices than n_slices at init) or
 * when probe adjoints are given but no wandqs_run has completed. */
wandqs_status wandqs_backward(wandqs_ctx* ctx, const double* h_dL_dprobe,
                              const double* d_dL_dfields, const double* d_dL_dparticles,
                              double* h_dL_dtheta, double* d_dL_dparticles0);

/* Number of driver parameters theta (0 for NULL). */
int32_t wandqs_num_theta(const wandqs_ctx* ctx);

/* Slices on the adjoint tape (-1 without a usable tape). */
int64_t wandqs_tape_slices(const wandqs_ctx* ctx);

/* Number of plasma macroparticles P of the context (0 for NULL). */
int64_t wandqs_num_particles(const wandqs_ctx* ctx);

/* Releases host resources; does not free the caller's workspace.  NULL is a no-op. */
void wandqs_destroy(wandqs_ctx* ctx);

/* Message of the last error of ctx (or of the last failed wandqs_init when ctx is NULL). */
const char* wandqs_last_error(const wandqs_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* WANDQS_H */
