/* ars.h -- C ABI of the MI355X (gfx950) all-regime, well-balanced
 * finite-volume step of Padioleau, Tremblin, Audit, Kestener and Kokh,
 * "A high performance and portable all-Mach regime flow solver code with
 * well-balanced gravity", arXiv 1903.09043.
 *
 * The library advances the compressible Navier-Stokes equations with gravity
 * (Sec. 1, eq. navier_stokes_gravity_nc, ideal gas of Sec. 4) on a uniform
 * Cartesian grid with the explicit scheme of Sec. 2: acoustic / transport
 * splitting with a relaxation Riemann solver (Sec. 2.1.2-2.1.3), the
 * relaxation of the gravitational potential (Sec. 2.1.4) that makes the
 * total energy rho e + rho u^2/2 + rho Phi conservative (eq.
 * conservation_of_energy, eq. all_regime_scheme), the low-Mach correction
 * theta = min(Ma, 1) (eq. low_mach_correction), the well-balanced gravity
 * source (eq. well_balanced_formula) and first-order viscous and heat
 * fluxes (Sec. 2.2).  The multi-dimensional update is unsplit: every face is
 * evaluated from U^n with one time step.
 *
 * Conventions
 *  - All arithmetic is IEEE FP64.  Gravity points along -e_z where z is the
 *    LAST active axis (y in 2D, z in 3D); Phi = g z at cell centres.
 *  - State: caller-owned device array of ars_state_len() doubles, SoA,
 *    variable-major: [rho][m_0]..[m_{D-1}][E], each variable a
 *    contiguous n_0 x n_1 x n_2 array with axis 0 fastest.
 *    E = rho e + rho |u|^2 / 2 (gravity excluded).
 *  - Every device buffer (state, scratch state, workspace, t, dt, schedules,
 *    adjoint fields) is owned by the caller and passed as a raw device
 *    pointer; the library never allocates device memory in the step,
 *    adjoint or batch calls, which are therefore safe to capture in a graph.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *  - A context is not thread-safe; calls on one context must be ordered.
 *  - Every function returns an ars_status; launches are asynchronous and a
 *    numerical fault found by a kernel (rho <= 0, p <= 0, L <= 0 or a
 *    non-finite value) is latched in the workspace and reported by the next
 *    call that synchronises (ars_diagnostics, ars_fault).
 */
#ifndef ARS_H
#define ARS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ARS_OK = 0,
  ARS_EINVAL = -1,        /* bad argument or configuration */
  ARS_ENOMEM = -2,        /* host allocation failed */
  ARS_EDEVICE = -3,       /* HIP runtime / launch error */
  ARS_ENONPHYS = -4,      /* latched numerical fault (see ars_diag.fault_cell) */
  ARS_EUNSUPPORTED = -5,  /* valid configuration this build does not run */
  ARS_ESCRATCH = -6,      /* state larger than the library's static scratch (ars_step_noalloc) */
  ARS_ENOCONV = -7        /* implicit solve of ars_step_imex did not converge */
} ars_status;

enum { ARS_BC_PERIODIC = 0, ARS_BC_WALL = 1, ARS_BC_OUTFLOW = 2 };
enum { ARS_T_ADIABATIC = 0, ARS_T_FIXED = 1 };
enum {
  ARS_PROB_UNIFORM = 0,     /* params: rho, u0, u1, u2, p */
  ARS_PROB_RB = 1,          /* params: T_bottom, T_top, rho of bottom cell (<= 0: its T), amp */
  ARS_PROB_GRESHO = 2,      /* params: Ma                     (Sec. 4.2) */
  ARS_PROB_SOD = 3,         /* no params                       (Sec. 4.1) */
  ARS_PROB_ISOTHERMAL = 4   /* no params: p = rho, T = 1       (Sec. 4.3) */
};

/* Problem description (Sec. 1 closures and Sec. 4 set-ups).
 *  dim        2 or 3 on the GPU (1 is accepted by ars_validate).
 *  n[a], L[a] cells and box length along axis a (unused axes: 1, 1.0).
 *  gamma      ideal-gas adiabatic index (> 1); R = 1 so T = p / rho.
 *  g          gravity magnitude along -z (Phi = g z); 0 allowed.
 *  mu, kappa  constant dynamic viscosity and heat conductivity (>= 0);
 *             Stokes bulk viscosity eta = -2 mu / 3.
 *  K          sub-characteristic factor: a_{i+1/2} = K max(rho_i c_i,
 *             rho_{i+1} c_{i+1}), K >= 1 (the paper only requires >=).
 *  cfl        dt = cfl / max_i lambda_i (see dt_mode).
 *  low_mach   1: theta = min(|u*| / max(c_L, c_R), 1); 0: theta = 1.
 *  dt_mode    0: lambda_i = sum_d (|u_d| + c)/dx_d + 2 D_i sum_d dx_d^-2
 *                with D_i = max(4 mu/3, kappa (gamma-1)) / rho_i;
 *             1: hyperbolic part only;
 *             2: lambda_i = sum_d |u_d|/dx_d + the diffusive part (no sound
 *                speed: the step ars_step_imex allows; ars_step itself is
 *                unstable with it).
 *  bc[a][s]   per axis a, side s (0 low, 1 high): periodic / wall / outflow.
 *             Walls only on the gravity axis; gravity needs walls on it;
 *             periodic must be set on both sides.
 *  wall_noslip 1: ghost velocity -u (no-slip); 0: only the normal component
 *             flips (free slip).
 *  thermal[s], T_wall[s]  bottom / top wall: adiabatic (T_ghost = T) or
 *             fixed temperature (T_ghost = 2 T_wall - T).
 *  energy_form 0: the scheme of eq. all_regime_scheme on the total energy
 *             E + rho Phi with the relaxation of the potential (Sec. 2.1.4);
 *             1: the non-conservative energy scheme of App. B (energy
 *             without the potential, source (uS)_i = (u*_{i+1/2} S_{i+1/2} +
 *             u*_{i-1/2} S_{i-1/2})/2 along the gravity axis, no relaxation
 *             step).  With g = 0 the two coincide.  Every entry point,
 *             the adjoint step included, takes both forms.
 */
typedef struct ars_config {
  int32_t dim;
  int32_t n[3];
  double L[3];
  double gamma, g, mu, kappa, K, cfl;
  int32_t low_mach;
  int32_t dt_mode;
  int32_t bc[3][2];
  int32_t wall_noslip;
  int32_t thermal[2];
  double T_wall[2];
  int32_t energy_form;
  int32_t pad_;
} ars_config;

/* Diagnostics of a state (Sec. 4 reports max velocity, mean absolute
 * velocity, local Mach number and kinetic energy).  Sums are volume
 * integrals (cell volume dV); e_total = sum (E + rho Phi) dV.
 * nu_bot / nu_top: horizontal mean of the wall conductive heat flux over
 * the conductive-profile flux (T_bottom - T_top)/depth (fixed-T walls).
 * fault / fault_cell: the latched numerical fault (1, smallest cell index),
 * cleared by the call that reports it. */
typedef struct ars_diag {
  double mass, mom[3], e_total, e_kin, e_int, e_grav;
  double max_u, mean_u, max_mach, nu_bot, nu_top;
  int64_t fault_cell;
  int32_t fault;
  int32_t pad_;
} ars_diag;

typedef struct ars_ctx ars_ctx;

/* Host-only check of a configuration (no device needed).  ARS_EINVAL for
 * an out-of-range field or more than 2^31 cells (a 1290^3 grid; its state
 * pair takes 172 GB of the 288 GB of one MI355X). */
int ars_validate(const ars_config* cfg);

/* Create / destroy a context (host memory only; no device allocation).
 * Returns ARS_EUNSUPPORTED for dim == 1. */
int ars_create(const ars_config* cfg, ars_ctx** out);
void ars_destroy(ars_ctx* ctx);

/* Number of doubles of one state: (dim + 2) * n_0 * n_1 * n_2. */
size_t ars_state_len(const ars_ctx* ctx);
/* Bytes of the caller-owned workspace every device call takes (256-byte
 * aligned device memory; contents managed by the library). */
size_t ars_workspace_bytes(const ars_ctx* ctx);
/* Prepare a freshly allocated workspace (clears the rate slots and the
 * fault latch).  Call once before its first use.  Asynchronous. */
int ars_workspace_init(ars_ctx* ctx, void* d_work, void* stream);

/* Launch shape of the fused step: number of planes one workgroup marches
 * through along the vertical axis (results do not depend on it).  The
 * default, set by ars_create from the grid: in 3D about 1536 (tile, chunk)
 * shares; in 2D a share of about sqrt(segments x planes) / 13 planes (one
 * plane for small grids, whose step time is the latency of one march). */
int ars_set_zchunk(ars_ctx* ctx, int zchunk);
int ars_get_zchunk(const ars_ctx* ctx);

/* Tile of the 3D fused step: output cells per workgroup in x and y (plus a
 * 2-cell halo on each side), each a compiled kernel; results do not depend
 * on it.  ARS_TILE3_32x10 (36 x 14 positions, the default) or
 * ARS_TILE3_16x20 (20 x 24).  Choosing a tile resets the vertical share
 * to that tile's default.  2D problems have one tile (EUNSUPPORTED for the
 * other). */
enum { ARS_TILE3_32x10 = 0, ARS_TILE3_16x20 = 1 };
int ars_set_tile3(ars_ctx* ctx, int tile);
int ars_get_tile3(const ars_ctx* ctx);

/* Build an initial state (Sec. 4 problems; hydrostatic bases from the
 * discrete equilibrium eq. well_balanced_formula, Sec. 4.3/4.5) on the
 * host and copy it to d_state (synchronous on `stream`).  RB perturbation:
 * p = rho (T + amp (2 U_i - 1)), U_i the i-th SplitMix64 output of `seed`
 * scaled to [0,1) by its top 53 bits, i the linear cell index. */
int ars_init_state(ars_ctx* ctx, int problem, const double* params, int n_params, uint64_t seed,
                   double* d_state, void* stream);
/* Same, into a host array of ars_state_len() doubles (no device use). */
int ars_init_state_host(const ars_ctx* ctx, int problem, const double* params, int n_params, uint64_t seed,
                        double* h_state);

/* Rayleigh-Benard initial state with a caller temperature perturbation
 * (Sec. 4.5 set-up; the base is the discrete hydrostatic equilibrium of eq.
 * well_balanced_formula with the linear temperature T_k of level k, as for
 * ARS_PROB_RB):  rho = rho_k,  m = rho u0,
 *   E = rho (T_k + dT) / (gamma - 1) + |m|^2 / (2 rho)
 * params: T_bottom, T_top, rho of the bottom cell (<= 0: T_bottom), as for
 * ARS_PROB_RB (a fourth value is ignored).  d_dT: device field of
 * ars_state_len()/(dim+2) doubles in the layout of one state variable.
 * d_u0 (nullable): device initial velocity, dim fields in the momentum
 * layout; NULL is rest, and then the state equals ars_init_state with the
 * SplitMix64 perturbation replaced by dT.  Forms the base density column
 * (nz values) on the host, stages it in d_state (the first nz doubles of
 * the x-momentum field, overwritten afterwards) and writes every cell on
 * the device; allocates nothing (synchronous on `stream`).  EINVAL for a
 * configuration without walls on the vertical axis or a NULL pointer. */
int ars_init_rb_dT(ars_ctx* ctx, const double* params, int n_params, const double* d_dT, const double* d_u0,
                   double* d_state, void* stream);
/* Transpose of the map dT -> U^0 of ars_init_rb_dT at the state it built:
 *   d_g_dT = (dU^0/d dT)^T d_lam = d_lam[E] rho / (gamma - 1)  (overwritten)
 * d_state0: that initial state (its density); d_lam: adjoint of U^0 in the
 * state layout.  Asynchronous. */
int ars_init_rb_dT_adjoint(ars_ctx* ctx, const double* d_state0, const double* d_lam, double* d_g_dT,
                           void* stream);

/* dt = cfl / max_i lambda_i of d_state (time-step kernel, Sec. 3.2),
 * written to the device double *d_dt.  Also prepares the workspace for
 * ars_step.  Asynchronous. */
int ars_compute_dt(ars_ctx* ctx, const double* d_state, void* d_work, double* d_dt, void* stream);

/* Advance n_steps explicit steps (eq. all_regime_scheme + dissipative
 * fluxes + relaxation, Sec. 2).  Step s uses dt = cfl / max lambda of its
 * own input state; the first dt is read from *d_dt (as left by
 * ars_compute_dt or a previous ars_step), and on return *d_dt holds the
 * next step's dt and *d_t has been advanced by the sum of the dts used.
 * d_tmp: caller scratch state of the same size.  The result is in d_state.
 * d_dt_log (nullable): receives the dt of every step (n_steps doubles).
 * Asynchronous; numerical faults are latched. */
int ars_step(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, int n_steps, double* d_t, double* d_dt,
             double* d_dt_log, void* stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ars_step
 * without d_tmp and d_work.  Its scratch -- the 256-byte control block
 * (CFL rate slots, fault latch) and the ping-pong state -- is a static
 * device array of the library, one per GPU, held until the process ends:
 * 256 + 8 * ARS_NOALLOC_MAX_STATE bytes (about 1 MiB).  The call allocates
 * nothing.  Returns ARS_ESCRATCH, launching nothing, when
 * ars_state_len(ctx) > ARS_NOALLOC_MAX_STATE (e.g. 2D grids up to 256 x 128
 * fit; larger problems use ars_step).  Results, *d_t, *d_dt and d_dt_log are
 * those of ars_step bit for bit; a numerical fault during the call leaves
 * *d_dt = NaN (no fault cell: ars_step reports it).  Every call on one GPU
 * shares that GPU's scratch and resets it at its start: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller.  Asynchronous. */
#define ARS_NOALLOC_MAX_STATE 131072
int ars_step_noalloc(ars_ctx* ctx, double* d_state, int n_steps, double* d_t, double* d_dt, double* d_dt_log,
                     void* stream);

/* Same with a prescribed per-step dt schedule d_dt_sched[n_steps] (device);
 * used with a frozen schedule by the adjoint and finite-difference checks.
 * *d_t advanced; *d_dt untouched. */
int ars_step_sched(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, int n_steps,
                   const double* d_dt_sched, double* d_t, void* stream);

/* ars_step's n_steps >= 1 steps (CFL dt on the device, *d_dt in and out,
 * optional dt log) out of place, with no copy: step 1 reads d_in (never
 * written), the intermediate states alternate between the scratch states
 * d_a and d_b, and the last step writes d_out; the same argument rules and
 * errors as ars_step_sched_to below (d_dt must not be NULL).  For the
 * forward sweep of a checkpointing schedule, whose stores are then choices
 * of d_out.  Asynchronous. */
int ars_step_to(ars_ctx* ctx, const double* d_in, double* d_a, double* d_b, double* d_out, void* d_work,
                int n_steps, double* d_t, double* d_dt, double* d_dt_log, void* stream);

/* The same n_steps >= 1 steps out of place, with no copy: step 1 reads
 * d_in (never written), the intermediate states alternate between the
 * scratch states d_a and d_b (steps 1, 3, ... write d_a, steps 2, 4, ...
 * d_b), and the last step writes d_out instead.  For a checkpointing
 * schedule whose state lives in several buffers (the adjoint's revolve
 * plan: restore, advance, store): the restore is a choice of d_in, the
 * store a choice of d_out.  EINVAL for a NULL pointer, n_steps < 1,
 * d_a == d_b, d_in equal to d_a or d_b, d_out equal to d_a or d_b, or
 * d_out == d_in with n_steps == 1 (a step cannot run in place).
 * Asynchronous; *d_t advanced by the dts used (d_t may be NULL). */
int ars_step_sched_to(ars_ctx* ctx, const double* d_in, double* d_a, double* d_b, double* d_out, void* d_work,
                      int n_steps, const double* d_dt_sched, double* d_t, void* stream);

/* Implicit acoustic (IMEX) step: the further work named in the paper's
 * Conclusion (solve the acoustic part implicitly to lift the acoustic CFL
 * condition while keeping the well-balanced gravity source); the paper
 * prints no scheme.  Reading: the acoustic step of Sec. 2.1.2 with its
 * interface values u*, Pi* taken at the end of the step (backward Euler on
 * the linear relaxation system at the frozen a, S and theta of t^n):
 *   u*_j  = (u_L + u_R)/2 - (Pi_R - Pi_L - S_j) / (2 a_j)    (0 at walls)
 *   Pi*_j = (Pi_L + Pi_R)/2 - (a_j theta_j / 2)(u^n_R - u^n_L)
 *   u_{d,i} = u^n_{d,i} - (dt/dx_d) tau_i ([Pi*]_{d,i} - S-bar_{d,i})
 *   Pi_i    = p_i - rho_i c_i^2 sum_d (dt/dx_d) [u*]_{d,i}
 * u is eliminated (its rows are explicit in Pi) and the system for Pi,
 * rows scaled by 1 / (rho c^2), is solved to a relative residual tol: by
 * conjugate gradients when every axis is periodic or walled at both ends
 * (the operator is then symmetric positive definite), else (outflow) by
 * BiCGSTAB.  The acoustic dissipation of Pi* acts on u^n: with the
 * low-Mach correction (theta ~ Ma) steps far above the acoustic limit are
 * stable, without it (theta = 1) only steps near it.  The
 * implicit (u*, Pi*) then enter the acoustic cell values, transport,
 * update and relaxation of eq. all_regime_scheme as in ars_step.  Dissipative
 * fluxes stay explicit.  dt of step s = d_dt_sched[s] (device); with
 * dt_mode = 2 ars_compute_dt gives the transport + diffusive CFL step that
 * this call allows (the acoustic limit is lifted).  d_tmp: scratch state;
 * d_work: the ars_step workspace (fault latch); d_work_imex:
 * ars_workspace_bytes_imex bytes, caller-owned.  *h_iters (nullable): total
 * solver iterations.  Synchronises (the solver reads its residual); returns
 * ARS_ENOCONV if a solve does not reach tol within max_iter iterations,
 * ARS_EUNSUPPORTED for the energy form of App. B. */
size_t ars_workspace_bytes_imex(const ars_ctx* ctx);
int ars_step_imex(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, void* d_work_imex, int n_steps,
                  const double* d_dt_sched, double* d_t, double tol, int max_iter, int* h_iters, void* stream);

/* Reference path: the same step as separate phase kernels (ghosts and
 * primitives, faces, acoustic cell values, fluxes, update) with their
 * intermediate arrays in a second caller-owned buffer d_work_ref of
 * ars_workspace_bytes_ref bytes; kept to check the fused kernel bit for
 * bit.  dt of step s is d_dt_sched[s]. */
size_t ars_workspace_bytes_ref(const ars_ctx* ctx);
int ars_step_ref(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, void* d_work_ref, int n_steps,
                 const double* d_dt_sched, void* stream);

/* Adjoint of one step at a frozen time step (the gradient is that of the
 * discrete step of eq. all_regime_scheme + Sec. 2.2 with dt held fixed):
 *   d_lam_n = (dU^{n+1}/dU^n)^T d_lam_np1          (overwritten)
 *   d_param_grad[0] += <d_lam_np1, dU^{n+1}/dmu>, d_param_grad[1] += ... dkappa
 * d_state_n is U^n (the step's input), *d_dt the step's dt (device).
 * Non-smooth operations differentiate the branch taken by the forward step
 * (max/min: first argument on ties; upwind: u* >= 0 takes the left cell).
 * d_param_grad may be NULL; with mu = kappa = 0 the dissipative terms are
 * absent and no parameter derivative is produced.  d_work_adj: caller
 * buffer of ars_workspace_bytes_adjoint bytes.  Deterministic (no atomics).
 * d_lam_n must not alias d_lam_np1.  Asynchronous.
 * 3D problems with periodic lateral sides of at least 5 cells and walls at
 * both vertical ends (or periodic ends with g = 0), conservative energy
 * form, run three fused tile marches whose workspace is 17 doubles per cell;
 * every other configuration runs the reference path below. */
size_t ars_workspace_bytes_adjoint(const ars_ctx* ctx);
int ars_step_adjoint(ars_ctx* ctx, const double* d_state_n, const double* d_lam_np1, double* d_lam_n,
                     const double* d_dt, double* d_param_grad, void* d_work_adj, void* stream);

/* Reference path of the adjoint step: the same product by phase kernels
 * over padded arrays (forward phases recomputed, then the reverse of each
 * phase as a gather), every configuration, with a workspace of
 * ars_workspace_bytes_adjoint_ref bytes; same arguments and contract as
 * ars_step_adjoint.  Kept to check the fused marches. */
size_t ars_workspace_bytes_adjoint_ref(const ars_ctx* ctx);
int ars_step_adjoint_ref(ars_ctx* ctx, const double* d_state_n, const double* d_lam_np1, double* d_lam_n,
                         const double* d_dt, double* d_param_grad, void* d_work_adj, void* stream);

/* Kinetic-energy objective J = sum (1/2) |m|^2 / rho dV of d_state into the
 * device scalar *d_ke, and (if d_grad is not NULL) its gradient dJ/dU in
 * state layout (d/drho = -|u|^2 dV/2, d/dm = u dV, d/dE = 0).  Uses the
 * workspace's reduction area.  Asynchronous. */
int ars_kinetic_energy(ars_ctx* ctx, const double* d_state, double* d_grad, double* d_ke, void* d_work,
                       void* stream);

/* Nusselt-number objective at a fixed-temperature wall (side 0: bottom,
 * 1: top of the gravity axis) of d_state into the device scalar *d_nu:
 * the horizontal mean of the two-point wall conductive flux,
 * 2 (T_wall - T_0)/dz at the bottom or 2 (T_{n-1} - T_wall)/dz at the top,
 * times depth / (T_bottom - T_top) (the conductive profile gives 1; the
 * quantity the diagnostics report as nu_bot / nu_top).  If d_grad is not
 * NULL it receives dNu/dU in state layout (zero except on the
 * wall-adjacent plane).  ARS_EINVAL unless the gravity axis has walls on
 * both sides, that side is a fixed-T wall and the wall temperatures
 * differ.  Uses the workspace's reduction area.  Asynchronous. */
int ars_nusselt(ars_ctx* ctx, const double* d_state, int side, double* d_grad, double* d_nu, void* d_work,
                void* stream);

/* Kinetic-energy spectrum of the horizontal plane at index kz of the
 * gravity axis (Sec. 4.5, 3D case, where it is taken on the middle plane,
 * kz = n_z / 2): with w_c = sqrt(rho) u_c on the plane for every velocity
 * component and W_c its discrete Fourier transform (kernel
 * exp(-2 pi i k.x / n), integer wave numbers k_j = j for j < (n+1)/2, else
 * j - n), d_spec[s] = sum over the k with round(|k|) = s of
 * sum_c |W_c(k)|^2 / (2 N^2), N the cell count of the plane, for
 * s < ars_spectrum_len(); the entries sum to the plane mean of
 * rho |u|^2 / 2.  In 2D the plane is a line along x and s = |k_x|.
 * d_work_spec: caller-owned device scratch of ars_workspace_bytes_spectrum
 * bytes (no contents kept between calls).  ARS_EINVAL for a NULL pointer
 * or kz outside [0, n_z); ARS_EUNSUPPORTED for a plane side above 2048.
 * A cell with rho <= 0 makes the result NaN.  Deterministic; asynchronous. */
int ars_spectrum_len(const ars_ctx* ctx); /* floor(|(n_x/2, n_y/2)| + 1/2) + 1 */
size_t ars_workspace_bytes_spectrum(const ars_ctx* ctx);
int ars_spectrum(ars_ctx* ctx, const double* d_state, int kz, double* d_spec, void* d_work_spec, void* stream);

/* Binomial checkpointing plan (host only) for reversing n steps with s
 * snapshot slots, slot 0 holding U^0 and slots used as a stack.  Writes up
 * to cap actions of 4 int32 {op, step, arg, 0}:
 *   op 0 ADVANCE  the working state from step `step` to step `arg`
 *   op 1 STORE    the working state (at step `step`) into slot `arg`
 *   op 2 RESTORE  slot `arg` (holding step `step`) into the working state
 *   op 3 ADJOINT  of step `step` (the working state is U^step)
 * Returns the number of actions (call with cap = 0 to size the array) or
 * ARS_EINVAL; *forward_steps = total steps advanced, which is the minimum
 * ars_revolve_cost(n, s) over all such schedules. */
int ars_revolve_plan(int n, int s, int32_t* actions, int cap, int64_t* forward_steps);
int64_t ars_revolve_cost(int n, int s);

/* ---- Batched problems -------------------------------------------------
 * Many independent 2D problems (each its own ars_config: size, mu, kappa,
 * boundaries, theta switch) advanced by one persistent launch; each
 * instance keeps its own CFL time step (Sec. 2 step with the time-step
 * rule of the single-problem calls) and its results equal those of
 * ars_step on that instance alone, bit for bit.  One workgroup owns one
 * instance for all steps (largest instances first), so no workgroup ever
 * waits for another.
 *
 * States: one caller-owned device array of ars_batch_state_len() doubles;
 * instance k occupies ars_batch_state_offset(k) onward, in the state layout
 * of the single-problem calls.  d_tmps: a second array of the same length
 * (ping-pong).  d_table: caller-owned device buffer of
 * ars_batch_table_bytes() bytes holding the instance table (per-instance
 * parameters, pointers, t, next dt and fault latch).
 *
 * ars_batch_create   validates every config (dim must be 2, else
 *                    ARS_EUNSUPPORTED); host only.
 * ars_batch_set_tiling  rows = row segments of 60 columns per workgroup
 *                    (4 or 8); zc = per-instance vertical chunk counts
 *                    (each must divide that instance's nz; NULL = the
 *                    built-in cost model).  Results do not depend on the
 *                    tiling.  Invalidates the captured graph; call
 *                    ars_batch_bind again afterwards.
 * ars_batch_bind     writes the table for these buffers (t = 0) and
 *                    synchronises `stream`.
 * ars_batch_step     advances every instance n_steps steps, dt of each step
 *                    = cfl / (max rate of its current state).  Asynchronous.
 * ars_batch_capture  captures the same launch (n_steps) into a hipGraph on
 *                    `stream` (which must not be NULL); ars_batch_replay
 *                    launches it.  A replay continues from the table's
 *                    current t and states.
 * ars_batch_read     copies per-instance t, next dt and the fault cell
 *                    (-1: none) to host arrays of n entries (each may be
 *                    NULL); synchronises; ARS_ENONPHYS if any instance
 *                    latched a fault. */
typedef struct ars_batch ars_batch;
int ars_batch_create(int n_inst, const ars_config* cfgs, ars_batch** out);
void ars_batch_destroy(ars_batch* b);
size_t ars_batch_state_len(const ars_batch* b);
size_t ars_batch_state_offset(const ars_batch* b, int k);
size_t ars_batch_table_bytes(const ars_batch* b);
int ars_batch_set_tiling(ars_batch* b, int rows, const int* zc);
int ars_batch_get_tiling(const ars_batch* b, int* rows, int* zc);
int ars_batch_bind(ars_batch* b, double* d_states, double* d_tmps, void* d_table, void* stream);
int ars_batch_step(ars_batch* b, void* d_table, int n_steps, void* stream);
int ars_batch_capture(ars_batch* b, void* d_table, int n_steps, void* stream);
int ars_batch_replay(ars_batch* b, void* stream);
int ars_batch_read(const ars_batch* b, const void* d_table, double* h_t, double* h_dt, int64_t* h_fault_cell,
                   void* stream);

/* ---- Launch shapes and autotuning --------------------------------------
 * ars_set_tiling / ars_get_tiling: the fused step's launch shape, zchunk =
 * smallest vertical share of planes a workgroup takes (>= 1) and wg_per_cu
 * = workgroups per compute unit (0: as many as are resident at once, up to
 * 32).  Results never depend on either, only time does.
 *
 * ars_autotune times the fused step (trial_steps steps after one untimed
 * step, per candidate) for candidate (tile, zchunk, wg_per_cu) triples (both
 * tiles of ars_set_tile3 in 3D) on a copy of d_state, keeps the fastest in
 * ctx and returns it in *out (may be NULL).
 * d_state is not modified; the workspace's rate slots and fault latch are
 * reset (as by ars_workspace_init).  It allocates and frees a temporary
 * device copy of two states: a set-up call, never to be captured.
 *
 * ars_batch_autotune times the batched launch over rows in {4, 8} and
 * vertical chunking policies (zc_policy 0: the cost model, 1: no chunks,
 * 2: twice, 3: half the model's chunks), applies the fastest with
 * ars_batch_set_tiling and rebinds the table (t = 0).  d_states is
 * restored to its contents at the call; it allocates a temporary copy.
 *
 * cache_path (may be NULL): text file of tuned shapes, one line per key
 * "<key> <a> <b> <ms_per_step> [<tile>]"; a key found there is applied without
 * timing (from_cache = 1), otherwise the result is appended.  Keys name
 * the device (architecture, compute units) and the problem (dimension,
 * grid, boundary kinds, theta and dissipation switches; for a batch a hash
 * of all instances' shapes and switches). */
typedef struct ars_tune_result {
  int32_t zchunk, wg_per_cu;  /* fused step */
  int32_t rows, zc_policy;    /* batch */
  int32_t from_cache, n_candidates;
  double ms_per_step;         /* of the chosen shape */
  int32_t tile3, pad_;        /* fused step, 3D: ARS_TILE3_* */
} ars_tune_result;
int ars_set_tiling(ars_ctx* ctx, int zchunk, int wg_per_cu);
int ars_get_tiling(const ars_ctx* ctx, int* zchunk, int* wg_per_cu);
int ars_autotune(ars_ctx* ctx, const double* d_state, void* d_work, int trial_steps, const char* cache_path,
                 void* stream, ars_tune_result* out);
int ars_batch_autotune(ars_batch* b, double* d_states, double* d_tmps, void* d_table, int trial_steps,
                       const char* cache_path, void* stream, ars_tune_result* out);

/* Diagnostics of d_state into *h_out (synchronises `stream`).  Returns
 * ARS_ENONPHYS (and clears the latch) if a fault was latched. */
int ars_diagnostics(ars_ctx* ctx, const double* d_state, void* d_work, ars_diag* h_out, void* stream);

/* Read (and clear) the fault latch without diagnostics (synchronises). */
int ars_fault(ars_ctx* ctx, void* d_work, int64_t* fault_cell, void* stream);

const char* ars_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* ARS_H */
