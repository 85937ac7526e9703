/*
 * mgrit.h -- C ABI of the MI355X (gfx950) MGRIT library for the 2D eddy-current
 * problem of an induction machine (arXiv:1912.03106).
 *
 * The library solves the space-time system of Sec. 2 (block lower-bidiagonal
 * system A u = g built from a one-step integrator Phi, eq. 2) for the
 * backward-Euler discretisation (eq. 8) of the semi-discrete eddy-current
 * system M u' + K(u) u = f(t) (eq. 7) on P1 triangles, either sequentially
 * (forward block solve) or with FAS-MGRIT (Algorithm 1) in a V-cycle with
 * F/FCF relaxation and optional spatial coarsening between nested meshes
 * (Sec. 2.2).  Every step runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point
 *  - Unknowns are the non-Dirichlet nodes of a mesh, in increasing node-id
 *    order; n_l is their count on level l.
 *  - Time-major arrays: point t of a trajectory is the contiguous vector
 *    u[t*n .. t*n+n-1].  Level l has N_l = N_t / (m_0 ... m_{l-1}) steps of
 *    size m_0 ... m_{l-1} dt, m_0 = m and m_l = m_coarse (or m) for l >= 1.
 *  - Host pointers unless a field says otherwise.  The library copies what it
 *    needs during mgrit_setup; the caller keeps ownership of every array it
 *    passes and may free it after the call returns.
 *  - Every function returns MGRIT_OK (0) or a negative mgrit_status; no C++
 *    exception crosses this boundary.  mgrit_last_error() gives the message.
 *  - A handle is not thread-safe: one handle per host thread.  Work runs on
 *    the HIP stream given to mgrit_setup; calls that return results to the
 *    host synchronize that stream before returning.
 */
#ifndef MGRIT_H
#define MGRIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGRIT_ABI_VERSION 2
#define MGRIT_MAX_LEVELS 8
#define MGRIT_MAX_HISTORY 128

typedef enum {
  MGRIT_OK = 0,
  MGRIT_INVALID_ARGUMENT = -1,
  MGRIT_NOT_NESTED = -2,          /* spatial coarsening between non-nested meshes */
  MGRIT_OUT_OF_MEMORY = -3,
  MGRIT_HIP_ERROR = -4,
  MGRIT_PCG_NOT_CONVERGED = -5,   /* a linear solve hit pcg_max_iter */
  MGRIT_NEWTON_NOT_CONVERGED = -6,/* a nonlinear step hit newton_max_iter (Sec. 5.2) */
  MGRIT_NOT_CONVERGED = -7,       /* MGRIT hit max_iter before tol (Table 2) */
  MGRIT_NONFINITE = -8,           /* NaN or Inf in an input or an iterate */
  MGRIT_UNSUPPORTED = -9
} mgrit_status;

/* One triangulation (Sec. 3.4).  n_r, n_theta > 0 declare the structured
 * polar numbering node id = i*n_theta + j (i radial, j angular, periodic in j);
 * spatial coarsening needs it.  Triangles must be counter-clockwise. */
typedef struct {
  int32_t n_r, n_theta;
  int32_t n_nodes, n_tri;
  const double*  xy;          /* [n_nodes][2] node coordinates, m               */
  const int32_t* tri;         /* [n_tri][3] node ids                            */
  const int32_t* cell_mat;    /* [n_tri] index into the material table          */
  const int32_t* cell_phase;  /* [n_tri] -1 = no source, else phase 0, 1 or 2   */
  const int32_t* cell_sign;   /* [n_tri] winding direction (+1 / -1 / 0)        */
  const uint8_t* dirichlet;   /* [n_nodes] 1 = A fixed to 0                     */
  const int32_t* cell_bar;    /* [n_tri] rotor bar 0 .. n_bars-1, -1 elsewhere; read only
                               * with circuit = 1 and n_bars > 0 (may be NULL otherwise) */
} mgrit_mesh;

/* Materials, source and time grid (Sec. 3.1-3.3).
 * nu(B^2) = bh_k1 exp(bh_k2 B^2) + bh_k3 in materials with iron[k] = 1 when
 * nonlinear != 0; otherwise nu = nu[k].  The coil current density of a cell
 * is sign * J0 * amplitude * b_phase(t), b_p(t) = sgn(sin(2 pi freq t +
 * phases[p] + phase_offset) - c(t)), carrier c = triangle (0) or sawtooth (1)
 * of frequency f_carrier; sgn(0) = 0.  ramp_periods = R > 0 multiplies the
 * source by the start-up factor (1 - cos(pi t f / R)) / 2 for t < R / f and
 * by 1 afterwards (nonlinear model, Sec. 3.3); 0 = no ramp. */
typedef struct {
  int32_t n_materials;
  const double*  nu;          /* [n_materials] reluctivity, A m / Wb */
  const double*  sigma;       /* [n_materials] conductivity, S / m   */
  const int32_t* iron;        /* [n_materials] 1 = saturating law applies */
  int32_t nonlinear;
  double bh_k1, bh_k2, bh_k3;
  double J0, amplitude, freq, f_carrier, phase_offset;
  double phases[3];
  int32_t carrier;            /* 0 triangle (c(0) = 1), 1 sawtooth */
  double dt;                  /* finest step; t_i = i * dt */
  int64_t n_steps;            /* N_t on the finest level */
  double ramp_periods;        /* start-up ramp length in electric periods (0 = none) */
  int32_t signal;             /* 0: the PWM signals b_p; 1: the sine references themselves
                               * drive the coils (the smooth source of Sec. 4.1) */
  double t_start;             /* time origin: point i samples the source at t_start + i dt
                               * (a window of a longer horizon; 0 = the horizon's start) */
  /* Field-circuit coupling (Sec. 3.1, the stator coil and rotor bar circuit
   * equations), linear model only.  circuit = 1: the coils are stranded
   * conductors with winding function turns_density * cell_sign on the cells
   * of each phase, fed by the phase voltages v_s(t) = v0 * amplitude * b_s(t)
   * (times the start-up ramp) through the phase resistance r_phase:
   *   l_z d/dt (X_s^T a) + r_phase i_s = v_s(t),  X_s = turns_density F_s;
   * J0 is unused.  With n_bars > 0 the cells of bar k (cell_bar) are a solid
   * conductor with voltage distribution 1 / l_z carrying the voltage v_k and
   * the current i_k = G_k v_k - d/dt(integral of sigma A over bar k),
   * G_k = sigma area_k / l_z; two end rings with resistance ring_r between
   * neighbouring bars close the cage: i = -(1 / (2 ring_r)) L v, L the
   * periodic path Laplacian over the bars.  No circuit inductance: the
   * currents and voltages are algebraic, fixed by two consecutive states, so
   * MGRIT's state stays the vector potential.  With n_bars = 0 the bar cells
   * are plain conductors (bar voltages 0), as with circuit = 0.  Inside
   * mgrit_solve a coupled step's linear solve (for a' - Z w, Z = A^-1 B^T)
   * starts from its guess of a' less Z times the circuit unknowns of the
   * latest step from the same time point, and pcg_tol_eta / residual_eta
   * apply as in the uncoupled model.  With them, pcg_tol <= 1e-14 is
   * advised: the right-hand side (M/dt) a is dominated by the bars' sigma/dt
   * rows, and with 1e-12 the iteration levels off near 1e-8 of rho_0. */
  int32_t circuit;            /* 0: current-driven coils (sign * J0 * amplitude * b_p); 1: coupled */
  double turns_density;       /* turns per m^2 of slot (> 0 with circuit = 1) */
  double l_z;                 /* axial length, m (> 0) */
  double r_phase;             /* stator phase resistance, ohm (> 0) */
  double v0;                  /* phase-voltage amplitude, V */
  int32_t n_bars;             /* rotor bars with circuit equations, 0 .. 32 */
  double ring_r;              /* end-ring resistance between neighbouring bars, ohm (> 0 with bars) */
} mgrit_physics;

typedef struct {
  int32_t n_levels;           /* MGRIT levels (>= 1); level 0 is the finest   */
  const mgrit_mesh* meshes;   /* [n_levels] mesh of every level               */
  mgrit_physics phys;
} mgrit_problem;

enum { MGRIT_FP64 = 0, MGRIT_FP32_IR = 1 };
enum { MGRIT_R_NORMALIZED = 0, MGRIT_R_TRANSPOSE = 1, MGRIT_R_INJECTION = 2 };

typedef struct {
  int32_t m;                  /* temporal coarsening factor between levels 0 and 1 (> 1) */
  int32_t gamma;              /* CF relaxations after the first F (1 = FCF)    */
  int32_t precision;          /* MGRIT_FP64 or MGRIT_FP32_IR                    */
  int32_t restriction;        /* MGRIT_R_*                                      */
  double  tol;                /* stop at rho_k <= tol * rho_0 (C-point residual)*/
  int32_t max_iter;           /* MGRIT iterations (coarse corrections)         */
  double  pcg_tol;            /* relative residual of every linear solve       */
  int32_t pcg_max_iter;
  int32_t pcg_check_every;    /* PCG iterations between host reads of the active-column count
                               * (the points where column compaction can happen; default 4) */
  double  ir_inner_tol;       /* relative tolerance of the inner CG: FP32 refinement steps and
                               * Newton corrections; a solve with an early stop at eta times its
                               * start residual uses min(0.1, max(ir_inner_tol, eta / 2)) */
  int32_t ir_max_iter;        /* refinement sweeps                              */
  double  newton_tol;         /* ||R(u^k)|| <= newton_tol ||R(u_prev)||        */
  int32_t newton_max_iter;
  int32_t warm_start;         /* 0: every solve starts from its input; 1: from the previous
                               * iterate at the same point; 2: as 1, and the level-0
                               * F-relaxation solves add the change of their input since
                               * that iterate was computed, u_j + (u_{j-1} - u_{j-1}^old)
                               * (Phi is nearly the identity on slowly varying changes at small
                               * steps, so this start is much closer; then pcg_tol_eta can be
                               * larger at the same accuracy) */
  int32_t device_pointers;    /* 1: u_init / u_out of mgrit_solve are device pointers */
  int32_t profile_kernels;    /* 1: time every PCG pass with HIP events (mgrit_stats.kernel_*) */
  int32_t autotune;           /* 1: time the batched-PCG tile shapes at setup and keep the fastest */
  int32_t pcg_kernel;         /* batched-PCG kernels: 0 choose (autotuner), 1 general sparse rows,
                               * 2 diagonal window (periodic polar stencil only, else UNSUPPORTED) */
  int32_t coarse_inverse;     /* linear model: 1 = the coarsest level (<= 8192 unknowns) steps with
                               * a stored A^{-1} (exact implicit Euler) instead of PCG; 2 = also
                               * every intermediate level <= 16384 unknowns (batched steps become
                               * one FP64 matrix-core product each); 0 = PCG everywhere */
  int32_t seq_kernel;         /* mgrit_seq_solve: 0 choose, 1 one persistent work-group (linear
                               * PCG or, nonlinear, the whole Newton sweep), 2 cooperative grid
                               * (linear) / batched Newton kernels step by step (nonlinear),
                               * 3 linear model: exact steps with the finest level's stored
                               * inverse (built by the first call, n^2 doubles; the build time is
                               * reported in time_nested_s).  With circuit = 1 the choices 0-2 step
                               * with the batched step and its circuit elimination one column at a
                               * time; 3 eliminates the circuit unknowns after each inverse step. */
  int32_t use_graphs;         /* 1: replay each check interval of CG iterations from a captured
                               * hipGraph (not while profile_kernels = 1: launches stay eager so
                               * that HIP events time each pass) */
  int32_t newton_halvings;    /* damped Newton (Sec. 5.1): per column, the first step length
                               * lambda in 1, 1/2, ..., 2^-newton_halvings with
                               * ||R(u + lambda d)|| < (1 - 1e-4 lambda) ||R(u)||, else the
                               * last one; 0 = plain Newton */
  double  pcg_tol_eta;        /* > 0: the linear solves of the level-0 F- and C-relaxation of
                               * mgrit_solve stop at ||r|| <= max(pcg_tol ||b||, eta ||r_0||), r_0
                               * the residual of their start (see warm_start), which shrinks as
                               * MGRIT converges; their Newton iterations likewise at
                               * ||R|| <= max(newton_tol ||R(u_prev)||, eta ||R(start)||).  The
                               * C-point residual keeps pcg_tol unless residual_eta > 0; all
                               * coarse levels keep the strict tolerances.  0 = strict */
  int32_t precision_coarse;   /* arithmetic of the linear solves on levels >= 1: -1 = precision,
                               * else MGRIT_FP64 or MGRIT_FP32_IR (level 0 always uses precision) */
  int32_t coarse_model;       /* coarsest-level propagator: 0 implicit Euler (Sec. 2.1
                               * re-discretisation), 1 implicit Euler plus the learned correction
                               * (needs mgrit_train_coarse or mgrit_set_coarse_weights) */
  int32_t compact_columns;    /* k > 0: when at most compact_fraction of a batched CG's columns
                               * still iterate and at least k columns would drop out, gather the
                               * iterating ones densely (same iterates, fewer masked lanes);
                               * 0 = never */
  double  compact_fraction;   /* see compact_columns (default 0.9; compact_columns default 64) */
  int32_t pcg_prefetch;       /* diagonal-window PCG kernels: rows of loads in flight per wave,
                               * 1, 2 or 4; 0 = the autotuner's choice (1 without autotune).
                               * Results do not depend on it. */
  double  residual_eta;       /* > 0: the level-0 C-point residual solves (Alg. 1, the residual
                               * before restriction) also stop at residual_eta times their
                               * warm-start residual.  Their warm start is the current C-point
                               * value, so that residual is proportional to the MGRIT residual
                               * and the stop is relative to it; 0 = pcg_tol only (default). */
  int32_t pcg_rows_narrow;    /* rows per work-group of the batched PCG passes once at most 128
                               * columns still iterate (shorter dependent-load walks): 0 = the
                               * autotuner's choice, -1 = never switch, 16/32/64/128/256 = this */
  int32_t cycle;              /* 0 V-cycles; 1 F-cycles: the coarse problem of a level is
                               * approximated by an F-cycle and then a V-cycle on the next level
                               * (Sec. 2.1, Fig. 4) */
  int32_t nested;             /* 1: start from the nested-iteration guess (Sec. 2.1): the coarsest
                               * time-stepping problem solved sequentially, then per finer level
                               * its points interpolated to the C-points and one V-cycle, all with
                               * the sine references as the source (Sec. 4.1); u_init is ignored */
  double  loss_tol;           /* > 0: stop once the Joule losses at the C-points change by less than
                               * loss_tol (relative, every C-point) between two successive
                               * iterations (Sec. 5.1 uses 1e-2) instead of the residual test */
  int32_t m_coarse;           /* temporal coarsening factor between levels l >= 1 and l + 1 (Sec. 4.1:
                               * a large factor m on the first level, a small one below); 0 = m.
                               * n_steps must be divisible by m * m_coarse^(levels - 2) */
  int32_t coarse_persistent;  /* nonlinear model, coarse levels.  0 = one persistent work-group
                               * runs the coarsest level's whole sequential Newton sweep (every
                               * Newton, CG and step-length iteration on the device) when the
                               * level has at most 16384 unknowns; 1 = that at any size, and in
                               * addition one persistent work-group per column for batches of at
                               * most 256 columns on levels >= 1 (FP64 inner CG; Newton and CG
                               * iterations then counted per column; slower than the batched
                               * kernels on the 32x256 level); -1 = never (batched kernels) */
  int32_t pcg_check_narrow;   /* PCG iterations between host reads of the active-column count for
                               * batches of at most 128 columns (coarse levels: no compaction, and
                               * each read is a device-to-host round trip); 0 = pcg_check_every;
                               * default 16; both at most 64 */
  int32_t pcg_rows_per_block; /* rows per work-group of the batched PCG passes: 0 = the
                               * autotuner's choice, else 16, 32, 64, 128 or 256 */
  int32_t pcg_cols_per_lane;  /* columns per lane of the batched PCG passes: 0 = the autotuner's
                               * choice, else 1 or 2.  With pcg_kernel, pcg_prefetch and
                               * pcg_rows_narrow these pin the whole kernel shape (hardware-counter
                               * runs, where timings would steer the autotuner); results do not
                               * depend on the shape. */
} mgrit_params;

typedef struct {
  int32_t iterations;         /* coarse corrections performed                   */
  int32_t converged;
  int32_t n_history;
  double  rho[MGRIT_MAX_HISTORY];     /* C-point residual norm per iteration     */
  int64_t phi_columns[MGRIT_MAX_LEVELS];   /* Phi applications per level        */
  int64_t pcg_sweeps[MGRIT_MAX_LEVELS];    /* batched PCG iterations per level   */
  int64_t newton_sweeps[MGRIT_MAX_LEVELS];
  /* batched PCG passes per level: [0] pass A (new direction, p.Ap), [1] pass B
   * (x, r update).  Launches and device time count every launch (including
   * the few at the end of a check interval that find every column converged
   * and exit at once); kernel_columns sums the unconverged columns the
   * launches worked on. */
  int64_t kernel_launches[2][MGRIT_MAX_LEVELS];
  int64_t kernel_columns[MGRIT_MAX_LEVELS];
  double  kernel_time_s[2][MGRIT_MAX_LEVELS];   /* needs profile_kernels = 1 */
  double  time_relax_s;       /* finest-level F/C relaxation time (device events) */
  double  time_total_s;
  int32_t coarse_fallback;    /* coarse_model = 1: iteration after which the residual grew and
                               * the coarsest level went back to implicit Euler; -1 = never */
  double  time_nested_s;      /* nested = 1: time of the nested-iteration start (in time_total_s);
                               * mgrit_seq_solve with seq_kernel = 3: time of the inverse build */
  double  loss_change[MGRIT_MAX_HISTORY];  /* loss_tol > 0: largest relative change of the C-point
                               * Joule losses against the previous iteration (-1 for the first) */
  double  time_phi_s[MGRIT_MAX_LEVELS];    /* profile_kernels = 1: wall time of each level's Phi
                               * applications and coarsest solve (stream drained around each) */
} mgrit_stats;

/* Fill *par with the defaults (m = 16, FCF, FP64, normalized restriction,
 * tol 1e-8, pcg_tol 1e-12, ...). */
void mgrit_default_params(mgrit_params* par);

/* Build the level hierarchy on the device: assembles K, M/dt_l, the Jacobi
 * diagonal and the phase load vectors on every level (eq. 7, 8), builds the
 * spatial transfers between consecutive levels whose meshes differ (nodal
 * interpolation P_s in the logical polar coordinates and R_s from P_s^T,
 * Sec. 3.4; MGRIT_NOT_NESTED if the meshes are not nested) and allocates the
 * space-time storage.  hip_stream: a hipStream_t (NULL = default stream).
 * On success *out owns all device memory until mgrit_destroy. */
int mgrit_setup(const mgrit_problem* prob, const mgrit_params* par,
                void* hip_stream, void** out);

/* FAS-MGRIT V-cycles (Algorithm 1, Sec. 2.1) until rho_k <= tol rho_0.
 * u0:     [n_0] initial value A(t_0) (NULL = 0).
 * u_init: [(N_t+1)][n_0] initial space-time guess, row 0 ignored (NULL = 0).
 * u_out:  [(N_t+1)][n_0] result: the relaxed iterate of the last iteration.
 * Returns MGRIT_NOT_CONVERGED (with u_out and *st filled) if max_iter is hit. */
int mgrit_solve(void* h, const double* u0, const double* u_init, double* u_out,
                mgrit_stats* st);

/* Joule losses P(t_i) = l_z (du/dt)^T M (du/dt), du/dt = (u_i - u_{i-1}) / dt the
 * backward difference of the implicit-Euler grid, M the sigma-weighted mass
 * matrix, l_z = 1 m (Sec. 3.1, the loss integral), at every point of the
 * iterate the last mgrit_solve on this handle returned: p [N_t + 1], p[0] = 0,
 * in W per metre of axial length.  A device pointer when device_pointers = 1.
 * INVALID_ARGUMENT before a completed solve. */
int mgrit_joule_losses(void* h, double* p);

/* Circuit quantities of a level-0 trajectory (circuit = 1; Sec. 3.1, the
 * stator coil and rotor bar circuit equations).  u: [(N_t+1)][n_0] time-major
 * (a device pointer when device_pointers = 1), e.g. the output of
 * mgrit_solve or mgrit_seq_solve.  out (host): [N_t][3 + 2 n_bars]; row i-1
 * holds for the step t_{i-1} -> t_i the stator phase currents i_1..3 (A),
 * the bar voltages v_1..nb (V) and the bar currents (A), each from the
 * circuit equations of that step alone:
 *   i_s = (v_s(t_i) - l_z X_s^T (u_i - u_{i-1}) / dt) / r_phase,
 *   C v = Y'^T (u_i - u_{i-1}) / dt,   i_bar = -L v / (2 ring_r).
 * UNSUPPORTED without a circuit. */
int mgrit_circuit_values(void* h, const double* u, double* out);

/* Sequential forward block solve (Sec. 2) on the finest level, on the GPU:
 * u_out [(N_t+1)][n_0] = (u0, Phi_1(u0), ...).  u0 may be NULL (= 0). */
int mgrit_seq_solve(void* h, const double* u0, double* u_out, mgrit_stats* st);

/* The one-step integrator Phi of level `level` (eq. 2 with eq. 8), batched:
 * u_next[k] = Phi(u_prev[k]) from t = i_from[k] * dt_level to
 * (i_from[k] + 1) * dt_level, forcing at the new time included.
 * u_prev, u_next: [B][n_level] time-major; i_from: [B].  Host pointers. */
int phi_step(void* h, int32_t level, int32_t B, const int64_t* i_from,
             const double* u_prev, double* u_next);

/* Allocation-free phi_step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same operation, layout and errors as phi_step, except that
 * i_from [B], u_prev [B][n_level] and u_next [B][n_level] are DEVICE
 * pointers owned by the caller.  Every workspace of the call lives in one
 * static device array of the library, 134.8 MiB per GPU, which each GPU the
 * library runs on holds until the process ends; the call allocates nothing
 * (no hipMalloc / hipFree, no allocating library routine) and does not use
 * graph replay or column compaction (the same iterates as phi_step).
 * Limits: n_level * round_up(B, 64) <= 2^21 (e.g. B <= 64 on the 64 x 512
 * mesh, B <= 1024 on 16 x 128), B <= 32768, pcg_max_iter <= 65472: else
 * MGRIT_INVALID_ARGUMENT.  The nonlinear model (its Newton workspace does not
 * fit): MGRIT_UNSUPPORTED.  The array is shared by every call on one GPU and keeps
 * the last call's contents: calls that overlap on one GPU (other threads,
 * handles or streams) race, so the caller serialises them.  The handle's
 * device must be current.  Returns after the stream is synchronized. */
int phi_step_noalloc(void* h, int32_t level, int32_t B, const int64_t* i_from,
                     const double* u_prev, double* u_next);

/* Sizes of a level: unknowns, steps, stored entries of the operator (fixed
 * row width times n), and kernel_shape[5] of its batched PCG kernels as the
 * autotuner chose them: rows per work-group, columns per lane, kernel family
 * (1 general sparse rows, 2 diagonal window), rows of loads in flight per
 * wave (1, 2 or 4; diagonal window only, else 1) and rows per work-group once
 * at most 128 columns still iterate (0 = unchanged).  Any output pointer may
 * be NULL. */
int mgrit_level_info(void* h, int32_t level, int64_t* n, int64_t* n_steps, int64_t* nnz,
                     int32_t* kernel_shape);

/* ---- Learned coarse propagator (coarsest level, coarse_model = 1) ----------
 * MGRIT admits any coarse propagator (Sec. 2.1: re-discretisation is one
 * choice); with FAS the fixed point is the fine solution whatever it is.  The
 * learned one is Psi(u) = p + s_out delta, p the implicit-Euler coarse step of
 * u, delta a 3-layer message-passing network (width 64, tanh) on the coarsest
 * mesh's interior-node graph.  Node features (F = m + 7): u/s_u, p/s_u, the
 * node's forcing at T_k + j dT/m (j = 0..m) over s_f, conductor / iron / coil
 * flags (node touches such a cell) and (r - r_in)/(r_out - r_in) with r_in,
 * r_out the radii of the mesh's first and last node.  The weight blob is FP32
 * (the master copy; products use its bf16 rounding and accumulate in FP32):
 *   [s_u, s_f, s_out, 0], W_in[F][64], b_in[64],
 *   3 x {Ws[64][64], Wn[64][64], b[64]}, w_out[64], b_out[1].
 * Layer l: h_l = h_{l-1} + tanh(h_{l-1} Ws + mean_neighbours(h_{l-1}) Wn + b);
 * h_0 = tanh(x W_in + b_in); delta = h_3 w_out + b_out. */
typedef struct {
  int32_t n_traj;        /* trajectories generated (columns of one batched Phi)     */
  int32_t epochs;
  int32_t batch;         /* samples per Adam step                                    */
  double  lr;            /* Adam rate (cosine decay to lr/10 over the run)           */
  double  amp_spread;    /* source amplitude factors uniform in [1 - s, 1 + s]       */
  double  val_fraction;  /* trajectories held out for validation                     */
  uint64_t seed;
  double  perturb;       /* at every coarse step each trajectory's state moves towards a
                          * random other trajectory's by a factor uniform in
                          * [-perturb, perturb] before the pair is taken (0 = none)  */
} mgrit_train_params;

typedef struct {
  int64_t n_train, n_val;   /* (u_k, u_{k+1}) pairs                                  */
  int64_t steps;            /* Adam steps                                            */
  double  loss_first, loss_last;  /* mean scaled squared error, first / last epoch   */
  /* sqrt(sum ||Psi(u_k) - u_{k+1}||^2 / sum ||u_{k+1} - u_k||^2) with Psi = implicit
   * Euler (ie) or the trained propagator (learned), on both sets */
  double  train_err_ie, train_err_learned, val_err_ie, val_err_learned;
  double  time_data_s, time_train_s;
} mgrit_train_stats;

/* Trains the learned coarse propagator of a hierarchy with two or more levels:
 * n_traj trajectories of the level above the coarsest (its own Phi, each with
 * a source amplitude factor and a phase shift drawn from seed), restricted to
 * the coarsest mesh every m steps, give the pairs (u_k, u_{k+1}); p = implicit
 * Euler on the coarsest level; loss = mean ((Psi - u_{k+1}) / s_out)^2; Adam
 * (beta 0.9 / 0.999, eps 1e-8) from Glorot-uniform weights with a zero output
 * layer.  Replaces the handle's weights.  Errors: INVALID_ARGUMENT, UNSUPPORTED. */
int mgrit_train_coarse(void* h, const mgrit_train_params* tp, mgrit_train_stats* ts);

/* Number of weights of the learned propagator (0 if the hierarchy has none). */
int64_t mgrit_coarse_n_params(void* h);
/* Copy a weight blob in (resets the Adam moments) or out; n must equal
 * mgrit_coarse_n_params; the three scales must be > 0. */
int mgrit_set_coarse_weights(void* h, const float* w, int64_t n);
int mgrit_get_coarse_weights(void* h, float* w, int64_t n);
/* Psi for B samples on the coarsest level, evaluated as inside MGRIT (FP64
 * activations: a FAS correction is a difference of two evaluations, and FP32
 * rounding of the inputs would turn differences below ~1e-7 of the state into
 * noise); training and mgrit_coarse_gradient use FP32 (host arrays, user node order):
 * u, p [B][n_c] (p = the implicit-Euler step of u), k[B] input coarse steps
 * (T_k = k dT), amp / dphi [B] source amplitude factors and phase shifts (NULL =
 * 1 and 0).  psi [B][n_c] out. */
int mgrit_coarse_apply(void* h, int32_t B, const int64_t* k, const double* amp, const double* dphi,
                       const double* u, const double* p, double* psi);
/* Loss (mean scaled squared error against y [B][n_c]) and its gradient with
 * respect to every weight (FP32, the scales get 0), same arguments. */
int mgrit_coarse_gradient(void* h, int32_t B, const int64_t* k, const double* amp,
                          const double* dphi, const double* u, const double* p, const double* y,
                          double* loss, float* grad);
/* One Adam step of the weights with a given gradient (moments kept between calls). */
int mgrit_coarse_adam(void* h, const float* grad, double lr);

void mgrit_destroy(void* h);
const char* mgrit_strerror(int status);
const char* mgrit_last_error(void* h);   /* NULL handle: last setup error */

#ifdef __cplusplus
}
#endif
#endif /* MGRIT_H */
