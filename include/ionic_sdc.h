/*
 * ionic_sdc.h -- C ABI of the MI355X reaction + SDC library (libionic_sdc.so).
 *
 * What it computes.  The per-vertex ODE stage of the partitioned bidomain
 * strategy with spectral deferred correction (paper section 3.3.2): with the
 * extracellular coupling held fixed over a step (here: a fixed per-vertex
 * diffusion current I_diff), every mesh vertex carries the state
 * X = (v, w, c) of equation genODE and integrates dX/dt = F(X) with M~ = I,
 *     F = [ -(I_ion + I_stim) + I_diff ; G(v, w) ; S(v, w, c) ]
 * (equations parabolic, odes_con, odes).  One time step runs a predictor
 * over the M Gauss-Lobatto sub-intervals -- backward Euler by local Newton,
 * or the paper's Rosenbrock method ROS2 (section 3.3.1, equation
 * rb_system) -- and K linearised implicit corrections (equations residual,
 * sdc_ode, sdc; M = 2, K = 1 is the paper's trapezoidal correction).  With
 * ROS2 the step size can also be chosen adaptively from its embedded
 * solution (reaction_sdc_adaptive).  The
 * local Jacobian uses exact derivatives (text after equation rb_system) and a
 * sparsity fixed at compile time (the paper's CTSM technique).
 *
 * Conventions shared by every entry point.
 *  - Every function returns an int status: IONIC_OK (0) or a negative
 *    IONIC_E* code; ionic_last_error() gives a message (thread-local).  No
 *    C++ exception crosses the ABI.  Invalid arguments are rejected before
 *    any HIP call is made.
 *  - Units: V in mV, t in ms, currents in uA/cm^2 (= pA/pF with
 *    C_m = 1 uF/cm^2 in the voltage equation), concentrations in mM.
 *    I_stim follows the cell-model convention dV/dt = -(I_ion + I_stim), so a
 *    negative amplitude depolarises (the paper's +100 uA/cm^2 is -100 here).
 *  - Device pointers are HIP device addresses on the current device; the
 *    caller owns them and keeps them alive until the work that uses them has
 *    completed on the stream.  `hip_stream` is a hipStream_t passed as
 *    void* (NULL = the null stream).  Work is enqueued asynchronously unless
 *    a function says it synchronises.
 *  - State layout in HBM ("SoA planes"): plane i holds state i of all
 *    vertices, planes in the order of ionic_state_name(model, i).  A plane
 *    has ionic_plane_stride(n) elements (n rounded up to a multiple of 64).
 *    IONIC_FP64: every plane is double.  IONIC_MIXED: the first
 *    ionic_n_fp64_states(model) planes (V and the intracellular
 *    concentrations) are double and the remaining ones (gates) are float.
 *  - A handle is not thread-safe; different handles may be used
 *    concurrently on different streams.
 */
#ifndef IONIC_SDC_H
#define IONIC_SDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cell models (paper section 2).  IONIC_LR91: Luo-Rudy 1991, 8 states, with
 * the paper's modified conductances G_si = 0.02, G_Na = 4.0, G_K = 0.423
 * (section 4) unless params override them.  IONIC_TT06_EPI: ten Tusscher-
 * Panfilov 2006 epicardial cell, 19 states.  The two test models are scalar
 * problems with closed forms used to check the SDC machinery:
 * IONIC_TEST_LINEAR y' = lam*y + b + I_diff (params lam, b) and
 * IONIC_TEST_LOGISTIC y' = rate*y*(1-y) + I_diff (param rate). */
enum { IONIC_LR91 = 1, IONIC_TT06_EPI = 2, IONIC_TEST_LINEAR = 90, IONIC_TEST_LOGISTIC = 91 };

/* IONIC_FP64: everything in double.  IONIC_MIXED: F, J and the sparse solve
 * in float; V, the intracellular concentrations, the SDC residual and their
 * updates in double; gates stored and updated in float. */
enum { IONIC_FP64 = 0, IONIC_MIXED = 1 };

enum {
  IONIC_OK = 0,
  IONIC_EINVAL = -1,       /* bad argument (null pointer, size, range)          */
  IONIC_EUNSUPPORTED = -2, /* model / precision / node count not built          */
  IONIC_EHIP = -3,         /* a HIP runtime call failed (message has the code)  */
  IONIC_ENOMEM = -4,       /* a library-internal allocation failed              */
  IONIC_ESTATE = -5        /* handle used in a wrong state (e.g. mixed batch)   */
};

/* Predictor on each Gauss-Lobatto sub-interval.  IONIC_PRED_NEWTON:
 * backward Euler Y - X_m - dtau F(Y) = 0 by local Newton (the first-order
 * implicit integrator of the correction equation, section 3.3.2).
 * IONIC_PRED_ROS2: one step of the two-stage, second-order, L-stable
 * Rosenbrock method ROS2 (section 3.3.1, equation rb_system) with
 * gamma = 1 + 1/sqrt(2), exact Jacobian, both stages on one factorisation.
 * IONIC_PRED_RUSH_LARSEN: the gating states (every state after the
 * ionic_n_fp64_states core: gates, and for TT06 fCass and Rbar) take the
 * exponential step g + dtau F_g (e^z - 1)/z, z = dtau dF_g/dg, at frozen X_m
 * (exact for their rows, which are linear in the state itself); then
 * backward Euler by local Newton on the core alone with the gates held, with
 * the same stop rule as IONIC_PRED_NEWTON.  Without gating states it equals
 * IONIC_PRED_NEWTON. */
enum { IONIC_PRED_NEWTON = 0, IONIC_PRED_ROS2 = 1, IONIC_PRED_RUSH_LARSEN = 2 };

#define IONIC_MAX_NODES 5   /* Gauss-Lobatto nodes per step: 2..5 */
#define IONIC_MAX_SWEEPS 16 /* SDC corrections per step: 0..16   */

typedef struct ionic_sim ionic_sim; /* opaque, owned by the library */

typedef struct {
  int64_t n_vertices;   /* N >= 1 */
  int32_t model;        /* IONIC_LR91, ... */
  int32_t precision;    /* IONIC_FP64 or IONIC_MIXED */
  double newton_tol;    /* predictor stop: max_i |delta_i|/max(|Y_i|, scale_i) <= tol; >= 0.
                           IONIC_MIXED uses max(tol, 1e-6): an fp32 F cannot resolve less. */
  int32_t newton_maxit; /* 1..64; the last iterate is kept and counted when reached */
  int32_t n_params;     /* number of entries in params (0 = defaults) */
  const double* params; /* host; overrides of the model's leading parameters, see
                           ionic_param_name(); NULL/0 = defaults */
} ionic_config;

/* A structured grid of nodes for the diffusion current (paper section 3.1:
 * Q1 elements on quadrilaterals / hexahedra).  Vertex index i + nx*(j + ny*k),
 * x fastest; nx*ny*nz must equal the simulation's vertex count and be below
 * 2^31; an extent of 1 drops that direction (1D cables, 2D sheets).  h: node
 * spacing in cm, uniform.  sigma: the conductivity in the voltage equation, cm^2/ms (for the
 * paper's bidomain with sigma_e = lambda sigma_i this is the monodomain
 * sigma_i sigma_e/(sigma_i + sigma_e): the elliptic solve then gives
 * -A_i v - A_i u = -(lambda/(1+lambda)) A_i v exactly; 0.75e-3 for
 * sigma_i = sigma_e = 1.5e-3). */
typedef struct {
  int64_t nx, ny, nz;
  double h;
  double sigma;
} ionic_grid;

/* A structured grid with the two conductivity tensors of the bidomain model
 * (diagonal and constant in space, as in paper section 2; section 4 uses
 * 1.5e-3 for every entry).  Same node layout
 * and limits as ionic_grid.  Conductivities in cm^2/ms, per direction x, y, z. */
typedef struct {
  int64_t nx, ny, nz;
  double h;
  double sigma_i[3];
  double sigma_e[3];
} ionic_bidomain_grid;

/* Outcome of an elliptic solve. */
typedef struct {
  int64_t cg_iterations;      /* iterations of the last solve (summed over steps
                                 by reaction_bidomain_step)                        */
  double relative_residual;   /* ||b - A_ie u|| / ||b|| of the last solve            */
  int32_t converged;          /* 1 iff every solve reached rtol                      */
  int32_t reserved;
} ionic_elliptic_info;

/* Outcome of reaction_bidomain_implicit_step (sums over the steps of the call). */
typedef struct {
  int64_t steps;              /* time steps taken                                       */
  int64_t inner_passes;       /* passes of Algorithm 2's inner loop, summed               */
  int64_t cg_iterations;      /* elliptic CG iterations, summed                          */
  int64_t krylov_iterations;  /* BiCGSTAB iterations of the stage and correction systems */
  double last_change;         /* scaled change of the last pass of the last step          */
  int32_t inner_max;          /* most passes in one step                                 */
  int32_t converged;          /* 1 iff every step met inner_tol within max_inner          */
  int32_t krylov_max;         /* most BiCGSTAB iterations of one solve                   */
  int32_t krylov_converged;   /* 1 iff every BiCGSTAB solve met krylov_rtol              */
} ionic_implicit_info;

/* Outcome of reaction_sdc_adaptive. */
typedef struct {
  double t;            /* time reached (ms); equals t_end when reached == 1       */
  double dt_next;      /* step the controller proposes next                      */
  double err_last;     /* scaled embedded error of the last attempt (inf: non-finite) */
  int64_t accepted;    /* accepted attempts                                      */
  int64_t rejected;    /* rejected attempts                                      */
  int32_t reached;     /* 1 iff t_end was reached                                */
  int32_t failed;      /* 1 iff the run stopped early: attempts exhausted, or the
                          step fell below 1e-12 ms                               */
} ionic_adapt_result;

typedef struct {
  int64_t vertex_steps;      /* sum over launches of N * n_steps                  */
  int64_t newton_iters;      /* Newton iterations summed over vertices and nodes  */
  int64_t newton_solves;     /* predictor solves (vertices x steps x (M-1))       */
  int64_t n_nonconverged;    /* predictor solves that stopped at newton_maxit     */
  int64_t n_nonfinite;       /* vertices whose state was non-finite after a launch */
  int32_t newton_it_max;     /* largest iteration count of one solve              */
  int32_t reserved;
} ionic_stats;

/* ---- model description (host only; no GPU needed) ------------------------ */

/* Number of states of `model` (8, 19, 1, 1), or IONIC_EUNSUPPORTED. */
int ionic_n_states(int model);

/* Number of leading planes kept in double under IONIC_MIXED (2 for LR91: V, Cai;
 * 6 for TT06: V, Cai, CaSR, CaSS, Nai, Ki; 1 for the test models). */
int ionic_n_fp64_states(int model);

/* Name of state `idx` ("V", "Cai", ...), i.e. the plane order; NULL if out of range. */
const char* ionic_state_name(int model, int idx);

/* Number of overridable parameters and the name of parameter `idx`. */
int ionic_n_params(int model);
const char* ionic_param_name(int model, int idx);

/* Elements per plane for N vertices: N rounded up to a multiple of 64. */
int64_t ionic_plane_stride(int64_t n_vertices);

/* Bytes of device memory the caller must provide for the state of N vertices;
 * 0 for an unknown model/precision or N < 1. */
size_t ionic_state_bytes(int model, int precision, int64_t n_vertices);

/* Gauss-Lobatto nodes c[0..M-1] on [0, 1] and the integration matrix
 * S[m*M + j] = integral_{c_m}^{c_{m+1}} l_j(s) ds (m < M-1), l_j the Lagrange
 * basis of node j.  M = 2 gives the trapezoid [1/2, 1/2] of equation sdc.
 * Host only.  c needs M doubles, S needs (M-1)*M; either may be NULL. */
int ionic_lobatto(int n_nodes, double* c, double* S);

/* ---- lifetime -------------------------------------------------------------- */

/* Create a simulation over a caller-owned device buffer `state_dev` of
 * `state_bytes` >= ionic_state_bytes(...) bytes (it must outlive the handle)
 * and load the initial state X = (v, w, c) of every vertex (section 3.3,
 * equation genODE).
 *  x0: n_states x N doubles, row i = state i of every vertex (FP64 SoA,
 *      plane order), on the host (x0_on_device = 0) or on the device (1); it
 *      is converted into the precision layout on the GPU.
 *  x0 = NULL: every vertex starts at the model's resting state.  LR91: the
 *      solution X* of F(X) = 0 without stimulus or diffusion current, found
 *      on the GPU by Newton's method from V = -84 mV, [Ca]_i = 2e-4 mM and
 *      every gate at its steady state there.  TT06: the epicardial initial
 *      conditions printed with the model's publication (the model conserves
 *      charge, so F(X) = 0 has a one-parameter family of solutions; those
 *      conditions are the quiescent state of a paced cell).  Test models:
 *      y = 0.
 * Host x0: the call synchronises hip_stream before returning, so x0 may be
 * released afterwards; under IONIC_MIXED it converts through a temporary
 * device buffer (allocated and freed here, which waits for the device).
 * Device x0 or NULL: asynchronous, nothing is allocated once a destroyed
 * handle's statistics block can be reused; a device x0 must stay valid
 * until the work enqueued on hip_stream has run. */
int ionic_init(ionic_sim** out, const ionic_config* cfg, void* state_dev, size_t state_bytes,
               const double* x0, int x0_on_device, void* hip_stream);

/* Release the handle (not the state buffer).  Waits for the work the handle
 * has enqueued (on every stream it was given; after more than eight
 * distinct streams, for the device), then keeps its small statistics block
 * for the next ionic_init on the same device instead of freeing it.  NULL is
 * ignored. */
void ionic_destroy(ionic_sim* sim);

/* ---- the hot path ------------------------------------------------------------ */

/* Advance every vertex by n_steps steps of size dt (t_n = t0 + n*dt):
 * per step the predictor and n_sweeps corrections on n_nodes Gauss-Lobatto
 * nodes, all fused in one kernel launch with the state held in registers.
 *  i_stim_dev: N doubles (stimulus amplitude per vertex) or NULL (none);
 *              step n is stimulated iff stim_t_on <= t0 + (n + 1/2) dt < stim_t_off.
 *  i_diff_dev: N doubles, fixed diffusion current added to dV/dt, or NULL (0).
 * n_steps >= 0, dt > 0 and finite, 2 <= n_nodes <= IONIC_MAX_NODES,
 * 0 <= n_sweeps <= IONIC_MAX_SWEEPS.  Asynchronous.  Newton non-convergence
 * and non-finite states are not errors: they are counted in the stats. */
int reaction_sdc_step(ionic_sim* sim, double t0, double dt, int n_steps, int n_nodes,
                      int n_sweeps, const double* i_stim_dev, double stim_t_on,
                      double stim_t_off, const double* i_diff_dev, void* hip_stream);

/* Choose the predictor used by reaction_sdc_step and reaction_sdc_step_batch
 * on this handle (default IONIC_PRED_NEWTON).  With IONIC_PRED_ROS2 the
 * Newton settings of the config are unused and the Newton counters stay 0;
 * with IONIC_PRED_RUSH_LARSEN they count the core Newton iterations.
 * Host only; takes effect for work enqueued afterwards. */
int ionic_set_predictor(ionic_sim* sim, int predictor);

/* Processing order of the vertices in the mixed-precision step kernels
 * (reaction_sdc_step, reaction_sdc_step_batch, reaction_sdc_adaptive, and the
 * reaction steps of the diffusion and bidomain entries): lane slot k of the
 * launch advances vertex order_dev[k].  Every vertex computes exactly what it
 * computes in any other order (bit for bit) and the state stays in the
 * caller's vertex order in HBM; the order only decides which vertices share a
 * wavefront, and with it how far their Newton iteration counts differ (a
 * wavefront iterates until its last lane has converged).  On a structured
 * grid, blocks of 4 x 4 x 4 neighbouring vertices per wavefront keep a
 * depolarisation front inside few wavefronts.  IONIC_FP64 handles accept and
 * check the order but keep the identity mapping (no measurable gain there,
 * and the double kernels have no registers to spare for it); their results
 * are the same either way.
 *   order_dev: n int32 on the device, a permutation of [0, n) (checked here:
 *              copied to the host once; IONIC_EINVAL otherwise), caller-owned,
 *              read by every later launch, so it must outlive them; NULL
 *              restores the identity order.  n must equal the handle's vertex
 *              count.  Synchronises the device copy. */
int ionic_set_vertex_order(ionic_sim* sim, const int32_t* order_dev, int64_t n);

/* Adaptive time stepping from t0 to t_end with the ROS2 predictor and
 * n_sweeps corrections on n_nodes nodes (the paper's scheme: n_nodes = 2,
 * n_sweeps = 1), one step size for all vertices (section 3.3.1: the embedded
 * ROS2 solution chooses the next step; section 4: steps capped at dt_max).
 * Per attempt with step tau from t:
 *   err = max over vertices, sub-intervals and states of
 *         |X_i - X_hat_i| / max(|X_i|, scale_i)   (X_hat: embedded solution,
 *         scale_i: the per-state floor of the Newton stop);
 *   accepted iff err <= err_tol (a non-finite state rejects);
 *   next step tau * min(2, max(0.2, 0.9 sqrt(err_tol/err))), capped at dt_max.
 * Steps never cross the breakpoints stim_t_on, stim_t_off and t_end: a step
 * that would reach one is cut to end there exactly.  The stimulus is on for a
 * step from t iff stim_t_on <= t + tau/2 < stim_t_off.  The controller runs on
 * the device, so attempts queue without host round trips; the host checks
 * progress between batches of attempts.
 *  work_dev: caller-owned device buffer of >= ionic_state_bytes(...) bytes,
 *            the second state buffer of accept/reject; on return the result
 *            is in the handle's own state buffer.
 *  max_attempts: >= 1, cap on accepted + rejected attempts.
 *  history_dev: device array of 4 * max_attempts doubles or NULL; row a holds
 *            (t, tau, err, accepted) of attempt a.
 *  out: host; filled on return.
 * t_end > t0, 0 < dt_init, 0 < dt_max, err_tol > 0, all finite.
 * Synchronises hip_stream before returning. */
int reaction_sdc_adaptive(ionic_sim* sim, double t0, double t_end, double dt_init, double dt_max,
                          double err_tol, int n_nodes, int n_sweeps, const double* i_stim_dev,
                          double stim_t_on, double stim_t_off, const double* i_diff_dev,
                          void* work_dev, size_t work_bytes, int64_t max_attempts,
                          double* history_dev, ionic_adapt_result* out, void* hip_stream);

/* Diffusion current of the current V field (section 3.1, equation
 * semi-parabolic with lumped mass): i_diff_dev[p] = -sigma (M_L^{-1} A v)_p,
 * A the unit-conductivity Q1 stiffness matrix, M_L the lumped mass,
 * homogeneous Neumann boundaries.  i_diff_dev: N doubles on the device.
 * Asynchronous. */
int ionic_diffusion_current(ionic_sim* sim, const ionic_grid* grid, double* i_diff_dev,
                            void* hip_stream);

/* Reaction-diffusion stepping: n_steps times, the diffusion current of the
 * V field at the start of the step (ionic_diffusion_current into
 * i_diff_work_dev, N doubles) is held over one reaction step (reaction_sdc_step
 * with the handle's predictor, t_n = t0 + n dt).  The diffusion term is thus
 * explicit in time, which is stable only for dt <= h^2 / (2 sigma) (the
 * largest eigenvalue of M_L^{-1} A on these grids is 4/h^2 in 1, 2 and 3
 * dimensions); larger steps are rejected with IONIC_EINVAL.  Asynchronous. */
int reaction_diffusion_step(ionic_sim* sim, const ionic_grid* grid, double t0, double dt,
                            int n_steps, int n_nodes, int n_sweeps, const double* i_stim_dev,
                            double stim_t_on, double stim_t_off, double* i_diff_work_dev,
                            void* hip_stream);

/* Levels of the multigrid hierarchy the elliptic solve uses on this grid
 * (fine level included), 0 when the grid is small enough for the Jacobi
 * preconditioner.  One preconditioner application (a V-cycle) on L levels
 * is 4 L - 3 kernel launches, 4 L - 7 of them on the coarse levels.  Host only. */
int ionic_multigrid_levels(int64_t nx, int64_t ny, int64_t nz);

/* Device bytes of the work buffer of ionic_elliptic_solve and
 * reaction_bidomain_step for this grid and iteration cap (0 on bad sizes). */
size_t ionic_elliptic_work_bytes(int64_t nx, int64_t ny, int64_t nz, int max_iter);

/* The elliptic equation of the partitioned step (section 3.1, equation
 * semi-elliptic; section 3.3.2, Algorithm 2, first box): A_ie u = -A_i v for
 * the current V field, A_i and A_ie the Q1 stiffness matrices of sigma_i and
 * sigma_i + sigma_e, homogeneous Neumann boundaries.  u_dev (N doubles,
 * device) holds the initial guess and receives the solution, whose
 * lumped-mass mean is set to zero.  Conjugate gradients preconditioned by one
 * geometric multigrid V-cycle on the grid's tensor-product hierarchy (Jacobi
 * for grids of at most 512 nodes) until ||b - A_ie u|| <= rtol ||b|| or
 * max_iter iterations
 * (not an error: info->converged = 0); info->cg_iterations is the first
 * iteration count that meets rtol (the test runs on the device after every
 * iteration).  Reductions in a fixed order, so the result is reproducible bit
 * for bit.  The paper uses BiCGSTAB with algebraic multigrid for this system.
 * The host forms the exact inverse of the coarsest level once per grid and
 * conductivities (kept in the handle).
 * work_dev: ionic_elliptic_work_bytes(...) bytes, not shared with a solve
 * running at the same time.  Synchronises hip_stream (the host reads the
 * device's convergence flag between batches of iteration launches). */
int ionic_elliptic_solve(ionic_sim* sim, const ionic_bidomain_grid* grid, double* u_dev,
                         void* work_dev, size_t work_bytes, double rtol, int max_iter,
                         ionic_elliptic_info* info, void* hip_stream);

/* Partitioned bidomain stepping, one pass of Algorithm 2 per time step: u
 * from ionic_elliptic_solve with the V field at the start of the step
 * (initial guess: u_dev in the first step, the previous solution in the
 * second, the linear extrapolation from the last two in the third, then the
 * quadratic extrapolation from the last three), the current
 * -M_L^{-1} A_i (v + u) into i_diff_work_dev (N doubles), held over one
 * reaction step with the handle's predictor.  The
 * parabolic term is explicit in time: dt <= h^2 / (2 max_k sigma_i,k) is
 * required (IONIC_EINVAL otherwise).  With sigma_e = lambda sigma_i this is
 * reaction_diffusion_step with the monodomain sigma.  u_dev ends with the u of
 * the last step.  info (may be NULL) sums the iterations over the steps.
 * Synchronises hip_stream. */
int reaction_bidomain_step(ionic_sim* sim, const ionic_bidomain_grid* grid, double t0, double dt,
                           int n_steps, int n_nodes, int n_sweeps, const double* i_stim_dev,
                           double stim_t_on, double stim_t_off, double* u_dev, void* work_dev,
                           size_t work_bytes, double rtol, int max_iter, double* i_diff_work_dev,
                           ionic_elliptic_info* info, void* hip_stream);

/* Device bytes of the work buffer of reaction_bidomain_implicit_step for this
 * model, grid and iteration cap (0 on bad arguments). */
size_t ionic_implicit_work_bytes(int model, int64_t nx, int64_t ny, int64_t nz, int max_iter);

/* Partitioned bidomain stepping as the paper states Algorithm 2 (section
 * 3.3.2, the partitioned strategy with SDC), the parabolic term implicit: per
 * time step t^n -> t^n + dt from (X^n, u^n), passes k = 0, 1, ... of
 *   1. u^{k+1} from A_ie u = -A_i v^k (as ionic_elliptic_solve; v^0 = v^n);
 *   2. one ROS2 step (section 3.3.1, equation rb_system) from X^n of
 *      dX/dt = G(X; u^{k+1}), G the cell right-hand side with the current
 *      -M_L^{-1} A_i (v + u) in the voltage equation, whose Jacobian keeps
 *      -M_L^{-1} A_i v: both stages solve (I - gamma dt J_G(X^n)) k = ...;
 *   3. the correction of equation sdc: (I - dt J_G(X~)) eps =
 *      X^n - X~ + dt/2 (G(X^n; u^n) + G(X~; u^{k+1})), X^{k+1} = X~ + eps;
 *   4. stop once max_i |X^{k+1}_i - X^k_i| / max(|X^{k+1}_i|, s_i) <= inner_tol
 *      (s_i the Newton scale of each state) or after max_inner passes;
 * then X^{n+1} = X^{k+1}, u^{n+1} = u^{k+1}.  Each stage or correction system
 * couples the vertices through the v block only: every vertex's block is
 * eliminated onto V by the static sparse elimination, the remaining system
 * (S + c M_L^{-1} A_i) dv = r over the grid is solved by BiCGSTAB (the
 * paper's Krylov method) preconditioned by its diagonal to ||r|| <=
 * krylov_rtol ||b|| (b the reduced right-hand side), starting from the same
 * system's solution in the previous pass of the call (from zero in the
 * first pass), and each vertex's states follow from dv.  Any step
 * size is stable (dt = 0.05 ms at h = 0.01 cm, the paper's largest step, is
 * beyond reaction_bidomain_step's explicit limit).
 *  u_dev: N doubles, device: u^0 on entry (e.g. from ionic_elliptic_solve),
 *         the u of the last step on return.
 *  work_dev: ionic_implicit_work_bytes(model, nx, ny, nz, max_iter) bytes.
 *  max_iter: cap of every CG and BiCGSTAB solve (not an error when reached:
 *         info reports it).  Synchronises hip_stream (the host reads each
 *         pass's change).
 * IONIC_MIXED handles: the step runs on a double copy of the state (in the
 * work buffer), with F, J and the per-vertex eliminations in float and
 * everything else in double (the states, the right-hand sides including the
 * correction's residual, BiCGSTAB, the elliptic solve); the result is stored
 * back in the handle's layout.  inner_tol should then be >= 1e-6, the change
 * a float F resolves. */
int reaction_bidomain_implicit_step(ionic_sim* sim, const ionic_bidomain_grid* grid, double t0,
                                    double dt, int n_steps, const double* i_stim_dev,
                                    double stim_t_on, double stim_t_off, double* u_dev,
                                    void* work_dev, size_t work_bytes, double elliptic_rtol,
                                    double krylov_rtol, double inner_tol, int max_inner,
                                    int max_iter, ionic_implicit_info* info, void* hip_stream);

/* Store the step inputs of `sim` for reaction_sdc_step_batch (same meaning as
 * the arguments of reaction_sdc_step).  The batch advances the handle's own
 * step counter, so chunks of a long run keep t_n = t0 + n*dt exact. */
int ionic_set_inputs(ionic_sim* sim, double t0, double dt, int n_nodes, int n_sweeps,
                     const double* i_stim_dev, double stim_t_on, double stim_t_off,
                     const double* i_diff_dev);

/* Continuous-batching entry: advance n_sims handles by n_steps[i] steps each
 * in as few launches as possible (one per group of up to 24 handles).  All
 * handles must share model, precision, predictor, n_nodes, parameters and
 * Newton settings (else IONIC_ESTATE).  Each vertex computes exactly what a
 * reaction_sdc_step call on its own handle computes (bit-identical). */
int reaction_sdc_step_batch(ionic_sim* const* sims, const int* n_steps, int n_sims,
                            void* hip_stream);

/* Copy states of vertices [first, first+count) into out: n_states x count
 * doubles (row i = state i), on the host (out_on_device = 0) or the device.
 * Mixed layouts are widened to double on the GPU.  Synchronises hip_stream. */
int state_readback(ionic_sim* sim, double* out, int64_t first, int64_t count,
                   int out_on_device, void* hip_stream);

/* state_readback into a host buffer without allocating anything, for
 * callers that cannot allocate device memory (code that runs while a HIP
 * graph is being captured, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and synchronisation as
 * state_readback with out_on_device = 0 (out: n_states x count doubles on
 * the host, row i = state i).  The widened values are staged in a static
 * device array of 8 MiB that the library holds on every GPU it runs on until
 * the process ends: n_states * count * 8 bytes must not exceed 8 MiB (TT06:
 * 55,188 vertices; LR91: 131,072), else IONIC_EINVAL before any HIP call.
 * The current device must be the handle's.  All calls on one GPU share that
 * array, so calls that overlap in time on one GPU (other threads, other
 * streams) race; serialise them. */
int state_readback_noalloc(ionic_sim* sim, double* out, int64_t first, int64_t count,
                           void* hip_stream);

/* Set every voltage-dependent gate to its steady state at the vertex's
 * current V (TT06: fCass to its steady state at the current CaSS); other
 * states unchanged.  Builds initial fields such as spiral waves. Asynchronous. */
int ionic_gates_to_steady_state(ionic_sim* sim, void* hip_stream);

/* Cumulative statistics since init.  Both wait for the work the handle has
 * enqueued (the streams it was given), not for the whole device. */
int ionic_get_stats(ionic_sim* sim, ionic_stats* out);
int ionic_reset_stats(ionic_sim* sim);

/* Debug/test: F and the Jacobian at the current state of one vertex, evaluated
 * by the same device code as the hot path (float under IONIC_MIXED, widened).
 * F_out: n doubles, J_out: n*n doubles row-major (J[i*n+k] = dF_i/dX_k), host.
 * Entries outside the compile-time pattern are returned as 0.  Synchronises. */
int ionic_debug_jacobian(ionic_sim* sim, int64_t vertex, double i_stim, double i_diff,
                         double* F_out, double* J_out, void* hip_stream);

/* Message of the last failing call on this thread ("" if none). */
const char* ionic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IONIC_SDC_H */
