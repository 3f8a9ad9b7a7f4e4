/*
 * ads.h -- C-ABI of the MI355X (gfx950) alternating-direction isogeometric
 * wave solver.
 *
 * Method: Los, Behnoudfar, Paszynski, Calo, "Fast isogeometric solvers for
 * hyperbolic wave propagation problems" (arXiv:1911.08158).
 *   - P-wave problem u'' - Laplace(u) = f on the unit cube (Section 2),
 *     tensor-product B-splines, Newmark (beta = 1/4) implicit step whose
 *     left-hand side M + (tau^2/4) K is replaced by the Kronecker product of
 *     1D operators (M_d + (tau^2/4) K_d) (eq. pwave2).
 *   - Isotropic linear elasticity (Section 5): alternating-triangular
 *     decoupling (eq. decom, eq. pre, eq. corr) with a direction split of
 *     every diagonal block (eq. spill), i.e. the three-level scheme eq. gen.
 *   - Every split operator is inverted by three sets of 1D banded solves,
 *     along x-lines, then y-lines, then z-lines (Appendix).
 *
 * Conventions (all functions):
 *   - Coefficient arrays exchanged through this ABI are FP64 DEVICE arrays on
 *     the FULL index set, n_x * n_y * n_z entries per component with
 *     n_d = nelem[d] + p, laid out [z][y][x] (x fastest); elasticity arrays
 *     hold the three components one after the other ([c][z][y][x]).
 *   - Boundary conditions (ads_params.bc): with ADS_BC_DIRICHLET0 the first
 *     and last basis function of every direction are eliminated; boundary
 *     entries of input arrays are ignored and boundary entries of output
 *     arrays are written as 0.  With ADS_BC_NATURAL no function is
 *     eliminated and every entry is a degree of freedom.
 *   - The library never allocates device memory.  Every device byte it uses
 *     lives in the caller's workspace (size from ads_workspace_bytes); the
 *     caller keeps the workspace alive until ads_destroy and the stream is
 *     idle.  Input pointers are read during the call's enqueue only.
 *   - Work is enqueued on the HIP stream given to ads_create and is
 *     asynchronous unless a function says otherwise.  A NULL stream means the
 *     default stream.
 *   - Every function returns an ads_status; nothing throws or aborts across
 *     the ABI.  ads_last_error() gives a thread-local message for the last
 *     non-OK status.
 */
#ifndef ADS_H
#define ADS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADS_OK = 0,
  ADS_EINVAL = -1,   /* invalid argument (sizes, degree, tau, material, NULL) */
  ADS_ENOMEM = -2,   /* workspace too small / capacity exceeded             */
  ADS_EDEVICE = -3,  /* a HIP call failed                                    */
  ADS_ESTATE = -4,   /* call out of order (e.g. ads_step before ads_factor)   */
  ADS_ENUMERIC = -5  /* non-finite state detected                           */
} ads_status;

typedef enum { ADS_PWAVE = 0, ADS_ELASTIC = 1 } ads_problem;

/* Arithmetic of the right-hand side.  Without a wave-speed field it is the
 * Kronecker form of the stiffness (P-wave: eq. pwave2; elasticity: the
 * blocks of Upsilon, Section 5) over assembled 1D band matrices, three
 * band passes, HBM-bound (the default); with a field (P-wave), or when
 * ads_tune picks it, the sum-factorized Gauss quadrature.  In the Kronecker
 * form the mixed modes run the passes with stiffness-type bands (K, G, G^T)
 * in FP32 on differences formed in FP64; the mass passes, the
 * z-accumulation and the assembly stay FP64.  Sweeps, factors and the time
 * update are FP64 in every mode.  ADS_MIXED_BF16 (P-wave only, not
 * accepted by pools) contracts the predictor rounded to BF16, then a second
 * pass contracts the FP64 remainder and adds it (one correction step),
 * FP32 arithmetic in both: two right-hand-side launches per step. */
typedef enum {
  ADS_FP64 = 0,        /* FP64 band passes / sum-factorized quadrature       */
  ADS_MIXED_FP32 = 1,  /* FP32 contractions, FP64 combination and assembly   */
  ADS_MIXED_BF16 = 2   /* BF16 inputs + FP64-remainder correction pass       */
} ads_precision;

/* Boundary conditions on all six faces.  ADS_BC_NATURAL is the homogeneous
 * natural condition of the weak forms: zero normal derivative for the
 * P-wave (Section 2) and zero traction, sigma n = 0, for elasticity (the
 * traction-free condition of Section 5); the 1D mass, stiffness and mixed
 * matrices are then used on the full index set. */
typedef enum { ADS_BC_DIRICHLET0 = 0, ADS_BC_NATURAL = 1 } ads_bc;

/* Problem statement (Section 2 for the P-wave, Section 5 for elasticity):
 * unit cube, nelem[d] uniform elements per direction (x, y, z), spline
 * degree p with open uniform knots and maximal continuity C^{p-1}, nquad
 * Gauss points per element and direction (0 means p+1, exact for these
 * integrands; p+2 and p+3 give the same matrices up to rounding and are
 * taken by the Kronecker-form right-hand sides only: no wave-speed field,
 * no quadrature variant, not in pools), time step tau, density rho and Lame constants lambda, mu
 * (elasticity only; the P-wave has unit wave speed).  nelem[2] = 0 selects
 * the two-dimensional problem on the unit square, the setting of the paper's
 * exposition: the P-wave of Section 2 (K = K_x (x) M_y + M_x (x) K_y, split
 * left-hand side (M_x + eta K_x) (x) (M_y + eta K_y)), and elasticity in
 * plane strain, Section 5's 2D blocks (components x then y in the
 * predictor, y then x in the corrector), with the antiplane displacement
 * u_z as a third, decoupled component (it stays zero when it starts at
 * zero without load); the arrays have one z-layer (n_z = 1) and the
 * z-index of Gauss-point data runs over q points whose weights sum to 1. */
typedef struct {
  int32_t problem;     /* ads_problem   */
  int32_t nelem[3];    /* >= 1 each; nelem[2] = 0: two-dimensional */
  int32_t p;           /* 1 to 5 (the quadrature right-hand side, and with
                          it a wave-speed field, needs 2 or 3)          */
  int32_t nquad;       /* 0 (= p+1) or p+1 .. p+3 (above p+1: Kronecker
                          forms only, not in pools)                      */
  int32_t bc;          /* ads_bc        */
  int32_t precision;   /* ads_precision */
  double tau;          /* > 0           */
  double rho, lambda, mu;
} ads_params;

typedef struct ads_sim ads_sim;   /* opaque host handle owned by the library */

/* Workspace bytes needed by ads_create for these parameters (host-only;
 * ADS_EINVAL for invalid parameters). */
ads_status ads_workspace_bytes(const ads_params* prm, size_t* bytes);

/* Gauss points of direction d (0=x,1=y,2=z): nelem[d]*q physical abscissae in
 * element-major order, written to host memory.  These are the points at which
 * ads_project expects sampled data (host-only). */
ads_status ads_quad_points(const ads_params* prm, int32_t d, double* host_out);

/* Create a simulation.  dev_workspace: caller-owned device buffer of at least
 * ads_workspace_bytes (256-byte aligned).  dev_u0 / dev_v0: initial
 * displacement and velocity coefficients (full layout; NULL = zero).
 * Uploads basis tables and mass factors; synchronizes the stream before
 * returning.  *out receives the handle. */
ads_status ads_create(const ads_params* prm, void* dev_workspace, size_t bytes,
                      void* hip_stream, const double* dev_u0, const double* dev_v0,
                      ads_sim** out);

/* Isogeometric L2 projection (Appendix, last paragraph): coefficients u with
 * M u = b, b_i = int B_i g, for data g sampled at the Gauss points
 * (dev_vals: [(nelem_z q)][(nelem_y q)][(nelem_x q)] per component, component
 * count 1 or 3 as the problem).  Writes full-layout coefficients to
 * dev_coef.  dev_scratch must hold ads_project_scratch_bytes. */
ads_status ads_project_scratch_bytes(const ads_params* prm, size_t* bytes);
ads_status ads_project(ads_sim* sim, const double* dev_vals, double* dev_coef,
                       void* dev_scratch, size_t scratch_bytes);

/* The projection above with the library's own staging memory instead of
 * dev_scratch, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc);
 * it allocates nothing.  The staging memory is a static device array of
 * ADS_PROJECT_STATIC_BYTES per GPU, held until the process ends; ADS_ENOMEM
 * (nothing enqueued) when ads_project_scratch_bytes exceeds it (e.g. meshes
 * of 64^3 elements fit at p = 2 and 3, 128^3 does not).  Every call on one
 * GPU uses the same array: calls that overlap on one GPU (different
 * streams or threads) race and must be serialized by the caller.
 * Synchronizes the simulation's stream, like ads_project. */
#define ADS_PROJECT_STATIC_BYTES (64u << 20)
ads_status ads_project_static(ads_sim* sim, const double* dev_vals, double* dev_coef);

/* Load F(t_k) = amp[k] * b (Section 2 uses f_{n+1} in the step n -> n+1;
 * Section 5 uses f^n).  dev_b: load vector (full layout, per component);
 * host_amp[k], k = 0..namp-1, amplitude at t_k = k tau (0 beyond namp;
 * namp <= 4096). */
ads_status ads_set_load(ads_sim* sim, const double* dev_b, const double* host_amp,
                        int32_t namp);
/* Point load b_{ijk} = B_i(x_s) B_j(y_s) B_k(z_s) (P-wave; a delta tested
 * against the basis), amplitude as in ads_set_load. */
ads_status ads_set_point_load(ads_sim* sim, const double xs[3], const double* host_amp,
                              int32_t namp);

/* Factor the 1D banded operators for the current tau (banded LU without
 * pivoting, Appendix: O(n) per direction) and start the time stepping:
 * P-wave u''_0 = G^{-1}(F_0 - K u_0); elasticity U^{-1} = U^0 - tau V^0 + Z^0/2
 * with Z^0 = D^{-1} tau^2 (f^0 - Upsilon U^0).  Synchronizes the stream. */
ads_status ads_factor(ads_sim* sim);

/* Variable wave speed of the P-wave (before ads_factor): the stiffness of
 * the right-hand side becomes the Gauss quadrature of (c^2 grad B_i, grad w)
 * with dev_c2 = c^2 at every Gauss point, a device FP64 array laid out like
 * the data of ads_project ([z][y][x] over (E_z q) x (E_y q) x (E_x q)
 * points; NULL = c^2 = 1).  The direction-split left-hand side keeps the
 * constant c2ref (G = (x)_d (M_d + tau^2/4 c2ref K_d)), so the ADS step is a
 * preconditioned Newmark step; with c2ref >= max c^2 the discrete energy of
 * ads_energy stays conserved.  The library keeps the pointer: the caller
 * keeps the array alive and unchanged until ads_destroy.  ADS_EINVAL for
 * elasticity, a degree other than 2 or 3 (the quadrature kernels are
 * instantiated for those) or c2ref <= 0, ADS_ESTATE after ads_factor. */
ads_status ads_set_coefficient(ads_sim* sim, const double* dev_c2, double c2ref);

/* Time-stepping coefficient set of the P-wave (before ads_factor; default
 * ADS_SCHEME_NEWMARK).  ADS_SCHEME_NEWMARK is standard Newmark beta = 1/4,
 * gamma = 1/2 with the direction-split left-hand side (Section 2, eq. scheme
 * and eq. pwave2 read with the u''_n terms the printed equations drop).
 * ADS_SCHEME_LITERAL applies the coefficient set exactly as printed, a
 * diagnostic of that erratum: G a' = F - K(u + tau u'), u' += tau/2 a',
 * u += tau u' (old u'); it propagates waves at 1/sqrt(2) of the speed.
 * ADS_EINVAL for unknown schemes or elasticity; ADS_ESTATE after ads_factor. */
typedef enum { ADS_SCHEME_NEWMARK = 0, ADS_SCHEME_LITERAL = 1 } ads_scheme;
ads_status ads_set_scheme(ads_sim* sim, int32_t scheme);

/* Discrete energy of the current state (synchronous; one double written to
 * host memory).  P-wave:
 *   E = 1/2 u'.(G - tau^2/4 K) u' + 1/2 u.K u,
 * G the direction-split operator of eq. pwave2, K the stiffness (by FP64
 * quadrature).  Elasticity, with V = (U^n - U^{n-1})/tau and
 * W = (U^n + U^{n-1})/2:
 *   E = 1/2 V.(D - tau^2/4 Upsilon) V + 1/2 W.Upsilon W,
 * D = L (rho M)^{-1} L^T the alternating-triangular operator of eq. pre /
 * eq. corr with the split diagonal blocks of eq. spill.  Without load both
 * are constant from the first step on: the energy counterpart of the
 * stability discussion of Sections 3 and 6 (the paper's energy plots).
 * Uses the simulation's scratch fields (between steps only).  ADS_ESTATE
 * before ads_factor. */
ads_status ads_energy(ads_sim* sim, double* host_energy);

/* Advance nsteps time steps (asynchronous).  ADS_ESTATE before ads_factor.
 * P-wave: the steps advance (w, b, u''), w = u + tau u' + tau^2/4 u'' the
 * predictor of the next step and b = u' + tau/2 u'' the half-step velocity
 * (ADS_SCHEME_LITERAL: (w, u', u''), w = u + tau u'), so that each step's
 * right-hand side reads one field and its update two: with the solved
 * u''_{n+1}, the z-sweep forms w_{n+1} = w_n + tau b_n + tau^2 u''_{n+1} and
 * b_{n+1} = b_n + tau u''_{n+1} (the Newmark update of u and u' written in
 * these fields).  u and u' are formed from (w, b, u'') when they are read
 * (ads_get_state, ads_energy, ads_check_finite), w and b from (u, u', u'')
 * when the state is set. */
ads_status ads_step(ads_sim* sim, int32_t nsteps);

/* Autotuner of the right-hand side (measurement-driven): times every
 * variant on this mesh (HIP events, a few launches each; synchronizes) and
 * keeps the fastest.  P-wave: 0-2 are tile shapes of the quadrature kernel,
 * 3 is the Kronecker form (the default; not offered with a wave-speed
 * field), 4 the quadrature with its x-contractions on the matrix cores
 * (FP32 MFMA; offered in the mixed modes with a wave-speed field only,
 * elsewhere it runs as 0).  Elasticity: 0 is the quadrature (FP64), 3 the Kronecker form
 * (the default); for elasticity it then times the two forms of the
 * couplings (ads_set_coupling).  Then, per direction, it times the tile widths 4, 8 and 16
 * lines per wave of the step's sweeps (on copies of their jobs that solve in
 * place with a plain store: only the step's temporaries change, the state
 * does not) and keeps the fastest.  The choices are cached per (problem,
 * degree, precision, field or none, mesh) for later simulations in the
 * process.  *chosen
 * receives the variant index, host_ms[v] (may be NULL; entries v < cap) the
 * mean ms of variant v.  Call after ads_factor.  ADS_ESTATE for a
 * simulation owned by a pool (the pool chooses its launch shapes, see
 * ads_pool_tune). */
ads_status ads_tune(ads_sim* sim, int32_t* chosen, double* host_ms, int32_t cap);

/* Launch shapes of a simulation, set explicitly (measurement and tests; the
 * defaults and ads_tune choose them otherwise).  rhs_var: right-hand-side
 * variant as in ads_tune (-1 keeps the current one); rhs_tz: owned z-layers
 * per right-hand-side tile (0 = chosen from the occupancy, -1 keeps);
 * sweep_w (NULL keeps all): lines per wave tile of the x-, y- and z-sweeps
 * (4, 8 or 16; 0 = default, -1 keeps).  Results do not depend on the
 * shapes, except through the variant (the two right-hand-side forms round
 * differently).  ADS_EINVAL for a variant the problem or degree lacks or a
 * width that does not fit the LDS, ADS_ESTATE for a pooled simulation. */
ads_status ads_set_launch_shape(ads_sim* sim, int32_t rhs_var, int32_t rhs_tz, const int32_t* sweep_w);

/* Where the elasticity couplings of the alternating-triangular stages are
 * applied (eq. pre: -tau^2/2 Upsilon_ij Y_j, j < i; eq. corr: rho M Y_i -
 * tau^2/2 Upsilon_ij Z_j, j > i; five per step).  fused = 0 (the default):
 * by separate launches that write the coupled right-hand side to memory.
 * fused = 1: in the input stage of the in-plane (x, y) sweep of the solve
 * that consumes them, where a z-plane of at most 4,608 unknowns with its
 * work space fits the LDS (elsewhere by separate launches).  One workgroup
 * per z-plane then does the coupling's work, so the form pays only where
 * z-planes are many and small; ads_tune times both and keeps the faster.
 * The two forms round differently (z-band first, against x-band first).
 * ADS_EINVAL for a
 * P-wave simulation or fused not 0 or 1, ADS_ESTATE for a pooled
 * simulation.  ads_coupling_fused returns 1 when the step applies them in
 * the in-plane sweeps, else 0. */
ads_status ads_set_coupling(ads_sim* sim, int32_t fused);
int32_t ads_coupling_fused(const ads_sim* sim);

/* Copy the state out (full layout; asynchronous on the sim's stream).
 * P-wave: u, u', u'' (any pointer may be NULL).  Elasticity: U^n into dev_u,
 * U^{n-1} into dev_v, dev_a ignored. */
ads_status ads_get_state(ads_sim* sim, double* dev_u, double* dev_v, double* dev_a);
/* Replace the state (full layout) and the step index; the sim must be
 * re-factored (ads_factor) unless dev_a (P-wave) / dev_v = U^{n-1}
 * (elasticity) is given, in which case stepping can continue directly.
 * P-wave: u, u', u''; elasticity: U^n, U^{n-1}. */
ads_status ads_set_state(ads_sim* sim, const double* dev_u, const double* dev_v,
                         const double* dev_a, int64_t step);

/* Checkpoint: the time-stepping state itself (full layout; asynchronous on
 * the sim's stream), so that a restored simulation continues bitwise as the
 * original would (a round trip through ads_get_state / ads_set_state agrees
 * to rounding only, since the P-wave u and u' are formed from the stepping
 * state).
 * P-wave: dev_s0 = w = u + tau u' + tau^2/4 u'', dev_s1 = b = u' + tau/2 u''
 * (ADS_SCHEME_LITERAL: w = u + tau u', dev_s1 = u'), dev_s2 = u'';
 * elasticity: dev_s0 = U^n, dev_s1 = U^{n-1}, dev_s2 ignored.  Every
 * pointer but dev_s2 of
 * elasticity must be non-NULL.  Save: ADS_ESTATE before ads_factor.  Load
 * restores the state and the step index; stepping continues without
 * ads_factor if the sim was factored (the load may precede ads_factor). */
ads_status ads_checkpoint_save(ads_sim* sim, double* dev_s0, double* dev_s1, double* dev_s2);
ads_status ads_checkpoint_load(ads_sim* sim, const double* dev_s0, const double* dev_s1, const double* dev_s2,
                               int64_t step);

/* Step index (number of steps taken since the start). Synchronizes. */
ads_status ads_get_step(ads_sim* sim, int64_t* step);

/* Health check: synchronizes and returns ADS_ENUMERIC if the state holds a
 * non-finite value (NaN/Inf), ADS_OK otherwise.  Uses the workspace's
 * counter slot; not for use under graph capture. */
ads_status ads_check_finite(ads_sim* sim);

/* Kernel timing with HIP events recorded on the sim's stream around every
 * kernel that ads_step enqueues (measurement support; not part of the
 * method).  ads_profile(sim, 1) enables recording for subsequent ads_step
 * calls; ads_profile_read synchronizes and returns, for each kernel position
 * of one time step (in launch order), its mean duration in ms over the
 * recorded steps (host_ms, up to cap entries) and its kind (host_kind:
 * 0 = right-hand side, 1 = x-sweep, 2 = y-sweep, 3 = z-sweep, 4 = coupling
 * apply, 6 = x- and y-sweeps of every z-plane in one launch, used when a
 * plane fits in the 160 KiB LDS), plus the per-step durations in ms
 * (host_step_ms, up to step_cap
 * entries; *nsteps receives the count).  Reading resets the record. */
ads_status ads_profile(ads_sim* sim, int32_t enable);
ads_status ads_profile_read(ads_sim* sim, double* host_ms, int32_t* host_kind, int32_t cap,
                            int32_t* nlaunch, double* host_step_ms, int32_t step_cap,
                            int32_t* nsteps);

/* Release the host handle (and its timing events).  The caller frees the
 * workspace after the stream is idle. */
ads_status ads_destroy(ads_sim* sim);

/* Thread-local message of the last non-OK status (never NULL). */
const char* ads_last_error(void);

/* ------------------------------------------------------------------------
 * Batched pool (serving form; not a construct of the paper).  Many
 * simulations of different meshes, degrees (1 to 5), problems and precisions
 * live in one caller workspace and advance together: every pool step runs
 * ONE launch per kernel class and stage for all active simulations
 * (persistent kernels over device job tables), replayed from a hipGraph
 * captured once; the job tables are rewritten between replays when the
 * batch changes.  Results are bitwise identical to running each simulation
 * alone (per-output arithmetic does not depend on tiling or batching).
 * Limits: at most 128 free coefficients per direction in pooled
 * simulations; max_slots <= 256.
 * ------------------------------------------------------------------------ */
typedef struct ads_pool ads_pool;

/* Workspace: caller-owned device buffer (256-byte aligned) from which the
 * pool carves its job tables and every admitted simulation's workspace.
 * use_graph = 0 enqueues the launches directly instead of replaying. */
ads_status ads_pool_create(void* dev_workspace, size_t bytes, int32_t max_slots, void* hip_stream,
                           int32_t use_graph, ads_pool** out);
/* Admission by memory: carves a simulation for prm from the pool
 * workspace, with initial coefficients dev_u0 / dev_v0 as in ads_create
 * (full layout; NULL = zero); ADS_ENOMEM when no slot or not enough
 * contiguous bytes are free right now (try again after a retirement).  The
 * new slot is inactive: configure it through ads_pool_sim (ads_project,
 * ads_set_state, ads_set_load, ads_factor), then ads_pool_activate. */
ads_status ads_pool_admit(ads_pool* pool, const ads_params* prm, const double* dev_u0, const double* dev_v0,
                          int32_t* slot);
ads_status ads_pool_sim(ads_pool* pool, int32_t slot, ads_sim** sim);
/* Join the batch from the next pool step (the simulation must be factored). */
ads_status ads_pool_activate(ads_pool* pool, int32_t slot);
/* Advance every active simulation by nsteps steps (asynchronous).  The
 * active simulations are split into two branches of about equal unknowns
 * (largest first, each to the branch with fewer so far) whose launch
 * sequences run concurrently: the second branch on a stream of the pool's
 * own, forked from the pool's stream by an event at the start of a step and
 * joined back into it at its end, so that one branch's latency-bound
 * stages overlap the other's bandwidth-bound ones (a captured graph holds
 * the two chains).  Each simulation's launches stay in order on one
 * stream; the results are the same bits with one branch or two. */
ads_status ads_pool_step(ads_pool* pool, int32_t nsteps);
/* Number of concurrent branches of the following steps: 2 (the default) or
 * 1 (every launch class of the batch in one launch on the pool's stream).
 * Profiled steps (ads_pool_profile) use one.  ADS_EINVAL otherwise. */
ads_status ads_pool_set_branches(ads_pool* pool, int32_t n);
/* Leave the batch and release the slot's memory.  dev_u, dev_v, dev_a
 * (each may be NULL) receive the final state as ads_get_state gives it
 * (P-wave u, u', u''; elasticity U^n, U^{n-1}, dev_a ignored), copied on the
 * pool's stream before the release; the release is stream-ordered, so
 * later admissions reuse the memory after the copies. */
ads_status ads_pool_retire(ads_pool* pool, int32_t slot, double* dev_u, double* dev_v, double* dev_a);
/* Durations (ms) of the pool steps since the last call (synchronizes); at
 * most 65536 steps are timed between two calls, later ones are not. */
ads_status ads_pool_step_times(ads_pool* pool, double* host_ms, int32_t cap, int32_t* n);
/* Autotuner of the pool's launch shapes for the current batch (measurement-
 * driven; synchronizes): every P-wave right-hand-side class (degrees 2, 3)
 * times the quadrature tile variants, without a wave-speed field the
 * Kronecker form, and in mixed mode with one the MFMA x-stage (variant 4),
 * on the batch's own jobs; every sweep class times tile
 * widths of 4, 8 and 16 lines per wave (on a copy of its jobs that solves
 * in place with a plain store, so that no state changes); with elasticity
 * in the batch, the two forms of the couplings (ads_set_coupling) over the
 * batch's coupling and in-plane launches, for every pooled elasticity
 * simulation at once.  Each class keeps
 * its fastest shape; the choices are cached per class and batch shape and
 * the graph is captured again at the next step.  *nchanged receives the
 * number of classes (and 1 for the coupling form) whose shape changed; host_shape (may be NULL; cap
 * entries, launch positions as in ads_pool_profile_read) the shape of each
 * launch: right-hand sides their variant, sweeps their tile width, other
 * launches 0, launches with no simulation in the batch -1. */
ads_status ads_pool_tune(ads_pool* pool, int32_t* nchanged, int32_t* host_shape, int32_t cap);
/* Kernel timing of pool steps (measurement support): with enable = 1 the
 * following ads_pool_step calls enqueue the launches directly (no graph)
 * with HIP events around each; ads_pool_profile_read synchronizes and
 * returns the mean ms per launch position of one pool step over the
 * recorded steps (-1 for a class with no simulation in the batch, which is
 * not launched), its kind (0 = P-wave right-hand side, 5 = elasticity
 * right-hand side, 6 = x- and y-sweeps of the z-planes, 3 = z-sweeps,
 * 4 = coupling apply), degree and
 * mixed flag (host arrays of cap entries), and resets the record. */
ads_status ads_pool_profile(ads_pool* pool, int32_t enable);
ads_status ads_pool_profile_read(ads_pool* pool, double* host_ms, int32_t* host_kind, int32_t* host_p,
                                 int32_t* host_mixed, int32_t cap, int32_t* nlaunch);
/* Active slots and workspace bytes in use / free. */
ads_status ads_pool_info(ads_pool* pool, int32_t* active, size_t* used_bytes, size_t* free_bytes);
ads_status ads_pool_destroy(ads_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* ADS_H */
