/*
 * pmgrit.h -- C ABI of the MI355X (gfx950) MGRIT + p-multigrid solver for isogeometric
 * discretisations of the heat equation.
 *
 * Method: Tielen, Moeller, Vuik, "Combining p-multigrid and multigrid reduced in time methods
 * to obtain a scalable solver for Isogeometric Analysis" (arXiv 2107.05337).
 *   - Problem: d_t u - kappa Lap u = f on Omega x [0,T], u(.,0) = u0, u = 0 on the boundary
 *     (Sec. 2, eq:heat), tensor-product B-splines of degree p on n x n elements of width
 *     h = 1/n with open uniform knot vectors (Sec. 2), the theta-scheme in time (implicit
 *     Euler by default), so every time step solves (M + theta kappa dt K) u^{k+1} =
 *     (M - (1 - theta) kappa dt K) u^k + dt f (Sec. 2, eq:los; Sec. 4).
 *   - Time parallelism: MGRIT with coarsening factor m, FCF-relaxation, injection of the
 *     C-point residual, rediscretised coarse levels dt_l = m^l dt and ideal interpolation
 *     (Sec. 3, eq:mgrit, eq:mgrit_coarse and the MGRIT recursion).
 *   - Spatial solves: p-multigrid V-cycles (Sec. 4, steps 1-5) with an ILUT smoother at
 *     degree p, direct restriction to p = 1 with the lumped-mass L2 transfers
 *     (Sec. 4, eq:prolongation, eq:PM) and at p = 1 an exact solve or the paper's one
 *     h-multigrid W-cycle; or, as the paper's comparison, Jacobi-preconditioned CG (Sec. 4).
 *
 * Conventions for every call:
 *   - Return value: PMGRIT_OK (0) or a negative pmgrit_status; no call aborts the process;
 *     pmgrit_last_error() returns a thread-local message about the last failure.
 *   - Output handles and host output arguments are left untouched on error.
 *   - Host structs passed by pointer are copied at the call; the caller keeps ownership.
 *   - Device pointers ("_dev") are device memory of the handle's GPU that the caller owns and
 *     keeps alive until the work enqueued on the given stream has completed.  Streams are
 *     hipStream_t passed as void* (NULL = the default stream).
 *   - The handle owns every factor, schedule and workspace; all of them are allocated in
 *     pmgrit_create, so the solve calls allocate nothing on the device.
 *   - A handle is not thread-safe; use one handle per host thread / stream.
 *   - Degrees of freedom: the interior tensor-product B-splines (the first and last function
 *     per direction carry the homogeneous Dirichlet condition and are removed), numbered
 *     lexicographically with the first parameter direction fastest: dof = iy * Nin + ix,
 *     Nin = n + p - 2.  A time trajectory is (N_t + 1) x n_dof doubles, time-major.
 */
#ifndef PMGRIT_H
#define PMGRIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMGRIT_OK = 0,
  PMGRIT_E_ARG = -1,            /* invalid argument or size */
  PMGRIT_E_HIP = -2,            /* a HIP runtime call failed (message in pmgrit_last_error) */
  PMGRIT_E_OOM = -3,            /* device or host allocation failed */
  PMGRIT_E_FACTOR = -4,         /* ILUT produced a non-positive or non-finite pivot */
  PMGRIT_E_SPATIAL_NOCONV = -5, /* a spatial solve hit max_vcycles before its tolerance */
  PMGRIT_E_MGRIT_NOCONV = -6,   /* MGRIT hit max_iter before its tolerance */
  PMGRIT_E_NONFINITE = -7,      /* NaN or Inf in a residual */
  PMGRIT_E_STATE = -8           /* call not valid for this handle (e.g. host-only handle) */
} pmgrit_status;

/* One problem instance (Sec. 2, eq:heat; Sec. 5 benchmark setting).
 * Time discretisation: the theta-scheme of Sec. 2 (eq:los), every step solving
 *   (M + theta kappa dt K) u^{k+1} = (M - (1 - theta) kappa dt K) u^k + w_k f,
 *   w_k = dt (theta tfac(t_{k+1}) + (1 - theta) tfac(t_k)),
 * theta = 1 implicit (backward) Euler, 1/2 Crank-Nicolson, 0 forward Euler (then M is the
 * operator the spatial solver inverts; stable only for small kappa dt / h^2 on every MGRIT level).
 * Coarse MGRIT levels rediscretise with the same theta and dt_l = m^l dt.
 * domain 0: unit square (F = identity).  domain 1: quarter annulus with radii 1 and 2, first
 * parameter direction radial, second the exact rational quadratic quarter circle.
 * Source f(x, t) = tfac(t) * sum_q amp_q m(k_q, s) m(l_q, t) in parameter coordinates (s, t)
 * with m(0, .) = 1 and m(k, s) = sin(k pi s) for k >= 1, set by pmgrit_set_source_modes. */
typedef struct {
  int32_t degree_p; /* B-spline degree p >= 2 (the p = 1 level is the coarse space) */
  int32_t n_elems;  /* n elements per direction, h = 1/n, n >= 2 */
  int32_t domain;   /* 0 unit square, 1 quarter annulus */
  double kappa;     /* diffusion coefficient > 0 */
  double T;         /* end time > 0 */
  int32_t n_steps;  /* N_t >= 1 */
  double theta;     /* theta-scheme parameter in [0, 1] (1 = implicit Euler; no default: a
                     * zero-initialised struct asks for forward Euler) */
} pmgrit_problem;

/* MGRIT hierarchy and stopping rule (Sec. 3; Sec. 5).  Level l has floor(N_t / m^l)
 * intervals of size m^l dt; coarsening stops at max_levels levels or as soon as a level has
 * at most coarsest_max intervals.  Converged when the level-0 C-point residual after
 * FCF-relaxation, in the Euclidean norm over all C-points and dofs, is <= tol times its value
 * in the first iteration. */
typedef struct {
  int32_t cfactor;      /* m >= 2 */
  int32_t max_levels;   /* >= 2 (2 = two-level MGRIT) */
  int32_t coarsest_max; /* stop coarsening at <= this many intervals (e.g. 8) */
  double tol;           /* relative residual, e.g. 1e-10 */
  int32_t max_iter;     /* MGRIT iteration cap */
  int32_t use_graph;    /* 1: capture one iteration (coarse correction and the next relaxation,
                         * kernels only) as a HIP graph per set of trajectory buffers and stream,
                         * and replay it; 0: launch every kernel */
  int32_t cycle;        /* cycle type of the coarse-level solves (Sec. 3): 0 V-cycle (one cycle
                         * per level), 1 W-cycle (two cycles per level), 2 F-cycle (an F-cycle
                         * followed by a V-cycle per level); the coarsest level is always solved
                         * by sequential time stepping, so with two levels all three coincide */
} pmgrit_mgrit_opts;

/* Spatial solver (Sec. 4).  precision 0: FP64 V-cycle.  precision 1: V-cycle in FP32 as the
 * preconditioner of FP64 iterative refinement (residual, update and the p = 1 solve in FP64).
 * guess: initial iterate of every spatial solve -- 0 zero, 1 previous time point,
 * 2 current value of the target point (MGRIT), 3 learned warm start: the network's prediction
 * from the previous point, or the previous point itself if its FP64 residual is smaller (needs
 * pmgrit_net_load before solving).  With guess 3, sequential stepping predicts every step;
 * MGRIT predicts the level-0 F- and C-relaxation steps of its first iteration, step by step, and
 * uses guess 2 afterwards.  In MGRIT only instances of at most 64 elements per direction are
 * predicted; the others take guess 2 throughout (there the previous point already needs as few
 * V-cycles as the prediction, and the network's cost grows with the grid).
 * trsv_block: row-block size of the blocked triangular solves (0 = blocks of 64 consecutive
 * rows, the default; 1 = plain row level-scheduling; -1 = one grid line per block, split evenly
 * above 72 rows; k >= 2 = blocks of k rows). */
typedef struct {
  int32_t nu1, nu2;       /* pre-/post-smoothing steps (>= 1) */
  double ilut_droptol;    /* ILUT drop tolerance tau (relative to the row 2-norm) */
  int32_t ilut_fill;      /* 0: at most as many entries per row of L / U as A has there */
  double spatial_tol;     /* stop when ||b - A x||_2 <= spatial_tol ||b||_2 */
  int32_t max_vcycles;    /* V-cycle cap per spatial solve */
  int32_t precision;      /* 0 FP64, 1 FP32 V-cycle inside FP64 refinement */
  int32_t guess;          /* 0 zero, 1 previous, 2 current target, 3 learned */
  int32_t trsv_block;     /* see above */
  int32_t autotune;       /* 1: at create, time candidate LDS placements of the work vectors per
                           * launch group on probe solves and keep the fastest (in precision 1
                           * also the two-workgroups-per-CU build where the plan fits half of
                           * the CU's LDS) */
  double coarse_tol;      /* spatial tolerance of the solves on MGRIT levels >= 1 (0: spatial_tol);
                           * those only supply corrections, so it changes the convergence rate,
                           * not the fixed point that the level-0 stop test measures */
  int32_t lds_mask;       /* 0: automatic (the largest LDS placement that fits, or the autotuner's
                           * choice).  Otherwise the placement of every launch group: bits 1 y,
                           * 2 d, 4 s, 8 x select the work vectors kept in LDS; 16 (precision 1
                           * with bit 1 and without 4 and 8) selects the kernel build for two
                           * workgroups per CU; 32 (with bit 1) the 1024-thread build and 64 (with
                           * bit 1, at most 64 rows per triangular-solve level) the 512-thread
                           * build, both with 8 lanes per triangular-solve row.  Results do not
                           * depend on bits 1-16; the 8-lane builds sum each triangular-solve row in
                           * another order (rounding only).  PMGRIT_E_ARG if it does not fit a
                           * group's LDS or its rows, or is combined with autotune. */
  int32_t solver;         /* spatial solver: 0 p-multigrid V-cycles (Sec. 4); 1 conjugate gradients
                           * preconditioned by diag(A) (the comparison solver of Sec. 4 and Sec. 5),
                           * FP64 only (precision 0), max_vcycles then caps the CG iterations */
  int32_t coarse;         /* p = 1 solve of the V-cycle (step 3 of Sec. 4): 0 exact (fast
                           * diagonalisation), 1 one h-multigrid W-cycle from zero (the paper's
                           * choice: four-colour Gauss-Seidel pre- and post-smoothing, canonical
                           * prolongation, restriction by its transpose, Galerkin coarse operators,
                           * meshes halved while the element count is even and above 4, the
                           * coarsest solved exactly) */
} pmgrit_solver_opts;

typedef struct {
  int32_t mgrit_iters;    /* coarse corrections applied until convergence */
  double res_hist[64];    /* relative level-0 residual after each FCF (res_hist[0] = 1) */
  int64_t phi_calls;      /* spatial solves performed (all levels, all instances) */
  int64_t vcycles;        /* V-cycles performed */
  double t_setup_s;       /* wall time of pmgrit_create */
  double t_solve_s;       /* wall time of the solve call, device-synchronised */
} pmgrit_stats;

typedef struct pmgrit_handle pmgrit_handle;

/* Create a solver for n_instances problems (several instances of uneven p, h, kappa and
 * domain are batched into the same launches).  Assembles M, K and the transfer operators on
 * the host, factors ILUT(M + kappa dt_l K) for every time level, builds the triangular-solve
 * schedules and the exact p = 1 solve data, and uploads everything to hip_device.
 * hip_device = -1 builds the host-side data only (for inspection; solve calls then return
 * PMGRIT_E_STATE).  All instances share one set of MGRIT and solver options. */
pmgrit_status pmgrit_create(int32_t n_instances, const pmgrit_problem* probs, const pmgrit_mgrit_opts* mopts,
                            const pmgrit_solver_opts* sopts, int32_t hip_device, pmgrit_handle** out);
void pmgrit_destroy(pmgrit_handle* h);

/* Sizes of instance inst: n_dof (degree p interior dofs), grid_n = n + p (functions per
 * direction incl. the boundary ones), n_levels of the MGRIT hierarchy. */
pmgrit_status pmgrit_dims(const pmgrit_handle* h, int32_t inst, int64_t* n_dof, int32_t* grid_n,
                          int32_t* n_levels);

/* Source of instance inst: n_modes separable modes (k[q], l[q], amp[q]) as described above,
 * with time factor time_kind 0: 1, 1: exp(-t).  The load vector int f Phi_i is assembled on
 * the host with the degree-p Gauss rule. */
pmgrit_status pmgrit_set_source_modes(pmgrit_handle* h, int32_t inst, int32_t n_modes, const int32_t* k,
                                      const int32_t* l, const double* amp, int32_t time_kind);

/* Initial condition of instance inst as the L2 projection (consistent mass) of a sum of
 * modes (Sec. 3: g^0 is u0 projected on the spline space).  n_modes = 0 gives u0 = 0. */
pmgrit_status pmgrit_set_initial_modes(pmgrit_handle* h, int32_t inst, int32_t n_modes, const int32_t* k,
                                       const int32_t* l, const double* amp);

/* Initial coefficients of instance inst from a host array of n_dof doubles. */
pmgrit_status pmgrit_set_initial_coeffs(pmgrit_handle* h, int32_t inst, const double* u0_host);

/* MGRIT solve of every instance (Sec. 3).  u_out_dev[i] is instance i's trajectory buffer of
 * (N_t + 1) x n_dof doubles on the device; on return (after the stream is synchronised by the
 * call) it holds the converged trajectory.  Each instance stops on its own criterion: once its
 * relative C-point residual reaches tol, its trajectory is kept as it is while the others
 * iterate, so a batched instance returns what a solve of it alone would (mgrit_iters and
 * res_hist describe the slowest instance).  stats may be NULL. */
pmgrit_status pmgrit_solve_mgrit(pmgrit_handle* h, void* hip_stream, double* const* u_out_dev, pmgrit_stats* stats);

/* Sequential implicit Euler with the same spatial solver (block forward solve of eq:mgrit);
 * same buffers as pmgrit_solve_mgrit. */
pmgrit_status pmgrit_solve_sequential(pmgrit_handle* h, void* hip_stream, double* const* u_out_dev,
                                      pmgrit_stats* stats);

/* One batched spatial solve at time level `level` of instance inst (Sec. 4): for each of the
 * nrhs right-hand sides j, solve (M + kappa dt_level K) x_j = b_j by p-multigrid V-cycles to
 * the spatial tolerance, starting from the guess in x_j.  b_dev and x_dev are nrhs x n_dof
 * doubles (right-hand side j contiguous), nrhs <= 4096.  vcycles_dev (nrhs int32, may be NULL)
 * receives the V-cycle count of each solve.  Asynchronous on hip_stream. */
pmgrit_status pmgrit_phi(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nrhs, const double* b_dev,
                         double* x_dev, int32_t* vcycles_dev, void* hip_stream);

/* pmgrit_phi for callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same solves, but the kernels' per-workgroup scratch (work
 * vectors that do not fit in LDS, the h-multigrid levels) lives in a fixed device array of 2^23
 * doubles (64 MiB) per GPU instead of the handle's buffer, and the call itself allocates nothing.
 * The array is part of the library's code object, held by each GPU the library runs on until the
 * process ends; its address is resolved once per device in pmgrit_create.  Every call on one GPU
 * shares that GPU's array (no contents are carried between calls): calls that overlap in time on one
 * GPU, from any handle or stream, race and must be ordered by the caller.  Errors: as pmgrit_phi,
 * and PMGRIT_E_ARG when nrhs times the instance's per-workgroup scratch (6 n_dof,max + 32 doubles
 * plus the h-multigrid levels with solver option coarse = 1) exceeds 2^23 doubles. */
pmgrit_status pmgrit_phi_noalloc(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nrhs, const double* b_dev,
                                 double* x_dev, int32_t* vcycles_dev, void* hip_stream);

/* Host-side inspection of the assembled data of instance inst (valid for every handle).
 * which: 0 M, 1 K, 2 A_level = M + kappa dt_level K, 3 L of ILUT(A_level) (strict lower),
 * 4 U of ILUT(A_level) (upper incl. diagonal), 5 P_1^p (interior, n_dof x n_dof1),
 * 6 M1, 7 K1 (degree 1 interior).  Call with rp = NULL to get shape3 = {rows, cols, nnz};
 * then with arrays of those sizes.  Doubles are the FP64 values. */
pmgrit_status pmgrit_host_matrix(const pmgrit_handle* h, int32_t inst, int32_t level, int32_t which,
                                 int32_t* shape3, int32_t* rp, int32_t* ci, double* v);

/* Host-side inspection: lumped masses (n_dof and n_dof1 doubles), load vector (n_dof) and
 * initial coefficients (n_dof) of instance inst; NULL pointers are skipped. */
pmgrit_status pmgrit_host_vectors(const pmgrit_handle* h, int32_t inst, double* mlp, double* ml1, double* load,
                                  double* u0);

/* Host-side inspection of the triangular-solve schedule of ILUT factor `factor` (0 L, 1 U) at
 * `level`: out4 = {levels, blocks, block_size, max_rows_per_level}. */
pmgrit_status pmgrit_host_schedule(const pmgrit_handle* h, int32_t inst, int32_t level, int32_t factor,
                                   int32_t* out4);

/* Exact p = 1 solve on the host with the library's fast-diagonalisation data of `level`:
 * x = (M1 + kappa dt_level K1)^{-1} b, both n_dof1 doubles (host).  For testing the setup. */
pmgrit_status pmgrit_host_coarse_solve(const pmgrit_handle* h, int32_t inst, int32_t level, const double* b,
                                       double* x);

/* Learned warm start (not part of the paper).  A 4-layer 3x3 convolutional network over the
 * G x G tensor-product coefficient grid (G = n + p, the Dirichlet ring included) with channels
 * 3 -> 32 -> 32 -> 32 -> 1, zero padding and ReLU after the first three layers.  Input planes of a
 * sample (step k -> k + 1 of an instance, time level l): u_k / s_u; e / s_e with
 * e = (w F - kappa dt_l K u_k) / m, the residual of the step's equation at the previous point divided by
 * the row-sum-lumped mass m (w: the step's source weight, dt_l at coarse levels); and
 * ln(kappa dt_l n^2) / 4; s_u = rms(u_k), s_e = rms(e) over the interior (1 if zero).  Output y: guess
 * u_{k+1} = u_k + s_e y on the interior; training target t = (u_{k+1} - u_k) / s_e; loss = mean over
 * samples and interior points of (y - t)^2.
 * Weights, inputs and hidden activations (and hidden gradients) are BF16 with FP32 accumulation.
 * Parameters: a flat float array, per layer weights [cout][cin][3][3] then bias [cout]
 * (pmgrit_net_nparams() floats, FP32 master copy).  A handle holds one network. */
int64_t pmgrit_net_nparams(void);

/* Load (and reset the optimiser state) / save the parameters.  Errors: PMGRIT_E_ARG when n is not
 * pmgrit_net_nparams() or a pointer is NULL, PMGRIT_E_STATE for a host-only handle or (save) no
 * network loaded. */
pmgrit_status pmgrit_net_load(pmgrit_handle* h, const float* weights_host, int64_t n);
pmgrit_status pmgrit_net_save(const pmgrit_handle* h, float* weights_host, int64_t n);

/* Network inference on given planes: x_dev (nb x 3 x G x G float, device) -> y_dev (nb x G x G
 * float, device), asynchronous on hip_stream.  3 <= G <= 1024, 1 <= nb. */
pmgrit_status pmgrit_net_forward(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, float* y_dev,
                                 void* hip_stream);

/* Loss and gradient for given planes and targets t_dev (nb x G x G float, device), computed by the
 * library's backward kernels; grad_host (pmgrit_net_nparams() floats) and loss_host may be NULL.
 * Synchronises hip_stream. */
pmgrit_status pmgrit_net_grad(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, const float* t_dev,
                              float* grad_host, double* loss_host, void* hip_stream);

/* One Adam step (betas 0.9 / 0.999, eps 1e-8, bias-corrected) on given planes and targets;
 * loss_host (may be NULL) receives the batch loss before the step.  Synchronises hip_stream. */
pmgrit_status pmgrit_net_train_step(pmgrit_handle* h, int32_t G, int32_t nb, const float* x_dev, const float* t_dev,
                                    float lr, double* loss_host, void* hip_stream);

/* Input planes (x_dev, nb x 3 x G x G), targets (t_dev, may be NULL) and scales (s_dev, nb doubles)
 * of the samples (inst, k_host[j] -> k_host[j] + 1) at time level `level`, read from the
 * trajectory U_dev ((N_l + 1) x n_dof doubles, device) of instance inst.  0 <= k < N_t
 * (k + 1 <= N_t is read only when t_dev is given).  Asynchronous on hip_stream. */
pmgrit_status pmgrit_net_pack(pmgrit_handle* h, int32_t inst, int32_t level, int32_t nb, const int32_t* k_host,
                              const double* U_dev, float* x_dev, float* t_dev, double* s_dev, void* hip_stream);

typedef struct {
  int32_t epochs;   /* passes over all (instance, step) samples */
  int32_t batch;    /* samples per Adam step (>= 1) */
  float lr;         /* Adam learning rate */
  uint32_t seed;    /* shuffling (counter-based hash of (seed, epoch, index)) */
} pmgrit_train_opts;

typedef struct {
  int32_t epochs_done;
  int64_t adam_steps;
  double loss_first;  /* loss of the first batch */
  double loss_last;   /* mean loss over the last epoch's batches */
  double seconds;
} pmgrit_train_stats;

/* Train the handle's network (from its loaded parameters) on the level-0 steps of trajectories the
 * solver produced: U_dev[i] is instance i's (N_t + 1) x n_dof trajectory (device).  A batch holds
 * samples of one grid size; with several grid sizes their batches alternate.  Synchronous. */
pmgrit_status pmgrit_net_train(pmgrit_handle* h, const pmgrit_train_opts* opts, const double* const* U_dev,
                               void* hip_stream, pmgrit_train_stats* stats);

/* Launch configuration chosen at create for the first launch group (for logs and tests):
 * out8 = {precision, LDS placement mask (bit 0 triangular-solve vector y, 1 V-cycle correction
 * d, 2 V-cycle residual / p = 1 vector s, 3 FP64 iterate x; a clear bit means global
 * scratch), dynamic LDS bytes per workgroup, device LDS limit, scratch doubles per workgroup,
 * workgroup slots, MGRIT levels, instances}.  Errors: PMGRIT_E_ARG for NULL arguments. */
pmgrit_status pmgrit_info(const pmgrit_handle* h, int64_t* out8);

/* Launch group of an instance.  Instances are grouped by the LDS placement their sizes allow;
 * each group launches with its own configuration on its own stream, forked from and joined
 * back into the caller's stream at every sweep of sequential stepping, and once per MGRIT
 * iteration (with the learned guess, the groups holding a predicted instance also meet at every
 * sweep of the first relaxation).  out8 = {group id, number of groups, LDS mask
 * of the sweeps with at most as many workgroups as the device has CUs | LDS mask of the wider
 * sweeps << 8 (masks as in pmgrit_solver_opts.lds_mask), dynamic LDS bytes of the first,
 * off-block entries per lane of the triangular solves, instances in the group, largest dof
 * count in the group, workgroup slots}.  Errors: PMGRIT_E_ARG for a bad
 * instance or NULL out8, PMGRIT_E_STATE for a host-only handle. */
pmgrit_status pmgrit_group_info(const pmgrit_handle* h, int32_t inst, int64_t* out8);

/* Live per-launch timing of the spatial-solve kernel: HIP events recorded on the solve stream
 * around every launch.  enable = 1 resets the totals and turns timing on, 0 turns it off, -1
 * leaves it as is; out4 (may be NULL) receives {total kernel ms, launches, workgroups launched,
 * V-cycles performed} accumulated since the last reset. */
pmgrit_status pmgrit_profile(pmgrit_handle* h, int32_t enable, double* out4);

/* Live per-launch timing of one launch group (same events as pmgrit_profile, same reset):
 * out3 = {kernel ms, launches, workgroups launched} of the spatial-solve launches of group `group`
 * (0 <= group < the group count of pmgrit_group_info) since the last reset; graph replays are not
 * attributed to a group.  Synchronises the device.  Errors: PMGRIT_E_ARG (bad group or NULL
 * out3), PMGRIT_E_STATE (host-only handle). */
pmgrit_status pmgrit_group_profile(pmgrit_handle* h, int32_t group, double* out3);

/* V-cycles (CG iterations with solver 1) performed for each instance since create: out receives
 * n_instances counts.  Synchronises the device.  Errors: PMGRIT_E_ARG (NULL), PMGRIT_E_STATE
 * (host-only handle). */
pmgrit_status pmgrit_inst_vcycles(pmgrit_handle* h, int64_t* out);

const char* pmgrit_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMGRIT_H */
