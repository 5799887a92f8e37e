/*
 * trajam.h -- C ABI of the MI355X (gfx950) batched alternating-minimization (AM)
 * projection of Bernstein-polynomial trajectories.
 *
 * The operation (thesis ch. 6, "Projection Optimization", eqs projection_cost to
 * comp_zeta): every sample xi_i of a batch is projected onto
 *     { A xi = b_eq,  obstacle avoidance,  |velocity| <= v_max,  |acceleration| <= a_max }
 * by the AM fixed point of eqs (fixed_point_1)-(fixed_point_2).  One iteration is
 *   (a)  the closed-form polar step (alpha, beta, d) for every (sample, obstacle,
 *        time) and for the velocity / acceleration bounds of every (sample, time)
 *        (ch. 4 eqs collision_x..d_max, ch. 5 eqs zeta_2..compute_da);
 *   (c)  the multiplier update lam <- lam - rho F^T (F xb - e) (ch. 6 eq lag) and
 *        the residual |F xb - e|_2 (Alg 3, "compute the residuals");
 *   (b)  the equality-constrained QP with the fixed matrix [I + rho F^T F, A^T; A, 0]
 *        (ch. 6 eqs affine_trans / matrix_vec; ch. 5 eqs over_1..over_3), applied to
 *        all samples at once with a precomputed inverse.
 *
 * Conventions for every entry point:
 *   - every call returns a trajam_status; 0 is success and nothing else is;
 *   - no C++ exception crosses this boundary;
 *   - all argument validation happens on the host before any device work, so an
 *     invalid call never launches a kernel;
 *   - "device pointer" means memory the caller allocated on the current HIP device
 *     (for example a PyTorch tensor); the caller owns it, the library never frees it;
 *   - calls are asynchronous on the HIP stream the caller passes (NULL = the null
 *     stream); device errors surface as TRAJAM_ERR_DEVICE from the call that
 *     launched, or from a later call;
 *   - one solver handle is used by one host thread at a time.
 *
 * Layouts (row-major, C order):
 *   xi, xi_bar, lambda      [batch][dims][degree + 1]   scalar = solver precision
 *   obs_centre, obs_vel,
 *   obs_axes                [n_obstacles][dims]         scalar = solver precision
 *                           centre at t = 0 [m], constant velocity [m/s],
 *                           semi-axes [m] (> 0); obstacle centre at time t is
 *                           centre + t * vel
 *   boundary_host           [dims][4] double, HOST memory: (x0, v0, a0, xf) per axis
 *   res_trace               [iters][batch]   scalar = solver precision
 *   flags                   [batch] uint32
 * The solver precision is double for TRAJAM_FP64 and float for TRAJAM_FP32 and
 * TRAJAM_BF16_REFINE.
 */
#ifndef TRAJAM_H
#define TRAJAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TRAJAM_OK = 0,
    TRAJAM_ERR_INVALID = -1,     /* bad argument or problem description */
    TRAJAM_ERR_UNSUPPORTED = -2, /* valid request outside what this build supports */
    TRAJAM_ERR_NUMERIC = -3,     /* singular or non-finite fixed matrix at init */
    TRAJAM_ERR_DEVICE = -4,      /* a HIP call failed (allocation, launch, fault) */
    TRAJAM_ERR_CAPACITY = -5     /* batch larger than max_batch given at init */
} trajam_status;

typedef enum {
    TRAJAM_FP64 = 0,        /* every step in double */
    TRAJAM_FP32 = 1,        /* every step in float; fixed matrices computed in double */
    TRAJAM_BF16_REFINE = 2  /* float state; the QP product on bf16 matrix cores with
                               a hi/lo split, fp32 accumulation and one refinement
                               pass; boundary coefficients set from double values */
} trajam_precision;

/* Obstacle shape (thesis ch. 6 eq coll_multiagent_priest: axis-aligned ellipsoids;
 * ch. 4-5 use circles).  The polar step is the same closed form for both; the
 * sphere model only lets the kernel test |x~|^2 < r^2 without per-axis scaling. */
typedef enum {
    TRAJAM_ELLIPSOID = 0, /* semi-axes obs_axes[j][0..dims) */
    TRAJAM_SPHERE = 1     /* radius obs_axes[j][0]; the other entries are ignored */
} trajam_obstacle_model;

/* Per-sample status bits written to `flags`. */
#define TRAJAM_FLAG_NONFINITE 1u /* a residual or coefficient became NaN / Inf */
#define TRAJAM_FLAG_GREW 2u      /* last residual of the call exceeds the first */

/* One problem class: everything that fixes the KKT matrix (thesis ch. 6, the
 * "one-time computation" of M in eq affine_trans).  Host values. */
typedef struct {
    int32_t dims;          /* 2 or 3 */
    int32_t degree;        /* Bernstein degree n, 3 <= n <= 15; n + 1 coefficients per axis */
    int32_t n_steps;       /* n_p time samples, n + 1 <= n_p <= 256; t_k = k T / (n_p - 1) */
    double horizon;        /* T > 0 [s] */
    double v_max;          /* > 0: velocity bound; <= 0 removes that block from F */
    double a_max;          /* > 0: acceleration bound; <= 0 removes that block from F */
    double rho;            /* augmented-Lagrangian weight, > 0 */
    int32_t n_obstacles;   /* n_o >= 0; each obstacle adds one copy of P to F */
    int32_t n_agents;      /* 1 (single robot) or N in [2, 64] agents planned jointly
                              (thesis ch. 7, Paper IV): each agent has every single-robot row and
                              every unordered pair of agents adds one row per time
                              sample keeping them 2 * agent_radius apart; needs
                              precision FP64 or FP32 and degree <= 11 */
    double agent_radius;   /* > 0 when n_agents > 1 [m]; unused otherwise */
    int32_t max_batch;     /* largest batch a call may pass (>= 1) */
    int32_t precision;     /* a trajam_precision value */
    int32_t obstacle_model; /* a trajam_obstacle_model value */
    /* Workspace bounds (Paper III, eq bound_con): 1 adds the rows G = [-P; P] per axis,
     * lo[ax] <= p_ax(t) <= hi[ax] at every time sample, handled by the slack step
     * s = max(0, -G xb + tau) of the AM iteration (each row's residual is its
     * violation) and 2 rho P^T P in the fixed matrix; 0: none (lo, hi unused).  The
     * materialized polar variables of trajam_polar do not cover these rows. */
    int32_t workspace;
    double ws_lo[3], ws_hi[3];   /* per axis, lo <= hi, finite; entries past dims unused */
} trajam_problem;

typedef struct trajam_solver trajam_solver; /* opaque; owns device constants */

/* Validates `p`, computes the fixed matrices in double on the host (Bernstein
 * basis, H = I + rho F^T F, the inverse of its free block), uploads them and
 * returns a handle in *out.  Uses the current HIP device.
 * For n_agents > 1 it also builds the operator of the agents' deviations from their
 * mean (the pair rows' Gram is the complete-graph Laplacian, so the joint QP splits
 * exactly into the agent mean, moved by the single-robot operator, and the
 * deviations, moved by the operator of H + n_agents rho P^T P).
 * Errors: INVALID (bad field), UNSUPPORTED (a multi-agent problem in BF16_REFINE or
 * with degree > 11), NUMERIC (H not positive definite), DEVICE (allocation / copy
 * failed).  On error *out is NULL. */
trajam_status trajam_init(const trajam_problem *p, trajam_solver **out);

/* Frees the handle and its device memory (never the caller's buffers).  NULL is a
 * no-op.  The caller must make sure no work using the handle is still queued. */
void trajam_destroy(trajam_solver *s);

/* Runs `iters` AM iterations on `batch` samples (thesis ch. 6 eqs comp_alpha to
 * comp_zeta, in that order), in one launch.
 *   xi            device, [batch][dims][n+1]: the samples to project (read only)
 *   boundary_host host,   [dims][4]: (x0, v0, a0, xf) of eq eq_modify11
 *   obs_*         device, [n_obstacles][dims] (see layouts above); obs_vel == NULL
 *                 means static obstacles (a faster loop than passing zeros).  All
 *                 three NULL: reuse the obstacles packed last (by a previous call or by
 *                 trajam_set_obstacles), which skips the packing launch; otherwise
 *                 obs_centre and obs_axes may be NULL only when n_obstacles == 0
 *   xi_bar        device, [batch][dims][n+1]: in = initial iterate (a copy of xi for a
 *                 cold start, or a warm start), out = iterate after `iters` steps
 *   lambda        device, [batch][dims][n+1]: in = initial multiplier (zeros for a
 *                 cold start), out = multiplier after `iters` steps
 *   res_trace     device, [iters][batch] or NULL: res_trace[k][i] = |F xb_i^k - e|_2,
 *                 the residual of iterate k after its own polar step
 *   flags         device, [batch] or NULL: TRAJAM_FLAG_* bits of this call
 *   stream        hipStream_t or NULL
 * The state of the iteration is (xi_bar, lambda), so a call with iters = a followed
 * by a call with iters = b gives the same result as one call with iters = a + b.
 * Multi-agent problems (n_agents = N > 1): a sample is a joint sample of N
 * trajectories, so xi, xi_bar and lambda are [batch][N][dims][n+1] and
 * boundary_host is [N][dims][4]; res_trace and flags stay per joint sample, and the
 * residual covers every row of every agent and every pair once.  Each agent has the
 * obstacle and kinematic rows; a pair's row targets the exterior of a sphere of
 * radius 2 * agent_radius around the other agent (eqs sphere_proposed to com_d_i).
 * The per-agent boundary coefficients live on the device and are re-uploaded only
 * when boundary_host changes; such a call synchronizes the stream (so, under graph
 * capture, keep the boundary of the captured call).
 * Errors: INVALID (NULL handle or required pointer, iters < 0, batch < 0),
 * CAPACITY (batch > max_batch), DEVICE (launch failed).  batch == 0 or iters == 0
 * is a successful no-op. */
trajam_status trajam_project(trajam_solver *s, int32_t batch, const void *xi,
                             const double *boundary_host, const void *obs_centre,
                             const void *obs_vel, const void *obs_axes, void *xi_bar,
                             void *lambda, int32_t iters, void *res_trace, uint32_t *flags,
                             void *stream);

/* ---- penalty continuation ------------------------------------------------------
 * Thesis ch. 4 (Alg 1) raises the penalty weights while the residuals stay above a
 * threshold; ch. 7 precomputes the QP inverse for ten increasing penalties and uses
 * them in later iterations.  Here: a ladder of `levels` penalties rho * growth^l
 * (l = 0 .. levels-1), each with its own fixed QP operator computed in double on the
 * host; every sample carries a level, an iteration count and a reference residual.
 * An iteration runs steps (a), (c), (b) with its level's penalty in the multiplier
 * update and its level's operator in the QP; then the count rises, and when it
 * reaches `window` the level goes up by one (at most levels - 1) if the iteration's
 * residual is above `tol` and above stall_ratio times the reference (0 before the
 * first check), the reference becomes that residual and the count restarts. */
#define TRAJAM_CONT_MAX_LEVELS 16
typedef struct {
    int32_t levels;      /* 1 .. TRAJAM_CONT_MAX_LEVELS; 1 = the plain iteration */
    double growth;       /* >= 1: rho_l = rho * growth^l */
    int32_t window;      /* >= 1: iterations between checks */
    double stall_ratio;  /* >= 0: a check raises the level when res > stall_ratio * reference */
    double tol;          /* >= 0: ... and res > tol */
} trajam_continuation;

/* Per-sample state, caller-owned device memory [batch]; zero it before a sample's first
 * call (level 0, no reference) and pass it back unchanged to continue. */
typedef struct {
    int32_t level;   /* index into the ladder */
    int32_t count;   /* iterations since the last check */
    double ref;      /* residual at the last check; 0 before the first */
} trajam_cont_state;

/* Computes and uploads the ladder's QP operators (host FP64, each checked like
 * trajam_init's) and enables trajam_project_continuation; c == NULL disables it.
 * Single robot, precision FP64 or FP32.  Allocates device memory (call at set-up).
 * Errors: INVALID (bad parameters), UNSUPPORTED (multi-agent or BF16_REFINE),
 * NUMERIC (a level's QP step does not contract in the solver's precision), DEVICE. */
trajam_status trajam_set_continuation(trajam_solver *s, const trajam_continuation *c);

/* trajam_project with the penalty continuation set by trajam_set_continuation; the
 * iteration's state is (xi_bar, lambda, state), so a call with iters = a followed by
 * one with iters = b equals one with a + b.  Runs the wave-per-sample kernel (its tuned
 * samples per workgroup when that variant is the tuned one).  Arguments and errors as
 * trajam_project, plus state (device, [batch] trajam_cont_state, in/out) and INVALID
 * when no continuation is set. */
trajam_status trajam_project_continuation(trajam_solver *s, int32_t batch, const void *xi,
                                          const double *boundary_host, const void *obs_centre,
                                          const void *obs_vel, const void *obs_axes, void *xi_bar,
                                          void *lambda, trajam_cont_state *state, int32_t iters,
                                          void *res_trace, uint32_t *flags, void *stream);

/* Steps (a) and the residual norm only, at the given coefficients, without
 * touching any multiplier (thesis Alg 3, "compute the residuals set r").
 *   xi_bar   device, [batch][dims][n+1] ([batch][N][dims][n+1] for N > 1 agents)
 *   res_l2   device, [batch]: |F xb - e|_2
 *   res_max  device, [batch] or NULL: largest |component| of F xb - e
 * Errors: as trajam_project. */
trajam_status trajam_residuals(trajam_solver *s, int32_t batch, const void *xi_bar,
                               const void *obs_centre, const void *obs_vel,
                               const void *obs_axes, void *res_l2, void *res_max,
                               void *stream);

/* The fixed matrices trajam_init computes and uploads, returned in double on the
 * host for inspection and CPU tests.  Host only: no device work, no handle.
 * Any output pointer may be NULL.
 *   P, Pd, Pdd  [n_steps][n+1]  basis rows and their first / second time derivatives
 *   H           [n+1][n+1]      I + rho F^T F (one axis; every axis is the same)
 *   W           [n-3][n+1]      the QP update operator of the free coefficients
 *                               3..n-1: delta_free = W z, where z holds the KKT
 *                               defect g at free coefficients and the boundary
 *                               defect (xi*_b - xb_b) at coefficients 0, 1, 2, n
 * Errors: INVALID, UNSUPPORTED (as trajam_init), NUMERIC. */
trajam_status trajam_fixed_matrices(const trajam_problem *p, double *P, double *Pd,
                                    double *Pdd, double *H, double *W);

/* Contraction of the QP step in the problem's precision: the spectral radius of
 * I - W~ H_ff, where W~ is the free-coefficient operator as the device applies it
 * (FP64: W_ff = H_ff^-1; FP32: W_ff rounded to float; BF16_REFINE: the bf16 hi + lo
 * split of the float W_ff) and H_ff the free block of the QP Hessian (thesis ch. 6:
 * the QP's fixed KKT matrix, eq over_3).  The delta-form step xb_f += W~ (q - H_ff
 * xb_f) multiplies its error by I - W~ H_ff, so reduced precision is usable only
 * when this is well below 1; for joint problems the larger of the mean and the
 * deviation operators is returned.  Estimated by ||E^256||_F^(1/256) (at most a factor
 * n_f^(1/512) above the radius).  trajam_init fails with NUMERIC when it is >= 0.5.
 * Host only: no device work, no handle.  Errors: INVALID (NULL rho or problem),
 * UNSUPPORTED, NUMERIC (as trajam_init). */
trajam_status trajam_qp_contraction(const trajam_problem *p, double *rho);

/* Kernel variants of trajam_project.  Both run every iteration of a call in one
 * launch and compute the same arithmetic per sample; they differ in how a sample's
 * time samples map to lanes. */
typedef enum {
    TRAJAM_KERNEL_MULTIWAVE = 0, /* one lane per time sample: ceil(n_steps / 64) waves per
                                    sample, exchanging partial sums through LDS */
    TRAJAM_KERNEL_WAVE = 1       /* one wave per sample: ceil(n_steps / 64) time samples
                                    per lane, no block barrier inside the iteration */
} trajam_kernel;

/* Launch shape of trajam_project: kernel variant and samples per workgroup (spw).
 * MULTIWAVE needs spw * roundup64(n_steps) <= 256, WAVE needs spw * 64 <= 256.
 * The autotuner picks it; results do not depend on spw, and the two variants agree
 * to rounding (they sum F^T r over time samples in different orders).
 * Errors: INVALID. */
trajam_status trajam_set_launch(trajam_solver *s, int32_t kernel, int32_t samples_per_workgroup);
trajam_status trajam_get_launch(const trajam_solver *s, int32_t *kernel,
                                int32_t *samples_per_workgroup);

/* Boundary coefficients xi_0, xi_1, xi_2, xi_n implied by (x0, v0, a0, xf) for
 * one axis (the unique solution of the four boundary rows).  Host only. */
trajam_status trajam_boundary_coefficients(const trajam_problem *p, const double *b4,
                                           double *coef4);

/* Packs obstacles into the solver (the same packing trajam_project does per call) so
 * that calls which take no obstacle arguments -- trajam_ragged_launch -- use them.
 * Same layouts and NULL rules as trajam_project.  Errors: INVALID, DEVICE. */
trajam_status trajam_set_obstacles(trajam_solver *s, const void *obs_centre, const void *obs_vel,
                                   const void *obs_axes, void *stream);

/* Autotuner: times every launch shape of trajam_project (both kernel variants, each
 * valid samples-per-workgroup; joint samples per workgroup for multi-agent problems)
 * for `probe_iters` iterations on the given inputs with HIP events, applies the
 * fastest with trajam_set_launch and returns it; the current shape is kept unless
 * another is more than 3 % faster.  Results are
 * cached per process, keyed by (GPU architecture, dims, n_steps, n_obstacles rounded
 * up to a power of two, batch rounded up to a power of two, precision); a cached key
 * is applied without timing.  When the environment variable TRAJAM_AUTOTUNE_CACHE
 * names a file, the cache is read from and appended to it (one key per line).
 * xi_bar and lambda are overwritten (used as scratch).  Synchronizes the stream.
 * Errors: as trajam_project. */
trajam_status trajam_autotune(trajam_solver *s, int32_t batch, const void *xi,
                              const double *boundary_host, const void *obs_centre,
                              const void *obs_vel, const void *obs_axes, void *xi_bar,
                              void *lambda, int32_t probe_iters, int32_t *kernel,
                              int32_t *samples_per_workgroup, void *stream);

/* ---- ragged batches: many problems in one persistent launch ---------------------
 * Each item is one problem (its own solver, hence fixed matrices and obstacles, and
 * its own batch).  A plan uploads the problem table once; every launch zeroes a
 * device work counter and runs one persistent kernel whose waves take (problem,
 * sample) units longest-problem-first until none is left (single-robot and
 * multi-agent problems each have their own table, counter and kernel, launched one
 * after the other).  Launches never allocate or synchronize, so they can be
 * captured in a graph.  Multi-agent items take [batch][N][dims][n+1] buffers and
 * [N][dims][4] boundary rows.  Restrictions of this build: FP32 solvers,
 * degree <= 11, n_steps <= 128, obstacles set with trajam_set_obstacles before the
 * plan is created. */
typedef struct {
    trajam_solver *solver;       /* problem class (FP32) */
    int32_t batch;               /* samples of this problem (<= max_batch) */
    const void *xi;              /* device [batch][dims][degree+1] */
    const double *boundary_host; /* host [dims][4] ([N][dims][4] for N agents), read at
                                    plan creation */
    void *xi_bar;                /* device in/out, as trajam_project */
    void *lambda;                /* device in/out */
    void *res_trace;             /* device [iters][batch] float or NULL */
    uint32_t *flags;             /* device [batch] or NULL */
} trajam_ragged_item;

typedef struct trajam_ragged_plan trajam_ragged_plan;

/* Errors: INVALID (bad item), UNSUPPORTED (item outside the restrictions above),
 * DEVICE (allocation / copy).  On error *out is NULL. */
trajam_status trajam_ragged_plan_create(const trajam_ragged_item *items, int32_t n_items,
                                        int32_t iters, trajam_ragged_plan **out);
/* Runs `iters` AM iterations for every sample of every item.  Errors: INVALID, DEVICE. */
trajam_status trajam_ragged_launch(trajam_ragged_plan *plan, void *stream);
void trajam_ragged_plan_destroy(trajam_ragged_plan *plan);

/* Materialised polar variables of step (a) at the given coefficients (thesis ch. 6,
 * eqs comp_alpha, comp_beta, comp_d for the obstacles; alpha_v, compute_dv and
 * alpha_a, compute_da for the kinematic blocks): the values one AM iteration's polar
 * step takes at xi_bar, for inspection, checking and consumers that want them in
 * memory; the projection itself never materialises them.  Single robot only.
 *   xi_bar     device, [batch][dims][n+1]
 *   obstacles  as trajam_project (all NULL: the obstacles packed last)
 *   obs_alpha, obs_beta, obs_d   device, [batch][n_obstacles][n_steps] or NULL each
 *              (a NULL array is not computed; in 2D beta is the constant pi/2, so
 *              callers usually pass NULL for it):
 *              u = (p(t) - c(t)) ./ semi-axes (1 / radius on every axis for the sphere
 *              model), alpha = atan2(u_y, u_x), beta = atan2(|(u_x, u_y)|, u_z)
 *              (pi/2 in 2D), d = max(1, |u|)
 *   kin        device, [batch][6][n_steps] or NULL: alpha_v, beta_v, d_v, alpha_a,
 *              beta_a, d_a with d = min(1, |v| / bound); all 0 for a disabled block
 * Rows are unpadded: entry (b, j, t) is at (b * n_obstacles + j) * n_steps + t.  Scalar
 * type = solver precision.  Errors: INVALID, UNSUPPORTED (n_agents > 1), CAPACITY,
 * DEVICE. */
trajam_status trajam_polar(trajam_solver *s, int32_t batch, const void *xi_bar, const void *obs_centre,
                           const void *obs_vel, const void *obs_axes, void *obs_alpha, void *obs_beta,
                           void *obs_d, void *kin, void *stream);

/* ---- projection-guided sampling loop (thesis ch. 6, Alg 3) -------------------
 * One CEM iteration on the device is: trajam_cem_sample -> trajam_project (cold
 * start) -> trajam_residuals -> trajam_cem_cost -> trajam_cem_select ->
 * trajam_cem_update.  dim = dims * (degree + 1); every array is a device pointer of
 * the solver precision unless typed otherwise; all calls are asynchronous on
 * `stream` and never synchronize, so a whole iteration can be captured in a graph. */

/* xi[i] = mu + chol z[i] for i < n (Alg 3, "draw N_b samples from N(mu, Sigma)").
 *   mu [dim], chol [dim][dim] lower-triangular Cholesky factor of Sigma,
 *   z [n][dim] standard normal draws (the caller's random numbers),
 *   xi [n][dims][degree+1] output.
 *   xi_bar, lambda [n][dims][degree+1]: optional outputs, NULL to skip; when given
 *   they receive the cold start of the projection that follows (xi_bar = xi,
 *   lambda = 0) from the same launch.
 * Errors: INVALID, CAPACITY (n > max_batch), DEVICE. */
trajam_status trajam_cem_sample(trajam_solver *s, int32_t n, const void *mu, const void *chol,
                                const void *z, void *xi, void *xi_bar, void *lambda, void *stream);

/* Receding-horizon control (thesis ch. 5, Paper II, Implementation Details: an MPC on
 * the batch optimizer that starts every control cycle from the preceding cycle's
 * solution, multipliers included).  Between two cycles the time origin moves on by
 * delta seconds: every sample's coefficients xi_bar [batch][n_agents][D][n_v] (the
 * layout of trajam_project) are re-expressed as the Bernstein coefficients of the same
 * polynomials on the window [delta, delta + T] (T the horizon; delta < 0 or > T
 * extrapolates), written to xi_next and xi_bar_next (the next cycle's samples and
 * its starting iterate), and lambda_next = lambda if keep_lambda, else 0 (lambda may
 * then be NULL).  Storage in the solver's state precision (double for FP64, else
 * float); FP64 arithmetic.  Outputs may alias the inputs (each coefficient row is read
 * whole before it is written).  The next cycle's boundary rows (the executed
 * trajectory's state at delta) and obstacles are the caller's.  Errors: INVALID,
 * CAPACITY (batch > max_batch), UNSUPPORTED (degree above 15), DEVICE. */
trajam_status trajam_mpc_shift(trajam_solver *s, int32_t batch, double delta, int32_t keep_lambda,
                               const void *xi_bar, const void *lambda, void *xi_next, void *xi_bar_next,
                               void *lambda_next, void *stream);

/* The sampling loop's standard normal draws from an in-library counter-based
 * generator (thesis ch. 6, Alg 3 draws N_b samples per iteration): z[i], i < count, of
 * the stream (key, counter).  Block b = i / 4 is Philox4x64 with 10 rounds (Salmon,
 * Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) of the
 * 256-bit counter (counter + b mod 2^64, 0, 0, 0) under the 128-bit key (key, 0); its
 * words x_0..x_3 give the uniforms u_j = (floor(x_j / 2^11) + 1/2) 2^-53 and the
 * normals sqrt(-2 ln u_0) (cos, sin)(2 pi u_1), sqrt(-2 ln u_2) (cos, sin)(2 pi u_3)
 * (Box-Muller), in FP64 arithmetic, stored as double (fp64 = 1) or float (0).  The
 * draws of CEM iteration l with N_b samples of dimension D n_v are z[l N_b D n_v + ...]
 * of one stream, so a run is reproduced by (key, counter).  No solver needed; errors
 * through trajam_last_error(NULL): INVALID, DEVICE. */
trajam_status trajam_normals(int64_t count, uint64_t key, uint64_t counter, int32_t fp64, void *z, void *stream);

/* Augmented cost of Alg 3: c_aug[i] = sum_t |Pdd xb_i(t)|^2 + res[i], and the residual
 * key res_key[i] = floor(res[i] / quantum) (int32, clamped), the resolution at which
 * residuals are compared.  xi_bar [n][dims][degree+1], res [n] (from trajam_residuals),
 * c_aug [n], res_key [n] int32.  Errors: INVALID (quantum <= 0), CAPACITY, DEVICE. */
trajam_status trajam_cem_cost(trajam_solver *s, int32_t n, const void *xi_bar, const void *res,
                              double quantum, void *c_aug, int32_t *res_key, void *stream);

/* ConstraintEliteSet and EliteSet of Alg 3: proj_idx [n_proj] = the indices of the
 * n_proj smallest (res_key, c_aug, index) in ascending order; elite_idx [n_elite] =
 * the n_elite of those with the smallest (c_aug, index), ascending (elite_idx[0] is
 * the returned trajectory).  One workgroup; n <= 4096.
 * Errors: INVALID (1 <= n_elite <= n_proj <= n violated, n > 4096), DEVICE. */
trajam_status trajam_cem_select(trajam_solver *s, int32_t n, const int32_t *res_key,
                                const void *c_aug, int32_t n_proj, int32_t n_elite,
                                int32_t *proj_idx, int32_t *elite_idx, void *stream);

/* Distribution update (eqs update_mean, update_covariance) with weights
 * w_e = exp(-(c_aug_e - min c_aug) / (gamma * std)) over the elite set (std = population
 * standard deviation of its c_aug; gamma alone when std is 0):
 *   mu <- (1 - sigma) mu + sigma sum w_e xb_e / sum w_e
 *   Sigma <- (1 - sigma) Sigma + sigma sum w_e (xb_e - mu)(xb_e - mu)^T / sum w_e  (new mu)
 *   chol <- Cholesky factor of Sigma + 1e-10 I.
 * mu [dim], Sigma [dim][dim], chol [dim][dim] in/out; elite_idx [n_elite] int32;
 * xi_bar and c_aug indexed by elite_idx.  One workgroup.
 * Errors: INVALID (sigma not in (0, 1], gamma <= 0, n_elite < 1), DEVICE. */
trajam_status trajam_cem_update(trajam_solver *s, int32_t n_elite, const int32_t *elite_idx,
                                const void *xi_bar, const void *c_aug, double sigma, double gamma,
                                void *mu, void *Sigma, void *chol, void *stream);

/* ---- learned warm start ------------------------------------------------------
 * A fully connected ReLU network (no thesis counterpart: a learned initialization
 * of the projection) trained and evaluated with these kernels.  Parameters are one
 * flat float array: for each layer l, W_l [width[l+1]][width[l]] row-major, then
 * b_l [width[l+1]].  Hidden layers apply ReLU; the last layer is linear.  These
 * calls take no solver handle; on error trajam_last_error(NULL) holds the message.
 * precision: 0 = fp32 products on the VALU, 1 = bf16 products on matrix cores with
 * fp32 accumulation. */
#define TRAJAM_MLP_MAX_LAYERS 8
#define TRAJAM_FLAG_COLD_FALLBACK 4u /* warm start rejected; the sample continues from its cold probe */

typedef struct {
    int32_t n_layers;                          /* 1 .. TRAJAM_MLP_MAX_LAYERS */
    int32_t width[TRAJAM_MLP_MAX_LAYERS + 1];  /* width[0] inputs .. width[n_layers] outputs */
} trajam_mlp_shape;

/* Number of parameters of the shape.  Errors: INVALID. */
trajam_status trajam_mlp_param_count(const trajam_mlp_shape *shape, int64_t *n_params);

/* y [batch][width[L]] = network(x [batch][width[0]]); acts receives the hidden
 * activations, layer after layer, each [batch][width[l]] (l = 1 .. L-1), for the
 * backward pass.  Device pointers.  Errors: INVALID, DEVICE. */
trajam_status trajam_mlp_forward(const trajam_mlp_shape *shape, int32_t batch, int32_t precision,
                                 const float *params, const float *x, float *acts, float *y,
                                 void *stream);

/* Inference layout of the parameters: per layer W^T [in][out] (transposed), then the
 * bias, in a separate buffer of n_params floats.  Errors: INVALID, DEVICE. */
trajam_status trajam_mlp_pack_infer(const trajam_mlp_shape *shape, const float *params,
                                    float *packed, void *stream);

/* Inference only: y [batch][width[L]] = network(x) in one launch from the packed
 * parameters of trajam_mlp_pack_infer (fp32 products, activations kept on chip;
 * every width <= 512).  Same result as trajam_mlp_forward with precision 0 up to the
 * order of the sums.  Errors: INVALID, UNSUPPORTED (a width above 512), DEVICE. */
trajam_status trajam_mlp_infer(const trajam_mlp_shape *shape, int32_t batch, const float *packed,
                               const float *x, float *y, void *stream);

/* grads [n_params] = d loss / d params given dy = d loss / d y [batch][width[L]], the
 * input x and the activations of the forward call.  scratch: 2 * batch * max hidden
 * width floats (NULL allowed for a single-layer network): the two input-gradient
 * buffers, the idle one of which also holds the partial weight gradients when a
 * weight-gradient product (K = batch) is split over the batch; the partials are added
 * in a fixed order, so the result does not depend on timing.  Errors: INVALID, DEVICE. */
trajam_status trajam_mlp_backward(const trajam_mlp_shape *shape, int32_t batch, int32_t precision,
                                  const float *params, const float *x, const float *acts,
                                  const float *dy, float *grads, float *scratch, void *stream);

/* trajam_mlp_backward without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid hipMalloc).  The two input-gradient
 * buffers live in a static per-device array of TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS floats
 * (8 MiB) that the library holds on every GPU it runs on until the process ends; its
 * device address is looked up on the first call on each device.  Every call on one GPU
 * shares that array, so calls that overlap in time on one GPU (two streams, two host
 * threads) race and must be serialized by the caller; a later call may overwrite what
 * an earlier one left there (nothing in it is meant to outlive a call).  Same arguments,
 * results and errors as trajam_mlp_backward, plus CAPACITY when 2 * batch * (largest
 * hidden width) exceeds TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS (for a single-layer network
 * no workspace is needed). */
#define TRAJAM_MLP_NOALLOC_SCRATCH_FLOATS 2097152
trajam_status trajam_mlp_backward_noalloc(const trajam_mlp_shape *shape, int32_t batch, int32_t precision,
                                          const float *params, const float *x, const float *acts,
                                          const float *dy, float *grads, void *stream);

/* Mean squared error over count values: loss[0] = mean (y - t)^2, dy = 2 (y - t) / count.
 * loss is a device array of TRAJAM_MLP_MSE_LOSS_FLOATS floats: loss[1..] is the
 * workspace of the per-workgroup partial sums (added in a fixed order, so the loss does
 * not depend on timing), overwritten by every call.  Errors: INVALID, DEVICE. */
#define TRAJAM_MLP_MSE_LOSS_FLOATS 513
trajam_status trajam_mlp_mse(int64_t count, const float *y, const float *target, float *dy,
                             float *loss, void *stream);

/* One Adam step (Kingma & Ba) with bias correction for step >= 1, in place on params,
 * m, v [n].  Errors: INVALID, DEVICE. */
trajam_status trajam_mlp_adam(int64_t n, float *params, const float *grads, float *m, float *v,
                              int32_t step, float lr, float beta1, float beta2, float eps,
                              void *stream);

/* The warm start is a learned jump of the AM state: a short cold probe (k0 AM
 * iterations with trajam_project from xi_bar = xi, lambda = 0) gives the state
 * (xb, lam); the network maps it to the state at which the cold iteration would
 * first reach the residual tolerance, (xb + d_xb, lam + d_lam); a per-sample check
 * keeps the probe state wherever the jump does not lower the residual.
 *
 * Network input rows x[b] = [(xb[b] - xi[b]), lam[b]] * inv_scale, each
 * [dims][n_coeffs]: x is [batch][2 * dims * n_coeffs].  Errors: INVALID, DEVICE. */
trajam_status trajam_warm_features(int32_t batch, int32_t dims, int32_t n_coeffs, const float *xi,
                                   const float *xb, const float *lam, float inv_scale, float *x,
                                   void *stream);

/* Jump from the network output y [batch][dims * n_coeffs] = d_xb / out_scale: on the
 * free coefficients (3 .. n-1) xb_out = xb + out_scale * d_xb and lam_out = xb_out - xi;
 * on the boundary ones xb_out = xb (already exact) and lam_out = lam.  Outputs must
 * not alias xb or lam (the fallback needs the probe state).  Errors: INVALID, DEVICE. */
trajam_status trajam_warm_apply(int32_t batch, int32_t dims, int32_t n_coeffs, const float *y,
                                float out_scale, const float *xi, const float *xb, const float *lam,
                                float *xb_out, float *lam_out, void *stream);

/* Fused warm jump on the matrix cores: trajam_warm_features, the network and
 * trajam_warm_apply in one launch, 16 samples per workgroup, every product on
 * v_mfma_f32_16x16x16_bf16 (weights and activations rounded to bf16, fp32 accumulation,
 * bias and ReLU in fp32).  The parameters are first packed by trajam_warm_pack_mfma
 * (flat fp32 layout in, the matrix-core operand order out; packed == NULL only returns
 * the byte size in *packed_bytes).  Network: 1..4 layers, every width <= 256, width[0] =
 * 2 dims nv, last width = dims nv.  Outputs must not alias xb or lam.
 * Errors: INVALID, UNSUPPORTED (shape), DEVICE. */
trajam_status trajam_warm_pack_mfma(const trajam_mlp_shape *shape, const float *params, void *packed,
                                    int64_t *packed_bytes, void *stream);
trajam_status trajam_warm_jump(const trajam_mlp_shape *shape, int32_t batch, int32_t dims, int32_t n_coeffs,
                               const void *packed, float in_scale, float out_scale, const float *xi,
                               const float *xb, const float *lam, float *xb_out, float *lam_out, void *stream);

/* Per-sample fallback: where res_warm[b] (residual of the jumped state xb) is not
 * below res_cold[b] (the probe's last residual), or is NaN, or the jumped state is
 * not finite, the sample keeps the probe state (xb = xb_src, lam = lam_src) and
 * flags[b] = TRAJAM_FLAG_COLD_FALLBACK; otherwise flags[b] = 0 (flags may be NULL).
 * Errors: INVALID, DEVICE. */
trajam_status trajam_warm_fallback(int32_t batch, int32_t dims, int32_t n_coeffs,
                                   const float *res_warm, const float *res_cold, const float *xb_src,
                                   const float *lam_src, float *xb, float *lam, uint32_t *flags,
                                   void *stream);

/* ------------------------------------------------------------------------------
 * Heading / multi-circle variant (thesis ch. 5, Paper II: Problem Formulation, the
 * reformulated problem eqs reform_cost..d_bound, the augmented Lagrangian eq
 * reform_formulation and Alg 2).  A rectangular robot is n_c circles at offsets r_m on
 * its heading axis; it tracks x_des(t) with the cost sum_t (xdd^2 + ydd^2 + psidd^2 +
 * |p - p_des|^2) under |v| <= v_max, |a| <= a_max and every circle outside every
 * axis-aligned elliptical obstacle.  Per sample the state is the Bernstein
 * coefficients of x, c, y, s (c, s: slack copies of cos psi, sin psi) and psi, and the
 * multipliers of the same rows.  One iteration, in Alg 2's order:
 *   1. xi      <- the QP with the fixed matrix Q + rho F'F of each position group
 *                 (x with c, y with s) under A xi = b;
 *   2. psi_t   <- atan2(s, c) at the time steps, on the branch nearest the current
 *                 heading; xi_psi <- the QP with the fixed matrix Pdd'Pdd + rho P'P of
 *                 eq compute_convex_surrogate under A_psi xi_psi = b_psi;
 *   3-4.        the polar step: angles and radii of every (circle, obstacle, step)
 *                 row (centre x + r_m cos psi, angles scaled by the semi-axes, d >= 1)
 *                 and of the velocity / acceleration rows (d <= 1) (eqs zeta_2..compute_da);
 *   5. lam     <- lam - rho F'(F xi - g); lam_psi <- lam_psi - rho P'(P xi_psi - psi_t).
 * Before the first iteration the state's coefficients fixed by the boundary rows
 * (0, 1, 2, n of x and y; 0, n of psi) are set from them and the first polar step is
 * taken at that state.  Residuals of an iterate: |F xi - g| over both groups and
 * |psi_t - P xi_psi|.
 *
 * Layouts: state, lambda [batch][5][degree + 1] (rows x, c, y, s, psi), res_trace
 * [iters][batch][2], all device memory in the handle's precision (double for
 * TRAJAM_FP64, float for TRAJAM_FP32). */
#define TRAJAM_HEADING_MAX_CIRCLES 8

typedef struct trajam_heading trajam_heading;

typedef struct {
    int32_t degree;      /* Bernstein degree n in [4, 11] */
    int32_t n_steps;     /* time steps t_k = k T / (n_steps - 1), in [n + 1, 128] */
    double horizon;      /* T [s] > 0 */
    double v_max;        /* > 0 [m/s] */
    double a_max;        /* > 0 [m/s^2] */
    double rho;          /* > 0, one penalty weight for every block */
    int32_t n_circles;   /* footprint circles, in [1, 8] */
    double radii[TRAJAM_HEADING_MAX_CIRCLES];  /* offsets r_m [m] on the heading axis */
    int32_t n_obstacles; /* >= 0; fixes the row count of F, hence the QP operator */
    int32_t precision;   /* TRAJAM_FP64 or TRAJAM_FP32 */
    int32_t max_batch;   /* >= 1 */
} trajam_heading_problem;

/* Handle with both fixed QP operators (inverses of the free blocks, computed in FP64
 * on the host) and the basis tables on the current device.  Errors (message through
 * trajam_last_error(NULL)): INVALID, NUMERIC, DEVICE. */
trajam_status trajam_heading_create(const trajam_heading_problem *p, trajam_heading **out);
void trajam_heading_destroy(trajam_heading *h);
const char *trajam_heading_last_error(const trajam_heading *h);

/* The scene, from HOST memory (copied before the call returns; it first waits for the
 * device, since a projection in flight reads the tables): boundary [10] = (x0, vx0,
 * ax0, xf, y0, vy0, ay0, yf, psi0, psif); x_des [2][n_steps] desired x and y at the
 * time steps; obstacles [n_obstacles][6] = (cx, cy, vx, vy, a, b): centre at t = 0 [m],
 * constant velocity [m/s], semi-axes [m] > 0 (inflated by the footprint circles'
 * radius).  Errors: INVALID, DEVICE. */
trajam_status trajam_heading_set_scene(trajam_heading *h, const double *boundary, const double *x_des,
                                       const double *obstacles);

/* `iters` iterations of Alg 2 for every sample, in place: state and lambda are read
 * as the start and hold the result (zero lambda for a cold start).  res_trace may be
 * NULL.  With iters = 0 the state's boundary coefficients are set and nothing else.
 * Errors: INVALID (no scene, negative sizes, NULL), CAPACITY, DEVICE. */
trajam_status trajam_heading_project(trajam_heading *h, int32_t batch, void *state, void *lambda, int32_t iters,
                                     void *res_trace, void *stream);

/* Receding horizon for the heading variant (thesis ch. 5, Paper II, Implementation
 * Details: each control cycle starts from the preceding one's solution, both
 * multipliers included): every row of every sample of `state` (x, c, y, s, psi) is
 * re-expressed, in place, on the window moved on by delta seconds (the same
 * polynomial, S(delta) as for trajam_mpc_shift); lambda's rows are carried over
 * unchanged (keep_lambda = 1) or cleared (0).  The next cycle's boundary rows, desired
 * path and obstacles are the caller's (trajam_heading_set_scene).  Errors: INVALID,
 * CAPACITY, DEVICE. */
trajam_status trajam_heading_shift(trajam_heading *h, int32_t batch, double delta, int32_t keep_lambda, void *state,
                                   void *lambda, void *stream);

/* Static description of a status code.  Never NULL. */
const char *trajam_status_string(trajam_status st);

/* Message of the last failed call on this handle (empty if none).  Valid until
 * the next call on the handle.  NULL handle: the message of the last failed
 * trajam_init on this thread. */
const char *trajam_last_error(const trajam_solver *s);

#ifdef __cplusplus
}
#endif

#endif /* TRAJAM_H */
