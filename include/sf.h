/*
 * sf.h - C ABI of the MI355X safety-filter (SF) library.
 *
 * The SF projects a sampled joint multi-robot trajectory xi onto the
 * inter-robot, obstacle and workspace constraints and the start/goal
 * equalities (projection problem, eqs. proj_cost..proj_robot) by L
 * applications of the fixed-point operator T (eq. fixed_point), whose steps are
 * the alternating-minimisation updates of the Appendix (eqs. alpha_step ..
 * xi_step) on the augmented Lagrangian (eq. aug_lag).  The planar SF (n_dim =
 * 2) has every entry point; the 3D spheroid variant (n_dim = 3, below) has the
 * fused forward and its adjoint.
 *
 * Layouts (all float32, contiguous, device memory unless marked host):
 *   coefficient arrays (xi, xi_bar, lambda and their gradients): problems
 *     concatenated in batch order; problem b holds [N_DIM=2][n_b][n_coef],
 *     i.e. the paper's stacking (all robots' x coefficients, then all y);
 *   boundary: [sum_b n_b][2][2]  = (b_{i,0}, b_{i,K}) positions per robot;
 *   obstacles: [sum_b M_b][3]    = centre x, centre y, a_o (inflated size:
 *     the minimum distance between a robot centre and the obstacle centre);
 *   residual: [B][4] = ||r_1||, ||r_2|| of the returned xi_bar (metres),
 *     ||z^L - z^{L-1}|| with z = (xi_bar, lambda), and a status word stored
 *     as a float (0 = finite outputs, 1 = non-finite value in the outputs).
 *   The robot size a is the minimum centre-to-centre distance (diag(a, a)
 *   is M_r of the inter-robot constraint); box = p_min, p_max per problem.
 *
 * 3D (cfg.n_dim = 3; problem formulation and Appendix eqs. inter_robot_polar,
 * workspace_polar, f_e): robots are axis-aligned spheroids with minimum
 * centre distances a (x, y) and b (z), M_r = diag(a, a, b); obstacles are
 * spheroids diag(a_o, a_o, b_o) inflated by the robot.  Layouts change to
 *   coefficient arrays: [3][n_b][n_coef] per problem (x, then y, then z);
 *   boundary: [sum_b n_b][2][3]; obstacles: [sum_b M_b][5] = x, y, z, a_o, b_o;
 *   robot_a (sf_setup): [B][2] = a, b; box: [B][2][3].
 * The paper gives a closed form for the alpha step only (Appendix, after eq.
 * d_step) and refers the beta and d steps to prior work.  This library reads
 * them as: beta = atan2(rho_xy / a, dz / b) with rho_xy = dx cos(alpha) +
 * dy sin(alpha), the polar angle of Delta in the spheroid's scaled coordinates
 * (for a != b this is not the Euclidean argmin of eq. beta_step with d held
 * fixed), and d = max(1, s) with s the scaled length of Delta, the exact
 * minimiser over d >= 1 in scaled coordinates; together they put e on the ray
 * of Delta.  For n_dim = 3, sf_project (SF_SAVE_FOR_BACKWARD, SF_GRAPH,
 * obstacle motion and early exit included) and sf_project_backward run; the
 * adjoint chains through the same alpha, beta and d steps, with the Jacobian
 * of r_1 = (1 - 1/s) Delta on active rows (identity at Delta = 0).  SF_PLAIN
 * and SF_UNFUSED run the forward's stages as separate launches (prep; per
 * iteration the constraint sweep and the update; the final pass) with the
 * same bits; sf_smoothness returns SF_ERR_INVALID_ARG.  Each workgroup visits
 * the candidate partners and obstacles of each robot
 * (sf_set_candidate_lists).
 *
 * Ownership: the caller allocates every array and the workspace; the library
 * owns only the host-side plan.  Calls never retain caller pointers (the
 * forward copies what the backward needs into the workspace).  All work is
 * asynchronous on the given hipStream_t (passed as void*).  Calls on one plan
 * must be serialised by the caller; the workspace of a plan must not be shared
 * with another plan.
 *
 * Errors: functions return 0 on success or a negative SF_ERR_* code and never
 * throw.  sf_last_error_detail() gives a thread-local message for the last
 * failing call.  Numerical divergence inside a problem does not fail the call:
 * it shows in that problem's status word.
 */
#ifndef SF_H_
#define SF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SF_OK 0
#define SF_ERR_INVALID_ARG (-1)     /* NULL pointer, bad count or parameter */
#define SF_ERR_SHAPE (-2)           /* sizes the library cannot handle */
#define SF_ERR_WORKSPACE_SMALL (-3) /* workspace smaller than sf_setup reported */
#define SF_ERR_NOT_SAVED (-4)       /* backward without a saved forward */
#define SF_ERR_HIP (-5)             /* HIP runtime error (detail has the code) */
#define SF_ERR_NONFINITE (-6)       /* non-finite host input */

/* sf_project flags */
#define SF_SAVE_FOR_BACKWARD 1 /* keep checkpoints for sf_project_backward */
#define SF_PLAIN 2             /* unfused per-stage kernels, one problem per launch */
#define SF_GRAPH 4             /* capture the launch once per argument set, replay after */
#define SF_UNFUSED 8           /* the per-stage kernels of SF_PLAIN, each launch covering the
                                  whole batch (batched but unfused) */

typedef struct sf_plan sf_plan_t;

typedef struct {
  int32_t n_dim;            /* workspace dimension n_d: 2, or 3 (spheroids) */
  int32_t n_coef;           /* basis size n_xi per axis, 2..32 (Bernstein, eq. poly) */
  int32_t n_steps;          /* time samples T = K + 1, 2..4096 */
  int32_t checkpoint_every; /* k >= 1: the forward stores (xi_bar, lambda) every k
                               iterates; the backward recomputes the rest */
  int32_t max_iters;        /* largest n_iters a saved forward may use (sizes the
                               checkpoint area); >= 0 */
  int32_t threads;          /* threads per workgroup for the fused kernels:
                               256, 512 or 1024; 0 = autotuned */
  double rho;               /* augmented-Lagrangian penalty rho > 0 (eq. aug_lag) */
  int32_t objective;        /* SF_OBJECTIVE_PROJECTION (0) or SF_OBJECTIVE_ACCEL (1) */
} sf_config_t;

/*
 * Objectives of the xi_bar step.  PROJECTION is the safety filter: the cost
 * 1/2 ||xi_bar - xi||^2 of the projection problem (eq. proj_cost), whose
 * KKT matrix is [I + rho H, A^T; A, 0].  ACCEL replaces the distance to the
 * sample by the smoothness cost 1/2 sum over robots, axes and time samples of
 * the squared second derivative in tau (the trajectory optimiser of the paper's
 * problem formulation, used to build its dataset): the identity block becomes
 * Q = Wdd^T Wdd per robot and axis, Wdd the second tau-derivative of the
 * Bernstein basis at the T samples.  The constraints, their updates and the
 * mode split are unchanged.  With ACCEL the xi argument of sf_project is not
 * read (it may be NULL) and sf_project_backward returns g_xi = 0.
 */
#define SF_OBJECTIVE_PROJECTION 0
#define SF_OBJECTIVE_ACCEL 1

/*
 * Build a plan for a batch of B problems and report the workspace it needs.
 *
 * The KKT matrix of the xi_bar step (Appendix, "Solution Process": M, with
 * the workspace terms rho G^T G kept) does not depend on xi, so its inverse is
 * factored once here, in FP64 on the host, per distinct (robot, obstacle)
 * count, and stored in float32 (Appendix, eq. batch_comp and the remark
 * before it: the matrix does not depend on the sample, so its factor is
 * computed ahead of the iterations; it must be rebuilt when rho or the basis
 * changes).
 *
 *   cfg            host; see sf_config_t.
 *   n_problems     B >= 1.
 *   n_robots       host int32[B], each 1..64 for n_dim = 2, 1..1024 for n_dim =
 *                  3 (a problem's state must also fit
 *                  the LDS of one workgroup, else SF_ERR_SHAPE).
 *   n_obs          host int32[B], each 0..4096.
 *   robot_a        host float[B], a > 0 (n_dim = 3: float[B][2] = a, b > 0).
 *   box            host float[B][2][n_dim] = p_min, p_max; p_min < p_max per axis.
 *   workspace      NULL: only *workspace_bytes is set and *plan is left alone.
 *                  Otherwise a device buffer of at least *workspace_bytes bytes,
 *                  256-byte aligned, that this plan uses until sf_destroy; the
 *                  plan's constant tables are copied into it on `stream`.
 *   workspace_bytes in/out: required size (out); with a workspace, its size (in).
 *   stream         hipStream_t or NULL (default stream).
 *   plan           out: the new plan (only when workspace != NULL).
 */
int sf_setup(const sf_config_t* cfg, int32_t n_problems, const int32_t* n_robots,
             const int32_t* n_obs, const float* robot_a, const float* box,
             void* workspace, size_t* workspace_bytes, void* stream, sf_plan_t** plan);

/*
 * Run n_iters applications of the fixed-point operator T (eq. fixed_point)
 * from the warm start (xi_bar^0, lambda^0) (eq. NN_loss's initialisation) for
 * every problem of the plan, and report the residual of the returned iterate
 * (eq. primal_residual, read as sqrt(||r_1||^2 + ||r_2||^2)).
 *
 * One iteration (Appendix, eqs. alpha_step..xi_step, in the order given there):
 * closed-form alpha/d steps on every robot pair and robot-obstacle pair at every
 * time sample, the slack s step, lambda^{l+1} = lambda^l - rho F^T r_1 -
 * rho G^T r_2, and the equality-constrained xi_bar step.
 *
 *   xi          flow sample xi (the projection target), coefficient layout.
 *   xi0, lam0   warm start, coefficient layout.
 *   boundary    [sum n][2][n_dim]; obstacles [sum M][3] ([sum M][5] for n_dim = 3;
 *               may be NULL if sum M = 0).
 *   n_iters     L >= 0 (L = 0 copies the warm start and reports its residual).
 *   flags       SF_SAVE_FOR_BACKWARD | SF_PLAIN | SF_UNFUSED | SF_GRAPH.  Saving
 *               requires n_iters <= cfg.max_iters and is not combined with
 *               SF_PLAIN or SF_UNFUSED; SF_PLAIN and SF_UNFUSED exclude each
 *               other.  All paths compute the same bits.
 *   xi_out, lam_out  coefficient layout, must not alias the inputs.
 *   residual    [B][4] (see the layout notes above).
 * Input arrays are read during the call's kernels only.
 */
int sf_project(sf_plan_t* plan, void* workspace, const float* xi, const float* xi0,
               const float* lam0, const float* boundary, const float* obstacles,
               int32_t n_iters, int32_t flags, float* xi_out, float* lam_out,
               float* residual, void* stream);

/*
 * Vector-Jacobian product of the last saved sf_project call (the unrolled
 * chain of T, Sec. "Fixed-Point Representation"; "Differentiability" in the
 * Appendix), for the scalar
 *   <g_xi_out, xi_bar^L> + <g_lam_out, lambda^L>
 *   + sum_b (g_residual[b][0] ||r_1|| + g_residual[b][1] ||r_2||)
 *   + fp_weight * sum_l ||z^{l+1} - z^l||^2   (eq. NN_loss's L_FP terms).
 * Iterates between checkpoints are recomputed.  Non-smooth points: a pair
 * exactly at distance a, or a coordinate exactly on a box bound, counts as
 * inactive; norm gradients at a zero norm are zero.
 *
 *   g_xi_out, g_lam_out  coefficient layout; either may be NULL (= zero).
 *   g_residual           [B][4] or NULL; columns 2 and 3 are ignored.
 *   g_xi, g_xi0, g_lam0  outputs, coefficient layout; each may be NULL (skipped).
 * Returns SF_ERR_NOT_SAVED unless the latest sf_project on this plan saved.
 */
int sf_project_backward(sf_plan_t* plan, void* workspace, const float* g_xi_out,
                        const float* g_lam_out, const float* g_residual, float fp_weight,
                        float* g_xi, float* g_xi0, float* g_lam0, void* stream);

/*
 * sf_project_backward for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same reverse sweep and the same results, bit for bit, but the iterates a
 * checkpoint segment recomputes go to a static device array of the library
 * (32 MiB per GPU, held from the first use on that GPU until the process ends)
 * instead of the plan's workspace, and the thread count is not autotuned (the
 * plan's current choice is used).  The call allocates nothing.
 *
 * Same arguments, layouts and errors as sf_project_backward, plus
 * SF_ERR_SHAPE when the recompute area, 8 * checkpoint_every * (floats of one
 * coefficient array of the batch) bytes, exceeds 32 MiB.  Every call on one
 * GPU shares the array: calls that overlap in time on one GPU (other streams,
 * other threads, other plans) race and must be serialised by the caller.
 */
int sf_project_backward_static(sf_plan_t* plan, void* workspace, const float* g_xi_out,
                               const float* g_lam_out, const float* g_residual,
                               float fp_weight, float* g_xi, float* g_xi0, float* g_lam0,
                               void* stream);

/* Free the plan (host memory and cached graphs).  NULL is accepted.  The
 * workspace stays the caller's. */
void sf_destroy(sf_plan_t* plan);

/* Static description of an SF_* code. */
const char* sf_error_string(int code);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char* sf_last_error_detail(void);

/* Threads per workgroup the plan's fused kernels use (after autotuning). */
int sf_plan_threads(const sf_plan_t* plan);

/*
 * Forward generation of the plan: the number of sf_project calls (and
 * sf_set_obstacle_motion calls) made on it so far, -1 for a NULL plan.
 * sf_project_backward always differentiates the latest saved forward; a
 * caller that keeps several forwards alive (an autograd graph, say) records
 * the generation right after its sf_project and compares it before
 * sf_project_backward: a different value means a later call replaced the
 * saved state that this backward would use.
 */
int64_t sf_forward_generation(const sf_plan_t* plan);

/*
 * Optional per-problem early exit of later sf_project calls on this plan
 * (iteration control around eq. fixed_point; the residual is that of eq.
 * primal_residual, read as sqrt(||r_1||^2 + ||r_2||^2)).  With check_every = c
 * > 0, at every iteration l that is a multiple of c the residual of the
 * current iterate xi_bar^l is formed as part of that iteration's constraint
 * pass (n_dim = 3: by a residual pass just before it); if it is <= tol, the
 * problem completes iteration l and stops, so it
 * returns xi_bar^{l+1}, lambda^{l+1} (and their residual, as always).  Other
 * problems of the batch continue.  n_iters stays the upper bound.  The
 * iterations each problem ran are available from sf_project_iterations, and
 * sf_project_backward differentiates each problem's own chain.
 *
 *   tol          >= 0, finite (metres).
 *   check_every  0 turns early exit off (the default); otherwise >= 1.
 * Not available with SF_PLAIN or SF_UNFUSED (sf_project then fails with
 * SF_ERR_INVALID_ARG).
 */
int sf_set_early_exit(sf_plan_t* plan, float tol, int32_t check_every);

/*
 * n_dim = 3: switch the candidate lists of the constraint pass on (the
 * default) or off for later sf_project and sf_project_backward calls.  The
 * spheroid rows of eqs. inter_robot_polar and workspace_polar add nothing
 * unless the scaled offset lies inside the unit ball, so each robot keeps,
 * per 16-step window, a list of the partners and obstacles that can reach it
 * there (window boxes widened by a skin, rebuilt when a coefficient has moved
 * further than the skin since the last build) and visits only those, in the
 * same order as the full pass: both give the same bits.  Off, every pair and
 * obstacle is visited at every step (for verification and timing).
 *
 *   enable   0 = off, otherwise on.
 * Returns 1 when the lists are in use after the call, 0 when they are off
 * (switched off, or their LDS did not fit at sf_setup), SF_ERR_INVALID_ARG
 * for a NULL plan or n_dim = 2 (the planar fused kernels always use lists;
 * SF_PLAIN visits every pair).
 */
int sf_set_candidate_lists(sf_plan_t* plan, int32_t enable);

/*
 * Copy the number of iterations each problem ran in the last sf_project call
 * on this plan (n_iters for every problem without early exit) into iters,
 * device int32[B], asynchronously on stream.
 */
int sf_project_iterations(const sf_plan_t* plan, const void* workspace, int32_t* iters,
                          void* stream);

/*
 * Moving obstacles (the dynamic-obstacle scenarios of the paper's evaluation,
 * where obstacles come with their velocity): obstacle m's centre at
 * tau = k / (T - 1) is c_m + d_m tau, with d_m the displacement over the
 * horizon (velocity times its duration).  displacement: device
 * float[sum M][n_dim] in the obstacles' order, copied into the workspace (asynchronously on
 * stream); NULL makes every obstacle static again (the default).  It applies
 * to later sf_project calls and invalidates a saved forward.  The constraint
 * stage, the candidate lists (per-window obstacle boxes) and the adjoint use
 * the moving centres; the centres do not depend on xi, so the adjoint gains
 * no term.
 */
int sf_set_obstacle_motion(sf_plan_t* plan, void* workspace, const float* displacement,
                           void* stream);

/*
 * Candidate selection around the SF (the planning pipeline of the paper's
 * "Validation and Benchmarking" section: its three-stage figure and
 * "Qualitative Validation").  Sampled candidate trajectories of one context
 * are ranked by their primal residual (eq. primal_residual), the k best are
 * refined by sf_project, and the refined candidate returned is the feasible
 * one with the least smoothness cost.  A candidate's residual row is the
 * [4]-row of sf_project (n_iters = 0 gives the residual of the warm start, i.e.
 * of the raw sample when xi0 = xi); its ranking key is ||r_1||^2 + ||r_2||^2
 * in float32 with each operation rounded separately, +inf when the status word
 * is set or the key is not finite.  Ties go to the lower index.
 */

/*
 * Smoothness cost of each problem's trajectory xi (the plan's coefficient
 * layout): (1/n) sum_i sum_k |d^2 p_i/dt^2 (t_k)|^2, the squared acceleration
 * norm summed over the T time steps and averaged over the robots ("Smoothness
 * Cost" of "Implementation Details"), with t = tau t_final.  cost: device
 * float[B].  t_final > 0 (seconds).  Asynchronous on stream.
 */
int sf_smoothness(const sf_plan_t* plan, const void* workspace, const float* xi,
                  float t_final, float* cost, void* stream);

/*
 * Indices of the k candidates with the smallest ranking keys, in increasing
 * key order (ties: lower index first).  residual: device float[n][4];
 * idx: device int32[k].  1 <= k <= n <= 8192.  Asynchronous on stream.
 */
int sf_rank_residual(const float* residual, int32_t n_candidates, int32_t k, int32_t* idx,
                     void* stream);

/*
 * Index of the chosen candidate: among those whose key is <= tol^2 (tol^2
 * rounded in float32; "feasible") the least cost, ties by key then index;
 * when none is feasible, the least key, ties by index.  A non-finite cost
 * counts as +inf.  residual: device float[n][4]; cost: device float[n];
 * idx: device int32[1].  1 <= n <= 8192, tol >= 0.  Asynchronous on stream.
 */
int sf_select_best(const float* residual, const float* cost, int32_t n_candidates, float tol,
                   int32_t* idx, void* stream);

/*
 * Gather of equal-size blocks (e.g. the coefficient blocks of candidates that
 * share n): dst[q] = src[idx[q]] for q < k, blocks of block_floats floats.
 * src: device float[n_blocks][block_floats]; idx: device int32[k]; dst:
 * device float[k][block_floats].  An index outside 0..n_blocks-1 yields a
 * block of NaN.  k <= 65535.  Asynchronous on stream.
 */
int sf_gather_blocks(const float* src, int32_t n_blocks, const int32_t* idx, int32_t k,
                     int32_t block_floats, float* dst, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SF_H_ */
