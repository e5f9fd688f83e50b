/*
 * rpba.h -- C ABI of librpba, the MI355X (gfx950) implementation of the
 * data-parallel hot path of covariance-weighted consensus bundle adjustment
 * (H. Mayer, "RPBA: Robust Parallel Bundle Adjustment Based on Covariance
 * Information", arXiv 1910.08138).
 *
 * Problem statement (paper Sec. 2): cameras P_i (here rotation R_i, world to
 * camera, and projection centre C_i), points X_j, observations x_k of point j
 * in camera i with 2x2 covariance C_xk (weight W_k = C_xk^-1), residual
 * v_k = g_k(P_i, X_j) - x_k with the calibrated pinhole
 *     p = R_i (X_j - C_i),  g = (f p1/p3 + cx, f p2/p3 + cy).
 * The cameras are split into L sub-blocks and each camera belongs to exactly
 * one of them (Sec. 4); points seen by cameras of two or more sub-blocks are
 * tie points (TPs).
 *
 * One outer iteration of the method (Sec. 5) is
 *     rpba_intersect          eq:bars + refined re-weighting (Sec. 5.1)
 *     [rpba_robust_reweight + rpba_intersect]   parallel robust variant (Sec. 5.3)
 *     rpba_subblock_lm_step   eq:bact, one LM iteration per call (Sec. 5.4)
 *     rpba_consensus          exchange of cameras and TPs (Sec. 5)
 *
 * Memory: every pointer argument is a DEVICE pointer unless it is marked
 * HOST.  All device memory (including the workspace) is allocated and owned
 * by the caller; the library never allocates or frees device memory.  The
 * handle is host memory owned by the library, released by rpba_destroy.  All
 * buffers named in the descriptor must outlive the handle.
 *
 * Asynchrony: every call except rpba_workspace_size / rpba_create only
 * enqueues kernels on the stream given at creation and returns.  Results
 * (stats, covariances, statuses) are in device memory; read them after
 * synchronising the stream.  rpba_create synchronises once.
 *
 * Errors: calls return a status code; no exception crosses the ABI.
 * rpba_last_error() returns a thread-local description of the last failure.
 * One host thread at a time per handle.
 */
#ifndef RPBA_H
#define RPBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPBA_OK = 0,
  RPBA_ERR_ARG = 1,        /* invalid argument or problem (message says which) */
  RPBA_ERR_HIP = 2,        /* a HIP runtime call failed */
  RPBA_ERR_WORKSPACE = 3,  /* workspace too small or misaligned (256 B) */
  RPBA_ERR_NOT_SPD = 4,    /* a reduced camera system was not positive definite */
  RPBA_ERR_STATE = 5,      /* call not valid in the handle's state */
  RPBA_WARN_NONCONVERGED = 100 /* an iterative solve ended above its tolerance (rpba_step_status) */
} rpba_status;

/* precision policy */
enum { RPBA_FP64 = 0, RPBA_MIXED = 1 };
/* solver of the reduced camera system: Cholesky everywhere; PCG everywhere
 * (block-Jacobi or learned blocks); AUTO: PCG with block-Jacobi on the
 * sub-blocks of at least pcg_min_cams cameras, Cholesky on the others;
 * AUTO_LEARNED: the same cut, PCG with the learned blocks */
enum { RPBA_SOLVER_CHOL = 0, RPBA_SOLVER_PCG_BJ = 1, RPBA_SOLVER_PCG_LEARNED = 2, RPBA_SOLVER_AUTO = 3,
       RPBA_SOLVER_AUTO_LEARNED = 4 };
/* schedule of the dense Cholesky factorisation: one persistent launch over
 * a tile task list with per-tile ready flags (dataflow), or three launches
 * per tile column (stepwise) */
enum { RPBA_CHOL_DEFAULT = 0, RPBA_CHOL_STEPWISE = 1, RPBA_CHOL_DATAFLOW = 2 };
/* per-point status written by rpba_intersect */
enum {
  RPBA_PT_OK = 0,
  RPBA_PT_NOT_CONVERGED = 1, /* Gauss-Newton did not reach int_tol in int_maxit iterations */
  RPBA_PT_BEHIND = 2,        /* some p3 <= 0 */
  RPBA_PT_ILL = 3,           /* 3x3 Cholesky pivot <= 1e-12 * largest diagonal */
  RPBA_PT_ELIMINATED = 4,    /* removed by the robust step */
  RPBA_PT_FILTERED = 5       /* plain variants: |X| > 1e10 or a reprojection error above filter_px */
};
/* variant of the method (Sec. 4 and the comparisons of Sec. 6.3-6.4):
 *   EXTENDED       the covariance-weighted consensus: every point intersected
 *                  (eq:bars), tie-point copies weighted by the information
 *                  from the cameras outside their sub-block (Sec. 5.1)
 *   ALL_CAMERAS    as EXTENDED, tie-point copies weighted by the information
 *                  from all cameras (Omega = H)
 *   SCALAR         as EXTENDED, tie-point copies weighted by rho_t I
 *   PLAIN          ADMM consensus (eq:admm7-eq:admm9): no intersection; a
 *                  tie-point copy is pulled towards X_j - Xtilde_j^l with
 *                  weight rho_t I, the consensus averages the copies (X_j)
 *                  and updates Xtilde_j^l += X_j^l - X_j; rpba_intersect only
 *                  evaluates the residuals at X_j (and applies the filters)
 *   PLAIN_REFINED  PLAIN with the tie-point weights of Sec. 5.1 evaluated at
 *                  X_j (Omega = H - H^(l), points not moved)
 * rho_t = rho * rho_growth^t after t calls of rpba_consensus. */
enum { RPBA_VARIANT_EXTENDED = 0, RPBA_VARIANT_ALL_CAMERAS = 1, RPBA_VARIANT_SCALAR = 2, RPBA_VARIANT_PLAIN = 3,
       RPBA_VARIANT_PLAIN_REFINED = 4 };
/* damping of the LM steps (Sec. 5.4 fixes lambda; adapting it is the
 * alternative the paper names, Sec. 5.4 and 7): ADAPTIVE keeps one lambda per
 * sub-block, starting at opt->lambda; a step that raises the sub-block's cost
 * (or whose system cannot be factorised) is taken back and lambda multiplied
 * by lambda_up, an accepted step divides it by lambda_down. */
enum { RPBA_DAMPING_FIXED = 0, RPBA_DAMPING_ADAPTIVE = 1 };
/* what rpba_robust_reweight does with flagged observations (Sec. 5.3) */
enum { RPBA_ROBUST_WEIGHT = 0, RPBA_ROBUST_ELIMINATE_POINTS = 1, RPBA_ROBUST_DELETE_OBS = 2 };

typedef struct rpba_problem rpba_problem;

typedef struct {
  int32_t M, N, K, L;        /* cameras, points, observations, sub-blocks */
  double f, cx, cy;          /* shared pinhole intrinsics [px] */
  double sigma_px;           /* a-priori std. dev. of an image coordinate; W = I / sigma^2 when obs_info is NULL */
  double *cam_R;             /* [M][9] row-major world->camera rotation; read at create, written by rpba_consensus */
  double *cam_C;             /* [3][M] projection centres (SoA); same ownership as cam_R */
  double *pts;               /* [3][N] points (SoA); read at create (start values), written by rpba_intersect / rpba_consensus */
  const double *obs_xy;      /* [2][K] measured pixel coordinates (SoA) */
  const double *obs_info;    /* [3][K] (w11, w12, w22) of W_k = C_xk^-1, or NULL */
  const int32_t *obs_cam;    /* HOST [K] camera of each observation, in [0, M) */
  const int32_t *obs_pt;     /* HOST [K] point of each observation, in [0, N) */
  const int32_t *cam_block;  /* HOST [M] sub-block of each camera, in [0, L) */
  double *cam_intr;          /* [2][M] (f, k1) of every camera (SoA) when opt->intrinsics = 1, else ignored (may be
                                NULL); same ownership as cam_R */
} rpba_problem_desc;

typedef struct {
  int32_t precision;     /* RPBA_FP64 or RPBA_MIXED */
  int32_t solver;        /* RPBA_SOLVER_* */
  double lambda;         /* LM damping, N + lambda diag(N) (Sec. 5.4): 1e-4 */
  double int_tol;        /* intersection stop: |dX| <= int_tol (1 + |X|): 1e-12 */
  int32_t int_maxit;     /* intersection iterations: 20 */
  int32_t pcg_maxit;     /* PCG iterations per refinement sweep: 200 */
  double pcg_tol;        /* PCG relative residual: 1e-8 */
  double ir_tol;         /* iterative refinement relative residual (FP64): 1e-10 */
  int32_t ir_maxit;      /* refinement sweeps: 6 */
  int32_t pcg_min_cams;  /* RPBA_SOLVER_AUTO(_LEARNED): sub-blocks with at least this many cameras use PCG: 150 */
  double t_v;            /* robust threshold on the normalised residual (Sec. 5.3): 4 (parallel variant; the
                            serial variant uses 3) */
  double down_weight;    /* weight multiplier of flagged observations: 1e-4 */
  int32_t chol_tile;     /* Cholesky tile edge, 32 or 64 (0 = library choice) */
  int32_t chol_schedule; /* RPBA_CHOL_*; DEFAULT = dataflow */
  int32_t robust;        /* 1: the intersection keeps its residuals for rpba_robust_reweight (Sec. 5.3);
                            0: it does not, and rpba_robust_reweight returns RPBA_ERR_STATE: 0 */
  int32_t pair_lanes;    /* lanes per camera-pair block in the Schur pass: 4, 8 or 16 (0 = 8) */
  int32_t variant;       /* RPBA_VARIANT_*: EXTENDED */
  double rho;            /* scalar tie-point weight of SCALAR / PLAIN variants [1/unit^2]: 1000 */
  double rho_growth;     /* factor applied to rho at every rpba_consensus (Sec. 6.3): 1.01 */
  double filter_px;      /* PLAIN variants: a point with a reprojection error above this is filtered: 1000 */
  int32_t covariance;    /* 1: the workspace holds one more array of the size of the dense RCS, for
                            rpba_covariance: 0 */
  int32_t damping;       /* RPBA_DAMPING_FIXED (lambda throughout) or RPBA_DAMPING_ADAPTIVE: FIXED */
  double lambda_up;      /* adaptive: factor on a sub-block's lambda after a rejected step: 10 */
  double lambda_down;    /* adaptive: divisor after an accepted step: 10 */
  double lambda_min;     /* adaptive: bounds of lambda: 1e-12 */
  double lambda_max;     /*   : 1e8 */
  int32_t intrinsics;    /* 1: every camera has its own focal length f and first radial distortion parameter k1,
                            estimated with its pose (Sec. 6, the n (6 + 2) camera parameters of the Final data
                            sets): pixel f (1 + k1 |q|^2) q + (cx, cy) with q = (p1/p3, p2/p3), start values in
                            desc->cam_intr, desc->f unused, 8 rows of the reduced camera system per camera.
                            Needs RPBA_SOLVER_CHOL and RPBA_VARIANT_EXTENDED (RPBA_ERR_ARG otherwise).  0: the
                            shared pinhole desc->f: 0 */
} rpba_options;

/* Fill *opt with the defaults listed above.  HOST pointer. */
rpba_status rpba_default_options(rpba_options *opt);

/* Bytes of device workspace rpba_create needs for this problem (host-side
 * planning; reads the HOST topology arrays only).  *bytes is HOST. */
rpba_status rpba_workspace_size(const rpba_problem_desc *desc, const rpba_options *opt, size_t *bytes);

/* Validate the problem, plan the data layout (Sec. 4: camera-unique split,
 * TPs derived from it) and pack the observation streams into the workspace.
 * Checks: indices in range, every point observed at least twice, every
 * camera observed at least once, every sub-block non-empty, no repeated
 * (camera, point) pair (host, on the topology arrays); every value of cam_R,
 * cam_C, pts, obs_xy and obs_info finite and every obs_info matrix positive
 * definite (one device reduction; RPBA_ERR_ARG names the counts).
 * `workspace` is a device buffer of at
 * least rpba_workspace_size bytes, 256-byte aligned, owned by the caller for
 * the life of the handle.  `stream` is a hipStream_t (NULL = default).
 * *out is HOST. */
rpba_status rpba_create(const rpba_problem_desc *desc, const rpba_options *opt, void *workspace, size_t bytes,
                        void *stream, rpba_problem **out);

/* Intersection of every valid point with all cameras fixed (eq:bars): undamped
 * Gauss-Newton on the point, covariance Sigma_j = (sum B^T W B)^-1, and for
 * each (point, sub-block) copy the refined weight Omega_j^l = H_j - H_j^(l),
 * the point information from cameras outside l (Sec. 5.1).  The point
 * position uses all cameras.  Sets every copy X_j^l = Xbar_j.  Points that
 * fail get a non-zero status and weight zero from then on (Sec. 5.4).
 *   cov    [6][N] (xx, xy, xz, yy, yz, zz) or NULL
 *   status [N] RPBA_PT_* or NULL
 *   stats  [4]: weighted cost sum v^T W v, sigma0 [px] (unit weights,
 *          redundancy 2K_valid - n_p M - 3N_valid, eq:sigma0, n_p = 6 or 8
 *          with intrinsics), RMS [px], N_valid;
 *          or NULL
 * Writes Xbar to desc->pts. */
rpba_status rpba_intersect(rpba_problem *h, double *cov, int32_t *status, double *stats);

/* Robust estimation (Sec. 5.3), for a handle created with opt->robust = 1
 * (else RPBA_ERR_STATE), after rpba_intersect: per camera, sigma0_i = 1.4826
 * MAD of the whitened residual components of the last intersection (over the
 * observations of valid points that are not deleted); an observation with
 * sqrt(v^T W v) / sigma0_i > opt->t_v is flagged.  mode:
 *   RPBA_ROBUST_WEIGHT: flagged observations get the weight multiplier
 *     opt->down_weight, every other observation 1 (both variants, after basic
 *     convergence);
 *   RPBA_ROBUST_ELIMINATE_POINTS: the same, and every point with a flagged
 *     observation gets RPBA_PT_ELIMINATED (parallel variant, at the end;
 *     t_v = 4);
 *   RPBA_ROBUST_DELETE_OBS: flagged observations are deleted (multiplier 0)
 *     and a flagged point left with fewer than two observations gets
 *     RPBA_PT_ELIMINATED (serial variant, at the end; t_v = 3).
 * A deleted observation stays deleted in later calls: it enters no scale,
 * flag, cost or statistic.  Any other mode: RPBA_ERR_ARG.
 * stats [2]: flagged observations, eliminated points (or NULL). */
rpba_status rpba_robust_reweight(rpba_problem *h, int32_t mode, double *stats);

/* Covariances of the sub-block adjustment (Sec. 2: M = N^-1 through the
 * Schur complement; the paper sets lambda = 1e-6 after convergence for them,
 * Sec. 5.4), for a handle created with opt->covariance = 1 (else
 * RPBA_ERR_STATE), after rpba_intersect, with no sub-block solved by PCG
 * (else RPBA_ERR_STATE).  At the current state (the cameras, and the copies
 * as the next LM step would take them) the normal equations of every
 * sub-block are assembled with damping `lambda` (N + lambda diag N), the
 * reduced camera system S is factorised and inverted, and
 *   cam_cov  [M][n_p][n_p] DEVICE, row-major, caller camera order: the
 *                       camera's diagonal block of S^-1 (rotation increment,
 *                       centre, with intrinsics f and k1; n_p = 6 or 8), or
 *                       NULL;
 *   copy_cov [NC][6]    DEVICE, copy order of rpba_get_copies: the point
 *                       block M_XX = V^-1 + V^-1 (sum_{i,k} Y_i^T (S^-1)_ik
 *                       Y_k) V^-1 of the copy (xx, xy, xz, yy, yz, zz), V its
 *                       damped point block with the tie-point weight, Y_i
 *                       the camera-point block of its observation in camera
 *                       i; zeros for copies of invalid points; or NULL.
 * The parameters of the camera and point blocks are those of the LM step.
 * A camera or copy covariance is that of the sub-block's system, i.e. with
 * the tie points weighted by the information from the other sub-blocks.
 * RPBA_ERR_NOT_SPD if a system is not positive definite; RPBA_ERR_ARG for a
 * negative or non-finite lambda.  Leaves the state unchanged; the next LM
 * step re-assembles its system.  Asynchronous on the handle's stream after
 * one synchronisation (the factorisation check). */
rpba_status rpba_covariance(rpba_problem *h, double lambda, double *cam_cov, double *copy_cov);

/* Per sub-block damping (HOST lambda [L]) and whether its last step was
 * taken back (HOST rejected [L]); with RPBA_DAMPING_FIXED lambda and 0.
 * Either may be NULL.  Synchronises the handle's stream. */
rpba_status rpba_get_damping(rpba_problem *h, double *lambda, int32_t *rejected);

/* Result of the last rpba_robust_reweight: sigma_cam [M] the per-camera
 * scales sigma0_i (0 for a camera without a valid observation), obs_weight
 * [K] the weight multipliers (1 or down_weight), both HOST, in the caller's
 * camera and observation order; either may be NULL.  Synchronises the
 * handle's stream. */
rpba_status rpba_get_robust(rpba_problem *h, double *sigma_cam, double *obs_weight);

/* One LM iteration of every active sub-block (eq:bact): normal equations of
 * the sub-block's cameras and point copies with the TPs as stochastic control
 * points, cost sum v^T W v + (X - Xbar)^T Omega (X - Xbar); damping
 * N + lambda diag(N); Schur complement onto the cameras (reduced camera system
 * S, outer products accumulated straight into S); S solved by Cholesky
 * (FP64 MFMA) or PCG; back-substitution; update R <- Exp([w]x) R, C += dc,
 * X^l += dX.  With RPBA_DAMPING_FIXED every step is accepted; with
 * RPBA_DAMPING_ADAPTIVE a step that raises its sub-block's cost is taken back
 * (block_stats: cost after = cost before, step norm 0) and the sub-block's
 * lambda adapted (rpba_get_damping).
 *   active      [L] uint8 (0 = skip) or NULL for all
 *   block_stats [L][4]: cost before, cost after, step norm, solver iterations
 *               (or NULL) */
rpba_status rpba_subblock_lm_step(rpba_problem *h, const uint8_t *active, double *block_stats);

/* Outcome of the last rpba_subblock_lm_step, per sub-block (synchronises the
 * handle's stream).  A sub-block whose reduced camera system had a
 * non-positive Cholesky pivot (or a non-positive-definite 6x6 diagonal block
 * under PCG) is counted in *n_not_spd; its cameras and point copies were left
 * unchanged (block_stats: cost after = cost before, iterations -1).  An
 * iterative sub-block whose FP64 refinement residual |e - S x| / |e| ended
 * above ir_tol is counted in *n_nonconverged; its step was applied.  Both
 * outputs HOST, either may be NULL.  Returns RPBA_ERR_NOT_SPD if any
 * sub-block failed, else RPBA_WARN_NONCONVERGED if any did not converge,
 * else RPBA_OK. */
rpba_status rpba_step_status(rpba_problem *h, int32_t *n_not_spd, int32_t *n_nonconverged);

/* Improvement test that ends a loop (Sec. 5.4), for n loops at once (one per
 * sub-block for the inner LM loop, or one for the outer loop on the RMS).
 * HOST arrays, no GPU work.  For every loop q with active[q] != 0 the step
 * with cost[q] is short when best[q] / cost[q] < ratio (1.01); the first
 * short step is tolerated (grace[q] = 1), the second ends the loop
 * (active[q] = 0); then best[q] = min(best[q], cost[q]).  Start a loop with
 * best = the cost before its first step, grace = 0, active = 1.  Returns the
 * number of loops still active, or -1 for a NULL array or n < 0. */
int32_t rpba_ratio_update(int32_t n, const double *cost, double ratio, double *best, uint8_t *grace, uint8_t *active);

/* Consensus exchange (Sec. 5): cameras go back to desc->cam_R / cam_C (and
 * with intrinsics their f and k1 to desc->cam_intr); every
 * point's start value for the next intersection is the mean of its sub-block
 * copies (eq:admm8 form), written to desc->pts.  PLAIN variants also update
 * the copies' dual offsets (eq:admm9); every variant then multiplies rho_t by
 * rho_growth.
 *   stats [2]: largest distance of a copy from its point's mean, number of TPs
 *         (or NULL) */
rpba_status rpba_consensus(rpba_problem *h, double *stats);

/* Wait for the work queued on the handle's stream, then release the handle
 * (host memory only; caller buffers are untouched and may be freed once this
 * returns). */
rpba_status rpba_destroy(rpba_problem *h);

/* Thread-local message of the last non-OK status. */
const char *rpba_last_error(void);

/* ---------------------------------------------------------------- inspection
 * Synchronous helpers for tests and tools; all pointers HOST.
 * rpba_num_copies: number of (sub-block, point) copies.
 * rpba_get_copies: copies in library order with sub-block, original point
 *   index, X^l [n][3] and Omega [n][6]; any pointer may be NULL.
 * rpba_get_block_rcs: assembles the reduced camera system of every sub-block at
 *   the current state (as an LM step would, without solving) and copies S of
 *   sub-block l (n6 x n6 row-major, both triangles: the mirrored lower
 *   triangle for Cholesky sub-blocks, the stored FP32 blocks for iterative
 *   ones) and e; n6 = n_p cameras of l (n_p = 6, or 8 with intrinsics),
 *   cameras in ascending original index
 *   (the library orders the cameras of a sub-block by its own rule and
 *   reorders the copy).
 * rpba_block_cameras: number of cameras of sub-block l. */
int64_t rpba_num_copies(rpba_problem *h);
rpba_status rpba_get_copies(rpba_problem *h, int32_t *blk, int32_t *pt, double *X, double *omega);
rpba_status rpba_get_block_rcs(rpba_problem *h, int32_t l, double *S, double *e);
int32_t rpba_block_cameras(rpba_problem *h, int32_t l);
/* rpba_get_block_solution: the camera step (n6 values) of sub-block l from the
 * last rpba_subblock_lm_step, cameras in ascending original index.
 * rpba_block_solver: 0 = Cholesky, 1 = iterative.
 * rpba_camera_order: cam_orig[M] = the caller's index of every camera in the
 *   library's order (the order of the preconditioner's probe vectors and
 *   training samples).
 * rpba_get_precond_blocks: the 6x6 CG preconditioner blocks (row-major) of the
 *   cameras of iterative sub-block l used by the last rpba_subblock_lm_step,
 *   P [ncam][36], cameras in ascending original index. */
rpba_status rpba_get_block_solution(rpba_problem *h, int32_t l, double *x);
int32_t rpba_block_solver(rpba_problem *h, int32_t l);
rpba_status rpba_camera_order(rpba_problem *h, int32_t *cam_orig);
/* rpba_factor_flops: work of one factorisation of the sub-blocks solved by
 *   Cholesky (Sec. 2), HOST out[3]:
 *   [0] the method's FP64 operations on the tiles the factor can hold (tiles
 *       that stay zero are skipped): T^3/3 per diagonal factor, T^3 per panel
 *       solve, 2 T^3 per tile product below the diagonal and T^3 per product
 *       onto a diagonal tile, plus the forward substitution folded into the
 *       right-hand-side row (2 T^2 per product, T^2 per solve);
 *   [1] the dense count sum over the sub-blocks of (n_p n)^3/3 + (n_p n)^2;
 *   [2] the FP64 matrix-core operations the persistent launch issues: 2 T^3
 *       per tile product and panel solve (right-hand-side row included) and
 *       the 16 x 16 block products inside every diagonal tile. */
rpba_status rpba_factor_flops(rpba_problem *h, double *out);
rpba_status rpba_get_precond_blocks(rpba_problem *h, int32_t l, double *P);

/* ------------------------------------------------ learned block preconditioner
 * With RPBA_SOLVER_PCG_LEARNED or _AUTO_LEARNED the CG preconditioner keeps the block-diagonal
 * form of block-Jacobi (paper Sec. 3 and 5.4) with blocks
 * P_i = G^-T L L^T G^-1, S_ii = G G^T, L = I + strict lower part from a
 * 26 -> 64 -> 64 -> 21 network (tanh) on per-camera features, exp(.) on the
 * diagonal: SPD for any output, block-Jacobi for a zero output (the default
 * until weights are set).
 * rpba_precond_num_params: number of FP32 network parameters (W1[64][26],
 *   b1[64], W2[64][64], b2[64], W3[21][64], b3[21]).
 * rpba_set_precond_weights: copy the parameters (DEVICE, FP32) into the
 *   workspace.
 * rpba_precond_num_samples: cameras of the iterative sub-blocks.
 * rpba_precond_sample_stride: floats per training sample for nz probes:
 *   features (26), G^-1 (36, row-major lower), z_i (6 nz), (S z)_i (6 nz).
 * rpba_precond_harvest: assemble the systems at the current state and write one
 *   sample per camera of the iterative sub-blocks; z: DEVICE [nz][M][6] probe
 *   vectors indexed by the library's camera order (random signs supplied by
 *   the caller); out: DEVICE [samples][stride].
 * rpba_precond_train_scratch: bytes of DEVICE scratch for rpba_precond_train_step.
 * rpba_precond_train_step: on `stream`, the loss
 *   (1 / (nz nsamp)) sum |z_i - P_i (S z)_i|^2 of the samples and its gradient
 *   (grad[NPAR], DEVICE); with `apply`, one Adam step (beta 0.9 / 0.999,
 *   eps 1e-8, step count t >= 1) on W with moments m, v (DEVICE).  loss: DEVICE
 *   [1] or NULL. */
int32_t rpba_precond_num_params(void);
rpba_status rpba_set_precond_weights(rpba_problem *h, const float *W);
int32_t rpba_precond_num_samples(rpba_problem *h);
int32_t rpba_precond_sample_stride(int32_t nz);
rpba_status rpba_precond_harvest(rpba_problem *h, const float *z, int32_t nz, float *out);
size_t rpba_precond_train_scratch(int32_t nsamp);
rpba_status rpba_precond_train_step(const float *samples, int32_t nsamp, int32_t nz, float *W, float *m, float *v,
                                    int32_t t, float lr, void *scratch, float *grad, float *loss, int32_t apply,
                                    void *stream);

/* rpba_precond_train_step_noalloc: the same training step for callers that
 *   cannot allocate device memory (code under HIP graph capture, tight
 *   serving or training loops, harnesses that forbid hipMalloc).  Arguments
 *   as rpba_precond_train_step without `scratch`: the per-sample activations
 *   and gradients and the loss partials live in a device array of the
 *   library itself, one per GPU (about 9 MB), held until the process ends.
 *   nsamp at most RPBA_TRAIN_NOALLOC_MAX_SAMPLES, else RPBA_ERR_ARG.  Calls no
 *   allocating routine.  Every call on one GPU shares that GPU's array: calls
 *   that overlap on one GPU (on different streams, or from several threads)
 *   race; calls in one stream's order do not.  Every value a call reads from
 *   the array it has written itself, so nothing needs clearing between
 *   calls.  RPBA_ERR_HIP if the array's address cannot be looked up. */
#define RPBA_TRAIN_NOALLOC_MAX_SAMPLES 8192
rpba_status rpba_precond_train_step_noalloc(const float *samples, int32_t nsamp, int32_t nz, float *W, float *m,
                                            float *v, int32_t t, float lr, float *grad, float *loss, int32_t apply,
                                            void *stream);

/* ------------------------------------------------------- sub-block partition
 * Sub-block construction (Sec. 5.2) by partitioning the visibility graph:
 * one node per camera, an edge between two cameras weighted by the number of
 * points both observe, node weight = cube root of the summed observation
 * counts of the points the camera sees.  Multilevel recursive bisection
 * (heavy-edge coarsening, greedy graph growing, Fiduccia-Mattheyses
 * refinement) into `parts` sub-blocks of balanced node weight with few
 * shared points; optionally followed by a pass that balances the cost model
 * c_l = cost_cams3 n_l^3 + cost_obs K_l (n_l cameras and K_l observations of
 * sub-block l) by moving boundary cameras out of the most expensive part.
 * Host code only: no device memory, no stream. */
typedef struct {
  int32_t parts;         /* number of sub-blocks L, in [1, M]: 1 */
  double imbalance;      /* allowed excess of a sub-block's node weight over its share: 0.05 */
  int32_t min_cams;      /* fewer sub-blocks if they would average fewer cameras than this (0: no
                            limit); the paper uses 70: 0 */
  int32_t refine_passes; /* refinement passes per level: 4 */
  double cost_cams3;     /* cost model, see above; both 0 = no cost pass: 0 */
  double cost_obs;       /*   : 0 */
  uint64_t seed;         /* matching order and growing seeds: 0 */
} rpba_partition_options;

/* Fill *opt with the defaults listed above.  HOST pointer. */
rpba_status rpba_partition_default_options(rpba_partition_options *opt);

/* Partition the cameras.  All pointers HOST.
 *   obs_cam, obs_pt [K]  camera and point of each observation
 *   cam_block [M]        out: sub-block of each camera, in [0, L_used)
 *   node_weight [M]      out: the node weights, or NULL
 *   stats [8]            out, or NULL: L_used; edge cut (sum of the edge
 *                        weights between sub-blocks); tie points (points seen
 *                        in >= 2 sub-blocks); point copies (sum over points of
 *                        the sub-blocks seeing them); largest sub-block node
 *                        weight / mean; largest cost / mean cost (0 without a
 *                        cost model); fewest and most cameras in a sub-block
 * L_used = parts, or less with min_cams.  Every sub-block gets at least one
 * camera.  The result depends only on the inputs and options (seed included).
 * RPBA_ERR_ARG: M, N or K < 1, an index out of range, parts outside [1, M], a
 * negative imbalance, min_cams, refine_passes or cost coefficient. */
rpba_status rpba_partition(int32_t M, int32_t N, int32_t K, const int32_t *obs_cam, const int32_t *obs_pt,
                           const rpba_partition_options *opt, int32_t *cam_block, double *node_weight,
                           double *stats);

/* ---------------------------------------------------------------- execution
 * rpba_set_graph: when on, each of rpba_intersect, rpba_subblock_lm_step and
 *   rpba_consensus is captured into a HIP graph on its first call and replayed
 *   on later calls with the same pointer arguments (re-captured when they
 *   change).  The stream given at creation must then not be the NULL stream.
 * rpba_set_timing: when on (graphs are bypassed), every phase is bracketed by
 *   HIP events on the handle's stream and the call synchronises; counters are
 *   reset.  rpba_get_timing copies (HOST) per-phase milliseconds, kernel
 *   launches and calls for phases 0..n-1: intersection, point blocks, Schur
 *   diagonal blocks and right-hand side, Cholesky forward, Cholesky
 *   backward, update, consensus, robust, iterative solver, Schur
 *   off-diagonal (camera pair) blocks, caller-order export of the
 *   intersection; returns the number of phases. */
rpba_status rpba_set_graph(rpba_problem *h, int32_t on);
rpba_status rpba_set_timing(rpba_problem *h, int32_t on);
int32_t rpba_get_timing(rpba_problem *h, double *ms, int64_t *launches, int64_t *calls, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* RPBA_H */
