// Internal state shared by the librpba kernels and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rpba.h"

namespace rpba {

// sets the message rpba_last_error returns (host-only parts of the library)
rpba_status report_error(rpba_status s, const char* msg);

// Device view of one problem: every pointer lives in the caller's workspace
// (or is one of the caller's own arrays, prefix u_).
struct Dev {
  int32_t M, N, K, L;
  int64_t NC;
  int32_t T;              // Cholesky tile edge
  int32_t np;             // parameters per camera: 6 (pose), 8 with intrinsics (pose, f, k1)
  int32_t int_maxit;
  int32_t has_info;
  double f, cx, cy, w0;   // w0 = 1 / sigma_px^2
  double lambda, int_tol;

  // caller arrays (original order)
  double* u_camR;         // [M][9]
  double* u_camC;         // [3][M]
  double* u_intr;         // [2][M] (f, k1) with intrinsics, else null
  double* u_pts;          // [3][N]
  const double* u_xy;     // [2][K]
  const double* u_info;   // [3][K] or null

  // cameras, internal (sub-block-major) order
  double* cam;            // [M][CAM_STRIDE] R row-major, C
  double* camN;           // [M][CAM_STRIDE] updated cameras of the current step
  double* intr;           // [M][2] (f, k1) with intrinsics, else null
  double* intrN;          // [M][2] updated intrinsics of the current step, else null
  const int32_t* cam_blk;
  const int32_t* blk_cam_off;
  const int32_t* cam_orig;

  // points, internal order
  double* P0;             // [3][N] start values of the next intersection
  double* Xbar;           // [3][N] last intersection
  int32_t* status;        // [N]
  const int32_t* pt_orig;
  const int32_t* pt_new;  // [N] internal index of caller point o
  double* pxs;            // [N][4] X (3), status: latest point per internal index, exported to u_pts
  double* covi;           // [N][6] covariance of the last intersection, internal order
  const int32_t* pt_copy_off;
  const int32_t* pt_copies;

  // observations, LM order
  double* xy;             // [K][2]
  double* info;           // [K][3] or null
  double* rw;             // [K] robust weight multiplier
  double* res;            // [K][2] residuals of the last intersection, point-major (valid points
                          // only), or null when the handle keeps none (no robust re-weighting)
  const int32_t* obs_cam;
  const int32_t* obs_copy;
  const int32_t* obs_orig;
  const int32_t* cam_obs_off;
  const int32_t* cam_obs;
  const int32_t* cam_obs_c;  // copy of each cam_obs entry
  // camera-major copies (cam_obs order) for the diagonal Schur pass
  double* cm_xy;          // [K][2] pixel
  double* cm_rw;          // [K] robust weight multiplier (kept with rw)
  int* rw_unit;           // [1] 1 while every robust weight is 1 (the Schur passes then skip reading them)
  double* cm_info;        // [K][3] or null
  // intersection stream, point-major (see the plan)
  const int32_t* pm_off;
  const int32_t* pm_k;
  const int32_t* pm_pos;
  int32_t* pm_code;       // [K] camera slot / PM_GLOBAL | camera, PM_DOWN (see the plan)
  const int32_t* iwg_cam_off;
  const int32_t* iwg_cams;
  double* pm_xy;          // [K][2]
  double* pm_w;           // [K][3] r W (with obs_info only)
  double down_weight;     // weight multiplier of robustly flagged observations

  // copies (sub-block, point)
  const int32_t* copy_off;
  const int32_t* copy_pt;
  const int32_t* copy_blk;
  const int64_t* blk_copy_off;
  double* Xc;             // [NC][3] X_j^l (valid when the sub-block is not fresh)
  int32_t* blk_fresh;     // [L] 1: every copy of the sub-block is still at Xbar (set by the
                          // intersection, cleared by the sub-block's next update)
  int32_t variant;        // RPBA_VARIANT_*
  double* rho_t;          // [1] scalar tie-point weight of this outer iteration (SCALAR, PLAIN)
  double rho_growth;      // factor applied to rho_t by every consensus
  double filter_px;       // PLAIN variants: reprojection error above which a point is filtered
  double* Xt;             // [NC][3] PLAIN variants: dual offset Xtilde of every copy (eq:admm9)
  int32_t* rec_valid;     // [1] 1: the copy records of the fresh sub-blocks hold their point
                          // blocks at the current state (written by the intersection; cleared by
                          // a robust re-weighting and by anything that reuses the record array)
  double* Om;             // [NC][6] refined tie-point weight (FP64 path)
  float* Omf;             // the same region as [NC][6] floats on the mixed path (om_f32)
  int32_t om_f32;         // 1: the refined weights are stored in FP32
  double* cpk;            // [NC][CPK] X (3), valid (1 or 0), damped V^-1 (6), g_X (3), spare (3);
                          // on the mixed path [NC][CPK32]: X (3 doubles), then
                          // as floats V^-1 (6), g_X (3), valid
  int32_t cpk_f32;        // 1: compact FP32 copy records
  const int32_t* nb_off;
  const int32_t* nb_cam;
  // pair blocks (see the plan) and the block-sparse matrix of iterative sub-blocks
  const int32_t* pb_row;
  const int64_t* pb_ent_off;
  const int32_t* pb_ent;
  const int32_t* od_pb;
  int64_t n_od;
  int32_t pb_lanes;        // lanes per camera-pair block (4, 8 or 16)
  const int32_t* pb_bsr;
  const int32_t* pb_bsr_t;
  const uint8_t* blk_pcg;  // [L] 1 = iterative solver (block-sparse output)
  float* bsr;              // [nbsr][36] FP32 blocks of the reduced camera systems
  const int32_t* bsr_row_off;  // [M+1]
  const int32_t* bsr_col;      // local column camera of each block
  float* Pblk;             // [M][36] preconditioner blocks (row-major 6x6)

  // dense reduced camera systems
  double* S;              // tiles, lower triangle per sub-block
  double* Ld;             // [diag] factor tiles L(k,k)
  double* Li;             // [diag] inverse tiles L(k,k)^-1
  double* y;              // padded right-hand sides, updated in place
  double* ys;             // forward-solved segments L^-1 e, then backward-updated
  double* x;              // solution (camera steps)
  const int32_t* nt;
  const int64_t* rcs_off;
  const uint8_t* tile_nz;  // [rcs_total / T^2] tile of the factor may be nonzero (plan's numbering)
  const int64_t* diag_off;
  const int64_t* vec_off;
  int32_t* blk_fail;      // [L] factorisation failed (non-positive pivot): step not applied
  int32_t* blk_nc;        // [L] iterative solve ended above its refinement tolerance
  const uint8_t* active;  // [L] or null (set per call)
  // adaptive damping: per sub-block lambda, or null for the fixed d.lambda
  double* lam_blk;        // [L]
  int32_t* blk_rej;       // [L] the last step was taken back
  double* XcOld;          // [3 NC] the copies before the step
  double lam_up, lam_down, lam_min, lam_max;

  // accumulators
  double* acc_int;        // [4 + L] cost, sum |v|^2, K_valid, N_valid; then per sub-block the cost
                          // of its copies at the intersection (the cost before its next LM step)
  double* acc_blk;        // [L][4] cost before, cost after, |step|^2, iterations
  double* acc_cons;       // [2]
  double* cons_part;      // [2 * ceil(N / 256)] per-workgroup partials of the consensus statistics
  double* int_part;       // [4 * ceil(N / INT_WG)] per-workgroup partials of the intersection statistics
  double* upd_part;       // [16 * ceil(NC / 256)] per-workgroup, per-slot partials of the update's costs
  double* acc_rob;        // [2]
};

// damping of sub-block l's normal equations
__host__ __device__ __forceinline__ double lam_of(const Dev& d, int l) { return d.lam_blk ? d.lam_blk[l] : d.lambda; }

// one 128-byte record per copy for the current LM step (64 bytes, CPK32
// doubles, on the mixed path)
constexpr int CPK = 16;
constexpr int CPK32 = 8;

// In-tile layout of the RCS tiles, chosen for the FP64 matrix cores: element
// (r, c) of a T x T tile lives at ((r / 16) (T / 4) + c / 4) 64 + r % 16 +
// 16 (c % 4), so that the 16 x 4 operand fragment a 64-lane wave feeds to one
// v_mfma_f64_16x16x4 (lane -> row lane % 16, column lane / 16) is one
// contiguous 512-byte load.
__host__ __device__ __forceinline__ int mf_idx(int T, int r, int c) {
  return ((r >> 4) * (T >> 2) + (c >> 2)) * 64 + (r & 15) + 16 * (c & 3);
}

// offset of element (row, col), col <= row, of sub-block l's tiled RCS
__host__ __device__ __forceinline__ int64_t rcs_elem(const Dev& d, int l, int row, int col) {
  const int T = d.T;
  const int tr = row / T, tc = col / T;
  return d.rcs_off[l] + ((int64_t)tr * (tr + 1) / 2 + tc) * T * T + mf_idx(T, row % T, col % T);
}

// kernel launchers (all asynchronous on `st`)
void launch_gather(const Dev& d, hipStream_t st);
// counts into cnt[0] the non-finite values of the caller's state and
// observation arrays and into cnt[1] the information matrices that are not
// positive definite (cnt zeroed by the caller)
void launch_check_inputs(const Dev& d, int32_t* cnt, hipStream_t st);
void launch_init_rcs(const Dev& d, hipStream_t st);
// the intersection itself (point records, and covariances if want_cov), then
// the caller-order export of points, covariances, statuses and the statistics
void launch_intersect(const Dev& d, bool want_cov, hipStream_t st);
void launch_intersect_export(const Dev& d, double* cov, int32_t* status_out, double* stats, hipStream_t st);
void launch_copy_prep(const Dev& d, hipStream_t st);
// covariances (rpba_covariance): Y [rcs_total] scratch of the RCS tile
// layout; the inverse S^-1 of every dense sub-block replaces its factor in S
void launch_cov_inverse(const Dev& d, double* Y, int nt_max, hipStream_t st);
// ends a dataflow factorisation that no backward launch follows: failure
// flags from exhausted waits, control words readied for the next step
void launch_df_finish(const Dev& d, int* ctl, hipStream_t st);
void launch_cov_outputs(const Dev& d, double* cam_cov, double* copy_cov, hipStream_t st);
void launch_schur_diag(const Dev& d, bool fp32, bool dense, int64_t rcs_total, hipStream_t st);
void launch_schur_offdiag(const Dev& d, bool fp32, hipStream_t st);
void launch_chol_potrf(const Dev& d, int k, const int32_t* pot, int64_t npot, hipStream_t st);
void launch_chol_trsm(const Dev& d, int k, const int32_t* trsm, int64_t ntrsm, hipStream_t st);
void launch_chol_update(const Dev& d, int k, const int32_t* upd, int64_t nupd, hipStream_t st);
// the whole forward factorisation of all dense sub-blocks as one persistent
// launch over a task list (see rpba_chol.hip); ctl = [ticket, epoch, errors].
// chol_dataflow_resident_per_cu: its workgroups that fit on one CU at once
// (0 if the query fails)
int chol_dataflow_resident_per_cu(int T);
void launch_chol_dataflow(const Dev& d, const int32_t* tasks, int ntask, int* flags, int64_t nflags, int* ctl,
                          int nworkers, hipStream_t st);
// the backward substitution as one persistent launch (ctl[3] = its ticket)
void launch_chol_backward_dataflow(const Dev& d, const int32_t* tasks, int ntask, int* xflags, int* ctl,
                                   int nworkers, hipStream_t st);
// ctl: the persistent launches' control words (its error word marks every
// sub-block failed)
void launch_rhs_extract(const Dev& d, const int* ctl, hipStream_t st);
// readies the control words after the workspace is zeroed (next epoch)
void launch_df_reset(int* ctl, hipStream_t st);
void launch_chol_backward(const Dev& d, const int32_t* items, int64_t n_items, hipStream_t st);
void launch_update(const Dev& d, double* block_stats, hipStream_t st);
void launch_consensus(const Dev& d, double* stats, hipStream_t st);
// PLAIN variants: every copy starts at its point's start value, duals zero
void launch_init_copies(const Dev& d, hipStream_t st);
void launch_zero(double* p, int64_t n, hipStream_t st);
void launch_zero_wide(double* p, int64_t n, hipStream_t st);  // p 16-byte aligned
void launch_zero_i32(int32_t* p, int64_t n, hipStream_t st);
void launch_rcs_extract(const Dev& d, int l, double* S_out, double* e_out, hipStream_t st);
void launch_bsr_extract(const Dev& d, int l, double* S_out, double* e_out, hipStream_t st);
int robust_lds_values();
void launch_robust(const Dev& d, double* spill, const int64_t* spill_off, int32_t* bad, double* sigma_cam, double t_v,
                   double down_weight, int mode, double* stats, hipStream_t st);
size_t pcg_lds_bytes(int max_n);
int mlp_num_params();
int mlp_num_features();
int mlp_scratch_per_sample();
void launch_mean_diag(const Dev& d, float* mean_diag, hipStream_t st);
void launch_precond_learned(const Dev& d, const float* W, const float* mean_diag, const float* cam_tpfrac,
                            hipStream_t st);
void launch_harvest(const Dev& d, const float* mean_diag, const float* cam_tpfrac, const float* z, int nz,
                    const int32_t* cams, int ncams, float* out, hipStream_t st);
void launch_train_step(const float* samples, int nsamp, int nz, float* W, float* m, float* v, int t, float lr,
                       float* scratch, float* grad, float* loss_part, bool apply, hipStream_t st);
void launch_sum_f32(const float* parts, int n, float* out, hipStream_t st);
// the training step without a caller workspace: samples per call at most
// TRAIN_NOALLOC_MAX_SAMPLES; train_noalloc_scratch returns the current
// device's copy of the library's own scratch array (null and *err on a HIP
// failure), the loss partials start train_noalloc_parts_offset() floats in
constexpr int TRAIN_NOALLOC_MAX_SAMPLES = RPBA_TRAIN_NOALLOC_MAX_SAMPLES;
float* train_noalloc_scratch(hipError_t* err);
size_t train_noalloc_parts_offset();
void launch_pcg(const Dev& d, const int32_t* blocks, int nblocks, int max_n, int pcg_maxit, double pcg_tol,
                double ir_tol, int ir_maxit, hipStream_t st);
// in-bounds layout check of the FP64 MFMA tile product: C = A B^T (64x64, row-major)
void launch_selftest_gemm(const double* A, const double* B, double* C, hipStream_t st);

}  // namespace rpba
