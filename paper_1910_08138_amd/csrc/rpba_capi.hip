// C ABI of librpba (declared in include/rpba.h): argument checking, the
// workspace layout, the host-side plan upload and the per-call kernel
// sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rpba.h"
#include "../../include/rpba_testing.h"
#include "rpba_device.hpp"
#include "rpba_internal.hpp"
#include "rpba_plan.hpp"

using namespace rpba;

namespace {

thread_local std::string g_err;

rpba_status fail(rpba_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace

// the message rpba_last_error returns, for the host-only parts of the library
rpba_status rpba::report_error(rpba_status s, const char* msg) { return fail(s, msg); }

namespace {

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(RPBA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Layout {
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t off = total;
    total += (bytes + 255) & ~(size_t)255;
    return off;
  }
};

// byte offsets of every workspace array
struct WsMap {
  size_t cam_blk, blk_cam_off, cam_orig, pt_orig, pt_new, tile_nz, pt_copy_off, pt_copies, obs_cam, obs_copy, obs_orig, cam_obs_off,
      cam_obs, copy_off, copy_pt, copy_blk, blk_copy_off, nb_off, nb_cam, nt, rcs_off, diag_off, vec_off, fwd_items,
      bwd_items, upd_items, pot_items, blk_fail, pb_row, pb_ent_off, pb_ent, od_pb, pb_bsr, pb_bsr_t, blk_pcg, bsr_row_off, bsr_col, bsr,
      Pblk, pcg_list, mean_diag, cam_tpfrac, mlp_w, pcg_cams, rob_bad, rob_off, rob_vals, rob_sigma, pm_off, pm_k,
      pm_pos, pm_cam, iwg_cam_off, iwg_cams, pm_xy, pm_w, cam_obs_c, df_tasks, df_flags,
      df_ctl, blk_fresh, dfb_tasks, dfb_flags, cm_xy, cm_rw, rw_unit, cm_info, blk_nc, chk, rec_valid, rho_t, Xt, covY,
      lam_blk, blk_rej, XcOld;
  size_t cam, camN, intr, intrN, P0, Xbar, pxs, covi, status, xy, info, rw, res, Xc, Om, cpk, S, Ld, Li, y, ys, x, acc_int, acc_blk, acc_cons, cons_part, int_part, upd_part,
      acc_rob;
  size_t total;
};

// doubles of global staging for the robust medians: cameras whose residual
// components do not fit the workgroup's LDS
int64_t robust_spill_values(const Plan& P, std::vector<int64_t>* off = nullptr) {
  int64_t tot = 0;
  if (off) off->assign(P.M, 0);
  for (int i = 0; i < P.M; ++i) {
    const int64_t n2 = 2 * (int64_t)(P.cam_obs_off[i + 1] - P.cam_obs_off[i]);
    if (n2 > robust_lds_values()) {
      if (off) (*off)[i] = tot;
      tot += n2;
    }
  }
  return tot;
}

WsMap layout_for(const Plan& P, bool keep_res, bool plain, bool cov, bool adaptive) {
  Layout L;
  WsMap m;
  const size_t i4 = 4, i8 = 8, f8 = 8;
  m.cam_blk = L.add(i4 * P.M);
  m.blk_cam_off = L.add(i4 * (P.L + 1));
  m.cam_orig = L.add(i4 * P.M);
  m.pt_orig = L.add(i4 * P.N);
  m.pt_new = L.add(i4 * P.N);
  m.pt_copy_off = L.add(i4 * (P.N + 1));
  m.pt_copies = L.add(i4 * P.NC);
  m.obs_cam = L.add(i4 * P.K);
  m.obs_copy = L.add(i4 * P.K);
  m.obs_orig = L.add(i4 * P.K);
  m.cam_obs_off = L.add(i4 * (P.M + 1));
  m.cam_obs = L.add(i4 * P.K);
  m.copy_off = L.add(i4 * (P.NC + 1));
  m.copy_pt = L.add(i4 * P.NC);
  m.copy_blk = L.add(i4 * P.NC);
  m.blk_copy_off = L.add(i8 * (P.L + 1));
  m.nb_off = L.add(i4 * (P.M + 1));
  m.nb_cam = L.add(i4 * P.nb_cam.size());
  m.nt = L.add(i4 * P.L);
  m.rcs_off = L.add(i8 * P.L);
  m.tile_nz = L.add(P.tile_nz.size());
  m.diag_off = L.add(i8 * P.L);
  m.vec_off = L.add(i8 * P.L);
  m.fwd_items = L.add(i4 * P.fwd_items.size());
  m.bwd_items = L.add(i4 * P.bwd_items.size());
  m.upd_items = L.add(i4 * P.upd_items.size());
  m.pot_items = L.add(i4 * P.pot_items.size());
  m.blk_fail = L.add(i4 * P.L);
  m.blk_nc = L.add(i4 * P.L);
  m.chk = L.add(i4 * 4);
  m.rec_valid = L.add(i4 * 4);
  m.rho_t = L.add(f8 * 2);
  m.Xt = L.add(plain ? f8 * 3 * P.NC : 0);
  m.covY = L.add(cov ? f8 * P.rcs_total : 0);
  m.lam_blk = L.add(f8 * P.L);
  m.blk_rej = L.add(i4 * P.L);
  m.XcOld = L.add(adaptive ? f8 * 3 * P.NC : 0);
  m.pb_row = L.add(i4 * P.pb_row.size());
  m.pb_ent_off = L.add(i8 * P.pb_ent_off.size());
  m.pb_ent = L.add(i4 * P.pb_ent.size());
  m.od_pb = L.add(i4 * P.od_pb.size());
  m.pb_bsr = L.add(i4 * P.pb_bsr.size());
  m.pb_bsr_t = L.add(i4 * P.pb_bsr_t.size());
  m.blk_pcg = L.add(P.L);
  m.bsr_row_off = L.add(i4 * P.bsr_row_off.size());
  m.bsr_col = L.add(i4 * P.bsr_col.size());
  m.bsr = L.add(4 * 36 * (size_t)P.nbsr);
  m.Pblk = L.add(4 * 36 * (size_t)P.M);
  m.pcg_list = L.add(i4 * P.L);
  m.mean_diag = L.add(4 * (size_t)P.L);
  m.cam_tpfrac = L.add(4 * (size_t)P.M);
  m.mlp_w = L.add(4 * (size_t)mlp_num_params());
  m.pcg_cams = L.add(i4 * P.M);
  m.rob_bad = L.add(i4 * P.N);
  m.rob_off = L.add(i8 * P.M);
  m.rob_vals = L.add(f8 * robust_spill_values(P));
  m.rob_sigma = L.add(f8 * P.M);
  m.pm_off = L.add(i4 * P.pm_off.size());
  m.pm_k = L.add(i4 * P.pm_k.size());
  m.pm_pos = L.add(i4 * P.pm_pos.size());
  m.pm_cam = L.add(i4 * P.pm_cam.size());
  m.iwg_cam_off = L.add(i4 * P.iwg_cam_off.size());
  m.iwg_cams = L.add(i4 * std::max<size_t>(1, P.iwg_cams.size()));
  m.pm_xy = L.add(f8 * 2 * P.K);
  m.pm_w = L.add(P.has_info ? f8 * 3 * P.K : 0);
  m.cam_obs_c = L.add(i4 * P.cam_obs_c.size());
  m.df_tasks = L.add(i4 * (P.rcs_total / ((int64_t)P.T * P.T)));
  m.df_flags = L.add(i4 * 2 * (P.rcs_total / ((int64_t)P.T * P.T)));  // ready flags, then partial-sum flags
  m.df_ctl = L.add(i4 * 4);
  m.blk_fresh = L.add(i4 * P.L);
  m.dfb_tasks = L.add(i4 * (P.vec_total / P.T));
  m.dfb_flags = L.add(i4 * (P.vec_total / P.T));
  m.cm_xy = L.add(f8 * 2 * P.K);
  m.cm_rw = L.add(f8 * P.K);
  m.rw_unit = L.add(4);
  m.cm_info = L.add(P.has_info ? f8 * 3 * P.K : 0);
  m.cam = L.add(f8 * CAM_STRIDE * P.M);
  m.camN = L.add(f8 * CAM_STRIDE * P.M);
  m.intr = L.add(P.np == 8 ? f8 * 2 * P.M : 0);  // (f, k1) per camera with intrinsics
  m.intrN = L.add(P.np == 8 ? f8 * 2 * P.M : 0);
  m.P0 = L.add(f8 * 3 * P.N);
  m.Xbar = L.add(f8 * 3 * P.N);
  m.pxs = L.add(f8 * 4 * P.N);
  m.covi = L.add(f8 * 6 * P.N);
  m.status = L.add(i4 * P.N);
  m.xy = L.add(f8 * 2 * P.K);
  m.info = L.add(P.has_info ? f8 * 3 * P.K : 0);
  m.rw = L.add(f8 * P.K);
  m.res = L.add(keep_res ? f8 * 2 * P.K : 0);
  m.Xc = L.add(f8 * 3 * P.NC);
  m.Om = L.add(f8 * 6 * P.NC);
  m.cpk = L.add(f8 * CPK * P.NC);
  m.S = L.add(f8 * P.rcs_total);
  m.Ld = L.add(f8 * P.diag_total);
  m.Li = L.add(f8 * P.diag_total);
  m.y = L.add(f8 * P.vec_total);
  m.ys = L.add(f8 * P.vec_total);
  m.x = L.add(f8 * P.vec_total);
  m.acc_int = L.add(f8 * (4 + P.L));
  m.acc_blk = L.add(f8 * 4 * P.L);
  m.acc_cons = L.add(f8 * 2);
  m.cons_part = L.add(f8 * 2 * ((P.N + 255) / 256));
  m.int_part = L.add(f8 * 4 * ((P.N + INT_WG - 1) / INT_WG));
  m.upd_part = L.add(f8 * 16 * ((P.NC + 255) / 256));
  m.acc_rob = L.add(f8 * 2);
  m.total = L.total;
  return m;
}

// one cached plan: rpba_workspace_size followed by rpba_create on the same
// topology plans once
std::mutex g_plan_mu;
std::shared_ptr<Plan> g_last_plan;

rpba_status get_plan(const rpba_problem_desc* d, const rpba_options* o, std::shared_ptr<Plan>& out) {
  int tile = o->chol_tile == 0 ? 64 : o->chol_tile;
  const int np = o->intrinsics ? 8 : 6;
  if (!d->obs_cam || !d->obs_pt || !d->cam_block) return fail(RPBA_ERR_ARG, "topology arrays must be non-NULL");
  uint64_t key = topology_key(d->M, d->N, d->K, d->L, d->obs_cam, d->obs_pt, d->cam_block, tile, np);
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    if (g_last_plan && g_last_plan->key == key) {
      out = g_last_plan;
      out->has_info = d->obs_info != nullptr;
      return RPBA_OK;
    }
  }
  auto P = std::make_shared<Plan>();
  std::string err = build_plan(d->M, d->N, d->K, d->L, d->obs_cam, d->obs_pt, d->cam_block, tile, np, *P);
  if (!err.empty()) return fail(RPBA_ERR_ARG, err);
  P->has_info = d->obs_info != nullptr;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_last_plan = P;
  }
  out = P;
  return RPBA_OK;
}

rpba_status check_desc(const rpba_problem_desc* d, const rpba_options* o) {
  if (!d || !o) return fail(RPBA_ERR_ARG, "desc and options must be non-NULL");
  if (o->intrinsics != 0 && o->intrinsics != 1) return fail(RPBA_ERR_ARG, "intrinsics must be 0 or 1");
  if ((!o->intrinsics && (!(d->f > 0) || !std::isfinite(d->f))) || !std::isfinite(d->cx) || !std::isfinite(d->cy))
    return fail(RPBA_ERR_ARG, "intrinsics must be finite, f > 0");
  if (o->intrinsics) {
    if (!d->cam_intr) return fail(RPBA_ERR_ARG, "intrinsics = 1 needs desc->cam_intr");
    if (o->solver != RPBA_SOLVER_CHOL) return fail(RPBA_ERR_ARG, "intrinsics = 1 needs RPBA_SOLVER_CHOL");
    if (o->variant != RPBA_VARIANT_EXTENDED) return fail(RPBA_ERR_ARG, "intrinsics = 1 needs RPBA_VARIANT_EXTENDED");
  }
  if (!d->obs_info && !(d->sigma_px > 0)) return fail(RPBA_ERR_ARG, "sigma_px must be > 0 without obs_info");
  if (!d->cam_R || !d->cam_C || !d->pts || !d->obs_xy) return fail(RPBA_ERR_ARG, "state and observation arrays must be non-NULL");
  if (o->precision != RPBA_FP64 && o->precision != RPBA_MIXED) return fail(RPBA_ERR_ARG, "unknown precision");
  if (o->solver < RPBA_SOLVER_CHOL || o->solver > RPBA_SOLVER_AUTO_LEARNED) return fail(RPBA_ERR_ARG, "unknown solver");
  if (!(o->lambda >= 0) || !(o->int_tol > 0) || o->int_maxit < 1) return fail(RPBA_ERR_ARG, "bad LM / intersection options");
  if (o->chol_tile != 0 && o->chol_tile != 32 && o->chol_tile != 64) return fail(RPBA_ERR_ARG, "chol_tile must be 0, 32 or 64");
  if (o->chol_schedule < RPBA_CHOL_DEFAULT || o->chol_schedule > RPBA_CHOL_DATAFLOW)
    return fail(RPBA_ERR_ARG, "chol_schedule must be RPBA_CHOL_DEFAULT, _STEPWISE or _DATAFLOW");
  if (o->robust != 0 && o->robust != 1) return fail(RPBA_ERR_ARG, "robust must be 0 or 1");
  if (o->variant < RPBA_VARIANT_EXTENDED || o->variant > RPBA_VARIANT_PLAIN_REFINED)
    return fail(RPBA_ERR_ARG, "unknown variant");
  if (!(o->rho > 0) || !std::isfinite(o->rho) || !(o->rho_growth > 0) || !std::isfinite(o->rho_growth) ||
      !(o->filter_px > 0))
    return fail(RPBA_ERR_ARG, "rho, rho_growth and filter_px must be positive and finite");
  if (o->covariance != 0 && o->covariance != 1) return fail(RPBA_ERR_ARG, "covariance must be 0 or 1");
  if (o->damping != RPBA_DAMPING_FIXED && o->damping != RPBA_DAMPING_ADAPTIVE)
    return fail(RPBA_ERR_ARG, "damping must be RPBA_DAMPING_FIXED or RPBA_DAMPING_ADAPTIVE");
  if (o->damping == RPBA_DAMPING_ADAPTIVE &&
      (!(o->lambda_up > 1.0) || !(o->lambda_down > 1.0) || !(o->lambda_min > 0.0) || !(o->lambda_max >= o->lambda_min) ||
       !std::isfinite(o->lambda_up) || !std::isfinite(o->lambda_down) || !std::isfinite(o->lambda_max)))
    return fail(RPBA_ERR_ARG, "adaptive damping needs lambda_up, lambda_down > 1 and 0 < lambda_min <= lambda_max, finite");
  if (o->pair_lanes != 0 && o->pair_lanes != 4 && o->pair_lanes != 8 && o->pair_lanes != 16)
    return fail(RPBA_ERR_ARG, "pair_lanes must be 0, 4, 8 or 16");
  return RPBA_OK;
}

bool pcg_bytes_ok(int max_n) { return pcg_lds_bytes(max_n) <= 150 * 1024; }

}  // namespace

// A captured call, replayed while its pointer arguments stay the same.
struct CallGraph {
  hipGraphExec_t exec = nullptr;
  const void* args[3] = {nullptr, nullptr, nullptr};
  bool valid = false;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    valid = false;
  }
};

enum Phase { PH_INTERSECT = 0, PH_COPY_PREP, PH_SCHUR, PH_CHOL_FWD, PH_CHOL_BWD, PH_UPDATE, PH_CONSENSUS, PH_ROBUST,
             PH_SOLVE_IT, PH_SCHUR_OD, PH_INT_EXPORT, NPHASE };

struct rpba_problem {
  std::shared_ptr<Plan> plan;
  WsMap map;
  Dev d;
  rpba_options opt;
  hipStream_t stream;
  char* ws;
  size_t max_lds_schur;
  std::vector<uint8_t> blk_pcg;
  // Cholesky work lists restricted to the sub-blocks solved densely
  std::vector<int64_t> pot_off, fwd_off, upd_off, bwd_off;
  // dataflow factorisation: task count and resident workers
  bool dataflow = true;
  int32_t df_ntask = 0, df_workers = 0, df_fwd_workers = 0, dfb_ntask = 0;
  int32_t nt_max_dense = 0;
  int32_t n_pcg = 0, max_pcg_n = 0, n_pcg_cams = 0;
  bool have_weights = false;
  bool any_dense = true;
  bool intersected = false;
  bool use_graph = false;
  CallGraph g_int, g_step, g_cons, g_rob[3];  // g_rob: one per RPBA_ROBUST_* mode
  bool timing = false;
  hipEvent_t ev[NPHASE + 1] = {};
  double ms[NPHASE] = {};
  int64_t launches[NPHASE] = {};
  int64_t calls[NPHASE] = {};
  ~rpba_problem() {
    // queued work may still read the workspace and the caller's arrays
    (void)hipStreamSynchronize(stream);
    g_int.reset();
    g_step.reset();
    g_cons.reset();
    for (CallGraph& g : g_rob) g.reset();
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

// Runs `body` on the handle's stream: eagerly, or through a graph captured on
// the first call with these pointer arguments and replayed afterwards.
template <typename F>
rpba_status run_call(rpba_problem* h, CallGraph& g, const void* a0, const void* a1, const void* a2, F body) {
  if (!h->use_graph || h->timing) {
    rpba_status s = body();
    if (s != RPBA_OK) return s;
    HIP_TRY(hipGetLastError());
    return RPBA_OK;
  }
  if (!(g.valid && g.args[0] == a0 && g.args[1] == a1 && g.args[2] == a2)) {
    g.reset();
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    rpba_status s = body();
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (s != RPBA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(RPBA_ERR_HIP, std::string("stream capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(RPBA_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    g.args[0] = a0;
    g.args[1] = a1;
    g.args[2] = a2;
    g.valid = true;
  }
  HIP_TRY(hipGraphLaunch(g.exec, h->stream));
  return RPBA_OK;
}

// event-timed phase (timing mode only)
struct PhaseTimer {
  rpba_problem* h;
  int ph;
  PhaseTimer(rpba_problem* h_, int ph_, int64_t nlaunch) : h(h_), ph(ph_) {
    if (h->timing) {
      (void)hipEventRecord(h->ev[0], h->stream);
      h->launches[ph] += nlaunch;
      h->calls[ph] += 1;
    }
  }
  ~PhaseTimer() {
    if (h->timing) {
      (void)hipEventRecord(h->ev[1], h->stream);
      (void)hipEventSynchronize(h->ev[1]);
      float t = 0;
      (void)hipEventElapsedTime(&t, h->ev[0], h->ev[1]);
      h->ms[ph] += t;
    }
  }
};

}  // namespace

extern "C" {

const char* rpba_last_error(void) { return g_err.c_str(); }

rpba_status rpba_default_options(rpba_options* o) {
  if (!o) return fail(RPBA_ERR_ARG, "NULL options");
  std::memset(o, 0, sizeof(*o));
  o->precision = RPBA_FP64;
  o->solver = RPBA_SOLVER_CHOL;
  o->lambda = 1e-4;
  o->int_tol = 1e-12;
  o->int_maxit = 20;
  o->pcg_maxit = 200;
  o->pcg_tol = 1e-8;
  o->ir_tol = 1e-10;
  o->ir_maxit = 6;
  o->pcg_min_cams = 150;
  o->t_v = 4.0;
  o->down_weight = 1e-4;
  o->chol_tile = 0;
  o->chol_schedule = RPBA_CHOL_DEFAULT;
  o->robust = 0;
  o->pair_lanes = 0;
  o->variant = RPBA_VARIANT_EXTENDED;
  o->rho = 1000.0;
  o->rho_growth = 1.01;
  o->filter_px = 1000.0;
  o->covariance = 0;
  o->damping = RPBA_DAMPING_FIXED;
  o->lambda_up = 10.0;
  o->lambda_down = 10.0;
  o->lambda_min = 1e-12;
  o->lambda_max = 1e8;
  o->intrinsics = 0;
  return RPBA_OK;
}

rpba_status rpba_workspace_size(const rpba_problem_desc* d, const rpba_options* o, size_t* bytes) {
  rpba_status s = check_desc(d, o);
  if (s != RPBA_OK) return s;
  if (!bytes) return fail(RPBA_ERR_ARG, "NULL bytes");
  std::shared_ptr<Plan> P;
  s = get_plan(d, o, P);
  if (s != RPBA_OK) return s;
  *bytes = layout_for(*P, o->robust != 0, o->variant >= RPBA_VARIANT_PLAIN, o->covariance != 0,
                      o->damping == RPBA_DAMPING_ADAPTIVE).total;
  return RPBA_OK;
}

rpba_status rpba_create(const rpba_problem_desc* d, const rpba_options* o, void* workspace, size_t bytes, void* stream,
                        rpba_problem** out) {
  rpba_status s = check_desc(d, o);
  if (s != RPBA_OK) return s;
  if (!out) return fail(RPBA_ERR_ARG, "NULL out");
  *out = nullptr;
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(RPBA_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  std::shared_ptr<Plan> P;
  s = get_plan(d, o, P);
  if (s != RPBA_OK) return s;
  WsMap m = layout_for(*P, o->robust != 0, o->variant >= RPBA_VARIANT_PLAIN, o->covariance != 0,
                      o->damping == RPBA_DAMPING_ADAPTIVE);
  if (bytes < m.total) return fail(RPBA_ERR_WORKSPACE, "workspace too small: need " + std::to_string(m.total));
  size_t lds = 0;

  std::unique_ptr<rpba_problem> h(new rpba_problem());
  h->plan = P;
  h->map = m;
  h->opt = *o;
  h->stream = (hipStream_t)stream;
  h->ws = (char*)workspace;
  h->max_lds_schur = lds;
  hipStream_t st = h->stream;
  char* w = h->ws;
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(w + off, src, n, hipMemcpyHostToDevice, st);
  };
  const Plan& p = *P;
  HIP_TRY(up(m.cam_blk, p.cam_blk.data(), 4 * p.cam_blk.size()));
  HIP_TRY(up(m.blk_cam_off, p.blk_cam_off.data(), 4 * p.blk_cam_off.size()));
  HIP_TRY(up(m.cam_orig, p.cam_orig.data(), 4 * p.cam_orig.size()));
  HIP_TRY(up(m.pt_orig, p.pt_orig.data(), 4 * p.pt_orig.size()));
  HIP_TRY(up(m.pt_new, p.pt_new.data(), 4 * p.pt_new.size()));
  HIP_TRY(up(m.pt_copy_off, p.pt_copy_off.data(), 4 * p.pt_copy_off.size()));
  HIP_TRY(up(m.pt_copies, p.pt_copies.data(), 4 * p.pt_copies.size()));
  HIP_TRY(up(m.obs_cam, p.obs_cam.data(), 4 * p.obs_cam.size()));
  HIP_TRY(up(m.obs_copy, p.obs_copy.data(), 4 * p.obs_copy.size()));
  HIP_TRY(up(m.obs_orig, p.obs_orig.data(), 4 * p.obs_orig.size()));
  HIP_TRY(up(m.cam_obs_off, p.cam_obs_off.data(), 4 * p.cam_obs_off.size()));
  HIP_TRY(up(m.cam_obs, p.cam_obs.data(), 4 * p.cam_obs.size()));
  HIP_TRY(up(m.cam_obs_c, p.cam_obs_c.data(), 4 * p.cam_obs_c.size()));
  HIP_TRY(up(m.pm_off, p.pm_off.data(), 4 * p.pm_off.size()));
  HIP_TRY(up(m.pm_k, p.pm_k.data(), 4 * p.pm_k.size()));
  HIP_TRY(up(m.pm_pos, p.pm_pos.data(), 4 * p.pm_pos.size()));
  HIP_TRY(up(m.pm_cam, p.pm_cam.data(), 4 * p.pm_cam.size()));
  HIP_TRY(up(m.iwg_cam_off, p.iwg_cam_off.data(), 4 * p.iwg_cam_off.size()));
  if (!p.iwg_cams.empty()) HIP_TRY(up(m.iwg_cams, p.iwg_cams.data(), 4 * p.iwg_cams.size()));
  HIP_TRY(up(m.copy_off, p.copy_off.data(), 4 * p.copy_off.size()));
  HIP_TRY(up(m.copy_pt, p.copy_pt.data(), 4 * p.copy_pt.size()));
  HIP_TRY(up(m.copy_blk, p.copy_blk.data(), 4 * p.copy_blk.size()));
  HIP_TRY(up(m.blk_copy_off, p.blk_copy_off.data(), 8 * p.blk_copy_off.size()));
  HIP_TRY(up(m.nb_off, p.nb_off.data(), 4 * p.nb_off.size()));
  HIP_TRY(up(m.nb_cam, p.nb_cam.data(), 4 * p.nb_cam.size()));
  HIP_TRY(up(m.nt, p.nt.data(), 4 * p.nt.size()));
  HIP_TRY(up(m.rcs_off, p.rcs_off.data(), 8 * p.rcs_off.size()));
  HIP_TRY(up(m.tile_nz, p.tile_nz.data(), p.tile_nz.size()));
  HIP_TRY(up(m.diag_off, p.diag_off.data(), 8 * p.diag_off.size()));
  HIP_TRY(up(m.vec_off, p.vec_off.data(), 8 * p.vec_off.size()));
  HIP_TRY(up(m.pb_row, p.pb_row.data(), 4 * p.pb_row.size()));
  HIP_TRY(up(m.pb_ent_off, p.pb_ent_off.data(), 8 * p.pb_ent_off.size()));
  HIP_TRY(up(m.pb_ent, p.pb_ent.data(), 4 * p.pb_ent.size()));
  {
    // camera-pair blocks by the number of rounds of a lane group, most first
    // (the plan orders them for 8 lanes; the order stays stable inside a class)
    // (with intrinsics the pair pass always takes eight lanes per block)
    const int G = o->pair_lanes == 0 || o->intrinsics ? 8 : o->pair_lanes;
    std::vector<int32_t> od = p.od_pb;
    auto rounds = [&](int32_t q) { return (p.pb_ent_off[q + 1] - p.pb_ent_off[q] + G - 1) / G; };
    if (G != 8) std::stable_sort(od.begin(), od.end(), [&](int32_t a, int32_t b) { return rounds(a) > rounds(b); });
    HIP_TRY(up(m.od_pb, od.data(), 4 * od.size()));
  }
  HIP_TRY(up(m.pb_bsr, p.pb_bsr.data(), 4 * p.pb_bsr.size()));
  HIP_TRY(up(m.pb_bsr_t, p.pb_bsr_t.data(), 4 * p.pb_bsr_t.size()));
  HIP_TRY(up(m.bsr_row_off, p.bsr_row_off.data(), 4 * p.bsr_row_off.size()));
  HIP_TRY(up(m.bsr_col, p.bsr_col.data(), 4 * p.bsr_col.size()));
  // solver of every sub-block
  h->blk_pcg.assign(p.L, 0);
  std::vector<int32_t> pcg_list;
  for (int l = 0; l < p.L; ++l) {
    const int ncam = p.blk_cam_off[l + 1] - p.blk_cam_off[l];
    bool it = o->solver == RPBA_SOLVER_PCG_BJ || o->solver == RPBA_SOLVER_PCG_LEARNED ||
              ((o->solver == RPBA_SOLVER_AUTO || o->solver == RPBA_SOLVER_AUTO_LEARNED) && ncam >= o->pcg_min_cams);
    if (it) {
      h->blk_pcg[l] = 1;
      pcg_list.push_back(l);
      h->max_pcg_n = std::max(h->max_pcg_n, 6 * ncam);
    }
  }
  h->n_pcg = (int32_t)pcg_list.size();
  {
    std::vector<int32_t> cams;
    for (int32_t l : pcg_list)
      for (int32_t i = p.blk_cam_off[l]; i < p.blk_cam_off[l + 1]; ++i) cams.push_back(i);
    h->n_pcg_cams = (int32_t)cams.size();
    HIP_TRY(up(m.pcg_cams, cams.data(), 4 * cams.size()));
    // tie-point fraction of every camera's observations (a feature of the
    // learned preconditioner)
    std::vector<float> tpf(p.M, 0.f);
    for (int32_t i = 0; i < p.M; ++i) {
      int32_t n = 0, tp = 0;
      for (int32_t q = p.cam_obs_off[i]; q < p.cam_obs_off[i + 1]; ++q) {
        const int32_t pt = p.copy_pt[p.obs_copy[p.cam_obs[q]]];
        ++n;
        tp += (p.pt_copy_off[pt + 1] - p.pt_copy_off[pt]) > 1;
      }
      tpf[i] = n ? (float)tp / (float)n : 0.f;
    }
    HIP_TRY(up(m.cam_tpfrac, tpf.data(), 4 * tpf.size()));
    std::vector<float> w0(mlp_num_params(), 0.f);  // zero network: block-Jacobi
    HIP_TRY(up(m.mlp_w, w0.data(), 4 * w0.size()));
  }
  if (pcg_bytes_ok(h->max_pcg_n) == false)
    return fail(RPBA_ERR_ARG, "a sub-block is too large for the single-workgroup iterative solver");
  HIP_TRY(up(m.blk_pcg, h->blk_pcg.data(), p.L));
  {
    std::vector<int64_t> roff;
    robust_spill_values(p, &roff);
    HIP_TRY(up(m.rob_off, roff.data(), 8 * roff.size()));
  }
  HIP_TRY(up(m.pcg_list, pcg_list.data(), 4 * pcg_list.size()));
  // Cholesky work lists without the iterative sub-blocks (same order, same
  // positions in the workspace arrays)
  {
    auto filt = [&](const std::vector<int32_t>& items, const std::vector<int64_t>& off, std::vector<int32_t>& out,
                    std::vector<int64_t>& out_off) {
      out.clear();
      out_off.assign(off.size(), 0);
      for (size_t k = 0; k + 1 < off.size(); ++k) {
        for (int64_t t = off[k]; t < off[k + 1]; ++t)
          if (!h->blk_pcg[items[t] >> 16]) out.push_back(items[t]);
        out_off[k + 1] = (int64_t)out.size();
      }
    };
    std::vector<int32_t> tmp;
    filt(p.pot_items, p.pot_off, tmp, h->pot_off);
    HIP_TRY(up(m.pot_items, tmp.data(), 4 * tmp.size()));
    filt(p.fwd_items, p.fwd_off, tmp, h->fwd_off);
    HIP_TRY(up(m.fwd_items, tmp.data(), 4 * tmp.size()));
    filt(p.upd_items, p.upd_off, tmp, h->upd_off);
    HIP_TRY(up(m.upd_items, tmp.data(), 4 * tmp.size()));
    filt(p.bwd_items, p.bwd_off, tmp, h->bwd_off);
    HIP_TRY(up(m.bwd_items, tmp.data(), 4 * tmp.size()));
    h->any_dense = false;
    h->nt_max_dense = 0;
    for (int l = 0; l < p.L; ++l)
      if (!h->blk_pcg[l]) {
        h->any_dense = true;
        h->nt_max_dense = std::max(h->nt_max_dense, p.nt[l]);
      }
    // dataflow task list (see dataflow_order)
    std::vector<int32_t> dense;
    for (int l = 0; l < p.L; ++l)
      if (!h->blk_pcg[l]) dense.push_back(l);
    tmp = dataflow_order(p, dense);
    if (tmp.empty() && !dense.empty()) return fail(RPBA_ERR_ARG, "internal: the dataflow task order is not topological");
    h->df_ntask = (int32_t)tmp.size();
    if (!tmp.empty()) HIP_TRY(up(m.df_tasks, tmp.data(), 4 * tmp.size()));
    // backward tasks: tile rows from the last one down
    tmp.clear();
    for (int k = h->nt_max_dense - 1; k >= 0; --k)
      for (int l : dense)
        if (p.nt[l] > k) tmp.push_back((l << 16) | (k << 8));
    h->dfb_ntask = (int32_t)tmp.size();
    if (!tmp.empty()) HIP_TRY(up(m.dfb_tasks, tmp.data(), 4 * tmp.size()));
    h->dataflow = o->chol_schedule != RPBA_CHOL_STEPWISE;
    int dev = 0, ncu = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    h->df_workers = ncu * (p.T == 64 ? 2 : 4);
    // the forward launch gets exactly the workgroups that can be resident
    // at once (a persistent grid; more would only start after the work is
    // done)
    h->df_fwd_workers = ncu * chol_dataflow_resident_per_cu(p.T);
    if (h->df_fwd_workers <= 0) return fail(RPBA_ERR_HIP, "dataflow Cholesky occupancy query failed");
  }

  Dev& D = h->d;
  std::memset(&D, 0, sizeof(D));
  D.M = p.M;
  D.N = p.N;
  D.K = p.K;
  D.L = p.L;
  D.NC = p.NC;
  D.T = p.T;
  D.np = p.np;
  D.int_maxit = o->int_maxit;
  D.has_info = p.has_info ? 1 : 0;
  D.down_weight = o->down_weight;
  D.cpk_f32 = o->precision == RPBA_MIXED ? 1 : 0;
  D.f = d->f;
  D.cx = d->cx;
  D.cy = d->cy;
  D.w0 = d->obs_info ? 0.0 : 1.0 / (d->sigma_px * d->sigma_px);
  D.lambda = o->lambda;
  D.int_tol = o->int_tol;
  D.u_camR = d->cam_R;
  D.u_camC = d->cam_C;
  D.u_intr = o->intrinsics ? d->cam_intr : nullptr;
  D.u_pts = d->pts;
  D.u_xy = d->obs_xy;
  D.u_info = d->obs_info;
  auto I = [&](size_t off) { return (int32_t*)(w + off); };
  auto F = [&](size_t off) { return (double*)(w + off); };
  D.cam = F(m.cam);
  D.camN = F(m.camN);
  D.intr = p.np == 8 ? F(m.intr) : nullptr;
  D.intrN = p.np == 8 ? F(m.intrN) : nullptr;
  D.cam_blk = I(m.cam_blk);
  D.blk_cam_off = I(m.blk_cam_off);
  D.cam_orig = I(m.cam_orig);
  D.P0 = F(m.P0);
  D.Xbar = F(m.Xbar);
  D.pxs = F(m.pxs);
  D.cm_xy = F(m.cm_xy);
  D.cm_rw = F(m.cm_rw);
  D.rw_unit = I(m.rw_unit);
  D.cm_info = p.has_info ? F(m.cm_info) : nullptr;
  D.covi = F(m.covi);
  D.status = I(m.status);
  D.pt_orig = I(m.pt_orig);
  D.pt_new = I(m.pt_new);
  D.pt_copy_off = I(m.pt_copy_off);
  D.pt_copies = I(m.pt_copies);
  D.xy = F(m.xy);
  D.info = p.has_info ? F(m.info) : nullptr;
  D.rw = F(m.rw);
  D.res = o->robust ? F(m.res) : nullptr;
  D.obs_cam = I(m.obs_cam);
  D.obs_copy = I(m.obs_copy);
  D.obs_orig = I(m.obs_orig);
  D.cam_obs_off = I(m.cam_obs_off);
  D.cam_obs_c = I(m.cam_obs_c);
  D.pm_off = I(m.pm_off);
  D.pm_k = I(m.pm_k);
  D.pm_pos = I(m.pm_pos);
  D.pm_code = I(m.pm_cam);
  D.iwg_cam_off = I(m.iwg_cam_off);
  D.iwg_cams = I(m.iwg_cams);
  D.pm_xy = F(m.pm_xy);
  D.pm_w = F(m.pm_w);
  D.cam_obs = I(m.cam_obs);
  D.copy_off = I(m.copy_off);
  D.copy_pt = I(m.copy_pt);
  D.copy_blk = I(m.copy_blk);
  D.blk_copy_off = (const int64_t*)(w + m.blk_copy_off);
  D.Xc = F(m.Xc);
  D.blk_fresh = I(m.blk_fresh);
  D.Om = F(m.Om);
  D.Omf = reinterpret_cast<float*>(D.Om);
  D.om_f32 = o->precision == RPBA_MIXED;
  D.cpk = F(m.cpk);
  D.nb_off = I(m.nb_off);
  D.nb_cam = I(m.nb_cam);
  D.pb_row = I(m.pb_row);
  D.pb_ent_off = (const int64_t*)(w + m.pb_ent_off);
  D.pb_ent = I(m.pb_ent);
  D.od_pb = I(m.od_pb);
  D.n_od = (int64_t)p.od_pb.size();
  D.pb_lanes = o->pair_lanes == 0 || o->intrinsics ? 8 : o->pair_lanes;
  D.pb_bsr = I(m.pb_bsr);
  D.pb_bsr_t = I(m.pb_bsr_t);
  D.blk_pcg = (const uint8_t*)(w + m.blk_pcg);
  D.bsr = (float*)(w + m.bsr);
  D.bsr_row_off = I(m.bsr_row_off);
  D.bsr_col = I(m.bsr_col);
  D.Pblk = (float*)(w + m.Pblk);
  D.S = F(m.S);
  D.Ld = F(m.Ld);
  D.Li = F(m.Li);
  D.y = F(m.y);
  D.ys = F(m.ys);
  D.x = F(m.x);
  D.nt = I(m.nt);
  D.rcs_off = (const int64_t*)(w + m.rcs_off);
  D.tile_nz = (const uint8_t*)(w + m.tile_nz);
  D.diag_off = (const int64_t*)(w + m.diag_off);
  D.vec_off = (const int64_t*)(w + m.vec_off);
  D.blk_fail = I(m.blk_fail);
  D.blk_nc = I(m.blk_nc);
  D.rec_valid = I(m.rec_valid);
  D.variant = o->variant;
  D.rho_t = F(m.rho_t);
  D.rho_growth = o->rho_growth;
  D.filter_px = o->filter_px;
  D.Xt = o->variant >= RPBA_VARIANT_PLAIN ? F(m.Xt) : nullptr;
  const bool adaptive = o->damping == RPBA_DAMPING_ADAPTIVE;
  D.lam_blk = adaptive ? F(m.lam_blk) : nullptr;
  D.blk_rej = I(m.blk_rej);
  D.XcOld = adaptive ? F(m.XcOld) : nullptr;
  D.lam_up = o->lambda_up;
  D.lam_down = o->lambda_down;
  D.lam_min = o->lambda_min;
  D.lam_max = o->lambda_max;
  D.acc_int = F(m.acc_int);
  D.acc_blk = F(m.acc_blk);
  D.acc_cons = F(m.acc_cons);
  D.cons_part = F(m.cons_part);
  D.int_part = F(m.int_part);
  D.upd_part = F(m.upd_part);
  D.acc_rob = F(m.acc_rob);

  // finite inputs, positive definite information matrices
  {
    int32_t* cnt = I(m.chk);
    launch_zero_i32(cnt, 2, st);
    launch_check_inputs(D, cnt, st);
    int32_t hc[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hc[0] || hc[1])
      return fail(RPBA_ERR_ARG, std::to_string(hc[0]) + " non-finite input values (cam_R, cam_C, cam_intr, pts, obs_xy, obs_info), " +
                                    std::to_string(hc[1]) + " obs_info matrices not positive definite");
  }
  // packing kernels, zero state, identity padding
  launch_gather(D, st);
  launch_zero(D.Xc, 3 * D.NC, st);
  launch_zero(D.Om, 6 * D.NC, st);
  launch_zero(D.cpk, CPK * D.NC, st);
  launch_zero(D.S, p.rcs_total, st);
  launch_zero(D.Ld, p.diag_total, st);
  launch_zero(D.Li, p.diag_total, st);
  launch_zero(D.y, p.vec_total, st);
  launch_zero(D.ys, p.vec_total, st);
  launch_zero(D.x, p.vec_total, st);
  launch_zero_i32(D.blk_fail, D.L, st);
  launch_zero_i32(D.blk_nc, D.L, st);
  launch_zero_i32(D.rec_valid, 1, st);
  launch_zero_i32((int32_t*)(w + m.df_flags), 2 * (p.rcs_total / ((int64_t)p.T * p.T)), st);
  launch_zero_i32((int32_t*)(w + m.df_ctl), 4, st);
  launch_df_reset((int32_t*)(w + m.df_ctl), st);
  launch_zero_i32(D.blk_fresh, D.L, st);
  launch_zero_i32((int32_t*)(w + m.dfb_flags), p.vec_total / p.T, st);
  launch_zero_i32((int32_t*)(w + m.rob_bad), D.N, st);
  launch_zero((double*)(w + m.rob_sigma), D.M, st);
  launch_init_rcs(D, st);
  HIP_TRY(hipMemcpyAsync(D.rho_t, &o->rho, sizeof(double), hipMemcpyHostToDevice, st));
  launch_zero_i32(D.blk_rej, D.L, st);
  if (adaptive) {
    const std::vector<double> lam0(p.L, o->lambda);
    HIP_TRY(hipMemcpyAsync(D.lam_blk, lam0.data(), 8 * (size_t)p.L, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // lam0 is a host temporary
  }
  if (o->variant >= RPBA_VARIANT_PLAIN) launch_init_copies(D, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  *out = h.release();
  return RPBA_OK;
}

rpba_status rpba_destroy(rpba_problem* h) {
  delete h;
  return RPBA_OK;
}

rpba_status rpba_intersect(rpba_problem* h, double* cov, int32_t* status, double* stats) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  rpba_status s = run_call(h, h->g_int, cov, status, stats, [&]() -> rpba_status {
    {
      PhaseTimer t(h, PH_INTERSECT, 3);
      launch_intersect(h->d, cov != nullptr, h->stream);
    }
    PhaseTimer t(h, PH_INT_EXPORT, 1);
    launch_intersect_export(h->d, cov, status, stats, h->stream);
    return RPBA_OK;
  });
  if (s != RPBA_OK) return s;
  h->intersected = true;
  return RPBA_OK;
}

static rpba_status assemble(rpba_problem* h, const uint8_t* active) {
  h->d.active = active;
  {
    PhaseTimer t(h, PH_COPY_PREP, 3);
    launch_copy_prep(h->d, h->stream);
  }
  {
    const bool fp32 = h->opt.precision == RPBA_MIXED;
    {
      PhaseTimer t(h, PH_SCHUR, 1 + (h->any_dense ? 2 : 0));
      launch_schur_diag(h->d, fp32, h->any_dense, h->plan->rcs_total, h->stream);
    }
    if (h->d.n_od) {
      PhaseTimer t(h, PH_SCHUR_OD, 1);
      launch_schur_offdiag(h->d, fp32, h->stream);
    }
  }
  HIP_TRY(hipGetLastError());
  return RPBA_OK;
}

// Forward factorisation of the dense reduced camera systems, step k = 0 ..
// nt - 1, three launches per step over all sub-blocks: diagonal factor,
// panel solves, trailing update.
static rpba_status chol_forward(rpba_problem* h, const int32_t* pot, const int32_t* fwd, const int32_t* upd) {
  hipStream_t st = h->stream;
  if (h->dataflow) {
    launch_chol_dataflow(h->d, (const int32_t*)(h->ws + h->map.df_tasks), h->df_ntask,
                         (int*)(h->ws + h->map.df_flags), h->plan->rcs_total / ((int64_t)h->plan->T * h->plan->T),
                         (int*)(h->ws + h->map.df_ctl), h->df_fwd_workers, st);
    return RPBA_OK;
  }
  for (int k = 0; k < h->nt_max_dense; ++k) {
    launch_chol_potrf(h->d, k, pot + h->pot_off[k], h->pot_off[k + 1] - h->pot_off[k], st);
    launch_chol_trsm(h->d, k, fwd + h->fwd_off[k], h->fwd_off[k + 1] - h->fwd_off[k], st);
    launch_chol_update(h->d, k, upd + h->upd_off[k], h->upd_off[k + 1] - h->upd_off[k], st);
  }
  return RPBA_OK;
}

rpba_status rpba_subblock_lm_step(rpba_problem* h, const uint8_t* active, double* block_stats) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  if (!h->intersected) return fail(RPBA_ERR_STATE, "rpba_intersect must run before the first LM step");
  const Plan& p = *h->plan;
  rpba_status s = run_call(h, h->g_step, active, block_stats, nullptr, [&]() -> rpba_status {
    rpba_status s1 = assemble(h, active);
    if (s1 != RPBA_OK) return s1;
    const int32_t* pot = (const int32_t*)(h->ws + h->map.pot_items);
    const int32_t* fwd = (const int32_t*)(h->ws + h->map.fwd_items);
    const int32_t* upd = (const int32_t*)(h->ws + h->map.upd_items);
    const int32_t* bwd = (const int32_t*)(h->ws + h->map.bwd_items);
    if (h->any_dense) {
      {
        PhaseTimer t(h, PH_CHOL_FWD, h->dataflow ? 1 : 3 * h->nt_max_dense);
        rpba_status s2 = chol_forward(h, pot, fwd, upd);
        if (s2 != RPBA_OK) return s2;
      }
      {
        PhaseTimer t(h, PH_CHOL_BWD, h->dataflow ? 3 : h->nt_max_dense + 1);
        launch_rhs_extract(h->d, (const int*)(h->ws + h->map.df_ctl), h->stream);
        if (h->dataflow)
          launch_chol_backward_dataflow(h->d, (const int32_t*)(h->ws + h->map.dfb_tasks), h->dfb_ntask,
                                        (int*)(h->ws + h->map.dfb_flags), (int*)(h->ws + h->map.df_ctl),
                                        h->df_workers, h->stream);
        else
          for (int s2 = 0; s2 < p.nt_max; ++s2)
            launch_chol_backward(h->d, bwd + h->bwd_off[s2], h->bwd_off[s2 + 1] - h->bwd_off[s2], h->stream);
      }
    }
    if (h->n_pcg) {
      const bool learned = h->opt.solver == RPBA_SOLVER_PCG_LEARNED || h->opt.solver == RPBA_SOLVER_AUTO_LEARNED;
      PhaseTimer t(h, PH_SOLVE_IT, learned ? 3 : 2);
      if (learned) launch_mean_diag(h->d, (float*)(h->ws + h->map.mean_diag), h->stream);
      launch_precond_learned(h->d, learned ? (const float*)(h->ws + h->map.mlp_w) : nullptr,
                             (const float*)(h->ws + h->map.mean_diag), (const float*)(h->ws + h->map.cam_tpfrac),
                             h->stream);
      launch_pcg(h->d, (const int32_t*)(h->ws + h->map.pcg_list), h->n_pcg, h->max_pcg_n, h->opt.pcg_maxit,
                 h->opt.pcg_tol, h->opt.ir_tol, h->opt.ir_maxit, h->stream);
    }
    {
      PhaseTimer t(h, PH_UPDATE, 4);
      launch_update(h->d, block_stats, h->stream);
    }
    return RPBA_OK;
  });
  h->d.active = nullptr;
  return s;
}

rpba_status rpba_consensus(rpba_problem* h, double* stats) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  return run_call(h, h->g_cons, stats, nullptr, nullptr, [&]() -> rpba_status {
    PhaseTimer t(h, PH_CONSENSUS, 4);
    launch_consensus(h->d, stats, h->stream);
    return RPBA_OK;
  });
}

rpba_status rpba_set_graph(rpba_problem* h, int32_t on) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  h->use_graph = on != 0;
  if (!h->use_graph) {
    h->g_int.reset();
    h->g_step.reset();
    h->g_cons.reset();
  }
  return RPBA_OK;
}

rpba_status rpba_set_timing(rpba_problem* h, int32_t on) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  if (on && !h->ev[0]) {
    HIP_TRY(hipEventCreate(&h->ev[0]));
    HIP_TRY(hipEventCreate(&h->ev[1]));
  }
  h->timing = on != 0;
  for (int q = 0; q < NPHASE; ++q) {
    h->ms[q] = 0;
    h->launches[q] = 0;
    h->calls[q] = 0;
  }
  return RPBA_OK;
}

int32_t rpba_get_timing(rpba_problem* h, double* ms, int64_t* launches, int64_t* calls, int32_t n) {
  if (!h) return -1;
  for (int q = 0; q < NPHASE && q < n; ++q) {
    if (ms) ms[q] = h->ms[q];
    if (launches) launches[q] = h->launches[q];
    if (calls) calls[q] = h->calls[q];
  }
  return NPHASE;
}

rpba_status rpba_robust_reweight(rpba_problem* h, int32_t mode, double* stats) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  if (mode != RPBA_ROBUST_WEIGHT && mode != RPBA_ROBUST_ELIMINATE_POINTS && mode != RPBA_ROBUST_DELETE_OBS)
    return fail(RPBA_ERR_ARG, "mode must be RPBA_ROBUST_WEIGHT, RPBA_ROBUST_ELIMINATE_POINTS or RPBA_ROBUST_DELETE_OBS");
  if (!h->opt.robust) return fail(RPBA_ERR_STATE, "the handle was created without opt->robust: no residuals are kept");
  if (!h->intersected) return fail(RPBA_ERR_STATE, "rpba_intersect must run before rpba_robust_reweight");
  CallGraph& g = h->g_rob[mode];
  return run_call(h, g, stats, nullptr, nullptr, [&]() -> rpba_status {
    PhaseTimer t(h, PH_ROBUST, stats ? 4 : 3);
    launch_robust(h->d, (double*)(h->ws + h->map.rob_vals), (const int64_t*)(h->ws + h->map.rob_off),
                  (int32_t*)(h->ws + h->map.rob_bad), (double*)(h->ws + h->map.rob_sigma), h->opt.t_v,
                  h->opt.down_weight, mode, stats, h->stream);
    return RPBA_OK;
  });
}

rpba_status rpba_covariance(rpba_problem* h, double lambda, double* cam_cov, double* copy_cov) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(RPBA_ERR_ARG, "lambda must be finite and >= 0");
  if (!h->opt.covariance) return fail(RPBA_ERR_STATE, "the handle was created without opt->covariance");
  if (!h->intersected) return fail(RPBA_ERR_STATE, "rpba_intersect must run before rpba_covariance");
  if (h->n_pcg) return fail(RPBA_ERR_STATE, "a sub-block is solved by PCG: it has no factor to invert");
  const Plan& p = *h->plan;
  const double lam0 = h->d.lambda;
  double* const lam_blk0 = h->d.lam_blk;
  h->d.lambda = lambda;
  h->d.lam_blk = nullptr;  // one damping for every sub-block here
  // the intersection's fused copy records carry its damping: rebuild them
  launch_zero_i32(h->d.rec_valid, 1, h->stream);
  rpba_status s = assemble(h, nullptr);
  if (s == RPBA_OK)
    s = chol_forward(h, (const int32_t*)(h->ws + h->map.pot_items), (const int32_t*)(h->ws + h->map.fwd_items),
                     (const int32_t*)(h->ws + h->map.upd_items));
  // the dataflow launch hands its control words on through the step's last
  // kernel: no backward substitution follows here, so finish it explicitly
  if (s == RPBA_OK && h->dataflow) launch_df_finish(h->d, (int*)(h->ws + h->map.df_ctl), h->stream);
  h->d.lambda = lam0;
  h->d.lam_blk = lam_blk0;
  h->d.active = nullptr;
  if (s != RPBA_OK) return s;
  std::vector<int32_t> bad(p.L);
  HIP_TRY(hipMemcpyAsync(bad.data(), h->d.blk_fail, 4 * (size_t)p.L, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int l = 0; l < p.L; ++l)
    if (bad[l]) return fail(RPBA_ERR_NOT_SPD, "sub-block " + std::to_string(l) + ": system not positive definite");
  h->d.lambda = lambda;  // the copy pass rebuilds V with the same damping
  h->d.lam_blk = nullptr;
  launch_cov_inverse(h->d, (double*)(h->ws + h->map.covY), p.nt_max, h->stream);
  launch_cov_outputs(h->d, cam_cov, copy_cov, h->stream);
  h->d.lambda = lam0;
  h->d.lam_blk = lam_blk0;
  HIP_TRY(hipGetLastError());
  // the RCS storage now holds S^-1: the next step assembles it afresh
  return RPBA_OK;
}

rpba_status rpba_get_damping(rpba_problem* h, double* lambda, int32_t* rejected) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const int L = h->plan->L;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (lambda) {
    if (h->d.lam_blk) HIP_TRY(hipMemcpy(lambda, h->d.lam_blk, 8 * (size_t)L, hipMemcpyDeviceToHost));
    else
      for (int l = 0; l < L; ++l) lambda[l] = h->d.lambda;
  }
  if (rejected) {
    if (h->d.lam_blk) HIP_TRY(hipMemcpy(rejected, h->d.blk_rej, 4 * (size_t)L, hipMemcpyDeviceToHost));
    else
      for (int l = 0; l < L; ++l) rejected[l] = 0;
  }
  return RPBA_OK;
}

rpba_status rpba_get_robust(rpba_problem* h, double* sigma_cam, double* obs_weight) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const Plan& p = *h->plan;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (sigma_cam) {
    std::vector<double> t(p.M);
    HIP_TRY(hipMemcpy(t.data(), h->ws + h->map.rob_sigma, 8 * (size_t)p.M, hipMemcpyDeviceToHost));
    for (int i = 0; i < p.M; ++i) sigma_cam[p.cam_orig[i]] = t[i];
  }
  if (obs_weight) {
    std::vector<double> t(p.K);
    HIP_TRY(hipMemcpy(t.data(), h->d.rw, 8 * (size_t)p.K, hipMemcpyDeviceToHost));
    for (int k = 0; k < p.K; ++k) obs_weight[p.obs_orig[k]] = t[k];
  }
  return RPBA_OK;
}

int64_t rpba_num_copies(rpba_problem* h) { return h ? h->plan->NC : -1; }

int32_t rpba_block_cameras(rpba_problem* h, int32_t l) {
  if (!h || l < 0 || l >= h->plan->L) return -1;
  return h->plan->blk_cam_off[l + 1] - h->plan->blk_cam_off[l];
}


rpba_status rpba_get_copies(rpba_problem* h, int32_t* blk, int32_t* pt, double* X, double* omega) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const Plan& p = *h->plan;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (blk) std::memcpy(blk, p.copy_blk.data(), 4 * p.NC);
  if (pt)
    for (int64_t c = 0; c < p.NC; ++c) pt[c] = p.pt_orig[p.copy_pt[c]];
  if (X) {
    // copies of a sub-block not updated since the last intersection are at Xbar
    HIP_TRY(hipMemcpy(X, h->d.Xc, 8 * 3 * p.NC, hipMemcpyDeviceToHost));
    std::vector<int32_t> fresh(p.L);
    HIP_TRY(hipMemcpy(fresh.data(), h->d.blk_fresh, 4 * (size_t)p.L, hipMemcpyDeviceToHost));
    std::vector<double> xb(3 * (size_t)p.N);
    HIP_TRY(hipMemcpy(xb.data(), h->d.Xbar, 8 * 3 * (size_t)p.N, hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < p.NC; ++c)
      if (fresh[p.copy_blk[c]])
        for (int r = 0; r < 3; ++r) X[3 * c + r] = xb[(size_t)r * p.N + p.copy_pt[c]];
  }
  if (omega) {
    if (h->d.om_f32) {
      std::vector<float> om((size_t)6 * p.NC);
      HIP_TRY(hipMemcpy(om.data(), h->d.Omf, 4 * om.size(), hipMemcpyDeviceToHost));
      for (size_t q = 0; q < om.size(); ++q) omega[q] = om[q];
    } else {
      HIP_TRY(hipMemcpy(omega, h->d.Om, 8 * 6 * p.NC, hipMemcpyDeviceToHost));
    }
  }
  return RPBA_OK;
}

// caller rank (position in ascending original index) of each internal camera
// position of sub-block l
static std::vector<int32_t> block_caller_rank(const Plan& p, int32_t l) {
  const int32_t b = p.blk_cam_off[l], n = p.blk_cam_off[l + 1] - b;
  std::vector<int32_t> q(n), rank(n);
  for (int32_t a = 0; a < n; ++a) q[a] = a;
  std::sort(q.begin(), q.end(), [&](int32_t x, int32_t y) { return p.cam_orig[b + x] < p.cam_orig[b + y]; });
  for (int32_t r = 0; r < n; ++r) rank[q[r]] = r;
  return rank;
}

// S of sub-block l assembled at the current state, rows and columns in the
// caller's camera order (the library keeps its own order inside a
// sub-block).  Runs the assembly kernels of an LM step without solving.
rpba_status rpba_get_block_rcs(rpba_problem* h, int32_t l, double* S, double* e) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const Plan& p = *h->plan;
  if (l < 0 || l >= p.L) return fail(RPBA_ERR_ARG, "sub-block out of range");
  if (!h->intersected) return fail(RPBA_ERR_STATE, "rpba_intersect must run first");
  rpba_status s = assemble(h, nullptr);
  if (s != RPBA_OK) return s;
  const int np = p.np;
  int n6 = np * (p.blk_cam_off[l + 1] - p.blk_cam_off[l]);
  // stage through the x / ys vectors is not possible for a full matrix: use
  // the Ld array (free outside a step) when large enough, else the cpk array
  size_t need = (size_t)n6 * n6 + n6;
  double* stage = nullptr;
  if ((int64_t)need <= p.diag_total * 2) stage = h->d.Ld;  // Ld and Li are contiguous in the layout
  else if ((int64_t)need <= CPK * p.NC) stage = h->d.cpk;
  else return fail(RPBA_ERR_STATE, "no staging space for this sub-block");
  if (h->blk_pcg[l]) {
    launch_zero(stage, (int64_t)n6 * n6, h->stream);
    launch_bsr_extract(h->d, l, stage, stage + (size_t)n6 * n6, h->stream);
  } else {
    launch_rcs_extract(h->d, l, stage, stage + (size_t)n6 * n6, h->stream);
  }
  // staging in the copy records overwrites them: the next LM step rebuilds them
  if (stage == h->d.cpk) launch_zero_i32(h->d.rec_valid, 1, h->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<double> Si((size_t)n6 * n6), ei(n6);
  HIP_TRY(hipMemcpy(Si.data(), stage, 8 * (size_t)n6 * n6, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ei.data(), stage + (size_t)n6 * n6, 8 * (size_t)n6, hipMemcpyDeviceToHost));
  // a Cholesky sub-block stores its lower triangle only: mirror it before
  // the reordering moves entries across the diagonal
  if (!h->blk_pcg[l])
    for (int r = 0; r < n6; ++r)
      for (int c = r + 1; c < n6; ++c) Si[(size_t)r * n6 + c] = Si[(size_t)c * n6 + r];
  const std::vector<int32_t> rank = block_caller_rank(p, l);
  auto to = [&](int r) { return np * rank[r / np] + r % np; };
  if (S)
    for (int r = 0; r < n6; ++r)
      for (int c = 0; c < n6; ++c) S[(size_t)to(r) * n6 + to(c)] = Si[(size_t)r * n6 + c];
  if (e)
    for (int r = 0; r < n6; ++r) e[to(r)] = ei[r];
  return RPBA_OK;
}

rpba_status rpba_get_block_solution(rpba_problem* h, int32_t l, double* x) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const Plan& p = *h->plan;
  if (l < 0 || l >= p.L) return fail(RPBA_ERR_ARG, "sub-block out of range");
  const int np = p.np;
  int n6 = np * (p.blk_cam_off[l + 1] - p.blk_cam_off[l]);
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<double> xi(n6);
  HIP_TRY(hipMemcpy(xi.data(), h->d.x + p.vec_off[l], 8 * (size_t)n6, hipMemcpyDeviceToHost));
  const std::vector<int32_t> rank = block_caller_rank(p, l);
  for (int r = 0; r < n6; ++r) x[np * rank[r / np] + r % np] = xi[r];
  return RPBA_OK;
}

int32_t rpba_block_solver(rpba_problem* h, int32_t l) {
  if (!h || l < 0 || l >= h->plan->L) return -1;
  return h->blk_pcg[l] ? 1 : 0;
}

rpba_status rpba_camera_order(rpba_problem* h, int32_t* cam_orig) {
  if (!h || !cam_orig) return fail(RPBA_ERR_ARG, "NULL argument");
  std::memcpy(cam_orig, h->plan->cam_orig.data(), 4 * (size_t)h->plan->M);
  return RPBA_OK;
}

rpba_status rpba_factor_flops(rpba_problem* h, double* out) {
  if (!h || !out) return fail(RPBA_ERR_ARG, "NULL argument");
  const Plan& p = *h->plan;
  const double T = p.T, T2 = T * T, T3 = T2 * T;
  // 16 x 16 block products inside one diagonal tile: trailing updates of
  // the panels plus the blocks of the inverse, 2 * 16^3 operations each
  const int nbk = p.T / 16;
  int64_t blk16 = 0;
  for (int kb = 0; kb < nbk; ++kb) blk16 += (int64_t)(nbk - 1 - kb) * (nbk - kb) / 2;
  for (int r = 1; r < nbk; ++r)
    for (int j = 0; j < r; ++j) blk16 += r - j + 1;
  const double diag_mfma = 2.0 * 4096.0 * (double)blk16;
  double alg = 0.0, dense = 0.0, mfma = 0.0;
  for (int l = 0; l < p.L; ++l) {
    if (h->blk_pcg[l]) continue;
    const double n6 = (double)p.np * (p.blk_cam_off[l + 1] - p.blk_cam_off[l]);
    dense += n6 * n6 * n6 / 3.0 + n6 * n6;
    const int nt = p.nt[l];
    const uint8_t* z = p.tile_nz.data() + p.rcs_off[l] / ((int64_t)p.T * p.T);
    auto nz = [&](int i, int j) { return z[(int64_t)i * (i + 1) / 2 + j] != 0; };
    for (int j = 0; j < nt; ++j)
      for (int i = j; i <= nt; ++i) {
        if (!nz(i, j)) continue;
        int64_t prods = 0;
        for (int k = 0; k < j; ++k) prods += nz(i, k) && nz(j, k);
        if (i == nt) {
          alg += 2.0 * T2 * prods + T2;
        } else if (i == j) {
          alg += T3 * prods + T3 / 3.0;
        } else {
          alg += 2.0 * T3 * prods + T3;
        }
        mfma += 2.0 * T3 * prods + (i == j ? diag_mfma : 2.0 * T3);
      }
  }
  out[0] = alg;
  out[1] = dense;
  out[2] = mfma;
  return RPBA_OK;
}

rpba_status rpba_get_precond_blocks(rpba_problem* h, int32_t l, double* P) {
  if (!h || !P) return fail(RPBA_ERR_ARG, "NULL argument");
  const Plan& p = *h->plan;
  if (l < 0 || l >= p.L) return fail(RPBA_ERR_ARG, "sub-block out of range");
  if (!h->blk_pcg[l]) return fail(RPBA_ERR_STATE, "sub-block is not solved iteratively");
  const int32_t b = p.blk_cam_off[l], n = p.blk_cam_off[l + 1] - b;
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<float> t((size_t)36 * n);
  HIP_TRY(hipMemcpy(t.data(), h->d.Pblk + (size_t)36 * b, 4 * t.size(), hipMemcpyDeviceToHost));
  const std::vector<int32_t> rank = block_caller_rank(p, l);
  for (int32_t a = 0; a < n; ++a)
    for (int q = 0; q < 36; ++q) P[(size_t)36 * rank[a] + q] = t[(size_t)36 * a + q];
  return RPBA_OK;
}

rpba_status rpba_step_status(rpba_problem* h, int32_t* n_not_spd, int32_t* n_nonconverged) {
  if (!h) return fail(RPBA_ERR_ARG, "NULL handle");
  const int L = h->plan->L;
  HIP_TRY(hipStreamSynchronize(h->stream));
  std::vector<int32_t> f(L), nc(L);
  HIP_TRY(hipMemcpy(f.data(), h->d.blk_fail, 4 * (size_t)L, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(nc.data(), h->d.blk_nc, 4 * (size_t)L, hipMemcpyDeviceToHost));
  int32_t a = 0, b = 0;
  for (int l = 0; l < L; ++l) {
    a += f[l] != 0;
    b += nc[l] != 0;
  }
  if (n_not_spd) *n_not_spd = a;
  if (n_nonconverged) *n_nonconverged = b;
  if (a) return fail(RPBA_ERR_NOT_SPD, std::to_string(a) + " sub-block(s) with a reduced camera system that is not positive definite");
  if (b) return fail(RPBA_WARN_NONCONVERGED, std::to_string(b) + " iterative sub-block(s) above the refinement tolerance");
  return RPBA_OK;
}

int32_t rpba_ratio_update(int32_t n, const double* cost, double ratio, double* best, uint8_t* grace, uint8_t* active) {
  if (n < 0 || (n > 0 && (!cost || !best || !grace || !active))) return -1;
  int32_t live = 0;
  for (int32_t q = 0; q < n; ++q) {
    if (!active[q]) continue;
    const bool slow = best[q] / cost[q] < ratio;
    if (slow && grace[q]) active[q] = 0;
    if (slow) grace[q] = 1;
    best[q] = std::min(best[q], cost[q]);
    live += active[q] != 0;
  }
  return live;
}

int32_t rpba_precond_num_params(void) { return mlp_num_params(); }

int32_t rpba_precond_sample_stride(int32_t nz) { return mlp_num_features() + 36 + 12 * nz; }

int32_t rpba_precond_num_samples(rpba_problem* h) { return h ? h->n_pcg_cams : -1; }

rpba_status rpba_set_precond_weights(rpba_problem* h, const float* W) {
  if (!h || !W) return fail(RPBA_ERR_ARG, "NULL argument");
  HIP_TRY(hipMemcpyAsync(h->ws + h->map.mlp_w, W, 4 * (size_t)mlp_num_params(), hipMemcpyDeviceToDevice, h->stream));
  h->have_weights = true;
  return RPBA_OK;
}

rpba_status rpba_precond_harvest(rpba_problem* h, const float* z, int32_t nz, float* out) {
  if (!h || !z || !out || nz < 1) return fail(RPBA_ERR_ARG, "bad harvest arguments");
  if (!h->intersected) return fail(RPBA_ERR_STATE, "rpba_intersect must run first");
  if (h->n_pcg == 0) return fail(RPBA_ERR_STATE, "no sub-block uses the iterative solver");
  rpba_status s = assemble(h, nullptr);
  if (s != RPBA_OK) return s;
  launch_mean_diag(h->d, (float*)(h->ws + h->map.mean_diag), h->stream);
  launch_harvest(h->d, (const float*)(h->ws + h->map.mean_diag), (const float*)(h->ws + h->map.cam_tpfrac), z, nz,
                 (const int32_t*)(h->ws + h->map.pcg_cams), h->n_pcg_cams, out, h->stream);
  HIP_TRY(hipGetLastError());
  return RPBA_OK;
}

size_t rpba_precond_train_scratch(int32_t nsamp) {
  return 4 * ((size_t)nsamp * mlp_scratch_per_sample() + (size_t)((nsamp + 255) / 256) + 64);
}

rpba_status rpba_precond_train_step(const float* samples, int32_t nsamp, int32_t nz, float* W, float* m, float* v,
                                    int32_t t, float lr, void* scratch, float* grad, float* loss, int32_t apply,
                                    void* stream) {
  if (!samples || nsamp < 1 || nz < 1 || !W || !grad || !scratch || (apply && (!m || !v || t < 1)))
    return fail(RPBA_ERR_ARG, "bad training arguments");
  float* sc = (float*)scratch;
  float* parts = sc + (size_t)nsamp * mlp_scratch_per_sample();
  launch_train_step(samples, nsamp, nz, W, m, v, t, lr, sc, grad, parts, apply != 0, (hipStream_t)stream);
  if (loss) launch_sum_f32(parts, (nsamp + 255) / 256, loss, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return RPBA_OK;
}

rpba_status rpba_precond_train_step_noalloc(const float* samples, int32_t nsamp, int32_t nz, float* W, float* m,
                                            float* v, int32_t t, float lr, float* grad, float* loss, int32_t apply,
                                            void* stream) {
  if (!samples || nsamp < 1 || nz < 1 || !W || !grad || (apply && (!m || !v || t < 1)))
    return fail(RPBA_ERR_ARG, "bad training arguments");
  if (nsamp > RPBA_TRAIN_NOALLOC_MAX_SAMPLES)
    return fail(RPBA_ERR_ARG, "rpba_precond_train_step_noalloc: " + std::to_string(nsamp) +
                                  " samples exceed the maximum of " + std::to_string(RPBA_TRAIN_NOALLOC_MAX_SAMPLES) +
                                  " per call");
  hipError_t e = hipSuccess;
  float* sc = train_noalloc_scratch(&e);
  if (!sc) return fail(RPBA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  float* parts = sc + train_noalloc_parts_offset();
  launch_train_step(samples, nsamp, nz, W, m, v, t, lr, sc, grad, parts, apply != 0, (hipStream_t)stream);
  if (loss) launch_sum_f32(parts, (nsamp + 255) / 256, loss, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return RPBA_OK;
}

rpba_status rpba_selftest_gemm(const double* A, const double* B, double* C, void* stream) {
  launch_selftest_gemm(A, B, C, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return RPBA_OK;
}

}  // extern "C"
