// librpba kernels of the FP64 path: packing, intersection with covariance and
// refined tie-point weights (eq:bars, Sec. 5.1), the sub-block normal
// equations with tie-point priors and their Schur complement (eq:bact,
// Sec. 2 and 5.4), back-substitution / update / new cost, and the consensus
// exchange (Sec. 5).
#include "rpba_device.hpp"
#include "rpba_internal.hpp"
#include "rpba_plan.hpp"

namespace rpba {

namespace {

constexpr int NT = 256;  // threads per workgroup of the streaming kernels

inline unsigned grid_for(int64_t n, int per = NT) { return (unsigned)((n + per - 1) / per); }

// weight of LM-order observation k; unit: every robust multiplier is 1 and
// is not read
__device__ __forceinline__ W2<double> obs_weight(const Dev& d, int64_t k, bool unit) {
  const double r = unit ? 1.0 : d.rw[k];
  if (d.has_info) {
    const double* w = d.info + 3 * k;
    return {r * w[0], r * w[1], r * w[2]};
  }
  return {r * d.w0, 0.0, r * d.w0};
}

// one observation of a copy (LM order): camera index, pixel, weight and the
// camera itself from `cams` (the cameras of the step or the updated ones;
// CAL: with its f and k1)
template <bool CAL>
struct CopyObs {
  int cam;
  double x, y;
  W2<double> W;
  double cm[CAL ? 14 : 12];
};
template <bool CAL>
__device__ __forceinline__ void copy_obs(const Dev& d, const double* cams, const double* intrs, int64_t k, bool unit,
                                         CopyObs<CAL>& o) {
  o.cam = d.obs_cam[k];
  const double2 v = reinterpret_cast<const double2*>(d.xy)[k];
  o.x = v.x;
  o.y = v.y;
  o.W = obs_weight(d, k, unit);
  const double2* g = reinterpret_cast<const double2*>(cams + (int64_t)CAM_STRIDE * o.cam);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double2 w = g[q];
    o.cm[2 * q] = w.x;
    o.cm[2 * q + 1] = w.y;
  }
  if constexpr (CAL) {
    const double2 fk = reinterpret_cast<const double2*>(intrs)[o.cam];
    o.cm[CAM_F] = fk.x;
    o.cm[CAM_K1] = fk.y;
  }
}

// f(observation) over the observations [k0, k1) of a copy, in order (one at
// a time: a second one in flight costs more occupancy than it hides);
// cameras from `cams` and, with intrinsics, their f and k1 from `intrs`
template <bool CAL, typename F>
__device__ __forceinline__ void for_copy_obs(const Dev& d, const double* cams, const double* intrs, int k0, int k1,
                                             bool unit, F&& f) {
  for (int k = k0; k < k1; ++k) {
    CopyObs<CAL> a;
    copy_obs<CAL>(d, cams, intrs, k, unit, a);
    f(a);
  }
}

// sum over a workgroup of 256 threads of `n` doubles; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* [NV][8] */) {
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q * 8 + wv] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = sh[q * 8 + 0] + sh[q * 8 + 1] + sh[q * 8 + 2] + sh[q * 8 + 3];
}

// ------------------------------------------------------------------ packing
__global__ void k_gather_obs(Dev d) {
  int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (k >= d.K) return;
  int64_t o = d.obs_orig[k];
  d.xy[2 * k] = d.u_xy[o];
  d.xy[2 * k + 1] = d.u_xy[(int64_t)d.K + o];
  if (d.has_info) {
    d.info[3 * k] = d.u_info[o];
    d.info[3 * k + 1] = d.u_info[(int64_t)d.K + o];
    d.info[3 * k + 2] = d.u_info[2 * (int64_t)d.K + o];
  }
  d.rw[k] = 1.0;
  if (d.res) {
    d.res[2 * k] = 0.0;
    d.res[2 * k + 1] = 0.0;
  }
}

// input check of rpba_create: non-finite values of the caller's arrays, and
// information matrices that are not positive definite (w11 > 0, det > 0)
__global__ void k_check_inputs(Dev d, int32_t* cnt) {
  const int64_t n1 = 9 * (int64_t)d.M, n2 = n1 + 3 * (int64_t)d.M, n3 = n2 + 3 * (int64_t)d.N,
                n4 = n3 + 2 * (int64_t)d.K, n5 = n4 + (d.u_info ? 3 * (int64_t)d.K : 0),
                n6 = n5 + (d.u_intr ? 2 * (int64_t)d.M : 0);
  int bad = 0, npd = 0;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n6; t += (int64_t)gridDim.x * NT) {
    const double v = t < n1 ? d.u_camR[t] : t < n2 ? d.u_camC[t - n1] : t < n3 ? d.u_pts[t - n2]
                   : t < n4 ? d.u_xy[t - n3] : t < n5 ? d.u_info[t - n4] : d.u_intr[t - n5];
    // (a focal length must be positive as well)
    bad += !isfinite(v) || (t >= n5 && t < n5 + d.M && !(v > 0.0));
  }
  if (d.u_info)
    for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < d.K; k += (int64_t)gridDim.x * NT) {
      const double a = d.u_info[k], b = d.u_info[(int64_t)d.K + k], c = d.u_info[2 * (int64_t)d.K + k];
      npd += !(a > 0.0 && a * c - b * b > 0.0);
    }
  for (int o = 32; o > 0; o >>= 1) {
    bad += __shfl_xor(bad, o);
    npd += __shfl_xor(npd, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (bad) atomicAdd(&cnt[0], bad);
    if (npd) atomicAdd(&cnt[1], npd);
  }
}

// camera-major copies of the pixels and weights (after k_gather_obs)
__global__ void k_gather_cm(Dev d) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= d.K) return;
  const int64_t k = d.cam_obs[t];
  if (t == 0) *d.rw_unit = 1;  // k_gather_obs set every robust weight to 1
  d.cm_xy[2 * t] = d.xy[2 * k];
  d.cm_xy[2 * t + 1] = d.xy[2 * k + 1];
  d.cm_rw[t] = d.rw[k];
  if (d.has_info)
    for (int q = 0; q < 3; ++q) d.cm_info[3 * t + q] = d.info[3 * k + q];
}

__global__ void k_gather_cams(Dev d) {
  int i = blockIdx.x * NT + threadIdx.x;
  if (i >= d.M) return;
  int o = d.cam_orig[i];
  double* c = d.cam + (int64_t)CAM_STRIDE * i;
  for (int q = 0; q < 9; ++q) c[q] = d.u_camR[9 * (int64_t)o + q];
  for (int r = 0; r < 3; ++r) c[9 + r] = d.u_camC[(int64_t)r * d.M + o];
  if (d.intr) {
    d.intr[2 * (int64_t)i] = d.u_intr[o];
    d.intr[2 * (int64_t)i + 1] = d.u_intr[(int64_t)d.M + o];
  }
}

__global__ void k_gather_pts(Dev d) {
  int j = blockIdx.x * NT + threadIdx.x;
  if (j >= d.N) return;
  int o = d.pt_orig[j];
  for (int r = 0; r < 3; ++r) {
    double v = d.u_pts[(int64_t)r * d.N + o];
    d.P0[(int64_t)r * d.N + j] = v;
    d.Xbar[(int64_t)r * d.N + j] = v;
  }
  d.status[j] = 0;
}

__global__ void k_zero(double* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) p[t] = 0.0;
}
// the same for a large 16-byte aligned array: 16-byte stores, four per
// thread and round
__global__ void k_zero_wide(double* p, int64_t n) {
  double2* q = reinterpret_cast<double2*>(p);
  const int64_t n2 = n / 2, stride = (int64_t)gridDim.x * NT;
  const double2 z = make_double2(0.0, 0.0);
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n2; t += 4 * stride) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (t + u * stride < n2) q[t + u * stride] = z;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) p[n - 1] = 0.0;
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) p[t] = 0;
}

// identity on the padded rows of the last diagonal tile of every sub-block
__global__ void k_pad_identity(Dev d) {
  int l = blockIdx.x;
  int n6 = d.np * (d.blk_cam_off[l + 1] - d.blk_cam_off[l]);
  int nt = d.nt[l];
  const int T = d.T;
  for (int r = threadIdx.x; r < T; r += NT) {
    int gr = (nt - 1) * T + r;
    if (gr >= n6) d.S[rcs_elem(d, l, gr, gr)] = 1.0;
  }
}

// point-major copies of the pixel coordinates and the weights (LM order ->
// intersection stream)
__global__ void k_gather_pm(Dev d) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= d.K) return;
  const int64_t k = d.pm_k[i];
  d.pm_xy[2 * i] = d.xy[2 * k];
  d.pm_xy[2 * i + 1] = d.xy[2 * k + 1];
  const double r = d.rw[k];
  if (d.has_info) {
    for (int q = 0; q < 3; ++q) d.pm_w[3 * i + q] = r * d.info[3 * k + q];
  } else {
    d.pm_code[i] = (d.pm_code[i] & ~(PM_DOWN | PM_DEL)) | (r != 1.0 ? PM_DOWN : 0) | (r == 0.0 ? PM_DEL : 0);
  }
}

// ------------------------------------------------------------ prior centre
// Centre of the tie-point prior of copy c of point p: the intersected point
// Xbar (the method and its ablations), or for the plain variants the
// consensus point minus the copy's dual offset, X_j - Xtilde_j^l (eq:admm7)
__device__ __forceinline__ void prior_centre(const Dev& d, int p, int64_t c, double (&xb)[3]) {
  if (d.Xt) {
    xb[0] = d.P0[p] - d.Xt[3 * c];
    xb[1] = d.P0[(int64_t)d.N + p] - d.Xt[3 * c + 1];
    xb[2] = d.P0[2 * (int64_t)d.N + p] - d.Xt[3 * c + 2];
  } else {
    xb[0] = d.Xbar[p];
    xb[1] = d.Xbar[(int64_t)d.N + p];
    xb[2] = d.Xbar[2 * (int64_t)d.N + p];
  }
}

// ------------------------------------------------------------ copy records
// The record of copy c for the Schur pass of the next LM step: X, the damped
// point block's inverse V*^-1 (zero if V* did not factorise), g_X, valid.
// FP64 path: 16 doubles (X, 1, V*^-1, g_X, spare).  Mixed path: X in FP64,
// then V*^-1, g_X and the valid flag rounded to FP32 (the precision that
// path's Schur pass computes in).
__device__ __forceinline__ void put_record(const Dev& d, int64_t c, const double (&X)[3], const double (&inv)[6],
                                           const double (&g)[3], bool ok) {
  if (d.cpk_f32) {
    uint32_t w[16];
    __builtin_memcpy(w, X, 24);
    float f[10];
    for (int q = 0; q < 6; ++q) f[q] = (float)inv[q];
    for (int q = 0; q < 3; ++q) f[6 + q] = ok ? (float)g[q] : 0.f;
    f[9] = 1.f;
    __builtin_memcpy(w + 6, f, 40);
    uint4* p4 = reinterpret_cast<uint4*>(d.cpk + CPK32 * c);
    for (int q = 0; q < 4; ++q) p4[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
  } else {
    double2* p2 = reinterpret_cast<double2*>(d.cpk + CPK * c);
    p2[0] = make_double2(X[0], X[1]);
    p2[1] = make_double2(X[2], 1.0);
    p2[2] = make_double2(inv[0], inv[1]);
    p2[3] = make_double2(inv[2], inv[3]);
    p2[4] = make_double2(inv[4], inv[5]);
    p2[5] = make_double2(ok ? g[0] : 0.0, ok ? g[1] : 0.0);
    p2[6] = make_double2(ok ? g[2] : 0.0, 0.0);
  }
}

// zero record: the Schur pass skips the copy
__device__ __forceinline__ void zero_record(const Dev& d, int64_t c) {
  if (d.cpk_f32) {
    uint4* p4 = reinterpret_cast<uint4*>(d.cpk + CPK32 * c);
    for (int q = 0; q < 4; ++q) p4[q] = make_uint4(0u, 0u, 0u, 0u);
  } else {
    double2* p2 = reinterpret_cast<double2*>(d.cpk + CPK * c);
    for (int q = 0; q < CPK / 2; ++q) p2[q] = make_double2(0.0, 0.0);
  }
}

// ------------------------------------------------------------ intersection
// One thread per point (internal order).  A workgroup's INT_WG consecutive
// points read their observations (point-major, copy by copy) and the cameras
// they see from LDS, where the workgroup stages them once: every
// Gauss-Newton pass then costs LDS traffic only (observations or cameras
// beyond the staging caps are read from memory).  Gauss-Newton with cameras
// fixed (eq:bars); on convergence: covariance, refined weights
// Omega^l = H - H^(l) of every copy (Sec. 5.1), residuals stored.
constexpr int IT = INT_WG;  // threads per intersection workgroup

// staged components of a camera: R, C, and with intrinsics its f and k1
constexpr int STAGE_CM = 14;
struct Stage {
  double cams[INT_CAM_CAP * STAGE_CM];  // component-major: component q of slot s at q * INT_CAM_CAP + s
  double2 xy[INT_OBS_CAP];
  int32_t code[INT_OBS_CAP];
};

// observation i of the stream, in two parts: its head (pixel, weight and
// code) and the camera the code names.  OLDS: the workgroup's observations
// are all staged (a workgroup-uniform choice, so the common path carries no
// per-lane test of where they live).  The camera is read from its LDS slot
// unconditionally; the rare camera beyond the staging cap is then replaced
// from memory in a branch of its own.
struct ObsHead {
  double x, y;
  W2<double> W;
  int32_t code;
};

template <bool INFO, bool OLDS>
__device__ __forceinline__ ObsHead obs_head(const Dev& d, const Stage& sg, int b0, int i) {
  ObsHead o;
  if (OLDS) {
    const double2 v = sg.xy[i - b0];
    o.x = v.x;
    o.y = v.y;
    o.code = sg.code[i - b0];
  } else {
    const double2 v = reinterpret_cast<const double2*>(d.pm_xy)[i];
    o.x = v.x;
    o.y = v.y;
    o.code = d.pm_code[i];
  }
  if (INFO) {
    const double* w = d.pm_w + 3 * (int64_t)i;
    o.W = {w[0], w[1], w[2]};
  } else {
    const double w = (o.code & PM_DOWN) ? ((o.code & PM_DEL) ? 0.0 : d.down_weight * d.w0) : d.w0;
    o.W = {w, 0.0, w};
  }
  return o;
}

// the camera of an observation code; CAL: with its f and k1 (intrinsics)
template <bool CAL>
__device__ __forceinline__ void obs_cam(const Dev& d, const Stage& sg, int32_t code, double (&cm)[CAL ? 14 : 12]) {
  constexpr int NQ = CAL ? 14 : 12;
  const int f = code & PM_FIELD;
  const bool glb = (code & PM_GLOBAL) != 0;
  const int sl = glb ? 0 : f;
#pragma unroll
  for (int q = 0; q < NQ; ++q) cm[q] = sg.cams[q * INT_CAM_CAP + sl];
  if (__builtin_expect(glb, 0)) {
    const double2* g = reinterpret_cast<const double2*>(d.cam + (int64_t)CAM_STRIDE * f);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double2 v = g[q];
      cm[2 * q] = v.x;
      cm[2 * q + 1] = v.y;
    }
    if constexpr (CAL) {
      const double2 fk = reinterpret_cast<const double2*>(d.intr)[f];
      cm[CAM_F] = fk.x;
      cm[CAM_K1] = fk.y;
    }
  }
}

template <bool INFO, bool OLDS, bool CAL>
__device__ __forceinline__ int32_t obs_get(const Dev& d, const Stage& sg, int b0, int i, double& x, double& y,
                                           W2<double>& W, double (&cm)[CAL ? 14 : 12]) {
  const ObsHead o = obs_head<INFO, OLDS>(d, sg, b0, i);
  x = o.x;
  y = o.y;
  W = o.W;
  obs_cam<CAL>(d, sg, o.code, cm);
  return o.code;
}

// per-workgroup sums of the copies' costs by sub-block (the cost before the
// next LM step of a fresh sub-block): a few LDS slots keyed by sub-block,
// flushed with one atomic each; a sub-block that finds no slot adds to memory
constexpr int CSLOT = 16;
struct CostSlots {
  int key[CSLOT];
  double sum[CSLOT];
};
__device__ __forceinline__ void cost_add(const Dev& d, CostSlots& cs, int l, double v) {
  for (int t = 0; t < CSLOT; ++t) {
    const int q = (l + t) & (CSLOT - 1);
    int k = cs.key[q];
    if (k == -1) k = atomicCAS(&cs.key[q], -1, l);
    if (k == -1 || k == l) {
      atomicAdd(&cs.sum[q], v);
      return;
    }
  }
  atomicAdd(&d.acc_int[4 + l], v);
}

// refined weight Omega of copy c (FP32 storage on the mixed path)
__device__ __forceinline__ void om_load(const Dev& d, int64_t c, double (&om)[6]) {
  if (d.om_f32) {
    const float2* f = reinterpret_cast<const float2*>(d.Omf + 6 * c);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float2 v = f[q];
      om[2 * q] = v.x;
      om[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 6; ++q) om[q] = d.Om[6 * c + q];
  }
}

// latest point of internal index j and its status, written whole so that
// the record lines fill completely (exported to the caller's order by
// k_export_pts)
__device__ __forceinline__ void put_pxs(const Dev& d, int j, const double (&X)[3], int st) {
  double2* p = reinterpret_cast<double2*>(d.pxs + 4 * (int64_t)j);
  p[0] = make_double2(X[0], X[1]);
  p[1] = make_double2(X[2], (double)st);
}

// one point: Gauss-Newton to convergence, then the final pass (covariance,
// residuals, refined weights of the copies); accv gets the point's share of
// the statistics
// VAR: the variant of the method (RPBA_VARIANT_*): the tie-point weights
// Omega of the copies, and for the plain variants an evaluation at the
// consensus point instead of Gauss-Newton (no copy records: their copies are
// never reset)
template <bool INFO, bool OLDS, int VAR, bool CAL>
__device__ __forceinline__ void intersect_point(const Dev& d, Stage& sg, CostSlots& cs, int b0, int j, int want_cov,
                                                double (&accv)[4]) {
  constexpr bool PLAIN = VAR >= RPBA_VARIANT_PLAIN;
  if (j < d.N && d.status[j] == 0) {
    const int c0 = d.pt_copy_off[j], c1 = d.pt_copy_off[j + 1], n = c1 - c0;
    const int i0 = d.pm_off[j], i1 = d.pm_off[j + 1];
    double X[3] = {d.P0[j], d.P0[(int64_t)d.N + j], d.P0[2 * (int64_t)d.N + j]};
    int st = PLAIN ? 0 : 1;  // not converged (the plain variants evaluate at the consensus point)
    double h[6], g[3], lch[6];
    for (int it = 0; !PLAIN && it < d.int_maxit; ++it) {
      for (int q = 0; q < 6; ++q) h[q] = 0.0;
      g[0] = g[1] = g[2] = 0.0;
      bool behind = false;
      // two observations per trip into independent sums (two independent
      // dependency chains for the scheduler), added at the end of the pass
      double h2[6] = {0, 0, 0, 0, 0, 0}, g2[3] = {0, 0, 0};
      int i = i0;
      // the heads of the next pair are read while this pair is computed
      // (indices clamped into the point's own range)
      ObsHead ha, hb;
      if (i0 < i1) {
        ha = obs_head<INFO, OLDS>(d, sg, b0, i0);
        hb = obs_head<INFO, OLDS>(d, sg, b0, min(i0 + 1, i1 - 1));
      }
      for (; i + 1 < i1; i += 2) {
        double cma[CAL ? 14 : 12], cmb[CAL ? 14 : 12];
        obs_cam<CAL>(d, sg, ha.code, cma);
        obs_cam<CAL>(d, sg, hb.code, cmb);
        const ObsHead na = obs_head<INFO, OLDS>(d, sg, b0, min(i + 2, i1 - 1));
        const ObsHead nb = obs_head<INFO, OLDS>(d, sg, b0, min(i + 3, i1 - 1));
        Lin<double> La, Lb;
        linearise_cam<CAL, double>(cma, cma + CAM_F, X, d.f, d.cx, d.cy, La);
        linearise_cam<CAL, double>(cmb, cmb + CAM_F, X, d.f, d.cx, d.cy, Lb);
        // a deleted observation (weight 0) neither counts nor fails the point
        if ((!(La.z > 0.0) && ha.W.a > 0.0) || (!(Lb.z > 0.0) && hb.W.a > 0.0)) behind = true;
        add_point_normals<double>(La, ha.W, La.g0 - ha.x, La.g1 - ha.y, h, g);
        add_point_normals<double>(Lb, hb.W, Lb.g0 - hb.x, Lb.g1 - hb.y, h2, g2);
        ha = na;
        hb = nb;
      }
      if (i < i1) {  // ha holds the head of observation i
        double cm[CAL ? 14 : 12];
        obs_cam<CAL>(d, sg, ha.code, cm);
        Lin<double> L;
        linearise_cam<CAL, double>(cm, cm + CAM_F, X, d.f, d.cx, d.cy, L);
        if (!(L.z > 0.0) && ha.W.a > 0.0) behind = true;
        add_point_normals<double>(L, ha.W, L.g0 - ha.x, L.g1 - ha.y, h, g);
      }
      for (int q = 0; q < 6; ++q) h[q] += h2[q];
      for (int q = 0; q < 3; ++q) g[q] += g2[q];
      if (behind) {
        st = 2;
        break;
      }
      if (!chol3(h, lch)) {
        st = 3;
        break;
      }
      double mg[3] = {-g[0], -g[1], -g[2]}, dX[3];
      chol3_solve(lch, mg, dX);
      X[0] += dX[0];
      X[1] += dX[1];
      X[2] += dX[2];
      double nd = sqrt(dX[0] * dX[0] + dX[1] * dX[1] + dX[2] * dX[2]);
      double nx2 = sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
      if (nd <= d.int_tol * (1.0 + nx2)) {
        st = 0;
        break;
      }
    }
    // final pass at the converged point, two sweeps over the point's
    // observations.  The first forms the normals H (summed copy by copy), the
    // residuals, the cost and the statistics.  Once H is complete, the second
    // forms each copy's normals H^(l), gradient g^(l) and cost again and
    // finishes the copy at its last observation: refined weight, record and
    // cost.  Forming the copies' sums again costs less than keeping them in
    // memory until H is known.
    double cost = 0.0, sq = 0.0, nobs = 0.0;
    double vmax = 0.0;  // largest squared reprojection error (filters)
    if (st == 0) {
      for (int q = 0; q < 6; ++q) h[q] = 0.0;
      double hl[6] = {0, 0, 0, 0, 0, 0}, gd[3] = {0, 0, 0};
      bool behind = false;
      for (int i = i0; i < i1; ++i) {
        double x, y, cm[CAL ? 14 : 12];
        W2<double> W;
        const int32_t code = obs_get<INFO, OLDS, CAL>(d, sg, b0, i, x, y, W, cm);
        Lin<double> L;
        linearise_cam<CAL, double>(cm, cm + CAM_F, X, d.f, d.cx, d.cy, L);
        const bool live = W.a > 0.0;  // not deleted by the robust step
        if (!(L.z > 0.0) && live) behind = true;
        const double v0 = L.g0 - x, v1 = L.g1 - y;
        add_point_normals<double>(L, W, v0, v1, hl, gd);
        // the residual takes the place of the pixel in LDS (the second sweep
        // reads it there, and the workgroup copies them out coalesced)
        if (OLDS) sg.xy[i - b0] = make_double2(v0, v1);
        else if (d.res) reinterpret_cast<double2*>(d.res)[i] = make_double2(v0, v1);
        cost += wquad(W, v0, v1);
        if (PLAIN && live) vmax = fmax(vmax, v0 * v0 + v1 * v1);
        if (live) {
          sq += v0 * v0 + v1 * v1;
          nobs += 1.0;
        }
        if (code & PM_LAST) {  // a copy complete: its normals join H
          for (int q = 0; q < 6; ++q) {
            h[q] += hl[q];
            hl[q] = 0.0;
          }
        }
      }
      if (behind) st = 2;
      else if (!chol3(h, lch)) st = 3;
      // filters of the plain variants (Sec. 6.3): very far points, and points
      // with a reprojection error above filter_px
      else if (PLAIN && (!(X[0] * X[0] + X[1] * X[1] + X[2] * X[2] <= 1e20) || vmax > d.filter_px * d.filter_px))
        st = 5;
    }
    double inv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (st == 0) {
      chol3_inverse(lch, inv);
      for (int r = 0; r < 3; ++r) {
        d.Xbar[(int64_t)r * d.N + j] = X[r];
        d.P0[(int64_t)r * d.N + j] = X[r];
      }
      const double rho = (VAR == RPBA_VARIANT_SCALAR || VAR == RPBA_VARIANT_PLAIN) ? *d.rho_t : 0.0;
      // Every copy restarts at Xbar with the same cameras, so the point block
      // of its sub-block, sum_(k in l) B^T W B + Omega^l = H^(l) + (H - H^(l)),
      // is H itself: the damped V* = H + lambda diag(H) and its inverse are
      // the same for every copy, and each copy's record gets its own g^(l).
      double hv[6] = {h[0] * (1.0 + d.lambda), h[1], h[2], h[3] * (1.0 + d.lambda), h[4], h[5] * (1.0 + d.lambda)};
      double lv[6], vi[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      bool vok = false;
      if (VAR == RPBA_VARIANT_EXTENDED) {
        vok = chol3(hv, lv);
        if (vok) chol3_inverse(lv, vi);
      }
      // second sweep: copy by copy; the copies are reset to Xbar through the
      // sub-blocks' fresh flags
      double hu[6] = {0, 0, 0, 0, 0, 0}, g3[3] = {0, 0, 0}, cc = 0.0;  // H^(l), g^(l), cost of the copy
      int u2 = 0;
      int64_t c = n > 0 ? d.pt_copies[c0] : 0;
      int lc = n > 0 ? d.copy_blk[c] : 0;
      for (int i = i0; i < i1; ++i) {
        const ObsHead o = obs_head<INFO, OLDS>(d, sg, b0, i);  // staged: (x, y) is the residual
        double cm[CAL ? 14 : 12];
        obs_cam<CAL>(d, sg, o.code, cm);
        Lin<double> L;
        linearise_cam<CAL, double>(cm, cm + CAM_F, X, d.f, d.cx, d.cy, L);
        const double v0 = OLDS ? o.x : L.g0 - o.x, v1 = OLDS ? o.y : L.g1 - o.y;
        add_point_normals<double>(L, o.W, v0, v1, hu, g3);
        cc += wquad(o.W, v0, v1);
        if (o.code & PM_LAST) {
          // Omega of a tie-point copy: information from the cameras outside l
          // (EXTENDED, PLAIN_REFINED), from all cameras (ALL_CAMERAS), or
          // rho_t I (SCALAR, PLAIN); zero for a point seen by one sub-block only
          double o6[6];
          for (int q = 0; q < 6; ++q) {
            const double sc = (q == 0 || q == 3 || q == 5) ? rho : 0.0;
            o6[q] = n == 1 ? 0.0
                    : (VAR == RPBA_VARIANT_EXTENDED || VAR == RPBA_VARIANT_PLAIN_REFINED) ? h[q] - hu[q]
                    : VAR == RPBA_VARIANT_ALL_CAMERAS ? h[q]
                                                      : sc;
          }
          if (d.om_f32) {
            float2* om = reinterpret_cast<float2*>(d.Omf + 6 * c);
            om[0] = make_float2((float)o6[0], (float)o6[1]);
            om[1] = make_float2((float)o6[2], (float)o6[3]);
            om[2] = make_float2((float)o6[4], (float)o6[5]);
          } else {
            double2* om = reinterpret_cast<double2*>(d.Om + 6 * c);
            om[0] = make_double2(o6[0], o6[1]);
            om[1] = make_double2(o6[2], o6[3]);
            om[2] = make_double2(o6[4], o6[5]);
          }
          if (!PLAIN) {
            if (VAR == RPBA_VARIANT_EXTENDED) {
              put_record(d, c, X, vi, g3, vok);
            } else {
              // the copy's own point block H^(l) + Omega^l, damped
              double hv2[6], lv2[6], vi2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
              for (int q = 0; q < 6; ++q) hv2[q] = hu[q] + o6[q];
              hv2[0] *= 1.0 + d.lambda;
              hv2[3] *= 1.0 + d.lambda;
              hv2[5] *= 1.0 + d.lambda;
              const bool ok2 = chol3(hv2, lv2);
              if (ok2) chol3_inverse(lv2, vi2);
              put_record(d, c, X, vi2, g3, ok2);
            }
            cost_add(d, cs, lc, cc);
          }
          for (int q = 0; q < 6; ++q) hu[q] = 0.0;
          for (int q = 0; q < 3; ++q) g3[q] = 0.0;
          cc = 0.0;
          if (++u2 < n) {
            c = d.pt_copies[c0 + u2];
            lc = d.copy_blk[c];
          }
        }
      }
      accv[0] = cost;
      accv[1] = sq;
      accv[2] = nobs;
      accv[3] = 1.0;
    } else if (!PLAIN) {
      // a point that fails here: its copies drop out of the Schur pass (a
      // point needs a degenerate geometry to fail after converging)
      for (int u2 = 0; u2 < n; ++u2) zero_record(d, d.pt_copies[c0 + u2]);
    }
    d.status[j] = st;
    put_pxs(d, j, X, st);
    if (want_cov) {
      double2* cv = reinterpret_cast<double2*>(d.covi + 6 * (int64_t)j);
      cv[0] = make_double2(inv[0], inv[1]);
      cv[1] = make_double2(inv[2], inv[3]);
      cv[2] = make_double2(inv[4], inv[5]);
    }
  } else if (j < d.N) {
    const double z[3] = {0.0, 0.0, 0.0};
    put_pxs(d, j, z, d.status[j]);
    // a point left out before (failed or eliminated): no copy of it in the
    // Schur pass
    if (!PLAIN)
      for (int c = d.pt_copy_off[j]; c < d.pt_copy_off[j + 1]; ++c) zero_record(d, d.pt_copies[c]);
  }
}

template <bool INFO, int VAR, bool CAL>
__global__ __launch_bounds__(IT) void k_intersect(Dev d, int want_cov) {
  __shared__ Stage sg;
  __shared__ double sh[4 * (IT / 64)];
  __shared__ CostSlots cs;
  if (blockIdx.x == 0) {
    // the copies restart at Xbar (their records written below); the plain
    // variants keep their copies where the sub-blocks left them
    if (VAR < RPBA_VARIANT_PLAIN)
      for (int l = threadIdx.x; l < d.L; l += IT) d.blk_fresh[l] = 1;
    // (with adaptive damping every sub-block has its own lambda: the point
    // blocks are rebuilt by the point-block pass instead)
    if (threadIdx.x == 0) *d.rec_valid = VAR < RPBA_VARIANT_PLAIN && !d.lam_blk ? 1 : 0;
  }
  if (threadIdx.x < CSLOT) {
    cs.key[threadIdx.x] = -1;
    cs.sum[threadIdx.x] = 0.0;
  }
  const int j0 = blockIdx.x * IT;
  const int b0 = d.pm_off[j0];
  const int nobs = d.pm_off[min(j0 + IT, d.N)] - b0;
  const int nst = min(nobs, INT_OBS_CAP);
  {
    // every load of the staging is issued before the first LDS write (one
    // round of memory latency for the indices, one for the data): each
    // thread owns whole camera slots and a fixed set of observations
    constexpr int CS = (INT_CAM_CAP + IT - 1) / IT, OS = (INT_OBS_CAP + IT - 1) / IT;
    const int cb = d.iwg_cam_off[blockIdx.x], nc = d.iwg_cam_off[blockIdx.x + 1] - cb;
    int ci[CS];
#pragma unroll
    for (int u = 0; u < CS; ++u) {
      const int sl = threadIdx.x + u * IT;
      ci[u] = sl < nc ? d.iwg_cams[cb + sl] : -1;
    }
    // unconditional loads at clamped indices (in range: every workgroup has
    // observations, since every point has at least two), stores guarded; no
    // array is filled under a condition, so all of them stay in registers
    const double2* gxy = reinterpret_cast<const double2*>(d.pm_xy) + b0;
    double2 ov[OS];
    int32_t oc[OS];
#pragma unroll
    for (int u = 0; u < OS; ++u) {
      const int t = max(0, min((int)threadIdx.x + u * IT, nst - 1));
      ov[u] = gxy[t];
      oc[u] = d.pm_code[b0 + t];
    }
    constexpr int NQ2 = CAL ? 7 : 6;  // double2 per staged camera (with intrinsics its f and k1 last)
    double2 cv[CS][NQ2];
#pragma unroll
    for (int u = 0; u < CS; ++u) {
      const double2* g = reinterpret_cast<const double2*>(d.cam + (int64_t)CAM_STRIDE * max(ci[u], 0));
#pragma unroll
      for (int q = 0; q < 6; ++q) cv[u][q] = g[q];
      if constexpr (CAL) cv[u][NQ2 - 1] = reinterpret_cast<const double2*>(d.intr)[max(ci[u], 0)];
    }
#pragma unroll
    for (int u = 0; u < OS; ++u) {
      const int t = threadIdx.x + u * IT;
      if (t < nst) {
        sg.xy[t] = ov[u];
        sg.code[t] = oc[u];
      }
    }
#pragma unroll
    for (int u = 0; u < CS; ++u)
      if (ci[u] >= 0) {
        const int sl = threadIdx.x + u * IT;
#pragma unroll
        for (int q = 0; q < NQ2; ++q) {
          sg.cams[(2 * q) * INT_CAM_CAP + sl] = cv[u][q].x;
          sg.cams[(2 * q + 1) * INT_CAM_CAP + sl] = cv[u][q].y;
        }
      }
  }
  __syncthreads();
  const int j = j0 + threadIdx.x;
  double accv[4] = {0.0, 0.0, 0.0, 0.0};
  if (nobs <= INT_OBS_CAP) {
    intersect_point<INFO, true, VAR, CAL>(d, sg, cs, b0, j, want_cov, accv);
    // residuals of the workgroup's stream, one coalesced copy (the slots of
    // points left invalid hold their pixels: residuals are only read for
    // valid points), as streaming stores: only a robust re-weighting reads
    // them, long after
    __syncthreads();
    double2* res = reinterpret_cast<double2*>(d.res) + b0;
    for (int t = threadIdx.x; d.res && t < nobs; t += IT) {
      const double2 v = sg.xy[t];
      __builtin_nontemporal_store(v.x, &res[t].x);
      __builtin_nontemporal_store(v.y, &res[t].y);
    }
  } else {
    intersect_point<INFO, false, VAR, CAL>(d, sg, cs, b0, j, want_cov, accv);
  }
  // workgroup sum of the statistics, one partial per value (k_int_reduce
  // adds them up: atomics of every workgroup on the same four words would
  // queue up in the cache)
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) accv[q] += __shfl_xor(accv[q], o);
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; ++q) sh[q * (IT / 64) + (threadIdx.x >> 6)] = accv[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < IT / 64; ++w) v += sh[threadIdx.x * (IT / 64) + w];
    d.int_part[4 * (int64_t)blockIdx.x + threadIdx.x] = v;
  }
  if (threadIdx.x < CSLOT && cs.key[threadIdx.x] >= 0)
    atomicAdd(&d.acc_int[4 + cs.key[threadIdx.x]], cs.sum[threadIdx.x]);
}

// statistics of an intersection from its sums: cost, sigma0 (redundancy
// 2 K_valid - 6 M - 3 N_valid), RMS reprojection error, valid points
__device__ void intersect_stats(const Dev& d, double* stats) {
  double cost = d.acc_int[0], sq = d.acc_int[1], kv = d.acc_int[2], nv = d.acc_int[3];
  double red = 2.0 * kv - (double)d.np * d.M - 3.0 * nv;
  stats[0] = cost;
  stats[1] = red > 0 ? sqrt(sq / red) : 0.0;
  stats[2] = kv > 0 ? sqrt(sq / (2.0 * kv)) : 0.0;
  stats[3] = nv;
}

// Caller-order export: one thread per caller point o gathers the internal
// record of its point, so that the caller's arrays are written line by line
// (points and covariances of invalid points are left as they were)
__global__ __launch_bounds__(NT) void k_export_pts(Dev d, double* cov, int32_t* status_out, double* stats) {
  const int o = blockIdx.x * NT + threadIdx.x;
  if (stats && o == 0) intersect_stats(d, stats);  // the intersection's sums are complete
  if (o >= d.N) return;
  const int j = d.pt_new[o];
  // both gathers issued together; the caller's arrays are written with
  // streaming stores (nothing in the library reads them back)
  const double2* p = reinterpret_cast<const double2*>(d.pxs + 4 * (int64_t)j);
  const double2 a = p[0], b = p[1];
  double2 c0, c1, c2;
  if (cov) {
    const double2* c = reinterpret_cast<const double2*>(d.covi + 6 * (int64_t)j);
    c0 = c[0];
    c1 = c[1];
    c2 = c[2];
  }
  const int st = (int)b.y;
  if (status_out) __builtin_nontemporal_store(st, status_out + o);
  if (st != 0) return;
  __builtin_nontemporal_store(a.x, d.u_pts + o);
  __builtin_nontemporal_store(a.y, d.u_pts + (int64_t)d.N + o);
  __builtin_nontemporal_store(b.x, d.u_pts + 2 * (int64_t)d.N + o);
  if (cov) {
    __builtin_nontemporal_store(c0.x, cov + o);
    __builtin_nontemporal_store(c0.y, cov + (int64_t)d.N + o);
    __builtin_nontemporal_store(c1.x, cov + 2 * (int64_t)d.N + o);
    __builtin_nontemporal_store(c1.y, cov + 3 * (int64_t)d.N + o);
    __builtin_nontemporal_store(c2.x, cov + 4 * (int64_t)d.N + o);
    __builtin_nontemporal_store(c2.y, cov + 5 * (int64_t)d.N + o);
  }
}

// ------------------------------------------------ sub-block normal equations
// One thread per copy: damped point block V* = (sum B^T W B + Omega)(1 + lambda
// on the diagonal), its FP64 inverse, g_X = sum B^T W v + Omega (X - Xbar),
// and the cost before the step.  Packs (X, V*^-1, g_X) for the Schur pass.
// Copies of fresh sub-blocks are skipped while the intersection's records
// are valid (it wrote them at this very state); so are whole workgroups.
// J: arithmetic of the Jacobians and of the per-observation products (FP32
// on the mixed path, with the projection, the residual and the cost in FP64
// and the sums added to the FP64 prior before the FP64 inverse).
template <typename J, bool CAL>
__global__ __launch_bounds__(NT) void k_copy_prep(Dev d) {
  __shared__ double sh[8];
  __shared__ int l_first, s_skip;
  const bool unit = *d.rw_unit != 0;
  const bool recs = *d.rec_valid != 0;
  int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (threadIdx.x == 0) {
    l_first = d.copy_blk[blockIdx.x * (int64_t)NT];
    const int l_last = d.copy_blk[min((int64_t)blockIdx.x * NT + NT, d.NC) - 1];
    int skip = recs ? 1 : 0;
    for (int l = l_first; skip && l <= l_last; ++l) skip = d.blk_fresh[l];
    s_skip = skip;
    for (int q = 0; q < 8; ++q) sh[q] = 0.0;
  }
  __syncthreads();
  // a skipped workgroup holds copies of fresh sub-blocks only, whose sums
  // the reduction does not read: its slots are left as they are
  if (s_skip) return;
  if (c < d.NC && !(recs && d.blk_fresh[d.copy_blk[c]])) {
    // the copy's indices, flags and point are loaded together, ahead of the
    // tests that use them (the copy's own data stays behind them: holding it
    // across the tests costs more occupancy than it saves here)
    const int l = d.copy_blk[c], p = d.copy_pt[c];
    const int k0 = d.copy_off[c], k1 = d.copy_off[c + 1];
    const bool act = d.active == nullptr || d.active[l];
    const int stp = d.status[p], fresh = d.blk_fresh[l];
    double xb[3];
    prior_centre(d, p, c, xb);
    if (act && stp == 0) {
      double X[3] = {xb[0], xb[1], xb[2]};
      if (!fresh)
        for (int r = 0; r < 3; ++r) X[r] = d.Xc[3 * c + r];
      double om[6];
      om_load(d, c, om);
      double dx[3] = {X[0] - xb[0], X[1] - xb[1], X[2] - xb[2]};
      double gp[3];
      sym3_mul(om, dx, gp);
      double cost = dx[0] * gp[0] + dx[1] * gp[1] + dx[2] * gp[2];
      // in FP64 the sums start from the prior (the oracle's order); in FP32
      // they start from zero and the prior is added in FP64
      J hj[6], gj[3];
      for (int q = 0; q < 6; ++q) hj[q] = sizeof(J) == 8 ? (J)om[q] : J(0);
      for (int q = 0; q < 3; ++q) gj[q] = sizeof(J) == 8 ? (J)gp[q] : J(0);
      for (int k = k0; k < k1; ++k) {
        const int ic = d.obs_cam[k];
        const double* cm = d.cam + (int64_t)CAM_STRIDE * ic;
        Lin<J> L;
        double g0, g1, z;
        linearise_split_cam<CAL, J>(cm, CAL ? d.intr + 2 * (int64_t)ic : nullptr, X, d.f, d.cx, d.cy, L, g0, g1, z);
        const double v0 = g0 - d.xy[2 * k], v1 = g1 - d.xy[2 * k + 1];
        const W2<double> W = obs_weight(d, k, unit);
        add_point_normals<J>(L, W2<J>{(J)W.a, (J)W.b, (J)W.c}, (J)v0, (J)v1, hj, gj);
        cost += wquad(W, v0, v1);
      }
      double h[6], g[3];
      for (int q = 0; q < 6; ++q) h[q] = sizeof(J) == 8 ? (double)hj[q] : om[q] + (double)hj[q];
      for (int q = 0; q < 3; ++q) g[q] = sizeof(J) == 8 ? (double)gj[q] : gp[q] + (double)gj[q];
      const double lam = lam_of(d, l);
      h[0] *= 1.0 + lam;
      h[3] *= 1.0 + lam;
      h[5] *= 1.0 + lam;
      double lch[6], inv[6];
      bool ok = chol3(h, lch);
      if (ok) chol3_inverse(lch, inv);
      else
        for (int q = 0; q < 6; ++q) inv[q] = 0.0;
      put_record(d, c, X, inv, g, ok);
      int slot = l - l_first;
      if (slot >= 0 && slot < 8) atomicAdd(&sh[slot], cost);
      else atomicAdd(&d.acc_blk[4 * l + 0], cost);
    } else {
      zero_record(d, c);  // the Schur pass skips the copy
    }
  }
  __syncthreads();
  // the workgroup's sums per slot, added up per sub-block by k_slots_reduce
  if (threadIdx.x < 8) d.upd_part[16 * (int64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x];
}

// start of an LM step: per sub-block the statistics (cost before from the
// intersection for a fresh sub-block whose records are valid, else summed by
// the point-block pass) and the failure flags
__global__ void k_step_begin(Dev d) {
  const int l = blockIdx.x * NT + threadIdx.x;
  if (l >= d.L) return;
  const bool fresh = *d.rec_valid != 0 && d.blk_fresh[l] != 0;
  double* a = d.acc_blk + 4 * l;
  a[0] = fresh ? d.acc_int[4 + l] : 0.0;
  a[1] = 0.0;
  a[2] = 0.0;
  a[3] = 0.0;
  d.blk_fail[l] = 0;
  d.blk_nc[l] = 0;
}

// ------------------------------------------------------- update of the step
// One thread per camera: new pose R <- Exp([w]x) R, C <- C + dc into camN.
__global__ void k_cam_update(Dev d) {
  const int i = blockIdx.x * NT + threadIdx.x;
  int l = -1;
  double s2 = 0.0;
  if (i < d.M) {
    l = d.cam_blk[i];
    const double* c = d.cam + (int64_t)CAM_STRIDE * i;
    double* n = d.camN + (int64_t)CAM_STRIDE * i;
    const bool act = (d.active == nullptr || d.active[l]) && d.blk_fail[l] == 0;
    if (!act) {
      for (int q = 0; q < CAM_STRIDE; ++q) n[q] = c[q];
      if (d.intr) {
        d.intrN[2 * (int64_t)i] = d.intr[2 * (int64_t)i];
        d.intrN[2 * (int64_t)i + 1] = d.intr[2 * (int64_t)i + 1];
      }
    } else {
      const int a = i - d.blk_cam_off[l];
      const double* dx = d.x + d.vec_off[l] + d.np * a;
      double w[3] = {dx[0], dx[1], dx[2]};
      rotate_left(w, c, n);
      for (int r = 0; r < 3; ++r) n[9 + r] = c[9 + r] + dx[3 + r];
      for (int q = 0; q < 6; ++q) s2 += dx[q] * dx[q];
      // intrinsics: f and k1 updated additively
      if (d.intr) {
        d.intrN[2 * (int64_t)i] = d.intr[2 * (int64_t)i] + dx[6];
        d.intrN[2 * (int64_t)i + 1] = d.intr[2 * (int64_t)i + 1] + dx[7];
        s2 += dx[6] * dx[6] + dx[7] * dx[7];
      }
    }
  }
  // the cameras of a sub-block are consecutive: a wave inside one sub-block
  // sums its squares first and adds them with one atomic
  const int l0 = __shfl(l, 0);
  if (__all(l == l0)) {
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
    if ((threadIdx.x & 63) == 0 && l0 >= 0 && s2 != 0.0) atomicAdd(&d.acc_blk[4 * l0 + 2], s2);
  } else if (l >= 0 && s2 != 0.0) {
    atomicAdd(&d.acc_blk[4 * l + 2], s2);
  }
}

// One thread per copy: dX = V*^-1 (-g_X - sum_k Y_k^T dC_i(k)) with Y_k at the
// old cameras, X^l += dX, and the cost after the step at the new cameras.
// J: arithmetic of the Jacobians and per-observation products of the first
// pass (FP32 on the mixed path; residuals, the 3x3 solve, the point and the
// cost after the step stay FP64).
template <typename J, bool CAL>
__global__ __launch_bounds__(NT) void k_back_update(Dev d) {
  __shared__ double sh[16];
  __shared__ int l_first;
  const bool unit = *d.rw_unit != 0;
  int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (threadIdx.x == 0) {
    l_first = d.copy_blk[blockIdx.x * (int64_t)NT];
    for (int q = 0; q < 16; ++q) sh[q] = 0.0;
  }
  __syncthreads();
  if (c < d.NC) {
    // the copy's inputs are loaded together, ahead of the tests that use them
    const int l = d.copy_blk[c], p = d.copy_pt[c];
    const int k0 = d.copy_off[c], k1 = d.copy_off[c + 1];
    const bool act = (d.active == nullptr || d.active[l]) && d.blk_fail[l] == 0;
    const int stp = d.status[p], fresh = d.blk_fresh[l];
    double xb[3];
    prior_centre(d, p, c, xb);
    const double xc[3] = {d.Xc[3 * c], d.Xc[3 * c + 1], d.Xc[3 * c + 2]};
    double om[6];
    om_load(d, c, om);
    if (act && stp == 0) {
      // the point block V* and g_X are rebuilt from the same linearisation
      // that forms Y^T dC (as in the point-block pass: no stored inverse is
      // read back), then V* dX = -g_X - sum_k Y_k^T dC_i(k)
      double X[3] = {xb[0], xb[1], xb[2]};
      if (!fresh)
        for (int r = 0; r < 3; ++r) X[r] = xc[r];
      double dx0[3] = {X[0] - xb[0], X[1] - xb[1], X[2] - xb[2]};
      double gp[3];
      sym3_mul(om, dx0, gp);
      // in FP64 the sums start from the prior (the oracle's order); in FP32
      // they start from zero and the prior is added in FP64
      J hj[6], gj[3], bt[3] = {J(0), J(0), J(0)};
      for (int q = 0; q < 6; ++q) hj[q] = sizeof(J) == 8 ? (J)om[q] : J(0);
      for (int q = 0; q < 3; ++q) gj[q] = sizeof(J) == 8 ? (J)gp[q] : J(0);
      const int base = d.blk_cam_off[l];
      const double* xs = d.x + d.vec_off[l];
      constexpr int NP = CAL ? 8 : 6;
      for_copy_obs<CAL>(d, d.cam, d.intr, k0, k1, unit, [&](const CopyObs<CAL>& o) {
        Lin<J> L;
        double g0, g1, z;
        linearise_split_cam<CAL, J>(o.cm, o.cm + CAM_F, X, d.f, d.cx, d.cy, L, g0, g1, z);
        const W2<J> W{(J)o.W.a, (J)o.W.b, (J)o.W.c};
        add_point_normals<J>(L, W, (J)(g0 - o.x), (J)(g1 - o.y), hj, gj);
        const double* dCd = xs + NP * (o.cam - base);
        J dC[NP];
        for (int q = 0; q < NP; ++q) dC[q] = (J)dCd[q];
        // t = A dC = Ar w - B dc (+ Ai (df, dk1)) ; Y^T dC = B^T W t
        J t0 = L.Ar[0][0] * dC[0] + L.Ar[0][1] * dC[1] + L.Ar[0][2] * dC[2] -
               (L.B[0][0] * dC[3] + L.B[0][1] * dC[4] + L.B[0][2] * dC[5]);
        J t1 = L.Ar[1][0] * dC[0] + L.Ar[1][1] * dC[1] + L.Ar[1][2] * dC[2] -
               (L.B[1][0] * dC[3] + L.B[1][1] * dC[4] + L.B[1][2] * dC[5]);
        if constexpr (CAL) {
          t0 += L.Ai[0][0] * dC[6] + L.Ai[0][1] * dC[7];
          t1 += L.Ai[1][0] * dC[6] + L.Ai[1][1] * dC[7];
        }
        J wt0 = W.a * t0 + W.b * t1, wt1 = W.b * t0 + W.c * t1;
        for (int s = 0; s < 3; ++s) bt[s] += L.B[0][s] * wt0 + L.B[1][s] * wt1;
      });
      double h[6], g[3];
      for (int q = 0; q < 6; ++q) h[q] = sizeof(J) == 8 ? (double)hj[q] : om[q] + (double)hj[q];
      for (int q = 0; q < 3; ++q) g[q] = sizeof(J) == 8 ? (double)gj[q] : gp[q] + (double)gj[q];
      const double lam = lam_of(d, l);
      h[0] *= 1.0 + lam;
      h[3] *= 1.0 + lam;
      h[5] *= 1.0 + lam;
      double lch[6], dX[3] = {0.0, 0.0, 0.0};
      if (chol3(h, lch)) {
        double rhs[3] = {-g[0] - (double)bt[0], -g[1] - (double)bt[1], -g[2] - (double)bt[2]};
        chol3_solve(lch, rhs, dX);
      }
      double Xn[3] = {X[0] + dX[0], X[1] + dX[1], X[2] + dX[2]};
      if (d.XcOld)  // adaptive damping: the copy before the step, to take it back
        for (int r = 0; r < 3; ++r) d.XcOld[3 * c + r] = X[r];
      d.Xc[3 * c] = Xn[0];
      d.Xc[3 * c + 1] = Xn[1];
      d.Xc[3 * c + 2] = Xn[2];
      double dx[3] = {Xn[0] - xb[0], Xn[1] - xb[1], Xn[2] - xb[2]};
      double og[3];
      sym3_mul(om, dx, og);
      double cost = dx[0] * og[0] + dx[1] * og[1] + dx[2] * og[2];
      for_copy_obs<CAL>(d, d.camN, d.intrN, k0, k1, unit, [&](const CopyObs<CAL>& o) {
        Lin<double> L;
        linearise_cam<CAL, double>(o.cm, o.cm + CAM_F, Xn, d.f, d.cx, d.cy, L);
        cost += wquad(o.W, L.g0 - o.x, L.g1 - o.y);
      });
      double s2 = dX[0] * dX[0] + dX[1] * dX[1] + dX[2] * dX[2];
      int slot = l - l_first;
      if (slot >= 0 && slot < 8) {
        atomicAdd(&sh[slot], cost);
        atomicAdd(&sh[8 + slot], s2);
      } else {
        atomicAdd(&d.acc_blk[4 * l + 1], cost);
        atomicAdd(&d.acc_blk[4 * l + 2], s2);
      }
    }
  }
  __syncthreads();
  // the workgroup's sums per slot, added up per sub-block by k_slots_reduce
  // (atomics of the many workgroups of one sub-block on its two words would
  // queue up in the cache)
  if (threadIdx.x < 16) d.upd_part[16 * (int64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x];
}

// per sub-block sums of the copy passes' slots: the cost before the step
// (point-block pass, UPD false) or the cost after it and the squared step of
// the copies (update pass, UPD true), from the slots of the workgroups that
// hold the sub-block's copies (one workgroup per sub-block, threads over
// those workgroups); added to what is already there (the camera steps' squares,
// the cost before of fresh sub-blocks, and the rare overflow adds)
template <bool UPD>
__global__ __launch_bounds__(NT) void k_slots_reduce(Dev d) {
  __shared__ double sh[2 * (NT / 64)];
  const int l = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the point-block pass skipped every copy of a fresh sub-block whose
  // records the intersection wrote: nothing to add (uniform over the workgroup)
  if (!UPD && *d.rec_valid != 0 && d.blk_fresh[l]) return;
  const int64_t c0 = d.blk_copy_off[l], c1 = d.blk_copy_off[l + 1];
  double a = 0.0, b = 0.0;
  if (c1 > c0) {
    // one workgroup per sub-block, U workgroups' slots per thread in flight
    constexpr int U = 4;
    const int64_t w0 = c0 / NT, w1 = (c1 - 1) / NT;
    for (int64_t wb = w0 + threadIdx.x; wb <= w1; wb += U * NT) {
      int slot[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t w = wb + u * NT;
        slot[u] = w <= w1 ? l - d.copy_blk[w * NT] : -1;
      }
      double va[U], vb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t w = wb + u * NT;
        const bool in = slot[u] >= 0 && slot[u] < 8;
        va[u] = in ? d.upd_part[16 * w + slot[u]] : 0.0;
        vb[u] = UPD && in ? d.upd_part[16 * w + 8 + slot[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a += va[u];
        b += vb[u];
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    if (UPD) b += __shfl_xor(b, o);
  }
  if (lane == 0) {
    sh[wv] = a;
    sh[NT / 64 + wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      sa += sh[w];
      sb += sh[NT / 64 + w];
    }
    if (UPD) {
      d.acc_blk[4 * l + 1] += sa;
      d.acc_blk[4 * l + 2] += sb;
    } else {
      d.acc_blk[4 * l + 0] += sa;
    }
  }
}

// adaptive damping: a step that raised its sub-block's cost, or could not
// be factorised, is taken back (cameras not committed, copies restored by
// k_restore_copies) and the sub-block's lambda grows by lam_up; an accepted
// step divides it by lam_down (within [lam_min, lam_max])
__device__ __forceinline__ bool step_rejected(const Dev& d, int l) {
  const double* a = d.acc_blk + 4 * l;
  return d.lam_blk && (d.active == nullptr || d.active[l]) && (d.blk_fail[l] != 0 || a[1] > a[0]);
}

// after the update: the new cameras become the current ones (those of an
// accepted step), and the per-sub-block statistics of the step are written
// out
__global__ void k_update_finish(Dev d, double* bs) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t < (int64_t)CAM_STRIDE * d.M && !step_rejected(d, d.cam_blk[t / CAM_STRIDE])) d.cam[t] = d.camN[t];
  if (d.intr && t < 2 * (int64_t)d.M && !step_rejected(d, d.cam_blk[t / 2])) d.intr[t] = d.intrN[t];
  if (t >= d.L) return;
  const int l = (int)t;
  bool act = d.active == nullptr || d.active[l];
  const double* a = d.acc_blk + 4 * l;
  const bool rej = step_rejected(d, l);
  if (act && d.blk_fail[l] == 0 && !rej) d.blk_fresh[l] = 0;  // its copies were written by the update
  if (d.lam_blk && act) {
    d.blk_rej[l] = rej ? 1 : 0;
    d.lam_blk[l] = rej ? fmin(d.lam_blk[l] * d.lam_up, d.lam_max) : fmax(d.lam_blk[l] / d.lam_down, d.lam_min);
  }
  if (bs) {
    bs[4 * l + 0] = act ? a[0] : 0.0;
    bs[4 * l + 1] = act ? (d.blk_fail[l] || rej ? a[0] : a[1]) : 0.0;
    bs[4 * l + 2] = act && !rej ? sqrt(a[2]) : 0.0;
    bs[4 * l + 3] = act ? (d.blk_fail[l] ? -1.0 : (a[3] > 0 ? a[3] : 1.0)) : 0.0;
  }
}

// adaptive damping: copies of a sub-block whose step was taken back return
// to where they were before it
__global__ void k_restore_copies(Dev d) {
  const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (c >= d.NC) return;
  const int l = d.copy_blk[c];
  if ((d.active == nullptr || d.active[l]) && d.blk_rej[l] && d.blk_fail[l] == 0 && d.status[d.copy_pt[c]] == 0)
    for (int r = 0; r < 3; ++r) d.Xc[3 * c + r] = d.XcOld[3 * c + r];
}

// --------------------------------------------------------------- consensus
__global__ __launch_bounds__(NT) void k_consensus_pts(Dev d) {
  __shared__ double sh[8];
  int j = blockIdx.x * NT + threadIdx.x;
  double dmax = 0.0, ntp = 0.0;
  if (j < d.N) {
    int c0 = d.pt_copy_off[j], c1 = d.pt_copy_off[j + 1];
    if (c1 - c0 > 1) ntp = 1.0;
    if (d.status[j] == 0) {
      // copy positions: a fresh sub-block's copies are still at Xbar.  The
      // first CU copies are gathered into registers with their loads issued
      // together (indices clamped into the point's range); further copies,
      // rare, are read in a loop.
      const double xb[3] = {d.Xbar[j], d.Xbar[(int64_t)d.N + j], d.Xbar[2 * (int64_t)d.N + j]};
      constexpr int CU = 4;
      const int n = c1 - c0;
      // unconditional gathers (indices clamped into the copy array, so no
      // array is filled under a condition and all stay in registers)
      double xu[CU][3];
      int cu[CU], fr[CU];
#pragma unroll
      for (int u = 0; u < CU; ++u) cu[u] = d.pt_copies[min(c0 + max(0, min(u, n - 1)), (int)d.NC - 1)];
#pragma unroll
      for (int u = 0; u < CU; ++u) {
        fr[u] = d.blk_fresh[d.copy_blk[cu[u]]];
        xu[u][0] = d.Xc[3 * (int64_t)cu[u]];
        xu[u][1] = d.Xc[3 * (int64_t)cu[u] + 1];
        xu[u][2] = d.Xc[3 * (int64_t)cu[u] + 2];
      }
#pragma unroll
      for (int u = 0; u < CU; ++u)
        if (fr[u]) {
          xu[u][0] = xb[0];
          xu[u][1] = xb[1];
          xu[u][2] = xb[2];
        }
      // (xb copied into the closure: an array captured by reference would be
      // kept in scratch memory)
      auto copy_x = [&d, b0 = xb[0], b1 = xb[1], b2 = xb[2]](int c, double (&x)[3]) {
        if (d.blk_fresh[d.copy_blk[c]]) {
          x[0] = b0;
          x[1] = b1;
          x[2] = b2;
        } else {
          x[0] = d.Xc[3 * (int64_t)c];
          x[1] = d.Xc[3 * (int64_t)c + 1];
          x[2] = d.Xc[3 * (int64_t)c + 2];
        }
      };
      double m[3] = {0, 0, 0};
#pragma unroll
      for (int u = 0; u < CU; ++u)
        if (u < n) {
          m[0] += xu[u][0];
          m[1] += xu[u][1];
          m[2] += xu[u][2];
        }
      for (int cc = c0 + CU; cc < c1; ++cc) {
        double x[3];
        copy_x(d.pt_copies[cc], x);
        m[0] += x[0];
        m[1] += x[1];
        m[2] += x[2];
      }
      if (n > 0) {
        double inv = 1.0 / (double)n;
        for (int r = 0; r < 3; ++r) m[r] *= inv;
      } else {  // no copy: the consensus is the intersection itself
        for (int r = 0; r < 3; ++r) m[r] = xb[r];
      }
#pragma unroll
      for (int u = 0; u < CU; ++u)
        if (u < n) {
          double e0 = xu[u][0] - m[0], e1 = xu[u][1] - m[1], e2 = xu[u][2] - m[2];
          dmax = fmax(dmax, sqrt(e0 * e0 + e1 * e1 + e2 * e2));
        }
      for (int cc = c0 + CU; cc < c1; ++cc) {
        double x[3];
        copy_x(d.pt_copies[cc], x);
        double e0 = x[0] - m[0], e1 = x[1] - m[1], e2 = x[2] - m[2];
        dmax = fmax(dmax, sqrt(e0 * e0 + e1 * e1 + e2 * e2));
      }
      // plain variants: the dual offsets Xtilde_j^l += X_j^l - X_j (eq:admm9)
      // (their copies are never fresh)
      if (d.Xt) {
        for (int u = 0; u < n; ++u) {
          const int64_t c = d.pt_copies[c0 + u];
          for (int r = 0; r < 3; ++r) d.Xt[3 * c + r] += d.Xc[3 * c + r] - m[r];
        }
      }
      for (int r = 0; r < 3; ++r) d.P0[(int64_t)r * d.N + j] = m[r];
      put_pxs(d, j, m, 0);
    } else {
      const double z[3] = {0.0, 0.0, 0.0};
      put_pxs(d, j, z, d.status[j]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmax(dmax, __shfl_xor(dmax, o));
    ntp += __shfl_xor(ntp, o);
  }
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wv] = dmax;
    sh[4 + wv] = ntp;
  }
  __syncthreads();
  // one partial per workgroup (k_consensus_reduce sums them: atomics of every
  // workgroup on the same two words would queue up in the cache)
  if (threadIdx.x == 0) {
    d.cons_part[2 * blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    d.cons_part[2 * blockIdx.x + 1] = sh[4] + sh[5] + sh[6] + sh[7];
  }
}

// the four statistics of an intersection from the per-workgroup partials
// (one workgroup of 1,024 threads, a fixed order: the sums are reproducible)
// the intersection's per-workgroup partials, summed by INT_RED_WG
// workgroups whose sums are added to acc_int[0..3] (zeroed with the launch):
// a few dozen atomic adds per word instead of one workgroup reading them all
constexpr int INT_RED_WG = 64;
__global__ __launch_bounds__(1024) void k_int_reduce(Dev d, int nwg) {
  __shared__ double sh[4 * 16];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const double4* p4 = reinterpret_cast<const double4*>(d.int_part);
  for (int t = blockIdx.x * (int)blockDim.x + threadIdx.x; t < nwg; t += (int)(gridDim.x * blockDim.x)) {
    const double4 a = p4[t];
    v[0] += a.x;
    v[1] += a.y;
    v[2] += a.z;
    v[3] += a.w;
  }
  for (int q = 0; q < 4; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int q = 0; q < 4; ++q) sh[16 * q + wv] = v[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[16 * threadIdx.x + w];
    atomicAdd(&d.acc_int[threadIdx.x], s);
  }
}

// largest copy spread and tie-point count from the per-workgroup partials
// (one workgroup of 1,024 threads)
__global__ __launch_bounds__(1024) void k_consensus_reduce(Dev d, int nwg) {
  __shared__ double sh[32];
  double mx = 0.0, sum = 0.0;
  constexpr int U = 8;  // partials in flight per thread
  const double2* p2 = reinterpret_cast<const double2*>(d.cons_part);
  for (int t0 = threadIdx.x; t0 < nwg; t0 += U * (int)blockDim.x) {
    double2 a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      a[u] = t < nwg ? p2[t] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mx = fmax(mx, a[u].x);
      sum += a[u].y;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o));
    sum += __shfl_xor(sum, o);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wv] = mx;
    sh[16 + wv] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m2 = 0.0, s2 = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      m2 = fmax(m2, sh[q]);
      s2 += sh[16 + q];
    }
    d.acc_cons[0] = m2;
    d.acc_cons[1] = s2;
  }
}

__global__ void k_consensus_cams(Dev d, double* stats) {
  int i = blockIdx.x * NT + threadIdx.x;
  if (stats && i == 0) {  // the point pass's sums are complete
    stats[0] = d.acc_cons[0];
    stats[1] = d.acc_cons[1];
  }
  if (i == 0) *d.rho_t *= d.rho_growth;  // the scalar weight of the next outer iteration
  if (i >= d.M) return;
  int o = d.cam_orig[i];
  const double* c = d.cam + (int64_t)CAM_STRIDE * i;
  for (int q = 0; q < 9; ++q) d.u_camR[9 * (int64_t)o + q] = c[q];
  for (int r = 0; r < 3; ++r) d.u_camC[(int64_t)r * d.M + o] = c[9 + r];
  if (d.intr) {
    d.u_intr[o] = d.intr[2 * (int64_t)i];
    d.u_intr[(int64_t)d.M + o] = d.intr[2 * (int64_t)i + 1];
  }
}

// dense copy-out of one sub-block's RCS (row-major n6 x n6 lower) and rhs
__global__ void k_rcs_extract(Dev d, int l, double* S_out, double* e_out) {
  int n6 = d.np * (d.blk_cam_off[l + 1] - d.blk_cam_off[l]);
  int64_t tot = (int64_t)n6 * n6;
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < tot; t += (int64_t)gridDim.x * NT) {
    int row = (int)(t / n6), col = (int)(t % n6);
    double v = 0.0;
    if (col <= row) v = d.S[rcs_elem(d, l, row, col)];
    S_out[t] = v;
  }
  for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < n6; t += (int64_t)gridDim.x * NT)
    e_out[t] = d.y[d.vec_off[l] + t];
}

// dense copy-out of an iterative sub-block's block-sparse RCS (output zeroed first)
__global__ void k_bsr_extract(Dev d, int l, double* S_out, double* e_out) {
  const int base = d.blk_cam_off[l];
  const int ncam = d.blk_cam_off[l + 1] - base;
  const int n6 = 6 * ncam;
  for (int a = blockIdx.x; a < ncam; a += gridDim.x) {
    const int i = base + a;
    for (int b = d.bsr_row_off[i]; b < d.bsr_row_off[i + 1]; ++b) {
      const int a2 = d.bsr_col[b];
      for (int t = threadIdx.x; t < 36; t += NT)
        S_out[(int64_t)(6 * a + t / 6) * n6 + 6 * a2 + t % 6] = (double)d.bsr[(int64_t)b * 36 + t];
    }
    if (threadIdx.x < 6) e_out[6 * a + threadIdx.x] = d.y[d.vec_off[l] + 6 * a + threadIdx.x];
  }
}

// ------------------------------------------------------------ covariance
// element (r, c) of the symmetric matrix held as a lower triangle in the RCS
// storage of sub-block l
__device__ __forceinline__ double rcs_sym(const Dev& d, int l, int r, int c) {
  return r >= c ? d.S[rcs_elem(d, l, r, c)] : d.S[rcs_elem(d, l, c, r)];
}

// Camera covariance: the camera's np x np diagonal block of S^-1 of its
// sub-block (the RCS storage holds S^-1 after the inverse launches), written
// row-major in the caller's camera order.
__global__ void k_cov_cams(Dev d, double* out) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= d.M) return;
  const int np = d.np;
  const int l = d.cam_blk[i], a = i - d.blk_cam_off[l];
  double* o = out + (int64_t)np * np * d.cam_orig[i];
  for (int r = 0; r < np; ++r)
    for (int c = 0; c < np; ++c) o[np * r + c] = rcs_sym(d, l, np * a + r, np * a + c);
}

// Point-copy covariance (Sec. 2): M_XX = V^-1 + V^-1 (sum_{k,k'} Y_k^T
// M(i_k, i_k') Y_k') V^-1 with M = S^-1 of the copy's sub-block, V the damped
// point block with the tie-point weight and Y_k = A_k^T W_k B_k of the copy's
// observation k in camera i_k, at the state the system was assembled at (FP64
// on both paths).  One thread per copy, the sum as sum_k Y_k^T (sum_k' M Y_k');
// zeros for copies of invalid points.  Output (xx, xy, xz, yy, yz, zz) in copy
// order.
template <int NP>
__device__ __forceinline__ void cov_obs(const Dev& d, int64_t k, const double (&X)[3], bool unit, double (&Y)[NP][3],
                                        double (&BtWB)[6]) {
  const int ic = d.obs_cam[k];
  const double* cm = d.cam + (int64_t)CAM_STRIDE * ic;
  Lin<double> L;
  linearise_cam<NP == 8, double>(cm, NP == 8 ? d.intr + 2 * (int64_t)ic : nullptr, X, d.f, d.cx, d.cy, L);
  const W2<double> W = obs_weight(d, k, unit);
  double WB[2][3];
  for (int c = 0; c < 3; ++c) {
    WB[0][c] = W.a * L.B[0][c] + W.b * L.B[1][c];
    WB[1][c] = W.b * L.B[0][c] + W.c * L.B[1][c];
  }
  for (int c = 0; c < 3; ++c) {
    for (int u = 0; u < 3; ++u) {
      Y[u][c] = L.Ar[0][u] * WB[0][c] + L.Ar[1][u] * WB[1][c];
      Y[3 + u][c] = -(L.B[0][u] * WB[0][c] + L.B[1][u] * WB[1][c]);
    }
    if constexpr (NP == 8)
      for (int u = 0; u < 2; ++u) Y[6 + u][c] = L.Ai[0][u] * WB[0][c] + L.Ai[1][u] * WB[1][c];
  }
  BtWB[0] = L.B[0][0] * WB[0][0] + L.B[1][0] * WB[1][0];
  BtWB[1] = L.B[0][0] * WB[0][1] + L.B[1][0] * WB[1][1];
  BtWB[2] = L.B[0][0] * WB[0][2] + L.B[1][0] * WB[1][2];
  BtWB[3] = L.B[0][1] * WB[0][1] + L.B[1][1] * WB[1][1];
  BtWB[4] = L.B[0][1] * WB[0][2] + L.B[1][1] * WB[1][2];
  BtWB[5] = L.B[0][2] * WB[0][2] + L.B[1][2] * WB[1][2];
}

template <int NP>
__global__ __launch_bounds__(NT) void k_cov_copies(Dev d, double* out) {
  const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (c >= d.NC) return;
  double* o = out + 6 * c;
  const int l = d.copy_blk[c], p = d.copy_pt[c];
  double Mx[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (d.status[p] == 0) {
    const bool unit = *d.rw_unit != 0;
    const int k0 = d.copy_off[c], k1 = d.copy_off[c + 1], b0 = d.blk_cam_off[l];
    double xb[3];
    prior_centre(d, p, c, xb);
    double X[3] = {xb[0], xb[1], xb[2]};
    if (!d.blk_fresh[l])
      for (int r = 0; r < 3; ++r) X[r] = d.Xc[3 * c + r];
    double h[6];
    om_load(d, c, h);
    double Y[NP][3], bwb[6];
    for (int k = k0; k < k1; ++k) {
      cov_obs<NP>(d, k, X, unit, Y, bwb);
      for (int q = 0; q < 6; ++q) h[q] += bwb[q];
    }
    h[0] *= 1.0 + d.lambda;
    h[3] *= 1.0 + d.lambda;
    h[5] *= 1.0 + d.lambda;
    double lch[6], vi[6];
    if (chol3(h, lch)) {
      chol3_inverse(lch, vi);
      double T3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int k1i = k0; k1i < k1; ++k1i) {
        double Y1[NP][3];
        cov_obs<NP>(d, k1i, X, unit, Y1, bwb);
        const int a1 = d.obs_cam[k1i] - b0;
        double G[NP][3];
        for (int u = 0; u < NP; ++u) G[u][0] = G[u][1] = G[u][2] = 0.0;
        for (int k2i = k0; k2i < k1; ++k2i) {
          double Y2[NP][3];
          cov_obs<NP>(d, k2i, X, unit, Y2, bwb);
          const int a2 = d.obs_cam[k2i] - b0;
          for (int u = 0; u < NP; ++u)
            for (int v = 0; v < NP; ++v) {
              const double m = rcs_sym(d, l, NP * a1 + u, NP * a2 + v);
              for (int q = 0; q < 3; ++q) G[u][q] += m * Y2[v][q];
            }
        }
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) {
            double sacc = 0.0;
            for (int u = 0; u < NP; ++u) sacc += Y1[u][r] * G[u][q];
            T3[r][q] += sacc;
          }
      }
      const double V[3][3] = {{vi[0], vi[1], vi[2]}, {vi[1], vi[3], vi[4]}, {vi[2], vi[4], vi[5]}};
      double VT[3][3];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) VT[r][q] = V[r][0] * T3[0][q] + V[r][1] * T3[1][q] + V[r][2] * T3[2][q];
      const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
      for (int e = 0; e < 6; ++e) {
        const int r = rr[e], q = cc[e];
        Mx[e] = V[r][q] + VT[r][0] * V[0][q] + VT[r][1] * V[1][q] + VT[r][2] * V[2][q];
      }
    }
  }
  for (int e = 0; e < 6; ++e) o[e] = Mx[e];
}

}  // namespace

// ------------------------------------------------------------- launchers
void launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = grid_for(n);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_zero, dim3(g), dim3(NT), 0, st, p, n);
}

void launch_zero_wide(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = grid_for((n / 2 + 3) / 4);
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_zero_wide, dim3(g), dim3(NT), 0, st, p, n);
}

void launch_zero_i32(int32_t* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  unsigned g = grid_for(n);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_zero_i32, dim3(g), dim3(NT), 0, st, p, n);
}

void launch_gather(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_obs, dim3(grid_for(d.K)), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_gather_pm, dim3(grid_for(d.K)), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_gather_cm, dim3(grid_for(d.K)), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_gather_cams, dim3(grid_for(d.M)), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_gather_pts, dim3(grid_for(d.N)), dim3(NT), 0, st, d);
}

void launch_check_inputs(const Dev& d, int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_check_inputs, dim3(1024), dim3(NT), 0, st, d, cnt);
}

void launch_init_rcs(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_pad_identity, dim3(d.L), dim3(NT), 0, st, d);
}

template <int VAR, bool CAL = false>
static void launch_intersect_var(const Dev& d, bool want_cov, hipStream_t st) {
  if (d.has_info)
    hipLaunchKernelGGL((k_intersect<true, VAR, CAL>), dim3(grid_for(d.N, IT)), dim3(IT), 0, st, d, (int)want_cov);
  else
    hipLaunchKernelGGL((k_intersect<false, VAR, CAL>), dim3(grid_for(d.N, IT)), dim3(IT), 0, st, d, (int)want_cov);
}

void launch_intersect(const Dev& d, bool want_cov, hipStream_t st) {
  launch_zero(d.acc_int, 4 + (int64_t)d.L, st);
  switch (d.variant) {
    case RPBA_VARIANT_ALL_CAMERAS: launch_intersect_var<RPBA_VARIANT_ALL_CAMERAS>(d, want_cov, st); break;
    case RPBA_VARIANT_SCALAR: launch_intersect_var<RPBA_VARIANT_SCALAR>(d, want_cov, st); break;
    case RPBA_VARIANT_PLAIN: launch_intersect_var<RPBA_VARIANT_PLAIN>(d, want_cov, st); break;
    case RPBA_VARIANT_PLAIN_REFINED: launch_intersect_var<RPBA_VARIANT_PLAIN_REFINED>(d, want_cov, st); break;
    default:
      // (intrinsics come with the extended variant only)
      if (d.np == 8) launch_intersect_var<RPBA_VARIANT_EXTENDED, true>(d, want_cov, st);
      else launch_intersect_var<RPBA_VARIANT_EXTENDED>(d, want_cov, st);
      break;
  }
  hipLaunchKernelGGL(k_int_reduce, dim3(INT_RED_WG), dim3(1024), 0, st, d, (int)grid_for(d.N, IT));
}

void launch_intersect_export(const Dev& d, double* cov, int32_t* status_out, double* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_export_pts, dim3(grid_for(d.N)), dim3(NT), 0, st, d, cov, status_out, stats);
}

void launch_cov_outputs(const Dev& d, double* cam_cov, double* copy_cov, hipStream_t st) {
  if (cam_cov) hipLaunchKernelGGL(k_cov_cams, dim3(grid_for(d.M)), dim3(NT), 0, st, d, cam_cov);
  if (copy_cov && d.np == 8) hipLaunchKernelGGL(k_cov_copies<8>, dim3(grid_for(d.NC)), dim3(NT), 0, st, d, copy_cov);
  else if (copy_cov) hipLaunchKernelGGL(k_cov_copies<6>, dim3(grid_for(d.NC)), dim3(NT), 0, st, d, copy_cov);
}

void launch_copy_prep(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_step_begin, dim3(grid_for(d.L)), dim3(NT), 0, st, d);
  if (d.np == 8) {
    if (d.cpk_f32) hipLaunchKernelGGL((k_copy_prep<float, true>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_copy_prep<double, true>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
  } else {
    if (d.cpk_f32) hipLaunchKernelGGL((k_copy_prep<float, false>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_copy_prep<double, false>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
  }
  hipLaunchKernelGGL(k_slots_reduce<false>, dim3(d.L), dim3(NT), 0, st, d);
}

void launch_update(const Dev& d, double* block_stats, hipStream_t st) {
  hipLaunchKernelGGL(k_cam_update, dim3(grid_for(d.M)), dim3(NT), 0, st, d);
  if (d.np == 8) {
    if (d.cpk_f32) hipLaunchKernelGGL((k_back_update<float, true>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_back_update<double, true>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
  } else {
    if (d.cpk_f32) hipLaunchKernelGGL((k_back_update<float, false>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_back_update<double, false>), dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
  }
  hipLaunchKernelGGL(k_slots_reduce<true>, dim3(d.L), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_update_finish, dim3(grid_for(std::max<int64_t>((int64_t)CAM_STRIDE * d.M, d.L))), dim3(NT), 0,
                     st, d, block_stats);
  if (d.lam_blk) hipLaunchKernelGGL(k_restore_copies, dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
}

__global__ void k_init_copies(Dev d) {
  const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (c >= d.NC) return;
  const int p = d.copy_pt[c];
  for (int r = 0; r < 3; ++r) {
    d.Xc[3 * c + r] = d.P0[(int64_t)r * d.N + p];
    d.Xt[3 * c + r] = 0.0;
  }
}

void launch_init_copies(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_init_copies, dim3(grid_for(d.NC)), dim3(NT), 0, st, d);
}

void launch_consensus(const Dev& d, double* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_consensus_pts, dim3(grid_for(d.N)), dim3(NT), 0, st, d);
  hipLaunchKernelGGL(k_consensus_reduce, dim3(1), dim3(1024), 0, st, d, (int)grid_for(d.N));
  hipLaunchKernelGGL(k_export_pts, dim3(grid_for(d.N)), dim3(NT), 0, st, d, (double*)nullptr, (int32_t*)nullptr,
                     (double*)nullptr);
  hipLaunchKernelGGL(k_consensus_cams, dim3(grid_for(d.M)), dim3(NT), 0, st, d, stats);
}

void launch_bsr_extract(const Dev& d, int l, double* S_out, double* e_out, hipStream_t st) {
  hipLaunchKernelGGL(k_bsr_extract, dim3(256), dim3(NT), 0, st, d, l, S_out, e_out);
}

void launch_rcs_extract(const Dev& d, int l, double* S_out, double* e_out, hipStream_t st) {
  hipLaunchKernelGGL(k_rcs_extract, dim3(1024), dim3(NT), 0, st, d, l, S_out, e_out);
}

}  // namespace rpba
