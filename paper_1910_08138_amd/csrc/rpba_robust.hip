// Robust re-weighting (paper Sec. 5.3): per camera the scale sigma0_i =
// 1.4826 MAD of the whitened residual components of its observations (from
// the last intersection); an observation whose normalised residual
// sqrt(v^T W v) / sigma0_i exceeds t_v is flagged.  Three modes:
//   RPBA_ROBUST_WEIGHT          flagged observations down-weighted by a
//                               factor (1e-4 by default), the others 1;
//   RPBA_ROBUST_ELIMINATE_POINTS the same, and every point holding a flagged
//                               observation removed (parallel variant);
//   RPBA_ROBUST_DELETE_OBS      flagged observations deleted (weight 0), and
//                               points left with fewer than two observations
//                               removed (serial variant).
// A deleted observation stays deleted: it enters no scale, flag or count.
// Whitening z = L^T v with W = L L^T (Cholesky of the 2x2 weight).
//
// The medians are exact order statistics: a radix select over the 64-bit
// order-preserving keys of the doubles, one workgroup per camera, values
// staged in LDS (or in a global scratch slice for cameras with very many
// observations).  Median of an even count = mean of the two middle values.
#include "rpba_device.hpp"
#include "rpba_internal.hpp"
#include "rpba_plan.hpp"

namespace rpba {

namespace {

constexpr int RT = 256;
constexpr int LDS_VALS = 8192;  // doubles staged in LDS per camera

__device__ __forceinline__ uint64_t okey(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ double okey_inv(uint64_t k) {
  const uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)u);
}

// k-th smallest (0-based) of vals[0..n), returned to every thread: eight
// radix passes over the keys, one byte each from the top; after each pass one
// wave scans the 256-bin histogram (4 bins per lane) to find the bin holding
// the k-th key.
__device__ double select_kth(const double* vals, int n, int k, uint32_t* hist, uint64_t* sh_prefix, int* sh_k) {
  uint64_t prefix = 0, mask = 0;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = threadIdx.x; b < 256; b += RT) hist[b] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += RT) {
      const uint64_t kk = okey(vals[t]);
      if ((kk & mask) == prefix) atomicAdd(&hist[(kk >> shift) & 255], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
      const uint32_t own = h0 + h1 + h2 + h3;
      uint32_t inc = own;
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
      }
      const uint32_t exc = inc - own;
      if ((uint32_t)k >= exc && (uint32_t)k < inc) {
        uint32_t kk = (uint32_t)k - exc;
        int b = 4 * lane;
        if (kk >= h0) {
          kk -= h0;
          ++b;
          if (kk >= h1) {
            kk -= h1;
            ++b;
            if (kk >= h2) {
              kk -= h2;
              ++b;
            }
          }
        }
        *sh_k = (int)kk;
        *sh_prefix = prefix | ((uint64_t)b << shift);
      }
    }
    __syncthreads();
    k = *sh_k;
    prefix = *sh_prefix;
    mask |= (uint64_t)255 << shift;
    __syncthreads();
  }
  return okey_inv(prefix);
}

__device__ __forceinline__ double median(const double* vals, int n, uint32_t* hist, uint64_t* shp, int* shk) {
  const double a = select_kth(vals, n, (n - 1) / 2, hist, shp, shk);
  const double b = select_kth(vals, n, n / 2, hist, shp, shk);
  return 0.5 * (a + b);
}

// base weight W0 (without the robust multiplier)
__device__ __forceinline__ W2<double> base_weight(const Dev& d, int64_t k) {
  if (d.has_info) {
    const double* w = d.info + 3 * k;
    return {w[0], w[1], w[2]};
  }
  return {d.w0, 0.0, d.w0};
}

__global__ __launch_bounds__(RT) void k_robust_scale(Dev d, double* spill, const int64_t* spill_off, double t_v,
                                                     double down_weight, int mode, int32_t* bad,
                                                     double* sigma_cam) {
  __shared__ double lds[LDS_VALS];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t shp;
  __shared__ int shk, cnt;
  __shared__ double sh_flag[RT / 64];
  const int i = blockIdx.x;
  const int o0 = d.cam_obs_off[i], o1 = d.cam_obs_off[i + 1];
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  double* vals = (2 * (o1 - o0) <= LDS_VALS) ? lds : spill + spill_off[i];
  // whitened residual components of the camera's observations of valid points
  for (int t = o0 + threadIdx.x; t < o1; t += RT) {
    const int k = d.cam_obs[t];
    if (d.status[d.copy_pt[d.obs_copy[k]]] != 0 || d.rw[k] == 0.0) continue;
    const W2<double> W = base_weight(d, k);
    const double l11 = sqrt(W.a), l21 = W.b / l11, l22 = sqrt(W.c - l21 * l21);
    const int64_t pos = d.pm_pos[k];  // residuals are stored point-major
    const double v0 = d.res[2 * pos], v1 = d.res[2 * pos + 1];
    const int at = atomicAdd(&cnt, 2);
    vals[at] = l11 * v0 + l21 * v1;
    vals[at + 1] = l22 * v1;
  }
  __syncthreads();
  const int n = cnt;
  double s0 = 0.0;
  if (n > 0) {
    const double med = median(vals, n, hist, &shp, &shk);
    for (int t = threadIdx.x; t < n; t += RT) vals[t] = fabs(vals[t] - med);
    __syncthreads();
    s0 = 1.4826 * median(vals, n, hist, &shp, &shk);
  }
  if (threadIdx.x == 0) sigma_cam[i] = s0;
  // flags and weights
  double nflag = 0.0;
  for (int t = o0 + threadIdx.x; t < o1; t += RT) {
    const int k = d.cam_obs[t];
    const int pt = d.copy_pt[d.obs_copy[k]];
    const bool deleted = d.rw[k] == 0.0;
    double w = deleted ? 0.0 : 1.0;
    if (d.status[pt] == 0 && !deleted) {
      const int64_t pos = d.pm_pos[k];
      const double v0 = d.res[2 * pos], v1 = d.res[2 * pos + 1];
      const double vb = sqrt(wquad(base_weight(d, k), v0, v1));
      if (s0 > 0.0 && vb > t_v * s0) {
        w = mode == RPBA_ROBUST_DELETE_OBS ? 0.0 : down_weight;
        nflag += 1.0;
        bad[pt] = 1;
      }
    }
    d.rw[k] = w;
    d.cm_rw[t] = w;  // the diagonal Schur pass's camera-major copy
    if (w != 1.0) *d.rw_unit = 0;  // from now on the Schur passes read the weights
    const int64_t pos = d.pm_pos[k];  // the intersection's copy of the weight
    if (d.has_info) {
      for (int q = 0; q < 3; ++q) d.pm_w[3 * pos + q] = w * d.info[3 * (int64_t)k + q];
    } else {
      d.pm_code[pos] = (d.pm_code[pos] & ~(PM_DOWN | PM_DEL)) | (w != 1.0 ? PM_DOWN : 0) | (w == 0.0 ? PM_DEL : 0);
    }
  }
  for (int o = 32; o > 0; o >>= 1) nflag += __shfl_xor(nflag, o);
  if ((threadIdx.x & 63) == 0) sh_flag[threadIdx.x >> 6] = nflag;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&d.acc_rob[0], sh_flag[0] + sh_flag[1] + sh_flag[2] + sh_flag[3]);
}

// flagged points: removed in the two eliminating modes (every one, or those
// left with fewer than two observations); the flags are cleared for the next call
__global__ void k_robust_eliminate(Dev d, int32_t* bad, int mode) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *d.rec_valid = 0;  // the weights changed: copy records are rebuilt by the next step
  if (j >= d.N) return;
  if (bad[j]) {
    bool drop = mode == RPBA_ROBUST_ELIMINATE_POINTS;
    if (mode == RPBA_ROBUST_DELETE_OBS) {
      int live = 0;
      for (int i = d.pm_off[j]; i < d.pm_off[j + 1]; ++i) live += d.rw[d.pm_k[i]] != 0.0;
      drop = live < 2;
    }
    if (drop && d.status[j] == 0) {
      d.status[j] = 4;
      atomicAdd(&d.acc_rob[1], 1.0);
    }
    bad[j] = 0;
  }
}

__global__ void k_copy_stats2(const double* src, double* dst) {
  if (threadIdx.x == 0) {
    dst[0] = src[0];
    dst[1] = src[1];
  }
}

}  // namespace

int robust_lds_values() { return LDS_VALS; }

void launch_robust(const Dev& d, double* spill, const int64_t* spill_off, int32_t* bad, double* sigma_cam, double t_v,
                   double down_weight, int mode, double* stats, hipStream_t st) {
  launch_zero(d.acc_rob, 2, st);
  hipLaunchKernelGGL(k_robust_scale, dim3(d.M), dim3(RT), 0, st, d, spill, spill_off, t_v, down_weight, mode, bad,
                     sigma_cam);
  hipLaunchKernelGGL(k_robust_eliminate, dim3((d.N + 255) / 256), dim3(256), 0, st, d, bad, mode);
  if (stats) hipLaunchKernelGGL(k_copy_stats2, dim3(1), dim3(64), 0, st, (const double*)d.acc_rob, stats);
}

}  // namespace rpba
