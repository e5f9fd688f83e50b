// Learned block preconditioner for the iterative solution of the reduced
// camera system.  Keeps the block-diagonal form of block-Jacobi (paper Sec. 3
// and 5.4: CG preconditioned by the inverses of the 6x6 camera blocks) and
// replaces each inverse block S_ii^-1 = G^-T G^-1 (S_ii = G G^T) by
//     P_i = G^-T L L^T G^-1,
// L = I + strict lower part from a small network's output, exp(.) on its
// diagonal: symmetric positive definite for every output, exactly
// block-Jacobi for a zero output.
//
// Network: 26 features -> 64 -> 64 (tanh) -> 21 outputs, FP32.  Features of
// camera block i: log(S_ii[q][q] / mean diagonal of the sub-block) (6), the 15
// correlations of S_ii, log(1 + observations), log(1 + neighbour blocks), the
// off-diagonal mass sum_k |S_ik|_F / |S_ii|_F, log10(lambda), the tie-point
// fraction of the camera's observations.
//
// Training (on the GPU, by these kernels): samples (features, G^-1, probe
// pairs (z_i, (S z)_i)) harvested from the systems the method assembles; loss
// (Hutchinson estimate of a block SPAI objective)
//     (1 / (nz nsamp)) sum_samples sum_probes |z_i - P_i (S z)_i|^2,
// backward pass per sample, per-parameter gradient sums in a fixed order, Adam.
#include "rpba_device.hpp"
#include "rpba_internal.hpp"

#include <mutex>
#include <vector>

namespace rpba {

namespace {

constexpr int NF = 26, NH = 64, NO = 21;
constexpr int NPAR = NF * NH + NH + NH * NH + NH + NH * NO + NO;
constexpr int OW1 = 0, OB1 = OW1 + NF * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NO;

// inverse Cholesky factor of a symmetric positive definite 6x6 (row-major);
// returns false on a non-positive pivot
__device__ bool inv_chol6(const float* S, float* Gi) {
  double G[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) G[r][c] = 0.0;
  bool ok = true;
  for (int j = 0; j < 6; ++j) {
    double s = S[6 * j + j];
    for (int k = 0; k < j; ++k) s -= G[j][k] * G[j][k];
    if (!(s > 0.0)) {
      ok = false;
      s = 1.0;
    }
    G[j][j] = sqrt(s);
    for (int r = j + 1; r < 6; ++r) {
      double t = S[6 * r + j];
      for (int k = 0; k < j; ++k) t -= G[r][k] * G[j][k];
      G[r][j] = t / G[j][j];
    }
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) Gi[6 * r + c] = 0.f;
  double X[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) X[r][c] = 0.0;
  for (int c = 0; c < 6; ++c) {
    X[c][c] = 1.0 / G[c][c];
    for (int r = c + 1; r < 6; ++r) {
      double s = 0.0;
      for (int m = c; m < r; ++m) s += G[r][m] * X[m][c];
      X[r][c] = -s / G[r][r];
    }
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c <= r; ++c) Gi[6 * r + c] = (float)X[r][c];
  return ok;
}

__device__ void forward(const float* __restrict__ W, const float* f, float* h1, float* h2, float* o) {
  for (int j = 0; j < NH; ++j) {
    float s = W[OB1 + j];
    for (int i = 0; i < NF; ++i) s += W[OW1 + j * NF + i] * f[i];
    h1[j] = tanhf(s);
  }
  for (int j = 0; j < NH; ++j) {
    float s = W[OB2 + j];
    for (int i = 0; i < NH; ++i) s += W[OW2 + j * NH + i] * h1[i];
    h2[j] = tanhf(s);
  }
  for (int j = 0; j < NO; ++j) {
    float s = W[OB3 + j];
    for (int i = 0; i < NH; ++i) s += W[OW3 + j * NH + i] * h2[i];
    o[j] = s;
  }
}

__device__ void lower_from_output(const float* o, float* Lm) {
  for (int q = 0; q < 36; ++q) Lm[q] = 0.f;
  int t = 0;
  for (int r = 1; r < 6; ++r)
    for (int c = 0; c < r; ++c) Lm[6 * r + c] = o[t++];
  for (int r = 0; r < 6; ++r) Lm[6 * r + r] = expf(o[15 + r]);
}

// P = Gi^T Lm Lm^T Gi
__device__ void spd_block(const float* Gi, const float* Lm, float* P) {
  float M[36];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      float s = 0.f;
      for (int m = 0; m < 6; ++m) s += Lm[6 * m + r] * Gi[6 * m + c];
      M[6 * r + c] = s;
    }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      float s = 0.f;
      for (int m = 0; m < 6; ++m) s += M[6 * m + r] * M[6 * m + c];
      P[6 * r + c] = s;
    }
}

// mean diagonal entry of every iterative sub-block's RCS
__global__ void k_mean_diag(Dev d, float* mean_diag) {
  __shared__ double red[4];
  const int l = blockIdx.x;
  if (!d.blk_pcg[l]) return;
  const int base = d.blk_cam_off[l];
  const int ncam = d.blk_cam_off[l + 1] - base;
  double s = 0.0;
  for (int a = threadIdx.x; a < ncam; a += blockDim.x) {
    const float* S = d.bsr + (int64_t)d.pb_bsr[d.nb_off[base + a + 1] - 1] * 36;
    for (int q = 0; q < 6; ++q) s += S[7 * q];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) mean_diag[l] = (float)((red[0] + red[1] + red[2] + red[3]) / (6.0 * ncam));
}

__device__ void features(const Dev& d, int i, const float* mean_diag, const float* cam_tpfrac, float* f) {
  const int l = d.cam_blk[i];
  const int b0 = d.bsr_row_off[i], b1 = d.bsr_row_off[i + 1];
  const float* S = d.bsr + (int64_t)d.pb_bsr[d.nb_off[i + 1] - 1] * 36;
  float dg[6];
  for (int q = 0; q < 6; ++q) {
    dg[q] = S[7 * q];
    f[q] = logf(dg[q] / mean_diag[l]);
  }
  int t = 6;
  for (int r = 1; r < 6; ++r)
    for (int c = 0; c < r; ++c) f[t++] = S[6 * r + c] / sqrtf(dg[r] * dg[c]);
  float fro_ii = 0.f;
  for (int q = 0; q < 36; ++q) fro_ii += S[q] * S[q];
  const int a = i - d.blk_cam_off[l];
  float off = 0.f;
  for (int b = b0; b < b1; ++b) {
    if (d.bsr_col[b] == a) continue;
    const float* B = d.bsr + (int64_t)b * 36;
    float fr = 0.f;
    for (int q = 0; q < 36; ++q) fr += B[q] * B[q];
    off += sqrtf(fr);
  }
  f[21] = log1pf((float)(d.cam_obs_off[i + 1] - d.cam_obs_off[i]));
  f[22] = log1pf((float)(b1 - b0 - 1));
  f[23] = off / sqrtf(fro_ii);
  f[24] = log10f((float)d.lambda);
  f[25] = cam_tpfrac[i];
}

// preconditioner blocks for every camera of an iterative sub-block: learned
// (network W) or, with W = NULL, block-Jacobi S_ii^-1 = G^-T G^-1 through the
// same arithmetic
__global__ void k_precond_learned(Dev d, const float* __restrict__ W, const float* mean_diag, const float* cam_tpfrac) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.M) return;
  const int l = d.cam_blk[i];
  if (!d.blk_pcg[l] || (d.active && !d.active[l])) return;
  float h1[NH], h2[NH], o[NO], Gi[36], Lm[36];
  const float* S = d.bsr + (int64_t)d.pb_bsr[d.nb_off[i + 1] - 1] * 36;
  if (!inv_chol6(S, Gi)) d.blk_fail[l] = 1;
  if (W) {
    float f[NF];
    features(d, i, mean_diag, cam_tpfrac, f);
    forward(W, f, h1, h2, o);
  } else {
    for (int q = 0; q < NO; ++q) o[q] = 0.f;  // block-Jacobi: L = I
  }
  lower_from_output(o, Lm);
  spd_block(Gi, Lm, d.Pblk + (int64_t)i * 36);
}

// training samples of the current systems: (f, G^-1, z_i (nz), w_i = (S z)_i (nz))
__global__ void k_harvest(Dev d, const float* mean_diag, const float* cam_tpfrac, const float* __restrict__ z, int nz,
                          const int32_t* __restrict__ cams, int ncams, float* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncams) return;
  const int i = cams[s];
  const int stride = NF + 36 + 12 * nz;
  float* o = out + (int64_t)s * stride;
  features(d, i, mean_diag, cam_tpfrac, o);
  const float* S = d.bsr + (int64_t)d.pb_bsr[d.nb_off[i + 1] - 1] * 36;
  inv_chol6(S, o + NF);
  const int base = d.blk_cam_off[d.cam_blk[i]];
  for (int t = 0; t < nz; ++t) {
    const float* zt = z + (int64_t)t * d.M * 6;
    float w[6] = {0, 0, 0, 0, 0, 0};
    for (int b = d.bsr_row_off[i]; b < d.bsr_row_off[i + 1]; ++b) {
      const float* B = d.bsr + (int64_t)b * 36;
      const float* zc = zt + 6 * (int64_t)(base + d.bsr_col[b]);
      for (int q = 0; q < 6; ++q)
        for (int c = 0; c < 6; ++c) w[q] += B[6 * q + c] * zc[c];
    }
    for (int q = 0; q < 6; ++q) {
      o[NF + 36 + 6 * t + q] = zt[6 * (int64_t)i + q];
      o[NF + 36 + 6 * nz + 6 * t + q] = w[q];
    }
  }
}

// ---------------------------------------------------------------- training
// per sample: forward, loss, backward down to the pre-activations; stores
// h1, h2 (64 each), dout (21), dh2, dh1 (64 each) for the parameter sums
constexpr int SCR = NH + NH + NO + NH + NH;

__global__ void k_train_samples(const float* __restrict__ W, const float* __restrict__ samples, int nsamp, int nz,
                                float* scratch, float* loss_part) {
  __shared__ float red[4];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  float loss = 0.f;
  if (s < nsamp) {
    const int stride = NF + 36 + 12 * nz;
    const float* sm = samples + (int64_t)s * stride;
    const float* f = sm;
    const float* Gi = sm + NF;
    float* sc = scratch + (int64_t)s * SCR;
    float* h1 = sc;
    float* h2 = sc + NH;
    float* dout = sc + 2 * NH;
    float* dh2 = dout + NO;
    float* dh1 = dh2 + NH;
    float o[NO], Lm[36], dLm[36];
    forward(W, f, h1, h2, o);
    lower_from_output(o, Lm);
    for (int q = 0; q < 36; ++q) dLm[q] = 0.f;
    for (int t = 0; t < nz; ++t) {
      const float* z = sm + NF + 36 + 6 * t;
      const float* w = sm + NF + 36 + 6 * nz + 6 * t;
      float u[6], a[6], v[6], p[6], res[6], qv[6], bq[6];
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Gi[6 * r + m] * w[m];
        u[r] = x;
      }
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Lm[6 * m + r] * u[m];
        a[r] = x;
      }
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Lm[6 * r + m] * a[m];
        v[r] = x;
      }
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Gi[6 * m + r] * v[m];
        p[r] = x;
      }
      for (int r = 0; r < 6; ++r) {
        res[r] = z[r] - p[r];
        loss += res[r] * res[r];
      }
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Gi[6 * r + m] * (-2.f * res[m]);
        qv[r] = x;
      }
      for (int r = 0; r < 6; ++r) {
        float x = 0.f;
        for (int m = 0; m < 6; ++m) x += Lm[6 * m + r] * qv[m];
        bq[r] = x;
      }
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) dLm[6 * r + c] += qv[r] * a[c] + u[r] * bq[c];
    }
    const float scale = 1.f / ((float)nz * (float)nsamp);
    loss *= scale;
    int t = 0;
    for (int r = 1; r < 6; ++r)
      for (int c = 0; c < r; ++c) dout[t++] = dLm[6 * r + c] * scale;
    for (int r = 0; r < 6; ++r) dout[15 + r] = dLm[7 * r] * Lm[7 * r] * scale;
    for (int i = 0; i < NH; ++i) {
      float x = 0.f;
      for (int j = 0; j < NO; ++j) x += dout[j] * W[OW3 + j * NH + i];
      dh2[i] = x * (1.f - h2[i] * h2[i]);
    }
    for (int i = 0; i < NH; ++i) {
      float x = 0.f;
      for (int j = 0; j < NH; ++j) x += dh2[j] * W[OW2 + j * NH + i];
      dh1[i] = x * (1.f - h1[i] * h1[i]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one thread per parameter: gradient = sum over samples (fixed order)
__global__ void k_train_param_grads(const float* __restrict__ samples, int nsamp, int nz, const float* __restrict__ scratch,
                                    float* grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NPAR) return;
  const int stride = NF + 36 + 12 * nz;
  double g = 0.0;
  if (q < OB1) {
    const int j = (q - OW1) / NF, i = (q - OW1) % NF;
    for (int s = 0; s < nsamp; ++s) g += (double)scratch[(int64_t)s * SCR + 2 * NH + NO + NH + j] * samples[(int64_t)s * stride + i];
  } else if (q < OW2) {
    const int j = q - OB1;
    for (int s = 0; s < nsamp; ++s) g += scratch[(int64_t)s * SCR + 2 * NH + NO + NH + j];
  } else if (q < OB2) {
    const int j = (q - OW2) / NH, i = (q - OW2) % NH;
    for (int s = 0; s < nsamp; ++s) g += (double)scratch[(int64_t)s * SCR + 2 * NH + NO + j] * scratch[(int64_t)s * SCR + i];
  } else if (q < OW3) {
    const int j = q - OB2;
    for (int s = 0; s < nsamp; ++s) g += scratch[(int64_t)s * SCR + 2 * NH + NO + j];
  } else if (q < OB3) {
    const int j = (q - OW3) / NH, i = (q - OW3) % NH;
    for (int s = 0; s < nsamp; ++s) g += (double)scratch[(int64_t)s * SCR + 2 * NH + j] * scratch[(int64_t)s * SCR + NH + i];
  } else {
    const int j = q - OB3;
    for (int s = 0; s < nsamp; ++s) g += scratch[(int64_t)s * SCR + 2 * NH + j];
  }
  grad[q] = (float)g;
}

__global__ void k_adam(float* W, const float* grad, float* m, float* v, int t, float lr, float b1, float b2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NPAR) return;
  const float g = grad[q];
  const float mq = b1 * m[q] + (1.f - b1) * g;
  const float vq = b2 * v[q] + (1.f - b2) * g * g;
  m[q] = mq;
  v[q] = vq;
  const float mh = mq / (1.f - powf(b1, (float)t));
  const float vh = vq / (1.f - powf(b2, (float)t));
  W[q] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_sum_f32(const float* parts, int n, float* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += parts[q];
  out[0] = (float)s;
}

}  // namespace

// Scratch of the training step that allocates nothing: per-sample
// activations and gradients (SCR floats each) for at most
// TRAIN_NOALLOC_MAX_SAMPLES samples, then the per-workgroup loss partials.
// One copy per GPU, held until the process ends.
constexpr size_t kNoAllocFloats =
    (size_t)TRAIN_NOALLOC_MAX_SAMPLES * SCR + (TRAIN_NOALLOC_MAX_SAMPLES + 255) / 256 + 64;
static __device__ __align__(256) float scratch[kNoAllocFloats];

float* train_noalloc_scratch(hipError_t* err) {
  // the array's device address, looked up once per device with that device
  // current (each GPU holds its own copy at its own address); host code uses
  // only this address, never the array's name
  static std::mutex mu;
  static std::vector<float*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *err = e;
      return nullptr;
    }
    addr[dev] = static_cast<float*>(ptr);
  }
  *err = hipSuccess;
  return addr[dev];
}

size_t train_noalloc_parts_offset() { return (size_t)TRAIN_NOALLOC_MAX_SAMPLES * SCR; }

void launch_sum_f32(const float* parts, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(64), 0, st, parts, n, out);
}

int mlp_num_params() { return NPAR; }
int mlp_num_features() { return NF; }
int mlp_scratch_per_sample() { return SCR; }

void launch_mean_diag(const Dev& d, float* mean_diag, hipStream_t st) {
  hipLaunchKernelGGL(k_mean_diag, dim3(d.L), dim3(256), 0, st, d, mean_diag);
}

void launch_precond_learned(const Dev& d, const float* W, const float* mean_diag, const float* cam_tpfrac,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_precond_learned, dim3((d.M + 127) / 128), dim3(128), 0, st, d, W, mean_diag, cam_tpfrac);
}

void launch_harvest(const Dev& d, const float* mean_diag, const float* cam_tpfrac, const float* z, int nz,
                    const int32_t* cams, int ncams, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_harvest, dim3((ncams + 127) / 128), dim3(128), 0, st, d, mean_diag, cam_tpfrac, z, nz, cams,
                     ncams, out);
}

void launch_train_step(const float* samples, int nsamp, int nz, float* W, float* m, float* v, int t, float lr,
                       float* scratch, float* grad, float* loss_part, bool apply, hipStream_t st) {
  const int g = (nsamp + 255) / 256;
  hipLaunchKernelGGL(k_train_samples, dim3(g), dim3(256), 0, st, W, samples, nsamp, nz, scratch, loss_part);
  hipLaunchKernelGGL(k_train_param_grads, dim3((NPAR + 255) / 256), dim3(256), 0, st, samples, nsamp, nz, scratch,
                     grad);
  if (apply)
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, st, W, grad, m, v, t, lr, 0.9f, 0.999f, 1e-8f);
}

}  // namespace rpba
