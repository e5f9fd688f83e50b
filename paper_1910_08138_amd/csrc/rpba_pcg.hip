// Iterative solution of the reduced camera system of a sub-block: conjugate
// gradients preconditioned block-diagonally by one 6x6 block per camera (the
// inverses of the diagonal blocks, "block-Jacobi", paper Sec. 3 and 5.4, or the
// learned blocks), run in FP32 on the FP32 block-sparse RCS, inside an
// iterative refinement whose residual r = e - S x is accumulated in FP64.
//
// One workgroup per sub-block keeps every vector of the system in LDS and
// runs all refinement sweeps and CG iterations without leaving the kernel;
// the workgroups of all iterative sub-blocks run concurrently in one launch.
// CG: x0 = 0; stop when |r|_2 <= tol |b|_2 after an update (same rule as the
// oracle).
#include "rpba_device.hpp"
#include "rpba_internal.hpp"

namespace rpba {

namespace {

constexpr int PW = 8;          // waves per workgroup
constexpr int PT = 64 * PW;    // threads per workgroup

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// sum over the workgroup (all threads return the total)
__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < PW; ++q) t += red[q];
  return t;
}

// out = S v for the sub-block (rows base .. base + ncam - 1), accumulating in A
template <typename A, typename V>
__device__ __forceinline__ void spmv(const Dev& d, int base, int ncam, const V* v, A* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int a = w; a < ncam; a += PW) {
    const int i = base + a;
    const int b0 = d.bsr_row_off[i], b1 = d.bsr_row_off[i + 1];
    A s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = b0 + lane; b < b1; b += 64) {
      const float* blk = d.bsr + (int64_t)b * 36;
      const V* xv = v + 6 * d.bsr_col[b];
      A xs[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) xs[c] = (A)xv[c];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        A t = 0;
#pragma unroll
        for (int c = 0; c < 6; ++c) t += (A)blk[6 * q + c] * xs[c];
        s[q] += t;
      }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = wsum(s[q]);
    if (lane < 6) {
      A sv = 0;
#pragma unroll
      for (int q = 0; q < 6; ++q)
        if (q == lane) sv = s[q];
      out[6 * a + lane] = sv;
    }
  }
}

// z = P rr (block-diagonal, FP32)
__device__ __forceinline__ void precond(const Dev& d, int base, int ncam, const float* rr, float* z) {
  for (int t = threadIdx.x; t < 6 * ncam; t += PT) {
    const int a = t / 6, q = t % 6;
    const float* P = d.Pblk + (int64_t)(base + a) * 36 + 6 * q;
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) s += P[c] * rr[6 * a + c];
    z[t] = s;
  }
}

__global__ __launch_bounds__(PT) void k_pcg(Dev d, const int32_t* __restrict__ blocks, int pcg_maxit, double pcg_tol,
                                            double ir_tol, int ir_maxit) {
  extern __shared__ double sm[];
  __shared__ double red[PW];
  const int l = blocks[blockIdx.x];
  if (d.active && !d.active[l]) return;
  const int base = d.blk_cam_off[l];
  const int ncam = d.blk_cam_off[l + 1] - base;
  const int n = 6 * ncam;
  double* e = sm;            // [n] FP64
  double* x = e + n;         // [n] FP64 solution
  double* r = x + n;         // [n] FP64 refinement residual
  float* rr = (float*)(r + n);
  float* z = rr + n;
  float* p = z + n;
  float* q = p + n;
  float* dd = q + n;
  const int64_t vb = d.vec_off[l];
  for (int t = threadIdx.x; t < n; t += PT) {
    e[t] = d.y[vb + t];
    x[t] = 0.0;
    r[t] = e[t];
  }
  __syncthreads();
  double ee = 0.0;
  for (int t = threadIdx.x; t < n; t += PT) ee += e[t] * e[t];
  const double ne = sqrt(wg_sum(ee, red));
  int iters = 0;
  for (int sweep = 0; sweep < ir_maxit && d.blk_fail[l] == 0; ++sweep) {
    double rn = 0.0;
    for (int t = threadIdx.x; t < n; t += PT) rn += r[t] * r[t];
    rn = sqrt(wg_sum(rn, red));
    if (!(rn > ir_tol * ne)) break;
    // inner CG on S dd = r in FP32
    for (int t = threadIdx.x; t < n; t += PT) {
      rr[t] = (float)r[t];
      dd[t] = 0.f;
    }
    __syncthreads();
    precond(d, base, ncam, rr, z);
    __syncthreads();
    double rz = 0.0, b2 = 0.0;
    for (int t = threadIdx.x; t < n; t += PT) {
      p[t] = z[t];
      rz += (double)rr[t] * z[t];
      b2 += (double)rr[t] * rr[t];
    }
    rz = wg_sum(rz, red);
    const double nb = sqrt(wg_sum(b2, red));
    for (int it = 0; it < pcg_maxit; ++it) {
      __syncthreads();
      spmv<float, float>(d, base, ncam, p, q);
      __syncthreads();
      double pq = 0.0;
      for (int t = threadIdx.x; t < n; t += PT) pq += (double)p[t] * q[t];
      pq = wg_sum(pq, red);
      const float alpha = (float)(rz / pq);
      double r2 = 0.0;
      for (int t = threadIdx.x; t < n; t += PT) {
        dd[t] += alpha * p[t];
        rr[t] -= alpha * q[t];
        r2 += (double)rr[t] * rr[t];
      }
      r2 = wg_sum(r2, red);
      ++iters;
      if (!(sqrt(r2) > pcg_tol * nb)) break;
      precond(d, base, ncam, rr, z);
      __syncthreads();
      double rz2 = 0.0;
      for (int t = threadIdx.x; t < n; t += PT) rz2 += (double)rr[t] * z[t];
      rz2 = wg_sum(rz2, red);
      const float beta = (float)(rz2 / rz);
      rz = rz2;
      for (int t = threadIdx.x; t < n; t += PT) p[t] = z[t] + beta * p[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += PT) x[t] += (double)dd[t];
    __syncthreads();
    // r = e - S x with the stored FP32 matrix, FP64 accumulation
    spmv<double, double>(d, base, ncam, x, r);
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += PT) r[t] = e[t] - r[t];
    __syncthreads();
  }
  // the refinement residual the sweeps ended with (r = e - S x of the last
  // sweep, or e itself when no sweep ran)
  double rf = 0.0;
  for (int t = threadIdx.x; t < n; t += PT) rf += r[t] * r[t];
  rf = sqrt(wg_sum(rf, red));
  for (int t = threadIdx.x; t < n; t += PT) d.x[vb + t] = x[t];
  if (threadIdx.x == 0) {
    d.acc_blk[4 * l + 3] = (double)iters;
    if (d.blk_fail[l] == 0 && !(rf <= ir_tol * ne)) d.blk_nc[l] = 1;
  }
}

}  // namespace

size_t pcg_lds_bytes(int max_n) { return (size_t)max_n * (3 * sizeof(double) + 5 * sizeof(float)); }

void launch_pcg(const Dev& d, const int32_t* blocks, int nblocks, int max_n, int pcg_maxit, double pcg_tol,
                double ir_tol, int ir_maxit, hipStream_t st) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_pcg, dim3(nblocks), dim3(PT), pcg_lds_bytes(max_n), st, d, blocks, pcg_maxit, pcg_tol, ir_tol,
                     ir_maxit);
}

}  // namespace rpba
