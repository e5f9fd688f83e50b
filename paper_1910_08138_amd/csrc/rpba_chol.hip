// Batched tiled Cholesky of the reduced camera systems of all sub-blocks
// (paper Sec. 2: the RCS is solved by Cholesky factorisation instead of being
// inverted), with the forward substitution of the right-hand side folded into
// the factorisation and a tiled backward substitution.
//
// Storage per sub-block: the lower triangle of S in T x T tiles (tile (i, j),
// i >= j, row-major inside, at (i (i + 1) / 2 + j) T^2), padded to nt T with
// an identity block.  Off-diagonal factor tiles overwrite S in place; the
// diagonal factor L(k,k) and its inverse go to separate arrays.
//
// Right-looking schedule, one launch per panel step k for all sub-blocks at
// once.  Launch k holds
//   * panel items (l, i, k), i >= k: apply the step k-1 update to A(k,k) and
//     A(i,k) in registers, factor A(k,k) in LDS (each item redundantly),
//     invert it, L(i,k) = A(i,k) L(k,k)^-T as a tile product, and
//     y_i -= L(i,k) L(k,k)^-1 y_k;
//   * update items (l, i, j), k < j <= i: A(i,j) -= L(i,k-1) L(j,k-1)^T.
// Every tile product runs on the FP64 matrix cores (v_mfma_f64_16x16x4).
// Backward launch k: x_k = L(k,k)^-T z_k, z_j -= L(k,j)^T x_k for j < k.
#include "rpba_internal.hpp"

namespace rpba {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int NT = 256;

template <int T>
struct Acc {
  static constexpr int NB = T / 32;  // 16x16 blocks per wave side
  v4d v[NB][NB];
  __device__ void zero() {
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int q = 0; q < NB; ++q) v[p][q] = v4d{0.0, 0.0, 0.0, 0.0};
  }
};

// Row / column of component e of block (p, q) held by this lane.  The 4
// waves split the tile in quadrants; inside a 16x16 block the FP64
// matrix-core result puts component e of lane l at (l / 16 + 4 e, l % 16).
template <int T>
__device__ __forceinline__ void acc_rc(int p, int q, int e, int& r, int& c) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  r = (wv >> 1) * (T / 2) + 16 * p + (lane >> 4) + 4 * e;
  c = (wv & 1) * (T / 2) + 16 * q + (lane & 15);
}

// acc += A B^T for T x T tiles in LDS (row stride T + 2)
template <int T>
__device__ __forceinline__ void gemm_nt(const double* __restrict__ A, const double* __restrict__ B, Acc<T>& acc) {
  constexpr int LD = T + 2;
  constexpr int NB = T / 32;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = (wv >> 1) * (T / 2), c0 = (wv & 1) * (T / 2);
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < T; k += 4) {
    double a[NB], b[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      a[q] = A[(r0 + 16 * q + lr) * LD + k + lk];
      b[q] = B[(c0 + 16 * q + lr) * LD + k + lk];
    }
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int q = 0; q < NB; ++q) acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc.v[p][q], 0, 0, 0);
  }
}

template <int T>
__device__ __forceinline__ void load_tile(const double* __restrict__ g, double* s) {
  constexpr int LD = T + 2;
  for (int e = threadIdx.x; e < T * T; e += NT) s[(e / T) * LD + (e % T)] = g[e];
}

// s = g - acc (element-wise), g global tile, s LDS
template <int T>
__device__ __forceinline__ void store_diff(const double* __restrict__ g, const Acc<T>& acc, double* s) {
  constexpr int LD = T + 2;
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        s[r * LD + c] = g[r * T + c] - acc.v[p][q][e];
      }
}

// Left-looking Cholesky of the lower triangle of an LDS tile; sets *fail on a
// non-positive pivot (the pivot is then replaced by 1 to keep values finite).
template <int T>
__device__ void potrf_lds(double* D, int* fail) {
  constexpr int LD = T + 2;
  constexpr int P = NT / T;  // threads per row
  const int r = threadIdx.x / P, p = threadIdx.x % P;
  for (int c = 0; c < T; ++c) {
    double s = 0.0;
    if (r >= c)
      for (int m = p; m < c; m += P) s += D[r * LD + m] * D[c * LD + m];
#pragma unroll
    for (int o = 1; o < P; o <<= 1) s += __shfl_xor(s, o);
    if (r == c && p == 0) {
      double dv = D[c * LD + c] - s;
      if (!(dv > 0.0)) {
        *fail = 1;
        dv = 1.0;
      }
      D[c * LD + c] = sqrt(dv);
    }
    __syncthreads();
    if (r > c && p == 0) D[r * LD + c] = (D[r * LD + c] - s) / D[c * LD + c];
    __syncthreads();
  }
}

// G = L^-1 (lower) from the lower triangle of L, both LDS tiles
template <int T>
__device__ void trtri_lds(const double* Lt, double* G) {
  constexpr int LD = T + 2;
  constexpr int P = NT / T;
  const int j = threadIdx.x / P, p = threadIdx.x % P;
  for (int e = threadIdx.x; e < T * T; e += NT) G[(e / T) * LD + (e % T)] = 0.0;
  __syncthreads();
  for (int r = 0; r < T; ++r) {
    if (j < r) {
      double s = 0.0;
      for (int m = j + p; m < r; m += P) s += Lt[r * LD + m] * G[m * LD + j];
#pragma unroll
      for (int o = 1; o < P; o <<= 1) s += __shfl_xor(s, o);
      if (p == 0) G[r * LD + j] = -s / Lt[r * LD + r];
    } else if (j == r && p == 0) {
      G[r * LD + r] = 1.0 / Lt[r * LD + r];
    }
    __syncthreads();
  }
}

template <int T>
__global__ __launch_bounds__(NT) void k_chol_forward(Dev d, int k, const int32_t* __restrict__ items) {
  constexpr int LD = T + 2;
  constexpr int64_t T2 = (int64_t)T * T;
  extern __shared__ double sm[];
  double* bA = sm;                 // L(i,k-1), then A(i,k) updated, then L(i,k)
  double* bB = sm + T * LD;        // L(k,k-1), then A(k,k) updated and factored
  double* bG = sm + 2 * T * LD;    // L(k,k)^-1
  double* yv = sm + 3 * T * LD;    // [T] y_k
  double* ysv = yv + T;            // [T] L(k,k)^-1 y_k
  __shared__ int fail;

  const int it = items[blockIdx.x];
  const int l = it >> 16, i = (it >> 8) & 255, j = it & 255;
  if (d.active && !d.active[l]) return;
  const int64_t base = d.rcs_off[l];
  auto tile = [&](int ti, int tj) { return d.S + base + ((int64_t)ti * (ti + 1) / 2 + tj) * T2; };

  if (j > k) {
    // trailing update of step k-1
    load_tile<T>(tile(i, k - 1), bA);
    load_tile<T>(tile(j, k - 1), bB);
    __syncthreads();
    Acc<T> acc;
    acc.zero();
    gemm_nt<T>(bA, bB, acc);
    double* C = tile(i, j);
#pragma unroll
    for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
      for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int r, c;
          acc_rc<T>(p, q, e, r, c);
          C[r * T + c] -= acc.v[p][q][e];
        }
    return;
  }

  // panel item (l, i, k)
  if (threadIdx.x == 0) fail = 0;
  if (k > 0) {
    load_tile<T>(tile(k, k - 1), bB);
    if (i > k) load_tile<T>(tile(i, k - 1), bA);
    __syncthreads();
    Acc<T> accD, accO;
    accD.zero();
    gemm_nt<T>(bB, bB, accD);
    if (i > k) {
      accO.zero();
      gemm_nt<T>(bA, bB, accO);
    }
    __syncthreads();
    store_diff<T>(tile(k, k), accD, bB);
    if (i > k) store_diff<T>(tile(i, k), accO, bA);
  } else {
    load_tile<T>(tile(k, k), bB);
    if (i > k) load_tile<T>(tile(i, k), bA);
  }
  const int64_t vb = d.vec_off[l];
  for (int t = threadIdx.x; t < T; t += NT) yv[t] = d.y[vb + (int64_t)k * T + t];
  __syncthreads();
  potrf_lds<T>(bB, &fail);
  trtri_lds<T>(bB, bG);
  // ys_k = L(k,k)^-1 y_k
  for (int r = threadIdx.x; r < T; r += NT) {
    double s = 0.0;
    for (int m = 0; m <= r; ++m) s += bG[r * LD + m] * yv[m];
    ysv[r] = s;
  }
  __syncthreads();
  if (i == k) {
    const int64_t db = d.diag_off[l] + (int64_t)k * T2;
    for (int e = threadIdx.x; e < T * T; e += NT) {
      int r = e / T, c = e % T;
      d.Ld[db + e] = c <= r ? bB[r * LD + c] : 0.0;
      d.Li[db + e] = bG[r * LD + c];
    }
    for (int t = threadIdx.x; t < T; t += NT) d.ys[vb + (int64_t)k * T + t] = ysv[t];
    if (threadIdx.x == 0 && fail) d.blk_fail[l] = 1;
    return;
  }
  // L(i,k) = A(i,k) L(k,k)^-T
  Acc<T> accT;
  accT.zero();
  gemm_nt<T>(bA, bG, accT);
  __syncthreads();
  double* Lik = tile(i, k);
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        Lik[r * T + c] = accT.v[p][q][e];
        bA[r * LD + c] = accT.v[p][q][e];
      }
  __syncthreads();
  // y_i -= L(i,k) ys_k
  for (int r = threadIdx.x; r < T; r += NT) {
    double s = 0.0;
    for (int c = 0; c < T; ++c) s += bA[r * LD + c] * ysv[c];
    d.y[vb + (int64_t)i * T + r] -= s;
  }
}

// backward substitution step k: x_k = L(k,k)^-T z_k; z_j -= L(k,j)^T x_k
template <int T>
__global__ __launch_bounds__(NT) void k_chol_backward(Dev d, const int32_t* __restrict__ items) {
  constexpr int64_t T2 = (int64_t)T * T;
  __shared__ double zk[T], xk[T];
  const int it = items[blockIdx.x];
  const int l = it >> 16, k = (it >> 8) & 255, j = it & 255;
  if (d.active && !d.active[l]) return;
  const int64_t vb = d.vec_off[l];
  for (int t = threadIdx.x; t < T; t += NT) zk[t] = d.ys[vb + (int64_t)k * T + t];
  __syncthreads();
  const double* Li = d.Li + d.diag_off[l] + (int64_t)k * T2;
  for (int r = threadIdx.x; r < T; r += NT) {
    double s = 0.0;
    for (int m = r; m < T; ++m) s += Li[(int64_t)m * T + r] * zk[m];
    xk[r] = s;
  }
  __syncthreads();
  if (j == k) {
    for (int t = threadIdx.x; t < T; t += NT) d.x[vb + (int64_t)k * T + t] = xk[t];
    return;
  }
  const double* Lkj = d.S + d.rcs_off[l] + ((int64_t)k * (k + 1) / 2 + j) * T2;
  for (int c = threadIdx.x; c < T; c += NT) {
    double s = 0.0;
    for (int r = 0; r < T; ++r) s += Lkj[(int64_t)r * T + c] * xk[r];
    d.ys[vb + (int64_t)j * T + c] -= s;
  }
}

__global__ __launch_bounds__(NT) void k_selftest_gemm(const double* A, const double* B, double* C) {
  constexpr int T = 64, LD = T + 2;
  extern __shared__ double sm[];
  load_tile<T>(A, sm);
  load_tile<T>(B, sm + T * LD);
  __syncthreads();
  Acc<T> acc;
  acc.zero();
  gemm_nt<T>(sm, sm + T * LD, acc);
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        C[r * T + c] = acc.v[p][q][e];
      }
}

template <int T>
size_t fwd_lds() {
  return (size_t)(3 * T * (T + 2) + 2 * T) * sizeof(double);
}

}  // namespace

void launch_chol_forward(const Dev& d, int k, const int32_t* items, int64_t n_items, hipStream_t st) {
  if (n_items <= 0) return;
  if (d.T == 64)
    hipLaunchKernelGGL(k_chol_forward<64>, dim3((unsigned)n_items), dim3(NT), fwd_lds<64>(), st, d, k, items);
  else
    hipLaunchKernelGGL(k_chol_forward<32>, dim3((unsigned)n_items), dim3(NT), fwd_lds<32>(), st, d, k, items);
}

void launch_chol_backward(const Dev& d, const int32_t* items, int64_t n_items, hipStream_t st) {
  if (n_items <= 0) return;
  if (d.T == 64)
    hipLaunchKernelGGL(k_chol_backward<64>, dim3((unsigned)n_items), dim3(NT), 0, st, d, items);
  else
    hipLaunchKernelGGL(k_chol_backward<32>, dim3((unsigned)n_items), dim3(NT), 0, st, d, items);
}

void launch_selftest_gemm(const double* A, const double* B, double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_selftest_gemm, dim3(1), dim3(NT), 2 * 64 * 66 * sizeof(double), st, A, B, C);
}

}  // namespace rpba
