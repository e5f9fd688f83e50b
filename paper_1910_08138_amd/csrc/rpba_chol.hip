// Batched tiled Cholesky of the reduced camera systems of all sub-blocks
// (paper Sec. 2: the RCS is solved by Cholesky factorisation instead of being
// inverted), with the forward substitution folded into the factorisation and
// a tiled backward substitution.
//
// Storage per sub-block: the lower triangle of S in T x T tiles (tile (i, j),
// i >= j, at (i (i + 1) / 2 + j) T^2, in-tile layout mf_idx), padded to nt T
// with an identity block, followed by one more tile row i = nt whose row 0
// holds the right-hand side e^T.  Factorising the augmented matrix turns that
// row into (L^-1 e)^T: the forward substitution comes for free.
//
// Right-looking schedule, three launches per step k for all sub-blocks:
//   potrf  (l):          L(k,k) and L(k,k)^-1 of the diagonal tile, one
//                        workgroup per sub-block, tile held in registers;
//   trsm   (l, i, k):    L(i,k) = A(i,k) L(k,k)^-T, k < i <= nt;
//   update (l, i, j):    A(i,j) -= L(i,k) L(j,k)^T, k < j <= i, j < nt.
// The tile products run on the FP64 matrix cores (v_mfma_f64_16x16x4) with
// operands read straight from memory in the matrix-core layout.
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

// acc += A B^T for T x T tiles stored in the matrix-core layout
template <int T>
__device__ __forceinline__ void gemm_nt_mf(const double* __restrict__ A, const double* __restrict__ B, Acc<T>& acc) {
  constexpr int NB = T / 32;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rb0 = (wv >> 1) * NB, cb0 = (wv & 1) * NB;
#pragma unroll 4
  for (int kg = 0; kg < T / 4; ++kg) {
    double a[NB], b[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      a[q] = A[((rb0 + q) * (T / 4) + kg) * 64 + lane];
      b[q] = B[((cb0 + q) * (T / 4) + kg) * 64 + lane];
    }
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int q = 0; q < NB; ++q) acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc.v[p][q], 0, 0, 0);
  }
}

template <int T>
__device__ __forceinline__ double* tile_ptr(const Dev& d, int l, int i, int j) {
  return d.S + d.rcs_off[l] + ((int64_t)i * (i + 1) / 2 + j) * (int64_t)T * T;
}

// Diagonal tile of step k: Cholesky factor and its inverse.  The 256 threads
// form a 16 x 16 grid, each holding a B x B block (B = T / 16) of the tile in
// registers; one column (resp. row) is broadcast through LDS per step.
template <int T>
__global__ __launch_bounds__(NT) void k_chol_potrf(Dev d, int k, const int32_t* __restrict__ items) {
  constexpr int B = T / 16;
  __shared__ double Lsh[T][T + 1];
  __shared__ double rowx[T];
  __shared__ double piv;
  __shared__ int fail;
  const int l = items[blockIdx.x] >> 16;
  if (d.active && !d.active[l]) return;
  const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
  const double* A = tile_ptr<T>(d, l, k, k);
  double a[B][B];
#pragma unroll
  for (int rr = 0; rr < B; ++rr)
#pragma unroll
    for (int ss = 0; ss < B; ++ss) a[rr][ss] = A[mf_idx(T, ti * B + rr, tj * B + ss)];
  if (threadIdx.x == 0) fail = 0;
  // right-looking factorisation; per column one pivot broadcast and one
  // column broadcast through LDS, updates as predicated multiply-adds (no
  // divergent branches: entries outside the active part are masked to zero
  // or left untouched by selects)
  for (int cb = 0; cb < 16; ++cb) {
#pragma unroll
    for (int cc = 0; cc < B; ++cc) {
      const int c = cb * B + cc;
      if (threadIdx.x == cb * 16 + cb) {
        double dv = a[cc][cc];
        if (!(dv > 0.0)) {
          fail = 1;
          dv = 1.0;
        }
        piv = sqrt(dv);
      }
      __syncthreads();
      const double p = piv;
      const double ip = 1.0 / p;
      if (tj == cb) {
#pragma unroll
        for (int rr = 0; rr < B; ++rr) {
          const int r = ti * B + rr;
          const double v = a[rr][cc];
          const double nv = r > c ? v * ip : (r == c ? p : v);
          a[rr][cc] = nv;
          Lsh[r][c] = nv;
        }
      }
      __syncthreads();
      double ls[B];
#pragma unroll
      for (int ss = 0; ss < B; ++ss) {
        const int s = tj * B + ss;
        ls[ss] = s > c ? Lsh[s][c] : 0.0;
      }
#pragma unroll
      for (int rr = 0; rr < B; ++rr) {
        const int r = ti * B + rr;
        const double lr = r > c ? Lsh[r][c] : 0.0;
#pragma unroll
        for (int ss = 0; ss < B; ++ss) a[rr][ss] -= lr * ls[ss];
      }
    }
  }
  __syncthreads();
  // inverse X = L^-1 by a right-looking forward substitution on X = I
  double x[B][B];
#pragma unroll
  for (int rr = 0; rr < B; ++rr)
#pragma unroll
    for (int ss = 0; ss < B; ++ss) x[rr][ss] = (ti * B + rr == tj * B + ss) ? 1.0 : 0.0;
  for (int cb = 0; cb < 16; ++cb) {
#pragma unroll
    for (int cc = 0; cc < B; ++cc) {
      const int c = cb * B + cc;
      if (ti == cb) {
        const double inv = 1.0 / Lsh[c][c];
#pragma unroll
        for (int ss = 0; ss < B; ++ss) {
          x[cc][ss] *= inv;
          rowx[tj * B + ss] = x[cc][ss];
        }
      }
      __syncthreads();
      double xs[B];
#pragma unroll
      for (int ss = 0; ss < B; ++ss) xs[ss] = rowx[tj * B + ss];
#pragma unroll
      for (int rr = 0; rr < B; ++rr) {
        const int r = ti * B + rr;
        const double lr = r > c ? Lsh[r][c] : 0.0;
#pragma unroll
        for (int ss = 0; ss < B; ++ss) x[rr][ss] -= lr * xs[ss];
      }
      __syncthreads();
    }
  }
  double* Li = d.Li + d.diag_off[l] + (int64_t)k * T * T;
#pragma unroll
  for (int rr = 0; rr < B; ++rr)
#pragma unroll
    for (int ss = 0; ss < B; ++ss) Li[mf_idx(T, ti * B + rr, tj * B + ss)] = x[rr][ss];
  if (threadIdx.x == 0 && fail) d.blk_fail[l] = 1;
}

// L(i,k) = A(i,k) L(k,k)^-T, in place (the right-hand-side row i = nt included)
template <int T>
__global__ __launch_bounds__(NT) void k_chol_trsm(Dev d, int k, const int32_t* __restrict__ items) {
  const int it = items[blockIdx.x];
  const int l = it >> 16, i = (it >> 8) & 255;
  if (d.active && !d.active[l]) return;
  double* Aik = tile_ptr<T>(d, l, i, k);
  const double* Li = d.Li + d.diag_off[l] + (int64_t)k * T * T;
  Acc<T> acc;
  acc.zero();
  gemm_nt_mf<T>(Aik, Li, acc);
  __syncthreads();  // every wave has read A(i,k) before it is overwritten
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        Aik[mf_idx(T, r, c)] = acc.v[p][q][e];
      }
}

// Trailing update A(i,j) -= L(i,k) L(j,k)^T.  Each wave owns a (T/2) x (T/2)
// quadrant; no LDS.
template <int T>
__global__ __launch_bounds__(NT) void k_chol_update(Dev d, int k, const int32_t* __restrict__ items) {
  const int it = items[blockIdx.x];
  const int l = it >> 16, i = (it >> 8) & 255, j = it & 255;
  if (d.active && !d.active[l]) return;
  const double* Aik = tile_ptr<T>(d, l, i, k);
  const double* Ajk = tile_ptr<T>(d, l, j, k);
  double* C = tile_ptr<T>(d, l, i, j);
  Acc<T> acc;
  acc.zero();
  gemm_nt_mf<T>(Aik, Ajk, acc);
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        C[mf_idx(T, r, c)] -= acc.v[p][q][e];
      }
}

// ys = L^-1 e: row 0 of the factored right-hand-side tile row
template <int T>
__global__ void k_rhs_extract(Dev d) {
  const int l = blockIdx.x;
  if (d.active && !d.active[l]) return;
  const int nt = d.nt[l];
  const int64_t vb = d.vec_off[l];
  for (int t = threadIdx.x; t < nt * T; t += blockDim.x) {
    const int k = t / T, c = t % T;
    d.ys[vb + t] = tile_ptr<T>(d, l, nt, k)[mf_idx(T, 0, c)];
  }
}

// backward substitution step k: x_k = L(k,k)^-T z_k; z_j -= L(k,j)^T x_k.
// P = 256 / T threads share each output element (strided partial sums,
// reduced with lane shuffles).
template <int T>
__global__ __launch_bounds__(NT) void k_chol_backward(Dev d, const int32_t* __restrict__ items) {
  constexpr int P = NT / T;
  __shared__ double zk[T], xk[T];
  const int it = items[blockIdx.x];
  const int l = it >> 16, k = (it >> 8) & 255, j = it & 255;
  if (d.active && !d.active[l]) return;
  const int64_t vb = d.vec_off[l];
  for (int t = threadIdx.x; t < T; t += NT) zk[t] = d.ys[vb + (int64_t)k * T + t];
  __syncthreads();
  const int r = threadIdx.x / P, part = threadIdx.x % P;
  const double* Li = d.Li + d.diag_off[l] + (int64_t)k * T * T;
  double s = 0.0;
#pragma unroll
  for (int m0 = 0; m0 < T; m0 += P) {
    const int m = m0 + part;
    s += m >= r ? Li[mf_idx(T, m, r)] * zk[m] : 0.0;
  }
#pragma unroll
  for (int o = 1; o < P; o <<= 1) s += __shfl_xor(s, o);
  if (part == 0) xk[r] = s;
  __syncthreads();
  if (j == k) {
    for (int t = threadIdx.x; t < T; t += NT) d.x[vb + (int64_t)k * T + t] = xk[t];
    return;
  }
  const double* Lkj = tile_ptr<T>(d, l, k, j);
  double u = 0.0;
#pragma unroll
  for (int m0 = 0; m0 < T; m0 += P) {
    const int m = m0 + part;
    u += Lkj[mf_idx(T, m, r)] * xk[m];
  }
#pragma unroll
  for (int o = 1; o < P; o <<= 1) u += __shfl_xor(u, o);
  if (part == 0) d.ys[vb + (int64_t)j * T + r] -= u;
}

// C = A B^T for row-major 64 x 64 tiles through the matrix-core tile product
__global__ __launch_bounds__(NT) void k_selftest_gemm(const double* A, const double* B, double* C) {
  constexpr int T = 64;
  extern __shared__ double sm[];
  double* a = sm;
  double* b = sm + T * T;
  for (int e = threadIdx.x; e < T * T; e += NT) {
    const int r = e / T, c = e % T;
    a[mf_idx(T, r, c)] = A[e];
    b[mf_idx(T, r, c)] = B[e];
  }
  __syncthreads();
  Acc<T> acc;
  acc.zero();
  gemm_nt_mf<T>(a, b, acc);
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

}  // namespace

void launch_chol_step(const Dev& d, int k, const int32_t* pot, int64_t npot, const int32_t* trsm, int64_t ntrsm,
                      const int32_t* upd, int64_t nupd, hipStream_t st) {
  if (d.T == 64) {
    if (npot) hipLaunchKernelGGL(k_chol_potrf<64>, dim3((unsigned)npot), dim3(NT), 0, st, d, k, pot);
    if (ntrsm) hipLaunchKernelGGL(k_chol_trsm<64>, dim3((unsigned)ntrsm), dim3(NT), 0, st, d, k, trsm);
    if (nupd) hipLaunchKernelGGL(k_chol_update<64>, dim3((unsigned)nupd), dim3(NT), 0, st, d, k, upd);
  } else {
    if (npot) hipLaunchKernelGGL(k_chol_potrf<32>, dim3((unsigned)npot), dim3(NT), 0, st, d, k, pot);
    if (ntrsm) hipLaunchKernelGGL(k_chol_trsm<32>, dim3((unsigned)ntrsm), dim3(NT), 0, st, d, k, trsm);
    if (nupd) hipLaunchKernelGGL(k_chol_update<32>, dim3((unsigned)nupd), dim3(NT), 0, st, d, k, upd);
  }
}

void launch_rhs_extract(const Dev& d, hipStream_t st) {
  if (d.T == 64) hipLaunchKernelGGL(k_rhs_extract<64>, dim3(d.L), dim3(NT), 0, st, d);
  else hipLaunchKernelGGL(k_rhs_extract<32>, dim3(d.L), dim3(NT), 0, st, d);
}

void launch_chol_backward(const Dev& d, const int32_t* items, int64_t n_items, hipStream_t st) {
  if (n_items <= 0) return;
  if (d.T == 64)
    hipLaunchKernelGGL(k_chol_backward<64>, dim3((unsigned)n_items), dim3(NT), 0, st, d, items);
  else
    hipLaunchKernelGGL(k_chol_backward<32>, dim3((unsigned)n_items), dim3(NT), 0, st, d, items);
}

void launch_selftest_gemm(const double* A, const double* B, double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_selftest_gemm, dim3(1), dim3(NT), 2 * 64 * 64 * sizeof(double), st, A, B, C);
}

}  // namespace rpba
