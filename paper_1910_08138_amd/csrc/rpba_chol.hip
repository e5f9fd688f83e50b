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

#include <algorithm>

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

// acc += A B^T for T x T tiles stored in the matrix-core layout.  Every
// operand fragment of the wave is loaded before the first product, so the
// tile costs one memory latency rather than one per k step.
template <int T, bool NEG = false>
__device__ __forceinline__ void gemm_nt_mf(const double* __restrict__ A, const double* __restrict__ B, Acc<T>& acc) {
  constexpr int NB = T / 32, KG = T / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rb0 = (wv >> 1) * NB, cb0 = (wv & 1) * NB;
  double a[KG][NB], b[KG][NB];
#pragma unroll
  for (int kg = 0; kg < KG; ++kg)
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      a[kg][q] = NEG ? -A[((rb0 + q) * (T / 4) + kg) * 64 + lane] : A[((rb0 + q) * (T / 4) + kg) * 64 + lane];
      b[kg][q] = B[((cb0 + q) * (T / 4) + kg) * 64 + lane];
    }
  __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the products
#pragma unroll
  for (int kg = 0; kg < KG; ++kg)
#pragma unroll
    for (int p = 0; p < NB; ++p)
#pragma unroll
      for (int q = 0; q < NB; ++q)
        acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kg][p], b[kg][q], acc.v[p][q], 0, 0, 0);
}

// The same product with the k range in four groups, double-buffered: the
// operands of group g + 1 are in flight while group g is multiplied (fewer
// registers than loading everything up front).
// device-coherent element access (relaxed atomics at agent scope): used for
// the tiles that workgroups of one persistent launch hand to each other
__device__ __forceinline__ double coh_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coh_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int T, bool NEG = false, bool COH_A = false, bool COH_B = false>
__device__ __forceinline__ void gemm_nt_mf_pipe(const double* __restrict__ A, const double* __restrict__ B,
                                                Acc<T>& acc) {
  constexpr int NB = T / 32, KG = T / 4, G = 4, KGB = KG / G;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rb0 = (wv >> 1) * NB, cb0 = (wv & 1) * NB;
  double a[2][KGB][NB], b[2][KGB][NB];
  auto load = [&](int g, int buf) {
#pragma unroll
    for (int kk = 0; kk < KGB; ++kk)
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int kg = g * KGB + kk;
        const double* pa = A + ((rb0 + q) * (T / 4) + kg) * 64 + lane;
        const double* pb = B + ((cb0 + q) * (T / 4) + kg) * 64 + lane;
        const double av = COH_A ? coh_load(pa) : *pa;
        a[buf][kk][q] = NEG ? -av : av;
        b[buf][kk][q] = COH_B ? coh_load(pb) : *pb;
      }
  };
  load(0, 0);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g + 1 < G) load(g + 1, (g + 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < KGB; ++kk)
#pragma unroll
      for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int q = 0; q < NB; ++q)
          acc.v[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[g & 1][kk][p], b[g & 1][kk][q], acc.v[p][q], 0, 0, 0);
  }
}

template <int T>
__device__ __forceinline__ double* tile_ptr(const Dev& d, int l, int i, int j) {
  return d.S + d.rcs_off[l] + ((int64_t)i * (i + 1) / 2 + j) * (int64_t)T * T;
}

// ---- diagonal tile: factor and inverse, blocked by 16 inside the tile.
// The tile sits in LDS (row-major, row stride T + 1).  For each 16-wide
// column block kb one wave factors the whole panel below the diagonal
// (lane = row; the pivot is broadcast with readlane, the rest of the step's
// column through one LDS store and broadcast reads, which keeps the scalar
// registers free and the round trip off the chain of pivots) and the trailing blocks are updated on the matrix cores.  The
// 16 x 16 diagonal factor blocks are inverted by one wave each (lane =
// column, forward substitution) and the inverse of the whole factor is
// assembled block row by block row:
//   Linv(i,i) = D_i^-1,  Linv(i,j) = -D_i^-1 sum_{k=j}^{i-1} L(i,k) Linv(k,j).
template <int T>
struct DiagLds {
  static constexpr int LD = T + 1;
  double A[T * LD];         // tile, then its factor (lower blocks)
  double X[T * LD];         // inverse of the factor (lower blocks)
  double Y[4][16 * 17];     // per-wave 16 x 16 staging
  double ipv[T];            // 1 / L(c,c)
  int fail;
};

__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / sqrt(d) for d > 0: hardware estimate and two Newton steps
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * (1.5 - 0.5 * d * y * y);
  y = y * (1.5 - 0.5 * d * y * y);
  return y;
}

// one wave: factor columns o .. o + 15 of rows o .. T - 1 (right-looking
// inside the panel); lane q holds row o + q
template <int T>
__device__ __forceinline__ void factor_panel(DiagLds<T>& sm, int o) {
  constexpr int LD = DiagLds<T>::LD;
  const int lane = threadIdx.x & 63;
  const bool live = o + lane < T;
  const int row = live ? o + lane : T - 1;
  double a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = sm.A[row * LD + o + c];
  // the step's column goes to the other rows through LDS (the wave's own
  // stores are seen by its later loads), one broadcast read per element.
  // The next pivot does not wait for that round trip: lane c + 1 updates its
  // own diagonal entry with its own column value, and the pivot is read from
  // there while the broadcast reads are in flight.
  // The sixteen steps have no branches (a failed pivot and the reciprocal
  // pivots are recorded with selects and stored afterwards), and each step
  // computes the next pivot while its column broadcast is in flight.
  double* colb = sm.Y[0];
  double piv = bcast(a[0], 0);
  bool bad = !(piv > 0.0);
  double dcc = bad ? 1.0 : piv;
  double ip = rsqrt_nr(dcc);
  double myip = 0.0;  // lane c: 1 / L(o + c, o + c)
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    myip = lane == c ? ip : myip;
    const double colv = lane > c ? a[c] * ip : (lane == c ? dcc * ip : 0.0);
    a[c] = colv;
    if (c < 15) {
      const double dn = a[c + 1] - colv * colv;
      colb[lane] = colv;
      double cb[16];
#pragma unroll
      for (int s2 = c + 1; s2 < 16; ++s2) cb[s2] = colb[s2];
      piv = bcast(dn, c + 1);
      const bool nonpos = !(piv > 0.0);  // uniform
      bad = bad || nonpos;
      dcc = nonpos ? 1.0 : piv;
      ip = rsqrt_nr(dcc);
#pragma unroll
      for (int s2 = c + 1; s2 < 16; ++s2) a[s2] -= colv * cb[s2];
    }
  }
  if (lane < 16) sm.ipv[o + lane] = myip;
  if (bad && lane == 0) sm.fail = 1;
  if (live) {
#pragma unroll
    for (int c = 0; c < 16; ++c) sm.A[row * LD + o + c] = a[c];
  }
}

// one wave: X(o.., o..) = inverse of the 16 x 16 factor block at (o, o);
// lane s computes column s
template <int T>
__device__ __forceinline__ void invert16(DiagLds<T>& sm, int o) {
  constexpr int LD = DiagLds<T>::LD;
  const int lane = threadIdx.x & 63, s = lane & 15;
  double x[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    double acc = (t == s) ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < t; ++u) acc -= sm.A[(o + t) * LD + o + u] * x[u];
    x[t] = acc * sm.ipv[o + t];
  }
  if (lane < 16) {
#pragma unroll
    for (int t = 0; t < 16; ++t) sm.X[(o + t) * LD + o + s] = x[t];
  }
}

// acc += P Q^T for 16 x 16 blocks of LDS matrices (row stride LD), P at
// (pr, pc), Q at (qr, qc); `neg` negates P
template <int LD>
__device__ __forceinline__ v4d mf16_nt(const double* P, int pr, int pc, const double* Q, int qr, int qc, v4d acc,
                                       bool neg) {
  const int lane = threadIdx.x & 63;
  const int rr = lane & 15, kk0 = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    double a = P[(pr + rr) * LD + pc + 4 * kk + kk0];
    const double b = Q[(qr + rr) * LD + qc + 4 * kk + kk0];
    if (neg) a = -a;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// acc += P Q for 16 x 16 blocks (P row stride LDP, Q row stride LDQ)
template <int LDP, int LDQ>
__device__ __forceinline__ v4d mf16_nn(const double* P, int pr, int pc, const double* Q, int qr, int qc, v4d acc) {
  const int lane = threadIdx.x & 63;
  const int rr = lane & 15, kk0 = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const double a = P[(pr + rr) * LDP + pc + 4 * kk + kk0];
    const double b = Q[(qr + 4 * kk + kk0) * LDQ + qc + rr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

template <int LD>
__device__ __forceinline__ v4d ld16(const double* P, int pr, int pc) {
  const int lane = threadIdx.x & 63;
  v4d v;
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = P[(pr + (lane >> 4) + 4 * e) * LD + pc + (lane & 15)];
  return v;
}

template <int LD>
__device__ __forceinline__ void st16(double* P, int pr, int pc, v4d v, bool neg) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; ++e) P[(pr + (lane >> 4) + 4 * e) * LD + pc + (lane & 15)] = neg ? -v[e] : v[e];
}

// block (r, j), j < r, of the inverse of the factor, from the blocks of the
// rows above it and the inverse diagonal block of row r:
//   Linv(r,j) = -D_r^-1 sum_{k=j}^{r-1} L(r,k) Linv(k,j)   (one wave)
template <int T>
__device__ __forceinline__ void inverse_block(DiagLds<T>& sm, int r, int j) {
  constexpr int LD = DiagLds<T>::LD;
  const int wv = threadIdx.x >> 6;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int k = j; k < r; ++k) acc = mf16_nn<LD, LD>(sm.A, 16 * r, 16 * k, sm.X, 16 * k, 16 * j, acc);
  st16<17>(sm.Y[wv], 0, 0, acc, false);
  v4d y = {0.0, 0.0, 0.0, 0.0};
  y = mf16_nn<LD, 17>(sm.X, 16 * r, 16 * r, sm.Y[wv], 0, 0, y);
  st16<LD>(sm.X, 16 * r, 16 * j, y, true);
}

// Factor sm.A (T x T, lower part used) and leave L^-1 in sm.X (lower blocks
// valid, diagonal blocks lower triangular).  All threads of the workgroup.
// Wave 0 factors the 16-wide panels one after the other; while it does, the
// other waves build the inverse of what is already factored: wave 1 inverts
// the diagonal block of the previous panel, waves 2 and 3 the block row two
// panels back (it needs that row's inverted diagonal block).  What is left at
// the end is the last diagonal block and the last two block rows.
template <int T>
__device__ void factor_inverse_tile(DiagLds<T>& sm) {
  constexpr int LD = DiagLds<T>::LD, NBK = T / 16;
  const int wv = threadIdx.x >> 6;
  for (int kb = 0; kb < NBK; ++kb) {
    const int o = 16 * kb;
    if (wv == 0) {
      factor_panel<T>(sm, o);
    } else if (wv == 1) {
      if (kb >= 1) invert16<T>(sm, o - 16);
    } else {
      for (int j = wv - 2; j < kb - 2; j += 2) inverse_block<T>(sm, kb - 2, j);
    }
    __syncthreads();
    // trailing update A(ib,jb) -= L(ib,kb) L(jb,kb)^T, kb < jb <= ib
    const int m = NBK - 1 - kb;
    if (m > 0) {
      for (int t = wv; t < m * (m + 1) / 2; t += 4) {
        int ib = 0;
        while ((ib + 1) * (ib + 2) / 2 <= t) ++ib;
        const int jb = t - ib * (ib + 1) / 2;
        const int I = 16 * (kb + 1 + ib), J = 16 * (kb + 1 + jb);
        v4d acc = ld16<LD>(sm.A, I, J);
        acc = mf16_nt<LD>(sm.A, I, o, sm.A, J, o, acc, true);
        st16<LD>(sm.A, I, J, acc, false);
      }
      __syncthreads();
    }
  }
  if (wv == 0) {
    invert16<T>(sm, 16 * (NBK - 1));
  } else {
    for (int j = wv - 1; j < NBK - 2; j += 3) inverse_block<T>(sm, NBK - 2, j);
  }
  __syncthreads();
  for (int j = wv; j < NBK - 1; j += 4) inverse_block<T>(sm, NBK - 1, j);
  __syncthreads();
}

// Diagonal tile of step k: the inverse of its Cholesky factor (the factor
// itself is not needed: the panel solves and the backward substitution use
// the inverse).  One workgroup per sub-block.
template <int T>
__global__ __launch_bounds__(NT) void k_chol_potrf(Dev d, int k, const int32_t* __restrict__ items) {
  constexpr int LD = DiagLds<T>::LD;
  __shared__ DiagLds<T> sm;
  const int l = items[blockIdx.x] >> 16;
  if (d.active && !d.active[l]) return;
  const double* A = tile_ptr<T>(d, l, k, k);
  if (threadIdx.x == 0) sm.fail = 0;
  for (int idx = threadIdx.x; idx < T * T; idx += NT) {
    const int blk = idx >> 6, w = idx & 63;
    const int r = (blk / (T / 4)) * 16 + (w & 15), c = (blk % (T / 4)) * 4 + (w >> 4);
    sm.A[r * LD + c] = A[idx];
  }
  __syncthreads();
  factor_inverse_tile<T>(sm);
  double* Li = d.Li + d.diag_off[l] + (int64_t)k * T * T;
  for (int idx = threadIdx.x; idx < T * T; idx += NT) {
    const int blk = idx >> 6, w = idx & 63;
    const int r = (blk / (T / 4)) * 16 + (w & 15), c = (blk % (T / 4)) * 4 + (w >> 4);
    Li[idx] = r >= c ? sm.X[r * LD + c] : 0.0;
  }
  if (threadIdx.x == 0 && sm.fail) d.blk_fail[l] = 1;
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
  // acc = C - L(i,k) L(j,k)^T, C read with the operands
  Acc<T> acc;
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        acc.v[p][q][e] = C[mf_idx(T, r, c)];
      }
  gemm_nt_mf<T, true>(Aik, Ajk, acc);
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        C[mf_idx(T, r, c)] = acc.v[p][q][e];
      }
}

// ys = L^-1 e: row 0 of the factored right-hand-side tile row.  A wait of
// the persistent forward launch that ran out of budget (ctl[2], never set by
// the stepwise launches) marks every sub-block failed.
template <int T>
__global__ void k_rhs_extract(Dev d, const int* ctl) {
  const int l = blockIdx.x;
  if (threadIdx.x == 0 && ctl[2] != 0) d.blk_fail[l] = 1;
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


// ---- one persistent launch for the whole forward factorisation ----------
// Every tile (i, j), j <= i, j < nt, of every dense sub-block that can be
// nonzero in the factor (the right-hand-side row i = nt included) is one
// task.  The plan lists the tasks (dataflow_order: by latest start along
// the chain of diagonal tiles, in a topological order), so a task only ever
// waits for tasks listed before it: the tiles (i,k), (j,k), k < j, that are
// both nonzero, and for j < i the diagonal tile (j,j).  Workgroups take
// list positions from a ticket counter, so a task being waited for is always
// held by a running workgroup and the launch cannot deadlock.  A finished
// tile publishes a ready flag equal to the call's epoch; waits are bounded,
// and a wait that runs out of its budget is counted as an error (the
// sub-blocks are then reported as failed instead of hanging).
//
// Left-looking per tile: acc = A(i,j) - sum_k L(i,k) L(j,k)^T in registers
// (tiles that stay zero left out), then for i == j the diagonal factor and
// its inverse, for i > j the panel solve L(i,j) = acc L(j,j)^-T.
constexpr int DF_SPIN_LIMIT = 1 << 20;

__device__ __forceinline__ int df_flag_load(const int* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// thread 0 waits for the flags; the workgroup then reads the tiles with
// device-coherent loads
__device__ __forceinline__ void df_wait(const int* f1, const int* f2, int epoch, int* err) {
  if (threadIdx.x == 0) {
    int spins = 0;
    // an exhausted wait anywhere ends all later waits at once, so a broken
    // dependency costs one wait budget, not one per task
    while ((df_flag_load(f1) != epoch || (f2 && df_flag_load(f2) != epoch)) && df_flag_load(err) == 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > DF_SPIN_LIMIT) {
        atomicAdd(err, 1);
        break;
      }
    }
  }
  __syncthreads();
}

// the tile was written with device-coherent stores: every wave waits until
// its stores are complete, then thread 0 sets the flag
__device__ __forceinline__ void df_publish(int* f, int epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wave 0 checks the flags of columns k .. min(j, k + 64) - 1 of tile rows
// r1 and r2 (r2 < 0: r1 only) at once; returns (to every thread) the first
// column that is not ready yet, or j.  A column whose product has a tile
// that stays zero (nz1, nz2: the rows' nonzero-tile flags) counts as ready.
__device__ __forceinline__ int df_poll(const int* row1, const int* row2, const uint8_t* nz1, const uint8_t* nz2, int k,
                                       int j, int epoch, int* sh) {
  if (threadIdx.x < 64) {
    const int kk = k + threadIdx.x;
    bool ready = true;
    if (kk < j && nz1[kk] && nz2[kk])
      ready = df_flag_load(row1 + kk) == epoch && (row2 == nullptr || df_flag_load(row2 + kk) == epoch);
    const unsigned long long not_ready = __ballot(!ready);
    if (threadIdx.x == 0) *sh = not_ready ? k + __ffsll((long long)not_ready) - 1 : min(j, k + 64);
  }
  __syncthreads();
  const int r = *sh;
  __syncthreads();
  return r;
}

// ctl = [forward ticket, epoch, exhausted waits, backward ticket].  The
// launches of one LM step share an epoch; the step's last kernel
// (k_df_finish) marks every sub-block failed if a wait ran out, then readies
// ctl for the next step (tickets 0, next epoch, no errors).  k_df_reset
// readies it once after the workspace is zeroed.
__global__ void k_df_reset(int* ctl) {
  if (threadIdx.x == 0) {
    ctl[0] = 0;
    ctl[1] = ctl[1] + 1;
    ctl[2] = 0;
    ctl[3] = 0;
  }
}

// one workgroup
__global__ void k_df_finish(Dev d, int* ctl) {
  const bool err = ctl[2] != 0;
  for (int l = threadIdx.x; l < d.L; l += blockDim.x)
    if (err) d.blk_fail[l] = 1;
  __syncthreads();  // every thread has read the error word
  if (threadIdx.x == 0) {
    ctl[0] = 0;
    ctl[1] = ctl[1] + 1;
    ctl[2] = 0;
    ctl[3] = 0;
  }
}

// A nonzero sub-diagonal tile (j, j-1) of the factor is solved by the task
// of diagonal tile j: its own task only sums its products and publishes the
// partial sums (second half of the flag array); the diagonal task solves it
// with the inverse of diagonal tile j-1, publishes it, and subtracts its
// product from its own sums in LDS.  One hand-over through memory less on
// the chain diagonal (j-1) -> tile (j, j-1) -> diagonal (j).
template <int T>
__global__ __launch_bounds__(NT, 2) void k_chol_dataflow(Dev d, const int32_t* __restrict__ tasks, int ntask, int* flags,
                                                      int64_t nflags, int* ctl) {
  constexpr int LD = DiagLds<T>::LD;
  __shared__ DiagLds<T> sm;
  __shared__ int s_task, s_poll;
  const int epoch = ctl[1];
  int* err = ctl + 2;
  int* pflags = flags + nflags;
  for (;;) {
    __syncthreads();  // the previous task is done with s_task and LDS
    if (threadIdx.x == 0) s_task = atomicAdd(ctl, 1);
    __syncthreads();
    const int t = s_task;
    if (t >= ntask) break;
    const int it = tasks[t];
    const int l = it >> 16, i = (it >> 8) & 255, j = it & 255;
    if (d.active && !d.active[l]) continue;
    const int64_t tile0 = d.rcs_off[l] / (T * T);
    auto fl = [&](int r, int c) { return flags + tile0 + (int64_t)r * (r + 1) / 2 + c; };
    auto pfl = [&](int r, int c) { return pflags + tile0 + (int64_t)r * (r + 1) / 2 + c; };
    double* C = tile_ptr<T>(d, l, i, j);
    Acc<T> acc;
#pragma unroll
    for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
      for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int r, c;
          acc_rc<T>(p, q, e, r, c);
          acc.v[p][q][e] = C[mf_idx(T, r, c)];
        }
    // tiles (i,k) and (j,k) of the row: flags of row r start at fl(r, 0);
    // products with a tile that stays zero are left out
    const uint8_t* nzi = d.tile_nz + tile0 + (int64_t)i * (i + 1) / 2;
    const uint8_t* nzj = d.tile_nz + tile0 + (int64_t)j * (j + 1) / 2;
    const int nt = d.nt[l];
    const bool partial = i == j + 1 && i < nt && nzi[j];  // sub-diagonal tile: products only
    const bool fused = i == j && j >= 1 && nzj[j - 1];     // diagonal task that solves (j, j-1)
    const int kend = fused ? j - 1 : j;
    int kready = 0;  // every k < kready is known to be ready
    for (int k = 0; k < kend; ++k) {
      if (!nzi[k] || !nzj[k]) continue;
      if (k >= kready) {
        kready = df_poll(fl(i, 0), i == j ? nullptr : fl(j, 0), nzi, nzj, k, kend, epoch, &s_poll);
        if (kready == k) {
          df_wait(fl(i, k), i == j ? nullptr : fl(j, k), epoch, err);
          kready = k + 1;
        }
      }
      gemm_nt_mf_pipe<T, true, true, true>(tile_ptr<T>(d, l, i, k), tile_ptr<T>(d, l, j, k), acc);
    }
    if (partial) {
      // the partial sums of tile (i, j), for the diagonal task i
#pragma unroll
      for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
        for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int r, c;
            acc_rc<T>(p, q, e, r, c);
            coh_store(C + mf_idx(T, r, c), acc.v[p][q][e]);
          }
      df_publish(pfl(i, j), epoch);
      continue;
    }
    if (i == j) {
      // diagonal: factor and inverse through LDS
      if (threadIdx.x == 0) sm.fail = 0;
#pragma unroll
      for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
        for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int r, c;
            acc_rc<T>(p, q, e, r, c);
            sm.A[r * LD + c] = acc.v[p][q][e];
          }
      if (fused) {
        // tile (j, j-1), its sums already in LDS as the diagonal's are:
        // the partial sums staged (matrix-core layout), solved with the
        // inverse of diagonal tile j-1, stored and published; then
        // A(j,j) -= L(j,j-1) L(j,j-1)^T from the copy in LDS
        double* Cs = tile_ptr<T>(d, l, j, j - 1);
        // the partial sums are usually ready long before diagonal tile j-1:
        // staged first, so that only the solve waits for it
        df_wait(pfl(j, j - 1), nullptr, epoch, err);
        for (int idx = threadIdx.x; idx < T * T; idx += NT) sm.X[idx] = coh_load(Cs + idx);
        df_wait(fl(j - 1, j - 1), nullptr, epoch, err);  // (its barrier also orders the LDS stores)
        const double* Lim = d.Li + d.diag_off[l] + (int64_t)(j - 1) * T * T;
        Acc<T> out;
        out.zero();
        gemm_nt_mf_pipe<T, false, false, true>(sm.X, Lim, out);
        __syncthreads();  // every wave has read the partial sums
#pragma unroll
        for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
          for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              int r, c;
              acc_rc<T>(p, q, e, r, c);
              coh_store(Cs + mf_idx(T, r, c), out.v[p][q][e]);
              sm.X[mf_idx(T, r, c)] = out.v[p][q][e];
            }
        df_publish(fl(j, j - 1), epoch);  // (its barrier also orders the LDS stores)
        out.zero();
        gemm_nt_mf_pipe<T, true, false, false>(sm.X, sm.X, out);
#pragma unroll
        for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
          for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              int r, c;
              acc_rc<T>(p, q, e, r, c);
              sm.A[r * LD + c] += out.v[p][q][e];
            }
      }
      __syncthreads();
      factor_inverse_tile<T>(sm);
      double* Li = d.Li + d.diag_off[l] + (int64_t)j * T * T;
      for (int idx = threadIdx.x; idx < T * T; idx += NT) {
        const int blk = idx >> 6, w = idx & 63;
        const int r = (blk / (T / 4)) * 16 + (w & 15), c = (blk % (T / 4)) * 4 + (w >> 4);
        coh_store(Li + idx, r >= c ? sm.X[r * LD + c] : 0.0);
      }
      if (threadIdx.x == 0 && sm.fail) d.blk_fail[l] = 1;
      df_publish(fl(j, j), epoch);
    } else {
      // panel solve: L(i,j) = acc Li(j,j)^T with acc staged in LDS in the
      // matrix-core layout
#pragma unroll
      for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
        for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int r, c;
            acc_rc<T>(p, q, e, r, c);
            sm.A[mf_idx(T, r, c)] = acc.v[p][q][e];
          }
      df_wait(fl(j, j), nullptr, epoch, err);  // also orders the LDS stores
      const double* Li = d.Li + d.diag_off[l] + (int64_t)j * T * T;
      Acc<T> out;
      out.zero();
      gemm_nt_mf_pipe<T, false, false, true>(sm.A, Li, out);
#pragma unroll
      for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
        for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int r, c;
            acc_rc<T>(p, q, e, r, c);
            coh_store(C + mf_idx(T, r, c), out.v[p][q][e]);
          }
      df_publish(fl(i, j), epoch);
    }
  }
}


// ---- one persistent launch for the backward substitution ------------------
// Task (l, k) produces x_k = L(k,k)^-T z_k with z_k = y_k - sum_{m > k}
// L(m,k)^T x_m (y = L^-1 e from the forward factorisation).  Tasks are
// numbered by k descending, so a task only waits for tasks with smaller
// numbers; x segments are handed over with device-coherent stores and a ready
// flag per segment (same epoch and error word as the forward launch).
template <int T>
__global__ __launch_bounds__(NT) void k_chol_backward_df(Dev d, const int32_t* __restrict__ tasks, int ntask,
                                                         int* xflags, int* ctl) {
  constexpr int P = NT / T;
  __shared__ double z[T], xm[T];
  __shared__ int s_task;
  const int epoch = ctl[1];
  int* err = ctl + 2;
  const int r = threadIdx.x / P, part = threadIdx.x % P;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_task = atomicAdd(ctl + 3, 1);
    __syncthreads();
    const int t = s_task;
    if (t >= ntask) break;
    const int it = tasks[t];
    const int l = it >> 16, k = (it >> 8) & 255;
    if (d.active && !d.active[l]) continue;
    const int nt = d.nt[l];
    const int64_t vb = d.vec_off[l];
    int* xf = xflags + vb / T;
    for (int q = threadIdx.x; q < T; q += NT) z[q] = d.ys[vb + (int64_t)k * T + q];
    __syncthreads();
    // this thread's columns of L(k,k)^-T, loaded before any wait
    const double* Li = d.Li + d.diag_off[l] + (int64_t)k * T * T;
    double li[T / P];
#pragma unroll
    for (int q = 0; q < T / P; ++q) {
      const int m = q * P + part;
      li[q] = m >= r ? Li[mf_idx(T, m, r)] : 0.0;
    }
    double zr = 0.0;  // this thread's share of the update of z[r]
    const uint8_t* nz = d.tile_nz + d.rcs_off[l] / (T * T);
    for (int m = nt - 1; m > k; --m) {
      if (!nz[(int64_t)m * (m + 1) / 2 + k]) continue;  // L(m,k) stays zero
      // the tile L(m,k) does not depend on x_m: load it before waiting
      const double* Lmk = tile_ptr<T>(d, l, m, k);
      double lv[T / P];
#pragma unroll
      for (int q = 0; q < T / P; ++q) lv[q] = Lmk[mf_idx(T, q * P + part, r)];
      df_wait(xf + m, nullptr, epoch, err);
      for (int q = threadIdx.x; q < T; q += NT) xm[q] = coh_load(d.x + vb + (int64_t)m * T + q);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < T / P; ++q) zr += lv[q] * xm[q * P + part];
      __syncthreads();  // xm is reloaded next round
    }
#pragma unroll
    for (int o = 1; o < P; o <<= 1) zr += __shfl_xor(zr, o);
    if (part == 0) z[r] -= zr;
    __syncthreads();
    double sx = 0.0;
#pragma unroll
    for (int q = 0; q < T / P; ++q) sx += li[q] * z[q * P + part];
#pragma unroll
    for (int o = 1; o < P; o <<= 1) sx += __shfl_xor(sx, o);
    if (part == 0) coh_store(d.x + vb + (int64_t)k * T + r, sx);
    df_publish(xf + k, epoch);
  }
}

// ------------------------------------------------------------ covariance
// Inverse of the reduced camera system of every dense sub-block from its
// Cholesky factor (Sec. 2: M_CC = S^-1), in three launches:
//   diag:    Y(J,J) = L(J,J)^-T, the stored inverse diagonal tile transposed;
//   panel:   one workgroup per tile column J of a sub-block, down the column:
//            Y(I,J) = -(sum_{K=J}^{I-1} Y(K,J) L(I,K)^T) L(I,I)^-T, I > J,
//            so that Y = (L^-1)^T tile by tile (X = L^-1, Y(I,J) = X(I,J)^T);
//   product: one workgroup per tile (I,J), I >= J:
//            S^-1(I,J) = sum_{K>=I} X(K,I)^T X(K,J) = sum_K Y(K,I) Y(K,J)^T,
//            written over the factor in the RCS storage.
// Y has the tile layout of the RCS.  Every product runs on the FP64 matrix
// cores; a tile column's chain stays in one workgroup, which reads the tiles
// it wrote itself after a barrier.
template <int T>
__device__ __forceinline__ double* ytile(const Dev& d, double* Y, int l, int i, int j) {
  return Y + d.rcs_off[l] + ((int64_t)i * (i + 1) / 2 + j) * (int64_t)T * T;
}

template <int T>
__global__ __launch_bounds__(NT) void k_cov_diag(Dev d, double* Y) {
  const int l = blockIdx.y, J = blockIdx.x;
  if (J >= d.nt[l]) return;
  const double* Li = d.Li + d.diag_off[l] + (int64_t)J * T * T;
  double* y = ytile<T>(d, Y, l, J, J);
  for (int idx = threadIdx.x; idx < T * T; idx += NT) {
    const int blk = idx >> 6, w = idx & 63;
    const int r = (blk / (T / 4)) * 16 + (w & 15), c = (blk % (T / 4)) * 4 + (w >> 4);
    y[idx] = Li[mf_idx(T, c, r)];
  }
}

template <int T>
__global__ __launch_bounds__(NT) void k_cov_panel(Dev d, double* Y) {
  __shared__ double stage[T * T];
  const int l = blockIdx.y, J = blockIdx.x, nt = d.nt[l];
  if (J >= nt) return;
  for (int I = J + 1; I < nt; ++I) {
    Acc<T> acc;
    acc.zero();
    for (int K = J; K < I; ++K) gemm_nt_mf<T>(ytile<T>(d, Y, l, K, J), tile_ptr<T>(d, l, I, K), acc);
#pragma unroll
    for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
      for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int r, c;
          acc_rc<T>(p, q, e, r, c);
          stage[mf_idx(T, r, c)] = acc.v[p][q][e];
        }
    __syncthreads();
    Acc<T> out;
    out.zero();
    gemm_nt_mf<T, true>(stage, d.Li + d.diag_off[l] + (int64_t)I * T * T, out);
    double* y = ytile<T>(d, Y, l, I, J);
#pragma unroll
    for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
      for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int r, c;
          acc_rc<T>(p, q, e, r, c);
          y[mf_idx(T, r, c)] = out.v[p][q][e];
        }
    __syncthreads();  // the tile is read by every wave in the next rows
  }
}

template <int T>
__global__ __launch_bounds__(NT) void k_cov_product(Dev d, const double* Y) {
  const int l = blockIdx.y, nt = d.nt[l];
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= (int)blockIdx.x) ++I;
  const int J = (int)blockIdx.x - I * (I + 1) / 2;
  if (I >= nt) return;
  Acc<T> acc;
  acc.zero();
  for (int K = I; K < nt; ++K)
    gemm_nt_mf<T>(ytile<T>(d, const_cast<double*>(Y), l, K, I), ytile<T>(d, const_cast<double*>(Y), l, K, J), acc);
  double* m = tile_ptr<T>(d, l, I, J);
#pragma unroll
  for (int p = 0; p < Acc<T>::NB; ++p)
#pragma unroll
    for (int q = 0; q < Acc<T>::NB; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int r, c;
        acc_rc<T>(p, q, e, r, c);
        m[mf_idx(T, r, c)] = acc.v[p][q][e];
      }
}

}  // namespace

void launch_chol_potrf(const Dev& d, int k, const int32_t* pot, int64_t npot, hipStream_t st) {
  if (npot <= 0) return;
  if (d.T == 64) hipLaunchKernelGGL(k_chol_potrf<64>, dim3((unsigned)npot), dim3(NT), 0, st, d, k, pot);
  else hipLaunchKernelGGL(k_chol_potrf<32>, dim3((unsigned)npot), dim3(NT), 0, st, d, k, pot);
}

void launch_chol_trsm(const Dev& d, int k, const int32_t* trsm, int64_t ntrsm, hipStream_t st) {
  if (ntrsm <= 0) return;
  if (d.T == 64) hipLaunchKernelGGL(k_chol_trsm<64>, dim3((unsigned)ntrsm), dim3(NT), 0, st, d, k, trsm);
  else hipLaunchKernelGGL(k_chol_trsm<32>, dim3((unsigned)ntrsm), dim3(NT), 0, st, d, k, trsm);
}

void launch_chol_update(const Dev& d, int k, const int32_t* upd, int64_t nupd, hipStream_t st) {
  if (nupd <= 0) return;
  if (d.T == 64) hipLaunchKernelGGL(k_chol_update<64>, dim3((unsigned)nupd), dim3(NT), 0, st, d, k, upd);
  else hipLaunchKernelGGL(k_chol_update<32>, dim3((unsigned)nupd), dim3(NT), 0, st, d, k, upd);
}

int chol_dataflow_resident_per_cu(int T) {
  int n = 0;
  const hipError_t e = T == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_chol_dataflow<64>, NT, 0)
                               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_chol_dataflow<32>, NT, 0);
  return e == hipSuccess ? n : 0;
}

void launch_chol_dataflow(const Dev& d, const int32_t* tasks, int ntask, int* flags, int64_t nflags, int* ctl,
                          int nworkers, hipStream_t st) {
  if (ntask > 0) {
    const unsigned g = (unsigned)std::max(1, std::min(ntask, nworkers));
    if (d.T == 64)
      hipLaunchKernelGGL(k_chol_dataflow<64>, dim3(g), dim3(NT), 0, st, d, tasks, ntask, flags, nflags, ctl);
    else
      hipLaunchKernelGGL(k_chol_dataflow<32>, dim3(g), dim3(NT), 0, st, d, tasks, ntask, flags, nflags, ctl);
  }
}

void launch_df_reset(int* ctl, hipStream_t st) { hipLaunchKernelGGL(k_df_reset, dim3(1), dim3(64), 0, st, ctl); }

void launch_df_finish(const Dev& d, int* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_df_finish, dim3(1), dim3(256), 0, st, d, ctl);
}

void launch_chol_backward_dataflow(const Dev& d, const int32_t* tasks, int ntask, int* xflags, int* ctl,
                                   int nworkers, hipStream_t st) {
  if (ntask > 0) {
    const unsigned g = (unsigned)std::max(1, std::min(ntask, nworkers));
    if (d.T == 64)
      hipLaunchKernelGGL(k_chol_backward_df<64>, dim3(g), dim3(NT), 0, st, d, tasks, ntask, xflags, ctl);
    else
      hipLaunchKernelGGL(k_chol_backward_df<32>, dim3(g), dim3(NT), 0, st, d, tasks, ntask, xflags, ctl);
  }
  hipLaunchKernelGGL(k_df_finish, dim3(1), dim3(256), 0, st, d, ctl);
}

void launch_rhs_extract(const Dev& d, const int* ctl, hipStream_t st) {
  if (d.T == 64) hipLaunchKernelGGL(k_rhs_extract<64>, dim3(d.L), dim3(NT), 0, st, d, ctl);
  else hipLaunchKernelGGL(k_rhs_extract<32>, dim3(d.L), dim3(NT), 0, st, d, ctl);
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

template <int T>
static void launch_cov_inverse_t(const Dev& d, double* Y, int nt_max, hipStream_t st) {
  hipLaunchKernelGGL(k_cov_diag<T>, dim3((unsigned)nt_max, (unsigned)d.L), dim3(NT), 0, st, d, Y);
  hipLaunchKernelGGL(k_cov_panel<T>, dim3((unsigned)nt_max, (unsigned)d.L), dim3(NT), 0, st, d, Y);
  hipLaunchKernelGGL(k_cov_product<T>, dim3((unsigned)(nt_max * (nt_max + 1) / 2), (unsigned)d.L), dim3(NT), 0, st,
                     d, (const double*)Y);
}

void launch_cov_inverse(const Dev& d, double* Y, int nt_max, hipStream_t st) {
  if (d.T == 64) launch_cov_inverse_t<64>(d, Y, nt_max, st);
  else launch_cov_inverse_t<32>(d, Y, nt_max, st);
}

}  // namespace rpba
