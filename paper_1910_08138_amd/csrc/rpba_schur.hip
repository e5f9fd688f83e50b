// Schur complement of the sub-block normal equations onto the cameras (the
// reduced camera system, RCS), paper Sec. 2 and 5.4: the outer products of
// the observations of every point copy are accumulated straight into the RCS,
//   S_(i,i2) = [i == i2] U*_i - sum_(copies c) sum_(k1 in i, k2 in i2) Y_k1 V*_c^-1 Y_k2^T,
//   e_i      = -g_Ci + sum_(k1 in i) Y_k1 V*_c^-1 g_Xc,
// with U*_i the damped camera block, Y_k = A_k^T W_k B_k, V*_c the damped point
// block (its FP64 inverse comes from the point-block pass).
//
// Camera blocks are NP x NP: NP = 6 (pose), or 8 with intrinsics (pose, the
// camera's f and k1; Sec. 6).
//
// Each NP x NP block is owned by one group of lanes that sums the contributions of
// its observation pairs in registers and writes the block once: no atomics,
// deterministic order.  Diagonal blocks (one 64-lane wave per camera) also
// reduce U*, g_C and e; off-diagonal blocks take a group of 4, 8 or 16 lanes
// each (an option the autotuner picks).
//
// T is the arithmetic of the Jacobians and of the accumulation: double on the
// FP64 path, float on the mixed path (X - C is formed in FP64 first).  Output
// per sub-block: the dense tiled lower triangle (FP64) for sub-blocks solved by
// Cholesky, or full 6x6 blocks of a block-sparse matrix (FP32) for sub-blocks
// solved iteratively.
#include "rpba_device.hpp"
#include "rpba_internal.hpp"
#include "rpba_plan.hpp"

namespace rpba {

namespace {

constexpr int NT = 256;

// weight of the observation at position t of its camera's list (camera-major
// copies of the robust multiplier and of the information matrix); unit:
// every robust multiplier is 1 and is not read
template <typename T>
__device__ __forceinline__ W2<T> cm_weight_t(const Dev& d, int64_t t, bool unit) {
  const double r = unit ? 1.0 : d.cm_rw[t];
  if (d.has_info) {
    const double* w = d.cm_info + 3 * t;
    return {(T)(r * w[0]), (T)(r * w[1]), (T)(r * w[2])};
  }
  return {(T)(r * d.w0), T(0), (T)(r * d.w0)};
}

// camera i: rotation in T, centre in FP64; with intrinsics (NP = 8) its f
// and k1 in T
template <typename T, int NP>
struct CamReg {
  T R[9];
  double C[3];
  T fk[2];
  __device__ void load(const Dev& d, int i) {
    const double* c = d.cam + (int64_t)CAM_STRIDE * i;
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = (T)c[q];
    C[0] = c[9];
    C[1] = c[10];
    C[2] = c[11];
    if constexpr (NP == 8) {
      fk[0] = (T)d.intr[2 * (int64_t)i];
      fk[1] = (T)d.intr[2 * (int64_t)i + 1];
    }
  }
  __device__ void lin(const double X[3], const Dev& d, Lin<T>& L) const {
    const T d0 = (T)(X[0] - C[0]), d1 = (T)(X[1] - C[1]), d2 = (T)(X[2] - C[2]);
    if constexpr (NP == 8) linearise_cal_d<T>(R, d0, d1, d2, fk[0], fk[1], (T)d.cx, (T)d.cy, L);
    else linearise_d<T>(R, d0, d1, d2, (T)d.f, (T)d.cx, (T)d.cy, L);
  }
};

// camera Jacobian A (2 x NP) = [Ar | -B | Ai] of one observation
template <typename T, int NP>
__device__ __forceinline__ void a_block(const Lin<T>& L, T A[2][NP]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    A[0][q] = L.Ar[0][q];
    A[1][q] = L.Ar[1][q];
    A[0][3 + q] = -L.B[0][q];
    A[1][3 + q] = -L.B[1][q];
  }
  if constexpr (NP == 8) {
    A[0][6] = L.Ai[0][0];
    A[1][6] = L.Ai[1][0];
    A[0][7] = L.Ai[0][1];
    A[1][7] = L.Ai[1][1];
  }
}

// Y = A^T W B (NP x 3) of one observation
template <typename T, int NP>
__device__ __forceinline__ void y_block(const Lin<T>& L, const W2<T>& W, T Y[NP][3]) {
  T WB0[3], WB1[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    WB0[s] = W.a * L.B[0][s] + W.b * L.B[1][s];
    WB1[s] = W.b * L.B[0][s] + W.c * L.B[1][s];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      Y[r][s] = L.Ar[0][r] * WB0[s] + L.Ar[1][r] * WB1[s];
      Y[3 + r][s] = -(L.B[0][r] * WB0[s] + L.B[1][r] * WB1[s]);
    }
  if constexpr (NP == 8) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) Y[6 + r][s] = L.Ai[0][r] * WB0[s] + L.Ai[1][r] * WB1[s];
  }
}

// Z = Y V^-1 with V^-1 symmetric (xx, xy, xz, yy, yz, zz)
template <typename T, int NP>
__device__ __forceinline__ void z_block(const T Y[NP][3], const T Vi[6], T Z[NP][3]) {
#pragma unroll
  for (int r = 0; r < NP; ++r) {
    Z[r][0] = Y[r][0] * Vi[0] + Y[r][1] * Vi[1] + Y[r][2] * Vi[2];
    Z[r][1] = Y[r][0] * Vi[1] + Y[r][1] * Vi[3] + Y[r][2] * Vi[4];
    Z[r][2] = Y[r][0] * Vi[2] + Y[r][1] * Vi[4] + Y[r][2] * Vi[5];
  }
}

// index of (r, s), r <= s, in a packed NP x NP upper triangle
template <int NP>
__host__ __device__ constexpr int upn(int r, int s) { return r * NP - r * (r - 1) / 2 + (s - r); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// Inputs of one observation k of copy c to the Schur pass, loaded ahead of
// use: the copy's point (FP64) and damped inverse, g_X (diagonal pass only),
// the pixel and the weight, converted to T.
template <typename T>
struct ObsIn {
  double X[3];
  T Vi[6], gX[3], x, y;
  W2<T> W;
  bool valid;
};

// inputs of one observation of copy c; k is the observation's position in
// its camera's list: pixel (diagonal pass only) and weight come from the
// camera-major copies, read in order by the camera's wave or pair group
template <typename T, bool DIAG>
__device__ __forceinline__ void obs_in_load(const Dev& d, int k, int c, bool in_range, bool unit, ObsIn<T>& o) {
  o.valid = false;
  if (!in_range) return;
  if constexpr (sizeof(T) == 4) {
    // compact record of the mixed path: X (3 doubles), V*^-1 (6 floats),
    // g_X (3 floats), valid (float)
    const uint4* p4 = reinterpret_cast<const uint4*>(d.cpk + CPK32 * (int64_t)c);
    uint32_t w[16];
    const uint4 a = p4[0], b = p4[1], e = p4[2];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    w[8] = e.x; w[9] = e.y; w[10] = e.z; w[11] = e.w;
    if (DIAG) {
      const uint4 f4 = p4[3];
      w[12] = f4.x; w[13] = f4.y; w[14] = f4.z; w[15] = f4.w;
    } else {
      const uint4 f4 = p4[3];
      w[15] = f4.w;
      w[12] = w[13] = w[14] = 0u;
    }
    __builtin_memcpy(o.X, w, 24);
    float f[10];
    __builtin_memcpy(f, w + 6, 40);
    o.valid = f[9] != 0.f;
    for (int q = 0; q < 6; ++q) o.Vi[q] = (T)f[q];
    if (DIAG)
      for (int q = 0; q < 3; ++q) o.gX[q] = (T)f[6 + q];
  } else {
    const double2* pk = reinterpret_cast<const double2*>(d.cpk + CPK * (int64_t)c);
    const double2 p0 = pk[0], p1 = pk[1], p2 = pk[2], p3 = pk[3], p4 = pk[4];
    o.valid = p1.y != 0.0;  // point not valid (or sub-block inactive): zero record
    o.X[0] = p0.x;
    o.X[1] = p0.y;
    o.X[2] = p1.x;
    o.Vi[0] = (T)p2.x;
    o.Vi[1] = (T)p2.y;
    o.Vi[2] = (T)p3.x;
    o.Vi[3] = (T)p3.y;
    o.Vi[4] = (T)p4.x;
    o.Vi[5] = (T)p4.y;
    if (DIAG) {
      const double2 p5 = pk[5], p6 = pk[6];
      o.gX[0] = (T)p5.x;
      o.gX[1] = (T)p5.y;
      o.gX[2] = (T)p6.x;
    }
  }
  if (DIAG) {
    const double2 xy = reinterpret_cast<const double2*>(d.cm_xy)[k];
    o.x = (T)xy.x;
    o.y = (T)xy.y;
  }
  o.W = cm_weight_t<T>(d, k, unit);
}

// One wave per camera: diagonal block S_(i,i) = U*_i - sum_k Y_k V*^-1 Y_k^T
// and e_i.  Neighbouring cameras (which see the same points, so read the same
// copy records) run on one XCD.
template <typename T, int NP>
__global__ __launch_bounds__(NT) void k_schur_diag(Dev d) {
  constexpr int NU = NP * (NP + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int i = xcd_block(blockIdx.x, gridDim.x) * (NT / 64) + (threadIdx.x >> 6);
  if (i >= d.M) return;
  const int l = d.cam_blk[i];
  if (d.active && !d.active[l]) return;
  const bool unit = *d.rw_unit != 0;
  CamReg<T, NP> cm;
  cm.load(d, i);
  T acc[NU], U[NU], gC[NP], ep[NP];
#pragma unroll
  for (int q = 0; q < NU; ++q) acc[q] = U[q] = T(0);
#pragma unroll
  for (int q = 0; q < NP; ++q) gC[q] = ep[q] = T(0);

  auto process = [&](const ObsIn<T>& o) {
    Lin<T> L;
    cm.lin(o.X, d, L);
    const W2<T> W = o.W;
    const T v0 = L.g0 - o.x, v1 = L.g1 - o.y;
    T A[2][NP], WA[2][NP];
    a_block<T, NP>(L, A);
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      WA[0][q] = W.a * A[0][q] + W.b * A[1][q];
      WA[1][q] = W.b * A[0][q] + W.c * A[1][q];
    }
    const T Wv0 = W.a * v0 + W.b * v1, Wv1 = W.b * v0 + W.c * v1;
#pragma unroll
    for (int r = 0; r < NP; ++r) {
#pragma unroll
      for (int s = r; s < NP; ++s) U[upn<NP>(r, s)] += A[0][r] * WA[0][s] + A[1][r] * WA[1][s];
      gC[r] += A[0][r] * Wv0 + A[1][r] * Wv1;
    }
    T Y[NP][3], Z[NP][3];
    y_block<T, NP>(L, W, Y);
    z_block<T, NP>(Y, o.Vi, Z);
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      ep[r] += Z[r][0] * o.gX[0] + Z[r][1] * o.gX[1] + Z[r][2] * o.gX[2];
#pragma unroll
      for (int s = r; s < NP; ++s) acc[upn<NP>(r, s)] -= Z[r][0] * Y[s][0] + Z[r][1] * Y[s][1] + Z[r][2] * Y[s][2];
    }
  };
  const int o0 = d.cam_obs_off[i], o1 = d.cam_obs_off[i + 1];
  if constexpr (sizeof(T) == 4) {
    // FP32: a two-stage software pipeline over the camera's observations
    // (indices two rounds ahead, the copy record, pixel and weight one round
    // ahead); in FP64 the extra registers would cost occupancy
    int t = o0 + lane;
    int kB = 0, cB = 0;
    ObsIn<T> cur;
    {
      int kA = 0, cA = 0;
      if (t < o1) {
        kA = t;
        cA = d.cam_obs_c[t];
      }
      if (t + 64 < o1) {
        kB = t + 64;
        cB = d.cam_obs_c[t + 64];
      }
      obs_in_load<T, true>(d, kA, cA, t < o1, unit, cur);
    }
    for (; t < o1; t += 64) {
      int kC = 0, cC = 0;
      if (t + 128 < o1) {
        kC = t + 128;
        cC = d.cam_obs_c[t + 128];
      }
      ObsIn<T> nxt;
      obs_in_load<T, true>(d, kB, cB, t + 64 < o1, unit, nxt);
      if (cur.valid) process(cur);
      cur = nxt;
      kB = kC;
      cB = cC;
    }
  } else {
    for (int t = o0 + lane; t < o1; t += 64) {
      ObsIn<T> cur;
      obs_in_load<T, true>(d, t, d.cam_obs_c[t], true, unit, cur);
      if (cur.valid) process(cur);
    }
  }
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    acc[q] = wave_sum(acc[q]);
    U[q] = wave_sum(U[q]);
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    gC[q] = wave_sum(gC[q]);
    ep[q] = wave_sum(ep[q]);
  }
  const int a = i - d.blk_cam_off[l];
  if (lane < NP * NP) {
    const int r = lane / NP, s = lane % NP;
    const int u = r <= s ? upn<NP>(r, s) : upn<NP>(s, r);
    // select the lane's entry from the register arrays
    double uv = 0.0, av = 0.0;
#pragma unroll
    for (int q = 0; q < NU; ++q)
      if (q == u) {
        uv = (double)U[q];
        av = (double)acc[q];
      }
    if (r == s) uv = (uv == 0.0) ? 1.0 : uv * (1.0 + lam_of(d, l));
    const double val = uv + av;
    if (NP == 6 && d.blk_pcg && d.blk_pcg[l]) {
      d.bsr[(int64_t)d.pb_bsr[d.nb_off[i + 1] - 1] * 36 + lane] = (float)val;
    } else if (s <= r) {
      d.S[rcs_elem(d, l, NP * a + r, NP * a + s)] = val;
    }
  }
  if (lane < NP) {
    double g = 0.0, e = 0.0;
#pragma unroll
    for (int q = 0; q < NP; ++q)
      if (q == lane) {
        g = (double)gC[q];
        e = (double)ep[q];
      }
    d.y[d.vec_off[l] + NP * a + lane] = -g + e;
    // dense sub-blocks: e^T is row 0 of the right-hand-side tile row
    if (!(NP == 6 && d.blk_pcg && d.blk_pcg[l])) d.S[rcs_elem(d, l, d.nt[l] * d.T, NP * a + lane)] = -g + e;
  }
}

// One G-lane group per off-diagonal pair block (i, i2), i2 < i in the sub-block.
template <typename T, int G, int NP>
__global__ __launch_bounds__(NT) void k_schur_offdiag(Dev d) {
  const int gl = threadIdx.x & (G - 1);
  const int64_t t = (int64_t)blockIdx.x * (NT / G) + (threadIdx.x / G);
  if (t >= d.n_od) return;  // uniform over the lane group
  const int q = d.od_pb[t];
  const int i1 = d.pb_row[q];
  const int l = d.cam_blk[i1];
  if (d.active && !d.active[l]) return;
  const int base = d.blk_cam_off[l];
  const int a2 = d.nb_cam[q];
  const int i2 = base + a2;
  const bool unit = *d.rw_unit != 0;
  CamReg<T, NP> c1, c2;
  c1.load(d, i1);
  c2.load(d, i2);
  T acc[NP * NP];
#pragma unroll
  for (int u = 0; u < NP * NP; ++u) acc[u] = T(0);
  for (int64_t e = d.pb_ent_off[q] + gl; e < d.pb_ent_off[q + 1]; e += G) {
    const int c = d.pb_ent[3 * e], t1 = d.pb_ent[3 * e + 1], t2 = d.pb_ent[3 * e + 2];
    ObsIn<T> o;
    obs_in_load<T, false>(d, t1, c, true, unit, o);
    if (!o.valid) continue;
    Lin<T> L1, L2;
    c1.lin(o.X, d, L1);
    c2.lin(o.X, d, L2);
    T Y1[NP][3], Y2[NP][3], Z1[NP][3];
    y_block<T, NP>(L1, o.W, Y1);
    y_block<T, NP>(L2, cm_weight_t<T>(d, t2, unit), Y2);
    z_block<T, NP>(Y1, o.Vi, Z1);
#pragma unroll
    for (int r = 0; r < NP; ++r)
#pragma unroll
      for (int s = 0; s < NP; ++s) acc[NP * r + s] -= Z1[r][0] * Y2[s][0] + Z1[r][1] * Y2[s][1] + Z1[r][2] * Y2[s][2];
  }
#pragma unroll
  for (int u = 0; u < NP * NP; ++u) acc[u] = group_sum<G>(acc[u]);
  const int a1 = i1 - base;
  // (the block-sparse matrix of the iterative solver holds 6 x 6 blocks:
  // intrinsics are solved directly)
  const bool sparse = NP == 6 && d.blk_pcg && d.blk_pcg[l];
#pragma unroll
  for (int u = 0; u < NP * NP; ++u) {
    if ((u & (G - 1)) != gl) continue;
    const int r = u / NP, s = u % NP;
    if (sparse) {
      d.bsr[(int64_t)d.pb_bsr[q] * 36 + u] = (float)acc[u];
      d.bsr[(int64_t)d.pb_bsr_t[q] * 36 + 6 * s + r] = (float)acc[u];
    } else {
      d.S[rcs_elem(d, l, NP * a1 + r, NP * a2 + s)] = (double)acc[u];
    }
  }
}

}  // namespace

void launch_schur_diag(const Dev& d, bool fp32, bool dense, int64_t rcs_total, hipStream_t st) {
  if (dense) {
    // every lower element not covered by a pair block is zero; the padded
    // identity of the last diagonal tile is restored as well
    launch_zero_wide(d.S, rcs_total, st);
    launch_init_rcs(d, st);
  }
  const unsigned gd = (unsigned)((d.M + 3) / 4);
  if (d.np == 8) {
    if (fp32) hipLaunchKernelGGL((k_schur_diag<float, 8>), dim3(gd), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_schur_diag<double, 8>), dim3(gd), dim3(NT), 0, st, d);
  } else {
    if (fp32) hipLaunchKernelGGL((k_schur_diag<float, 6>), dim3(gd), dim3(NT), 0, st, d);
    else hipLaunchKernelGGL((k_schur_diag<double, 6>), dim3(gd), dim3(NT), 0, st, d);
  }
}

template <int G, int NP>
static void launch_offdiag_lanes(const Dev& d, bool fp32, hipStream_t st) {
  const unsigned go = (unsigned)((d.n_od + NT / G - 1) / (NT / G));
  if (!go) return;
  if (fp32) hipLaunchKernelGGL((k_schur_offdiag<float, G, NP>), dim3(go), dim3(NT), 0, st, d);
  else hipLaunchKernelGGL((k_schur_offdiag<double, G, NP>), dim3(go), dim3(NT), 0, st, d);
}

void launch_schur_offdiag(const Dev& d, bool fp32, hipStream_t st) {
  if (d.np == 8) launch_offdiag_lanes<8, 8>(d, fp32, st);  // intrinsics: eight lanes per block
  else if (d.pb_lanes == 4) launch_offdiag_lanes<4, 6>(d, fp32, st);
  else if (d.pb_lanes == 16) launch_offdiag_lanes<16, 6>(d, fp32, st);
  else launch_offdiag_lanes<8, 6>(d, fp32, st);
}

}  // namespace rpba
