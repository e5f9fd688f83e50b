// Device-side geometry and small dense algebra for the librpba kernels.
//
// Camera model (paper Sec. 2, calibrated pinhole): p = R (X - C),
// g = (f p1/p3 + cx, f p2/p3 + cy).  With u = p1/p3, w = p2/p3:
//   dg/dX            = (f/p3) [[1, 0, -u], [0, 1, -w]] R            (B, 2x3)
//   dg/d(rotation)   = f [[-u w, 1 + u^2, -w], [-(1 + w^2), u w, u]]  (rotation
//                      increment left-multiplied, R <- Exp([d]x) R, Sec. 5.4)
//   dg/dC            = -B
// The camera Jacobian A (2x6) is [Ar | -B] with parameter order
// (rotation x, y, z, centre x, y, z).
//
// With intrinsics (Sec. 6: the focal length f and the first radial
// distortion parameter k1 of every camera estimated with its pose) the pixel
// is f (1 + k1 r2) q + c with q = (u, w), r2 = |q|^2.  With M = (1 + k1 r2) I
// + 2 k1 q q^T, B and Ar are those of the pinhole with the camera's f,
// multiplied by M on the left, and A gains the columns dg/df = (1 + k1 r2) q
// and dg/dk1 = f r2 q: A (2x8) = [Ar | -B | Ai], parameter order (rotation,
// centre, f, k1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpba {

// camera record in device memory: R (row-major, 9) then C (3).  With
// intrinsics the cameras' f and k1 are an array of their own ([M][2]); a
// kernel that holds a camera in registers appends them at CAM_F, CAM_K1.
constexpr int CAM_STRIDE = 12;
constexpr int CAM_F = 12, CAM_K1 = 13;

template <typename T>
struct Lin {
  T g0, g1;      // projected pixel
  T z;           // depth p3
  T B[2][3];     // dg/dX
  T Ar[2][3];    // dg/d(rotation increment)
  T Ai[2][2];    // with intrinsics: dg/df, dg/dk1
};

// Position of workgroup b of an n-workgroup grid in an order that gives each
// of the 8 XCDs one contiguous run of the work: the dispatcher hands
// workgroups to the XCDs round-robin (b runs on XCD b % 8), so position
// (b % 8) * share + b / 8 keeps neighbouring work items, which read the same
// records, on one XCD and in its L2.  A bijection of [0, n) for every n.
__device__ __forceinline__ int xcd_block(int b, int n) {
  constexpr int NX = 8;
  const int q = n / NX, r = n % NX, x = b % NX, s = b / NX;
  return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// 1 / x: in FP64 the hardware reciprocal estimate refined by two Newton
// steps (within an ulp or two for the depths met here, cheaper than the
// correctly rounded division); in FP32 the plain division (a refined
// estimate there measured no faster and moved the mixed path's results)
template <typename T>
__device__ __forceinline__ T recip(T x) {
  return T(1) / x;
}
template <>
__device__ __forceinline__ double recip<double>(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  y = y * (2.0 - x * y);
  return y;
}

// linearisation from the offset d = X - C (formed by the caller, in FP64 when T
// is float, so that large coordinates do not cancel in single precision)
template <typename T>
__device__ __forceinline__ void linearise_d(const T* __restrict__ R, T d0, T d1, T d2, T f, T cx, T cy, Lin<T>& o) {
  T p0 = R[0] * d0 + R[1] * d1 + R[2] * d2;
  T p1 = R[3] * d0 + R[4] * d1 + R[5] * d2;
  T p2 = R[6] * d0 + R[7] * d1 + R[8] * d2;
  o.z = p2;
  T iz = recip(p2);
  T u = p0 * iz, w = p1 * iz;
  o.g0 = f * u + cx;
  o.g1 = f * w + cy;
  T fz = f * iz;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o.B[0][c] = fz * (R[c] - u * R[6 + c]);
    o.B[1][c] = fz * (R[3 + c] - w * R[6 + c]);
  }
  o.Ar[0][0] = -f * u * w;
  o.Ar[0][1] = f * (T(1) + u * u);
  o.Ar[0][2] = -f * w;
  o.Ar[1][0] = -f * (T(1) + w * w);
  o.Ar[1][1] = f * u * w;
  o.Ar[1][2] = f * u;
}

// with intrinsics: the pinhole Jacobians with the camera's f, then the
// distortion (M on the left) and the two intrinsic columns
template <typename T>
__device__ __forceinline__ void distort(Lin<T>& o, T u, T w, T f, T k1) {
  const T r2 = u * u + w * w, s = T(1) + k1 * r2;
  const T m00 = s + T(2) * k1 * u * u, m01 = T(2) * k1 * u * w, m11 = s + T(2) * k1 * w * w;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T b0 = o.B[0][c], b1 = o.B[1][c], a0 = o.Ar[0][c], a1 = o.Ar[1][c];
    o.B[0][c] = m00 * b0 + m01 * b1;
    o.B[1][c] = m01 * b0 + m11 * b1;
    o.Ar[0][c] = m00 * a0 + m01 * a1;
    o.Ar[1][c] = m01 * a0 + m11 * a1;
  }
  o.Ai[0][0] = s * u;
  o.Ai[1][0] = s * w;
  o.Ai[0][1] = f * r2 * u;
  o.Ai[1][1] = f * r2 * w;
}

template <typename T>
__device__ __forceinline__ void linearise_cal_d(const T* __restrict__ R, T d0, T d1, T d2, T f, T k1, T cx, T cy,
                                                Lin<T>& o) {
  linearise_d<T>(R, d0, d1, d2, f, cx, cy, o);
  const T iz = recip(o.z);
  const T p0 = R[0] * d0 + R[1] * d1 + R[2] * d2, p1 = R[3] * d0 + R[4] * d1 + R[5] * d2;
  const T u = p0 * iz, w = p1 * iz, s = T(1) + k1 * (u * u + w * w);
  o.g0 = f * s * u + cx;
  o.g1 = f * s * w + cy;
  distort<T>(o, u, w, f, k1);
}

// camera record cm (CAM_STRIDE layout) at X: the pinhole with the shared f,
// or with intrinsics (CAL) the camera's own f and k1 at fk
template <bool CAL, typename T>
__device__ __forceinline__ void linearise_cam(const T* __restrict__ cm, const T* __restrict__ fk, const T X[3], T f,
                                              T cx, T cy, Lin<T>& o) {
  if constexpr (CAL)
    linearise_cal_d<T>(cm, X[0] - cm[9], X[1] - cm[10], X[2] - cm[11], fk[0], fk[1], cx, cy, o);
  else
    linearise_d<T>(cm, X[0] - cm[9], X[1] - cm[10], X[2] - cm[11], f, cx, cy, o);
}

template <typename T>
__device__ __forceinline__ void linearise(const T* __restrict__ R, const T* __restrict__ C, const T X[3], T f,
                                          T cx, T cy, Lin<T>& o) {
  linearise_d<T>(R, X[0] - C[0], X[1] - C[1], X[2] - C[2], f, cx, cy, o);
}

// Projection and residual in FP64, Jacobians in J (the mixed path's split:
// FP64 state and residuals, FP32 Jacobians and per-observation products).
// For J = double the arithmetic is that of linearise<double>.  o.g0, o.g1
// and o.z hold the projection rounded to J; g0, g1 the FP64 projection.
template <typename J>
__device__ __forceinline__ void linearise_split(const double* __restrict__ R, const double* __restrict__ C,
                                                const double X[3], double f, double cx, double cy, Lin<J>& o,
                                                double& g0, double& g1, double& z) {
  const double d0 = X[0] - C[0], d1 = X[1] - C[1], d2 = X[2] - C[2];
  const double p0 = R[0] * d0 + R[1] * d1 + R[2] * d2;
  const double p1 = R[3] * d0 + R[4] * d1 + R[5] * d2;
  const double p2 = R[6] * d0 + R[7] * d1 + R[8] * d2;
  z = p2;
  const double iz = recip(p2);
  const double u = p0 * iz, w = p1 * iz;
  g0 = f * u + cx;
  g1 = f * w + cy;
  const J fz = (J)(f * iz), uj = (J)u, wj = (J)w, fj = (J)f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o.B[0][c] = fz * ((J)R[c] - uj * (J)R[6 + c]);
    o.B[1][c] = fz * ((J)R[3 + c] - wj * (J)R[6 + c]);
  }
  o.Ar[0][0] = -fj * uj * wj;
  o.Ar[0][1] = fj * (J(1) + uj * uj);
  o.Ar[0][2] = -fj * wj;
  o.Ar[1][0] = -fj * (J(1) + wj * wj);
  o.Ar[1][1] = fj * uj * wj;
  o.Ar[1][2] = fj * uj;
  o.g0 = (J)g0;
  o.g1 = (J)g1;
  o.z = (J)z;
}

// the same for a camera record (CAM_STRIDE layout); with intrinsics (CAL)
// the camera's own f and k1 at fk: projection in FP64, Jacobians in J
template <bool CAL, typename J>
__device__ __forceinline__ void linearise_split_cam(const double* __restrict__ cm, const double* __restrict__ fk,
                                                    const double X[3], double f, double cx, double cy, Lin<J>& o,
                                                    double& g0, double& g1, double& z) {
  if constexpr (!CAL) {
    linearise_split<J>(cm, cm + 9, X, f, cx, cy, o, g0, g1, z);
  } else {
    const double fc = fk[0], k1 = fk[1];
    linearise_split<J>(cm, cm + 9, X, fc, cx, cy, o, g0, g1, z);
    const double iz = recip(z);
    const double d0 = X[0] - cm[9], d1 = X[1] - cm[10], d2 = X[2] - cm[11];
    const double u = (cm[0] * d0 + cm[1] * d1 + cm[2] * d2) * iz, w = (cm[3] * d0 + cm[4] * d1 + cm[5] * d2) * iz;
    const double s = 1.0 + k1 * (u * u + w * w);
    g0 = fc * s * u + cx;
    g1 = fc * s * w + cy;
    o.g0 = (J)g0;
    o.g1 = (J)g1;
    distort<J>(o, (J)u, (J)w, (J)fc, (J)k1);
  }
}

// weight matrix of one observation [[a, b], [b, c]]
template <typename T>
struct W2 {
  T a, b, c;
};

template <typename T>
__device__ __forceinline__ T wquad(const W2<T>& W, T v0, T v1) {
  return W.a * v0 * v0 + T(2) * W.b * v0 * v1 + W.c * v1 * v1;
}

// Rodrigues' formula: R_out = Exp([w]x) R_in (series below 1e-8 rad).
__device__ __forceinline__ void rotate_left(const double w[3], const double* Rin, double* Rout) {
  double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double th = sqrt(th2);
  double a, b;
  if (th < 1e-8) {
    a = 1.0;
    b = 0.5;
  } else {
    double sn, cs;
    sincos(th, &sn, &cs);
    a = sn / th;
    b = (1.0 - cs) / th2;
  }
  // E = I + a K + b K^2 with K = [w]x, K^2 = w w^T - th2 I
  double E[9];
  E[0] = 1.0 + b * (w[0] * w[0] - th2);
  E[4] = 1.0 + b * (w[1] * w[1] - th2);
  E[8] = 1.0 + b * (w[2] * w[2] - th2);
  E[1] = -a * w[2] + b * w[0] * w[1];
  E[3] = a * w[2] + b * w[0] * w[1];
  E[2] = a * w[1] + b * w[0] * w[2];
  E[6] = -a * w[1] + b * w[0] * w[2];
  E[5] = -a * w[0] + b * w[1] * w[2];
  E[7] = a * w[0] + b * w[1] * w[2];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Rout[3 * r + c] = E[3 * r] * Rin[c] + E[3 * r + 1] * Rin[3 + c] + E[3 * r + 2] * Rin[6 + c];
}

// 1 / sqrt(x) in FP64: the hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// Symmetric 3x3 stored as (xx, xy, xz, yy, yz, zz).
// Cholesky with the pivot test pivot > 1e-12 * max diagonal; on success
// writes the lower factor with its diagonal held as reciprocals,
// l = (1/l00, l10, l20, 1/l11, l21, 1/l22), so that the solves and the
// inverse below multiply instead of divide.
__device__ __forceinline__ bool chol3(const double h[6], double l[6]) {
  double dmax = fmax(h[0], fmax(h[3], h[5]));
  if (!(dmax > 0.0)) return false;
  double thr = 1e-12 * dmax;
  double p0 = h[0];
  if (!(p0 > thr)) return false;
  l[0] = rsqrt_nr(p0);
  l[1] = h[1] * l[0];
  l[2] = h[2] * l[0];
  double p1 = h[3] - l[1] * l[1];
  if (!(p1 > thr)) return false;
  l[3] = rsqrt_nr(p1);
  l[4] = (h[4] - l[2] * l[1]) * l[3];
  double p2 = h[5] - l[2] * l[2] - l[4] * l[4];
  if (!(p2 > thr)) return false;
  l[5] = rsqrt_nr(p2);
  return true;
}

// x = (L L^T)^-1 b
__device__ __forceinline__ void chol3_solve(const double l[6], const double b[3], double x[3]) {
  double y0 = b[0] * l[0];
  double y1 = (b[1] - l[1] * y0) * l[3];
  double y2 = (b[2] - l[2] * y0 - l[4] * y1) * l[5];
  x[2] = y2 * l[5];
  x[1] = (y1 - l[4] * x[2]) * l[3];
  x[0] = (y0 - l[1] * x[1] - l[2] * x[2]) * l[0];
}

// inverse (sym6 layout) from the Cholesky factor: Inv = L^-T L^-1
__device__ __forceinline__ void chol3_inverse(const double l[6], double inv[6]) {
  // M = L^-1 (lower)
  double m00 = l[0];
  double m11 = l[3];
  double m22 = l[5];
  double m10 = -l[1] * m00 * m11;
  double m21 = -l[4] * m11 * m22;
  double m20 = -(l[2] * m00 + l[4] * m10) * m22;
  inv[0] = m00 * m00 + m10 * m10 + m20 * m20;
  inv[1] = m11 * m10 + m21 * m20;
  inv[2] = m22 * m20;
  inv[3] = m11 * m11 + m21 * m21;
  inv[4] = m22 * m21;
  inv[5] = m22 * m22;
}

__device__ __forceinline__ void sym3_mul(const double s[6], const double x[3], double y[3]) {
  y[0] = s[0] * x[0] + s[1] * x[1] + s[2] * x[2];
  y[1] = s[1] * x[0] + s[3] * x[1] + s[4] * x[2];
  y[2] = s[2] * x[0] + s[4] * x[1] + s[5] * x[2];
}

// B^T W B (sym6) and B^T W v added into h, g.
template <typename T>
__device__ __forceinline__ void add_point_normals(const Lin<T>& L, const W2<T>& W, T v0, T v1, T h[6], T g[3]) {
  T WB0[3], WB1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    WB0[c] = W.a * L.B[0][c] + W.b * L.B[1][c];
    WB1[c] = W.b * L.B[0][c] + W.c * L.B[1][c];
  }
  T Wv0 = W.a * v0 + W.b * v1, Wv1 = W.b * v0 + W.c * v1;
  h[0] += L.B[0][0] * WB0[0] + L.B[1][0] * WB1[0];
  h[1] += L.B[0][0] * WB0[1] + L.B[1][0] * WB1[1];
  h[2] += L.B[0][0] * WB0[2] + L.B[1][0] * WB1[2];
  h[3] += L.B[0][1] * WB0[1] + L.B[1][1] * WB1[1];
  h[4] += L.B[0][1] * WB0[2] + L.B[1][1] * WB1[2];
  h[5] += L.B[0][2] * WB0[2] + L.B[1][2] * WB1[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] += L.B[0][c] * Wv0 + L.B[1][c] * Wv1;
}

// atomic max of a non-negative double through its bit pattern
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

}  // namespace rpba
