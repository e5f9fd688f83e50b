// Plain FP64 CPU oracle for covariance-weighted consensus bundle adjustment
// (H. Mayer, "RPBA: Robust Parallel Bundle Adjustment Based on Covariance
// Information", arXiv 1910.08138).
//
// TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
// HIP path is checked against.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it; the product never does.  It
// shares no code, header, table or helper with the HIP library.
//
// Everything is double precision, written for reading rather than speed:
// small fixed-size matrices are plain arrays with explicit loops, the reduced
// camera system of each sub-block is a dense matrix factorised by a textbook
// Cholesky.  OpenMP only distributes independent points / sub-blocks; every
// sum that crosses items is done serially in a fixed order.
//
// Paper passages followed (by section / equation label):
//   Sec. 2  -- residual v_k = g_k(P_i, X_j) - x_k, weighted normal equations
//              (eq:normalw), point/camera split of N and the Schur complement
//              (reduced camera system), LM damping.
//   Sec. 5  -- sub-block adjustment with tie points as stochastic control
//              points (eq:batp, eq:bact); intersection of points with cameras
//              fixed giving the point and its covariance (eq:bars); switching
//              between the two without a dual update.
//   Sec. 5.1 -- refined re-weighting: the tie-point weight for sub-block l is
//              the point normal matrix built from cameras outside l only,
//              while the point position uses all cameras.
//   Sec. 5.3 -- sigma0 (eq:sigma0); per-camera MAD scale (factor 1.4826);
//              parallel robust variant (weighting inside the intersection,
//              threshold 4, down-weight 1e-4, whole points eliminated);
//              serial variant (threshold 3, down-weight 1e-4, then the
//              flagged observations deleted and points left in one camera
//              eliminated).
//   Sec. 5.4 -- outer products accumulated straight into the RCS; incremental
//              three-parameter rotation; N + lambda diag(N), lambda = 1e-4;
//              ratio rule for convergence; points whose intersection does not
//              converge are dropped.
//   Sec. 2.3/3 (former work) -- block-Jacobi preconditioned CG on the RCS.
//
// Readings taken where the paper is silent (listed in the design notes):
//   * camera model: calibrated pinhole, p = R (X - C), pixel f p/p3 + c;
//     rotation update R <- Exp([w]x) R (Rodrigues), centre update C <- C + dc;
//     per-camera parameter order (w_x, w_y, w_z, c_x, c_y, c_z).
//   * intrinsics (the f + k1 per camera of the Final data sets, Sec. 6):
//     pixel f (1 + k1 r2) q + c with q = (p1/p3, p2/p3), r2 = |q|^2, the
//     principal point shared and fixed; f and k1 updated additively and
//     appended to the camera's parameters (w, c, f, k1).
//   * the tie-point term of eq:bact is the squared Mahalanobis distance
//     (X - Xbar)^T Omega (X - Xbar).
//   * damping multiplies the diagonal of the full N (including Omega) and is
//     applied to camera and point blocks before the Schur complement; every
//     step is accepted.
//   * intersection: undamped Gauss-Newton, stop when |dX| <= tol (1 + |X|),
//     at most maxit iterations; statuses NOT_CONVERGED, BEHIND_CAMERA,
//     ILL_CONDITIONED (3x3 Cholesky pivot <= 1e-12 * max diagonal); failed
//     points get weight zero from then on.
//   * sigma0 redundancy r = 2 K_valid - n_p M - 3 N_valid (n_p = 6, or 8 with
//     intrinsics), unit weights, pixels.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

enum PointStatus { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_BEHIND = 2, ST_ILL = 3, ST_ELIMINATED = 4, ST_FILTERED = 5 };

// Variants of the method compared in the paper (Sec. 4, Sec. 6.3-6.4):
//   EXTENDED      covariance-weighted consensus (Sec. 5, 5.1): points
//                 intersected, tie-point copies weighted by the information
//                 from the cameras outside their sub-block
//   ALL_CAMERAS   the same with the information from all cameras
//   SCALAR        the same with the scalar weight rho_t I
//   PLAIN         ADMM consensus (eq:admm7 to eq:admm9): no intersection,
//                 copies pulled towards X_j - Xtilde_j^l with weight rho_t I,
//                 X_j = mean of the copies, Xtilde_j^l += X_j^l - X_j
//   PLAIN_REFINED PLAIN with the weights of Sec. 5.1 at the mean point
// rho_t grows by a constant factor per outer iteration (Sec. 6.3).
enum Variant { V_EXTENDED = 0, V_ALL_CAMERAS = 1, V_SCALAR = 2, V_PLAIN = 3, V_PLAIN_REFINED = 4 };

// ---------------------------------------------------------------- 3x3 / small
struct Cam {
  double R[3][3];
  double C[3];
  double f = 0.0, k1 = 0.0;  // own focal length and radial distortion (estimated with intrinsics only)
};

// Rodrigues' formula for the rotation of the axis-angle vector w
// (Sec. 5.4: three-parameter incremental rotation).  Small angles use the
// second-order series I + [w]x + 1/2 [w]x^2.
void rodrigues(const double w[3], double R[3][3]) {
  double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
  double K2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int m = 0; m < 3; ++m) s += K[i][m] * K[m][j];
      K2[i][j] = s;
    }
  double a, b;
  if (th < 1e-8) {
    a = 1.0;
    b = 0.5;
  } else {
    a = std::sin(th) / th;
    b = (1.0 - std::cos(th)) / (th * th);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * K2[i][j];
}

struct Obs2 {  // weight matrix of one observation: [[w11, w12], [w12, w22]]
  double w11, w12, w22;
};

// Projection g_k(P_i, X_j) and its Jacobians (Sec. 2, eq:ta):
//   p = R (X - C); g = (f p1/p3 + cx, f p2/p3 + cy)
//   dg/dp = (f/p3) [[1, 0, -p1/p3], [0, 1, -p2/p3]]
//   dp/dw = -[p]x (rotation increment left-multiplied), dp/dC = -R, dp/dX = R
// A = dg/d(w, C) (2x6), B = dg/dX (2x3).  With intrinsics A has two more
// columns, dg/df and dg/dk1 (see linearise_cal); they are zero otherwise.
struct Lin {
  double g[2];
  double p[3];
  double A[2][8];
  double B[2][3];
};

void linearise(const Cam& cam, const double X[3], double f, double cx, double cy, Lin& o) {
  double d[3] = {X[0] - cam.C[0], X[1] - cam.C[1], X[2] - cam.C[2]};
  for (int r = 0; r < 3; ++r) o.p[r] = cam.R[r][0] * d[0] + cam.R[r][1] * d[1] + cam.R[r][2] * d[2];
  double z = o.p[2];
  o.g[0] = f * o.p[0] / z + cx;
  o.g[1] = f * o.p[1] / z + cy;
  double Jp[2][3] = {{f / z, 0.0, -f * o.p[0] / (z * z)}, {0.0, f / z, -f * o.p[1] / (z * z)}};
  double mpx[3][3] = {{0, o.p[2], -o.p[1]}, {-o.p[2], 0, o.p[0]}, {o.p[1], -o.p[0], 0}};  // -[p]x
  for (int r = 0; r < 2; ++r) {
    for (int c = 0; c < 3; ++c) {
      double sB = 0, sW = 0;
      for (int m = 0; m < 3; ++m) {
        sB += Jp[r][m] * cam.R[m][c];
        sW += Jp[r][m] * mpx[m][c];
      }
      o.B[r][c] = sB;
      o.A[r][c] = sW;
      o.A[r][3 + c] = -sB;
    }
    o.A[r][6] = o.A[r][7] = 0.0;
  }
}

// Projection with the camera's own focal length f and first (quadratic)
// radial distortion parameter k1, both estimated with the pose (Sec. 6: the
// Final data sets, n (6 + 2) camera parameters).  The distortion acts on the
// normalised image coordinates q = (p1/p3, p2/p3), r2 = |q|^2:
//   g = f (1 + k1 r2) q + c
//   dg/dq = f ((1 + k1 r2) I + 2 k1 q q^T),  dq/dp = (1/p3) [[1, 0, -q1], [0, 1, -q2]]
//   dg/df = (1 + k1 r2) q,  dg/dk1 = f r2 q
// Camera parameter order (w_x, w_y, w_z, c_x, c_y, c_z, f, k1).
void linearise_cal(const Cam& cam, const double X[3], double cx, double cy, Lin& o) {
  double d[3] = {X[0] - cam.C[0], X[1] - cam.C[1], X[2] - cam.C[2]};
  for (int r = 0; r < 3; ++r) o.p[r] = cam.R[r][0] * d[0] + cam.R[r][1] * d[1] + cam.R[r][2] * d[2];
  double z = o.p[2];
  double q[2] = {o.p[0] / z, o.p[1] / z};
  double r2 = q[0] * q[0] + q[1] * q[1];
  double s = 1.0 + cam.k1 * r2;
  o.g[0] = cam.f * s * q[0] + cx;
  o.g[1] = cam.f * s * q[1] + cy;
  double Dq[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) Dq[r][c] = cam.f * ((r == c ? s : 0.0) + 2.0 * cam.k1 * q[r] * q[c]);
  double dqdp[2][3] = {{1.0 / z, 0.0, -q[0] / z}, {0.0, 1.0 / z, -q[1] / z}};
  double Jp[2][3];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) Jp[r][c] = Dq[r][0] * dqdp[0][c] + Dq[r][1] * dqdp[1][c];
  double mpx[3][3] = {{0, o.p[2], -o.p[1]}, {-o.p[2], 0, o.p[0]}, {o.p[1], -o.p[0], 0}};  // -[p]x
  for (int r = 0; r < 2; ++r) {
    for (int c = 0; c < 3; ++c) {
      double sB = 0, sW = 0;
      for (int m = 0; m < 3; ++m) {
        sB += Jp[r][m] * cam.R[m][c];
        sW += Jp[r][m] * mpx[m][c];
      }
      o.B[r][c] = sB;
      o.A[r][c] = sW;
      o.A[r][3 + c] = -sB;
    }
    o.A[r][6] = s * q[r];
    o.A[r][7] = cam.f * r2 * q[r];
  }
}

// Cholesky of a symmetric 3x3; pivot test relative to the largest diagonal.
bool chol3(const double H[3][3], double Lc[3][3]) {
  double dmax = std::max(H[0][0], std::max(H[1][1], H[2][2]));
  if (!(dmax > 0)) return false;
  double thr = 1e-12 * dmax;
  std::memset(Lc, 0, sizeof(double) * 9);
  double p0 = H[0][0];
  if (!(p0 > thr)) return false;
  Lc[0][0] = std::sqrt(p0);
  Lc[1][0] = H[1][0] / Lc[0][0];
  Lc[2][0] = H[2][0] / Lc[0][0];
  double p1 = H[1][1] - Lc[1][0] * Lc[1][0];
  if (!(p1 > thr)) return false;
  Lc[1][1] = std::sqrt(p1);
  Lc[2][1] = (H[2][1] - Lc[2][0] * Lc[1][0]) / Lc[1][1];
  double p2 = H[2][2] - Lc[2][0] * Lc[2][0] - Lc[2][1] * Lc[2][1];
  if (!(p2 > thr)) return false;
  Lc[2][2] = std::sqrt(p2);
  return true;
}

void chol3_solve(const double Lc[3][3], const double b[3], double x[3]) {
  double y[3];
  for (int i = 0; i < 3; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= Lc[i][k] * y[k];
    y[i] = s / Lc[i][i];
  }
  for (int i = 2; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 3; ++k) s -= Lc[k][i] * x[k];
    x[i] = s / Lc[i][i];
  }
}

void chol3_inverse(const double Lc[3][3], double Inv[3][3]) {
  for (int c = 0; c < 3; ++c) {
    double e[3] = {0, 0, 0}, x[3];
    e[c] = 1.0;
    chol3_solve(Lc, e, x);
    for (int r = 0; r < 3; ++r) Inv[r][c] = x[r];
  }
}

// Dense Cholesky S = L L^T (row-major n x n, lower triangle used).  Returns
// false on a non-positive pivot.
bool chol_dense(int n, std::vector<double>& S) {
  for (int j = 0; j < n; ++j) {
    double d = S[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= S[(size_t)j * n + k] * S[(size_t)j * n + k];
    if (!(d > 0)) return false;
    double ljj = std::sqrt(d);
    S[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = S[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= S[(size_t)i * n + k] * S[(size_t)j * n + k];
      S[(size_t)i * n + j] = s / ljj;
    }
  }
  return true;
}

void chol_dense_solve(int n, const std::vector<double>& L, const std::vector<double>& b, std::vector<double>& x) {
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  x.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
}

// ---------------------------------------------------------------- problem
struct Copy {        // a point as seen inside one sub-block
  int blk, pt;
  std::vector<int> obs;  // observation indices, cameras of blk only
  double X[3];           // the sub-block's own estimate X_j^l
  double Om[3][3];       // refined tie-point weight (Sec. 5.1)
};

struct Problem {
  int M, N, K, L;
  int ncp = 6;  // parameters per camera: 6 (pose), 8 with intrinsics (pose, f, k1)
  double f, cx, cy, sigma;
  double lambda, int_tol;
  int int_maxit;
  int variant = V_EXTENDED;
  double rho_t = 1000.0, rho_growth = 1.01, filter_px = 1000.0;
  // adaptive damping (Sec. 5.4, 7): per sub-block lambda, a step that raises
  // the sub-block's cost is taken back and lambda multiplied by lam_up, an
  // accepted step divides it by lam_down, within [lam_min, lam_max]
  int damping = 0;
  double lam_up = 10.0, lam_down = 10.0, lam_min = 1e-12, lam_max = 1e8;
  std::vector<double> lam_blk;
  std::vector<int> rejected;
  std::vector<Cam> cams;
  std::vector<double> X;        // [N][3] global point (start value / intersection result)
  std::vector<double> Xbar;     // [N][3] last intersection result
  std::vector<double> Sig;      // [N][6] covariance (xx, xy, xz, yy, yz, zz)
  std::vector<int> status;      // [N]
  std::vector<double> xy;       // [K][2]
  std::vector<int> ocam, opt;   // [K]
  std::vector<Obs2> info;       // [K] base weight matrix
  std::vector<double> rw;       // [K] robust weight multiplier
  std::vector<int> cblk;        // [M]
  std::vector<std::vector<int>> pt_obs;    // point -> observations
  std::vector<std::vector<int>> blk_cams;  // sub-block -> cameras (ascending)
  std::vector<int> cam_local;              // camera -> index inside its sub-block
  std::vector<Copy> copies;                // sorted by (blk, pt)
  std::vector<std::vector<int>> blk_copies;
  std::vector<std::vector<int>> pt_copies;
  std::vector<double> last_res;            // [K][2] residuals of the last intersection
  std::vector<double> Xt;                  // [copies][3] dual offsets of the plain variants
};

Obs2 weight_of(const Problem& P, int k) {
  Obs2 w = P.info[k];
  w.w11 *= P.rw[k];
  w.w12 *= P.rw[k];
  w.w22 *= P.rw[k];
  return w;
}

// projection of observation k's camera at X: the shared pinhole, or with
// intrinsics the camera's own f and k1
void lin_obs(const Problem& P, int k, const double X[3], Lin& o) {
  if (P.ncp == 8) linearise_cal(P.cams[P.ocam[k]], X, P.cx, P.cy, o);
  else linearise(P.cams[P.ocam[k]], X, P.f, P.cx, P.cy, o);
}

double wnorm2(const Obs2& w, const double v[2]) {
  return w.w11 * v[0] * v[0] + 2 * w.w12 * v[0] * v[1] + w.w22 * v[1] * v[1];
}

// B^T W B (3x3) and B^T W v (3) of one observation, added into H, g.
void add_point_normals(const Lin& li, const Obs2& w, const double v[2], double H[3][3], double g[3]) {
  double WB[2][3];
  for (int c = 0; c < 3; ++c) {
    WB[0][c] = w.w11 * li.B[0][c] + w.w12 * li.B[1][c];
    WB[1][c] = w.w12 * li.B[0][c] + w.w22 * li.B[1][c];
  }
  double Wv[2] = {w.w11 * v[0] + w.w12 * v[1], w.w12 * v[0] + w.w22 * v[1]};
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) H[r][c] += li.B[0][r] * WB[0][c] + li.B[1][r] * WB[1][c];
    g[r] += li.B[0][r] * Wv[0] + li.B[1][r] * Wv[1];
  }
}

// Intersection of one point with all cameras fixed (eq:bars): Gauss-Newton on
// the three coordinates, then covariance H^-1 and the refined weights.
void intersect_point(Problem& P, int j) {
  if (P.status[j] != ST_OK) return;
  const std::vector<int>& ol = P.pt_obs[j];
  double X[3] = {P.X[3 * j], P.X[3 * j + 1], P.X[3 * j + 2]};
  const bool plain = P.variant == V_PLAIN || P.variant == V_PLAIN_REFINED;
  int st = ST_NOT_CONVERGED;
  auto normals = [&](const double* Xc, double H[3][3], double g[3], bool& behind) {
    std::memset(H, 0, sizeof(double) * 9);
    g[0] = g[1] = g[2] = 0;
    behind = false;
    for (int k : ol) {
      Lin li;
      lin_obs(P, k, Xc, li);
      if (!(li.p[2] > 0) && P.rw[k] != 0) behind = true;  // a deleted observation does not count
      double v[2] = {li.g[0] - P.xy[2 * k], li.g[1] - P.xy[2 * k + 1]};
      add_point_normals(li, weight_of(P, k), v, H, g);
    }
  };
  // the plain variants do not move the point: they evaluate at the consensus
  // point X_j
  if (plain) st = ST_OK;
  for (int it = 0; !plain && it < P.int_maxit; ++it) {
    double H[3][3], g[3], Lc[3][3];
    bool behind;
    normals(X, H, g, behind);
    if (behind) {
      st = ST_BEHIND;
      break;
    }
    if (!chol3(H, Lc)) {
      st = ST_ILL;
      break;
    }
    double mg[3] = {-g[0], -g[1], -g[2]}, dX[3];
    chol3_solve(Lc, mg, dX);
    for (int r = 0; r < 3; ++r) X[r] += dX[r];
    double nd = std::sqrt(dX[0] * dX[0] + dX[1] * dX[1] + dX[2] * dX[2]);
    double nx = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    if (nd <= P.int_tol * (1.0 + nx)) {
      st = ST_OK;
      break;
    }
  }
  if (st == ST_OK) {
    // final evaluation at the converged point
    double H[3][3], g[3], Lc[3][3];
    bool behind;
    normals(X, H, g, behind);
    double vmax = 0;  // largest reprojection error, for the filters of the plain variants
    for (int k : ol) {
      if (!plain) break;
      if (P.rw[k] == 0) continue;
      Lin li;
      lin_obs(P, k, X, li);
      vmax = std::max(vmax, std::hypot(li.g[0] - P.xy[2 * k], li.g[1] - P.xy[2 * k + 1]));
    }
    if (behind) st = ST_BEHIND;
    else if (!chol3(H, Lc)) st = ST_ILL;
    else if (plain && (!(std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]) <= 1e10) || vmax > P.filter_px))
      st = ST_FILTERED;
    else {
      double Inv[3][3];
      chol3_inverse(Lc, Inv);
      double* s = &P.Sig[6 * j];
      s[0] = Inv[0][0]; s[1] = Inv[0][1]; s[2] = Inv[0][2];
      s[3] = Inv[1][1]; s[4] = Inv[1][2]; s[5] = Inv[2][2];
      for (int r = 0; r < 3; ++r) P.Xbar[3 * j + r] = P.X[3 * j + r] = X[r];
      // refined weights: Omega^l = H - H^(l), H^(l) from the cameras of l
      for (int ci : P.pt_copies[j]) {
        Copy& cp = P.copies[ci];
        double Hl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, gl[3] = {0, 0, 0};
        for (int k : cp.obs) {
          Lin li;
          lin_obs(P, k, X, li);
          double v[2] = {li.g[0] - P.xy[2 * k], li.g[1] - P.xy[2 * k + 1]};
          add_point_normals(li, weight_of(P, k), v, Hl, gl);
        }
        // tie-point weight by variant; zero for a point seen by one sub-block
        const bool tp = P.pt_copies[j].size() > 1;
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double o = 0;
            if (tp) {
              if (P.variant == V_EXTENDED || P.variant == V_PLAIN_REFINED) o = H[r][c] - Hl[r][c];
              else if (P.variant == V_ALL_CAMERAS) o = H[r][c];
              else o = r == c ? P.rho_t : 0.0;
            }
            cp.Om[r][c] = o;
          }
        if (!plain)
          for (int r = 0; r < 3; ++r) cp.X[r] = X[r];  // X^l starts at Xbar
      }
      for (int k : ol) {
        Lin li;
        lin_obs(P, k, X, li);
        P.last_res[2 * k] = li.g[0] - P.xy[2 * k];
        P.last_res[2 * k + 1] = li.g[1] - P.xy[2 * k + 1];
      }
    }
  }
  P.status[j] = st;
}

void point_stats(const Problem& P, double* stats) {
  double wcost = 0, sq = 0;
  long kv = 0, nv = 0;
  for (int j = 0; j < P.N; ++j) {
    if (P.status[j] != ST_OK) continue;
    ++nv;
    for (int k : P.pt_obs[j]) {
      if (P.rw[k] == 0) continue;  // deleted by the robust step
      double v[2] = {P.last_res[2 * k], P.last_res[2 * k + 1]};
      wcost += wnorm2(weight_of(P, k), v);
      sq += v[0] * v[0] + v[1] * v[1];
      ++kv;
    }
  }
  double red = 2.0 * kv - (double)P.ncp * P.M - 3.0 * nv;
  stats[0] = wcost;
  stats[1] = red > 0 ? std::sqrt(sq / red) : 0.0;
  stats[2] = kv > 0 ? std::sqrt(sq / (2.0 * kv)) : 0.0;
  stats[3] = (double)nv;
}

// ------------------------------------------------- sub-block LM step (eq:bact)
struct BlockSystem {
  int n6 = 0, nc = 0;                      // n6: rows of the RCS, np per camera
  int np = 6;                              // parameters per camera
  std::vector<int> cps;                    // valid copies of the block
  std::vector<double> U;                   // [ncam][np][np] damped
  std::vector<double> gC;                  // [ncam][np]
  std::vector<double> Vinv;                // [nc][3][3] of the damped V
  std::vector<double> gX;                  // [nc][3]
  std::vector<double> S, e;                // dense RCS and right-hand side
  std::vector<std::vector<double>> Y;      // per copy, per observation: N_CX block (np x 3)
  double cost = 0;
  bool ok = true;
};

// centre of the tie-point prior of a copy: Xbar, or for the plain variants
// X_j - Xtilde_j^l (eq:admm7)
void prior_centre(const Problem& P, const Copy& cp, double xb[3]) {
  const bool plain = P.variant == V_PLAIN || P.variant == V_PLAIN_REFINED;
  const int id = (int)(&cp - P.copies.data());
  for (int r = 0; r < 3; ++r) xb[r] = plain ? P.X[3 * cp.pt + r] - P.Xt[3 * (size_t)id + r] : P.Xbar[3 * cp.pt + r];
}

double copy_cost(const Problem& P, const Copy& cp) {
  double c = 0;
  for (int k : cp.obs) {
    Lin li;
    lin_obs(P, k, cp.X, li);
    double v[2] = {li.g[0] - P.xy[2 * k], li.g[1] - P.xy[2 * k + 1]};
    c += wnorm2(weight_of(P, k), v);
  }
  double xb[3];
  prior_centre(P, cp, xb);
  double d[3] = {cp.X[0] - xb[0], cp.X[1] - xb[1], cp.X[2] - xb[2]};
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) c += d[r] * cp.Om[r][s] * d[s];
  return c;
}

// Normal equations of sub-block l with tie-point priors, and the Schur
// complement S = U* - Y V*^-1 Y^T with e = -g_C + Y V*^-1 g_X (Sec. 2, 5.4).
void build_block(const Problem& P, int l, BlockSystem& B) {
  const std::vector<int>& cams = P.blk_cams[l];
  int nca = (int)cams.size();
  const int np = P.ncp;
  B.np = np;
  B.n6 = np * nca;
  B.cps.clear();
  for (int ci : P.blk_copies[l])
    if (P.status[P.copies[ci].pt] == ST_OK) B.cps.push_back(ci);
  B.nc = (int)B.cps.size();
  B.U.assign((size_t)nca * np * np, 0.0);
  B.gC.assign((size_t)nca * np, 0.0);
  B.Vinv.assign((size_t)B.nc * 9, 0.0);
  B.gX.assign((size_t)B.nc * 3, 0.0);
  B.S.assign((size_t)B.n6 * B.n6, 0.0);
  B.e.assign(B.n6, 0.0);
  B.cost = 0;
  B.ok = true;
  const double lam = P.damping ? P.lam_blk[l] : P.lambda;

  // camera blocks U_i, gradients g_C
  std::vector<std::vector<double>>& Ys = B.Y;
  Ys.assign(B.nc, {});
  for (int q = 0; q < B.nc; ++q) {
    const Copy& cp = P.copies[B.cps[q]];
    double V[3][3], gx[3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) V[r][c] = cp.Om[r][c];
    double xb[3];
    prior_centre(P, cp, xb);
    double d[3] = {cp.X[0] - xb[0], cp.X[1] - xb[1], cp.X[2] - xb[2]};
    for (int r = 0; r < 3; ++r) gx[r] = cp.Om[r][0] * d[0] + cp.Om[r][1] * d[1] + cp.Om[r][2] * d[2];
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) B.cost += d[r] * cp.Om[r][s] * d[s];
    Ys[q].assign(cp.obs.size() * np * 3, 0.0);
    for (size_t t = 0; t < cp.obs.size(); ++t) {
      int k = cp.obs[t];
      int a = P.cam_local[P.ocam[k]];
      Lin li;
      lin_obs(P, k, cp.X, li);
      double v[2] = {li.g[0] - P.xy[2 * k], li.g[1] - P.xy[2 * k + 1]};
      Obs2 w = weight_of(P, k);
      B.cost += wnorm2(w, v);
      double WA[2][8], WB[2][3], Wv[2];
      for (int c = 0; c < np; ++c) {
        WA[0][c] = w.w11 * li.A[0][c] + w.w12 * li.A[1][c];
        WA[1][c] = w.w12 * li.A[0][c] + w.w22 * li.A[1][c];
      }
      for (int c = 0; c < 3; ++c) {
        WB[0][c] = w.w11 * li.B[0][c] + w.w12 * li.B[1][c];
        WB[1][c] = w.w12 * li.B[0][c] + w.w22 * li.B[1][c];
      }
      Wv[0] = w.w11 * v[0] + w.w12 * v[1];
      Wv[1] = w.w12 * v[0] + w.w22 * v[1];
      double* U = &B.U[(size_t)a * np * np];
      for (int r = 0; r < np; ++r) {
        for (int c = 0; c < np; ++c) U[r * np + c] += li.A[0][r] * WA[0][c] + li.A[1][r] * WA[1][c];
        B.gC[a * np + r] += li.A[0][r] * Wv[0] + li.A[1][r] * Wv[1];
        for (int c = 0; c < 3; ++c) Ys[q][(t * np + r) * 3 + c] = li.A[0][r] * WB[0][c] + li.A[1][r] * WB[1][c];
      }
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) V[r][c] += li.B[0][r] * WB[0][c] + li.B[1][r] * WB[1][c];
        gx[r] += li.B[0][r] * Wv[0] + li.B[1][r] * Wv[1];
      }
    }
    // damping of the point block, then its inverse (FP64 3x3)
    for (int r = 0; r < 3; ++r) V[r][r] *= (1.0 + lam);
    double Lc[3][3], Inv[3][3];
    if (!chol3(V, Lc)) {
      B.ok = false;
      return;
    }
    chol3_inverse(Lc, Inv);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) B.Vinv[(size_t)q * 9 + r * 3 + c] = Inv[r][c];
    for (int r = 0; r < 3; ++r) B.gX[q * 3 + r] = gx[r];
  }
  // damped camera blocks on the diagonal of S
  for (int a = 0; a < nca; ++a) {
    double* U = &B.U[(size_t)a * np * np];
    for (int r = 0; r < np; ++r) {
      if (U[r * np + r] == 0.0) U[r * np + r] = 1.0;  // camera without any valid observation: parameter held
      else U[r * np + r] *= (1.0 + lam);
    }
    for (int r = 0; r < np; ++r) {
      for (int c = 0; c < np; ++c) B.S[(size_t)(np * a + r) * B.n6 + np * a + c] += U[r * np + c];
      B.e[np * a + r] -= B.gC[a * np + r];
    }
  }
  // outer products of every pair of observations of a copy (Sec. 5.4)
  for (int q = 0; q < B.nc; ++q) {
    const Copy& cp = P.copies[B.cps[q]];
    const double* Vi = &B.Vinv[(size_t)q * 9];
    const double* gx = &B.gX[q * 3];
    size_t m = cp.obs.size();
    for (size_t t1 = 0; t1 < m; ++t1) {
      const double* Y1 = &Ys[q][t1 * np * 3];
      int a1 = P.cam_local[P.ocam[cp.obs[t1]]];
      double Z[8][3];  // Z = Y1 V*^-1
      for (int r = 0; r < np; ++r)
        for (int c = 0; c < 3; ++c) Z[r][c] = Y1[r * 3 + 0] * Vi[0 * 3 + c] + Y1[r * 3 + 1] * Vi[1 * 3 + c] + Y1[r * 3 + 2] * Vi[2 * 3 + c];
      for (int r = 0; r < np; ++r) B.e[np * a1 + r] += Z[r][0] * gx[0] + Z[r][1] * gx[1] + Z[r][2] * gx[2];
      for (size_t t2 = 0; t2 < m; ++t2) {
        const double* Y2 = &Ys[q][t2 * np * 3];
        int a2 = P.cam_local[P.ocam[cp.obs[t2]]];
        for (int r = 0; r < np; ++r)
          for (int c = 0; c < np; ++c)
            B.S[(size_t)(np * a1 + r) * B.n6 + np * a2 + c] -= Z[r][0] * Y2[c * 3 + 0] + Z[r][1] * Y2[c * 3 + 1] + Z[r][2] * Y2[c * 3 + 2];
      }
    }
  }
}

// Back-substitution dX_c = V*^-1 (-g_X - sum_k Y_k^T dC_i(k)).
void back_substitute(const Problem& P, int l, const BlockSystem& B, const std::vector<double>& dC, std::vector<double>& dX) {
  dX.assign((size_t)B.nc * 3, 0.0);
  for (int q = 0; q < B.nc; ++q) {
    const Copy& cp = P.copies[B.cps[q]];
    double rhs[3] = {-B.gX[q * 3], -B.gX[q * 3 + 1], -B.gX[q * 3 + 2]};
    for (int k : cp.obs) {
      int a = P.cam_local[P.ocam[k]];
      Lin li;
      lin_obs(P, k, cp.X, li);
      Obs2 w = weight_of(P, k);
      double WB[2][3];
      for (int c = 0; c < 3; ++c) {
        WB[0][c] = w.w11 * li.B[0][c] + w.w12 * li.B[1][c];
        WB[1][c] = w.w12 * li.B[0][c] + w.w22 * li.B[1][c];
      }
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int r = 0; r < B.np; ++r) s += (li.A[0][r] * WB[0][c] + li.A[1][r] * WB[1][c]) * dC[B.np * a + r];
        rhs[c] -= s;
      }
    }
    const double* Vi = &B.Vinv[(size_t)q * 9];
    for (int r = 0; r < 3; ++r) dX[q * 3 + r] = Vi[r * 3] * rhs[0] + Vi[r * 3 + 1] * rhs[1] + Vi[r * 3 + 2] * rhs[2];
  }
  (void)l;
}

void apply_update(Problem& P, int l, const BlockSystem& B, const std::vector<double>& dC, const std::vector<double>& dX) {
  const std::vector<int>& cams = P.blk_cams[l];
  const int np = B.np;
  for (size_t a = 0; a < cams.size(); ++a) {
    Cam& cm = P.cams[cams[a]];
    double w[3] = {dC[np * a], dC[np * a + 1], dC[np * a + 2]}, Rw[3][3], Rn[3][3];
    rodrigues(w, Rw);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Rn[r][c] = Rw[r][0] * cm.R[0][c] + Rw[r][1] * cm.R[1][c] + Rw[r][2] * cm.R[2][c];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) cm.R[r][c] = Rn[r][c];
    for (int r = 0; r < 3; ++r) cm.C[r] += dC[np * a + 3 + r];
    if (np == 8) {  // intrinsics: additive updates
      cm.f += dC[np * a + 6];
      cm.k1 += dC[np * a + 7];
    }
  }
  for (int q = 0; q < B.nc; ++q) {
    Copy& cp = P.copies[B.cps[q]];
    for (int r = 0; r < 3; ++r) cp.X[r] += dX[q * 3 + r];
  }
}

// raise or lower the sub-block's damping after a rejected / accepted step
void adapt_lambda(Problem& P, int l, bool rejected) {
  if (!P.damping) return;
  P.rejected[l] = rejected ? 1 : 0;
  P.lam_blk[l] = rejected ? std::min(P.lam_blk[l] * P.lam_up, P.lam_max) : std::max(P.lam_blk[l] / P.lam_down, P.lam_min);
}

int lm_step_block(Problem& P, int l, double* bs) {
  BlockSystem B;
  build_block(P, l, B);
  bs[0] = B.cost;
  if (!B.ok) {
    adapt_lambda(P, l, true);
    return 1;
  }
  std::vector<double> Lf = B.S;
  if (!chol_dense(B.n6, Lf)) {
    adapt_lambda(P, l, true);
    return 2;
  }
  std::vector<double> dC, dX;
  chol_dense_solve(B.n6, Lf, B.e, dC);
  back_substitute(P, l, B, dC, dX);
  // the state before the step, to take a rejected step back exactly
  std::vector<Cam> cams0;
  std::vector<std::array<double, 3>> X0;
  if (P.damping) {
    for (int i : P.blk_cams[l]) cams0.push_back(P.cams[i]);
    for (int ci : B.cps) X0.push_back({P.copies[ci].X[0], P.copies[ci].X[1], P.copies[ci].X[2]});
  }
  apply_update(P, l, B, dC, dX);
  double c = 0, nrm = 0;
  for (int ci : B.cps) c += copy_cost(P, P.copies[ci]);
  for (double x : dC) nrm += x * x;
  for (double x : dX) nrm += x * x;
  bs[1] = c;
  bs[2] = std::sqrt(nrm);
  bs[3] = 1.0;
  if (P.damping) {
    const bool rej = c > bs[0];
    if (rej) {
      for (size_t a = 0; a < cams0.size(); ++a) P.cams[P.blk_cams[l][a]] = cams0[a];
      for (size_t q = 0; q < X0.size(); ++q)
        for (int r = 0; r < 3; ++r) P.copies[B.cps[q]].X[r] = X0[q][r];
      bs[1] = bs[0];
      bs[2] = 0.0;
    }
    adapt_lambda(P, l, rej);
  }
  return 0;
}

// ------------------------------------------------- robust weights (Sec. 5.3)
double median_sorted(const std::vector<double>& a) {
  size_t n = a.size();
  if (n == 0) return 0.0;
  return 0.5 * (a[(n - 1) / 2] + a[n / 2]);
}

}  // namespace

// ============================================================== C interface
extern "C" {

struct orc_problem {
  Problem P;
};

orc_problem* orc_create(int M, int N, int K, int L, double f, double cx, double cy, double sigma_px,
                        const double* cam_R, const double* cam_C, const double* pts, const double* obs_xy,
                        const int32_t* obs_cam, const int32_t* obs_pt, const double* obs_info,
                        const int32_t* cam_block, double lambda, double int_tol, int int_maxit, int variant,
                        double rho, double rho_growth, double filter_px) {
  orc_problem* h = new orc_problem;
  Problem& P = h->P;
  P.variant = variant;
  P.rho_t = rho;
  P.rho_growth = rho_growth;
  P.filter_px = filter_px;
  P.M = M; P.N = N; P.K = K; P.L = L;
  P.f = f; P.cx = cx; P.cy = cy; P.sigma = sigma_px;
  P.lambda = lambda; P.int_tol = int_tol; P.int_maxit = int_maxit;
  P.cams.resize(M);
  for (int i = 0; i < M; ++i) {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) P.cams[i].R[r][c] = cam_R[(size_t)i * 9 + r * 3 + c];
    for (int r = 0; r < 3; ++r) P.cams[i].C[r] = cam_C[(size_t)r * M + i];
  }
  P.X.resize((size_t)3 * N);
  for (int j = 0; j < N; ++j)
    for (int r = 0; r < 3; ++r) P.X[3 * j + r] = pts[(size_t)r * N + j];
  P.Xbar = P.X;
  P.Sig.assign((size_t)6 * N, 0.0);
  P.status.assign(N, ST_OK);
  P.xy.resize((size_t)2 * K);
  P.ocam.assign(obs_cam, obs_cam + K);
  P.opt.assign(obs_pt, obs_pt + K);
  P.info.resize(K);
  P.rw.assign(K, 1.0);
  P.last_res.assign((size_t)2 * K, 0.0);
  double w0 = 1.0 / (sigma_px * sigma_px);
  for (int k = 0; k < K; ++k) {
    P.xy[2 * k] = obs_xy[k];
    P.xy[2 * k + 1] = obs_xy[(size_t)K + k];
    if (obs_info) P.info[k] = {obs_info[k], obs_info[(size_t)K + k], obs_info[(size_t)2 * K + k]};
    else P.info[k] = {w0, 0.0, w0};
  }
  P.cblk.assign(cam_block, cam_block + M);
  P.blk_cams.assign(L, {});
  P.cam_local.assign(M, 0);
  for (int i = 0; i < M; ++i) {
    P.cam_local[i] = (int)P.blk_cams[P.cblk[i]].size();
    P.blk_cams[P.cblk[i]].push_back(i);
  }
  P.pt_obs.assign(N, {});
  for (int k = 0; k < K; ++k) P.pt_obs[P.opt[k]].push_back(k);
  // copies: one per (sub-block, point) pair, sorted by (sub-block, point);
  // the observations of a copy sorted by camera
  std::vector<int> ord(K);
  for (int k = 0; k < K; ++k) ord[k] = k;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    int la = P.cblk[P.ocam[a]], lb = P.cblk[P.ocam[b]];
    if (la != lb) return la < lb;
    if (P.opt[a] != P.opt[b]) return P.opt[a] < P.opt[b];
    if (P.ocam[a] != P.ocam[b]) return P.ocam[a] < P.ocam[b];
    return a < b;
  });
  P.blk_copies.assign(L, {});
  P.pt_copies.assign(N, {});
  for (int q = 0; q < K;) {
    int k0 = ord[q];
    int l = P.cblk[P.ocam[k0]], j = P.opt[k0];
    Copy c;
    c.blk = l;
    c.pt = j;
    while (q < K && P.cblk[P.ocam[ord[q]]] == l && P.opt[ord[q]] == j) c.obs.push_back(ord[q++]);
    for (int r = 0; r < 3; ++r) c.X[r] = P.X[3 * c.pt + r];
    std::memset(c.Om, 0, sizeof(c.Om));
    int id = (int)P.copies.size();
    P.copies.push_back(std::move(c));
    P.blk_copies[l].push_back(id);
    P.pt_copies[j].push_back(id);
  }
  P.Xt.assign(3 * P.copies.size(), 0.0);
  return h;
}

void orc_destroy(orc_problem* h) { delete h; }

// One intersection of every valid point (eq:bars + refined weights).
void orc_intersect(orc_problem* h, double* stats) {
  Problem& P = h->P;
#pragma omp parallel for schedule(dynamic, 256)
  for (int j = 0; j < P.N; ++j) intersect_point(P, j);
  if (stats) point_stats(P, stats);
}

// Per-camera MAD scale and robust flagging (Sec. 5.3), from the residuals of
// the last intersection.  Returns the number of flagged observations.
// mode 0: flagged observations weighted down by down_weight (both variants,
//         after basic convergence);
// mode 1: the same, and points with a flagged observation ELIMINATED
//         (parallel variant);
// mode 2: flagged observations deleted (weight 0), and points left with fewer
//         than two observations ELIMINATED (serial variant).
// Deleted observations stay deleted and take no part in scales or flags.
int orc_robust_reweight(orc_problem* h, double t_v, double down_weight, int mode, double* sigma_cam) {
  Problem& P = h->P;
  std::vector<std::vector<double>> comp(P.M);
  for (int k = 0; k < P.K; ++k) {
    if (P.status[P.opt[k]] != ST_OK || P.rw[k] == 0) continue;
    const Obs2& w = P.info[k];
    double l11 = std::sqrt(w.w11), l21 = w.w12 / l11, l22 = std::sqrt(w.w22 - l21 * l21);
    double v0 = P.last_res[2 * k], v1 = P.last_res[2 * k + 1];
    comp[P.ocam[k]].push_back(l11 * v0 + l21 * v1);
    comp[P.ocam[k]].push_back(l22 * v1);
  }
  std::vector<double> s0(P.M, 0.0);
  for (int i = 0; i < P.M; ++i) {
    std::vector<double> a = comp[i];
    std::sort(a.begin(), a.end());
    double med = median_sorted(a);
    for (double& x : a) x = std::fabs(x - med);
    std::sort(a.begin(), a.end());
    s0[i] = 1.4826 * median_sorted(a);
    if (sigma_cam) sigma_cam[i] = s0[i];
  }
  int nflag = 0;
  std::vector<char> bad(P.N, 0);
  for (int k = 0; k < P.K; ++k) {
    if (P.rw[k] == 0) continue;  // deleted earlier
    P.rw[k] = 1.0;
    if (P.status[P.opt[k]] != ST_OK) continue;
    double v[2] = {P.last_res[2 * k], P.last_res[2 * k + 1]};
    double vb = std::sqrt(wnorm2(P.info[k], v));
    double s = s0[P.ocam[k]];
    if (s > 0 && vb > t_v * s) {
      P.rw[k] = mode == 2 ? 0.0 : down_weight;
      ++nflag;
      bad[P.opt[k]] = 1;
    }
  }
  for (int j = 0; j < P.N; ++j) {
    if (!bad[j] || P.status[j] != ST_OK) continue;
    int live = 0;
    for (int k : P.pt_obs[j]) live += P.rw[k] != 0;
    if (mode == 1 || (mode == 2 && live < 2)) P.status[j] = ST_ELIMINATED;
  }
  return nflag;
}

// One LM step on every active sub-block (eq:bact).  block_stats[L][4] =
// (cost before, cost after, step norm, solver iterations).  Returns the
// number of sub-blocks whose system could not be factorised.
int orc_lm_step(orc_problem* h, const uint8_t* active, double* block_stats) {
  Problem& P = h->P;
  int fails = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : fails)
  for (int l = 0; l < P.L; ++l) {
    double* bs = &block_stats[4 * l];
    bs[0] = bs[1] = bs[2] = bs[3] = 0.0;
    if (active && !active[l]) continue;
    if (lm_step_block(P, l, bs) != 0) ++fails;
  }
  return fails;
}

// Consensus exchange: every point's start value for the next intersection is
// the mean of its sub-block copies (eq:admm8 form).  stats[0] = largest
// distance of a copy from that mean, stats[1] = number of tie points.
void orc_consensus(orc_problem* h, double* stats) {
  Problem& P = h->P;
  double dmax = 0;
  long ntp = 0;
  for (int j = 0; j < P.N; ++j) {
    const std::vector<int>& cl = P.pt_copies[j];
    if (cl.size() > 1) ++ntp;
    if (P.status[j] != ST_OK) continue;
    double m[3] = {0, 0, 0};
    for (int ci : cl)
      for (int r = 0; r < 3; ++r) m[r] += P.copies[ci].X[r];
    for (int r = 0; r < 3; ++r) m[r] /= (double)cl.size();
    for (int ci : cl) {
      const double* x = P.copies[ci].X;
      double d = std::sqrt((x[0] - m[0]) * (x[0] - m[0]) + (x[1] - m[1]) * (x[1] - m[1]) + (x[2] - m[2]) * (x[2] - m[2]));
      dmax = std::max(dmax, d);
    }
    for (int r = 0; r < 3; ++r) P.X[3 * j + r] = m[r];
    // plain variants: dual update Xtilde_j^l += X_j^l - X_j (eq:admm9)
    if (P.variant == V_PLAIN || P.variant == V_PLAIN_REFINED)
      for (int ci : cl)
        for (int r = 0; r < 3; ++r) P.Xt[3 * (size_t)ci + r] += P.copies[ci].X[r] - m[r];
  }
  P.rho_t *= P.rho_growth;  // the scalar weight of the next outer iteration (Sec. 6.3)
  if (stats) {
    stats[0] = dmax;
    stats[1] = (double)ntp;
  }
}

void orc_get_cameras(orc_problem* h, double* cam_R, double* cam_C) {
  Problem& P = h->P;
  for (int i = 0; i < P.M; ++i) {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) cam_R[(size_t)i * 9 + r * 3 + c] = P.cams[i].R[r][c];
    for (int r = 0; r < 3; ++r) cam_C[(size_t)r * P.M + i] = P.cams[i].C[r];
  }
}

void orc_set_cameras(orc_problem* h, const double* cam_R, const double* cam_C) {
  Problem& P = h->P;
  for (int i = 0; i < P.M; ++i) {
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) P.cams[i].R[r][c] = cam_R[(size_t)i * 9 + r * 3 + c];
    for (int r = 0; r < 3; ++r) P.cams[i].C[r] = cam_C[(size_t)r * P.M + i];
  }
}

// Intrinsics (Sec. 6, the Final data sets): every camera gets its own focal
// length f [M] and radial distortion k1 [M], estimated with its pose from now
// on (8 parameters per camera).
void orc_set_intrinsics(orc_problem* h, const double* f, const double* k1) {
  Problem& P = h->P;
  P.ncp = 8;
  for (int i = 0; i < P.M; ++i) {
    P.cams[i].f = f[i];
    P.cams[i].k1 = k1[i];
  }
}

void orc_get_intrinsics(orc_problem* h, double* f, double* k1) {
  Problem& P = h->P;
  for (int i = 0; i < P.M; ++i) {
    f[i] = P.ncp == 8 ? P.cams[i].f : P.f;
    k1[i] = P.ncp == 8 ? P.cams[i].k1 : 0.0;
  }
}

void orc_get_points(orc_problem* h, double* pts) {
  Problem& P = h->P;
  for (int j = 0; j < P.N; ++j)
    for (int r = 0; r < 3; ++r) pts[(size_t)r * P.N + j] = P.X[3 * j + r];
}

void orc_get_intersection(orc_problem* h, double* xbar, double* cov, int32_t* status) {
  Problem& P = h->P;
  for (int j = 0; j < P.N; ++j) {
    if (xbar)
      for (int r = 0; r < 3; ++r) xbar[(size_t)r * P.N + j] = P.Xbar[3 * j + r];
    if (cov)
      for (int r = 0; r < 6; ++r) cov[(size_t)r * P.N + j] = P.Sig[6 * j + r];
    if (status) status[j] = P.status[j];
  }
}

int orc_num_copies(orc_problem* h) { return (int)h->P.copies.size(); }

// Copies in (sub-block, point) order: sub-block, point, X^l (3), Omega (6:
// xx, xy, xz, yy, yz, zz).
void orc_get_copies(orc_problem* h, int32_t* blk, int32_t* pt, double* X, double* om) {
  Problem& P = h->P;
  for (size_t c = 0; c < P.copies.size(); ++c) {
    const Copy& cp = P.copies[c];
    if (blk) blk[c] = cp.blk;
    if (pt) pt[c] = cp.pt;
    if (X)
      for (int r = 0; r < 3; ++r) X[3 * c + r] = cp.X[r];
    if (om) {
      double* o = &om[6 * c];
      o[0] = cp.Om[0][0]; o[1] = cp.Om[0][1]; o[2] = cp.Om[0][2];
      o[3] = cp.Om[1][1]; o[4] = cp.Om[1][2]; o[5] = cp.Om[2][2];
    }
  }
}

// Test hook: place every copy X_j^l by hand (copies in (sub-block, point)
// order, [n][3]), e.g. to pin the consensus mean against hand-computed values.
void orc_set_copies(orc_problem* h, const double* X) {
  Problem& P = h->P;
  for (size_t c = 0; c < P.copies.size(); ++c)
    for (int r = 0; r < 3; ++r) P.copies[c].X[r] = X[3 * c + r];
}

// Test hook: replace the residuals of the last intersection ([2][K], pixels),
// e.g. to pin the robust scale against a hand-computed MAD.
void orc_set_residuals(orc_problem* h, const double* res) {
  Problem& P = h->P;
  for (int k = 0; k < P.K; ++k) {
    P.last_res[2 * k] = res[k];
    P.last_res[2 * k + 1] = res[(size_t)P.K + k];
  }
}

// Dual offsets Xtilde of the copies of the plain variants ([n][3], copies in
// (sub-block, point) order).
void orc_get_duals(orc_problem* h, double* Xt) {
  std::memcpy(Xt, h->P.Xt.data(), sizeof(double) * h->P.Xt.size());
}

void orc_get_weights(orc_problem* h, double* w) {
  std::memcpy(w, h->P.rw.data(), sizeof(double) * h->P.K);
}

void orc_get_residuals(orc_problem* h, double* res /*[2][K]*/) {
  Problem& P = h->P;
  for (int k = 0; k < P.K; ++k) {
    res[k] = P.last_res[2 * k];
    res[(size_t)P.K + k] = P.last_res[2 * k + 1];
  }
}

// Dense RCS and right-hand side of sub-block l at the current state (n6 x n6,
// n6 = parameters per camera x cameras; row-major, both triangles).  Returns
// n6, or -1 if a point block is singular.
int orc_block_rcs(orc_problem* h, int l, double* S, double* e) {
  BlockSystem B;
  build_block(h->P, l, B);
  if (!B.ok) return -1;
  if (S) std::memcpy(S, B.S.data(), sizeof(double) * B.S.size());
  if (e) std::memcpy(e, B.e.data(), sizeof(double) * B.e.size());
  return B.n6;
}

// The Schur-path step of sub-block l without applying it: dC [np n_l], dX for
// the block's valid copies in (point) order [3 nc].  Returns nc, or <0.
int orc_block_step(orc_problem* h, int l, double* dC_out, double* dX_out) {
  Problem& P = h->P;
  BlockSystem B;
  build_block(P, l, B);
  if (!B.ok) return -1;
  std::vector<double> Lf = B.S;
  if (!chol_dense(B.n6, Lf)) return -2;
  std::vector<double> dC, dX;
  chol_dense_solve(B.n6, Lf, B.e, dC);
  back_substitute(P, l, B, dC, dX);
  std::memcpy(dC_out, dC.data(), sizeof(double) * dC.size());
  std::memcpy(dX_out, dX.data(), sizeof(double) * dX.size());
  return B.nc;
}

// Covariances from the normal equations of every sub-block (Sec. 2: the
// inverse of N through the Schur complement), with damping lam in place of
// lambda.  cam_cov [M][np][np] (np = 6, or 8 with intrinsics; row-major, caller
// order): the camera's diagonal
// block of M_CC = S^-1 of its sub-block.  copy_cov [n_copies][6] (xx, xy, xz,
// yy, yz, zz): M_XX = V^-1 + V^-1 (sum_{i,k} Y_i^T M_ik Y_k) V^-1 of the copy,
// V its damped point block (with the tie-point weight), Y_i the N_CX block of
// its observation in camera i; zeros for copies of invalid points.  The
// inverse S^-1 is formed column by column from the dense Cholesky factor.
// Returns 0, or -(l + 1) if sub-block l cannot be factorised.
int orc_covariance(orc_problem* h, double lam, double* cam_cov, double* copy_cov) {
  Problem& P = h->P;
  const double lam0 = P.lambda;
  const int damping0 = P.damping;
  P.lambda = lam;
  P.damping = 0;
  int rc = 0;
  if (copy_cov) std::fill(copy_cov, copy_cov + 6 * P.copies.size(), 0.0);
  for (int l = 0; l < P.L && rc == 0; ++l) {
    BlockSystem B;
    build_block(P, l, B);
    std::vector<double> Lf = B.S;
    if (!B.ok || !chol_dense(B.n6, Lf)) {
      rc = -(l + 1);
      break;
    }
    const int n = B.n6;
    std::vector<double> Minv((size_t)n * n), col, unit(n, 0.0);
    for (int c = 0; c < n; ++c) {
      unit[c] = 1.0;
      chol_dense_solve(n, Lf, unit, col);
      unit[c] = 0.0;
      for (int r = 0; r < n; ++r) Minv[(size_t)r * n + c] = col[r];
    }
    const std::vector<int>& cams = P.blk_cams[l];
    const int np = B.np;
    if (cam_cov)
      for (size_t a = 0; a < cams.size(); ++a)
        for (int r = 0; r < np; ++r)
          for (int c = 0; c < np; ++c)
            cam_cov[(size_t)cams[a] * np * np + r * np + c] = Minv[(np * a + r) * n + np * a + c];
    if (!copy_cov) continue;
    for (int q = 0; q < B.nc; ++q) {
      const int id = B.cps[q];
      const Copy& cp = P.copies[id];
      const double* Vi = &B.Vinv[(size_t)q * 9];
      double Tm[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // sum_{i,k} Y_i^T M_ik Y_k
      const size_t m = cp.obs.size();
      for (size_t t1 = 0; t1 < m; ++t1)
        for (size_t t2 = 0; t2 < m; ++t2) {
          const double* Y1 = &B.Y[q][t1 * np * 3];
          const double* Y2 = &B.Y[q][t2 * np * 3];
          const int a1 = P.cam_local[P.ocam[cp.obs[t1]]], a2 = P.cam_local[P.ocam[cp.obs[t2]]];
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
              double s = 0.0;
              for (int u = 0; u < np; ++u)
                for (int v = 0; v < np; ++v) s += Y1[u * 3 + r] * Minv[(size_t)(np * a1 + u) * n + np * a2 + v] * Y2[v * 3 + c];
              Tm[r][c] += s;
            }
        }
      double VT[3][3], Mx[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) VT[r][c] = Vi[r * 3 + 0] * Tm[0][c] + Vi[r * 3 + 1] * Tm[1][c] + Vi[r * 3 + 2] * Tm[2][c];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Mx[r][c] = Vi[r * 3 + c] + VT[r][0] * Vi[0 * 3 + c] + VT[r][1] * Vi[1 * 3 + c] + VT[r][2] * Vi[2 * 3 + c];
      double* o = copy_cov + 6 * (size_t)id;
      o[0] = Mx[0][0]; o[1] = Mx[0][1]; o[2] = Mx[0][2];
      o[3] = Mx[1][1]; o[4] = Mx[1][2]; o[5] = Mx[2][2];
    }
  }
  P.lambda = lam0;
  P.damping = damping0;
  return rc;
}

// Adaptive damping on (mode 1) or off (0); every sub-block starts at lambda.
void orc_set_damping(orc_problem* h, int mode, double up, double down, double lmin, double lmax) {
  Problem& P = h->P;
  P.damping = mode;
  P.lam_up = up;
  P.lam_down = down;
  P.lam_min = lmin;
  P.lam_max = lmax;
  P.lam_blk.assign(P.L, P.lambda);
  P.rejected.assign(P.L, 0);
}

// Per sub-block damping and whether its last step was rejected.
void orc_get_damping(orc_problem* h, double* lam, int32_t* rejected) {
  Problem& P = h->P;
  for (int l = 0; l < P.L; ++l) {
    if (lam) lam[l] = P.damping ? P.lam_blk[l] : P.lambda;
    if (rejected) rejected[l] = P.damping ? P.rejected[l] : 0;
  }
}

// Linearisation of one observation (for finite-difference pins).
void orc_linearise(const double* R9, const double* C3, const double* X3, double f, double cx, double cy,
                   double* g2, double* A12, double* B6) {
  Cam cm;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) cm.R[r][c] = R9[r * 3 + c];
  for (int r = 0; r < 3; ++r) cm.C[r] = C3[r];
  Lin li;
  linearise(cm, X3, f, cx, cy, li);
  g2[0] = li.g[0];
  g2[1] = li.g[1];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 6; ++c) A12[r * 6 + c] = li.A[r][c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) B6[r * 3 + c] = li.B[r][c];
}

// the same with the camera's own f and k1: A16 is dg/d(w, C, f, k1) (2x8)
void orc_linearise_cal(const double* R9, const double* C3, const double* X3, double f, double k1, double cx,
                       double cy, double* g2, double* A16, double* B6) {
  Cam cm;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) cm.R[r][c] = R9[r * 3 + c];
  for (int r = 0; r < 3; ++r) cm.C[r] = C3[r];
  cm.f = f;
  cm.k1 = k1;
  Lin li;
  linearise_cal(cm, X3, cx, cy, li);
  g2[0] = li.g[0];
  g2[1] = li.g[1];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 8; ++c) A16[r * 8 + c] = li.A[r][c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) B6[r * 3 + c] = li.B[r][c];
}

void orc_rodrigues(const double* w3, double* R9) {
  double R[3][3];
  rodrigues(w3, R);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R9[r * 3 + c] = R[r][c];
}

// Dense Cholesky of an n x n SPD matrix (row-major, in place; lower triangle
// holds L, upper triangle untouched).  Returns 0 or 1 on a non-positive pivot.
int orc_cholesky(int n, double* A) {
  std::vector<double> S(A, A + (size_t)n * n);
  if (!chol_dense(n, S)) return 1;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = S[(size_t)i * n + j];
  return 0;
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
