// FP64 CPU oracle, iterative part: block-preconditioned conjugate gradients on
// a reduced camera system and the learned block preconditioner's network.
//
// TEST INFRASTRUCTURE ONLY (see rpba_oracle.cpp).  Shares nothing with the HIP
// library.
//
// Passages: the RCS is solved by CG preconditioned with the inverses of the
// 6x6 camera blocks on the diagonal ("block-Jacobi", paper Sec. 3 and 5.4);
// stronger preconditioners exist (Sec. 3).  The learned preconditioner keeps
// the block-diagonal form and replaces each inverse block S_ii^-1 = G^-T G^-1
// (S_ii = G G^T) by G^-T L L^T G^-1, with L = I + strict lower part from the
// network output and exp(.) on the diagonal, so a zero output gives exactly
// block-Jacobi and every block stays symmetric positive definite.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// Cholesky of a dense n x n SPD matrix (row-major), lower factor in place.
bool chol(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0)) return false;
    A[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / A[j * n + j];
    }
  }
  return true;
}

// inverse of a lower-triangular 6x6 (row-major)
void tri_inverse6(const double* L, double* X) {
  std::memset(X, 0, sizeof(double) * 36);
  for (int c = 0; c < 6; ++c) {
    X[c * 6 + c] = 1.0 / L[c * 6 + c];
    for (int r = c + 1; r < 6; ++r) {
      double s = 0;
      for (int m = c; m < r; ++m) s += L[r * 6 + m] * X[m * 6 + c];
      X[r * 6 + c] = -s / L[r * 6 + r];
    }
  }
}

// P = Ginv^T Lm Lm^T Ginv for Ginv = G^-1 (lower), Lm lower
void spd_block(const double* Ginv, const double* Lm, double* P) {
  double M[36];  // Lm^T Ginv
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      double s = 0;
      for (int m = 0; m < 6; ++m) s += Lm[m * 6 + r] * Ginv[m * 6 + c];
      M[r * 6 + c] = s;
    }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) {
      double s = 0;
      for (int m = 0; m < 6; ++m) s += M[m * 6 + r] * M[m * 6 + c];
      P[r * 6 + c] = s;
    }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// ------------------------------------------------------------------ network
// Features per camera block (26): the 6 log diagonal entries of S_ii scaled by
// the sub-block mean, its 15 correlations, log(1 + observations), log(1 +
// neighbour blocks), the off-diagonal mass sum_k |S_ik|_F / |S_ii|_F,
// log10(lambda) and the tie-point fraction of its observations.
// Network: 26 -> 64 -> 64 -> 21 with tanh hidden units.
constexpr int NF = 26, NH = 64, NO = 21;
constexpr int NPAR = NF * NH + NH + NH * NH + NH + NH * NO + NO;

struct Net {
  const double *W1, *b1, *W2, *b2, *W3, *b3;
  explicit Net(const double* p) {
    W1 = p;
    b1 = W1 + NF * NH;
    W2 = b1 + NH;
    b2 = W2 + NH * NH;
    W3 = b2 + NH;
    b3 = W3 + NH * NO;
  }
};

// o = network(f); also the hidden activations for the backward pass
void forward(const Net& n, const double* f, double* h1, double* h2, double* o) {
  for (int j = 0; j < NH; ++j) {
    double s = n.b1[j];
    for (int i = 0; i < NF; ++i) s += n.W1[j * NF + i] * f[i];
    h1[j] = std::tanh(s);
  }
  for (int j = 0; j < NH; ++j) {
    double s = n.b2[j];
    for (int i = 0; i < NH; ++i) s += n.W2[j * NH + i] * h1[i];
    h2[j] = std::tanh(s);
  }
  for (int j = 0; j < NO; ++j) {
    double s = n.b3[j];
    for (int i = 0; i < NH; ++i) s += n.W3[j * NH + i] * h2[i];
    o[j] = s;
  }
}

// Lm from the network output: strict lower part o[0..14] (row-major order of
// (r, c), r > c), diagonal exp(o[15..20])
void lower_from_output(const double* o, double* Lm) {
  std::memset(Lm, 0, sizeof(double) * 36);
  int q = 0;
  for (int r = 1; r < 6; ++r)
    for (int c = 0; c < r; ++c) Lm[r * 6 + c] = o[q++];
  for (int r = 0; r < 6; ++r) Lm[r * 6 + r] = std::exp(o[15 + r]);
}

}  // namespace

extern "C" {

// Preconditioned CG on a dense symmetric n x n system (row-major, both
// triangles), x0 = 0, stop when |r|_2 <= tol |e|_2 after an update or after
// maxit iterations.  P: n/6 row-major 6x6 blocks applied block-diagonally, or
// NULL for block-Jacobi (inverses of the diagonal 6x6 blocks of S).  Returns
// the iteration count, or -1 when a diagonal block is not positive definite.
int orc_pcg(int n, const double* S, const double* e, const double* P, double tol, int maxit, double* x,
            double* res_hist) {
  const int nb = n / 6;
  std::vector<double> Pb((size_t)nb * 36);
  if (P) {
    std::memcpy(Pb.data(), P, sizeof(double) * Pb.size());
  } else {
    for (int b = 0; b < nb; ++b) {
      double G[36], Gi[36], I6[36];
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) G[r * 6 + c] = S[(size_t)(6 * b + r) * n + 6 * b + c];
      if (!chol(6, G)) return -1;
      for (int r = 0; r < 6; ++r)
        for (int c = r + 1; c < 6; ++c) G[r * 6 + c] = 0.0;
      tri_inverse6(G, Gi);
      std::memset(I6, 0, sizeof(I6));
      for (int r = 0; r < 6; ++r) I6[r * 6 + r] = 1.0;
      spd_block(Gi, I6, &Pb[(size_t)b * 36]);
    }
  }
  auto apply_P = [&](const std::vector<double>& r, std::vector<double>& z) {
    for (int b = 0; b < nb; ++b)
      for (int q = 0; q < 6; ++q) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Pb[(size_t)b * 36 + q * 6 + m] * r[6 * b + m];
        z[6 * b + q] = s;
      }
  };
  std::vector<double> xv(n, 0.0), r(e, e + n), z(n), p(n), Ap(n);
  const double ne = std::sqrt(dot(r, r));
  apply_P(r, z);
  p = z;
  double rz = dot(r, z);
  int it = 0;
  if (ne == 0.0) {
    std::memcpy(x, xv.data(), sizeof(double) * n);
    return 0;
  }
  while (it < maxit) {
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int j = 0; j < n; ++j) s += S[(size_t)i * n + j] * p[j];
      Ap[i] = s;
    }
    const double alpha = rz / dot(p, Ap);
    for (int i = 0; i < n; ++i) {
      xv[i] += alpha * p[i];
      r[i] -= alpha * Ap[i];
    }
    ++it;
    const double nr = std::sqrt(dot(r, r));
    if (res_hist) res_hist[it - 1] = nr / ne;
    if (nr <= tol * ne) break;
    apply_P(r, z);
    const double rz2 = dot(r, z);
    const double beta = rz2 / rz;
    rz = rz2;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  std::memcpy(x, xv.data(), sizeof(double) * n);
  return it;
}

int orc_mlp_num_params(void) { return NPAR; }

// Features of every camera block of a dense RCS (n x n, both triangles).
// obs_count[nb], tp_frac[nb]; out feat[nb][26].
void orc_mlp_features(int n, const double* S, const double* obs_tp /*[nb][2]: observations, tie-point fraction*/,
                      double lambda, double* feat) {
  const int nb = n / 6;
  double mean_diag = 0;
  for (int i = 0; i < n; ++i) mean_diag += S[(size_t)i * n + i];
  mean_diag /= n;
  for (int b = 0; b < nb; ++b) {
    double* f = feat + (size_t)b * NF;
    double dg[6];
    for (int q = 0; q < 6; ++q) {
      dg[q] = S[(size_t)(6 * b + q) * n + 6 * b + q];
      f[q] = std::log(dg[q] / mean_diag);
    }
    int t = 6;
    for (int r = 1; r < 6; ++r)
      for (int c = 0; c < r; ++c) f[t++] = S[(size_t)(6 * b + r) * n + 6 * b + c] / std::sqrt(dg[r] * dg[c]);
    double fro_ii = 0, off = 0;
    int nnb = 0;
    for (int b2 = 0; b2 < nb; ++b2) {
      double fr = 0;
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          double v = S[(size_t)(6 * b + r) * n + 6 * b2 + c];
          fr += v * v;
        }
      if (b2 == b) fro_ii = fr;
      else if (fr > 0) {
        off += std::sqrt(fr);
        ++nnb;
      }
    }
    f[21] = std::log1p(obs_tp[2 * b]);
    f[22] = std::log1p((double)nnb);
    f[23] = off / std::sqrt(fro_ii);
    f[24] = std::log10(lambda);
    f[25] = obs_tp[2 * b + 1];
  }
}

// Preconditioner blocks P_i = G^-T Lm Lm^T G^-1 from the network output for
// every block of a dense RCS; params may be NULL (zero output: block-Jacobi).
// Ginv_out (optional): the inverse Cholesky factors G^-1 per block.
void orc_mlp_blocks(int n, const double* S, const double* feat, const double* params, double* P, double* Ginv_out) {
  const int nb = n / 6;
  for (int b = 0; b < nb; ++b) {
    double G[36], Gi[36], Lm[36], o[NO], h1[NH], h2[NH];
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) G[r * 6 + c] = (c <= r) ? S[(size_t)(6 * b + r) * n + 6 * b + c] : 0.0;
    chol(6, G);
    for (int r = 0; r < 6; ++r)
      for (int c = r + 1; c < 6; ++c) G[r * 6 + c] = 0.0;
    tri_inverse6(G, Gi);
    if (Ginv_out) std::memcpy(Ginv_out + (size_t)b * 36, Gi, sizeof(Gi));
    if (params) {
      Net net(params);
      forward(net, feat + (size_t)b * NF, h1, h2, o);
    } else {
      std::memset(o, 0, sizeof(o));
    }
    lower_from_output(o, Lm);
    spd_block(Gi, Lm, P + (size_t)b * 36);
  }
}

// Hutchinson estimate of the SPAI-type loss of the block preconditioner,
//   loss = (1/nz) sum_z sum_i |z_i - P_i (S z)_i|^2 / (nb),
// for probes z[nz][n] with w = S z given; returns the loss and its gradient
// with respect to the network parameters (grad[NPAR]).  Ginv: per block the
// inverse Cholesky factor of S_ii (row-major lower 6x6).
// zw: [nz][2][6 nb] = (z, w = S z) probe pairs.
double orc_mlp_loss_grad(int nb, int nz, const double* Ginv, const double* feat, const double* params,
                         const double* zw, double* grad) {
  std::memset(grad, 0, sizeof(double) * NPAR);
  Net net(params);
  double loss = 0;
  const int n = 6 * nb;
  for (int b = 0; b < nb; ++b) {
    const double* f = feat + (size_t)b * NF;
    const double* Gi = Ginv + (size_t)b * 36;
    double h1[NH], h2[NH], o[NO], Lm[36];
    forward(net, f, h1, h2, o);
    lower_from_output(o, Lm);
    double dLm[36];
    std::memset(dLm, 0, sizeof(dLm));
    for (int t = 0; t < nz; ++t) {
      const double* z = zw + (size_t)t * 2 * n + 6 * b;
      const double* w = zw + (size_t)t * 2 * n + n + 6 * b;
      // u = Gi w ; a = Lm^T u ; v = Lm a ; p = Gi^T v ; res = z - p
      double u[6], a[6], v[6], p[6], res[6], q[6], bq[6];
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Gi[r * 6 + m] * w[m];
        u[r] = s;
      }
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Lm[m * 6 + r] * u[m];
        a[r] = s;
      }
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Lm[r * 6 + m] * a[m];
        v[r] = s;
      }
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Gi[m * 6 + r] * v[m];
        p[r] = s;
      }
      double l2 = 0;
      for (int r = 0; r < 6; ++r) {
        res[r] = z[r] - p[r];
        l2 += res[r] * res[r];
      }
      loss += l2;
      // dloss/dp = -2 res ; dv = Gi dp ; dLm += dv a^T + u (Lm^T dv)^T
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Gi[r * 6 + m] * (-2.0 * res[m]);
        q[r] = s;  // dv
      }
      for (int r = 0; r < 6; ++r) {
        double s = 0;
        for (int m = 0; m < 6; ++m) s += Lm[m * 6 + r] * q[m];
        bq[r] = s;  // da = Lm^T dv
      }
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) dLm[r * 6 + c] += q[r] * a[c] + u[r] * bq[c];
    }
    // back to the output: strict lower entries directly, diagonal through exp
    double dout[NO];
    int qn = 0;
    for (int r = 1; r < 6; ++r)
      for (int c = 0; c < r; ++c) dout[qn++] = dLm[r * 6 + c];
    for (int r = 0; r < 6; ++r) dout[15 + r] = dLm[r * 6 + r] * Lm[r * 6 + r];
    const double scale = 1.0 / ((double)nz * nb);
    for (int j = 0; j < NO; ++j) dout[j] *= scale;
    // layer 3
    double* gW1 = grad;
    double* gb1 = gW1 + NF * NH;
    double* gW2 = gb1 + NH;
    double* gb2 = gW2 + NH * NH;
    double* gW3 = gb2 + NH;
    double* gb3 = gW3 + NH * NO;
    double dh2[NH], dh1[NH];
    for (int i = 0; i < NH; ++i) dh2[i] = 0;
    for (int j = 0; j < NO; ++j) {
      gb3[j] += dout[j];
      for (int i = 0; i < NH; ++i) {
        gW3[j * NH + i] += dout[j] * h2[i];
        dh2[i] += dout[j] * net.W3[j * NH + i];
      }
    }
    for (int i = 0; i < NH; ++i) dh2[i] *= 1.0 - h2[i] * h2[i];
    for (int i = 0; i < NH; ++i) dh1[i] = 0;
    for (int j = 0; j < NH; ++j) {
      gb2[j] += dh2[j];
      for (int i = 0; i < NH; ++i) {
        gW2[j * NH + i] += dh2[j] * h1[i];
        dh1[i] += dh2[j] * net.W2[j * NH + i];
      }
    }
    for (int i = 0; i < NH; ++i) dh1[i] *= 1.0 - h1[i] * h1[i];
    for (int j = 0; j < NH; ++j) {
      gb1[j] += dh1[j];
      for (int i = 0; i < NF; ++i) gW1[j * NF + i] += dh1[j] * f[i];
    }
  }
  return loss / ((double)nz * nb);
}

}  // extern "C"
