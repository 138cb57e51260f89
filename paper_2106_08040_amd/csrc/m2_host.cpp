// Model M2 weights on the host (paper: Methods, "Technical details regarding the parameter
// identification", M2: Eq. LSfitM2, its stacked form Eq. LSfitM2_alternative and the truncated-SVD
// regularisation Eq. approx_low_rank), from the Gram matrix G = M^H M and b = M^H y that
// fpn_m2_system forms on the device.
//
// With M = U Sigma V^H, U_s^H M = Sigma_s V_s^H and U_s^H y = Sigma_s^{-1} V_s^H b, so for real w
//   || U_s^H (M w - y) ||^2 = w^T A_s w + 2 f_s^T w + sum_{i<s} |v_i^H b|^2 / lambda_i,
//   A_s = Re(V_s Lambda_s V_s^H),  f_s = -Re(V_s V_s^H b),  G = V Lambda V^H (Lambda = Sigma^2):
// the eigenvectors of the Hermitian J x J matrix G (cyclic complex Jacobi) give the truncation, and
// the non-negative quadratic program min 1/2 w^T A_s w + f_s^T w, w >= 0, is solved by a primal-dual
// interior-point method (Mehrotra predictor-corrector), as the paper solves it.
#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fpn.h"

namespace fpn_internal {
fpn_status fail(fpn_status s, const std::string& msg);
}

namespace {

using cd = std::complex<double>;

// Eigenvalues (descending) and eigenvectors (columns of V, n x n row-major) of a Hermitian matrix.
void jacobi_hermitian(int n, std::vector<cd> A, std::vector<double>& lam, std::vector<cd>& V) {
  V.assign(size_t(n) * n, cd(0.0));
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  auto at = [&](int r, int c) -> cd& { return A[size_t(r) * n + c]; };
  double total = 0.0;
  for (const cd& x : A) total += std::norm(x);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(at(p, q));
    if (off <= 1e-30 * total) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd g = at(p, q);
        const double ag = std::abs(g);
        if (ag <= 1e-300 || ag * ag <= 1e-34 * total) continue;
        const cd e = g / ag;  // phase of the coupling
        const double a = at(p, p).real(), d = at(q, q).real();
        const double th = (d - a) / (2.0 * ag);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // J = diag(1, conj(e)) [[c, s], [-s, c]]
        const cd jpp = c, jpq = s, jqp = -s * std::conj(e), jqq = c * std::conj(e);
        for (int k = 0; k < n; ++k) {  // A <- A J
          const cd xp = at(k, p), xq = at(k, q);
          at(k, p) = xp * jpp + xq * jqp;
          at(k, q) = xp * jpq + xq * jqq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^H A
          const cd yp = at(p, k), yq = at(q, k);
          at(p, k) = std::conj(jpp) * yp + std::conj(jqp) * yq;
          at(q, k) = std::conj(jpq) * yp + std::conj(jqq) * yq;
        }
        at(p, q) = at(q, p) = 0.0;
        at(p, p) = at(p, p).real();
        at(q, q) = at(q, q).real();
        for (int k = 0; k < n; ++k) {  // V <- V J
          cd& vp = V[size_t(k) * n + p];
          cd& vq = V[size_t(k) * n + q];
          const cd xp = vp, xq = vq;
          vp = xp * jpp + xq * jqp;
          vq = xp * jpq + xq * jqq;
        }
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return at(x, x).real() > at(y, y).real(); });
  lam.resize(n);
  std::vector<cd> W(size_t(n) * n);
  for (int j = 0; j < n; ++j) {
    lam[j] = at(ord[j], ord[j]).real();
    for (int k = 0; k < n; ++k) W[size_t(k) * n + j] = V[size_t(k) * n + ord[j]];
  }
  V.swap(W);
}

// In-place Cholesky of a symmetric positive definite n x n matrix (lower factor); false if not PD.
bool cholesky(int n, std::vector<double>& H) {
  for (int j = 0; j < n; ++j) {
    double d = H[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= H[size_t(j) * n + k] * H[size_t(j) * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    H[size_t(j) * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = H[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) v -= H[size_t(i) * n + k] * H[size_t(j) * n + k];
      H[size_t(i) * n + j] = v / d;
    }
  }
  return true;
}

void chol_solve(int n, const std::vector<double>& Lf, std::vector<double>& x) {
  for (int i = 0; i < n; ++i) {
    double v = x[i];
    for (int k = 0; k < i; ++k) v -= Lf[size_t(i) * n + k] * x[k];
    x[i] = v / Lf[size_t(i) * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < n; ++k) v -= Lf[size_t(k) * n + i] * x[k];
    x[i] = v / Lf[size_t(i) * n + i];
  }
}

// min 1/2 w^T Q w + f^T w subject to w >= 0 (Q symmetric positive semidefinite); false if the
// iteration does not reach the tolerance.
bool ipm_nonneg_qp(int n, std::vector<double> Q, std::vector<double> f, std::vector<double>& w) {
  double sc = 0.0;
  for (int i = 0; i < n; ++i) sc = std::max(sc, Q[size_t(i) * n + i]);
  for (double v : f) sc = std::max(sc, std::fabs(v));
  w.assign(n, 0.0);
  if (!(sc > 0.0)) return true;
  for (double& v : Q) v /= sc;
  for (double& v : f) v /= sc;
  std::vector<double> z(n, 1.0), rd(n), H(size_t(n) * n), dwa(n), dza(n), dw(n), dz(n);
  w.assign(n, 1.0);
  double fmax = 0.0;
  for (double v : f) fmax = std::max(fmax, std::fabs(v));
  auto step_to_boundary = [&](const std::vector<double>& x, const std::vector<double>& dx) {
    double a = 1.0;
    for (int i = 0; i < n; ++i)
      if (dx[i] < 0.0) a = std::min(a, -x[i] / dx[i]);
    return a;
  };
  for (int it = 0; it < 300; ++it) {
    double mu = 0.0, rmax = 0.0;
    for (int i = 0; i < n; ++i) {
      double v = f[i] - z[i];
      for (int k = 0; k < n; ++k) v += Q[size_t(i) * n + k] * w[k];
      rd[i] = v;
      rmax = std::max(rmax, std::fabs(v));
      mu += w[i] * z[i];
    }
    mu /= n;
    if (rmax <= 1e-13 * (1.0 + fmax) && mu <= 1e-15) return true;
    H = Q;
    for (int i = 0; i < n; ++i) H[size_t(i) * n + i] += z[i] / w[i] + 1e-15;
    if (!cholesky(n, H)) return false;
    // predictor (affine scaling)
    for (int i = 0; i < n; ++i) dwa[i] = -rd[i] - z[i];
    chol_solve(n, H, dwa);
    for (int i = 0; i < n; ++i) dza[i] = -z[i] - z[i] / w[i] * dwa[i];
    const double ap = step_to_boundary(w, dwa), ad = step_to_boundary(z, dza);
    double mua = 0.0;
    for (int i = 0; i < n; ++i) mua += (w[i] + ap * dwa[i]) * (z[i] + ad * dza[i]);
    mua /= n;
    const double sig = std::pow(mua / mu, 3.0);
    // corrector
    for (int i = 0; i < n; ++i) dw[i] = -rd[i] - z[i] + (sig * mu - dwa[i] * dza[i]) / w[i];
    chol_solve(n, H, dw);
    for (int i = 0; i < n; ++i) dz[i] = (sig * mu - dwa[i] * dza[i]) / w[i] - z[i] - z[i] / w[i] * dw[i];
    const double a1 = std::min(1.0, 0.995 * step_to_boundary(w, dw));
    const double a2 = std::min(1.0, 0.995 * step_to_boundary(z, dz));
    for (int i = 0; i < n; ++i) {
      w[i] += a1 * dw[i];
      z[i] += a2 * dz[i];
    }
  }
  return false;
}

}  // namespace

extern "C" {

fpn_status fpn_m2_weights(int32_t J, const double* G, const double* b, double yy, int32_t s, double* w_out,
                          double* resid_out, double* reduced_out, int32_t* rank_out) {
  if (J < 1 || J > 8192) return fpn_internal::fail(FPN_E_ARG, "J outside [1, 8192]");
  if (!G || !b || !w_out) return fpn_internal::fail(FPN_E_ARG, "NULL argument");
  if (s < 0) return fpn_internal::fail(FPN_E_ARG, "s < 0");
  const int n = J;
  std::vector<cd> A(size_t(n) * n);
  for (size_t e = 0; e < A.size(); ++e) A[e] = cd(G[2 * e], G[2 * e + 1]);
  for (const cd& x : A)
    if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return fpn_internal::fail(FPN_E_ARG, "G not finite");
  std::vector<double> lam;
  std::vector<cd> V;
  jacobi_hermitian(n, A, lam, V);
  int r = 0;
  for (int i = 0; i < n; ++i)
    if (lam[i] > lam[0] * 1e-14 && lam[i] > 0.0) ++r;
  const int se = (s == 0) ? r : std::min(int(s), r);
  std::vector<double> Q(size_t(n) * n, 0.0), f(n, 0.0);
  double cc = 0.0;
  for (int i = 0; i < se; ++i) {
    cd vb(0.0);  // v_i^H b
    for (int k = 0; k < n; ++k) vb += std::conj(V[size_t(k) * n + i]) * cd(b[2 * k], b[2 * k + 1]);
    cc += std::norm(vb) / lam[i];
    for (int p = 0; p < n; ++p) {
      const cd vp = V[size_t(p) * n + i];
      f[p] -= (vp * vb).real();
      for (int q = 0; q < n; ++q) Q[size_t(p) * n + q] += lam[i] * (vp * std::conj(V[size_t(q) * n + i])).real();
    }
  }
  // objective w^T Q w + 2 f^T w + cc: the QP minimises half of it
  std::vector<double> w;
  if (!ipm_nonneg_qp(n, Q, f, w)) return fpn_internal::fail(FPN_E_RANGE, "interior-point iteration did not converge");
  double red = cc, full = yy;
  for (int p = 0; p < n; ++p) {
    double qw = 0.0, gw = 0.0;
    for (int q = 0; q < n; ++q) {
      qw += Q[size_t(p) * n + q] * w[q];
      gw += G[2 * (size_t(p) * n + q)] * w[q];
    }
    red += w[p] * qw + 2.0 * f[p] * w[p];
    full += w[p] * gw - 2.0 * b[2 * p] * w[p];
  }
  for (int p = 0; p < n; ++p) w_out[p] = w[p];
  if (resid_out) *resid_out = full;
  if (reduced_out) *reduced_out = red;
  if (rank_out) *rank_out = se;
  return FPN_OK;
}

}  // extern "C"
