// Host builder of the easy-axis-frame Galerkin tables (see structure.hpp for the identities).
#include "structure.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "physics.hpp"

namespace fpn {
namespace {

inline int idx(int l, int m) { return l * l + l + m; }

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Real orthonormal harmonics (no Condon-Shortley phase) up to degree Lmax at one point.
void real_sh_point(int Lmax, double ct, double st, double phi, double* Y) {
  std::vector<double> pl((Lmax + 1) * (Lmax + 1));
  auto P = [&](int l, int m) -> double& { return pl[l * (Lmax + 1) + m]; };
  double pmm = std::sqrt(1.0 / (4.0 * kPi));
  for (int m = 0; m <= Lmax; ++m) {
    if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
    P(m, m) = pmm;
    if (m + 1 <= Lmax) P(m + 1, m) = std::sqrt(2.0 * m + 3.0) * ct * pmm;
    for (int l = m + 2; l <= Lmax; ++l) {
      double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
      double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
      P(l, m) = a * (ct * P(l - 1, m) - b * P(l - 2, m));
    }
  }
  const double r2 = std::sqrt(2.0);
  for (int l = 0; l <= Lmax; ++l) {
    Y[idx(l, 0)] = P(l, 0);
    for (int m = 1; m <= l; ++m) {
      Y[idx(l, m)] = r2 * P(l, m) * std::cos(m * phi);
      Y[idx(l, -m)] = r2 * P(l, m) * std::sin(m * phi);
    }
  }
}

struct Dense {
  int n;
  std::vector<double> a;
  explicit Dense(int n_) : n(n_), a(size_t(n_) * n_, 0.0) {}
  double& operator()(int i, int j) { return a[size_t(i) * n + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * n + j]; }
};

std::unique_ptr<OperatorTables> build(int L) {
  if (L < 1 || L > 32) throw std::runtime_error("L out of range");
  const int L1 = L + 1;
  const int N = (L + 1) * (L + 1), N1 = (L1 + 1) * (L1 + 1);
  std::vector<int> deg(N1), ord(N1);
  for (int l = 0; l <= L1; ++l)
    for (int m = -l; m <= l; ++m) { deg[idx(l, m)] = l; ord[idx(l, m)] = m; }

  // Quadrature exact for spherical polynomials of degree 2*L1 + 1.
  const int nt = L1 + 3, nph = 2 * L1 + 6;
  std::vector<double> gx, gw;
  gauss_legendre(nt, gx, gw);
  const int Q = nt * nph;
  std::vector<double> Y(size_t(Q) * N1), W(Q), mv(size_t(Q) * 3);
  for (int a = 0; a < nt; ++a) {
    const double ct = gx[a], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    for (int b = 0; b < nph; ++b) {
      const int q = a * nph + b;
      const double ph = 2.0 * kPi * b / nph;
      real_sh_point(L1, ct, st, ph, &Y[size_t(q) * N1]);
      W[q] = gw[a] * 2.0 * kPi / nph;
      mv[3 * q + 0] = st * std::cos(ph);
      mv[3 * q + 1] = st * std::sin(ph);
      mv[3 * q + 2] = ct;
    }
  }
  // Coordinate multiplication matrices (only |l_i - l_j| = 1 is nonzero).
  std::vector<Dense> M(3, Dense(N1));
  for (int i = 0; i < N1; ++i)
    for (int j = i + 1; j < N1; ++j) {
      if (deg[j] != deg[i] + 1 || std::abs(std::abs(ord[j]) - std::abs(ord[i])) > 1) continue;
      double s[3] = {0, 0, 0};
      for (int q = 0; q < Q; ++q) {
        const double yy = W[q] * Y[size_t(q) * N1 + i] * Y[size_t(q) * N1 + j];
        s[0] += yy * mv[3 * q];
        s[1] += yy * mv[3 * q + 1];
        s[2] += yy * mv[3 * q + 2];
      }
      for (int a = 0; a < 3; ++a) {
        const double v = std::fabs(s[a]) < 1e-15 ? 0.0 : s[a];
        M[a](i, j) = v;
        M[a](j, i) = v;
      }
    }
  // Z2 = Mz Mz (truncated to degree L; the intermediate runs to L+1).
  Dense Z2(N);
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N1; ++k) {
      const double a = M[2](i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < N; ++j) Z2(i, j) += a * M[2](k, j);
    }
  // Rotation generators J_a (matrix [J_a]_{ji} = int Y_j (m x grad)_a Y_i); J_z directly.
  std::vector<Dense> J(3, Dense(N));
  const int eps[6][4] = {{0, 1, 2, 1}, {1, 2, 0, 1}, {2, 0, 1, 1}, {0, 2, 1, -1}, {2, 1, 0, -1}, {1, 0, 2, -1}};
  for (int e = 0; e < 6; ++e) {
    const int a = eps[e][0], b = eps[e][1], c = eps[e][2], sg = eps[e][3];
    if (a == 2) continue;
    for (int i = 0; i < N; ++i) {
      const int li = deg[i];
      if (li == 0) continue;
      for (int j = li * li; j < (li + 1) * (li + 1); ++j) {
        double s = 0.0;
        for (int k = (li - 1) * (li - 1); k < li * li; ++k) s += M[b](j, k) * M[c](k, i);
        J[a](j, i) += (2.0 * li + 1.0) * sg * s;
      }
    }
  }
  for (int l = 1; l <= L; ++l)
    for (int m = 1; m <= l; ++m) {
      J[2](idx(l, -m), idx(l, m)) = -m;   // d/dphi cos(m phi) = -m sin(m phi)
      J[2](idx(l, m), idx(l, -m)) = m;
    }

  auto t = std::make_unique<OperatorTables>();
  t->L = L;
  t->N = N;
  std::vector<ShEntry>& E = t->sh;
  auto add = [&](int i, int j, int kind, double v, double scale) {
    if (std::fabs(v) > 1e-13 * scale) E.push_back({i, j, kind, v});
  };
  auto ll = [&](int i) { return double(deg[i]) * (deg[i] + 1.0); };
  for (int i = 0; i < N; ++i) add(i, i, K_LAM, -ll(i), 1.0);
  double sZ = 0, sM = 0, sJ = 0;
  for (double v : Z2.a) sZ = std::max(sZ, std::fabs(v));
  for (int a = 0; a < 3; ++a)
    for (double v : M[a].a) sM = std::max(sM, std::fabs(v));
  for (int a = 0; a < 3; ++a)
    for (double v : J[a].a) sJ = std::max(sJ, std::fabs(v));
  const double sL = ll(N - 1) + 6.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      // G: anisotropy drift
      const double g = 0.5 * (ll(i) - ll(j) + 6.0) * Z2(i, j) - (i == j ? 1.0 : 0.0);
      add(i, j, K_G, g, sL * sZ);
      // P: anisotropy precession [Mz Jz]_{ji}
      double p = 0.0;
      for (int k = 0; k < N; ++k) p += M[2](j, k) * J[2](k, i);
      add(i, j, K_P, p, sM * sJ);
      // F and R for each axis
      const int kf[3] = {K_FX, K_FY, K_FZ}, kr[3] = {K_RX, K_RY, K_RZ};
      for (int a = 0; a < 3; ++a) {
        add(i, j, kf[a], 0.5 * (ll(i) - ll(j) + 2.0) * M[a](i, j), sL * sM);
        add(i, j, kr[a], J[a](j, i), sJ);
      }
    }

  // Block order.
  t->n0 = (L + 1) + ((L + 1) % 2);
  t->nblk = L + 1;
  t->perm.clear();
  for (int k = 0; k <= L; ++k) {
    t->boff.push_back(int(t->perm.size()));
    if (k == 0) {
      for (int l = 0; l <= L; ++l) t->perm.push_back(idx(l, 0));
      if ((L + 1) % 2) t->perm.push_back(-1);
    } else {
      for (int l = k; l <= L; ++l) {
        t->perm.push_back(idx(l, k));
        t->perm.push_back(idx(l, -k));
      }
    }
    t->bn.push_back(int(t->perm.size()) - t->boff.back());
  }
  t->Np = int(t->perm.size());
  t->pos.assign(N, -1);
  for (int p = 0; p < t->Np; ++p)
    if (t->perm[p] >= 0) t->pos[t->perm[p]] = p;
  std::vector<int> blk_of(t->Np);
  for (int k = 0; k <= L; ++k)
    for (int p = t->boff[k]; p < t->boff[k] + t->bn[k]; ++p) blk_of[p] = k;

  // Row-wise tables in block order, sorted by column.
  std::vector<std::vector<ShEntry>> rows(t->Np);
  for (const ShEntry& e : E) {
    const int p = t->pos[e.row], c = t->pos[e.col];
    if (std::abs(blk_of[p] - blk_of[c]) > 1) throw std::runtime_error("coupling beyond neighbouring |m| blocks");
    rows[p].push_back({p, c, e.kind, e.val});
  }
  t->seg.assign(size_t(4) * t->Np, 0);
  for (int p = 0; p < t->Np; ++p) {
    auto& r = rows[p];
    std::stable_sort(r.begin(), r.end(), [](const ShEntry& a, const ShEntry& b) { return a.col < b.col; });
    const int k = blk_of[p];
    const int start = int(t->colkind.size());
    int nB = 0, nD = 0;
    for (const ShEntry& e : r) {
      if (blk_of[e.col] == k - 1) ++nB;
      else if (blk_of[e.col] == k) ++nD;
      t->colkind.push_back(uint32_t(e.col) | (uint32_t(e.kind) << 16));
      t->val.push_back(float(e.val));
      t->val64.push_back(e.val);
    }
    t->seg[4 * p + 0] = start;
    t->seg[4 * p + 1] = start + nB;
    t->seg[4 * p + 2] = start + nB + nD;
    t->seg[4 * p + 3] = int(t->colkind.size());
  }
  // Column-wise upper coupling entries.
  std::vector<std::vector<ShEntry>> cols(t->Np);
  for (int p = 0; p < t->Np; ++p)
    for (const ShEntry& e : rows[p])
      if (blk_of[e.col] == blk_of[p] + 1) cols[e.col].push_back(e);
  t->cptr.assign(t->Np + 1, 0);
  for (int c = 0; c < t->Np; ++c) {
    t->cptr[c] = int(t->crowkind.size());
    for (const ShEntry& e : cols[c]) {
      t->crowkind.push_back(uint32_t(e.row) | (uint32_t(e.kind) << 16));
      t->cval.push_back(float(e.val));
      t->cval64.push_back(e.val);
    }
  }
  t->cptr[t->Np] = int(t->crowkind.size());
  return t;
}

}  // namespace

const OperatorTables& operator_tables(int L) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<OperatorTables>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(L);
  if (it != cache.end()) return *it->second;
  auto t = build(L);
  const OperatorTables& ref = *t;
  cache[L] = std::move(t);
  return ref;
}

void kind_multipliers(double inv2tau, double sigma, double beta_T, double alpha, const double h[3],
                      double mult[K_COUNT]) {
  mult[K_LAM] = inv2tau;
  mult[K_G] = inv2tau * sigma;
  mult[K_P] = inv2tau * 2.0 * sigma / alpha;
  mult[K_FX] = inv2tau * beta_T * h[0];
  mult[K_FY] = inv2tau * beta_T * h[1];
  mult[K_FZ] = inv2tau * beta_T * h[2];
  mult[K_RX] = inv2tau * beta_T * h[0] / alpha;
  mult[K_RY] = inv2tau * beta_T * h[1] / alpha;
  mult[K_RZ] = inv2tau * beta_T * h[2] / alpha;
}

void dense_operator(const OperatorTables& t, const double mult[K_COUNT], double* A) {
  std::fill(A, A + size_t(t.N) * t.N, 0.0);
  for (const ShEntry& e : t.sh) A[size_t(e.row) * t.N + e.col] += mult[e.kind] * e.val;
}

bool easy_axis_frame(const double n[3], double R[9]) {
  const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(std::fabs(nn - 1.0) <= 1e-6)) return false;
  const double z[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
  double a[3] = {1.0, 0.0, 0.0};
  if (std::fabs(z[0]) >= 0.9) { a[0] = 0.0; a[1] = 1.0; }
  double u[3] = {a[1] * z[2] - a[2] * z[1], a[2] * z[0] - a[0] * z[2], a[0] * z[1] - a[1] * z[0]};
  const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (double& x : u) x /= un;
  const double v[3] = {z[1] * u[2] - z[2] * u[1], z[2] * u[0] - z[0] * u[2], z[0] * u[1] - z[1] * u[0]};
  for (int r = 0; r < 3; ++r) {
    R[3 * r + 0] = u[r];
    R[3 * r + 1] = v[r];
    R[3 * r + 2] = z[r];
  }
  return true;
}

}  // namespace fpn
