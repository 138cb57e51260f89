// Galerkin operator tables of the Fokker-Planck equation in the easy-axis frame.
//
// Paper basis: Eq. FP-general with the drift of Eq. convection.  Writing
// Phi = beta H'.m + sigma (z.m)^2 (easy axis = z) the equation becomes
//   2 tau df/dt = Lap f - div( f (grad Phi - m x grad Phi / alpha) ),
// and its Galerkin matrix on real spherical harmonics Y_i (degree <= L) is
//   2 tau A = Lam + sigma (G + (2/alpha) P) + beta sum_a H'_a (F_a + R_a / alpha).
// Every piece is derived from the coordinate-multiplication matrices
// M_a[i][j] = int m_a Y_i Y_j by exact identities:
//   F_a[i][j] = (l_i(l_i+1) - l_j(l_j+1) + 2)/2 * M_a[i][j]          (drift of a linear potential)
//   G[i][j]   = (l_i(l_i+1) - l_j(l_j+1) + 6)/2 * (M_z M_z)[i][j] - delta_ij  (drift of z^2)
//   [J_a]_{ji} = (2 l_i + 1) eps_abc sum_{l_k = l_i - 1} M_b[j][k] M_c[k][i]  (J = m x grad)
//   R_a[i][j] = [J_a]_{ji},  P[i][j] = [M_z J_z]_{ji}
// M_a itself is computed by exact Gauss quadrature with a normalised associated-
// Legendre recurrence.  Everything here is FP64 host code.
#pragma once
#include <cstdint>
#include <vector>

namespace fpn {

// Entry kinds; the per-instance multiplier of kind k (times 1/(2 tau)) is
//   LAM: 1, G: sigma, P: 2 sigma/alpha, FZ/FX/FY: beta h_a, RZ/RX/RY: beta h_a / alpha.
enum Kind : int { K_LAM = 0, K_G = 1, K_P = 2, K_FZ = 3, K_RZ = 4, K_FX = 5, K_FY = 6, K_RX = 7, K_RY = 8, K_COUNT = 9 };

struct ShEntry {
  int row, col, kind;   // flat SH indices i = l*l + l + m
  double val;
};

// Block order: block k holds |m| = k.  Block 0: l = 0..L (cos type), padded with one
// identity slot when L+1 is odd so every block has even size.  Block k >= 1:
// position 2(l-k) + t for l = k..L, t = 0 (cos, m = +k), t = 1 (sin, m = -k).
struct OperatorTables {
  int L = 0, N = 0, Np = 0, nblk = 0, n0 = 0;
  std::vector<int> perm;       // block position -> SH index (-1 = pad)
  std::vector<int> pos;        // SH index -> block position
  std::vector<int> boff, bn;   // block offsets and sizes (block order)
  std::vector<ShEntry> sh;     // all entries, SH order (host reference)
  // Device tables (block order).  Row segments: for row p,
  // seg[4p+0] = first B entry (cols in block k-1), seg[4p+1] = first D entry (block k),
  // seg[4p+2] = first C entry (block k+1), seg[4p+3] = end.
  std::vector<int32_t> seg;
  std::vector<uint32_t> colkind;   // col | (kind << 16)
  std::vector<float> val;
  std::vector<double> val64;
  // Upper coupling blocks by column: for a column c in block b >= 1, the entries
  // (row in block b-1, value) of C_{b-1}; cptr has Np+1 offsets.
  std::vector<int32_t> cptr;
  std::vector<uint32_t> crowkind;  // row | (kind << 16)
  std::vector<float> cval;
  std::vector<double> cval64;
};

// Cached per L (thread-safe).  1 <= L <= 32.
const OperatorTables& operator_tables(int L);

// Dense A (1/s) in SH order from the entries of `t` with the given multipliers.
void dense_operator(const OperatorTables& t, const double mult[K_COUNT], double* A_out);

// Multipliers of every kind for a particle (FP64).
void kind_multipliers(double inv2tau, double sigma, double beta_T, double alpha,
                      const double h_easy[3], double mult[K_COUNT]);

// Rotation with R * e_z = n (row-major); false if |n| differs from 1 by more than 1e-6.
bool easy_axis_frame(const double n[3], double R[9]);

}  // namespace fpn
