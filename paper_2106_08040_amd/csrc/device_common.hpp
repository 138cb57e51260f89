// Shared device-side definitions of the fpn kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace fpn {

// Per-instance status codes (the FPN_INST_* values of fpn.h).  kInstTolUnmet keeps the outputs (finite,
// accuracy not certified); every other non-zero code leaves NaN outputs.
enum : int {
  kInstOk = 0,
  kInstBadParam = 1,
  kInstNonfinite = 2,
  kInstSingular = 3,
  kInstUnresolved = 4,
  kInstTolUnmet = 5
};
__host__ __device__ inline bool inst_failed(int s) { return s != kInstOk && s != kInstTolUnmet; }
// |m|^2 above which a sampled state is not a probability density: (1 + 1e-3)^2
constexpr float kMaxM2 = 1.002001f;

// Per-instance data prepared by the instance kernel (FP64).
struct InstParams {
  double inv2tau, sigma, beta_T, alpha;  // particle scalars
  double R[9];                           // easy-axis frame, row-major, R e_z = n
  double off[3];                         // static offset mu0*H [T], lab frame
  double D, sigK;                        // diameter [m] and d sigma / d K = V_C / (k_B T) (tangents)
};

// Tangent directions (parameter derivatives) carried by the sensitivity solves.
enum : int { kNTan = 5 };  // D, K, alpha, easy-axis polar angle, easy-axis azimuth

// Lab-frame rotation axis whose infinitesimal rotation moves the easy axis n = R e_z along the
// polar (prm 3: e_phi) or azimuthal (prm 4: e_z) direction.  A rotation of n by e is the same as
// rotating the field by -e and the result by +e, so the angle derivatives need no frame derivative.
template <typename T>
__host__ __device__ inline void tan_axis(int prm, const double* R, T e[3]) {
  if (prm == 4) {
    e[0] = 0; e[1] = 0; e[2] = 1;
    return;
  }
  const double ph = atan2(R[5], R[2]);
  e[0] = T(-sin(ph)); e[1] = T(cos(ph)); e[2] = 0;
}

// d/dp of kind multiplier `kind` (kind numbering of structure.hpp; multipliers as in kind_mult)
// for the field h (easy frame) of the same time: prm 0..2 differentiate the particle scalars, prm 3, 4
// rotate the field by h x e' with e' = R^T e.
template <typename T>
__host__ __device__ inline T tan_mult_t(int prm, int kind, T inv2tau, T sigma, T alpha, T beta, T D, T sigK,
                                        const T h[3], const T ep[3]) {
  const T s = inv2tau;
  const T ia = T(1) / alpha;
  const T m[9] = {s, s * sigma, s * T(2) * sigma * ia, s * beta * h[2], s * beta * h[2] * ia,
                  s * beta * h[0], s * beta * h[1], s * beta * h[0] * ia, s * beta * h[1] * ia};
  const bool over_alpha = (kind == 2 || kind == 4 || kind == 7 || kind == 8);
  switch (prm) {
    case 0: return kind == 0 ? T(-3) * m[0] / D : T(0);
    case 1: return kind == 1 ? s * sigK : (kind == 2 ? s * T(2) * sigK * ia : T(0));
    case 2: {
      const T g = ia - T(2) * alpha / (T(1) + alpha * alpha);  // d ln(1/2tau) / d alpha
      return m[kind] * (over_alpha ? g - ia : g);
    }
    default: {
      if (kind < 3) return T(0);
      const T d[3] = {h[1] * ep[2] - h[2] * ep[1], h[2] * ep[0] - h[0] * ep[2], h[0] * ep[1] - h[1] * ep[0]};
      const T c = (kind == 3 || kind == 4) ? d[2] : ((kind == 5 || kind == 7) ? d[0] : d[1]);
      return s * beta * c * (over_alpha ? ia : T(1));
    }
  }
}

// Device copies of the operator tables of one degree L (see structure.hpp).
struct DevTables {
  int L, N, Np, n0, nnz, nnzc;
  int32_t* seg;        // [4*Np]
  uint32_t* colkind;   // [nnz]
  float* val;          // [nnz]
  double* val64;       // [nnz]
  int32_t* cptr;       // [Np+1]
  uint32_t* crowkind;  // [nnzc]
  float* cval;         // [nnzc]
  double* cval64;      // [nnzc]
  uint16_t* ell_col;   // [kNSlRow][Np] fixed-slot rows (stepper)
  float* ell_val;      // [kNSlRow][Np]
  float* ell_lo;       // [kNSlRow][Np] low-order parts: value = ell_val + ell_lo (the register-layout
                       // stepper reads the first kNSlD rows, the diagonal-block slots)
  uint16_t* ecol_row;  // [kNSlCol][Np] fixed-slot columns of the lower coupling
  float* ecol_val;     // [kNSlCol][Np]
  float* win_b;        // [kNWin][Np] window coefficients (see above)
  float* win_c;        // [kNWin][Np]
  float* win_s;        // [kNWin][Np]
  int32_t* boff;       // [L+1]
  int32_t* bn;         // [L+1]
  int64_t inv_doubles; // sum of bn^2
};

// Fixed-slot (ELL) layout of the operator rows used by the time stepper.  Every row of
// the block-ordered matrix has one slot group per entry kind; the kind of a slot is
// static, so its multiplier is a uniform value and the loops over slots unroll.
//   same |m| block (D):  LAM 1, G 3, P 2, FZ 2, RZ 1
//   block k-1 (B):       FX 2, FY 2, RX 1, RY 1
//   block k+1 (C):       FX 2, FY 2, RX 1, RY 1
// and, by column, the entries of the coupling to block k-1 (C of the previous block):
//   FX 2, FY 2, RX 1, RY 1.  Unused slots hold index 0 and value 0.
enum : int {
  kSlD = 0, kNSlD = 9,
  kSlB = 9, kNSlB = 6,
  kSlC = 15, kNSlC = 6,
  kNSlRow = 21,
  kNSlCol = 6,
  kNKindD = 5  // kinds 0..4 occur in the diagonal-block slots
};
// kind of every row slot and column slot (kind numbering of structure.hpp)
constexpr int kSlotKindRow[kNSlRow] = {0, 1, 1, 1, 2, 2, 3, 3, 4,   // D: LAM G G G P P FZ FZ RZ
                                       5, 5, 6, 6, 7, 8,            // B: FX FX FY FY RX RY
                                       5, 5, 6, 6, 7, 8};           // C
constexpr int kSlotKindCol[kNSlCol] = {5, 5, 6, 6, 7, 8};

// Window layout of the couplings between neighbouring |m| blocks (block-local indices; row or
// column i, type t = i & 1; d = 0, 1, 2 for degree offsets -1, 0, +1).  Slot e = d (same type)
// or 3 + d (other type).  Kinds: same type FX, RY, FX; other type FY, RX, FY (d = 0, 1, 2).
//   B (row i of block K >= 2 -> block K-1):   same i + 2d,      other i + 1 - 2t + 2d
//   C (row i of block K >= 1 -> block K+1):   same i - 4 + 2d,  other i - 3 - 2t + 2d
//     (block 0, cos only:                     same 2i - 4 + 2d, other 2i - 3 + 2d)
//   S (column i of block K >= 2, rows of block K-1): same i + 2d, other i + 1 - 2t + 2d
enum : int { kNWin = 6 };

// RODAS4 (Hairer & Wanner), in the form
//   (I/(h g) - J) K_i = f(t + al_i h, y + sum_j a_ij K_j) + sum_j (c_ij/h) K_j + h gi_i f_t,
//   y_{n+1} = y_n + sum_i m_i K_i.
// Stage abscissae al = {0, 0.386, 0.21, 0.63, 1, 1}; gamma = 1/4.
struct Rodas4 {
  static constexpr float g = 0.25f;
};

}  // namespace fpn
