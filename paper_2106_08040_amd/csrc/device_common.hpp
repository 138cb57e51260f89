// Shared device-side definitions of the fpn kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace fpn {

// Per-instance data prepared by the instance kernel (FP64).
struct InstParams {
  double inv2tau, sigma, beta_T, alpha;  // particle scalars
  double R[9];                           // easy-axis frame, row-major, R e_z = n
  double off[3];                         // static offset mu0*H [T], lab frame
};

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
  int32_t* boff;       // [L+1]
  int32_t* bn;         // [L+1]
  int64_t inv_doubles; // sum of bn^2
};

// RODAS4 (Hairer & Wanner), in the form
//   (I/(h g) - J) K_i = f(t + al_i h, y + sum_j a_ij K_j) + sum_j (c_ij/h) K_j + h gi_i f_t,
//   y_{n+1} = y_n + sum_i m_i K_i.
// Stage abscissae al = {0, 0.386, 0.21, 0.63, 1, 1}; gamma = 1/4.
struct Rodas4 {
  static constexpr float g = 0.25f;
};

}  // namespace fpn
