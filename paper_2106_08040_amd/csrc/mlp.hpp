// Surrogate network kernels (mlp.hip): launch wrappers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fpn {
namespace mlp {

enum : int {
  kEpiBiasGelu = 0,  // C = bf16(gelu(acc + bias)) (+ transposed copy, + FP32 pre-activation)
  kEpiBias = 1,      // Cf = acc + bias (FP32)
  kEpiGeluGrad = 2,  // C = bf16(acc * gelu'(zin)) (+ transposed copy)
  kEpiAtomic = 3     // Cf += acc (FP32 atomics; split over K)
};

// C[M][N] = A[M][K] B[N][K]^T; K % 32 == 0, lda and ldb multiples of 8 (16-byte rows).
struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int M, N, K;
  int64_t lda, ldb;
  uint16_t* C;       // BF16 output [M][ldc]        (kEpiBiasGelu, kEpiGeluGrad)
  uint16_t* Ct;      // optional transposed copy [N][ldct]
  float* Cf;         // FP32 output [M][ldc]        (kEpiBias, kEpiAtomic)
  int64_t ldc, ldct;
  const float* bias; // [N]
  float* z_out;      // optional FP32 pre-activation [M][ldz] (kEpiBiasGelu)
  const float* zin;  // pre-activation read by kEpiGeluGrad [M][ldz]
  int64_t ldz;
  // optional low-order BF16 parts (same layouts as A and C): with Alo the product is
  // (A + Alo) B^T, two matrix-core products per tile; with Clo (kEpiBiasGelu) the output is written
  // as C + Clo, Clo = bf16(value - C), so an activation carries about 16 significant bits
  const uint16_t* Alo;
  uint16_t* Clo;
};

hipError_t gemm_nt(int epi, const GemmArgs& g, int ksplit, hipStream_t stream);
hipError_t cast_weights(const float* W, int out, int in, int in_pad, uint16_t* Wb, uint16_t* Wt, hipStream_t s);
hipError_t cast_input(const float* x, int64_t n, int64_t rows, int in, int in_pad, const float* mean,
                      const float* istd, uint16_t* xb, uint16_t* xt, int64_t ldt, hipStream_t s,
                      uint16_t* xlo = nullptr);
hipError_t loss_grad(const float* y, const float* t, int64_t n, int64_t rows, int out, uint16_t* dz, uint16_t* dzt,
                     int64_t ldt, double* loss_sum, hipStream_t s);
hipError_t bias_grad(const uint16_t* dzt, int64_t ldt, int64_t rows, int out, float* db, hipStream_t s);
hipError_t fill(float* p, int64_t n, float v, hipStream_t s);
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);

}  // namespace mlp
}  // namespace fpn
