// Surrogate network kernels: BF16 MFMA products with FP32 accumulation, fused epilogues,
// loss, bias gradients and Adam on FP32 master weights.
//
// Every product is C = A B^T with A [M][K] and B [N][K] row-major BF16 (K a multiple of 32):
//   forward        z = a W^T + b          A = activations, B = W           (epilogue: bias, GELU)
//   backward data  da = dz W              A = dz,          B = W^T stored  (epilogue: * gelu'(z))
//   weight grad    dW = dz^T a            A = dz^T stored, B = a^T stored  (epilogue: FP32 atomic add,
//                                                                           split over K)
// so the forward and backward epilogues also write the transposed copies the next product needs.
// The forward products take the activations as a pair of BF16 arrays (hi + lo, about 16 significant
// bits): rounding every layer's activations to one BF16 value is what limits the network's accuracy,
// the BF16 weights are what it was trained with.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.hpp"

namespace fpn {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// erf by the rational approximation of Abramowitz & Stegun, Handbook of Mathematical Functions,
// formula 7.1.26 (|error| <= 1.5e-7 for all x; odd symmetry for x < 0).  The activations are rounded to
// BF16 (relative spacing 2^-8) right after, so this is far below what the products can see, and it
// costs a reciprocal, an exponential and six FMAs instead of a full-precision erf.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  const float r = fmaf(-p * t, __expf(-ax * ax), 1.0f);
  return copysignf(r, x);
}
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

constexpr int BM = 128, BN = 128, BK = 32, LDT = BK + 8;  // LDS row stride 80 B (bank spread)

// Tile of 128 x 128 per 256-thread workgroup; wave w owns rows 64 (w >> 1), cols 64 (w & 1),
// as 4 x 4 MFMA 16x16x32 tiles.  blockIdx.z splits K (weight gradients).  SPLIT: A is given as
// g.A + g.Alo (a second LDS tile and a second product per k-step).
template <int EPI, bool SPLIT>
__global__ void __launch_bounds__(256) gemm_nt_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][BM * LDT];
  __shared__ __align__(16) uint16_t Bs[2][BN * LDT];
  __shared__ __align__(16) uint16_t Al[SPLIT ? 2 : 1][SPLIT ? BM * LDT : 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int ksplit = gridDim.z;
  const int kchunk = ((g.K / BK + ksplit - 1) / ksplit) * BK;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(g.K, kbeg + kchunk);
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  // global -> register staging: thread t loads rows (t >> 2) and 64 + (t >> 2), 8 elements at k (t & 3) * 8
  const int lr = tid >> 2, lk = (tid & 3) * 8;
  uint4 ra[2], rb[2], rl[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int r = lr + 64 * p;
      const int gm = m0 + r, gn = n0 + r;
      ra[p] = (gm < g.M && k0 < kend) ? *reinterpret_cast<const uint4*>(g.A + int64_t(gm) * g.lda + k0 + lk)
                                      : make_uint4(0, 0, 0, 0);
      rb[p] = (gn < g.N && k0 < kend) ? *reinterpret_cast<const uint4*>(g.B + int64_t(gn) * g.ldb + k0 + lk)
                                      : make_uint4(0, 0, 0, 0);
      if constexpr (SPLIT)
        rl[p] = (gm < g.M && k0 < kend) ? *reinterpret_cast<const uint4*>(g.Alo + int64_t(gm) * g.lda + k0 + lk)
                                        : make_uint4(0, 0, 0, 0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int r = lr + 64 * p;
      *reinterpret_cast<uint4*>(&As[buf][r * LDT + lk]) = ra[p];
      *reinterpret_cast<uint4*>(&Bs[buf][r * LDT + lk]) = rb[p];
      if constexpr (SPLIT) *reinterpret_cast<uint4*>(&Al[buf][r * LDT + lk]) = rl[p];
    }
  };
  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    load(kbeg);
    stash(0);
  }
  __syncthreads();
  const int ar = lane & 15, ak = (lane >> 4) * 8;
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) load(kbeg + (it + 1) * BK);
    bf16x8 af[4], bfr[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) af[a] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 16 * a + ar) * LDT + ak]);
#pragma unroll
    for (int b = 0; b < 4; ++b) bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 16 * b + ar) * LDT + ak]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    if constexpr (SPLIT) {
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = *reinterpret_cast<const bf16x8*>(&Al[buf][(wm + 16 * a + ar) * LDT + ak]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
    if (it + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }

  // accumulator layout: lane holds column (lane & 15), rows 4 (lane >> 4) + e of each 16 x 16 tile
  const int cn = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int n = n0 + wn + 16 * b + cn;
    if (n >= g.N) continue;
    const float bias = (EPI == kEpiBiasGelu || EPI == kEpiBias) ? g.bias[n] : 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + 16 * a + rq + e;
        if (m >= g.M) continue;
        const float v = acc[a][b][e];
        if constexpr (EPI == kEpiBiasGelu) {
          const float z = v + bias;
          if (g.z_out) g.z_out[int64_t(m) * g.ldz + n] = z;
          const float av = gelu(z);
          const uint16_t o = f2bf(av);
          g.C[int64_t(m) * g.ldc + n] = o;
          if (g.Clo) g.Clo[int64_t(m) * g.ldc + n] = f2bf(av - bf2f(o));
          if (g.Ct) g.Ct[int64_t(n) * g.ldct + m] = o;
        } else if constexpr (EPI == kEpiBias) {
          g.Cf[int64_t(m) * g.ldc + n] = v + bias;
        } else if constexpr (EPI == kEpiGeluGrad) {
          const float d = v * gelu_grad(g.zin[int64_t(m) * g.ldz + n]);
          const uint16_t o = f2bf(d);
          g.C[int64_t(m) * g.ldc + n] = o;
          if (g.Ct) g.Ct[int64_t(n) * g.ldct + m] = o;
        } else {  // kEpiAtomic
          atomicAdd(g.Cf + int64_t(m) * g.ldc + n, v);
        }
      }
    }
  }
}

hipError_t gemm_nt(int epi, const GemmArgs& g, int ksplit, hipStream_t stream) {
  if (g.K % BK != 0 || g.M < 0 || g.N < 0 || ksplit < 1) return hipErrorInvalidValue;
  if (g.M == 0 || g.N == 0) return hipSuccess;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, ksplit);
  const bool split = g.Alo != nullptr;
  if (split && (epi == kEpiGeluGrad || epi == kEpiAtomic)) return hipErrorInvalidValue;  // forward products only
  switch (epi) {
    case kEpiBiasGelu:
      if (split) hipLaunchKernelGGL((gemm_nt_kernel<kEpiBiasGelu, true>), grid, dim3(256), 0, stream, g);
      else hipLaunchKernelGGL((gemm_nt_kernel<kEpiBiasGelu, false>), grid, dim3(256), 0, stream, g);
      break;
    case kEpiBias:
      if (split) hipLaunchKernelGGL((gemm_nt_kernel<kEpiBias, true>), grid, dim3(256), 0, stream, g);
      else hipLaunchKernelGGL((gemm_nt_kernel<kEpiBias, false>), grid, dim3(256), 0, stream, g);
      break;
    case kEpiGeluGrad: hipLaunchKernelGGL((gemm_nt_kernel<kEpiGeluGrad, false>), grid, dim3(256), 0, stream, g); break;
    case kEpiAtomic: hipLaunchKernelGGL((gemm_nt_kernel<kEpiAtomic, false>), grid, dim3(256), 0, stream, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP32 master weights [out][in] -> BF16 W [out][in_pad] and W^T [in_pad][out], zero padded.
__global__ void cast_weights_kernel(const float* W, int out, int in, int in_pad, uint16_t* Wb, uint16_t* Wt) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(out) * in_pad) return;
  const int o = int(e / in_pad), i = int(e % in_pad);
  const uint16_t v = (i < in) ? f2bf(W[int64_t(o) * in + i]) : uint16_t(0);
  Wb[e] = v;
  if (Wt) Wt[int64_t(i) * out + o] = v;
}

// Standardised input rows: xb[m][j] = (x[m][j] - mean[j]) / std[j] for j < in, 0 up to in_pad;
// rows m >= n (padding to the tile) are zero.  Optional transposed copy xt[in_pad][ldt].
__global__ void cast_input_kernel(const float* x, int64_t n, int64_t rows, int in, int in_pad, const float* mean,
                                  const float* istd, uint16_t* xb, uint16_t* xt, int64_t ldt, uint16_t* xlo) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * in_pad) return;
  const int64_t m = e / in_pad;
  const int j = int(e % in_pad);
  float v = 0.0f;
  if (m < n && j < in) v = (x[m * in + j] - mean[j]) * istd[j];
  const uint16_t b = f2bf(v);
  xb[e] = b;
  if (xlo) xlo[e] = f2bf(v - bf2f(b));
  if (xt) xt[int64_t(j) * ldt + m] = b;
}

// dL/dy for L = mean (y - t)^2 over n rows x `out` columns; rows >= n (tile padding) get 0.
// Writes dz (BF16, row-major and transposed) and accumulates the loss sum in FP64.
__global__ void loss_grad_kernel(const float* y, const float* t, int64_t n, int64_t rows, int out, uint16_t* dz,
                                 uint16_t* dzt, int64_t ldt, double* loss_sum) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double part = 0.0;
  if (e < rows * out) {
    const int64_t m = e / out;
    const int j = int(e % out);
    float g = 0.0f;
    if (m < n) {
      const float d = y[e] - t[e];
      part = double(d) * double(d);
      g = 2.0f * d / float(double(n) * out);
    }
    const uint16_t b = f2bf(g);
    dz[e] = b;
    dzt[int64_t(j) * ldt + m] = b;
  }
  // wavefront sum, then one FP64 atomic per wavefront
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if ((threadIdx.x & 63) == 0 && loss_sum) atomicAdd(loss_sum, part);
}

// db[j] = sum_m dzt[j][m] (FP32), one workgroup per output unit.
__global__ void bias_grad_kernel(const uint16_t* dzt, int64_t ldt, int64_t rows, float* db) {
  const int j = blockIdx.x;
  float s = 0.0f;
  for (int64_t m = threadIdx.x; m < rows; m += blockDim.x) s += bf2f(dzt[int64_t(j) * ldt + m]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = red[0];
}

__global__ void fill_kernel(float* p, int64_t n, float v) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// Adam (Kingma & Ba) on FP32 master parameters; bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

static inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

hipError_t cast_weights(const float* W, int out, int in, int in_pad, uint16_t* Wb, uint16_t* Wt, hipStream_t s) {
  const int64_t n = int64_t(out) * in_pad;
  hipLaunchKernelGGL(cast_weights_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, W, out, in, in_pad, Wb, Wt);
  return hipGetLastError();
}
hipError_t cast_input(const float* x, int64_t n, int64_t rows, int in, int in_pad, const float* mean,
                      const float* istd, uint16_t* xb, uint16_t* xt, int64_t ldt, hipStream_t s, uint16_t* xlo) {
  const int64_t e = rows * in_pad;
  if (e == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_input_kernel, dim3(blocks(e, 256)), dim3(256), 0, s, x, n, rows, in, in_pad, mean, istd,
                     xb, xt, ldt, xlo);
  return hipGetLastError();
}
hipError_t loss_grad(const float* y, const float* t, int64_t n, int64_t rows, int out, uint16_t* dz, uint16_t* dzt,
                     int64_t ldt, double* loss_sum, hipStream_t s) {
  const int64_t e = rows * out;
  if (e == 0) return hipSuccess;
  hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks(e, 256)), dim3(256), 0, s, y, t, n, rows, out, dz, dzt, ldt,
                     loss_sum);
  return hipGetLastError();
}
hipError_t bias_grad(const uint16_t* dzt, int64_t ldt, int64_t rows, int out, float* db, hipStream_t s) {
  hipLaunchKernelGGL(bias_grad_kernel, dim3(out), dim3(256), 0, s, dzt, ldt, rows, db);
  return hipGetLastError();
}
hipError_t fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace mlp
}  // namespace fpn
