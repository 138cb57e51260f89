// Definitions shared by the time-stepper kernels (register-resident and wide block layouts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"

namespace fpn {

// Block geometry of the |m| ordering: block 0 holds l = 0..L (cos type, padded to even size),
// block k >= 1 holds the (cos, sin) pairs of l = k..L.
template <int L>
struct Geo {
  static constexpr int N = (L + 1) * (L + 1);
  static constexpr int n0 = (L + 1) + ((L + 1) & 1);
  static constexpr int Np = N + (n0 - (L + 1));
  static constexpr int nb(int k) { return k == 0 ? n0 : 2 * (L + 1 - k); }
  static constexpr int off(int k) {
    int o = 0;
    for (int j = 0; j < k; ++j) o += nb(j);
    return o;
  }
  static constexpr int qmax = (n0 / 2 > L) ? n0 / 2 : L;  // largest block row length per half-wave
  static constexpr int S = (Np + 63) / 64;    // vector slots per lane
  static constexpr int NpA = (Np + 3) & ~3;   // padded vector length in LDS
};

// A zero the optimiser cannot see through: table indices offset by it are not hoisted out of
// the time loop (the tables are loop-invariant, and hoisting keeps one register per entry live).
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// A (wavefront-uniform) pointer the optimiser cannot see through: addresses derived from it are
// formed after this point, so the per-block table addresses are not all hoisted out of the time loop.
// (The offset is an opaque zero: the asm operand is a fresh scalar, whatever register class the
// pointer itself ends up in.)
template <typename T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
  return p + opaque_zero();
}

// |v| for the step-error maximum, with NaN mapped to +inf: fmaxf ignores a NaN operand, an infinity
// survives the maximum and marks the attempt as non-finite.
__device__ __forceinline__ float err_abs(float v) {
  const float a = fabsf(v);
  return a == a ? a : __builtin_inff();
}

// Zeroes a wavefront's LDS scratch up to its step-controller scalars `ctl` (the struct's last
// member), before each instance and after a non-finite attempt: window reads past a block edge
// carry weight 0 and need finite data there.
template <typename WL>
__device__ __forceinline__ void clear_wave_scratch(WL& w, int lane) {
  float* f = reinterpret_cast<float*>(&w);
  const int nf = int((reinterpret_cast<const char*>(w.ctl) - reinterpret_cast<const char*>(&w)) / 4);
  for (int e = lane; e < nf; e += 64) f[e] = 0.0f;
}

// Sum of a value over the two 32-lane halves (lane and lane ^ 32).
__device__ __forceinline__ float half_sum(float v) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Largest absolute value over the wavefront, returned as a wavefront-uniform (scalar) value so that
// control flow that depends on it stays uniform.
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  v = fmaxf(v, __shfl_xor(v, 8));
  v = fmaxf(v, __shfl_xor(v, 4));
  v = fmaxf(v, __shfl_xor(v, 2));
  v = fmaxf(v, __shfl_xor(v, 1));
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  const float m = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m)));
}

// Partial pivoting of the Schur-block Gauss-Jordan: the pivot of a column is the remaining row with
// the largest |entry|.  The comparison key of a row is its |entry| with the low `B` mantissa bits
// replaced by the row index (a candidate key is at least 2^B, a finished row's key is 0), so one
// unsigned maximum over the lanes yields the pivot row.  NaN compares above every finite value and
// is then caught as a non-finite pivot.
template <int B>
__device__ __forceinline__ uint32_t pivot_key(float v, int row, bool candidate) {
  const uint32_t mag = __float_as_uint(v) & 0x7fffffffu;
  return candidate ? ((((mag >> B) + 1u) << B) | uint32_t(row)) : 0u;
}

// Maximum of a key over each 16-lane row of the wavefront (every lane of the row receives it):
// DPP butterflies within quads, then the half-row and row mirrors.
__device__ __forceinline__ uint32_t row16_max(uint32_t k) {
  k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0xB1, 0xF, 0xF, false)));   // quad: 1 0 3 2
  k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x4E, 0xF, 0xF, false)));   // quad: 2 3 0 1
  k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x141, 0xF, 0xF, false)));  // row half mirror
  k = max(k, uint32_t(__builtin_amdgcn_update_dpp(0, int(k), 0x140, 0xF, 0xF, false)));  // row mirror
  return k;
}

// Wavefront-uniform maximum of a key over lanes 0..31 (rows 0 and 1) or over all 64 lanes.
__device__ __forceinline__ uint32_t max32_uniform(uint32_t k) {
  k = row16_max(k);
  return max(uint32_t(__builtin_amdgcn_readlane(int(k), 0)), uint32_t(__builtin_amdgcn_readlane(int(k), 16)));
}
__device__ __forceinline__ uint32_t max64_uniform(uint32_t k) {
  k = row16_max(k);
  const uint32_t a = max(uint32_t(__builtin_amdgcn_readlane(int(k), 0)), uint32_t(__builtin_amdgcn_readlane(int(k), 16)));
  const uint32_t b = max(uint32_t(__builtin_amdgcn_readlane(int(k), 32)), uint32_t(__builtin_amdgcn_readlane(int(k), 48)));
  return max(a, b);
}

// RODAS4 (Hairer & Wanner) in the form
//   (I/(h g) - J) K_i = f(t + al_i h, y + sum_j a_ij K_j) + sum_j (c_ij/h) K_j + h gm_i f_t,
//   y_{n+1} = y + sum_j a_6j K_j + K_6,  g = 1/4; K_6 is the embedded error estimate.
static __constant__ float kRodasAlpha[6] = {0.0f, 0.386f, 0.21f, 0.63f, 1.0f, 1.0f};
static __constant__ float kRodasGamma[6] = {0.25f, -0.1043f, 0.1035f, -0.03620000000000023f, 0.0f, 0.0f};
static __constant__ float kRodasA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.544f, 0, 0, 0, 0},
    {0.9466785280815826f, 0.2557011698983284f, 0, 0, 0},
    {3.314825187068521f, 2.896124015972201f, 0.9986419139977817f, 0, 0},
    {1.221224509226641f, 6.019134481288629f, 12.53708332932087f, -0.6878860361058950f, 0},
    {1.221224509226641f, 6.019134481288629f, 12.53708332932087f, -0.6878860361058950f, 1.0f}};
static __constant__ float kRodasC[6][5] = {
    {0, 0, 0, 0, 0},
    {-5.668800000000000f, 0, 0, 0, 0},
    {-2.430093356833875f, -0.2063599157091915f, 0, 0, 0},
    {-0.1073529058151375f, -9.594562251023355f, -20.47028614809616f, 0, 0},
    {7.496443313967647f, -10.24680431464352f, -33.99990352819905f, 11.70890893206160f, 0},
    {8.083246795921522f, -7.981132988064893f, -31.52159432874371f, 16.31930543123136f, -6.058818238834054f}};

// Adaptive settling: largest step, in sample spacings, while no sample is recorded (the error
// control sizes the steps; this only bounds them).
constexpr double kSettleSpan = 8.0;

struct StepArgs {
  const InstParams* ip;
  const int32_t* inst_idx;
  int n_inst;
  const double* c0;
  int64_t c_stride;
  double amp[3], freq[3], phase[3];  // drive
  double period;
  int settle;
  int Ns;
  int r_fixed;   // > 0: fixed substeps per sample interval; 0: adaptive
  int r_max;     // adaptive: smallest step = sample spacing / r_max
  float tol;     // adaptive: bound on max |K6| (embedded RODAS4 error) per step
  float* msamp;  // [n_total][3][Ns]
  float* dmdt;   // [n_total][3][Ns] dm/dt at the samples (right-hand side of the ODE), may be null
  int32_t* status;
  int32_t* steps_out;  // [n_total] time steps taken (may be null)
  int32_t* queue;      // work counter of this launch, zero at launch
  const double* c0t;   // tangents: initial states [n_total][kNTan][c_stride] (FP64)
  float* mtan;         // tangents: samples [n_total][kNTan][3][Ns]; null without tangents
  float* tws;          // register layout with tangents: workspace per resident wavefront (8 NT NpA floats)
};

}  // namespace fpn
