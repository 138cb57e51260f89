// Surrogate evaluation kernels: instance features, ensemble combination with an error
// estimate, compaction of the instances handed to the solver, gather and scatter.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "physics.hpp"
#include "surrogate.hpp"

namespace fpn {
namespace sur {

// x[i] = (log D, sigma, alpha, n_x, n_y, n_z, offset_x / 12 mT, offset_y / 12 mT), sigma = K V / (k_B T)
// with V = pi D^3 / 6: the anisotropy barrier in units of k_B T, the exponent of the Neel relaxation
// time, which the response of stiff particles follows (K is log D, sigma and T away).
// n and -n describe the same particle (the anisotropy energy is even in n), so the axis is
// mapped to the half-space n_z > 0 (ties broken by n_y, then n_x).  Instances with
// non-physical parameters get status 1 and NaN features.
__global__ void features_kernel(int64_t n, const double* D, const double* Ms, const double* K,
                                const double* alpha, const double* T, const double* nax, const double* off,
                                float* x, int32_t* status) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a0 = nax[3 * i], a1 = nax[3 * i + 1], a2 = nax[3 * i + 2];
  const double nn = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
  const bool ok = D[i] > 0.0 && Ms[i] > 0.0 && K[i] > 0.0 && alpha[i] > 0.0 && T[i] > 0.0 && isfinite(D[i]) &&
                  isfinite(K[i]) && isfinite(alpha[i]) && fabs(nn - 1.0) <= 1e-6 &&
                  (off == nullptr || (isfinite(off[3 * i]) && isfinite(off[3 * i + 1])));
  status[i] = ok ? 0 : 1;
  float* xi = x + 8 * i;
  if (!ok) {
    for (int j = 0; j < 8; ++j) xi[j] = __builtin_nanf("");
    return;
  }
  const bool flip = (a2 < 0.0) || (a2 == 0.0 && (a1 < 0.0 || (a1 == 0.0 && a0 < 0.0)));
  if (flip) {
    a0 = -a0;
    a1 = -a1;
    a2 = -a2;
  }
  xi[0] = float(log(D[i]));
  xi[1] = float(K[i] * (kPi / 6.0) * D[i] * D[i] * D[i] / (kBoltzmann * T[i]));
  xi[2] = float(alpha[i]);
  xi[3] = float(a0);
  xi[4] = float(a1);
  xi[5] = float(a2);
  xi[6] = off ? float(off[3 * i] / 12e-3) : 0.0f;
  xi[7] = off ? float(off[3 * i + 1] / 12e-3) : 0.0f;
}

// One wavefront per instance.  y = (ya + yb) / 2 / out_scale is written as harmonics 1..Kh of x and
// y (network layout [ch][k][re, im], 4 Kh values); bin 0 is zero (Phi_0 of a periodic signal).
// err = calib * ||ya - yb|| / ||ya + yb|| * 2; instances with err > tol (or non-finite) are appended
// to `list` (order of arrival; the caller treats the list as a set).
__global__ void combine_kernel(int64_t n, int Kh, const float* ya, const float* yb, float inv_scale, float calib,
                               float tol, const int32_t* status, float* harm, float* err, int32_t* used,
                               int32_t* list, int32_t* count) {
  const int64_t i = int64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int W = 4 * Kh;
  const float* a = ya + i * W;
  const float* b = yb + i * W;
  float* h = harm + i * 2 * (Kh + 1) * 2;
  const bool bad = status[i] != 0;
  float dd = 0.0f, ss = 0.0f;
  for (int j = lane; j < W; j += 64) {
    const float u = a[j], v = b[j];
    dd += (u - v) * (u - v);
    ss += (u + v) * (u + v);
    const int c = j / (2 * Kh), k = (j / 2) % Kh, ri = j & 1;
    h[(c * (Kh + 1) + k + 1) * 2 + ri] = bad ? __builtin_nanf("") : 0.5f * (u + v) * inv_scale;
  }
  if (lane < 4) h[((lane >> 1) * (Kh + 1)) * 2 + (lane & 1)] = bad ? __builtin_nanf("") : 0.0f;
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_xor(dd, o);
    ss += __shfl_xor(ss, o);
  }
  if (lane == 0) {
    const float e = calib * 2.0f * sqrtf(dd) / sqrtf(ss);
    const bool fall = !bad && !(e <= tol);
    err[i] = bad ? __builtin_nanf("") : e;
    used[i] = fall ? 1 : 0;
    if (fall) list[atomicAdd(count, 1)] = int32_t(i);
  }
}

// One wavefront per row: the ensemble mean y = (ya + yb) / 2 * inv_scale (network layout kept) and
// err = calib * 2 ||ya - yb|| / ||ya + yb||, the same estimate as combine_kernel.
__global__ void mean_spread_kernel(int64_t n, int W, const float* ya, const float* yb, float inv_scale,
                                   float calib, float* y, float* err) {
  const int64_t i = int64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const float* a = ya + i * W;
  const float* b = yb + i * W;
  float dd = 0.0f, ss = 0.0f;
  for (int j = lane; j < W; j += 64) {
    const float u = a[j], v = b[j];
    dd += (u - v) * (u - v);
    ss += (u + v) * (u + v);
    if (y) y[i * W + j] = 0.5f * (u + v) * inv_scale;
  }
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_xor(dd, o);
    ss += __shfl_xor(ss, o);
  }
  if (lane == 0 && err) err[i] = calib * 2.0f * sqrtf(dd) / sqrtf(ss);
}

__global__ void axpy_kernel(int64_t n, float a, const float* x, float* y) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) y[j] = fmaf(a, x[j], y[j]);
}

__global__ void scale_kernel(int64_t n, const float* src, float a, float* dst) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = src[j] * a;
}

__global__ void gather_kernel(int cnt, const int32_t* list, const double* D, const double* Ms, const double* K,
                              const double* alpha, const double* T, const double* nax, const double* off,
                              double* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cnt) return;
  const int64_t i = list[j];
  // out: D, Ms, K, alpha, T [cnt] each, then easy axis [cnt][3], offset [cnt][3]
  out[j] = D[i];
  out[cnt + j] = Ms[i];
  out[2 * cnt + j] = K[i];
  out[3 * cnt + j] = alpha[i];
  out[4 * cnt + j] = T[i];
  for (int c = 0; c < 3; ++c) {
    out[5 * cnt + 3 * j + c] = nax[3 * i + c];
    out[8 * cnt + 3 * j + c] = off ? off[3 * i + c] : 0.0;
  }
}

__global__ void scatter_kernel(int cnt, int per, const int32_t* list, const float* src, const int32_t* st_src,
                               float* harm, int32_t* status, float* err) {
  const int j = blockIdx.x;
  if (j >= cnt) return;
  const int64_t i = list[j];
  for (int e = threadIdx.x; e < per; e += blockDim.x) harm[i * per + e] = src[int64_t(j) * per + e];
  if (threadIdx.x == 0) {
    status[i] = st_src[j];
    err[i] = 0.0f;
  }
}

__global__ void zero_i32_kernel(int32_t* p, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = 0;
}

hipError_t features(int64_t n, const double* D, const double* Ms, const double* K, const double* alpha,
                    const double* T, const double* nax, const double* off, float* x, int32_t* status,
                    hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, D, Ms, K, alpha, T, nax,
                     off, x, status);
  return hipGetLastError();
}

hipError_t combine(int64_t n, int Kh, const float* ya, const float* yb, float inv_scale, float calib, float tol,
                   const int32_t* status, float* harm, float* err, int32_t* used, int32_t* list, int32_t* count,
                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, s, count, 1);
  hipLaunchKernelGGL(combine_kernel, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, n, Kh, ya, yb, inv_scale, calib,
                     tol, status, harm, err, used, list, count);
  return hipGetLastError();
}

hipError_t mean_spread(int64_t n, int W, const float* ya, const float* yb, float inv_scale, float calib, float* y,
                       float* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(mean_spread_kernel, dim3(unsigned((n + 3) / 4)), dim3(256), 0, s, n, W, ya, yb, inv_scale,
                     calib, y, err);
  return hipGetLastError();
}

hipError_t axpy(int64_t n, float a, const float* x, float* y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t scale(int64_t n, const float* src, float a, float* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, src, a, dst);
  return hipGetLastError();
}

hipError_t gather(int cnt, const int32_t* list, const double* D, const double* Ms, const double* K,
                  const double* alpha, const double* T, const double* nax, const double* off, double* out,
                  hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, s, cnt, list, D, Ms, K, alpha,
                     T, nax, off, out);
  return hipGetLastError();
}

hipError_t scatter(int cnt, int per, const int32_t* list, const float* src, const int32_t* st_src, float* harm,
                   int32_t* status, float* err, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(unsigned(cnt)), dim3(128), 0, s, cnt, per, list, src, st_src, harm, status,
                     err);
  return hipGetLastError();
}

}  // namespace sur
}  // namespace fpn
