// Data-driven model fits and the distance measure (paper: Methods, "Data-driven physically
// motivated models" M0/M1 with the closed-form scale of "Technical details regarding the parameter
// identification", and "Distance Measure": Eq. mix, Eq. error1, Eq. globalMeasure), on system
// matrices laid out as the solver writes its harmonics.
//
// A system matrix of one dictionary element (or one measurement) is [n_pos][n_ch][n_bins][2] FP32:
// positions (offset fields) outermost, then receive channel, frequency bin, (re, im).  A batch of
// them is contiguous, which is exactly fpn_solve's harm_out when the instances are ordered
// element-major, position-minor.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <string>

#include "../../include/fpn.h"
#include "capi_internal.hpp"

using namespace fpn_internal;

namespace {

// One workgroup per (dictionary element, measurement) pair, one thread per (channel, bin) row:
//   a_k   = sum_nu S_k(nu) conj(Phi_k(nu)) / sum_nu |Phi_k(nu)|^2        (FP64 sums)
//   eps_k = sqrt(sum_nu |S_k(nu) - a_k Phi_k(nu)|^2 / N) / max_nu |S_k(nu)|
// Two passes over the row (the residual is summed directly, not from the normal equations, so an
// almost exact fit keeps its small error).  Consecutive threads read consecutive bins (8 bytes
// each) of one position: coalesced.
__global__ void fit_rows_kernel(const float2* __restrict__ phi, const float2* __restrict__ S, int n_pos, int rows,
                                const int32_t* __restrict__ pair_phi, const int32_t* __restrict__ pair_s,
                                float2* __restrict__ a_out, float* __restrict__ err_out) {
  const int64_t p = blockIdx.x;
  const int64_t stride = rows;  // float2 per position
  const float2* F = phi + int64_t(pair_phi[p]) * n_pos * stride;
  const float2* M = S + int64_t(pair_s[p]) * n_pos * stride;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    double nr = 0.0, ni = 0.0, den = 0.0, smax = 0.0;
    for (int v = 0; v < n_pos; ++v) {
      const float2 f = F[v * stride + r];
      const float2 s = M[v * stride + r];
      // s * conj(f)
      nr += double(s.x) * f.x + double(s.y) * f.y;
      ni += double(s.y) * f.x - double(s.x) * f.y;
      den += double(f.x) * f.x + double(f.y) * f.y;
      smax = fmax(smax, sqrt(double(s.x) * s.x + double(s.y) * s.y));
    }
    const double ar = den > 0.0 ? nr / den : 0.0;
    const double ai = den > 0.0 ? ni / den : 0.0;
    double res = 0.0;
    for (int v = 0; v < n_pos; ++v) {
      const float2 f = F[v * stride + r];
      const float2 s = M[v * stride + r];
      const double dr = s.x - (ar * f.x - ai * f.y);
      const double di = s.y - (ar * f.y + ai * f.x);
      res += dr * dr + di * di;
    }
    if (a_out) a_out[p * rows + r] = make_float2(float(ar), float(ai));
    if (err_out) err_out[p * rows + r] = float(sqrt(res / n_pos) / smax);
  }
}

// One workgroup per parameter group: rows of err [n_ang][n_ch][n_bins] for the group, reduced over
// angles and channels for every bin of kset (eps_freq) and then over kset (eps_global), FP64.
__global__ void nrmse_global_kernel(const float* __restrict__ err, int n_ang, int n_ch, int n_bins,
                                    const int32_t* __restrict__ kset, int n_k, float* __restrict__ eps_freq,
                                    float* __restrict__ eps_global) {
  const int64_t g = blockIdx.x;
  const float* E = err + g * int64_t(n_ang) * n_ch * n_bins;
  __shared__ double part[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_k; j += blockDim.x) {
    const int k = kset[j];
    double s = 0.0;
    for (int a = 0; a < n_ang; ++a)
      for (int c = 0; c < n_ch; ++c) {
        const double e = E[(int64_t(a) * n_ch + c) * n_bins + k];
        s += e * e;
      }
    const double f2 = s / (double(n_ang) * n_ch);
    if (eps_freq) eps_freq[g * n_k + j] = float(sqrt(f2));
    acc += f2;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && eps_global) eps_global[g] = float(sqrt(part[0] / n_k));
}

// Model M2 dictionary matrix, transposed: Mt[j][r] = w_r a_{j,theta}(c, k) Phi_{j,theta}(nu, c, k) and
// y[r] = w_r S_theta(nu, c, k), rows r = ((theta n_ch + c) n_k + kk) n_pos + nu for the bins kset[kk],
// with the row weight w_r = 1 / max_nu |S_theta(nu, c, k)| (the paper's per-frequency infinity-norm
// weighting, applied per receive channel).  Dictionary element of pair j at angle theta: j n_ang + theta.
// One workgroup per (j, theta, c, kk) row block of n_pos rows; j = J is the data column y.
__global__ void m2_build_kernel(const float2* __restrict__ phi, const float2* __restrict__ a,
                                const float2* __restrict__ S, int n_pos, int n_ch, int n_bins, int J, int n_ang,
                                const int32_t* __restrict__ kset, int n_k, float2* __restrict__ Mt,
                                float2* __restrict__ y) {
  const int blk = blockIdx.x;  // ((j * n_ang + th) * n_ch + c) * n_k + kk, j in [0, J]
  const int kk = blk % n_k;
  const int c = (blk / n_k) % n_ch;
  const int th = (blk / (n_k * n_ch)) % n_ang;
  const int j = blk / (n_k * n_ch * n_ang);
  const int k = kset[kk];
  const int64_t rows = int64_t(n_ang) * n_ch * n_k * n_pos;
  const int64_t r0 = ((int64_t(th) * n_ch + c) * n_k + kk) * n_pos;
  const int64_t rs = int64_t(n_ch) * n_bins;  // float2 between positions
  const float2* Sm = S + int64_t(th) * n_pos * rs + c * n_bins + k;
  // row weight: largest |S| over the positions (every thread computes it; n_pos is small)
  float smax = 0.0f;
  for (int v = 0; v < n_pos; ++v) {
    const float2 q = Sm[v * rs];
    smax = fmaxf(smax, sqrtf(q.x * q.x + q.y * q.y));
  }
  const float wr = 1.0f / smax;
  if (j == J) {
    for (int v = threadIdx.x; v < n_pos; v += blockDim.x) {
      const float2 q = Sm[v * rs];
      y[r0 + v] = make_float2(wr * q.x, wr * q.y);
    }
    return;
  }
  const int64_t el = int64_t(j) * n_ang + th;
  const float2 av = a[(el * n_ch + c) * n_bins + k];
  const float2* F = phi + el * n_pos * rs + c * n_bins + k;
  float2* out = Mt + int64_t(j) * rows + r0;
  for (int v = threadIdx.x; v < n_pos; v += blockDim.x) {
    const float2 f = F[v * rs];
    out[v] = make_float2(wr * (av.x * f.x - av.y * f.y), wr * (av.x * f.y + av.y * f.x));
  }
}

// G = conj(Mt) Mt^T (J x J, Hermitian) and b = conj(Mt) y, FP64 sums.  Column J of the extended
// matrix [Mt; y] gives b (pairs (j, J)) and ||y||^2 (pair (J, J)).  32 x 32 output tile per
// workgroup (256 threads, 4 outputs each), rows staged through LDS 64 at a time.
constexpr int kGT = 32, kGR = 64;
__global__ void m2_gram_kernel(const float2* __restrict__ Mt, const float2* __restrict__ y, int J, int64_t rows,
                               double2* __restrict__ G, double2* __restrict__ b, double* __restrict__ yy) {
  const int tj = blockIdx.y * kGT, tk = blockIdx.x * kGT;
  if (tk + kGT <= tj) return;  // lower tiles: Hermitian mirror of an upper one
  __shared__ float2 A[kGT][kGR + 1], B[kGT][kGR + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty in 0..7: rows ty, ty + 8, ...
  double acc_r[4] = {0, 0, 0, 0}, acc_i[4] = {0, 0, 0, 0};
  auto col = [&](int j) -> const float2* { return j < J ? Mt + int64_t(j) * rows : (j == J ? y : nullptr); };
  for (int64_t r0 = 0; r0 < rows; r0 += kGR) {
    for (int e = threadIdx.x; e < kGT * kGR; e += blockDim.x) {
      const int jj = e / kGR, rr = e % kGR;
      const int64_t r = r0 + rr;
      const float2* pa = col(tj + jj);
      const float2* pb = col(tk + jj);
      A[jj][rr] = (pa && r < rows) ? pa[r] : make_float2(0.0f, 0.0f);
      B[jj][rr] = (pb && r < rows) ? pb[r] : make_float2(0.0f, 0.0f);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kGR; ++rr) {
      const float2 q = B[tx][rr];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float2 p = A[ty + 8 * u][rr];
        // conj(p) * q
        acc_r[u] += double(p.x) * q.x + double(p.y) * q.y;
        acc_i[u] += double(p.x) * q.y - double(p.y) * q.x;
      }
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u) {
    const int j = tj + ty + 8 * u, k = tk + tx;
    if (j > J || k > J || k < j) continue;
    if (k < J) {
      G[int64_t(j) * J + k] = make_double2(acc_r[u], acc_i[u]);
      G[int64_t(k) * J + j] = make_double2(acc_r[u], -acc_i[u]);
    } else if (j < J) {
      b[j] = make_double2(acc_r[u], acc_i[u]);
    } else {
      *yy = acc_r[u];
    }
  }
}

// S_model[theta](nu, c, k) = sum_j w_j a_{j,theta}(c, k) Phi_{j,theta}(nu, c, k): one thread per
// (theta, nu, c, k) output.
__global__ void m2_model_kernel(const float2* __restrict__ phi, const float2* __restrict__ a,
                                const double* __restrict__ w, int n_pos, int n_ch, int n_bins, int J, int n_ang,
                                float2* __restrict__ model) {
  const int64_t per = int64_t(n_pos) * n_ch * n_bins;
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= per * n_ang) return;
  const int th = int(e / per);
  const int64_t rem = e - int64_t(th) * per;  // (nu, c, k)
  const int64_t ck = rem % (int64_t(n_ch) * n_bins);
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < J; ++j) {
    const int64_t el = int64_t(j) * n_ang + th;
    const float2 f = phi[el * per + rem];
    const float2 av = a[el * n_ch * n_bins + ck];
    const double wj = w[j];
    sr += wj * (double(av.x) * f.x - double(av.y) * f.y);
    si += wj * (double(av.x) * f.y + double(av.y) * f.x);
  }
  model[e] = make_float2(float(sr), float(si));
}

// Eq. error1 of model rows against measured rows, matrix by matrix (same layout, no fit).
__global__ void rows_error_kernel(const float2* __restrict__ model, const float2* __restrict__ S, int n_pos,
                                  int rows, float* __restrict__ err) {
  const int64_t p = blockIdx.x;
  const float2* F = model + p * n_pos * rows;
  const float2* M = S + p * n_pos * rows;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    double res = 0.0, smax = 0.0;
    for (int v = 0; v < n_pos; ++v) {
      const float2 f = F[int64_t(v) * rows + r];
      const float2 s = M[int64_t(v) * rows + r];
      const double dr = double(s.x) - f.x, di = double(s.y) - f.y;
      res += dr * dr + di * di;
      smax = fmax(smax, sqrt(double(s.x) * s.x + double(s.y) * s.y));
    }
    err[p * rows + r] = float(sqrt(res / n_pos) / smax);
  }
}

}  // namespace

extern "C" {

fpn_status fpn_fit_rows(fpn_ctx ctx, const float* phi, const float* S, int32_t n_pos, int32_t n_ch, int32_t n_bins,
                        int64_t n_pairs, const int32_t* pair_phi, const int32_t* pair_s, float* a_out,
                        float* err_out, void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n_pairs < 0 || n_pairs > (int64_t(1) << 31) - 1) return fail(FPN_E_ARG, "n_pairs outside [0, 2^31)");
  if (n_pos < 1 || n_ch < 1 || n_bins < 1 || int64_t(n_ch) * n_bins > (int64_t(1) << 20))
    return fail(FPN_E_ARG, "n_pos, n_ch, n_bins must be >= 1 and n_ch * n_bins <= 2^20");
  if (n_pairs == 0) return FPN_OK;
  if (!phi || !S || !pair_phi || !pair_s) return fail(FPN_E_ARG, "NULL input");
  if (!a_out && !err_out) return fail(FPN_E_ARG, "a_out and err_out are both NULL");
  FPN_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(fit_rows_kernel, dim3(unsigned(n_pairs)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const float2*>(phi), reinterpret_cast<const float2*>(S), int(n_pos),
                     int(n_ch * n_bins), pair_phi, pair_s, reinterpret_cast<float2*>(a_out), err_out);
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

fpn_status fpn_nrmse_global(fpn_ctx ctx, const float* err_rows, int64_t n_groups, int32_t n_ang, int32_t n_ch,
                            int32_t n_bins, const int32_t* kset, int32_t n_k, float* eps_freq, float* eps_global,
                            void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n_groups < 0 || n_groups > (int64_t(1) << 31) - 1) return fail(FPN_E_ARG, "n_groups outside [0, 2^31)");
  if (n_ang < 1 || n_ch < 1 || n_bins < 1 || n_k < 1) return fail(FPN_E_ARG, "n_ang, n_ch, n_bins, n_k must be >= 1");
  if (n_groups == 0) return FPN_OK;
  if (!err_rows || !kset) return fail(FPN_E_ARG, "NULL input");
  if (!eps_freq && !eps_global) return fail(FPN_E_ARG, "eps_freq and eps_global are both NULL");
  FPN_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(nrmse_global_kernel, dim3(unsigned(n_groups)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), err_rows, int(n_ang), int(n_ch), int(n_bins), kset,
                     int(n_k), eps_freq, eps_global);
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

// k = mx n + my (n + 1): with (mx, my) = (-k, k) + t (n + 1, -n) for integer t, the order sum
// f(t) = |(n + 1) t - k| + |k - n t| is convex in t with its real minimum between k / (n + 1) and k / n,
// so the integer minimiser is among the integers of that interval and its two neighbours.
fpn_status fpn_mixing_order(int32_t k, int32_t n_dens, int32_t* mx, int32_t* my) {
  if (!mx || !my) return fail(FPN_E_ARG, "NULL output");
  if (n_dens < 1 || n_dens > 4096 || std::llabs(int64_t(k)) > (int64_t(1) << 24))
    return fail(FPN_E_ARG, "n_dens outside [1, 4096] or |k| > 2^24");
  const int64_t n = n_dens, kk = k;
  auto fl = [](int64_t a, int64_t b) { return a / b - ((a % b != 0) && ((a < 0) != (b < 0))); };
  const int64_t lo = std::min(fl(kk, n + 1), fl(kk, n)) - 1;
  const int64_t hi = std::max(fl(kk, n + 1), fl(kk, n)) + 2;
  int64_t best = -1, bt = 0;
  int ties = 0;
  for (int64_t t = lo; t <= hi; ++t) {
    const int64_t ax = -kk + (n + 1) * t, ay = kk - n * t;
    const int64_t f = std::llabs(ax) + std::llabs(ay);
    if (best < 0 || f < best) {
      best = f;
      bt = t;
      ties = 0;
    } else if (f == best) {
      ++ties;
    }
  }
  if (ties) return fail(FPN_E_ARG, "mixing order is not unique for this k and n_dens");
  *mx = int32_t(-kk + (n + 1) * bt);
  *my = int32_t(kk - n * bt);
  return FPN_OK;
}

fpn_status fpn_frequency_index_set(int32_t Mx, int32_t My, int32_t n_dens, int32_t* k_out, int32_t* count) {
  if (!count) return fail(FPN_E_ARG, "NULL count");
  if (Mx < 0 || My < 0 || Mx > 1024 || My > 1024 || n_dens < 1 || n_dens > 4096)
    return fail(FPN_E_ARG, "Mx, My outside [0, 1024] or n_dens outside [1, 4096]");
  int32_t c = 0;
  for (int32_t a = 0; a <= Mx; ++a)
    for (int32_t b = 0; b <= My; ++b) {
      if ((a == 0 && b == 0) || (a == 0 && b == 1) || (a == 1 && b == 0)) continue;
      if (k_out) k_out[c] = a * n_dens + b * (n_dens + 1);
      ++c;
    }
  *count = c;
  return FPN_OK;
}

fpn_status fpn_m2_system(fpn_ctx ctx, const float* phi, const float* a, const float* S, int32_t n_pos, int32_t n_ch,
                         int32_t n_bins, int32_t J, int32_t n_ang, const int32_t* kset, int32_t n_k, double* G_out,
                         double* b_out, double* yy_out, void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n_pos < 1 || n_ch < 1 || n_bins < 1 || J < 1 || n_ang < 1 || n_k < 1)
    return fail(FPN_E_ARG, "n_pos, n_ch, n_bins, J, n_ang, n_k must be >= 1");
  if (J > 8192) return fail(FPN_E_RANGE, "J > 8192");
  if (!phi || !a || !S || !kset || !G_out || !b_out || !yy_out) return fail(FPN_E_ARG, "NULL argument");
  const int64_t rows = int64_t(n_ang) * n_ch * n_k * n_pos;
  const int64_t blocks = int64_t(J + 1) * n_ang * n_ch * n_k;
  if (blocks > (int64_t(1) << 31) - 1 || rows * int64_t(J) > (int64_t(1) << 34))
    return fail(FPN_E_RANGE, "dictionary matrix larger than 2^34 entries");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(ctx->device));
  FPN_HIP(ctx->m2_mt.ensure(size_t(rows) * J * 2));
  FPN_HIP(ctx->m2_y.ensure(size_t(rows) * 2));
  float2* Mt = reinterpret_cast<float2*>(ctx->m2_mt.p);
  float2* y = reinterpret_cast<float2*>(ctx->m2_y.p);
  hipLaunchKernelGGL(m2_build_kernel, dim3(unsigned(blocks)), dim3(128), 0, s, reinterpret_cast<const float2*>(phi),
                     reinterpret_cast<const float2*>(a), reinterpret_cast<const float2*>(S), int(n_pos), int(n_ch),
                     int(n_bins), int(J), int(n_ang), kset, int(n_k), Mt, y);
  FPN_HIP(hipGetLastError());
  const unsigned t = unsigned((J + 1 + kGT - 1) / kGT);
  hipLaunchKernelGGL(m2_gram_kernel, dim3(t, t), dim3(256), 0, s, Mt, y, int(J), rows,
                     reinterpret_cast<double2*>(G_out), reinterpret_cast<double2*>(b_out), yy_out);
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

fpn_status fpn_m2_model(fpn_ctx ctx, const float* phi, const float* a, const double* w, int32_t n_pos, int32_t n_ch,
                        int32_t n_bins, int32_t J, int32_t n_ang, float* model_out, void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n_pos < 1 || n_ch < 1 || n_bins < 1 || J < 1 || n_ang < 1)
    return fail(FPN_E_ARG, "n_pos, n_ch, n_bins, J, n_ang must be >= 1");
  if (!phi || !a || !w || !model_out) return fail(FPN_E_ARG, "NULL argument");
  const int64_t total = int64_t(n_ang) * n_pos * n_ch * n_bins;
  if ((total + 255) / 256 > (int64_t(1) << 31) - 1) return fail(FPN_E_RANGE, "model too large");
  FPN_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(m2_model_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const float2*>(phi),
                     reinterpret_cast<const float2*>(a), w, int(n_pos), int(n_ch), int(n_bins), int(J), int(n_ang),
                     reinterpret_cast<float2*>(model_out));
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

fpn_status fpn_rows_error(fpn_ctx ctx, const float* model, const float* S, int32_t n_pos, int32_t n_ch, int32_t n_bins,
                          int64_t n_mat, float* err_out, void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n_mat < 0 || n_mat > (int64_t(1) << 31) - 1) return fail(FPN_E_ARG, "n_mat outside [0, 2^31)");
  if (n_pos < 1 || n_ch < 1 || n_bins < 1) return fail(FPN_E_ARG, "n_pos, n_ch, n_bins must be >= 1");
  if (n_mat == 0) return FPN_OK;
  if (!model || !S || !err_out) return fail(FPN_E_ARG, "NULL argument");
  FPN_HIP(hipSetDevice(ctx->device));
  hipLaunchKernelGGL(rows_error_kernel, dim3(unsigned(n_mat)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const float2*>(model), reinterpret_cast<const float2*>(S), int(n_pos),
                     int(n_ch * n_bins), err_out);
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

}  // extern "C"
