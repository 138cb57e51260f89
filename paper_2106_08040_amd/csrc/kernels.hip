// HIP kernels of the fpn solver for gfx950 (MI355X).
//
//   instance_prep      a1: particle scalars + easy-axis frame per instance (FP64)
//   stationary_fp64    a3: stationary density of the field at t = 0 (FP64 block solve)
//   (the FP32 time stepper, rows a4/a5, lives in stepper.hip)
//   harmonics_fp64     a6: Phi_k = (2 pi i k / T) DFT_k(m) with FP64 accumulation
//
// Paper basis: Eq. FP-general + Eq. convection (operator), Eq. mean_magmom_FP (moment),
// Eq. MPI_model_fourier / phi-hat of model M1 (harmonics).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "physics.hpp"

namespace fpn {

// ------------------------------------------------------------- a1: instance ---

__global__ void instance_prep_kernel(int64_t n, const double* D, const double* Ms, const double* K,
                                     const double* alpha, const double* temp, const double* easy,
                                     const double* offset, InstParams* ip, int32_t* status) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double d = D[i], ms = Ms[i], k = K[i], a = alpha[i], T = temp[i];
  const double nx = easy[3 * i], ny = easy[3 * i + 1], nz = easy[3 * i + 2];
  const double nn = sqrt(nx * nx + ny * ny + nz * nz);
  bool ok = isfinite(d) && isfinite(ms) && isfinite(k) && isfinite(a) && isfinite(T) && d > 0 && ms > 0 &&
            k >= 0 && a > 0 && T > 0 && fabs(nn - 1.0) <= 1e-6;
  double off[3] = {0, 0, 0};
  if (offset) {
    for (int c = 0; c < 3; ++c) {
      off[c] = offset[3 * i + c];
      ok = ok && isfinite(off[c]);
    }
  }
  InstParams p;
  const ParticleScalars s = particle_scalars(ok ? d : 1e-8, ok ? ms : 1.0, ok ? k : 0.0, ok ? a : 1.0, ok ? T : 300.0);
  p.inv2tau = s.inv2tau;
  p.sigma = s.sigma;
  p.beta_T = s.beta_T;
  p.alpha = s.alpha;
  // frame: R = [u v n] with u = normalize(a x n), a = e_x unless n is close to x
  const double z0 = ok ? nx / nn : 0.0, z1 = ok ? ny / nn : 0.0, z2 = ok ? nz / nn : 1.0;
  double ax = 1.0, ay = 0.0;
  if (fabs(z0) >= 0.9) { ax = 0.0; ay = 1.0; }
  double u0 = ay * z2, u1 = -ax * z2, u2 = ax * z1 - ay * z0;
  const double un = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
  u0 /= un; u1 /= un; u2 /= un;
  const double v0 = z1 * u2 - z2 * u1, v1 = z2 * u0 - z0 * u2, v2 = z0 * u1 - z1 * u0;
  p.R[0] = u0; p.R[1] = v0; p.R[2] = z0;
  p.R[3] = u1; p.R[4] = v1; p.R[5] = z1;
  p.R[6] = u2; p.R[7] = v2; p.R[8] = z2;
  for (int c = 0; c < 3; ++c) p.off[c] = off[c];
  p.D = ok ? d : 1e-8;
  p.sigK = ok ? kPi * d * d * d / 6.0 / (kBoltzmann * T) : 0.0;
  ip[i] = p;
  status[i] = ok ? 0 : 1;
}

// ------------------------------------------------------ a3: stationary FP64 ---
// One workgroup (256 threads) per instance.  Solves A' c = c00 e_0 where A' is the
// Galerkin matrix at the initial field with row 0 replaced by e_0^T (total probability),
// by block elimination over |m| blocks with partially pivoted Gauss-Jordan inverses.
// Block inverses are kept in global workspace `wsinv` (sum bn^2 doubles per instance).

constexpr int kStatThreads = 256;
constexpr int kMaxBlk = 48;  // largest |m| block for L <= 24 is 2L = 48

__global__ void __launch_bounds__(kStatThreads)
stationary_kernel(DevTables t, const int32_t* inst_idx, int n_inst, const InstParams* ip,
                  const double* field_lab, double3 drive0, double* c_out, int64_t c_stride,
                  double* wsinv, int32_t* status) {
  const int w = blockIdx.x;
  if (w >= n_inst) return;
  const int inst = inst_idx[w];
  const int tid = threadIdx.x;
  __shared__ double S[kMaxBlk * kMaxBlk];
  __shared__ double U[kMaxBlk * kMaxBlk];
  __shared__ double mult[9];
  __shared__ int perm[kMaxBlk];
  __shared__ int s_ok;
  extern __shared__ double vec[];  // [2*Np]: g/x and rhs
  const int Np = t.Np;
  double* x = vec;
  if (status[inst] != 0) {
    for (int p = tid; p < Np; p += blockDim.x) c_out[inst * c_stride + p] = __builtin_nan("");
    return;
  }
  const InstParams P = ip[inst];
  if (tid == 0) s_ok = 1;
  if (tid < 9) {
    double B[3];
    if (field_lab) {
      B[0] = field_lab[3 * inst]; B[1] = field_lab[3 * inst + 1]; B[2] = field_lab[3 * inst + 2];
    } else {
      B[0] = drive0.x + P.off[0]; B[1] = drive0.y + P.off[1]; B[2] = drive0.z + P.off[2];
    }
    double h[3];
    for (int c = 0; c < 3; ++c) h[c] = P.R[0 * 3 + c] * B[0] + P.R[1 * 3 + c] * B[1] + P.R[2 * 3 + c] * B[2];
    const double ia = 1.0 / P.alpha, b = P.beta_T, s2 = P.inv2tau;
    const double m9[9] = {s2, s2 * P.sigma, s2 * 2.0 * P.sigma * ia, s2 * b * h[2], s2 * b * h[2] * ia,
                          s2 * b * h[0], s2 * b * h[1], s2 * b * h[0] * ia, s2 * b * h[1] * ia};
    mult[tid] = m9[tid];
  }
  for (int p = tid; p < Np; p += blockDim.x) x[p] = 0.0;
  __syncthreads();
  const double c00 = 0.28209479177387814;  // 1/sqrt(4 pi): total probability one
  const int pad = (t.n0 != t.L + 1) ? t.n0 - 1 : -1;
  int64_t invoff = 0;
  double* ws = wsinv + int64_t(w) * t.inv_doubles;
  // ---- forward: factor and eliminate
  for (int k = 0; k <= t.L; ++k) {
    const int off = t.boff[k], n = t.bn[k];
    const int offp = k > 0 ? t.boff[k - 1] : 0, np = k > 0 ? t.bn[k - 1] : 0;
    const double* Sp = ws + invoff - int64_t(np) * np;
    // U = B_k Sinv_{k-1}
    if (k > 0) {
      for (int e = tid; e < n * np; e += blockDim.x) {
        const int i = e / np, c = e % np;
        const int row = off + i;
        double acc = 0.0;
        for (int q = t.seg[4 * row]; q < t.seg[4 * row + 1]; ++q) {
          const uint32_t ck = t.colkind[q];
          acc += mult[ck >> 16] * t.val64[q] * Sp[(int(ck & 0xffff) - offp) * np + c];
        }
        U[i * kMaxBlk + c] = acc;
      }
    }
    for (int e = tid; e < n * n; e += blockDim.x) S[(e / n) * kMaxBlk + (e % n)] = 0.0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const int row = off + i;
      if (row == 0 || row == pad) {
        S[i * kMaxBlk + i] = 1.0;
        continue;
      }
      for (int q = t.seg[4 * row + 1]; q < t.seg[4 * row + 2]; ++q) {
        const uint32_t ck = t.colkind[q];
        S[i * kMaxBlk + (int(ck & 0xffff) - off)] += mult[ck >> 16] * t.val64[q];
      }
    }
    __syncthreads();
    if (k > 0) {  // S -= U C_{k-1}
      for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        const int col = off + c;
        double acc = 0.0;
        for (int q = t.cptr[col]; q < t.cptr[col + 1]; ++q) {
          const uint32_t rk = t.crowkind[q];
          const int r = int(rk & 0xffff);
          if (r == 0) continue;  // row 0 replaced by the normalisation
          acc += U[i * kMaxBlk + (r - offp)] * mult[rk >> 16] * t.cval64[q];
        }
        S[i * kMaxBlk + c] -= acc;
      }
      __syncthreads();
    }
    // Gauss-Jordan with partial (row) pivoting
    for (int p = 0; p < n; ++p) {
      if (tid == 0) {
        int best = p;
        double bv = fabs(S[p * kMaxBlk + p]);
        for (int r = p + 1; r < n; ++r) {
          const double v = fabs(S[r * kMaxBlk + p]);
          if (v > bv) { bv = v; best = r; }
        }
        perm[p] = best;
        if (!(bv > 0.0) || !isfinite(bv)) s_ok = 0;
      }
      __syncthreads();
      const int r = perm[p];
      if (r != p)
        for (int j = tid; j < n; j += blockDim.x) {
          const double tmp = S[p * kMaxBlk + j];
          S[p * kMaxBlk + j] = S[r * kMaxBlk + j];
          S[r * kMaxBlk + j] = tmp;
        }
      __syncthreads();
      const double piv = 1.0 / S[p * kMaxBlk + p];
      // column p multipliers and pivot row, read before update
      for (int e = tid; e < n; e += blockDim.x) {
        U[e] = S[e * kMaxBlk + p];          // column p
        U[kMaxBlk + e] = S[p * kMaxBlk + e];  // row p
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v;
        if (i == p && j == p) v = piv;
        else if (i == p) v = U[kMaxBlk + j] * piv;
        else if (j == p) v = -U[i] * piv;
        else v = S[i * kMaxBlk + j] - U[i] * piv * U[kMaxBlk + j];
        S[i * kMaxBlk + j] = v;
      }
      __syncthreads();
    }
    // undo the row interchanges on the columns of the inverse
    for (int p = n - 1; p >= 0; --p) {
      const int r = perm[p];
      if (r != p)
        for (int i = tid; i < n; i += blockDim.x) {
          const double tmp = S[i * kMaxBlk + p];
          S[i * kMaxBlk + p] = S[i * kMaxBlk + r];
          S[i * kMaxBlk + r] = tmp;
        }
      __syncthreads();
    }
    for (int e = tid; e < n * n; e += blockDim.x) ws[invoff + e] = S[(e / n) * kMaxBlk + (e % n)];
    // g_k = Sinv (b_k - B_k g_{k-1})
    double* tv = U;  // reuse as temp
    for (int i = tid; i < n; i += blockDim.x) {
      const int row = off + i;
      double v = (row == 0) ? c00 : 0.0;
      if (k > 0 && row != 0 && row != pad)
        for (int q = t.seg[4 * row]; q < t.seg[4 * row + 1]; ++q) {
          const uint32_t ck = t.colkind[q];
          v -= mult[ck >> 16] * t.val64[q] * x[int(ck & 0xffff)];
        }
      tv[i] = v;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += S[i * kMaxBlk + j] * tv[j];
      x[off + i] = acc;
    }
    __syncthreads();
    invoff += int64_t(n) * n;
  }
  // ---- backward: x_k = g_k - Sinv_k C_k x_{k+1}
  for (int k = t.L - 1; k >= 0; --k) {
    const int off = t.boff[k], n = t.bn[k];
    invoff -= int64_t(t.bn[k + 1]) * t.bn[k + 1];
    const double* Sk = ws + invoff - int64_t(n) * n;
    double* tv = U;
    for (int i = tid; i < n; i += blockDim.x) {
      const int row = off + i;
      double v = 0.0;
      if (row != 0 && row != pad)
        for (int q = t.seg[4 * row + 2]; q < t.seg[4 * row + 3]; ++q) {
          const uint32_t ck = t.colkind[q];
          v += mult[ck >> 16] * t.val64[q] * x[int(ck & 0xffff)];
        }
      tv[i] = v;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += Sk[i * n + j] * tv[j];
      S[i] = x[off + i] - acc;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) x[off + i] = S[i];
    __syncthreads();
  }
  bool fin = true;
  for (int p = tid; p < Np; p += blockDim.x) {
    c_out[inst * c_stride + p] = x[p];
    fin = fin && isfinite(x[p]);
  }
  if (!fin) atomicAnd(&s_ok, 0);
  __syncthreads();
  if (tid == 0 && !s_ok) status[inst] = 3;
}

// ------------------------------------------ a8: stationary-state tangents ---
// d c0 / d p for the five instance parameters p (D, K, alpha, easy-axis polar and azimuth angle):
// differentiating A'(p) c0(p) = c00 e_0 (row 0 of A' is the fixed normalisation) gives
//   A' c0_p = -(dA/dp) c0  with row 0 (and the padding row) of the right-hand side zero,
// solved with the block inverses the stationary kernel left in `wsinv` (same instance slot).
// dA/dp is the operator with the parameter derivatives of the kind multipliers (tan_mult).
__global__ void __launch_bounds__(kStatThreads)
stationary_tangent_kernel(DevTables t, const int32_t* inst_idx, int n_inst, const InstParams* ip, double3 drive0,
                          const double* c0, int64_t c_stride, const double* wsinv, double* ct, int32_t* status) {
  const int w = blockIdx.x;
  if (w >= n_inst) return;
  const int inst = inst_idx[w];
  const int tid = threadIdx.x;
  const int Np = t.Np;
  extern __shared__ double vec[];  // x [Np], tv [kMaxBlk]
  double* x = vec;
  __shared__ double tv[kMaxBlk];
  __shared__ double dm[kNTan][9];
  __shared__ double mult[9];
  double* out = ct + int64_t(inst) * kNTan * c_stride;
  if (status[inst] != 0) {
    for (int e = tid; e < kNTan * Np; e += blockDim.x) out[(e / Np) * c_stride + e % Np] = __builtin_nan("");
    return;
  }
  const InstParams P = ip[inst];
  if (tid < kNTan * 9 + 9) {
    const double B[3] = {drive0.x + P.off[0], drive0.y + P.off[1], drive0.z + P.off[2]};
    double h[3];
    for (int c = 0; c < 3; ++c) h[c] = P.R[0 * 3 + c] * B[0] + P.R[1 * 3 + c] * B[1] + P.R[2 * 3 + c] * B[2];
    if (tid < kNTan * 9) {
      const int prm = tid / 9;
      double e[3], ep[3];
      tan_axis(prm, P.R, e);
      for (int c = 0; c < 3; ++c) ep[c] = P.R[0 * 3 + c] * e[0] + P.R[1 * 3 + c] * e[1] + P.R[2 * 3 + c] * e[2];
      dm[prm][tid % 9] = tan_mult_t<double>(prm, tid % 9, P.inv2tau, P.sigma, P.alpha, P.beta_T, P.D, P.sigK, h, ep);
    } else {
      const double ia = 1.0 / P.alpha, b = P.beta_T, s2 = P.inv2tau;
      const double m9[9] = {s2, s2 * P.sigma, s2 * 2.0 * P.sigma * ia, s2 * b * h[2], s2 * b * h[2] * ia,
                            s2 * b * h[0], s2 * b * h[1], s2 * b * h[0] * ia, s2 * b * h[1] * ia};
      mult[tid - kNTan * 9] = m9[tid - kNTan * 9];
    }
  }
  __syncthreads();
  const double* cin = c0 + int64_t(inst) * c_stride;
  const int pad = (t.n0 != t.L + 1) ? t.n0 - 1 : -1;
  const double* ws = wsinv + int64_t(w) * t.inv_doubles;
  for (int prm = 0; prm < kNTan; ++prm) {
    // forward: g_k = Sinv_k (b_k - B_k g_{k-1}), b = -(dA/dp) c0 (rows 0 and pad: 0)
    int64_t invoff = 0;
    for (int k = 0; k <= t.L; ++k) {
      const int off = t.boff[k], n = t.bn[k];
      for (int i = tid; i < n; i += blockDim.x) {
        const int row = off + i;
        double v = 0.0;
        if (row != 0 && row != pad) {
          for (int q = t.seg[4 * row]; q < t.seg[4 * row + 3]; ++q) {
            const uint32_t ck = t.colkind[q];
            v -= dm[prm][ck >> 16] * t.val64[q] * cin[int(ck & 0xffff)];
          }
          if (k > 0)
            for (int q = t.seg[4 * row]; q < t.seg[4 * row + 1]; ++q) {
              const uint32_t ck = t.colkind[q];
              const int kind = ck >> 16;
              v -= mult[kind] * t.val64[q] * x[int(ck & 0xffff)];
            }
        }
        tv[i] = v;
      }
      __syncthreads();
      for (int i = tid; i < n; i += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += ws[invoff + int64_t(i) * n + j] * tv[j];
        x[off + i] = acc;
      }
      __syncthreads();
      invoff += int64_t(n) * n;
    }
    // backward: x_k = g_k - Sinv_k C_k x_{k+1}
    for (int k = t.L - 1; k >= 0; --k) {
      const int off = t.boff[k], n = t.bn[k];
      invoff -= int64_t(t.bn[k + 1]) * t.bn[k + 1];
      const double* Sk = ws + invoff - int64_t(n) * n;
      for (int i = tid; i < n; i += blockDim.x) {
        const int row = off + i;
        double v = 0.0;
        if (row != 0 && row != pad)
          for (int q = t.seg[4 * row + 2]; q < t.seg[4 * row + 3]; ++q) {
            const uint32_t ck = t.colkind[q];
            v += mult[ck >> 16] * t.val64[q] * x[int(ck & 0xffff)];
          }
        tv[i] = v;
      }
      __syncthreads();
      double nv[2] = {0.0, 0.0};
      for (int i = tid, r = 0; i < n; i += blockDim.x, ++r) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += Sk[int64_t(i) * n + j] * tv[j];
        nv[r] = x[off + i] - acc;
      }
      __syncthreads();
      for (int i = tid, r = 0; i < n; i += blockDim.x, ++r) x[off + i] = nv[r];
      __syncthreads();
    }
    for (int p = tid; p < Np; p += blockDim.x) out[int64_t(prm) * c_stride + p] = x[p];
    __syncthreads();
  }
}

// -------------------------------------------------------- a6: harmonics ---
// Phi_k = (2 pi i k / T) (1/N_s) sum_j m(t_j) e^{-2 pi i j k / N_s}, FP64 accumulation.
// One workgroup per instance: its samples (and the twiddle table, when both fit in 64 KiB) are staged
// in LDS; each thread owns one (channel, bin) and keeps two partial sums (even and odd j) so that
// consecutive multiply-adds do not wait on each other.  The twiddle index (j k) mod N_s is carried
// exactly in int32 (k < N_s / 2, so 2k < N_s and one subtraction keeps it reduced).
template <bool kTwLds>
__global__ void harmonics_kernel(const float* msamp, int Ns, int n_harm, int nch, double period,
                                 const double2* tw, float* harm, const int32_t* status, int64_t n, int st_div) {
  const int64_t inst = blockIdx.x;
  if (inst >= n) return;
  extern __shared__ double2 hsm[];  // [N_s] twiddles (kTwLds), then [nch][N_s] samples
  float* ml = reinterpret_cast<float*>(kTwLds ? hsm + Ns : hsm);
  const double2* twl = kTwLds ? hsm : tw;
  if (kTwLds)
    for (int e = threadIdx.x; e < Ns; e += blockDim.x) hsm[e] = tw[e];
  const float* src = msamp + inst * 3 * Ns;
  for (int e = threadIdx.x; e < nch * Ns; e += blockDim.x) ml[e] = src[e];
  __syncthreads();
  const bool bad = inst_failed(status[inst / st_div]);  // st_div > 1: several sample sets per instance
  const int nk = n_harm + 1;
  for (int e = threadIdx.x; e < nch * nk; e += blockDim.x) {
    const int c = e / nk, k = e % nk;
    const float* mc = ml + c * Ns;
    const int k2 = 2 * k;
    double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
    int r0 = 0, r1 = k;  // (j k) mod N_s for the even and the odd sample of a pair
    int j = 0;
    for (; j + 1 < Ns; j += 2) {
      const double2 t0 = twl[r0], t1 = twl[r1];  // (cos, sin)(2 pi r / N_s)
      const double a0 = double(mc[j]), a1 = double(mc[j + 1]);
      re0 += a0 * t0.x;
      im0 -= a0 * t0.y;
      re1 += a1 * t1.x;
      im1 -= a1 * t1.y;
      r0 += k2;
      if (r0 >= Ns) r0 -= Ns;
      r1 += k2;
      if (r1 >= Ns) r1 -= Ns;
    }
    if (j < Ns) {
      const double2 t0 = twl[r0];
      re0 += double(mc[j]) * t0.x;
      im0 -= double(mc[j]) * t0.y;
    }
    const double re = re0 + re1, im = im0 + im1;
    const double sc = 2.0 * kPi * k / period / Ns;
    float* out = harm + ((inst * nch + c) * nk + k) * 2;
    if (bad) {
      out[0] = __builtin_nanf("");
      out[1] = __builtin_nanf("");
    } else {
      out[0] = float(-sc * im);
      out[1] = float(sc * re);
    }
  }
}

// Equilibrium model (model M0, Eq. Langevin): the moment follows the field without delay or
// anisotropy, m(t_j) = L(beta |B(t_j)|) B(t_j) / |B(t_j)|, L(x) = coth(x) - 1/x, at the samples
// t_j = settle T + j T / N_s of the recorded period.  One thread per (instance, sample), FP64,
// stored as FP32 in the stepper's sample layout [n][3][N_s].
__global__ void equilibrium_kernel(int64_t n, int Ns, int settle, EqDrive d, const InstParams* ip,
                                   const int32_t* status, float* m) {
  const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= n * Ns) return;
  const int64_t i = e / Ns;
  const int j = int(e - i * Ns);
  float* out = m + i * 3 * Ns + j;
  if (status[i] != 0) {
    for (int c = 0; c < 3; ++c) out[c * Ns] = __builtin_nanf("");
    return;
  }
  const InstParams p = ip[i];
  double b[3];
  for (int c = 0; c < 3; ++c) {
    // drive phase in cycles, reduced to [0, 1) before the cosine: t is up to a few periods long
    double cyc = d.freq[c] * (double(settle) * d.period) + d.freq[c] * d.period * double(j) / double(Ns);
    cyc -= floor(cyc);
    b[c] = p.off[c] + d.amp[c] * cos(2.0 * kPi * cyc + d.phase[c]);
  }
  const double bn = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  const double x = p.beta_T * bn;
  double Lx;
  if (x < 1e-2) {
    const double x2 = x * x;  // Taylor series of coth(x) - 1/x
    Lx = x * (1.0 / 3.0 - x2 * (1.0 / 45.0 - x2 * (2.0 / 945.0)));
  } else {
    Lx = 1.0 / tanh(x) - 1.0 / x;
  }
  const double s = bn > 0.0 ? Lx / bn : 0.0;
  for (int c = 0; c < 3; ++c) out[c * Ns] = float(s * b[c]);
}

// Field of largest magnitude over the samples of one period, one thread per instance (FP64).  Ties:
// the first sample whose squared magnitude is within a relative 1e-9 of the largest, so that the choice
// does not hang on the last bits of the cosines.
struct PeakDrive {
  double amp[3], freq[3], phase[3], period;
};

__global__ void peak_field_kernel(int64_t n, const double* offset, PeakDrive d, int Ns, double* field) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double o[3] = {offset[3 * i], offset[3 * i + 1], offset[3 * i + 2]};
  auto field_at = [&](int j, double* b) {
    for (int c = 0; c < 3; ++c) {
      double cyc = d.freq[c] * d.period * double(j) / double(Ns);
      cyc -= floor(cyc);
      b[c] = o[c] + d.amp[c] * cos(2.0 * kPi * cyc + d.phase[c]);
    }
  };
  double best = -1.0;
  for (int j = 0; j < Ns; ++j) {
    double b[3];
    field_at(j, b);
    best = fmax(best, b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  }
  for (int j = 0; j < Ns; ++j) {
    double b[3];
    field_at(j, b);
    if (b[0] * b[0] + b[1] * b[1] + b[2] * b[2] >= best * (1.0 - 1e-9)) {
      for (int c = 0; c < 3; ++c) field[3 * i + c] = b[c];
      return;
    }
  }
}

// Queue order of a degree bucket of a plan launched again without a cost hint: the instances are
// sorted by the time steps the previous launch took (steps[instance], written by the stepper), most
// first, so the persistent stepper starts the longest solves first and ends on the shortest.  One
// workgroup sorts one chunk of up to kOrderChunk queue entries (bitonic network in LDS; equal counts
// by instance index, so the order does not depend on the order it starts from).  Results never
// depend on the order.
constexpr int kOrderChunk = 4096;

__global__ void __launch_bounds__(1024) order_kernel(int32_t* idx, int cnt, const int32_t* steps) {
  __shared__ int32_t key[kOrderChunk];
  __shared__ int32_t val[kOrderChunk];
  const int base = blockIdx.x * kOrderChunk;
  const int m = min(kOrderChunk, cnt - base);
  int P = 1;
  while (P < m) P <<= 1;
  for (int e = threadIdx.x; e < P; e += blockDim.x) {
    const int32_t v = e < m ? idx[base + e] : INT32_MAX;
    key[e] = e < m ? -steps[v] : INT32_MAX;  // padding sorts last
    val[e] = v;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int e = threadIdx.x; e < P; e += blockDim.x) {
        const int x = e ^ j;
        if (x > e) {
          const bool up = (e & k) == 0;
          const bool gt = key[e] > key[x] || (key[e] == key[x] && val[e] > val[x]);
          if (gt == up) {
            const int32_t tk = key[e];
            key[e] = key[x];
            key[x] = tk;
            const int32_t tv = val[e];
            val[e] = val[x];
            val[x] = tv;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < m; e += blockDim.x) idx[base + e] = val[e];
}

__global__ void fill_i32_kernel(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------- launchers ---

void launch_equilibrium(int64_t n, int Ns, int settle, const EqDrive& d, const InstParams* ip,
                        const int32_t* status, float* m, hipStream_t stream) {
  const int64_t total = n * Ns;
  if (total <= 0) return;
  hipLaunchKernelGGL(equilibrium_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, stream, n, Ns, settle, d,
                     ip, status, m);
}

void launch_peak_field(int64_t n, const double* offset, const double* amp, const double* freq, const double* phase,
                       double period, int Ns, double* field_out, hipStream_t stream) {
  if (n <= 0) return;
  PeakDrive d;
  for (int c = 0; c < 3; ++c) {
    d.amp[c] = amp[c];
    d.freq[c] = freq[c];
    d.phase[c] = phase[c];
  }
  d.period = period;
  hipLaunchKernelGGL(peak_field_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream, n, offset, d, Ns,
                     field_out);
}

void launch_order(int32_t* idx, int cnt, const int32_t* steps, hipStream_t stream) {
  if (cnt <= 1) return;
  hipLaunchKernelGGL(order_kernel, dim3(unsigned((cnt + kOrderChunk - 1) / kOrderChunk)), dim3(1024), 0, stream, idx,
                     cnt, steps);
}

void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
}

void launch_instance_prep(int64_t n, const double* D, const double* Ms, const double* K, const double* alpha,
                          const double* temp, const double* easy, const double* offset, InstParams* ip,
                          int32_t* status, hipStream_t stream) {
  const int bs = 256;
  const int64_t grid = (n + bs - 1) / bs;
  hipLaunchKernelGGL(instance_prep_kernel, dim3(grid), dim3(bs), 0, stream, n, D, Ms, K, alpha, temp, easy,
                     offset, ip, status);
}

void launch_stationary(const DevTables& t, const int32_t* idx, int n_inst, const InstParams* ip,
                       const double* field_lab, double3 drive0, double* c_out, int64_t c_stride, double* wsinv,
                       int32_t* status, hipStream_t stream) {
  const size_t shm = size_t(t.Np) * sizeof(double);
  hipLaunchKernelGGL(stationary_kernel, dim3(n_inst), dim3(kStatThreads), shm, stream, t, idx, n_inst, ip,
                     field_lab, drive0, c_out, c_stride, wsinv, status);
}

void launch_stationary_tangent(const DevTables& t, const int32_t* idx, int n_inst, const InstParams* ip,
                               double3 drive0, const double* c0, int64_t c_stride, const double* wsinv, double* ct,
                               int32_t* status, hipStream_t stream) {
  const size_t shm = size_t(t.Np) * sizeof(double);
  hipLaunchKernelGGL(stationary_tangent_kernel, dim3(n_inst), dim3(kStatThreads), shm, stream, t, idx, n_inst, ip,
                     drive0, c0, c_stride, wsinv, ct, status);
}

void launch_harmonics(const float* msamp, int Ns, int n_harm, int nch, double period, const double2* tw,
                      float* harm, const int32_t* status, int64_t n, hipStream_t stream, int st_div) {
  if (n <= 0) return;
  const int items = nch * (n_harm + 1);
  const int threads = std::min(512, std::max(64, (items + 63) / 64 * 64));  // one (channel, bin) per thread
  const size_t samples = size_t(nch) * Ns * sizeof(float);
  const size_t with_tw = size_t(Ns) * sizeof(double2) + samples;
  if (with_tw <= 64 * 1024)
    hipLaunchKernelGGL(harmonics_kernel<true>, dim3(n), dim3(threads), with_tw, stream, msamp, Ns, n_harm, nch,
                       period, tw, harm, status, n, st_div);
  else
    hipLaunchKernelGGL(harmonics_kernel<false>, dim3(n), dim3(threads), samples, stream, msamp, Ns, n_harm, nch,
                       period, tw, harm, status, n, st_div);
}

// grad[i][p] = sum over channels, bins and (re, im) of dL/dPhi[i] * dPhi/dp[i][p], FP64 accumulation;
// one workgroup per instance.  NaN for instances with a non-zero status.
__global__ void contract_kernel(const float* dL, const float* dharm, int per, double* grad, const int32_t* status,
                                int64_t n) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  __shared__ double red[kNTan][256];
  double acc[kNTan] = {0, 0, 0, 0, 0};
  const float* g = dL + i * per;
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const double w = g[e];
    for (int p = 0; p < kNTan; ++p) acc[p] += w * double(dharm[(i * kNTan + p) * per + e]);
  }
  for (int p = 0; p < kNTan; ++p) red[p][threadIdx.x] = acc[p];
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o)
      for (int p = 0; p < kNTan; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < kNTan) grad[i * kNTan + threadIdx.x] = inst_failed(status[i]) ? __builtin_nan("") : red[threadIdx.x][0];
}

void launch_contract(const float* dL, const float* dharm, int per, double* grad, const int32_t* status, int64_t n,
                     hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(contract_kernel, dim3(n), dim3(256), 0, stream, dL, dharm, per, grad, status, n);
}

}  // namespace fpn
