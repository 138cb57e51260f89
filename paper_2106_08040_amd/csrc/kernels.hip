// HIP kernels of the fpn solver for gfx950 (MI355X).
//
//   instance_prep      a1: particle scalars + easy-axis frame per instance (FP64)
//   stationary_fp64    a3: stationary density of the field at t = 0 (FP64 block solve)
//   stepper<L>         a4/a5: FP32 RODAS4 over the drive, one wavefront per instance,
//                      block inverses resident in VGPRs, m(t_j) samples written out
//   harmonics_fp64     a6: Phi_k = (2 pi i k / T) DFT_k(m) with FP64 accumulation
//
// Paper basis: Eq. FP-general + Eq. convection (operator), Eq. mean_magmom_FP (moment),
// Eq. MPI_model_fourier / phi-hat of model M1 (harmonics).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "physics.hpp"

namespace fpn {

// ------------------------------------------------------------------ helpers ---

// Completes this wavefront's outstanding LDS traffic and orders memory accesses.
__device__ __forceinline__ void wsync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}
template <int I, int E, typename F>
__device__ __forceinline__ void static_for_down(F&& f) {  // I, I-1, ..., E
  if constexpr (I >= E) {
    f(std::integral_constant<int, I>{});
    static_for_down<I - 1, E>(f);
  }
}

// Kind multipliers (1/s per unit table value) of the Galerkin operator, see structure.hpp.
__device__ __forceinline__ float kind_mult(int kind, float inv2tau, float sigma, float alpha, float beta,
                                           float hx, float hy, float hz) {
  switch (kind) {
    case 0: return inv2tau;
    case 1: return inv2tau * sigma;
    case 2: return inv2tau * 2.0f * sigma / alpha;
    case 3: return inv2tau * beta * hz;
    case 4: return inv2tau * beta * hz / alpha;
    case 5: return inv2tau * beta * hx;
    case 6: return inv2tau * beta * hy;
    case 7: return inv2tau * beta * hx / alpha;
    default: return inv2tau * beta * hy / alpha;
  }
}

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

// ---------------------------------------------------------- a4/a5: stepper ---

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
  static constexpr int S = (Np + 63) / 64;  // vector slots per lane
};

template <int Q>
struct Arr {
  float v[Q];
};
template <int L, int K>
struct Store : Store<L, K - 1> {
  Arr<Geo<L>::nb(K) / 2> a;
};
template <int L>
struct Store<L, -1> {};
template <int K, int L>
__device__ __forceinline__ auto& blk(Store<L, L>& s) {
  return static_cast<Store<L, K>&>(s).a.v;
}

// Per-wavefront LDS scratch (floats).
struct WaveLds {
  static constexpr int kVec = 640;  // >= Np for L <= 24
  float X[32 * 32];    // dense scratch: Sinv_{k-1} copy, then D_k  ([row][parity][16])
  float Ub[32 * 32];   // U = B_k Sinv_{k-1}                         ([row][parity][16])
  float xin[kVec];     // matvec input
  float V[kVec];       // solve right-hand side
  float G[kVec];       // solve result
  float T[32];         // block-local right-hand side, [parity][16]
  float col[64];       // pivot columns [parity][32]
  float row[64];       // pivot rows [r][parity][16]
  float mk[16];        // -h g * multiplier(t_n) per kind
  float ms[16];        // multiplier at the current stage time per kind
  float mm[4];         // misc
};

// In-place inverse of the lane-distributed block (lane: row i = lane&31, column
// parity h = lane>>5, a[q] = A[i][h + 2q]) by Gauss-Jordan with 2x2 pivots on the
// (cos, sin) pairs (rows/cols 2qq, 2qq+1).
template <int Q>
__device__ __forceinline__ bool gj2_invert(float (&a)[Q], int i, int h, WaveLds& w) {
  constexpr int n = 2 * Q;
  const bool act = i < n;
  bool ok = true;
  for (int qq = 0; qq < Q; ++qq) {
    const int r0 = 2 * qq;
    const float cv = a[qq];  // (i, r0 + h)
    if (act) w.col[h * 32 + i] = cv;
    const int r = i - r0;
    const bool inR = act && (r == 0 || r == 1);
    if (inR) {
#pragma unroll
      for (int q = 0; q < Q; ++q) w.row[(r * 2 + h) * 16 + q] = a[q];
    }
    wsync();
    const float P00 = w.col[r0], P01 = w.col[32 + r0];
    const float P10 = w.col[r0 + 1], P11 = w.col[32 + r0 + 1];
    const float det = P00 * P11 - P01 * P10;
    ok = ok && (det != 0.0f) && isfinite(det);
    const float id = 1.0f / det;
    const float Pi00 = P11 * id, Pi01 = -P01 * id, Pi10 = -P10 * id, Pi11 = P00 * id;
    const float g0 = act ? w.col[i] : 0.0f;
    const float g1 = act ? w.col[32 + i] : 0.0f;
    float G0 = g0 * Pi00 + g1 * Pi10;
    float G1 = g0 * Pi01 + g1 * Pi11;
    float s = 1.0f;
    float newc = (h == 0) ? -G0 : -G1;
    if (inR) {
      s = 0.0f;
      G0 = (r == 0) ? -Pi00 : -Pi10;
      G1 = (r == 0) ? -Pi01 : -Pi11;
      newc = (r == 0) ? ((h == 0) ? Pi00 : Pi01) : ((h == 0) ? Pi10 : Pi11);
    }
    const float* w0 = w.row + (0 * 2 + h) * 16;
    const float* w1 = w.row + (1 * 2 + h) * 16;
#pragma unroll
    for (int q = 0; q < Q; ++q) a[q] = fmaf(-G1, w1[q], fmaf(-G0, w0[q], s * a[q]));
    a[qq] = act ? newc : 0.0f;
    wsync();
  }
  return ok;
}

struct StepArgs {
  const InstParams* ip;
  const int32_t* inst_idx;
  int n_inst;
  const double* c0;
  int64_t c_stride;
  const float4* drive;  // [spp][5]: H(t_n + al h) for al = 0, .386, .21, .63 and dH/dt(t_n)
  int spp;              // steps per period
  int substeps;
  int settle;
  int Ns;
  float h;
  float* msamp;         // [n_total][3][Ns]
  int32_t* status;
};

template <int L>
struct StepperCtx {
  const float* hv;        // not used directly
};

template <int L, int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
stepper_kernel(StepArgs A, DevTables t) {
  using Gm = Geo<L>;
  constexpr int Np = Gm::Np;
  constexpr int S = Gm::S;
  extern __shared__ __align__(16) unsigned char smem[];
  // tables
  int32_t* seg = reinterpret_cast<int32_t*>(smem);
  uint32_t* colkind = reinterpret_cast<uint32_t*>(seg + 4 * Np);
  float* val = reinterpret_cast<float*>(colkind + t.nnz);
  int32_t* cptr = reinterpret_cast<int32_t*>(val + t.nnz);
  uint32_t* crowkind = reinterpret_cast<uint32_t*>(cptr + Np + 1);
  float* cval = reinterpret_cast<float*>(crowkind + t.nnzc);
  size_t tbytes = (size_t(4 * Np) + t.nnz * 2 + (Np + 1) + t.nnzc * 2) * 4;
  tbytes = (tbytes + 15) & ~size_t(15);
  WaveLds* wl = reinterpret_cast<WaveLds*>(smem + tbytes);

  for (int e = threadIdx.x; e < 4 * Np; e += blockDim.x) seg[e] = t.seg[e];
  for (int e = threadIdx.x; e < t.nnz; e += blockDim.x) { colkind[e] = t.colkind[e]; val[e] = t.val[e]; }
  for (int e = threadIdx.x; e <= Np; e += blockDim.x) cptr[e] = t.cptr[e];
  for (int e = threadIdx.x; e < t.nnzc; e += blockDim.x) { crowkind[e] = t.crowkind[e]; cval[e] = t.cval[e]; }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int slot = blockIdx.x * WAVES + wid;
  if (slot >= A.n_inst) return;
  const int inst = A.inst_idx[slot];
  WaveLds& w = wl[wid];
  const int i = lane & 31, h = lane >> 5;
  float* ms_out = A.msamp + int64_t(inst) * 3 * A.Ns;
  if (A.status[inst] != 0) {
    for (int j = lane; j < 3 * A.Ns; j += 64) ms_out[j] = __builtin_nanf("");
    return;
  }
  const InstParams P = A.ip[inst];
  const float inv2tau = float(P.inv2tau), sigma = float(P.sigma), alpha = float(P.alpha), beta = float(P.beta_T);
  float R[9], off[3];
  for (int c = 0; c < 9; ++c) R[c] = float(P.R[c]);
  for (int c = 0; c < 3; ++c) off[c] = float(P.off[c]);

  // state in block order: lane holds positions lane + 64 s
  float y[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int p = lane + 64 * s;
    y[s] = (p < Np) ? float(A.c0[int64_t(inst) * A.c_stride + p]) : 0.0f;
  }
  Store<L, L> st;

  const float hstep = A.h;
  const float hg = hstep * Rodas4::g;
  const int total = (A.settle + 1) * A.spp;
  const int first_rec = A.settle * A.spp;
  const float rc = 2.0466534158929770f;  // sqrt(4 pi / 3)
  constexpr int pX = Gm::off(1), pY = Gm::off(1) + 1, pZ = 1;
  bool ok = true;

  // per-lane multiplier for kind `lane` at lab field B (lab frame, tesla)
  auto mult_lane = [&](float4 B) -> float {
    const float bx = B.x + off[0], by = B.y + off[1], bz = B.z + off[2];
    const float hx = R[0] * bx + R[3] * by + R[6] * bz;
    const float hy = R[1] * bx + R[4] * by + R[7] * bz;
    const float hz = R[2] * bx + R[5] * by + R[8] * bz;
    return kind_mult(lane < 9 ? lane : 0, inv2tau, sigma, alpha, beta, hx, hy, hz);
  };
  auto dmult_lane = [&](float4 dB) -> float {
    const float hx = R[0] * dB.x + R[3] * dB.y + R[6] * dB.z;
    const float hy = R[1] * dB.x + R[4] * dB.y + R[7] * dB.z;
    const float hz = R[2] * dB.x + R[5] * dB.y + R[8] * dB.z;
    return (lane < 3) ? 0.0f : kind_mult(lane < 9 ? lane : 0, inv2tau, sigma, alpha, beta, hx, hy, hz);
  };
  // y_out = A(ms) x  (x in w.xin), rows lane + 64 s
  auto matvec = [&](float (&out)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      float acc = 0.0f;
      if (p < Np) {
        const int e1 = seg[4 * p + 3];
        for (int e = seg[4 * p]; e < e1; ++e) {
          const uint32_t ck = colkind[e];
          acc = fmaf(w.ms[ck >> 16] * val[e], w.xin[ck & 0xffff], acc);
        }
      }
      out[s] = acc;
    }
  };
  // Block-tridiagonal solve M x = V with the resident inverses; result in w.G.
  auto solve = [&]() {
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      if (h == 0 && i < n) {
        const int row = off0 + i;
        float tv = w.V[row];
        if constexpr (K > 0) {
          const int e1 = seg[4 * row + 1];
          for (int e = seg[4 * row]; e < e1; ++e) {
            const uint32_t ck = colkind[e];
            tv = fmaf(-w.mk[ck >> 16] * val[e], w.G[ck & 0xffff], tv);
          }
        }
        w.T[(i & 1) * 16 + (i >> 1)] = tv;
      }
      wsync();
      auto& a = blk<K>(st);
      float part = 0.0f;
#pragma unroll
      for (int q = 0; q < Q; ++q) part = fmaf(a[q], w.T[h * 16 + q], part);
      part += __shfl_xor(part, 32);
      if (h == 0 && i < n) w.G[off0 + i] = part;
      wsync();
    });
    static_for_down<L - 1, 0>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      if (h == 0 && i < n) {
        const int row = off0 + i;
        float tv = 0.0f;
        const int e1 = seg[4 * row + 3];
        for (int e = seg[4 * row + 2]; e < e1; ++e) {
          const uint32_t ck = colkind[e];
          tv = fmaf(w.mk[ck >> 16] * val[e], w.G[ck & 0xffff], tv);
        }
        w.T[(i & 1) * 16 + (i >> 1)] = tv;
      }
      wsync();
      auto& a = blk<K>(st);
      float part = 0.0f;
#pragma unroll
      for (int q = 0; q < Q; ++q) part = fmaf(a[q], w.T[h * 16 + q], part);
      part += __shfl_xor(part, 32);
      if (h == 0 && i < n) w.G[off0 + i] -= part;
      wsync();
    });
  };
  // Factor M = I - h g A(t_n): block inverses of the Schur complements into registers.
  auto factor = [&]() {
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      const bool act = i < n;
      if constexpr (K > 0) {
        constexpr int np = Gm::nb(K - 1), Qp = np / 2, offp = Gm::off(K - 1);
        auto& ap = blk<K - 1>(st);
        if (i < np) {
#pragma unroll
          for (int q = 0; q < Qp; ++q) w.X[i * 32 + h * 16 + q] = ap[q];
        }
        wsync();
        float u[Qp];
#pragma unroll
        for (int q = 0; q < Qp; ++q) u[q] = 0.0f;
        if (act) {
          const int row = off0 + i;
          const int e1 = seg[4 * row + 1];
          for (int e = seg[4 * row]; e < e1; ++e) {
            const uint32_t ck = colkind[e];
            const float me = w.mk[ck >> 16] * val[e];
            const float* xr = w.X + (int(ck & 0xffff) - offp) * 32 + h * 16;
#pragma unroll
            for (int q = 0; q < Qp; ++q) u[q] = fmaf(me, xr[q], u[q]);
          }
#pragma unroll
          for (int q = 0; q < Qp; ++q) w.Ub[i * 32 + h * 16 + q] = u[q];
        }
        wsync();
      }
      // D_k (with identity) into X
      if (act) {
#pragma unroll
        for (int q = 0; q < Q; ++q) w.X[i * 32 + h * 16 + q] = 0.0f;
      }
      wsync();
      if (act) {
        const int row = off0 + i;
        const int e1 = seg[4 * row + 2];
        for (int e = seg[4 * row + 1]; e < e1; ++e) {
          const uint32_t ck = colkind[e];
          const int c = int(ck & 0xffff) - off0;
          if ((c & 1) == h) w.X[i * 32 + h * 16 + (c >> 1)] += w.mk[ck >> 16] * val[e];
        }
        if ((i & 1) == h) w.X[i * 32 + h * 16 + (i >> 1)] += 1.0f;
      }
      wsync();
      auto& a = blk<K>(st);
#pragma unroll
      for (int q = 0; q < Q; ++q) a[q] = act ? w.X[i * 32 + h * 16 + q] : 0.0f;
      if constexpr (K > 0) {
        constexpr int offp = Gm::off(K - 1);
        if (act) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int c = off0 + h + 2 * q;
            float acc = 0.0f;
            const int e1 = cptr[c + 1];
            for (int e = cptr[c]; e < e1; ++e) {
              const uint32_t rk = crowkind[e];
              const int rl = int(rk & 0xffff) - offp;
              acc = fmaf(w.mk[rk >> 16] * cval[e], w.Ub[i * 32 + (rl & 1) * 16 + (rl >> 1)], acc);
            }
            a[q] -= acc;
          }
        }
      }
      ok = gj2_invert<Q>(a, i, h, w) && ok;
    });
  };

  float K1[S], K2[S], K3[S], K4[S], K5[S], ft[S], yt[S];
  constexpr float a21 = 1.544f;
  constexpr float a31 = 0.9466785280815826f, a32 = 0.2557011698983284f;
  constexpr float a41 = 3.314825187068521f, a42 = 2.896124015972201f, a43 = 0.9986419139977817f;
  constexpr float a51 = 1.221224509226641f, a52 = 6.019134481288629f, a53 = 12.53708332932087f,
                  a54 = -0.6878860361058950f;
  constexpr float c21 = -5.668800000000000f;
  constexpr float c31 = -2.430093356833875f, c32 = -0.2063599157091915f;
  constexpr float c41 = -0.1073529058151375f, c42 = -9.594562251023355f, c43 = -20.47028614809616f;
  constexpr float c51 = 7.496443313967647f, c52 = -10.24680431464352f, c53 = -33.99990352819905f,
                  c54 = 11.70890893206160f;
  constexpr float c61 = 8.083246795921522f, c62 = -7.981132988064893f, c63 = -31.52159432874371f,
                  c64 = 16.31930543123136f, c65 = -6.058818238834054f;
  constexpr float gm1 = 0.25f, gm2 = -0.1043f, gm3 = 0.1035f, gm4 = -0.03620000000000023f;
  const float ih = 1.0f / hstep;

  // stage: write x (registers) to xin, rhs = A(ms) x + extra, solve, return hg * x
  auto stage_solve = [&](float (&xv)[S], float (&extra)[S], float (&kout)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      if (p < Np) w.xin[p] = xv[s];
    }
    wsync();
    float r[S];
    matvec(r);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      if (p < Np) w.V[p] = r[s] + extra[s];
    }
    wsync();
    solve();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      kout[s] = (p < Np) ? hg * w.G[p] : 0.0f;
    }
  };

  for (int n = 0; n < total && ok; ++n) {
    const int dn = n % A.spp;
    if (n >= first_rec && (n - first_rec) % A.substeps == 0) {
      const int j = (n - first_rec) / A.substeps;
      const float vx = __shfl(y[pX >> 6], pX & 63), vy = __shfl(y[pY >> 6], pY & 63), vz = __shfl(y[pZ >> 6], pZ & 63);
      if (lane < 3) {
        const float r0 = lane == 0 ? R[0] : (lane == 1 ? R[3] : R[6]);
        const float r1 = lane == 0 ? R[1] : (lane == 1 ? R[4] : R[7]);
        const float r2 = lane == 0 ? R[2] : (lane == 1 ? R[5] : R[8]);
        const float mv = rc * (r0 * vx + r1 * vy + r2 * vz);
        ms_out[lane * A.Ns + j] = mv;
      }
      ok = ok && isfinite(vx) && isfinite(vy) && isfinite(vz);
    }
    const float4* dr = A.drive + int64_t(dn) * 5;
    const float4* drn = A.drive + int64_t((dn + 1) % A.spp) * 5;
    // factorisation multipliers: -h g * A(t_n)
    {
      const float mt = mult_lane(dr[0]);
      if (lane < 9) { w.mk[lane] = -hg * mt; w.ms[lane] = mt; }
      wsync();
    }
    factor();
    // f_t = A'(t_n) y
    {
      const float md = dmult_lane(dr[4]);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        if (p < Np) w.xin[p] = y[s];
      }
      if (lane < 9) w.ms[lane] = md;
      wsync();
      matvec(ft);
      wsync();
      const float mt = mult_lane(dr[0]);
      if (lane < 9) w.ms[lane] = mt;
      wsync();
    }
    // stage 1 (al = 0): rhs = A(t_n) y + h g1 f_t
    float ex[S];
#pragma unroll
    for (int s = 0; s < S; ++s) ex[s] = hstep * gm1 * ft[s];
    stage_solve(y, ex, K1);
    // stage 2 (al = .386)
    {
      const float mt = mult_lane(dr[1]);
      if (lane < 9) w.ms[lane] = mt;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        yt[s] = fmaf(a21, K1[s], y[s]);
        ex[s] = c21 * ih * K1[s] + hstep * gm2 * ft[s];
      }
      stage_solve(yt, ex, K2);
    }
    // stage 3 (al = .21)
    {
      const float mt = mult_lane(dr[2]);
      if (lane < 9) w.ms[lane] = mt;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        yt[s] = fmaf(a32, K2[s], fmaf(a31, K1[s], y[s]));
        ex[s] = ih * (c31 * K1[s] + c32 * K2[s]) + hstep * gm3 * ft[s];
      }
      stage_solve(yt, ex, K3);
    }
    // stage 4 (al = .63)
    {
      const float mt = mult_lane(dr[3]);
      if (lane < 9) w.ms[lane] = mt;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        yt[s] = fmaf(a43, K3[s], fmaf(a42, K2[s], fmaf(a41, K1[s], y[s])));
        ex[s] = ih * (c41 * K1[s] + c42 * K2[s] + c43 * K3[s]) + hstep * gm4 * ft[s];
      }
      stage_solve(yt, ex, K4);
    }
    // stage 5 (al = 1)
    {
      const float mt = mult_lane(drn[0]);
      if (lane < 9) w.ms[lane] = mt;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        yt[s] = fmaf(a54, K4[s], fmaf(a53, K3[s], fmaf(a52, K2[s], fmaf(a51, K1[s], y[s]))));
        ex[s] = ih * (c51 * K1[s] + c52 * K2[s] + c53 * K3[s] + c54 * K4[s]);
      }
      stage_solve(yt, ex, K5);
    }
    // stage 6 (al = 1): argument y + sum a6j K_j = yt + K5; y_{n+1} = that + K6
    {
      float K6[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        yt[s] += K5[s];
        ex[s] = ih * (c61 * K1[s] + c62 * K2[s] + c63 * K3[s] + c64 * K4[s] + c65 * K5[s]);
      }
      stage_solve(yt, ex, K6);
#pragma unroll
      for (int s = 0; s < S; ++s) y[s] = yt[s] + K6[s];
    }
  }
  if (!ok) {
    for (int j = lane; j < 3 * A.Ns; j += 64) ms_out[j] = __builtin_nanf("");
    if (lane == 0) A.status[inst] = 2;
  }
}

// -------------------------------------------------------- a6: harmonics ---
// Phi_k = (2 pi i k / T) (1/N_s) sum_j m(t_j) e^{-2 pi i j k / N_s}, FP64 accumulation.
// One workgroup per instance; the twiddle index (j k) mod N_s is carried exactly in int32.
__global__ void harmonics_kernel(const float* msamp, int Ns, int n_harm, int nch, double period,
                                 const double2* tw, float* harm, const int32_t* status, int64_t n) {
  const int64_t inst = blockIdx.x;
  if (inst >= n) return;
  extern __shared__ float ml[];  // [3][Ns]
  const float* src = msamp + inst * 3 * Ns;
  for (int e = threadIdx.x; e < 3 * Ns; e += blockDim.x) ml[e] = src[e];
  __syncthreads();
  const bool bad = status[inst] != 0;
  const int nk = n_harm + 1;
  for (int e = threadIdx.x; e < nch * nk; e += blockDim.x) {
    const int c = e / nk, k = e % nk;
    double re = 0.0, im = 0.0;
    int r = 0;
    const float* mc = ml + c * Ns;
    for (int j = 0; j < Ns; ++j) {
      const double2 t = tw[r];  // (cos, sin)(2 pi r / N_s)
      re += double(mc[j]) * t.x;
      im -= double(mc[j]) * t.y;
      r += k;
      if (r >= Ns) r -= Ns;
    }
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

// ------------------------------------------------------------- launchers ---

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

constexpr int kWaves = 4;

size_t stepper_lds_bytes(const DevTables& t) {
  size_t tbytes = (size_t(4 * t.Np) + size_t(t.nnz) * 2 + (t.Np + 1) + size_t(t.nnzc) * 2) * 4;
  tbytes = (tbytes + 15) & ~size_t(15);
  return tbytes + kWaves * sizeof(WaveLds);
}

template <int L>
static hipError_t launch_stepper_L(const StepLaunch& s, const DevTables& t, hipStream_t stream) {
  StepArgs a;
  a.ip = s.ip;
  a.inst_idx = s.inst_idx;
  a.n_inst = s.n_inst;
  a.c0 = s.c0;
  a.c_stride = s.c_stride;
  a.drive = s.drive;
  a.spp = s.spp;
  a.substeps = s.substeps;
  a.settle = s.settle;
  a.Ns = s.Ns;
  a.h = s.h;
  a.msamp = s.msamp;
  a.status = s.status;
  const size_t shm = stepper_lds_bytes(t);
  auto kern = stepper_kernel<L, kWaves>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  if (e != hipSuccess) return e;
  const int grid = (s.n_inst + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kWaves), shm, stream, a, t);
  return hipGetLastError();
}

hipError_t launch_stepper(int L, const StepLaunch& s, const DevTables& t, hipStream_t stream) {
  switch (L) {
#define FPN_CASE(LL) \
  case LL: return launch_stepper_L<LL>(s, t, stream);
    FPN_CASE(10) FPN_CASE(16)

#undef FPN_CASE
    default: return hipErrorInvalidValue;
  }
}

void launch_harmonics(const float* msamp, int Ns, int n_harm, int nch, double period, const double2* tw,
                      float* harm, const int32_t* status, int64_t n, hipStream_t stream) {
  const size_t shm = size_t(3) * Ns * sizeof(float);
  hipLaunchKernelGGL(harmonics_kernel, dim3(n), dim3(256), shm, stream, msamp, Ns, n_harm, nch, period, tw, harm,
                     status, n);
}

}  // namespace fpn
