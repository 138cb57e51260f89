// FP32 time stepper for large degrees (L = 17..24): the same RODAS4 integration as stepper.hip, with
// a block layout that fits |m| blocks of up to 64 rows.
//
// One wavefront per instance; lane i owns row i of the block being factored.  A block's Schur
// complement is built and inverted in registers (Gauss-Jordan with partial pivoting, columns rotated
// by one after every pivot so all register indexing is static) and the
// inverse is written to a per-instance workspace in global memory, column-quad-major so that a
// wavefront reads 1 KiB contiguous per quad of columns in the stage solves.  The state vector stays
// in registers, the stage and gather vectors in LDS (xin, V, G) or in the workspace (K1..K5, f_t,
// which only their own lane reads).  The operator tables are read from global memory (they are
// shared by every wavefront and stay in L2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "physics.hpp"
#include "stepper_common.hpp"

namespace fpn {

template <int L>
struct WGeo {
  using G = Geo<L>;
  static constexpr int NB = G::n0 > G::nb(1) ? G::n0 : G::nb(1);  // largest block
  static constexpr int XS = NB + 1;                                // odd LDS row stride
  static constexpr int XR = NB + 4;                                // rows incl. window overhang
  static constexpr int q4(int k) { return (G::nb(k) + 3) / 4; }
  static constexpr int ioff(int k) {
    int o = 0;
    for (int j = 0; j < k; ++j) o += 4 * q4(j) * G::nb(j);
    return o;
  }
  static constexpr int INV = ioff(L + 1);        // floats of all block inverses
  static constexpr int WS = INV + 6 * G::NpA;    // + K1..K5 and f_t
};

template <int L>
struct WideLds {
  static constexpr int NpA = Geo<L>::NpA;
  static constexpr int kX = WGeo<L>::XR * WGeo<L>::XS;
  static constexpr int kA = (((kX > 2 * NpA) ? kX : 2 * NpA) + 3) & ~3;  // keeps T 16-byte aligned
  float a[kA];        // X (factorisation) | xin, V (stages)
  float g[NpA];       // G (block-solve result)
  float T[64];        // block right-hand side
  float prow[2][64];  // pivot row
  float cw[6][64];    // Schur coefficients of one block, multiplier included
  float mk[16];
  float ms[16];
  double msd[16];     // FP64 multipliers of the right-hand side evaluation (stage or time-derivative)
  double ctl[6];      // step controller: time, next step size, this step size, landed, last attempt rejected
  float xlo[NpA];     // low-order part of the stage argument (xin + xlo)
  __device__ float* X() { return a; }
  __device__ float* xin() { return a; }
  __device__ float* V() { return a + NpA; }
  __device__ float* G() { return g; }
};

// FP64 multiplier of operator kind `kind` (kind numbering of structure.hpp) at time tt: the kinds of the
// field use its value with the static offset (deriv = false) or its time derivative (deriv = true,
// field-free kinds 0..2 give 0).  Field mu0 H_a(t) = amp_a cos(2 pi f_a t + phase_a) with the cycles
// reduced in FP64, frame and particle scalars from the FP64 instance data.
__device__ inline double kind_mult_d(int kind, const InstParams& Q, const double* amp, const double* freq,
                                     const double* phase, double tt, bool deriv) {
  double b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double cyc = freq[a] * tt;
    const double x = 2.0 * (cyc - floor(cyc)) + phase[a] * 0.3183098861837907;
    b[a] = deriv ? -amp[a] * 2.0 * kPi * freq[a] * sinpi(x) : amp[a] * cospi(x) + Q.off[a];
  }
  const double hx = Q.R[0] * b[0] + Q.R[3] * b[1] + Q.R[6] * b[2];
  const double hy = Q.R[1] * b[0] + Q.R[4] * b[1] + Q.R[7] * b[2];
  const double hz = Q.R[2] * b[0] + Q.R[5] * b[1] + Q.R[8] * b[2];
  const double s2 = Q.inv2tau, sb = Q.inv2tau * Q.beta_T, ia = 1.0 / Q.alpha;
  switch (kind) {
    case 0: return deriv ? 0.0 : s2;
    case 1: return deriv ? 0.0 : s2 * Q.sigma;
    case 2: return deriv ? 0.0 : s2 * 2.0 * Q.sigma * ia;
    case 3: return sb * hz;
    case 4: return sb * hz * ia;
    case 5: return sb * hx;
    case 6: return sb * hy;
    case 7: return sb * hx * ia;
    default: return sb * hy * ia;
  }
}

// s + e = a + b exactly, s = fl(a + b) (Knuth's branch-free two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// In-place inverse of an n x n block, row `lane` in a[0..n-1], by Gauss-Jordan with partial pivoting
// (single rows).  Pivot k works on column 0 of the rotated order (original column k): the remaining
// row with the largest |entry| pivots, and the new pivot column is appended at n - 1, so after n
// pivots the columns are back in their original order and all register indexing is static.  The
// tableau then holds the inverse with rows and columns permuted; X (row stride XS) puts it back.
// kRow0 (block 0): row 0 is e_0 and pivots column 0, which conserves c_00 exactly (see stepper.hip).
// As there, a pivot row keeps its scale P (pivot-column entry 1) and is divided by P once at the end.
template <int n, int XS, bool kRow0, typename WL>
__device__ __forceinline__ bool gj_piv_invert_wide(float (&a)[n], int lane, WL& w, float* X) {
  const bool act = lane < n;
  bool ok = true;
  bool cand = act;
  int mycol = 0;  // column this row pivoted
  int cpiv = 0;   // lane k: pivot row of column k
  float myip = 1.0f;  // 1 / pivot of this row (deferred scale)
#pragma unroll 1
  for (int k = 0; k < n; ++k) {
    const float g = a[0];
    const uint32_t best = max64_uniform(pivot_key<6>(g, lane, cand));
    const int p = (kRow0 && k == 0) ? 0 : int(best & 63u);
    const float P = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g), p));
    ok = ok && (P != 0.0f) && isfinite(P);
    const float ip = 1.0f / P;
    const bool isp = (lane == p);
    if (isp) {
#pragma unroll
      for (int q = 1; q < n; ++q) w.prow[0][q] = a[q];
    }
    if (lane == k) cpiv = p;
    wsync();
    const float G = isp ? 0.0f : g * ip;
#pragma unroll
    for (int q = 1; q < n; ++q) {
      a[q - 1] = fmaf(-G, w.prow[0][q], a[q]);
      if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    a[n - 1] = act ? (isp ? 1.0f : -G) : 0.0f;
    if (isp) {
      cand = false;
      mycol = k;
      myip = ip;
    }
    wsync();
  }
  // inverse entry (a, b) = tableau entry (pivot row of column a, column pivoted by row b)
  if (act) {
#pragma unroll
    for (int q = 0; q < n; ++q) X[lane * XS + q] = a[q] * myip;
  }
  wsync();
  const float* xr = X + cpiv * XS;
#pragma unroll
  for (int q = 0; q < n; ++q) a[q] = act ? xr[__builtin_amdgcn_readlane(mycol, q)] : 0.0f;
  wsync();
  return ok;
}

// Bytes of dynamic LDS before the LDS-resident workspace (WAVES = 1): the wavefront scratch, rounded
// to 16 bytes for the float4 inverse quads.
template <int L, int WAVES>
constexpr size_t wide_lds_scratch_bytes() {
  return (WAVES * sizeof(WideLds<L>) + 15) & ~size_t(15);
}

// WAVES = 4: four instances per workgroup, each wavefront's workspace (block inverses, K1..K5, f_t) in
// global memory (`ws`, one slot per resident wavefront).  WAVES = 1: one instance per workgroup with its
// workspace in LDS behind the scratch (48 KB at L = 17 .. 114 KB at L = 24), so the block solves read the
// inverses at LDS rather than L2 latency; fewer instances are resident at once.
template <int L, int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
stepper_wide_kernel(StepArgs A, DevTables t, float* ws) {
  using Gm = Geo<L>;
  using WG = WGeo<L>;
  using WL = WideLds<L>;
  constexpr int Np = Gm::Np;
  constexpr int NpA = Gm::NpA;
  constexpr int S = Gm::S;
  constexpr int XS = WG::XS;
  extern __shared__ __align__(16) unsigned char smem[];
  WL* wl = reinterpret_cast<WL*>(smem);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));  // uniform per wavefront
  const int slot = blockIdx.x * WAVES + wid;  // resident wavefront index
  // persistent: every wavefront takes instances from the launch's queue until it is drained
  for (;;) {
  int qk = 0;
  if (lane == 0) qk = atomicAdd(A.queue, 1);
  qk = __builtin_amdgcn_readfirstlane(__shfl(qk, 0));
  if (qk >= A.n_inst) break;
  const int inst = A.inst_idx[qk];
  WL& w = wl[wid];
  clear_wave_scratch(w, lane);
  wsync();
  float* inv;
  if constexpr (WAVES == 1) {
    inv = reinterpret_cast<float*>(smem + wide_lds_scratch_bytes<L, WAVES>());
  } else {
    inv = ws + int64_t(slot) * WG::WS;
  }
  float* Kg = inv + WG::INV;  // K1..K5 at j * NpA, f_t at 5 * NpA
  const uint16_t* ecol = t.ell_col;
  const float* eval = t.ell_val;
  const float* elo = t.ell_lo;
  const float* wB = t.win_b;
  const float* wC = t.win_c;
  const float* wS = t.win_s;
  float* ms_out = A.msamp + int64_t(inst) * 3 * A.Ns;
  float* dd_out = A.dmdt ? A.dmdt + int64_t(inst) * 3 * A.Ns : nullptr;
  if (A.status[inst] != 0) {
    for (int j = lane; j < 3 * A.Ns; j += 64) ms_out[j] = __builtin_nanf("");
    if (dd_out)
      for (int j = lane; j < 3 * A.Ns; j += 64) dd_out[j] = __builtin_nanf("");
    if (A.steps_out && lane == 0) A.steps_out[inst] = 0;
    continue;
  }
  const InstParams P = A.ip[inst];
  const float inv2tau = float(P.inv2tau), sigma = float(P.sigma), alpha = float(P.alpha), beta = float(P.beta_T);
  float R[9], off[3];
  for (int c = 0; c < 9; ++c) R[c] = float(P.R[c]);
  for (int c = 0; c < 3; ++c) off[c] = float(P.off[c]);

  // the state is carried as an unevaluated sum y + ylo of two FP32 values (about 48 bits): the slow
  // relaxation of a stiff particle moves it by much less than one FP32 unit per step, and a state
  // rounded to FP32 after every step loses or biases those increments
  float y[S], ylo[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int p = lane + 64 * s;
    const double c = (p < Np) ? A.c0[int64_t(inst) * A.c_stride + p] : 0.0;
    y[s] = float(c);
    ylo[s] = float(c - double(y[s]));
  }
  const float rc = 2.0466534158929770f;  // sqrt(4 pi / 3)
  constexpr int pX = Gm::off(1), pY = Gm::off(1) + 1, pZ = 1;
  bool ok = true;

  auto field = [&](double tt, float& bx, float& by, float& bz, bool deriv) {
    float v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double cyc = A.freq[a] * tt;
      const float x = float(2.0 * (cyc - floor(cyc))) + float(A.phase[a] * 0.3183098861837907);
      if (!deriv) {
        v[a] = float(A.amp[a]) * cospif(x);
      } else {
        v[a] = -float(A.amp[a] * 2.0 * kPi * A.freq[a]) * sinpif(x);
      }
    }
    bx = v[0]; by = v[1]; bz = v[2];
  };
  auto mult_lane = [&](double tt) -> float {
    float bx, by, bz;
    field(tt, bx, by, bz, false);
    bx += off[0]; by += off[1]; bz += off[2];
    const float hx = R[0] * bx + R[3] * by + R[6] * bz;
    const float hy = R[1] * bx + R[4] * by + R[7] * bz;
    const float hz = R[2] * bx + R[5] * by + R[8] * bz;
    return kind_mult(lane < 9 ? lane : 0, inv2tau, sigma, alpha, beta, hx, hy, hz);
  };
  // FP64 multiplier of kind `lane` (lanes 0..8) at time tt (field value or its time derivative)
  auto mult_lane_d = [&](double tt, bool deriv) -> double {
    return kind_mult_d(lane < 9 ? lane : 0, A.ip[inst], A.amp, A.freq, A.phase, tt, deriv);
  };
  // dst[p] = add * dst[p] + (A(msd) (xin + xlo))[p] for the rows p = lane + 64 s, in FP64: every
  // entry as hi + lo, the FP64 kind multipliers, the two-part stage argument.  The right-hand side of a
  // nearly relaxed stiff particle is a small difference of large terms; FP32 rounding of the terms,
  // the multipliers or the sums biases its slow relaxation (a resolved L = 17 particle's moment moved by
  // 1e-5 independently of the step size), FP64 leaves only the final rounding of the small result.
  auto matvec = [&](float* dst, bool add) {
    const float* xin = w.xin();
    const float* xl = w.xlo;
    double m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = w.msd[k];
#pragma unroll 1
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      const float* ev = opaque_ptr(eval);
      const float* el = opaque_ptr(elo);
      const uint16_t* ec = opaque_ptr(ecol);
      if (p < Np) {
        // table reads, then gathers, then the sums, one slot group at a time (one wait per phase)
        double acc = 0.0;
        constexpr int kG = 7;
        static_assert(kNSlRow % kG == 0, "row slots come in whole groups");
#pragma unroll
        for (int g0 = 0; g0 < kNSlRow; g0 += kG) {
          int ci[kG];
          float hv[kG], lv[kG], xh[kG], xo[kG];
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            ci[u] = ec[(g0 + u) * Np + p];
            hv[u] = ev[(g0 + u) * Np + p];
            lv[u] = el[(g0 + u) * Np + p];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            xh[u] = xin[ci[u]];
            xo[u] = xl[ci[u]];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u)
            acc = fma(m[kSlotKindRow[g0 + u]] * (double(hv[u]) + double(lv[u])), double(xh[u]) + double(xo[u]), acc);
        }
        dst[p] = add ? float(double(dst[p]) + acc) : float(acc);
      }
    }
  };
  // x = M^{-1} V with the stored block inverses; result in G
  // Block solves read the inverses from the workspace.  The column quads of the next block are
  // requested before the current block's right-hand side is formed (two alternating register
  // buffers), so the memory latency overlaps the LDS work of the current block.
  constexpr int kNQ = WG::q4(0) > WG::q4(1) ? WG::q4(0) : WG::q4(1);  // largest quad count of a block
  auto load_quads = [&](auto KK, float4 (&cq)[kNQ]) {
    constexpr int K = decltype(KK)::value;
    constexpr int n = Gm::nb(K), nq = WG::q4(K);
    const float4* iv = reinterpret_cast<const float4*>(opaque_ptr(inv) + WG::ioff(K));
    if (lane < n) {
#pragma unroll
      for (int q = 0; q < nq; ++q) cq[q] = iv[q * n + lane];
    }
  };
  auto block_apply = [&](auto KK, float* G, bool subtract, const float4 (&cq)[kNQ]) {
    constexpr int K = decltype(KK)::value;
    constexpr int n = Gm::nb(K), off0 = Gm::off(K), nq = WG::q4(K);
    if (lane < n) {
      // four independent partial sums (one per quad component), not one dependent chain
      float px = 0.0f, py = 0.0f, pz = 0.0f, pw = 0.0f;
#pragma unroll
      for (int q = 0; q < nq; ++q) {
        const float4 c = cq[q];
        const float4 tv = *reinterpret_cast<const float4*>(&w.T[4 * q]);
        px = fmaf(c.x, tv.x, px);
        py = fmaf(c.y, tv.y, py);
        pz = fmaf(c.z, tv.z, pz);
        pw = fmaf(c.w, tv.w, pw);
      }
      const float part = (px + py) + (pz + pw);
      if (subtract) G[off0 + lane] -= part;
      else G[off0 + lane] = part;
    }
    wsync();
  };
  auto solve = [&]() {
    float* V = w.V();
    float* G = w.G();
    float mk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) mk[k] = w.mk[k];
    const float mFX = mk[5], mFY = mk[6], mRX = mk[7], mRY = mk[8];
    float4 qa[kNQ], qb[kNQ];
    load_quads(std::integral_constant<int, 0>{}, qa);
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), off0 = Gm::off(K);
      if constexpr (K + 1 <= L) load_quads(std::integral_constant<int, K + 1>{}, (K % 2 == 0) ? qb : qa);
      const float* ev = opaque_ptr(eval);
      const uint16_t* ec = opaque_ptr(ecol);
      const float* wb = opaque_ptr(wB);
      if (lane < n) {
        const int row = off0 + lane;
        float tv = V[row];
        // (loads first, then the sums: one wait per phase instead of one per coupling)
        if constexpr (K == 1) {
          int ci[kNSlB];
          float cv[kNSlB], gv[kNSlB];
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) {
            ci[u] = ec[(kSlB + u) * Np + row];
            cv[u] = ev[(kSlB + u) * Np + row];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) gv[u] = G[ci[u]];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) tv = fmaf(-mk[kSlotKindRow[kSlB + u]] * cv[u], gv[u], tv);
        } else if constexpr (K >= 2) {
          constexpr int offp = Gm::off(K - 1);
          const int tt = lane & 1;
          const float* gs = G + offp + lane;
          const float* go = G + offp + lane + 1 - 2 * tt;
          float wv[6], gsv[3], gov[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            wv[d] = wb[d * Np + row];
            wv[3 + d] = wb[(3 + d) * Np + row];
            gsv[d] = gs[2 * d];
            gov[d] = go[2 * d];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            tv = fmaf(-(d == 1 ? mRY : mFX) * wv[d], gsv[d], tv);
            tv = fmaf(-(d == 1 ? mRX : mFY) * wv[3 + d], gov[d], tv);
          }
        }
        w.T[lane] = tv;
      }
      wsync();
      block_apply(KK, G, false, (K % 2 == 0) ? qa : qb);
      __builtin_amdgcn_sched_barrier(0);
    });
    load_quads(std::integral_constant<int, L - 1>{}, ((L - 1) % 2 == 0) ? qa : qb);
    static_for_down<L - 1, 0>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), off0 = Gm::off(K);
      if constexpr (K >= 1) load_quads(std::integral_constant<int, K - 1>{}, (K % 2 == 0) ? qb : qa);
      const float* wc = opaque_ptr(wC);
      if (lane < n) {
        const int row = off0 + lane;
        float tv = 0.0f;
        constexpr int offn = Gm::off(K + 1);
        const int tt = (K > 0) ? (lane & 1) : 0;
        const float* gs = G + offn + ((K > 0) ? lane - 4 : 2 * lane - 4);
        const float* go = G + offn + ((K > 0) ? lane - 3 - 2 * tt : 2 * lane - 3);
        float wv[6], gsv[3], gov[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          wv[d] = wc[d * Np + row];
          wv[3 + d] = wc[(3 + d) * Np + row];
          gsv[d] = gs[2 * d];
          gov[d] = go[2 * d];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          tv = fmaf((d == 1 ? mRY : mFX) * wv[d], gsv[d], tv);
          tv = fmaf((d == 1 ? mRX : mFY) * wv[3 + d], gov[d], tv);
        }
        w.T[lane] = tv;
      }
      wsync();
      block_apply(KK, G, true, (K % 2 == 0) ? qa : qb);
      __builtin_amdgcn_sched_barrier(0);
    });
  };
  // factor M = I - h g A(t_n) (multipliers in w.mk): Schur-complement inverses into the workspace.
  // X holds the previous block's inverse (rows) on entry to each block.
  auto factor = [&]() {
    float* X = w.X();
    float mk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) mk[k] = w.mk[k];
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), off0 = Gm::off(K);
      const bool act = lane < n;
      constexpr int np = (K > 0) ? Gm::nb(K > 0 ? K - 1 : 0) : 1;
      float u[np];  // U = B_K Sinv_{K-1}, row `lane`
#pragma unroll
      for (int q = 0; q < np; ++q) u[q] = 0.0f;
      if constexpr (K > 0) {
        constexpr int offp = Gm::off(K - 1);
        if (act) {
          const int row = off0 + lane;
          if constexpr (K == 1) {
            const float* ev = opaque_ptr(eval);
            const uint16_t* ec = opaque_ptr(ecol);
            int ci[kNSlB];
            float cv[kNSlB];
#pragma unroll
            for (int u2 = 0; u2 < kNSlB; ++u2) {
              ci[u2] = ec[(kSlB + u2) * Np + row];
              cv[u2] = ev[(kSlB + u2) * Np + row];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int sl = kSlB; sl < kSlB + kNSlB; ++sl) {
              const float me = mk[kSlotKindRow[sl]] * cv[sl - kSlB];
              const float* xr = X + (ci[sl - kSlB] - offp) * XS;
#pragma unroll
              for (int q = 0; q < np; ++q) {
                u[q] = fmaf(me, xr[q], u[q]);
                if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          } else {
            const int tt = lane & 1;
            const float* xs = X + lane * XS;                // rows lane + 2d
            const float* xo = X + (lane + 1 - 2 * tt) * XS;  // rows lane + 1 - 2t + 2d
            const float* wb = opaque_ptr(wB);
            float wv[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) wv[d] = wb[d * Np + row];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float ms_ = (d == 1 ? mk[8] : mk[5]) * wv[d];
              const float mo_ = (d == 1 ? mk[7] : mk[6]) * wv[3 + d];
#pragma unroll
              for (int q = 0; q < np; ++q) {
                u[q] = fmaf(mo_, xo[2 * d * XS + q], fmaf(ms_, xs[2 * d * XS + q], u[q]));
                if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
      wsync();
      // S_K = I + (-h g) D_K assembled in X
      if (act) {
#pragma unroll
        for (int q = 0; q < n; ++q) X[lane * XS + q] = 0.0f;
      }
      wsync();
      if (act) {
        const int row = off0 + lane;
        const float* ev = opaque_ptr(eval);
        const uint16_t* ec = opaque_ptr(ecol);
        // table reads first, then LDS atomic adds (several slots can share a column)
        int cl[kNSlD];
        float cv[kNSlD];
#pragma unroll
        for (int u2 = 0; u2 < kNSlD; ++u2) {
          cl[u2] = int(ec[(kSlD + u2) * Np + row]) - off0;
          cv[u2] = ev[(kSlD + u2) * Np + row];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u2 = 0; u2 < kNSlD; ++u2)
          __hip_atomic_fetch_add(X + lane * XS + cl[u2], mk[kSlotKindRow[kSlD + u2]] * cv[u2], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
        __hip_atomic_fetch_add(X + lane * XS + lane, 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
      wsync();
      if constexpr (K >= 1) {
        // stage the coefficients of C_{K-1} (with the kind multipliers) for broadcast reads:
        // K = 1: by row j of block 0 (window of row j); K >= 2: by column c of block K (S window)
        constexpr int nc = (K == 1) ? np : n;
        constexpr int base = (K == 1) ? 0 : off0;
        const float* wt = opaque_ptr((K == 1) ? wC : wS);
        if (lane < nc) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            w.cw[d][lane] = (d == 1 ? mk[8] : mk[5]) * wt[d * Np + base + lane];
            w.cw[3 + d][lane] = (d == 1 ? mk[7] : mk[6]) * wt[(3 + d) * Np + base + lane];
          }
        }
        wsync();
      }
      if constexpr (K == 1) {
        // S_1 -= U C_0 by rows j of block 0 (cos type): C_0 row j reaches block-1 columns
        // 2j - 4 + 2d (same window) and 2j - 3 + 2d (other window)
        if (act) {
          float* xr = X + lane * XS;
#pragma unroll
          for (int c = 0; c < n; ++c) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < np; ++j) {
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                if (2 * j - 4 + 2 * d == c) acc = fmaf(u[j], w.cw[d][j], acc);
                if (2 * j - 3 + 2 * d == c) acc = fmaf(u[j], w.cw[3 + d][j], acc);
              }
            }
            xr[c] -= acc;
            if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else if constexpr (K >= 2) {
        // S_K -= U C_{K-1}: column c takes U[c + 2d] (same type) and U[c + 1 - 2 t_c + 2d] (other type)
        if (act) {
          float* xr = X + lane * XS;
#pragma unroll
          for (int c = 0; c < n; ++c) {
            float acc = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const int js = c + 2 * d, jo = c + 1 - 2 * (c & 1) + 2 * d;
              if (js < np) acc = fmaf(w.cw[d][c], u[js], acc);
              if (jo < np) acc = fmaf(w.cw[3 + d][c], u[jo], acc);
            }
            xr[c] -= acc;
            if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      wsync();
      float a[n];
#pragma unroll
      for (int q = 0; q < n; ++q) a[q] = act ? X[lane * XS + q] : 0.0f;
      ok = gj_piv_invert_wide<n, XS, K == 0>(a, lane, w, X) && ok;
      // inverse -> workspace (column quads) and -> X rows for the next block's U
      if (act) {
        float4* iv = reinterpret_cast<float4*>(opaque_ptr(inv) + WG::ioff(K));
#pragma unroll
        for (int q = 0; q < WG::q4(K); ++q) {
          float4 v;
          v.x = (4 * q + 0 < n) ? a[(4 * q + 0) < n ? 4 * q + 0 : 0] : 0.0f;
          v.y = (4 * q + 1 < n) ? a[(4 * q + 1) < n ? 4 * q + 1 : 0] : 0.0f;
          v.z = (4 * q + 2 < n) ? a[(4 * q + 2) < n ? 4 * q + 2 : 0] : 0.0f;
          v.w = (4 * q + 3 < n) ? a[(4 * q + 3) < n ? 4 * q + 3 : 0] : 0.0f;
          iv[q * n + lane] = v;
        }
#pragma unroll
        for (int q = 0; q < n; ++q) X[lane * XS + q] = a[q];
      }
      wsync();
      __builtin_amdgcn_sched_barrier(0);
    });
  };

  float* Kv = Kg;                // K1..K5 at j * NpA
  float* ft = Kg + 5 * NpA;
  auto rodas_step = [&](double tn, double hs) -> float {
    const float hf = float(hs);
    const float hg = hf * 0.25f;
    const float ih = 1.0f / hf;
    {
      // both multiplier sets of t_n before the factorisation (their shared sin/cos work is not kept
      // live across it): M's in mk, the time derivatives for f_t in ms
      const float mt = mult_lane(tn);
      const double md = mult_lane_d(tn, true);
      if (lane < 9) {
        w.mk[lane] = -hg * mt;
        w.msd[lane] = md;
      }
      wsync();
    }
    factor();
    {  // f_t = A'(t_n) y
      float* xin = w.xin();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        if (p < Np) {
          xin[p] = y[s];
          w.xlo[p] = ylo[s];
        }
      }
      wsync();
      matvec(ft, false);
      wsync();
    }
    for (int stg = 0; stg < 6; ++stg) {
      const double mt = mult_lane_d(tn + double(kRodasAlpha[stg]) * hs, false);
      if (lane < 9) w.msd[lane] = mt;
      // stage argument -> xin, extra right-hand-side terms -> V
      float* xin = w.xin();
      float* V = w.V();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        if (p < Np) {
          // stage increment sum_j a_ij K_j added to the two-part state: xin + xlo = y + ylo + increment
          float u = ylo[s];
          float ev = hf * kRodasGamma[stg] * ft[p];
          for (int j = 0; j < stg; ++j) {
            const float kj = Kv[j * NpA + p];
            u = fmaf(kRodasA[stg][j], kj, u);
            ev = fmaf(kRodasC[stg][j] * ih, kj, ev);
          }
          float hi, lo;
          two_sum(y[s], u, hi, lo);
          xin[p] = hi;
          w.xlo[p] = lo;
          V[p] = ev;
        }
      }
      wsync();
      matvec(V, true);
      wsync();
      solve();
      if (stg < 5) {
        const float* G = w.G();
        float* kd = Kv + stg * NpA;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int p = lane + 64 * s;
          if (p < Np) kd[p] = hg * G[p];
        }
      }
      wsync();
    }
    // y_{n+1} = (stage-6 argument) + K6 ; embedded error K6
    // embedded error estimate max |K6|; the candidate (stage-6 argument in xin) + K6 stays in LDS until
    // the step is accepted
    float emax = 0.0f;
    {
      const float* G = w.G();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        emax = fmaxf(emax, (p < Np) ? err_abs(hg * G[p]) : 0.0f);
      }
    }
    return wave_max(emax);
  };
  // y + ylo <- y_{n+1} = (stage-6 argument) + K6 of the step just taken
  auto accept = [&](float hg) {
    const float* xin = w.xin();
    const float* G = w.G();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      float hi = 0.0f, lo = 0.0f;
      if (p < Np) two_sum(xin[p], w.xlo[p] + hg * G[p], hi, lo);
      y[s] = hi;
      ylo[s] = lo;
    }
  };

  const double dt = A.period / A.Ns;
  const int n_int = (A.settle + 1) * A.Ns;
  const int first_rec = A.settle * A.Ns;
  // The controller's FP64 scalars live in LDS across a step (re-read after it).
  if (lane == 0) {
    w.ctl[1] = dt;  // step size, kept across sample intervals
    w.ctl[4] = 0.0;
  }
  int steps = 0;
  const float c00_0 = __shfl(y[0], 0);  // c_00 = 1 / sqrt(4 pi): total probability
  bool unres = false;   // |m| > 1 + 1e-3 or c_00 changed at a sample
  bool forced = false;  // a step accepted at the smallest step size with its estimate above tol
  // a probability density has |m| <= 1 and keeps c_00 (conserved exactly by the solves); a state that
  // breaks either is not resolved by the degree (status FPN_INST_UNRESOLVED, the instance stops)
  auto state_ok = [&](float vx, float vy, float vz) -> bool {
    const bool fin = isfinite(vx) && isfinite(vy) && isfinite(vz);
    const bool phys = (rc * rc) * (vx * vx + vy * vy + vz * vz) <= kMaxM2 && __shfl(y[0], 0) == c00_0;
    if (fin && !phys) unres = true;
    return fin && phys;
  };
  for (int j = 0; j < n_int && ok; ++j) {
    const double tj = j * dt;
    const float vx = __shfl(y[pX >> 6], pX & 63), vy = __shfl(y[pY >> 6], pY & 63),
                vz = __shfl(y[pZ >> 6], pZ & 63);
    if (!state_ok(vx, vy, vz)) {
      ok = false;
      break;
    }
    if (j >= first_rec) {
      const int js = j - first_rec;
      if (lane < 3) {
        const float r0 = lane == 0 ? R[0] : (lane == 1 ? R[3] : R[6]);
        const float r1 = lane == 0 ? R[1] : (lane == 1 ? R[4] : R[7]);
        const float r2 = lane == 0 ? R[2] : (lane == 1 ? R[5] : R[8]);
        ms_out[lane * A.Ns + js] = rc * (r0 * vx + r1 * vy + r2 * vz);
      }
      if (dd_out) {
        // dm/dt at the sample: rows l = 1 of A(t_j) y (the ODE's right-hand side), rotated like m
        const float mt = mult_lane(tj);
        if (lane < 9) w.ms[lane] = mt;
        float* xs = w.xin();
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int p = lane + 64 * s;
          if (p < Np) xs[p] = y[s];
        }
        wsync();
        float acc = 0.0f;
        if (lane < 3) {
          const int row = lane == 0 ? pX : (lane == 1 ? pY : pZ);  // rows < 64
          for (int g = 0; g < kNSlRow; ++g)
          {
            const float x = xs[ecol[g * Np + row]], mk = w.ms[kSlotKindRow[g]];
            acc = fmaf(mk * eval[g * Np + row], x, acc);
            acc = fmaf(mk * elo[g * Np + row], x, acc);
          }
        }
        const float ax = __shfl(acc, 0), ay = __shfl(acc, 1), az = __shfl(acc, 2);
        if (lane < 3) {
          const float r0 = lane == 0 ? R[0] : (lane == 1 ? R[3] : R[6]);
          const float r1 = lane == 0 ? R[1] : (lane == 1 ? R[4] : R[7]);
          const float r2 = lane == 0 ? R[2] : (lane == 1 ? R[5] : R[8]);
          dd_out[lane * A.Ns + js] = rc * (r0 * ax + r1 * ay + r2 * az);
        }
        wsync();
      }
    }
    // fixed: r_fixed equal steps per sample interval.  adaptive: steps of any size up to the sample
    // spacing, each accepted (max |K6| <= tol) or redone on its own.  The last step of an interval
    // lands on the next sample time.  (One call site of the stage routine keeps it inlined.)
    // Adaptive settling (span): the settling periods are one interval, stepped with up to kSettleSpan
    // sample spacings per step, the last step landing on the first recorded sample time; the state
    // checks then follow every accepted step (as in stepper.hip).
    const bool fixedr = A.r_fixed > 0;
    const bool span = !fixedr && j < first_rec;
    if (lane == 0) w.ctl[0] = tj;
    wsync();
    for (;;) {
      const double dtv = A.period / A.Ns;
      const double tend = double(span ? A.settle * A.Ns : j + 1) * dtv;
      const double t = w.ctl[0];
      if (!(t < tend - 1e-9 * dtv)) break;
      double hs = fixedr ? dtv / A.r_fixed : w.ctl[1];
      bool landed = false;
      if (hs >= (tend - t) * (fixedr ? 0.75 : 0.95)) {
        hs = tend - t;
        landed = true;
      }
      if (lane == 0) {
        w.ctl[2] = hs;
        w.ctl[3] = landed ? 1.0 : 0.0;
      }
      const float e = rodas_step(t, hs);
      ++steps;
      const double dt2 = A.period / A.Ns;
      const double hmin = dt2 / (A.r_max > 0 ? A.r_max : 64);
      const double t2 = w.ctl[0], hst = w.ctl[1], hs2 = w.ctl[2];
      const bool landed2 = w.ctl[3] != 0.0, after_reject = w.ctl[4] != 0.0;
      const double tend2 = double(span ? A.settle * A.Ns : j + 1) * dt2;
      // e = +inf for a non-finite attempt (an overflow of the FP32 factorisation, which a long step can
      // cause): rejected like any other (5x shorter, on cleared scratch) unless it is the smallest step
      if (!isfinite(e) && (fixedr || hs2 <= hmin * 1.06)) {
        ok = false;
        break;
      }
      const float fac = 0.9f * sqrtf(sqrtf(A.tol / fmaxf(e, 1e-30f)));
      // reject this step only (y is unchanged).  A step no longer than hmin / 0.95 is always accepted:
      // the landing rule could stretch its retry back to the same length.
      if (!fixedr && e > A.tol && hs2 > hmin * 1.06) {
        if (!isfinite(e) || !ok) {
          clear_wave_scratch(w, lane);
          ok = true;
        }
        if (lane == 0) {
          w.ctl[1] = fmax(hmin, hs2 * double(fmaxf(0.2f, fac)));
          w.ctl[4] = 1.0;
        }
        wsync();
        continue;
      }
      if (!fixedr && e > A.tol) forced = true;
      accept(float(hs2) * 0.25f);
      // no growth right after a rejected attempt (avoids grow / reject cycles)
      const double hn = hs2 * double(fminf(after_reject ? 1.0f : 4.0f, fmaxf(0.2f, fac)));
      if (lane == 0) {
        w.ctl[0] = landed2 ? tend2 : t2 + hs2;
        w.ctl[1] = fmin(span ? kSettleSpan * dt2 : dt2, fmax(hmin, landed2 ? fmax(hn, hst) : hn));
        w.ctl[4] = 0.0;
      }
      wsync();
      if (span) {
        const float ux = __shfl(y[pX >> 6], pX & 63), uy = __shfl(y[pY >> 6], pY & 63),
                    uz = __shfl(y[pZ >> 6], pZ & 63);
        if (!state_ok(ux, uy, uz)) {
          ok = false;
          break;
        }
      }
    }
    if (span) j = first_rec - 1;  // continue at the first recorded sample
  }
  if (!ok) {
    for (int j = lane; j < 3 * A.Ns; j += 64) ms_out[j] = __builtin_nanf("");
    if (dd_out)
      for (int j = lane; j < 3 * A.Ns; j += 64) dd_out[j] = __builtin_nanf("");
    if (lane == 0) A.status[inst] = unres ? kInstUnresolved : kInstNonfinite;
  } else if (forced) {
    if (lane == 0) A.status[inst] = kInstTolUnmet;
  }
  if (A.steps_out && lane == 0) A.steps_out[inst] = steps;
  }  // queue
}

#ifndef FPN_WIDE_WAVES
#define FPN_WIDE_WAVES 4
#endif
constexpr int kWideWaves = FPN_WIDE_WAVES;

template <int L>
int64_t stepper_wide_ws_floats_L() {
  return WGeo<L>::WS;
}

template <int L, int WV>
constexpr size_t wide_lds_bytes() {
  return WV == 1 ? wide_lds_scratch_bytes<L, 1>() + size_t(WGeo<L>::WS) * sizeof(float) : WV * sizeof(WideLds<L>);
}

template <int L>
hipError_t launch_stepper_wide_L(const StepLaunch& s, const DevTables& t, float* ws, hipStream_t stream) {
  StepArgs a;
  a.ip = s.ip;
  a.inst_idx = s.inst_idx;
  a.n_inst = s.n_inst;
  a.c0 = s.c0;
  a.c_stride = s.c_stride;
  for (int c = 0; c < 3; ++c) {
    a.amp[c] = s.amp[c];
    a.freq[c] = s.freq[c];
    a.phase[c] = s.phase[c];
  }
  a.period = s.period;
  a.settle = s.settle;
  a.Ns = s.Ns;
  a.r_fixed = s.r_fixed;
  a.r_max = s.r_max;
  a.tol = s.tol;
  a.msamp = s.msamp;
  a.dmdt = s.dmdt;
  a.status = s.status;
  a.steps_out = s.steps_out;
  a.queue = s.queue;
  a.c0t = nullptr;  // tangents are carried by the register-layout stepper only
  a.mtan = nullptr;
  a.tws = nullptr;
  auto go = [&](auto WVC) -> hipError_t {
    constexpr int WV = decltype(WVC)::value;
    constexpr size_t shm = wide_lds_bytes<L, WV>();
    static_assert(shm <= 160 * 1024, "wide stepper LDS exceeds a compute unit");
    auto kern = stepper_wide_kernel<L, WV>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
    if (e != hipSuccess) return e;
    int grid = (s.n_inst + WV - 1) / WV;
    if (s.grid > 0) grid = std::min(grid, s.grid);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WV), shm, stream, a, t, ws);
    return hipGetLastError();
  };
  if (s.waves == 1) return go(std::integral_constant<int, 1>{});
  if (s.waves != 0 && s.waves != kWideWaves) return hipErrorInvalidValue;
  return go(std::integral_constant<int, kWideWaves>{});
}

template <int L>
hipError_t stepper_wide_occupancy_L(int waves, int* waves_per_block, int* blocks_per_cu) {
  auto occ = [&](auto WVC) -> hipError_t {
    constexpr int WV = decltype(WVC)::value;
    constexpr size_t shm = wide_lds_bytes<L, WV>();
    auto kern = stepper_wide_kernel<L, WV>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
    if (e != hipSuccess) return e;
    *waves_per_block = WV;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, 64 * WV, shm);
  };
  if (waves == 1) return occ(std::integral_constant<int, 1>{});
  if (waves != 0 && waves != kWideWaves) return hipErrorInvalidValue;
  return occ(std::integral_constant<int, kWideWaves>{});
}

#define FPN_WINST(LL)                                                                                  \
  template hipError_t launch_stepper_wide_L<LL>(const StepLaunch&, const DevTables&, float*, hipStream_t); \
  template int64_t stepper_wide_ws_floats_L<LL>();                                                     \
  template hipError_t stepper_wide_occupancy_L<LL>(int, int*, int*);
#if !defined(FPN_L_BEGIN)
#define FPN_L_BEGIN 17
#define FPN_L_END 24
#endif
#if FPN_L_BEGIN <= 17 && 17 <= FPN_L_END
FPN_WINST(17)
#endif
#if FPN_L_BEGIN <= 18 && 18 <= FPN_L_END
FPN_WINST(18)
#endif
#if FPN_L_BEGIN <= 19 && 19 <= FPN_L_END
FPN_WINST(19)
#endif
#if FPN_L_BEGIN <= 20 && 20 <= FPN_L_END
FPN_WINST(20)
#endif
#if FPN_L_BEGIN <= 21 && 21 <= FPN_L_END
FPN_WINST(21)
#endif
#if FPN_L_BEGIN <= 22 && 22 <= FPN_L_END
FPN_WINST(22)
#endif
#if FPN_L_BEGIN <= 23 && 23 <= FPN_L_END
FPN_WINST(23)
#endif
#if FPN_L_BEGIN <= 24 && 24 <= FPN_L_END
FPN_WINST(24)
#endif

}  // namespace fpn
