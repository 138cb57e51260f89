// FP32 time stepper (rows a4/a5): one wavefront per instance, linearly implicit
// L-stable RODAS4 with per-step error control.
//
// The Galerkin ODE dc/dt = A(t) c (paper: Eq. FP-general with the drift of
// Eq. convection, easy-axis frame) is integrated over (settle + 1) drive periods.
// Every step factors M = I - h g A(t_n) by block elimination over the |m| blocks
// (block-tridiagonal ordering): the Schur complement of each block is inverted by
// Gauss-Jordan with partial pivoting, and the inverses stay in VGPRs for the six
// stage solves.  Moments are sampled at t_j (Eq. mean_magmom_FP).
//
// Lane layout of a block (n <= 32 rows): lane = 32 h + i holds row i, columns
// h, h + 2, h + 4, ... (a[q] = S[i][h + 2q]).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_common.hpp"
#include "device_util.hpp"
#include "kernels.hpp"
#include "physics.hpp"
#include "stepper_common.hpp"

namespace fpn {

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

// Per-wavefront LDS, sized by the degree.  The factorisation scratch (X, Ub) and the stage vectors
// share `u`.  A scratch row holds the two column parities of a block row side by side, kH slots each
// (kH = the longest half row of any block), with a row stride kXS = 2 kH + 1 (odd, so the rows of a
// half-wave fall in different LDS banks).  X has 2 kH + 5 rows (window reads overhang a block by up
// to five rows), Ub 2 kH rows.  With tangents (NT > 0) three more vectors hold the step-start state,
// the tangent stage argument and the current primal stage increment, and three multiplier tables
// hold the parameter derivatives.
template <int L, int NT>
struct WaveLds {
  static constexpr int NpA = Geo<L>::NpA;
  static constexpr int kH = Geo<L>::qmax;
  static constexpr int kXS = 2 * kH + 1;
  static constexpr int kUbOff = (2 * kH + 5) * kXS;
  static constexpr int kFac = kUbOff + 2 * kH * kXS;
  // every lane reads a scratch row i < 32 (masked when i is past the block): keep 32 rows in bounds
  static constexpr int kUnion0 = (kFac > 9 * NpA) ? kFac : 9 * NpA;
  static constexpr int kUnion = (kUnion0 > 32 * kXS) ? kUnion0 : 32 * kXS;
  static constexpr int kTanV = NT > 0 ? 3 * NpA : 4;
  float u[kUnion];
  float T[2 * kH];     // block right-hand side [parity][kH]
  int pv[64];          // pivot row of every column, [parity][kH]
  float row[4 * kH];   // pivot row [parity][kH]
  float mk[16];        // -h g * multiplier(t_n) per kind
  float ms[16];        // multiplier at the current stage time per kind
  float tv[kTanV];                     // y0 | xt | kc
  float dmi[NT > 0 ? NT : 1][12];      // d multiplier / d p at the stage time
  float dmn[NT > 0 ? NT : 1][12];      // ... at t_n
  float ddm[NT > 0 ? NT : 1][12];      // d (time derivative of the multiplier) / d p at t_n
  double ctl[6];                       // step controller: time, next step size, this step size, landed,
                                       // last attempt rejected, steps taken (accepted and rejected)
  __device__ float* X() { return u; }
  __device__ float* Ub() { return u + kUbOff; }
  __device__ float* xin() { return u; }
  __device__ float* V() { return u + NpA; }
  __device__ float* G() { return u + 2 * NpA; }
  __device__ float* Kv(int j) { return u + (3 + j) * NpA; }  // K1..K5
  __device__ float* ft() { return u + 8 * NpA; }
  __device__ float* y0() { return tv; }
  __device__ float* xt() { return tv + NpA; }
  __device__ float* kc() { return tv + 2 * NpA; }
};

// In-place inverse of the lane-distributed block by Gauss-Jordan with partial pivoting (single
// rows).  Column c = 2 qq + hc is held by the lanes of parity hc; the remaining row with the largest
// |S[i][c]| becomes its pivot.  The slots rotate by one after every column pair, so the pivot column
// is always slot 0 and all register indexing is static; after Q pairs the slots are back in order.
// The tableau then holds the inverse with rows and columns permuted (row i of the tableau belongs to
// the column it pivoted, column c to the row that pivoted it); the LDS scratch X (row stride kXS, one
// half of kH slots per parity) puts it back in order.  kRow0 (block 0): row 0 is e_0 (the probability
// row of M = I - h g A, A having a zero row 0) and pivots column 0, so it stays e_0 and the total
// probability c_00 is conserved exactly by every solve.
// Pivot rows are not divided by their pivot P when they pivot: a row is kept as P times the
// normalised tableau row (its pivot-column entry 1 instead of 1/P) and scaled by 1/P once at the end.
// Every later update of a row is linear in it, so the stored row stays P times the true one, and a
// row is broadcast only at its own pivot step, before any scaling, so the broadcast rows are the ones
// the plain algorithm uses.  This saves a multiply per entry and column.
template <int Q, bool kRow0, typename W>
__device__ __forceinline__ bool gj_piv_invert(float (&a)[Q], int i, int h, W& w, float* X) {
  constexpr int n = 2 * Q;
  constexpr int kH = W::kH;
  constexpr int kXS = 2 * kH + 1;
  const bool act = i < n;
  bool ok = true;
  bool cand = act;  // row not yet a pivot
  int mycol = 0;    // column this row pivoted
  float myip = 1.0f;  // 1 / pivot of this row: the row's deferred scale
  int* pv = w.pv;  // pivot row of column c at [(c & 1) kH + (c >> 1)]
#pragma unroll 1
  for (int qq = 0; qq < Q; ++qq) {
#pragma unroll
    for (int hc = 0; hc < 2; ++hc) {
      // the column's entry of this lane's row: own slot 0 (parity hc) or the partner lane's
      const float own = a[0];
      auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(own), __float_as_uint(own), false, false);
      const float g = (h == hc) ? own : __uint_as_float(h == 0 ? sw[1] : sw[0]);
      const uint32_t best = max32_uniform(pivot_key<5>(g, i, cand));
      const int p = (kRow0 && hc == 0 && qq == 0) ? 0 : int(best & 31u);
      const float P = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g), p));
      ok = ok && (P != 0.0f) && isfinite(P);
      const float ip = __builtin_amdgcn_rcpf(P);  // hardware reciprocal (1 ulp)
      const bool isp = (i == p);
      if (isp) {
#pragma unroll
        for (int q = 0; q < Q; ++q) w.row[h * kH + q] = a[q];
      }
      if (i == 0 && h == 0) pv[hc * kH + qq] = p;
      wsync();
      float rv[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) rv[q] = w.row[h * kH + q];
      __builtin_amdgcn_sched_barrier(0);
      // pivot row: unchanged (deferred scale 1 / P, pivot-column entry P / P = 1); other rows:
      // row - g / P * pivot row, pivot-column entry -g / P
      const float G = isp ? 0.0f : g * ip;
      const float pc = act ? (isp ? 1.0f : -G) : 0.0f;
      if (hc == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) a[q] = fmaf(-G, rv[q], a[q]);
        if (h == 0) a[0] = pc;
      } else {
        const float a0 = fmaf(-G, rv[0], a[0]);
#pragma unroll
        for (int q = 1; q < Q; ++q) a[q - 1] = fmaf(-G, rv[q], a[q]);
        a[Q - 1] = (h == 1) ? pc : a0;
      }
      if (isp) {
        cand = false;
        mycol = 2 * qq + hc;
        myip = ip;
      }
      wsync();
    }
  }
  // tableau entry (i, j) -> inverse entry (mycol, pivot row of column j)
  int pj[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) pj[q] = pv[h * kH + q];
  __builtin_amdgcn_sched_barrier(0);
  if (act) {
#pragma unroll
    for (int q = 0; q < Q; ++q) X[mycol * kXS + (pj[q] & 1) * kH + (pj[q] >> 1)] = a[q] * myip;
  }
  wsync();
#pragma unroll
  for (int q = 0; q < Q; ++q) a[q] = act ? X[i * kXS + h * kH + q] : 0.0f;
  wsync();
  return ok;
}

// Row i of a block inverse (this lane's half a[0..Q-1]) times the half vector t[0..Q-1], summed over
// both halves: four independent partial sums, so the products do not form one dependent chain.
template <int Q>
__device__ __forceinline__ float dot_half(const float (&a)[Q], const float* t) {
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q & 3] = fmaf(a[q], t[q], acc[q & 3]);
  return half_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

template <int L, int WAVES, int NT>
__global__ void __launch_bounds__(64 * WAVES)
stepper_kernel(StepArgs A, DevTables t) {
  using Gm = Geo<L>;
  using WL = WaveLds<L, NT>;
  constexpr int kH = WL::kH;    // half-row slots of the factorisation scratch
  constexpr int kXS = WL::kXS;  // its row stride
  constexpr int NpA = Gm::NpA;
  constexpr int Np = Gm::Np;
  constexpr int S = Gm::S;
  extern __shared__ __align__(16) unsigned char smem[];
  // fixed-slot operator tables: indices (u16) then values (f32), slot-major; the diagonal-block slots
  // also carry the low-order part of their value (elo).  The column slots of the block-1 coupling are
  // read from global memory (once per step).
  uint16_t* ecol = reinterpret_cast<uint16_t*>(smem);          // [kNSlRow][Np]
  constexpr size_t b16 = ((size_t(kNSlRow) * Np * 2) + 15) & ~size_t(15);
  float* eval = reinterpret_cast<float*>(smem + b16);          // [kNSlRow][Np]
  float* elo = eval + kNSlRow * Np;                            // [kNSlD][Np]
  float* wB = elo + kNSlD * Np;                                // [kNWin][Np] window coefficients
  float* wC = wB + kNWin * Np;
  float* wS = wC + kNWin * Np;
  constexpr size_t tb = (b16 + size_t(kNSlRow + kNSlD + 3 * kNWin) * Np * 4 + 15) & ~size_t(15);
  WL* wl = reinterpret_cast<WL*>(smem + tb);
  const uint16_t* crow = t.ecol_row;                           // [kNSlCol][Np] (global)
  const float* cvl = t.ecol_val;                               // [kNSlCol][Np] (global)
  for (int e = threadIdx.x; e < kNSlRow * Np; e += blockDim.x) { ecol[e] = t.ell_col[e]; eval[e] = t.ell_val[e]; }
  for (int e = threadIdx.x; e < kNSlD * Np; e += blockDim.x) elo[e] = t.ell_lo[e];
  // wB, wC slot-major like the global tables; wS column-major ([column][6]): the Schur update reads
  // the six weights of one column together (three 8-byte broadcast reads)
  for (int e = threadIdx.x; e < kNWin * Np; e += blockDim.x) {
    wB[e] = t.win_b[e];
    wC[e] = t.win_c[e];
    const int d = e / Np, c = e - d * Np;
    wS[c * kNWin + d] = t.win_s[e];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  // tangent workspace of this resident wavefront (lane-private rows): state, saved state,
  // stage increments [5 stages][NT] and time-derivative terms, NpA floats each
  float* tws = (NT > 0) ? A.tws + int64_t(blockIdx.x * WAVES + wid) * (8 * NT) * NpA : nullptr;
  auto TY = [&](int p) { return tws + p * NpA; };
  auto TYS = [&](int p) { return tws + (NT + p) * NpA; };
  auto TK = [&](int j, int p) { return tws + (2 * NT + j * NT + p) * NpA; };
  auto TF = [&](int p) { return tws + (7 * NT + p) * NpA; };
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
  const int i = lane & 31, h = lane >> 5;
  float* ms_out = A.msamp + int64_t(inst) * 3 * A.Ns;
  float* dd_out = A.dmdt ? A.dmdt + int64_t(inst) * 3 * A.Ns : nullptr;
  float* mt_out = (NT > 0) ? A.mtan + int64_t(inst) * NT * 3 * A.Ns : nullptr;
  if (A.status[inst] != 0) {
    for (int j = lane; j < 3 * A.Ns; j += 64) ms_out[j] = __builtin_nanf("");
    if (dd_out)
      for (int j = lane; j < 3 * A.Ns; j += 64) dd_out[j] = __builtin_nanf("");
    if constexpr (NT > 0)
      for (int j = lane; j < NT * 3 * A.Ns; j += 64) mt_out[j] = __builtin_nanf("");
    if (A.steps_out && lane == 0) A.steps_out[inst] = 0;
    continue;
  }
  const InstParams P = A.ip[inst];
  const float inv2tau = float(P.inv2tau), sigma = float(P.sigma), alpha = float(P.alpha), beta = float(P.beta_T);
  float R[9], off[3];
  for (int c = 0; c < 9; ++c) R[c] = float(P.R[c]);
  for (int c = 0; c < 3; ++c) off[c] = float(P.off[c]);

  // The state is kept as an unevaluated sum y + ylo of two FP32 parts (compensated accumulation):
  // a step adds a small increment to it, and rounding the sum to one FP32 number at every step would
  // accumulate a relative error of order sqrt(steps) * 2^-24 over the thousands of steps of a solve.
  float y[S], ylo[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int p = lane + 64 * s;
    const double c = (p < Np) ? A.c0[int64_t(inst) * A.c_stride + p] : 0.0;
    y[s] = float(c);
    ylo[s] = float(c - double(y[s]));
  }
  float ep[3] = {0.0f, 0.0f, 0.0f};  // R^T e for the tangent direction of this lane (lane / 9)
  if constexpr (NT > 0) {
    for (int pp = 0; pp < NT; ++pp) {
      const double* src = A.c0t + (int64_t(inst) * NT + pp) * A.c_stride;
      float* dst = TY(pp);
      for (int q = lane; q < Np; q += 64) dst[q] = float(src[q]);
    }
    double e[3];
    tan_axis(lane < 9 * NT ? lane / 9 : 3, P.R, e);
    for (int c = 0; c < 3; ++c) ep[c] = float(P.R[0 * 3 + c] * e[0] + P.R[1 * 3 + c] * e[1] + P.R[2 * 3 + c] * e[2]);
  }
  Store<L, L> st;
  const float rc = 2.0466534158929770f;  // sqrt(4 pi / 3)
  constexpr int pX = Gm::off(1), pY = Gm::off(1) + 1, pZ = 1;
  bool ok = true;

  // drive: mu0 H_a(t) = amp_a cos(2 pi (f_a t) + phase_a); cycles reduced in FP64
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
  // multiplier of kind `lane` (lanes 0..8) at time tt
  auto mult_lane = [&](double tt) -> float {
    float bx, by, bz;
    field(tt, bx, by, bz, false);
    bx += off[0]; by += off[1]; bz += off[2];
    const float hx = R[0] * bx + R[3] * by + R[6] * bz;
    const float hy = R[1] * bx + R[4] * by + R[7] * bz;
    const float hz = R[2] * bx + R[5] * by + R[8] * bz;
    return kind_mult(lane < 9 ? lane : 0, inv2tau, sigma, alpha, beta, hx, hy, hz);
  };
  auto dmult_lane = [&](double tt) -> float {
    float bx, by, bz;
    field(tt, bx, by, bz, true);
    const float hx = R[0] * bx + R[3] * by + R[6] * bz;
    const float hy = R[1] * bx + R[4] * by + R[7] * bz;
    const float hz = R[2] * bx + R[5] * by + R[8] * bz;
    return (lane < 3) ? 0.0f : kind_mult(lane < 9 ? lane : 0, inv2tau, sigma, alpha, beta, hx, hy, hz);
  };
  // parameter derivative of multiplier kind (lane % 9) for direction lane / 9 (lanes < 9 NT), from the
  // field (deriv = false) or its time derivative (deriv = true, constant kinds give 0)
  auto tan_lane = [&](double tt, bool deriv) -> float {
    float bx, by, bz;
    field(tt, bx, by, bz, deriv);
    if (!deriv) { bx += off[0]; by += off[1]; bz += off[2]; }
    const float hh[3] = {R[0] * bx + R[3] * by + R[6] * bz, R[1] * bx + R[4] * by + R[7] * bz,
                         R[2] * bx + R[5] * by + R[8] * bz};
    const int kind = lane % 9, prm = lane / 9;
    if (lane >= 9 * NT || (deriv && kind < 3)) return 0.0f;
    return tan_mult_t<float>(prm, kind, inv2tau, sigma, alpha, beta, float(P.D), float(P.sigK), hh, ep);
  };
  // dst[p] = add * dst[p] + (A(ms) src)[p] for the rows p = lane + 64 s (one row slot at a time).
  // Diagonal-block entries are applied as hi + lo (the table's FP32 value and its low-order part),
  // summed per kind and scaled by the kind's multiplier at the end: rounding them to FP32 would bias
  // the operator itself, and the slow relaxation modes of an anisotropic particle, whose rates are
  // small differences of large entries, are sensitive to such a bias (rounding of the sums is not a
  // bias: it changes with the state from one evaluation to the next).
  auto matvec = [&](float* dst, bool add, const float* xin) {
    float m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = w.ms[k];
#pragma unroll 1
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      const int z = opaque_zero();
      const uint16_t* ec = ecol + z;
      const float* ev = eval + z;
      const float* el = elo + z;
      if (p < Np) {
        // table reads, then gathers, then the sums, one slot group at a time: the LDS latency is paid
        // twice per group rather than twice per coupling (the scheduler otherwise waits after every load)
        float acc = 0.0f;
        {
          int ci[kNSlD];
          float hv[kNSlD], lv[kNSlD], xv[kNSlD];
#pragma unroll
          for (int u = 0; u < kNSlD; ++u) {
            ci[u] = ec[(kSlD + u) * Np + p];
            hv[u] = ev[(kSlD + u) * Np + p];
            lv[u] = el[u * Np + p];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kNSlD; ++u) xv[u] = xin[ci[u]];
          __builtin_amdgcn_sched_barrier(0);
          float sh[kNKindD], sl[kNKindD];
#pragma unroll
          for (int k = 0; k < kNKindD; ++k) sh[k] = sl[k] = 0.0f;
#pragma unroll
          for (int u = 0; u < kNSlD; ++u) {
            sh[kSlotKindRow[kSlD + u]] = fmaf(hv[u], xv[u], sh[kSlotKindRow[kSlD + u]]);
            sl[kSlotKindRow[kSlD + u]] = fmaf(lv[u], xv[u], sl[kSlotKindRow[kSlD + u]]);
          }
#pragma unroll
          for (int k = 0; k < kNKindD; ++k) acc = fmaf(m[k], sl[k], fmaf(m[k], sh[k], acc));
        }
        float acc2 = 0.0f;  // the coupling slots: a second, independent partial sum
        constexpr int kG = 6;
        static_assert((kNSlB + kNSlC) % kG == 0, "coupling slots come in whole groups");
#pragma unroll
        for (int g0 = kSlB; g0 < kNSlRow; g0 += kG) {
          int ci[kG];
          float cv[kG], xv[kG];
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            ci[u] = ec[(g0 + u) * Np + p];
            cv[u] = ev[(g0 + u) * Np + p];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u) xv[u] = xin[ci[u]];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u) acc2 = fmaf(m[kSlotKindRow[g0 + u]] * cv[u], xv[u], acc2);
        }
        acc += acc2;
        dst[p] = add ? dst[p] + acc : acc;
      }
    }
  };
  // tangent right-hand side of direction pp: V[p] += (A(t_i) xt + A_p(t_i) yt + A_p(t_n) K_i
  //   + h gm_i dA_p/dt(t_n) y)[p], one pass over the table with four gathers
  auto matvec_tan = [&](int pp, float hgm) {
    float* V = w.V();
    const float* xt = w.xt();
    const float* yt = w.xin();
    const float* kc = w.kc();
    const float* y0 = w.y0();
    float m[9], a1[9], a2[9], a3[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      m[k] = w.ms[k];
      a1[k] = w.dmi[pp][k];
      a2[k] = w.dmn[pp][k];
      a3[k] = hgm * w.ddm[pp][k];
    }
#pragma unroll 1
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      const int z = opaque_zero();
      const uint16_t* ec = ecol + z;
      const float* ev = eval + z;
      if (p < Np) {
        // table reads, then the four gathers, then the sums, seven couplings at a time
        constexpr int kG = 7;
        float acc = 0.0f;
#pragma unroll
        for (int g0 = 0; g0 < kNSlRow; g0 += kG) {
          int ci[kG];
          float cv[kG], gx[kG], gy[kG], gk[kG], g0v[kG];
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            ci[u] = ec[(g0 + u) * Np + p];
            cv[u] = ev[(g0 + u) * Np + p];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            gx[u] = xt[ci[u]];
            gy[u] = yt[ci[u]];
            gk[u] = kc[ci[u]];
            g0v[u] = y0[ci[u]];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            const int kd = kSlotKindRow[g0 + u];
            float g = m[kd] * gx[u];
            g = fmaf(a1[kd], gy[u], g);
            g = fmaf(a2[kd], gk[u], g);
            g = fmaf(a3[kd], g0v[u], g);
            acc = fmaf(cv[u], g, acc);
          }
        }
        V[p] += acc;
      }
    }
  };
  // block-tridiagonal solve M x = V with the resident inverses; result in G
  auto solve = [&]() {
    float* V = w.V();
    float* G = w.G();
    float mk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) mk[k] = w.mk[k];
    const float mFX = mk[5], mFY = mk[6], mRX = mk[7], mRY = mk[8];
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      if (h == 0 && i < n) {
        const int row = off0 + i;
        float tv = V[row];
        // (loads first, then the sums: one LDS wait per phase instead of one per coupling)
        if constexpr (K == 1) {
          const int z = opaque_zero();
          int ci[kNSlB];
          float cv[kNSlB], gv[kNSlB];
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) {
            ci[u] = ecol[z + (kSlB + u) * Np + row];
            cv[u] = eval[z + (kSlB + u) * Np + row];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) gv[u] = G[ci[u]];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < kNSlB; ++u) tv = fmaf(-mk[kSlotKindRow[kSlB + u]] * cv[u], gv[u], tv);
        } else if constexpr (K >= 2) {
          constexpr int offp = Gm::off(K - 1);
          const int z = opaque_zero();
          const int t = i & 1;
          const float* gs = G + offp + i;
          const float* go = G + offp + i + 1 - 2 * t;
          float wv[6], gsv[3], gov[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            wv[d] = wB[z + d * Np + row];
            wv[3 + d] = wB[z + (3 + d) * Np + row];
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
        w.T[(i & 1) * kH + (i >> 1)] = tv;
      }
      wsync();
      auto& a = blk<K>(st);
      float part = dot_half<Q>(a, w.T + h * kH);
      if (h == 0 && i < n) G[off0 + i] = part;
      wsync();
      __builtin_amdgcn_sched_barrier(0);
    });
    static_for_down<L - 1, 0>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      if (h == 0 && i < n) {
        const int row = off0 + i;
        float tv = 0.0f;
        {
          constexpr int offn = Gm::off(K + 1);
          const int z = opaque_zero();
          const int t = (K > 0) ? (i & 1) : 0;
          const float* gs = G + offn + ((K > 0) ? i - 4 : 2 * i - 4);
          const float* go = G + offn + ((K > 0) ? i - 3 - 2 * t : 2 * i - 3);
          float wv[6], gsv[3], gov[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            wv[d] = wC[z + d * Np + row];
            wv[3 + d] = wC[z + (3 + d) * Np + row];
            gsv[d] = gs[2 * d];
            gov[d] = go[2 * d];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            tv = fmaf((d == 1 ? mRY : mFX) * wv[d], gsv[d], tv);
            tv = fmaf((d == 1 ? mRX : mFY) * wv[3 + d], gov[d], tv);
          }
        }
        w.T[(i & 1) * kH + (i >> 1)] = tv;
      }
      wsync();
      auto& a = blk<K>(st);
      float part = dot_half<Q>(a, w.T + h * kH);
      if (h == 0 && i < n) G[off0 + i] -= part;
      wsync();
      __builtin_amdgcn_sched_barrier(0);
    });
  };
  // factor M = I - h g A(t_n) (multipliers in w.mk): Schur-complement inverses into registers
  auto factor = [&]() {
    float* X = w.X();
    float* Ub = w.Ub();
    float mk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) mk[k] = w.mk[k];
    static_for<0, L + 1>([&](auto KK) {
      constexpr int K = decltype(KK)::value;
      constexpr int n = Gm::nb(K), Q = n / 2, off0 = Gm::off(K);
      const bool act = i < n;
      constexpr int Qpv = (K > 0) ? Gm::nb(K > 0 ? K - 1 : 0) / 2 : 1;
      float u[Qpv];      // U = B_K Sinv_{K-1}: row i, columns of parity h
      float uo[Qpv];     // the same row, columns of the other parity (partner lane)
      if constexpr (K > 0) {
        constexpr int np = Gm::nb(K - 1), Qp = np / 2, offp = Gm::off(K - 1);
        auto& ap = blk<K - 1>(st);
        if (i < np) {
#pragma unroll
          for (int q = 0; q < Qp; ++q) X[i * kXS + h * kH + q] = ap[q];
        }
        wsync();
#pragma unroll
        for (int q = 0; q < Qp; ++q) u[q] = 0.0f;
        if (act) {
          const int row = off0 + i;
          const int z = opaque_zero();
          // table entries first (one LDS wait), then each coupling's row of the inverse
          if constexpr (K == 1) {
            int ci[kNSlB];
            float cv[kNSlB];
#pragma unroll
            for (int u2 = 0; u2 < kNSlB; ++u2) {
              ci[u2] = ecol[z + (kSlB + u2) * Np + row];
              cv[u2] = eval[z + (kSlB + u2) * Np + row];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u2 = 0; u2 < kNSlB; ++u2) {
              const float me = mk[kSlotKindRow[kSlB + u2]] * cv[u2];
              const float* xr = X + (ci[u2] - offp) * kXS + h * kH;
              float xv[Qp];
#pragma unroll
              for (int q = 0; q < Qp; ++q) xv[q] = xr[q];
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int q = 0; q < Qp; ++q) u[q] = fmaf(me, xv[q], u[q]);
            }
          } else {
            const int t = i & 1;
            const float* xs = X + i * kXS + h * kH;                // rows i + 2d
            const float* xo = X + (i + 1 - 2 * t) * kXS + h * kH;  // rows i + 1 - 2t + 2d
            float wv[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) wv[d] = wB[z + d * Np + row];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float ms_ = (d == 1 ? mk[8] : mk[5]) * wv[d];
              const float mo_ = (d == 1 ? mk[7] : mk[6]) * wv[3 + d];
              float xsv[Qp], xov[Qp];
#pragma unroll
              for (int q = 0; q < Qp; ++q) {
                xsv[q] = xs[2 * kXS * d + q];
                xov[q] = xo[2 * kXS * d + q];
              }
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int q = 0; q < Qp; ++q) u[q] = fmaf(mo_, xov[q], fmaf(ms_, xsv[q], u[q]));
            }
          }
        }
        if constexpr (K == 1) {
          if (act) {
#pragma unroll
            for (int q = 0; q < Qp; ++q) Ub[i * kXS + h * kH + q] = u[q];
          }
          wsync();
        } else {
#pragma unroll
          for (int q = 0; q < Qp; ++q) {
            auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(u[q]), __float_as_uint(u[q]), false, false);
            uo[q] = __uint_as_float(h == 0 ? r[1] : r[0]);
          }
        }
      }
      if (act) {
#pragma unroll
        for (int q = 0; q < Q; ++q) X[i * kXS + h * kH + q] = 0.0f;
      }
      wsync();
      if (act) {
        // diagonal-block entries of M: table reads first, then LDS atomic adds (entries of several
        // slots can share a column; the adds need no wait in between)
        const int row = off0 + i;
        const int z = opaque_zero();
        int cl[kNSlD];
        float cv[kNSlD];
#pragma unroll
        for (int u2 = 0; u2 < kNSlD; ++u2) {
          cl[u2] = int(ecol[z + (kSlD + u2) * Np + row]) - off0;
          cv[u2] = eval[z + (kSlD + u2) * Np + row];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u2 = 0; u2 < kNSlD; ++u2) {
          if ((cl[u2] & 1) == h)
            __hip_atomic_fetch_add(X + i * kXS + h * kH + (cl[u2] >> 1), mk[kSlotKindRow[kSlD + u2]] * cv[u2],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        if ((i & 1) == h)
          __hip_atomic_fetch_add(X + i * kXS + h * kH + (i >> 1), 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
      wsync();
      // work on a local copy: the indexed pivot-column access must not touch the store itself.  Rows
      // i >= n lie inside the scratch (rows 0..36) and are read unconditionally, then masked.
      float a[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) a[q] = X[i * kXS + h * kH + q];
#pragma unroll
      for (int q = 0; q < Q; ++q) a[q] = act ? a[q] : 0.0f;
      if constexpr (K == 1) {
        constexpr int offp = Gm::off(K - 1);
        if (act) {
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int c = off0 + h + 2 * q;
            float acc = 0.0f;
            const int z = opaque_zero();
            int rl[kNSlCol];
            float cv[kNSlCol], uv[kNSlCol];
#pragma unroll
            for (int sl = 0; sl < kNSlCol; ++sl) {
              rl[sl] = int(crow[z + sl * Np + c]) - offp;
              cv[sl] = cvl[z + sl * Np + c];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int sl = 0; sl < kNSlCol; ++sl) uv[sl] = Ub[i * kXS + (rl[sl] & 1) * kH + (rl[sl] >> 1)];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int sl = 0; sl < kNSlCol; ++sl) acc = fmaf(mk[kSlotKindCol[sl]] * cv[sl], uv[sl], acc);
            a[q] -= acc;
          }
        }
      } else if constexpr (K >= 2) {
        // S_K -= U C_{K-1}: column c = h + 2q takes U[i][c + 2d] (own parity) and
        // U[i][c + 1 - 2h + 2d] (other parity) with the window weights of column c
        constexpr int Qp = Gm::nb(K - 1) / 2;
        if (act) {
          const int z = opaque_zero();
          // window weights of four columns per LDS wait
          constexpr int kC = 4;
#pragma unroll
          for (int q0 = 0; q0 < Q; q0 += kC) {
            float wv[kC][6];
#pragma unroll
            for (int qq = 0; qq < kC; ++qq) {
              if (q0 + qq < Q) {
                const float2* src = reinterpret_cast<const float2*>(wS + z + (off0 + h + 2 * (q0 + qq)) * kNWin);
#pragma unroll
                for (int d2 = 0; d2 < 3; ++d2) {
                  const float2 v = src[d2];
                  wv[qq][2 * d2] = v.x;
                  wv[qq][2 * d2 + 1] = v.y;
                }
              }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int qq = 0; qq < kC; ++qq) {
              const int q = q0 + qq;
              if (q < Q) {
                float acc = 0.0f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                  if (q + d < Qp) {
                    acc = fmaf((d == 1 ? mk[8] : mk[5]) * wv[qq][d], u[q + d], acc);
                    acc = fmaf((d == 1 ? mk[7] : mk[6]) * wv[qq][3 + d], uo[q + d], acc);
                  }
                }
                a[q] -= acc;
              }
            }
          }
        }
      }
      ok = gj_piv_invert<Q, K == 0>(a, i, h, w, X) && ok;
      auto& sa = blk<K>(st);
#pragma unroll
      for (int q = 0; q < Q; ++q) sa[q] = a[q];
      __builtin_amdgcn_sched_barrier(0);
    });
  };

  // one RODAS4 step of size hs from t_n; returns max |K6| (embedded error estimate)
  auto rodas_step = [&](double tn, double hs) -> float {
    const float hf = float(hs);
    const float hg = hf * 0.25f;
    const float ih = 1.0f / hf;
    {
      // both multiplier sets of t_n before the factorisation (their shared sin/cos work is not kept
      // live across it): M's in mk, the time derivatives for f_t in ms
      const float mt = mult_lane(tn);
      const float md = dmult_lane(tn);
      if (lane < 9) {
        w.mk[lane] = -hg * mt;
        w.ms[lane] = md;
      }
      wsync();
    }
    factor();
    {  // f_t = A'(t_n) y  -> LDS
      float* xin = w.xin();
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        if (p < Np) xin[p] = y[s] + ylo[s];
      }
      wsync();
      matvec(w.ft(), false, w.xin());
      wsync();
      if constexpr (NT > 0) {
        // step-start state and the tangents' time-derivative terms dA/dt(t_n) y_p (same multipliers)
        float* y0 = w.y0();
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int p = lane + 64 * s;
          if (p < Np) y0[p] = y[s] + ylo[s];
        }
        const float dn = tan_lane(tn, false), dd = tan_lane(tn, true);
        if (lane < 9 * NT) {
          w.dmn[lane / 9][lane % 9] = dn;
          w.ddm[lane / 9][lane % 9] = dd;
        }
        for (int pp = 0; pp < NT; ++pp) {
          float* xt = w.xt();
          const float* yp = TY(pp);
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int p = lane + 64 * s;
            if (p < Np) xt[p] = yp[p];
          }
          wsync();
          matvec(TF(pp), false, w.xt());
          wsync();
        }
      }
    }
    for (int stg = 0; stg < 6; ++stg) {
      const float mt = mult_lane(tn + double(kRodasAlpha[stg]) * hs);
      if (lane < 9) w.ms[lane] = mt;
      // r = 0: the primal stage; r = 1..NT: the tangent directions of the same stage (same
      // factorisation, right-hand sides from the primal stage).  One call site of the block solve keeps
      // it inlined, so the inverses stay in registers.
#pragma unroll 1
      for (int r = 0; r <= NT; ++r) {
        float* V = w.V();
        const int pp = r - 1;
        if (r == 0) {
          // stage argument -> xin, extra right-hand-side terms -> V (no per-lane copies kept: registers)
          float* xin = w.xin();
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int p = lane + 64 * s;
            if (p < Np) {
              float sv = ylo[s];
              float ev = hf * kRodasGamma[stg] * w.ft()[p];
              for (int j = 0; j < stg; ++j) {
                const float kj = w.Kv(j)[p];
                sv = fmaf(kRodasA[stg][j], kj, sv);
                ev = fmaf(kRodasC[stg][j] * ih, kj, ev);
              }
              xin[p] = y[s] + sv;
              V[p] = ev;
            }
          }
          wsync();
          matvec(V, true, w.xin());
        } else if constexpr (NT > 0) {
          float* xt = w.xt();
          const float* yp = TY(pp);
          const float* fp = TF(pp);
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int p = lane + 64 * s;
            if (p < Np) {
              float yv = yp[p];
              float ev = hf * kRodasGamma[stg] * fp[p];
              for (int j = 0; j < stg; ++j) {
                const float kj = TK(j, pp)[p];
                yv = fmaf(kRodasA[stg][j], kj, yv);
                ev = fmaf(kRodasC[stg][j] * ih, kj, ev);
              }
              xt[p] = yv;
              V[p] = ev;
            }
          }
          wsync();
          matvec_tan(pp, hf * kRodasGamma[stg]);
        }
        wsync();
        solve();
        const float* G = w.G();
        if (r == 0) {
          if (stg < 5) {
            float* kd = w.Kv(stg);
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const int p = lane + 64 * s;
              if (p < Np) kd[p] = hg * G[p];
            }
          }
          if constexpr (NT > 0) {
            float* kc = w.kc();
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const int p = lane + 64 * s;
              if (p < Np) kc[p] = hg * G[p];
            }
            const float tm = tan_lane(tn + double(kRodasAlpha[stg]) * hs, false);
            if (lane < 9 * NT) w.dmi[lane / 9][lane % 9] = tm;
          }
        } else if constexpr (NT > 0) {
          const float* xt = w.xt();
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int p = lane + 64 * s;
            if (p < Np) {
              const float kt = hg * G[p];
              if (stg < 5) TK(stg, pp)[p] = kt;
              else TY(pp)[p] = xt[p] + kt;
            }
          }
        }
        wsync();
      }
    }
    // embedded error estimate max |K6|.  The candidate y_{n+1} = (stage-6 argument, in xin) + K6 stays in
    // LDS (with tangents K6 was kept in kc, G holds the last tangent solve) until the step is accepted.
    float emax = 0.0f;
    {
      const float* k6 = (NT > 0) ? w.kc() : w.G();
      const float sc = (NT > 0) ? 1.0f : hg;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = lane + 64 * s;
        emax = fmaxf(emax, (p < Np) ? err_abs(sc * k6[p]) : 0.0f);
      }
    }
    return wave_max(emax);
  };
  // y + ylo <- y_{n+1} = y_n + sum_j a_6j K_j + K6 of the step just taken (the stage-6 argument plus
  // K6): the increment is formed apart from y and added to it by an exact two-sum
  auto accept = [&](float hg) {
    const float* k6 = (NT > 0) ? w.kc() : w.G();
    const float sc = (NT > 0) ? 1.0f : hg;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int p = lane + 64 * s;
      if (p < Np) {
        float d = fmaf(sc, k6[p], ylo[s]);
#pragma unroll
        for (int j = 0; j < 5; ++j) d = fmaf(kRodasA[5][j], w.Kv(j)[p], d);
        const float t = y[s] + d;
        const float bb = t - y[s];
        ylo[s] = (y[s] - (t - bb)) + (d - bb);
        y[s] = t;
      }
    }
  };

  const double dt = A.period / A.Ns;
  const int n_int = (A.settle + 1) * A.Ns;
  const int first_rec = A.settle * A.Ns;
  // The controller's FP64 scalars live in LDS across a step (re-read after it), so they take no
  // registers while the step runs.
  if (lane == 0) {
    w.ctl[1] = dt;  // step size, kept across sample intervals
    w.ctl[4] = 0.0;
    w.ctl[5] = 0.0;
  }
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
    const float vx = __shfl(y[pX >> 6] + ylo[pX >> 6], pX & 63), vy = __shfl(y[pY >> 6] + ylo[pY >> 6], pY & 63),
                vz = __shfl(y[pZ >> 6] + ylo[pZ >> 6], pZ & 63);
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
          if (p < Np) xs[p] = y[s] + ylo[s];
        }
        wsync();
        float acc = 0.0f;
        if (lane < 3) {
          const int row = lane == 0 ? pX : (lane == 1 ? pY : pZ);  // rows < 64
          for (int g = 0; g < kNSlRow; ++g) {
            const float x = xs[ecol[g * Np + row]], mk = w.ms[kSlotKindRow[g]];
            acc = fmaf(mk * eval[g * Np + row], x, acc);
            if (g < kNSlD) acc = fmaf(mk * elo[g * Np + row], x, acc);
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
      if constexpr (NT > 0) {
        // d m / d p = R d m' / d p, plus e x m for the axis angles (rotation of the frame)
        const float mx = rc * (R[0] * vx + R[1] * vy + R[2] * vz);
        const float my = rc * (R[3] * vx + R[4] * vy + R[5] * vz);
        const float mz = rc * (R[6] * vx + R[7] * vy + R[8] * vz);
        for (int pp = 0; pp < NT; ++pp) {
          const float own = lane < Np ? TY(pp)[lane] : 0.0f;  // rows pX, pY, pZ lie in the first 64 for L <= 16
          const float tx = __shfl(own, pX), ty = __shfl(own, pY), tz = __shfl(own, pZ);
          if (lane < 3) {
            const float r0 = lane == 0 ? R[0] : (lane == 1 ? R[3] : R[6]);
            const float r1 = lane == 0 ? R[1] : (lane == 1 ? R[4] : R[7]);
            const float r2 = lane == 0 ? R[2] : (lane == 1 ? R[5] : R[8]);
            float v = rc * (r0 * tx + r1 * ty + r2 * tz);
            if (pp >= 3) {
              double e[3];
              tan_axis(pp, P.R, e);
              const float ex = float(e[0]), ey = float(e[1]), ez = float(e[2]);
              v += (lane == 0) ? (ey * mz - ez * my) : ((lane == 1) ? (ez * mx - ex * mz) : (ex * my - ey * mx));
            }
            mt_out[(pp * 3 + lane) * A.Ns + js] = v;
          }
        }
      }
    }
    // fixed: r_fixed equal steps per sample interval.  adaptive: steps of any size up to the sample
    // spacing, each accepted (max |K6| <= tol) or redone on its own.  The last step of an interval
    // lands on the next sample time.  (One call site of the stage routine keeps it inlined.)
    // Adaptive settling (span): no sample is recorded before the first recorded one, so the settling
    // periods are one interval, stepped with up to kSettleSpan sample spacings per step as the error
    // control allows, the last step landing on the first recorded sample time; the state checks then
    // follow every accepted step.
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
      if constexpr (NT > 0) {
        if (!fixedr)
          for (int pp = 0; pp < NT; ++pp)
            for (int q = lane; q < Np; q += 64) TYS(pp)[q] = TY(pp)[q];
      }
      const float e = rodas_step(t, hs);
      const double dt2 = A.period / A.Ns;
      const double hmin = dt2 / (A.r_max > 0 ? A.r_max : 64);
      const double t2 = w.ctl[0], hst = w.ctl[1], hs2 = w.ctl[2], nst = w.ctl[5];
      const bool landed2 = w.ctl[3] != 0.0, after_reject = w.ctl[4] != 0.0;
      const double tend2 = double(span ? A.settle * A.Ns : j + 1) * dt2;
      // e = +inf for a non-finite attempt (an overflow of the FP32 factorisation, which a long step can
      // cause): rejected like any other (5x shorter, on cleared scratch) unless it is the smallest step
      if (!isfinite(e) && (fixedr || hs2 <= hmin * 1.06)) {
        if (lane == 0) w.ctl[5] = nst + 1.0;
        ok = false;
        break;
      }
      const float fac = 0.9f * sqrtf(sqrtf(A.tol / fmaxf(e, 1e-30f)));
      // reject this step only (y is unchanged).  A step no longer than hmin / 0.95 is always accepted:
      // the landing rule could stretch its retry back to the same length.
      if (!fixedr && e > A.tol && hs2 > hmin * 1.06) {
        if constexpr (NT > 0) {
          for (int pp = 0; pp < NT; ++pp)
            for (int q = lane; q < Np; q += 64) TY(pp)[q] = TYS(pp)[q];
        }
        if (!isfinite(e) || !ok) {
          clear_wave_scratch(w, lane);
          ok = true;
        }
        if (lane == 0) {
          w.ctl[1] = fmax(hmin, hs2 * double(fmaxf(0.2f, fac)));
          w.ctl[4] = 1.0;
          w.ctl[5] = nst + 1.0;
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
        w.ctl[5] = nst + 1.0;
      }
      wsync();
      if (span) {
        const float ux = __shfl(y[pX >> 6] + ylo[pX >> 6], pX & 63),
                    uy = __shfl(y[pY >> 6] + ylo[pY >> 6], pY & 63),
                    uz = __shfl(y[pZ >> 6] + ylo[pZ >> 6], pZ & 63);
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
    if constexpr (NT > 0)
      for (int j = lane; j < NT * 3 * A.Ns; j += 64) mt_out[j] = __builtin_nanf("");
    if (lane == 0) A.status[inst] = unres ? kInstUnresolved : kInstNonfinite;
  } else if (forced) {
    if (lane == 0) A.status[inst] = kInstTolUnmet;
  }
  wsync();
  if (A.steps_out && lane == 0) A.steps_out[inst] = int(w.ctl[5]);
  }  // queue
}

// Instances (wavefronts) per workgroup.  Every degree has the 8-wavefront kernel; degrees up to
// kMultiWavesMaxL also have 12- and 16-wavefront kernels, which share the operator tables in LDS
// among more instances at a smaller register budget per wavefront (a workgroup of 64 w threads
// needs w / 4 wavefronts per SIMD).  The fastest one per degree is picked by measurement
// (fpn_autotune).  With tangents the workgroup has 4 wavefronts (more LDS per wavefront).
constexpr int kWaves = kStepperWaves;
constexpr int kTanWaves = 4;
constexpr int kMultiWavesMaxL = kStepperMultiWavesMaxL;
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS of one compute unit

template <int L, int WV, int NT>
constexpr size_t stepper_lds_bytes() {
  constexpr int Np = Geo<L>::Np;
  constexpr size_t b16 = ((size_t(kNSlRow) * Np * 2) + 15) & ~size_t(15);
  constexpr size_t tb = (b16 + size_t(kNSlRow + kNSlD + 3 * kNWin) * Np * 4 + 15) & ~size_t(15);
  return tb + WV * sizeof(WaveLds<L, NT>);
}

template <int L, int WV, int NT>
hipError_t launch_stepper_cfg(const StepLaunch& s, const DevTables& t, hipStream_t stream) {
  constexpr size_t shm = stepper_lds_bytes<L, WV, NT>();
  if (shm > kMaxLdsBytes) return hipErrorInvalidConfiguration;
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
  a.c0t = s.c0t;
  a.mtan = s.mtan;
  a.tws = s.tws;
  auto kern = stepper_kernel<L, WV, NT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  if (e != hipSuccess) return e;
  int grid = (s.n_inst + WV - 1) / WV;
  if (s.grid > 0) grid = std::min(grid, s.grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WV), shm, stream, a, t);
  return hipGetLastError();
}

template <int L>
hipError_t launch_stepper_L(const StepLaunch& s, const DevTables& t, hipStream_t stream) {
  if (s.mtan) return launch_stepper_cfg<L, kTanWaves, kNTan>(s, t, stream);
  if constexpr (L <= kMultiWavesMaxL) {
    if (s.waves == 12) return launch_stepper_cfg<L, 12, 0>(s, t, stream);
    if (s.waves == 16) return launch_stepper_cfg<L, 16, 0>(s, t, stream);
  }
  if (s.waves != 0 && s.waves != kWaves) return hipErrorInvalidValue;
  return launch_stepper_cfg<L, kWaves, 0>(s, t, stream);
}

template <int L, int WV, int NT>
hipError_t stepper_occupancy_cfg(int* waves_per_block, int* blocks_per_cu) {
  constexpr size_t shm = stepper_lds_bytes<L, WV, NT>();
  *waves_per_block = WV;
  *blocks_per_cu = 0;
  if (shm > kMaxLdsBytes) return hipSuccess;  // does not fit: reported as zero workgroups per CU
  const void* kern = reinterpret_cast<const void*>(stepper_kernel<L, WV, NT>);
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, 64 * WV, shm);
}

template <int L>
hipError_t stepper_occupancy_L(const DevTables&, bool tangents, int waves, int* waves_per_block, int* blocks_per_cu) {
  if (tangents) return stepper_occupancy_cfg<L, kTanWaves, kNTan>(waves_per_block, blocks_per_cu);
  if constexpr (L <= kMultiWavesMaxL) {
    if (waves == 12) return stepper_occupancy_cfg<L, 12, 0>(waves_per_block, blocks_per_cu);
    if (waves == 16) return stepper_occupancy_cfg<L, 16, 0>(waves_per_block, blocks_per_cu);
  }
  if (waves != 0 && waves != kWaves) return hipErrorInvalidValue;
  return stepper_occupancy_cfg<L, kWaves, 0>(waves_per_block, blocks_per_cu);
}

#define FPN_INST(LL)                                                                          \
  template hipError_t launch_stepper_L<LL>(const StepLaunch&, const DevTables&, hipStream_t); \
  template hipError_t stepper_occupancy_L<LL>(const DevTables&, bool, int, int*, int*);
#if !defined(FPN_L_BEGIN)
#define FPN_L_BEGIN 1
#define FPN_L_END 16
#endif
#if FPN_L_BEGIN <= 1 && 1 <= FPN_L_END
FPN_INST(1)
#endif
#if FPN_L_BEGIN <= 2 && 2 <= FPN_L_END
FPN_INST(2)
#endif
#if FPN_L_BEGIN <= 3 && 3 <= FPN_L_END
FPN_INST(3)
#endif
#if FPN_L_BEGIN <= 4 && 4 <= FPN_L_END
FPN_INST(4)
#endif
#if FPN_L_BEGIN <= 5 && 5 <= FPN_L_END
FPN_INST(5)
#endif
#if FPN_L_BEGIN <= 6 && 6 <= FPN_L_END
FPN_INST(6)
#endif
#if FPN_L_BEGIN <= 7 && 7 <= FPN_L_END
FPN_INST(7)
#endif
#if FPN_L_BEGIN <= 8 && 8 <= FPN_L_END
FPN_INST(8)
#endif
#if FPN_L_BEGIN <= 9 && 9 <= FPN_L_END
FPN_INST(9)
#endif
#if FPN_L_BEGIN <= 10 && 10 <= FPN_L_END
FPN_INST(10)
#endif
#if FPN_L_BEGIN <= 11 && 11 <= FPN_L_END
FPN_INST(11)
#endif
#if FPN_L_BEGIN <= 12 && 12 <= FPN_L_END
FPN_INST(12)
#endif
#if FPN_L_BEGIN <= 13 && 13 <= FPN_L_END
FPN_INST(13)
#endif
#if FPN_L_BEGIN <= 14 && 14 <= FPN_L_END
FPN_INST(14)
#endif
#if FPN_L_BEGIN <= 15 && 15 <= FPN_L_END
FPN_INST(15)
#endif
#if FPN_L_BEGIN <= 16 && 16 <= FPN_L_END
FPN_INST(16)
#endif

}  // namespace fpn
