// C ABI of libfpn (include/fpn.h): argument validation, launch planning, context state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fpn.h"
#include "capi_internal.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "physics.hpp"
#include "structure.hpp"

using namespace fpn_internal;

namespace fpn_internal {
thread_local std::string g_last_error;
fpn_status fail(fpn_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace fpn_internal

namespace {

fpn_status get_tables(fpn_ctx ctx, int L, const fpn::DevTables** out) {
  auto it = ctx->tables.find(L);
  if (it != ctx->tables.end()) {
    *out = &it->second.t;
    return FPN_OK;
  }
  const fpn::OperatorTables* h = nullptr;
  try {
    h = &fpn::operator_tables(L);
  } catch (const std::exception& e) {
    return fail(FPN_E_RANGE, e.what());
  }
  TableSet ts;
  fpn::DevTables& t = ts.t;
  t.L = L;
  t.N = h->N;
  t.Np = h->Np;
  t.n0 = h->n0;
  t.nnz = int(h->colkind.size());
  t.nnzc = int(h->crowkind.size());
  t.inv_doubles = 0;
  for (int b : h->bn) t.inv_doubles += int64_t(b) * b;
  auto up = [&](auto** dst, const auto& src) -> hipError_t {
    using E = typename std::remove_reference<decltype(src)>::type::value_type;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(src.size(), 1) * sizeof(E));
    if (e != hipSuccess) return e;
    ts.allocs.push_back(p);
    e = hipMemcpy(p, src.data(), src.size() * sizeof(E), hipMemcpyHostToDevice);
    *dst = reinterpret_cast<typename std::remove_pointer<typename std::remove_reference<decltype(dst)>::type>::type>(p);
    return e;
  };
  std::vector<int32_t> boff(h->boff.begin(), h->boff.end()), bn(h->bn.begin(), h->bn.end());
  if (h->Np > 65535) return fail(FPN_E_RANGE, "operator tables too large for 16-bit indexing");
  // fixed-slot layout (see device_common.hpp): fill the slots of each kind in column order
  const int Np = h->Np;
  std::vector<uint16_t> ecol(size_t(fpn::kNSlRow) * Np, 0), crow(size_t(fpn::kNSlCol) * Np, 0);
  std::vector<float> eval(size_t(fpn::kNSlRow) * Np, 0.0f), cvl(size_t(fpn::kNSlCol) * Np, 0.0f);
  std::vector<float> elo(size_t(fpn::kNSlRow) * Np, 0.0f);  // value - float(value) of every row slot
  std::vector<int> blk_of(Np);
  for (int k = 0; k <= L; ++k)
    for (int p = h->boff[k]; p < h->boff[k] + h->bn[k]; ++p) blk_of[p] = k;
  auto place = [&](std::vector<uint16_t>& ix, std::vector<float>& vv, const int* kinds, int first, int count,
                   int line, int kind, int other, float v) -> int {
    for (int s = first; s < first + count; ++s) {
      if (kinds[s] != kind || vv[size_t(s) * Np + line] != 0.0f) continue;
      ix[size_t(s) * Np + line] = uint16_t(other);
      vv[size_t(s) * Np + line] = v;
      return s;
    }
    return -1;
  };
  // padding slots (value 0) point inside the block they would address, so every index is in range
  for (int p = 0; p < Np; ++p) {
    const int k = blk_of[p];
    for (int s = 0; s < fpn::kNSlRow; ++s) {
      int def = p;
      if (s >= fpn::kSlB && s < fpn::kSlB + fpn::kNSlB && k > 0) def = h->boff[k - 1];
      if (s >= fpn::kSlC && s < fpn::kSlC + fpn::kNSlC && k < L) def = h->boff[k + 1];
      ecol[size_t(s) * Np + p] = uint16_t(def);
    }
    for (int s = 0; s < fpn::kNSlCol; ++s) crow[size_t(s) * Np + p] = uint16_t(k > 0 ? h->boff[k - 1] : p);
  }
  for (int p = 0; p < Np; ++p) {
    for (int e = h->seg[4 * p]; e < h->seg[4 * p + 3]; ++e) {
      const int col = int(h->colkind[e] & 0xffffu), kind = int(h->colkind[e] >> 16);
      const float v = float(h->val64[e]);
      const int rel = blk_of[col] - blk_of[p];
      const int first = rel == 0 ? fpn::kSlD : (rel < 0 ? fpn::kSlB : fpn::kSlC);
      const int count = rel == 0 ? fpn::kNSlD : (rel < 0 ? fpn::kNSlB : fpn::kNSlC);
      const int slot = place(ecol, eval, fpn::kSlotKindRow, first, count, p, kind, col, v);
      if (slot < 0) return fail(FPN_E_RANGE, "operator row does not fit the fixed-slot layout");
      elo[size_t(slot) * Np + p] = float(h->val64[e] - double(v));
      if (rel > 0 && place(crow, cvl, fpn::kSlotKindCol, 0, fpn::kNSlCol, col, kind, p, v) < 0)
        return fail(FPN_E_RANGE, "operator column does not fit the fixed-slot layout");
    }
  }
  // window coefficients of the neighbour-block couplings (layout in device_common.hpp)
  std::vector<float> wb(size_t(fpn::kNWin) * Np, 0.0f), wc(size_t(fpn::kNWin) * Np, 0.0f), ws(size_t(fpn::kNWin) * Np, 0.0f);
  {
    // expected kind of window slot e: same FX RY FX, other FY RX FY
    const int ekind[6] = {fpn::K_FX, fpn::K_RY, fpn::K_FX, fpn::K_FY, fpn::K_RX, fpn::K_FY};
    for (int p = 0; p < Np; ++p) {
      const int K = blk_of[p], i = p - h->boff[K], tr = (K > 0) ? (i & 1) : 0;
      for (int e = h->seg[4 * p]; e < h->seg[4 * p + 3]; ++e) {
        const int col = int(h->colkind[e] & 0xffffu), kind = int(h->colkind[e] >> 16);
        const float v = h->val[e];
        const int Kc = blk_of[col], c = col - h->boff[Kc];
        int slot = -1;
        if (Kc == K - 1 && K >= 2) {  // B window of row p
          if (((c - i) & 1) == 0) slot = (c - i) / 2;
          else slot = 3 + (c - i - 1 + 2 * tr) / 2;
          if (slot < 0 || slot > 5 || ekind[slot] != kind) return fail(FPN_E_RANGE, "B coupling outside its window");
          wb[size_t(slot) * Np + p] = v;
        }
        if (Kc == K + 1) {  // C window of row p
          const int bs = (K >= 1) ? i - 4 : 2 * i - 4;
          const int bo = (K >= 1) ? i - 3 - 2 * tr : 2 * i - 3;
          if (((c - bs) & 1) == 0) slot = (c - bs) / 2;
          else slot = 3 + (c - bo) / 2;
          if (slot < 0 || slot > 5 || ekind[slot] != kind) return fail(FPN_E_RANGE, "C coupling outside its window");
          wc[size_t(slot) * Np + p] = v;
          if (Kc >= 2) {  // S window of column col: rows of block Kc-1 = K
            const int tc = c & 1;
            int ss;
            if (((i - c) & 1) == 0) ss = (i - c) / 2;
            else ss = 3 + (i - c - 1 + 2 * tc) / 2;
            if (ss < 0 || ss > 5 || ekind[ss] != kind) return fail(FPN_E_RANGE, "Schur coupling outside its window");
            ws[size_t(ss) * Np + col] = v;
          }
        }
      }
    }
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(&t.seg, h->seg);
  if (e == hipSuccess) e = up(&t.colkind, h->colkind);
  if (e == hipSuccess) e = up(&t.val, h->val);
  if (e == hipSuccess) e = up(&t.val64, h->val64);
  if (e == hipSuccess) e = up(&t.cptr, h->cptr);
  if (e == hipSuccess) e = up(&t.crowkind, h->crowkind);
  if (e == hipSuccess) e = up(&t.cval, h->cval);
  if (e == hipSuccess) e = up(&t.cval64, h->cval64);
  if (e == hipSuccess) e = up(&t.ell_col, ecol);
  if (e == hipSuccess) e = up(&t.ell_val, eval);
  if (e == hipSuccess) e = up(&t.ell_lo, elo);
  if (e == hipSuccess) e = up(&t.ecol_row, crow);
  if (e == hipSuccess) e = up(&t.ecol_val, cvl);
  if (e == hipSuccess) e = up(&t.win_b, wb);
  if (e == hipSuccess) e = up(&t.win_c, wc);
  if (e == hipSuccess) e = up(&t.win_s, ws);
  if (e == hipSuccess) e = up(&t.boff, boff);
  if (e == hipSuccess) e = up(&t.bn, bn);
  if (e != hipSuccess) {
    for (void* p : ts.allocs) (void)hipFree(p);
    return fail(e == hipErrorOutOfMemory ? FPN_E_NOMEM : FPN_E_DEVICE, hipGetErrorString(e));
  }
  auto res = ctx->tables.emplace(L, std::move(ts));
  *out = &res.first->second.t;
  return FPN_OK;
}

// Records a pair of events around `launch` on `stream` when timing is on.
template <typename F>
fpn_status timed(fpn_ctx ctx, int which, hipStream_t stream, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->timing) {
    FPN_HIP(hipEventCreate(&a));
    FPN_HIP(hipEventCreate(&b));
    FPN_HIP(hipEventRecord(a, stream));
  }
  fpn_status st = launch();
  if (ctx->timing) {
    FPN_HIP(hipEventRecord(b, stream));
    ctx->events.push_back({which, {a, b}});
  }
  return st;
}

fpn_status validate_drive(const fpn_drive* d) {
  if (!d) return fail(FPN_E_ARG, "drive is NULL");
  if (!(d->period > 0.0) || !std::isfinite(d->period)) return fail(FPN_E_ARG, "drive.period must be > 0");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(d->amp[a]) || !std::isfinite(d->freq[a]) || !std::isfinite(d->phase[a]))
      return fail(FPN_E_ARG, "drive has a non-finite entry");
    if (d->freq[a] < 0.0) return fail(FPN_E_ARG, "drive.freq must be >= 0");
    const double cyc = d->freq[a] * d->period;
    if (d->amp[a] != 0.0 && std::fabs(cyc - std::round(cyc)) > 1e-9 * std::max(1.0, cyc))
      return fail(FPN_E_ARG, "drive.freq * period must be an integer (T-periodic drive)");
  }
  return FPN_OK;
}

// Twiddle table e^{2 pi i j / N_s}, j < N_s (FP64, built on the host) for `Ns`: made on first use and
// never rewritten or freed while the context lives.
fpn_status ensure_twiddle(fpn_ctx ctx, int Ns, hipStream_t stream, const double2** out) {
  auto it = ctx->twiddles.find(Ns);
  if (it == ctx->twiddles.end()) {
    std::vector<double2> tw(Ns);
    for (int j = 0; j < Ns; ++j) {
      const double a = 2.0 * fpn::kPi * double(j) / double(Ns);
      tw[j] = make_double2(std::cos(a), std::sin(a));
    }
    fpn_internal::DevBuf<double2> buf;
    FPN_HIP(buf.ensure(Ns));
    hipError_t e = hipMemcpyAsync(buf.p, tw.data(), Ns * sizeof(double2), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      buf.release();
      FPN_HIP(e);
    }
    it = ctx->twiddles.emplace(Ns, buf).first;
  }
  *out = it->second.p;
  return FPN_OK;
}

fpn_status validate_batch(const fpn_batch* b, int64_t n) {
  if (!b) return fail(FPN_E_ARG, "batch is NULL");
  if (!b->D || !b->Ms || !b->K || !b->alpha || !b->temp || !b->easy_axis || !b->L)
    return fail(FPN_E_ARG, "batch has a NULL array");
  for (int64_t i = 0; i < n; ++i)
    if (b->L[i] < 1 || b->L[i] > FPN_MAX_L)
      return fail(FPN_E_RANGE, "batch.L[" + std::to_string(i) + "] = " + std::to_string(b->L[i]) +
                                   " outside [1, " + std::to_string(FPN_MAX_L) + "]");
  return FPN_OK;
}

// Instances grouped by L (ascending), each group in batch order.
std::vector<std::pair<int, std::vector<int32_t>>> group_by_L(const int32_t* L, int64_t n) {
  std::map<int, std::vector<int32_t>> g;
  for (int64_t i = 0; i < n; ++i) g[L[i]].push_back(int32_t(i));
  return {g.begin(), g.end()};
}

}  // namespace

namespace fpn {
hipError_t launch_stepper(int L, const StepLaunch& s, const DevTables& t, float* ws, hipStream_t stream) {
  switch (L) {
#define FPN_CASE(LL) \
  case LL: return launch_stepper_L<LL>(s, t, stream);
    FPN_CASE(1) FPN_CASE(2) FPN_CASE(3) FPN_CASE(4) FPN_CASE(5) FPN_CASE(6) FPN_CASE(7) FPN_CASE(8)
    FPN_CASE(9) FPN_CASE(10) FPN_CASE(11) FPN_CASE(12) FPN_CASE(13) FPN_CASE(14) FPN_CASE(15) FPN_CASE(16)
#undef FPN_CASE
#define FPN_WCASE(LL) \
  case LL: return launch_stepper_wide_L<LL>(s, t, ws, stream);
    FPN_WCASE(17) FPN_WCASE(18) FPN_WCASE(19) FPN_WCASE(20) FPN_WCASE(21) FPN_WCASE(22) FPN_WCASE(23) FPN_WCASE(24)
#undef FPN_WCASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t stepper_occupancy(int L, const DevTables& t, bool tangents, int waves, int* waves_per_block,
                             int* blocks_per_cu) {
  switch (L) {
#define FPN_CASE(LL) \
  case LL: return stepper_occupancy_L<LL>(t, tangents, waves, waves_per_block, blocks_per_cu);
    FPN_CASE(1) FPN_CASE(2) FPN_CASE(3) FPN_CASE(4) FPN_CASE(5) FPN_CASE(6) FPN_CASE(7) FPN_CASE(8)
    FPN_CASE(9) FPN_CASE(10) FPN_CASE(11) FPN_CASE(12) FPN_CASE(13) FPN_CASE(14) FPN_CASE(15) FPN_CASE(16)
#undef FPN_CASE
#define FPN_WCASE(LL) \
  case LL: return stepper_wide_occupancy_L<LL>(waves, waves_per_block, blocks_per_cu);
    FPN_WCASE(17) FPN_WCASE(18) FPN_WCASE(19) FPN_WCASE(20) FPN_WCASE(21) FPN_WCASE(22) FPN_WCASE(23) FPN_WCASE(24)
#undef FPN_WCASE
    default: return hipErrorInvalidValue;
  }
}

int64_t stepper_ws_floats(int L) {
  switch (L) {
#define FPN_WCASE(LL) \
  case LL: return stepper_wide_ws_floats_L<LL>();
    FPN_WCASE(17) FPN_WCASE(18) FPN_WCASE(19) FPN_WCASE(20) FPN_WCASE(21) FPN_WCASE(22) FPN_WCASE(23) FPN_WCASE(24)
#undef FPN_WCASE
    default: return 0;
  }
}
}  // namespace fpn

extern "C" {

const char* fpn_status_string(fpn_status s) {
  switch (s) {
    case FPN_OK: return "ok";
    case FPN_E_ARG: return "invalid argument";
    case FPN_E_RANGE: return "value out of supported range";
    case FPN_E_DEVICE: return "HIP device error";
    case FPN_E_NOMEM: return "device out of memory";
    case FPN_E_UNSUPPORTED: return "unsupported";
    case FPN_E_IO: return "file error";
    default: return "unknown status";
  }
}

const char* fpn_last_error(void) { return g_last_error.c_str(); }

fpn_status fpn_create(fpn_ctx* out, int device) {
  if (!out) return fail(FPN_E_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  FPN_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(FPN_E_ARG, "device index out of range");
  if (fpn_status s = fpn_internal::static_scratch_init(device)) return s;
  auto* c = new fpn_ctx_s();
  c->device = device;
  *out = c;
  return FPN_OK;
}

fpn_status fpn_destroy(fpn_ctx ctx) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->tables)
    for (void* p : kv.second.allocs) (void)hipFree(p);
  for (auto& kv : ctx->twiddles) kv.second.release();
  ctx->twiddles.clear();
  ctx->ip.release();
  ctx->c0.release();
  ctx->wsinv.release();
  ctx->msamp.release();
  ctx->eq_m.release();
  ctx->idx.release();
  ctx->steps.release();
  ctx->wide_ws.release();
  ctx->m2_mt.release();
  ctx->trunc_field.release();
  ctx->m2_y.release();
  for (fpn_plan_s* pl : {ctx->solve_plan, ctx->tangent_plan}) {
    if (pl) {
      plan_release(pl);
      delete pl;
    }
  }
  for (auto* b : {&ctx->sur_x, &ctx->sur_ya, &ctx->sur_yb, &ctx->sur_h, &ctx->sur_r}) b->release();
  for (auto* b : {&ctx->sur_list, &ctx->sur_count, &ctx->sur_st}) b->release();
  ctx->sur_g.release();
  for (auto& e : ctx->events) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  delete ctx;
  return FPN_OK;
}

}  // extern "C"

namespace fpn_internal {

void plan_release(fpn_plan_s* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  for (hipStream_t s : p->side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  p->side.clear();
  p->ev.clear();
  p->cap = nullptr;
  p->ip.release();
  p->c0.release();
  p->wsinv.release();
  p->own_m.release();
  p->wide_ws.release();
  p->idx.release();
  p->steps.release();
  p->queue.release();
  p->c0t.release();
  p->own_mt.release();
  p->own_dh.release();
  p->tws.release();
}

}  // namespace fpn_internal

namespace {

fpn_status validate_opts(const fpn_drive* drive, const fpn_solve_opts* opts) {
  if (!opts) return fail(FPN_E_ARG, "opts is NULL");
  if (fpn_status s = validate_drive(drive)) return s;
  const int Ns = opts->samples_per_period, r = opts->substeps, Kh = opts->n_harm;
  if (Ns < 2) return fail(FPN_E_ARG, "samples_per_period must be >= 2");
  if (opts->settle_periods < 0) return fail(FPN_E_ARG, "settle_periods must be >= 0");
  if (r < 0 || r > 64) return fail(FPN_E_ARG, "substeps must be in [0, 64]");
  if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) return fail(FPN_E_ARG, "tol must be finite and >= 0");
  if (Kh < 0 || 2 * Kh >= Ns) return fail(FPN_E_ARG, "n_harm must satisfy 0 <= n_harm < samples_per_period/2");
  if (int64_t(Ns) * std::max(r, 1) * (opts->settle_periods + 1) > (int64_t(1) << 30))
    return fail(FPN_E_ARG, "too many time steps");
  if (opts->flags & ~uint32_t(FPN_OUT_M | FPN_OUT_HARM | FPN_HARM_Z | FPN_OUT_DMDT)) return fail(FPN_E_ARG, "unknown flag");
  // the harmonics kernel stages one instance's samples (all channels) in 64 KiB of LDS
  const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
  if (int64_t(nch) * Ns * int64_t(sizeof(float)) > FPN_MAX_HARM_LDS)
    return fail(FPN_E_RANGE, "samples_per_period too large for the harmonics (channels * N_s * 4 bytes > 64 KiB)");
  return FPN_OK;
}

fpn_status occupancy(fpn_ctx ctx, int L, const fpn::DevTables& t, bool tangents, int wg, int* waves, int* blocks) {
  const int key = L + (tangents ? 1000 : 0) + 10000 * wg;
  auto it = ctx->occupancy.find(key);
  if (it == ctx->occupancy.end()) {
    int w = 0, b = 0;
    FPN_HIP(fpn::stepper_occupancy(L, t, tangents, wg, &w, &b));
    it = ctx->occupancy.emplace(key, std::make_pair(w, b)).first;
  }
  if (it->second.second < 1) return fail(FPN_E_DEVICE, "stepper configuration does not fit on a compute unit");
  if (ctx->cus == 0) {
    hipDeviceProp_t prop;
    FPN_HIP(hipGetDeviceProperties(&prop, ctx->device));
    ctx->cus = prop.multiProcessorCount;
  }
  *waves = it->second.first;
  *blocks = it->second.second;
  return FPN_OK;
}

// Groups the batch by degree, orders the groups (most expensive first) and the instances within each
// group (by cost_hint, largest first, when given), and sizes every workspace.
fpn_status plan_build(fpn_plan_s* p, fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                      const fpn_batch* batch, int64_t n, const float* cost_hint, float* m_out, float* harm_out,
                      int32_t* status, hipStream_t stream, bool tangent = false, float* dm_out = nullptr,
                      float* dharm_out = nullptr) {
  const bool want_m = opts->flags & FPN_OUT_M, want_h = opts->flags & FPN_OUT_HARM;
  const int Ns = opts->samples_per_period;
  p->ctx = ctx;
  p->dmdt = nullptr;
  p->drive = *drive;
  p->opts = *opts;
  p->batch = *batch;
  p->batch.L = nullptr;
  p->n = n;
  p->m_out = want_m ? m_out : nullptr;
  p->harm_out = want_h ? harm_out : nullptr;
  p->status = status;
  p->tangent = tangent;
  std::map<int, std::vector<int32_t>> byL;
  for (int64_t i = 0; i < n; ++i) {
    if (tangent && batch->L[i] > 16)
      return fail(FPN_E_RANGE, "parameter sensitivities are available for L <= 16");
    byL[batch->L[i]].push_back(int32_t(i));
  }
  p->groups.clear();
  p->order.clear();
  p->order.reserve(n);
  p->np_max = 0;
  for (auto& kv : byL) {
    fpn_internal::PlanGroup g;
    g.L = kv.first;
    if (fpn_status s = get_tables(ctx, g.L, &g.t)) return s;
    p->np_max = std::max<int64_t>(p->np_max, g.t->Np);
    auto& ids = kv.second;
    double per = 0.0;  // per-step work of degree L: sum of cubed block sizes
    for (int k = 0; k <= g.L; ++k) per += std::pow(double(k == 0 ? g.t->n0 : 2 * (g.L + 1 - k)), 3.0);
    double longest = 0.0;  // steps of the longest instance (per-step work units below)
    if (cost_hint) {
      std::stable_sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) { return cost_hint[a] > cost_hint[b]; });
      for (int32_t i : ids) g.cost += per * double(cost_hint[i]);
      longest = per * double(cost_hint[ids.front()]);
    } else {
      g.cost = per * double(ids.size());
      longest = per;
    }
    g.est = longest;
    g.cnt = int(ids.size());
    p->groups.push_back(g);
    byL[g.L] = ids;
  }
  std::stable_sort(p->groups.begin(), p->groups.end(),
                   [](const fpn_internal::PlanGroup& a, const fpn_internal::PlanGroup& b) { return a.cost > b.cost; });
  int64_t start = 0, ws_total = 0, inv_total = 0, tws_total = 0;
  for (auto& g : p->groups) {
    g.start = start;
    auto& ids = byL[g.L];
    p->order.insert(p->order.end(), ids.begin(), ids.end());
    start += g.cnt;
    int waves = 0, blocks = 0;
    g.waves = tangent ? 0 : ctx->stepper_waves[g.L];
    if (g.L > 16 && g.waves == 0) {
      // wide layout: global workspace (more instances resident) or LDS workspace (shorter steps), by the
      // predicted bucket duration max(longest instance, total work / resident instances) x step time
      int wg = 0, bg = 0, wl = 0, bl = 0;
      if (fpn_status s = occupancy(ctx, g.L, *g.t, false, fpn::kWideGlobalWaves, &wg, &bg)) return s;
      if (fpn_status s = occupancy(ctx, g.L, *g.t, false, fpn::kWideLdsWaves, &wl, &bl)) return s;
      // (g.cost: the bucket's work, g.est: its longest instance's, both in per-step work units)
      const double eg = std::max(g.est, g.cost / double(int64_t(wg) * bg * ctx->cus));
      const double el = fpn::kWideLdsStepRatio * std::max(g.est, g.cost / double(int64_t(wl) * bl * ctx->cus));
      g.waves = el < eg ? fpn::kWideLdsWaves : fpn::kWideGlobalWaves;
    }
    if (fpn_status s = occupancy(ctx, g.L, *g.t, tangent, g.waves, &waves, &blocks)) return s;
    g.grid = std::max(1, std::min((g.cnt + waves - 1) / waves, blocks * ctx->cus));
    // without a cost hint, a bucket with more instances than resident wavefronts is ordered on the
    // device by the step counts of the plan's previous launch, longest first (the instances queued
    // last run after the rest)
    g.order = !cost_hint && int64_t(g.cnt) > int64_t(g.grid) * waves;
    g.est = std::max(g.est, g.cost / double(int64_t(g.grid) * waves));
    if (g.L > 16 && g.waves == fpn::kWideLdsWaves) g.est *= fpn::kWideLdsStepRatio;
    g.ws_off = ws_total;
    if (g.waves != fpn::kWideLdsWaves) ws_total += int64_t(g.grid) * waves * fpn::stepper_ws_floats(g.L);
    g.tws_off = tws_total;
    if (g.L <= 16) tws_total += int64_t(g.grid) * waves * fpn::stepper_reg_ws_floats(g.L, tangent);
    g.inv_off = inv_total;
    inv_total += int64_t(g.cnt) * g.t->inv_doubles;
  }
  if (want_h || tangent)
    if (fpn_status s = ensure_twiddle(ctx, Ns, stream, &p->twiddle)) return s;
  FPN_HIP(p->ip.ensure(n));
  FPN_HIP(p->c0.ensure(size_t(n) * p->np_max));
  FPN_HIP(p->idx.ensure(n));
  FPN_HIP(p->steps.ensure(n));
  FPN_HIP(p->queue.ensure(std::max<size_t>(p->groups.size(), 1)));
  FPN_HIP(p->wsinv.ensure(size_t(inv_total)));
  if (ws_total) FPN_HIP(p->wide_ws.ensure(size_t(ws_total)));
  p->msamp = m_out;
  if (!want_m) {
    FPN_HIP(p->own_m.ensure(size_t(n) * 3 * Ns));
    p->msamp = p->own_m.p;
  }
  if (tws_total) FPN_HIP(p->tws.ensure(size_t(tws_total)));
  if (tangent) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    FPN_HIP(p->c0t.ensure(size_t(n) * fpn::kNTan * p->np_max));
    p->mtan = dm_out;
    if (!p->mtan) {
      FPN_HIP(p->own_mt.ensure(size_t(n) * fpn::kNTan * 3 * Ns));
      p->mtan = p->own_mt.p;
    }
    p->dharm = dharm_out;
    if (!p->dharm) {
      FPN_HIP(p->own_dh.ensure(size_t(n) * fpn::kNTan * nch * (opts->n_harm + 1) * 2));
      p->dharm = p->own_dh.p;
    }
  }
  FPN_HIP(hipMemcpyAsync(p->idx.p, p->order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  // Worker streams for concurrent degree buckets: the caller's stream and up to three side streams
  // (default priority), as many as the runtime's hardware queues by default (4), so no two workers
  // share a queue (a bucket queued behind another worker's kernel on a shared queue waits for all of
  // it).  Buckets on one worker run one after another, so each bucket goes, longest predicted
  // duration first, to the worker with the least predicted time so far (the launch order within a
  // worker stays the cost order).  Worker 0 is the caller's stream.
  const size_t nwork = std::min<size_t>(p->groups.size(), 4);
  const size_t nside = nwork > 1 ? nwork - 1 : 0;
  {
    std::vector<size_t> by_est(p->groups.size());
    for (size_t i = 0; i < by_est.size(); ++i) by_est[i] = i;
    std::stable_sort(by_est.begin(), by_est.end(),
                     [&](size_t a, size_t b) { return p->groups[a].est > p->groups[b].est; });
    std::vector<double> load(std::max<size_t>(nwork, 1), 0.0);
    for (size_t i : by_est) {
      const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
      p->groups[i].stream = int(k);
      load[k] += p->groups[i].est;
    }
  }
  while (p->side.size() < nside) {
    hipStream_t s = nullptr;
    FPN_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    p->side.push_back(s);
  }
  while (p->ev.size() < 1 + p->side.size()) {
    hipEvent_t e = nullptr;
    FPN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    p->ev.push_back(e);
  }
  return FPN_OK;
}

// Launches the planned solve on `stream` (kernel launches, event records and stream waits only, so
// the sequence can be captured into a graph).  Degree buckets run on side streams when there are
// several of them.
fpn_status plan_launch(fpn_plan_s* p, hipStream_t stream, bool timing) {
  fpn_ctx ctx = p->ctx;
  const fpn_solve_opts* opts = &p->opts;
  const fpn_drive* drive = &p->drive;
  const int64_t n = p->n;
  const int Ns = opts->samples_per_period;
  auto tm = [&](int which, hipStream_t s, auto&& f) -> fpn_status {
    if (!timing) return f();
    return timed(ctx, which, s, f);
  };
  fpn::launch_fill_i32(p->queue.p, int(p->groups.size()), 0, stream);
  FPN_HIP(hipGetLastError());
  if (fpn_status s = tm(0, stream, [&]() -> fpn_status {
        fpn::launch_instance_prep(n, p->batch.D, p->batch.Ms, p->batch.K, p->batch.alpha, p->batch.temp,
                                  p->batch.easy_axis, p->batch.offset, p->ip.p, p->status, stream);
        FPN_HIP(hipGetLastError());
        return FPN_OK;
      }))
    return s;
  if (p->reorder && p->history) {
    for (const auto& g : p->groups) {
      if (!g.order) continue;
      fpn::launch_order(p->idx.p + g.start, g.cnt, p->steps.p, stream);
      FPN_HIP(hipGetLastError());
    }
  }
  double3 d0;
  d0.x = drive->amp[0] * std::cos(drive->phase[0]);
  d0.y = drive->amp[1] * std::cos(drive->phase[1]);
  d0.z = drive->amp[2] * std::cos(drive->phase[2]);
  // The stationary starts of every bucket first, on the caller's stream: they take milliseconds
  // alone, but one issued beside the persistent stepper kernels of other buckets gets few compute
  // units and delays its own bucket's stepper by seconds.
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    const auto& g = p->groups[gi];
    const int32_t* idx = p->idx.p + g.start;
    if (fpn_status s = tm(1, stream, [&]() -> fpn_status {
          fpn::launch_stationary(*g.t, idx, g.cnt, p->ip.p, nullptr, d0, p->c0.p, p->np_max, p->wsinv.p + g.inv_off,
                                 p->status, stream);
          FPN_HIP(hipGetLastError());
          if (p->tangent) {
            fpn::launch_stationary_tangent(*g.t, idx, g.cnt, p->ip.p, d0, p->c0.p, p->np_max,
                                           p->wsinv.p + g.inv_off, p->c0t.p, p->status, stream);
            FPN_HIP(hipGetLastError());
          }
          return FPN_OK;
        }))
      return s;
  }
  const bool fork = !p->side.empty();
  if (fork) {
    FPN_HIP(hipEventRecord(p->ev[0], stream));
    for (hipStream_t s : p->side) FPN_HIP(hipStreamWaitEvent(s, p->ev[0], 0));
  }
  for (size_t gi = 0; gi < p->groups.size(); ++gi) {
    const auto& g = p->groups[gi];
    hipStream_t gs = (fork && g.stream > 0) ? p->side[size_t(g.stream - 1) % p->side.size()] : stream;
    const int32_t* idx = p->idx.p + g.start;
    fpn::StepLaunch sl;
    sl.ip = p->ip.p;
    sl.inst_idx = idx;
    sl.n_inst = g.cnt;
    sl.c0 = p->c0.p;
    sl.c_stride = p->np_max;
    for (int c = 0; c < 3; ++c) {
      sl.amp[c] = drive->amp[c];
      sl.freq[c] = drive->freq[c];
      sl.phase[c] = drive->phase[c];
    }
    sl.period = drive->period;
    sl.settle = opts->settle_periods;
    sl.Ns = Ns;
    sl.r_fixed = opts->substeps;
    sl.r_max = 64;
    sl.tol = float(opts->tol > 0.0 ? opts->tol : 5e-6);
    sl.msamp = p->msamp;
    sl.dmdt = p->dmdt;
    sl.status = p->status;
    sl.steps_out = p->steps.p;
    sl.queue = p->queue.p + gi;
    sl.grid = g.grid;
    sl.waves = g.waves;
    if (g.L <= 16 && p->tws.p) sl.tws = p->tws.p + g.tws_off;
    if (p->tangent) {
      sl.c0t = p->c0t.p;
      sl.mtan = p->mtan;
    }
    if (fpn_status s = tm(2, gs, [&]() -> fpn_status {
          FPN_HIP(fpn::launch_stepper(g.L, sl, *g.t, p->wide_ws.p ? p->wide_ws.p + g.ws_off : nullptr, gs));
          return FPN_OK;
        }))
      return s;
  }
  if (fork) {
    for (size_t k = 0; k < p->side.size(); ++k) {
      FPN_HIP(hipEventRecord(p->ev[1 + k], p->side[k]));
      FPN_HIP(hipStreamWaitEvent(stream, p->ev[1 + k], 0));
    }
  }
  if (p->harm_out) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    if (fpn_status s = tm(3, stream, [&]() -> fpn_status {
          fpn::launch_harmonics(p->msamp, Ns, opts->n_harm, nch, drive->period, p->twiddle, p->harm_out,
                                p->status, n, stream);
          FPN_HIP(hipGetLastError());
          return FPN_OK;
        }))
      return s;
  }
  if (p->tangent) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    fpn::launch_harmonics(p->mtan, Ns, opts->n_harm, nch, drive->period, p->twiddle, p->dharm, p->status,
                          n * fpn::kNTan, stream, fpn::kNTan);
    FPN_HIP(hipGetLastError());
  }
  p->history = true;  // the steppers issued above write every instance's step count
  return FPN_OK;
}

fpn_status check_outputs(const fpn_solve_opts* opts, float* m_out, float* harm_out, int32_t* status, int64_t n) {
  const bool want_m = opts->flags & FPN_OUT_M, want_h = opts->flags & FPN_OUT_HARM;
  if (want_m && !m_out) return fail(FPN_E_ARG, "FPN_OUT_M set but m_out is NULL");
  if (want_h && !harm_out) return fail(FPN_E_ARG, "FPN_OUT_HARM set but harm_out is NULL");
  if (!status) return fail(FPN_E_ARG, "status is NULL");
  if (n > (int64_t(1) << 31) - 1) return fail(FPN_E_ARG, "n too large");
  return FPN_OK;
}

}  // namespace

namespace fpn_internal {
fpn_status validate_solve_opts(const fpn_drive* drive, const fpn_solve_opts* opts) { return validate_opts(drive, opts); }
fpn_status validate_solve_batch(const fpn_batch* batch, int64_t n) { return validate_batch(batch, n); }
fpn_status validate_solve_outputs(const fpn_solve_opts* opts, float* m_out, float* harm_out, int32_t* status,
                                  int64_t n) {
  return check_outputs(opts, m_out, harm_out, status, n);
}
}  // namespace fpn_internal

extern "C" {

fpn_status fpn_solve(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                     int64_t n, float* m_out, float* dmdt_out, float* harm_out, int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = validate_opts(drive, opts)) return s;
  if (n == 0) return FPN_OK;  // nothing to do (empty outputs may be NULL)
  if (fpn_status s = check_outputs(opts, m_out, harm_out, status, n)) return s;
  const bool want_dmdt = opts->flags & FPN_OUT_DMDT;
  if (want_dmdt && !dmdt_out) return fail(FPN_E_ARG, "FPN_OUT_DMDT set but dmdt_out is NULL");
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  if (!ctx->solve_plan) ctx->solve_plan = new fpn_plan_s();
  fpn_plan_s* p = ctx->solve_plan;
  ctx->last_plan = nullptr;
  if (fpn_status s = plan_build(p, ctx, drive, opts, batch, n, nullptr, m_out, harm_out, status, stream)) return s;
  p->dmdt = want_dmdt ? dmdt_out : nullptr;
  if (fpn_status s = plan_launch(p, stream, ctx->timing)) return s;
  ctx->last_plan = p;
  return FPN_OK;
}

fpn_status fpn_last_steps(fpn_ctx ctx, int64_t* total_steps) {
  if (!ctx || !total_steps) return fail(FPN_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  const fpn_plan_s* p = ctx->last_plan;
  const int64_t n = p ? p->n : 0;
  std::vector<int32_t> h(n);
  if (n > 0) {
    FPN_HIP(hipDeviceSynchronize());
    FPN_HIP(hipMemcpy(h.data(), p->steps.p, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  int64_t sum = 0;
  for (int32_t v : h) sum += v;
  *total_steps = sum;
  return FPN_OK;
}

fpn_status fpn_solve_tangent(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                             int64_t n, float* m_out, float* harm_out, float* dm_out, float* dharm_out,
                             int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = validate_opts(drive, opts)) return s;
  if (n == 0) return FPN_OK;
  if (fpn_status s = check_outputs(opts, m_out, harm_out, status, n)) return s;
  if (opts->flags & FPN_OUT_DMDT) return fail(FPN_E_ARG, "FPN_OUT_DMDT is written by fpn_solve only");
  if ((opts->flags & FPN_OUT_M) && !dm_out) return fail(FPN_E_ARG, "FPN_OUT_M set but dm_out is NULL");
  if ((opts->flags & FPN_OUT_HARM) && !dharm_out) return fail(FPN_E_ARG, "FPN_OUT_HARM set but dharm_out is NULL");
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  if (!ctx->tangent_plan) ctx->tangent_plan = new fpn_plan_s();
  fpn_plan_s* p = ctx->tangent_plan;
  ctx->last_plan = nullptr;
  if (fpn_status s = plan_build(p, ctx, drive, opts, batch, n, nullptr, m_out, harm_out, status, stream, true,
                                (opts->flags & FPN_OUT_M) ? dm_out : nullptr,
                                (opts->flags & FPN_OUT_HARM) ? dharm_out : nullptr))
    return s;
  if (fpn_status s = plan_launch(p, stream, ctx->timing)) return s;
  ctx->last_plan = p;
  return FPN_OK;
}

fpn_status fpn_adjoint(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                       int64_t n, const float* dL_dharm, double* grad_out, float* harm_out, int32_t* status,
                       void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = validate_opts(drive, opts)) return s;
  if (n == 0) return FPN_OK;
  if (!dL_dharm || !grad_out || !status) return fail(FPN_E_ARG, "dL_dharm, grad_out and status are required");
  if (fpn_status s = validate_batch(batch, n)) return s;
  fpn_solve_opts o = *opts;
  o.flags = (opts->flags & FPN_HARM_Z) | (harm_out ? FPN_OUT_HARM : 0);
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  if (!ctx->tangent_plan) ctx->tangent_plan = new fpn_plan_s();
  fpn_plan_s* p = ctx->tangent_plan;
  ctx->last_plan = nullptr;
  if (fpn_status s = plan_build(p, ctx, drive, &o, batch, n, nullptr, nullptr, harm_out, status, stream, true)) return s;
  if (fpn_status s = plan_launch(p, stream, ctx->timing)) return s;
  ctx->last_plan = p;
  const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
  fpn::launch_contract(dL_dharm, p->dharm, nch * (opts->n_harm + 1) * 2, grad_out, status, n, stream);
  FPN_HIP(hipGetLastError());
  return FPN_OK;
}

fpn_status fpn_plan_create(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                           int64_t n, const float* cost_hint, float* m_out, float* harm_out, int32_t* status,
                           fpn_plan* out) {
  if (!ctx || !out) return fail(FPN_E_ARG, "NULL argument");
  *out = nullptr;
  if (n < 1) return fail(FPN_E_ARG, "a plan needs n >= 1");
  if (fpn_status s = validate_opts(drive, opts)) return s;
  if (opts->flags & FPN_OUT_DMDT) return fail(FPN_E_ARG, "FPN_OUT_DMDT is written by fpn_solve only");
  if (fpn_status s = check_outputs(opts, m_out, harm_out, status, n)) return s;
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  auto* p = new fpn_plan_s();
  if (fpn_status s = plan_build(p, ctx, drive, opts, batch, n, cost_hint, m_out, harm_out, status, nullptr)) {
    plan_release(p);
    delete p;
    return s;
  }
  p->reorder = true;
  FPN_HIP(hipDeviceSynchronize());
  *out = p;
  return FPN_OK;
}

fpn_status fpn_plan_launch(fpn_plan p, void* stream) {
  if (!p) return fail(FPN_E_ARG, "plan is NULL");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  FPN_HIP(hipSetDevice(p->ctx->device));
  return plan_launch(p, reinterpret_cast<hipStream_t>(stream), p->ctx->timing);
}

fpn_status fpn_plan_graph_launch(fpn_plan p, void* stream) {
  if (!p) return fail(FPN_E_ARG, "plan is NULL");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  FPN_HIP(hipSetDevice(p->ctx->device));
  if (!p->exec) {
    if (!p->cap) FPN_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    FPN_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed));
    fpn_status s = plan_launch(p, p->cap, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (s != FPN_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    FPN_HIP(e);
    p->graph = g;
    FPN_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  }
  FPN_HIP(hipGraphLaunch(p->exec, reinterpret_cast<hipStream_t>(stream)));
  return FPN_OK;
}

fpn_status fpn_plan_steps(fpn_plan p, int32_t* steps_out) {
  if (!p || !steps_out) return fail(FPN_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(p->ctx->mu);
  FPN_HIP(hipSetDevice(p->ctx->device));
  FPN_HIP(hipDeviceSynchronize());
  FPN_HIP(hipMemcpy(steps_out, p->steps.p, p->n * sizeof(int32_t), hipMemcpyDeviceToHost));
  return FPN_OK;
}

fpn_status fpn_plan_destroy(fpn_plan p) {
  if (!p) return fail(FPN_E_ARG, "plan is NULL");
  (void)hipSetDevice(p->ctx->device);
  (void)hipDeviceSynchronize();
  plan_release(p);
  delete p;
  return FPN_OK;
}

fpn_status fpn_stepper_wave_options(int32_t L, int32_t* waves, int32_t* count) {
  if (!waves || !count) return fail(FPN_E_ARG, "NULL argument");
  if (L < 1 || L > FPN_MAX_L) return fail(FPN_E_ARG, "L out of range");
  int tmp[3];
  const int c = fpn::stepper_wave_options(L, tmp);
  for (int k = 0; k < c; ++k) waves[k] = tmp[k];
  *count = c;
  return FPN_OK;
}

namespace {
// the context's workgroup size for degree L after checking it is compiled and fits (lock held)
fpn_status set_waves_locked(fpn_ctx ctx, int L, int waves) {
  int opts[3];
  const int c = fpn::stepper_wave_options(L, opts);
  bool known = false;
  for (int k = 0; k < c; ++k) known = known || opts[k] == waves;
  if (L > 16) known = known || waves == fpn::kWideGlobalWaves || waves == fpn::kWideLdsWaves;
  if (waves != 0 && !known) return fail(FPN_E_ARG, "workgroup size not compiled for this degree");
  if (waves != 0) {
    const fpn::DevTables* t = nullptr;
    if (fpn_status s = get_tables(ctx, L, &t)) return s;
    int w = 0, b = 0;
    if (fpn_status s = occupancy(ctx, L, *t, false, waves, &w, &b)) return s;
  }
  ctx->stepper_waves[L] = waves;
  return FPN_OK;
}
}  // namespace

fpn_status fpn_set_stepper_waves(fpn_ctx ctx, int32_t L, int32_t waves) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (L < 1 || L > FPN_MAX_L) return fail(FPN_E_ARG, "L out of range");
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  return set_waves_locked(ctx, L, waves);
}

fpn_status fpn_autotune(fpn_ctx ctx, int32_t L, int32_t* waves_out, double* ns_per_step_out) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (L < 1 || L > FPN_MAX_L) return fail(FPN_E_ARG, "L out of range");
  int opts[3];
  const int nopt = fpn::stepper_wave_options(L, opts);
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  const fpn::DevTables* t = nullptr;
  if (fpn_status s = get_tables(ctx, L, &t)) return s;
  // probe size: twice the resident instances of the largest configuration that fits
  int64_t slots = 1;
  bool fits[3] = {false, false, false};
  for (int k = 0; k < nopt; ++k) {
    int w = 0, b = 0;
    const int key_waves = (L <= 16) ? opts[k] : 0;
    if (occupancy(ctx, L, *t, false, key_waves, &w, &b) != FPN_OK) continue;
    fits[k] = true;
    slots = std::max<int64_t>(slots, int64_t(w) * b * ctx->cus);
  }
  const int64_t n = std::min<int64_t>(2 * slots, 16384);
  // probe batch: one magnetite-like particle (D 20 nm, K 2 kJ/m^3, alpha 0.1, 295 K), easy axes on a
  // golden-angle spiral, offsets on a ring of 6 mT; a 40 us drive with 3 and 4 cycles on x and y,
  // 64 samples, no settling, two fixed steps per sample (the step count does not depend on the
  // configuration, so times compare directly)
  std::vector<double> hD(n, 20e-9), hMs(n, 474e3), hK(n, 2e3), hA(n, 0.1), hT(n, 295.0), hE(3 * n), hO(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double z = 1.0 - (2.0 * double(i) + 1.0) / double(n);
    const double r = std::sqrt(std::max(0.0, 1.0 - z * z)), ph = 2.399963229728653 * double(i);
    hE[3 * i] = r * std::cos(ph);
    hE[3 * i + 1] = r * std::sin(ph);
    hE[3 * i + 2] = z;
    const double a = 0.6180339887498949 * double(i) * 6.283185307179586;
    hO[3 * i] = 6e-3 * std::cos(a);
    hO[3 * i + 1] = 6e-3 * std::sin(a);
    hO[3 * i + 2] = 0.0;
  }
  std::vector<int32_t> hL(n, L);
  fpn_internal::DevBuf<double> dD, dMs, dK, dA, dT, dE, dO;
  fpn_internal::DevBuf<float> dm;
  fpn_internal::DevBuf<int32_t> dst;
  auto release = [&]() {
    dD.release(); dMs.release(); dK.release(); dA.release(); dT.release(); dE.release(); dO.release();
    dm.release(); dst.release();
  };
  const int Ns = 64;
  hipError_t he = hipSuccess;
  for (auto* b : {&dD, &dMs, &dK, &dA, &dT}) he = (he == hipSuccess) ? b->ensure(n) : he;
  if (he == hipSuccess) he = dE.ensure(3 * n);
  if (he == hipSuccess) he = dO.ensure(3 * n);
  if (he == hipSuccess) he = dm.ensure(size_t(n) * 3 * Ns);
  if (he == hipSuccess) he = dst.ensure(n);
  const std::pair<fpn_internal::DevBuf<double>*, const std::vector<double>*> ups[] = {
      {&dD, &hD}, {&dMs, &hMs}, {&dK, &hK}, {&dA, &hA}, {&dT, &hT}, {&dE, &hE}, {&dO, &hO}};
  for (const auto& u : ups)
    if (he == hipSuccess)
      he = hipMemcpy(u.first->p, u.second->data(), u.second->size() * sizeof(double), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    release();
    return fail(FPN_E_DEVICE, hipGetErrorString(he));
  }
  fpn_batch b{dD.p, dMs.p, dK.p, dA.p, dT.p, dE.p, dO.p, hL.data()};
  const double T = 40e-6;
  fpn_drive dr{{10e-3, 8e-3, 0.0}, {3.0 / T, 4.0 / T, 0.0}, {0.0, 0.3, 0.0}, T};
  fpn_solve_opts o{Ns, 0, 0, 2, FPN_OUT_M, 0.0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fpn_status status = FPN_OK;
  double best = 0.0;
  int best_k = -1;
  const int saved = ctx->stepper_waves[L];
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) status = fail(FPN_E_DEVICE, "event");
  for (int k = 0; k < nopt && status == FPN_OK; ++k) {
    double ns = std::numeric_limits<double>::infinity();
    if (fits[k]) {
      ctx->stepper_waves[L] = (L <= 16) ? opts[k] : 0;
      fpn_plan_s p;
      status = plan_build(&p, ctx, &dr, &o, &b, n, nullptr, dm.p, nullptr, dst.p, nullptr);
      float ms = 0.0f;
      if (status == FPN_OK) status = plan_launch(&p, nullptr, false);  // first run: code and caches warm
      if (status == FPN_OK && (hipEventRecord(e0, nullptr) != hipSuccess)) status = fail(FPN_E_DEVICE, "event");
      if (status == FPN_OK) status = plan_launch(&p, nullptr, false);
      if (status == FPN_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        status = fail(FPN_E_DEVICE, "timing");
      std::vector<int32_t> steps(n);
      if (status == FPN_OK &&
          hipMemcpy(steps.data(), p.steps.p, n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        status = fail(FPN_E_DEVICE, "steps");
      (void)hipDeviceSynchronize();
      plan_release(&p);
      int64_t tot = 0;
      for (int32_t v : steps) tot += v;
      if (status == FPN_OK && tot > 0) ns = double(ms) * 1e6 / double(tot);
    }
    if (ns_per_step_out) ns_per_step_out[k] = ns;
    if (ns < std::numeric_limits<double>::infinity() && (best_k < 0 || ns < best)) {
      best = ns;
      best_k = k;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  release();
  if (status != FPN_OK || best_k < 0) {
    ctx->stepper_waves[L] = saved;
    return status != FPN_OK ? status : fail(FPN_E_DEVICE, "no stepper configuration fits");
  }
  ctx->stepper_waves[L] = (L <= 16) ? opts[best_k] : 0;
  if (waves_out) *waves_out = opts[best_k];
  return FPN_OK;
}

fpn_status fpn_timing_enable(fpn_ctx ctx, int enable) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto& e : ctx->events) {
    (void)hipEventSynchronize(e.second.second);
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  ctx->events.clear();
  for (int k = 0; k < 4; ++k) { ctx->ms[k] = 0.0; ctx->launches[k] = 0; }
  ctx->timing = enable != 0;
  return FPN_OK;
}

fpn_status fpn_timing_read(fpn_ctx ctx, double* ms_out, int64_t* launches_out) {
  if (!ctx || !ms_out || !launches_out) return fail(FPN_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  for (auto& e : ctx->events) {
    FPN_HIP(hipEventSynchronize(e.second.second));
    float ms = 0.0f;
    FPN_HIP(hipEventElapsedTime(&ms, e.second.first, e.second.second));
    ctx->ms[e.first] += ms;
    ctx->launches[e.first] += 1;
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  ctx->events.clear();
  for (int k = 0; k < 4; ++k) {
    ms_out[k] = ctx->ms[k];
    launches_out[k] = ctx->launches[k];
  }
  return FPN_OK;
}

fpn_status fpn_equilibrium(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                           int64_t n, float* m_out, float* harm_out, int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = validate_opts(drive, opts)) return s;
  if (n == 0) return FPN_OK;
  if (opts->flags & FPN_OUT_DMDT) return fail(FPN_E_ARG, "FPN_OUT_DMDT is written by fpn_solve only");
  if (fpn_status s = check_outputs(opts, m_out, harm_out, status, n)) return s;
  if (fpn_status s = validate_batch(batch, n)) return s;
  const int Ns = opts->samples_per_period;
  if (int64_t(n) * Ns >= (int64_t(1) << 31)) return fail(FPN_E_ARG, "n * samples_per_period must be < 2^31");
  const bool want_m = opts->flags & FPN_OUT_M, want_h = opts->flags & FPN_OUT_HARM;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  float* m = m_out;
  if (!want_m) {
    FPN_HIP(ctx->eq_m.ensure(size_t(n) * 3 * Ns));
    m = ctx->eq_m.p;
  }
  const double2* tw = nullptr;
  if (want_h)
    if (fpn_status s = ensure_twiddle(ctx, Ns, stream, &tw)) return s;
  FPN_HIP(ctx->ip.ensure(n));
  fpn::launch_instance_prep(n, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp, batch->easy_axis,
                            batch->offset, ctx->ip.p, status, stream);
  FPN_HIP(hipGetLastError());
  fpn::EqDrive d;
  for (int c = 0; c < 3; ++c) {
    d.amp[c] = drive->amp[c];
    d.freq[c] = drive->freq[c];
    d.phase[c] = drive->phase[c];
  }
  d.period = drive->period;
  fpn::launch_equilibrium(n, Ns, opts->settle_periods, d, ctx->ip.p, status, m, stream);
  FPN_HIP(hipGetLastError());
  if (want_h) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    // timed like the solver's harmonics (fpn_timing_enable / fpn_timing_read, slot 3)
    return timed(ctx, 3, stream, [&]() -> fpn_status {
      fpn::launch_harmonics(m, Ns, opts->n_harm, nch, drive->period, tw, harm_out, status, n, stream);
      FPN_HIP(hipGetLastError());
      return FPN_OK;
    });
  }
  return FPN_OK;
}

namespace {

// Stationary states of degree L[i] (host array) under the per-instance fields `field` [n][3] (device),
// reduced on the host to the lab-frame moments m [n][3] (host vector).  Shared by fpn_stationary and
// fpn_truncation_estimate; the caller holds the context lock.
fpn_status stationary_moments(fpn_ctx ctx, const fpn_batch* batch, const int32_t* L, int64_t n, const double* field,
                              std::vector<double>* m, int32_t* status, hipStream_t stream) {
  auto groups = group_by_L(L, n);
  std::map<int, const fpn::DevTables*> tabs;
  int64_t inv_max = 0, np_max = 0;
  size_t maxg = 0;
  for (auto& g : groups) {
    const fpn::DevTables* t = nullptr;
    if (fpn_status s = get_tables(ctx, g.first, &t)) return s;
    tabs[g.first] = t;
    inv_max = std::max<int64_t>(inv_max, t->inv_doubles);
    np_max = std::max<int64_t>(np_max, t->Np);
    maxg = std::max(maxg, g.second.size());
  }
  FPN_HIP(ctx->ip.ensure(n));
  FPN_HIP(ctx->c0.ensure(size_t(n) * np_max));
  FPN_HIP(ctx->idx.ensure(n));
  FPN_HIP(ctx->wsinv.ensure(maxg * size_t(inv_max)));
  std::vector<int32_t> order;
  for (auto& g : groups) order.insert(order.end(), g.second.begin(), g.second.end());
  FPN_HIP(hipMemcpyAsync(ctx->idx.p, order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  fpn::launch_instance_prep(n, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp, batch->easy_axis,
                            nullptr, ctx->ip.p, status, stream);
  FPN_HIP(hipGetLastError());
  int64_t start = 0;
  double3 zero;
  zero.x = zero.y = zero.z = 0.0;
  for (auto& g : groups) {
    const fpn::DevTables& t = *tabs[g.first];
    const int cnt = int(g.second.size());
    fpn::launch_stationary(t, ctx->idx.p + start, cnt, ctx->ip.p, field, zero, ctx->c0.p, np_max, ctx->wsinv.p,
                           status, stream);
    FPN_HIP(hipGetLastError());
    start += cnt;
  }
  // moments from the block-order states: (1,+1) at n0, (1,-1) at n0+1, (1,0) at 1
  std::vector<fpn::InstParams> hip_ip(n);
  std::vector<double> c(size_t(n) * np_max);
  FPN_HIP(hipMemcpyAsync(hip_ip.data(), ctx->ip.p, n * sizeof(fpn::InstParams), hipMemcpyDeviceToHost, stream));
  FPN_HIP(hipMemcpyAsync(c.data(), ctx->c0.p, c.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  m->assign(size_t(n) * 3, 0.0);
  const double rc = std::sqrt(4.0 * fpn::kPi / 3.0);
  for (int64_t i = 0; i < n; ++i) {
    const int n0 = tabs[L[i]]->n0;
    const double* ci = c.data() + i * np_max;
    const double mp[3] = {rc * ci[n0], rc * ci[n0 + 1], rc * ci[1]};
    for (int a = 0; a < 3; ++a)
      (*m)[3 * i + a] = hip_ip[i].R[3 * a] * mp[0] + hip_ip[i].R[3 * a + 1] * mp[1] + hip_ip[i].R[3 * a + 2] * mp[2];
  }
  return FPN_OK;
}

}  // namespace

fpn_status fpn_stationary(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const double* field, double* m_out,
                          int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (n == 0) return FPN_OK;
  if (!field || !m_out || !status) return fail(FPN_E_ARG, "field, m_out and status are required");
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  std::vector<double> m;
  if (fpn_status s = stationary_moments(ctx, batch, batch->L, n, field, &m, status, stream)) return s;
  FPN_HIP(hipMemcpyAsync(m_out, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  return FPN_OK;
}

fpn_status fpn_select_degree(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const fpn_drive* drive,
                             int32_t samples_per_period, double tol, int32_t L_max, int32_t* L_out, double* est_out,
                             int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (n == 0) return FPN_OK;
  if (!drive || !L_out || !status) return fail(FPN_E_ARG, "drive, L_out and status are required");
  if (samples_per_period < 1) return fail(FPN_E_ARG, "samples_per_period < 1");
  if (!(drive->period > 0.0) || !std::isfinite(drive->period)) return fail(FPN_E_ARG, "drive period must be > 0");
  if (!(tol > 0.0)) return fail(FPN_E_ARG, "tol must be > 0");
  if (L_max < 3 || L_max > FPN_MAX_L) return fail(FPN_E_RANGE, "L_max must be in 3..24");
  if (fpn_status s = validate_batch(batch, n)) return s;
  int lo = L_max;
  for (int64_t i = 0; i < n; ++i) {
    if (batch->L[i] < 3 || batch->L[i] > L_max) return fail(FPN_E_RANGE, "the starting degrees must be in 3..L_max");
    lo = std::min(lo, int(batch->L[i]));
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  FPN_HIP(ctx->trunc_field.ensure(size_t(n) * 3));
  fpn::launch_peak_field(n, batch->offset, drive->amp, drive->freq, drive->phase, drive->period, samples_per_period,
                         ctx->trunc_field.p, stream);
  FPN_HIP(hipGetLastError());
  // moments of every degree lo - 2 .. L_max for every instance (each degree one batch of stationary solves)
  const int nd = L_max - (lo - 2) + 1;
  std::vector<std::vector<double>> m(static_cast<size_t>(nd));
  std::vector<int32_t> Ld(n);
  for (int d = 0; d < nd; ++d) {
    std::fill(Ld.begin(), Ld.end(), int32_t(lo - 2 + d));
    if (fpn_status s = stationary_moments(ctx, batch, Ld.data(), n, ctx->trunc_field.p, &m[size_t(d)], status, stream))
      return s;
  }
  std::vector<int32_t> st(n);
  FPN_HIP(hipMemcpyAsync(st.data(), status, n * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  std::vector<double> est(n);
  for (int64_t i = 0; i < n; ++i) {
    L_out[i] = L_max;
    est[i] = std::nan("");
    if (st[i] != 0) continue;
    for (int L = batch->L[i]; L <= L_max; ++L) {
      const double* a = m[size_t(L - (lo - 2))].data() + 3 * i;
      const double* b = m[size_t(L - 2 - (lo - 2))].data() + 3 * i;
      const double e = std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                                 (a[2] - b[2]) * (a[2] - b[2]));
      L_out[i] = L;
      est[i] = e;
      if (e <= tol) break;
    }
  }
  if (est_out) {
    FPN_HIP(hipMemcpyAsync(est_out, est.data(), n * sizeof(double), hipMemcpyHostToDevice, stream));
    FPN_HIP(hipStreamSynchronize(stream));
  }
  return FPN_OK;
}

fpn_status fpn_truncation_estimate(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const fpn_drive* drive,
                                   int32_t samples_per_period, double* est_out, int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (n == 0) return FPN_OK;
  if (!drive || !est_out || !status) return fail(FPN_E_ARG, "drive, est_out and status are required");
  if (samples_per_period < 1) return fail(FPN_E_ARG, "samples_per_period < 1");
  if (!(drive->period > 0.0) || !std::isfinite(drive->period)) return fail(FPN_E_ARG, "drive period must be > 0");
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::vector<int32_t> Llow(n);
  for (int64_t i = 0; i < n; ++i) {
    if (batch->L[i] < 3) return fail(FPN_E_RANGE, "the truncation estimate needs L >= 3");
    Llow[i] = batch->L[i] - 2;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  FPN_HIP(ctx->trunc_field.ensure(size_t(n) * 3));
  fpn::launch_peak_field(n, batch->offset, drive->amp, drive->freq, drive->phase, drive->period, samples_per_period,
                         ctx->trunc_field.p, stream);
  FPN_HIP(hipGetLastError());
  std::vector<double> ma, mb;
  if (fpn_status s = stationary_moments(ctx, batch, batch->L, n, ctx->trunc_field.p, &ma, status, stream)) return s;
  if (fpn_status s = stationary_moments(ctx, batch, Llow.data(), n, ctx->trunc_field.p, &mb, status, stream)) return s;
  std::vector<int32_t> st(n);
  FPN_HIP(hipMemcpyAsync(st.data(), status, n * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  std::vector<double> est(n);
  for (int64_t i = 0; i < n; ++i) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) d2 += (ma[3 * i + a] - mb[3 * i + a]) * (ma[3 * i + a] - mb[3 * i + a]);
    est[i] = st[i] == 0 ? std::sqrt(d2) : std::nan("");
  }
  FPN_HIP(hipMemcpyAsync(est_out, est.data(), n * sizeof(double), hipMemcpyHostToDevice, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  return FPN_OK;
}

fpn_status fpn_host_operator(int32_t L, double D, double Ms, double K, double alpha, double temp,
                             const double field_easy[3], double* A_out) {
  if (!field_easy || !A_out) return fail(FPN_E_ARG, "NULL argument");
  if (L < 1 || L > 32) return fail(FPN_E_RANGE, "L outside [1, 32]");
  if (!(D > 0) || !(Ms > 0) || !(K >= 0) || !(alpha > 0) || !(temp > 0))
    return fail(FPN_E_ARG, "non-physical particle parameter");
  const fpn::ParticleScalars s = fpn::particle_scalars(D, Ms, K, alpha, temp);
  double mult[fpn::K_COUNT];
  fpn::kind_multipliers(s.inv2tau, s.sigma, s.beta_T, s.alpha, field_easy, mult);
  try {
    fpn::dense_operator(fpn::operator_tables(L), mult, A_out);
  } catch (const std::exception& e) {
    return fail(FPN_E_RANGE, e.what());
  }
  return FPN_OK;
}

fpn_status fpn_host_frame(const double n[3], double R_out[9]) {
  if (!n || !R_out) return fail(FPN_E_ARG, "NULL argument");
  if (!fpn::easy_axis_frame(n, R_out)) return fail(FPN_E_ARG, "|n| differs from 1");
  return FPN_OK;
}

int64_t fpn_host_table_nnz(int32_t L) {
  if (L < 1 || L > 32) return -1;
  try {
    return int64_t(fpn::operator_tables(L).colkind.size());
  } catch (...) {
    return -1;
  }
}

}  // extern "C"
