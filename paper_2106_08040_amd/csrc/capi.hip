// C ABI of libfpn (include/fpn.h): argument validation, launch planning, context state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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
  std::vector<int> blk_of(Np);
  for (int k = 0; k <= L; ++k)
    for (int p = h->boff[k]; p < h->boff[k] + h->bn[k]; ++p) blk_of[p] = k;
  auto place = [&](std::vector<uint16_t>& ix, std::vector<float>& vv, const int* kinds, int first, int count,
                   int line, int kind, int other, float v) -> bool {
    for (int s = first; s < first + count; ++s) {
      if (kinds[s] != kind || vv[size_t(s) * Np + line] != 0.0f) continue;
      ix[size_t(s) * Np + line] = uint16_t(other);
      vv[size_t(s) * Np + line] = v;
      return true;
    }
    return false;
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
      const float v = h->val[e];
      const int rel = blk_of[col] - blk_of[p];
      const int first = rel == 0 ? fpn::kSlD : (rel < 0 ? fpn::kSlB : fpn::kSlC);
      const int count = rel == 0 ? fpn::kNSlD : (rel < 0 ? fpn::kNSlB : fpn::kNSlC);
      if (!place(ecol, eval, fpn::kSlotKindRow, first, count, p, kind, col, v))
        return fail(FPN_E_RANGE, "operator row does not fit the fixed-slot layout");
      if (rel > 0 && !place(crow, cvl, fpn::kSlotKindCol, 0, fpn::kNSlCol, col, kind, p, v))
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

fpn_status ensure_twiddle(fpn_ctx ctx, int Ns, hipStream_t stream) {
  if (ctx->tw_N == Ns) return FPN_OK;
  std::vector<double2> tw(Ns);
  for (int j = 0; j < Ns; ++j) {
    const double a = 2.0 * fpn::kPi * double(j) / double(Ns);
    tw[j] = make_double2(std::cos(a), std::sin(a));
  }
  FPN_HIP(ctx->twiddle.ensure(Ns));
  FPN_HIP(hipMemcpyAsync(ctx->twiddle.p, tw.data(), Ns * sizeof(double2), hipMemcpyHostToDevice, stream));
  FPN_HIP(hipStreamSynchronize(stream));
  ctx->tw_N = Ns;
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
  ctx->twiddle.release();
  ctx->ip.release();
  ctx->c0.release();
  ctx->wsinv.release();
  ctx->msamp.release();
  ctx->idx.release();
  ctx->steps.release();
  ctx->wide_ws.release();
  for (auto* b : {&ctx->sur_x, &ctx->sur_ya, &ctx->sur_yb, &ctx->sur_h}) b->release();
  for (auto* b : {&ctx->sur_list, &ctx->sur_count, &ctx->sur_st}) b->release();
  ctx->sur_g.release();
  for (auto& e : ctx->events) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  delete ctx;
  return FPN_OK;
}

fpn_status fpn_solve(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts, const fpn_batch* batch,
                     int64_t n, float* m_out, float* harm_out, int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (!opts) return fail(FPN_E_ARG, "opts is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = validate_drive(drive)) return s;
  const int Ns = opts->samples_per_period, r = opts->substeps, Kh = opts->n_harm;
  if (Ns < 2) return fail(FPN_E_ARG, "samples_per_period must be >= 2");
  if (opts->settle_periods < 0) return fail(FPN_E_ARG, "settle_periods must be >= 0");
  if (r < 0 || r > 64) return fail(FPN_E_ARG, "substeps must be in [0, 64]");
  if (!(opts->tol >= 0.0) || !std::isfinite(opts->tol)) return fail(FPN_E_ARG, "tol must be finite and >= 0");
  if (Kh < 0 || 2 * Kh >= Ns) return fail(FPN_E_ARG, "n_harm must satisfy 0 <= n_harm < samples_per_period/2");
  if (int64_t(Ns) * std::max(r, 1) * (opts->settle_periods + 1) > (int64_t(1) << 30))
    return fail(FPN_E_ARG, "too many time steps");
  if (opts->flags & ~uint32_t(FPN_OUT_M | FPN_OUT_HARM | FPN_HARM_Z)) return fail(FPN_E_ARG, "unknown flag");
  const bool want_m = opts->flags & FPN_OUT_M, want_h = opts->flags & FPN_OUT_HARM;
  if (n == 0) return FPN_OK;  // nothing to do (empty outputs may be NULL)
  if (want_m && !m_out) return fail(FPN_E_ARG, "FPN_OUT_M set but m_out is NULL");
  if (want_h && !harm_out) return fail(FPN_E_ARG, "FPN_OUT_HARM set but harm_out is NULL");
  if (!status) return fail(FPN_E_ARG, "status is NULL");
  if (n > (int64_t(1) << 31) - 1) return fail(FPN_E_ARG, "n too large");
  if (fpn_status s = validate_batch(batch, n)) return s;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));

  auto groups = group_by_L(batch->L, n);
  int Lmax = 0;
  for (auto& g : groups) Lmax = std::max(Lmax, g.first);
  std::map<int, const fpn::DevTables*> tabs;
  int64_t inv_max = 0, np_max = 0;
  for (auto& g : groups) {
    const fpn::DevTables* t = nullptr;
    if (fpn_status s = get_tables(ctx, g.first, &t)) return s;
    tabs[g.first] = t;
    inv_max = std::max<int64_t>(inv_max, t->inv_doubles);
    np_max = std::max<int64_t>(np_max, t->Np);
  }
  if (want_h)
    if (fpn_status s = ensure_twiddle(ctx, Ns, stream)) return s;
  FPN_HIP(ctx->ip.ensure(n));
  FPN_HIP(ctx->c0.ensure(size_t(n) * np_max));
  FPN_HIP(ctx->idx.ensure(n));
  FPN_HIP(ctx->steps.ensure(n));
  ctx->steps_n = n;
  float* msamp = m_out;
  if (!want_m) {
    FPN_HIP(ctx->msamp.ensure(size_t(n) * 3 * Ns));
    msamp = ctx->msamp.p;
  }
  // largest group bounds the stationary workspace; the wide-layout stepper needs its own
  size_t maxg = 0, wide = 0;
  for (auto& g : groups) {
    maxg = std::max(maxg, g.second.size());
    wide = std::max(wide, g.second.size() * size_t(fpn::stepper_ws_floats(g.first)));
  }
  FPN_HIP(ctx->wsinv.ensure(maxg * size_t(inv_max)));
  if (wide) FPN_HIP(ctx->wide_ws.ensure(wide));
  std::vector<int32_t> order;
  order.reserve(n);
  for (auto& g : groups) order.insert(order.end(), g.second.begin(), g.second.end());
  FPN_HIP(hipMemcpyAsync(ctx->idx.p, order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream));

  if (fpn_status s = timed(ctx, 0, stream, [&]() -> fpn_status {
        fpn::launch_instance_prep(n, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp, batch->easy_axis,
                                  batch->offset, ctx->ip.p, status, stream);
        FPN_HIP(hipGetLastError());
        return FPN_OK;
      }))
    return s;
  double3 d0;
  d0.x = drive->amp[0] * std::cos(drive->phase[0]);
  d0.y = drive->amp[1] * std::cos(drive->phase[1]);
  d0.z = drive->amp[2] * std::cos(drive->phase[2]);
  int64_t start = 0;
  for (auto& g : groups) {
    const fpn::DevTables& t = *tabs[g.first];
    const int cnt = int(g.second.size());
    const int32_t* idx = ctx->idx.p + start;
    if (fpn_status s = timed(ctx, 1, stream, [&]() -> fpn_status {
          fpn::launch_stationary(t, idx, cnt, ctx->ip.p, nullptr, d0, ctx->c0.p, np_max, ctx->wsinv.p, status,
                                 stream);
          FPN_HIP(hipGetLastError());
          return FPN_OK;
        }))
      return s;
    fpn::StepLaunch sl;
    sl.ip = ctx->ip.p;
    sl.inst_idx = idx;
    sl.n_inst = cnt;
    sl.c0 = ctx->c0.p;
    sl.c_stride = np_max;
    for (int c = 0; c < 3; ++c) {
      sl.amp[c] = drive->amp[c];
      sl.freq[c] = drive->freq[c];
      sl.phase[c] = drive->phase[c];
    }
    sl.period = drive->period;
    sl.settle = opts->settle_periods;
    sl.Ns = Ns;
    sl.r_fixed = r;
    sl.r_max = 64;
    sl.tol = float(opts->tol > 0.0 ? opts->tol : 5e-6);
    sl.msamp = msamp;
    sl.status = status;
    sl.steps_out = ctx->steps.p;
    if (fpn_status s = timed(ctx, 2, stream, [&]() -> fpn_status {
          FPN_HIP(fpn::launch_stepper(g.first, sl, t, ctx->wide_ws.p, stream));
          return FPN_OK;
        }))
      return s;
    start += cnt;
  }
  if (want_h) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    if (fpn_status s = timed(ctx, 3, stream, [&]() -> fpn_status {
          fpn::launch_harmonics(msamp, Ns, Kh, nch, drive->period, ctx->twiddle.p, harm_out, status, n, stream);
          FPN_HIP(hipGetLastError());
          return FPN_OK;
        }))
      return s;
  }
  return FPN_OK;
}

fpn_status fpn_last_steps(fpn_ctx ctx, int64_t* total_steps) {
  if (!ctx || !total_steps) return fail(FPN_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  FPN_HIP(hipSetDevice(ctx->device));
  std::vector<int32_t> h(ctx->steps_n);
  if (ctx->steps_n > 0) {
    FPN_HIP(hipDeviceSynchronize());
    FPN_HIP(hipMemcpy(h.data(), ctx->steps.p, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  int64_t sum = 0;
  for (int32_t v : h) sum += v;
  *total_steps = sum;
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
  auto groups = group_by_L(batch->L, n);
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
  std::vector<double> m(size_t(n) * 3);
  const double rc = std::sqrt(4.0 * fpn::kPi / 3.0);
  for (int64_t i = 0; i < n; ++i) {
    const int n0 = tabs[batch->L[i]]->n0;
    const double* ci = c.data() + i * np_max;
    const double mp[3] = {rc * ci[n0], rc * ci[n0 + 1], rc * ci[1]};
    for (int a = 0; a < 3; ++a)
      m[3 * i + a] = hip_ip[i].R[3 * a] * mp[0] + hip_ip[i].R[3 * a + 1] * mp[1] + hip_ip[i].R[3 * a + 2] * mp[2];
  }
  FPN_HIP(hipMemcpyAsync(m_out, m.data(), m.size() * sizeof(double), hipMemcpyHostToDevice, stream));
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
