// C ABI of the surrogate evaluation (include/fpn.h, "surrogate evaluation" section):
// features, two-member ensemble forward, error estimate, and the solver for every instance
// whose estimate exceeds the tolerance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/fpn.h"
#include "capi_internal.hpp"
#include "surrogate.hpp"

using namespace fpn_internal;

extern "C" {

fpn_status fpn_surrogate_features(fpn_ctx ctx, const fpn_batch* batch, int64_t n, float* x, int32_t* status,
                                  void* stream) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (n == 0) return FPN_OK;
  if (!batch || !x || !status) return fail(FPN_E_ARG, "NULL argument");
  if (!batch->D || !batch->Ms || !batch->K || !batch->alpha || !batch->temp || !batch->easy_axis)
    return fail(FPN_E_ARG, "batch has a NULL array");
  FPN_HIP(hipSetDevice(ctx->device));
  FPN_HIP(fpn::sur::features(n, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp, batch->easy_axis,
                             batch->offset, x, status, reinterpret_cast<hipStream_t>(stream)));
  return FPN_OK;
}

fpn_status fpn_surrogate_predict(fpn_ctx ctx, const fpn_surrogate* sur, double tol, const fpn_drive* drive,
                                 const fpn_solve_opts* opts, const fpn_batch* batch, int64_t n, float* harm_out,
                                 float* err_out, int32_t* used_solver, int32_t* status, int64_t* n_fallback,
                                 void* stream) {
  if (!ctx || !sur || !opts || !batch) return fail(FPN_E_ARG, "NULL argument");
  if (n < 0 || n > (int64_t(1) << 30)) return fail(FPN_E_ARG, "n outside [0, 2^30]");
  if (n_fallback) *n_fallback = 0;
  if (!sur->net[0] || !sur->net[1]) return fail(FPN_E_ARG, "surrogate needs two networks");
  const fpn_mlp a = sur->net[0], b = sur->net[1];
  const int Kh = opts->n_harm;
  if (a->w != b->w) return fail(FPN_E_ARG, "ensemble members differ in shape");
  if (a->w.front() != 8 || a->w.back() != 4 * Kh)
    return fail(FPN_E_ARG, "networks must map 8 features to 4 * n_harm outputs");
  if (a->device != ctx->device || b->device != ctx->device) return fail(FPN_E_ARG, "networks on another device");
  const bool resid = sur->res[0] || sur->res[1];
  if (resid) {
    if (!sur->res[0] || !sur->res[1]) return fail(FPN_E_ARG, "residual stage needs two networks");
    if (sur->res[0]->w != a->w || sur->res[1]->w != a->w) return fail(FPN_E_ARG, "residual networks differ in shape");
    if (sur->res[0]->device != ctx->device || sur->res[1]->device != ctx->device)
      return fail(FPN_E_ARG, "networks on another device");
    if (!(sur->res_scale > 0.0f) || !std::isfinite(sur->res_scale)) return fail(FPN_E_ARG, "res_scale must be > 0");
  }
  if (!(sur->out_scale > 0.0f) || !std::isfinite(sur->out_scale) || !(sur->err_calib > 0.0f) ||
      !std::isfinite(sur->err_calib))
    return fail(FPN_E_ARG, "out_scale and err_calib must be finite and > 0");
  if (!(tol >= 0.0)) return fail(FPN_E_ARG, "tol must be >= 0");
  if (opts->flags & FPN_HARM_Z) return fail(FPN_E_ARG, "the surrogate predicts the x and y channels only");
  if (n == 0) return FPN_OK;
  if (!harm_out || !err_out || !used_solver || !status) return fail(FPN_E_ARG, "NULL output");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(ctx->device));
  const int W = 4 * Kh;
  FPN_HIP(ctx->sur_x.ensure(size_t(n) * 8));
  FPN_HIP(ctx->sur_ya.ensure(size_t(n) * W));
  FPN_HIP(ctx->sur_yb.ensure(size_t(n) * W));
  FPN_HIP(ctx->sur_list.ensure(size_t(n)));
  FPN_HIP(ctx->sur_count.ensure(1));
  if (fpn_status e = fpn_surrogate_features(ctx, batch, n, ctx->sur_x.p, status, stream)) return e;
  if (fpn_status e = fpn_mlp_forward(a, ctx->sur_x.p, n, ctx->sur_ya.p, stream)) return e;
  if (fpn_status e = fpn_mlp_forward(b, ctx->sur_x.p, n, ctx->sur_yb.p, stream)) return e;
  if (resid) {  // member k's output += res[k](x) / res_scale
    FPN_HIP(ctx->sur_r.ensure(size_t(n) * W));
    float* ys[2] = {ctx->sur_ya.p, ctx->sur_yb.p};
    for (int k = 0; k < 2; ++k) {
      if (fpn_status e = fpn_mlp_forward(sur->res[k], ctx->sur_x.p, n, ctx->sur_r.p, stream)) return e;
      FPN_HIP(fpn::sur::axpy(n * W, 1.0f / sur->res_scale, ctx->sur_r.p, ys[k], s));
    }
  }
  FPN_HIP(fpn::sur::combine(n, Kh, ctx->sur_ya.p, ctx->sur_yb.p, 1.0f / sur->out_scale, sur->err_calib, float(tol),
                            status, harm_out, err_out, used_solver, ctx->sur_list.p, ctx->sur_count.p, s));
  int32_t cnt = 0;
  FPN_HIP(hipMemcpyAsync(&cnt, ctx->sur_count.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FPN_HIP(hipStreamSynchronize(s));
  if (n_fallback) *n_fallback = cnt;
  if (cnt == 0) return FPN_OK;
  if (!drive) return fail(FPN_E_ARG, "drive is NULL but instances need the solver");
  // the solver's launch plan needs the fallback instances' degrees on the host
  std::vector<int32_t> list(cnt), Lsub(cnt);
  FPN_HIP(hipMemcpy(list.data(), ctx->sur_list.p, cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int j = 0; j < cnt; ++j) Lsub[j] = batch->L[list[j]];
  FPN_HIP(ctx->sur_g.ensure(size_t(cnt) * 11));
  const int per = 2 * (Kh + 1) * 2;
  FPN_HIP(ctx->sur_h.ensure(size_t(cnt) * per));
  FPN_HIP(ctx->sur_st.ensure(size_t(cnt)));
  FPN_HIP(fpn::sur::gather(cnt, ctx->sur_list.p, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp,
                           batch->easy_axis, batch->offset, ctx->sur_g.p, s));
  fpn_batch sub;
  double* g = ctx->sur_g.p;
  sub.D = g;
  sub.Ms = g + cnt;
  sub.K = g + 2 * int64_t(cnt);
  sub.alpha = g + 3 * int64_t(cnt);
  sub.temp = g + 4 * int64_t(cnt);
  sub.easy_axis = g + 5 * int64_t(cnt);
  sub.offset = g + 8 * int64_t(cnt);
  sub.L = Lsub.data();
  fpn_solve_opts o = *opts;
  o.flags = FPN_OUT_HARM;
  if (fpn_status e = fpn_solve(ctx, drive, &o, &sub, cnt, nullptr, nullptr, ctx->sur_h.p, ctx->sur_st.p, stream)) return e;
  FPN_HIP(fpn::sur::scatter(cnt, per, ctx->sur_list.p, ctx->sur_h.p, ctx->sur_st.p, harm_out, status, err_out, s));
  // the call is synchronous as a whole (the fallback count had to be read)
  FPN_HIP(hipStreamSynchronize(s));
  return FPN_OK;
}

}  // extern "C"
