// C ABI of the surrogate model handle (include/fpn.h, "surrogate model" section): a two-member
// ensemble with its output scale and error calibration that can be trained, evaluated, written to a
// file and read back.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fpn.h"
#include "capi_internal.hpp"
#include "surrogate.hpp"

using namespace fpn_internal;

namespace {

constexpr char kMagic[8] = {'F', 'P', 'N', 'S', 'U', 'R', '1', '\0'};
constexpr uint32_t kVersion = 2;

// FNV-1a over the bytes written before the trailer (detects truncated or altered files)
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t k = 0; k < n; ++k) h = (h ^ c[k]) * 1099511628211ull;
  }
};

struct Writer {
  FILE* f;
  Fnv sum;
  bool ok = true;
  void put(const void* p, size_t n) {
    if (!ok) return;
    ok = std::fwrite(p, 1, n, f) == n;
    sum.add(p, n);
  }
};

struct Reader {
  FILE* f;
  Fnv sum;
  bool ok = true;
  void get(void* p, size_t n) {
    if (!ok) return;
    ok = std::fread(p, 1, n, f) == n;
    if (ok) sum.add(p, n);
  }
};

fpn_status free_model(fpn_sur_model m) {
  for (fpn_mlp* arr : {m->net, m->res})
    for (int k = 0; k < 2; ++k)
      if (arr[k]) {
        fpn_mlp_destroy(arr[k]);
        arr[k] = nullptr;
      }
  m->r.release();
  m->ya.release();
  m->yb.release();
  m->t.release();
  delete m;
  return FPN_OK;
}

}  // namespace

extern "C" {

fpn_status fpn_surrogate_init(fpn_ctx ctx, int32_t n_layers, const int32_t* widths, const uint64_t seeds[2],
                              fpn_sur_model* out) {
  if (!ctx || !widths || !seeds || !out) return fail(FPN_E_ARG, "NULL argument");
  *out = nullptr;
  auto* m = new fpn_sur_model_s();
  m->device = ctx->device;
  for (int k = 0; k < 2; ++k)
    if (fpn_status e = fpn_mlp_create(ctx, n_layers, widths, seeds[k], &m->net[k])) {
      free_model(m);
      return e;
    }
  *out = m;
  return FPN_OK;
}

fpn_status fpn_surrogate_destroy(fpn_sur_model m) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  (void)hipSetDevice(m->device);
  return free_model(m);
}

fpn_status fpn_surrogate_member(fpn_sur_model m, int32_t k, fpn_mlp* out) {
  if (!m || !out || k < 0 || k > 3) return fail(FPN_E_ARG, "NULL model or output, or member not in 0..3");
  if (k >= 2 && !m->res[0]) return fail(FPN_E_ARG, "the model has no residual stage");
  *out = k < 2 ? m->net[k] : m->res[k - 2];
  return FPN_OK;
}

fpn_status fpn_surrogate_add_residual(fpn_ctx ctx, fpn_sur_model m, const uint64_t seeds[2]) {
  if (!ctx || !m || !seeds) return fail(FPN_E_ARG, "NULL argument");
  if (m->res[0]) return fail(FPN_E_ARG, "the model already has a residual stage");
  if (m->device != ctx->device) return fail(FPN_E_ARG, "model on another device");
  const std::vector<int>& w = m->net[0]->w;
  std::vector<int32_t> w32(w.begin(), w.end());
  for (int k = 0; k < 2; ++k)
    if (fpn_status e = fpn_mlp_create(ctx, int32_t(w32.size()) - 1, w32.data(), seeds[k], &m->res[k])) {
      if (m->res[0]) fpn_mlp_destroy(m->res[0]);
      m->res[0] = m->res[1] = nullptr;
      return e;
    }
  m->res_scale = 1.0f;
  return FPN_OK;
}

fpn_status fpn_surrogate_set_residual_scale(fpn_sur_model m, float res_scale) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  if (!m->res[0]) return fail(FPN_E_ARG, "the model has no residual stage");
  if (!(res_scale > 0.0f) || !std::isfinite(res_scale)) return fail(FPN_E_ARG, "res_scale must be finite and > 0");
  m->res_scale = res_scale;
  return FPN_OK;
}

fpn_status fpn_surrogate_set_scales(fpn_sur_model m, float out_scale, float err_calib) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  if (!(out_scale > 0.0f) || !std::isfinite(out_scale) || !(err_calib > 0.0f) || !std::isfinite(err_calib))
    return fail(FPN_E_ARG, "out_scale and err_calib must be finite and > 0");
  m->out_scale = out_scale;
  m->err_calib = err_calib;
  return FPN_OK;
}

fpn_status fpn_surrogate_view(fpn_sur_model m, fpn_surrogate* view) {
  if (!m || !view) return fail(FPN_E_ARG, "NULL argument");
  view->net[0] = m->net[0];
  view->net[1] = m->net[1];
  view->out_scale = m->out_scale;
  view->err_calib = m->err_calib;
  view->res[0] = m->res[0];
  view->res[1] = m->res[1];
  view->res_scale = m->res_scale;
  return FPN_OK;
}

fpn_status fpn_surrogate_infer(fpn_ctx ctx, fpn_sur_model m, const float* x, int64_t n, float* y, float* err_est,
                               void* stream) {
  if (!ctx || !m) return fail(FPN_E_ARG, "NULL context or model");
  if (m->device != ctx->device) return fail(FPN_E_ARG, "model on another device");
  if (n < 0 || n > (int64_t(1) << 30)) return fail(FPN_E_ARG, "n outside [0, 2^30]");
  if (n == 0) return FPN_OK;
  if (!x || (!y && !err_est)) return fail(FPN_E_ARG, "NULL x, or neither y nor err_est");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(m->device));
  const int W = m->net[0]->w.back();
  FPN_HIP(m->ya.ensure(size_t(n) * W));
  FPN_HIP(m->yb.ensure(size_t(n) * W));
  if (fpn_status e = fpn_mlp_forward(m->net[0], x, n, m->ya.p, stream)) return e;
  if (fpn_status e = fpn_mlp_forward(m->net[1], x, n, m->yb.p, stream)) return e;
  if (m->res[0]) {  // member k's output += res[k](x) / res_scale
    FPN_HIP(m->r.ensure(size_t(n) * W));
    float* ys[2] = {m->ya.p, m->yb.p};
    for (int k = 0; k < 2; ++k) {
      if (fpn_status e = fpn_mlp_forward(m->res[k], x, n, m->r.p, stream)) return e;
      FPN_HIP(fpn::sur::axpy(n * W, 1.0f / m->res_scale, m->r.p, ys[k], s));
    }
  }
  FPN_HIP(fpn::sur::mean_spread(n, W, m->ya.p, m->yb.p, 1.0f / m->out_scale, m->err_calib, y, err_est, s));
  return FPN_OK;
}

fpn_status fpn_surrogate_train_step(fpn_ctx ctx, fpn_sur_model m, const float* x, const float* y_true, int64_t n,
                                    float lr, double* loss_out, void* stream) {
  if (!ctx || !m) return fail(FPN_E_ARG, "NULL context or model");
  if (m->device != ctx->device) return fail(FPN_E_ARG, "model on another device");
  if (n < 1 || n > (int64_t(1) << 22)) return fail(FPN_E_ARG, "n outside [1, 2^22]");
  if (!x || !y_true) return fail(FPN_E_ARG, "NULL x or y_true");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(FPN_E_ARG, "lr must be finite and > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(m->device));
  const int W = m->net[0]->w.back();
  FPN_HIP(m->t.ensure(size_t(n) * W));
  FPN_HIP(fpn::sur::scale(n * W, y_true, m->out_scale, m->t.p, s));
  for (int k = 0; k < 2; ++k)
    if (fpn_status e = fpn_mlp_train_step(m->net[k], x, m->t.p, n, lr, loss_out ? loss_out + k : nullptr, stream))
      return e;
  return FPN_OK;
}

fpn_status fpn_surrogate_save(fpn_sur_model m, const char* path) {
  if (!m || !path) return fail(FPN_E_ARG, "NULL model or path");
  FPN_HIP(hipSetDevice(m->device));
  FPN_HIP(hipDeviceSynchronize());
  const fpn_mlp a = m->net[0];
  const int32_t nl = a->nl;
  const int64_t np = a->nparam;
  const int w0 = a->w[0];
  std::vector<float> buf(static_cast<size_t>(np)), nrm(2 * static_cast<size_t>(w0));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(FPN_E_IO, std::string("cannot open ") + path + " for writing");
  Writer wr{f};
  wr.put(kMagic, sizeof kMagic);
  wr.put(&kVersion, sizeof kVersion);
  wr.put(&nl, sizeof nl);
  for (int l = 0; l <= nl; ++l) {
    const int32_t wl = a->w[l];
    wr.put(&wl, sizeof wl);
  }
  wr.put(&m->out_scale, sizeof(float));
  wr.put(&m->err_calib, sizeof(float));
  const int32_t has_res = m->res[0] ? 1 : 0;
  wr.put(&has_res, sizeof has_res);
  wr.put(&m->res_scale, sizeof(float));
  for (int k = 0; k < (has_res ? 4 : 2) && wr.ok; ++k) {
    const fpn_mlp net = k < 2 ? m->net[k] : m->res[k - 2];
    const int64_t t = net->t;
    wr.put(&t, sizeof t);
    if (hipMemcpy(nrm.data(), net->norm.p, nrm.size() * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
      std::fclose(f);
      return fail(FPN_E_DEVICE, "reading the input normalisation");
    }
    wr.put(nrm.data(), nrm.size() * sizeof(float));
    for (const float* src : {net->P.p, net->Am.p, net->Av.p}) {
      if (hipMemcpy(buf.data(), src, size_t(np) * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        std::fclose(f);
        return fail(FPN_E_DEVICE, "reading the parameters");
      }
      wr.put(buf.data(), size_t(np) * sizeof(float));
    }
  }
  const uint64_t sum = wr.sum.h;
  if (wr.ok) wr.ok = std::fwrite(&sum, sizeof sum, 1, f) == 1;
  const bool closed = std::fclose(f) == 0;
  if (!wr.ok || !closed) return fail(FPN_E_IO, std::string("writing ") + path + " failed");
  return FPN_OK;
}

fpn_status fpn_surrogate_create(fpn_ctx ctx, const char* weights_path, fpn_sur_model* out) {
  if (!ctx || !weights_path || !out) return fail(FPN_E_ARG, "NULL argument");
  *out = nullptr;
  FILE* f = std::fopen(weights_path, "rb");
  if (!f) return fail(FPN_E_IO, std::string("cannot open ") + weights_path);
  Reader rd{f};
  auto bad = [&](const std::string& why) {
    std::fclose(f);
    return fail(FPN_E_IO, std::string(weights_path) + ": " + why);
  };
  char magic[8];
  uint32_t ver = 0;
  int32_t nl = 0;
  rd.get(magic, sizeof magic);
  rd.get(&ver, sizeof ver);
  rd.get(&nl, sizeof nl);
  if (!rd.ok || std::memcmp(magic, kMagic, sizeof kMagic) != 0) return bad("not a surrogate model file");
  if (ver != 1 && ver != kVersion) return bad("unsupported version");
  if (nl < 1 || nl > 16) return bad("layer count outside [1, 16]");
  std::vector<int32_t> w(nl + 1);
  rd.get(w.data(), w.size() * sizeof(int32_t));
  float scales[2];
  rd.get(scales, sizeof scales);
  int32_t has_res = 0;
  float res_scale = 1.0f;
  if (ver >= 2) {
    rd.get(&has_res, sizeof has_res);
    rd.get(&res_scale, sizeof res_scale);
  }
  if (!rd.ok) return bad("truncated header");
  if (has_res != 0 && has_res != 1) return bad("bad residual flag");
  const uint64_t seeds[2] = {0, 0};
  fpn_sur_model m = nullptr;
  if (fpn_status e = fpn_surrogate_init(ctx, nl, w.data(), seeds, &m)) {
    std::fclose(f);
    return e;
  }
  if (fpn_status e = fpn_surrogate_set_scales(m, scales[0], scales[1])) {
    free_model(m);
    std::fclose(f);
    return e;
  }
  if (has_res) {
    if (fpn_status e = fpn_surrogate_add_residual(ctx, m, seeds)) {
      free_model(m);
      std::fclose(f);
      return e;
    }
    if (fpn_status e = fpn_surrogate_set_residual_scale(m, res_scale)) {
      free_model(m);
      std::fclose(f);
      return e;
    }
  }
  const int64_t np = m->net[0]->nparam;
  std::vector<float> buf(static_cast<size_t>(np)), nrm(2 * static_cast<size_t>(w[0]));
  for (int k = 0; k < (has_res ? 4 : 2); ++k) {
    const fpn_mlp net = k < 2 ? m->net[k] : m->res[k - 2];
    int64_t t = 0;
    rd.get(&t, sizeof t);
    rd.get(nrm.data(), nrm.size() * sizeof(float));
    if (!rd.ok || t < 0) {
      free_model(m);
      return bad("truncated member");
    }
    net->t = t;
    hipError_t e = hipMemcpy(net->norm.p, nrm.data(), nrm.size() * sizeof(float), hipMemcpyHostToDevice);
    for (float* dst : {net->P.p, net->Am.p, net->Av.p}) {
      rd.get(buf.data(), size_t(np) * sizeof(float));
      if (!rd.ok) break;
      if (e == hipSuccess) e = hipMemcpy(dst, buf.data(), size_t(np) * sizeof(float), hipMemcpyHostToDevice);
    }
    if (!rd.ok) {
      free_model(m);
      return bad("truncated parameters");
    }
    if (e != hipSuccess) {
      free_model(m);
      std::fclose(f);
      return fail(FPN_E_DEVICE, hipGetErrorString(e));
    }
    net->dirty = true;
  }
  const uint64_t expect = rd.sum.h;
  uint64_t sum = 0;
  const bool got = std::fread(&sum, sizeof sum, 1, f) == 1;
  char extra;
  const bool tail = std::fread(&extra, 1, 1, f) == 1;
  std::fclose(f);
  if (!got || sum != expect || tail) {
    free_model(m);
    return fail(FPN_E_IO, std::string(weights_path) + ": checksum mismatch or trailing bytes");
  }
  *out = m;
  return FPN_OK;
}

}  // extern "C"
