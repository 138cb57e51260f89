// C ABI of the surrogate network (include/fpn.h, "surrogate network" section): parameter
// storage, forward, gradient and Adam training step on one device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fpn.h"
#include "capi_internal.hpp"
#include "mlp.hpp"

using namespace fpn_internal;

namespace {

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

fpn_status ensure_work(fpn_mlp m, int64_t rows, bool train) {
  const int nl = m->nl;
  m->act.resize(nl);
  m->act_lo.resize(nl);
  m->actT.resize(nl);
  m->z.resize(nl);
  if (rows <= m->rows_cap && (!train || m->train_cap)) return FPN_OK;
  rows = std::max(rows, m->rows_cap);
  for (int l = 0; l < nl; ++l) {
    FPN_HIP(m->act[l].ensure(size_t(rows) * m->inpad[l]));
    FPN_HIP(m->act_lo[l].ensure(size_t(rows) * m->inpad[l]));
    if (train) {
      FPN_HIP(m->actT[l].ensure(size_t(rows) * m->inpad[l]));
      if (l > 0) FPN_HIP(m->z[l].ensure(size_t(rows) * m->inpad[l]));
    }
  }
  FPN_HIP(m->y.ensure(size_t(rows) * m->w[nl]));
  if (train) {
    int wmax = 0;
    for (int v : m->w) wmax = std::max(wmax, v);
    for (int k = 0; k < 2; ++k) {
      FPN_HIP(m->dz[k].ensure(size_t(rows) * wmax));
      FPN_HIP(m->dzT[k].ensure(size_t(rows) * wmax));
    }
    FPN_HIP(m->loss.ensure(1));
  }
  m->rows_cap = rows;
  m->train_cap = m->train_cap || train;
  return FPN_OK;
}

fpn_status refresh_weights(fpn_mlp m, hipStream_t s) {
  if (!m->dirty) return FPN_OK;
  for (int l = 0; l < m->nl; ++l)
    FPN_HIP(fpn::mlp::cast_weights(m->P.p + m->offW[l], m->w[l + 1], m->w[l], m->inpad[l], m->Wb[l].p, m->Wt[l].p, s));
  m->dirty = false;
  return FPN_OK;
}

// Forward over `rows` rows of x (n real rows); training keeps transposes and pre-activations.  The
// activations go from layer to layer as BF16 pairs (act + act_lo); the transposed copies the weight
// gradients read stay single BF16.
fpn_status forward(fpn_mlp m, const float* x, int64_t n, int64_t rows, bool train, float* y_out, hipStream_t s) {
  const int nl = m->nl;
  FPN_HIP(fpn::mlp::cast_input(x, n, rows, m->w[0], m->inpad[0], m->norm.p, m->norm.p + m->w[0], m->act[0].p,
                               train ? m->actT[0].p : nullptr, rows, s, m->act_lo[0].p));
  for (int l = 0; l < nl; ++l) {
    fpn::mlp::GemmArgs g{};
    g.A = m->act[l].p;
    g.Alo = m->act_lo[l].p;
    g.lda = m->inpad[l];
    g.B = m->Wb[l].p;
    g.ldb = m->inpad[l];
    g.M = int(rows);
    g.N = m->w[l + 1];
    g.K = m->inpad[l];
    g.bias = m->P.p + m->offB[l];
    if (l < nl - 1) {
      g.C = m->act[l + 1].p;
      g.Clo = m->act_lo[l + 1].p;
      g.ldc = m->inpad[l + 1];
      g.Ct = train ? m->actT[l + 1].p : nullptr;
      g.ldct = rows;
      g.z_out = train ? m->z[l + 1].p : nullptr;
      g.ldz = m->inpad[l + 1];
      FPN_HIP(fpn::mlp::gemm_nt(fpn::mlp::kEpiBiasGelu, g, 1, s));
    } else {
      g.Cf = y_out;
      g.ldc = m->w[nl];
      FPN_HIP(fpn::mlp::gemm_nt(fpn::mlp::kEpiBias, g, 1, s));
    }
  }
  return FPN_OK;
}

// Gradient of the mean-square loss into m->G (zeroed first) and the loss sum into m->loss.
fpn_status gradient(fpn_mlp m, const float* x, const float* t, int64_t n, hipStream_t s) {
  const int nl = m->nl;
  const int64_t rows = (n + 31) / 32 * 32;
  if (fpn_status e = ensure_work(m, rows, true)) return e;
  if (fpn_status e = refresh_weights(m, s)) return e;
  if (fpn_status e = forward(m, x, n, rows, true, m->y.p, s)) return e;
  FPN_HIP(fpn::mlp::fill(m->G.p, m->nparam, 0.0f, s));
  // zero the FP64 loss accumulator with a kernel (no memset nodes under graph capture)
  FPN_HIP(fpn::mlp::fill(reinterpret_cast<float*>(m->loss.p), 2, 0.0f, s));
  int cur = 0;
  FPN_HIP(fpn::mlp::loss_grad(m->y.p, t, n, rows, m->w[nl], m->dz[cur].p, m->dzT[cur].p, rows, m->loss.p, s));
  for (int l = nl - 1; l >= 0; --l) {
    const int out = m->w[l + 1], in = m->w[l];
    {  // dW_l += dz^T a_l
      fpn::mlp::GemmArgs g{};
      g.A = m->dzT[cur].p;
      g.lda = rows;
      g.B = m->actT[l].p;
      g.ldb = rows;
      g.M = out;
      g.N = in;
      g.K = int(rows);
      g.Cf = m->G.p + m->offW[l];
      g.ldc = in;
      const int tiles = ((out + 127) / 128) * ((in + 127) / 128);
      const int ks = int(std::max<int64_t>(1, std::min<int64_t>(rows / 32, (1024 + tiles - 1) / tiles)));
      FPN_HIP(fpn::mlp::gemm_nt(fpn::mlp::kEpiAtomic, g, ks, s));
    }
    FPN_HIP(fpn::mlp::bias_grad(m->dzT[cur].p, rows, rows, out, m->G.p + m->offB[l], s));
    if (l > 0) {  // dz_{l-1} = (dz W_l) * gelu'(z_l)
      fpn::mlp::GemmArgs g{};
      g.A = m->dz[cur].p;
      g.lda = out;
      g.B = m->Wt[l].p;
      g.ldb = out;
      g.M = int(rows);
      g.N = in;
      g.K = out;
      g.C = m->dz[cur ^ 1].p;
      g.ldc = in;
      g.Ct = m->dzT[cur ^ 1].p;
      g.ldct = rows;
      g.zin = m->z[l].p;
      g.ldz = m->inpad[l];
      FPN_HIP(fpn::mlp::gemm_nt(fpn::mlp::kEpiGeluGrad, g, 1, s));
      cur ^= 1;
    }
  }
  return FPN_OK;
}

}  // namespace

extern "C" {

fpn_status fpn_mlp_create(fpn_ctx ctx, int32_t n_layers, const int32_t* widths, uint64_t seed, fpn_mlp* out) {
  if (!ctx || !widths || !out) return fail(FPN_E_ARG, "NULL argument");
  *out = nullptr;
  if (n_layers < 1 || n_layers > 16) return fail(FPN_E_ARG, "n_layers must be in [1, 16]");
  for (int l = 0; l <= n_layers; ++l)
    if (widths[l] < 1 || widths[l] > 8192) return fail(FPN_E_ARG, "layer width outside [1, 8192]");
  for (int l = 1; l < n_layers; ++l)
    if (widths[l] % 32 != 0) return fail(FPN_E_ARG, "hidden widths must be multiples of 32");
  if (widths[n_layers] % 32 != 0) return fail(FPN_E_ARG, "the output width must be a multiple of 32");
  FPN_HIP(hipSetDevice(ctx->device));
  auto* m = new fpn_mlp_s();
  m->device = ctx->device;
  m->nl = n_layers;
  m->w.assign(widths, widths + n_layers + 1);
  m->inpad.resize(n_layers + 1);
  for (int l = 0; l <= n_layers; ++l) m->inpad[l] = (m->w[l] + 31) / 32 * 32;
  int64_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->offW.push_back(off);
    off += int64_t(m->w[l + 1]) * m->w[l];
    m->offB.push_back(off);
    off += m->w[l + 1];
  }
  m->nparam = off;
  // default initialisation: U(-1/sqrt(in), 1/sqrt(in)) for weights and biases
  std::vector<float> h(off);
  uint64_t st = seed;
  for (int l = 0; l < n_layers; ++l) {
    const double sc = 1.0 / std::sqrt(double(m->w[l]));
    for (int64_t e = m->offW[l]; e < m->offB[l] + m->w[l + 1]; ++e)
      h[e] = float((double(splitmix(st) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0) * sc);
  }
  auto cleanup = [&](fpn_status s) {
    for (auto* b : {&m->P, &m->G, &m->Am, &m->Av, &m->norm}) b->release();
    for (auto& b : m->Wb) b.release();
    for (auto& b : m->Wt) b.release();
    delete m;
    return s;
  };
  hipError_t e = m->P.ensure(off);
  if (e == hipSuccess) e = m->G.ensure(off);
  if (e == hipSuccess) e = m->Am.ensure(off);
  if (e == hipSuccess) e = m->Av.ensure(off);
  if (e == hipSuccess) e = m->norm.ensure(2 * size_t(m->w[0]));
  if (e != hipSuccess) return cleanup(fail(FPN_E_NOMEM, hipGetErrorString(e)));
  std::vector<float> nrm(2 * m->w[0]);
  for (int j = 0; j < m->w[0]; ++j) {
    nrm[j] = 0.0f;
    nrm[m->w[0] + j] = 1.0f;
  }
  std::vector<float> zeros(off, 0.0f);
  e = hipMemcpy(m->P.p, h.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->Am.p, zeros.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->Av.p, zeros.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->norm.p, nrm.data(), nrm.size() * sizeof(float), hipMemcpyHostToDevice);
  m->Wb.resize(n_layers);
  m->Wt.resize(n_layers);
  for (int l = 0; l < n_layers && e == hipSuccess; ++l) {
    e = m->Wb[l].ensure(size_t(m->w[l + 1]) * m->inpad[l]);
    if (e == hipSuccess) e = m->Wt[l].ensure(size_t(m->w[l + 1]) * m->inpad[l]);
  }
  if (e != hipSuccess) return cleanup(fail(FPN_E_DEVICE, hipGetErrorString(e)));
  *out = m;
  return FPN_OK;
}

fpn_status fpn_mlp_destroy(fpn_mlp m) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (auto* b : {&m->P, &m->G, &m->Am, &m->Av, &m->norm, &m->y}) b->release();
  for (auto& b : m->Wb) b.release();
  for (auto& b : m->Wt) b.release();
  for (auto& b : m->act) b.release();
  for (auto& b : m->act_lo) b.release();
  for (auto& b : m->actT) b.release();
  for (auto& b : m->z) b.release();
  for (int k = 0; k < 2; ++k) {
    m->dz[k].release();
    m->dzT[k].release();
  }
  m->loss.release();
  delete m;
  return FPN_OK;
}

int64_t fpn_mlp_num_params(fpn_mlp m) { return m ? m->nparam : -1; }

fpn_status fpn_mlp_shape(fpn_mlp m, int32_t* n_layers, int32_t* widths) {
  if (!m || !n_layers) return fail(FPN_E_ARG, "NULL argument");
  *n_layers = m->nl;
  if (widths)
    for (int l = 0; l <= m->nl; ++l) widths[l] = m->w[l];
  return FPN_OK;
}

fpn_status fpn_mlp_params(fpn_mlp m, float* dst, const float* src, void* stream) {
  if (!m || (!dst && !src)) return fail(FPN_E_ARG, "NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(m->device));
  if (src) {
    FPN_HIP(hipMemcpyAsync(m->P.p, src, m->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    m->dirty = true;
  }
  if (dst) FPN_HIP(hipMemcpyAsync(dst, m->P.p, m->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  return FPN_OK;
}

fpn_status fpn_mlp_set_input_norm(fpn_mlp m, const float* mean, const float* stdev) {
  if (!m || !mean || !stdev) return fail(FPN_E_ARG, "NULL argument");
  std::vector<float> nrm(2 * m->w[0]);
  for (int j = 0; j < m->w[0]; ++j) {
    if (!(stdev[j] > 0.0f) || !std::isfinite(stdev[j]) || !std::isfinite(mean[j]))
      return fail(FPN_E_ARG, "input scale must be finite and > 0");
    nrm[j] = mean[j];
    nrm[m->w[0] + j] = 1.0f / stdev[j];
  }
  FPN_HIP(hipSetDevice(m->device));
  FPN_HIP(hipDeviceSynchronize());
  FPN_HIP(hipMemcpy(m->norm.p, nrm.data(), nrm.size() * sizeof(float), hipMemcpyHostToDevice));
  return FPN_OK;
}

fpn_status fpn_mlp_forward(fpn_mlp m, const float* x, int64_t n, float* y, void* stream) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  if (n < 0 || n > (int64_t(1) << 30)) return fail(FPN_E_ARG, "n outside [0, 2^30]");
  if (n == 0) return FPN_OK;
  if (!x || !y) return fail(FPN_E_ARG, "NULL x or y");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(m->device));
  if (fpn_status e = refresh_weights(m, s)) return e;
  const int64_t chunk = int64_t(1) << 17;
  if (fpn_status e = ensure_work(m, std::min(n, chunk), false)) return e;
  for (int64_t b = 0; b < n; b += chunk) {
    const int64_t c = std::min(chunk, n - b);
    if (fpn_status e = forward(m, x + b * m->w[0], c, c, false, y + b * m->w[m->nl], s)) return e;
  }
  return FPN_OK;
}

fpn_status fpn_mlp_gradient(fpn_mlp m, const float* x, const float* t, int64_t n, float* grad, double* loss,
                            void* stream) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  if (n < 1 || n > (int64_t(1) << 22)) return fail(FPN_E_ARG, "n outside [1, 2^22]");
  if (!x || !t) return fail(FPN_E_ARG, "NULL x or t");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FPN_HIP(hipSetDevice(m->device));
  if (fpn_status e = gradient(m, x, t, n, s)) return e;
  if (grad) FPN_HIP(hipMemcpyAsync(grad, m->G.p, m->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (loss) FPN_HIP(hipMemcpyAsync(loss, m->loss.p, sizeof(double), hipMemcpyDeviceToDevice, s));
  return FPN_OK;
}

fpn_status fpn_mlp_train_step(fpn_mlp m, const float* x, const float* t, int64_t n, float lr, double* loss,
                              void* stream) {
  if (!m) return fail(FPN_E_ARG, "NULL model");
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(FPN_E_ARG, "lr must be finite and > 0");
  if (fpn_status e = fpn_mlp_gradient(m, x, t, n, nullptr, loss, stream)) return e;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  m->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = float(1.0 - std::pow(0.9, double(m->t))), c2 = float(1.0 - std::pow(0.999, double(m->t)));
  FPN_HIP(fpn::mlp::adam(m->P.p, m->G.p, m->Am.p, m->Av.p, m->nparam, lr, b1, b2, 1e-8f, c1, c2, s));
  m->dirty = true;
  return FPN_OK;
}

}  // extern "C"
