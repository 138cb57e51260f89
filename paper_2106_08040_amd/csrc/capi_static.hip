// fpn_solve_static: the solve of one degree L <= 16 without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).
//
// Every per-call buffer (instance parameters, instance list, launch queue counter, FP64 stationary
// states and their block workspace, the samples when the caller does not want them) is carved out of
// `scratch`, a fixed device array of this translation unit.  In host code the array's name is a
// stand-in, not a device address: its address on each GPU is looked up once with hipGetSymbolAddress
// (static_scratch_init, called by fpn_create with the device current) and only that pointer is used.
// All calls on one GPU share the array and keep the last call's contents: the queue counter is
// cleared by a fill kernel at the start of every call, everything else is written before it is read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "capi_internal.hpp"
#include "kernels.hpp"
#include "stepper_common.hpp"

namespace {

constexpr int kMaxNp = (16 + 1) * (16 + 1) + 1;  // vector length of L = 16 in the |m| block order
constexpr int64_t kMaxInvDoubles = 6308;         // sum of squared block sizes at L = 16 (stationary workspace)
constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
// byte offsets of the parts of the array
constexpr size_t kOffIp = 0;
constexpr size_t kOffIdx = kOffIp + align_up(sizeof(fpn::InstParams) * FPN_STATIC_MAX_N);
constexpr size_t kOffQueue = kOffIdx + align_up(sizeof(int32_t) * FPN_STATIC_MAX_N);
constexpr size_t kOffC0 = kOffQueue + align_up(sizeof(int32_t));
constexpr size_t kOffInv = kOffC0 + align_up(sizeof(double) * kMaxNp * FPN_STATIC_MAX_N);
constexpr size_t kOffM = kOffInv + align_up(sizeof(double) * kMaxInvDoubles * FPN_STATIC_MAX_N);
constexpr size_t kBytes = kOffM + align_up(sizeof(float) * 3 * FPN_STATIC_MAX_NS * FPN_STATIC_MAX_N);
static_assert(kBytes <= FPN_STATIC_SCRATCH_BYTES, "static scratch layout exceeds its declared size");

static __device__ __align__(256) unsigned char scratch[FPN_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
void* g_addr[64] = {nullptr};  // device address of `scratch` per GPU

__global__ void iota_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

}  // namespace

namespace fpn_internal {

fpn_status static_scratch_init(int device) {
  if (device < 0 || device >= 64) return fail(FPN_E_RANGE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_addr[device]) return FPN_OK;
  void* ptr = nullptr;
  FPN_HIP(hipSetDevice(device));
  FPN_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(FPN_E_DEVICE, "hipGetSymbolAddress returned NULL for the static scratch");
  g_addr[device] = ptr;
  return FPN_OK;
}

}  // namespace fpn_internal

using fpn_internal::fail;

extern "C" fpn_status fpn_solve_static(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                                       const fpn_batch* batch, int64_t n, float* m_out, float* harm_out,
                                       int32_t* status, void* stream_) {
  if (!ctx) return fail(FPN_E_ARG, "ctx is NULL");
  if (n < 0) return fail(FPN_E_ARG, "n < 0");
  if (fpn_status s = fpn_internal::validate_solve_opts(drive, opts)) return s;
  if (n == 0) return FPN_OK;
  if (fpn_status s = fpn_internal::validate_solve_outputs(opts, m_out, harm_out, status, n)) return s;
  if (opts->flags & FPN_OUT_DMDT) return fail(FPN_E_ARG, "fpn_solve_static has no dm/dt output");
  if (fpn_status s = fpn_internal::validate_solve_batch(batch, n)) return s;
  if (n > FPN_STATIC_MAX_N) return fail(FPN_E_RANGE, "fpn_solve_static: n > FPN_STATIC_MAX_N");
  const int Ns = opts->samples_per_period;
  if (Ns > FPN_STATIC_MAX_NS) return fail(FPN_E_RANGE, "fpn_solve_static: samples_per_period > FPN_STATIC_MAX_NS");
  const int L = batch->L[0];
  for (int64_t i = 1; i < n; ++i)
    if (batch->L[i] != L) return fail(FPN_E_ARG, "fpn_solve_static: every instance must have the same L");
  if (L > 16) return fail(FPN_E_RANGE, "fpn_solve_static: L > 16");
  std::lock_guard<std::mutex> lk(ctx->mu);
  // tables and twiddles are looked up, never built here (building them allocates)
  auto ti = ctx->tables.find(L);
  if (ti == ctx->tables.end())
    return fail(FPN_E_ARG, "fpn_solve_static: no operator tables for this L in the context (run fpn_solve first)");
  const fpn::DevTables& t = ti->second.t;
  const double2* tw = nullptr;
  if (opts->flags & FPN_OUT_HARM) {
    auto wi = ctx->twiddles.find(Ns);
    if (wi == ctx->twiddles.end())
      return fail(FPN_E_ARG, "fpn_solve_static: no twiddle table for this N_s in the context (run fpn_solve first)");
    tw = wi->second.p;
  }
  const int waves_cfg = ctx->stepper_waves[L];
  const int occ_key = L + 10000 * waves_cfg;
  auto oi = ctx->occupancy.find(occ_key);
  int waves = 0, blocks = 0;
  if (oi != ctx->occupancy.end()) {
    waves = oi->second.first;
    blocks = oi->second.second;
  } else {
    FPN_HIP(fpn::stepper_occupancy(L, t, false, waves_cfg, &waves, &blocks));
  }
  if (blocks < 1) return fail(FPN_E_DEVICE, "stepper configuration does not fit on a compute unit");
  int cus = ctx->cus;
  if (cus == 0) FPN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    base = static_cast<unsigned char*>(g_addr[ctx->device]);
  }
  if (!base) return fail(FPN_E_DEVICE, "static scratch address not initialised for this device");

  hipStream_t stream = reinterpret_cast<hipStream_t>(stream_);
  FPN_HIP(hipSetDevice(ctx->device));
  auto* ip = reinterpret_cast<fpn::InstParams*>(base + kOffIp);
  auto* idx = reinterpret_cast<int32_t*>(base + kOffIdx);
  auto* queue = reinterpret_cast<int32_t*>(base + kOffQueue);
  auto* c0 = reinterpret_cast<double*>(base + kOffC0);
  auto* wsinv = reinterpret_cast<double*>(base + kOffInv);
  float* msamp = (opts->flags & FPN_OUT_M) ? m_out : reinterpret_cast<float*>(base + kOffM);
  const int nn = int(n);

  fpn::launch_fill_i32(queue, 1, 0, stream);
  hipLaunchKernelGGL(iota_kernel, dim3((nn + 255) / 256), dim3(256), 0, stream, idx, nn);
  fpn::launch_instance_prep(n, batch->D, batch->Ms, batch->K, batch->alpha, batch->temp, batch->easy_axis,
                            batch->offset, ip, status, stream);
  FPN_HIP(hipGetLastError());
  double3 d0;
  d0.x = drive->amp[0] * std::cos(drive->phase[0]);
  d0.y = drive->amp[1] * std::cos(drive->phase[1]);
  d0.z = drive->amp[2] * std::cos(drive->phase[2]);
  fpn::launch_stationary(t, idx, nn, ip, nullptr, d0, c0, t.Np, wsinv, status, stream);
  FPN_HIP(hipGetLastError());
  fpn::StepLaunch sl;
  sl.ip = ip;
  sl.inst_idx = idx;
  sl.n_inst = nn;
  sl.c0 = c0;
  sl.c_stride = t.Np;
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
  sl.msamp = msamp;
  sl.status = status;
  sl.steps_out = nullptr;
  sl.queue = queue;
  sl.grid = std::max(1, std::min((nn + waves - 1) / waves, blocks * cus));
  sl.waves = waves_cfg;
  FPN_HIP(fpn::launch_stepper(L, sl, t, nullptr, stream));
  if (opts->flags & FPN_OUT_HARM) {
    const int nch = (opts->flags & FPN_HARM_Z) ? 3 : 2;
    fpn::launch_harmonics(msamp, Ns, opts->n_harm, nch, drive->period, tw, harm_out, status, n, stream);
    FPN_HIP(hipGetLastError());
  }
  return FPN_OK;
}
