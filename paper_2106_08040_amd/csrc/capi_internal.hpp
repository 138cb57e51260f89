// Private state and helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fpn.h"
#include "device_common.hpp"

namespace fpn_internal {

fpn_status fail(fpn_status s, const std::string& msg);
// argument checks of fpn_solve, shared with fpn_solve_static
fpn_status validate_solve_opts(const fpn_drive* drive, const fpn_solve_opts* opts);
fpn_status validate_solve_batch(const fpn_batch* batch, int64_t n);
fpn_status validate_solve_outputs(const fpn_solve_opts* opts, float* m_out, float* harm_out, int32_t* status,
                                  int64_t n);
// looks up the device address of fpn_solve_static's scratch array on `device` (once per device)
fpn_status static_scratch_init(int device);

#define FPN_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::fpn_internal::fail(e_ == hipErrorOutOfMemory ? FPN_E_NOMEM : FPN_E_DEVICE,  \
                                  std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  hipError_t ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

struct TableSet {
  fpn::DevTables t{};
  std::vector<void*> allocs;
};

}  // namespace fpn_internal

struct fpn_plan_s;

namespace fpn_internal {
// One |m|-degree bucket of a solve: instances [start, start + cnt) of the plan's order.
struct PlanGroup {
  int L = 0;
  int64_t start = 0;
  int cnt = 0;
  const fpn::DevTables* t = nullptr;
  int grid = 0;          // persistent workgroups of the stepper
  int waves = 0;         // instances per workgroup (0: the default for L)
  int64_t ws_off = 0;    // floats into the wide-layout workspace
  int64_t inv_off = 0;   // doubles into the stationary workspace
  int64_t tws_off = 0;   // floats into the tangent workspace
  double cost = 0.0;     // predicted work (for the launch order)
  double est = 0.0;      // predicted duration (per-step work x the longer of total steps / slots and the
                         // longest instance's steps), for the assignment to streams
  int stream = 0;        // side stream of the bucket (longest-first onto the least loaded stream)
  bool order = false;    // no cost hint and more instances than resident wavefronts: a plan launched
                         // again sorts the bucket's queue by the previous launch's step counts
};
void plan_release(fpn_plan_s* p);
}  // namespace fpn_internal

struct fpn_ctx_s {
  int device = 0;
  std::mutex mu;
  std::map<int, fpn_internal::TableSet> tables;
  // DFT twiddle tables, one per sample count N_s; a table is written once and kept until fpn_destroy,
  // so plans and captured graphs that hold its address stay valid whatever N_s later calls use
  std::map<int, fpn_internal::DevBuf<double2>> twiddles;
  fpn_internal::DevBuf<fpn::InstParams> ip;
  fpn_internal::DevBuf<double> c0;
  fpn_internal::DevBuf<double> wsinv;
  fpn_internal::DevBuf<float> msamp;
  fpn_internal::DevBuf<float> eq_m;     // equilibrium model: samples when the caller wants none
  fpn_internal::DevBuf<int32_t> idx;
  fpn_internal::DevBuf<int32_t> steps;
  fpn_internal::DevBuf<float> wide_ws;  // wide-layout stepper: block inverses and stage vectors
  int64_t steps_n = 0;
  // surrogate evaluation workspace
  fpn_internal::DevBuf<float> sur_x, sur_ya, sur_yb, sur_h, sur_r;
  fpn_internal::DevBuf<int32_t> sur_list, sur_count, sur_st;
  fpn_internal::DevBuf<double> sur_g;
  // model M2 dictionary matrix (transposed) and data vector, complex FP32 as float pairs
  fpn_internal::DevBuf<float> m2_mt, m2_y;
  // truncation estimate: the field of largest magnitude per instance
  fpn_internal::DevBuf<double> trunc_field;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
  double ms[4] = {0, 0, 0, 0};
  int64_t launches[4] = {0, 0, 0, 0};
  fpn_plan_s* solve_plan = nullptr;   // reused by fpn_solve
  fpn_plan_s* tangent_plan = nullptr; // reused by fpn_solve_tangent and fpn_adjoint
  fpn_plan_s* last_plan = nullptr;    // the one of the two used by the most recent call (fpn_last_steps)
  // (L, tangents, workgroup size) -> (waves per workgroup, workgroups per CU)
  std::map<int, std::pair<int, int>> occupancy;
  int cus = 0;
  int stepper_waves[25] = {0};  // workgroup size per degree (0: default), set by fpn_autotune
};

// A solve bound to its inputs and outputs: the degree buckets in launch order, the instance
// order within them, and every workspace the launch needs.
struct fpn_plan_s {
  fpn_ctx ctx = nullptr;
  fpn_drive drive{};
  fpn_solve_opts opts{};
  fpn_batch batch{};          // device pointers (the host L array is not kept)
  int64_t n = 0;
  float* m_out = nullptr;
  float* harm_out = nullptr;
  int32_t* status = nullptr;
  const double2* twiddle = nullptr;  // the context's table for this plan's N_s
  float* msamp = nullptr;     // m_out or the plan's own sample buffer
  float* dmdt = nullptr;      // dmdt_out of fpn_solve (null for plans and tangent solves)
  int64_t np_max = 0;
  std::vector<fpn_internal::PlanGroup> groups;
  std::vector<int32_t> order;  // host copy of the instance order
  fpn_internal::DevBuf<fpn::InstParams> ip;
  fpn_internal::DevBuf<double> c0, wsinv;
  fpn_internal::DevBuf<float> own_m, wide_ws;
  fpn_internal::DevBuf<int32_t> idx, steps, queue;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;   // [0] fork, [1 + i] join of side stream i
  hipStream_t cap = nullptr;    // capture stream for the graph
  // tangents (parameter sensitivities), L <= 16
  bool tangent = false;
  float* mtan = nullptr;        // [n][kNTan][3][Ns]: caller's dm_out or own_mt
  float* dharm = nullptr;       // [n][kNTan][ch][K_h+1][2]: caller's or own_dh
  fpn_internal::DevBuf<double> c0t;
  fpn_internal::DevBuf<float> own_mt, own_dh, tws;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool history = false;         // steps holds the step counts of a completed launch of this plan
  bool reorder = false;         // launches after the first order the buckets by those counts
};

struct fpn_mlp_s {
  int device = 0;
  int nl = 0;                   // number of affine layers
  std::vector<int> w;           // widths [nl + 1]
  std::vector<int> inpad;       // padded input width of each layer (multiple of 32)
  std::vector<int64_t> offW, offB;
  int64_t nparam = 0;
  fpn_internal::DevBuf<float> P, G, Am, Av;   // FP32 master parameters, gradient, Adam moments
  fpn_internal::DevBuf<float> norm;           // mean[in], 1/std[in]
  std::vector<fpn_internal::DevBuf<uint16_t>> Wb, Wt;
  bool dirty = true;
  int64_t t = 0;                // Adam step count
  // workspace (rows = capacity of the current buffers)
  int64_t rows_cap = 0;
  bool train_cap = false;
  std::vector<fpn_internal::DevBuf<uint16_t>> act, actT;  // act[l] [rows][inpad l] (l = 0..nl-1)
  std::vector<fpn_internal::DevBuf<uint16_t>> act_lo;     // low-order BF16 parts of act[l] (forward products)
  std::vector<fpn_internal::DevBuf<float>> z;             // z[l] pre-activation feeding act[l], l = 1..nl-1
  fpn_internal::DevBuf<float> y;                          // [rows][out]
  fpn_internal::DevBuf<uint16_t> dz[2], dzT[2];
  fpn_internal::DevBuf<double> loss;
};

// A surrogate model: the two ensemble members, the output scale and the error calibration, with the
// workspace of fpn_surrogate_infer / fpn_surrogate_train_step.
struct fpn_sur_model_s {
  int device = 0;
  fpn_mlp net[2] = {nullptr, nullptr};
  float out_scale = 1.0f;
  float err_calib = 1.0f;
  fpn_mlp res[2] = {nullptr, nullptr};  // optional residual stage
  float res_scale = 1.0f;
  fpn_internal::DevBuf<float> ya, yb, t, r;
};
