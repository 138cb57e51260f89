// Launch entry points of the fpn kernels (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.hpp"

namespace fpn {

struct StepLaunch {
  const InstParams* ip;
  const int32_t* inst_idx;   // instances of this launch (indices into the batch)
  int n_inst;
  const double* c0;          // stationary states, block order, stride c_stride
  int64_t c_stride;
  double amp[3], freq[3], phase[3], period;  // drive
  int settle;
  int Ns;
  int r_fixed;               // > 0 fixed substeps per sample interval, 0 adaptive
  int r_max;                 // adaptive: smallest step = sample spacing / r_max
  float tol;
  float* msamp;              // [n][3][Ns]
  float* dmdt = nullptr;      // [n][3][Ns] dm/dt at the samples, may be null
  int32_t* status;
  int32_t* steps_out;        // [n] steps taken, may be null
  int32_t* queue;            // work counter, zero when the launch starts
  int grid;                  // workgroups to launch (0: one wavefront per instance)
  const double* c0t = nullptr;  // tangents (L <= 16): initial states [n][kNTan][c_stride]
  float* mtan = nullptr;        // tangents: samples [n][kNTan][3][Ns]; null for a plain solve
  float* tws = nullptr;         // L <= 16: workspace, stepper_reg_ws_floats(L, tangents) per resident wavefront
  int waves = 0;                // L <= 16 without tangents: instances per workgroup (0: the default, 8;
                                // stepper_wave_options lists the others compiled for L)
};

template <int L>
hipError_t launch_stepper_L(const StepLaunch& s, const DevTables& t, hipStream_t stream);
// wide block layout (L = 17..24): needs a workspace of stepper_ws_floats(L) floats per instance
template <int L>
hipError_t launch_stepper_wide_L(const StepLaunch& s, const DevTables& t, float* ws, hipStream_t stream);
template <int L>
int64_t stepper_wide_ws_floats_L();
int64_t stepper_ws_floats(int L);  // 0 for the register layout (L <= 16); per resident wavefront
template <int L>
hipError_t stepper_occupancy_L(const DevTables& t, bool tangents, int waves, int* waves_per_block,
                               int* blocks_per_cu);
template <int L>
hipError_t stepper_wide_occupancy_L(int waves, int* waves_per_block, int* blocks_per_cu);
// wavefronts per workgroup and resident workgroups per CU of the stepper for degree L, for the
// workgroup size `waves` (0: the default); blocks_per_cu = 0 when that configuration does not fit
hipError_t stepper_occupancy(int L, const DevTables& t, bool tangents, int waves, int* waves_per_block,
                             int* blocks_per_cu);
// Instances (wavefronts) per workgroup of the primal register-layout stepper: 8 for every degree, and
// 12 and 16 as well for L <= kStepperMultiWavesMaxL.
constexpr int kStepperWaves = 8;
constexpr int kStepperMultiWavesMaxL = 13;
// workgroup sizes compiled for the primal stepper of degree L (at most 3 written to out); the wide
// layout (L = 17..24) reports one entry, 0: there a plan picks between 4 instances per workgroup with
// the workspace in global memory and 1 instance per workgroup with the workspace in LDS (a context can
// force either with fpn_set_stepper_waves(L, 4 or 1)); the autotuner leaves that choice to the plans
constexpr int kWideLdsWaves = 1;
constexpr int kWideGlobalWaves = 4;
// time per step of the LDS-resident wide layout relative to the global-workspace one (measured on
// MI355X: 256 instances at L = 24, both layouts holding all of them resident, 1.23 s against 1.69 s);
// plans weigh it against the resident instances of each layout
constexpr double kWideLdsStepRatio = 0.72;
inline int stepper_wave_options(int L, int* out) {
  if (L < 1 || L > 24) return 0;
  if (L > 16) {
    out[0] = 0;
    return 1;
  }
  out[0] = kStepperWaves;
  if (L > kStepperMultiWavesMaxL) return 1;
  out[1] = 12;
  out[2] = 16;
  return 3;
}
// register-layout stepper workspace per resident wavefront (floats): the tangent vectors (none without
// tangents)
inline int64_t stepper_reg_ws_floats(int L, bool tangents) {
  return tangents ? int64_t(8 * kNTan) * (((L + 1) * (L + 1) + 1 + 3) & ~3) : 0;
}

void launch_instance_prep(int64_t n, const double* D, const double* Ms, const double* K, const double* alpha,
                          const double* temp, const double* easy, const double* offset, InstParams* ip,
                          int32_t* status, hipStream_t stream);
void launch_stationary(const DevTables& t, const int32_t* idx, int n_inst, const InstParams* ip,
                       const double* field_lab, double3 drive0, double* c_out, int64_t c_stride, double* wsinv,
                       int32_t* status, hipStream_t stream);
hipError_t launch_stepper(int L, const StepLaunch& s, const DevTables& t, float* ws, hipStream_t stream);
// field mu0 H(t_j) [T] (lab frame) of largest magnitude over the samples t_j = j T / Ns of one period,
// per instance (offset [n][3] + the drive); field_out [n][3]
void launch_peak_field(int64_t n, const double* offset, const double* amp, const double* freq, const double* phase,
                       double period, int Ns, double* field_out, hipStream_t stream);
void launch_stationary_tangent(const DevTables& t, const int32_t* idx, int n_inst, const InstParams* ip,
                               double3 drive0, const double* c0, int64_t c_stride, const double* wsinv, double* ct,
                               int32_t* status, hipStream_t stream);
// drive of the equilibrium model: mu0 H_a(t) = amp_a cos(2 pi freq_a t + phase_a) + offset_a
struct EqDrive {
  double amp[3], freq[3], phase[3], period;
};
// m [n][3][Ns] of the equilibrium model (NaN for instances with a non-zero status)
void launch_equilibrium(int64_t n, int Ns, int settle, const EqDrive& d, const InstParams* ip,
                        const int32_t* status, float* m, hipStream_t stream);
void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t stream);
// sorts the queue entries idx[0..cnt) of one degree bucket by steps[instance] (the previous launch's
// time steps), most first; chunks of 4096 entries are sorted apart
void launch_order(int32_t* idx, int cnt, const int32_t* steps, hipStream_t stream);
void launch_harmonics(const float* msamp, int Ns, int n_harm, int nch, double period, const double2* tw,
                      float* harm, const int32_t* status, int64_t n, hipStream_t stream, int st_div = 1);
void launch_contract(const float* dL, const float* dharm, int per, double* grad, const int32_t* status, int64_t n,
                     hipStream_t stream);

}  // namespace fpn
