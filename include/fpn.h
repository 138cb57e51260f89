/*
 * fpn.h -- C ABI of the MI355X Neel-rotation Fokker-Planck solver (libfpn.so).
 *
 * Physics (arXiv 2106.08040, Methods, "Particle magnetization model"):
 *   mean moment  m(t) = int_{S^2} m f(m,t) dm          (Eq. mean_magmom_FP, reported / m0)
 *   df/dt = div(grad f)/(2 tau) - div(b f)             (Eq. FP-general)
 *   b = p1 H x m + p2 (m x H) x m + p3 (n.m) n x m + p4 (n.m)(m x n) x m   (Eq. convection)
 *   with p1..p4, tau, gamma~ as defined right after Eq. convection, beta and V_C as in model M0.
 * Signal (Eq. MPI_model_fourier and the phi-hat definition of model M1):
 *   Phi_k = (1/T) int_0^T dm/dt e^{-2 pi i t k / T} dt, evaluated as
 *   (2 pi i k / T) (1/N_s) sum_j m(t_j) e^{-2 pi i j k / N_s}  (exact integration by parts
 *   of the periodic moment, rectangle rule on m).
 *
 * Discretisation: real spherical-harmonic Galerkin expansion of degree <= L,
 * solved in the easy-axis frame; L-stable linearly implicit stepping (RODAS4)
 * in FP32 with the stationary initial state computed in FP64.
 *
 * Conventions shared by every call:
 *   - Fields are mu0*H in tesla, lab frame.  Outputs are lab frame.
 *   - Every instance array is DEVICE memory unless stated otherwise; the caller
 *     owns all buffers and keeps them alive until the stream has completed.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*, NULL = default
 *     stream).  Argument errors are detected on the host before any launch and
 *     returned synchronously; numerical failures are per instance in `status`
 *     (outputs of a failed instance are NaN) and the call still returns FPN_OK.
 *   - All calls are thread-safe for distinct contexts; one context per host thread.
 */
#ifndef FPN_H
#define FPN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fpn_status;
enum {
  FPN_OK = 0,
  FPN_E_ARG = -1,          /* invalid argument (NULL pointer, bad size, bad option) */
  FPN_E_RANGE = -2,        /* value out of the supported range (e.g. L) */
  FPN_E_DEVICE = -3,       /* HIP runtime error */
  FPN_E_NOMEM = -4,        /* device allocation failed */
  FPN_E_UNSUPPORTED = -7,  /* valid request the library does not implement */
  FPN_E_IO = -8            /* a file could not be read or written, or is not a valid model file */
};

/* per-instance status codes written to `status[i]` */
enum {
  FPN_INST_OK = 0,
  FPN_INST_BAD_PARAM = 1,  /* non-finite or non-positive parameter, |n| != 1 */
  FPN_INST_NONFINITE = 2,  /* non-finite state during stepping */
  FPN_INST_SINGULAR = 3,   /* zero pivot in a block inversion */
  FPN_INST_UNRESOLVED = 4, /* the Galerkin degree does not resolve the particle: at some sample time
                              (settling included) the state is not a probability density, |m| > 1 + 1e-3
                              or c_00 (total probability, conserved exactly by the solver) changed;
                              the solve stops there */
  FPN_INST_TOL_UNMET = 5   /* outputs ARE written (finite), but some step at the smallest step size
                              (sample spacing / 64) was accepted with its error estimate above `tol`:
                              their accuracy is not certified */
};

/* Static description of a status code (never NULL). */
const char* fpn_status_string(fpn_status s);
/* Detail text of the last error on the calling host thread ("" if none). */
const char* fpn_last_error(void);

typedef struct fpn_ctx_s* fpn_ctx;

/* Create a context bound to HIP device `device`.  The context owns the per-L
 * operator tables, drive tables and workspace; the caller owns *out and frees it
 * with fpn_destroy.  Errors: FPN_E_ARG (out == NULL), FPN_E_DEVICE. */
fpn_status fpn_create(fpn_ctx* out, int device);
fpn_status fpn_destroy(fpn_ctx ctx);

/* Drive field (Eq. complete-problem's H_DF):
 *   mu0 H_a(t) = amp[a] * cos(2 pi freq[a] t + phase[a])   [T],  a = x, y, z.
 * `period` is the repetition time T [s]; every freq[a]*period must be an
 * integer (checked to 1e-9), so the field is T-periodic.  Host memory. */
typedef struct {
  double amp[3];
  double freq[3];
  double phase[3];
  double period;
} fpn_drive;

/* Flags for fpn_solve_opts.flags */
enum {
  FPN_OUT_M = 1u,          /* write m_out */
  FPN_OUT_HARM = 2u,       /* write harm_out */
  FPN_HARM_Z = 4u,         /* harm_out has 3 channels (x, y, z) instead of 2 (x, y) */
  FPN_OUT_DMDT = 8u        /* write dmdt_out (fpn_solve only) */
};

/* Host memory. */
typedef struct {
  int32_t samples_per_period;  /* N_s >= 2 */
  int32_t settle_periods;      /* >= 0; the period with index settle_periods is recorded */
  int32_t n_harm;              /* K_h: harmonic bins 0..K_h, 0 <= K_h < N_s/2 */
  int32_t substeps;            /* 1..64: fixed time steps per sample interval;
                                  0: adaptive: every RODAS4 step is accepted or redone on its own
                                  embedded error, step sizes between 1/64 of the sample spacing and
                                  the sample spacing, the last step of each interval ending on the
                                  sample time (while settling, where nothing is sampled, up to 8
                                  sample spacings per step, the last one ending on the first recorded
                                  sample time); an attempt that overflows is redone 5x shorter, and
                                  the instance ends FPN_INST_NONFINITE only when that happens at the
                                  smallest step (with fixed steps: at once) */
  uint32_t flags;              /* FPN_OUT_* */
  double tol;                  /* adaptive: bound on the embedded error max|K6| of every step,
                                  0 selects the default 5e-6; ignored when substeps > 0 */
} fpn_solve_opts;

/* One batch of instances in structure-of-arrays form.  Instance parameters
 * (paper: D, M_S, K^anis, alpha, T_B, easy axis n, selection-field offset) are
 * DEVICE arrays of length n in SI units; `L` (Galerkin degree per instance) is a
 * HOST array because the launch plan depends on it. */
typedef struct {
  const double* D;         /* core diameter [m] */
  const double* Ms;        /* saturation magnetisation [A/m] */
  const double* K;         /* uniaxial anisotropy constant [J/m^3], >= 0 */
  const double* alpha;     /* damping, > 0 */
  const double* temp;      /* temperature T_B [K] */
  const double* easy_axis; /* [n][3], unit vectors (|n| = 1 within 1e-6) */
  const double* offset;    /* [n][3], static offset mu0*H_SF [T] */
  const int32_t* L;        /* HOST [n], 1 <= L <= FPN_MAX_L */
} fpn_batch;

#define FPN_MAX_L 24
/* channels * samples_per_period * 4 bytes must not exceed this (one instance's samples are staged in
 * LDS by the harmonics reduction): N_s <= 8192 with 2 channels, <= 5461 with 3; else FPN_E_RANGE */
#define FPN_MAX_HARM_LDS 65536

/* Periodic response of every instance to drive + offset (the system-matrix columns).
 * Procedure: stationary density of the field at t = 0 (FP64), then
 * (settle_periods + 1) periods of FP32 time stepping; the last period is sampled
 * at t_j = settle_periods*T + j T / N_s.
 * Outputs (DEVICE, may be NULL when the matching flag is off):
 *   m_out    [n][3][N_s]          float, dimensionless <m> (lab frame)
 *   dmdt_out [n][3][N_s]          float, d<m>/dt [1/s] at the same samples (lab frame): the rows
 *                                 l = 1 of the ODE's right-hand side A(t_j) c(t_j) (the derivative of
 *                                 the mean moment of the averaged equation of motion, model section).
 *                                 Accuracy: within 2e-3 relative (rel-L2 over an instance; measured
 *                                 3e-4 .. 6e-4 against the FP64 oracle), far below
 *                                 that of m and harm_out: A's l = 1 rows are stiff (|A| ~ 1/tau) and
 *                                 multiply the FP32 state error of the fast modes (~1e-6), which the
 *                                 slow moment m does not see.  harm_out does not use dmdt_out.
 *   harm_out [n][ch][K_h+1][2]    float, (re, im) of Phi_k [1/s], ch = 2 or 3.  Accuracy (adaptive
 *                                 steps): rel-L2 within 1e-5 per instance; per bin the error is close
 *                                 to a constant absolute level (about 3e-7 of the largest harmonic of
 *                                 the channel), so small harmonics are relatively less accurate
 *   status   [n]                  int32, FPN_INST_* (required)
 * Instances with a non-zero status other than FPN_INST_TOL_UNMET get NaN in every output.
 * Errors: FPN_E_ARG, FPN_E_RANGE (L, N_s above FPN_MAX_HARM_LDS), FPN_E_DEVICE, FPN_E_NOMEM. */
fpn_status fpn_solve(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                     const fpn_batch* batch, int64_t n,
                     float* m_out, float* dmdt_out, float* harm_out, int32_t* status, void* stream);

/* Equilibrium-model columns (paper: model M0 of the data-driven models section, Eq. Langevin):
 * the moment follows the field at once and ignores the anisotropy and the easy axis,
 * m(t) = L(beta |B(t)|) B(t) / |B(t)| with L(x) = coth(x) - 1/x, beta = V_C M_S / (k_B T) per tesla,
 * B = drive + offset.  Sampled at the same times as fpn_solve and reduced to the same harmonics, so the
 * outputs are directly comparable with the Fokker-Planck ones.  Arguments, layouts and errors as
 * fpn_solve (K, alpha, easy_axis are checked but do not enter; batch->L must be valid and is unused;
 * FPN_OUT_DMDT is rejected; n * samples_per_period < 2^31); FP64 evaluation, FP32 outputs.
 * Asynchronous. */
fpn_status fpn_equilibrium(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                           const fpn_batch* batch, int64_t n,
                           float* m_out, float* harm_out, int32_t* status, void* stream);

/* ---- parameter sensitivities (gradients) ----
 * Derivatives of the outputs with respect to the five instance parameters, in this order:
 *   0: D [1/m]   1: K [1/(J/m^3)]   2: alpha   3: polar angle of the easy axis   4: its azimuth
 * (angles of n = (sin th cos ph, sin th sin ph, cos th) in radians; at the poles the azimuth
 * derivative is zero and the polar one is taken along ph = atan2(n_y, n_x)).
 * They are computed as tangents of the discrete solve (forward mode): every RODAS4 stage of the
 * primal solve is differentiated with respect to the parameters and the five tangent systems are
 * solved with the same factorisation, in FP32; the stationary initial state is differentiated in
 * FP64 (same block inverses).  The result is the exact derivative of the computed outputs for the
 * step sequence that the primal error control chose.  Available for L <= 16 (FPN_E_RANGE otherwise). */
#define FPN_NPARAM 5

/* As fpn_solve, plus dm_out [n][5][3][N_s] (FPN_OUT_M) and dharm_out [n][5][ch][K_h+1][2] (FPN_OUT_HARM),
 * the parameter derivatives of m_out and harm_out.  Asynchronous. */
fpn_status fpn_solve_tangent(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                             const fpn_batch* batch, int64_t n, float* m_out, float* harm_out,
                             float* dm_out, float* dharm_out, int32_t* status, void* stream);

/* Gradient of a scalar loss through the harmonics: given dL_dharm [n][ch][K_h+1][2] (DEVICE FP32,
 * same layout as harm_out), writes grad_out [n][5] (DEVICE FP64) = sum over channels, bins, re/im of
 * dL/dPhi * dPhi/dp, accumulated in FP64 (NaN for failed instances).  harm_out may be NULL; opts->flags
 * only selects FPN_HARM_Z.  Asynchronous. */
fpn_status fpn_adjoint(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                       const fpn_batch* batch, int64_t n, const float* dL_dharm, double* grad_out,
                       float* harm_out, int32_t* status, void* stream);

/* ---- solve plans: reusable schedules and graph capture ----
 * A plan binds one solve to its inputs and outputs (device pointers that must stay valid and
 * unchanged in shape for the plan's lifetime; their contents may change between launches) and fixes
 * its schedule: instances are grouped by degree L, the groups are launched most expensive first on
 * concurrent streams, and every stepper launch is persistent (each wavefront takes instances from a
 * queue until it is drained), so uneven step counts do not idle whole workgroups.  Within a group
 * instances start in order of decreasing cost_hint (HOST [n], e.g. the step counts of an earlier run
 * from fpn_plan_steps).  With cost_hint NULL the first launch keeps batch order, and every later
 * launch (eager or a graph captured after the first launch) starts the instances of each group that
 * has more instances than resident wavefronts in order of decreasing step count of the launch before
 * it, sorted on the device; the instances queued last then run after the others, and the shortest
 * go there.  Outputs do not depend on the schedule.  Launches of one plan must be ordered (one stream,
 * or synchronised): they share the plan's workspace and outputs.
 * The plan owns its workspace; plans are independent of fpn_solve's and of each other. */
typedef struct fpn_plan_s* fpn_plan;

/* Build a plan (synchronous).  Errors as fpn_solve; n >= 1. */
fpn_status fpn_plan_create(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                           const fpn_batch* batch, int64_t n, const float* cost_hint,
                           float* m_out, float* harm_out, int32_t* status, fpn_plan* out);
/* Run the plan on `stream` (asynchronous), as fpn_solve would. */
fpn_status fpn_plan_launch(fpn_plan plan, void* stream);
/* Run the plan as one HIP graph: the first call captures the launch sequence (on a stream of the
 * plan's own) and instantiates it; every call launches the graph on `stream` (asynchronous). */
fpn_status fpn_plan_graph_launch(fpn_plan plan, void* stream);
/* Time steps taken per instance by the plan's last run (HOST int32 [n]; synchronises). */
fpn_status fpn_plan_steps(fpn_plan plan, int32_t* steps_out);
fpn_status fpn_plan_destroy(fpn_plan plan);

/* ---- Launch configuration and autotuner (batching of uneven degrees) ----
 * The register-layout stepper (L <= 16) is compiled for several workgroup sizes: 8 instances per
 * workgroup for every degree, and 12 and 16 for L <= 13.  A larger workgroup shares the per-degree
 * operator tables in LDS among more instances, so more instances fit on a compute unit, at a smaller
 * register budget per instance.  Which is fastest depends on L; results are bitwise identical for
 * every size (each instance is integrated by one wavefront in the same order).  The context keeps
 * one size per degree, used by fpn_solve and fpn_plan_create (a plan keeps the size it was built
 * with); the tangent stepper of fpn_solve_tangent and fpn_adjoint has a size of its own. */

/* Workgroup sizes compiled for degree L: *count (1..3) sizes written to waves (capacity >= 3).
 * For L = 17..24 (one configuration) the single entry is 0.  Errors: FPN_E_ARG. */
fpn_status fpn_stepper_wave_options(int32_t L, int32_t* waves, int32_t* count);

/* Use workgroup size `waves` (one of fpn_stepper_wave_options(L), or 0 for the default) for degree L
 * in this context.  For L = 17..24 (the wide layout, whose option list is just 0) `waves` is 0, 4 or
 * 1: 4 keeps each instance's block inverses and stage vectors in a global workspace with 4 instances
 * per workgroup, 1 keeps them in LDS with 1 instance per workgroup (about 28 % shorter steps at L = 24,
 * fewer instances resident), 0 lets each plan choose per degree bucket from its predicted duration
 * (the longest instance against the bucket's work over the resident instances of each layout).
 * Outputs do not depend on the choice.  Errors: FPN_E_ARG (size not compiled for L), FPN_E_DEVICE
 * (the configuration does not fit on a compute unit of this device). */
fpn_status fpn_set_stepper_waves(fpn_ctx ctx, int32_t L, int32_t waves);

/* Autotuner: time every workgroup size of degree L that fits on this device on a fixed synthetic
 * probe batch (one particle, D = 20 nm, K = 2 kJ/m^3, alpha = 0.1, 295 K, easy axes on a spiral,
 * 6 mT offsets on a ring; a 40 us drive with 3 and 4 cycles on x and y, 64 samples, 2 fixed steps
 * per sample; twice as many instances as the largest configuration keeps resident, at most 16384)
 * and keep the fastest for this context.  waves_out (may be NULL): the chosen size.
 * ns_per_step_out (may be NULL, capacity >= 3): measured time per instance-step of each size, in
 * the order of fpn_stepper_wave_options, +inf for a size that does not fit.  Allocates and frees
 * its probe buffers and synchronises the device; the chosen size persists until changed.
 * Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_autotune(fpn_ctx ctx, int32_t L, int32_t* waves_out, double* ns_per_step_out);

/* Time steps taken by the most recent fpn_solve, fpn_solve_tangent or fpn_adjoint on this context,
 * summed over its instances (synchronises with that call).  0 before the first such call and after
 * one that failed while setting up or launching; a call rejected for its arguments leaves the previous
 * count.  Plans (fpn_plan_*) report theirs through fpn_plan_steps.  HOST output.
 * Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_last_steps(fpn_ctx ctx, int64_t* total_steps);

/* Stationary mean moment under a static field (FP64 on the device):
 * the null vector of the Galerkin operator with total probability 1.
 *   field  [n][3] DEVICE, mu0*H [T] lab frame
 *   m_out  [n][3] DEVICE, dimensionless <m> (lab frame)
 *   status [n]    DEVICE int32 */
fpn_status fpn_stationary(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const double* field,
                          double* m_out, int32_t* status, void* stream);

/* Truncation estimate of the Galerkin degree (an a-posteriori indicator, not part of the paper):
 * the paper discretises Eq. FP-general with finite volumes; a spherical-harmonic expansion cut at
 * degree L converges spectrally to the same solution, and this call estimates how far the degree-L
 * solution of each instance is from it.  Per instance: the field mu0 H(t_j) of largest magnitude
 * over the samples t_j = j T / samples_per_period of one drive period (offset + drive; the first
 * sample within a relative 1e-9 of the largest squared magnitude), the stationary moments
 * (Eq. mean_magmom_FP / m0, FP64, as fpn_stationary) of degrees L and L - 2 under that static field,
 * and est = |m_L - m_{L-2}| (Euclidean, dimensionless).  Checked against finite-volume solutions
 * of Eq. FP-general and higher-degree solves, it bounds the rel-L2 truncation error of the periodic
 * m(t) at degree L within a factor of about 2..20 from above; it is a heuristic, not a proof.
 *   batch  as for fpn_solve (L[i] >= 3 on the host)
 *   est_out [n] DEVICE double (NaN where status != 0)
 *   status  [n] DEVICE int32, FPN_INST_* of the stationary solves
 * Synchronises `stream`.  Errors: FPN_E_ARG, FPN_E_RANGE (some L < 3), FPN_E_DEVICE. */
fpn_status fpn_truncation_estimate(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const fpn_drive* drive,
                                   int32_t samples_per_period, double* est_out, int32_t* status, void* stream);

/* Degree selection by the truncation estimate: per instance the smallest L in batch->L[i] .. L_max
 * whose fpn_truncation_estimate value is <= tol (the largest sampled field, stationary moments of
 * degrees L and L - 2); L_max where none is (est_out then holds that degree's estimate, > tol).
 * batch->L[i] is the smallest degree allowed (for instance a stability rule), 3 <= batch->L[i] <= L_max.
 * Costs one batch of FP64 stationary solves per degree from min(L) - 2 to L_max.
 *   tol     > 0, on |m_L - m_{L-2}| (dimensionless)
 *   L_max   3..24
 *   L_out   [n] HOST int32 (L_max where status != 0)
 *   est_out [n] DEVICE double, may be NULL: the estimate at the chosen degree (NaN where status != 0)
 *   status  [n] DEVICE int32, FPN_INST_* of the stationary solves
 * Synchronises `stream`.  Errors: FPN_E_ARG, FPN_E_RANGE, FPN_E_DEVICE. */
fpn_status fpn_select_degree(fpn_ctx ctx, const fpn_batch* batch, int64_t n, const fpn_drive* drive,
                             int32_t samples_per_period, double tol, int32_t L_max, int32_t* L_out, double* est_out,
                             int32_t* status, void* stream);

/* Kernel timing (diagnostic).  When enabled, every kernel launch of fpn_solve and
 * fpn_stationary is bracketed by HIP events recorded on the launch stream; reading
 * synchronises those events and returns the accumulated device time.
 *   fpn_timing_enable: enable != 0 starts (and clears) the counters, 0 stops them.
 *   fpn_timing_read:   ms_out[4] and launches_out[4] (HOST) receive, in this order,
 *                      instance preparation, stationary solve, time stepper, harmonics.
 * Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_timing_enable(fpn_ctx ctx, int enable);
fpn_status fpn_timing_read(fpn_ctx ctx, double* ms_out, int64_t* launches_out);

/* ---- surrogate network ----
 * A multilayer perceptron (not part of the paper) that maps instance features to signal
 * harmonics: affine layers z_l = W_l a_{l-1} + b_l with a_l = gelu(z_l) (exact erf form) on every
 * layer but the last.  Products run on BF16 matrix cores with FP32 accumulation; the master
 * parameters, gradients and Adam moments are FP32.  Inputs are standardised inside the network:
 * x' = (x - mean) / std (fpn_mlp_set_input_norm; default mean 0, std 1).
 * Parameter layout (flat FP32): for each layer l, W_l [out][in] row-major, then b_l [out].
 * A model belongs to the device of the context it was created with; calls on one model must not
 * overlap (they share its workspace). */
typedef struct fpn_mlp_s* fpn_mlp;

/* widths[0..n_layers]: input width, hidden widths (multiples of 32), output width (multiple of 32).
 * Weights and biases start U(-1/sqrt(in), 1/sqrt(in)) from `seed`.  Errors: FPN_E_ARG, FPN_E_NOMEM. */
fpn_status fpn_mlp_create(fpn_ctx ctx, int32_t n_layers, const int32_t* widths, uint64_t seed, fpn_mlp* out);
fpn_status fpn_mlp_destroy(fpn_mlp m);
/* number of FP32 parameters (-1 for NULL) */
int64_t fpn_mlp_num_params(fpn_mlp m);
/* Layer count (HOST int32) and, when widths is not NULL, widths[0..n_layers] (HOST, capacity >= 17). */
fpn_status fpn_mlp_shape(fpn_mlp m, int32_t* n_layers, int32_t* widths);
/* Copy the parameters out to `dst` and/or in from `src` (DEVICE, flat layout above; either may
 * be NULL).  Asynchronous on `stream`. */
fpn_status fpn_mlp_params(fpn_mlp m, float* dst, const float* src, void* stream);
/* Input standardisation, HOST arrays [input width]; std > 0.  Synchronous. */
fpn_status fpn_mlp_set_input_norm(fpn_mlp m, const float* mean, const float* stdev);
/* y [n][out] = network(x [n][in]) (DEVICE FP32).  n <= 2^30, processed in chunks of 2^17 rows. */
fpn_status fpn_mlp_forward(fpn_mlp m, const float* x, int64_t n, float* y, void* stream);
/* Gradient of loss = mean over n x out elements of (y - t)^2 (t DEVICE [n][out]).
 * grad (DEVICE, flat layout, may be NULL) and loss (DEVICE, one double, may be NULL).  n <= 2^22. */
fpn_status fpn_mlp_gradient(fpn_mlp m, const float* x, const float* t, int64_t n, float* grad, double* loss,
                            void* stream);
/* One Adam step (b1 = 0.9, b2 = 0.999, eps = 1e-8, learning rate lr) on that gradient. */
fpn_status fpn_mlp_train_step(fpn_mlp m, const float* x, const float* t, int64_t n, float lr, double* loss,
                              void* stream);

/* ---- surrogate evaluation ----
 * Harmonics 1..K_h of the x and y channels predicted by a two-member network ensemble from the
 * instance features, with the solver as the fallback and as the reference its error is measured against:
 *   features x = (log D, sigma, alpha, n_x, n_y, n_z, offset_x / 12 mT, offset_y / 12 mT) with
 *   sigma = K (pi D^3 / 6) / (k_B T) (the anisotropy barrier in units of k_B T, which sets the Neel
 *   relaxation time), the axis taken in the half-space n_z > 0 (n and -n describe the same particle);
 *   K must be > 0;
 *   prediction = (y_a + y_b) / 2 / out_scale, network output layout [channel x, y][k = 1..K_h][re, im]
 *   (y_k = net[k](x), plus res[k](x) / res_scale with a residual stage);
 *   error estimate = err_calib * ||y_a - y_b|| / ||(y_a + y_b) / 2||  (err_calib is fitted on held-out
 *   solver results so that the estimate bounds the relative L2 error of the prediction). */
typedef struct {
  fpn_mlp net[2];     /* widths: 8 inputs, 4 * K_h outputs, identical shapes */
  float out_scale;    /* network output = Phi [1/s] * out_scale */
  float err_calib;    /* > 0 */
  fpn_mlp res[2];     /* optional residual stage (both NULL: none), same widths: member k's output is
                         net[k](x) + res[k](x) / res_scale, res[k] trained on the residual of net[k]
                         multiplied by res_scale */
  float res_scale;    /* > 0 when res[] is set */
} fpn_surrogate;

/* Features x [n][8] (DEVICE FP32) and status [n] (FPN_INST_BAD_PARAM for non-physical instances,
 * whose features are NaN).  Asynchronous. */
fpn_status fpn_surrogate_features(fpn_ctx ctx, const fpn_batch* batch, int64_t n, float* x, int32_t* status,
                                  void* stream);

/* Evaluate every instance with the ensemble; instances whose error estimate exceeds `tol` (or is
 * not finite) are solved with fpn_solve(drive, opts) instead (opts->n_harm = K_h; FPN_HARM_Z not
 * allowed).  Outputs (DEVICE): harm_out [n][2][K_h+1][2] as fpn_solve's (bin 0 = 0), err_out [n]
 * (the estimate; 0 where the solver ran), used_solver [n] (1 where the solver ran), status [n].
 * n_fallback (HOST, may be NULL) receives the number of solver instances.  Synchronous: the
 * fallback count is read back before the solver is planned.  Errors: FPN_E_ARG, FPN_E_RANGE,
 * FPN_E_DEVICE, FPN_E_NOMEM. */
fpn_status fpn_surrogate_predict(fpn_ctx ctx, const fpn_surrogate* sur, double tol, const fpn_drive* drive,
                                 const fpn_solve_opts* opts, const fpn_batch* batch, int64_t n, float* harm_out,
                                 float* err_out, int32_t* used_solver, int32_t* status, int64_t* n_fallback,
                                 void* stream);

/* ---- surrogate model ----
 * An owning handle for a two-member ensemble (the fpn_surrogate above): both networks, the output
 * scale and the error calibration, so a trained surrogate can be written to a file and read back
 * (in this or another process, on any device).  Calls on one model must not overlap.
 *
 * File format (little-endian, written by fpn_surrogate_save):
 *   char magic[8] = "FPNSUR1\0"; uint32 version = 2; int32 n_layers; int32 widths[n_layers + 1];
 *   float out_scale; float err_calib; int32 has_residual; float res_scale;
 *   then for each member k = 0, 1 (and, with a residual stage, its members 2, 3): int64 adam_steps;
 *   float norm[2 * widths[0]] (input mean, then 1 / std, as the network applies them);
 *   float params[P]; float adam_m[P]; float adam_v[P] (P = sum over layers of (in + 1) * out, layout
 *   as fpn_mlp_params);
 *   uint64 FNV-1a hash of every preceding byte.
 * Version-1 files (no residual fields or members) are read as well.
 * A model read back evaluates bit for bit as the one saved, and continues training from the same
 * Adam state. */
typedef struct fpn_sur_model_s* fpn_sur_model;

/* A new model: two networks of widths[0..n_layers] (as fpn_mlp_create), member k initialised from
 * seeds[k] (HOST), out_scale = err_calib = 1.  Errors: FPN_E_ARG, FPN_E_NOMEM, FPN_E_DEVICE. */
fpn_status fpn_surrogate_init(fpn_ctx ctx, int32_t n_layers, const int32_t* widths, const uint64_t seeds[2],
                              fpn_sur_model* out);
/* A model read from `weights_path` (a file written by fpn_surrogate_save), on ctx's device.
 * Errors: FPN_E_ARG (NULL argument), FPN_E_IO (unreadable, not a model file, truncated, hash
 * mismatch, trailing bytes), FPN_E_NOMEM, FPN_E_DEVICE. */
fpn_status fpn_surrogate_create(fpn_ctx ctx, const char* weights_path, fpn_sur_model* out);
/* Write the model to `path` (synchronises the device).  Errors: FPN_E_ARG, FPN_E_IO, FPN_E_DEVICE. */
fpn_status fpn_surrogate_save(fpn_sur_model m, const char* path);
fpn_status fpn_surrogate_destroy(fpn_sur_model m);
/* Member k as an fpn_mlp handle owned by the model (for fpn_mlp_* calls: input normalisation,
 * parameters, per-member training): k = 0, 1 the ensemble, k = 2, 3 the residual stage (FPN_E_ARG if
 * the model has none). */
fpn_status fpn_surrogate_member(fpn_sur_model m, int32_t k, fpn_mlp* out);
/* Add a residual stage: two networks of the members' widths, member k initialised from seeds[k]
 * (HOST), res_scale = 1; FPN_E_ARG if the model has one.  Errors: FPN_E_ARG, FPN_E_NOMEM, FPN_E_DEVICE. */
fpn_status fpn_surrogate_add_residual(fpn_ctx ctx, fpn_sur_model m, const uint64_t seeds[2]);
/* res_scale of the residual stage (finite, > 0; FPN_E_ARG without a stage). */
fpn_status fpn_surrogate_set_residual_scale(fpn_sur_model m, float res_scale);
/* out_scale: network output = prediction * out_scale; err_calib: the estimate's constant.  Both finite
 * and > 0, else FPN_E_ARG. */
fpn_status fpn_surrogate_set_scales(fpn_sur_model m, float out_scale, float err_calib);
/* Fill an fpn_surrogate (non-owning view: member handles and scales) for fpn_surrogate_predict. */
fpn_status fpn_surrogate_view(fpn_sur_model m, fpn_surrogate* view);
/* Ensemble evaluation without fallback: y [n][W] = (y_a + y_b) / 2 / out_scale (W = output width, the
 * networks' layout; y_k includes the residual stage) and err_est [n] = err_calib * ||y_a - y_b|| /
 * ||(y_a + y_b) / 2||, from features
 * x [n][widths[0]] (all DEVICE FP32; y or err_est may be NULL, not both).  n <= 2^30.  Asynchronous.
 * Errors: FPN_E_ARG, FPN_E_NOMEM, FPN_E_DEVICE. */
fpn_status fpn_surrogate_infer(fpn_ctx ctx, fpn_sur_model m, const float* x, int64_t n, float* y, float* err_est,
                               void* stream);
/* One Adam step (fpn_mlp_train_step) of each ensemble member (not the residual stage, which is trained
 * through its member handles) on the same minibatch: features x [n][widths[0]],
 * targets y_true [n][W] in prediction units (multiplied by out_scale inside); loss_out (DEVICE, two
 * doubles, may be NULL) receives each member's summed squared error in network units.  1 <= n <= 2^22.
 * Asynchronous.  Errors: FPN_E_ARG, FPN_E_NOMEM, FPN_E_DEVICE. */
fpn_status fpn_surrogate_train_step(fpn_ctx ctx, fpn_sur_model m, const float* x, const float* y_true, int64_t n,
                                    float lr, double* loss_out, void* stream);

/* ---- data-driven model fits and distance measure ----
 * Paper: Methods, "Data-driven physically motivated models" (models M0 and M1), "Technical details
 * regarding the parameter identification" (closed-form scale of M0/M1) and "Distance Measure"
 * (Eq. mix, Eq. error1, Eq. globalMeasure).
 * A system matrix (one dictionary element, or one measured matrix) is [n_pos][n_ch][n_bins][2] FP32:
 * offset positions outermost, then receive channel, frequency bin k = 0..n_bins-1, (re, im); a batch
 * of them is contiguous.  fpn_solve's harm_out is such a batch when its instances are ordered
 * element-major, position-minor (n_bins = K_h + 1). */

/* For each pair p (DEVICE int32 pair_phi[p], pair_s[p]: indices of a dictionary element of `phi` and a
 * measured matrix of `S`) and every row (channel c, bin k), over the n_pos positions nu:
 *   a[p][c][k]   = sum_nu S(nu) conj(Phi(nu)) / sum_nu |Phi(nu)|^2   (0 for an all-zero Phi row)
 *   err[p][c][k] = sqrt(sum_nu |S(nu) - a Phi(nu)|^2 / n_pos) / max_nu |S(nu)|   (Eq. error1)
 * Sums in FP64.  a_out [n_pairs][n_ch][n_bins][2], err_out [n_pairs][n_ch][n_bins] (DEVICE FP32, one
 * may be NULL); an all-zero S row gives err = NaN.  Pair indices must lie inside phi and S (not
 * checked on the device).  Asynchronous.  Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_fit_rows(fpn_ctx ctx, const float* phi, const float* S, int32_t n_pos, int32_t n_ch, int32_t n_bins,
                        int64_t n_pairs, const int32_t* pair_phi, const int32_t* pair_s, float* a_out,
                        float* err_out, void* stream);

/* Per-frequency and global NRMSE of n_groups parameter groups: err_rows [n_groups][n_ang][n_ch][n_bins]
 * (fpn_fit_rows's err_out for pairs ordered group-major, angle-minor), kset [n_k] DEVICE int32 bins
 * (the graded set I_freq, each < n_bins):
 *   eps_freq[g][j] = sqrt(mean over angles and channels of err[g][.][.][kset[j]]^2)
 *   eps_global[g]  = sqrt(mean over j of eps_freq[g][j]^2)                    (Eq. globalMeasure)
 * The mean over receive channels is folded into the per-frequency measure, as the paper states its
 * sums also run over the channels.  DEVICE FP32 outputs (one may be NULL), FP64 sums.  Asynchronous.
 * Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_nrmse_global(fpn_ctx ctx, const float* err_rows, int64_t n_groups, int32_t n_ang, int32_t n_ch,
                            int32_t n_bins, const int32_t* kset, int32_t n_k, float* eps_freq, float* eps_global,
                            void* stream);

/* Mixing orders of bin k (Eq. mix): the integers (mx, my) with k = mx n_dens + my (n_dens + 1) and the
 * smallest |mx| + |my| (unique).  HOST, no device needed.  Errors: FPN_E_ARG (NULL output,
 * n_dens outside [1, 4096], |k| > 2^24). */
fpn_status fpn_mixing_order(int32_t k, int32_t n_dens, int32_t* mx, int32_t* my);
/* The graded bin set I_freq = { mx n_dens + my (n_dens + 1) : 0 <= mx <= Mx, 0 <= my <= My } without
 * (mx, my) = (0,0), (0,1), (1,0), mx-major.  k_out (HOST, capacity (Mx+1)(My+1), may be NULL) and
 * count (HOST).  Errors: FPN_E_ARG. */
fpn_status fpn_frequency_index_set(int32_t Mx, int32_t My, int32_t n_dens, int32_t* k_out, int32_t* count);

/* Model M2 (paper: "Technical details regarding the parameter identification", M2: Eq. LSfitM2,
 * Eq. LSfitM2_alternative, Eq. approx_low_rank).  The dictionary holds J parameter pairs at n_ang
 * angles: element j * n_ang + theta of phi (layout as above), its M1 scale a [J * n_ang][n_ch][n_bins][2]
 * (fpn_fit_rows's a_out for pairs in that order) and the measured matrices S [n_ang][...].  The
 * weighted dictionary matrix M has rows (theta, c, k in kset, position) and columns j:
 *   M[r][j] = a_{j,theta}(c,k) Phi_{j,theta}(nu,c,k) / max_nu |S_theta(nu,c,k)|,  y[r] = S_theta(nu,c,k) / (same)
 * (the paper's per-frequency infinity-norm weighting, per receive channel).  This call forms, on the
 * device with FP64 sums, G = M^H M (G_out [J][J][2], Hermitian), b = M^H y (b_out [J][2]) and
 * yy_out = ||y||^2 (all DEVICE FP64).  Workspace: the context keeps M (J * rows complex FP32).
 * Asynchronous.  Errors: FPN_E_ARG, FPN_E_RANGE (J > 8192 or more than 2^34 entries), FPN_E_NOMEM,
 * FPN_E_DEVICE. */
fpn_status fpn_m2_system(fpn_ctx ctx, const float* phi, const float* a, const float* S, int32_t n_pos, int32_t n_ch,
                         int32_t n_bins, int32_t J, int32_t n_ang, const int32_t* kset, int32_t n_k, double* G_out,
                         double* b_out, double* yy_out, void* stream);
/* Non-negative weights of model M2 from G, b, yy (HOST arrays as fpn_m2_system writes them): the
 * eigenvectors of G give the truncated SVD of M; with s > 0 only the s largest singular values are kept
 * (s = 0: every eigenvalue above 1e-14 of the largest), and min over real w >= 0 of
 * ||U_s^H (M w - y)||^2 is solved by a primal-dual interior-point method.  w_out [J] (HOST), resid_out
 * (HOST, may be NULL) = ||M w - y||^2, reduced_out (may be NULL) = the truncated objective, rank_out (may
 * be NULL) = the number of singular values kept.  No device needed.  Errors: FPN_E_ARG, FPN_E_RANGE (the
 * interior-point iteration did not converge). */
fpn_status fpn_m2_weights(int32_t J, const double* G, const double* b, double yy, int32_t s, double* w_out,
                          double* resid_out, double* reduced_out, int32_t* rank_out);
/* The M2 system matrices S_model[theta] = sum_j w_j a_{j,theta} Phi_{j,theta} (w DEVICE FP64 [J]; phi and a as
 * for fpn_m2_system; model_out [n_ang][n_pos][n_ch][n_bins][2] DEVICE FP32, FP64 sums).  Asynchronous.
 * Errors: FPN_E_ARG, FPN_E_RANGE, FPN_E_DEVICE. */
fpn_status fpn_m2_model(fpn_ctx ctx, const float* phi, const float* a, const double* w, int32_t n_pos, int32_t n_ch,
                        int32_t n_bins, int32_t J, int32_t n_ang, float* model_out, void* stream);
/* Eq. error1 rows of n_mat model matrices against the measured ones of the same index (no fit):
 * err_out [n_mat][n_ch][n_bins] (DEVICE FP32, FP64 sums).  Asynchronous.  Errors: FPN_E_ARG, FPN_E_DEVICE. */
fpn_status fpn_rows_error(fpn_ctx ctx, const float* model, const float* S, int32_t n_pos, int32_t n_ch, int32_t n_bins,
                          int64_t n_mat, float* err_out, void* stream);

/* ---- allocation-free solve ----
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same solve as fpn_solve for a batch of ONE Galerkin degree
 * L <= 16, with no device (or host-side library) allocation: every per-call buffer lives in a fixed
 * device array of the library, FPN_STATIC_SCRATCH_BYTES on each GPU the library runs on, held until
 * the process ends.  Hence n <= FPN_STATIC_MAX_N and samples_per_period <= FPN_STATIC_MAX_NS, else
 * FPN_E_RANGE; all batch.L[i] equal, else FPN_E_ARG; FPN_OUT_DMDT is not available (FPN_E_ARG).
 * The context must already hold the operator tables of that L and the twiddle table of that N_s,
 * which an earlier fpn_solve on the context with the same L and N_s builds; otherwise FPN_E_ARG.
 * All calls on one GPU share the array (whatever the context or stream), and it keeps the last call's
 * contents: calls that overlap on one GPU race, so serialise them.  Asynchronous on `stream`;
 * outputs, statuses and the other errors as fpn_solve. */
#define FPN_STATIC_MAX_N 128
#define FPN_STATIC_MAX_NS 2048
#define FPN_STATIC_SCRATCH_BYTES (12u << 20)
fpn_status fpn_solve_static(fpn_ctx ctx, const fpn_drive* drive, const fpn_solve_opts* opts,
                            const fpn_batch* batch, int64_t n, float* m_out, float* harm_out, int32_t* status,
                            void* stream);

/* ---- host-only helpers (no device needed; used to check the operator build) ---- */

/* Dense Galerkin operator A (1/s) of one particle in its easy-axis frame, built
 * from the library's own operator tables: dc/dt = A c with c in flat SH order
 * i = l*l + l + m.  field_easy is mu0*H [T] in the easy-axis frame (n = z).
 * A_out: HOST, (L+1)^2 x (L+1)^2 row-major doubles.  Errors: FPN_E_ARG, FPN_E_RANGE. */
fpn_status fpn_host_operator(int32_t L, double D, double Ms, double K, double alpha, double temp,
                             const double field_easy[3], double* A_out);

/* The rotation R (row-major 3x3, HOST) with R * (0,0,1) = n used to map lab vectors
 * into the easy-axis frame (v_easy = R^T v_lab).  Errors: FPN_E_ARG (|n| not 1). */
fpn_status fpn_host_frame(const double n[3], double R_out[9]);

/* Number of nonzeros of the operator tables for degree L (diagnostic). */
int64_t fpn_host_table_nnz(int32_t L);

#ifdef __cplusplus
}
#endif

#endif /* FPN_H */
