// Surrogate evaluation kernels (surrogate.hip): launch wrappers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fpn {
namespace sur {

hipError_t features(int64_t n, const double* D, const double* Ms, const double* K, const double* alpha,
                    const double* T, const double* nax, const double* off, float* x, int32_t* status,
                    hipStream_t s);
hipError_t combine(int64_t n, int Kh, const float* ya, const float* yb, float inv_scale, float calib, float tol,
                   const int32_t* status, float* harm, float* err, int32_t* used, int32_t* list, int32_t* count,
                   hipStream_t s);
// y = (ya + yb) / 2 * inv_scale and err = calib * 2 ||ya - yb|| / ||ya + yb|| per row of W values
// (either output may be NULL)
hipError_t mean_spread(int64_t n, int W, const float* ya, const float* yb, float inv_scale, float calib, float* y,
                       float* err, hipStream_t s);
// y += a * x (n values)
hipError_t axpy(int64_t n, float a, const float* x, float* y, hipStream_t s);
// dst = a * src (n values)
hipError_t scale(int64_t n, const float* src, float a, float* dst, hipStream_t s);
hipError_t gather(int cnt, const int32_t* list, const double* D, const double* Ms, const double* K,
                  const double* alpha, const double* T, const double* nax, const double* off, double* out,
                  hipStream_t s);
hipError_t scatter(int cnt, int per, const int32_t* list, const float* src, const int32_t* st_src, float* harm,
                   int32_t* status, float* err, hipStream_t s);

}  // namespace sur
}  // namespace fpn
