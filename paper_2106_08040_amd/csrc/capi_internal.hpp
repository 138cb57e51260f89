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

struct fpn_ctx_s {
  int device = 0;
  std::mutex mu;
  std::map<int, fpn_internal::TableSet> tables;
  fpn_internal::DevBuf<double2> twiddle;
  int tw_N = 0;
  fpn_internal::DevBuf<fpn::InstParams> ip;
  fpn_internal::DevBuf<double> c0;
  fpn_internal::DevBuf<double> wsinv;
  fpn_internal::DevBuf<float> msamp;
  fpn_internal::DevBuf<int32_t> idx;
  fpn_internal::DevBuf<int32_t> steps;
  int64_t steps_n = 0;
  // kernel timing
  bool timing = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
  double ms[4] = {0, 0, 0, 0};
  int64_t launches[4] = {0, 0, 0, 0};
};
