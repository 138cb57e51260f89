// Device helpers shared by the fpn kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace fpn {

// ------------------------------------------------------------------ helpers ---

// Orders the memory accesses of the lanes of one wavefront: what a lane wrote before the call is
// seen by every lane of the same wavefront after it.  A wavefront's LDS and global-memory operations
// are performed in program order (the AMDGPU memory model needs no wait counter at wavefront
// scope), so this is a fence for the compiler only: a write followed by a read of another lane's
// data does not wait for the write to complete before the read is issued.
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}
template <int I, int E, typename F>
__device__ __forceinline__ void static_for_down(F&& f) {  // I, I-1, ..., E
  if constexpr (I >= E) {
    f(std::integral_constant<int, I>{});
    static_for_down<I - 1, E>(f);
  }
}

// Kind multipliers (1/s per unit table value) of the Galerkin operator, see structure.hpp.
__device__ __forceinline__ float kind_mult(int kind, float inv2tau, float sigma, float alpha, float beta,
                                           float hx, float hy, float hz) {
  switch (kind) {
    case 0: return inv2tau;
    case 1: return inv2tau * sigma;
    case 2: return inv2tau * 2.0f * sigma / alpha;
    case 3: return inv2tau * beta * hz;
    case 4: return inv2tau * beta * hz / alpha;
    case 5: return inv2tau * beta * hx;
    case 6: return inv2tau * beta * hy;
    case 7: return inv2tau * beta * hx / alpha;
    default: return inv2tau * beta * hy / alpha;
  }
}

}  // namespace fpn
