// Device helpers shared by the fpn kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace fpn {

// ------------------------------------------------------------------ helpers ---

// Completes this wavefront's outstanding LDS traffic and orders memory accesses.
__device__ __forceinline__ void wsync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

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
