#pragma once
// Small device helpers shared by the kernels: compile-time loops, wave-wide
// broadcasts and the LDS ordering of a single wave.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#define SI __attribute__((always_inline))

namespace rbfsl {

template <int B0, typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, B0 + Is>{}), ...);
}
// compile-time loop over B0..E-1 (f receives an integral_constant)
template <int B0, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    if constexpr (E > B0) sfor_impl<B0>(f, std::make_integer_sequence<int, E - B0>{});
}

// value of v in lane `lane` (wave-uniform), through two readlanes
__device__ __forceinline__ double bcast_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// LDS writes by some lanes of this wave become visible to its other lanes
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace rbfsl
