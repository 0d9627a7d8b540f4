// Device helpers shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cashash_internal.h"

namespace cashash {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Loads through pointers known to address global memory (pointers read from
// device tables would otherwise be treated as generic and use flat loads).
template <class T>
__device__ __forceinline__ T gload(const T* p) {
#if __HIP_DEVICE_COMPILE__
    return *(const __attribute__((address_space(1))) T*)(p);
#else
    return *p;  // host pass: parsed only, never run
#endif
}
// Store through a pointer known to address global memory (a generic store
// would also count against the LDS wait counter).
template <class T>
__device__ __forceinline__ void gstore(T* p, T v) {
#if __HIP_DEVICE_COMPILE__
    *(__attribute__((address_space(1))) T*)(p) = v;
#else
    *p = v;  // host pass: parsed only, never run
#endif
}
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ ulonglong2 gload(const ulonglong2* p) {
    const u64x2_t v = gload(reinterpret_cast<const u64x2_t*>(p));
    return make_ulonglong2(v.x, v.y);
}
__device__ __forceinline__ uint4 gload(const uint4* p) {
    const u32x4_t v = gload(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gload(const float2* p) {
    const f32x2_t v = gload(reinterpret_cast<const f32x2_t*>(p));
    return make_float2(v.x, v.y);
}
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 gload(const uint2* p) {
    const u32x2_t v = gload(reinterpret_cast<const u32x2_t*>(p));
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ void gstore(ulonglong2* p, ulonglong2 v) {
    gstore(reinterpret_cast<u64x2_t*>(p), u64x2_t{v.x, v.y});
}
__device__ __forceinline__ void gstore(float2* p, float2 v) {
    gstore(reinterpret_cast<f32x2_t*>(p), f32x2_t{v.x, v.y});
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (lane >= d) v += t;
    }
    return v;
}

}  // namespace cashash

// Launch and return the launch error, if any.
#define CH_LAUNCH(...)                                  \
    do {                                                \
        hipLaunchKernelGGL(__VA_ARGS__);                \
        hipError_t e_ = hipGetLastError();              \
        if (e_ != hipSuccess) return e_;                \
    } while (0)
