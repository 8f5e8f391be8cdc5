// Wavefront-level primitives: the one-lane DPP shift that hands a value from lane l-1 to lane l,
// wavefront maxima and minima, LDS progress words, and the wait that makes this wavefront's
// global stores complete before it publishes them.
#pragma once

#include <hip/hip_runtime.h>

namespace dlr {

// lane l receives lane l-1's value; lane 0 receives `first`
__device__ __forceinline__ float shift_in(float first, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, first),
                                                                  __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double shift_in(double first, double v) {
    const long long f = __builtin_bit_cast(long long, first), x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(x & 0xffffffffll), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(x >> 32), 0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Wavefront all-reductions for max and min (exact in any order).  Within each row of 16 lanes:
// DPP exchanges with lane xor 1 and xor 2 (quad permutations), then rotations by 4 and 8; the four
// row results are then read from lanes 0, 16, 32 and 48.  VALU only, no LDS round trips.  Every
// lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = dpp_i32<CTRL>((int)(x & 0xffffffffll)), hi = dpp_i32<CTRL>((int)(x >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRor4 = 0x124, kDppRor8 = 0x128;
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppRor4>(v));
    v = fmax(v, dpp_f64<kDppRor8>(v));
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp_f64<kDppXor1>(v));
    v = fmin(v, dpp_f64<kDppXor2>(v));
    v = fmin(v, dpp_f64<kDppRor4>(v));
    v = fmin(v, dpp_f64<kDppRor8>(v));
    return fmin(fmin(readlane_f64(v, 0), readlane_f64(v, 16)), fmin(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_i32<kDppXor1>(v));
    v = min(v, dpp_i32<kDppXor2>(v));
    v = min(v, dpp_i32<kDppRor4>(v));
    v = min(v, dpp_i32<kDppRor8>(v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Progress words of LDS rings.  The LDS unit executes a wavefront's LDS instructions in
// issue order, so a ring write followed by a progress store is seen in that order by any
// wavefront that reads the progress word first and the ring afterwards; compiler barriers keep
// the compiler from reordering them.  Relaxed atomics are used on purpose: a release or acquire
// at workgroup scope would also wait for this wavefront's outstanding global loads (the
// prefetched chunks), which is what the rings must not do.
__device__ __forceinline__ int lds_load(int* p) {
    const int v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return v;
}
__device__ __forceinline__ void lds_store(int* p, int v) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until this wavefront's vector memory operations have completed (vmcnt(0); expcnt and
// lgkmcnt unconstrained).
__device__ __forceinline__ void wait_vm_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

}  // namespace dlr
