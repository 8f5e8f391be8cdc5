// Wavefront-level primitives shared by the sweep kernels: the one-lane DPP shift that
// hands a value from lane l-1 to lane l, LDS progress words, and the wait that makes this
// wavefront's global stores complete before it publishes them.
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
