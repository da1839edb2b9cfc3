// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace dfmg {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Remapping the hardware block id so that each XCD works
// on one contiguous eighth of the rows keeps neighbouring rows (which share
// most of the vector entries a stencil row reads) in the same L2.
__device__ __forceinline__ int xcd_block(int hw, int grid) {
    const int per = grid >> 3;  // grid is a multiple of 8
    return (hw & 7) * per + (hw >> 3);
}

// A load of a value that is the same for the whole block (a problem's
// damping) as a vector load: it then travels beside the block's other loads,
// where a scalar load would be waited for by the first later scalar load (the
// kernel arguments).  The relaxed atomic keeps the compiler from turning it
// into a scalar load.
template <class T>
__device__ __forceinline__ T uniform_vload(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// the wide flags of calls without flags (never written)
__device__ int kNoStop[kStopLanes] = {};

// A problem's stop flag from its wide form (0 when there are no flags): lane i
// reads copy i, unconditionally, so the value stays per lane and the compiler
// tests it where it is used.
__device__ __forceinline__ int stop_flag(const int *stopw, int prob) {
    const int lane = threadIdx.x & 63;
    return stopw ? stopw[prob * kStopLanes + lane] : kNoStop[lane];
}

// A load from a wave-uniform address of data the kernel does not write (the
// local inverses): through the constant address space, so the compiler reads
// it with scalar loads (one per wave, from the scalar cache) instead of one
// vector load per lane.
template <class T>
__device__ __forceinline__ T scalar_ld(const T *p) {
    return *reinterpret_cast<const __attribute__((address_space(4))) T *>(
        reinterpret_cast<uintptr_t>(p));
}

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Sum over the block (wave shuffles, then the waves in a fixed order); the
// result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

}  // namespace dfmg
