// Block reductions for the fused dot products of the CG iteration.  Each block
// writes one partial; a single-block kernel sums the partials in a fixed
// order, so every dot product is reproducible run to run.  (No block waits for
// another and no device-scope fence is issued inside a streaming kernel.)
#pragma once

#include <hip/hip_runtime.h>

namespace hb {

// Sum over a wave64 by butterfly exchanges.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the whole block (all threads must call it); result valid in every thread.
// `scratch` needs blockDim.x / 64 doubles of shared memory.
__device__ inline double block_sum(double v, double *scratch)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();  // scratch may still be in use by a previous call
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nwaves; ++i) s += scratch[i];
    return s;
}

// Workgroups are dispatched to the 8 XCDs of the device in turn (id mod 8).
// Give each XCD a contiguous range of tiles so that tiles sharing data
// (neighbouring elements) are served by the same L2.  A bijection on [0, n).
__device__ inline int xcd_remap(int bid, int n)
{
    constexpr int X = 8;
    const int per = n / X, rem = n % X;
    const int xcd = bid % X, k = bid / X;
    return xcd * per + (xcd < rem ? xcd : rem) + k;
}

}  // namespace hb
