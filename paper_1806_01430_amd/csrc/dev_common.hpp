// Device helpers shared by the kernels: FP64 wave / block sums and the
// deterministic "last block finishes" reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ofl {
namespace k {

constexpr int kWave = 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Called by every thread of the block with its own partial.  Thread 0 of each
// block publishes the block's sum; the block that completes last adds all
// partials, in block order, to target[0] and returns the counter to zero.  The
// combination order depends only on the grid, so results are reproducible.
__device__ inline void reduce_finish(double v, double *partials, unsigned *counter, double *target) {
    __shared__ double wsum[16];
    __shared__ int last;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_sum(v);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i) t += wsum[i];
        const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        __hip_atomic_store(&partials[bid], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == nb - 1) ? 1 : 0;
    }
    __syncthreads();
    if (last && w == 0) {
        __threadfence();
        double s = 0.0;
        for (unsigned i = lane; i < nb; i += kWave)
            s += __hip_atomic_load(&partials[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s = wave_sum(s);
        if (lane == 0) {
            target[0] = target[0] + s;
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace k
}  // namespace ofl
