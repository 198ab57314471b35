// Device helpers shared by the kernels: FP64 wave / block sums and the
// deterministic "last block finishes" reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ofl {
namespace k {

constexpr int kWave = 64;

// SplitMix64 (Steele, Lea & Flood 2014) output function and the
// counter-based U[0,1) value of element e under a stream key: the top 24 bits
// of mix64(key + (e + 1) * golden), scaled by 2^-24.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline float uniform24(uint64_t key, int64_t e) {
    return (float)(mix64(key + (uint64_t)(e + 1) * kGolden) >> 40) * (1.0f / 16777216.0f);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Called by every thread of the block with its own partial.  Thread 0 of each
// block publishes the block's sum; the block that completes last adds all
// partials, in block order, to target[0] and returns the counter to zero.  The
// combination order depends only on the grid, so results are reproducible.
// Ordering: each block's counter increment is a release (its partial is
// written back before the increment), and only the reading lanes of the last
// block acquire, each with an acquire load of the counter (it reads the final
// increment, which continues every block's release sequence).  An acquire in
// every block would invalidate the L2 of its XCD once per block, evicting
// lines that the blocks still running there are about to read.
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
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == nb - 1) ? 1 : 0;
    }
    __syncthreads();
    if (last && w == 0) {
        (void)__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
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
