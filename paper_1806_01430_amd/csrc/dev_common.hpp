// Device helpers shared by the kernels: the counter-based uniform values, the
// FP64 wave sum and the fixed-order sum of per-block partials.
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

// slot[0] += partials[0] + ... + partials[n-1], summed in a fixed order by
// one whole block of kOrderedSumThreads threads: thread t adds partials t,
// t + 256, ... (loads unrolled so that they overlap), then a tree over the
// threads in LDS.  The order depends only on n, so the result is
// reproducible run to run.
constexpr int kOrderedSumThreads = 256;

__device__ inline void ordered_sum_into(const double *__restrict__ partials, int n, double *slot) {
    __shared__ double t[kOrderedSumThreads];
    const int tid = threadIdx.x;
    double s = 0.0;
    int i = tid;
    for (; i + 3 * kOrderedSumThreads < n; i += 4 * kOrderedSumThreads) {
        const double a = partials[i], b = partials[i + kOrderedSumThreads];
        const double c = partials[i + 2 * kOrderedSumThreads], d = partials[i + 3 * kOrderedSumThreads];
        s += a;
        s += b;
        s += c;
        s += d;
    }
    for (; i < n; i += kOrderedSumThreads) s += partials[i];
    t[tid] = s;
    __syncthreads();
#pragma unroll
    for (int h = kOrderedSumThreads / 2; h > 0; h >>= 1) {
        if (tid < h) t[tid] += t[tid + h];
        __syncthreads();
    }
    if (tid == 0) slot[0] = slot[0] + t[0];
}

}  // namespace k
}  // namespace ofl
