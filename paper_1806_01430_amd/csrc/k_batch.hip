// Grouped kernels of instance batches: one launch runs one nest of every
// instance.  The grid is persistent (a few blocks per CU) and walks a global
// range of work units -- 1024-element runs for the initialisation, output
// tiles for the product, sweep items for the stencil, groups of rows for the
// copy -- finding each unit's instance by binary search over the job table.
// The per-unit code is the single-instance kernels' own (gemm_tile.hpp,
// stencil_item.hpp), so a grouped launch computes bit for bit what the
// single launches compute for the same tile shape.
//
// Blocks are renumbered so that each XCD takes a contiguous run of logical
// block indices; with units dealt round-robin over logical blocks, the units
// in flight on one XCD at a time are neighbours (tiles of one product share
// A panels, stencil items of one grid share halo rows in that XCD's L2).
#include <hip/hip_runtime.h>

#include <mutex>

#include "batch_jobs.hpp"
#include "dev_common.hpp"
#include "gemm_tile.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "stencil_item.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;

__device__ inline int logical_block() {
    const int nb = gridDim.x;
    return (nb % 8) ? (int)blockIdx.x : (int)(blockIdx.x % 8) * (nb / 8) + (int)blockIdx.x / 8;
}

// Last job whose first unit is <= u (jobs sorted by begin, jobs[0].begin = 0).
template <typename Job, typename Index>
__device__ inline int find_job(const Job *jobs, int njobs, Index u, Index Job::*begin) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*begin <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_init_grouped(const InitJob *__restrict__ jobs, int njobs,
                                                           int64_t nunits) {
    for (int64_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int j = find_job(jobs, njobs, u, &InitJob::unit_begin);
        float *x = jobs[j].x;
        const int64_t n = jobs[j].n;
        const uint64_t key = jobs[j].key;
        const int64_t e0 = (u - jobs[j].unit_begin) * kInitUnit;
#pragma unroll
        for (int t = 0; t < kInitUnit / kThreads; ++t) {
            const int64_t e = e0 + t * kThreads + threadIdx.x;
            if (e < n) x[e] = uniform24(key, e);
        }
    }
}

template <int BM, int BK>
__global__ __launch_bounds__(kThreads) void k_gemm_grouped(const GemmJob *__restrict__ jobs, int njobs, int ntiles) {
    __shared__ GemmLds<BM, BM, BK> sm;
    for (int t = logical_block(); t < ntiles; t += gridDim.x) {
        const int j = find_job(jobs, njobs, t, &GemmJob::tile_begin);
        const GemmJob jb = jobs[j];
        const int lt = t - jb.tile_begin;
        const int m0 = (lt / jb.tiles_n) * BM, n0 = (lt % jb.tiles_n) * BM;
        if (jb.vec) gemm_f32_tile<BM, BM, BK, true>(jb.A, jb.B, jb.C, jb.M, jb.N, jb.K, m0, n0, sm);
        else gemm_f32_tile<BM, BM, BK, false>(jb.A, jb.B, jb.C, jb.M, jb.N, jb.K, m0, n0, sm);
    }
}

// One wave per item; the item's residual terms go, summed over the wave, to
// partials[item] (the finish kernel adds them per instance in item order).
template <int JR>
__global__ __launch_bounds__(kThreads) void k_stencil_grouped(const StencilJob *__restrict__ jobs, int njobs,
                                                              int nitems, double *__restrict__ partials) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = gridDim.x * kWaves;
    for (int w = logical_block() * kWaves + wib; w < nitems; w += nwaves) {
        const int j = find_job(jobs, njobs, w, &StencilJob::item_begin);
        const Geo g = jobs[j].g;
        const __amdgpu_buffer_rsrc_t rp =
            __builtin_amdgcn_make_buffer_rsrc((void *)jobs[j].p, (short)0, g.bytes, kBufferConfig);
        const __amdgpu_buffer_rsrc_t rq =
            __builtin_amdgcn_make_buffer_rsrc((void *)jobs[j].q, (short)0, g.bytes, kBufferConfig);
        double acc = stencil_item<JR>(rp, rq, g, w - jobs[j].item_begin, lane, 0.0);
        acc = wave_sum(acc);
        if (lane == 0) partials[w] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_stencil_finish(const StencilJob *__restrict__ jobs, int njobs,
                                                             int nitems, const double *__restrict__ partials,
                                                             int64_t slot) {
    __shared__ double wsum[kWaves];
    const int j = blockIdx.x;
    const int b = jobs[j].item_begin, e = j + 1 < njobs ? jobs[j + 1].item_begin : nitems;
    double s = 0.0;
    for (int i = b + (int)threadIdx.x; i < e; i += kThreads) s += partials[i];
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w];
        double *target = jobs[j].res + slot;
        *target = *target + t;
    }
}

__global__ __launch_bounds__(kThreads) void k_copy_grouped(const CopyJob *__restrict__ jobs, int njobs, int nunits) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = gridDim.x * kWaves;
    for (int u = logical_block() * kWaves + wib; u < nunits; u += nwaves) {
        const int j = find_job(jobs, njobs, u, &CopyJob::unit_begin);
        const CopyJob c = jobs[j];
        const int bytes = c.I * c.J * c.K * 4;
        const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)c.q, (short)0, bytes, kBufferConfig);
        const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)c.p, (short)0, bytes, kBufferConfig);
        copy_rows(rp, rq, c.J, c.K, c.rows, (u - c.unit_begin) * kRows, lane);
    }
}

template <typename F>
int occupancy_of(F kernel) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

constexpr int kCfgBM[kGemmCfgs] = {64, 64, 64, 128, 128, 128, 256, 256};
constexpr int kCfgBK[kGemmCfgs] = {16, 32, 64, 16, 32, 64, 16, 32};

}  // namespace

void gemm_cfg_shape(int cfg, int *bm, int *bk) {
    if (cfg < 0 || cfg >= kGemmCfgs) cfg = 1;
    *bm = kCfgBM[cfg];
    *bk = kCfgBK[cfg];
}

int grouped_gemm_occupancy(int cfg) {
    static std::once_flag once;
    static int table[kGemmCfgs];
    std::call_once(once, [] {
        table[0] = occupancy_of(k_gemm_grouped<64, 16>);
        table[1] = occupancy_of(k_gemm_grouped<64, 32>);
        table[2] = occupancy_of(k_gemm_grouped<64, 64>);
        table[3] = occupancy_of(k_gemm_grouped<128, 16>);
        table[4] = occupancy_of(k_gemm_grouped<128, 32>);
        table[5] = occupancy_of(k_gemm_grouped<128, 64>);
        table[6] = occupancy_of(k_gemm_grouped<256, 16>);
        table[7] = occupancy_of(k_gemm_grouped<256, 32>);
    });
    return table[(cfg < 0 || cfg >= kGemmCfgs) ? 1 : cfg];
}

int grouped_stencil_occupancy(int JR) {
    static std::once_flag once;
    static int table[3];
    std::call_once(once, [] {
        table[0] = occupancy_of(k_stencil_grouped<2>);
        table[1] = occupancy_of(k_stencil_grouped<4>);
        table[2] = occupancy_of(k_stencil_grouped<8>);
    });
    return table[JR == 2 ? 0 : (JR == 4 ? 1 : 2)];
}

int grouped_copy_occupancy() {
    static std::once_flag once;
    static int n = 1;
    std::call_once(once, [] { n = occupancy_of(k_copy_grouped); });
    return n;
}

hipError_t init_grouped(const InitJob *jobs, int njobs, int64_t nunits, unsigned blocks, hipStream_t s) {
    if (njobs <= 0 || nunits <= 0) return hipSuccess;
    return launch(k_init_grouped, dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, nunits);
}

hipError_t gemm_grouped(int cfg, const GemmJob *jobs, int njobs, int ntiles, unsigned blocks, hipStream_t s) {
    if (njobs <= 0 || ntiles <= 0) return hipSuccess;
    switch (cfg) {
    case 0: return launch((k_gemm_grouped<64, 16>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 1: return launch((k_gemm_grouped<64, 32>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 2: return launch((k_gemm_grouped<64, 64>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 3: return launch((k_gemm_grouped<128, 16>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 4: return launch((k_gemm_grouped<128, 32>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 5: return launch((k_gemm_grouped<128, 64>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 6: return launch((k_gemm_grouped<256, 16>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    case 7: return launch((k_gemm_grouped<256, 32>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, ntiles);
    default: return hipErrorInvalidValue;
    }
}

hipError_t stencil_grouped(int JR, const StencilJob *jobs, int njobs, int nitems, double *partials, unsigned blocks,
                           hipStream_t s) {
    if (njobs <= 0 || nitems <= 0) return hipSuccess;
    if (JR == 2) return launch((k_stencil_grouped<2>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, nitems, partials);
    if (JR == 4) return launch((k_stencil_grouped<4>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, nitems, partials);
    if (JR == 8) return launch((k_stencil_grouped<8>), dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, nitems, partials);
    return hipErrorInvalidValue;
}

hipError_t stencil_finish(const StencilJob *jobs, int njobs, int nitems, const double *partials, int64_t slot,
                          hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    return launch(k_stencil_finish, dim3((unsigned)njobs), dim3(kThreads), 0, s, jobs, njobs, nitems, partials, slot);
}

hipError_t copy_grouped(const CopyJob *jobs, int njobs, int nunits, unsigned blocks, hipStream_t s) {
    if (njobs <= 0 || nunits <= 0) return hipSuccess;
    return launch(k_copy_grouped, dim3(blocks), dim3(kThreads), 0, s, jobs, njobs, nunits);
}

}  // namespace k
}  // namespace ofl
