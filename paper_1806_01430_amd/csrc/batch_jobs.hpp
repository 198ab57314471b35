// Work tables of the grouped kernels that run one nest of every instance of a
// batch in a single launch.  Each table lists one job per instance, sorted as
// the host chose, with the prefix index of the job's first work unit; a
// persistent grid walks the global unit range and finds a unit's job by
// binary search over those prefixes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "stencil_item.hpp"

namespace ofl {
namespace k {

constexpr int kInitUnit = 1024;   // elements per unit of the grouped initialisation

struct InitJob {
    float *x;
    int64_t n;
    uint64_t key;
    int64_t unit_begin;
};

struct GemmJob {
    const float *A, *B;
    float *C;
    int M, N, K;
    int tiles_n;       // tiles along N
    int tile_begin;
    int vec;           // K and N multiples of 4: 16-byte global loads
};

struct StencilJob {
    const float *p;
    float *q;
    double *res;       // residual buffer of the instance (slot added at launch)
    Geo g;
    int item_begin;
};

struct CopyJob {
    float *p;
    const float *q;
    int I, J, K;
    int rows;          // (I - 2) * (J - 2)
    int unit_begin;    // units of kRows rows
};

// FP32 tile shapes of the grouped product: index -> (BM = BN, BK).
constexpr int kGemmCfgs = 8;
void gemm_cfg_shape(int cfg, int *bm, int *bk);

Geo make_geo(int64_t I, int64_t J, int64_t K, int JR, int IC, int kout = kOut);
int cu_count();
int grouped_gemm_occupancy(int cfg);
int grouped_stencil_occupancy(int JR);
int grouped_copy_occupancy();

hipError_t init_grouped(const InitJob *jobs, int njobs, int64_t nunits, unsigned blocks, hipStream_t s);
hipError_t gemm_grouped(int cfg, const GemmJob *jobs, int njobs, int ntiles, unsigned blocks, hipStream_t s);
hipError_t stencil_grouped(int JR, const StencilJob *jobs, int njobs, int nitems, double *partials, unsigned blocks,
                           hipStream_t s);
// res[slot] += sum of the job's item partials, in item order (one block per job)
hipError_t stencil_finish(const StencilJob *jobs, int njobs, int nitems, const double *partials, int64_t slot,
                          hipStream_t s);
hipError_t copy_grouped(const CopyJob *jobs, int njobs, int nunits, unsigned blocks, hipStream_t s);

}  // namespace k
}  // namespace ofl
