// Element-wise, copy, cast, transpose, sum-of-squares and initialisation
// kernels.  All are bound by HBM bandwidth: 16-byte vector accesses where the
// element count allows, grid-stride loops sized to a few waves per SIMD.
#include <hip/hip_runtime.h>

#include "dev_common.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kThreads = 256;

// Blocks for work_items units of per_thread items, at most cap (256 CUs x 32
// blocks by default: grid-stride beyond that).  The element-wise updates and
// the cast (one 16-byte piece of each operand per thread and iteration) take
// the larger cap kStreamCap, so that on large arrays more blocks keep more
// loads in flight: at 8192 x 8192 (16384 blocks of 4 pieces per thread
// instead of 8192 of 8) on gfx950 add_scaled 148 vs 175 us, avg2 158 vs 178,
// cast_bf16 74 vs 83, scale 79 vs 84; init_uniform and the sum of squares
// gained nothing.
constexpr int64_t kStreamCap = 65536;
inline unsigned grid_for(int64_t work_items, int per_thread = 1, int64_t cap = 8192) {
    int64_t blocks = (work_items + (int64_t)kThreads * per_thread - 1) / ((int64_t)kThreads * per_thread);
    if (blocks < 1) blocks = 1;
    if (blocks > cap) blocks = cap;
    return (unsigned)blocks;
}

__global__ __launch_bounds__(kThreads) void k_fill_zero(uint4 *dst, int64_t n16, unsigned char *tail, int ntail) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads) void k_init_uniform(float *x, int64_t n, uint64_t key) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += stride) {
        const int64_t e = g * 4;
        float4 v;
        v.x = uniform24(key, e);
        v.y = uniform24(key, e + 1);
        v.z = uniform24(key, e + 2);
        v.w = uniform24(key, e + 3);
        reinterpret_cast<float4 *>(x)[g] = v;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const int64_t e = n4 * 4 + threadIdx.x;
        x[e] = uniform24(key, e);
    }
}

__global__ __launch_bounds__(kThreads) void k_add_scaled(float *C, const float *A, float alpha, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += stride) {
        float4 c = reinterpret_cast<float4 *>(C)[g];
        const float4 a = reinterpret_cast<const float4 *>(A)[g];
        c.x = c.x + alpha * a.x;
        c.y = c.y + alpha * a.y;
        c.z = c.z + alpha * a.z;
        c.w = c.w + alpha * a.w;
        reinterpret_cast<float4 *>(C)[g] = c;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const int64_t e = n4 * 4 + threadIdx.x;
        C[e] = C[e] + alpha * A[e];
    }
}

__global__ __launch_bounds__(kThreads) void k_avg2(float *S, const float *X, const float *Y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += stride) {
        const float4 x = reinterpret_cast<const float4 *>(X)[g];
        const float4 y = reinterpret_cast<const float4 *>(Y)[g];
        float4 s;
        s.x = 0.5f * (x.x + y.x);
        s.y = 0.5f * (x.y + y.y);
        s.z = 0.5f * (x.z + y.z);
        s.w = 0.5f * (x.w + y.w);
        reinterpret_cast<float4 *>(S)[g] = s;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const int64_t e = n4 * 4 + threadIdx.x;
        S[e] = 0.5f * (X[e] + Y[e]);
    }
}

__global__ __launch_bounds__(kThreads) void k_scale(float *D, float beta, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += stride) {
        float4 d = reinterpret_cast<float4 *>(D)[g];
        d.x = beta * d.x;
        d.y = beta * d.y;
        d.z = beta * d.z;
        d.w = beta * d.w;
        reinterpret_cast<float4 *>(D)[g] = d;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const int64_t e = n4 * 4 + threadIdx.x;
        D[e] = beta * D[e];
    }
}

__global__ __launch_bounds__(kThreads) void k_copy16(uint4 *dst, const uint4 *src, int64_t n16,
                                                     unsigned char *dtail, const unsigned char *stail, int ntail) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) dtail[threadIdx.x] = stail[threadIdx.x];
}

// Copies and fills of kLargeBytes and more (restores of a large grid's set-up
// content): one 16-byte piece per lane, no grid-stride loop, streaming loads
// and stores -- the form that moves the 1 GB grids fastest (no dirty lines
// are left behind for the next kernel to write back).
constexpr uint64_t kLargeBytes = (uint64_t)512 << 20;
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_copy16_stream(u32x4v *dst, const u32x4v *src, int64_t n16,
                                                            unsigned char *dtail, const unsigned char *stail,
                                                            int ntail) {
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) dtail[threadIdx.x] = stail[threadIdx.x];
}

__global__ __launch_bounds__(kThreads) void k_fill_zero_stream(u32x4v *dst, int64_t n16, unsigned char *tail,
                                                               int ntail) {
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(u32x4v{0u, 0u, 0u, 0u}, dst + i);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__device__ inline unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__global__ __launch_bounds__(kThreads) void k_cast_bf16(unsigned short *dst, const float *src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += stride) {
        const float4 v = reinterpret_cast<const float4 *>(src)[g];
        uint2 o;
        o.x = (unsigned)bf16_rne(v.x) | ((unsigned)bf16_rne(v.y) << 16);
        o.y = (unsigned)bf16_rne(v.z) | ((unsigned)bf16_rne(v.w) << 16);
        reinterpret_cast<uint2 *>(dst)[g] = o;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const int64_t e = n4 * 4 + threadIdx.x;
        dst[e] = bf16_rne(src[e]);
    }
}

// T[c][r] = X[r][c]; 64 x 64 tiles through LDS (+1 column of padding so the
// transposed read hits 64 distinct banks).
constexpr int kTile = 64;
__global__ __launch_bounds__(kThreads) void k_transpose(const float *__restrict__ X, float *__restrict__ T,
                                                        int64_t R, int64_t Cc) {
    __shared__ float tile[kTile][kTile + 1];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kTile, r0 = (int64_t)blockIdx.y * kTile;
#pragma unroll
    for (int r = ty; r < kTile; r += kThreads / kTile) {
        const int64_t row = r0 + r, col = c0 + tx;
        if (row < R && col < Cc) tile[r][tx] = X[row * Cc + col];
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < kTile; r += kThreads / kTile) {
        const int64_t orow = c0 + r, ocol = r0 + tx;   // T is Cc x R
        if (orow < Cc && ocol < R) T[orow * R + ocol] = tile[tx][r];
    }
}

// The same transpose with 16-byte accesses, for R and Cc multiples of 4: a
// thread reads four float4 pieces of the tile's rows and, after the barrier,
// writes four float4 pieces of T, each gathering 4 consecutive tile rows of
// one column from LDS (row pitch 65: the 64 lanes of a wave hit 64 distinct
// banks).
__global__ __launch_bounds__(kThreads) void k_transpose4(const float *__restrict__ X, float *__restrict__ T,
                                                         int64_t R, int64_t Cc) {
    __shared__ float tile[kTile][kTile + 1];
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * kTile, r0 = (int64_t)blockIdx.y * kTile;
    const int q = t % 16;   // float4 piece within a 64-wide row
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = t / 16 + 16 * i;
        const int64_t row = r0 + r, col = c0 + 4 * q;
        if (row < R && col < Cc) {   // Cc % 4 == 0: the piece is whole
            const float4 v = *reinterpret_cast<const float4 *>(X + row * Cc + col);
            tile[r][4 * q] = v.x;
            tile[r][4 * q + 1] = v.y;
            tile[r][4 * q + 2] = v.z;
            tile[r][4 * q + 3] = v.w;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = t / 16 + 16 * i;
        const int64_t orow = c0 + c, ocol = r0 + 4 * q;   // T is Cc x R
        if (orow < Cc && ocol < R) {   // R % 4 == 0: the piece is whole
            float4 v;
            v.x = tile[4 * q][c];
            v.y = tile[4 * q + 1][c];
            v.z = tile[4 * q + 2][c];
            v.w = tile[4 * q + 3][c];
            *reinterpret_cast<float4 *>(T + orow * R + ocol) = v;
        }
    }
}

// s[0] += sum of x[e]^2 in FP64 (the FP32 values widened exactly).  The sum
// kernel leaves one partial per block with a plain store (per thread in
// element order, U loads of 16 bytes in flight; the waves of a block then in
// wave order); k_sumsq_finish, launched next on the same stream, adds the
// partials in a fixed order.  No atomics and no grid-wide release: a release
// per block would write back the L2 of its XCD once per block.
template <int U>
__global__ __launch_bounds__(kThreads) void k_sumsq(const float *__restrict__ x, int64_t n, double *partials) {
    __shared__ double wsum[kThreads / kWave];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = n / 4;
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    double acc = 0.0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n4; g += U * stride) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = g + u * stride < n4 ? x4[g + u * stride] : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double a = v[u].x, b = v[u].y, c = v[u].z, d = v[u].w;
            acc = acc + a * a;
            acc = acc + b * b;
            acc = acc + c * c;
            acc = acc + d * d;
        }
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < (int)(n - n4 * 4)) {
        const double a = x[n4 * 4 + threadIdx.x];
        acc = acc + a * a;
    }
    acc = wave_sum(acc);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / kWave; ++i) t += wsum[i];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kOrderedSumThreads) void k_sumsq_finish(const double *__restrict__ partials, int n,
                                                                     double *s_out) {
    ordered_sum_into(partials, n, s_out);
}

// out[i] = element idx[i] of src, widened to double (dtype 0 f32, 1 f64,
// 2 bf16): the probes of an output check.
__global__ __launch_bounds__(kThreads) void k_gather_probes(const void *__restrict__ src, int dtype,
                                                            const int64_t *__restrict__ idx, int n,
                                                            double *__restrict__ out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int64_t e = idx[i];
    double v;
    if (dtype == 1) {
        v = static_cast<const double *>(src)[e];
    } else if (dtype == 2) {
        v = (double)__uint_as_float((unsigned)static_cast<const unsigned short *>(src)[e] << 16);
    } else {
        v = (double)static_cast<const float *>(src)[e];
    }
    out[i] = v;
}

}  // namespace

hipError_t gather_probes(const void *src, int dtype, const int64_t *idx, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_gather_probes, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, src,
                  dtype, idx, n, out);
}

hipError_t fill_zero(void *dst, uint64_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int ntail = (int)(bytes - (uint64_t)n16 * 16);
    if (bytes >= kLargeBytes && (n16 + kThreads - 1) / kThreads < ((int64_t)1 << 31))
        return launch(k_fill_zero_stream, dim3((unsigned)((n16 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                      static_cast<u32x4v *>(dst), n16, static_cast<unsigned char *>(dst) + n16 * 16, ntail);
    return launch(k_fill_zero, dim3(grid_for(n16 > 0 ? n16 : 1, 4)), dim3(kThreads), 0, s,
                       static_cast<uint4 *>(dst), n16, static_cast<unsigned char *>(dst) + n16 * 16, ntail);
}

hipError_t init_uniform(float *x, int64_t n, uint64_t key, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_init_uniform, dim3(grid_for(n / 4 + 1, 2)), dim3(kThreads), 0, s, x, n, key);
}

hipError_t add_scaled(float *C, const float *A, float alpha, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_add_scaled, dim3(grid_for(n / 4 + 1, 4, kStreamCap)), dim3(kThreads), 0, s, C, A, alpha, n);
}

hipError_t avg2(float *S, const float *X, const float *Y, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_avg2, dim3(grid_for(n / 4 + 1, 4, kStreamCap)), dim3(kThreads), 0, s, S, X, Y, n);
}

hipError_t scale(float *D, float beta, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_scale, dim3(grid_for(n / 4 + 1, 4, kStreamCap)), dim3(kThreads), 0, s, D, beta, n);
}

hipError_t copy_bytes(void *dst, const void *src, uint64_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int ntail = (int)(bytes - (uint64_t)n16 * 16);
    if (bytes >= kLargeBytes && (n16 + kThreads - 1) / kThreads < ((int64_t)1 << 31))
        return launch(k_copy16_stream, dim3((unsigned)((n16 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                      static_cast<u32x4v *>(dst), static_cast<const u32x4v *>(src), n16,
                      static_cast<unsigned char *>(dst) + n16 * 16,
                      static_cast<const unsigned char *>(src) + n16 * 16, ntail);
    return launch(k_copy16, dim3(grid_for(n16 > 0 ? n16 : 1, 4)), dim3(kThreads), 0, s,
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n16,
                       static_cast<unsigned char *>(dst) + n16 * 16,
                       static_cast<const unsigned char *>(src) + n16 * 16, ntail);
}

hipError_t cast_bf16(uint16_t *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return launch(k_cast_bf16, dim3(grid_for(n / 4 + 1, 4, kStreamCap)), dim3(kThreads), 0, s,
                       reinterpret_cast<unsigned short *>(dst), src, n);
}

hipError_t transpose(const float *X, float *T, int64_t R, int64_t Cc, hipStream_t s) {
    if (R <= 0 || Cc <= 0) return hipSuccess;
    dim3 grid((unsigned)((Cc + kTile - 1) / kTile), (unsigned)((R + kTile - 1) / kTile));
    if (grid.y > 65535) return hipErrorInvalidValue;
    // 16-byte accesses when both sides are multiples of 4 (buffers are
    // 16-byte aligned): 8192 x 8192 in 102 us instead of 138 us
    if (R % 4 == 0 && Cc % 4 == 0) return launch(k_transpose4, grid, dim3(kThreads), 0, s, X, T, R, Cc);
    return launch(k_transpose, grid, dim3(kThreads), 0, s, X, T, R, Cc);
}

constexpr int kSumsqUnroll = 4;

int64_t sumsq_partials(int64_t n) { return grid_for(n / 4 + 1, 2 * kSumsqUnroll); }

hipError_t sumsq(const float *x, int64_t n, double *s_out, const ReduceScratch &rs, hipStream_t s) {
    const unsigned blocks = (unsigned)sumsq_partials(n);
    if ((int64_t)blocks > rs.capacity) return hipErrorInvalidValue;
    const hipError_t e = launch(k_sumsq<kSumsqUnroll>, dim3(blocks), dim3(kThreads), 0, s, x, n, rs.partials);
    if (e != hipSuccess) return e;
    return launch(k_sumsq_finish, dim3(1), dim3(kOrderedSumThreads), 0, s, (const double *)rs.partials,
                  (int)blocks, s_out);
}

}  // namespace k
}  // namespace ofl
