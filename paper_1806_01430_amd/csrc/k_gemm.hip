// Dense matrix product C = A * B (row-major) on the MFMA matrix cores.
//
// FP32: v_mfma_f32_16x16x4_f32 (gfx950 has no XF32, so the product is true
// FP32 with FP32 accumulation).  BF16: v_mfma_f32_16x16x32_bf16 with FP32
// accumulation.  A block of 256 threads (4 waves, 2 x 2) owns a BM x BN tile
// of C; each wave a (BM/2) x (BN/2) sub-tile as (BM/32) x (BN/32) 16x16
// accumulators.  K advances in slabs of BK staged through LDS, double
// buffered: the next slab is fetched from global memory into registers while
// the current one feeds the MFMAs.
//
// Within one MFMA the k index of lane l's operands is (l / 16, slot); any
// assignment of real k values to (lane group, slot) gives the same sum as
// long as A and B use the same one.  Here lane group g takes the contiguous
// run k = g*S .. g*S + S - 1 of the slab, so every lane reads its A operands
// with one wide LDS load.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// receives a contiguous run of output tiles (rows of tiles share A panels in
// that XCD's L2).
__device__ inline int xcd_swizzle(int bid, int nblocks) {
    const int nx = 8;
    if (nblocks % nx) return bid;
    return (bid % nx) * (nblocks / nx) + bid / nx;
}

template <int BM, int BN, int BK, bool VEC>
__global__ __launch_bounds__(kThreads) void k_gemm_f32(const float *__restrict__ A, const float *__restrict__ B,
                                                       float *__restrict__ C, int M, int N, int K) {
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LDA = BK + 4;          // As[m][k], 16-byte aligned rows, conflict-free b128 reads
    constexpr int LDB = BN + 4;          // Bs[k][n]
    constexpr int A_PER = BM * BK / 4 / kThreads;
    constexpr int B_PER = BK * BN / 4 / kThreads;
    static_assert(A_PER * 4 * kThreads == BM * BK && B_PER * 4 * kThreads == BK * BN, "tile / thread mismatch");
    __shared__ float As[2][BM * LDA];
    __shared__ float Bs[2][BK * LDB];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int tiles_n = (N + BN - 1) / BN;
    const int tiles = tiles_n * ((M + BM - 1) / BM);
    const int t = xcd_swizzle(blockIdx.x, tiles);
    const int m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * BN;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    float4 ra[A_PER], rb[B_PER];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (BK / 4), c4 = (idx % (BK / 4)) * 4;
            const int gm = m0 + row, gk = k0 + c4;
            if (VEC) {
                ra[s] = (gm < M && gk < K) ? *reinterpret_cast<const float4 *>(A + (size_t)gm * K + gk)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                const float *src = A + (size_t)gm * K + gk;
                const bool rin = gm < M;
                ra[s].x = (rin && gk < K) ? src[0] : 0.f;
                ra[s].y = (rin && gk + 1 < K) ? src[1] : 0.f;
                ra[s].z = (rin && gk + 2 < K) ? src[2] : 0.f;
                ra[s].w = (rin && gk + 3 < K) ? src[3] : 0.f;
            }
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
            const int gk = k0 + row, gn = n0 + c4;
            if (VEC) {
                rb[s] = (gk < K && gn < N) ? *reinterpret_cast<const float4 *>(B + (size_t)gk * N + gn)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                const float *src = B + (size_t)gk * N + gn;
                const bool kin = gk < K;
                rb[s].x = (kin && gn < N) ? src[0] : 0.f;
                rb[s].y = (kin && gn + 1 < N) ? src[1] : 0.f;
                rb[s].z = (kin && gn + 2 < N) ? src[2] : 0.f;
                rb[s].w = (kin && gn + 3 < N) ? src[3] : 0.f;
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (BK / 4), c4 = (idx % (BK / 4)) * 4;
            *reinterpret_cast<float4 *>(&As[buf][row * LDA + c4]) = ra[s];
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
            *reinterpret_cast<float4 *>(&Bs[buf][row * LDB + c4]) = rb[s];
        }
    };
    const int r = lane & 15, g = lane >> 4;
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            float4 af[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const float4 *>(&As[buf][(wm * WM + i * 16 + r) * LDA + ks + 4 * g]);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float bf[TN];
#pragma unroll
                for (int j = 0; j < TN; ++j) bf[j] = Bs[buf][(ks + 4 * g + s) * LDB + wn * WN + j * 16 + r];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const float a = s == 0 ? af[i].x : s == 1 ? af[i].y : s == 2 ? af[i].z : af[i].w;
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    };

    const int nk = (K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        compute(cur);
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    // lane l, register e of a 16x16 accumulator: row 4*(l/16) + e, column l % 16
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * WM + i * 16 + 4 * g + e, col = n0 + wn * WN + j * 16 + r;
                if (row < M && col < N) C[(size_t)row * N + col] = acc[i][j][e];
            }
}

// BF16 inputs: As[m][k] and Bs[n][k] (B transposed on its way into LDS) so
// that each lane's 8 consecutive k values are one 16-byte LDS read.
template <int BM, int BN>
__global__ __launch_bounds__(kThreads) void k_gemm_bf16(const unsigned short *__restrict__ A,
                                                        const unsigned short *__restrict__ B, float *__restrict__ C,
                                                        int M, int N, int K) {
    constexpr int BK = 32;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LD = BK + 8;           // in bf16 elements (80 bytes per row)
    __shared__ unsigned short As[BM * LD];
    __shared__ unsigned short Bs[BN * LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int tiles_n = (N + BN - 1) / BN;
    const int tiles = tiles_n * ((M + BM - 1) / BM);
    const int t = xcd_swizzle(blockIdx.x, tiles);
    const int m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * BN;
    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += BK) {
        // A: BM x 32 elements, element-wise guarded
        for (int idx = tid; idx < BM * BK; idx += kThreads) {
            const int row = idx / BK, kk = idx % BK, gm = m0 + row, gk = k0 + kk;
            As[row * LD + kk] = (gm < M && gk < K) ? A[(size_t)gm * K + gk] : (unsigned short)0;
        }
        // B: 32 x BN elements read along n, stored transposed
        for (int idx = tid; idx < BK * BN; idx += kThreads) {
            const int kk = idx / BN, col = idx % BN, gk = k0 + kk, gn = n0 + col;
            Bs[col * LD + kk] = (gk < K && gn < N) ? B[(size_t)gk * N + gn] : (unsigned short)0;
        }
        __syncthreads();
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[(wm * WM + i * 16 + r) * LD + 8 * g]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[(wn * WN + j * 16 + r) * LD + 8 * g]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * WM + i * 16 + 4 * g + e, col = n0 + wn * WN + j * 16 + r;
                if (row < M && col < N) C[(size_t)row * N + col] = acc[i][j][e];
            }
}

template <int BM, int BN, int BK>
hipError_t launch_f32(const float *A, const float *B, float *C, int M, int N, int K, hipStream_t s) {
    const unsigned tiles = (unsigned)(((M + BM - 1) / BM) * ((N + BN - 1) / BN));
    const bool vec = (K % 4 == 0) && (N % 4 == 0);
    if (vec)
        return launch((k_gemm_f32<BM, BN, BK, true>), dim3(tiles), dim3(kThreads), 0, s, A, B, C, M, N, K);
    else
        return launch((k_gemm_f32<BM, BN, BK, false>), dim3(tiles), dim3(kThreads), 0, s, A, B, C, M, N, K);
}

}  // namespace

hipError_t gemm_f32(const float *A, const float *B, float *C, int64_t M, int64_t N, int64_t K, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return fill_zero(C, (uint64_t)M * N * sizeof(float), s);
    if (M > (1 << 30) || N > (1 << 30) || K > (1 << 30)) return hipErrorInvalidValue;
    // large products: 128 x 128 tiles; smaller ones: 64 x 64 so the grid still covers the CUs
    if ((M / 128) * (N / 128) >= 512) return launch_f32<128, 128, 32>(A, B, C, (int)M, (int)N, (int)K, s);
    return launch_f32<64, 64, 32>(A, B, C, (int)M, (int)N, (int)K, s);
}

hipError_t gemm_bf16(const uint16_t *A, const uint16_t *B, float *C, int64_t M, int64_t N, int64_t K,
                     hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return fill_zero(C, (uint64_t)M * N * sizeof(float), s);
    if (M > (1 << 30) || N > (1 << 30) || K > (1 << 30)) return hipErrorInvalidValue;
    const unsigned tiles = (unsigned)(((M + 63) / 64) * ((N + 63) / 64));
    return launch((k_gemm_bf16<64, 64>), dim3(tiles), dim3(kThreads), 0, s,
                       reinterpret_cast<const unsigned short *>(A), reinterpret_cast<const unsigned short *>(B), C,
                       (int)M, (int)N, (int)K);
}

}  // namespace k
}  // namespace ofl
