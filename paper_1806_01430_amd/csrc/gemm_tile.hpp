// One BM x BN output tile of the FP32 product C = A * B on the MFMA matrix
// cores (v_mfma_f32_16x16x4_f32; gfx950 has no XF32, so the product is true
// FP32 with FP32 accumulation), shared by the single-product kernel and the
// grouped persistent kernel of instance batches.
//
// A block of 256 threads (4 waves, 2 x 2) owns the tile; each wave a
// (BM/2) x (BN/2) sub-tile as (BM/32) x (BN/32) 16x16 accumulators.  K
// advances in slabs of BK staged through LDS, double buffered: the next slab
// is fetched from global memory into registers while the current one feeds
// the MFMAs.  The function ends with a block barrier, so a caller may start
// the next tile on the same LDS at once.
//
// Within one MFMA the k index of lane l's operands is (l / 16, slot); any
// assignment of real k values to (lane group, slot) gives the same sum as
// long as A and B use the same one.  Here lane group g takes the contiguous
// run k = g*S .. g*S + S - 1 of the slab, so every lane reads its A operands
// with one wide LDS load.
#pragma once

#include <hip/hip_runtime.h>

namespace ofl {
namespace k {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kGemmThreads = 256;

// A slab of A is staged chunk-major: the 16-byte chunk c (k = 4c .. 4c+3) of
// row m at float offset c*BM*4 + 4m, loaded with rows fastest (a wave takes
// chunks 4h .. 4h+3 of 16 consecutive rows), so that an operand read (16
// consecutive rows, one chunk) and a staging write each cover 256 contiguous
// bytes per 16 lanes; rows padded to BK+4 floats left the operand reads
// two-way bank conflicted on gfx950.  B stays row-major Bs[k][n] (its reads
// walk n).
template <int BM, int BN, int BK>
struct GemmLds {
    float As[2][BM * BK];
    float Bs[2][BK * (BN + 4)];   // Bs[k][n]
};

template <int BM, int BN, int BK, bool VEC>
__device__ inline void gemm_f32_tile(const float *__restrict__ A, const float *__restrict__ B, float *__restrict__ C,
                                     int M, int N, int K, int m0, int n0, GemmLds<BM, BN, BK> &sm) {
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LDB = BN + 4;          // Bs[k][n]
    static_assert((BK == 16 || BK == 32 || BK == 64) && BM % 16 == 0, "4, 8 or 16 chunks per row, 16-row groups");
    // row and chunk of staged A piece p (0 .. BM BK/4 - 1): p = r16 + 16 (c_lo
    // + 4 (group + BM/16 c_hi)) is chunk c_lo + 4 c_hi of row 16 group + r16
    auto piece = [](int p, int &row, int &c) {
        const int rest = p / 64;
        row = (rest % (BM / 16)) * 16 + (p % 16);
        c = (p / 16) % 4 + 4 * (rest / (BM / 16));
    };
    constexpr int A_PER = BM * BK / 4 / kGemmThreads;
    constexpr int B_PER = BK * BN / 4 / kGemmThreads;
    static_assert(A_PER * 4 * kGemmThreads == BM * BK && B_PER * 4 * kGemmThreads == BK * BN, "tile / thread mismatch");
    auto &As = sm.As;
    auto &Bs = sm.Bs;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    float4 ra[A_PER], rb[B_PER];
    auto gload = [&](int k0) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            int row, c;
            piece(tid + s * kGemmThreads, row, c);
            const int gm = m0 + row, gk = k0 + 4 * c;
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
            const int idx = tid + s * kGemmThreads, row = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
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
            int row, c;
            piece(tid + s * kGemmThreads, row, c);
            *reinterpret_cast<float4 *>(&As[buf][c * BM * 4 + 4 * row]) = ra[s];
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int idx = tid + s * kGemmThreads, row = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
            *reinterpret_cast<float4 *>(&Bs[buf][row * LDB + c4]) = rb[s];
        }
    };
    const int r = lane & 15, g = lane >> 4;
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            float4 af[TM];
            const int c = ks / 4 + g;                       // this lane group's chunk
            const int off = c * BM * 4 + 4 * r;               // + 4 * (16-row group base)
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const float4 *>(&As[buf][off + 4 * (wm * WM + i * 16)]);
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

}  // namespace k
}  // namespace ofl
