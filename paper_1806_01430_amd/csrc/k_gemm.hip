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

// Split-precision / low-precision product on k-contiguous operands:
// C[i][j] = (sum_k A'[i][k] B'[j][k]) * sa[i] * sb[j]   (scales optional),
// A' is Mp x Kp, B' is Np x Kp (B stored transposed), both zero-padded to
// whole tiles, so loads need no bounds checks.  T = bf16 (MFMA 16x16x32 bf16)
// or fp8 e4m3 (MFMA 16x16x32 fp8).  A slab is 128 bytes of k per row; each
// lane takes a contiguous 32-byte run of the slab for its lane group.
typedef long fp8x8;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T, int BM, int BN, bool SCALED>
__global__ __launch_bounds__(kThreads) void k_gemm_nt(const T *__restrict__ A, const T *__restrict__ B,
                                                      float *__restrict__ C, int M, int N, int Kp,
                                                      const float *__restrict__ sa, const float *__restrict__ sb) {
    constexpr int SLAB = 128;                       // bytes of k per row per slab
    constexpr int LDS_ROW = SLAB + 16;              // padded row: conflict-free 16-byte reads
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int A_PER = BM * SLAB / 16 / kThreads;
    constexpr int B_PER = BN * SLAB / 16 / kThreads;
    static_assert(A_PER * 16 * kThreads == BM * SLAB && B_PER * 16 * kThreads == BN * SLAB, "tile mismatch");
    __shared__ __attribute__((aligned(16))) unsigned char As[2][BM * LDS_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[2][BN * LDS_ROW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int tiles_n = (N + BN - 1) / BN;
    const int tiles = tiles_n * ((M + BM - 1) / BM);
    const int t = xcd_swizzle(blockIdx.x, tiles);
    const int m0 = (t / tiles_n) * BM, n0 = (t % tiles_n) * BN;
    const size_t row_bytes = (size_t)Kp * sizeof(T);
    const unsigned char *Ab = reinterpret_cast<const unsigned char *>(A) + (size_t)m0 * row_bytes;
    const unsigned char *Bb = reinterpret_cast<const unsigned char *>(B) + (size_t)n0 * row_bytes;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    u32x4 ra[A_PER], rb[B_PER];
    auto gload = [&](int slab) {
        const size_t kb = (size_t)slab * SLAB;
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (SLAB / 16), c = (idx % (SLAB / 16)) * 16;
            ra[s] = *reinterpret_cast<const u32x4 *>(Ab + (size_t)row * row_bytes + kb + c);
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (SLAB / 16), c = (idx % (SLAB / 16)) * 16;
            rb[s] = *reinterpret_cast<const u32x4 *>(Bb + (size_t)row * row_bytes + kb + c);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (SLAB / 16), c = (idx % (SLAB / 16)) * 16;
            *reinterpret_cast<u32x4 *>(&As[buf][row * LDS_ROW + c]) = ra[s];
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            const int idx = tid + s * kThreads, row = idx / (SLAB / 16), c = (idx % (SLAB / 16)) * 16;
            *reinterpret_cast<u32x4 *>(&Bs[buf][row * LDS_ROW + c]) = rb[s];
        }
    };
    const int r = lane & 15, g = lane >> 4;
    auto compute = [&](int buf) {
        // lane group g owns bytes [32g, 32g+32) of the slab: two 16-byte reads
        u32x4 af[TM][2], bfr[TN][2];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                af[i][h] = *reinterpret_cast<const u32x4 *>(&As[buf][(wm * WM + i * 16 + r) * LDS_ROW + 32 * g + 16 * h]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int h = 0; h < 2; ++h)
                bfr[j][h] = *reinterpret_cast<const u32x4 *>(&Bs[buf][(wn * WN + j * 16 + r) * LDS_ROW + 32 * g + 16 * h]);
        if constexpr (sizeof(T) == 2) {
            // 16 bf16 per lane = two MFMA steps of 8
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i][h]),
                                                                            __builtin_bit_cast(bf16x8, bfr[j][h]),
                                                                            acc[i][j], 0, 0, 0);
        } else {
            // 32 fp8 per lane = four MFMA steps of 8
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                            const fp8x8 a8 = (fp8x8)(((unsigned long)af[i][h][2 * q + 1] << 32) | af[i][h][2 * q]);
                            const fp8x8 b8 = (fp8x8)(((unsigned long)bfr[j][h][2 * q + 1] << 32) | bfr[j][h][2 * q]);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a8, b8, acc[i][j], 0, 0, 0);
                        }
        }
    };

    const int nslab = (int)(row_bytes / SLAB);
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nslab; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nslab) gload(kt + 1);
        compute(cur);
        if (kt + 1 < nslab) sstore(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * WM + i * 16 + 4 * g + e, col = n0 + wn * WN + j * 16 + r;
                if (row < M && col < N) {
                    float v = acc[i][j][e];
                    if (SCALED) v = v * (sa[row] * sb[col]);
                    C[(size_t)row * N + col] = v;
                }
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

// ---------------------------------------------------------------- split-precision GEMM
namespace {
constexpr int kNT = 128;   // tile of the k-contiguous product (rows of A', rows of B')

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Workspace layout of one product: [A' | B' | float area], A' omitted when
// bf16 inputs are already tile-aligned.  float area (fp8 only): row scales,
// column scales, their inverses, and per-slice column maxima.
struct NtLayout {
    int64_t Mp = 0, Np = 0, Kp = 0, kx = 0;
    int elem = 2;
    bool a_copy = true;    // A' is written (else A is used in place)
    bool b_pad = true;     // B' has a padded region that must read as zero
    int64_t a_bytes = 0, b_bytes = 0, f_off = 0, total = 0;
};

NtLayout nt_layout(int64_t M, int64_t N, int64_t K, int variant) {
    NtLayout L;
    L.elem = variant == 2 ? 1 : 2;
    L.kx = variant == 3 ? K : 3 * K;
    L.Mp = round_up(M, kNT);
    L.Np = round_up(N, kNT);
    L.Kp = round_up(L.kx, 128 / L.elem);
    L.a_copy = variant != 3 || L.Mp != M || L.Kp != K;
    L.b_pad = L.Np != N || L.Kp != L.kx;
    L.a_bytes = L.a_copy ? L.Mp * L.Kp * L.elem : 0;
    L.b_bytes = L.Np * L.Kp * L.elem;
    L.f_off = round_up(L.a_bytes + L.b_bytes, 256);
    const int64_t nf = variant == 2 ? 2 * (L.Mp + L.Np) + (int64_t)kColSlices * L.Np : 0;
    L.total = round_up(L.f_off + nf * (int64_t)sizeof(float), 256);
    return L;
}

bool nt_sizes_ok(int64_t M, int64_t N, int64_t K) {
    return M <= (1 << 28) && N <= (1 << 22) && K <= (1 << 26);
}
}  // namespace

int64_t gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int variant) {
    if (M <= 0 || N <= 0 || K <= 0 || variant < 1 || variant > 3) return 0;
    return nt_layout(M, N, K, variant).total;
}

int gemm_launches(int64_t M, int64_t N, int64_t K, int variant) {
    if (M <= 0 || N <= 0) return 0;
    if (K <= 0) return 1;
    if (variant == 0) return 1;
    const NtLayout L = nt_layout(M, N, K, variant);
    int n = (L.b_pad ? 1 : 0) + 2 + (L.a_copy ? 1 : 0);   // [zero B'], B', product, [A']
    if (variant == 2) n += 3;                               // row scales, column maxima, column scales
    return n;
}

hipError_t gemm_split(const float *A, const float *B, float *C, int64_t M, int64_t N, int64_t K, int variant,
                      void *ws, int64_t ws_bytes, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return fill_zero(C, (uint64_t)M * N * sizeof(float), s);
    if ((variant != 1 && variant != 2) || !nt_sizes_ok(M, N, 3 * K)) return hipErrorInvalidValue;
    const NtLayout L = nt_layout(M, N, K, variant);
    if (L.total > ws_bytes || !ws) return hipErrorInvalidValue;
    unsigned char *w = static_cast<unsigned char *>(ws);
    void *Ap = w, *Bp = w + L.a_bytes;
    float *f = reinterpret_cast<float *>(w + L.f_off);
    float *sa = f, *sb = f + L.Mp, *isa = sb + L.Np, *isb = isa + L.Mp, *colmax = isb + L.Np;
    const unsigned tiles = (unsigned)((L.Mp / kNT) * (L.Np / kNT));
    hipError_t e = L.b_pad ? fill_zero(Bp, (uint64_t)L.b_bytes, s) : hipSuccess;
    if (variant == 1) {
        if (e == hipSuccess) e = prep_a(A, Ap, nullptr, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 0, s);
        if (e == hipSuccess) e = split_bt(B, Bp, nullptr, (int)K, (int)N, (int)L.Kp, 0, s);
        if (e == hipSuccess)
            e = launch((k_gemm_nt<unsigned short, kNT, kNT, false>), dim3(tiles), dim3(kThreads), 0, s,
                       static_cast<const unsigned short *>(Ap), static_cast<const unsigned short *>(Bp), C, (int)M,
                       (int)N, (int)L.Kp, (const float *)nullptr, (const float *)nullptr);
        return e;
    }
    if (e == hipSuccess) e = row_scales(A, sa, isa, (int)M, (int)K, s);
    if (e == hipSuccess) e = col_scales(B, sb, isb, colmax, (int)K, (int)N, (int)L.Np, s);
    if (e == hipSuccess) e = prep_a(A, Ap, sa, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 1, s);
    if (e == hipSuccess) e = split_bt(B, Bp, sb, (int)K, (int)N, (int)L.Kp, 1, s);
    if (e == hipSuccess)
        e = launch((k_gemm_nt<unsigned char, kNT, kNT, true>), dim3(tiles), dim3(kThreads), 0, s,
                   static_cast<const unsigned char *>(Ap), static_cast<const unsigned char *>(Bp), C, (int)M, (int)N,
                   (int)L.Kp, (const float *)isa, (const float *)isb);
    return e;
}

hipError_t gemm_bf16(const uint16_t *A, const uint16_t *B, float *C, int64_t M, int64_t N, int64_t K, void *ws,
                     int64_t ws_bytes, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0) return fill_zero(C, (uint64_t)M * N * sizeof(float), s);
    if (!nt_sizes_ok(M, N, K)) return hipErrorInvalidValue;
    const NtLayout L = nt_layout(M, N, K, 3);
    if (L.total > ws_bytes || !ws) return hipErrorInvalidValue;
    unsigned char *w = static_cast<unsigned char *>(ws);
    void *Bp = w + L.a_bytes;
    const void *Ause = A;
    const unsigned tiles = (unsigned)((L.Mp / kNT) * (L.Np / kNT));
    hipError_t e = L.b_pad ? fill_zero(Bp, (uint64_t)L.b_bytes, s) : hipSuccess;
    if (L.a_copy) {
        if (e == hipSuccess) e = prep_a(A, w, nullptr, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 2, s);
        Ause = w;
    }
    if (e == hipSuccess) e = split_bt(B, Bp, nullptr, (int)K, (int)N, (int)L.Kp, 2, s);
    if (e == hipSuccess)
        e = launch((k_gemm_nt<unsigned short, kNT, kNT, false>), dim3(tiles), dim3(kThreads), 0, s,
                   static_cast<const unsigned short *>(Ause), static_cast<const unsigned short *>(Bp), C, (int)M,
                   (int)N, (int)L.Kp, (const float *)nullptr, (const float *)nullptr);
    return e;
}

}  // namespace k
}  // namespace ofl
