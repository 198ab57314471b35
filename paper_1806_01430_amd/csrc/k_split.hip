// Operand preparation for the split-precision GEMM variants.
//
// A product in lower precision with one refinement pass: with A = Ah + Al and
// B = Bh + Bl (hi = rounded value, lo = rounded remainder),
//   A B  ~  Ah Bh + Ah Bl + Al Bh,
// which is a single GEMM over K' = 3K of A' = [Ah | Ah | Al] (rows of A) with
// B' = [Bh ; Bl ; Bh].  Both operands are written k-contiguous (B' stored
// transposed, one row per column of B) and zero-padded to whole tiles, so the
// GEMM kernel needs no bounds checks on its loads.
//
// FP8 (e4m3): each row of A and each column of B gets a power-of-two scale s
// with amax * s <= 224 (inside the range of either e4m3 variant); the scale
// factors out of every dot product and is undone in the GEMM epilogue.
#include <hip/hip_runtime.h>

#include "dev_common.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kThreads = 256;

__device__ inline unsigned short bf16_rne_bits(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// hi / lo parts of x in the operand type
struct Bf16Parts {
    unsigned short hi, lo;
};
__device__ inline Bf16Parts split_bf16(float x) {
    const unsigned short h = bf16_rne_bits(x);
    return {h, bf16_rne_bits(x - bf16_value(h))};
}
struct Fp8Parts {
    unsigned char hi, lo;
};
__device__ inline unsigned char fp8_bits(float x) {
    return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
}
__device__ inline float fp8_value(unsigned char b) { return __builtin_amdgcn_cvt_f32_fp8((int)b, 0); }
__device__ inline Fp8Parts split_fp8(float xs) {
    const unsigned char h = fp8_bits(xs);
    return {h, fp8_bits(xs - fp8_value(h))};
}

// Largest power of two s with amax * s <= 224 (1 when amax is 0 or not
// finite).  With amax = m 2^E, m in [0.5, 1), and 224 = 0.875 * 2^8:
// s = 2^(8 - E) when m <= 0.875, else 2^(7 - E); exact, no division.
__device__ inline float pow2_scale(float amax) {
    if (!(amax > 0.0f) || !(amax <= 3.4028235e38f)) return 1.0f;
    int E;
    const float m = frexpf(amax, &E);
    int e = (m <= 0.875f ? 8 : 7) - E;
    e = e < -126 ? -126 : (e > 126 ? 126 : e);
    return ldexpf(1.0f, e);
}

// A' rows.  Each thread reads kPrepV elements of A (lanes on consecutive k,
// so every load and store instruction is coalesced) and writes each one's
// parts to all segments of the row: MODE 0 bf16 split [hi | hi | lo],
// MODE 1 e4m3 split of A * sa[i], MODE 2 plain bf16 copy.  The same threads
// zero the row's padding k' >= kx; rows i >= M are written as zero.
constexpr int kPrepV = 4;
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_prep_a(const void *__restrict__ Av, void *__restrict__ Apv,
                                                     const float *__restrict__ sa, int M, int K, int Kp, int kx) {
    constexpr int nseg = MODE == 2 ? 1 : 3;
    const int i = blockIdx.x;
    const int pad = Kp - kx;                  // zero tail of the row
    const float scale = (MODE == 1 && i < M) ? sa[i] : 1.0f;
#pragma unroll
    for (int e = 0; e < kPrepV; ++e) {
        const int kk = (blockIdx.y * kPrepV + e) * kThreads + threadIdx.x;
        if (kk < K) {
            unsigned hi = 0, lo = 0;
            if (i < M) {
                if (MODE == 2) {
                    hi = static_cast<const unsigned short *>(Av)[(size_t)i * K + kk];
                } else {
                    const float a = static_cast<const float *>(Av)[(size_t)i * K + kk];
                    if (MODE == 0) {
                        const Bf16Parts p = split_bf16(a);
                        hi = p.hi;
                        lo = p.lo;
                    } else {
                        const Fp8Parts p = split_fp8(a * scale);
                        hi = p.hi;
                        lo = p.lo;
                    }
                }
            }
            if (MODE == 1) {
                unsigned char *row = static_cast<unsigned char *>(Apv) + (size_t)i * Kp;
                row[kk] = (unsigned char)hi;
                row[K + kk] = (unsigned char)hi;
                row[2 * K + kk] = (unsigned char)lo;
            } else {
                unsigned short *row = static_cast<unsigned short *>(Apv) + (size_t)i * Kp;
                row[kk] = (unsigned short)hi;
                if (nseg == 3) {
                    row[K + kk] = (unsigned short)hi;
                    row[2 * K + kk] = (unsigned short)lo;
                }
            }
        }
        if (kk < pad) {
            if (MODE == 1) static_cast<unsigned char *>(Apv)[(size_t)i * Kp + kx + kk] = 0;
            else static_cast<unsigned short *>(Apv)[(size_t)i * Kp + kx + kk] = 0;
        }
    }
}

// The same rows with 4 consecutive k per lane (16-byte loads, 8-byte bf16
// or 4-byte e4m3 stores per segment) when K is a multiple of 4: same parts,
// same bits.
template <int MODE>   // 0: bf16 hi/lo split, 1: e4m3 split of A * sa[i]
__global__ __launch_bounds__(kThreads) void k_prep_a4(const float *__restrict__ A, void *__restrict__ Apv,
                                                      const float *__restrict__ sa, int M, int K, int Kp, int kx) {
    const int i = blockIdx.x;
    const int kk = (blockIdx.y * kThreads + (int)threadIdx.x) * 4;
    const float scale = (MODE == 1 && i < M) ? sa[i] : 1.0f;
    if (kk < K) {
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < M) a = *reinterpret_cast<const float4 *>(A + (size_t)i * K + kk);
        const float v[4] = {a.x, a.y, a.z, a.w};
        if (MODE == 0) {
            unsigned hi[2] = {0, 0}, lo[2] = {0, 0};
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const Bf16Parts q = split_bf16(v[t]);
                hi[t >> 1] |= (unsigned)q.hi << (16 * (t & 1));
                lo[t >> 1] |= (unsigned)q.lo << (16 * (t & 1));
            }
            unsigned short *row = static_cast<unsigned short *>(Apv) + (size_t)i * Kp;
            *reinterpret_cast<uint2 *>(row + kk) = make_uint2(hi[0], hi[1]);
            *reinterpret_cast<uint2 *>(row + K + kk) = make_uint2(hi[0], hi[1]);
            *reinterpret_cast<uint2 *>(row + 2 * K + kk) = make_uint2(lo[0], lo[1]);
        } else {
            unsigned hi = 0, lo = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const Fp8Parts q = split_fp8(v[t] * scale);
                hi |= (unsigned)q.hi << (8 * t);
                lo |= (unsigned)q.lo << (8 * t);
            }
            unsigned char *row = static_cast<unsigned char *>(Apv) + (size_t)i * Kp;
            *reinterpret_cast<unsigned *>(row + kk) = hi;
            *reinterpret_cast<unsigned *>(row + K + kk) = hi;
            *reinterpret_cast<unsigned *>(row + 2 * K + kk) = lo;
        }
    }
    if (kk < Kp - kx) {   // the row's zero tail, 4 elements at a time
        if (MODE == 0)
            *reinterpret_cast<uint2 *>(static_cast<unsigned short *>(Apv) + (size_t)i * Kp + kx + kk) = make_uint2(0, 0);
        else
            *reinterpret_cast<unsigned *>(static_cast<unsigned char *>(Apv) + (size_t)i * Kp + kx + kk) = 0u;
    }
}

// B'^T: row j (< N) of the output holds column j of B: [hi | lo | hi | 0 ...]
// (or the plain bf16 column for the bf16-input product).  64 x 64 tiles of B
// through LDS, so both the read of B and the write of B'^T are coalesced.
constexpr int kT = 64;
template <int MODE>   // 0: bf16 hi/lo split of f32, 1: fp8 split of f32 * sb, 2: plain bf16 copy
__global__ __launch_bounds__(kThreads) void k_split_bt(const void *__restrict__ Bv, void *__restrict__ Btv,
                                                       const float *__restrict__ sb, int K, int N, int Kp) {
    __shared__ float tile[kT][kT + 1];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int k0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    for (int r = ty; r < kT; r += kThreads / kT) {
        const int kk = k0 + r, j = j0 + tx;
        float v = 0.0f;
        if (kk < K && j < N) {
            if (MODE == 2) v = bf16_value(static_cast<const unsigned short *>(Bv)[(size_t)kk * N + j]);
            else v = static_cast<const float *>(Bv)[(size_t)kk * N + j];
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < kT; r += kThreads / kT) {
        const int j = j0 + r, kk = k0 + tx;
        if (j >= N || kk >= K) continue;
        const float x = tile[tx][r];
        if (MODE == 0) {
            unsigned short *Bt = static_cast<unsigned short *>(Btv) + (size_t)j * Kp;
            const Bf16Parts s = split_bf16(x);
            Bt[kk] = s.hi;
            Bt[K + kk] = s.lo;
            Bt[2 * K + kk] = s.hi;
        } else if (MODE == 1) {
            unsigned char *Bt = static_cast<unsigned char *>(Btv) + (size_t)j * Kp;
            const Fp8Parts s = split_fp8(x * sb[j]);
            Bt[kk] = s.hi;
            Bt[K + kk] = s.lo;
            Bt[2 * K + kk] = s.hi;
        } else {
            unsigned short *Bt = static_cast<unsigned short *>(Btv) + (size_t)j * Kp;
            Bt[kk] = bf16_rne_bits(x);
        }
    }
}

// The split of B (MODE 0 / 1) when K and N are whole 64-element tiles:
// 16-byte loads of 4 columns, and per output row 8 k values at a time
// (16-byte bf16 / 8-byte e4m3 stores per segment); same parts, same bits.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_split_bt8(const float *__restrict__ B, void *__restrict__ Btv,
                                                        const float *__restrict__ sb, int K, int N, int Kp) {
    constexpr int P = kT + 4;   // row pitch in floats (16-byte aligned rows)
    __shared__ __attribute__((aligned(16))) float tile[kT][P];
    const int k0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = tid + u * kThreads, r = c >> 4, q = c & 15;   // k-row r, columns 4q .. 4q + 3
        *reinterpret_cast<float4 *>(&tile[r][4 * q]) =
            *reinterpret_cast<const float4 *>(B + (size_t)(k0 + r) * N + j0 + 4 * q);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = tid + u * kThreads, j = c >> 3, q = c & 7;   // output row j, k values 8q .. 8q + 7
        const float scale = MODE == 1 ? sb[j0 + j] : 1.0f;
        if (MODE == 0) {
            unsigned hi[4] = {0, 0, 0, 0}, lo[4] = {0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const Bf16Parts p = split_bf16(tile[8 * q + t][j]);
                hi[t >> 1] |= (unsigned)p.hi << (16 * (t & 1));
                lo[t >> 1] |= (unsigned)p.lo << (16 * (t & 1));
            }
            unsigned short *row = static_cast<unsigned short *>(Btv) + (size_t)(j0 + j) * Kp + k0 + 8 * q;
            *reinterpret_cast<uint4 *>(row) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
            *reinterpret_cast<uint4 *>(row + K) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
            *reinterpret_cast<uint4 *>(row + 2 * K) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        } else {
            unsigned hi[2] = {0, 0}, lo[2] = {0, 0};
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const Fp8Parts p = split_fp8(tile[8 * q + t][j] * scale);
                hi[t >> 2] |= (unsigned)p.hi << (8 * (t & 3));
                lo[t >> 2] |= (unsigned)p.lo << (8 * (t & 3));
            }
            unsigned char *row = static_cast<unsigned char *>(Btv) + (size_t)(j0 + j) * Kp + k0 + 8 * q;
            *reinterpret_cast<uint2 *>(row) = make_uint2(hi[0], hi[1]);
            *reinterpret_cast<uint2 *>(row + K) = make_uint2(lo[0], lo[1]);
            *reinterpret_cast<uint2 *>(row + 2 * K) = make_uint2(hi[0], hi[1]);
        }
    }
}

// The plain bf16 transpose of B (MODE 2) when K and N are whole 64-element
// tiles: 16-byte loads of 8 columns and 16-byte stores of 8 k values (the
// form above moves 2 bytes per lane); other shapes take the form above.
__global__ __launch_bounds__(kThreads) void k_transpose_bf16(const unsigned short *__restrict__ B,
                                                             unsigned short *__restrict__ Bt, int K, int N, int Kp) {
    constexpr int P = kT + 8;   // row pitch in elements (16-byte aligned rows)
    __shared__ __attribute__((aligned(16))) unsigned short tile[kT][P];
    const int k0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = tid + u * kThreads, r = c >> 3, q = c & 7;   // k-row r, columns 8q .. 8q + 7
        *reinterpret_cast<uint4 *>(&tile[r][8 * q]) =
            *reinterpret_cast<const uint4 *>(B + (size_t)(k0 + r) * N + j0 + 8 * q);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int c = tid + u * kThreads, j = c >> 3, q = c & 7;   // output row j, k values 8q .. 8q + 7
        unsigned w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            w[t] = (unsigned)tile[8 * q + 2 * t][j] | ((unsigned)tile[8 * q + 2 * t + 1][j] << 16);
        *reinterpret_cast<uint4 *>(Bt + (size_t)(j0 + j) * Kp + k0 + 8 * q) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Row scales of A: one wave per row, max |A[i][k]| -> s_i; inv_s_i.
__global__ __launch_bounds__(kThreads) void k_row_scale(const float *__restrict__ A, float *__restrict__ s,
                                                        float *__restrict__ inv, int M, int K, bool vec) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
    if (row >= M) return;
    // the maximum does not depend on the order it is taken in: 16-byte loads
    // when every row starts 16-byte aligned (vec)
    float m = 0.0f;
    const float *a = A + (size_t)row * K;
    if (vec) {
        for (int k = 4 * lane; k < K; k += 4 * kWave) {
            const float4 v = *reinterpret_cast<const float4 *>(a + k);
            m = fmaxf(fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y))), fmaxf(fabsf(v.z), fabsf(v.w)));
        }
    } else {
        for (int k = lane; k < K; k += kWave) m = fmaxf(m, fabsf(a[k]));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (lane == 0) {
        const float sc = pow2_scale(m);
        s[row] = sc;
        inv[row] = 1.0f / sc;
    }
}

// Column maxima of |B| in two deterministic stages: block (x, y) takes 64
// columns and slice y of the k range, combining its 4 row lanes in LDS;
// then one thread per column reduces the kColSlices partial maxima.
__global__ __launch_bounds__(kThreads) void k_col_max(const float *__restrict__ B, float *__restrict__ part, int K,
                                                      int N, int ld_part) {
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + tx;
    const int rows = (K + kColSlices - 1) / kColSlices;
    const int k0 = blockIdx.y * rows, k1 = min(K, k0 + rows);
    float m = 0.0f;
    if (j < N)
        for (int k = k0 + ty; k < k1; k += 4) m = fmaxf(m, fabsf(B[(size_t)k * N + j]));
    red[ty][tx] = m;
    __syncthreads();
    if (ty == 0 && j < N)
        part[(size_t)blockIdx.y * ld_part + j] = fmaxf(fmaxf(red[0][tx], red[1][tx]), fmaxf(red[2][tx], red[3][tx]));
}

__global__ __launch_bounds__(kThreads) void k_col_scale(const float *__restrict__ part, float *__restrict__ s,
                                                        float *__restrict__ inv, int N, int ld_part) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= N) return;
    float m = 0.0f;
    for (int y = 0; y < kColSlices; ++y) m = fmaxf(m, part[(size_t)y * ld_part + j]);
    const float sc = pow2_scale(m);
    s[j] = sc;
    inv[j] = 1.0f / sc;
}

}  // namespace

hipError_t prep_a(const void *A, void *Ap, const float *sa, int M, int K, int Mp, int Kp, int mode, hipStream_t s) {
    const int kx = mode == 2 ? K : 3 * K;
    const int span = K > Kp - kx ? K : Kp - kx;   // k range the threads of one row cover
    const dim3 grid((unsigned)Mp, (unsigned)((span + kThreads * kPrepV - 1) / (kThreads * kPrepV)));
    if (grid.y > 65535 || K <= 0) return hipErrorInvalidValue;
    if (mode != 2 && K % 4 == 0) {
        const dim3 g4((unsigned)Mp, (unsigned)((span + kThreads * 4 - 1) / (kThreads * 4)));
        if (mode == 0)
            return launch((k_prep_a4<0>), g4, dim3(kThreads), 0, s, static_cast<const float *>(A), Ap, sa, M, K, Kp,
                          kx);
        return launch((k_prep_a4<1>), g4, dim3(kThreads), 0, s, static_cast<const float *>(A), Ap, sa, M, K, Kp, kx);
    }
    if (mode == 0) return launch((k_prep_a<0>), grid, dim3(kThreads), 0, s, A, Ap, sa, M, K, Kp, kx);
    if (mode == 1) return launch((k_prep_a<1>), grid, dim3(kThreads), 0, s, A, Ap, sa, M, K, Kp, kx);
    return launch((k_prep_a<2>), grid, dim3(kThreads), 0, s, A, Ap, sa, M, K, Kp, kx);
}

hipError_t split_bt(const void *B, void *Bt, const float *sb, int K, int N, int Kp, int mode, hipStream_t s) {
    dim3 grid((unsigned)((K + kT - 1) / kT), (unsigned)((N + kT - 1) / kT));
    if (grid.y > 65535) return hipErrorInvalidValue;
    if (mode != 2 && K % kT == 0 && N % kT == 0) {
        const float *Bf = static_cast<const float *>(B);
        if (mode == 0) return launch((k_split_bt8<0>), grid, dim3(kThreads), 0, s, Bf, Bt, sb, K, N, Kp);
        return launch((k_split_bt8<1>), grid, dim3(kThreads), 0, s, Bf, Bt, sb, K, N, Kp);
    }
    if (mode == 0) return launch((k_split_bt<0>), grid, dim3(kThreads), 0, s, B, Bt, sb, K, N, Kp);
    if (mode == 1) return launch((k_split_bt<1>), grid, dim3(kThreads), 0, s, B, Bt, sb, K, N, Kp);
    if (K % kT == 0 && N % kT == 0 && Kp % 8 == 0)
        return launch(k_transpose_bf16, grid, dim3(kThreads), 0, s, static_cast<const unsigned short *>(B),
                      static_cast<unsigned short *>(Bt), K, N, Kp);
    return launch((k_split_bt<2>), grid, dim3(kThreads), 0, s, B, Bt, sb, K, N, Kp);
}

hipError_t row_scales(const float *A, float *s_out, float *inv_out, int M, int K, hipStream_t s) {
    const unsigned blocks = (unsigned)((M + (kThreads / kWave) - 1) / (kThreads / kWave));
    const bool vec = K % 4 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0;
    return launch(k_row_scale, dim3(blocks), dim3(kThreads), 0, s, A, s_out, inv_out, M, K, vec);
}

hipError_t col_scales(const float *B, float *s_out, float *inv_out, float *part, int K, int N, int ld_part,
                      hipStream_t s) {
    hipError_t e = launch(k_col_max, dim3((unsigned)((N + 63) / 64), (unsigned)kColSlices), dim3(kThreads), 0, s, B,
                          part, K, N, ld_part);
    if (e != hipSuccess) return e;
    return launch(k_col_scale, dim3((unsigned)((N + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                  (const float *)part, s_out, inv_out, N, ld_part);
}

}  // namespace k
}  // namespace ofl
