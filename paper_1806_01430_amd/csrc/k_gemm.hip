// Dense matrix products C = A * B (row-major) on the MFMA matrix cores.
//
// FP32: one BM x BN tile per block (gemm_tile.hpp).  bf16 inputs and the
// split-precision forms: one product over k-contiguous, tile-padded operands
// (k_gemm_nt) after preparation passes (k_split.hip).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "gemm_tile.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// receives a contiguous run of output tiles.
__device__ inline int xcd_swizzle(int bid, int nblocks) {
    const int nx = 8;
    if (nblocks % nx) return bid;
    return (bid % nx) * (nblocks / nx) + bid / nx;
}

// Output tile (tm, tn) of block bid: the XCD's contiguous run of tiles is
// walked in groups of kGroupRows tile rows, column by column inside a group,
// so that the blocks an XCD runs at one time form a square of tiles (8 x 8
// with 64 resident blocks) and share 8 A panels and 8 B panels in its L2;
// walking whole tile rows instead streams all of B once per tile row
// (8192 x 8192 bf16: 8.9 GB read per product against 2 GB grouped).
constexpr int kGroupRows = 8;
__device__ inline void tile_of(int bid, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int t = xcd_swizzle(bid, tiles_m * tiles_n);
    const int per_group = kGroupRows * tiles_n;
    const int g = t / per_group, idx = t - g * per_group;
    const int rows = min(kGroupRows, tiles_m - g * kGroupRows);
    tm = g * kGroupRows + idx % rows;
    tn = idx / rows;
}

template <int BM, int BN, int BK, bool VEC>
__global__ __launch_bounds__(kThreads) void k_gemm_f32(const float *__restrict__ A, const float *__restrict__ B,
                                                       float *__restrict__ C, int M, int N, int K) {
    __shared__ GemmLds<BM, BN, BK> sm;
    int tm, tn;
    tile_of(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, tm, tn);
    gemm_f32_tile<BM, BN, BK, VEC>(A, B, C, M, N, K, tm * BM, tn * BN, sm);
}

// Split-precision / low-precision product on k-contiguous operands:
// C[i][j] = (sum_k A'[i][k] B'[j][k]) * sa[i] * sb[j]   (scales optional),
// A' is Mp x Kp, B' is Np x Kp (B stored transposed), both zero-padded to
// whole tiles, so loads need no bounds checks.  T = bf16 (MFMA 16x16x32 bf16)
// or fp8 e4m3 (MFMA 16x16x32 fp8).  A slab is 128 bytes of k per row; each
// lane takes a contiguous 32-byte run of the slab for its lane group.
typedef long fp8x8;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
// Block shape BM x BN, WGM x WGN waves (each a (BM/WGM) x (BN/WGN) tile of
// 16 x 16 MFMA tiles), MINB blocks per CU, NSET register sets of staged
// slabs: with two, the slab two ahead is in flight from global memory while
// the current one is computed (two compute periods to arrive); with one, the
// next slab's loads go out before the current slab is computed (one period),
// and the fragments of each half-slab are read just before its MFMAs -- the
// register budget of the 256 x 256 block (128 accumulators per wave at two
// waves per SIMD).
//
// LDS layout of a staged slab (LAY), both staged row by row (8 lanes per
// 128-byte row, the coalesced order of the global loads): 0 = row-major rows
// padded to 144 bytes; 1 = chunk-major: the 16-byte chunk c of row R at
// c * rows * 16 + 16 (R ^ 2c) (the XOR keeps a row's eight chunks in
// distinct slots of one 256-byte span).  Measured on gfx950: layout 1 is
// 4-5% faster (BF16x3 at 4096); both leave half of the LDS cycles bank
// conflicted.  A chunk-major layout without the XOR, staged with rows
// fastest, had no conflicts at all but ran 16% slower: the loads of a wave
// then touch 16 rows at 64 bytes each instead of 8 rows at 128 bytes, and
// the global side, not LDS, is what limits these kernels.
template <typename T, int BM, int BN, int WGM, int WGN, int MINB, int NSET, int LAY, bool SCALED>
__global__ __launch_bounds__(WGM * WGN * 64, MINB) void k_gemm_nt(const T *__restrict__ A, const T *__restrict__ B,
                                                               float *__restrict__ C, int M, int N, int Kp,
                                                               const float *__restrict__ sa,
                                                               const float *__restrict__ sb) {
    constexpr int NT = WGM * WGN * 64;              // threads
    constexpr int SLAB = 128;                       // bytes of k per row per slab
    constexpr int LDS_ROW = LAY == 0 ? SLAB + 16 : SLAB;   // padded row (layout 0)
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int A_PER = BM * SLAB / 16 / NT;
    constexpr int B_PER = BN * SLAB / 16 / NT;
    static_assert(A_PER * 16 * NT == BM * SLAB && B_PER * 16 * NT == BN * SLAB, "tile mismatch");
    static_assert(NSET == 1 || NSET == 2, "one or two staging sets");
    static_assert(BM % 16 == 0 && BN % 16 == 0, "whole 16-row groups");
    __shared__ __attribute__((aligned(16))) unsigned char As[2][BM * LDS_ROW];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[2][BN * LDS_ROW];
    // byte offset of chunk c (16 bytes) of row R in a staged slab of ROWS rows
    auto at = [](int ROWS, int R, int c) {
        return LAY == 0 ? R * LDS_ROW + 16 * c : c * ROWS * 16 + 16 * (R ^ (2 * c));
    };
    // the row and chunk of staged piece p (0 .. 8 ROWS - 1): row by row
    auto piece = [](int, int p, int &row, int &c) {
        row = p / (SLAB / 16);
        c = p % (SLAB / 16);
    };

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    int tm, tn;
    tile_of(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const size_t row_bytes = (size_t)Kp * sizeof(T);
    const unsigned char *Ab = reinterpret_cast<const unsigned char *>(A) + (size_t)m0 * row_bytes;
    const unsigned char *Bb = reinterpret_cast<const unsigned char *>(B) + (size_t)n0 * row_bytes;

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    u32x4 ra[NSET][A_PER], rb[NSET][B_PER];
    auto gload = [&](int slab, int set) {
        const size_t kb = (size_t)slab * SLAB;
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            int row, c;
            piece(BM, tid + s * NT, row, c);
            ra[set][s] = *reinterpret_cast<const u32x4 *>(Ab + (size_t)row * row_bytes + kb + 16 * c);
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            int row, c;
            piece(BN, tid + s * NT, row, c);
            rb[set][s] = *reinterpret_cast<const u32x4 *>(Bb + (size_t)row * row_bytes + kb + 16 * c);
        }
    };
    auto sstore = [&](int buf, int set) {
#pragma unroll
        for (int s = 0; s < A_PER; ++s) {
            int row, c;
            piece(BM, tid + s * NT, row, c);
            *reinterpret_cast<u32x4 *>(&As[buf][at(BM, row, c)]) = ra[set][s];
        }
#pragma unroll
        for (int s = 0; s < B_PER; ++s) {
            int row, c;
            piece(BN, tid + s * NT, row, c);
            *reinterpret_cast<u32x4 *>(&Bs[buf][at(BN, row, c)]) = rb[set][s];
        }
    };
    const int r = lane & 15, g = lane >> 4;
    // lane group g owns bytes [32g, 32g+32) of the slab: two 16-byte halves
    // h, each feeding one k-step of every accumulator
    auto mfma_half = [&](const u32x4 (&af)[TM], const u32x4 (&bfr)[TN]) {
        if constexpr (sizeof(T) == 2) {
            // 8 bf16 per lane and MFMA
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                                        __builtin_bit_cast(bf16x8, bfr[j]), acc[i][j],
                                                                        0, 0, 0);
        } else {
            // 16 fp8 per lane and half: two MFMA steps of 8
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        const fp8x8 a8 = (fp8x8)(((unsigned long)af[i][2 * q + 1] << 32) | af[i][2 * q]);
                        const fp8x8 b8 = (fp8x8)(((unsigned long)bfr[j][2 * q + 1] << 32) | bfr[j][2 * q]);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a8, b8, acc[i][j], 0, 0, 0);
                    }
        }
    };
    // a lane's byte offset of chunk c in the 16-row group that starts at row
    // R0 (a multiple of 16): the group's base plus a per-lane part, so the
    // group bases fold into instruction offsets
    auto lane_off = [&](int ROWS, int c) { return at(ROWS, r, c); };
    auto read_half = [&](int buf, int h, u32x4 (&af)[TM], u32x4 (&bfr)[TN]) {
        const int oa = lane_off(BM, 2 * g + h), ob = lane_off(BN, 2 * g + h);
#pragma unroll
        for (int i = 0; i < TM; ++i)
            af[i] = *reinterpret_cast<const u32x4 *>(&As[buf][oa + (wm * WM + i * 16) * (LAY == 0 ? LDS_ROW : 16)]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
            bfr[j] = *reinterpret_cast<const u32x4 *>(&Bs[buf][ob + (wn * WN + j * 16) * (LAY == 0 ? LDS_ROW : 16)]);
    };
    auto compute = [&](int buf) {
        if constexpr (NSET == 2) {
            // all reads of the slab issued before the first MFMA
            u32x4 af[2][TM], bfr[2][TN];
            read_half(buf, 0, af[0], bfr[0]);
            read_half(buf, 1, af[1], bfr[1]);
            mfma_half(af[0], bfr[0]);
            mfma_half(af[1], bfr[1]);
        } else if constexpr (sizeof(T) == 2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                u32x4 af[TM], bfr[TN];
                read_half(buf, h, af, bfr);
                mfma_half(af, bfr);
            }
        } else {
            // fp8: four k-steps of 8 bytes per lane, each read just before
            // its MFMAs (8-byte fragments keep the register count in budget)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                fp8x8 af[TM], bfr[TN];
                const int oa = lane_off(BM, 2 * g + (q >> 1)) + 8 * (q & 1);
                const int ob = lane_off(BN, 2 * g + (q >> 1)) + 8 * (q & 1);
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    af[i] = *reinterpret_cast<const fp8x8 *>(
                        &As[buf][oa + (wm * WM + i * 16) * (LAY == 0 ? LDS_ROW : 16)]);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    bfr[j] = *reinterpret_cast<const fp8x8 *>(
                        &Bs[buf][ob + (wn * WN + j * 16) * (LAY == 0 ? LDS_ROW : 16)]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(af[i], bfr[j], acc[i][j], 0, 0, 0);
            }
        }
    };

    const int nslab = (int)(row_bytes / SLAB);
    if constexpr (NSET == 2) {
        // slab kt lives in LDS buffer kt & 1 and, before that, in register
        // set kt & 1; iteration kt loads slab kt + 2 into the set slab kt
        // left, computes slab kt and writes slab kt + 1 to the other buffer
        gload(0, 0);
        sstore(0, 0);
        if (nslab > 1) gload(1, 1);
        __syncthreads();
        auto iteration = [&](int kt, auto SET) {
            constexpr int set = decltype(SET)::value;      // = kt & 1
            if (kt + 2 < nslab) gload(kt + 2, set);
            compute(set);
            if (kt + 1 < nslab) sstore(set ^ 1, set ^ 1);
            __syncthreads();
        };
        for (int kt = 0; kt < nslab; kt += 2) {
            iteration(kt, std::integral_constant<int, 0>());
            if (kt + 1 < nslab) iteration(kt + 1, std::integral_constant<int, 1>());
        }
    } else {
        // iteration kt loads slab kt + 1 into the one register set, computes
        // slab kt from LDS buffer kt & 1, then stages slab kt + 1 in the other
        gload(0, 0);
        sstore(0, 0);
        __syncthreads();
        for (int kt = 0; kt < nslab; ++kt) {
            if (kt + 1 < nslab) gload(kt + 1, 0);
            compute(kt & 1);
            if (kt + 1 < nslab) sstore((kt + 1) & 1, 0);
            __syncthreads();
        }
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

// The k-contiguous product with the operand slabs loaded straight into LDS
// (buffer loads with the LDS bit: each lane's 16 bytes land at the
// instruction's LDS base + 16 lane), for 256 x 256 blocks of 8 waves (2 x 4,
// each 128 x 64).  128-byte slabs (whole 128-byte lines per row, one request
// to L2 per line) in two LDS stages of 64 KB; the loads hold no registers.
// A slab holds two half-slabs of 64 bytes, each one MFMA k-step for bf16
// (lane group g supplies chunk 4h + g of half h); for fp8 the whole slab is
// one k-step of the 128-deep MFMA.  The loads of slab kt + 1 go out after
// the barrier inside step kt - 1 (once every wave has read slab kt - 1) and
// are waited for at the barrier inside step kt, a lead of one slab.  bf16
// step kt: read half 1 of slab kt, MFMAs of half 0, barrier, read half 0 of
// slab kt + 1, MFMAs of half 1, so that LDS reads always overlap MFMAs of the
// other register set.  A wave waits for its own loads by counting its
// outstanding memory operations; the barrier then makes every wave's part
// visible.  Stage layout: row R at R * 128, chunk c in slot c ^ (R & 7); one
// load instruction fills 8 rows (8 lanes per row).
//
// Measured on gfx950 against the register-staged form (bf16 8192^3 product
// 1.02 -> 0.79 ms): a form with 64-byte slabs in four stages (a lead of three
// half-slabs) came between the two; it sends 64-byte requests to L2, twice as
// many as here.
constexpr int kRawBuffer = 0x00020000;   // raw buffer resource, gfx9 family
constexpr int kDmaThreads = 512;

// s_waitcnt immediates (gfx9 encoding): no vector memory operation of the
// wave outstanding; no LDS read outstanding
constexpr int kVm0 = (7 << 4) | (15 << 8);
constexpr int kLgkm0 = 15 | (3 << 14) | (7 << 4);

template <typename T, bool SCALED>
__global__ __launch_bounds__(kDmaThreads, 1) void k_gemm_nt_dma(const T *__restrict__ A, const T *__restrict__ B,
                                                                float *__restrict__ C, int M, int N, int Kp,
                                                                const float *__restrict__ sa,
                                                                const float *__restrict__ sb) {
    constexpr int BM = 256, BN = 256, WGM = 2, WGN = 4, WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
    constexpr int SL = 128;
    constexpr int STAGE = (BM + BN) * SL;
    constexpr int PER_WAVE = BM / 8 / (kDmaThreads / 64);   // load instructions per wave per operand
    __shared__ __attribute__((aligned(1024))) unsigned char lds[2 * STAGE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WGN, wn = wave % WGN;
    int tm, tn;
    tile_of(blockIdx.x, (M + BM - 1) / BM, (N + BN - 1) / BN, tm, tn);
    const int row_bytes = Kp * (int)sizeof(T);
    const int nslab = row_bytes / SL;
    const unsigned char *Ab = reinterpret_cast<const unsigned char *>(A) + (size_t)tm * BM * row_bytes;
    const unsigned char *Bb = reinterpret_cast<const unsigned char *>(B) + (size_t)tn * BN * row_bytes;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc((void *)Ab, (short)0, BM * row_bytes, kRawBuffer);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, BN * row_bytes, kRawBuffer);
    // row lane / 8 of the instruction's 8, the chunk that belongs in slot lane % 8
    const int vo = (lane >> 3) * row_bytes + 16 * ((lane & 7) ^ ((lane >> 3) & 7));
    auto issue = [&](int slab) {
        unsigned char *st = lds + (slab & 1) * STAGE;
#pragma unroll
        for (int h = 0; h < PER_WAVE; ++h) {
            const int u = PER_WAVE * wave + h;   // rows [8u, 8u + 8) of A and of B
            const int off = vo + u * 8 * row_bytes + slab * SL;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (__attribute__((address_space(3))) void *)(st + u * 1024), 16,
                                                     off, 0, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rb, (__attribute__((address_space(3))) void *)(st + BM * SL + u * 1024), 16, off, 0, 0, 0);
        }
        asm volatile("" ::: "memory");
    };
    // this wave's loads complete and its LDS reads done (waits as builtins,
    // so the compiler knows that nothing issued before them is pending), then
    // the block barrier
    auto wait_barrier = [&]() {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(kVm0);
        __builtin_amdgcn_s_waitcnt(kLgkm0);
        asm volatile("s_barrier" ::: "memory");
    };
    const int r = lane & 15, g = lane >> 4;
    auto read = [&](int slab, int h, u32x4(&af)[TM], u32x4(&bf)[TN]) {
        const unsigned char *st = lds + (slab & 1) * STAGE;
        const int lo = r * SL + 16 * ((4 * h + g) ^ (r & 7));
#pragma unroll
        for (int i = 0; i < TM; ++i)
            af[i] = *reinterpret_cast<const u32x4 *>(st + (wm * WM + i * 16) * SL + lo);
#pragma unroll
        for (int j = 0; j < TN; ++j)
            bf[j] = *reinterpret_cast<const u32x4 *>(st + BM * SL + (wn * WN + j * 16) * SL + lo);
    };

    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // bf16: one half-slab per MFMA k-step
    auto mfma = [&](const u32x4(&af)[TM], const u32x4(&bf)[TN]) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, af[i]),
                                                                    __builtin_bit_cast(bf16x8, bf[j]), acc[i][j], 0, 0,
                                                                    0);
    };
    // fp8: the whole slab in one MFMA k-step of 128 (v_mfma_f32_16x16x128_f8f6f4,
    // e4m3 x e4m3, no block scales): lane group g supplies chunk g of each
    // half, 32 bytes
    auto mfma8 = [&](const u32x4(&a0)[TM], const u32x4(&a1)[TM], const u32x4(&b0)[TN], const u32x4(&b1)[TN]) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const i32x8 a = {(int)a0[i][0], (int)a0[i][1], (int)a0[i][2], (int)a0[i][3],
                                 (int)a1[i][0], (int)a1[i][1], (int)a1[i][2], (int)a1[i][3]};
                const i32x8 b = {(int)b0[j][0], (int)b0[j][1], (int)b0[j][2], (int)b0[j][3],
                                 (int)b1[j][0], (int)b1[j][1], (int)b1[j][2], (int)b1[j][3]};
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[i][j], 0, 0, 0, 0, 0, 0);
            }
    };

    u32x4 fa[2][TM], fb[2][TN];
    if constexpr (sizeof(T) == 2) {
        issue(0);
        wait_barrier();
        if (nslab > 1) issue(1);
        read(0, 0, fa[0], fb[0]);
        for (int kt = 0; kt + 1 < nslab; ++kt) {
            read(kt, 1, fa[1], fb[1]);
            mfma(fa[0], fb[0]);
            // slab kt + 1 has landed and every wave has read slab kt: slab
            // kt + 2 takes its stage
            wait_barrier();
            if (kt + 2 < nslab) issue(kt + 2);
            read(kt + 1, 0, fa[0], fb[0]);
            mfma(fa[1], fb[1]);
        }
        read(nslab - 1, 1, fa[1], fb[1]);
        mfma(fa[0], fb[0]);
        __builtin_amdgcn_s_waitcnt(kLgkm0);
        mfma(fa[1], fb[1]);
    } else {
        // fp8: one MFMA step needs both halves of a slab, so a step reads the
        // whole slab and then multiplies it (the LDS reads of one wave overlap
        // the MFMAs of the other wave on its SIMD); slab kt + 1 goes out once
        // every wave has read slab kt - 1
        issue(0);
        for (int kt = 0; kt < nslab; ++kt) {
            wait_barrier();
            if (kt + 1 < nslab) issue(kt + 1);
            read(kt, 0, fa[0], fb[0]);
            read(kt, 1, fa[1], fb[1]);
            mfma8(fa[0], fa[1], fb[0], fb[1]);
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = tm * BM + wm * WM + i * 16 + 4 * g + e, col = tn * BN + wn * WN + j * 16 + r;
                if (row < M && col < N) {
                    float v = acc[i][j][e];
                    if (SCALED) v = v * (sa[row] * sb[col]);
                    C[(size_t)row * N + col] = v;
                }
            }
}

// FP32 product with the slabs of A and B loaded straight into LDS, for
// shapes of whole 128 x 128 tiles and whole 32-deep k slabs: 128 x 128 blocks
// of 4 waves (64 x 64 each, v_mfma_f32_16x16x4f32), two LDS stages of 32 KB
// (two blocks per CU), the loads of slab kt + 1 issued after the barrier of
// step kt, once every wave has read slab kt - 1.  A slab of A: row R (128
// bytes of k) at R * 128, its 16-byte chunk c in slot c ^ (R & 7); a slab of
// B: k-row r (512 bytes of n) at r * 512, its chunk c in slot
// c ^ (4 ((r >> 2) & 3)), so that the four lane groups of an operand read
// (k-rows 4 apart, 64 bytes each) fall on four different 64-byte spans.
// Lane group g of a k-step of 16 takes k = 4 g .. 4 g + 3 (as the
// register-staged tile does).
constexpr int kF32DmaThreads = 256;

__global__ __launch_bounds__(kF32DmaThreads, 2) void k_gemm_f32_dma(const float *__restrict__ A,
                                                                    const float *__restrict__ B,
                                                                    float *__restrict__ C, int M, int N, int K) {
    constexpr int BM = 128, BN = 128, BK = 32, WM = 64, WN = 64, TM = WM / 16, TN = WN / 16;
    constexpr int A_STAGE = BM * BK * 4, STAGE = A_STAGE + BK * BN * 4;   // 16 KB + 16 KB
    constexpr int PER_WAVE = A_STAGE / 1024 / (kF32DmaThreads / 64);     // load instructions per wave per operand
    __shared__ __attribute__((aligned(1024))) unsigned char lds[2 * STAGE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn;
    tile_of(blockIdx.x, M / BM, N / BN, tm, tn);
    const int nslab = K / BK;
    const unsigned char *Ab = reinterpret_cast<const unsigned char *>(A + (size_t)tm * BM * K);
    const unsigned char *Bb = reinterpret_cast<const unsigned char *>(B + (size_t)tn * BN);
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc((void *)Ab, (short)0, BM * K * 4, kRawBuffer);
    const __amdgpu_buffer_rsrc_t rb =
        __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, (K - 1) * N * 4 + BN * 4, kRawBuffer);
    // A: instruction u fills rows 8u .. 8u + 7 (8 lanes per row); B: k-rows
    // 2u, 2u + 1 (32 lanes per row)
    const int ra_row = lane >> 3, ra_ch = (lane & 7) ^ ((lane >> 3) & 7);
    const int va = ra_row * K * 4 + 16 * ra_ch;
    const int rb_row = lane >> 5;
    auto issue = [&](int slab) {
        unsigned char *st = lds + (slab & 1) * STAGE;
#pragma unroll
        for (int h = 0; h < PER_WAVE; ++h) {
            const int u = PER_WAVE * wave + h;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (__attribute__((address_space(3))) void *)(st + u * 1024), 16,
                                                     va + u * 8 * K * 4 + slab * BK * 4, 0, 0, 0);
            const int kr = 2 * u + rb_row;                               // k-row of the slab
            const int ch = (lane & 31) ^ (4 * ((kr >> 2) & 3));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rb, (__attribute__((address_space(3))) void *)(st + A_STAGE + u * 1024), 16,
                (slab * BK + kr) * N * 4 + 16 * ch, 0, 0, 0);
        }
        asm volatile("" ::: "memory");
    };
    auto wait_barrier = [&]() {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(kVm0);
        __builtin_amdgcn_s_waitcnt(kLgkm0);
        asm volatile("s_barrier" ::: "memory");
    };
    const int r = lane & 15, g = lane >> 4;
    floatx4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&](int slab) {
        const unsigned char *st = lds + (slab & 1) * STAGE;
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            const int c = ks / 4 + g;                                    // this lane group's chunk of A
            floatx4 af[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const floatx4 *>(st + (wm * WM + i * 16 + r) * 128 + 16 * (c ^ (r & 7)));
            const int x = 4 * ((ks / 4 + g) & 3);                        // B swizzle of k-rows ks + 4g + s
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int kr = ks + 4 * g + s4;
                float bf[TN];
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int n = wn * WN + j * 16 + r;
                    bf[j] = *reinterpret_cast<const float *>(st + A_STAGE + kr * 512 + 16 * ((n >> 2) ^ x) +
                                                             4 * (n & 3));
                }
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const float a = af[i][s4];
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    };
    issue(0);
    for (int kt = 0; kt < nslab; ++kt) {
        // slab kt has landed and every wave has read slab kt - 1, so slab
        // kt + 1 takes its stage
        wait_barrier();
        if (kt + 1 < nslab) issue(kt + 1);
        compute(kt);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = tm * BM + wm * WM + i * 16 + 4 * g + e, col = tn * BN + wn * WN + j * 16 + r;
                C[(size_t)row * N + col] = acc[i][j][e];
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
    // large products: 128 x 128 tiles (with LDS-direct loads when the shape
    // is whole tiles and slabs and the operands fit the 31-bit offsets of a
    // buffer load, unless knob OFL_GEMM_F32_FORM=reg); smaller ones: 64 x 64
    // so that the grid still covers the CUs
    if ((M / 128) * (N / 128) >= 512) {
        const char *form = std::getenv("OFL_GEMM_F32_FORM");
        const bool dma = !(form && form[0] == 'r') && M % 128 == 0 && N % 128 == 0 && K % 32 == 0 &&
                         128 * K * 4 < ((int64_t)1 << 31) && K * N * 4 < ((int64_t)1 << 31);
        if (dma)
            return launch(k_gemm_f32_dma, dim3((unsigned)((M / 128) * (N / 128))), dim3(kF32DmaThreads), 0, s, A, B,
                          C, (int)M, (int)N, (int)K);
        return launch_f32<128, 128, 32>(A, B, C, (int)M, (int)N, (int)K, s);
    }
    return launch_f32<64, 64, 32>(A, B, C, (int)M, (int)N, (int)K, s);
}

// ---------------------------------------------------------------- split-precision GEMM
namespace {
// Tile of the k-contiguous product (rows of A' x rows of B'): 128 x 128
// (4 waves of 64 x 64, two blocks per CU), or 256 x 256 (8 waves of
// 128 x 64, one block per CU: a third less LDS traffic per MFMA) for
// products of at least 256 such tiles.  An earlier 256 x 256 form with 4
// waves of 128 x 128 (one wave per SIMD) measured slower than 128 x 128 at
// 4096 (521 vs 472 us, bf16x3): its LDS and global latencies stayed exposed.
// Knob OFL_GEMM_NT_TILE=128/256 forces a tile.
int nt_tile(int64_t M, int64_t N) {
    if (const char *e = std::getenv("OFL_GEMM_NT_TILE")) {
        if (std::atoi(e) == 256) return 256;
        if (std::atoi(e) == 128) return 128;
    }
    return ((M + 255) / 256) * ((N + 255) / 256) >= 256 ? 256 : 128;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Workspace layout of one product: [A' | B' | float area], A' omitted when
// bf16 inputs are already tile-aligned.  float area (fp8 only): row scales,
// column scales, their inverses, and per-slice column maxima.
struct NtLayout {
    int tile = 128;
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
    L.tile = nt_tile(M, N);
    L.Mp = round_up(M, L.tile);
    L.Np = round_up(N, L.tile);
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

template <typename T, bool SCALED>
hipError_t launch_nt(const NtLayout &L, const void *A, const void *B, float *C, int64_t M, int64_t N,
                     const float *sa, const float *sb, hipStream_t s) {
    const unsigned tiles = (unsigned)((L.Mp / L.tile) * (L.Np / L.tile));
    // knob OFL_GEMM_NT_LAYOUT=0/1: the LDS layout of the staged slabs
    const char *lay = std::getenv("OFL_GEMM_NT_LAYOUT");
    const bool cm = !(lay && lay[0] == '0');
    const T *a = static_cast<const T *>(A), *b = static_cast<const T *>(B);
    const int m = (int)M, n = (int)N, kp = (int)L.Kp;
    // 256 x 256 tiles: the form with LDS-direct loads, unless knob
    // OFL_GEMM_NT_FORM=reg asks for the register-staged one or a tile's panel
    // (256 rows) exceeds the 31-bit offsets of a buffer load
    const char *form = std::getenv("OFL_GEMM_NT_FORM");
    const bool dma = !(form && form[0] == 'r') && 256 * L.Kp * (int64_t)sizeof(T) < ((int64_t)1 << 31);
    if (L.tile == 256 && dma)
        return launch((k_gemm_nt_dma<T, SCALED>), dim3(tiles), dim3(kDmaThreads), 0, s, a, b, C, m, n, kp, sa, sb);
    if (L.tile == 256)
        return cm ? launch((k_gemm_nt<T, 256, 256, 2, 4, 1, 1, 1, SCALED>), dim3(tiles), dim3(512), 0, s, a, b, C, m,
                           n, kp, sa, sb)
                  : launch((k_gemm_nt<T, 256, 256, 2, 4, 1, 1, 0, SCALED>), dim3(tiles), dim3(512), 0, s, a, b, C, m,
                           n, kp, sa, sb);
    return cm ? launch((k_gemm_nt<T, 128, 128, 2, 2, 2, 2, 1, SCALED>), dim3(tiles), dim3(kThreads), 0, s, a, b, C, m,
                       n, kp, sa, sb)
              : launch((k_gemm_nt<T, 128, 128, 2, 2, 2, 2, 0, SCALED>), dim3(tiles), dim3(kThreads), 0, s, a, b, C, m,
                       n, kp, sa, sb);
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
    hipError_t e = L.b_pad ? fill_zero(Bp, (uint64_t)L.b_bytes, s) : hipSuccess;
    if (variant == 1) {
        if (e == hipSuccess) e = prep_a(A, Ap, nullptr, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 0, s);
        if (e == hipSuccess) e = split_bt(B, Bp, nullptr, (int)K, (int)N, (int)L.Kp, 0, s);
        if (e == hipSuccess) e = launch_nt<unsigned short, false>(L, Ap, Bp, C, M, N, nullptr, nullptr, s);
        return e;
    }
    if (e == hipSuccess) e = row_scales(A, sa, isa, (int)M, (int)K, s);
    if (e == hipSuccess) e = col_scales(B, sb, isb, colmax, (int)K, (int)N, (int)L.Np, s);
    if (e == hipSuccess) e = prep_a(A, Ap, sa, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 1, s);
    if (e == hipSuccess) e = split_bt(B, Bp, sb, (int)K, (int)N, (int)L.Kp, 1, s);
    if (e == hipSuccess) e = launch_nt<unsigned char, true>(L, Ap, Bp, C, M, N, isa, isb, s);
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
    hipError_t e = L.b_pad ? fill_zero(Bp, (uint64_t)L.b_bytes, s) : hipSuccess;
    if (L.a_copy) {
        if (e == hipSuccess) e = prep_a(A, w, nullptr, (int)M, (int)K, (int)L.Mp, (int)L.Kp, 2, s);
        Ause = w;
    }
    if (e == hipSuccess) e = split_bt(B, Bp, nullptr, (int)K, (int)N, (int)L.Kp, 2, s);
    if (e == hipSuccess) e = launch_nt<unsigned short, false>(L, Ause, Bp, C, M, N, nullptr, nullptr, s);
    return e;
}

}  // namespace k
}  // namespace ofl
