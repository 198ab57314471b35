// 19-point weighted-Jacobi sweep with the FP64 residual, and the interior copy
// (definition and per-item code in stencil_item.hpp).  The plane-local sums x
// and y are formed once per loaded plane and reused by the three output
// planes that need them.
//
// Per-wave forms (gfx950, wave64): a work item is 64 consecutive k (lanes
// 1..62 produce outputs, lanes 0 and 63 only supply the k-1 / k+1
// neighbours; or two columns per lane), JR consecutive rows j and a run of IC
// planes along i.  A wave marches along i holding a, x, y of three planes in
// registers, with the next three planes already in flight in a register
// ring: every element of p is loaded once per work item (plus two halo rows
// and two halo planes), the k neighbours arrive through DPP lane shifts, and
// no LDS is used.  Waves loop over work items (grid sized to the resident
// wave slots, so there is no tail round).  These serve grids below 192
// interior planes, where launches and latency, not bandwidth, set the time.
//
// Band form (k_stencil19b, grids of 192 and more interior planes): a block
// owns a band of rows across the whole row; each plane's rows are staged in
// LDS as one contiguous range with aligned 16-byte loads, which is what the
// memory system serves near copy speed on rows of arbitrary alignment, and
// the waves march along i as above.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "dev_common.hpp"
#include "kernels.hpp"
#include "launch.hpp"
#include "batch_jobs.hpp"
#include "stencil_item.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kThreads = kStencilThreads;

// The residual: every wave stores the sum of its squared differences in
// partials[wave] (a plain store: no atomics and no fences in the sweep, whose
// blocks would otherwise serialise on one counter and write back or
// invalidate their XCD's L2 once per block), and k_residual_finish, launched
// after the sweep on the same stream, adds the partials in wave order.
template <int JR, int SP>
__global__ __launch_bounds__(kThreads) void k_stencil19(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                        double *partials) {
    const int lane = threadIdx.x & (kWave - 1);
    // blocks are dealt to the 8 XCDs round-robin: renumber them so that one
    // XCD takes a contiguous run of work items (neighbouring j-runs share
    // their halo rows in that XCD's L2); gridDim.x is a multiple of 8
    const int nb = gridDim.x;
    const int lb = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = nb * kWavesPerBlock;
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, g.bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, g.bytes, kBufferConfig);
    double acc = 0.0;
    for (int w = lb * kWavesPerBlock + wib; w < g.items; w += nwaves) acc = stencil_item<JR, SP>(rp, rq, g, w, lane, acc);
    acc = wave_sum(acc);
    if (lane == 0) partials[lb * kWavesPerBlock + wib] = acc;
}

// The sweep with two columns per lane (stencil_item_w); same grid logic.
template <int JR, int SP>
__global__ __launch_bounds__(kThreads) void k_stencil19w(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                         double *partials) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nb = gridDim.x;
    const int lb = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = nb * kWavesPerBlock;
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, g.bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, g.bytes, kBufferConfig);
    double acc = 0.0;
    for (int w = lb * kWavesPerBlock + wib; w < g.items; w += nwaves) acc = stencil_item_w<JR, SP>(rp, rq, g, w, lane, acc);
    acc = wave_sum(acc);
    if (lane == 0) partials[lb * kWavesPerBlock + wib] = acc;
}

// Band sweep for grids whose interior row spans at most 8 k-tiles of 128
// columns.  A block of 16 waves owns a band of TB = 64 / NKT rows covering
// every column of the interior (NKT waves across a row, each 128 columns with
// two columns per lane; 16 / NKT row groups of 4 rows) and a run of planes.
// Per plane the block stages the TB + 2 rows it reads -- one contiguous range
// of the plane -- in LDS through 16-byte loads and stores (the loads of a plane
// go out one step before it is staged), then
// every wave derives a, x, y of its 4 rows x 128 columns from LDS (lanes 0 and
// 63 read the tile's halo columns) and marches along i with a, x, y of three
// planes in registers, as stencil_item does.  Per point the arithmetic is that
// of stencil_item, in the same order.  One barrier per plane: a plane's staging
// buffer (two buffers, alternating) is written only after every wave has
// passed the barrier of the step after the one that last read it.
//
// DMA variant (DMA = true): the plane loads go straight from memory into LDS
// (buffer loads with the LDS bit: each lane's 16 bytes land at the wave's LDS
// base + 16 lane), three staging buffers, and planes i+2 and i+3 in flight
// while plane i is produced -- a lead of two steps at no register cost.  A
// wave waits for its own loads of the plane it derives next by counting its
// outstanding memory operations (s_waitcnt vmcnt: loads and stores of a wave
// complete in order of issue for this count), then the block barrier makes
// every wave's loads of that plane visible.
constexpr int kBandThreads = 1024;
constexpr int kBandChunks = 3;                               // 16-byte pieces per thread per plane
constexpr int kBandCap = kBandChunks * kBandThreads * 4;     // floats per staging buffer

// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector
// memory operations of the wave are outstanding, and nothing else
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

struct GeoB {
    int I, J, K;
    int IC;                  // planes per item
    int TB;                  // rows per band
    int nbands, nic, items;  // items: band fastest, then plane run
    int bytes;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <int NKT, int SP, bool DMA, int LP = 0>
__global__ __launch_bounds__(kBandThreads) void k_stencil19b(const float *__restrict__ p, float *__restrict__ q, GeoB g,
                                                             double *partials) {
    constexpr int RG = 16 / NKT;
    static_assert(RG * NKT == 16, "16 waves per block");
    constexpr int NBUF = DMA ? 3 : 2;
    __shared__ __attribute__((aligned(16))) float lds[NBUF][kBandCap];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int kt = wv % NKT, rg = wv / NKT;
    const int nb = gridDim.x;
    const int lb = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int I = g.I, J = g.J, K = g.K;
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, g.bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, g.bytes, kBufferConfig);
    const int c0 = 1 + kOutV * kt + 2 * lane;                 // this lane's first column
    const bool cols_full = kOutV * (kt + 1) <= K - 2;         // every lane's two columns interior
    const bool out0 = c0 <= K - 2, out1 = c0 + 1 <= K - 2;
    const int edge = lane == 0 ? c0 - 1 : lane == kWave - 1 ? c0 + 2 : c0;   // halo column read
    const int voff = c0 * 4;
    double acc = 0.0;

    for (int it = lb; it < g.items; it += nb) {
        const int bt = it % g.nbands, ic = it / g.nbands;
        const int jb = 1 + bt * g.TB;
        const int ib = 1 + ic * g.IC, ie = min(ib + g.IC, I - 1);
        const int rend = min(jb + g.TB + 1, J);               // rows [jb-1, rend) are staged
        const int wr = jb + 4 * rg;                           // this wave's first output row
        const bool full = cols_full && wr + 3 <= J - 2;
        const int jlast = J - 2 - wr;

        f32x4 st[kBandChunks];
        f32x2 Pa[3][4], Px[3][4], Py[3][4];

        // global loads of plane i's staged range (none past ie)
        auto issue = [&](int i, f32x4 (&v)[kBandChunks]) {
            const int ii = min(i, I - 1);
            const int f0 = (ii * J + jb - 1) * K, f1 = (ii * J + rend) * K;
            const int a0 = f0 & ~3;
#pragma unroll
            for (int u = 0; u < kBandChunks; ++u) {
                const int e = a0 + 4 * (u * kBandThreads + tid);
                v[u] = __builtin_bit_cast(
                    f32x4, __builtin_amdgcn_raw_buffer_load_b128(rp, (i <= ie && e < f1) ? e * 4 : kOutOfRange, 0, LP));
            }
        };
        auto stage = [&](const f32x4 (&v)[kBandChunks], float *buf) {
#pragma unroll
            for (int u = 0; u < kBandChunks; ++u) *(f32x4 *)(buf + 4 * (u * kBandThreads + tid)) = v[u];
        };
        // DMA form: plane i's staged range straight into buf (kBandChunks
        // memory operations per wave, issued whether or not they are masked)
        auto issue_lds = [&](int i, float *buf) {
            const int ii = min(i, I - 1);
            const int f0 = (ii * J + jb - 1) * K, f1 = (ii * J + rend) * K;
            const int a0 = f0 & ~3;
#pragma unroll
            for (int u = 0; u < kBandChunks; ++u) {
                const int e = a0 + 4 * (u * kBandThreads + tid);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rp, (__attribute__((address_space(3))) void *)(buf + 4 * (u * kBandThreads + wv * kWave)), 16,
                    (i <= ie && e < f1) ? e * 4 : kOutOfRange, 0, 0, LP);
            }
            asm volatile("" ::: "memory");
        };
        // wait until this wave has at most N memory operations outstanding,
        // then the block barrier (after the wave's LDS reads have completed)
        auto wait_barrier = [&](auto NC) {
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(decltype(NC)::value));
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        };
        // a, x, y of this wave's 4 rows of plane i from the staged plane
        auto derive = [&](const float *buf, int i, f32x2 (&a)[4], f32x2 (&x)[4], f32x2 (&y)[4]) {
            const int sh = ((min(i, I - 1) * J + jb - 1) * K) & 3;   // staged range starts sh floats early
            f32x2 v[6], h[6];
            float e[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const float *row = buf + (4 * rg + r) * K + sh;
                v[r] = f32x2{row[c0], row[c0 + 1]};
                e[r] = row[edge];
            }
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                h[r].x = from_left_or(v[r].y, e[r]) + v[r].y;
                h[r].y = v[r].x + from_right_or(v[r].x, e[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[r] = v[r + 1];
                x[r].x = (v[r].x + v[r + 2].x) + h[r + 1].x;
                x[r].y = (v[r].y + v[r + 2].y) + h[r + 1].y;
                y[r].x = h[r].x + h[r + 2].x;
                y[r].y = h[r].y + h[r + 2].y;
            }
        };
        auto point = [&](float am, float an, float ac, float xm, float xn, float xc, float yc) {
            const float F = (am + an) + xc;
            const float E = (xm + xn) + yc;
            const float t0 = 0.25f * ac;
            const float t1 = 0.0625f * F;
            const float t2 = 0.03125f * E;
            return (t0 + t1) + t2;
        };
        // step k of the run (output plane i = ib + k): stage plane i+1 (its
        // loads went out one step earlier), load plane i+2, derive plane i+1,
        // produce plane i.  DMA form: wait for plane i+1 (loaded two steps
        // earlier), load plane i+3 into the buffer plane i left, derive plane
        // i+1, produce plane i; WAIT is the wave's memory operations issued
        // after plane i+1's loads (2 S + 3 from the third step on, S stores
        // per step).
        auto step = [&](auto S, auto FULLC, int i, auto WAIT) {
            constexpr bool FULL = decltype(FULLC)::value;
            constexpr int k3 = decltype(S)::value;
            constexpr int m = k3, c = (k3 + 1) % 3, n = (k3 + 2) % 3;
            float *buf;
            if constexpr (DMA) {
                // plane t is staged in buffer (t - ib + 1) mod 3
                buf = lds[(k3 + 2) % 3];
                wait_barrier(WAIT);
                issue_lds(i + 3, lds[(k3 + 1) % 3]);
            } else {
                buf = lds[(i + 1 - ib) & 1];               // plane t is staged in buffer (t - ib) mod 2
                stage(st, buf);
                __syncthreads();
                issue(i + 2, st);
            }
            derive(buf, i + 1, Pa[n], Px[n], Py[n]);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v0 = point(Pa[m][r].x, Pa[n][r].x, Pa[c][r].x, Px[m][r].x, Px[n][r].x, Px[c][r].x, Py[c][r].x);
                const float v1 = point(Pa[m][r].y, Pa[n][r].y, Pa[c][r].y, Px[m][r].y, Px[n][r].y, Px[c][r].y, Py[c][r].y);
                const int base = ((i * J + wr + r) * K) * 4;
                const double d0 = (double)v0 - (double)Pa[c][r].x;
                const double d1 = (double)v1 - (double)Pa[c][r].y;
                if constexpr (FULL) {
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, f32x2{v0, v1}), rq, base + voff, 0,
                                                          SP);
                    acc = __builtin_fma(d0, d0, acc);
                    acc = __builtin_fma(d1, d1, acc);
                } else {
                    const bool ok0 = out0 && r <= jlast, ok1 = out1 && r <= jlast;
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v0), rq,
                                                          ok0 ? base + voff : kOutOfRange, 0, SP);
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v1), rq,
                                                          ok1 ? base + voff + 4 : kOutOfRange, 0, SP);
                    acc = __builtin_fma(ok0 ? d0 : 0.0, d0, acc);
                    acc = __builtin_fma(ok1 ? d1 : 0.0, d1, acc);
                }
            }
        };

        // every wave passes the same barriers whichever store path it takes
        auto run = [&](auto FULLC) {
            constexpr int SPS = decltype(FULLC)::value ? 4 : 8;   // stores per step and wave
            using W0 = std::integral_constant<int, 0>;
            if constexpr (DMA) {
                // the previous item's last reads of the staging buffers are
                // done, and all of its loads (masked ones write zeros) landed
                wait_barrier(W0());
                issue_lds(ib - 1, lds[0]);
                issue_lds(ib, lds[1]);
                issue_lds(ib + 1, lds[2]);
                wait_barrier(std::integral_constant<int, 2 * kBandChunks>());
                derive(lds[0], ib - 1, Pa[0], Px[0], Py[0]);
                wait_barrier(std::integral_constant<int, kBandChunks>());
                issue_lds(ib + 2, lds[0]);
                derive(lds[1], ib, Pa[1], Px[1], Py[1]);
                using WA = std::integral_constant<int, kBandChunks>;
                using WB = std::integral_constant<int, SPS + kBandChunks>;
                using WC = std::integral_constant<int, 2 * SPS + kBandChunks>;
                // the first two steps have fewer operations behind their plane
                step(std::integral_constant<int, 0>(), FULLC, ib, WA());
                if (ib + 1 < ie) {
                    step(std::integral_constant<int, 1>(), FULLC, ib + 1, WB());
                    if (ib + 2 < ie) step(std::integral_constant<int, 2>(), FULLC, ib + 2, WC());
                }
                for (int i0 = ib + 3; i0 < ie; i0 += 3) {
                    step(std::integral_constant<int, 0>(), FULLC, i0, WC());
                    if (i0 + 1 < ie) {
                        step(std::integral_constant<int, 1>(), FULLC, i0 + 1, WC());
                        if (i0 + 2 < ie) step(std::integral_constant<int, 2>(), FULLC, i0 + 2, WC());
                    }
                }
            } else {
                // the previous item's last reads of the staging buffers are done
                __syncthreads();
                issue(ib - 1, st);
                stage(st, lds[1]);
                issue(ib, st);
                __syncthreads();
                derive(lds[1], ib - 1, Pa[0], Px[0], Py[0]);
                stage(st, lds[0]);
                issue(ib + 1, st);
                __syncthreads();
                derive(lds[0], ib, Pa[1], Px[1], Py[1]);
                for (int i0 = ib; i0 < ie; i0 += 3) {
                    step(std::integral_constant<int, 0>(), FULLC, i0, W0());
                    if (i0 + 1 < ie) {
                        step(std::integral_constant<int, 1>(), FULLC, i0 + 1, W0());
                        if (i0 + 2 < ie) step(std::integral_constant<int, 2>(), FULLC, i0 + 2, W0());
                    }
                }
            }
        };
        if (full)
            run(std::true_type());
        else
            run(std::false_type());
    }
    // DMA form: no load into this block's LDS may still be in flight when it ends
    if constexpr (DMA) __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    acc = wave_sum(acc);
    if (lane == 0) partials[lb * (kBandThreads / kWave) + wv] = acc;
}

// res_slot[0] += the n wave partials of a sweep, in a fixed order
// (ordered_sum_into), by one whole block of 256 threads: k_residual_finish,
// or the extra block of an interior copy launched next.
constexpr int kFinishThreads = kOrderedSumThreads;
static_assert(kFinishThreads == kThreads, "the copy's extra block runs the finish");

__global__ __launch_bounds__(kFinishThreads) void k_residual_finish(const double *__restrict__ partials, int n,
                                                                    double *res_slot) {
    ordered_sum_into(partials, n, res_slot);
}

// p[i][j][k] = q[i][j][k] on the interior: a wave copies ROWS consecutive
// rows (i, j) at a time.
// With fin_n > 0 the grid has one extra (last) block, which adds up the
// residual partials of the sweep launched before instead of copying.
template <int ROWS, int POL>
__global__ __launch_bounds__(kThreads) void k_copy_interior(float *__restrict__ p, const float *__restrict__ q,
                                                            int I, int J, int K, const double *fin_partials,
                                                            int fin_n, double *fin_slot) {
    const int copy_blocks = (int)gridDim.x - (fin_n > 0 ? 1 : 0);
    if ((int)blockIdx.x >= copy_blocks) {
        ordered_sum_into(fin_partials, fin_n, fin_slot);
        return;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int gwave = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int nwaves = copy_blocks * kWavesPerBlock;
    const int rows = (I - 2) * (J - 2);
    const int bytes = I * J * K * 4;
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, bytes, kBufferConfig);
    for (int row0 = gwave * ROWS; row0 < rows; row0 += nwaves * ROWS) copy_rows<ROWS, POL>(rp, rq, J, K, rows, row0, lane);
}

// p = q on the interior, plane-range form: in every interior plane i the
// elements p[i][1][1] .. p[i][J-2][K-2] lie in one contiguous range of
// (J-2) K - 2 floats, which is copied in 16-byte pieces aligned to the
// buffer, U pieces per lane in flight (loads first); the only elements of
// that range outside the interior are the boundary columns between
// consecutive rows (k = K-1, then k = 0 of the next row), and a piece that
// holds one of them (or straddles an end of the range) is written dword by
// dword without them.  Grid: x covers a plane's pieces, y the interior
// planes, plus one more row of blocks whose first block runs the residual
// finish of the sweep launched before (fin_n > 0).
template <int U, int LPOL, int SPOL>
__global__ __launch_bounds__(kThreads) void k_copy_interior_flat(float *__restrict__ p, const float *__restrict__ q,
                                                                 int I, int J, int K, float invK,
                                                                 const double *fin_partials, int fin_n,
                                                                 double *fin_slot) {
    const int plane = blockIdx.y;
    if (plane >= I - 2) {
        if (blockIdx.x == 0) ordered_sum_into(fin_partials, fin_n, fin_slot);
        return;
    }
    const int i = plane + 1;
    const int pbase = i * J * K;                      // first element of plane i
    const int s = pbase + K + 1;                      // p[i][1][1]
    const int e = pbase + (J - 2) * K + K - 1;        // one past p[i][J-2][K-2]
    const int bytes = I * J * K * 4;
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, bytes, kBufferConfig);
    const int g0 = (s >> 2) + blockIdx.x * (kThreads * U) + (int)threadIdx.x;   // first piece of this lane
    __attribute__((ext_vector_type(4))) unsigned v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = 4 * (g0 + u * kThreads);
        v[u] = __builtin_amdgcn_raw_buffer_load_b128(rq, f < e ? f * 4 : kOutOfRange, 0, LPOL);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int f = 4 * (g0 + u * kThreads);
        // column of the piece's first element (r < 2^24: exact in float, the
        // quotient off by at most one)
        const int r = f - pbase;
        int kq = (int)((float)r * invK);
        int k = r - kq * K;
        if (k < 0) k += K;
        if (k >= K) k -= K;
        const bool whole = f >= s && f + 4 <= e && k >= 1 && k + 3 <= K - 2;
        __builtin_amdgcn_raw_buffer_store_b128(v[u], rp, whole ? f * 4 : kOutOfRange, 0, SPOL);
        if (!whole && f < e) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int kt = k + t;
                if (kt >= K) kt -= K;
                const bool ok = f + t >= s && f + t < e && kt != 0 && kt != K - 1;
                __builtin_amdgcn_raw_buffer_store_b32(v[u][t], rp, ok ? (f + t) * 4 : kOutOfRange, 0, SPOL);
            }
        }
    }
}

// Sweep forms: one column per lane (62 outputs per wave), two columns per
// lane (126 outputs), two columns per lane with scalar-loaded halo columns
// (128 outputs, 8-byte stores on interior tiles).
enum Form { kFormOne = 0, kFormWide = 1, kFormBand = 2 };

struct Config {
    int JR;
    int form = kFormOne;
    bool store_nt = false;   // q written with the non-temporal policy
    Geo g;
    GeoB gb;                 // band form
    int nkt = 0;             // band form: waves across a row (1, 2, 4, 8)
    bool dma = false;        // band form: planes loaded straight into LDS
    bool load_nt = false;    // band form, 8 waves across: planes read with the streaming policy
    unsigned blocks;
    int waves_per_block = kWavesPerBlock;
};

// Waves across a row for the band form (a power of two covering the interior
// row in 128-column tiles), 0 when the row is too long for it.
int band_nkt(int64_t K) {
    const int64_t t = (K - 2 + kOutV - 1) / kOutV;
    return t <= 1 ? 1 : t <= 2 ? 2 : t <= 4 ? 4 : t <= 8 ? 8 : 0;
}

GeoB make_geo_band(int64_t I, int64_t J, int64_t K, int nkt, int IC) {
    GeoB g;
    g.I = (int)I;
    g.J = (int)J;
    g.K = (int)K;
    g.bytes = (int)(I * J * K * 4);
    g.TB = 64 / nkt;
    g.nbands = (int)((J - 2 + g.TB - 1) / g.TB);
    const int64_t ni = I - 2;
    if (IC > ni) IC = (int)ni;
    if (IC < 1) IC = 1;
    g.IC = IC;
    g.nic = (int)((ni + IC - 1) / IC);
    g.items = g.nbands * g.nic;
    return g;
}

int resident_blocks_per_cu(int JR, int form);
int band_blocks_per_cu(int nkt, bool dma);

bool valid_jr(int JR) { return JR == 2 || JR == 4 || JR == 8; }

// Tuning knobs, used by tuning sweeps: OFL_STENCIL_CFG="JR,IC" overrides the
// choice (JR rows per item, IC planes per work item, 0 = automatic) and then
// selects one column per lane unless a form is named: OFL_STENCIL_WIDE=0/1
// (one / two columns per lane) or OFL_STENCIL_FORM=1/w/b (one column, two
// columns, band), the latter taking precedence.  JR is one of 2, 4, 8 (the
// band form ignores it); IC = 0 keeps the automatic choice.
bool env_override(int &JR, int &IC) {
    const char *s = std::getenv("OFL_STENCIL_CFG");
    if (!s) return false;
    int a, b;
    if (std::sscanf(s, "%d,%d", &a, &b) != 2) return false;
    if (!((a == 2 || a == 4 || a == 8) && b >= 0)) return false;
    JR = a;
    IC = b;
    return true;
}

// Work items: JR rows, i-runs of IC planes; the grid holds at most one block
// per resident slot and waves loop over the items.  Defaults measured on
// gfx950 (sweep kernel time, median of interleaved runs):
//   fewer than 192 interior planes: JR = 4, IC = 6 (3 below 96 planes):
//     129x129x257 9.9 us (JR 8: 10.8; IC 4 / 8: 11.8 / 10.9; the band form
//     18.3 us: too few bands), 65x65x129 5.6 us
//   192 planes and more, rows of at most 8 k-tiles: the band form with
//     about one item per block (IC = interior planes / (blocks / bands)):
//     257x257x513 50.8 us (one column per lane, JR 8, IC 12: 55.1),
//     513x513x1025 412 us (IC 64: 415, IC 16: 440; two columns per lane,
//     JR 8, IC 16: 579)
//   longer rows: two columns per lane, JR = 8, IC = 16
Config choose(int64_t I, int64_t J, int64_t K) {
    Config c;
    const int64_t ni = I - 2;
    int JR = 0, IC = 0;
    const bool forced = env_override(JR, IC);
    if (!forced) JR = ni >= 192 ? 8 : 4;
    const bool band_default = !forced && ni >= 192 && band_nkt(K) > 0;
    const int ic_asked = IC;   // 0: automatic
    if (IC <= 0) IC = ni >= 384 ? 16 : ni >= 192 ? 12 : ni >= 96 ? 6 : 3;
    c.form = band_default ? kFormBand : !forced && ni >= 384 ? kFormWide : kFormOne;
    // q with the non-temporal policy on grids of 4 MB to 512 MB: measured
    // faster at 129x129x257 (9.9 vs 12.3 us) and 257x257x513 (54.4 vs 61.1),
    // slower at 513x513x1025 (654 vs 573) and 65x65x129 (6.4 vs 5.6);
    // OFL_STENCIL_NT=0/1 overrides
    const int64_t grid_bytes = I * J * K * 4;
    c.store_nt = grid_bytes >= ((int64_t)4 << 20) && grid_bytes <= ((int64_t)512 << 20);
    if (const char *nt = std::getenv("OFL_STENCIL_NT")) c.store_nt = nt[0] == '1';
    if (const char *lnt = std::getenv("OFL_STENCIL_LNT")) c.load_nt = lnt[0] == '1';
    if (const char *wd = std::getenv("OFL_STENCIL_WIDE")) c.form = wd[0] == '1' ? kFormWide : kFormOne;
    if (const char *fm = std::getenv("OFL_STENCIL_FORM")) {
        c.form = fm[0] == 'b' || fm[0] == 'd' ? kFormBand : fm[0] == 'w' ? kFormWide : kFormOne;
        c.dma = fm[0] == 'd';
    }
    if (c.form == kFormBand) {
        c.nkt = band_nkt(K);
        if (c.nkt > 0) {
            c.JR = JR;
            const int64_t slots = (int64_t)cu_count() * band_blocks_per_cu(c.nkt, c.dma);
            if (ic_asked <= 0) {
                // about one item per resident block: the fewest halo planes
                const int64_t nbands = (J - 2 + 64 / c.nkt - 1) / (64 / c.nkt);
                const int64_t runs = std::max<int64_t>(1, slots / nbands);
                IC = (int)((ni + runs - 1) / runs);
            }
            c.gb = make_geo_band(I, J, K, c.nkt, IC);
            const int64_t blocks = std::min<int64_t>(c.gb.items, slots);
            c.blocks = (unsigned)((blocks + 7) / 8 * 8);
            c.waves_per_block = kBandThreads / kWave;
            return c;
        }
        c.form = kFormWide;   // rows too long for the band form
    }
    if (!valid_jr(JR)) JR = 8;
    c.JR = JR;
    c.g = make_geo(I, J, K, JR, IC, c.form == kFormWide ? kOutW : kOut);
    const int64_t resident_blocks = (int64_t)cu_count() * resident_blocks_per_cu(JR, c.form);
    int64_t blocks = ((int64_t)c.g.items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > resident_blocks) blocks = resident_blocks;
    blocks = (blocks + 7) / 8 * 8;
    c.blocks = (unsigned)blocks;
    return c;
}

hipError_t launch_band(const Config &c, const float *p, float *q, double *partials, hipStream_t s) {
    const dim3 grid(c.blocks), block(kBandThreads);
#define OFL_BAND(N)                                                                                               \
    case N:                                                                                                       \
        if (c.dma)                                                                                                \
            return c.store_nt ? launch((k_stencil19b<N, kNonTemporal, true>), grid, block, 0, s, p, q, c.gb, partials) \
                              : launch((k_stencil19b<N, 0, true>), grid, block, 0, s, p, q, c.gb, partials);          \
        return c.store_nt ? launch((k_stencil19b<N, kNonTemporal, false>), grid, block, 0, s, p, q, c.gb, partials)    \
                          : launch((k_stencil19b<N, 0, false>), grid, block, 0, s, p, q, c.gb, partials);
    if (c.load_nt && c.nkt == 8 && !c.dma)   // tuning knob: planes read with the streaming policy
        return c.store_nt ? launch((k_stencil19b<8, kNonTemporal, false, kNonTemporal>), grid, block, 0, s, p, q,
                                   c.gb, partials)
                          : launch((k_stencil19b<8, 0, false, kNonTemporal>), grid, block, 0, s, p, q, c.gb, partials);
    switch (c.nkt) {
        OFL_BAND(1)
        OFL_BAND(2)
        OFL_BAND(4)
        OFL_BAND(8)
    default:
        return hipErrorInvalidValue;
    }
#undef OFL_BAND
}

template <int JR>
hipError_t launch_t(const Config &c, const float *p, float *q, double *partials, hipStream_t s) {
    const dim3 grid(c.blocks), block(kThreads);
    if (c.form == kFormWide) {
        if (c.store_nt) return launch((k_stencil19w<JR, kNonTemporal>), grid, block, 0, s, p, q, c.g, partials);
        return launch((k_stencil19w<JR, 0>), grid, block, 0, s, p, q, c.g, partials);
    }
    if (c.store_nt) return launch((k_stencil19<JR, kNonTemporal>), grid, block, 0, s, p, q, c.g, partials);
    return launch((k_stencil19<JR, 0>), grid, block, 0, s, p, q, c.g, partials);
}

template <typename Kern>
int occupancy_of(Kern kern) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

int resident_blocks_per_cu(int JR, int form) {
    static std::once_flag once;
    static int table[2][3];   // [one column, two columns][JR 2, 4, 8]
    std::call_once(once, [] {
        table[0][0] = occupancy_of(k_stencil19<2, 0>);
        table[0][1] = occupancy_of(k_stencil19<4, 0>);
        table[0][2] = occupancy_of(k_stencil19<8, 0>);
        table[1][0] = occupancy_of(k_stencil19w<2, 0>);
        table[1][1] = occupancy_of(k_stencil19w<4, 0>);
        table[1][2] = occupancy_of(k_stencil19w<8, 0>);
    });
    return table[form == kFormWide ? 1 : 0][JR == 2 ? 0 : JR == 4 ? 1 : 2];
}

int band_blocks_per_cu(int nkt, bool dma) {
    static std::once_flag once;
    static int table[2][4];
    std::call_once(once, [] {
        auto occ = [](auto kern) {
            int n = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kBandThreads, 0) != hipSuccess || n < 1) n = 1;
            return n;
        };
        table[0][0] = occ(k_stencil19b<1, 0, false>);
        table[0][1] = occ(k_stencil19b<2, 0, false>);
        table[0][2] = occ(k_stencil19b<4, 0, false>);
        table[0][3] = occ(k_stencil19b<8, 0, false>);
        table[1][0] = occ(k_stencil19b<1, 0, true>);
        table[1][1] = occ(k_stencil19b<2, 0, true>);
        table[1][2] = occ(k_stencil19b<4, 0, true>);
        table[1][3] = occ(k_stencil19b<8, 0, true>);
    });
    return table[dma ? 1 : 0][nkt == 1 ? 0 : nkt == 2 ? 1 : nkt == 4 ? 2 : 3];
}

}  // namespace

int cu_count() {
    static std::once_flag once;
    static int n = 256;
    std::call_once(once, [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            n = v;
    });
    return n;
}

// Work-item geometry of a sweep over an I x J x K grid with JR-row items and
// i-runs of IC planes (IC clamped to the interior).
Geo make_geo(int64_t I, int64_t J, int64_t K, int JR, int IC, int kout) {
    Geo g;
    const int64_t ni = I - 2, nj = J - 2;
    g.I = (int)I;
    g.J = (int)J;
    g.K = (int)K;
    g.bytes = (int)(I * J * K * 4);
    g.nkt = (int)((K - 2 + kout - 1) / kout);
    g.njt = (int)((nj + JR - 1) / JR);
    if (IC > ni) IC = (int)ni;
    if (IC < 1) IC = 1;
    g.IC = IC;
    g.nic = (int)((ni + IC - 1) / IC);
    g.items = (int)((int64_t)g.nkt * g.njt * g.nic);
    return g;
}

int64_t stencil_partials(int64_t I, int64_t J, int64_t K) {
    if (I < 3 || J < 3 || K < 3) return 1;
    // upper bound over every configuration the launcher may choose: one
    // partial per wave, one block per resident slot (at most 2048 threads
    // per CU), blocks rounded up to 8
    return ((int64_t)cu_count() * (2048 / kThreads) + 8) * kWavesPerBlock;
}

hipError_t residual_finish(ResidualFinish &fin, hipStream_t s) {
    const ResidualFinish f = fin;
    fin = ResidualFinish{};
    if (f.n <= 0) return hipSuccess;
    return launch(k_residual_finish, dim3(1), dim3(kFinishThreads), 0, s, f.partials, f.n, f.target);
}

hipError_t stencil19_sweep(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                           const ReduceScratch &rs, hipStream_t s, ResidualFinish &fin) {
    // a finish still owed reads the partials this sweep overwrites: do it first
    if (fin.n > 0) {
        const hipError_t e = residual_finish(fin, s);
        if (e != hipSuccess) return e;
    }
    if (I < 3 || J < 3 || K < 3) return hipSuccess;   // no interior: nothing written, residual unchanged
    // byte offsets are non-negative 32-bit ints: the loop may form offsets up
    // to five planes past the end (read as 0); dropped stores use 2^31
    if ((I + 6) * J * K * 4 >= (1ll << 31)) return hipErrorInvalidValue;
    const Config c = choose(I, J, K);
    const int waves = (int)c.blocks * c.waves_per_block;
    if ((int64_t)waves > rs.capacity) return hipErrorInvalidValue;
    const hipError_t e = c.form == kFormBand ? launch_band(c, p, q, rs.partials, s)
                         : c.JR == 8         ? launch_t<8>(c, p, q, rs.partials, s)
                         : c.JR == 4         ? launch_t<4>(c, p, q, rs.partials, s)
                                     : launch_t<2>(c, p, q, rs.partials, s);
    if (e != hipSuccess) return e;
    fin = ResidualFinish{rs.partials, waves, res_slot};
    return hipSuccess;
}

hipError_t stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                     const ReduceScratch &rs, hipStream_t s) {
    ResidualFinish fin;
    const hipError_t e = stencil19_sweep(p, q, I, J, K, res_slot, rs, s, fin);
    if (e != hipSuccess) return e;
    return residual_finish(fin, s);
}

// Tuning knob: OFL_COPY_CFG="ROWS,BLOCKS_PER_CU,NT" (ROWS in {2,4,8}, NT 0/1);
// true when it is set.
bool copy_env_override(int &rows_per_wave, int &bpc, int &nt) {
    const char *s = std::getenv("OFL_COPY_CFG");
    if (!s) return false;
    int a = 0, b = 0, c = 0;
    if (std::sscanf(s, "%d,%d,%d", &a, &b, &c) < 2) return false;
    if (a == 2 || a == 4 || a == 8) rows_per_wave = a;
    if (b >= 1 && b <= 64) bpc = b;
    nt = c == 1 ? 1 : 0;
    return true;
}

// Tuning knob: OFL_COPY_FLAT="U,LNT,SNT" for the plane-range form.
void flat_env_override(int &u, int &lnt, int &snt) {
    const char *e = std::getenv("OFL_COPY_FLAT");
    if (!e) return;
    int a = 0, b = 0, c = 0;
    if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && (a == 1 || a == 2 || a == 4)) {
        u = a;
        lnt = b == 1;
        snt = c == 1;
    }
}

template <int ROWS>
hipError_t launch_copy(float *p, const float *q, int64_t I, int64_t J, int64_t K, int bpc, int nt,
                       const ResidualFinish &f, hipStream_t s) {
    const int64_t rows = (I - 2) * (J - 2);
    int64_t blocks = (rows + kWavesPerBlock * ROWS - 1) / (kWavesPerBlock * ROWS);
    if (blocks > (int64_t)cu_count() * bpc) blocks = (int64_t)cu_count() * bpc;
    if (f.n > 0) ++blocks;   // the finish block
    if (nt)
        return launch((k_copy_interior<ROWS, kNonTemporal>), dim3((unsigned)blocks), dim3(kThreads), 0, s, p, q,
                      (int)I, (int)J, (int)K, f.partials, f.n, f.target);
    return launch((k_copy_interior<ROWS, 0>), dim3((unsigned)blocks), dim3(kThreads), 0, s, p, q, (int)I, (int)J,
                  (int)K, f.partials, f.n, f.target);
}

// Plane-range copy, U 16-byte pieces per lane, load / store policies
template <int U, int LPOL, int SPOL>
hipError_t launch_copy_flat_u(float *p, const float *q, int64_t I, int64_t J, int64_t K, const ResidualFinish &f,
                              hipStream_t s) {
    // pieces a plane's range may touch: its floats / 4, plus one for a
    // misaligned start and one for the end
    const int64_t pieces = ((J - 2) * K - 2) / 4 + 2;
    const int64_t bx = (pieces + kThreads * U - 1) / (kThreads * U);
    const dim3 grid((unsigned)bx, (unsigned)(I - 2 + (f.n > 0 ? 1 : 0)));
    const float invK = 1.0f / (float)K;
    return launch((k_copy_interior_flat<U, LPOL, SPOL>), grid, dim3(kThreads), 0, s, p, q, (int)I, (int)J, (int)K,
                  invK, f.partials, f.n, f.target);
}

// Tuning knob OFL_COPY_FLAT="U,LNT,SNT": pieces per lane (1, 2 or 4) and the
// streaming policy for the loads / stores (0 or 1), overriding the choice.
template <int U>
hipError_t launch_copy_flat_p(float *p, const float *q, int64_t I, int64_t J, int64_t K, int lnt, int snt,
                              const ResidualFinish &f, hipStream_t s) {
    if (lnt && snt) return launch_copy_flat_u<U, kNonTemporal, kNonTemporal>(p, q, I, J, K, f, s);
    if (lnt) return launch_copy_flat_u<U, kNonTemporal, 0>(p, q, I, J, K, f, s);
    if (snt) return launch_copy_flat_u<U, 0, kNonTemporal>(p, q, I, J, K, f, s);
    return launch_copy_flat_u<U, 0, 0>(p, q, I, J, K, f, s);
}

hipError_t launch_copy_flat(float *p, const float *q, int64_t I, int64_t J, int64_t K, int u, int lnt, int snt,
                            const ResidualFinish &f, hipStream_t s) {
    if (u == 1) return launch_copy_flat_p<1>(p, q, I, J, K, lnt, snt, f, s);
    if (u == 2) return launch_copy_flat_p<2>(p, q, I, J, K, lnt, snt, f, s);
    return launch_copy_flat_p<4>(p, q, I, J, K, lnt, snt, f, s);
}

hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s,
                         ResidualFinish *fin) {
    const ResidualFinish f = fin ? *fin : ResidualFinish{};
    if (fin) *fin = ResidualFinish{};
    if (I < 3 || J < 3 || K < 3) {   // nothing to copy: the finish still runs
        ResidualFinish g = f;
        return residual_finish(g, s);
    }
    if (I * J * K * 4 >= (1ll << 31)) return hipErrorInvalidValue;   // 32-bit buffer offsets
    // Forms measured on gfx950 (sweep + copy pair, the sweep's time depends
    // on what the copy leaves in the caches):
    //   grids of 512 MB and more: plane-range form, one 16-byte piece per
    //     lane, streaming loads and stores -- 513x513x1025 pair 746 us
    //     (copy 360 + sweep 386) against 833 (431 + 402) in the row form;
    //     the copy's streaming stores leave no dirty lines of p for the
    //     sweep to write back
    //   64 MB to 512 MB: plane-range form, two pieces per lane, cached --
    //     257x257x513 pair 90.8 us against 96.5 (streaming: 106.5; the
    //     grids partly stay in the 256 MB last-level cache)
    //   smaller: row form, 8 rows per wave and 16 blocks per CU up to 64 K
    //     interior rows, 2 rows and 32 blocks per CU beyond -- 129x129x257
    //     pair 19.2 us (plane-range forms 19.6-27.7)
    // Knobs: OFL_COPY_FORM=flat / rows forces a form, OFL_COPY_CFG and
    // OFL_COPY_FLAT its parameters.
    const int64_t grid_bytes = I * J * K * 4;
    const bool small = (I - 2) * (J - 2) <= 65536;
    int rows_per_wave = small ? 8 : 2, bpc = small ? 16 : 32, nt = 0;
    const bool cfg_set = copy_env_override(rows_per_wave, bpc, nt);
    const char *form = std::getenv("OFL_COPY_FORM");
    const bool flat_ok = (I - 2) <= 65535;
    bool flat = flat_ok && grid_bytes >= ((int64_t)64 << 20);
    if (form) flat = flat_ok && form[0] == 'f';
    if (flat) {
        const bool huge = grid_bytes >= ((int64_t)512 << 20);
        int u = huge ? 1 : 2, lnt = huge ? 1 : 0, snt = lnt;
        if (cfg_set) lnt = snt = nt;
        flat_env_override(u, lnt, snt);
        return launch_copy_flat(p, q, I, J, K, u, lnt, snt, f, s);
    }
    if (rows_per_wave == 2) return launch_copy<2>(p, q, I, J, K, bpc, nt, f, s);
    if (rows_per_wave == 8) return launch_copy<8>(p, q, I, J, K, bpc, nt, f, s);
    return launch_copy<4>(p, q, I, J, K, bpc, nt, f, s);
}

}  // namespace k
}  // namespace ofl
