// 19-point weighted-Jacobi sweep with the FP64 residual, and the interior copy.
//
// Sweep definition (centre 1/4, faces 1/16, edges 1/32; FP32, fixed order):
//   per plane m:  a_m = p[m][j][k]
//                 x_m = (p[m][j-1][k] + p[m][j+1][k]) + (p[m][j][k-1] + p[m][j][k+1])
//                 y_m = (p[m][j-1][k-1] + p[m][j-1][k+1]) + (p[m][j+1][k-1] + p[m][j+1][k+1])
//   F = (a_{i-1} + a_{i+1}) + x_i,  E = (x_{i-1} + x_{i+1}) + y_i,
//   q = (0.25 a_i + 0.0625 F) + 0.03125 E,   res += ((double)q - (double)a_i)^2.
// The plane-local sums x and y are formed once per loaded plane and reused by
// the three output planes that need them.
//
// Mapping (gfx950, wave64): a work item is 64 consecutive k (lanes 1..62
// produce outputs, lanes 0 and 63 only supply the k-1 / k+1 neighbours), JR
// consecutive rows j and a run of IC planes along i.  A wave marches along i
// holding a, x, y of three planes in registers, with the next three planes
// already in flight in a register ring: every element of p is loaded once per
// work item (plus two halo rows and two halo planes), the k neighbours arrive
// through DPP lane shifts, and no LDS is used.  Waves loop over work items
// (grid sized to the resident wave slots, so there is no tail round); the
// four waves of a block take neighbouring j-runs, sharing halo rows in L1.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "dev_common.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kThreads = 256;
constexpr int kOut = 62;          // output lanes per wave along k
constexpr int kWavesPerBlock = kThreads / kWave;

// Value of lane l-1 (k-1 neighbour) / lane l+1 (k+1 neighbour) of the wave.
// DPP wave_shr:1 / wave_shl:1; the end lanes get 0 and never produce output.
__device__ inline float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ inline float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

struct Geo {
    int I, J, K;
    int IC;                 // planes per work item
    int nkt, njt, nic;      // work items along k, j, i
    int items;              // nkt * njt * nic
    int bytes;              // size of p (and q) in bytes, < 2^31
};

constexpr int kBufferConfig = 0x00020000;   // raw buffer resource, gfx9 family

// The whole byte offset goes in the per-lane (VGPR) operand with a zero SGPR
// offset: the raw-buffer range check covers the VGPR offset, so an access
// at or past num_records reads 0 / is dropped and never touches memory.
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// One sweep.  Work item w (jt fastest, then kt, then ic) covers rows
// jb .. jb+JR-1, the 62 output columns of k-tile kt and planes [ib, ie).
// Plane sets P[0..2] hold a, x, y of planes i-1, i, i+1 with roles rotating
// every step (the i-loop is unrolled by three, so no register moves); the ring
// holds the next three raw planes in flight.  Loads are raw buffer loads; the
// loop body has no branches: loads beyond the work item are clamped into the
// array (their values feed no stored output), so refills are unconditional,
// and a store that must not happen gets an offset past num_records, which the
// raw-buffer range check drops.
constexpr int kOutOfRange = (int)0x80000000u;

template <int JR>
__global__ __launch_bounds__(kThreads) void k_stencil19(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                        double *res_slot, double *partials, unsigned *counter) {
    constexpr int R = JR + 2;
    const int lane = threadIdx.x & (kWave - 1);
    // blocks are dealt to the 8 XCDs round-robin: renumber them so that one
    // XCD takes a contiguous run of work items (neighbouring j-runs share
    // their halo rows in that XCD's L2); gridDim.x is a multiple of 8
    const int nb = gridDim.x;
    const int lb = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = nb * kWavesPerBlock;
    const int J = g.J, K = g.K;
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, g.bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, g.bytes, kBufferConfig);
    double acc = 0.0;

    for (int w = lb * kWavesPerBlock + wib; w < g.items; w += nwaves) {
        // k-tile fastest: the waves of a block take neighbouring k-tiles of
        // the same rows in lockstep, so the cache lines a tile boundary
        // straddles are fetched once and hit in L1 for the other wave
        const int kt = w % g.nkt;
        const int rest = w / g.nkt;
        const int jt = rest % g.njt;
        const int ic = rest / g.njt;
        const int k = kt * kOut + lane;             // lane 0 holds k-1 of the first output
        const int voff = k * 4;
        const int kld = min(k, K - 1) * 4;          // loads stay inside the row
        const bool kout = lane >= 1 && lane <= kOut && k <= K - 2;
        const int jb = 1 + jt * JR;                 // first output row
        const int ib = 1 + ic * g.IC;
        const int ie = min(ib + g.IC, g.I - 1);     // exclusive; ib < ie by construction
        const int jlast = J - 2 - jb;               // rows r <= jlast are interior

        float Pa[3][JR], Px[3][JR], Py[3][JR];
        float ring[3][R];

        // every load offset lies inside the array: planes past the last and
        // rows past the last are clamped (those values feed no stored output)
        auto load = [&](int i, float (&v)[R]) {
            const int ii = min(i, g.I - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = buf_load(rp, ((ii * J + min(jb - 1 + r, J - 1)) * K) * 4 + kld);
        };
        auto derive = [&](const float (&v)[R], float (&a)[JR], float (&x)[JR], float (&y)[JR]) {
            float h[R];                             // p[j][k-1] + p[j][k+1] per row
#pragma unroll
            for (int r = 0; r < R; ++r) h[r] = from_left(v[r]) + from_right(v[r]);
#pragma unroll
            for (int r = 0; r < JR; ++r) {
                a[r] = v[r + 1];
                x[r] = (v[r] + v[r + 2]) + h[r + 1];
                y[r] = h[r] + h[r + 2];
            }
        };
        auto step = [&](auto S, int i) {
            constexpr int s = decltype(S)::value;
            constexpr int m = s, c = (s + 1) % 3, n = (s + 2) % 3;
            // keep each step's use of its ring slot in place: hoisting the
            // later slots' use to the loop top would wait for the newest loads
            __builtin_amdgcn_sched_barrier(0);
            derive(ring[s], Pa[n], Px[n], Py[n]);            // plane i+1
            // the refill must not start before the slot's old value is consumed,
            // or old and new value need separate registers (a copy per iteration);
            // past the run's last plane it re-reads that plane (an L1 hit)
            __builtin_amdgcn_sched_barrier(0);
            load(min(i + 4, ie), ring[s]);
            const bool plane_ok = i < ie;
#pragma unroll
            for (int r = 0; r < JR; ++r) {
                const float F = (Pa[m][r] + Pa[n][r]) + Px[c][r];
                const float E = (Px[m][r] + Px[n][r]) + Py[c][r];
                const float t0 = 0.25f * Pa[c][r];
                const float t1 = 0.0625f * F;
                const float t2 = 0.03125f * E;
                const float v = (t0 + t1) + t2;
                const bool ok = kout && plane_ok && r <= jlast;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rq,
                                                      ok ? ((i * J + jb + r) * K) * 4 + voff : kOutOfRange, 0, 0);
                const double d = (double)v - (double)Pa[c][r];
                acc = __builtin_fma(ok ? d : 0.0, d, acc);
            }
        };

        {
            float r0[R], r1[R];
            load(ib - 1, r0);
            load(ib, r1);
            load(ib + 1, ring[0]);
            load(min(ib + 2, ie), ring[1]);
            load(min(ib + 3, ie), ring[2]);
            derive(r0, Pa[0], Px[0], Py[0]);
            derive(r1, Pa[1], Px[1], Py[1]);
        }
        for (int i0 = ib; i0 < ie; i0 += 3) {
            step(std::integral_constant<int, 0>(), i0);
            step(std::integral_constant<int, 1>(), i0 + 1);
            step(std::integral_constant<int, 2>(), i0 + 2);
        }
    }
    reduce_finish(acc, partials, counter, res_slot);
}

// p[i][j][k] = q[i][j][k] on the interior: a wave copies kRows consecutive
// rows (i, j) at a time.  Each row splits into a head [lo, a0) and a tail
// [a1, hi) of at most three elements and a 16-byte aligned middle [a0, a1);
// a pass moves up to 64 middle groups of every row plus the heads and tails.
// Raw buffer accesses without branches: every load reads a valid element
// (element 0 when the lane has nothing to move), so all loads of a pass
// overlap, and a store that must not happen carries an offset past
// num_records, which the range check drops.
constexpr int kRows = 4;

__global__ __launch_bounds__(kThreads) void k_copy_interior(float *__restrict__ p, const float *__restrict__ q,
                                                            int I, int J, int K) {
    const int lane = threadIdx.x & (kWave - 1);
    const int gwave = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int rows = (I - 2) * (J - 2);
    const int bytes = I * J * K * 4;
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, bytes, kBufferConfig);
    const int passes = ((K - 2) / 4 + kWave) / kWave;   // >= ceil(groups / 64), groups <= (K-2)/4
    for (int row0 = gwave * kRows; row0 < rows; row0 += nwaves * kRows) {
        int lo[kRows], a0[kRows], a1[kRows], hi[kRows];
        bool live[kRows];
#pragma unroll
        for (int t = 0; t < kRows; ++t) {
            live[t] = row0 + t < rows;
            const int row = live[t] ? row0 + t : rows - 1;
            const int i = 1 + row / (J - 2), j = 1 + row % (J - 2);
            const int base = (i * J + j) * K;
            lo[t] = base + 1;
            hi[t] = base + K - 1;                 // [lo, hi)
            a0[t] = (lo[t] + 3) & ~3;
            a1[t] = hi[t] & ~3;
            if (a1[t] < a0[t]) a1[t] = a0[t];     // no aligned group: all in head / tail
        }
        for (int pass = 0; pass < passes; ++pass) {
            __attribute__((ext_vector_type(4))) unsigned mid[kRows];
            unsigned hd[kRows], tl[kRows];
            int om[kRows], oh[kRows], ot[kRows];
#pragma unroll
            for (int t = 0; t < kRows; ++t) {
                const int em = a0[t] + 4 * (pass * kWave + lane);
                const int eh = lo[t] + lane, et = a1[t] + lane;
                om[t] = (live[t] && em < a1[t]) ? em * 4 : -1;
                oh[t] = (live[t] && pass == 0 && eh < a0[t] && eh < hi[t]) ? eh * 4 : -1;
                ot[t] = (live[t] && pass == 0 && et < hi[t] && et >= a0[t]) ? et * 4 : -1;
                mid[t] = __builtin_amdgcn_raw_buffer_load_b128(rq, om[t] < 0 ? 0 : om[t], 0, 0);
                hd[t] = __builtin_amdgcn_raw_buffer_load_b32(rq, oh[t] < 0 ? 0 : oh[t], 0, 0);
                tl[t] = __builtin_amdgcn_raw_buffer_load_b32(rq, ot[t] < 0 ? 0 : ot[t], 0, 0);
            }
#pragma unroll
            for (int t = 0; t < kRows; ++t) {
                __builtin_amdgcn_raw_buffer_store_b128(mid[t], rp, om[t] < 0 ? kOutOfRange : om[t], 0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(hd[t], rp, oh[t] < 0 ? kOutOfRange : oh[t], 0, 0);
                __builtin_amdgcn_raw_buffer_store_b32(tl[t], rp, ot[t] < 0 ? kOutOfRange : ot[t], 0, 0);
            }
        }
    }
}

struct Config {
    int JR;
    Geo g;
    unsigned blocks;
};

int resident_blocks_per_cu(int JR);

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

// Tuning knob: OFL_STENCIL_CFG="JR,IC" overrides the choice (JR in {2,4,8},
// IC planes per work item, 0 = automatic); used by tuning sweeps.
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

// Work items: JR = 8 rows, i-runs of IC planes; the grid holds at most one
// block per resident slot and waves loop over the items.
Config choose(int64_t I, int64_t J, int64_t K) {
    Config c;
    const int64_t ni = I - 2, nj = J - 2;
    int JR = 0, IC = 0;
    if (!env_override(JR, IC)) {
        JR = 8;
        IC = 0;
    }
    c.JR = JR;
    c.g.I = (int)I;
    c.g.J = (int)J;
    c.g.K = (int)K;
    c.g.bytes = (int)(I * J * K * 4);
    c.g.nkt = (int)((K - 2 + kOut - 1) / kOut);
    c.g.njt = (int)((nj + JR - 1) / JR);
    const int64_t per_plane_run = (int64_t)c.g.nkt * c.g.njt;
    const int64_t resident_blocks = (int64_t)cu_count() * resident_blocks_per_cu(JR);
    if (IC <= 0) {
        // measured on gfx950 (129^3-, 257^3- and 513^3-class grids): runs of
        // 48 planes (a few work items per resident wave) on grids with at
        // least 192 interior planes, 12 planes below that
        IC = ni >= 192 ? 48 : 12;
    }
    if (IC > ni) IC = (int)ni;
    c.g.IC = IC;
    c.g.nic = (int)((ni + IC - 1) / IC);
    c.g.items = (int)(per_plane_run * c.g.nic);
    int64_t blocks = ((int64_t)c.g.items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > resident_blocks) blocks = resident_blocks;
    blocks = (blocks + 7) / 8 * 8;
    c.blocks = (unsigned)blocks;
    return c;
}

template <int JR>
hipError_t launch_t(const Config &c, const float *p, float *q, double *res_slot, const ReduceScratch &rs,
                    hipStream_t s) {
    return launch((k_stencil19<JR>), dim3(c.blocks), dim3(kThreads), 0, s, p, q, c.g, res_slot, rs.partials,
                       rs.counter);
}

template <int JR>
int occupancy_t() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stencil19<JR>, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

int resident_blocks_per_cu(int JR) {
    static std::once_flag once;
    static int table[3];
    std::call_once(once, [] {
        table[0] = occupancy_t<2>();
        table[1] = occupancy_t<4>();
        table[2] = occupancy_t<8>();
    });
    return table[JR == 2 ? 0 : JR == 4 ? 1 : 2];
}

}  // namespace

int64_t stencil_partials(int64_t I, int64_t J, int64_t K) {
    if (I < 3 || J < 3 || K < 3) return 1;
    // upper bound over every configuration the launcher may choose: one block
    // per resident slot (at most 2048 threads per CU), rounded up to 8
    return (int64_t)cu_count() * (2048 / kThreads) + 8;
}

hipError_t stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                     const ReduceScratch &rs, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;   // no interior: nothing written, residual unchanged
    // byte offsets are non-negative 32-bit ints: the loop may form offsets up
    // to five planes past the end (read as 0); dropped stores use 2^31
    if ((I + 6) * J * K * 4 >= (1ll << 31)) return hipErrorInvalidValue;
    const Config c = choose(I, J, K);
    if ((int64_t)c.blocks > rs.capacity) return hipErrorInvalidValue;
    if (c.JR == 8) return launch_t<8>(c, p, q, res_slot, rs, s);
    if (c.JR == 4) return launch_t<4>(c, p, q, res_slot, rs, s);
    return launch_t<2>(c, p, q, res_slot, rs, s);
}

hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;
    if (I * J * K * 4 >= (1ll << 31)) return hipErrorInvalidValue;   // 32-bit buffer offsets
    const int64_t rows = (I - 2) * (J - 2);
    int64_t blocks = (rows + kWavesPerBlock * kRows - 1) / (kWavesPerBlock * kRows);
    if (blocks > (int64_t)cu_count() * 16) blocks = (int64_t)cu_count() * 16;
    return launch(k_copy_interior, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, q, (int)I, (int)J, (int)K);
}

}  // namespace k
}  // namespace ofl
