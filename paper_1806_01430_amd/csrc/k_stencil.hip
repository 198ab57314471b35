// 19-point weighted-Jacobi sweep with the FP64 residual, and the interior copy
// (definition and per-item code in stencil_item.hpp).  The plane-local sums x
// and y are formed once per loaded plane and reused by the three output
// planes that need them.
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

// The sweep with 128 output columns per wave (stencil_item_v): items whose
// tile lies wholly inside the interior take the mask-free path.
template <int JR, int SP>
__global__ __launch_bounds__(kThreads) void k_stencil19v(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                         double *partials) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nb = gridDim.x;
    const int lb = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int nwaves = nb * kWavesPerBlock;
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, g.bytes, kBufferConfig);
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc((void *)q, (short)0, g.bytes, kBufferConfig);
    const int nkt_full = (g.K - 2) / kOutV, njt_full = (g.J - 2) / JR;
    double acc = 0.0;
    for (int w = lb * kWavesPerBlock + wib; w < g.items; w += nwaves) {
        const int kt = w % g.nkt, jt = (w / g.nkt) % g.njt;
        if (kt < nkt_full && jt < njt_full)
            acc = stencil_item_v<JR, true, SP>(rp, rq, g, w, lane, acc);
        else
            acc = stencil_item_v<JR, false, SP>(rp, rq, g, w, lane, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) partials[lb * kWavesPerBlock + wib] = acc;
}

// res_slot[0] += the n wave partials of a sweep, in a fixed order: thread t
// sums partials t, t + 256, ... (loads unrolled so that they overlap), then a
// tree over the threads in LDS.  Executed by one whole block of 256 threads:
// k_residual_finish, or the extra block of an interior copy launched next.
constexpr int kFinishThreads = 256;
static_assert(kFinishThreads == kThreads, "the copy's extra block runs the finish");

__device__ inline void finish_block(const double *__restrict__ partials, int n, double *res_slot) {
    __shared__ double t[kFinishThreads];
    const int tid = threadIdx.x;
    double s = 0.0;
    int i = tid;
    for (; i + 3 * kFinishThreads < n; i += 4 * kFinishThreads) {
        const double a = partials[i], b = partials[i + kFinishThreads];
        const double c = partials[i + 2 * kFinishThreads], d = partials[i + 3 * kFinishThreads];
        s += a;
        s += b;
        s += c;
        s += d;
    }
    for (; i < n; i += kFinishThreads) s += partials[i];
    t[tid] = s;
    __syncthreads();
#pragma unroll
    for (int h = kFinishThreads / 2; h > 0; h >>= 1) {
        if (tid < h) t[tid] += t[tid + h];
        __syncthreads();
    }
    if (tid == 0) res_slot[0] = res_slot[0] + t[0];
}

__global__ __launch_bounds__(kFinishThreads) void k_residual_finish(const double *__restrict__ partials, int n,
                                                                    double *res_slot) {
    finish_block(partials, n, res_slot);
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
        finish_block(fin_partials, fin_n, fin_slot);
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

// Sweep forms: one column per lane (62 outputs per wave), two columns per
// lane (126 outputs), two columns per lane with scalar-loaded halo columns
// (128 outputs, 8-byte stores on interior tiles).
enum Form { kFormOne = 0, kFormWide = 1, kFormV = 2 };

struct Config {
    int JR;
    int form = kFormOne;
    bool store_nt = false;   // q written with the non-temporal policy
    Geo g;
    unsigned blocks;
};

int resident_blocks_per_cu(int JR, int form);

bool valid_jr(int JR, int form) {
    return form == kFormV ? (JR == 4 || JR == 6 || JR == 8) : (JR == 2 || JR == 4 || JR == 8);
}

// Tuning knobs, used by tuning sweeps: OFL_STENCIL_CFG="JR,IC" overrides the
// choice (JR rows per item, IC planes per work item, 0 = automatic) and then
// selects one column per lane unless a form is named: OFL_STENCIL_WIDE=0/1
// (one / two columns per lane) or OFL_STENCIL_FORM=1/w/v (one column, two
// columns, two columns with 128 outputs per wave), the latter taking
// precedence.  JR is one of 2, 4, 8 (forms 1 and w) or 4, 6, 8 (form v).
bool env_override(int &JR, int &IC) {
    const char *s = std::getenv("OFL_STENCIL_CFG");
    if (!s) return false;
    int a, b;
    if (std::sscanf(s, "%d,%d", &a, &b) != 2) return false;
    if (!((a == 2 || a == 4 || a == 6 || a == 8) && b >= 0)) return false;
    JR = a;
    IC = b;
    return true;
}

// Work items: JR rows, i-runs of IC planes; the grid holds at most one block
// per resident slot and waves loop over the items.  Defaults measured on
// gfx950 (sweep kernel time, median of interleaved runs):
//   fewer than 192 interior planes: JR = 4, IC = 6 (3 below 96 planes):
//     129x129x257 10.2 us (JR 8: 10.8; IC 4 / 8: 11.8 / 10.9), 65x65x129 5.6 us
//   192 .. 383 planes: JR = 8, IC = 12: 257x257x513 54.5 us (IC 24: 55.5,
//     IC 48: 61.8, two columns per lane: 57.5)
//   384 and more: two columns per lane, JR = 8, IC = 16: 513x513x1025 574 us
//     (one column per lane, IC 48: 599)
Config choose(int64_t I, int64_t J, int64_t K) {
    Config c;
    const int64_t ni = I - 2;
    int JR = 0, IC = 0;
    const bool forced = env_override(JR, IC);
    if (!forced) JR = ni >= 192 ? 8 : 4;
    if (IC <= 0) IC = ni >= 384 ? 16 : ni >= 192 ? 12 : ni >= 96 ? 6 : 3;
    c.form = !forced && ni >= 384 ? kFormWide : kFormOne;
    // q with the non-temporal policy on grids of 4 MB to 512 MB: measured
    // faster at 129x129x257 (9.9 vs 12.3 us) and 257x257x513 (54.4 vs 61.1),
    // slower at 513x513x1025 (654 vs 573) and 65x65x129 (6.4 vs 5.6);
    // OFL_STENCIL_NT=0/1 overrides
    const int64_t grid_bytes = I * J * K * 4;
    c.store_nt = grid_bytes >= ((int64_t)4 << 20) && grid_bytes <= ((int64_t)512 << 20);
    if (const char *nt = std::getenv("OFL_STENCIL_NT")) c.store_nt = nt[0] == '1';
    if (const char *wd = std::getenv("OFL_STENCIL_WIDE")) c.form = wd[0] == '1' ? kFormWide : kFormOne;
    if (const char *fm = std::getenv("OFL_STENCIL_FORM"))
        c.form = fm[0] == 'v' ? kFormV : fm[0] == 'w' ? kFormWide : kFormOne;
    if (!valid_jr(JR, c.form)) JR = 8;
    c.JR = JR;
    c.g = make_geo(I, J, K, JR, IC, c.form == kFormV ? kOutV : c.form == kFormWide ? kOutW : kOut);
    const int64_t resident_blocks = (int64_t)cu_count() * resident_blocks_per_cu(JR, c.form);
    int64_t blocks = ((int64_t)c.g.items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > resident_blocks) blocks = resident_blocks;
    blocks = (blocks + 7) / 8 * 8;
    c.blocks = (unsigned)blocks;
    return c;
}

template <int JR>
hipError_t launch_t(const Config &c, const float *p, float *q, double *partials, hipStream_t s) {
    const dim3 grid(c.blocks), block(kThreads);
    if (c.form == kFormV) {
        if constexpr (JR == 2) {
            return hipErrorInvalidValue;
        } else {
            if (c.store_nt) return launch((k_stencil19v<JR, kNonTemporal>), grid, block, 0, s, p, q, c.g, partials);
            return launch((k_stencil19v<JR, 0>), grid, block, 0, s, p, q, c.g, partials);
        }
    }
    if constexpr (JR == 6) {
        return hipErrorInvalidValue;
    } else {
        if (c.form == kFormWide) {
            if (c.store_nt) return launch((k_stencil19w<JR, kNonTemporal>), grid, block, 0, s, p, q, c.g, partials);
            return launch((k_stencil19w<JR, 0>), grid, block, 0, s, p, q, c.g, partials);
        }
        if (c.store_nt) return launch((k_stencil19<JR, kNonTemporal>), grid, block, 0, s, p, q, c.g, partials);
        return launch((k_stencil19<JR, 0>), grid, block, 0, s, p, q, c.g, partials);
    }
}

template <typename Kern>
int occupancy_of(Kern kern) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kThreads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

int resident_blocks_per_cu(int JR, int form) {
    static std::once_flag once;
    static int table[3][4];   // [form][JR 2, 4, 6, 8]
    std::call_once(once, [] {
        table[0][0] = occupancy_of(k_stencil19<2, 0>);
        table[0][1] = occupancy_of(k_stencil19<4, 0>);
        table[0][3] = occupancy_of(k_stencil19<8, 0>);
        table[1][0] = occupancy_of(k_stencil19w<2, 0>);
        table[1][1] = occupancy_of(k_stencil19w<4, 0>);
        table[1][3] = occupancy_of(k_stencil19w<8, 0>);
        table[2][1] = occupancy_of(k_stencil19v<4, 0>);
        table[2][2] = occupancy_of(k_stencil19v<6, 0>);
        table[2][3] = occupancy_of(k_stencil19v<8, 0>);
        table[0][2] = table[1][2] = table[2][0] = 1;
    });
    return table[form][JR / 2 - 1];
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
    const int waves = (int)c.blocks * kWavesPerBlock;
    if ((int64_t)waves > rs.capacity) return hipErrorInvalidValue;
    const hipError_t e = c.JR == 8   ? launch_t<8>(c, p, q, rs.partials, s)
                         : c.JR == 6 ? launch_t<6>(c, p, q, rs.partials, s)
                         : c.JR == 4 ? launch_t<4>(c, p, q, rs.partials, s)
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

// Tuning knob: OFL_COPY_CFG="ROWS,BLOCKS_PER_CU,NT" (ROWS in {2,4,8}, NT 0/1).
void copy_env_override(int &rows_per_wave, int &bpc, int &nt) {
    const char *s = std::getenv("OFL_COPY_CFG");
    if (!s) return;
    int a = 0, b = 0, c = 0;
    if (std::sscanf(s, "%d,%d,%d", &a, &b, &c) < 2) return;
    if (a == 2 || a == 4 || a == 8) rows_per_wave = a;
    if (b >= 1 && b <= 64) bpc = b;
    nt = c == 1 ? 1 : 0;
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

hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s,
                         ResidualFinish *fin) {
    const ResidualFinish f = fin ? *fin : ResidualFinish{};
    if (fin) *fin = ResidualFinish{};
    if (I < 3 || J < 3 || K < 3) {   // nothing to copy: the finish still runs
        ResidualFinish g = f;
        return residual_finish(g, s);
    }
    if (I * J * K * 4 >= (1ll << 31)) return hipErrorInvalidValue;   // 32-bit buffer offsets
    // measured on gfx950: 8 rows per wave and 16 blocks per CU up to 64 K
    // interior rows (129^2-class planes), 2 rows and 32 blocks per CU beyond
    const bool small = (I - 2) * (J - 2) <= 65536;
    int rows_per_wave = small ? 8 : 2, bpc = small ? 16 : 32, nt = 0;
    copy_env_override(rows_per_wave, bpc, nt);
    if (rows_per_wave == 2) return launch_copy<2>(p, q, I, J, K, bpc, nt, f, s);
    if (rows_per_wave == 8) return launch_copy<8>(p, q, I, J, K, bpc, nt, f, s);
    return launch_copy<4>(p, q, I, J, K, bpc, nt, f, s);
}

}  // namespace k
}  // namespace ofl
