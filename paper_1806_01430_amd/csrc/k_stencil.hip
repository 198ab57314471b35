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
// holding a, x, y of three planes in registers, with the next PD planes
// already in flight in a register ring: every element of p is loaded once per
// work item (plus two halo rows and two halo planes), the k neighbours arrive
// through DPP lane shifts, and no LDS is used.  Waves loop over work items
// (grid sized to the resident wave slots, so there is no tail round); the
// four waves of a block take neighbouring j-runs, sharing halo rows in L1.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "dev_common.hpp"
#include "kernels.hpp"

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
};

template <int JR, int PD>
__global__ __launch_bounds__(kThreads) void k_stencil19(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                        double *res_slot, double *partials, unsigned *counter) {
    const int lane = threadIdx.x & (kWave - 1);
    const int gwave = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int J = g.J, K = g.K;
    const size_t plane = (size_t)J * K;
    double acc = 0.0;

    for (int w = gwave; w < g.items; w += nwaves) {
        const int jt = w % g.njt;
        const int rest = w / g.njt;
        const int kt = rest % g.nkt;
        const int ic = rest / g.nkt;
        const int k = kt * kOut + lane;             // lane 0 holds k-1 of the first output
        const bool kin = k < K;
        const bool kout = lane >= 1 && lane <= kOut && k <= K - 2;
        const int jb = 1 + jt * JR;                 // first output row
        const int ib = 1 + ic * g.IC;
        const int ie = min(ib + g.IC, g.I - 1);     // exclusive; ib < ie by construction

        float am[JR], a0[JR], ap[JR], xm[JR], x0[JR], xp[JR], y0[JR], yp[JR];
        float ring[PD][JR + 2];

        auto load = [&](int i, float (&v)[JR + 2]) {
            const float *base = p + (size_t)i * plane + (size_t)(jb - 1) * K + k;
#pragma unroll
            for (int r = 0; r < JR + 2; ++r)
                v[r] = (kin && jb - 1 + r < J) ? base[(size_t)r * K] : 0.0f;
        };
        auto derive = [&](const float (&v)[JR + 2], float (&a)[JR], float (&x)[JR], float (&y)[JR]) {
            float vl[JR + 2], vr[JR + 2];
#pragma unroll
            for (int r = 0; r < JR + 2; ++r) {
                vl[r] = from_left(v[r]);
                vr[r] = from_right(v[r]);
            }
#pragma unroll
            for (int r = 0; r < JR; ++r) {
                a[r] = v[r + 1];
                x[r] = (v[r] + v[r + 2]) + (vl[r + 1] + vr[r + 1]);
                y[r] = (vl[r] + vr[r]) + (vl[r + 2] + vr[r + 2]);
            }
        };

        {
            float raw[JR + 2], ydummy[JR];
            load(ib - 1, raw);
#pragma unroll
            for (int s = 0; s < PD; ++s)
                if (ib + 1 + s <= ie) load(ib + 1 + s, ring[s]);
            derive(raw, am, xm, ydummy);
            load(ib, raw);
            derive(raw, a0, x0, y0);
        }
        for (int i0 = ib; i0 < ie; i0 += PD) {
#pragma unroll
            for (int s = 0; s < PD; ++s) {
                const int i = i0 + s;
                if (i < ie) {
                    derive(ring[s], ap, xp, yp);                    // plane i+1
                    if (i + 1 + PD <= ie) load(i + 1 + PD, ring[s]);
                    float *qrow = q + (size_t)i * plane + (size_t)jb * K + k;
#pragma unroll
                    for (int r = 0; r < JR; ++r) {
                        const float F = (am[r] + ap[r]) + x0[r];
                        const float E = (xm[r] + xp[r]) + y0[r];
                        const float t0 = 0.25f * a0[r];
                        const float t1 = 0.0625f * F;
                        const float t2 = 0.03125f * E;
                        const float v = (t0 + t1) + t2;
                        if (kout && jb + r <= J - 2) {
                            __builtin_nontemporal_store(v, qrow + (size_t)r * K);
                            const double d = (double)v - (double)a0[r];
                            acc = acc + d * d;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < JR; ++r) {
                        am[r] = a0[r];
                        a0[r] = ap[r];
                        xm[r] = x0[r];
                        x0[r] = xp[r];
                        y0[r] = yp[r];
                    }
                }
            }
        }
    }
    reduce_finish(acc, partials, counter, res_slot);
}

// p[i][j][k] = q[i][j][k] on the interior: one wave per row (i, j), 16-byte
// accesses on the aligned middle of the row, single elements at its ends.
__global__ __launch_bounds__(kThreads) void k_copy_interior(float *__restrict__ p, const float *__restrict__ q,
                                                            int I, int J, int K) {
    const int lane = threadIdx.x & (kWave - 1);
    const int gwave = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int rows = (I - 2) * (J - 2);
    for (int row = gwave; row < rows; row += nwaves) {
        const int i = 1 + row / (J - 2), j = 1 + row % (J - 2);
        const size_t base = ((size_t)i * J + j) * K;
        const size_t lo = base + 1, hi = base + K - 1;        // [lo, hi)
        const size_t a0 = (lo + 3) & ~(size_t)3, a1 = hi & ~(size_t)3;
        if (a0 < a1) {
            for (size_t e = a0 + 4 * (size_t)lane; e < a1; e += 4 * kWave)
                *reinterpret_cast<float4 *>(p + e) = *reinterpret_cast<const float4 *>(q + e);
            if (lo + lane < a0) p[lo + lane] = q[lo + lane];
            if (a1 + lane < hi) p[a1 + lane] = q[a1 + lane];
        } else {
            for (size_t e = lo + lane; e < hi; e += kWave) p[e] = q[e];
        }
    }
}

struct Config {
    int JR, PD;
    Geo g;
    unsigned blocks;
};

int resident_blocks_per_cu(int JR, int PD);

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

// Tuning knob: OFL_STENCIL_CFG="JR,PD,IC" overrides the choice (JR in {2,4,8},
// PD in {1,2,3}); used by the tuning sweeps.
bool env_override(int &JR, int &PD, int &IC) {
    const char *s = std::getenv("OFL_STENCIL_CFG");
    if (!s) return false;
    int a, b, c;
    if (std::sscanf(s, "%d,%d,%d", &a, &b, &c) != 3) return false;
    if (!((a == 2 || a == 4 || a == 8) && b >= 1 && b <= 3 && c >= 1)) return false;
    JR = a;
    PD = b;
    IC = c;
    return true;
}

Config choose(int64_t I, int64_t J, int64_t K) {
    Config c;
    const int64_t ni = I - 2, nj = J - 2;
    int JR, PD, IC;
    if (!env_override(JR, PD, IC)) {
        // large grids: long i-runs (halo planes negligible) and deep prefetch;
        // small grids: short runs so that enough work items exist
        const int64_t pts = ni * nj * (K - 2);
        if (pts >= (int64_t)32 << 20) {
            JR = 8;
            PD = 2;
            IC = 32;
        } else {
            JR = 4;
            PD = 2;
            IC = 8;
        }
    }
    if (IC > ni) IC = (int)ni;
    c.JR = JR;
    c.PD = PD;
    c.g.I = (int)I;
    c.g.J = (int)J;
    c.g.K = (int)K;
    c.g.IC = IC;
    c.g.nkt = (int)((K - 2 + kOut - 1) / kOut);
    c.g.njt = (int)((nj + JR - 1) / JR);
    c.g.nic = (int)((ni + IC - 1) / IC);
    c.g.items = c.g.nkt * c.g.njt * c.g.nic;
    const int64_t blocks_needed = ((int64_t)c.g.items + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t slots = (int64_t)cu_count() * resident_blocks_per_cu(JR, PD);
    c.blocks = (unsigned)(blocks_needed < slots ? blocks_needed : slots);
    if (c.blocks < 1) c.blocks = 1;
    return c;
}

template <int JR, int PD>
hipError_t launch_t(const Config &c, const float *p, float *q, double *res_slot, const ReduceScratch &rs,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_stencil19<JR, PD>), dim3(c.blocks), dim3(kThreads), 0, s, p, q, c.g, res_slot,
                       rs.partials, rs.counter);
    return hipGetLastError();
}

template <int JR, int PD>
int occupancy_t() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stencil19<JR, PD>, kThreads, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

int resident_blocks_per_cu(int JR, int PD) {
    static std::once_flag once;
    static int table[3][3];
    std::call_once(once, [] {
        table[0][0] = occupancy_t<2, 1>();
        table[0][1] = occupancy_t<2, 2>();
        table[0][2] = occupancy_t<2, 3>();
        table[1][0] = occupancy_t<4, 1>();
        table[1][1] = occupancy_t<4, 2>();
        table[1][2] = occupancy_t<4, 3>();
        table[2][0] = occupancy_t<8, 1>();
        table[2][1] = occupancy_t<8, 2>();
        table[2][2] = occupancy_t<8, 3>();
    });
    const int r = JR == 2 ? 0 : JR == 4 ? 1 : 2;
    return table[r][PD - 1];
}

}  // namespace

int64_t stencil_partials(int64_t I, int64_t J, int64_t K) {
    if (I < 3 || J < 3 || K < 3) return 1;
    // upper bound over every configuration the launcher may choose: one block
    // per resident slot, at most 2048 threads per CU
    return (int64_t)cu_count() * (2048 / kThreads);
}

hipError_t stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                     const ReduceScratch &rs, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;   // no interior: nothing written, residual unchanged
    if (J * K >= (1ll << 31) || I >= (1ll << 31)) return hipErrorInvalidValue;
    const Config c = choose(I, J, K);
    if ((int64_t)c.blocks > rs.capacity) return hipErrorInvalidValue;
#define OFL_STENCIL_CASE(jr, pd) \
    if (c.JR == jr && c.PD == pd) return launch_t<jr, pd>(c, p, q, res_slot, rs, s);
    OFL_STENCIL_CASE(2, 1) OFL_STENCIL_CASE(2, 2) OFL_STENCIL_CASE(2, 3)
    OFL_STENCIL_CASE(4, 1) OFL_STENCIL_CASE(4, 2) OFL_STENCIL_CASE(4, 3)
    OFL_STENCIL_CASE(8, 1) OFL_STENCIL_CASE(8, 2) OFL_STENCIL_CASE(8, 3)
#undef OFL_STENCIL_CASE
    return hipErrorInvalidValue;
}

hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;
    if ((I - 2) * (J - 2) >= (1ll << 31)) return hipErrorInvalidValue;
    const int64_t rows = (I - 2) * (J - 2);
    int64_t blocks = (rows + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > (int64_t)cu_count() * 16) blocks = (int64_t)cu_count() * 16;
    hipLaunchKernelGGL(k_copy_interior, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, q, (int)I, (int)J, (int)K);
    return hipGetLastError();
}

}  // namespace k
}  // namespace ofl
