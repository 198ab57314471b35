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
// Mapping (gfx950, wave64): a wave owns 64 consecutive k (lanes 1..62 produce
// outputs, lanes 0 and 63 only supply the k-1 / k+1 neighbours), JR
// consecutive rows j, and a run of IC planes along i.  It marches along i
// holding a, x, y of three planes in registers: every element of p is loaded
// once per wave (plus the two halo rows and two halo planes), the k
// neighbours arrive through DPP lane shifts, and no LDS is used.  Four waves
// of a block take four consecutive j-runs so that their halo rows are shared
// in the CU's L1.  The next plane is prefetched one step ahead.
#include <hip/hip_runtime.h>

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
    int IC;         // planes per wave
    int nkt, njt, njg;
};

template <int JR>
__global__ __launch_bounds__(kThreads) void k_stencil19(const float *__restrict__ p, float *__restrict__ q, Geo g,
                                                        double *res_slot, double *partials, unsigned *counter) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    int b = blockIdx.x;
    const int kt = b % g.nkt;
    b /= g.nkt;
    const int jg = b % g.njg;
    const int ic = b / g.njg;
    const int jt = jg * kWavesPerBlock + wave;
    double acc = 0.0;

    if (jt < g.njt) {
        const int J = g.J, K = g.K;
        const int k = kt * kOut + lane;             // lane 0 holds k-1 of the first output
        const bool kin = k < K;
        const bool kout = lane >= 1 && lane <= kOut && k <= K - 2;
        const int jb = 1 + jt * JR;                 // first output row
        const int ib = 1 + ic * g.IC;
        const int ie = min(ib + g.IC, g.I - 1);     // exclusive
        const size_t plane = (size_t)J * K;

        float am[JR], a0[JR], ap[JR], xm[JR], x0[JR], xp[JR], y0[JR], yp[JR];
        float nxt[JR + 2];

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

        if (ib < ie) {
            float raw[JR + 2], ydummy[JR];
            load(ib - 1, raw);
            derive(raw, am, xm, ydummy);
            load(ib, raw);
            derive(raw, a0, x0, y0);
            load(ib + 1, nxt);
            for (int i = ib; i < ie; ++i) {
                derive(nxt, ap, xp, yp);
                if (i + 2 <= ie) load(i + 2, nxt);
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
                        qrow[(size_t)r * K] = v;
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
    reduce_finish(acc, partials, counter, res_slot);
}

__global__ __launch_bounds__(kThreads) void k_copy_interior(float *__restrict__ p, const float *__restrict__ q,
                                                            int J, int K) {
    const int k = 1 + blockIdx.x * kThreads + threadIdx.x;
    const int j = 1 + blockIdx.y;
    const int i = 1 + blockIdx.z;
    if (k < K - 1) {
        const size_t e = ((size_t)i * J + j) * K + k;
        p[e] = q[e];
    }
}

// Choice of rows per wave and planes per wave: enough waves to fill 256 CUs
// (about 16 per CU) while keeping the i-runs long enough that the two halo
// planes stay a small overhead.
struct Config {
    int JR;
    Geo g;
    unsigned blocks;
};

Config choose(int64_t I, int64_t J, int64_t K) {
    Config c;
    const int64_t interior_j = J - 2, interior_i = I - 2;
    c.JR = (interior_j * (K - 2) >= 256 * 1024) ? 8 : 4;
    c.g.I = (int)I;
    c.g.J = (int)J;
    c.g.K = (int)K;
    c.g.nkt = (int)((K - 2 + kOut - 1) / kOut);
    c.g.njt = (int)((interior_j + c.JR - 1) / c.JR);
    c.g.njg = (c.g.njt + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t waves_per_chunk = (int64_t)c.g.nkt * c.g.njg * kWavesPerBlock;
    const int64_t target = 4096;
    int64_t nic = (target + waves_per_chunk - 1) / waves_per_chunk;
    if (nic < 1) nic = 1;
    if (nic > interior_i) nic = interior_i;
    int64_t IC = (interior_i + nic - 1) / nic;
    if (IC < 1) IC = 1;
    nic = (interior_i + IC - 1) / IC;
    c.g.IC = (int)IC;
    c.blocks = (unsigned)((int64_t)c.g.nkt * c.g.njg * nic);
    return c;
}

}  // namespace

int64_t stencil_partials(int64_t I, int64_t J, int64_t K) {
    if (I < 3 || J < 3 || K < 3) return 1;
    return choose(I, J, K).blocks;
}

hipError_t stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                     const ReduceScratch &rs, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;   // no interior: nothing written, residual unchanged
    const Config c = choose(I, J, K);
    if ((int64_t)c.blocks > rs.capacity) return hipErrorInvalidValue;
    if (c.JR == 8)
        hipLaunchKernelGGL(k_stencil19<8>, dim3(c.blocks), dim3(kThreads), 0, s, p, q, c.g, res_slot, rs.partials,
                           rs.counter);
    else
        hipLaunchKernelGGL(k_stencil19<4>, dim3(c.blocks), dim3(kThreads), 0, s, p, q, c.g, res_slot, rs.partials,
                           rs.counter);
    return hipGetLastError();
}

hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s) {
    if (I < 3 || J < 3 || K < 3) return hipSuccess;
    dim3 grid((unsigned)((K - 2 + kThreads - 1) / kThreads), (unsigned)(J - 2), (unsigned)(I - 2));
    if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_interior, grid, dim3(kThreads), 0, s, p, q, (int)J, (int)K);
    return hipGetLastError();
}

}  // namespace k
}  // namespace ofl
