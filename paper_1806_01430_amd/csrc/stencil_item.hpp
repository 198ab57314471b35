// Device building blocks of the 19-point sweep and the interior copy, shared
// by the single-grid kernels and the grouped kernels of instance batches.
//
// Sweep definition (centre 1/4, faces 1/16, edges 1/32; FP32, fixed order):
//   per plane m:  a_m = p[m][j][k]
//                 x_m = (p[m][j-1][k] + p[m][j+1][k]) + (p[m][j][k-1] + p[m][j][k+1])
//                 y_m = (p[m][j-1][k-1] + p[m][j-1][k+1]) + (p[m][j+1][k-1] + p[m][j+1][k+1])
//   F = (a_{i-1} + a_{i+1}) + x_i,  E = (x_{i-1} + x_{i+1}) + y_i,
//   q = (0.25 a_i + 0.0625 F) + 0.03125 E,   res += ((double)q - (double)a_i)^2.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.hpp"

namespace ofl {
namespace k {

constexpr int kStencilThreads = 256;
constexpr int kOut = 62;          // output lanes per wave along k
constexpr int kWavesPerBlock = kStencilThreads / kWave;

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

// Offset that the raw-buffer range check always drops (stores are not made,
// loads return zero without a memory access).
constexpr int kOutOfRange = (int)0x80000000u;

// One work item of the sweep.  Item w (k-tile fastest, then j-run, then
// i-run) covers rows jb .. jb+JR-1, the 62 output columns of k-tile kt and
// planes [ib, ie).  Plane sets P[0..2] hold a, x, y of planes i-1, i, i+1
// with roles rotating every step (the i-loop is unrolled by three, so no
// register moves); the ring holds the next three raw planes in flight.  Loads
// are raw buffer loads; the loop body branches only on wave-uniform values:
// loads of rows beyond the work item are clamped into the array (their values
// feed no stored output), and a refill past the run's last plane or a store
// that must not happen gets an offset past num_records, which the raw-buffer
// range check drops (a load so dropped returns zeros).  Returns acc plus
// the lane's squared differences.
// Cache policy of the buffer accesses: 0 = default, kNonTemporal = streaming
// (the "nt" bit: the line is not kept for reuse).
constexpr int kNonTemporal = 2;

template <int JR, int STORE_POLICY = 0>
__device__ inline double stencil_item(__amdgpu_buffer_rsrc_t rp, __amdgpu_buffer_rsrc_t rq, const Geo &g, int w,
                                      int lane, double acc) {
    constexpr int R = JR + 2;
    const int J = g.J, K = g.K;
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
        for (int r = 0; r < R; ++r)
            v[r] = buf_load(rp, i < 0 ? kOutOfRange : ((ii * J + min(jb - 1 + r, J - 1)) * K) * 4 + kld);
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
        // past the run's last plane there is nothing left to fetch: the
        // refill then reads past num_records (no memory access, zeros)
        __builtin_amdgcn_sched_barrier(0);
        load(i + 4 <= ie ? i + 4 : -1, ring[s]);
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
                                                  ok ? ((i * J + jb + r) * K) * 4 + voff : kOutOfRange, 0,
                                                  STORE_POLICY);
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
    return acc;
}

// The same sweep with two consecutive k per lane: a wave covers 128 k of
// each row with one 8-byte load (the lines a row window straddles are
// fetched once per 126 outputs instead of once per 62) and produces the 126
// columns k0+1 .. k0+126 (lane 0's first and lane 63's second value only
// supply neighbours).  Per point the arithmetic is that of stencil_item, in
// the same order, so the field is bit-identical; only the order in which the
// residual terms are summed differs.
constexpr int kOutW = 126;

typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ inline f32x2 buf_load2(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <int JR, int STORE_POLICY = 0>
__device__ inline double stencil_item_w(__amdgpu_buffer_rsrc_t rp, __amdgpu_buffer_rsrc_t rq, const Geo &g, int w,
                                        int lane, double acc) {
    constexpr int R = JR + 2;
    const int J = g.J, K = g.K;
    const int kt = w % g.nkt;
    const int rest = w / g.nkt;
    const int jt = rest % g.njt;
    const int ic = rest / g.njt;
    const int k = kt * kOutW + 2 * lane;        // this lane's first column
    // the 8-byte window stays inside the row: a lane whose first column is
    // the row's last reads the window one column earlier and takes its second
    // value; lanes past the row read anything (their values feed no output)
    const bool shifted = k > K - 2;
    const int kld = min(k, K - 2) * 4;
    const bool out0 = lane >= 1 && k <= K - 2;
    const bool out1 = lane <= 62 && k + 1 <= K - 2;
    const int voff0 = k * 4, voff1 = voff0 + 4;
    const int jb = 1 + jt * JR;
    const int ib = 1 + ic * g.IC;
    const int ie = min(ib + g.IC, g.I - 1);
    const int jlast = J - 2 - jb;

    f32x2 Pa[3][JR], Px[3][JR], Py[3][JR];
    f32x2 ring[3][R];

    auto load = [&](int i, f32x2 (&v)[R]) {
        const int ii = min(i, g.I - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const f32x2 t = buf_load2(rp, ((ii * J + min(jb - 1 + r, J - 1)) * K) * 4 + kld);
            v[r] = shifted ? f32x2{t.y, t.y} : t;
        }
    };
    auto derive = [&](const f32x2 (&v)[R], f32x2 (&a)[JR], f32x2 (&x)[JR], f32x2 (&y)[JR]) {
        f32x2 h[R];                             // p[j][k-1] + p[j][k+1] per row and column
#pragma unroll
        for (int r = 0; r < R; ++r) {
            h[r].x = from_left(v[r].y) + v[r].y;
            h[r].y = v[r].x + from_right(v[r].x);
        }
#pragma unroll
        for (int r = 0; r < JR; ++r) {
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
    auto step = [&](auto S, int i) {
        constexpr int s = decltype(S)::value;
        constexpr int m = s, c = (s + 1) % 3, n = (s + 2) % 3;
        __builtin_amdgcn_sched_barrier(0);
        derive(ring[s], Pa[n], Px[n], Py[n]);
        __builtin_amdgcn_sched_barrier(0);
        load(min(i + 4, ie), ring[s]);
        const bool plane_ok = i < ie;
#pragma unroll
        for (int r = 0; r < JR; ++r) {
            const float v0 = point(Pa[m][r].x, Pa[n][r].x, Pa[c][r].x, Px[m][r].x, Px[n][r].x, Px[c][r].x, Py[c][r].x);
            const float v1 = point(Pa[m][r].y, Pa[n][r].y, Pa[c][r].y, Px[m][r].y, Px[n][r].y, Px[c][r].y, Py[c][r].y);
            const bool row_ok = plane_ok && r <= jlast;
            const bool ok0 = out0 && row_ok, ok1 = out1 && row_ok;
            const int base = ((i * J + jb + r) * K) * 4;
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v0), rq,
                                                  ok0 ? base + voff0 : kOutOfRange, 0, STORE_POLICY);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v1), rq,
                                                  ok1 ? base + voff1 : kOutOfRange, 0, STORE_POLICY);
            const double d0 = (double)v0 - (double)Pa[c][r].x;
            const double d1 = (double)v1 - (double)Pa[c][r].y;
            acc = __builtin_fma(ok0 ? d0 : 0.0, d0, acc);
            acc = __builtin_fma(ok1 ? d1 : 0.0, d1, acc);
        }
    };

    {
        f32x2 r0[R], r1[R];
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
    return acc;
}

// Columns per wave in the band form (two per lane), and DPP wave shifts
// whose lane without a source keeps `edge` (the band form's halo columns).
constexpr int kOutV = 128;

__device__ inline float from_left_or(float v, float edge) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ inline float from_right_or(float v, float edge) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xF, 0xF, false));
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Rows row0 .. row0+ROWS-1 (of the (I-2)(J-2) interior rows (i, j)) of the
// interior copy p = q.  Each row splits into a head [lo, a0) and a tail
// [a1, hi) of at most three elements and a 16-byte aligned middle [a0, a1);
// a pass moves up to 64 middle groups of every row plus the heads and tails.
// Raw buffer accesses without branches: every load reads a valid element
// (element 0 when the lane has nothing to move), so all loads of a pass
// overlap, and a store that must not happen carries an offset past
// num_records, which the range check drops.
constexpr int kRows = 4;   // rows per work unit of the grouped copy

template <int ROWS = kRows, int POLICY = 0>
__device__ inline void copy_rows(__amdgpu_buffer_rsrc_t rp, __amdgpu_buffer_rsrc_t rq, int J, int K, int rows,
                                 int row0, int lane) {
    const int passes = ((K - 2) / 4 + kWave) / kWave;   // >= ceil(groups / 64), groups <= (K-2)/4
    int lo[ROWS], a0[ROWS], a1[ROWS], hi[ROWS];
    bool live[ROWS];
#pragma unroll
    for (int t = 0; t < ROWS; ++t) {
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
        __attribute__((ext_vector_type(4))) unsigned mid[ROWS];
        unsigned hd[ROWS], tl[ROWS];
        int om[ROWS], oh[ROWS], ot[ROWS];
#pragma unroll
        for (int t = 0; t < ROWS; ++t) {
            const int em = a0[t] + 4 * (pass * kWave + lane);
            const int eh = lo[t] + lane, et = a1[t] + lane;
            om[t] = (live[t] && em < a1[t]) ? em * 4 : -1;
            oh[t] = (live[t] && pass == 0 && eh < a0[t] && eh < hi[t]) ? eh * 4 : -1;
            ot[t] = (live[t] && pass == 0 && et < hi[t] && et >= a0[t]) ? et * 4 : -1;
            mid[t] = __builtin_amdgcn_raw_buffer_load_b128(rq, om[t] < 0 ? 0 : om[t], 0, POLICY);
            hd[t] = __builtin_amdgcn_raw_buffer_load_b32(rq, oh[t] < 0 ? 0 : oh[t], 0, POLICY);
            tl[t] = __builtin_amdgcn_raw_buffer_load_b32(rq, ot[t] < 0 ? 0 : ot[t], 0, POLICY);
        }
#pragma unroll
        for (int t = 0; t < ROWS; ++t) {
            __builtin_amdgcn_raw_buffer_store_b128(mid[t], rp, om[t] < 0 ? kOutOfRange : om[t], 0, POLICY);
            __builtin_amdgcn_raw_buffer_store_b32(hd[t], rp, oh[t] < 0 ? kOutOfRange : oh[t], 0, POLICY);
            __builtin_amdgcn_raw_buffer_store_b32(tl[t], rp, ot[t] < 0 ? kOutOfRange : ot[t], 0, POLICY);
        }
    }
}

}  // namespace k
}  // namespace ofl
