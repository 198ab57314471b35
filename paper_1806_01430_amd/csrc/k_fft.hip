// The FFT function block: the GPU implementation swapped in for an FFT
// library call (the analysis of Sec. 3.2, steps 1-2 and 1-3, finds FFT
// library calls beside loop statements as offloadable parts).  Each row of n
// complex values (real and imaginary parts interleaved, n a power of two) is
// replaced by its forward DFT
//   X[k] = sum_j x[j] exp(-2 pi i j k / n),
// computed by radix-2 self-sorting (Stockham) passes: in pass s (half-size
// ns = 2^s) butterfly j pairs a[j] and a[j + n/2], multiplies the second by
// the twiddle w(k n / (2 ns)) = exp(-2 pi i k / (2 ns)) with k = j mod ns,
// and writes the sum to position 2 (j - k) + k and the difference ns further
// on; after log2 n passes the spectrum is in natural order.
//
// Two passes run back to back in registers: pass s's butterflies g and
// g + n/4 produce exactly the four inputs of pass s+1's butterflies
// (g div ns) 2 ns + k and that + ns, so one thread takes a[g + m n/4],
// m = 0..3, does the four butterflies and stores four outputs at
// (g div ns) 4 ns + k + m ns.  The butterflies and their operands are those
// of the plain radix-2 passes, so the result has the same bits as the CPU
// form (host_nests.cpp), at half the LDS round trips and barriers.  The
// first pair reads the row from HBM, the last writes it back; odd log2 n
// begins with one plain pass.  Short rows share a block (below); rows of
// 256 to 4096 points take the register form further down.
//
// The inverse transform, x[j] = (1/n) sum_k X[k] exp(+2 pi i j k / n), is
// the forward one applied to the conjugated row, conjugated again and
// scaled by 1/n (exact: a power of two): the kernels conjugate as they read
// the row and conjugate and scale as they write it, so the passes, twiddles
// and bits are those of the forward transform (and of the CPU form, which
// does the same).
#include <algorithm>

#include "fft_limits.hpp"
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kFftThreads = 256;

__device__ inline float2 cmul(float2 v, float2 t) {
    return make_float2(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
}
// a value read from the row (conjugated for the inverse) and one written to
// it (conjugated and scaled by 1/n for the inverse)
__device__ inline float2 rd(float2 v, bool inv) { return inv ? make_float2(v.x, -v.y) : v; }
__device__ inline float2 wr(float2 v, bool inv, float sc) { return inv ? make_float2(v.x * sc, -v.y * sc) : v; }

// One plain radix-2 pass (half-size ns): src -> dst, by threads t of T.
// `put` = false skips the stores (a row past the end of the array); ci / co:
// src / dst is the row of an inverse transform (sc = 1/n).
__device__ inline void pass1(const float2 *__restrict__ src, float2 *__restrict__ dst, const float2 *w, int n,
                             int ns, int st, int t, int T, bool put, bool ci, bool co, float sc) {
    const int half = n >> 1;
    for (int j = t; j < half; j += T) {
        const int k = j & (ns - 1), o = ((j - k) << 1) + k;
        const float2 u = rd(src[j], ci), v = cmul(rd(src[j + half], ci), w[k * st]);
        if (put) {
            dst[o] = wr(make_float2(u.x + v.x, u.y + v.y), co, sc);
            dst[o + ns] = wr(make_float2(u.x - v.x, u.y - v.y), co, sc);
        }
    }
}

// Passes s and s + 1 (half-sizes ns and 2 ns): src -> dst, by threads t of T.
__device__ inline void pass2(const float2 *__restrict__ src, float2 *__restrict__ dst, const float2 *w, int n,
                             int ns, int t, int T, bool put, bool ci, bool co, float sc) {
    const int q4 = n >> 2, st = n / (2 * ns), st2 = st >> 1;
    for (int g = t; g < q4; g += T) {
        const int k = g & (ns - 1), base = ((g - k) << 2) + k;
        const float2 x0 = rd(src[g], ci), x1 = rd(src[g + q4], ci), x2 = rd(src[g + 2 * q4], ci),
                     x3 = rd(src[g + 3 * q4], ci);
        const float2 tw1 = w[k * st];
        const float2 m2 = cmul(x2, tw1), m3 = cmul(x3, tw1);
        const float2 u0 = make_float2(x0.x + m2.x, x0.y + m2.y), v0 = make_float2(x0.x - m2.x, x0.y - m2.y);
        const float2 u1 = make_float2(x1.x + m3.x, x1.y + m3.y), v1 = make_float2(x1.x - m3.x, x1.y - m3.y);
        const float2 p = cmul(u1, w[k * st2]), r = cmul(v1, w[(k + ns) * st2]);
        if (put) {
            dst[base] = wr(make_float2(u0.x + p.x, u0.y + p.y), co, sc);
            dst[base + 2 * ns] = wr(make_float2(u0.x - p.x, u0.y - p.y), co, sc);
            dst[base + ns] = wr(make_float2(v0.x + r.x, v0.y + r.y), co, sc);
            dst[base + 3 * ns] = wr(make_float2(v0.x - r.x, v0.y - r.y), co, sc);
        }
    }
}

// Rows of 2 to 128 points: a 256-thread block takes 256 / T rows, T =
// max(1, n/4) threads per row (one pass-pair group each), with two LDS
// buffers per row and one twiddle table for the block.  Threads of a row
// past the end read row 0 and store nothing; every thread reaches every
// barrier.
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(float2 *__restrict__ x, const float2 *__restrict__ tw,
                                                          int64_t rows, int n, int logn, bool inv) {
    extern __shared__ float2 lds[];
    const int T = n >= 4 ? n >> 2 : 1, rb = kFftThreads / T;
    const int sub = threadIdx.x / T, t = threadIdx.x - sub * T;
    const int64_t row = (int64_t)blockIdx.x * rb + sub;
    const bool valid = row < rows;
    float2 *w = lds, *a = lds + (n >> 1) + 2 * sub * n, *b = a + n;
    float2 *xr = x + (valid ? row : 0) * n;
    const int half = n >> 1;
    for (int m = threadIdx.x; m < half; m += blockDim.x) w[m] = tw[m];
    __syncthreads();
    const float sc = 1.0f / (float)n;
    int s = 0;
    const float2 *src = xr;
    if (logn & 1) {
        // one plain pass first; with n = 2 it is the whole transform
        pass1(xr, logn == 1 ? xr : a, w, n, 1, half, t, T, logn != 1 || valid, inv, inv && logn == 1, sc);
        if (logn == 1) return;
        __syncthreads();
        src = a;
        s = 1;
    }
    float2 *spare = (src == a) ? b : a;
    for (; s < logn; s += 2) {
        const bool last = s + 2 >= logn;
        float2 *dst = last ? xr : spare;
        pass2(src, dst, w, n, 1 << s, t, T, !last || valid, inv && src == xr, inv && last, sc);
        if (last) break;
        __syncthreads();
        spare = const_cast<float2 *>(src == xr ? b : src);
        src = dst;
    }
}

// Rows of 1024, 2048 and 4096 points: sixteen points per thread in registers,
// so four passes run per register stage (passes s..s+3 on the group
// a[g + m n/16], m = 0..15); stages at s = 0, 4 and 8 (the last of 2, 3 or 4
// passes), the
// first reading the row from HBM, the last writing it, with two LDS
// exchanges between them.  Within a stage the element at register index
// i = (m' << t) | d after t passes pairs with the one whose top bit differs;
// the pass's twiddle index is ((d << s) | k) n / 2^(s+t+1) with k = g mod 2^s,
// the d bits being the sum/difference choices of the passes done so far
// (latest highest).  After the stage register D goes to position
// (g - k) 2^r + k + D 2^s: the same butterflies on the same values as the
// plain passes.  LDS positions are padded by one slot per sixteen, which
// keeps the strided stores of the first two stages at two lanes per bank.
__device__ inline int fft_pad(int p) { return p + (p >> 4); }

template <int R, int S, int LOGN>
__device__ inline void fft_stage(float2 (&v)[1 << R], const float2 *__restrict__ tw, int k) {
    constexpr int R2 = 1 << R, H = R2 >> 1, N = 1 << LOGN;
#pragma unroll
    for (int t = 0; t < R; ++t) {
        float2 nv[R2];
#pragma unroll
        for (int rest = 0; rest < H; ++rest) {
            const int dbits = rest & ((1 << t) - 1), mlow = rest >> t;
            const float2 w = tw[((dbits << S) | k) * (N >> (S + t + 1))];
            const float2 a = v[rest], b = cmul(v[rest + H], w);
            nv[(mlow << (t + 1)) | dbits] = make_float2(a.x + b.x, a.y + b.y);
            nv[(mlow << (t + 1)) | (1 << t) | dbits] = make_float2(a.x - b.x, a.y - b.y);
        }
#pragma unroll
        for (int i = 0; i < R2; ++i) v[i] = nv[i];
    }
}

// The transform of one row whose sixteen first-stage points per thread are
// already in registers; ends with the row written back.
template <int LOGN, bool INV>
__device__ inline void fft_row16(float2 (&v)[16], float2 *__restrict__ xr, float2 *lds,
                                 const float2 *__restrict__ tw) {
    constexpr int N = 1 << LOGN, G16 = N / 16, R3 = LOGN - 8, G3 = N >> R3;
    const int tid = threadIdx.x;   // one 16-point group per thread in the first two stages
    fft_stage<4, 0, LOGN>(v, tw, 0);
#pragma unroll
    for (int d = 0; d < 16; ++d) lds[fft_pad((tid << 4) + d)] = v[d];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = lds[fft_pad(tid + m * G16)];
    __syncthreads();   // every read of this stage before its stores
    const int k = tid & 15;
    fft_stage<4, 4, LOGN>(v, tw, k);
#pragma unroll
    for (int d = 0; d < 16; ++d) lds[fft_pad(((tid - k) << 4) + k + (d << 4))] = v[d];
    __syncthreads();
    for (int g = tid; g < G3; g += G16) {   // G3 = 256 groups of 2^R3 points (16 at n = 4096); k = g
        float2 w[1 << R3];
#pragma unroll
        for (int m = 0; m < (1 << R3); ++m) w[m] = lds[fft_pad(g + m * G3)];
        fft_stage<R3, 8, LOGN>(w, tw, g);
#pragma unroll
        for (int d = 0; d < (1 << R3); ++d) xr[g + (d << 8)] = wr(w[d], INV, 1.0f / N);
    }
}

// Two rows per block: both rows' loads are issued first, so the second row
// streams in from HBM while the first is transformed.
constexpr int kFftRowsPerBlock = 2;

template <int LOGN, bool INV>
__global__ __launch_bounds__((1 << LOGN) / 16) void k_fft_rows16(float2 *__restrict__ x,
                                                                   const float2 *__restrict__ tw, int64_t rows) {
    constexpr int N = 1 << LOGN, G16 = N / 16;
    __shared__ float2 lds[N + N / 16];
    const int64_t r0 = (int64_t)blockIdx.x * kFftRowsPerBlock;
    const bool two = r0 + 1 < rows;
    float2 *x0 = x + r0 * N, *x1 = x0 + N;
    const int tid = threadIdx.x;
    float2 v0[16], v1[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) v0[m] = rd(x0[tid + m * G16], INV);
    if (two) {
#pragma unroll
        for (int m = 0; m < 16; ++m) v1[m] = rd(x1[tid + m * G16], INV);
    }
    fft_row16<LOGN, INV>(v0, x0, lds, tw);
    if (two) {
        __syncthreads();   // the first row's last LDS reads before the second row's stores
        fft_row16<LOGN, INV>(v1, x1, lds, tw);
    }
}

// Rows of 256 and 512 points: the same register form with T = n/16 threads
// per row and 64 / T rows per one-wave block, each row in its own LDS area;
// at 256 points the second stage is the last and writes the row back.
// Threads of a row past the end read row 0 and store nothing.
template <int LOGN, bool INV>
__global__ __launch_bounds__(64) void k_fft_rows16s(float2 *__restrict__ x, const float2 *__restrict__ tw,
                                                     int64_t rows) {
    constexpr int N = 1 << LOGN, T = N / 16, RW = 64 / T, R3 = LOGN - 8, P = N + N / 16;
    __shared__ float2 lds_all[RW * P];
    const int sub = threadIdx.x / T, tid = threadIdx.x - sub * T;
    const int64_t row = (int64_t)blockIdx.x * RW + sub;
    const bool valid = row < rows;
    float2 *xr = x + (valid ? row : 0) * N;
    float2 *lds = lds_all + sub * P;
    float2 v[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = rd(xr[tid + m * T], INV);
    fft_stage<4, 0, LOGN>(v, tw, 0);
#pragma unroll
    for (int d = 0; d < 16; ++d) lds[fft_pad((tid << 4) + d)] = v[d];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = lds[fft_pad(tid + m * T)];
    const int k = tid & 15;
    fft_stage<4, 4, LOGN>(v, tw, k);
    if constexpr (R3 == 0) {
        if (valid) {
#pragma unroll
            for (int d = 0; d < 16; ++d) xr[((tid - k) << 4) + k + (d << 4)] = wr(v[d], INV, 1.0f / N);
        }
    } else {
        __syncthreads();   // every read of this stage before its stores
#pragma unroll
        for (int d = 0; d < 16; ++d) lds[fft_pad(((tid - k) << 4) + k + (d << 4))] = v[d];
        __syncthreads();
        constexpr int G3 = N >> R3;   // 256 groups of 2^R3 points; k = g
        for (int g = tid; g < G3; g += T) {
            float2 w[1 << R3];
#pragma unroll
            for (int m = 0; m < (1 << R3); ++m) w[m] = lds[fft_pad(g + m * G3)];
            fft_stage<R3, 8, LOGN>(w, tw, g);
            if (valid) {
#pragma unroll
                for (int d = 0; d < (1 << R3); ++d) xr[g + (d << 8)] = wr(w[d], INV, 1.0f / N);
            }
        }
    }
}

// Real rows: the n real values of a row read as m = n/2 complex values z
// (z[j] = x[2j] + i x[2j+1]) have the transform Z (the complex kernels
// above); the spectrum of the real row follows from pairs of Z,
//   X[k] = E[k] + w^k O[k],  E[k] = (Z[k] + conj Z[m-k]) / 2,
//   O[k] = (Z[k] - conj Z[m-k]) / 2i,  w = exp(-2 pi i / n),
// with X[0] = Z0.x + Z0.y and X[m] = Z0.x - Z0.y real.  One thread per pair
// (k, m - k), k = 0 .. m/2, writes both bins in place (packed: X[0] and X[m]
// in the row's first two floats).  The CPU form does the same operations.
__device__ inline float2 rfft_bin(float2 a, float2 b, float2 t) {
    const float2 e = make_float2((a.x + b.x) * 0.5f, (a.y - b.y) * 0.5f);
    const float2 d = make_float2((a.x - b.x) * 0.5f, (a.y + b.y) * 0.5f);
    const float2 p = cmul(make_float2(d.y, -d.x), t);
    return make_float2(e.x + p.x, e.y + p.y);
}

__global__ __launch_bounds__(kFftThreads) void k_rfft_unpack(float2 *__restrict__ x, const float2 *__restrict__ tw,
                                                             int64_t rows, int m) {
    const int64_t pairs = m / 2 + 1, total = rows * pairs;
    for (int64_t u = blockIdx.x * (int64_t)kFftThreads + threadIdx.x; u < total;
         u += (int64_t)gridDim.x * kFftThreads) {
        const int64_t r = u / pairs;
        const int k = (int)(u - r * pairs);
        float2 *z = x + r * m;
        if (k == 0) {
            const float2 z0 = z[0];
            z[0] = make_float2(z0.x + z0.y, z0.x - z0.y);
        } else {
            const float2 a = z[k], b = z[m - k];
            const float2 yk = rfft_bin(a, b, tw[k]);
            if (2 * k != m) z[m - k] = rfft_bin(b, a, tw[m - k]);
            z[k] = yk;
        }
    }
}

// The inverse: from the packed spectrum back to Z of the half-length
// transform, per bin pair: E = (X[k] + conj X[m-k]) / 2 and
// O = (X[k] - conj X[m-k]) / 2 conj(w^k), Z[k] = E + i O (k = 0: E and O
// are the half-sum and half-difference of X0 and X(m)); then the inverse
// complex transform of m values, scaled by 1/m, gives z, i.e. the real row.
__device__ inline float2 irfft_bin(float2 a, float2 b, float2 t) {
    const float2 e = make_float2((a.x + b.x) * 0.5f, (a.y - b.y) * 0.5f);
    const float2 d = make_float2((a.x - b.x) * 0.5f, (a.y + b.y) * 0.5f);
    const float2 o = cmul(d, make_float2(t.x, -t.y));
    return make_float2(e.x - o.y, e.y + o.x);
}

__global__ __launch_bounds__(kFftThreads) void k_irfft_pack(float2 *__restrict__ x, const float2 *__restrict__ tw,
                                                            int64_t rows, int m) {
    const int64_t pairs = m / 2 + 1, total = rows * pairs;
    for (int64_t u = blockIdx.x * (int64_t)kFftThreads + threadIdx.x; u < total;
         u += (int64_t)gridDim.x * kFftThreads) {
        const int64_t r = u / pairs;
        const int k = (int)(u - r * pairs);
        float2 *z = x + r * m;
        if (k == 0) {
            const float2 p = z[0];   // (X0, X(m))
            z[0] = make_float2((p.x + p.y) * 0.5f, (p.x - p.y) * 0.5f);
        } else {
            const float2 a = z[k], b = z[m - k];
            const float2 zk = irfft_bin(a, b, tw[k]);
            if (2 * k != m) z[m - k] = irfft_bin(b, a, tw[m - k]);
            z[k] = zk;
        }
    }
}

template <bool INV>
hipError_t fft_rows_t(float2 *x2, const float2 *t2, int64_t rows, int64_t n, hipStream_t s) {
    const dim3 pairs((unsigned)((rows + kFftRowsPerBlock - 1) / kFftRowsPerBlock));
    if (n == 1024) return launch(k_fft_rows16<10, INV>, pairs, dim3(64), 0, s, x2, t2, rows);
    if (n == 2048) return launch(k_fft_rows16<11, INV>, pairs, dim3(128), 0, s, x2, t2, rows);
    if (n == 4096) return launch(k_fft_rows16<12, INV>, pairs, dim3(256), 0, s, x2, t2, rows);
    if (n == 256)
        return launch(k_fft_rows16s<8, INV>, dim3((unsigned)((rows + 3) / 4)), dim3(64), 0, s, x2, t2, rows);
    if (n == 512)
        return launch(k_fft_rows16s<9, INV>, dim3((unsigned)((rows + 1) / 2)), dim3(64), 0, s, x2, t2, rows);
    if (n > 128) return hipErrorInvalidValue;
    int logn = 0;
    while ((1ll << logn) < n) ++logn;
    const int64_t rb = kFftThreads / (n >= 4 ? n / 4 : 1);
    const uint32_t lds_bytes = (uint32_t)((rb * 2 * n + n / 2) * sizeof(float2));
    return launch(k_fft_rows, dim3((unsigned)((rows + rb - 1) / rb)), dim3(kFftThreads), lds_bytes, s, x2, t2, rows,
                  (int)n, logn, INV);
}

}  // namespace

hipError_t rfft_rows(float *x, int64_t rows, int64_t n, const float *tw, bool inverse, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (n < 2 || n > kFftMaxPoints || (n & (n - 1)) != 0 || rows > 0x7FFFFFFF || tw == nullptr)
        return hipErrorInvalidValue;
    const int64_t total = rows * (n / 4 + 1);
    const int64_t blocks = std::min<int64_t>((total + kFftThreads - 1) / kFftThreads, 65536);
    float2 *x2 = reinterpret_cast<float2 *>(x);
    const float2 *t2 = reinterpret_cast<const float2 *>(tw) + (n / 2 - 1);   // exp(-2 pi i k / n), k < n/2
    if (inverse) {
        hipError_t e = launch(k_irfft_pack, dim3((unsigned)blocks), dim3(kFftThreads), 0, s, x2, t2, rows, (int)(n / 2));
        if (e != hipSuccess) return e;
        return fft_rows(x, rows, n / 2, tw, true, s);
    }
    hipError_t e = fft_rows(x, rows, n / 2, tw, false, s);
    if (e != hipSuccess) return e;
    return launch(k_rfft_unpack, dim3((unsigned)blocks), dim3(kFftThreads), 0, s, x2, t2, rows, (int)(n / 2));
}

hipError_t fft_rows(float *x, int64_t rows, int64_t n, const float *tw, bool inverse, hipStream_t s) {
    if (rows <= 0 || n <= 1) return hipSuccess;   // a 1-point transform (either way) is the identity
    if (n > kFftMaxPoints || (n & (n - 1)) != 0 || rows > 0x7FFFFFFF || tw == nullptr) return hipErrorInvalidValue;
    const float2 *t2 = reinterpret_cast<const float2 *>(tw) + (n / 2 - 1);   // this length's table
    float2 *x2 = reinterpret_cast<float2 *>(x);
    return inverse ? fft_rows_t<true>(x2, t2, rows, n, s) : fft_rows_t<false>(x2, t2, rows, n, s);
}

}  // namespace k
}  // namespace ofl
