// The FFT function block: the GPU implementation swapped in for an FFT
// library call (the analysis of Sec. 3.2, steps 1-2 and 1-3, finds FFT
// library calls beside loop statements as offloadable parts).  Each row of n complex values (real and imaginary
// parts interleaved, n a power of two) is replaced by its forward DFT
//   X[k] = sum_j x[j] exp(-2 pi i j k / n),
// computed by radix-2 self-sorting (Stockham) passes: in pass s (half-size
// ns = 2^s) butterfly j pairs a[j] and a[j + n/2], scales the second by the
// twiddle exp(-2 pi i k / (2 ns)) with k = j mod ns, and writes the sum and
// difference to positions (j - k) * 2 + k and that + ns of the other buffer;
// after log2 n passes the spectrum is in natural order.
//
// One block per row: the row, a second buffer and the n/2 twiddles
// exp(-2 pi i m / n) (computed in double, rounded once) live in LDS, so a row
// is read from HBM once and written once; 40 KB of LDS at n = 2048.
#include "kernels.hpp"
#include "launch.hpp"

namespace ofl {
namespace k {

namespace {

constexpr int kFftMaxPoints = 2048;
constexpr double kTwoPi = 6.283185307179586;   // 2 pi rounded to double

__global__ __launch_bounds__(256) void k_fft_rows(float2 *__restrict__ x, int n) {
    extern __shared__ float2 lds[];
    const int half = n >> 1;
    float2 *a = lds, *b = lds + n, *w = lds + 2 * n;
    float2 *xr = x + (int64_t)blockIdx.x * n;
    for (int m = threadIdx.x; m < half; m += blockDim.x) {
        const double th = kTwoPi * (double)m / (double)n;
        w[m] = make_float2((float)cos(th), (float)-sin(th));
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) a[e] = xr[e];
    __syncthreads();
    for (int ns = 1, st = half; ns < n; ns <<= 1, st >>= 1) {
        for (int j = threadIdx.x; j < half; j += blockDim.x) {
            const int k = j & (ns - 1), o = ((j - k) << 1) + k;
            const float2 u = a[j], v = a[j + half], t = w[k * st];
            const float vr = v.x * t.x - v.y * t.y;
            const float vi = v.x * t.y + v.y * t.x;
            b[o] = make_float2(u.x + vr, u.y + vi);
            b[o + ns] = make_float2(u.x - vr, u.y - vi);
        }
        __syncthreads();
        float2 *tmp = a;
        a = b;
        b = tmp;
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) xr[e] = a[e];
}

}  // namespace

hipError_t fft_rows(float *x, int64_t rows, int64_t n, hipStream_t s) {
    if (rows <= 0 || n <= 0) return hipSuccess;
    if (n > kFftMaxPoints || (n & (n - 1)) != 0 || rows > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int threads = n >= 512 ? 256 : (n >= 128 ? (int)(n / 2) : 64);
    const uint32_t lds_bytes = (uint32_t)((2 * n + n / 2) * sizeof(float2));
    return launch(k_fft_rows, dim3((unsigned)rows), dim3(threads), lds_bytes, s, reinterpret_cast<float2 *>(x),
                  (int)n);
}

}  // namespace k
}  // namespace ofl
