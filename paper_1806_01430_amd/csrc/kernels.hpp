// Launchers of the gfx950 kernels, one per nest kind.  All launch on the given
// stream and return the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ofl {
namespace k {

// Device scratch used by the reductions: the per-block (or per-wave) partial
// sums a reduction kernel leaves for the ordered finish launched after it.
struct ReduceScratch {
    double *partials = nullptr;
    int64_t capacity = 0;   // number of partials
};

hipError_t fill_zero(void *dst, uint64_t bytes, hipStream_t s);
// out[i] = (double) element idx[i] of src (dtype 0 f32, 1 f64, 2 bf16), i < n.
hipError_t gather_probes(const void *src, int dtype, const int64_t *idx, int n, double *out, hipStream_t s);
hipError_t init_uniform(float *x, int64_t n, uint64_t key, hipStream_t s);
hipError_t add_scaled(float *C, const float *A, float alpha, int64_t n, hipStream_t s);
hipError_t avg2(float *S, const float *X, const float *Y, int64_t n, hipStream_t s);
hipError_t scale(float *D, float beta, int64_t n, hipStream_t s);
hipError_t copy_bytes(void *dst, const void *src, uint64_t bytes, hipStream_t s);
hipError_t cast_bf16(uint16_t *dst, const float *src, int64_t n, hipStream_t s);
hipError_t transpose(const float *X, float *T, int64_t R, int64_t Cc, hipStream_t s);
hipError_t sumsq(const float *x, int64_t n, double *s_out, const ReduceScratch &rs, hipStream_t s);
// In-place DFT of each of `rows` rows of n complex values (real and
// imaginary parts interleaved), n a power of two up to kFftMaxPoints (4096):
// forward, or with `inverse` the inverse transform scaled by 1/n;
// `tw` is the device copy of fft_twiddle_packed (the contiguous table of
// each row length, 4095 complex values).
hipError_t fft_rows(float *x, int64_t rows, int64_t n, const float *tw, bool inverse, hipStream_t s);
// In-place DFT of each of `rows` rows of n real values (n a power of two,
// 2 <= n <= kFftMaxPoints), written as the packed spectrum [Re X0, Re X(n/2),
// Re X1, Im X1, ..., Re X(n/2-1), Im X(n/2-1)]: the complex transform of the
// row read as n/2 complex values, then one unpacking pass; `inverse`: a
// packed spectrum replaced by its real row (one packing pass, then the
// inverse complex transform of n/2 values).
hipError_t rfft_rows(float *x, int64_t rows, int64_t n, const float *tw, bool inverse, hipStream_t s);
// The sweep writes q and one residual partial per wave; adding the partials
// to the sweep's residual slot is a separate step (ResidualFinish) that runs
// as a one-block kernel or as the extra block of an interior copy launched
// next on the same stream.  The partials live in the ReduceScratch area, so a
// finish must run before the next launch that writes partials.
struct ResidualFinish {
    const double *partials = nullptr;
    int n = 0;                 // 0: nothing owed
    double *target = nullptr;  // the sweep's residual slot
};
// Launch the sweep; a finish still owed in `fin` is launched first; on
// return `fin` holds the sweep's own finish.
hipError_t stencil19_sweep(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                           const ReduceScratch &rs, hipStream_t s, ResidualFinish &fin);
// Launch the finish owed in `fin` (if any) as one block; clears `fin`.
hipError_t residual_finish(ResidualFinish &fin, hipStream_t s);
// Sweep and finish (two launches).
hipError_t stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res_slot,
                     const ReduceScratch &rs, hipStream_t s);
// p = q on the interior; a finish owed in *fin runs as one extra block of
// the same launch (and *fin is cleared).
hipError_t copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K, hipStream_t s,
                         ResidualFinish *fin = nullptr);
hipError_t gemm_f32(const float *A, const float *B, float *C, int64_t M, int64_t N, int64_t K, hipStream_t s);

// Products on MFMA over k-contiguous, tile-padded operands prepared in a
// caller-provided workspace.  variant 1 = BF16x3 and 2 = FP8x2 (FP32 inputs
// split into hi/lo parts, one refinement pass), 3 = bf16 inputs.
constexpr int kColSlices = 32;   // k slices of the column-maximum pass
int64_t gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int variant);
int gemm_launches(int64_t M, int64_t N, int64_t K, int variant);
hipError_t gemm_split(const float *A, const float *B, float *C, int64_t M, int64_t N, int64_t K, int variant,
                      void *ws, int64_t ws_bytes, hipStream_t s);
hipError_t gemm_bf16(const uint16_t *A, const uint16_t *B, float *C, int64_t M, int64_t N, int64_t K, void *ws,
                     int64_t ws_bytes, hipStream_t s);
hipError_t prep_a(const void *A, void *Ap, const float *sa, int M, int K, int Mp, int Kp, int mode, hipStream_t s);
hipError_t split_bt(const void *B, void *Bt, const float *sb, int K, int N, int Kp, int mode, hipStream_t s);
hipError_t row_scales(const float *A, float *s_out, float *inv_out, int M, int K, hipStream_t s);
hipError_t col_scales(const float *B, float *s_out, float *inv_out, float *part, int K, int N, int ld_part,
                      hipStream_t s);

// Upper bound on partials the reductions need for a problem size.
int64_t sumsq_partials(int64_t n);
int64_t stencil_partials(int64_t I, int64_t J, int64_t K);

}  // namespace k
}  // namespace ofl
