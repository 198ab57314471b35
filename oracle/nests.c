/*
 * Oracle: plain serial CPU versions of every loop nest of the matrix
 * applications (TEST INFRASTRUCTURE ONLY -- never linked into the product).
 *
 * The paper's evaluation workload is a C/C++ matrix computation whose for-loop
 * nests are offloaded one gene bit at a time (Sec. 3.3, Sec. 4, Sec. 5.1.1).
 * The paper does not print those loops, so the nests here are the ones the
 * applications of this project define: each function is the plain textbook
 * definition of its nest, written out as serial loops in a fixed order.
 *
 *  - FP32 functions evaluate in exactly the order written (built with
 *    -O2 -ffp-contract=off, SSE arithmetic, no reassociation).
 *  - *_f64 twins compute the same quantity in double precision; they are the
 *    accuracy reference for results whose GPU evaluation order differs (GEMM).
 *
 * Random inputs come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), implemented here from its
 * published definition, counter-based so every element is independent.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

/* SplitMix64 output function (the "mix64" variant of the published generator). */
uint64_t or_sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The k-th output (k >= 1) of a SplitMix64 generator started from state s:
 * the state advances by GAMMA before every output. */
uint64_t or_sm64_nth(uint64_t s, uint64_t k)
{
    return or_sm64_mix(s + k * SM64_GAMMA);
}

/* INIT nest: x[idx] = U(seed, stream, idx) in [0,1).
 * Stream key = output number (stream+1) of SplitMix64 seeded with `seed`;
 * element idx = output number (idx+1) of SplitMix64 seeded with that key;
 * the top 24 bits scaled by 2^-24 are exact in FP32. */
void or_init_uniform(float *x, int64_t n, uint64_t seed, uint32_t stream)
{
    uint64_t key = or_sm64_nth(seed, (uint64_t)stream + 1u);
    for (int64_t idx = 0; idx < n; ++idx) {
        uint64_t z = or_sm64_nth(key, (uint64_t)idx + 1u);
        x[idx] = (float)(z >> 40) * (1.0f / 16777216.0f);
    }
}

/* GEMM nest: C[i][j] = sum_{k=0}^{Kd-1} A[i][k] * B[k][j], row-major,
 * A is M x Kd, B is Kd x N, C is M x N.  Each C element is accumulated in
 * FP32 in increasing k, starting from 0. */
void or_gemm_f32(const float *A, const float *B, float *C,
                 int64_t M, int64_t N, int64_t Kd)
{
    for (int64_t i = 0; i < M; ++i) {
        float *c = C + i * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0f;
        for (int64_t k = 0; k < Kd; ++k) {
            const float a = A[i * Kd + k];
            const float *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) {
                float prod = a * b[j];
                c[j] = c[j] + prod;
            }
        }
    }
}

/* Double-precision twin of the GEMM nest on the same FP32 inputs. */
void or_gemm_f64(const float *A, const float *B, double *C,
                 int64_t M, int64_t N, int64_t Kd)
{
    for (int64_t i = 0; i < M; ++i) {
        double *c = C + i * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < Kd; ++k) {
            const double a = (double)A[i * Kd + k];
            const float *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) c[j] += a * (double)b[j];
        }
    }
}

/* GEMM nest on bfloat16 inputs (stored as raw uint16 bit patterns),
 * FP32 accumulation in increasing k.  A bf16*bf16 product is exact in FP32. */
static float bf16_to_f32(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

void or_gemm_bf16(const uint16_t *A, const uint16_t *B, float *C,
                  int64_t M, int64_t N, int64_t Kd)
{
    for (int64_t i = 0; i < M; ++i) {
        float *c = C + i * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0f;
        for (int64_t k = 0; k < Kd; ++k) {
            const float a = bf16_to_f32(A[i * Kd + k]);
            const uint16_t *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) {
                float prod = a * bf16_to_f32(b[j]);
                c[j] = c[j] + prod;
            }
        }
    }
}

void or_gemm_bf16_f64(const uint16_t *A, const uint16_t *B, double *C,
                      int64_t M, int64_t N, int64_t Kd)
{
    for (int64_t i = 0; i < M; ++i) {
        double *c = C + i * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < Kd; ++k) {
            const double a = (double)bf16_to_f32(A[i * Kd + k]);
            const uint16_t *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) c[j] += a * (double)bf16_to_f32(b[j]);
        }
    }
}

/* ------------------------------------------------------------------
 * Split-precision GEMM (the mixed-precision product of the precision
 * configuration): with x = hi + lo, hi = round(x), lo = round(x - hi) in the
 * narrow format, the product is taken as Ah Bh + Ah Bl + Al Bh, i.e. the
 * base product plus one refinement pass (the bf16x3 scheme of Henry, Tang &
 * Heinecke 2019; the split itself goes back to Markidis et al. 2018).
 * Here every product of narrow values is exact in double and the sum is
 * taken in double, so the result is the split method's value up to FP64
 * rounding -- the GPU's only further difference is its FP32 accumulation.
 *
 * FP8 is OCP e4m3 ("E4M3FN"): 1 sign bit, 4 exponent bits with bias 7,
 * 3 fraction bits; normal values (1 + f/8) 2^(e-7) for e = 1..15 (e = 15,
 * f = 7 is NaN, so the largest finite value is 448); subnormals (f/8) 2^-6.
 * Rows of A and columns of B are scaled by powers of two into range first.
 * ------------------------------------------------------------------ */

/* Value of an e4m3 code (NaN code -> NAN). */
double or_e4m3_value(uint8_t c)
{
    const int e = (c >> 3) & 15, f = c & 7;
    double v;
    if (e == 15 && f == 7) return NAN;
    if (e == 0) v = ldexp((double)f, -9);            /* f/8 * 2^-6 */
    else v = ldexp(8.0 + f, e - 10);                  /* (8+f)/8 * 2^(e-7) */
    return (c & 0x80) ? -v : v;
}

/* Nearest e4m3 code to x, ties to even; |x| must not exceed 448. */
uint8_t or_e4m3_rne(double x)
{
    const uint8_t sign = (x < 0.0 || (x == 0.0 && signbit(x))) ? 0x80 : 0x00;
    const double a = fabs(x);
    double q;                                         /* spacing of codes around a */
    if (a < ldexp(1.0, -6)) {
        q = ldexp(1.0, -9);
    } else {
        int E;
        (void)frexp(a, &E);                           /* a = m 2^E, m in [0.5, 1) */
        q = ldexp(1.0, E - 4);                        /* 3 fraction bits below 2^(E-1) */
    }
    const double n = a / q;                           /* exact: q is a power of two */
    double r = floor(n);
    const double d = n - r;
    if (d > 0.5 || (d == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
    const double v = r * q;                           /* rounded magnitude */
    if (v == 0.0) return sign;
    if (v < ldexp(1.0, -6)) return (uint8_t)(sign | (uint8_t)(v / ldexp(1.0, -9)));
    int E;
    const double m = frexp(v, &E);                    /* v = m 2^E */
    const int ef = E - 1 + 7;
    const int f = (int)((2.0 * m - 1.0) * 8.0);
    return (uint8_t)(sign | (uint8_t)(ef << 3) | (uint8_t)f);
}

/* Largest power of two s with amax * s <= 224 (half the e4m3 maximum of 448,
 * which leaves room for the rounding of hi); 1 for amax 0 or not finite. */
double or_e4m3_scale(double amax)
{
    if (!(amax > 0.0) || !isfinite(amax)) return 1.0;
    double s = 1.0;
    while (amax * s > 224.0) s *= 0.5;
    while (amax * (2.0 * s) <= 224.0 && s < ldexp(1.0, 126)) s *= 2.0;
    if (s < ldexp(1.0, -126)) s = ldexp(1.0, -126);
    return s;
}

static double bf16_to_f64(uint16_t h) { return (double)bf16_to_f32(h); }
static uint16_t f32_to_bf16_rne(float f);

/* Split of one FP32 value: hi and lo as doubles, both on the narrow grid.
 * For fp8, xs is the value already multiplied by its power-of-two scale. */
static void split_bf16(float x, double *hi, double *lo)
{
    const uint16_t h = f32_to_bf16_rne(x);
    *hi = bf16_to_f64(h);
    const float r = (float)((double)x - *hi);         /* exact in FP32 */
    *lo = bf16_to_f64(f32_to_bf16_rne(r));
}

static void split_e4m3(float xs, double *hi, double *lo)
{
    *hi = or_e4m3_value(or_e4m3_rne((double)xs));
    const double r = (double)xs - *hi;                /* exact */
    *lo = or_e4m3_value(or_e4m3_rne(r));
}

/* C = Ah Bh + Ah Bl + Al Bh in double; variant 1 = bf16, 2 = e4m3 with a
 * power-of-two scale per row of A and per column of B. */
void or_gemm_split_f64(const float *A, const float *B, double *C,
                       int64_t M, int64_t N, int64_t Kd, int variant)
{
    double *ah = malloc(sizeof(double) * (size_t)(M * Kd + 1));
    double *al = malloc(sizeof(double) * (size_t)(M * Kd + 1));
    double *bh = malloc(sizeof(double) * (size_t)(Kd * N + 1));
    double *bl = malloc(sizeof(double) * (size_t)(Kd * N + 1));
    double *sa = malloc(sizeof(double) * (size_t)(M + 1));
    double *sb = malloc(sizeof(double) * (size_t)(N + 1));
    for (int64_t i = 0; i < M; ++i) {
        double amax = 0.0;
        for (int64_t k = 0; k < Kd; ++k) amax = fmax(amax, fabs((double)A[i * Kd + k]));
        sa[i] = variant == 2 ? or_e4m3_scale(amax) : 1.0;
    }
    for (int64_t j = 0; j < N; ++j) {
        double amax = 0.0;
        for (int64_t k = 0; k < Kd; ++k) amax = fmax(amax, fabs((double)B[k * N + j]));
        sb[j] = variant == 2 ? or_e4m3_scale(amax) : 1.0;
    }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < Kd; ++k) {
            const float x = A[i * Kd + k];
            if (variant == 2) split_e4m3((float)((double)x * sa[i]), &ah[i * Kd + k], &al[i * Kd + k]);
            else split_bf16(x, &ah[i * Kd + k], &al[i * Kd + k]);
        }
    for (int64_t k = 0; k < Kd; ++k)
        for (int64_t j = 0; j < N; ++j) {
            const float x = B[k * N + j];
            if (variant == 2) split_e4m3((float)((double)x * sb[j]), &bh[k * N + j], &bl[k * N + j]);
            else split_bf16(x, &bh[k * N + j], &bl[k * N + j]);
        }
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < Kd; ++k) {
                const double a1 = ah[i * Kd + k], a0 = al[i * Kd + k];
                const double b1 = bh[k * N + j], b0 = bl[k * N + j];
                acc += a1 * b1 + a1 * b0 + a0 * b1;
            }
            C[i * N + j] = acc / (sa[i] * sb[j]);
        }
    free(ah); free(al); free(bh); free(bl); free(sa); free(sb);
}

/* Element-wise nests. */
void or_add_scaled(float *C, const float *A, float alpha, int64_t n)
{   /* C[e] = C[e] + alpha*A[e] */
    for (int64_t e = 0; e < n; ++e) {
        float t = alpha * A[e];
        C[e] = C[e] + t;
    }
}

void or_avg2(float *S, const float *X, const float *Y, int64_t n)
{   /* S[e] = 0.5*(X[e] + Y[e]) */
    for (int64_t e = 0; e < n; ++e) {
        float t = X[e] + Y[e];
        S[e] = 0.5f * t;
    }
}

void or_scale(float *D, float beta, int64_t n)
{   /* D[e] = beta*D[e] */
    for (int64_t e = 0; e < n; ++e) D[e] = beta * D[e];
}

void or_copy(float *dst, const float *src, int64_t n)
{
    for (int64_t e = 0; e < n; ++e) dst[e] = src[e];
}

/* bfloat16 cast, round to nearest even (NaN kept quiet NaN). */
static uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

void or_cast_bf16(uint16_t *dst, const float *src, int64_t n)
{
    for (int64_t e = 0; e < n; ++e) dst[e] = f32_to_bf16_rne(src[e]);
}

/* TRANSPOSE nest: T[j][i] = X[i][j], X is R x Cc, T is Cc x R. */
void or_transpose(const float *X, float *T, int64_t R, int64_t Cc)
{
    for (int64_t i = 0; i < R; ++i)
        for (int64_t j = 0; j < Cc; ++j) T[j * R + i] = X[i * Cc + j];
}

/* REDUCE nest: s[0] = s[0] + sum_e (double)x[e]^2, serially in index order. */
void or_sumsq(const float *x, int64_t n, double *s)
{
    double acc = s[0];
    for (int64_t e = 0; e < n; ++e) {
        double v = (double)x[e];
        acc = acc + v * v;
    }
    s[0] = acc;
}

/*
 * STENCIL nest: one weighted-Jacobi sweep of the 19-point 3-D Laplacian
 * neighbourhood (centre, 6 faces, 12 edges) on p[i][j][k], k contiguous,
 * writing q on the interior only (Dirichlet boundary, never written).
 *
 * Weights: centre 1/4, each face 1/16, each edge 1/32 (sum 1/4+6/16+12/32=1).
 * Evaluation order (fixed, FP32), with plane-local partial sums of plane m:
 *   a_m = p[m][j][k]
 *   x_m = (p[m][j-1][k] + p[m][j+1][k]) + (p[m][j][k-1] + p[m][j][k+1])
 *   y_m = (p[m][j-1][k-1] + p[m][j-1][k+1]) + (p[m][j+1][k-1] + p[m][j+1][k+1])
 *   F   = (a_{i-1} + a_{i+1}) + x_i                 (the 6 faces)
 *   E   = (x_{i-1} + x_{i+1}) + y_i                 (the 12 edges)
 *   q   = (0.25*a_i + 0.0625*F) + 0.03125*E
 * Residual of the sweep: res[0] += sum over the interior, in i,j,k order,
 * of d*d with d = (double)q - (double)p[i][j][k].
 */
static float plane_x(const float *p, int64_t J, int64_t K, int64_t m, int64_t j, int64_t k)
{
    const float *r = p + (m * J + j) * K;
    float s1 = r[-K + k] + r[K + k];
    float s2 = r[k - 1] + r[k + 1];
    return s1 + s2;
}

static float plane_y(const float *p, int64_t J, int64_t K, int64_t m, int64_t j, int64_t k)
{
    const float *r = p + (m * J + j) * K;
    float s1 = r[-K + k - 1] + r[-K + k + 1];
    float s2 = r[K + k - 1] + r[K + k + 1];
    return s1 + s2;
}

void or_stencil19(const float *p, float *q, int64_t I, int64_t J, int64_t K, double *res)
{
    double acc = res[0];
    for (int64_t i = 1; i < I - 1; ++i)
        for (int64_t j = 1; j < J - 1; ++j)
            for (int64_t k = 1; k < K - 1; ++k) {
                float am = p[((i - 1) * J + j) * K + k];
                float a0 = p[(i * J + j) * K + k];
                float ap = p[((i + 1) * J + j) * K + k];
                float xm = plane_x(p, J, K, i - 1, j, k);
                float x0 = plane_x(p, J, K, i, j, k);
                float xp = plane_x(p, J, K, i + 1, j, k);
                float y0 = plane_y(p, J, K, i, j, k);
                float F = (am + ap) + x0;
                float E = (xm + xp) + y0;
                float t0 = 0.25f * a0;
                float t1 = 0.0625f * F;
                float t2 = 0.03125f * E;
                float v = (t0 + t1) + t2;
                q[(i * J + j) * K + k] = v;
                double d = (double)v - (double)a0;
                acc = acc + d * d;
            }
    res[0] = acc;
}

/* Double-precision twin of one sweep: all neighbours summed in double. */
void or_stencil19_f64(const double *p, double *q, int64_t I, int64_t J, int64_t K, double *res)
{
    double acc = res[0];
#define P(a, b, c) p[((a) * J + (b)) * K + (c)]
    for (int64_t i = 1; i < I - 1; ++i)
        for (int64_t j = 1; j < J - 1; ++j)
            for (int64_t k = 1; k < K - 1; ++k) {
                double faces = P(i - 1, j, k) + P(i + 1, j, k) + P(i, j - 1, k) + P(i, j + 1, k)
                             + P(i, j, k - 1) + P(i, j, k + 1);
                double edges = P(i - 1, j - 1, k) + P(i - 1, j + 1, k) + P(i + 1, j - 1, k) + P(i + 1, j + 1, k)
                             + P(i - 1, j, k - 1) + P(i - 1, j, k + 1) + P(i + 1, j, k - 1) + P(i + 1, j, k + 1)
                             + P(i, j - 1, k - 1) + P(i, j - 1, k + 1) + P(i, j + 1, k - 1) + P(i, j + 1, k + 1);
                double v = 0.25 * P(i, j, k) + faces / 16.0 + edges / 32.0;
                q[(i * J + j) * K + k] = v;
                double d = v - P(i, j, k);
                acc += d * d;
            }
#undef P
    res[0] = acc;
}

/* COPY-INTERIOR nest: p[i][j][k] = q[i][j][k] on the interior. */
void or_copy_interior(float *p, const float *q, int64_t I, int64_t J, int64_t K)
{
    for (int64_t i = 1; i < I - 1; ++i)
        for (int64_t j = 1; j < J - 1; ++j)
            for (int64_t k = 1; k < K - 1; ++k) {
                int64_t e = (i * J + j) * K + k;
                p[e] = q[e];
            }
}

void or_copy_interior_f64(double *p, const double *q, int64_t I, int64_t J, int64_t K)
{
    for (int64_t i = 1; i < I - 1; ++i)
        for (int64_t j = 1; j < J - 1; ++j)
            for (int64_t k = 1; k < K - 1; ++k) {
                int64_t e = (i * J + j) * K + k;
                p[e] = q[e];
            }
}

/* Initial field (host set-up, not a nest): the separable sine mode
 * p = sin(m*pi*i/(I-1)) * sin(m*pi*j/(J-1)) * sin(m*pi*k/(K-1)),
 * evaluated in double; `out32` gets it rounded to FP32 (may be NULL). */
void or_sin_field(float *out32, double *out64, int64_t I, int64_t J, int64_t K, int32_t m)
{
    const double pi = 3.14159265358979323846;
    for (int64_t i = 0; i < I; ++i) {
        double si = sin(m * pi * (double)i / (double)(I - 1));
        for (int64_t j = 0; j < J; ++j) {
            double sj = sin(m * pi * (double)j / (double)(J - 1));
            for (int64_t k = 0; k < K; ++k) {
                double sk = sin(m * pi * (double)k / (double)(K - 1));
                double v = si * sj * sk;
                int64_t e = (i * J + j) * K + k;
                if (out32) out32[e] = (float)v;
                if (out64) out64[e] = v;
            }
        }
    }
}

/* Loop-carried recurrences (rejected by the dependence check, always serial). */
void or_rec_prefix(float *v, const float *S, int64_t N, int64_t ld)
{   /* v[i] = v[i-1] + S[i][0], i = 1..N-1 */
    for (int64_t i = 1; i < N; ++i) v[i] = v[i - 1] + S[i * ld];
}

void or_rec_decay(float *w, const float *p, int64_t J, int64_t K)
{   /* w[k] = 0.5*w[k-1] + p[1][1][k], k = 1..K-1 */
    const float *row = p + (1 * J + 1) * K;
    for (int64_t k = 1; k < K; ++k) {
        float h = 0.5f * w[k - 1];
        w[k] = h + row[k];
    }
}

/* Sequential linear congruential fill (the "opaque library call" nest):
 * x_{e+1} = 1664525 * x_e + 1013904223 mod 2^32, x_0 = seed32;
 * L[e] = x_{e+1} scaled by 2^-32 to [0,1) in FP32 (top 24 bits). */
void or_lcg_fill(float *L, int64_t n, uint32_t seed32)
{
    uint32_t x = seed32;
    for (int64_t e = 0; e < n; ++e) {
        x = 1664525u * x + 1013904223u;
        L[e] = (float)(x >> 8) * (1.0f / 16777216.0f);
    }
}

/* Raw LCG states, for pinning the recurrence against its published constants. */
void or_lcg_states(uint32_t *out, int64_t n, uint32_t seed32)
{
    uint32_t x = seed32;
    for (int64_t e = 0; e < n; ++e) {
        x = 1664525u * x + 1013904223u;
        out[e] = x;
    }
}
