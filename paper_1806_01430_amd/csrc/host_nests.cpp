// Serial host nests.  FP32 expressions are evaluated exactly as written
// (this file is compiled with -ffp-contract=off), so a nest run here and the
// same nest run by its GPU kernel agree bit for bit wherever the kernel keeps
// the same per-element order (everything except the GEMM and the FP64 sums).
#include "host_nests.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace ofl {

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr double kTwoPi = 6.283185307179586;   // 2 pi rounded to double

// SplitMix64 output mix (Steele, Lea & Flood 2014).
inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline float bf16_bits_to_float(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

inline uint16_t float_to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

}  // namespace

uint64_t uniform_stream_key(uint64_t seed, uint32_t stream) {
    return mix64(seed + ((uint64_t)stream + 1u) * kGolden);
}

void fill_setup_sin(const Buffer &b, float *dst) {
    const int64_t I = b.dims[0], J = b.dims[1], K = b.dims[2];
    const double pi = 3.14159265358979323846;
    const double m = (double)b.sin_mode;
    std::vector<double> sk(K);
    for (int64_t k = 0; k < K; ++k) sk[k] = std::sin(m * pi * (double)k / (double)(K - 1));
    for (int64_t i = 0; i < I; ++i) {
        double si = std::sin(m * pi * (double)i / (double)(I - 1));
        for (int64_t j = 0; j < J; ++j) {
            double sij = si * std::sin(m * pi * (double)j / (double)(J - 1));
            float *row = dst + (i * J + j) * K;
            for (int64_t k = 0; k < K; ++k) row[k] = (float)(sij * sk[k]);
        }
    }
}

void fft_twiddle_table(float *w) {
    for (int64_t m = 0; m < kFftMaxPoints / 2; ++m) {
        const double th = kTwoPi * (double)m / (double)kFftMaxPoints;
        w[2 * m] = (float)std::cos(th);
        w[2 * m + 1] = (float)-std::sin(th);
    }
}

void fft_twiddle_packed(float *w) {
    std::vector<float> t(kFftMaxPoints);
    fft_twiddle_table(t.data());
    for (int64_t n = 2; n <= kFftMaxPoints; n <<= 1)
        for (int64_t m = 0; m < n / 2; ++m) {
            const int64_t at = n / 2 - 1 + m, from = m * (kFftMaxPoints / n);
            w[2 * at] = t[2 * from];
            w[2 * at + 1] = t[2 * from + 1];
        }
}

bool run_host_nest(const AppIR &app, const Nest &n, const std::vector<void *> &host, const int64_t *env,
                   uint64_t seed, const Deadline &dl) {
    auto F = [&](int i) { return static_cast<float *>(host[n.b[i]]); };
    auto cnt = [&](int i) { return app.bufs[n.b[i]].count; };
    switch (n.op) {
    case OP_INIT_UNIFORM:
        for (size_t t = 0; t < n.b.size(); ++t) {
            const uint64_t key = uniform_stream_key(seed, n.streams[t]);
            float *x = static_cast<float *>(host[n.b[t]]);
            const int64_t c = app.bufs[n.b[t]].count;
            for (int64_t e = 0; e < c; ++e) {
                if ((e & 0xFFFF) == 0 && dl.expired()) return false;
                x[e] = (float)(mix64(key + (uint64_t)(e + 1) * kGolden) >> 40) * (1.0f / 16777216.0f);
            }
        }
        return true;
    case OP_GEMM: {
        const Buffer &a = app.bufs[n.b[0]], &bb = app.bufs[n.b[1]];
        const int64_t M = a.dims[0], Kd = a.dims[1], N = bb.dims[1];
        const float *A = F(0), *B = F(1);
        float *C = F(2);
        for (int64_t i = 0; i < M; ++i) {
            if (dl.expired()) return false;
            float *c = C + i * N;
            for (int64_t j = 0; j < N; ++j) c[j] = 0.0f;
            for (int64_t k = 0; k < Kd; ++k) {
                const float av = A[i * Kd + k];
                const float *brow = B + k * N;
                for (int64_t j = 0; j < N; ++j) c[j] = c[j] + av * brow[j];
            }
        }
        return true;
    }
    case OP_GEMM_BF16: {
        const Buffer &a = app.bufs[n.b[0]], &bb = app.bufs[n.b[1]];
        const int64_t M = a.dims[0], Kd = a.dims[1], N = bb.dims[1];
        const uint16_t *A = static_cast<const uint16_t *>(host[n.b[0]]);
        const uint16_t *B = static_cast<const uint16_t *>(host[n.b[1]]);
        float *C = F(2);
        for (int64_t i = 0; i < M; ++i) {
            if (dl.expired()) return false;
            float *c = C + i * N;
            for (int64_t j = 0; j < N; ++j) c[j] = 0.0f;
            for (int64_t k = 0; k < Kd; ++k) {
                const float av = bf16_bits_to_float(A[i * Kd + k]);
                const uint16_t *brow = B + k * N;
                for (int64_t j = 0; j < N; ++j) c[j] = c[j] + av * bf16_bits_to_float(brow[j]);
            }
        }
        return true;
    }
    case OP_ADD_SCALED: {
        float *C = F(0);
        const float *A = F(1);
        const float al = (float)n.alpha;
        for (int64_t e = 0, c = cnt(0); e < c; ++e) C[e] = C[e] + al * A[e];
        return !dl.expired();
    }
    case OP_AVG2: {
        float *S = F(0);
        const float *X = F(1), *Y = F(2);
        for (int64_t e = 0, c = cnt(0); e < c; ++e) S[e] = 0.5f * (X[e] + Y[e]);
        return !dl.expired();
    }
    case OP_SCALE: {
        float *D = F(0);
        const float be = (float)n.alpha;
        for (int64_t e = 0, c = cnt(0); e < c; ++e) D[e] = be * D[e];
        return !dl.expired();
    }
    case OP_COPY:
        std::memcpy(host[n.b[0]], host[n.b[1]], app.bufs[n.b[0]].nbytes);
        return !dl.expired();
    case OP_CAST_BF16:
        for (size_t t = 0; t + 1 < n.b.size(); t += 2) {
            uint16_t *d = static_cast<uint16_t *>(host[n.b[t]]);
            const float *s = static_cast<const float *>(host[n.b[t + 1]]);
            for (int64_t e = 0, c = app.bufs[n.b[t]].count; e < c; ++e) d[e] = float_to_bf16_bits(s[e]);
        }
        return !dl.expired();
    case OP_TRANSPOSE: {
        const Buffer &x = app.bufs[n.b[0]];
        const int64_t R = x.dims[0], Cc = x.dims[1];
        const float *X = F(0);
        float *T = F(1);
        for (int64_t i = 0; i < R; ++i) {
            if ((i & 63) == 0 && dl.expired()) return false;
            for (int64_t j = 0; j < Cc; ++j) T[j * R + i] = X[i * Cc + j];
        }
        return true;
    }
    case OP_SUMSQ: {
        const float *x = F(0);
        double *s = static_cast<double *>(host[n.b[1]]);
        double acc = s[0];
        for (int64_t e = 0, c = cnt(0); e < c; ++e) {
            const double v = (double)x[e];
            acc = acc + v * v;
        }
        s[0] = acc;
        return !dl.expired();
    }
    case OP_STENCIL19: {
        const Buffer &g = app.bufs[n.b[0]];
        const int64_t I = g.dims[0], J = g.dims[1], K = g.dims[2];
        const float *p = F(0);
        float *q = F(1);
        double *res = static_cast<double *>(host[n.b[2]]) + env[n.slot_repeat];
        double acc = *res;
        const int64_t JK = J * K;
        for (int64_t i = 1; i < I - 1; ++i) {
            if (dl.expired()) {
                *res = acc;
                return false;
            }
            for (int64_t j = 1; j < J - 1; ++j) {
                const float *c0 = p + i * JK + j * K;   // row (i, j)
                const float *cm = c0 - JK, *cp = c0 + JK;
                for (int64_t k = 1; k < K - 1; ++k) {
                    // in-plane cross (x) of planes i-1, i, i+1 and diagonals (y) of plane i
                    const float xm = (cm[k - K] + cm[k + K]) + (cm[k - 1] + cm[k + 1]);
                    const float x0 = (c0[k - K] + c0[k + K]) + (c0[k - 1] + c0[k + 1]);
                    const float xp = (cp[k - K] + cp[k + K]) + (cp[k - 1] + cp[k + 1]);
                    const float y0 = (c0[k - K - 1] + c0[k - K + 1]) + (c0[k + K - 1] + c0[k + K + 1]);
                    const float faces = (cm[k] + cp[k]) + x0;
                    const float edges = (xm + xp) + y0;
                    const float v = (0.25f * c0[k] + 0.0625f * faces) + 0.03125f * edges;
                    q[i * JK + j * K + k] = v;
                    const double d = (double)v - (double)c0[k];
                    acc = acc + d * d;
                }
            }
        }
        *res = acc;
        return true;
    }
    case OP_COPY_INTERIOR: {
        const Buffer &g = app.bufs[n.b[0]];
        const int64_t I = g.dims[0], J = g.dims[1], K = g.dims[2];
        float *p = F(0);
        const float *q = F(1);
        for (int64_t i = 1; i < I - 1; ++i) {
            if (dl.expired()) return false;
            for (int64_t j = 1; j < J - 1; ++j) {
                const int64_t base = (i * J + j) * K;
                if (K > 2) std::memcpy(p + base + 1, q + base + 1, (size_t)(K - 2) * sizeof(float));
            }
        }
        return true;
    }
    case OP_REC_PREFIX: {
        float *v = F(0);
        const float *S = F(1);
        const int64_t N = app.bufs[n.b[0]].dims[0], ld = app.bufs[n.b[1]].dims[1];
        for (int64_t i = 1; i < N; ++i) v[i] = v[i - 1] + S[i * ld];
        return !dl.expired();
    }
    case OP_REC_DECAY: {
        float *w = F(0);
        const Buffer &g = app.bufs[n.b[1]];
        const float *row = F(1) + (1 * g.dims[1] + 1) * g.dims[2];
        for (int64_t k = 1; k < g.dims[2]; ++k) w[k] = 0.5f * w[k - 1] + row[k];
        return !dl.expired();
    }
    case OP_HOST_CODE: {
        // compiled from the nest's own source text: it runs to completion
        // (the deadline is checked at the nest's boundary)
        if (!n.host_fn) return false;
        n.host_fn(host.data(), env);
        return !dl.expired();
    }
    case OP_LCG_FILL: {
        float *L = F(0);
        uint32_t x = n.seed32;
        for (int64_t e = 0, c = cnt(0); e < c; ++e) {
            x = 1664525u * x + 1013904223u;
            L[e] = (float)(x >> 8) * (1.0f / 16777216.0f);
        }
        return !dl.expired();
    }
    case OP_FFT_ROWS: {
        // the CPU form of the FFT call: the same radix-2 self-sorting
        // (Stockham) passes as the GPU kernel, per row; the inverse conjugates
        // the row, transforms it forward, and conjugates and scales by 1/n; a
        // real row is transformed as half as many complex values and unpacked
        const Buffer &x = app.bufs[n.b[0]];
        const int64_t rows = x.dims[0], pts = x.dims[1] / 2, half = pts / 2, ws = kFftMaxPoints / std::max<int64_t>(pts, 1);
        std::vector<float> w(kFftMaxPoints), a(2 * pts), b(2 * pts);
        fft_twiddle_table(w.data());
        float *X = F(0);
        for (int64_t r = 0; r < rows; ++r) {
            if ((r & 15) == 0 && dl.expired()) return false;
            float *xr = X + r * 2 * pts;
            std::memcpy(a.data(), xr, 2 * pts * sizeof(float));
            if (n.real && n.inverse) {
                // a packed spectrum of 2 pts real values: back to the
                // half-length transform Z, bin pairs (k, pts - k), as the kernel does
                const int64_t wr = ws / 2;
                auto zbin = [&](int64_t ka, int64_t kb, int64_t kt, float &zr, float &zi) {
                    const float ar = a[2 * ka], ai = a[2 * ka + 1], br = a[2 * kb], bi = a[2 * kb + 1];
                    const float er = (ar + br) * 0.5f, ei = (ai - bi) * 0.5f;
                    const float dr = (ar - br) * 0.5f, di = (ai + bi) * 0.5f;
                    const float tr = w[2 * kt * wr], ti = -w[2 * kt * wr + 1];
                    const float orr = dr * tr - di * ti, oi = dr * ti + di * tr;
                    zr = er - oi;
                    zi = ei + orr;
                };
                for (int64_t k = 1; 2 * k <= pts; ++k) {
                    float yr, yi, qr = 0.f, qi = 0.f;
                    zbin(k, pts - k, k, yr, yi);
                    if (2 * k != pts) zbin(pts - k, k, pts - k, qr, qi);
                    a[2 * k] = yr;
                    a[2 * k + 1] = yi;
                    if (2 * k != pts) {
                        a[2 * (pts - k)] = qr;
                        a[2 * (pts - k) + 1] = qi;
                    }
                }
                const float p0 = a[0], p1 = a[1];
                a[0] = (p0 + p1) * 0.5f;
                a[1] = (p0 - p1) * 0.5f;
            }
            if (n.inverse)
                for (int64_t j = 0; j < pts; ++j) a[2 * j + 1] = -a[2 * j + 1];
            for (int64_t ns = 1, st = half; ns < pts; ns <<= 1, st >>= 1) {
                for (int64_t j = 0; j < half; ++j) {
                    const int64_t k = j & (ns - 1), o = ((j - k) << 1) + k;
                    const float ur = a[2 * j], ui = a[2 * j + 1];
                    const float vr0 = a[2 * (j + half)], vi0 = a[2 * (j + half) + 1];
                    const float tr = w[2 * k * st * ws], ti = w[2 * k * st * ws + 1];
                    const float vr = vr0 * tr - vi0 * ti;
                    const float vi = vr0 * ti + vi0 * tr;
                    b[2 * o] = ur + vr;
                    b[2 * o + 1] = ui + vi;
                    b[2 * (o + ns)] = ur - vr;
                    b[2 * (o + ns) + 1] = ui - vi;
                }
                a.swap(b);
            }
            if (n.real && !n.inverse) {
                // the row held 2 pts real values: unpack the spectrum of the
                // half-length transform, bin pairs (k, pts - k), as the kernel does
                const int64_t wr = ws / 2;   // twiddle stride of length 2 pts
                auto bin = [&](int64_t ka, int64_t kb, int64_t kt, float &yr, float &yi) {
                    const float ar = a[2 * ka], ai = a[2 * ka + 1], br = a[2 * kb], bi = a[2 * kb + 1];
                    const float er = (ar + br) * 0.5f, ei = (ai - bi) * 0.5f;
                    const float dr = (ar - br) * 0.5f, di = (ai + bi) * 0.5f;
                    const float orr = di, oi = -dr;
                    const float tr = w[2 * kt * wr], ti = w[2 * kt * wr + 1];
                    const float pr = orr * tr - oi * ti, pi = orr * ti + oi * tr;
                    yr = er + pr;
                    yi = ei + pi;
                };
                for (int64_t k = 1; 2 * k <= pts; ++k) {
                    float yr, yi, zr = 0.f, zi = 0.f;
                    bin(k, pts - k, k, yr, yi);
                    if (2 * k != pts) bin(pts - k, k, pts - k, zr, zi);
                    a[2 * k] = yr;
                    a[2 * k + 1] = yi;
                    if (2 * k != pts) {
                        a[2 * (pts - k)] = zr;
                        a[2 * (pts - k) + 1] = zi;
                    }
                }
                const float z0r = a[0], z0i = a[1];
                a[0] = z0r + z0i;
                a[1] = z0r - z0i;
            }
            if (n.inverse) {
                const float sc = 1.0f / (float)pts;
                for (int64_t j = 0; j < pts; ++j) {
                    a[2 * j] = a[2 * j] * sc;
                    a[2 * j + 1] = -a[2 * j + 1] * sc;
                }
            }
            std::memcpy(xr, a.data(), 2 * pts * sizeof(float));
        }
        return true;
    }
    default:
        return true;
    }
}

}  // namespace ofl
