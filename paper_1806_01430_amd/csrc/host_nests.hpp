// Serial host execution of a nest (gene bit 0, and the rejected nests that
// always stay on the CPU).  One thread, the nest's own loop order.
#pragma once

#include <chrono>
#include <cstdint>
#include <vector>

#include "ir.hpp"

namespace ofl {

struct Deadline {
    bool active = false;
    std::chrono::steady_clock::time_point until;
    bool expired() const { return active && std::chrono::steady_clock::now() > until; }
};

// Runs nest `n` on host arrays `host[b]`; `env` = repeat-variable values;
// `seed` = application seed.  Returns false if the deadline expired (checked
// once per outer-loop iteration), leaving the outputs partially written.
bool run_host_nest(const AppIR &app, const Nest &n, const std::vector<void *> &host, const int64_t *env,
                   uint64_t seed, const Deadline &dl);

// Host part of the counter-based generator: key of random stream `stream`.
uint64_t uniform_stream_key(uint64_t seed, uint32_t stream);

// Set-up content of a buffer (sine-mode field), written into `dst`.
void fill_setup_sin(const Buffer &b, float *dst);

// Twiddles of the FFT function block: w[2m], w[2m+1] = cos, -sin of
// 2 pi m / kFftMaxPoints (computed in double, rounded once), m <
// kFftMaxPoints / 2.  A row of n points uses entries m * (kFftMaxPoints / n):
// the angle 2 pi (m s) / (n s) is the same double for a power-of-two s.  The
// CPU form and the GPU kernel read this one table, so both multiply by the
// same values.
void fft_twiddle_table(float *w);

// The tables of every row length n = 2, 4, ..., kFftMaxPoints packed back to
// back, each contiguous: the n/2 twiddles of n points start at complex
// offset n/2 - 1 and are fft_twiddle_table's entries m * (kFftMaxPoints / n)
// (the same values; 2 (kFftMaxPoints - 1) floats in all).  The GPU kernel
// reads these, so its gathers stay dense at every row length.
void fft_twiddle_packed(float *w);

}  // namespace ofl
