// Size limit of the FFT function block, shared by the IR check, the CPU
// form, the twiddle table and the GPU kernel: rows of up to kFftMaxPoints
// complex values (a power of two); the twiddle table holds kFftMaxPoints / 2
// complex values.
#pragma once

namespace ofl {

constexpr int kFftMaxPoints = 4096;

}  // namespace ofl
