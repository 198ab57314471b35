// Error reporting shared by the C ABI entry points: the message is kept as
// the calling thread's last error (ofl_last_error) and the code returned.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace ofl {

int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);   // returns OFL_E_HIP

}  // namespace ofl
