// Error reporting shared by the C ABI sources: every entry point returns CMBX_OK or a
// negative code and leaves a message for cmbx_last_error in the calling thread.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace cmbx {

// The calling thread's last error message.
std::string& err_msg();
// Set the message (printf format) and return `code`.
int fail(int code, const char* fmt, ...);
// Clear the message and return CMBX_OK.
int ok();

}  // namespace cmbx

#define HIP_TRY(call)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) return cmbx::fail(CMBX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
