// Error reporting shared by the library's host files: both set the message
// that kpd_last_error returns and pass the code through.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

namespace kpd {

int api_fail(int code, const std::string& msg);
int api_hip_fail(hipError_t e, const char* what);

}  // namespace kpd
