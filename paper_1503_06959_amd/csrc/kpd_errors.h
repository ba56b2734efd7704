// Error reporting shared by the library's host files: both set the message
// that kpd_last_error returns and pass the code through.
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>

namespace kpd {

int api_fail(int code, const std::string& msg);
int api_hip_fail(hipError_t e, const char* what);

// Handles of every kind that the library has handed out and not yet
// released. Entry points check a handle here before touching it, so a
// closed (or never opened) handle fails with KPD_ESTATE instead of reading
// released memory. handle_add returns false when the host is out of memory.
bool handle_add(const void* h);
void handle_remove(const void* h);
bool handle_live(const void* h);

}  // namespace kpd
