// kpd_detect_layers for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the same detection over octaves and intra-octaves, with its
// workspace (layers, score maps, per-block counts) in a file-scope device
// array that every GPU the library runs on holds until the process ends.
//
// The array's name is a host-side stand-in in host code, not a device
// address: its address on each device is taken once with
// hipGetSymbolAddress (on the first call made with that device current)
// and only that address is handed to the kernels. Calls on one GPU share
// the array, so calls that overlap on one GPU race; the detection writes
// every workspace byte it reads before reading it, so nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/kpd.h"
#include "kpd_errors.h"

namespace {

constexpr size_t kStaticBytes = (size_t)KPD_STATIC_WORKSPACE;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticBytes];

std::mutex g_mu;
uint8_t* g_ptr[kMaxDevices] = {};

}  // namespace

extern "C" {

int kpd_detect_layers_static(const uint8_t* frame, size_t pitch_bytes, int width, int height, int fast_t,
                             int n_octaves, kpd_keypoint* out, uint32_t capacity, uint32_t* count, void* hip_stream)
{
    const size_t need = kpd_layers_bytes(width, height, n_octaves);
    if (need == 0) return KPD_EINVAL;   // kpd_layers_bytes set the message
    if (need > kStaticBytes)
        return kpd::api_fail(KPD_EINVAL, "the frame needs " + std::to_string(need) +
                                             " workspace bytes; the static workspace holds " +
                                             std::to_string(kStaticBytes));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers_static: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return kpd::api_fail(KPD_EINVAL, "device index out of range");
    uint8_t* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return kpd::api_hip_fail(e, "kpd_detect_layers_static: hipGetSymbolAddress");
            g_ptr[dev] = reinterpret_cast<uint8_t*>(p);
        }
        ws = g_ptr[dev];
    }
    return kpd_detect_layers(frame, pitch_bytes, width, height, fast_t, n_octaves, ws, kStaticBytes, out, capacity,
                             count, hip_stream);
}

}  // extern "C"
