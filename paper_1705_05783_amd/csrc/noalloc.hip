// Allocation-free variant of the learned basis' matrix-core inference.
//
// cams_cnn_forward_bf16 takes a caller workspace for the bfloat16 copy of
// the network's weights.  Callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that forbid allocation) use
// cams_cnn_forward_bf16_noalloc instead: the same kernels, with that
// workspace in a file-scope device array of fixed size.  Each GPU the
// library runs on holds one copy of the array until the process ends; its
// address on a device is looked up once (hipGetSymbolAddress, with that
// device current) and kept, and only that address is ever passed to a
// kernel.
#include <mutex>

#include "cams_internal.h"

namespace {

constexpr size_t kScratchBytes = 512 * 1024;   // >= the network's bfloat16 weights and FP32 biases
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t cams_cnn_noalloc_scratch_bytes(void) { return kScratchBytes; }

cams_status cams_cnn_forward_bf16_noalloc(void *stream, const float *params, const float *feat, int32_t batch,
                                          float *phi)
{
    if (!params || !feat || !phi || batch <= 0) return CAMS_E_ARG;
    if (cams::cnn_bf16_bytes() > kScratchBytes) return CAMS_E_NOMEM;   // the network outgrew the array
    void *ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return CAMS_E_DEVICE;
    cams::cnn_forward_bf16((hipStream_t)stream, params, feat, batch, ws, phi);
    return hipGetLastError() == hipSuccess ? CAMS_OK : CAMS_E_DEVICE;
}

}  // extern "C"
