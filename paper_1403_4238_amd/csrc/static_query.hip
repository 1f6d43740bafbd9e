// Device scratch of the allocation-free exemplar query
// (inpaint_find_exemplar_static): one file-scope device array per GPU, and
// its per-device address.
//
// In host code `scratch` names a host-side stand-in, not device memory; the
// device address comes from hipGetSymbolAddress, taken once per device (with
// that device current) by static_scratch_setup and kept in g_ptr.  Only that
// address is ever handed to kernels.
#include <mutex>

#include "inpaint_dev.h"

namespace inpaint {

namespace {

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_tried[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_tried[device]) {
        g_tried[device] = true;
        void *p = nullptr;
        g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (g_err[device] == hipSuccess) g_ptr[device] = p;
    }
    return g_err[device];
}

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace inpaint
