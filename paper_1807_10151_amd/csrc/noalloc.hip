// Device scratch of the allocation-free backprojection entry point
// (sp_backproject_noalloc): one statically sized array per GPU, in place of
// the buffers the context would allocate.  Its device address is looked up
// once per device, with that device current; host code never passes the
// array's own name to a kernel (on the host it only stands for the symbol).
#include <mutex>

#include "sp_internal.h"

namespace sp {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::once_flag g_once[MAX_DEVICES];
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::call_once(g_once[device], [device]() {
        void* p = nullptr;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
    });
    *ptr = g_ptr[device];
    return g_err[device];
}

}  // namespace sp
