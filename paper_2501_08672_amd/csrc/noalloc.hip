// Device scratch memory for the entry point that takes no workspace argument
// (gsl_render_bwd_noalloc): one file-scope array per GPU, created with the
// code object and held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it asks the runtime for the array's device address once per
// device, with that device current, and hands that address to the kernels.
#include <mutex>

#include "common.hpp"

static __device__ __align__(256) unsigned char scratch[gsl::kStaticScratchBytes];

namespace gsl {

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t static_scratch_address(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace gsl
