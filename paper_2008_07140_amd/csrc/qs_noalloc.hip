// Reduction scratch that needs no allocation: one static device array per
// GPU the library runs on, for qs_probabilities_noalloc (callers that cannot
// allocate device memory, e.g. under HIP graph capture).
#include <hip/hip_runtime.h>

#include <mutex>

#include "qs_internal.h"

namespace qs {

namespace {

// The largest scratch any PMEASURE reduction asks for: reduce_scratch_doubles
// with 1024 bins (8 MiB + 512 B), the same size a state allocates for itself.
constexpr size_t kScratchDoubles = QS_NOALLOC_SCRATCH_BYTES / sizeof(double);

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device (set once)

}  // namespace

size_t noalloc_scratch_doubles() { return kScratchDoubles; }

hipError_t noalloc_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        // the array's name is a host-side stand-in: its device address on the
        // current device comes from the runtime, once per device
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace qs
