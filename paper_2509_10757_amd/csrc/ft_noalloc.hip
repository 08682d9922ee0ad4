// Fixed device scratch of the allocation-free search entry point.
//
// ft_search_local_points_noalloc runs the same kernels as
// ft_search_local_points, but takes the view's workspace (cell offsets, cell
// records, per-map-point candidates, claim table) from one file-scope device
// array instead of a context's arena, so a caller that cannot allocate device
// memory (code under graph capture, serving loops that forbid it) can still
// search.  Every GPU the library runs on holds its own copy of the array for
// the life of the process.  The host-side name of the array is not a device
// address: host code uses only the address hipGetSymbolAddress returns for the
// current device, fetched once per device and kept.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "ft_internal.h"

namespace ft {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};
bool g_gfx950[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, char **out, bool *gfx950)
{
    *out = nullptr;
    *gfx950 = false;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        // `device` is current: the symbol resolves to that device's copy
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_gfx950[device] = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        g_ptr[device] = static_cast<char *>(p);
    }
    *out = g_ptr[device];
    *gfx950 = g_gfx950[device];
    return hipSuccess;
}

}  // namespace ft
