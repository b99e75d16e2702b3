// Device scratch of the entry point that allocates nothing
// (rtdm_multiply_noalloc): a file-scope static array that every GPU the
// library runs on holds from the first load of this code object until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it looks up the device address
// once per device, with that device current, and uses that address.
#include <mutex>

#include "internal.h"

namespace rtdm {

namespace {

static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

}  // namespace

double *static_scratch(int device)
{
    RT_CHECK(device >= 0 && device < kMaxDevices, RTDM_E_ARG, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        RT_HIP(hipGetDevice(&cur));
        RT_CHECK(cur == device, RTDM_E_STATE, "the static scratch is looked up with its device current");
        void *p = nullptr;
        RT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        RT_CHECK(p != nullptr, RTDM_E_HIP, "no device address for the static scratch");
        g_ptr[device] = static_cast<double *>(p);
    }
    return g_ptr[device];
}

}  // namespace rtdm
