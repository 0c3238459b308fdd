// Device-resident scratch for the entry point that allocates nothing (lbm_residual_noalloc):
// one file-scope array per device, held until the process ends.  Host code never uses the
// array's name as an address (in host code it is only a stand-in for the device symbol):
// each device's address is looked up once, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm.h"
#include "lbm_kernels.h"

namespace lbm {

static __device__ __align__(256) unsigned char scratch[LBM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_addr[MAX_DEVICES];
bool g_looked_up[MAX_DEVICES];
hipError_t g_status[MAX_DEVICES];

}  // namespace

hipError_t static_scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_lock);
    if (g_looked_up[device]) return g_status[device];
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;   // the caller makes it current
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_addr[device] = e == hipSuccess ? ptr : nullptr;
    g_status[device] = e;
    g_looked_up[device] = true;
    return e;
}

void *static_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> guard(g_lock);
    return g_looked_up[device] ? g_addr[device] : nullptr;
}

}  // namespace lbm
