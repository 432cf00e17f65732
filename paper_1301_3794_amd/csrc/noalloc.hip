// Scratch memory of the entry point that allocates nothing
// (dm_solve_pcg_noalloc): a file-scope device array, one copy per GPU the
// library runs on, held until the process ends.
//
// In host code the array's name is only a host-side stand-in, never a device
// address: its device address is looked up once per device, with that device
// current, by hipGetSymbolAddress (at operator build), and only that address
// is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "dm.h"
#include "op.h"

namespace dm {

static_assert(DM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) double scratch[DM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

std::mutex g_mu;
std::vector<double *> g_ptr;   // device -> address of `scratch` on it (NULL: not looked up)

}  // namespace

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0) throw DmError{DM_EINVAL, "bad device"};
    if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
    if (g_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw DmError{DM_EHIP, std::string("no-allocation scratch: hipGetSymbolAddress failed: ") +
                                   hipGetErrorString(e)};
    g_ptr[device] = static_cast<double *>(ptr);
}

double *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0 || device >= (int)g_ptr.size()) return nullptr;
    return g_ptr[device];
}

}  // namespace dm
