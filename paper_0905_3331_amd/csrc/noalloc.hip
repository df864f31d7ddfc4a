// noalloc.hip -- the fixed device work space of the allocation-free operator
// entry point (tmq_apply_Qhat_noalloc_dev).
//
// The array `scratch` below is part of the library's code object: every GPU
// the library runs on holds its own copy, at its own address, from the load
// of the code object until the process ends.  In host code the array's name
// is only a host-side stand-in, so host code never passes it to a kernel or a
// copy: the address of a device's copy is looked up once per device with
// hipGetSymbolAddress (with that device current, from tmq_lattice_create) and
// that address is what the entry point hands to its kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tmq.h"
#include "kernels.h"

namespace tmq {

static_assert(TMQ_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");
static __device__ __align__(256) unsigned char scratch[TMQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};
}  // namespace

// Look up the current device's copy of `scratch` (once per device; device must
// be the current one).  Returns the lookup's status.
hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_err[device] = e;
        g_done[device] = true;
    }
    return g_err[device];
}

// The device address of `device`'s copy (nullptr if the lookup has not run or failed).
void *noalloc_scratch(int device, size_t *bytes)
{
    if (bytes) *bytes = TMQ_NOALLOC_SCRATCH_BYTES;
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_done[device] && g_err[device] == hipSuccess ? g_ptr[device] : nullptr;
}

}  // namespace tmq
