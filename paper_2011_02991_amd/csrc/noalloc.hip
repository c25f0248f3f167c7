// noalloc.hip -- the fixed device scratch of the entry point that allocates
// nothing (qng_energy_grad_dev_noalloc).
//
// The array below is the whole workspace of that entry point: registers,
// reduction partials, raw products and plan images all live in it.  Every GPU
// the library runs on holds its own copy of the array (at its own address)
// from module load until the process ends.  In host code the name `scratch`
// is only a host-side stand-in: its device address is looked up once per
// device with hipGetSymbolAddress (at qng_create, with the device current) and
// only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "noalloc.hpp"

namespace qng {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_mu;
std::vector<void *> g_ptr;   // device address of `scratch`, per device (nullptr: not looked up yet)
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((int)g_ptr.size() <= device) g_ptr.resize(device + 1, nullptr);
    if (g_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

void *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    return (device >= 0 && device < (int)g_ptr.size()) ? g_ptr[device] : nullptr;
}

}  // namespace qng
