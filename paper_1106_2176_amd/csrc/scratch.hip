// scratch.hip -- the static device array behind fmm_evaluate_noalloc.
//
// A file-scope __device__ array of FMM_NOALLOC_SCRATCH_BYTES: every device
// the library runs on holds its own copy from module load until the process
// ends, so an evaluation that takes its buffers from it needs no allocation.
// In host code the array's name is only a host-side stand-in for the symbol;
// the device address of each device's copy comes from hipGetSymbolAddress,
// looked up once per device (with that device current) and kept.
#include <map>
#include <mutex>

#include "kernels.hpp"

namespace fmm {

static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void **ptr) {
    static std::mutex mu;
    static std::map<int, void *> addr;  // device -> address of its copy
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        it = addr.emplace(dev, p).first;
    }
    *ptr = it->second;
    return hipSuccess;
}

}  // namespace fmm
