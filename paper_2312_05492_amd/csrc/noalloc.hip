// noalloc.hip -- the library's static device workspace, for the entry point
// that allocates nothing (sz_decompress_noalloc).
//
// The workspace is a file-scope device array.  Each GPU holds its own copy,
// at its own address, from the time the library's code is loaded on it
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in): it asks the
// runtime for the device address once per device, at context creation, and
// uses that address from then on.
#include <map>
#include <mutex>

#include "dev_common.h"

namespace szi {

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void** ptr) {
    static std::mutex mu;
    static std::map<int, void*> addr;   // device -> address of its copy
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the caller makes it current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

// Host bytes to device memory through a kernel argument: no staging buffer
// and no host-to-device copy.
__global__ __launch_bounds__(256) void k_stage_words(uint32_t* dst, StageWords a) {
    for (uint32_t i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.w[i];
}

hipError_t launch_stage_words(uint32_t* dst, const StageWords& a, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stage_words, dim3(1), dim3(256), 0, st, dst, a);
    return hipGetLastError();
}

}  // namespace szi
