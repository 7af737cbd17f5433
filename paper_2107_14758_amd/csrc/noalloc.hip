// Static device workspace for the allocation-free entry point (vsr_apply_operator_noalloc).
//
// The workspace is one file-scope device array.  Each GPU that loads the library holds its
// own copy at its own address until the process ends.  Host code never uses the array's
// name as a device address: the address is looked up with hipGetSymbolAddress once per
// device (with that device current) and kept here, and kernels receive it as an argument.
// Every call on a GPU shares that GPU's copy; calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "vsr_internal.h"

namespace vsr {

constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;   // 64 MiB
constexpr int kMaxDevices = 64;

}  // namespace vsr

static __device__ __align__(256) double scratch[vsr::kStaticWorkspaceBytes / sizeof(double)];

namespace vsr {
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t static_workspace_bytes() { return kStaticWorkspaceBytes; }

void *static_workspace(size_t bytes) {
    if (bytes > kStaticWorkspaceBytes)
        throw Error(VSR_EINVAL, "the allocation-free call needs " + std::to_string(bytes) +
                                    " bytes of workspace; its static workspace holds " +
                                    std::to_string(kStaticWorkspaceBytes));
    int dev = -1;
    VSR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error(VSR_EINVAL, "device ordinal out of range for the static workspace");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        VSR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(VSR_EDEVICE, "hipGetSymbolAddress returned no address for the static workspace");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace vsr
