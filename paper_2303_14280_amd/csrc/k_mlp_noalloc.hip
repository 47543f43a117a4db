// The learned screener's loss gradient for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid allocation): the same
// kernels as snk_mlp_loss_grad, with their per-workgroup partial sums in a fixed device array
// instead of a buffer the library allocates.
#include "snk.h"
#include "snk_internal.h"

#include <cmath>
#include <mutex>

namespace snk {

const MlpNorm& mlp_norm(const snk_mlp* m);
const float* mlp_params(const snk_mlp* m);
int mlp_device(const snk_mlp* m);
void set_last_error(const char* msg);

namespace {

// One partial-sum record (kMlpParams gradients + the loss) per workgroup of 64 samples.
constexpr int64_t kNoAllocBlocks = kMlpNoAllocMaxSamples / 64;
constexpr int64_t kScratchFloats = kNoAllocBlocks * (kMlpParams + 1);   // 21.8 MB

// Each GPU holds its own copy of this array until the process ends.  In host code its name is
// not a device address: the address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_scratch[kMaxDevices] = {};

}  // namespace

// Looks up the device address of `scratch` on `device`, which must be current; once per device.
int mlp_scratch_init(int device)
{
    static_assert(kMlpNoAllocMaxSamples % 64 == 0, "whole workgroups of samples");
    if (device < 0 || device >= kMaxDevices) return SNK_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return SNK_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_last_error(hipGetErrorString(e));
        return SNK_E_DEVICE;
    }
    g_scratch[device] = static_cast<float*>(p);
    return SNK_OK;
}

}  // namespace snk

extern "C" int snk_mlp_loss_grad_noalloc(snk_mlp* m, const float* x, const float* target, int64_t n, float under,
                                         float* grads, void* stream)
{
    using namespace snk;
    if (!m || n <= 0 || !x || !target || !grads || !std::isfinite(under) || under <= 0.0f) {
        set_last_error("snk_mlp_loss_grad_noalloc: invalid argument");
        return SNK_E_ARG;
    }
    if (n > kMlpNoAllocMaxSamples) {
        set_last_error("snk_mlp_loss_grad_noalloc: more samples than the fixed scratch array holds "
                       "(at most 65536 per call)");
        return SNK_E_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SNK_E_DEVICE;
    if (dev != mlp_device(m)) {
        set_last_error("snk_mlp_loss_grad_noalloc: the network's device is not the current device");
        return SNK_E_ARG;
    }
    float* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ptr = dev < kMaxDevices ? g_scratch[dev] : nullptr;
    }
    if (!ptr) {
        // the network was made on this device (snk_mlp_create looks the array up there); a
        // context that reached this point without it is a library error
        set_last_error("snk_mlp_loss_grad_noalloc: scratch array not set up on this device");
        return SNK_E_DEVICE;
    }
    const hipError_t e = launch_mlp_grad(mlp_params(m), mlp_norm(m), x, target, nullptr, n, under, ptr, grads,
                                         (hipStream_t)stream);
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return SNK_E_DEVICE;
    }
    return SNK_OK;
}
