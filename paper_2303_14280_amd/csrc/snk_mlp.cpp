// C ABI of the learned block screener's network (declared in snk.h).
#include "snk.h"
#include "snk_internal.h"

#include <cmath>
#include <cstring>
#include <string>

using namespace snk;

struct snk_mlp {
    int device = 0;
    float* d_params = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_part = nullptr;
    int64_t part_cap = 0;
    MlpNorm norm{};
    float lo[16], hi[16];
    float margin = 0.0f;
    int has_range = 0;
};

namespace snk {
int mlp_scratch_init(int device);
// read by the screening host code
const MlpNorm& mlp_norm(const snk_mlp* m) { return m->norm; }
const float* mlp_params(const snk_mlp* m) { return m->d_params; }
int mlp_device(const snk_mlp* m) { return m->device; }
void mlp_range(const snk_mlp* m, float* lo, float* hi, float* margin, int* has_range)
{
    std::memcpy(lo, m->lo, sizeof(m->lo));
    std::memcpy(hi, m->hi, sizeof(m->hi));
    *margin = m->margin;
    *has_range = m->has_range;
}
}  // namespace snk

extern "C" {

int snk_mlp_nparams(void) { return kMlpParams; }

int snk_mlp_create(int device, snk_mlp** out)
{
    if (!out) return SNK_E_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return SNK_E_DEVICE;
    // the device address of the fixed scratch array of snk_mlp_loss_grad_noalloc, once per device
    if (mlp_scratch_init(device) != SNK_OK) return SNK_E_DEVICE;
    snk_mlp* m = new (std::nothrow) snk_mlp();
    if (!m) return SNK_E_NOMEM;
    m->device = device;
    const size_t bytes = (size_t)kMlpParams * sizeof(float);
    if (hipMalloc((void**)&m->d_params, bytes) != hipSuccess || hipMalloc((void**)&m->d_m, bytes) != hipSuccess ||
        hipMalloc((void**)&m->d_v, bytes) != hipSuccess) {
        snk_mlp_destroy(m);
        return SNK_E_NOMEM;
    }
    if (hipMemset(m->d_params, 0, bytes) != hipSuccess || hipMemset(m->d_m, 0, bytes) != hipSuccess ||
        hipMemset(m->d_v, 0, bytes) != hipSuccess) {
        snk_mlp_destroy(m);
        return SNK_E_DEVICE;
    }
    for (int j = 0; j < 16; ++j) {
        m->norm.mean[j] = 0.0f;
        m->norm.inv_std[j] = 1.0f;
        m->lo[j] = -INFINITY;
        m->hi[j] = INFINITY;
    }
    *out = m;
    return SNK_OK;
}

void snk_mlp_destroy(snk_mlp* m)
{
    if (!m) return;
    (void)hipFree(m->d_params);
    (void)hipFree(m->d_m);
    (void)hipFree(m->d_v);
    (void)hipFree(m->d_part);
    delete m;
}

int snk_mlp_set_params(snk_mlp* m, const float* params)
{
    if (!m || !params) return SNK_E_ARG;
    for (int i = 0; i < kMlpParams; ++i)
        if (!std::isfinite(params[i])) return SNK_E_ARG;
    if (hipMemcpy(m->d_params, params, (size_t)kMlpParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return SNK_E_DEVICE;
    return SNK_OK;
}

int snk_mlp_get_params(const snk_mlp* m, float* params)
{
    if (!m || !params) return SNK_E_ARG;
    if (hipMemcpy(params, m->d_params, (size_t)kMlpParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return SNK_E_DEVICE;
    return SNK_OK;
}

int snk_mlp_set_normalisation(snk_mlp* m, const float* mean, const float* std)
{
    if (!m || !mean || !std) return SNK_E_ARG;
    for (int j = 0; j < 16; ++j) {
        if (!std::isfinite(mean[j]) || !std::isfinite(std[j]) || !(std[j] > 0.0f)) return SNK_E_ARG;
        m->norm.mean[j] = mean[j];
        m->norm.inv_std[j] = 1.0f / std[j];
    }
    return SNK_OK;
}

int snk_mlp_set_range(snk_mlp* m, const float* lo, const float* hi, float margin)
{
    if (!m || !lo || !hi || !std::isfinite(margin) || margin < 0.0f) return SNK_E_ARG;
    for (int j = 0; j < 16; ++j) {
        if (std::isnan(lo[j]) || std::isnan(hi[j]) || lo[j] > hi[j]) return SNK_E_ARG;
        m->lo[j] = lo[j];
        m->hi[j] = hi[j];
    }
    m->margin = margin;
    m->has_range = 1;
    return SNK_OK;
}

int snk_mlp_forward(const snk_mlp* m, const float* x, int64_t n, float* y, int bf16, void* stream)
{
    if (!m || n < 0) return SNK_E_ARG;
    if (n == 0) return SNK_OK;
    if (!x || !y) return SNK_E_ARG;
    return launch_mlp_forward(m->d_params, m->norm, x, n, y, bf16 != 0, (hipStream_t)stream) == hipSuccess
               ? SNK_OK
               : SNK_E_DEVICE;
}

namespace {
int ensure_part(snk_mlp* m, int64_t n)
{
    const int64_t nblk = mlp_grad_blocks(n);
    if (nblk > m->part_cap) {
        (void)hipFree(m->d_part);
        m->d_part = nullptr;
        if (hipMalloc((void**)&m->d_part, (size_t)nblk * (kMlpParams + 1) * sizeof(float)) != hipSuccess) {
            m->part_cap = 0;
            return SNK_E_NOMEM;
        }
        m->part_cap = nblk;
    }
    return SNK_OK;
}
}  // namespace

int snk_mlp_backward(snk_mlp* m, const float* x, const float* dy, int64_t n, float* grads, void* stream)
{
    if (!m || n <= 0 || !x || !dy || !grads) return SNK_E_ARG;
    const int rc = ensure_part(m, n);
    if (rc) return rc;
    return launch_mlp_grad(m->d_params, m->norm, x, nullptr, dy, n, 1.0f, m->d_part, grads, (hipStream_t)stream) ==
                   hipSuccess
               ? SNK_OK
               : SNK_E_DEVICE;
}

int snk_mlp_loss_grad(snk_mlp* m, const float* x, const float* target, int64_t n, float under, float* grads,
                      void* stream)
{
    if (!m || n <= 0 || !x || !target || !grads || !std::isfinite(under) || under <= 0.0f) return SNK_E_ARG;
    const int64_t nblk = mlp_grad_blocks(n);
    if (nblk > m->part_cap) {
        (void)hipFree(m->d_part);
        m->d_part = nullptr;
        if (hipMalloc((void**)&m->d_part, (size_t)nblk * (kMlpParams + 1) * sizeof(float)) != hipSuccess) {
            m->part_cap = 0;
            return SNK_E_NOMEM;
        }
        m->part_cap = nblk;
    }
    return launch_mlp_grad(m->d_params, m->norm, x, target, nullptr, n, under, m->d_part, grads, (hipStream_t)stream) ==
                   hipSuccess
               ? SNK_OK
               : SNK_E_DEVICE;
}

int snk_mlp_adam_step(snk_mlp* m, const float* grads, float lr, int t, void* stream)
{
    if (!m || !grads || t < 1 || !std::isfinite(lr)) return SNK_E_ARG;
    return launch_mlp_adam(m->d_params, m->d_m, m->d_v, grads, lr, t, (hipStream_t)stream) == hipSuccess
               ? SNK_OK
               : SNK_E_DEVICE;
}

}  // extern "C"
