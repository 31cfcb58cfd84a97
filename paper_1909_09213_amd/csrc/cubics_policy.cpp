// Learned branching policy objects: parameters resident on the device, and
// the host side of the network's forward / gradient / Adam kernels.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/cubics.h"
#include "cubics_internal.h"

namespace cubics {
hipError_t launch_policy_round(const float *theta, uint16_t *w1b, uint16_t *w2b, hipStream_t st);
hipError_t launch_mlp_forward(const PolicyDev &P, const float *X, int ld, long long N, float *y, hipStream_t st);
hipError_t launch_mlp_grad(const PolicyDev &P, const float *X, int ld, const float *T, int ldt, long long N,
                           float *grad, float *loss, hipStream_t st);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, float lr, int step, hipStream_t st);
hipError_t launch_fill(float *p, int n, float v, hipStream_t st);
}  // namespace cubics

using namespace cubics;

int cubics_set_error(int code, const char *msg);
hipStream_t cubics_ctx_stream(const cubics_ctx *ctx);
int cubics_ctx_device(const cubics_ctx *ctx);

struct cubics_policy {
    const cubics_ctx *ctx = nullptr;
    void *mem = nullptr;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    uint16_t *w1b = nullptr, *w2b = nullptr;
    PolicyDev dev;
};

int policy_fill(const cubics_policy *pol, PolicyDev *out) {
    *out = pol->dev;
    return 0;
}

#define PCHK(expr)                                                                 \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) return cubics_set_error(CUBICS_EDEVICE, #expr " failed"); \
    } while (0)

extern "C" int cubics_policy_create(cubics_ctx *ctx, const float *theta, cubics_policy **out) {
    if (!out) return cubics_set_error(CUBICS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || !theta) return cubics_set_error(CUBICS_EINVAL, "ctx or theta is NULL");
    PCHK(hipSetDevice(cubics_ctx_device(ctx)));
    cubics_policy *p = new cubics_policy();
    p->ctx = ctx;
    const size_t nf = 4 * 512 + 64;  // theta, m, v, grad (512 each), loss
    const size_t bytes = nf * 4 + (64 * 16 + 64) * 2;
    if (hipMalloc(&p->mem, bytes) != hipSuccess) {
        delete p;
        return cubics_set_error(CUBICS_ENOMEM, "policy allocation failed");
    }
    float *f = (float *)p->mem;
    p->theta = f;
    p->m = f + 512;
    p->v = f + 1024;
    p->grad = f + 1536;
    p->loss = f + 2048;
    p->w1b = (uint16_t *)(f + nf);
    p->w2b = p->w1b + 64 * 16;
    p->dev.w1 = p->w1b;
    p->dev.b1 = p->theta + OFF_B1;
    p->dev.w2 = p->w2b;
    p->dev.b2 = p->theta + OFF_B2;
    hipStream_t st = cubics_ctx_stream(ctx);
    hipError_t e = hipMemcpyAsync(p->theta, theta, POLICY_NP * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_fill(p->m, 1024, 0.f, st);  // m and v
    if (e == hipSuccess) e = launch_policy_round(p->theta, p->w1b, p->w2b, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(p->mem);
        delete p;
        return cubics_set_error(CUBICS_EDEVICE, "policy upload failed");
    }
    *out = p;
    return CUBICS_OK;
}

extern "C" void cubics_policy_free(cubics_policy *p) {
    if (!p) return;
    if (p->mem) (void)hipFree(p->mem);
    delete p;
}

extern "C" int cubics_policy_get(const cubics_policy *p, float *theta) {
    if (!p || !theta) return cubics_set_error(CUBICS_EINVAL, "NULL argument");
    hipStream_t st = cubics_ctx_stream(p->ctx);
    PCHK(hipMemcpyAsync(theta, p->theta, POLICY_NP * 4, hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    return CUBICS_OK;
}

extern "C" int cubics_policy_set(cubics_policy *p, const float *theta) {
    if (!p || !theta) return cubics_set_error(CUBICS_EINVAL, "NULL argument");
    hipStream_t st = cubics_ctx_stream(p->ctx);
    PCHK(hipMemcpyAsync(p->theta, theta, POLICY_NP * 4, hipMemcpyHostToDevice, st));
    PCHK(launch_fill(p->m, 1024, 0.f, st));
    PCHK(launch_policy_round(p->theta, p->w1b, p->w2b, st));
    PCHK(hipStreamSynchronize(st));
    return CUBICS_OK;
}

extern "C" int cubics_mlp_forward(const cubics_policy *p, const float *x_dev, int32_t ld, int64_t N, float *y_dev) {
    if (!p || (N > 0 && (!x_dev || !y_dev)) || N < 0 || ld < POLICY_F)
        return cubics_set_error(CUBICS_EINVAL, "bad arguments");
    if (N == 0) return CUBICS_OK;
    hipStream_t st = cubics_ctx_stream(p->ctx);
    PCHK(launch_mlp_forward(p->dev, x_dev, ld, N, y_dev, st));
    PCHK(hipStreamSynchronize(st));
    return CUBICS_OK;
}

extern "C" int cubics_mlp_grad(const cubics_policy *p, const float *x_dev, int32_t ld, const float *t_dev,
                               int32_t ldt, int64_t N, float *grad_dev, float *loss_dev) {
    if (!p || N < 1 || !x_dev || !t_dev || ld < POLICY_F || ldt < 1)
        return cubics_set_error(CUBICS_EINVAL, "bad arguments");
    hipStream_t st = cubics_ctx_stream(p->ctx);
    float *g = grad_dev ? grad_dev : p->grad;
    float *l = loss_dev ? loss_dev : p->loss;
    PCHK(launch_mlp_grad(p->dev, x_dev, ld, t_dev, ldt, N, g, l, st));
    PCHK(hipStreamSynchronize(st));
    return CUBICS_OK;
}

extern "C" int cubics_mlp_train_step(cubics_policy *p, const float *x_dev, int32_t ld, const float *t_dev,
                                     int32_t ldt, int64_t N, float lr, int32_t step, float *loss_host) {
    if (!p || N < 1 || !x_dev || !t_dev || step < 1 || ld < POLICY_F || ldt < 1)
        return cubics_set_error(CUBICS_EINVAL, "bad arguments");
    hipStream_t st = cubics_ctx_stream(p->ctx);
    PCHK(launch_mlp_grad(p->dev, x_dev, ld, t_dev, ldt, N, p->grad, p->loss, st));
    PCHK(launch_adam(p->theta, p->m, p->v, p->grad, lr, step, st));
    PCHK(launch_policy_round(p->theta, p->w1b, p->w2b, st));
    if (loss_host) PCHK(hipMemcpyAsync(loss_host, p->loss, 4, hipMemcpyDeviceToHost, st));
    PCHK(hipStreamSynchronize(st));
    return CUBICS_OK;
}
