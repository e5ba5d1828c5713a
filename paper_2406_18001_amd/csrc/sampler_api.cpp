// Host side of the learned sampler's C-ABI: model lifetime, parameter
// transfer, inference, gradients, training and stand-alone selection.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.hpp"
#include "sampler.hpp"

using namespace kdcd;

namespace {

const int kMaxTrainBlocks = (SMP_MAX_BATCH + 127) / 128;

kdcd_status sync_status(hipStream_t st)
{
    return hipStreamSynchronize(st) == hipSuccess ? KDCD_OK : KDCD_ERR_HIP;
}

bool same_device(const kdcd_sampler *m)
{
    int d = -1;
    return hipGetDevice(&d) == hipSuccess && d == m->device;
}

}  // namespace

extern "C" {

kdcd_status kdcd_sampler_create(kdcd_sampler **out, uint64_t seed)
{
    if (!out) return KDCD_ERR_INVALID_ARG;
    *out = nullptr;
    auto *m = new kdcd_sampler();
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return KDCD_ERR_HIP;
    }
    const size_t np = sizeof(float) * SMP_NP;
    bool ok = hipMalloc(&m->params, np) == hipSuccess && hipMalloc(&m->mom, np) == hipSuccess &&
              hipMalloc(&m->vel, np) == hipSuccess &&
              hipMalloc(&m->gpart, np * (size_t)kMaxTrainBlocks) == hipSuccess &&
              hipMalloc(&m->lpart, sizeof(float) * kMaxTrainBlocks) == hipSuccess &&
              hipMalloc(&m->lacc, sizeof(double)) == hipSuccess;
    if (!ok) {
        kdcd_sampler_destroy(m);
        return KDCD_ERR_ALLOC;
    }
    std::vector<float> h(SMP_NP), z(SMP_NP, 0.0f);
    sampler_init_params(h.data(), seed);
    ok = hipMemcpy(m->params, h.data(), np, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->mom, z.data(), np, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(m->vel, z.data(), np, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        kdcd_sampler_destroy(m);
        return KDCD_ERR_HIP;
    }
    *out = m;
    return KDCD_OK;
}

void kdcd_sampler_destroy(kdcd_sampler *m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(m->params);
    (void)hipFree(m->mom);
    (void)hipFree(m->vel);
    (void)hipFree(m->gpart);
    (void)hipFree(m->lpart);
    (void)hipFree(m->lacc);
    delete m;
}

kdcd_status kdcd_sampler_get_params(const kdcd_sampler *m, float *params, kdcd_stream stream)
{
    if (!m || !params) return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    KDCD_HIP_TRY(hipMemcpyAsync(params, m->params, sizeof(float) * SMP_NP,
                                hipMemcpyDeviceToDevice, st));
    return sync_status(st);
}

kdcd_status kdcd_sampler_set_params(kdcd_sampler *m, const float *params, kdcd_stream stream)
{
    if (!m || !params) return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    std::vector<float> z(SMP_NP, 0.0f);
    KDCD_HIP_TRY(hipMemcpyAsync(m->params, params, sizeof(float) * SMP_NP,
                                hipMemcpyDeviceToDevice, st));
    KDCD_HIP_TRY(hipMemcpyAsync(m->mom, z.data(), sizeof(float) * SMP_NP, hipMemcpyHostToDevice, st));
    KDCD_HIP_TRY(hipMemcpyAsync(m->vel, z.data(), sizeof(float) * SMP_NP, hipMemcpyHostToDevice, st));
    m->step = 0;
    return sync_status(st);
}

kdcd_status kdcd_sampler_forward(const kdcd_sampler *m, const float *x, int64_t n, float *out,
                                 kdcd_stream stream)
{
    if (!m || !x || !out || n < 0) return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    if (n == 0) return KDCD_OK;
    KDCD_HIP_TRY(launch_mlp_forward(m->params, x, n, out, (hipStream_t)stream));
    return KDCD_OK;
}

kdcd_status kdcd_sampler_grad(const kdcd_sampler *m, const float *x, const float *t, int64_t n,
                              float *grad, float *loss, kdcd_stream stream)
{
    if (!m || !x || !t || !grad || !loss || n < 1 || n > SMP_MAX_BATCH) return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    TrainArgs a{};
    a.params = m->params;
    a.mom = m->mom;
    a.vel = m->vel;
    a.x = x;
    a.t = t;
    a.n = n;
    a.gpart = m->gpart;
    a.lpart = m->lpart;
    a.adam = 0;
    a.grad = grad;
    a.loss = loss;
    KDCD_HIP_TRY(launch_train_step(a, (hipStream_t)stream));
    return KDCD_OK;
}

kdcd_status kdcd_sampler_train(kdcd_sampler *m, const float *x, const float *t, int64_t n,
                               int32_t batch, int32_t epochs, float lr, float *epoch_loss,
                               kdcd_stream stream)
{
    if (!m || !x || !t || n < 1 || batch < 1 || batch > SMP_MAX_BATCH || epochs < 0 ||
        !std::isfinite(lr) || lr < 0.0f)
        return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    for (int32_t e = 0; e < epochs; ++e) {
        KDCD_HIP_TRY(launch_lacc(m->lacc, nullptr, false, st));
        for (int64_t o = 0; o < n; o += batch) {
            const int64_t nb = std::min<int64_t>(batch, n - o);
            m->step += 1;
            TrainArgs a{};
            a.params = m->params;
            a.mom = m->mom;
            a.vel = m->vel;
            a.x = x + 4 * o;
            a.t = t + o;
            a.n = nb;
            a.gpart = m->gpart;
            a.lpart = m->lpart;
            a.adam = 1;
            a.lr = lr;
            a.bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
            a.bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
            a.lacc = m->lacc;
            a.lweight = (double)nb / (double)n;
            KDCD_HIP_TRY(launch_train_step(a, st));
        }
        if (epoch_loss) KDCD_HIP_TRY(launch_lacc(m->lacc, epoch_loss + e, true, st));
    }
    return sync_status(st);
}

kdcd_status kdcd_sampler_keys(const kdcd_sampler *m, const float *x, int64_t n, double tau,
                              uint64_t seed, int64_t outer, float *keys, kdcd_stream stream)
{
    if (!m || !x || !keys || n < 0 || n >= ((int64_t)1 << 31) || !(tau > 0.0) ||
        !std::isfinite(tau) || outer < 0 || outer > (int64_t)0xFFFFFFFF)
        return KDCD_ERR_INVALID_ARG;
    if (!same_device(m)) return KDCD_ERR_INVALID_ARG;
    if (n == 0) return KDCD_OK;
    KDCD_HIP_TRY(launch_mlp_keys(m->params, x, n, tau, (uint32_t)outer, seed, keys,
                                 (hipStream_t)stream));
    return KDCD_OK;
}

kdcd_status kdcd_sampler_select(const float *keys, int64_t m, int32_t s, double epsilon,
                                uint64_t seed, int64_t outer, int32_t *S, kdcd_stream stream)
{
    if (!keys || !S || m < 1 || m >= ((int64_t)1 << 31) || s < 1 || s > kMaxSB || s > m ||
        !(epsilon >= 0.0 && epsilon <= 1.0) || outer < 0 || outer > (int64_t)0xFFFFFFFF)
        return KDCD_ERR_INVALID_ARG;
    const hipStream_t st = (hipStream_t)stream;
    void *ws = nullptr;
    const size_t bytes = select_workspace_bytes(m) + 256;
    if (hipMallocAsync(&ws, bytes, st) != hipSuccess) return KDCD_ERR_ALLOC;
    int32_t *status = static_cast<int32_t *>(ws);
    SelectArgs a{};
    a.ws = select_workspace(static_cast<char *>(ws) + 256, m);
    a.m = m;
    a.ns = s;
    a.topk = true;
    a.epsilon = epsilon;
    a.seed = seed;
    a.outer = (uint32_t)outer;
    a.keys = keys;
    a.S = S;
    a.status = status;
    kdcd_status rc = KDCD_OK;
    int32_t hs = 0;
    if (launch_fill_i32(status, 0, 1, st) != hipSuccess || launch_select_reset(a.ws, st) != hipSuccess ||
        launch_select(a, st) != hipSuccess ||
        hipMemcpyAsync(&hs, status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = KDCD_ERR_HIP;
    (void)hipFreeAsync(ws, st);
    if (hipStreamSynchronize(st) != hipSuccess) rc = KDCD_ERR_HIP;
    if (rc == KDCD_OK) rc = (kdcd_status)hs;
    return rc;
}

}  // extern "C"
