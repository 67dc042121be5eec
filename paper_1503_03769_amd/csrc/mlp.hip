// libpphd: C ABI of the learned birth proposal (include/pphd_mlp.h) over the
// kernels in mlp_kernels.h.  Every device array lives in the caller's
// workspace, carved here in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/pphd_mlp.h"
#include "mlp_internal.h"
#include "mlp_kernels.h"

using namespace pphd;
using namespace pphd::mlp;

namespace {

constexpr int LOSS_CHUNK = 1024;  // training steps whose losses are staged at once

pphd_status err(pphd_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
pphd_status err(pphd_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(s, buf);
}

#define MLP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return err(PPHD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define MLP_LAUNCHED(name)                                                                   \
    do {                                                                                     \
        hipError_t e_ = hipGetLastError();                                                   \
        if (e_ != hipSuccess) return err(PPHD_EDEVICE, "%s launch failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

struct Carve {
    size_t off = 0;
    template <typename P>
    P* take(char* base, size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

bool config_ok(const pphd_mlp_config* c, const char** why)
{
    if (!c) { *why = "config is NULL"; return false; }
    if (c->batch < TS || c->batch > 65536 || c->batch % TS) { *why = "batch must be a multiple of 64 in [64, 65536]"; return false; }
    if (c->dataset < c->batch || c->dataset % c->batch) { *why = "dataset must be a positive multiple of batch"; return false; }
    if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) || !(c->eps > 0)) {
        *why = "Adam parameters out of range";
        return false;
    }
    return true;
}

Norm norm_of(const pphd_model& m, uint64_t seed)
{
    Norm n;
    std::memset(&n, 0, sizeof n);
    n.sx = m.sensor_x;
    n.sy = m.sensor_y;
    n.cx = 0.5 * (m.region[0] + m.region[1]);
    n.cy = 0.5 * (m.region[2] + m.region[3]);
    n.hx = 0.5 * (m.region[1] - m.region[0]);
    n.hy = 0.5 * (m.region[3] - m.region[2]);
    n.sv = m.birth_sigma_v;
    n.log_scale_sum = std::log(n.hx) + std::log(n.hy) + 2.0 * std::log(n.sv);
    n.reg0 = m.region[0];
    n.reg1 = m.region[1];
    n.reg2 = m.region[2];
    n.reg3 = m.region[3];
    n.sigma_r = m.sigma_r;
    n.sigma_th = m.sigma_theta;
    n.key0 = (uint32_t)seed;
    n.key1 = (uint32_t)(seed >> 32);
    return n;
}

}  // namespace

struct pphd_mlp {
    pphd_model model;
    pphd_mlp_config cfg;
    hipStream_t stream = nullptr;
    uint64_t seed = 0;
    Norm nrm;
    float *theta = nullptr, *am = nullptr, *av = nullptr, *grad = nullptr;
    uint16_t *Wt2 = nullptr, *Wi2 = nullptr, *Wt3 = nullptr, *Wi3 = nullptr, *Wt4 = nullptr, *Wi4 = nullptr;
    float *dz = nullptr, *dx = nullptr;  // dataset
    float *bz = nullptr, *bx = nullptr;  // one explicit batch
    float* part = nullptr;
    double* ploss = nullptr;
    float* lossbuf = nullptr;
    double* zin = nullptr;
    float* out = nullptr;
    int64_t t = 0;  // Adam steps since the last parameter reset

    Net net() const { return Net{ theta, Wt2, Wi2, Wt3, Wi3, Wt4, Wi4 }; }
};

namespace {

size_t carve(pphd_mlp* h, char* base, const pphd_mlp_config& c)
{
    Carve L;
    const size_t B = (size_t)c.batch, D = (size_t)c.dataset, tiles = B / TS;
    // the BF16 copies first: their padding must read as zero
    h->Wt2 = L.take<uint16_t>(base, H * H * 2);
    h->Wi2 = L.take<uint16_t>(base, H * H * 2);
    h->Wt3 = L.take<uint16_t>(base, H * H * 2);
    h->Wi3 = L.take<uint16_t>(base, H * H * 2);
    h->Wt4 = L.take<uint16_t>(base, NOP * H * 2);
    h->Wi4 = L.take<uint16_t>(base, H * NOP * 2);
    const size_t weights_end = L.off;
    h->theta = L.take<float>(base, P_ALL * 4 + 64);
    h->am = L.take<float>(base, P_ALL * 4);
    h->av = L.take<float>(base, P_ALL * 4);
    h->grad = L.take<float>(base, P_ALL * 4);
    h->dz = L.take<float>(base, D * 2 * 4);
    h->dx = L.take<float>(base, D * 4 * 4);
    h->bz = L.take<float>(base, B * 2 * 4);
    h->bx = L.take<float>(base, B * 4 * 4);
    h->part = L.take<float>(base, tiles * P_ALL * 4);
    h->ploss = L.take<double>(base, tiles * 8);
    h->lossbuf = L.take<float>(base, LOSS_CHUNK * 4);
    h->zin = L.take<double>(base, B * 2 * 8);
    h->out = L.take<float>(base, B * NO * 4);
    (void)weights_end;
    return (L.off + 255) & ~(size_t)255;
}

pphd_status reduce(pphd_mlp* h, int mode, int ntiles, double inv_n, float* loss_out)
{
    const int t = (int)std::min<int64_t>(h->t, 1 << 30);
    Adam ad;
    ad.lr = (float)h->cfg.lr;
    ad.beta1 = (float)h->cfg.beta1;
    ad.beta2 = (float)h->cfg.beta2;
    ad.eps = (float)h->cfg.eps;
    ad.bc1 = (float)(1.0 / (1.0 - std::pow(h->cfg.beta1, (double)std::max(t, 1))));
    ad.bc2 = (float)(1.0 / (1.0 - std::pow(h->cfg.beta2, (double)std::max(t, 1))));
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P_ALL + RP - 1) / RP), dim3(NTHR), 0, h->stream, mode, h->part,
                       h->ploss, ntiles, inv_n, h->theta, h->am, h->av, h->grad, ad, h->Wt2, h->Wi2, h->Wt3,
                       h->Wi3, h->Wt4, h->Wi4, loss_out);
    MLP_LAUNCHED("k_mlp_reduce");
    return PPHD_OK;
}

pphd_status train_tiles(pphd_mlp* h, const float* z, const float* x, int64_t base, int64_t D, int n)
{
    const int tiles = (n + TS - 1) / TS;
    hipLaunchKernelGGL(k_mlp_train, dim3(tiles), dim3(NTHR), 0, h->stream, h->net(), h->nrm, z, x, base, D, n,
                       h->part, h->ploss);
    MLP_LAUNCHED("k_mlp_train");
    return PPHD_OK;
}

hipMemcpyKind kind_in(int32_t on_device) { return on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice; }
hipMemcpyKind kind_out(int32_t on_device) { return on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost; }

}  // namespace

namespace pphd {

pphd_status mlp_mixture_table(pphd_mlp* h, hipStream_t stream, const double* dz, int M, double* tab)
{
    if (M <= 0) return PPHD_OK;
    hipLaunchKernelGGL(k_mlp_infer, dim3((M + TS - 1) / TS), dim3(NTHR), 0, stream, h->net(), h->nrm, dz, M,
                       (float*)nullptr, tab);
    MLP_LAUNCHED("k_mlp_infer");
    return PPHD_OK;
}

pphd_status mlp_head_table(const pphd_model& m, hipStream_t stream, const double* dz, const float* raw, int M,
                           double* tab)
{
    if (M <= 0) return PPHD_OK;
    hipLaunchKernelGGL(k_mix_head, dim3((M + NTHR - 1) / NTHR), dim3(NTHR), 0, stream, norm_of(m, 0), dz, raw, M,
                       tab);
    MLP_LAUNCHED("k_mix_head");
    return PPHD_OK;
}

}  // namespace pphd

extern "C" {

pphd_status pphd_mlp_workspace_size(const pphd_mlp_config* cfg, size_t* bytes)
{
    const char* why = nullptr;
    if (!config_ok(cfg, &why)) return err(PPHD_EINVAL, "%s", why);
    if (!bytes) return err(PPHD_EINVAL, "bytes is NULL");
    pphd_mlp tmp;
    *bytes = carve(&tmp, nullptr, *cfg);
    return PPHD_OK;
}

pphd_status pphd_mlp_create(const pphd_model* model, const pphd_mlp_config* cfg, void* workspace,
                            size_t workspace_bytes, uint64_t seed, void* stream, pphd_mlp** out)
{
    const char* why = nullptr;
    if (!out) return err(PPHD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!model) return err(PPHD_EINVAL, "model is NULL");
    if (!config_ok(cfg, &why)) return err(PPHD_EINVAL, "%s", why);
    if (!(model->region[1] > model->region[0]) || !(model->region[3] > model->region[2]))
        return err(PPHD_EINVAL, "empty surveillance region");
    if (!(model->birth_sigma_v > 0) || !(model->sigma_r > 0) || !(model->sigma_theta > 0))
        return err(PPHD_EINVAL, "birth_sigma_v, sigma_r and sigma_theta must be > 0");
    if (!workspace || ((uintptr_t)workspace & 255)) return err(PPHD_EINVAL, "workspace must be 256-byte aligned");
    pphd_mlp* h = new (std::nothrow) pphd_mlp;
    if (!h) return err(PPHD_ENOMEM, "host allocation failed");
    const size_t need = carve(h, nullptr, *cfg);
    if (workspace_bytes < need) {
        delete h;
        return err(PPHD_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    }
    h->model = *model;
    h->cfg = *cfg;
    h->stream = (hipStream_t)stream;
    h->seed = seed;
    h->nrm = norm_of(*model, seed);
    carve(h, (char*)workspace, *cfg);
    hipError_t e = hipMemsetAsync(workspace, 0, need, h->stream);
    if (e != hipSuccess) {
        delete h;
        return err(PPHD_EDEVICE, "hipMemsetAsync failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return PPHD_OK;
}

pphd_status pphd_mlp_destroy(pphd_mlp* h)
{
    if (!h) return PPHD_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    delete h;
    if (e != hipSuccess) return err(PPHD_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return PPHD_OK;
}

pphd_status pphd_mlp_init_params(pphd_mlp* h, uint32_t init_id)
{
    if (!h) return err(PPHD_EINVAL, "handle is NULL");
    hipLaunchKernelGGL(k_mlp_init, dim3((P_ALL + NTHR - 1) / NTHR), dim3(NTHR), 0, h->stream, h->theta, h->am,
                       h->av, h->nrm.key0, h->nrm.key1, init_id);
    MLP_LAUNCHED("k_mlp_init");
    h->t = 0;
    return reduce(h, 2, 0, 0.0, nullptr);
}

pphd_status pphd_mlp_set_params(pphd_mlp* h, const float* params, int32_t on_device)
{
    if (!h || !params) return err(PPHD_EINVAL, "NULL argument");
    MLP_TRY(hipMemcpyAsync(h->theta, params, P_ALL * 4, kind_in(on_device), h->stream));
    MLP_TRY(hipMemsetAsync(h->am, 0, P_ALL * 4, h->stream));
    MLP_TRY(hipMemsetAsync(h->av, 0, P_ALL * 4, h->stream));
    if (!on_device) MLP_TRY(hipStreamSynchronize(h->stream));
    h->t = 0;
    return reduce(h, 2, 0, 0.0, nullptr);
}

pphd_status pphd_mlp_get_params(pphd_mlp* h, float* params, int32_t on_device)
{
    if (!h || !params) return err(PPHD_EINVAL, "NULL argument");
    MLP_TRY(hipMemcpyAsync(params, h->theta, P_ALL * 4, kind_out(on_device), h->stream));
    if (!on_device) MLP_TRY(hipStreamSynchronize(h->stream));
    return PPHD_OK;
}

pphd_status pphd_mlp_simulate(pphd_mlp* h, uint32_t run)
{
    if (!h) return err(PPHD_EINVAL, "handle is NULL");
    const int64_t D = h->cfg.dataset;
    hipLaunchKernelGGL(k_mlp_simulate, dim3((unsigned)((D + NTHR - 1) / NTHR)), dim3(NTHR), 0, h->stream, h->nrm,
                       h->model.birth_sigma_v, run, h->dz, h->dx, D);
    MLP_LAUNCHED("k_mlp_simulate");
    return PPHD_OK;
}

pphd_status pphd_mlp_read_dataset(pphd_mlp* h, int32_t first, int32_t n, float* z, float* x)
{
    if (!h) return err(PPHD_EINVAL, "handle is NULL");
    if (first < 0 || n < 0 || (int64_t)first + n > h->cfg.dataset) return err(PPHD_EINVAL, "range outside the dataset");
    if (n == 0) return PPHD_OK;
    if (z) MLP_TRY(hipMemcpyAsync(z, h->dz + 2 * (size_t)first, (size_t)n * 8, hipMemcpyDeviceToHost, h->stream));
    if (x) MLP_TRY(hipMemcpyAsync(x, h->dx + 4 * (size_t)first, (size_t)n * 16, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    return PPHD_OK;
}

pphd_status pphd_mlp_loss_grad(pphd_mlp* h, const float* z, const float* x, int32_t n, int32_t on_device,
                               float* grad, double* loss)
{
    if (!h || !z || !x) return err(PPHD_EINVAL, "NULL argument");
    if (n < 1 || n > h->cfg.batch) return err(PPHD_EINVAL, "n must be in [1, batch]");
    MLP_TRY(hipMemcpyAsync(h->bz, z, (size_t)n * 8, kind_in(on_device), h->stream));
    MLP_TRY(hipMemcpyAsync(h->bx, x, (size_t)n * 16, kind_in(on_device), h->stream));
    pphd_status s = train_tiles(h, h->bz, h->bx, 0, n, n);
    if (s != PPHD_OK) return s;
    s = reduce(h, 0, (n + TS - 1) / TS, 1.0 / n, h->lossbuf);
    if (s != PPHD_OK) return s;
    if (grad) MLP_TRY(hipMemcpyAsync(grad, h->grad, P_ALL * 4, hipMemcpyDeviceToHost, h->stream));
    float l = 0.0f;
    MLP_TRY(hipMemcpyAsync(&l, h->lossbuf, 4, hipMemcpyDeviceToHost, h->stream));
    MLP_TRY(hipStreamSynchronize(h->stream));
    if (loss) *loss = l;
    return PPHD_OK;
}

pphd_status pphd_mlp_train(pphd_mlp* h, int32_t steps, double lr, float* loss)
{
    if (!h) return err(PPHD_EINVAL, "handle is NULL");
    if (steps < 0) return err(PPHD_EINVAL, "steps must be >= 0");
    const double lr0 = h->cfg.lr;
    if (lr > 0) h->cfg.lr = lr;
    const int B = h->cfg.batch;
    const int64_t D = h->cfg.dataset;
    pphd_status s = PPHD_OK;
    for (int done = 0; done < steps && s == PPHD_OK;) {
        const int chunk = std::min(LOSS_CHUNK, steps - done);
        for (int i = 0; i < chunk && s == PPHD_OK; ++i) {
            const int64_t base = (h->t * (int64_t)B) % D;
            s = train_tiles(h, h->dz, h->dx, base, D, B);
            if (s != PPHD_OK) break;
            h->t += 1;
            s = reduce(h, 1, B / TS, 1.0 / B, loss ? h->lossbuf + i : nullptr);
        }
        if (s == PPHD_OK && loss) {
            hipError_t e = hipMemcpyAsync(loss + done, h->lossbuf, (size_t)chunk * 4, hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) s = err(PPHD_EDEVICE, "loss copy failed: %s", hipGetErrorString(e));
        }
        done += chunk;
    }
    h->cfg.lr = lr0;
    return s;
}

pphd_status pphd_mlp_forward(pphd_mlp* h, const double* z, int32_t n, int32_t on_device, float* out)
{
    if (!h || !z || !out) return err(PPHD_EINVAL, "NULL argument");
    if (n < 0 || n > h->cfg.batch) return err(PPHD_EINVAL, "n must be in [0, batch]");
    if (n == 0) return PPHD_OK;
    MLP_TRY(hipMemcpyAsync(h->zin, z, (size_t)n * 16, kind_in(on_device), h->stream));
    hipLaunchKernelGGL(k_mlp_infer, dim3((n + TS - 1) / TS), dim3(NTHR), 0, h->stream, h->net(), h->nrm, h->zin, n,
                       h->out, (double*)nullptr);
    MLP_LAUNCHED("k_mlp_infer");
    MLP_TRY(hipMemcpyAsync(out, h->out, (size_t)n * NO * 4, kind_out(on_device), h->stream));
    if (!on_device) MLP_TRY(hipStreamSynchronize(h->stream));
    return PPHD_OK;
}

pphd_status pphd_mlp_steps(pphd_mlp* h, int64_t* steps)
{
    if (!h || !steps) return err(PPHD_EINVAL, "NULL argument");
    *steps = h->t;
    return PPHD_OK;
}

}  // extern "C"
