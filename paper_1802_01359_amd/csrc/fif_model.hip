// Host runtime of the step-count proposal network: device memory of a model,
// forward pass, gradient, Adam step, parameter files.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fif.h"
#include "fif_model_internal.hpp"
#include "fif_net.hpp"

using namespace fif;

static_assert(kNetParams == FIF_NET_PARAMS, "parameter count of the header");
static_assert(kNetFeat == FIF_NET_FEATURES && kNetCin0 == FIF_NET_CHANNELS, "input shape of the header");

struct fif_model {
    int device = 0;
    int32_t max_batch = 0;
    void* mem = nullptr;
    float *p = nullptr, *m1 = nullptr, *m2 = nullptr, *g = nullptr;
    NetWeights W{};
    bf16* act[kNetLayers] = {};
    bf16 *dza = nullptr, *dzb = nullptr;
    float* part = nullptr;
    float *y = nullptr, *loss_b = nullptr, *hpart = nullptr, *loss = nullptr;
    int64_t step = 0;
    ~fif_model()
    {
        if (mem) (void)hipFree(mem);
    }
};

namespace {

constexpr int kHeadParts = kNetOut * kNetCh + kNetOut;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

int wchunks(int l, int B) { return (B * (net_len_in(l) / 2) + kNetWRows - 1) / kNetWRows; }
int wstride(int l) { return net_kp(l) * kNetCh + kNetCh; }

#define M_TRY(expr)                                                                            \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fif_internal_fail(FIF_ERR_DEVICE, std::string(#expr " failed: ") +           \
                                                         hipGetErrorString(e_));               \
    } while (0)

fif_status alloc_model(fif_model* m, int32_t Bm)
{
    m->max_batch = Bm;
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> parts;
    auto add = [&](void** ptr, size_t bytes) {
        parts.push_back({ptr, off});
        off = al(off + bytes);
    };
    const size_t P = sizeof(float) * kNetParams;
    add((void**)&m->p, P);
    add((void**)&m->m1, P);
    add((void**)&m->m2, P);
    add((void**)&m->g, P);
    for (int l = 0; l < kNetLayers; ++l) {
        add((void**)&m->W.wf[l], sizeof(bf16) * net_kp(l) * kNetCh);
        if (l > 0) add((void**)&m->W.wd[l], sizeof(bf16) * net_kf(l) * kNetCh);
        add((void**)&m->act[l], sizeof(bf16) * (size_t)Bm * (net_len_in(l) / 2) * kNetCh);
    }
    add((void**)&m->dza, sizeof(bf16) * (size_t)Bm * (kNetFeat / 2) * kNetCh);
    add((void**)&m->dzb, sizeof(bf16) * (size_t)Bm * (kNetFeat / 2) * kNetCh);
    size_t pmax = 0;
    for (int l = 0; l < kNetLayers; ++l) pmax = std::max(pmax, (size_t)wchunks(l, Bm) * wstride(l));
    add((void**)&m->part, sizeof(float) * pmax);
    add((void**)&m->y, sizeof(float) * (size_t)Bm * kNetOut);
    add((void**)&m->loss_b, sizeof(float) * (size_t)Bm);
    add((void**)&m->hpart, sizeof(float) * (size_t)Bm * kHeadParts);
    add((void**)&m->loss, sizeof(float));
    if (hipMalloc(&m->mem, off) != hipSuccess) return fif_internal_fail(FIF_ERR_NOMEM, "model allocation failed");
    for (auto& pr : parts) *pr.first = (char*)m->mem + pr.second;
    M_TRY(hipMemset(m->mem, 0, off));
    return FIF_OK;
}

fif_status upload_params(fif_model* m, const float* host)
{
    if (host)
        M_TRY(hipMemcpy(m->p, host, sizeof(float) * kNetParams, hipMemcpyHostToDevice));
    else
        M_TRY(hipMemset(m->p, 0, sizeof(float) * kNetParams));
    M_TRY(hipMemset(m->m1, 0, sizeof(float) * kNetParams));
    M_TRY(hipMemset(m->m2, 0, sizeof(float) * kNetParams));
    m->step = 0;
    k_pack_weights<<<dim3(64, kNetLayers), 256>>>(m->p, m->W);
    M_TRY(hipGetLastError());
    M_TRY(hipDeviceSynchronize());
    return FIF_OK;
}

fif_status check_call(const fif_model* m, const void* feats, int32_t B)
{
    if (!m) return fif_internal_fail(FIF_ERR_INVALID_ARG, "model is null");
    if (!feats) return fif_internal_fail(FIF_ERR_INVALID_ARG, "feats is null");
    if (B < 1 || B > m->max_batch)
        return fif_internal_fail(FIF_ERR_INVALID_ARG, "batch " + std::to_string(B) + " outside 1.." +
                                                          std::to_string(m->max_batch));
    if (((uintptr_t)feats) % 16) return fif_internal_fail(FIF_ERR_INVALID_ARG, "feats must be 16-byte aligned");
    int dev = -1;
    M_TRY(hipGetDevice(&dev));
    if (dev != m->device) return fif_internal_fail(FIF_ERR_INVALID_ARG, "model lives on another device");
    return FIF_OK;
}

// Six convolutions and the head (targets may be null).
void forward(fif_model* m, const bf16* x, int B, const float* targets, hipStream_t s)
{
    const bf16* in = x;
    for (int l = 0; l < kNetLayers; ++l) {
        const int lin = net_len_in(l);
        const int rows = B * (lin / 2);
        const unsigned grid = (unsigned)((rows + kNetRowsWG - 1) / kNetRowsWG);
        const float* bias = m->p + net_w_off(l) + net_kf(l) * kNetCh;
        if (l == 0)
            k_conv_fwd<kNetCin0><<<grid, kNetThreads, 0, s>>>(in, lin, m->W.wf[l], bias, m->act[l], rows);
        else
            k_conv_fwd<kNetCh><<<grid, kNetThreads, 0, s>>>(in, lin, m->W.wf[l], bias, m->act[l], rows);
        in = m->act[l];
    }
    // layer 5's pre-activation gradient goes to dza (used only with targets)
    k_head<<<B, 64, 0, s>>>(m->act[kNetLayers - 1], m->p + kNetHeadOff, m->p + kNetHeadOff + kNetOut * kNetCh, m->y,
                            targets, m->loss_b, m->hpart, m->dza, B);
}

// Gradient of the loss into m->g and the loss into m->loss (after forward
// with targets).
void backward(fif_model* m, const bf16* x, int B, hipStream_t s)
{
    bf16* dz = m->dza;     // gradient of layer l's pre-activation
    bf16* other = m->dzb;
    for (int l = kNetLayers - 1; l >= 0; --l) {
        const int lin = net_len_in(l);
        const int rows_out = B * (lin / 2);
        const bf16* in = l == 0 ? x : m->act[l - 1];
        const int nch = wchunks(l, B);
        if (l == 0)
            k_conv_bwd_w<kNetCin0><<<nch, kNetThreads, 0, s>>>(in, lin, dz, m->part, rows_out);
        else
            k_conv_bwd_w<kNetCh><<<nch, kNetThreads, 0, s>>>(in, lin, dz, m->part, rows_out);
        const int nw = net_kf(l) * kNetCh, n = nw + kNetCh;
        k_reduce_parts<<<(n + 255) / 256, 256, 0, s>>>(m->part, nch, wstride(l), nw, net_kp(l) * kNetCh, n,
                                                       m->g + net_w_off(l));
        if (l > 0) {
            const int rows_in = B * lin;
            k_conv_bwd_data<<<(unsigned)((rows_in + kNetRowsWG - 1) / kNetRowsWG), kNetThreads, 0, s>>>(dz, lin, m->W.wd[l],
                                                                                   m->act[l - 1], other, rows_in);
            std::swap(dz, other);
        }
    }
    k_reduce_parts<<<1, 256, 0, s>>>(m->hpart, B, kHeadParts, kHeadParts, 0, kHeadParts, m->g + kNetHeadOff);
    k_sum_loss<<<1, 64, 0, s>>>(m->loss_b, B, m->loss);
}

}  // namespace

namespace fif {

int32_t model_max_batch(const fif_model* m) { return m->max_batch; }
int model_device(const fif_model* m) { return m->device; }

const float* model_infer(fif_model* m, const uint16_t* feats, int32_t B, hipStream_t s)
{
    forward(m, (const bf16*)feats, B, nullptr, s);
    return m->y;
}

}  // namespace fif

extern "C" {

fif_status fif_model_create(fif_model** model, const float* params, int32_t max_batch)
{
    if (!model) return fif_internal_fail(FIF_ERR_INVALID_ARG, "model is null");
    *model = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20)) return fif_internal_fail(FIF_ERR_INVALID_ARG, "max_batch out of range");
    fif_model* m = new fif_model();
    fif_status st = FIF_OK;
    if (hipGetDevice(&m->device) != hipSuccess) st = fif_internal_fail(FIF_ERR_DEVICE, "no HIP device");
    if (st == FIF_OK) st = alloc_model(m, max_batch);
    if (st == FIF_OK) st = upload_params(m, params);
    if (st != FIF_OK) {
        delete m;
        return st;
    }
    *model = m;
    return FIF_OK;
}

fif_status fif_model_free(fif_model* model)
{
    delete model;
    return FIF_OK;
}

fif_status fif_model_get_params(const fif_model* m, float* params)
{
    if (!m || !params) return fif_internal_fail(FIF_ERR_INVALID_ARG, "null argument");
    M_TRY(hipDeviceSynchronize());
    M_TRY(hipMemcpy(params, m->p, sizeof(float) * kNetParams, hipMemcpyDeviceToHost));
    return FIF_OK;
}

fif_status fif_model_set_params(fif_model* m, const float* params)
{
    if (!m || !params) return fif_internal_fail(FIF_ERR_INVALID_ARG, "null argument");
    M_TRY(hipDeviceSynchronize());
    return upload_params(m, params);
}

fif_status fif_model_save(const fif_model* m, const char* path)
{
    if (!m || !path) return fif_internal_fail(FIF_ERR_INVALID_ARG, "null argument");
    std::vector<float> h(kNetParams);
    fif_status st = fif_model_get_params(m, h.data());
    if (st != FIF_OK) return st;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fif_internal_fail(FIF_ERR_INVALID_ARG, std::string("cannot write ") + path);
    const int32_t hdr[2] = {kNetParams, 0};
    bool ok = std::fwrite("FIFNET01", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 2, f) == 2 &&
              std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fif_internal_fail(FIF_ERR_INVALID_ARG, std::string("short write to ") + path);
    return FIF_OK;
}

fif_status fif_model_load(fif_model** model, const char* path, int32_t max_batch)
{
    if (!model || !path) return fif_internal_fail(FIF_ERR_INVALID_ARG, "null argument");
    *model = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fif_internal_fail(FIF_ERR_INVALID_ARG, std::string("cannot read ") + path);
    char magic[8];
    int32_t hdr[2];
    std::vector<float> h(kNetParams);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "FIFNET01", 8) == 0 &&
              std::fread(hdr, sizeof(int32_t), 2, f) == 2 && hdr[0] == kNetParams &&
              std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) return fif_internal_fail(FIF_ERR_INVALID_ARG, std::string("not a proposal network file: ") + path);
    return fif_model_create(model, h.data(), max_batch);
}

fif_status fif_model_forward(fif_model* m, const uint16_t* feats, int32_t B, float* out, void* stream)
{
    fif_status st = check_call(m, feats, B);
    if (st != FIF_OK) return st;
    if (!out) return fif_internal_fail(FIF_ERR_INVALID_ARG, "out is null");
    hipStream_t s = (hipStream_t)stream;
    forward(m, (const bf16*)feats, B, nullptr, s);
    M_TRY(hipMemcpyAsync(out, m->y, sizeof(float) * kNetOut * (size_t)B, hipMemcpyDeviceToDevice, s));
    M_TRY(hipGetLastError());
    return FIF_OK;
}

fif_status fif_model_grad(fif_model* m, const uint16_t* feats, const float* targets, int32_t B, float* grad,
                          float* loss, void* stream)
{
    fif_status st = check_call(m, feats, B);
    if (st != FIF_OK) return st;
    if (!targets) return fif_internal_fail(FIF_ERR_INVALID_ARG, "targets is null");
    hipStream_t s = (hipStream_t)stream;
    forward(m, (const bf16*)feats, B, targets, s);
    backward(m, (const bf16*)feats, B, s);
    if (grad) M_TRY(hipMemcpyAsync(grad, m->g, sizeof(float) * kNetParams, hipMemcpyDeviceToDevice, s));
    if (loss) M_TRY(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    M_TRY(hipGetLastError());
    return FIF_OK;
}

fif_status fif_model_train_step(fif_model* m, const uint16_t* feats, const float* targets, int32_t B, float lr,
                                float* loss, void* stream)
{
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fif_internal_fail(FIF_ERR_INVALID_ARG, "lr must be >= 0");
    fif_status st = fif_model_grad(m, feats, targets, B, nullptr, loss, stream);
    if (st != FIF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    k_adam<<<(kNetParams + 255) / 256, 256, 0, s>>>(m->p, m->m1, m->m2, m->g, kNetParams, lr, b1, b2, 1e-8f, c1, c2);
    k_pack_weights<<<dim3(64, kNetLayers), 256, 0, s>>>(m->p, m->W);
    M_TRY(hipGetLastError());
    return FIF_OK;
}

}  // extern "C"
