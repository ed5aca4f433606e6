// Host side of the CNN surrogate: parameter storage (FP32 master weights,
// BF16 packed copies), forward pass, one training step (MSE loss on the
// scaled 1-hour increment, backward pass, Adam), and the surrogate advance of
// a grid class with the residual check against the plain solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sft.h"
#include "sft_internal.h"

namespace sft {
void cnn_features(hipStream_t st, const void* Bin, int dtype, const float* feats, uint16_t* X0, int batch,
                  int H, int W);
// cap > 0 limits the blocks of the persistent launches (0: one wave over
// the compute units)
void cnn_conv_fwd(hipStream_t st, int cap, int cin, const uint16_t* x, const uint16_t* wf, const float* bias,
                  uint16_t* out, int batch, int H, int W);
void cnn_conv_fwd_first(hipStream_t st, int cap, const void* Bin, int dtype, const float* feats,
                        const uint16_t* wf, const float* bias, uint16_t* out, int batch, int H, int W);
void cnn_conv_fwd_out(hipStream_t st, int cap, const uint16_t* x, const uint16_t* wf, const float* bias,
                      const uint16_t* wf5, const float* b5, float* z, float* y, int batch, int H, int W);
void cnn_conv_out(hipStream_t st, const uint16_t* x4, const uint16_t* wf5, const float* b5, float* y,
                  int batch, int H, int W);
void cnn_conv_dgrad(hipStream_t st, int cap, int cin, const uint16_t* dz, const uint16_t* wd,
                    const uint16_t* act, uint16_t* dx, float* edge, int batch, int H, int W);
void cnn_wgrad(hipStream_t st, int cin, int cout, int cin_out, int cout_out, const uint16_t* x,
               const uint16_t* dz, float* part, float* bpart, int nblk, float* grad, float* gbias,
               int batch, int H, int W);
void cnn_loss_grad(hipStream_t st, const float* y, const void* Bin, const void* Bt, int dtype, uint16_t* dyb,
                   double* part, int nblk, size_t n);
void cnn_adam(hipStream_t st, float* p, const float* g, float* m, float* v, int n, float lr, float b1,
              float b2, float eps, float c1, float c2);
void cnn_pack(hipStream_t st, const float* Wm, int cin, int cout, int cip, int nout, int cop, uint16_t* wf,
              uint16_t* wd);
}  // namespace sft

using namespace sft;

namespace {
// five 3x3 layers: 6 -> 64 -> 64 -> 64 -> 64 -> 1 (weights W[co][ci][3][3], then bias);
// the first layer reads 16 packed input slots (field hi/lo sharing weight 0)
const int kCin[5] = {6, 64, 64, 64, 64};
const int kCout[5] = {64, 64, 64, 64, 1};
const int kWGB = 256;     // weight-gradient blocks (one per compute unit), each with its own partial
const int kRED = 1024;    // reduction blocks
}  // namespace

struct sft_net {
    int H = 0, W = 0, maxb = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t n = 0;
    int64_t woff[5], boff[5];
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    int step = 0;
    uint16_t* wf[5] = {};   // forward layouts (layer 5: one 32-wide tile, row 0 real)
    uint16_t* wd[5] = {};   // data-gradient layouts (layers 2..5)
    uint16_t* X0 = nullptr;
    uint16_t* X[4] = {};
    float *y = nullptr, *dxp = nullptr;   // dxp: pole-row edge scratch [B][4][np][64]
    uint16_t* dyb = nullptr;   // output gradient as 16 bf16 channels (channel 0 real)
    uint16_t* dz[2] = {};
    float *wpart = nullptr, *bpart = nullptr;
    double* losspart = nullptr;
    int last_batch = 0;
    bool acts_kept = false;   // the input and layer-4 activations of the last forward pass are held
    int grid_cap = 0;         // > 0: at most this many blocks per persistent / weight-gradient launch
    std::vector<void*> allocs;
    std::string err;
};

namespace {

int wgrad_blocks(const sft_net* net) { return net->grid_cap > 0 ? std::min(kWGB, net->grid_cap) : kWGB; }

sft_status nfail(sft_net* n, sft_status st, const char* msg)
{
    if (n) n->err = msg;
    return st;
}

template <typename T>
sft_status nalloc(sft_net* net, T** p, size_t count)
{
    if (hipMalloc((void**)p, (count ? count : 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return nfail(net, SFT_ERR_OOM, "device allocation failed");
    }
    net->allocs.push_back((void*)*p);
    return SFT_OK;
}

#define NTRY(x)                       \
    do {                              \
        sft_status s_ = (x);          \
        if (s_ != SFT_OK) return s_;  \
    } while (0)

void pack_all(sft_net* net)
{
    for (int l = 0; l < 4; ++l)
        cnn_pack(net->stream, net->p + net->woff[l], kCin[l], 64, l == 0 ? 16 : 64, 64, 64, net->wf[l],
                 l == 0 ? nullptr : net->wd[l]);
    cnn_pack(net->stream, net->p + net->woff[4], 64, 1, 64, 32, 16, net->wf[4], net->wd[4]);
}

// predict = true (inference only): the first layer forms its input channels
// from the field while staging its tiles, and the last hidden layer and the
// output layer's tap products run as one pass; the input and layer-4
// activations are not kept (the latter's buffer holds the tap products
// instead).  y is bitwise the same.
void forward(sft_net* net, int batch, const void* Bin, int dtype, const float* feats, bool predict = false)
{
    hipStream_t st = net->stream;
    const int H = net->H, W = net->W;
    if (predict) {
        cnn_conv_fwd_first(st, net->grid_cap, Bin, dtype, feats, net->wf[0], net->p + net->boff[0], net->X[0], batch, H, W);
    } else {
        cnn_features(st, Bin, dtype, feats, net->X0, batch, H, W);
        cnn_conv_fwd(st, net->grid_cap, 16, net->X0, net->wf[0], net->p + net->boff[0], net->X[0], batch, H, W);
    }
    for (int l = 1; l < (predict ? 3 : 4); ++l)
        cnn_conv_fwd(st, net->grid_cap, 64, net->X[l - 1], net->wf[l], net->p + net->boff[l], net->X[l], batch, H, W);
    if (predict)
        cnn_conv_fwd_out(st, net->grid_cap, net->X[2], net->wf[3], net->p + net->boff[3], net->wf[4], net->p + net->boff[4],
                         (float*)net->X[3], net->y, batch, H, W);
    else
        cnn_conv_out(st, net->X[3], net->wf[4], net->p + net->boff[4], net->y, batch, H, W);
    net->last_batch = batch;
    net->acts_kept = !predict;
}

}  // namespace

extern "C" {

sft_status sft_net_create(sft_net** out, int32_t nt, int32_t np, int32_t max_batch, void* hip_stream)
{
    if (!out || nt < 8 || np < 32 || (np & 1) || max_batch < 1) return SFT_ERR_ARG;
    sft_net* net = new sft_net();
    net->H = nt;
    net->W = np;
    net->maxb = max_batch;
    net->stream = (hipStream_t)hip_stream;
    if (!net->stream) {
        if (hipStreamCreate(&net->stream) != hipSuccess) {
            delete net;
            return SFT_ERR_HIP;
        }
        net->own_stream = true;
    }
    int64_t o = 0;
    for (int l = 0; l < 5; ++l) {
        net->woff[l] = o;
        o += (int64_t)kCout[l] * kCin[l] * 9;
        net->boff[l] = o;
        o += kCout[l];
    }
    net->n = o;
    const size_t plane = (size_t)nt * np;
    const size_t B = (size_t)max_batch;
    sft_status st = SFT_OK;
#define A_(x) \
    if (st == SFT_OK) st = (x)
    A_(nalloc(net, &net->p, net->n));
    A_(nalloc(net, &net->g, net->n));
    A_(nalloc(net, &net->m, net->n));
    A_(nalloc(net, &net->v, net->n));
    for (int l = 0; l < 4; ++l) {
        A_(nalloc(net, &net->wf[l], (size_t)9 * 64 * (l == 0 ? 16 : 64)));
        if (l) A_(nalloc(net, &net->wd[l], (size_t)9 * 64 * 64));
    }
    A_(nalloc(net, &net->wf[4], (size_t)9 * 32 * 64));
    A_(nalloc(net, &net->wd[4], (size_t)9 * 64 * 16));
    A_(nalloc(net, &net->X0, B * plane * 16));
    for (int l = 0; l < 4; ++l) A_(nalloc(net, &net->X[l], B * plane * 64));
    A_(nalloc(net, &net->y, B * plane));
    A_(nalloc(net, &net->dyb, B * plane * 16));
    A_(nalloc(net, &net->dxp, B * (size_t)4 * np * 64));
    A_(nalloc(net, &net->dz[0], B * plane * 64));
    A_(nalloc(net, &net->dz[1], B * plane * 64));
    A_(nalloc(net, &net->wpart, (size_t)kWGB * 9 * 64 * 64));
    A_(nalloc(net, &net->bpart, (size_t)kWGB * 64));
    A_(nalloc(net, &net->losspart, (size_t)kRED));
#undef A_
    if (st != SFT_OK) {
        for (void* q : net->allocs) (void)hipFree(q);
        if (net->own_stream) (void)hipStreamDestroy(net->stream);
        delete net;
        return st;
    }
    (void)hipMemsetAsync(net->p, 0, net->n * sizeof(float), net->stream);
    (void)hipMemsetAsync(net->m, 0, net->n * sizeof(float), net->stream);
    (void)hipMemsetAsync(net->v, 0, net->n * sizeof(float), net->stream);
    (void)hipMemsetAsync(net->g, 0, net->n * sizeof(float), net->stream);
    pack_all(net);
    *out = net;
    return SFT_OK;
}

sft_status sft_net_param_count(const sft_net* net, int64_t* n)
{
    if (!net || !n) return SFT_ERR_ARG;
    *n = net->n;
    return SFT_OK;
}

sft_status sft_net_set_params(sft_net* net, const float* params, int32_t on_device)
{
    if (!net || !params) return SFT_ERR_ARG;
    if (hipMemcpyAsync(net->p, params, net->n * sizeof(float),
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, net->stream) != hipSuccess)
        return SFT_ERR_HIP;
    if (!on_device && hipStreamSynchronize(net->stream) != hipSuccess) return SFT_ERR_HIP;
    (void)hipMemsetAsync(net->m, 0, net->n * sizeof(float), net->stream);
    (void)hipMemsetAsync(net->v, 0, net->n * sizeof(float), net->stream);
    net->step = 0;
    pack_all(net);
    return hipGetLastError() == hipSuccess ? SFT_OK : SFT_ERR_HIP;
}

static sft_status copy_vec(sft_net* net, float* dst, const float* src, int32_t on_device)
{
    if (hipMemcpyAsync(dst, src, net->n * sizeof(float),
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, net->stream) != hipSuccess)
        return SFT_ERR_HIP;
    if (!on_device && hipStreamSynchronize(net->stream) != hipSuccess) return SFT_ERR_HIP;
    return SFT_OK;
}

sft_status sft_net_get_params(sft_net* net, float* params, int32_t on_device)
{
    if (!net || !params) return SFT_ERR_ARG;
    return copy_vec(net, params, net->p, on_device);
}

sft_status sft_net_get_grads(sft_net* net, float* grads, int32_t on_device)
{
    if (!net || !grads) return SFT_ERR_ARG;
    return copy_vec(net, grads, net->g, on_device);
}

sft_status sft_net_forward(sft_net* net, int32_t batch, const void* b_in, int32_t dtype, const float* feats,
                           float* y)
{
    if (!net || !b_in || !feats || batch < 1 || batch > net->maxb) return SFT_ERR_ARG;
    if (dtype != SFT_DTYPE_F64 && dtype != SFT_DTYPE_F32) return SFT_ERR_ARG;
    forward(net, batch, b_in, dtype, feats);
    if (y)
        (void)hipMemcpyAsync(y, net->y, (size_t)batch * net->H * net->W * sizeof(float),
                             hipMemcpyDeviceToDevice, net->stream);
    return hipGetLastError() == hipSuccess ? SFT_OK : SFT_ERR_HIP;
}

sft_status sft_net_predict(sft_net* net, int32_t batch, const void* b_in, int32_t dtype, const float* feats,
                           float* y)
{
    if (!net || !b_in || !feats || batch < 1 || batch > net->maxb) return SFT_ERR_ARG;
    if (dtype != SFT_DTYPE_F64 && dtype != SFT_DTYPE_F32) return SFT_ERR_ARG;
    forward(net, batch, b_in, dtype, feats, true);
    if (y)
        (void)hipMemcpyAsync(y, net->y, (size_t)batch * net->H * net->W * sizeof(float),
                             hipMemcpyDeviceToDevice, net->stream);
    return hipGetLastError() == hipSuccess ? SFT_OK : SFT_ERR_HIP;
}

sft_status sft_net_get_activation(sft_net* net, int32_t layer, void* out)
{
    if (!net || !out || layer < 0 || layer > 4 || !net->last_batch) return SFT_ERR_ARG;
    if ((layer == 0 || layer == 4) && !net->acts_kept) return SFT_ERR_STATE;
    const size_t plane = (size_t)net->H * net->W * net->last_batch;
    const void* src = layer == 0 ? (const void*)net->X0 : (const void*)net->X[layer - 1];
    const size_t bytes = plane * (layer == 0 ? 16 : 64) * sizeof(uint16_t);
    if (hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, net->stream) != hipSuccess)
        return SFT_ERR_HIP;
    return SFT_OK;
}

sft_status sft_net_train_step(sft_net* net, int32_t batch, const void* b_in, const void* b_target,
                              int32_t dtype, const float* feats, float lr, int32_t apply, double* loss)
{
    if (!net || !b_in || !b_target || !feats || batch < 1 || batch > net->maxb) return SFT_ERR_ARG;
    if (dtype != SFT_DTYPE_F64 && dtype != SFT_DTYPE_F32) return SFT_ERR_ARG;
    hipStream_t st = net->stream;
    const int H = net->H, W = net->W;
    const size_t npx = (size_t)batch * H * W;
    forward(net, batch, b_in, dtype, feats);
    cnn_loss_grad(st, net->y, b_in, b_target, dtype, net->dyb, net->losspart, kRED, npx);
    // output layer: weight/bias gradient, then the gradient into the layer-4
    // output masked by its ReLU
    cnn_wgrad(st, 64, 16, 64, 1, net->X[3], net->dyb, net->wpart, net->bpart, wgrad_blocks(net), net->g + net->woff[4],
              net->g + net->boff[4], batch, H, W);
    cnn_conv_dgrad(st, net->grid_cap, 16, net->dyb, net->wd[4], net->X[3], net->dz[0], net->dxp, batch, H, W);
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        const uint16_t* xin = l == 0 ? net->X0 : net->X[l - 1];
        const int cin = l == 0 ? 16 : 64;
        cnn_wgrad(st, cin, 64, kCin[l], 64, xin, net->dz[cur], net->wpart, net->bpart, wgrad_blocks(net),
                  net->g + net->woff[l], net->g + net->boff[l], batch, H, W);
        if (l > 0) {
            cnn_conv_dgrad(st, net->grid_cap, 64, net->dz[cur], net->wd[l], net->X[l - 1], net->dz[cur ^ 1], net->dxp, batch,
                           H, W);
            cur ^= 1;
        }
    }
    if (apply) {
        net->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)net->step), c2 = 1.f - powf(b2, (float)net->step);
        cnn_adam(st, net->p, net->g, net->m, net->v, (int)net->n, lr, b1, b2, 1e-8f, c1, c2);
        pack_all(net);
    }
    if (loss) {
        std::vector<double> part(kRED);
        if (hipMemcpyAsync(part.data(), net->losspart, kRED * sizeof(double), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return SFT_ERR_HIP;
        double s = 0.0;
        for (double x : part) s += x;
        *loss = s / (double)npx;
    }
    return hipGetLastError() == hipSuccess ? SFT_OK : SFT_ERR_HIP;
}

sft_status sft_net_set_grid_limit(sft_net* net, int32_t max_blocks)
{
    if (!net || max_blocks < 0) return SFT_ERR_ARG;
    net->grid_cap = max_blocks;
    return SFT_OK;
}

sft_status sft_net_sync(sft_net* net)
{
    if (!net) return SFT_ERR_ARG;
    return hipStreamSynchronize(net->stream) == hipSuccess ? SFT_OK : SFT_ERR_HIP;
}

sft_status sft_net_destroy(sft_net* net)
{
    if (!net) return SFT_ERR_ARG;
    (void)hipStreamSynchronize(net->stream);
    for (void* q : net->allocs) (void)hipFree(q);
    if (net->own_stream) (void)hipStreamDestroy(net->stream);
    delete net;
    return SFT_OK;
}

}  // extern "C"

namespace sft {
// internal: used by the context's surrogate advance
sft_status net_predict(sft_net* net, hipStream_t st, int batch, const double* Bin,
                                    const float* feats, float** y_out)
{
    if (!net) return SFT_ERR_ARG;
    hipStream_t saved = net->stream;
    net->stream = st;
    forward(net, batch, Bin, SFT_DTYPE_F64, feats, true);
    net->stream = saved;
    *y_out = net->y;
    return SFT_OK;
}

void net_dims(const sft_net* net, int* H, int* W, int* maxb)
{
    *H = net->H;
    *W = net->W;
    *maxb = net->maxb;
}

}  // namespace sft
