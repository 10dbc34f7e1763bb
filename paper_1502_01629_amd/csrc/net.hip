// C-ABI of the learned warm start: network object, forward, loss and gradients, Adam, and the
// projection to a start of the SL iteration. Kernels in cnn.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/slhjb.h"
#include "internal.h"

using namespace slhjb;

namespace {
constexpr int kCin0 = 16;      // input feature channels (5 used)
constexpr int kMaxImages = 256;
constexpr int kMaxLayers = 14;
// The 4-level U-Net: two 3 x 3 convolutions per level (32, 64, 128 channels, 128 at the bottom),
// 2 x 2 average pooling down, nearest upsampling and concatenation with the skip up; layer l reads
// (cin, level) and writes cout channels. Inputs: 0 features, 1 out0, 2 pool(out1), 3 out2,
// 4 pool(out3), 5 out4, 6 pool(out5), 7 out6, 8 [up(out7), out5], 9 out8, 10 [up(out9), out3],
// 11 out10, 12 [up(out11), out1], 13 out12; the head reads out13.
struct UConv {
  int cin, cout, level;
};
constexpr UConv kUNet[kMaxLayers] = {{16, 32, 0},   {32, 32, 0},   {32, 64, 1},   {64, 64, 1},  {64, 128, 2},
                                     {128, 128, 2}, {128, 128, 3}, {128, 128, 3}, {256, 128, 2}, {128, 128, 2},
                                     {192, 64, 1},  {64, 64, 1},   {96, 32, 0},   {32, 32, 0}};
constexpr int kUNetMargin = 48;  // receptive-field radius of the U-Net (46 px), rounded up
}  // namespace

struct slhjb_net {
  slhjb_ctx* ctx = nullptr;
  int arch = 0;  // 0 dilated CNN, 1 U-Net
  int L = 0, C = 0;
  int dil[kMaxLayers] = {};
  int cin[kMaxLayers] = {};
  int cout[kMaxLayers] = {};
  int level[kMaxLayers] = {};
  int64_t nparam = 0;
  int64_t w_off[kMaxLayers] = {}, b_off[kMaxLayers] = {}, hw_off = 0, hb_off = 0;
  float* params = nullptr;
  float* grads = nullptr;
  float* wwork = nullptr;  // partial sums of the weight gradients (kWgradWorkFloats)
  float* m1 = nullptr;
  float* m2 = nullptr;
  uint16_t* wt[kMaxLayers] = {};
  uint16_t* wtt[kMaxLayers] = {};
  int step = 0;
  // activations, sized for `cap_px` pixels (at full resolution)
  long long cap_px = 0;
  uint16_t* feat = nullptr;
  uint16_t* act[kMaxLayers] = {};
  uint16_t* g[2] = {nullptr, nullptr};
  // U-Net: pooled tensors, concatenations and the gradients of every tensor
  uint16_t* pool[3] = {};
  uint16_t* cat[3] = {};
  uint16_t* gact[kMaxLayers] = {};
  uint16_t* gpool[3] = {};
  uint16_t* gcat[3] = {};
  float* delta = nullptr;
  float* uhat = nullptr;
  float* vstar = nullptr;
  uint8_t* mask = nullptr;
  CropSrc* d_src = nullptr;
  CropSrc* h_src = nullptr;  // pinned
  float* d_acc = nullptr;    // [0] sum of squared errors
  float* h_acc = nullptr;    // pinned
};

namespace {

int net_hip(slhjb_net* net, hipError_t e, const char* what) { return ctx_hip_fail(net->ctx, e, what); }

#define NET_TRY(expr)                                       \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return net_hip(net, _e, #expr);   \
  } while (0)

void free_acts(slhjb_net* net) {
  auto f = [](void* p) {
    if (p) hipFree(p);
  };
  f(net->feat);
  for (auto& a : net->act) f(a), a = nullptr;
  for (auto& a : net->gact) f(a), a = nullptr;
  for (int l = 0; l < 3; ++l) {
    f(net->pool[l]), net->pool[l] = nullptr;
    f(net->cat[l]), net->cat[l] = nullptr;
    f(net->gpool[l]), net->gpool[l] = nullptr;
    f(net->gcat[l]), net->gcat[l] = nullptr;
  }
  f(net->g[0]);
  f(net->g[1]);
  f(net->delta);
  f(net->uhat);
  f(net->vstar);
  f(net->mask);
  net->feat = nullptr;
  net->g[0] = net->g[1] = nullptr;
  net->delta = net->uhat = net->vstar = nullptr;
  net->mask = nullptr;
  net->cap_px = 0;
}

int ensure_acts(slhjb_net* net, long long px) {
  if (net->cap_px >= px) return SLHJB_OK;
  free_acts(net);
  const size_t C = (size_t)net->C;
  hipError_t e = hipMalloc(&net->feat, sizeof(uint16_t) * px * kCin0);
  if (net->arch == 1) {
    // level l holds px / 4^l pixels
    for (int l = 0; l < net->L && e == hipSuccess; ++l) {
      const size_t n = sizeof(uint16_t) * (px >> (2 * net->level[l])) * net->cout[l];
      e = hipMalloc(&net->act[l], n);
      if (e == hipSuccess) e = hipMalloc(&net->gact[l], n);
    }
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
      const size_t np = sizeof(uint16_t) * (px >> (2 * (l + 1))) * kUNet[2 * l + 1].cout;
      const size_t nc = sizeof(uint16_t) * (px >> (2 * l)) * kUNet[12 - 2 * l].cin;
      e = hipMalloc(&net->pool[l], np);
      if (e == hipSuccess) e = hipMalloc(&net->gpool[l], np);
      if (e == hipSuccess) e = hipMalloc(&net->cat[l], nc);
      if (e == hipSuccess) e = hipMalloc(&net->gcat[l], nc);
    }
  } else {
    for (int l = 0; l < net->L && e == hipSuccess; ++l) e = hipMalloc(&net->act[l], sizeof(uint16_t) * px * C);
    if (e == hipSuccess) e = hipMalloc(&net->g[0], sizeof(uint16_t) * px * C);
    if (e == hipSuccess) e = hipMalloc(&net->g[1], sizeof(uint16_t) * px * C);
  }
  if (e == hipSuccess) e = hipMalloc(&net->delta, sizeof(float) * px);
  if (e == hipSuccess) e = hipMalloc(&net->uhat, sizeof(float) * px);
  if (e == hipSuccess) e = hipMalloc(&net->vstar, sizeof(float) * px);
  if (e == hipSuccess) e = hipMalloc(&net->mask, px);
  if (e != hipSuccess) {
    free_acts(net);
    if (e == hipErrorOutOfMemory) return ctx_fail(net->ctx, SLHJB_E_NOMEM, "network activations");
    return net_hip(net, e, "network activations");
  }
  net->cap_px = px;
  return SLHJB_OK;
}

int pack(slhjb_net* net) {
  const hipStream_t s = ctx_stream(net->ctx);
  for (int l = 0; l < net->L; ++l)
    NET_TRY(launch_pack_weights(net->params + net->w_off[l], net->cout[l], net->cin[l], net->wt[l], net->wtt[l], s));
  return SLHJB_OK;
}

// pad: how far a window may reach past the frame (the U-Net's whole-frame inference)
int check_samples(slhjb_net* net, const slhjb_net_sample* smp, int count, int crop, bool need_target, int pad = 0) {
  if (!smp || count < 1 || count > kMaxImages || crop < 1 || crop > 4096)
    return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "need samples, 1 <= count <= 256, 1 <= crop <= 4096");
  if (net->arch == 1 && crop % 8 != 0)
    return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "the U-Net takes crops of a multiple of 8 pixels");
  for (int k = 0; k < count; ++k) {
    const slhjb_net_sample& q = smp[k];
    if (!q.v_hat || !q.node_class || (need_target && !q.v_star) || q.n < 1 || q.x0 < 0 || q.y0 < 0 ||
        q.x0 + crop > q.n + pad || q.y0 + crop > q.n + pad || !(q.eps > 0.0f) || !isfinite(q.eps) ||
        (!q.speed && !(q.speed_const > 0.0f)))
      return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "sample " + std::to_string(k) + " is invalid");
  }
  return SLHJB_OK;
}

// crops -> features -> conv layers -> head (delta)
int forward_core(slhjb_net* net, const slhjb_net_sample* smp, int count, int crop) {
  const long long px = (long long)count * crop * crop;
  int st = ensure_acts(net, px);
  if (st != SLHJB_OK) return st;
  const hipStream_t s = ctx_stream(net->ctx);
  // the pinned source table may still be read by the previous call's crop kernel
  NET_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < count; ++k) {
    const slhjb_net_sample& q = smp[k];
    CropSrc& c = net->h_src[k];
    c.uhat = q.v_hat;
    c.vstar = q.v_star;
    c.speed = q.speed;
    c.cls = q.node_class;
    c.speed_const = q.speed_const;
    c.leps = (float)(log10((double)q.eps) + 3.0);
    c.n = q.n;
    c.x0 = q.x0;
    c.y0 = q.y0;
  }
  NET_TRY(hipMemcpyAsync(net->d_src, net->h_src, sizeof(CropSrc) * count, hipMemcpyHostToDevice, s));
  int margin = 0;  // receptive-field radius: the sum of the dilations, or the U-Net's
  for (int l = 0; l < net->L; ++l) margin += net->dil[l];
  if (net->arch == 1) margin = kUNetMargin;
  NET_TRY(launch_crops(kCin0, net->d_src, count, crop, margin, net->feat, net->uhat, net->vstar, net->mask, s));
  if (net->arch == 1) {
    auto conv = [&](int l, const uint16_t* in) -> hipError_t {
      const int S = crop >> net->level[l];
      return launch_conv3x3(net->cin[l], net->cout[l], 0, in, net->wt[l], net->params + net->b_off[l], nullptr,
                            count, S, S, 1, 1, net->act[l], s);
    };
    uint16_t** A = net->act;
    NET_TRY(conv(0, net->feat));
    NET_TRY(conv(1, A[0]));
    for (int lv = 0; lv < 3; ++lv) {  // pool, then the two convolutions of the level below
      const int S = crop >> lv;
      NET_TRY(launch_pool2(A[2 * lv + 1], count, S, S, net->cout[2 * lv + 1], net->pool[lv], s));
      NET_TRY(conv(2 * lv + 2, net->pool[lv]));
      NET_TRY(conv(2 * lv + 3, A[2 * lv + 2]));
    }
    for (int lv = 2; lv >= 0; --lv) {  // upsample and concatenate with the skip, two convolutions
      const int S = crop >> lv;
      const int below = 2 * (2 - lv) + 7;  // out7, out9, out11: the last output of the level below
      const int skip = 2 * lv + 1;          // out5, out3, out1
      NET_TRY(launch_upcat(A[below], A[skip], count, S, S, net->cout[below], net->cout[skip], net->cat[lv], s));
      NET_TRY(conv(below + 1, net->cat[lv]));
      NET_TRY(conv(below + 2, A[below + 1]));
    }
  } else {
    for (int l = 0; l < net->L; ++l)
      NET_TRY(launch_conv3x3(net->cin[l], net->C, 0, l == 0 ? net->feat : net->act[l - 1], net->wt[l],
                             net->params + net->b_off[l], nullptr, count, crop, crop, net->dil[l], 1, net->act[l], s));
  }
  NET_TRY(launch_head_fwd(net->C, net->act[net->L - 1], net->params + net->hw_off, net->params + net->hb_off, px,
                          net->delta, s));
  return SLHJB_OK;
}

// Backward pass of the U-Net from the head gradient in gact[13]; the weight and bias gradients
// accumulate into net->grads (already zeroed).
int unet_backward(slhjb_net* net, int count, int crop) {
  const hipStream_t s = ctx_stream(net->ctx);
  uint16_t** A = net->act;
  uint16_t** G = net->gact;
  // weight gradient of layer l (input x), then the input gradient into gx, gated by the input
  // when `gated` (not for pooled inputs: their producer's ReLU gates after the unpooling)
  auto back = [&](int l, const uint16_t* x, uint16_t* gx, bool gated) -> hipError_t {
    const int S = crop >> net->level[l];
    hipError_t e = launch_conv3x3_wgrad(net->cin[l], net->cout[l], x, G[l], count, S, S, 1, net->grads + net->w_off[l],
                                        net->grads + net->b_off[l], net->wwork, s);
    if (e == hipSuccess && gx)
      e = launch_conv3x3(net->cin[l], net->cout[l], 1, G[l], net->wtt[l], nullptr, gated ? x : nullptr, count, S, S, 1,
                         0, gx, s);
    return e;
  };
  for (int lv = 0; lv <= 2; ++lv) {  // decoder, top level first
    const int below = 2 * (2 - lv) + 7, skip = 2 * lv + 1;
    const int S = crop >> lv;
    NET_TRY(back(below + 2, A[below + 1], G[below + 1], true));
    NET_TRY(back(below + 1, net->cat[lv], net->gcat[lv], true));
    NET_TRY(launch_upcat_bwd(net->gcat[lv], count, S, S, net->cout[below], net->cout[skip], G[below], s));
  }
  // bottom: out7 <- out6 <- pool2
  NET_TRY(back(7, A[6], G[6], true));
  NET_TRY(back(6, net->pool[2], net->gpool[2], false));
  for (int lv = 2; lv >= 0; --lv) {  // encoder, bottom level first
    const int S = crop >> lv;
    const int b = 2 * lv + 1;  // out5, out3, out1
    NET_TRY(launch_skip_combine(A[b], net->gcat[lv], net->cout[2 * (2 - lv) + 7], net->gpool[lv], count, S, S,
                                net->cout[b], G[b], s));
    NET_TRY(back(b, A[b - 1], G[b - 1], true));
    if (lv > 0) NET_TRY(back(b - 1, net->pool[lv - 1], net->gpool[lv - 1], false));
    else NET_TRY(back(0, net->feat, nullptr, false));
  }
  return SLHJB_OK;
}

}  // namespace

extern "C" {

int slhjb_net_create(slhjb_ctx* ctx, const slhjb_net_config* cfg, slhjb_net** out) {
  if (!ctx || !cfg || !out) return SLHJB_E_INVALID_ARG;
  *out = nullptr;
  if (cfg->arch != 0 && cfg->arch != 1) return ctx_fail(ctx, SLHJB_E_INVALID_ARG, "arch must be 0 or 1");
  if (cfg->arch == 0) {
    if (cfg->layers < 1 || cfg->layers > 12 || cfg->channels != 32)
      return ctx_fail(ctx, SLHJB_E_INVALID_ARG, "need 1 <= layers <= 12 and channels == 32");
    for (int l = 0; l < cfg->layers; ++l)
      if (cfg->dilation[l] < 1 || cfg->dilation[l] > 32)
        return ctx_fail(ctx, SLHJB_E_INVALID_ARG, "dilation in 1..32");
  }
  hipError_t e = hipSetDevice(ctx_device(ctx));
  if (e != hipSuccess) return ctx_hip_fail(ctx, e, "hipSetDevice");
  slhjb_net* net = new (std::nothrow) slhjb_net();
  if (!net) return SLHJB_E_NOMEM;
  net->ctx = ctx;
  net->arch = cfg->arch;
  net->L = cfg->arch == 1 ? kMaxLayers : cfg->layers;
  net->C = 32;  // channels of the last layer (the head's input)
  int64_t off = 0;
  for (int l = 0; l < net->L; ++l) {
    net->dil[l] = cfg->arch == 1 ? 1 : cfg->dilation[l];
    net->cin[l] = cfg->arch == 1 ? kUNet[l].cin : (l == 0 ? kCin0 : net->C);
    net->cout[l] = cfg->arch == 1 ? kUNet[l].cout : net->C;
    net->level[l] = cfg->arch == 1 ? kUNet[l].level : 0;
    net->w_off[l] = off;
    off += 9LL * net->cout[l] * net->cin[l];
    net->b_off[l] = off;
    off += net->cout[l];
  }
  net->hw_off = off;
  off += net->C;
  net->hb_off = off;
  off += 1;
  net->nparam = off;
  e = hipMalloc(&net->params, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&net->grads, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&net->wwork, sizeof(float) * kWgradWorkFloats);
  if (e == hipSuccess) e = hipMalloc(&net->m1, sizeof(float) * off);
  if (e == hipSuccess) e = hipMalloc(&net->m2, sizeof(float) * off);
  for (int l = 0; l < net->L && e == hipSuccess; ++l) {
    e = hipMalloc(&net->wt[l], sizeof(uint16_t) * 9 * net->cout[l] * net->cin[l]);
    if (e == hipSuccess) e = hipMalloc(&net->wtt[l], sizeof(uint16_t) * 9 * net->cout[l] * net->cin[l]);
  }
  if (e == hipSuccess) e = hipMalloc(&net->d_src, sizeof(CropSrc) * kMaxImages);
  if (e == hipSuccess) e = hipHostMalloc(&net->h_src, sizeof(CropSrc) * kMaxImages, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&net->d_acc, sizeof(float) * 4);
  if (e == hipSuccess) e = hipHostMalloc(&net->h_acc, sizeof(float) * 4, hipHostMallocDefault);
  const hipStream_t s = ctx_stream(ctx);
  if (e == hipSuccess) e = launch_zero_f32(net->params, off, s);
  if (e == hipSuccess) e = launch_zero_f32(net->grads, off, s);
  if (e == hipSuccess) e = launch_zero_f32(net->m1, off, s);
  if (e == hipSuccess) e = launch_zero_f32(net->m2, off, s);
  if (e == hipSuccess && pack(net) != SLHJB_OK) e = hipErrorUnknown;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    const int st = ctx_hip_fail(ctx, e, "network allocation");
    slhjb_net_destroy(net);
    return e == hipErrorOutOfMemory ? SLHJB_E_NOMEM : st;
  }
  *out = net;
  return SLHJB_OK;
}

int slhjb_net_destroy(slhjb_net* net) {
  if (!net) return SLHJB_E_INVALID_ARG;
  hipSetDevice(ctx_device(net->ctx));
  hipStreamSynchronize(ctx_stream(net->ctx));
  free_acts(net);
  for (void* p : {(void*)net->params, (void*)net->grads, (void*)net->wwork, (void*)net->m1, (void*)net->m2,
                  (void*)net->d_src, (void*)net->d_acc})
    if (p) hipFree(p);
  for (int l = 0; l < kMaxLayers; ++l) {
    if (net->wt[l]) hipFree(net->wt[l]);
    if (net->wtt[l]) hipFree(net->wtt[l]);
  }
  if (net->h_src) hipHostFree(net->h_src);
  if (net->h_acc) hipHostFree(net->h_acc);
  delete net;
  return SLHJB_OK;
}

int64_t slhjb_net_param_count(const slhjb_net* net) { return net ? net->nparam : -1; }

int slhjb_net_set_params(slhjb_net* net, const float* host) {
  if (!net || !host) return SLHJB_E_INVALID_ARG;
  for (int64_t i = 0; i < net->nparam; ++i)
    if (!isfinite(host[i])) return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "non-finite parameter");
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  const hipStream_t s = ctx_stream(net->ctx);
  NET_TRY(hipMemcpyAsync(net->params, host, sizeof(float) * net->nparam, hipMemcpyHostToDevice, s));
  NET_TRY(launch_zero_f32(net->m1, net->nparam, s));
  NET_TRY(launch_zero_f32(net->m2, net->nparam, s));
  net->step = 0;
  const int st = pack(net);
  if (st != SLHJB_OK) return st;
  NET_TRY(hipStreamSynchronize(s));  // the host array is pageable
  return SLHJB_OK;
}

int slhjb_net_get_params(slhjb_net* net, float* host) {
  if (!net || !host) return SLHJB_E_INVALID_ARG;
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  const hipStream_t s = ctx_stream(net->ctx);
  NET_TRY(hipMemcpyAsync(host, net->params, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, s));
  NET_TRY(hipStreamSynchronize(s));
  return SLHJB_OK;
}

int slhjb_net_get_grads(slhjb_net* net, float* host) {
  if (!net || !host) return SLHJB_E_INVALID_ARG;
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  const hipStream_t s = ctx_stream(net->ctx);
  NET_TRY(hipMemcpyAsync(host, net->grads, sizeof(float) * net->nparam, hipMemcpyDeviceToHost, s));
  NET_TRY(hipStreamSynchronize(s));
  return SLHJB_OK;
}

int slhjb_net_forward(slhjb_net* net, const slhjb_net_sample* samples, int32_t count, int32_t crop,
                      float* delta_out) {
  if (!net) return SLHJB_E_INVALID_ARG;
  if (!delta_out) return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "delta_out is NULL");
  int st = check_samples(net, samples, count, crop, false);
  if (st != SLHJB_OK) return st;
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  st = forward_core(net, samples, count, crop);
  if (st != SLHJB_OK) return st;
  const hipStream_t s = ctx_stream(net->ctx);
  NET_TRY(hipMemcpyAsync(delta_out, net->delta, sizeof(float) * count * crop * crop, hipMemcpyDeviceToDevice, s));
  NET_TRY(hipStreamSynchronize(s));
  return SLHJB_OK;
}

int slhjb_net_loss_grad(slhjb_net* net, const slhjb_net_sample* samples, int32_t count, int32_t crop,
                        double* loss_out) {
  if (!net) return SLHJB_E_INVALID_ARG;
  int st = check_samples(net, samples, count, crop, true);
  if (st != SLHJB_OK) return st;
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  st = forward_core(net, samples, count, crop);
  if (st != SLHJB_OK) return st;
  const hipStream_t s = ctx_stream(net->ctx);
  const long long px = (long long)count * crop * crop;
  // The loss is normalised by the number N of FREE pixels: the backward pass runs with weight 1
  // per pixel and the gradients are scaled by 1/N at the end, once N has been counted.
  NET_TRY(launch_zero_f32(net->d_acc, 4, s));
  NET_TRY(launch_zero_f32(net->grads, net->nparam, s));
  uint16_t* dy = net->arch == 1 ? net->gact[net->L - 1] : net->g[0];
  uint16_t* dx = net->g[1];
  NET_TRY(launch_loss_head_bwd(net->C, net->delta, net->uhat, net->vstar, net->mask, px, 1.0f,
                               net->act[net->L - 1], net->params + net->hw_off, dy, net->grads + net->hw_off,
                               net->grads + net->hb_off, net->d_acc, s));
  if (net->arch == 1) {
    st = unet_backward(net, count, crop);
    if (st != SLHJB_OK) return st;
  } else {
    for (int l = net->L - 1; l >= 0; --l) {
      const uint16_t* x = l == 0 ? net->feat : net->act[l - 1];
      NET_TRY(launch_conv3x3_wgrad(net->cin[l], net->C, x, dy, count, crop, crop, net->dil[l],
                                   net->grads + net->w_off[l], net->grads + net->b_off[l], net->wwork, s));
      if (l > 0) {
        NET_TRY(launch_conv3x3(net->cin[l], net->C, 1, dy, net->wtt[l], nullptr, net->act[l - 1], count, crop, crop,
                               net->dil[l], 0, dx, s));
        std::swap(dx, dy);
      }
    }
  }
  NET_TRY(launch_count_nonzero_u8(net->mask, px, (unsigned*)(net->d_acc + 1), s));
  NET_TRY(hipMemcpyAsync(net->h_acc, net->d_acc, sizeof(float) * 4, hipMemcpyDeviceToHost, s));
  NET_TRY(hipStreamSynchronize(s));
  unsigned nfree;
  memcpy(&nfree, &net->h_acc[1], sizeof(nfree));
  if (nfree == 0) return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "the crops hold no FREE node");
  NET_TRY(launch_scale_f32(net->grads, net->nparam, (float)(1.0 / (double)nfree), s));
  if (loss_out) *loss_out = (double)net->h_acc[0] / (double)nfree;
  return SLHJB_OK;
}

int slhjb_net_adam_step(slhjb_net* net, float lr) {
  if (!net) return SLHJB_E_INVALID_ARG;
  if (!(lr > 0.0f) || !isfinite(lr)) return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "lr must be > 0");
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  const hipStream_t s = ctx_stream(net->ctx);
  net->step += 1;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, net->step), c2 = 1.0 - pow(b2, net->step);
  // p -= lr m_hat / (sqrt(v_hat) + eps) with m_hat = m / c1, v_hat = v / c2
  const float lr_t = (float)(lr * sqrt(c2) / c1), eps_t = (float)(eps * sqrt(c2));
  NET_TRY(launch_adam(net->params, net->grads, net->m1, net->m2, net->nparam, lr_t, (float)b1, (float)b2, eps_t, s));
  return pack(net);
}

int slhjb_net_warm_start(slhjb_net* net, const slhjb_problem* problem, const float* v_hat, float* v_out) {
  if (!net) return SLHJB_E_INVALID_ARG;
  if (!problem || !v_hat || !v_out) return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "problem, v_hat, v_out needed");
  if (problem->n < 3 || problem->n > 4096 || !problem->node_class || !(problem->eps > 0.0f))
    return ctx_fail(net->ctx, SLHJB_E_INVALID_ARG, "need 3 <= n <= 4096, node_class and eps > 0");
  NET_TRY(hipSetDevice(ctx_device(net->ctx)));
  slhjb_net_sample q;
  memset(&q, 0, sizeof(q));
  q.v_hat = v_hat;
  q.v_star = nullptr;
  q.speed = problem->speed;
  q.speed_const = problem->speed_const;
  q.node_class = problem->node_class;
  q.eps = problem->eps;
  q.n = problem->n;
  // the U-Net's window: the frame padded to a multiple of 8 (edge replication)
  const int S = net->arch == 1 ? (problem->n + 7) / 8 * 8 : problem->n;
  int st = check_samples(net, &q, 1, S, false, S - problem->n);
  if (st != SLHJB_OK) return st;
  st = forward_core(net, &q, 1, S);
  if (st != SLHJB_OK) return st;
  const hipStream_t s = ctx_stream(net->ctx);
  NET_TRY(launch_project(net->uhat, net->delta, problem->node_class, problem->n, S, problem->target_value,
                         problem->v_out, v_out, s));
  NET_TRY(hipStreamSynchronize(s));
  return SLHJB_OK;
}

}  // extern "C"
