// Learned warm start: a small dilated convolutional network that maps the upsampled coarse
// solution and the problem data to a correction of u_hat, with its inference and training
// kernels (a serving addition beside the paper's own u_hat start; the SL iteration that follows
// converges to the same fixed point from any start).
//
// Layout: activations NHWC in bfloat16 ([image][y][x][channel]); conv weights per layer as
// Wt[tap][c_out][c_in] (tap = 3 x 3 dilated offsets, row-major) plus the transpose
// WtT[tap][c_in][c_out] for the data gradient; FP32 master parameters, gradients and Adam
// moments. The 3 x 3 convolutions are implicit GEMMs on the 16 x 16 x 16 BF16 matrix cores with
// FP32 accumulation:
//   forward   Y[p][co]  = b[co] + sum_t sum_ci X[p + off_t][ci] Wt[t][co][ci]          (then ReLU)
//   data grad dX[p][ci] = (X[p][ci] > 0) sum_t sum_co dY[p - off_t][co] WtT[t][ci][co]
//   weight grad dW[t][co][ci] = sum_p dY[p][co] X[p + off_t][ci]
// with zero padding outside each image. The 1 x 1 head (C -> 1), the loss and Adam run on the
// vector ALUs in FP32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace slhjb {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bfloat16 bits (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Operand fragments of v_mfma_f32_16x16x16_bf16 (64 lanes): lane l holds
//   A[l % 16][4 (l / 16) + j],  B[4 (l / 16) + j][l % 16],  D[4 (l / 16) + j][l % 16],  j = 0..3.
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ v4s load4(const uint16_t* p) {
  // four consecutive bfloat16 (8-byte aligned: channel offsets are multiples of 4)
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  v4s r;
  r.x = (short)(u.x & 0xffffu);
  r.y = (short)(u.x >> 16);
  r.z = (short)(u.y & 0xffffu);
  r.w = (short)(u.y >> 16);
  return r;
}

// ---- 3 x 3 dilated convolution, forward (MODE 0) or data gradient (MODE 1) ------------------
// One workgroup = 64 consecutive pixels of one row of one image, four wavefronts of 16 pixels;
// each wavefront computes its 16 pixels x COUT channels as COUT/16 MFMA blocks over
// K = 9 taps x CIN channels. MODE 0 reads X (CIN channels) and Wt, adds the bias and applies
// ReLU; MODE 1 reads dY (CIN = the layer's output channels) with negated offsets and WtT, and
// multiplies by the ReLU mask of the layer input `gate` (nullable).
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void conv3x3_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ gate, int H, int W, int dil,
                                                      int relu, uint16_t* __restrict__ out) {
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels");
  constexpr int NB = COUT / 16;
  const int img = blockIdx.z, y = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = blockIdx.x * 64 + wave * 16 + (lane & 15);  // the A-row pixel of this lane
  const int kg = (lane >> 4) * 4;                              // this lane's k offset in a block
  const size_t img_off = (size_t)img * H * W;
  v4f acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    int oy = (t / 3 - 1) * dil, ox = (t % 3 - 1) * dil;
    if (MODE == 1) {
      oy = -oy;
      ox = -ox;
    }
    const int yy = y + oy, xx = px + ox;
    const bool inb = yy >= 0 && yy < H && xx >= 0 && xx < W && px < W;
    const uint16_t* src = in + (img_off + (size_t)(inb ? yy : 0) * W + (inb ? xx : 0)) * CIN;
#pragma unroll
    for (int cb = 0; cb < CIN; cb += 16) {
      v4s a = inb ? load4(src + cb + kg) : v4s{0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // B[k][n] = weight of input channel cb + k for output channel 16 b + n
        const v4s bw = load4(w + ((size_t)t * COUT + 16 * b + (lane & 15)) * CIN + cb + kg);
        acc[b] = mfma16(a, bw, acc[b]);
      }
    }
  }
  // D rows are pixels 4 (lane / 16) + j of the wavefront, column = output channel
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int co = 16 * b + (lane & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = blockIdx.x * 64 + wave * 16 + kg + j;
      if (p >= W) continue;
      const size_t o = (img_off + (size_t)y * W + p) * COUT + co;
      float v = acc[b][j];
      if (MODE == 0) {
        v += bias[co];
        if (relu) v = fmaxf(v, 0.0f);
      } else if (gate) {
        v = gate[o] != 0 && !(gate[o] & 0x8000u) ? v : 0.0f;  // input > 0 (bf16 bits: nonzero, sign clear)
      }
      out[o] = f2bf(v);
    }
  }
}

// ---- weight gradient -------------------------------------------------------------------------
// grid (chunks, 9 taps). A workgroup sums over `chunk` consecutive pixels (flattened over the
// batch) for one tap: A[m = co][k = p] = dY[p][co], B[k = p][n = ci] = X[p + off_t][ci]; the four
// wavefronts take interleaved 16-pixel steps, reduce through LDS, and one atomic per weight adds
// the workgroup's sum to dW[t][co][ci] (FP32).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const uint16_t* __restrict__ x,
                                                            const uint16_t* __restrict__ dy, int images, int H,
                                                            int W, int dil, int chunk, float* __restrict__ dw) {
  constexpr int MB = COUT / 16, NB = CIN / 16;
  __shared__ float red[4][COUT * CIN];
  const int t = blockIdx.y;
  const int oy = (t / 3 - 1) * dil, ox = (t % 3 - 1) * dil;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kg = (lane >> 4) * 4;
  const long long total = (long long)images * H * W;
  const long long p0 = (long long)blockIdx.x * chunk;
  v4f acc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[m][nb] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int s = wave * 16; s < chunk; s += 64) {
    // this lane's four pixels p0 + s + kg + j
    v4s a[MB], b[NB];
#pragma unroll
    for (int m = 0; m < MB; ++m) a[m] = v4s{0, 0, 0, 0};
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) b[nb] = v4s{0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long p = p0 + s + kg + j;
      if (p >= total) continue;
      const int img = (int)(p / ((long long)H * W));
      const int rem = (int)(p - (long long)img * H * W);
      const int y = rem / W, xx = rem - y * W;
      const uint16_t* g = dy + (size_t)p * COUT + (lane & 15);
#pragma unroll
      for (int m = 0; m < MB; ++m) a[m][j] = (short)g[16 * m];
      const int sy = y + oy, sx = xx + ox;
      if (sy >= 0 && sy < H && sx >= 0 && sx < W) {
        const uint16_t* q = x + (((size_t)img * H + sy) * W + sx) * CIN + (lane & 15);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) b[nb][j] = (short)q[16 * nb];
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = mfma16(a[m], b[nb], acc[m][nb]);
  }
  // D[m = co][n = ci]: lane holds co = 16 m + kg + j, ci = 16 nb + lane % 16
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wave][(16 * m + kg + j) * CIN + 16 * nb + (lane & 15)] = acc[m][nb][j];
  __syncthreads();
  for (int e = threadIdx.x; e < COUT * CIN; e += 256) {
    const float v = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
    atomicAdd(&dw[(size_t)t * COUT * CIN + e], v);
  }
}

// bias gradient: db[co] += sum over the chunk's pixels of dY[p][co]
template <int COUT>
__global__ __launch_bounds__(256) void bias_grad_kernel(const uint16_t* __restrict__ dy, long long total, int chunk,
                                                        float* __restrict__ db) {
  __shared__ float red[256];
  const int co = threadIdx.x % COUT, part = threadIdx.x / COUT;
  constexpr int parts = 256 / COUT;
  const long long p0 = (long long)blockIdx.x * chunk;
  float s = 0.0f;
  for (int k = part; k < chunk; k += parts) {
    const long long p = p0 + k;
    if (p < total) s += bf2f(dy[(size_t)p * COUT + co]);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (part == 0) {
    float v = 0.0f;
    for (int q = 0; q < parts; ++q) v += red[q * COUT + co];
    atomicAdd(&db[co], v);
  }
}

// ---- head, loss, features, projection ----------------------------------------------------------
// delta[p] = hb + sum_c h[p][c] hw[c]
template <int C>
__global__ void head_fwd_kernel(const uint16_t* __restrict__ h, const float* __restrict__ hw, const float* __restrict__ hb,
                                long long total, float* __restrict__ delta) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= total) return;
  float s = hb[0];
#pragma unroll
  for (int c = 0; c < C; ++c) s = fmaf(bf2f(h[(size_t)p * C + c]), hw[c], s);
  delta[p] = s;
}

// Loss on FREE nodes of the batch, L = (1/N) sum (u_hat + delta - v*)^2 with N the number of
// masked pixels: ddelta = 2 (u_hat + delta - v*) / N; loss_acc[0] += the squared errors (then / N
// on the host); also the head gradient dh[p][c] = ddelta hw[c] (h > 0), dhw, dhb.
template <int C>
__global__ __launch_bounds__(256) void loss_head_bwd_kernel(const float* __restrict__ delta,
                                                            const float* __restrict__ uhat,
                                                            const float* __restrict__ vstar,
                                                            const uint8_t* __restrict__ mask, long long total,
                                                            float inv_n, const uint16_t* __restrict__ h,
                                                            const float* __restrict__ hw, uint16_t* __restrict__ dh,
                                                            float* __restrict__ dhw, float* __restrict__ dhb,
                                                            float* __restrict__ loss_acc) {
  __shared__ float sw[C + 2][4];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  float g = 0.0f, sq = 0.0f;
  if (p < total && mask[p]) {
    const float e = uhat[p] + delta[p] - vstar[p];
    sq = e * e;
    g = 2.0f * e * inv_n;
  }
  float part[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float hv = 0.0f;
    if (p < total) {
      hv = bf2f(h[(size_t)p * C + c]);
      dh[(size_t)p * C + c] = f2bf(hv > 0.0f ? g * hw[c] : 0.0f);
    }
    part[c] = g * hv;
  }
  // block sums of dhw, dhb and the loss: wavefront reduction, then LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float v = part[c];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sw[c][wave] = v;
  }
  float gv = g, sv = sq;
  for (int off = 32; off > 0; off >>= 1) {
    gv += __shfl_xor(gv, off, 64);
    sv += __shfl_xor(sv, off, 64);
  }
  if (lane == 0) {
    sw[C][wave] = gv;
    sw[C + 1][wave] = sv;
  }
  __syncthreads();
  if (threadIdx.x < C + 2) {
    const int c = threadIdx.x;
    const float v = (sw[c][0] + sw[c][1]) + (sw[c][2] + sw[c][3]);
    if (c < C) atomicAdd(&dhw[c], v);
    else if (c == C) atomicAdd(dhb, v);
    else atomicAdd(loss_acc, v);
  }
}

// Training crops (and whole frames for inference): image k of the batch is the S x S window at
// (x0, y0) of its source frame (side n). Features NHWC, CIN channels:
// [u_hat, c, target mask, log10(eps) + 3, 1 / (1 + d / 4), 0, ...] with d the distance in cells to
// the nearest side of the box (where the diffusion feet start to leave it); also u_hat, v* and the
// loss mask: FREE nodes at least `margin` cells (the receptive-field radius) from every window edge
// that lies inside the frame, where the zero padding of the window is not the box boundary.
template <int CIN>
__global__ void crop_kernel(const CropSrc* __restrict__ src, int S, int margin, uint16_t* __restrict__ out,
                            float* __restrict__ uhat, float* __restrict__ vstar, uint8_t* __restrict__ mask) {
  const int k = blockIdx.z;
  const int y = blockIdx.y, x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= S) return;
  const CropSrc c = src[k];
  const int gx = c.x0 + x, gy = c.y0 + y;
  const size_t q = (size_t)gy * c.n + gx;
  const size_t dst = ((size_t)k * S + y) * S + x;
  uint16_t* o = out + dst * CIN;
  const float u = c.uhat[q];
  const int d = min(min(gx, gy), min(c.n - 1 - gx, c.n - 1 - gy));
  o[0] = f2bf(u);
  o[1] = f2bf(c.speed ? c.speed[q] : c.speed_const);
  o[2] = f2bf(c.cls[q] == kTarget ? 1.0f : 0.0f);
  o[3] = f2bf(c.leps);
  o[4] = f2bf(1.0f / (1.0f + 0.25f * (float)d));
#pragma unroll
  for (int ch = 5; ch < CIN; ++ch) o[ch] = 0;
  uhat[dst] = u;
  vstar[dst] = c.vstar ? c.vstar[q] : 0.0f;
  bool inner = true;
  if (c.x0 > 0) inner &= x >= margin;
  if (c.y0 > 0) inner &= y >= margin;
  if (c.x0 + S < c.n) inner &= x < S - margin;
  if (c.y0 + S < c.n) inner &= y < S - margin;
  mask[dst] = (c.cls[q] == kFree && inner) ? 1 : 0;
}

// Start of the SL iteration from the network: clamp(u_hat + delta, 0, 1) on FREE nodes, the
// boundary data elsewhere (target_value on TARGET, v_out on OBSTACLE).
__global__ void project_kernel(const float* __restrict__ uhat, const float* __restrict__ delta,
                               const uint8_t* __restrict__ cls, long long total, float target_value, float v_out,
                               float* __restrict__ v) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int c = cls[p];
  v[p] = c == kFree ? fminf(fmaxf(uhat[p] + delta[p], 0.0f), 1.0f) : (c == kTarget ? target_value : v_out);
}

// Adam on the FP32 master parameters (bias-corrected step sizes precomputed on the host).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long long count, float lr_t, float b1, float b2, float eps_t) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
}

// bfloat16 copies of one layer's conv weights: Wt[t][co][ci] and WtT[t][ci][co]
__global__ void pack_weights_kernel(const float* __restrict__ w, int cout, int cin, uint16_t* __restrict__ wt,
                                    uint16_t* __restrict__ wtt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * cout * cin) return;
  const int t = i / (cout * cin), r = i - t * cout * cin;
  const int co = r / cin, ci = r - co * cin;
  const uint16_t b = f2bf(w[i]);
  wt[i] = b;
  wtt[((size_t)t * cin + ci) * cout + co] = b;
}

__global__ void zero_f32_kernel(float* p, long long count) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
}

__global__ void scale_f32_kernel(float* p, long long count, float a) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < count) p[i] *= a;
}

__global__ void count_nonzero_u8_kernel(const uint8_t* __restrict__ m, long long count, unsigned* __restrict__ out) {
  unsigned c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    c += m[i] != 0 ? 1u : 0u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

// ---- launchers ----------------------------------------------------------------------------------
static unsigned blocks_for(long long n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_conv3x3(int cin, int cout, int mode, const uint16_t* in, const uint16_t* w, const float* bias,
                          const uint16_t* gate, int images, int H, int W, int dil, int relu, uint16_t* out,
                          hipStream_t s) {
  dim3 grid((W + 63) / 64, H, images);
#define SLHJB_CONV(CI, CO, MO) conv3x3_kernel<CI, CO, MO><<<grid, 256, 0, s>>>(in, w, bias, gate, H, W, dil, relu, out)
  if (mode == 0) {
    if (cin == 16 && cout == 32) SLHJB_CONV(16, 32, 0);
    else if (cin == 32 && cout == 32) SLHJB_CONV(32, 32, 0);
    else return hipErrorInvalidValue;
  } else {
    // data gradient of a layer cin -> cout: reads cout channels, writes cin channels
    if (cin == 32 && cout == 32) SLHJB_CONV(32, 32, 1);
    else return hipErrorInvalidValue;
  }
#undef SLHJB_CONV
  return hipGetLastError();
}

hipError_t launch_conv3x3_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dy, int images, int H, int W,
                                int dil, float* dw, float* db, hipStream_t s) {
  const long long total = (long long)images * H * W;
  const int chunk = 4096;
  dim3 grid((unsigned)((total + chunk - 1) / chunk), 9);
  if (cin == 16 && cout == 32) conv3x3_wgrad_kernel<16, 32><<<grid, 256, 0, s>>>(x, dy, images, H, W, dil, chunk, dw);
  else if (cin == 32 && cout == 32) conv3x3_wgrad_kernel<32, 32><<<grid, 256, 0, s>>>(x, dy, images, H, W, dil, chunk, dw);
  else return hipErrorInvalidValue;
  if (cout != 32) return hipErrorInvalidValue;
  bias_grad_kernel<32><<<blocks_for(total, 1024), 256, 0, s>>>(dy, total, 1024, db);
  return hipGetLastError();
}

hipError_t launch_head_fwd(int c, const uint16_t* h, const float* hw, const float* hb, long long total, float* delta,
                           hipStream_t s) {
  if (c != 32) return hipErrorInvalidValue;
  head_fwd_kernel<32><<<blocks_for(total, 256), 256, 0, s>>>(h, hw, hb, total, delta);
  return hipGetLastError();
}

hipError_t launch_loss_head_bwd(int c, const float* delta, const float* uhat, const float* vstar, const uint8_t* mask,
                                long long total, float inv_n, const uint16_t* h, const float* hw, uint16_t* dh,
                                float* dhw, float* dhb, float* loss_acc, hipStream_t s) {
  if (c != 32) return hipErrorInvalidValue;
  loss_head_bwd_kernel<32><<<blocks_for(total, 256), 256, 0, s>>>(delta, uhat, vstar, mask, total, inv_n, h, hw, dh,
                                                                  dhw, dhb, loss_acc);
  return hipGetLastError();
}

hipError_t launch_crops(int cin, const CropSrc* src, int images, int S, int margin, uint16_t* feat, float* uhat,
                        float* vstar, uint8_t* mask, hipStream_t s) {
  if (cin != 16) return hipErrorInvalidValue;
  dim3 grid((S + 63) / 64, S, images);
  crop_kernel<16><<<grid, 64, 0, s>>>(src, S, margin, feat, uhat, vstar, mask);
  return hipGetLastError();
}

hipError_t launch_project(const float* uhat, const float* delta, const uint8_t* cls, long long total,
                          float target_value, float v_out, float* v, hipStream_t s) {
  project_kernel<<<blocks_for(total, 256), 256, 0, s>>>(uhat, delta, cls, total, target_value, v_out, v);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long count, float lr_t, float b1, float b2,
                       float eps_t, hipStream_t s) {
  adam_kernel<<<blocks_for(count, 256), 256, 0, s>>>(p, g, m, v, count, lr_t, b1, b2, eps_t);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* w, int cout, int cin, uint16_t* wt, uint16_t* wtt, hipStream_t s) {
  pack_weights_kernel<<<blocks_for(9LL * cout * cin, 256), 256, 0, s>>>(w, cout, cin, wt, wtt);
  return hipGetLastError();
}

hipError_t launch_scale_f32(float* p, long long count, float a, hipStream_t s) {
  scale_f32_kernel<<<blocks_for(count, 256), 256, 0, s>>>(p, count, a);
  return hipGetLastError();
}

hipError_t launch_count_nonzero_u8(const uint8_t* m, long long count, unsigned* out, hipStream_t s) {
  count_nonzero_u8_kernel<<<std::min(blocks_for(count, 256), 1024u), 256, 0, s>>>(m, count, out);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, long long count, hipStream_t s) {
  zero_f32_kernel<<<blocks_for(count, 256), 256, 0, s>>>(p, count);
  return hipGetLastError();
}

}  // namespace slhjb
