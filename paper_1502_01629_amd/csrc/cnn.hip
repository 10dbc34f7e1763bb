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

// Operand fragments of v_mfma_f32_16x16x32_bf16 (gfx950): lane l holds
//   A[l % 16][8 (l / 16) + j],  B[8 (l / 16) + j][l % 16] (j = 0..7),  D[4 (l / 16) + j][l % 16] (j = 0..3).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v4f mfma32(uint4 a, uint4 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ v4s as_v4s(uint2 u) { return __builtin_bit_cast(v4s, u); }

// ---- 3 x 3 (dilated) convolution, forward (MODE 0) or data gradient (MODE 1) -------------------
// Implicit GEMM: M = 64 consecutive pixels of one row of one image, N = COUT channels, K = 9 taps x
// CIN channels. The three input rows the taps read ([x0 - dil, x0 + 64 + dil) x KC channels) are
// staged in LDS one channel chunk of KC at a time, so every input element is read from memory once
// per workgroup instead of once per tap; the weights come through the caches. The four wavefronts
// split the output as CW channel groups x (4 / CW) pixel groups. K steps of 32 channels on the
// 16 x 16 x 32 matrix cores (of 16 on the 16 x 16 x 16 ones when CIN = 16).
// MODE 0 reads X (CIN channels) and Wt[t][co][ci], adds the bias and applies ReLU; MODE 1 reads dY
// (CIN = the layer's output channels) with negated offsets and the transposed weights, and zeroes
// the outputs where `gate` (the layer input, nullable) is not > 0.
template <int CIN, int COUT>
struct ConvShape {
  // staged channel chunk: 64 channels, or the largest of 32 / 16 that divides CIN (96 = 3 x 32)
  static constexpr int KC = CIN % 64 == 0 ? 64 : (CIN % 32 == 0 ? 32 : 16);
  static constexpr int KP = KC + 8;                   // LDS pitch per pixel (bf16): breaks bank conflicts
  static constexpr int KS = CIN % 32 == 0 ? 32 : 16;  // channels per MFMA step
  // channel groups: 4, 2 or 1, whichever divides the COUT / 16 channel blocks (96 = 2 x 3 x 16)
  static constexpr int CW = (COUT / 16) % 4 == 0 ? 4 : ((COUT / 16) % 2 == 0 ? 2 : 1);
  static constexpr int PW = 4 / CW;
  static constexpr int MB = 64 / PW / 16;             // 16-pixel blocks per wavefront
  static constexpr int NB = COUT / CW / 16;           // 16-channel blocks per wavefront
};

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void conv3x3_kernel(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias,
                                                      const uint16_t* __restrict__ gate, int H, int W, int dil,
                                                      int relu, uint16_t* __restrict__ out) {
  using S = ConvShape<CIN, COUT>;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0 && S::NB >= 1 && S::MB >= 1, "channels");
  static_assert(CIN % S::KC == 0 && S::KC % S::KS == 0, "the channel chunks tile CIN");
  static_assert(S::CW * S::NB * 16 == COUT && S::PW * S::MB * 16 == 64, "the wavefronts tile the output");
  extern __shared__ uint16_t xs[];  // [3][XW][KP]
  const int img = blockIdx.z, y = blockIdx.y, x0 = blockIdx.x * 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cw = wave % S::CW, pw = wave / S::CW;
  const int XW = 64 + 2 * dil;
  const int sg = MODE == 0 ? 1 : -1;
  const size_t img_off = (size_t)img * H * W;
  v4f acc[S::MB][S::NB];
#pragma unroll
  for (int m = 0; m < S::MB; ++m)
#pragma unroll
    for (int b = 0; b < S::NB; ++b) acc[m][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  const int kq = lane >> 4, l16 = lane & 15;
  for (int kc = 0; kc < CIN; kc += S::KC) {
    __syncthreads();  // the previous chunk's reads are done
    // stage rows y + sg (r - 1) dil, r = 0..2, in 16-byte pieces (8 channels)
    constexpr int V = S::KC / 8;
    const int total = 3 * XW * V;
    for (int e = threadIdx.x; e < total; e += 256) {
      const int r = e / (XW * V);
      const int rem = e - r * XW * V;
      const int xi = rem / V, c8 = rem - xi * V;
      const int yy = y + sg * (r - 1) * dil, xx = x0 - dil + xi;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = *reinterpret_cast<const uint4*>(in + (img_off + (size_t)yy * W + xx) * CIN + kc + 8 * c8);
      *reinterpret_cast<uint4*>(xs + ((size_t)r * XW + xi) * S::KP + 8 * c8) = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int r = t / 3;
      const int ox = sg * (t % 3 - 1) * dil;
#pragma unroll
      for (int ks = 0; ks < S::KC; ks += S::KS) {
        // B fragments: weights of channels kc + ks + (8 or 4) (l / 16) + j for output channel co
        uint4 bq[S::NB];
        uint2 bh[S::NB];
#pragma unroll
        for (int b = 0; b < S::NB; ++b) {
          const int co = (cw * S::NB + b) * 16 + l16;
          const uint16_t* wp = w + ((size_t)t * COUT + co) * CIN + kc + ks;
          if (S::KS == 32) bq[b] = *reinterpret_cast<const uint4*>(wp + 8 * kq);
          else bh[b] = *reinterpret_cast<const uint2*>(wp + 4 * kq);
        }
#pragma unroll
        for (int m = 0; m < S::MB; ++m) {
          const int px = (pw * S::MB + m) * 16 + l16;
          // staged row r holds y + sg (r - 1) dil: the tap's row in both modes
          const uint16_t* ap = xs + ((size_t)r * XW + px + dil + ox) * S::KP + ks;
          if (S::KS == 32) {
            const uint4 a = *reinterpret_cast<const uint4*>(ap + 8 * kq);
#pragma unroll
            for (int b = 0; b < S::NB; ++b) acc[m][b] = mfma32(a, bq[b], acc[m][b]);
          } else {
            const v4s a = as_v4s(*reinterpret_cast<const uint2*>(ap + 4 * kq));
#pragma unroll
            for (int b = 0; b < S::NB; ++b) acc[m][b] = mfma16(a, as_v4s(bh[b]), acc[m][b]);
          }
        }
      }
    }
  }
  // D rows are pixels 4 (l / 16) + j of the block, columns output channels
#pragma unroll
  for (int m = 0; m < S::MB; ++m)
#pragma unroll
    for (int b = 0; b < S::NB; ++b) {
      const int co = (cw * S::NB + b) * 16 + l16;
      const float bb = MODE == 0 ? bias[co] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = x0 + (pw * S::MB + m) * 16 + 4 * kq + j;
        if (p >= W) continue;
        const size_t o = (img_off + (size_t)y * W + p) * COUT + co;
        float v = acc[m][b][j];
        if (MODE == 0) {
          v += bb;
          if (relu) v = fmaxf(v, 0.0f);
        } else if (gate) {
          v = gate[o] != 0 && !(gate[o] & 0x8000u) ? v : 0.0f;  // input > 0 (bf16 bits: nonzero, sign clear)
        }
        out[o] = f2bf(v);
      }
    }
}

template <int CIN, int COUT>
size_t conv3x3_lds_bytes(int dil) {
  return sizeof(uint16_t) * 3 * (64 + 2 * dil) * ConvShape<CIN, COUT>::KP;
}

// ---- weight gradient -------------------------------------------------------------------------
// dW[t][co][ci] = sum_p dY[p][co] X[p + off_t][ci]: a GEMM with M = COUT, N = CIN and the pixels
// as K. grid (chunks, 9 taps). A workgroup walks `chunk` consecutive pixels (flattened over the
// batch) in steps of 64, staging dY and the tap-shifted X transposed in LDS ([channel][pixel]), so
// that the matrix-core fragments (8 consecutive pixels of one channel) are single 16-byte reads.
// The COUT/16 x CIN/16 output blocks are dealt to the four wavefronts; one atomic per weight and
// workgroup adds the sums to dW (FP32).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const uint16_t* __restrict__ x,
                                                            const uint16_t* __restrict__ dy, int images, int H,
                                                            int W, int dil, int chunk, float* __restrict__ dw) {
  constexpr int MBt = COUT / 16, NBt = CIN / 16, BLK = MBt * NBt;
  constexpr int NBLK = (BLK + 3) / 4;  // output blocks per wavefront
  constexpr int PP = 64 + 8;           // LDS pitch (pixels) of a channel row
  __shared__ uint16_t dyT[COUT * PP];
  __shared__ uint16_t xT[CIN * PP];
  const int t = blockIdx.y;
  const int oy = (t / 3 - 1) * dil, ox = (t % 3 - 1) * dil;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, l16 = lane & 15;
  const long long HW = (long long)H * W, total = (long long)images * HW;
  const long long p0 = (long long)blockIdx.x * chunk;
  v4f acc[NBLK];
#pragma unroll
  for (int q = 0; q < NBLK; ++q) acc[q] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int s = 0; s < chunk; s += 64) {
    __syncthreads();
    // stage 64 pixels: each thread moves 8 channels of one pixel (16 bytes) at a time
    for (int e = threadIdx.x; e < 64 * (COUT / 8); e += 256) {
      const int pl = e / (COUT / 8), c8 = e - pl * (COUT / 8);
      const long long p = p0 + s + pl;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (p < total) v = *reinterpret_cast<const uint4*>(dy + (size_t)p * COUT + 8 * c8);
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) dyT[(8 * c8 + j) * PP + pl] = h[j];
    }
    for (int e = threadIdx.x; e < 64 * (CIN / 8); e += 256) {
      const int pl = e / (CIN / 8), c8 = e - pl * (CIN / 8);
      const long long p = p0 + s + pl;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (p < total) {
        const long long img = p / HW;
        const int rem = (int)(p - img * HW);
        const int yy = rem / W + oy, xx = rem % W + ox;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
          v = *reinterpret_cast<const uint4*>(x + ((size_t)img * HW + (size_t)yy * W + xx) * CIN + 8 * c8);
      }
      const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) xT[(8 * c8 + j) * PP + pl] = h[j];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 64; ks += 32) {
#pragma unroll
      for (int q = 0; q < NBLK; ++q) {
        const int blk = wave + 4 * q;
        if (blk < BLK) {
          const int mb = blk / NBt, nb = blk - mb * NBt;
          const uint4 a = *reinterpret_cast<const uint4*>(dyT + (mb * 16 + l16) * PP + ks + 8 * kq);
          const uint4 b = *reinterpret_cast<const uint4*>(xT + (nb * 16 + l16) * PP + ks + 8 * kq);
          acc[q] = mfma32(a, b, acc[q]);
        }
      }
    }
  }
  // D[co][ci]: lane holds co = 16 mb + 4 (l / 16) + j, ci = 16 nb + l % 16
#pragma unroll
  for (int q = 0; q < NBLK; ++q) {
    const int blk = wave + 4 * q;
    if (blk < BLK) {
      const int mb = blk / NBt, nb = blk - mb * NBt;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        atomicAdd(&dw[((size_t)t * COUT + mb * 16 + 4 * kq + j) * CIN + nb * 16 + l16], acc[q][j]);
    }
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

// ---- U-Net glue: 2 x 2 average pooling, nearest upsampling with the skip concatenation, and their
// backward passes. Activations NHWC bfloat16; each thread moves 8 channels (16 bytes).
__device__ __forceinline__ void unpack8(uint4 v, float f[8]) {
  const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] = bf2f(h[j]);
}
__device__ __forceinline__ uint4 pack8(const float f[8]) {
  uint4 v;
  uint16_t* h = reinterpret_cast<uint16_t*>(&v);
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = f2bf(f[j]);
  return v;
}

// out[b][y][x][c] = bf16(((in[2y][2x] + in[2y][2x+1]) + (in[2y+1][2x] + in[2y+1][2x+1])) / 4)
__global__ void pool2_kernel(const uint16_t* __restrict__ in, long long opix, int Ho, int Wo, int C,
                             uint16_t* __restrict__ out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int V = C / 8;
  if (e >= opix * V) return;
  const long long p = e / V;
  const int c8 = (int)(e - p * V);
  const long long img = p / ((long long)Ho * Wo);
  const int rem = (int)(p - img * Ho * Wo);
  const int y = rem / Wo, x = rem - y * Wo;
  const int W = 2 * Wo;
  const size_t base = ((size_t)img * 2 * Ho + 2 * y) * W + 2 * x;
  float a[8], b[8], c[8], d[8], r[8];
  unpack8(*reinterpret_cast<const uint4*>(in + base * C + 8 * c8), a);
  unpack8(*reinterpret_cast<const uint4*>(in + (base + 1) * C + 8 * c8), b);
  unpack8(*reinterpret_cast<const uint4*>(in + (base + W) * C + 8 * c8), c);
  unpack8(*reinterpret_cast<const uint4*>(in + (base + W + 1) * C + 8 * c8), d);
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = ((a[j] + b[j]) + (c[j] + d[j])) * 0.25f;
  *reinterpret_cast<uint4*>(out + (size_t)p * C + 8 * c8) = pack8(r);
}

// out[b][y][x] = [low[b][y/2][x/2][0..Cu), skip[b][y][x][0..Cs)]
__global__ void upcat_kernel(const uint16_t* __restrict__ low, const uint16_t* __restrict__ skip, long long pix,
                             int H, int W, int Cu, int Cs, uint16_t* __restrict__ out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int C = Cu + Cs, V = C / 8;
  if (e >= pix * V) return;
  const long long p = e / V;
  const int c = 8 * (int)(e - p * V);
  uint4 v;
  if (c < Cu) {
    const long long img = p / ((long long)H * W);
    const int rem = (int)(p - img * H * W);
    const int y = rem / W, x = rem - y * W;
    v = *reinterpret_cast<const uint4*>(low + (((size_t)img * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu + c);
  } else {
    v = *reinterpret_cast<const uint4*>(skip + (size_t)p * Cs + (c - Cu));
  }
  *reinterpret_cast<uint4*>(out + (size_t)p * C + c) = v;
}

// gradient of the upsampled part: glow[b][Y][X][c] = bf16((g[2Y][2X] + g[2Y][2X+1]) + (g[2Y+1][2X] +
// g[2Y+1][2X+1])) over the first Cu channels of g (Cu + Cs channels per pixel)
__global__ void upcat_bwd_kernel(const uint16_t* __restrict__ g, long long opix, int Ho, int Wo, int Cu, int Cs,
                                 uint16_t* __restrict__ glow) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int V = Cu / 8, C = Cu + Cs;
  if (e >= opix * V) return;
  const long long p = e / V;
  const int c8 = (int)(e - p * V);
  const long long img = p / ((long long)Ho * Wo);
  const int rem = (int)(p - img * Ho * Wo);
  const int y = rem / Wo, x = rem - y * Wo;
  const int W = 2 * Wo;
  const size_t base = ((size_t)img * 2 * Ho + 2 * y) * W + 2 * x;
  float a[8], b[8], c[8], d[8], r[8];
  unpack8(*reinterpret_cast<const uint4*>(g + base * C + 8 * c8), a);
  unpack8(*reinterpret_cast<const uint4*>(g + (base + 1) * C + 8 * c8), b);
  unpack8(*reinterpret_cast<const uint4*>(g + (base + W) * C + 8 * c8), c);
  unpack8(*reinterpret_cast<const uint4*>(g + (base + W + 1) * C + 8 * c8), d);
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = (a[j] + b[j]) + (c[j] + d[j]);
  *reinterpret_cast<uint4*>(glow + (size_t)p * Cu + 8 * c8) = pack8(r);
}

// gradient of an encoder output e (C channels) that feeds both the skip (the channels Cu.. of the
// decoder's concatenation gradient gcat) and the pooling (gradient gpool at half resolution):
// out[p][c] = bf16(e[p][c] > 0 ? gcat[p][Cu + c] + gpool[p / 2][c] / 4 : 0)
__global__ void skip_combine_kernel(const uint16_t* __restrict__ e_act, const uint16_t* __restrict__ gcat, int Cu,
                                    const uint16_t* __restrict__ gpool, long long pix, int H, int W, int C,
                                    uint16_t* __restrict__ out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int V = C / 8;
  if (e >= pix * V) return;
  const long long p = e / V;
  const int c = 8 * (int)(e - p * V);
  const long long img = p / ((long long)H * W);
  const int rem = (int)(p - img * H * W);
  const int y = rem / W, x = rem - y * W;
  float a[8], gs[8], gp[8], r[8];
  unpack8(*reinterpret_cast<const uint4*>(e_act + (size_t)p * C + c), a);
  unpack8(*reinterpret_cast<const uint4*>(gcat + (size_t)p * (Cu + C) + Cu + c), gs);
  unpack8(*reinterpret_cast<const uint4*>(gpool + (((size_t)img * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c), gp);
#pragma unroll
  for (int j = 0; j < 8; ++j) r[j] = a[j] > 0.0f ? gs[j] + 0.25f * gp[j] : 0.0f;
  *reinterpret_cast<uint4*>(out + (size_t)p * C + c) = pack8(r);
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
  // a window may reach past the frame (the U-Net's whole-frame inference pads to a multiple of 8):
  // there the nearest frame node is replicated and the loss mask is 0
  const bool in_frame = c.x0 + x < c.n && c.y0 + y < c.n;
  const int gx = min(c.x0 + x, c.n - 1), gy = min(c.y0 + y, c.n - 1);
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
  mask[dst] = (c.cls[q] == kFree && inner && in_frame) ? 1 : 0;
}

// Start of the SL iteration from the network: clamp(u_hat + delta, 0, 1) on FREE nodes, the
// boundary data elsewhere (target_value on TARGET, v_out on OBSTACLE).
// uhat and delta are rows of `pitch` >= n values (the network's window), cls and v rows of n.
__global__ void project_kernel(const float* __restrict__ uhat, const float* __restrict__ delta,
                               const uint8_t* __restrict__ cls, int n, int pitch, float target_value, float v_out,
                               float* __restrict__ v) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= (long long)n * n) return;
  const int y = (int)(p / n), x = (int)(p - (long long)y * n);
  const size_t q = (size_t)y * pitch + x;
  const int c = cls[p];
  v[p] = c == kFree ? fminf(fmaxf(uhat[q] + delta[q], 0.0f), 1.0f) : (c == kTarget ? target_value : v_out);
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

// The (c_in, c_out) pairs of the two networks: the dilated CNN (16 -> 32, 32 -> 32) and the 4-level
// U-Net (32/64/128/128 channels; the decoder's first convolutions read the concatenation of the
// upsampled level below and the skip: 256, 192 and 96 channels).
#define SLHJB_FOR_LAYERS(X) \
  X(16, 32) X(32, 32) X(32, 64) X(64, 64) X(64, 128) X(128, 128) X(256, 128) X(192, 64) X(96, 32)

hipError_t launch_conv3x3(int cin, int cout, int mode, const uint16_t* in, const uint16_t* w, const float* bias,
                          const uint16_t* gate, int images, int H, int W, int dil, int relu, uint16_t* out,
                          hipStream_t s) {
  if (dil < 1 || dil > 32) return hipErrorInvalidValue;
  dim3 grid((W + 63) / 64, H, images);
  // data gradient of a layer cin -> cout: reads cout channels, writes cin channels
#define SLHJB_CONV(CI, CO)                                                                                 \
  if (mode == 0 && cin == CI && cout == CO) {                                                              \
    conv3x3_kernel<CI, CO, 0><<<grid, 256, conv3x3_lds_bytes<CI, CO>(dil), s>>>(in, w, bias, gate, H, W, dil, \
                                                                                relu, out);                \
    return hipGetLastError();                                                                              \
  }                                                                                                        \
  if (mode == 1 && cin == CI && cout == CO && CI != 16) {                                                  \
    conv3x3_kernel<CO, CI, 1><<<grid, 256, conv3x3_lds_bytes<CO, CI>(dil), s>>>(in, w, bias, gate, H, W, dil, \
                                                                                relu, out);                \
    return hipGetLastError();                                                                              \
  }
  SLHJB_FOR_LAYERS(SLHJB_CONV)
#undef SLHJB_CONV
  return hipErrorInvalidValue;
}

hipError_t launch_conv3x3_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dy, int images, int H, int W,
                                int dil, float* dw, float* db, hipStream_t s) {
  const long long total = (long long)images * H * W;
  // about 64 chunks per tap (a multiple of 64 pixels each): enough workgroups to fill the chip,
  // few atomics per weight
  long long chunk = (total + 63) / 64;
  chunk = std::max(2048LL, (chunk + 63) / 64 * 64);
  dim3 grid((unsigned)((total + chunk - 1) / chunk), 9);
  bool done = false;
#define SLHJB_WG(CI, CO)                                                                                    \
  if (!done && cin == CI && cout == CO) {                                                                   \
    conv3x3_wgrad_kernel<CI, CO><<<grid, 256, 0, s>>>(x, dy, images, H, W, dil, (int)chunk, dw);            \
    done = true;                                                                                            \
  }
  SLHJB_FOR_LAYERS(SLHJB_WG)
#undef SLHJB_WG
  if (!done) return hipErrorInvalidValue;
  if (cout == 32) bias_grad_kernel<32><<<blocks_for(total, 1024), 256, 0, s>>>(dy, total, 1024, db);
  else if (cout == 64) bias_grad_kernel<64><<<blocks_for(total, 1024), 256, 0, s>>>(dy, total, 1024, db);
  else if (cout == 128) bias_grad_kernel<128><<<blocks_for(total, 1024), 256, 0, s>>>(dy, total, 1024, db);
  else return hipErrorInvalidValue;
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

hipError_t launch_project(const float* uhat, const float* delta, const uint8_t* cls, int n, int pitch,
                          float target_value, float v_out, float* v, hipStream_t s) {
  project_kernel<<<blocks_for((long long)n * n, 256), 256, 0, s>>>(uhat, delta, cls, n, pitch, target_value, v_out, v);
  return hipGetLastError();
}

hipError_t launch_pool2(const uint16_t* in, int images, int H, int W, int C, uint16_t* out, hipStream_t s) {
  if (H % 2 || W % 2 || C % 8) return hipErrorInvalidValue;
  const long long opix = (long long)images * (H / 2) * (W / 2);
  pool2_kernel<<<blocks_for(opix * (C / 8), 256), 256, 0, s>>>(in, opix, H / 2, W / 2, C, out);
  return hipGetLastError();
}

hipError_t launch_upcat(const uint16_t* low, const uint16_t* skip, int images, int H, int W, int Cu, int Cs,
                        uint16_t* out, hipStream_t s) {
  if (H % 2 || W % 2 || Cu % 8 || Cs % 8) return hipErrorInvalidValue;
  const long long pix = (long long)images * H * W;
  upcat_kernel<<<blocks_for(pix * ((Cu + Cs) / 8), 256), 256, 0, s>>>(low, skip, pix, H, W, Cu, Cs, out);
  return hipGetLastError();
}

hipError_t launch_upcat_bwd(const uint16_t* g, int images, int H, int W, int Cu, int Cs, uint16_t* glow,
                            hipStream_t s) {
  if (H % 2 || W % 2 || Cu % 8 || Cs % 8) return hipErrorInvalidValue;
  const long long opix = (long long)images * (H / 2) * (W / 2);
  upcat_bwd_kernel<<<blocks_for(opix * (Cu / 8), 256), 256, 0, s>>>(g, opix, H / 2, W / 2, Cu, Cs, glow);
  return hipGetLastError();
}

hipError_t launch_skip_combine(const uint16_t* e_act, const uint16_t* gcat, int Cu, const uint16_t* gpool, int images,
                               int H, int W, int C, uint16_t* out, hipStream_t s) {
  if (H % 2 || W % 2 || Cu % 8 || C % 8) return hipErrorInvalidValue;
  const long long pix = (long long)images * H * W;
  skip_combine_kernel<<<blocks_for(pix * (C / 8), 256), 256, 0, s>>>(e_act, gcat, Cu, gpool, pix, H, W, C, out);
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
