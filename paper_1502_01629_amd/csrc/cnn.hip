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

// ---- 3 x 3 convolution with register tiles (dilation 1) --------------------------------------
// The same products as conv3x3_kernel, with a larger output tile per workgroup: TR rows x 64
// pixels x all COUT channels, dealt to the four wavefronts as PWG pixel groups x CWG channel groups
// of MB x NB 16 x 16 blocks. Every weight fragment a wavefront loads serves its MB pixel blocks and
// every staged input fragment its NB channel blocks. The TR + 2 input rows the tile reads are
// staged in LDS one channel chunk at a time. The results go through LDS (bias and ReLU, or the
// ReLU gate of the data gradient, applied on the way) so that each thread writes 16 contiguous
// bytes. Same operands, accumulation order and rounding as conv3x3_kernel.
template <int CIN, int COUT>
struct ConvTile {
  static constexpr int KC = ConvShape<CIN, COUT>::KC;
  static constexpr int KP = ConvShape<CIN, COUT>::KP;
  static constexpr int KS = ConvShape<CIN, COUT>::KS;
  static constexpr int CWG = (COUT == 128 || COUT >= 192) ? 2 : 1;
  static constexpr int PWG = 4 / CWG;
  static constexpr int NB = COUT / 16 / CWG;
  static constexpr int MB = COUT == 32 ? 8 : 4;
  static constexpr int TP = PWG * MB * 16;  // pixels per workgroup
  static constexpr int TR = TP / 64;        // rows per workgroup
  static constexpr int OP = COUT + 8;       // LDS pitch of an output pixel (bf16)
};

template <int CIN, int COUT>
size_t conv3x3_tile_lds_bytes() {
  using S = ConvTile<CIN, COUT>;
  const size_t stage = (size_t)(S::TR + 2) * 66 * S::KP, outs = (size_t)S::TP * S::OP;
  return sizeof(uint16_t) * (stage > outs ? stage : outs);
}

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3x3_tile_kernel(const uint16_t* __restrict__ in,
                                                           const uint16_t* __restrict__ w,
                                                           const float* __restrict__ bias,
                                                           const uint16_t* __restrict__ gate, int H, int W, int relu,
                                                           uint16_t* __restrict__ out) {
  using S = ConvTile<CIN, COUT>;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0 && S::NB >= 1 && S::NB * S::MB <= 32, "tile");
  static_assert(CIN % S::KC == 0 && S::KC % S::KS == 0, "the channel chunks tile CIN");
  static_assert(S::CWG * S::NB * 16 == COUT && S::TP % 64 == 0, "waves tile the output");
  constexpr int XW = 66;
  extern __shared__ uint16_t xs[];  // [TR + 2][XW][KP], then [TP][OP] for the results
  const int img = blockIdx.z, y0 = blockIdx.y * S::TR, x0 = blockIdx.x * 64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cw = wave % S::CWG, pw = wave / S::CWG;
  const int sg = MODE == 0 ? 1 : -1;
  const size_t img_off = (size_t)img * H * W;
  const int kq = lane >> 4, l16 = lane & 15;
  v4f acc[S::MB][S::NB];
#pragma unroll
  for (int m = 0; m < S::MB; ++m)
#pragma unroll
    for (int b = 0; b < S::NB; ++b) acc[m][b] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int kc = 0; kc < CIN; kc += S::KC) {
    __syncthreads();  // the previous chunk's reads are done
    // stage rows y0 - 1 .. y0 + TR, columns x0 - 1 .. x0 + 64, in 16-byte pieces (8 channels),
    // four loads of the thread in flight before their LDS stores
    constexpr int V = S::KC / 8;
    constexpr int total = (S::TR + 2) * XW * V;
    constexpr int SB = 4;
    for (int e0 = 0; e0 < total; e0 += 256 * SB) {
      uint4 v[SB];
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        const int e = e0 + threadIdx.x + 256 * i;
        const int q = e / (XW * V);
        const int rem = e - q * XW * V;
        const int xi = rem / V, c8 = rem - xi * V;
        const int yy = y0 - 1 + q, xx = x0 - 1 + xi;
        v[i] = make_uint4(0u, 0u, 0u, 0u);
        if (e < total && yy >= 0 && yy < H && xx >= 0 && xx < W)
          v[i] = *reinterpret_cast<const uint4*>(in + (img_off + (size_t)yy * W + xx) * CIN + kc + 8 * c8);
      }
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        const int e = e0 + threadIdx.x + 256 * i;
        const int q = e / (XW * V);
        const int rem = e - q * XW * V;
        const int xi = rem / V, c8 = rem - xi * V;
        if (e < total) *reinterpret_cast<uint4*>(xs + ((size_t)q * XW + xi) * S::KP + 8 * c8) = v[i];
      }
    }
    __syncthreads();
    // taps as a loop (not unrolled), so that the weight loads of one tap stay in that tap
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
      const int dy = sg * (t / 3 - 1), dx = sg * (t % 3 - 1);
#pragma unroll
      for (int ks = 0; ks < S::KC; ks += S::KS) {
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
          const int pl = (pw * S::MB + m) * 16 + l16;  // pixel of the tile: row pl / 64, column pl % 64
          const int q = pl / 64 + 1 + dy, xi = pl % 64 + 1 + dx;
          const uint16_t* ap = xs + ((size_t)q * XW + xi) * S::KP + ks;
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
  __syncthreads();  // the staged rows are no longer read
  // D rows are pixels 4 (l / 16) + j of the block, columns output channels
#pragma unroll
  for (int b = 0; b < S::NB; ++b) {
    const int co = (cw * S::NB + b) * 16 + l16;
    const float bb = MODE == 0 ? bias[co] : 0.0f;
#pragma unroll
    for (int m = 0; m < S::MB; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = acc[m][b][j];
        if (MODE == 0) {
          v += bb;
          if (relu) v = fmaxf(v, 0.0f);
        }
        xs[(size_t)((pw * S::MB + m) * 16 + 4 * kq + j) * S::OP + co] = f2bf(v);
      }
  }
  __syncthreads();
  constexpr int V8 = COUT / 8;
  for (int e = threadIdx.x; e < S::TP * V8; e += 256) {
    const int pl = e / V8, c8 = e - pl * V8;
    const int yy = y0 + pl / 64, xx = x0 + pl % 64;
    if (yy >= H || xx >= W) continue;
    const size_t o = (img_off + (size_t)yy * W + xx) * COUT + 8 * c8;
    uint4 v = *reinterpret_cast<const uint4*>(xs + (size_t)pl * S::OP + 8 * c8);
    if (MODE == 1 && gate) {
      // keep the gradient where the layer input is > 0 (bf16 bits: nonzero, sign clear)
      const uint4 gv = *reinterpret_cast<const uint4*>(gate + o);
      const uint32_t gw[4] = {gv.x, gv.y, gv.z, gv.w};
      uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t lo = gw[i] & 0xffffu, hi = gw[i] >> 16;
        const uint32_t keep = ((lo != 0u && !(lo & 0x8000u)) ? 0xffffu : 0u) |
                              ((hi != 0u && !(hi & 0x8000u)) ? 0xffff0000u : 0u);
        vw[i] &= keep;
      }
      v = make_uint4(vw[0], vw[1], vw[2], vw[3]);
    }
    *reinterpret_cast<uint4*>(out + o) = v;
  }
}

// ---- weight and bias gradients ------------------------------------------------------------------
// dW[t][co][ci] = sum_p dY[p][co] X[p + off_t][ci] and db[co] = sum_p dY[p][co]: GEMMs with the
// pixels as K. A workgroup owns a CO_T x CI_T block of (co, ci) for all nine taps and walks `steps`
// consecutive strips (64 pixels of one row of one image). Per strip it stages dY[strip][co block]
// and the three input rows X[y + (ty - 1) dil][x0 - dil .. x0 + 64 + dil][ci block] transposed in
// LDS, as runs of 8 pixels of one channel (one 16-byte matrix-core fragment). The runs are
// strided: run g of the strip holds pixels x0 + g + 8 j (j = 0..7), so a tap's column shift
// tx dil moves a fragment to another whole run (g + tx dil) and every LDS read is an aligned
// 16-byte read. The 8 x 8 transposes (8 channels x 8 pixels) happen in registers while staging.
// The (tap, ci block) units are dealt to the four wavefronts; each loads the dY fragments of its
// co blocks once per K step and reuses them for all its units. The bias gradient is one more
// product per co block, with a B operand of ones. Each workgroup writes its partial sums to its
// own slice of `work` ([tile][strip run][9][CO_T][CI_T] then [CO_T] for the bias, plain stores);
// wgrad_reduce_kernel adds the slices of every tile to dW and db.
template <int CIN, int COUT>
struct WgradShape {
  static constexpr int CO_T = COUT < 64 ? COUT : 64;
  static constexpr int CI_T = CIN % 64 == 0 ? 64 : (CIN % 48 == 0 ? 48 : (CIN % 32 == 0 ? 32 : 16));
  static constexpr int MBt = CO_T / 16, NBt = CI_T / 16;
  static constexpr int UNITS = 9 * NBt;       // (tap, ci block) pairs
  static constexpr int NU = (UNITS + 3) / 4;  // units per wavefront
  static constexpr int DYP = 9;               // LDS pitch of a dY channel, in 16-byte runs (8 + 1)
};

__device__ __forceinline__ uint32_t lohalves(uint32_t a, uint32_t b) { return (a & 0xffffu) | (b << 16); }
__device__ __forceinline__ uint32_t hihalves(uint32_t a, uint32_t b) { return (a >> 16) | (b & 0xffff0000u); }

// v[j] holds channels 0..7 of pixel j; on return o[c] holds pixels 0..7 of channel c
__device__ __forceinline__ void transpose8x8(const uint4 v[8], uint4 o[8]) {
#pragma unroll
  for (int c2 = 0; c2 < 4; ++c2) {
    uint32_t w[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) w[j] = c2 == 0 ? v[j].x : (c2 == 1 ? v[j].y : (c2 == 2 ? v[j].z : v[j].w));
    o[2 * c2] = make_uint4(lohalves(w[0], w[1]), lohalves(w[2], w[3]), lohalves(w[4], w[5]), lohalves(w[6], w[7]));
    o[2 * c2 + 1] = make_uint4(hihalves(w[0], w[1]), hihalves(w[2], w[3]), hihalves(w[4], w[5]), hihalves(w[6], w[7]));
  }
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const uint16_t* __restrict__ x,
                                                            const uint16_t* __restrict__ dy, int images, int H,
                                                            int W, int dil, int steps, float* __restrict__ work) {
  using S = WgradShape<CIN, COUT>;
  static_assert(COUT % S::CO_T == 0 && CIN % S::CI_T == 0 && S::MBt >= 1 && S::MBt <= 4, "tiles");
  extern __shared__ uint4 lds4[];
  const int NG = 8 + 2 * dil;           // runs per staged row and channel
  const int XP = NG + 1;                // LDS pitch of an X channel row, in runs (odd)
  uint4* dyT = lds4;                    // [CO_T][DYP]
  uint4* xT = lds4 + S::CO_T * S::DYP;  // [3][CI_T][XP]
  constexpr int CBLK = CIN / S::CI_T;
  const int co0 = (blockIdx.y / CBLK) * S::CO_T, ci0 = (blockIdx.y % CBLK) * S::CI_T;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, l16 = lane & 15;
  const int NS = (W + 63) / 64;
  const long long nsteps = (long long)images * H * NS;
  const long long s0 = (long long)blockIdx.x * steps;
  v4f acc[S::NU][S::MBt];
#pragma unroll
  for (int u = 0; u < S::NU; ++u)
#pragma unroll
    for (int m = 0; m < S::MBt; ++m) acc[u][m] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  v4f accb = v4f{0.0f, 0.0f, 0.0f, 0.0f};  // bias sums of co block `wave`
  const uint4 ones = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);  // bf16 1.0
  for (int k = 0; k < steps; ++k) {
    const long long st = s0 + k;
    if (st >= nsteps) break;
    const int img = (int)(st / ((long long)H * NS));
    const int rem = (int)(st - (long long)img * H * NS);
    const int y = rem / NS, x0 = (rem % NS) * 64;
    const int SW = min(64, W - x0);
    const size_t img_off = (size_t)img * H * W;
    __syncthreads();  // the previous strip's reads are done
    // dY runs: item (g, c8) -> channels co0 + 8 c8 .. + 7 of pixels x0 + g + 8 j (zero past the row)
    for (int e = threadIdx.x; e < 8 * (S::CO_T / 8); e += 256) {
      const int g = e % 8, c8 = e / 8;
      uint4 v[8], o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = g + 8 * j;
        v[j] = i < SW ? *reinterpret_cast<const uint4*>(dy + (img_off + (size_t)y * W + x0 + i) * COUT + co0 + 8 * c8)
                      : make_uint4(0u, 0u, 0u, 0u);
      }
      transpose8x8(v, o);
#pragma unroll
      for (int c = 0; c < 8; ++c) dyT[(8 * c8 + c) * S::DYP + g] = o[c];
    }
    // X runs: item (ty, sx, c8) -> channels ci0 + 8 c8 .. + 7 of row y + (ty - 1) dil, pixels
    // x0 - dil + sx + 8 j (zero outside the image)
    const int xitems = 3 * NG * (S::CI_T / 8);
    for (int e = threadIdx.x; e < xitems; e += 256) {
      const int c8 = e % (S::CI_T / 8);
      const int rs = e / (S::CI_T / 8);
      const int ty = rs / NG, sx = rs - ty * NG;
      const int yy = y + (ty - 1) * dil;
      uint4 v[8], o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int xx = x0 - dil + sx + 8 * j;
        v[j] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                   ? *reinterpret_cast<const uint4*>(x + (img_off + (size_t)yy * W + xx) * CIN + ci0 + 8 * c8)
                   : make_uint4(0u, 0u, 0u, 0u);
      }
      transpose8x8(v, o);
#pragma unroll
      for (int c = 0; c < 8; ++c) xT[((size_t)ty * S::CI_T + 8 * c8 + c) * XP + sx] = o[c];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int g = 4 * ks + kq;  // this lane's run of the strip
      uint4 a[S::MBt];
#pragma unroll
      for (int m = 0; m < S::MBt; ++m) a[m] = dyT[(m * 16 + l16) * S::DYP + g];
#pragma unroll
      for (int u = 0; u < S::NU; ++u) {
        const int unit = wave + 4 * u;
        if (unit < S::UNITS) {
          const int t = unit % 9, nb = unit / 9;
          const int ty = t / 3, tx = t - 3 * ty;
          const uint4 b = xT[((size_t)ty * S::CI_T + nb * 16 + l16) * XP + g + tx * dil];
#pragma unroll
          for (int m = 0; m < S::MBt; ++m) acc[u][m] = mfma32(a[m], b, acc[u][m]);
        }
      }
#pragma unroll
      for (int m = 0; m < S::MBt; ++m)
        if (m == wave) accb = mfma32(a[m], ones, accb);
    }
  }
  // D[co][ci]: lane holds co = 16 m + 4 (l / 16) + j, ci = 16 nb + l % 16 (tile-local)
  constexpr int TILE = 9 * S::CO_T * S::CI_T;
  float* part = work + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (TILE + S::CO_T);
#pragma unroll
  for (int u = 0; u < S::NU; ++u) {
    const int unit = wave + 4 * u;
    if (unit < S::UNITS) {
      const int t = unit % 9, nb = unit / 9;
#pragma unroll
      for (int m = 0; m < S::MBt; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          part[((size_t)t * S::CO_T + m * 16 + 4 * kq + j) * S::CI_T + nb * 16 + l16] = acc[u][m][j];
    }
  }
  if (wave < S::MBt && l16 == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) part[TILE + wave * 16 + 4 * kq + j] = accb[j];
  }
}

// dW[t][co][ci] += sum over the runs of the partial sums of the tile holding (co, ci); db[co] +=
// the same over the bias sums of the tiles with ci block 0. A workgroup of 512 threads takes 32
// consecutive elements of a tile; its 16 slices of 32 threads sum every 16th run, then LDS adds
// the 16 slice sums in a fixed order.
__global__ __launch_bounds__(512) void wgrad_reduce_kernel(const float* __restrict__ work, int runs, int co_t,
                                                           int ci_t, int cin, int cout, float* __restrict__ dw,
                                                           float* __restrict__ db) {
  __shared__ float red[16][33];
  const int tile = blockIdx.y;
  const int per = 9 * co_t * ci_t + co_t;
  const int el = threadIdx.x & 31, slice = threadIdx.x >> 5;
  const int e = blockIdx.x * 32 + el;
  float sum = 0.0f;
  if (e < per) {
    const float* p = work + (size_t)tile * runs * per + e;
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int r = slice;
    for (; r + 48 < runs; r += 64) {
#pragma unroll
      for (int i = 0; i < 4; ++i) part[i] += p[(size_t)(r + 16 * i) * per];
    }
    for (; r < runs; r += 16) part[0] += p[(size_t)r * per];
    sum = (part[0] + part[1]) + (part[2] + part[3]);
  }
  red[slice][el] = sum;
  __syncthreads();
  if (slice != 0 || e >= per) return;
  float total = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) total += red[i][el];
  const int cblk = cin / ci_t;
  const int co0 = (tile / cblk) * co_t, ci0 = (tile % cblk) * ci_t;
  if (e < 9 * co_t * ci_t) {
    const int t = e / (co_t * ci_t), rem = e - t * co_t * ci_t;
    const int co = rem / ci_t, ci = rem - co * ci_t;
    dw[((size_t)t * cout + co0 + co) * cin + ci0 + ci] += total;
  } else if (tile % cblk == 0 && db) {
    db[co0 + e - 9 * co_t * ci_t] += total;
  }
}

template <int CIN, int COUT>
size_t conv3x3_wgrad_lds_bytes(int dil) {
  using S = WgradShape<CIN, COUT>;
  return sizeof(uint4) * ((size_t)S::CO_T * S::DYP + 3 * (size_t)S::CI_T * (8 + 2 * dil + 1));
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
  for (int q = 0; q < C / 8; ++q) {
    float hv[8];
    unpack8(*reinterpret_cast<const uint4*>(h + (size_t)p * C + 8 * q), hv);
#pragma unroll
    for (int j = 0; j < 8; ++j) s = fmaf(hv[j], hw[8 * q + j], s);
  }
  delta[p] = s;
}

// Loss on FREE nodes of the batch, L = (1/N) sum (u_hat + delta - v*)^2 with N the number of
// masked pixels: ddelta = 2 (u_hat + delta - v*) / N; loss_acc[0] += the squared errors (then / N
// on the host); also the head gradient dh[p][c] = ddelta hw[c] (h > 0), dhw, dhb.
constexpr int kLossPix = 8;
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
  // kLossPix pixels per thread (strided by the block), their sums kept per thread
  float part[C];
#pragma unroll
  for (int c = 0; c < C; ++c) part[c] = 0.0f;
  float g_sum = 0.0f, sq = 0.0f;
  for (int k = 0; k < kLossPix; ++k) {
    const long long p = ((long long)blockIdx.x * kLossPix + k) * blockDim.x + threadIdx.x;
    if (p >= total) break;
    float g = 0.0f;
    if (mask[p]) {
      const float e = uhat[p] + delta[p] - vstar[p];
      sq += e * e;
      g = 2.0f * e * inv_n;
    }
    g_sum += g;
    // the pixel's C channels in 16-byte pieces
#pragma unroll
    for (int q = 0; q < C / 8; ++q) {
      float hv[8];
      unpack8(*reinterpret_cast<const uint4*>(h + (size_t)p * C + 8 * q), hv);
      float gh[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        gh[j] = hv[j] > 0.0f ? g * hw[8 * q + j] : 0.0f;
        part[8 * q + j] += g * hv[j];
      }
      *reinterpret_cast<uint4*>(dh + (size_t)p * C + 8 * q) = pack8(gh);
    }
  }
  const float g = g_sum;
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

// out += the number of nonzero bytes of m: 16 bytes per load, one atomic per workgroup
__global__ __launch_bounds__(256) void count_nonzero_u8_kernel(const uint8_t* __restrict__ m, long long count,
                                                               unsigned* __restrict__ out) {
  __shared__ unsigned red[4];
  unsigned c = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long first = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (long long i = first; i < count / 16; i += stride) {
    const uint4 v = reinterpret_cast<const uint4*>(m)[i];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b) c += ((w[q] >> (8 * b)) & 0xffu) != 0u ? 1u : 0u;
  }
  for (long long i = count / 16 * 16 + first; i < count; i += stride) c += m[i] != 0 ? 1u : 0u;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = (red[0] + red[1]) + (red[2] + red[3]);
    if (t) atomicAdd(out, t);
  }
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
  // dilation 1: the register-tiled kernel; data gradient of a layer cin -> cout: reads cout
  // channels, writes cin channels
#define SLHJB_TILE(CI, CO, MODE)                                                                           \
  {                                                                                                        \
    using S = ConvTile<CI, CO>;                                                                           \
    const size_t lds = conv3x3_tile_lds_bytes<CI, CO>();                                                   \
    if (lds > 64 * 1024) {                                                                                 \
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&conv3x3_tile_kernel<CI, CO, MODE>), \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
      if (e != hipSuccess) return e;                                                                       \
    }                                                                                                      \
    dim3 tgrid((W + 63) / 64, (H + S::TR - 1) / S::TR, images);                                            \
    conv3x3_tile_kernel<CI, CO, MODE><<<tgrid, 256, lds, s>>>(in, w, bias, gate, H, W, relu, out);         \
    return hipGetLastError();                                                                              \
  }
#define SLHJB_CONV(CI, CO)                                                                                 \
  if (dil == 1 && mode == 0 && cin == CI && cout == CO) SLHJB_TILE(CI, CO, 0)                              \
  if (dil == 1 && mode == 1 && cin == CI && cout == CO && CI != 16) SLHJB_TILE(CO, CI, 1)                  \
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
#undef SLHJB_TILE
  return hipErrorInvalidValue;
}

hipError_t launch_conv3x3_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dy, int images, int H, int W,
                                int dil, float* dw, float* db, float* work, hipStream_t s) {
  if (images <= 0 || H <= 0 || W <= 0 || dil < 1 || dil > 32 || !work) return hipErrorInvalidValue;
  const long long nsteps = (long long)images * H * ((W + 63) / 64);
  // about 256 workgroups in all for the 64 x 64 tiles (one per compute unit: their accumulators
  // fill the register file), 512 for the smaller ones; each over a run of consecutive strips
#define SLHJB_WG(CI, CO)                                                                                    \
  if (cin == CI && cout == CO) {                                                                            \
    using S = WgradShape<CI, CO>;                                                                           \
    const int tiles = (CO / S::CO_T) * (CI / S::CI_T);                                                      \
    const long long want = std::max(1LL, (S::CO_T * S::CI_T >= 4096 ? 256LL : 512LL) / tiles);              \
    const long long steps = std::max(1LL, (nsteps + want - 1) / want);                                      \
    const int runs = (int)((nsteps + steps - 1) / steps);                                                   \
    const long long per = 9LL * S::CO_T * S::CI_T + S::CO_T;                                                \
    if ((long long)tiles * runs * per > kWgradWorkFloats) return hipErrorInvalidValue;                      \
    const size_t lds = conv3x3_wgrad_lds_bytes<CI, CO>(dil);                                                \
    if (lds > 160 * 1024) return hipErrorInvalidValue;                                                      \
    if (lds > 64 * 1024) {                                                                                  \
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&conv3x3_wgrad_kernel<CI, CO>), \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
      if (e != hipSuccess) return e;                                                                        \
    }                                                                                                       \
    conv3x3_wgrad_kernel<CI, CO><<<dim3(runs, tiles), 256, lds, s>>>(x, dy, images, H, W, dil, (int)steps,   \
                                                                      work);                                \
    wgrad_reduce_kernel<<<dim3((unsigned)((per + 31) / 32), tiles), 512, 0, s>>>(work, runs, S::CO_T,        \
                                                                                  S::CI_T, CI, CO, dw, db);   \
    return hipGetLastError();                                                                               \
  }
  SLHJB_FOR_LAYERS(SLHJB_WG)
#undef SLHJB_WG
  return hipErrorInvalidValue;
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
  loss_head_bwd_kernel<32><<<blocks_for(total, 256 * kLossPix), 256, 0, s>>>(delta, uhat, vstar, mask, total, inv_n, h, hw, dh,
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
  const unsigned blocks = std::max(1u, std::min(blocks_for(count, 256 * 16 * 8), 256u));
  count_nonzero_u8_kernel<<<blocks, 256, 0, s>>>(m, count, out);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, long long count, hipStream_t s) {
  zero_f32_kernel<<<blocks_for(count, 256), 256, 0, s>>>(p, count);
  return hipGetLastError();
}

}  // namespace slhjb
