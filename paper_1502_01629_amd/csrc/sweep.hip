// Jacobi sweep kernels of the semi-Lagrangian Markov-chain scheme (Cacace & Falcone,
// Section 3, eqs. SLscheme2 / SLscheme3) for gfx950.
//
// The iterate is w = V* - v (V* = l / lambda), in which the discounted update is
//   SL2:  w_i = beta * max_a (1/K) sum_feet I[w](y)
//   SL3:  w_i = beta * max_a (sum_feet I[w](y) - L0 w_i) / (K - beta L0)
// where L0 is the sum over the feet of node i's own bilinear weight (K Lambda0 of
// eq. SLimplicit). Feet outside the closed box read w_outside and carry no self weight.
//
// Two kernels:
//  * sweep_general: any diffusion, any foot reach up to kMaxHalo-1 cells. The workgroup
//    stages its 64 x 16 node tile plus a halo in LDS and gathers the four cell corners of
//    every foot from there.
//  * sweep_ring1: sigma = 0 with every foot inside the first ring of cells (|h c a| <= dx
//    per axis, the regime the paper prescribes by eq. upper-bound). The interpolant in each
//    of the four cells around a node is a bilinear form A + B s + C t + D s t; with the
//    node's 3x3 neighbourhood in registers and the controls grouped by quadrant, a control
//    costs three FMAs (SL2) instead of a gather.
#include <algorithm>

#include "sweep_device.h"

namespace slhjb {

// Stage the node tile [tx0 - halo, tx0 + kTileW + halo) x [ty0 - halo, ty0 + kTileH + halo)
// in LDS; nodes outside the grid are stored as 0 and never carry weight.
__device__ __forceinline__ void load_tile(float* tile, const float* __restrict__ w_in, const SweepArgs& a, int tx0,
                                          int ty0, int LW, int LH) {
  const int n = a.n;
  const int total = LW * LH;
  for (int t = threadIdx.x; t < total; t += kThreads) {
    const int ly = t / LW;
    const int lx = t - ly * LW;
    const int gx = tx0 - a.halo + lx;
    const int gy = ty0 - a.halo + ly;
    float val = 0.0f;
    if (gx >= 0 && gx < n && gy >= 0 && gy < n) val = w_in[(size_t)gy * n + gx];
    tile[t] = val;
  }
}

// All pointers are separate __restrict__ kernel arguments: the compiler can then prove that the
// control table is never written during the kernel and fetch it with scalar loads.
#define SLHJB_SWEEP_PARAMS                                                                           \
  SweepArgs a, const float* __restrict__ w_in, float* __restrict__ w_out, const float* __restrict__ speed, \
      const uint8_t* __restrict__ cls, const float4* __restrict__ ctrl, unsigned* __restrict__ resid,        \
      unsigned* __restrict__ flags

template <int DIFF, int SCHEME, bool GEN>
__global__ __launch_bounds__(kThreads) void sweep_general(SLHJB_SWEEP_PARAMS) {
  extern __shared__ float tile[];
  const int tx0 = blockIdx.x * kTileW;
  const int ty0 = blockIdx.y * kTileH;
  const int LW = kTileW + 2 * a.halo;
  const int LH = kTileH + 2 * a.halo;
  load_tile(tile, w_in, a, tx0, ty0, LW, LH);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = tx0 + lane;
  const int n = a.n;
  float local = 0.0f;
  bool bad = false;
  for (int row = wave; row < kTileH; row += kThreads / 64) {
    const int j = ty0 + row;
    if (i < n && j < n) {
      const size_t idx = (size_t)j * n + i;
      const int c = cls[idx];
      float wn;
      if (c == kFree) {
        const float k = a.r * (speed ? speed[idx] : a.speed_const);
        const int node_li = (row + a.halo) * LW + lane + a.halo;
        const float wself = tile[node_li];
        if (GEN)
          wn = general_update<DIFF, SCHEME, false, true>(tile, LW, node_li, i, j, k, wself, ctrl, a, nullptr, 0,
                                                         node_cost(a, idx), node_noise(a, idx));
        else
          wn = general_update<DIFF, SCHEME>(tile, LW, node_li, i, j, k, wself, ctrl, a);
        local = fmaxf(local, fabsf(wn - wself));
        bad |= !isfinite(wn);
      } else {
        wn = c == kTarget ? a.w_target : a.w_obstacle;
      }
      w_out[idx] = wn;
    }
  }
  block_reduce_and_publish(local, bad, resid, flags);
}

template <int SCHEME>
__global__ __launch_bounds__(kThreads) void sweep_ring1(SLHJB_SWEEP_PARAMS) {
  extern __shared__ float tile[];
  const int tx0 = blockIdx.x * kTileW;
  const int ty0 = blockIdx.y * kTileH;
  const int LW = kTileW + 2 * a.halo;
  const int LH = kTileH + 2 * a.halo;
  load_tile(tile, w_in, a, tx0, ty0, LW, LH);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = tx0 + lane;
  const int n = a.n;
  const bool cols_interior = tx0 >= 1 && tx0 + kTileW - 1 <= n - 2;
  float local = 0.0f;
  bool bad = false;
  for (int row = wave; row < kTileH; row += kThreads / 64) {
    const int j = ty0 + row;
    if (j >= n) break;
    const bool interior = cols_interior && j >= 1 && j <= n - 2;  // uniform across the wavefront
    if (i < n) {
      const size_t idx = (size_t)j * n + i;
      const int c = cls[idx];
      float wn;
      if (c == kFree) {
        const float k = a.r * (speed ? speed[idx] : a.speed_const);
        const float* T = tile + (row + a.halo) * LW + lane + a.halo;
        if (interior) {
          wn = ring1_update<SCHEME, false>(T, LW, k, ctrl, a, false, false, false, false);
        } else {
          wn = ring1_update<SCHEME, true>(T, LW, k, ctrl, a, i == 0, i == n - 1, j == 0, j == n - 1);
        }
        local = fmaxf(local, fabsf(wn - T[0]));
        bad |= !isfinite(wn);
      } else {
        wn = c == kTarget ? a.w_target : a.w_obstacle;
      }
      w_out[idx] = wn;
    }
  }
  block_reduce_and_publish(local, bad, resid, flags);
}

#define SLHJB_SWEEP_ARGS a, a.w_in, a.w_out, a.speed, a.cls, a.ctrl, a.resid, a.flags

hipError_t launch_sweep(const SweepArgs& a, int diffusion, int scheme, int path, hipStream_t s) {
  dim3 grid((a.n + kTileW - 1) / kTileW, (a.n + kTileH - 1) / kTileH);
  const size_t lds = sizeof(float) * (kTileW + 2 * a.halo) * (kTileH + 2 * a.halo);
  if (path == 1) {
    if (scheme == kSL2) sweep_ring1<kSL2><<<grid, kThreads, lds, s>>>(SLHJB_SWEEP_ARGS);
    else sweep_ring1<kSL3><<<grid, kThreads, lds, s>>>(SLHJB_SWEEP_ARGS);
    return hipGetLastError();
  }
#define SLHJB_LAUNCH(D, S)                                                               \
  do {                                                                                   \
    if (path == 2) sweep_general<D, S, true><<<grid, kThreads, lds, s>>>(SLHJB_SWEEP_ARGS); \
    else sweep_general<D, S, false><<<grid, kThreads, lds, s>>>(SLHJB_SWEEP_ARGS);         \
  } while (0)
  switch (diffusion * 2 + scheme) {
  case kDiffNone * 2 + kSL2: SLHJB_LAUNCH(kDiffNone, kSL2); break;
  case kDiffNone * 2 + kSL3: SLHJB_LAUNCH(kDiffNone, kSL3); break;
  case kDiffIso * 2 + kSL2: SLHJB_LAUNCH(kDiffIso, kSL2); break;
  case kDiffIso * 2 + kSL3: SLHJB_LAUNCH(kDiffIso, kSL3); break;
  case kDiffRank1 * 2 + kSL2: SLHJB_LAUNCH(kDiffRank1, kSL2); break;
  default: SLHJB_LAUNCH(kDiffRank1, kSL3); break;
  }
#undef SLHJB_LAUNCH
  return hipGetLastError();
}

// ---- small helper kernels -------------------------------------------------------------

__global__ void v_to_w_kernel(const float* __restrict__ v, float* __restrict__ w, const uint8_t* __restrict__ cls,
                              int64_t count, float vstar, float w_target, float w_obstacle) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[t];
    w[t] = c == kFree ? vstar - v[t] : (c == kTarget ? w_target : w_obstacle);
  }
}

__global__ void w_to_v_kernel(const float* __restrict__ w, float* __restrict__ v, int64_t count, float vstar) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x)
    v[t] = vstar - w[t];
}

// Problem statistics in one pass: out[0] = bits of the minimum speed, out[1] = bits of the
// maximum speed (positive floats order like their bits), out[2] |= 1 if a speed is not finite
// or not > 0, out[3] += number of FREE nodes, out[4] |= 1 if a class value is not 0, 1 or 2.
// The caller initialises out to (0x7f7fffff, 0, 0, 0, 0). speed may be NULL.
__global__ void problem_stats_kernel(const float* __restrict__ speed, const uint8_t* __restrict__ cls,
                                     const float2* __restrict__ drift, float speed_const, int64_t count,
                                     unsigned* out) {
  float lo = INFINITY, hi = 0.0f, dmax = 0.0f;
  bool bad_speed = false, bad_cls = false, bad_drift = false;
  unsigned nfree = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls[t];
    nfree += c == kFree ? 1u : 0u;
    bad_cls |= c > kObstacle;
    float v = speed_const;
    if (speed) {
      v = speed[t];
      if (!(v > 0.0f) || !isfinite(v)) bad_speed = true;
      else {
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
      }
    }
    if (drift) {
      const float2 d = drift[t];
      if (!isfinite(d.x) || !isfinite(d.y)) bad_drift = true;
      else if (isfinite(v)) dmax = fmaxf(dmax, v * fmaxf(fabsf(d.x), fabsf(d.y)));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, 64));
    hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    dmax = fmaxf(dmax, __shfl_xor(dmax, off, 64));
    nfree += __shfl_xor(nfree, off, 64);
  }
  // one set of atomics per workgroup: same-address atomics from every wavefront serialise in L2
  __shared__ float slo[kThreads / 64], shi[kThreads / 64], sdm[kThreads / 64];
  __shared__ unsigned sfree[kThreads / 64];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    slo[threadIdx.x >> 6] = lo;
    shi[threadIdx.x >> 6] = hi;
    sdm[threadIdx.x >> 6] = dmax;
    sfree[threadIdx.x >> 6] = nfree;
  }
  if (bad_speed) atomicOr(&sbad, 1);
  if (bad_cls) atomicOr(&sbad, 2);
  if (bad_drift) atomicOr(&sbad, 4);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / 64; ++k) {
      lo = fminf(lo, slo[k]);
      hi = fmaxf(hi, shi[k]);
      dmax = fmaxf(dmax, sdm[k]);
      nfree += sfree[k];
    }
    if (speed) {
      if (lo < INFINITY) atomicMin(&out[0], __float_as_uint(lo));
      atomicMax(&out[1], __float_as_uint(hi));
    }
    atomicAdd(&out[3], nfree);
    if (sbad & 1) atomicOr(&out[2], 1u);
    if (sbad & 2) atomicOr(&out[4], 1u);
    if (drift) atomicMax(&out[5], __float_as_uint(dmax));  // non-negative: the bits order as the values
    if (sbad & 4) atomicOr(&out[6], 1u);
  }
}

// Largest value of a per-node field and whether any value is non-finite, negative or (positive)
// zero: one pass, one set of atomics per workgroup.
__global__ __launch_bounds__(kThreads) void field_stats_kernel(const float* __restrict__ f, int64_t count,
                                                               int positive, unsigned* __restrict__ out) {
  float hi = 0.0f;
  bool bad = false;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count; t += (int64_t)gridDim.x * kThreads) {
    const float v = f[t];
    if (!isfinite(v) || v < 0.0f || (positive && !(v > 0.0f))) bad = true;
    else hi = fmaxf(hi, v);
  }
  hi = wave_max(hi);
  __shared__ float shi[kThreads / 64];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) shi[threadIdx.x >> 6] = hi;
  if (bad) atomicOr(&sbad, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / 64; ++k) hi = fmaxf(hi, shi[k]);
    atomicMax(&out[0], __float_as_uint(hi));  // non-negative: the bits order as the values
    if (sbad) atomicOr(&out[1], 1u);
  }
}

__global__ void fill_u32_kernel(unsigned* p, unsigned value, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = value;
}

static int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_v_to_w(const float* v, float* w, const uint8_t* cls, int64_t count, float vstar, float w_target,
                         float w_obstacle, hipStream_t s) {
  v_to_w_kernel<<<grid_for(count), 256, 0, s>>>(v, w, cls, count, vstar, w_target, w_obstacle);
  return hipGetLastError();
}

hipError_t launch_w_to_v(const float* w, float* v, int64_t count, float vstar, hipStream_t s) {
  w_to_v_kernel<<<grid_for(count), 256, 0, s>>>(w, v, count, vstar);
  return hipGetLastError();
}

hipError_t launch_problem_stats(const float* speed, const uint8_t* cls, const float2* drift, float speed_const,
                                int64_t count, unsigned* out, hipStream_t s) {
  problem_stats_kernel<<<std::min(grid_for(count), 512), kThreads, 0, s>>>(speed, cls, drift, speed_const, count,
                                                                             out);
  return hipGetLastError();
}

hipError_t launch_field_stats(const float* f, int64_t count, int positive, unsigned* out, hipStream_t s) {
  field_stats_kernel<<<std::min(grid_for(count), 512), kThreads, 0, s>>>(f, count, positive, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, unsigned value, int count, hipStream_t s) {
  fill_u32_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, value, count);
  return hipGetLastError();
}

}  // namespace slhjb
