// Active-tile solver: the GPU form of the paper's per-patch computation with a fast-marching-like
// order (Section 4.2 "The role of causality", Section 4.3 computation step).
//
// The grid is cut into 32 x 16 node tiles. A pass takes a list of tiles; each workgroup stages
// its tile and an interpolation halo in LDS and runs Jacobi iterations of the scheme on the
// tile's FREE nodes, with the halo frozen, until no node moves by more than tol_inner (or
// max_inner iterations). Results go to a staging buffer, so every tile of a pass reads the
// iterate of the previous pass and the outcome does not depend on scheduling. A commit kernel
// writes the staged tiles back and flags a tile and its 8 neighbours for the next pass when it
// moved by more than the activation threshold. The next pass takes the flagged tiles; with keys
// (the arrival time of u_hat, min over the tile) only the frontier: flagged tiles with no flagged
// neighbour whose key is smaller by more than a slack. That is the order "by increasing u_hat"
// of the paper at tile granularity, and it keeps tiles whose upwind values are still moving from
// being iterated to convergence against stale halos.
#include "sweep_device.h"

namespace slhjb {

constexpr int kTW = 32, kTH = 16, kTN = kTW * kTH;  // nodes per tile; 2 per thread

template <int DIFF, int SCHEME, int PATH, bool INDEP>
__global__ __launch_bounds__(kThreads) void tile_pass_kernel(
    SweepArgs a, const float* __restrict__ w, const float* __restrict__ speed, const uint8_t* __restrict__ cls,
    const float4* __restrict__ ctrl, const int16_t* __restrict__ label, const int* __restrict__ list,
    const int* __restrict__ count, int tiles_x, float* __restrict__ outbuf, float* __restrict__ tchange,
    uint8_t* __restrict__ flag, int max_inner, float tol_inner, unsigned long long* __restrict__ updates) {
  extern __shared__ float lds[];
  const int R = a.halo;
  const int LW = kTW + 2 * R, LH = kTH + 2 * R, span = LW * LH;
  float* bufA = lds;
  float* bufB = lds + span;
  int16_t* labs = (int16_t*)(lds + 2 * span);
  __shared__ float red[kThreads / 64];
  const int n = a.n;
  const int total = *count;
  const int wave = threadIdx.x >> 6;
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int tid = list[slot];
    const int tx = tid % tiles_x, ty = tid / tiles_x;
    const int x0 = tx * kTW, y0 = ty * kTH;
    if (threadIdx.x == 0) flag[tid] = 0;
    for (int e = threadIdx.x; e < span; e += kThreads) {
      const int ly = e / LW, lx = e - ly * LW;
      const int gx = x0 - R + lx, gy = y0 - R + ly;
      const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n;
      const float val = in ? w[(size_t)gy * n + gx] : 0.0f;
      bufA[e] = val;
      bufB[e] = val;
      if (INDEP) labs[e] = in ? label[(size_t)gy * n + gx] : (int16_t)-32768;
    }
    // the two nodes of this thread
    int li[2], gi[2], gj[2];
    bool fr[2];
    float kk[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const int lx = q & (kTW - 1), ly = q / kTW;
      gi[r] = x0 + lx;
      gj[r] = y0 + ly;
      li[r] = (ly + R) * LW + lx + R;
      fr[r] = false;
      kk[r] = 0.0f;
      if (gi[r] < n && gj[r] < n) {
        const size_t idx = (size_t)gj[r] * n + gi[r];
        fr[r] = cls[idx] == kFree;
        if (fr[r]) kk[r] = a.r * (speed ? speed[idx] : a.speed_const);
      }
    }
    __syncthreads();  // tile staged
    float* cur = bufA;
    float* nxt = bufB;
    int it = 0;
    for (;;) {
      float lmax = 0.0f;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        // rows handled by this wavefront in this half: 2*wave + {0,1} + 8 r
        const int row0 = y0 + 2 * wave + 8 * r;
        if (fr[r]) {
          float v;
          if (PATH == 1) {
            const bool interior = x0 >= 1 && x0 + kTW - 1 <= n - 2 && row0 >= 1 && row0 + 1 <= n - 2;
            const float* T = cur + li[r];
            const int16_t* L = INDEP ? labs + li[r] : nullptr;
            if (interior) {
              v = ring1_update<SCHEME, false, INDEP>(T, LW, kk[r], ctrl, a, false, false, false, false, L);
            } else {
              v = ring1_update<SCHEME, true, INDEP>(T, LW, kk[r], ctrl, a, gi[r] == 0, gi[r] == n - 1, gj[r] == 0,
                                                    gj[r] == n - 1, L);
            }
          } else {
            v = general_update<DIFF, SCHEME, INDEP>(cur, LW, li[r], gi[r], gj[r], kk[r], cur[li[r]], ctrl, a,
                                                    INDEP ? labs : nullptr, INDEP ? labs[li[r]] : 0);
          }
          nxt[li[r]] = v;
          lmax = fmaxf(lmax, fabsf(v - cur[li[r]]));
        }
      }
      const int moving = __syncthreads_or(lmax > tol_inner);
      float* tmp = cur;
      cur = nxt;
      nxt = tmp;
      ++it;
      if (!moving || it >= max_inner) break;
    }
    // stage the tile and measure how far it moved during this visit
    float moved = 0.0f;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const float v = cur[li[r]];
      outbuf[(size_t)slot * kTN + q] = v;
      if (fr[r]) moved = fmaxf(moved, fabsf(v - w[(size_t)gj[r] * n + gi[r]]));
    }
    moved = wave_max(moved);
    if ((threadIdx.x & 63) == 0) red[wave] = moved;
    const int free_total = __syncthreads_count(fr[0]) + __syncthreads_count(fr[1]);
    if (threadIdx.x == 0) {
      float m = red[0];
#pragma unroll
      for (int k = 1; k < kThreads / 64; ++k) m = fmaxf(m, red[k]);
      tchange[slot] = m;
      atomicAdd(updates, (unsigned long long)it * (unsigned long long)free_total);
    }
    __syncthreads();
  }
}

// Write the staged tiles back and flag the neighbourhood of every tile that moved by more
// than `act`.
__global__ __launch_bounds__(kThreads) void tile_commit_kernel(const int* __restrict__ list, const int* __restrict__ count,
                                                               int tiles_x, int tiles_y, int n,
                                                               const float* __restrict__ outbuf,
                                                               const float* __restrict__ tchange, float act,
                                                               const uint8_t* __restrict__ cls, float* __restrict__ w,
                                                               uint8_t* __restrict__ flag, unsigned* __restrict__ resid) {
  const int total = *count;
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int tid = list[slot];
    const int tx = tid % tiles_x, ty = tid / tiles_x;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const int gx = tx * kTW + (q & (kTW - 1)), gy = ty * kTH + q / kTW;
      if (gx < n && gy < n) {
        const size_t idx = (size_t)gy * n + gx;
        if (cls[idx] == kFree) w[idx] = outbuf[(size_t)slot * kTN + q];
      }
    }
    if (threadIdx.x == 0) {
      const float m = tchange[slot];
      if (resid) atomicMax(resid, __float_as_uint(m));
      if (m > act) {
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int nx = tx + dx, ny = ty + dy;
            if (nx >= 0 && ny >= 0 && nx < tiles_x && ny < tiles_y) flag[ny * tiles_x + nx] = 1;
          }
      }
    }
  }
}

// The next pass: flagged tiles, restricted with keys to those with no flagged neighbour whose
// key is smaller by more than `slack`. The flagged tile of smallest key is always selected, so
// every pass makes progress.
__global__ void tile_select_kernel(const uint8_t* __restrict__ flag, const float* __restrict__ key, int tiles_x,
                                   int tiles_y, float slack, int* __restrict__ list, int* __restrict__ count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int tiles = tiles_x * tiles_y;
  bool on = false;
  if (t < tiles && flag[t]) {
    on = true;
    if (key) {
      const int tx = t % tiles_x, ty = t / tiles_x;
      const float kt = key[t];
      for (int dy = -1; dy <= 1 && on; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int nx = tx + dx, ny = ty + dy;
          if ((dx | dy) == 0 || nx < 0 || ny < 0 || nx >= tiles_x || ny >= tiles_y) continue;
          const int u = ny * tiles_x + nx;
          if (flag[u] && key[u] < kt - slack) {
            on = false;
            break;
          }
        }
    }
  }
  const unsigned long long mask = __ballot(on);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0 && mask) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, 0, 64);
  if (on) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = t;
}

// Key of a tile: the smallest arrival time T = -ln(w / V*) / lambda over its FREE nodes
// (+inf where w <= 0, i.e. not reached).
__global__ __launch_bounds__(kThreads) void tile_keys_kernel(const float* __restrict__ w, const uint8_t* __restrict__ cls,
                                                             int n, int tiles_x, float vstar, float lambda,
                                                             float* __restrict__ key) {
  __shared__ float red[kThreads / 64];
  const int tid = blockIdx.x;
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  float best = INFINITY;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int q = threadIdx.x + r * kThreads;
    const int gx = tx * kTW + (q & (kTW - 1)), gy = ty * kTH + q / kTW;
    if (gx < n && gy < n) {
      const size_t idx = (size_t)gy * n + gx;
      const float ww = w[idx];
      if (cls[idx] == kFree && ww > 0.0f) best = fminf(best, -logf(ww / vstar) / lambda);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = fminf(best, __shfl_xor(best, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
    for (int k = 1; k < kThreads / 64; ++k) m = fminf(m, red[k]);
    key[tid] = m;
  }
}

size_t tile_pass_lds_bytes(int halo, bool indep) {
  const size_t span = (size_t)(kTW + 2 * halo) * (kTH + 2 * halo);
  return 2 * span * sizeof(float) + (indep ? span * sizeof(int16_t) : 0);
}

hipError_t launch_tile_pass(const SweepArgs& a, int diffusion, int scheme, int path, bool indep, const int16_t* label,
                            const int* list, const int* count, int tiles_x, float* outbuf, float* tchange,
                            uint8_t* flag, int max_inner, float tol_inner, unsigned long long* updates, int grid,
                            hipStream_t s) {
  const size_t lds = tile_pass_lds_bytes(a.halo, indep);
#define SLHJB_TP(D, S, PA, IN)                                                                                  \
  tile_pass_kernel<D, S, PA, IN><<<grid, kThreads, lds, s>>>(a, a.w_in, a.speed, a.cls, a.ctrl, label, list, count, \
                                                             tiles_x, outbuf, tchange, flag, max_inner, tol_inner,  \
                                                             updates)
#define SLHJB_TP_S(D, PA, IN)          \
  do {                                 \
    if (scheme == kSL2) SLHJB_TP(D, kSL2, PA, IN); \
    else SLHJB_TP(D, kSL3, PA, IN);    \
  } while (0)
#define SLHJB_TP_I(D, PA)                \
  do {                                   \
    if (indep) SLHJB_TP_S(D, PA, true);  \
    else SLHJB_TP_S(D, PA, false);       \
  } while (0)
  if (path == 1) {
    SLHJB_TP_I(kDiffNone, 1);
  } else if (diffusion == kDiffNone) {
    SLHJB_TP_I(kDiffNone, 0);
  } else if (diffusion == kDiffIso) {
    SLHJB_TP_I(kDiffIso, 0);
  } else {
    SLHJB_TP_I(kDiffRank1, 0);
  }
#undef SLHJB_TP_I
#undef SLHJB_TP_S
#undef SLHJB_TP
  return hipGetLastError();
}

hipError_t launch_tile_commit(const int* list, const int* count, int tiles_x, int tiles_y, int n, const float* outbuf,
                              const float* tchange, float act, const uint8_t* cls, float* w, uint8_t* flag,
                              unsigned* resid, int grid, hipStream_t s) {
  tile_commit_kernel<<<grid, kThreads, 0, s>>>(list, count, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag,
                                               resid);
  return hipGetLastError();
}

hipError_t launch_tile_select(const uint8_t* flag, const float* key, int tiles_x, int tiles_y, float slack, int* list,
                              int* count, hipStream_t s) {
  const int tiles = tiles_x * tiles_y;
  tile_select_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(flag, key, tiles_x, tiles_y, slack, list, count);
  return hipGetLastError();
}

__global__ void iota_kernel(int* p, int count, int* count_out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = t;
  if (t == 0) *count_out = count;
}

hipError_t launch_iota(int* p, int count, int* count_out, hipStream_t s) {
  iota_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, count, count_out);
  return hipGetLastError();
}

hipError_t launch_tile_keys(const float* w, const uint8_t* cls, int n, int tiles_x, int tiles_y, float vstar,
                            float lambda, float* key, hipStream_t s) {
  tile_keys_kernel<<<tiles_x * tiles_y, kThreads, 0, s>>>(w, cls, n, tiles_x, vstar, lambda, key);
  return hipGetLastError();
}

}  // namespace slhjb
