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
// (the arrival time of u_hat, min over the tile) only a band of them: those whose key is within
// a window of the smallest flagged key. That is the order "by increasing u_hat" of the paper at
// tile granularity, bucketed so that a whole ring of tiles runs at once, and it keeps tiles
// whose upwind values are still moving from being iterated to convergence against stale halos.
#include <hip/hip_cooperative_groups.h>

#include "sweep_device.h"

namespace slhjb {

// Visit of an 8x8 tile by a 256-thread workgroup: lane = node, wavefront = a quarter of the
// controls (a quadrant on the first-ring path, a quarter of the list otherwise). Per inner
// iteration the four partial maxima go through LDS and wavefront 0 combines them in a fixed
// order, so the result does not depend on timing.
template <int DIFF, int SCHEME, int PATH, bool INDEP>
__device__ __forceinline__ void visit_tile_split(const SweepArgs& a, const float* __restrict__ w,
                                                 const float* __restrict__ speed, const uint8_t* __restrict__ cls,
                                                 const float4* __restrict__ ctrl, const int16_t* __restrict__ label,
                                                 int slot, int tid, int tiles_x, float* __restrict__ outbuf,
                                                 float* __restrict__ tchange, uint8_t* __restrict__ flag, int max_inner,
                                                 float tol_inner, unsigned long long* __restrict__ updates, float* lds,
                                                 float* red) {
  constexpr int kT = 8;
  const int R = a.halo;
  const int LW = kT + 2 * R, span = LW * LW;
  float* bufA = lds;
  float* bufB = lds + span;
  float* pn = lds + 2 * span;
  float* pd = pn + 256;
  int16_t* labs = (int16_t*)(pd + 256);
  const int n = a.n;
  const int node = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  const int x0 = tx * kT, y0 = ty * kT;
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
  const int lx = node & (kT - 1), ly = node / kT;
  const int gi = x0 + lx, gj = y0 + ly;
  const int li = (ly + R) * LW + lx + R;
  bool fr = false;
  float kk = 0.0f;
  if (gi < n && gj < n) {
    const size_t idx = (size_t)gj * n + gi;
    fr = cls[idx] == kFree;
    if (fr) kk = a.r * (speed ? speed[idx] : a.speed_const);
  }
  const bool interior = x0 >= 1 && x0 + kT - 1 <= n - 2 && y0 >= 1 && y0 + kT - 1 <= n - 2;
  const int quarter = a.n_controls / 4;  // the padded list length is a multiple of 4
  __syncthreads();
  float* cur = bufA;
  float* nxt = bufB;
  int it = 0;
  for (;;) {
    if (fr) {
      float num, den;
      if (PATH == 1) {
        const float* T = cur + li;
        const int16_t* L = INDEP ? labs + li : nullptr;
        if (interior)
          ring1_partial<SCHEME, false, INDEP>(T, LW, kk, ctrl, a, false, false, false, false, L, part, num, den);
        else
          ring1_partial<SCHEME, true, INDEP>(T, LW, kk, ctrl, a, gi == 0, gi == n - 1, gj == 0, gj == n - 1, L, part,
                                             num, den);
      } else {
        general_partial<DIFF, SCHEME, INDEP>(cur, LW, li, gi, gj, kk, cur[li], ctrl, a, INDEP ? labs : nullptr,
                                             INDEP ? labs[li] : 0, part * quarter, (part + 1) * quarter, num, den);
      }
      pn[part * 64 + node] = num;
      pd[part * 64 + node] = den;
    }
    __syncthreads();
    float lmax = 0.0f;
    if (part == 0 && fr) {
      float v;
      if (SCHEME == kSL2) {
        const float m = fmaxf(fmaxf(pn[node], pn[64 + node]), fmaxf(pn[128 + node], pn[192 + node]));
        constexpr int K = Feet<DIFF>::K;
        v = PATH == 1 ? a.beta * (cur[li] + m) : a.beta * m * (1.0f / (float)K);
      } else {
        float bn = pn[node], bd = pd[node];
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          const float qn = pn[q * 64 + node], qd = pd[q * 64 + node];
          if (qn * bd > bn * qd) {
            bn = qn;
            bd = qd;
          }
        }
        v = a.beta * bn / bd;
      }
      nxt[li] = v;
      lmax = fabsf(v - cur[li]);
    }
    const int moving = __syncthreads_or(lmax > tol_inner);
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
    ++it;
    if (!moving || it >= max_inner) break;
  }
  float moved = 0.0f;
  if (part == 0) {
    outbuf[(size_t)slot * 64 + node] = cur[li];
    if (fr) moved = fabsf(cur[li] - w[(size_t)gj * n + gi]);
  }
  moved = wave_max(moved);
  if ((threadIdx.x & 63) == 0) red[part] = moved;
  const int free_total = __syncthreads_count(part == 0 && fr);
  if (threadIdx.x == 0) {
    const float m = red[0];
    const bool unsettled = it >= max_inner && max_inner > 1;
    tchange[slot] = unsettled ? -fmaxf(m, 1e-30f) : m;
    atomicAdd(updates, (unsigned long long)it * (unsigned long long)free_total);
  }
  __syncthreads();
}

// One visit of tile `tid`, staged into slot `slot` of outbuf/tchange: Jacobi iterations in LDS
// against the frozen halo until no node moves by more than tol_inner (or max_inner).
template <int TW, int TH, int DIFF, int SCHEME, int PATH, bool INDEP>
__device__ __forceinline__ void visit_tile(const SweepArgs& a, const float* __restrict__ w,
                                           const float* __restrict__ speed, const uint8_t* __restrict__ cls,
                                           const float4* __restrict__ ctrl, const int16_t* __restrict__ label,
                                           int slot, int tid, int tiles_x, float* __restrict__ outbuf,
                                           float* __restrict__ tchange, uint8_t* __restrict__ flag, int max_inner,
                                           float tol_inner, unsigned long long* __restrict__ updates, float* lds,
                                           float* red) {
  if constexpr (TW * TH == 64) {
    visit_tile_split<DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, slot, tid, tiles_x, outbuf, tchange,
                                                flag, max_inner, tol_inner, updates, lds, red);
    return;
  } else {
  constexpr int kTW = TW, kTH = TH, kTN = TW * TH, NPT = kTN / kThreads;  // NPT nodes per thread
  static_assert(kTN % kThreads == 0 && 64 % TW == 0, "tile shape");
  const int R = a.halo;
  const int LW = kTW + 2 * R, LH = kTH + 2 * R, span = LW * LH;
  float* bufA = lds;
  float* bufB = lds + span;
  int16_t* labs = (int16_t*)(lds + 2 * span);
  const int n = a.n;
  const int wave = threadIdx.x >> 6;
  {
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
    // the NPT nodes of this thread
    int li[NPT], gi[NPT], gj[NPT];
    bool fr[NPT];
    float kk[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
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
      for (int r = 0; r < NPT; ++r) {
        // rows handled by this wavefront for its r-th node: 64/TW consecutive rows
        const int row0 = y0 + (64 * wave + kThreads * r) / kTW;
        if (fr[r]) {
          float v;
          if (PATH == 1) {
            const bool interior = x0 >= 1 && x0 + kTW - 1 <= n - 2 && row0 >= 1 && row0 + 64 / kTW - 1 <= n - 2;
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
    for (int r = 0; r < NPT; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const float v = cur[li[r]];
      outbuf[(size_t)slot * kTN + q] = v;
      if (fr[r]) moved = fmaxf(moved, fabsf(v - w[(size_t)gj[r] * n + gi[r]]));
    }
    moved = wave_max(moved);
    if ((threadIdx.x & 63) == 0) red[wave] = moved;
    int nf = 0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) nf += fr[r] ? 1 : 0;
    const int free_total = __syncthreads_count(nf >= 1) + (NPT > 1 ? __syncthreads_count(nf >= 2) : 0);
    if (threadIdx.x == 0) {
      float m = red[0];
#pragma unroll
      for (int k = 1; k < kThreads / 64; ++k) m = fmaxf(m, red[k]);
      // a visit that stopped at max_inner while still moving is marked by a negative sign
      const bool unsettled = it >= max_inner && max_inner > 1;
      tchange[slot] = unsettled ? -fmaxf(m, 1e-30f) : m;
      atomicAdd(updates, (unsigned long long)it * (unsigned long long)free_total);
    }
    __syncthreads();
  }
  }
}

template <int TW, int TH, int DIFF, int SCHEME, int PATH, bool INDEP>
__global__ __launch_bounds__(kThreads) void tile_pass_kernel(
    SweepArgs a, const float* __restrict__ w, const float* __restrict__ speed, const uint8_t* __restrict__ cls,
    const float4* __restrict__ ctrl, const int16_t* __restrict__ label, const int* __restrict__ list,
    const int* __restrict__ count, int tiles_x, float* __restrict__ outbuf, float* __restrict__ tchange,
    uint8_t* __restrict__ flag, int max_inner, float tol_inner, unsigned long long* __restrict__ updates) {
  extern __shared__ float lds[];
  __shared__ float red[kThreads / 64];
  const int total = *count;
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x)
    visit_tile<TW, TH, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, slot, list[slot], tiles_x, outbuf,
                                                  tchange, flag, max_inner, tol_inner, updates, lds, red);
}

// Write staged tile `tid` (slot `slot`) back and flag the neighbourhood of a tile that moved by
// more than `act`; the tile itself is flagged again only if its visit stopped before settling.
__device__ __forceinline__ void commit_tile(int slot, int tid, int tw, int th, int tiles_x, int tiles_y, int n,
                                            const float* __restrict__ outbuf, const float* __restrict__ tchange,
                                            float act, const uint8_t* __restrict__ cls, float* __restrict__ w,
                                            uint8_t* __restrict__ flag, unsigned* __restrict__ resid) {
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  const int tn = tw * th;
  for (int q = threadIdx.x; q < tn; q += kThreads) {
    const int gx = tx * tw + q % tw, gy = ty * th + q / tw;
    if (gx < n && gy < n) {
      const size_t idx = (size_t)gy * n + gx;
      if (cls[idx] == kFree) w[idx] = outbuf[(size_t)slot * tn + q];
    }
  }
  if (threadIdx.x == 0) {
    const float tc = tchange[slot];
    const float m = fabsf(tc);
    if (resid) atomicMax(resid, __float_as_uint(m));
    if (m > act) {
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int nx = tx + dx, ny = ty + dy;
          if ((dx | dy) == 0 && !(tc < 0.0f)) continue;
          if (nx >= 0 && ny >= 0 && nx < tiles_x && ny < tiles_y) flag[ny * tiles_x + nx] = 1;
        }
    }
  }
}

__global__ __launch_bounds__(kThreads) void tile_commit_kernel(const int* __restrict__ list, const int* __restrict__ count,
                                                               int tw, int th, int tiles_x, int tiles_y, int n,
                                                               const float* __restrict__ outbuf,
                                                               const float* __restrict__ tchange, float act,
                                                               const uint8_t* __restrict__ cls, float* __restrict__ w,
                                                               uint8_t* __restrict__ flag, unsigned* __restrict__ resid,
                                                               unsigned* __restrict__ pass_counter) {
  const int total = *count;
  if (pass_counter && blockIdx.x == 0 && threadIdx.x == 0 && total > 0) atomicAdd(pass_counter, 1u);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x)
    commit_tile(slot, list[slot], tw, th, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag, resid);
}

// Smallest key among the flagged tiles (keys are >= 0 or +inf, so their bits order like the
// values). `kmin` must hold +inf bits before the launch.
__global__ void tile_kmin_kernel(const uint8_t* __restrict__ flag, const float* __restrict__ key, int tiles,
                                 unsigned* __restrict__ kmin) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  float k = INFINITY;
  if (t < tiles && flag[t]) k = key[t];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) k = fminf(k, __shfl_xor(k, off, 64));
  if ((threadIdx.x & 63) == 0 && k < INFINITY) atomicMin(kmin, __float_as_uint(k));
}

// The next pass: the flagged tiles; with keys only those whose key is at most the band bound B
// (buckets of arrival times processed in increasing order: the paper's order by u_hat). B only
// grows: when no flagged tile is left at or below it, it jumps to the smallest flagged key plus
// `window`. Tiles re-flagged below B (their halo moved) rejoin at once. The flagged tile of
// smallest key is always selected, so every pass makes progress. `bound` holds B (float bits,
// -inf before the first pass); every thread derives the same new bound, block 0 stores it.
__global__ void tile_select_kernel(const uint8_t* __restrict__ flag, const float* __restrict__ key, int tiles,
                                   const unsigned* __restrict__ kmin, unsigned* __restrict__ bound, float window,
                                   int* __restrict__ list, int* __restrict__ count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  bool on = false;
  float B = INFINITY;
  if (key) {
    const float lo = __uint_as_float(*kmin);
    B = __uint_as_float(*bound);
    if (lo > B) B = lo + window;
    if (lo == INFINITY) B = INFINITY;  // only tiles without a finite key remain
  }
  if (t < tiles && flag[t]) on = !key || key[t] <= B;
  const unsigned long long mask = __ballot(on);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0 && mask) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, 0, 64);
  if (on) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = t;
  if (key && t == 0 && B < INFINITY) *bound = __float_as_uint(B);
}

// Key of a tile: the smallest arrival time T = -ln(w / V*) / lambda over its FREE nodes
// (+inf where w <= 0, i.e. not reached).
__global__ __launch_bounds__(kThreads) void tile_keys_kernel(const float* __restrict__ w, const uint8_t* __restrict__ cls,
                                                             int tw, int th, int n, int tiles_x, float vstar,
                                                             float lambda, float* __restrict__ key) {
  __shared__ float red[kThreads / 64];
  const int tid = blockIdx.x;
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  float best = INFINITY;
  for (int q = threadIdx.x; q < tw * th; q += kThreads) {
    const int gx = tx * tw + q % tw, gy = ty * th + q / tw;
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

size_t tile_pass_lds_bytes(int tw, int th, int halo, bool indep) {
  const size_t span = (size_t)(tw + 2 * halo) * (th + 2 * halo);
  const size_t partials = tw * th == 64 ? 2 * 256 * sizeof(float) : 0;
  return 2 * span * sizeof(float) + partials + (indep ? span * sizeof(int16_t) : 0);
}

template <int TW, int TH>
static void launch_tile_pass_shape(const SweepArgs& a, int diffusion, int scheme, int path, bool indep,
                                   const int16_t* label, const int* list, const int* count, int tiles_x, float* outbuf,
                                   float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                   unsigned long long* updates, int grid, hipStream_t s) {
  const size_t lds = tile_pass_lds_bytes(TW, TH, a.halo, indep);
#define SLHJB_TP(D, S, PA, IN)                                                                                      \
  tile_pass_kernel<TW, TH, D, S, PA, IN><<<grid, kThreads, lds, s>>>(a, a.w_in, a.speed, a.cls, a.ctrl, label, list, \
                                                                     count, tiles_x, outbuf, tchange, flag, max_inner, \
                                                                     tol_inner, updates)
#define SLHJB_TP_S(D, PA, IN)                      \
  do {                                             \
    if (scheme == kSL2) SLHJB_TP(D, kSL2, PA, IN); \
    else SLHJB_TP(D, kSL3, PA, IN);                \
  } while (0)
#define SLHJB_TP_I(D, PA)               \
  do {                                  \
    if (indep) SLHJB_TP_S(D, PA, true); \
    else SLHJB_TP_S(D, PA, false);      \
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
}

hipError_t launch_tile_pass(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                            const int16_t* label, const int* list, const int* count, int tiles_x, float* outbuf,
                            float* tchange, uint8_t* flag, int max_inner, float tol_inner, unsigned long long* updates,
                            int grid, hipStream_t s) {
  if (shape == 2)
    launch_tile_pass_shape<8, 8>(a, diffusion, scheme, path, indep, label, list, count, tiles_x, outbuf, tchange,
                                 flag, max_inner, tol_inner, updates, grid, s);
  else if (shape == 1)
    launch_tile_pass_shape<16, 16>(a, diffusion, scheme, path, indep, label, list, count, tiles_x, outbuf, tchange,
                                   flag, max_inner, tol_inner, updates, grid, s);
  else
    launch_tile_pass_shape<32, 16>(a, diffusion, scheme, path, indep, label, list, count, tiles_x, outbuf, tchange,
                                   flag, max_inner, tol_inner, updates, grid, s);
  return hipGetLastError();
}

hipError_t launch_tile_commit(const int* list, const int* count, int tw, int th, int tiles_x, int tiles_y, int n,
                              const float* outbuf, const float* tchange, float act, const uint8_t* cls, float* w,
                              uint8_t* flag, unsigned* resid, unsigned* pass_counter, int grid, hipStream_t s) {
  tile_commit_kernel<<<grid, kThreads, 0, s>>>(list, count, tw, th, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w,
                                               flag, resid, pass_counter);
  return hipGetLastError();
}

hipError_t launch_tile_select(const uint8_t* flag, const float* key, int tiles, unsigned* kmin, unsigned* bound,
                              float window, int* list, int* count, hipStream_t s) {
  if (key) {
    tile_kmin_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(flag, key, tiles, kmin);
  }
  tile_select_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(flag, key, tiles, kmin, bound, window, list, count);
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

hipError_t launch_tile_keys(const float* w, const uint8_t* cls, int tw, int th, int n, int tiles_x, int tiles_y,
                            float vstar, float lambda, float* key, hipStream_t s) {
  tile_keys_kernel<<<tiles_x * tiles_y, kThreads, 0, s>>>(w, cls, tw, th, n, tiles_x, vstar, lambda, key);
  return hipGetLastError();
}

// ---- the whole active-tile iteration in one cooperative launch -------------------------------
// Every workgroup runs the same loop of phases separated by grid barriers: (1) smallest flagged
// key, (2) selection of the band, (3) visits, (4) commits; when no tile is flagged, a check
// sweep of every tile (one Jacobi iteration each) measures the residual. All control decisions
// are taken from values read with device-scope atomics after a barrier and not written again
// before the next barrier, so every workgroup takes the same branch, and the loop is bounded by
// max_passes, so every workgroup reaches the end.
struct CoopState {
  unsigned count;     // length of the selected list
  unsigned kmin;      // bits of the smallest flagged key
  unsigned bound;     // bits of the band bound B
  unsigned resid;     // bits of the residual of the last check sweep
  unsigned passes;    // passes done (written by workgroup 0 at the end)
  unsigned status;    // 1 converged, 2 pass budget exhausted
  unsigned long long updates;
};

__device__ __forceinline__ unsigned ld_agent(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_barrier(cooperative_groups::grid_group& g) {
  __threadfence();
  g.sync();
  __threadfence();
}

template <int TW, int TH, int DIFF, int SCHEME, int PATH, bool INDEP>
__global__ __launch_bounds__(kThreads) void tile_solve_coop_kernel(
    SweepArgs a, float* __restrict__ w, const float* __restrict__ speed, const uint8_t* __restrict__ cls,
    const float4* __restrict__ ctrl, const int16_t* __restrict__ label, const float* __restrict__ key,
    int* __restrict__ list, int tiles_x, int tiles_y, float* __restrict__ outbuf, float* __restrict__ tchange,
    uint8_t* __restrict__ flag, int max_inner, float tol_inner, float act, float window, float tol, int max_passes,
    CoopState* __restrict__ st) {
  extern __shared__ float lds[];
  __shared__ float red[kThreads / 64];
  cooperative_groups::grid_group g = cooperative_groups::this_grid();
  const int tiles = tiles_x * tiles_y;
  const int n = a.n;
  const bool keyed = key != nullptr;
  int passes = 0;
  unsigned final_status = 2;
  while (passes < max_passes) {
    // (1) smallest flagged key
    if (keyed) {
      for (int base = blockIdx.x * kThreads; base < tiles; base += gridDim.x * kThreads) {
        const int t = base + threadIdx.x;
        float k = (t < tiles && flag[t]) ? key[t] : INFINITY;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) k = fminf(k, __shfl_xor(k, off, 64));
        if ((threadIdx.x & 63) == 0 && k < INFINITY) atomicMin(&st->kmin, __float_as_uint(k));
      }
    }
    grid_barrier(g);
    // (2) select the band
    float B = INFINITY;
    if (keyed) {
      const float lo = __uint_as_float(ld_agent(&st->kmin));
      B = __uint_as_float(ld_agent(&st->bound));
      if (lo > B) B = lo + window;
      if (lo == INFINITY) B = INFINITY;
    }
    for (int base = blockIdx.x * kThreads; base < tiles; base += gridDim.x * kThreads) {
      const int t = base + threadIdx.x;
      const bool on = t < tiles && flag[t] && (!keyed || key[t] <= B);
      const unsigned long long mask = __ballot(on);
      const int lane = threadIdx.x & 63;
      int pos = 0;
      if (lane == 0 && mask) pos = atomicAdd(&st->count, (unsigned)__popcll(mask));
      pos = __shfl(pos, 0, 64);
      if (on) list[pos + __popcll(mask & ((1ull << lane) - 1ull))] = t;
    }
    grid_barrier(g);
    const int cnt = (int)ld_agent(&st->count);
    if (blockIdx.x == 0 && threadIdx.x == 0 && keyed && B < INFINITY) st_agent(&st->bound, __float_as_uint(B));
    if (cnt > 0) {
      // (3) visits
      for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
        visit_tile<TW, TH, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, slot, list[slot], tiles_x, outbuf,
                                                      tchange, flag, max_inner, tol_inner, &st->updates, lds, red);
      grid_barrier(g);
      // (4) commits; workgroup 0 resets the selection state for the next pass
      for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
        commit_tile(slot, list[slot], TW, TH, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag, nullptr);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st_agent(&st->count, 0u);
        st_agent(&st->kmin, 0x7f800000u);
      }
      grid_barrier(g);
      ++passes;
      continue;
    }
    // nothing flagged: check sweep of every tile, one Jacobi iteration each
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      visit_tile<TW, TH, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, t, t, tiles_x, outbuf, tchange,
                                                    flag, 1, 0.0f, &st->updates, lds, red);
    grid_barrier(g);
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      commit_tile(t, t, TW, TH, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag, &st->resid);
    grid_barrier(g);
    ++passes;
    const float r = __uint_as_float(ld_agent(&st->resid));
    if (r <= tol) {
      final_status = 1;
      break;
    }
    grid_barrier(g);  // everyone has read the residual
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st_agent(&st->resid, 0u);
      st_agent(&st->kmin, 0x7f800000u);
    }
    grid_barrier(g);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&st->passes, (unsigned)passes);
    st_agent(&st->status, final_status);
  }
}

template <int TW, int TH, int DIFF, int SCHEME, int PATH, bool INDEP>
static hipError_t launch_coop_one(const SweepArgs& a, const int16_t* label, const float* key, int* list, int tiles_x,
                                  int tiles_y, float* outbuf, float* tchange, uint8_t* flag, int max_inner,
                                  float tol_inner, float act, float window, float tol, int max_passes, CoopState* st,
                                  int max_grid, int* grid_used, hipStream_t s) {
  auto kern = tile_solve_coop_kernel<TW, TH, DIFF, SCHEME, PATH, INDEP>;
  const size_t lds = tile_pass_lds_bytes(TW, TH, a.halo, INDEP);
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, lds);
  if (e != hipSuccess) return e;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int grid = per_cu * cus;
  if (grid > max_grid) grid = max_grid;
  if (grid < 1) return hipErrorInvalidConfiguration;
  *grid_used = grid;
  SweepArgs aa = a;
  float* wp = const_cast<float*>(a.w_in);
  const float* sp = a.speed;
  const uint8_t* cp = a.cls;
  const float4* ct = a.ctrl;
  void* args[] = {&aa, &wp, &sp, &cp, &ct, (void*)&label, (void*)&key, &list, &tiles_x, &tiles_y, &outbuf,
                  &tchange, &flag, &max_inner, &tol_inner, &act, &window, &tol, &max_passes, &st};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(kThreads), args, (unsigned)lds, s);
}

template <int TW, int TH>
static hipError_t launch_coop_shape(const SweepArgs& a, int diffusion, int scheme, int path, bool indep,
                                    const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                    float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                    float act, float window, float tol, int max_passes, CoopState* st, int max_grid,
                                    int* grid_used, hipStream_t s) {
#define SLHJB_CO(D, S, PA, IN)                                                                                   \
  return launch_coop_one<TW, TH, D, S, PA, IN>(a, label, key, list, tiles_x, tiles_y, outbuf, tchange, flag,     \
                                               max_inner, tol_inner, act, window, tol, max_passes, st, max_grid, \
                                               grid_used, s)
#define SLHJB_CO_S(D, PA, IN)                      \
  do {                                             \
    if (scheme == kSL2) SLHJB_CO(D, kSL2, PA, IN); \
    else SLHJB_CO(D, kSL3, PA, IN);                \
  } while (0)
#define SLHJB_CO_I(D, PA)               \
  do {                                  \
    if (indep) SLHJB_CO_S(D, PA, true); \
    else SLHJB_CO_S(D, PA, false);      \
  } while (0)
  if (path == 1) SLHJB_CO_I(kDiffNone, 1);
  if (diffusion == kDiffNone) SLHJB_CO_I(kDiffNone, 0);
  if (diffusion == kDiffIso) SLHJB_CO_I(kDiffIso, 0);
  SLHJB_CO_I(kDiffRank1, 0);
#undef SLHJB_CO_I
#undef SLHJB_CO_S
#undef SLHJB_CO
}

hipError_t launch_tile_solve_coop(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                                  const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                  float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                  float act, float window, float tol, int max_passes, void* state, int max_grid,
                                  int* grid_used, hipStream_t s) {
  CoopState* st = (CoopState*)state;
  if (shape == 2)
    return launch_coop_shape<8, 8>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                   tchange, flag, max_inner, tol_inner, act, window, tol, max_passes, st, max_grid,
                                   grid_used, s);
  if (shape == 1)
    return launch_coop_shape<16, 16>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                     tchange, flag, max_inner, tol_inner, act, window, tol, max_passes, st, max_grid,
                                     grid_used, s);
  return launch_coop_shape<32, 16>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                   tchange, flag, max_inner, tol_inner, act, window, tol, max_passes, st, max_grid,
                                   grid_used, s);
}

size_t coop_state_bytes() { return sizeof(CoopState); }

__global__ void coop_state_init_kernel(CoopState* st) {
  st->count = 0u;
  st->kmin = 0x7f800000u;
  st->bound = 0xff800000u;
  st->resid = 0u;
  st->passes = 0u;
  st->status = 0u;
  st->updates = 0ull;
}

hipError_t launch_coop_state_init(void* state, hipStream_t s) {
  coop_state_init_kernel<<<1, 1, 0, s>>>((CoopState*)state);
  return hipGetLastError();
}


// ---- device-driven passes for graph capture ---------------------------------------------------
// A pass is three launches with fixed arguments (parity q alternates between passes), so a batch
// of passes can be captured once into a graph and replayed: select -> visit -> commit. The band
// bound, the "nothing selected" jump, the check sweep when nothing is flagged and the final
// decision all happen on the device; the host only reads `done` between replays.
struct TileCtl {
  unsigned count[2];   // selected tiles of the pass with parity q
  unsigned nflag[2];   // flagged tiles seen by that selection
  unsigned kmin[2];    // bits of their smallest key
  unsigned bound;      // bits of the band bound B (-inf at start)
  unsigned resid;      // bits of the residual of the last check sweep
  unsigned checked;    // 1 after a check sweep, until the next selection reads it
  unsigned done;       // 1 once a check sweep met tol
  unsigned passes;     // passes that did work (check sweeps included)
  unsigned pad;
  unsigned long long updates;
};

__global__ void tilectl_init_kernel(TileCtl* c) {
  c->count[0] = c->count[1] = 0u;
  c->nflag[0] = c->nflag[1] = 0u;
  c->kmin[0] = c->kmin[1] = 0x7f800000u;
  c->bound = 0xff800000u;
  c->resid = 0u;
  c->checked = 0u;
  c->done = 0u;
  c->passes = 0u;
  c->pad = 0u;
  c->updates = 0ull;
}

// Also clears the outcome of the last check sweep once read: a workgroup that reads it after
// workgroup 0 cleared it sees "no check" and selects, which is what every workgroup does when the
// check failed; when it met tol nothing is cleared and every workgroup stops.
__global__ void tilectl_select_kernel(const uint8_t* __restrict__ flag, const float* __restrict__ key, int tiles,
                                      float tol, int q, int* __restrict__ list, TileCtl* __restrict__ c) {
  if (c->done) return;
  if (c->checked) {
    const bool ok = __uint_as_float(c->resid) <= tol;
    if (ok) {
      if (blockIdx.x == 0 && threadIdx.x == 0) c->done = 1u;
      return;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->checked = 0u;
    c->resid = 0u;
  }
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const float B = key ? __uint_as_float(c->bound) : INFINITY;
  bool fl = false, on = false;
  float k = INFINITY;
  if (t < tiles && flag[t]) {
    fl = true;
    if (key) k = key[t];
    on = !key || k <= B;
  }
  const unsigned long long fmask = __ballot(fl), mask = __ballot(on);
  const int lane = threadIdx.x & 63;
  if (key) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) k = fminf(k, __shfl_xor(k, off, 64));
  }
  int base = 0;
  if (lane == 0) {
    if (fmask) atomicAdd(&c->nflag[q], (unsigned)__popcll(fmask));
    if (key && k < INFINITY) atomicMin(&c->kmin[q], __float_as_uint(k));
    if (mask) base = atomicAdd(&c->count[q], (unsigned)__popcll(mask));
  }
  base = __shfl(base, 0, 64);
  if (on) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = t;
}

template <int TW, int TH, int DIFF, int SCHEME, int PATH, bool INDEP>
__global__ __launch_bounds__(kThreads) void tilectl_visit_kernel(
    SweepArgs a, const float* __restrict__ w, const float* __restrict__ speed, const uint8_t* __restrict__ cls,
    const float4* __restrict__ ctrl, const int16_t* __restrict__ label, const int* __restrict__ list, int tiles_x,
    int tiles, float* __restrict__ outbuf, float* __restrict__ tchange, uint8_t* __restrict__ flag, int max_inner,
    float tol_inner, float window, int q, TileCtl* __restrict__ c) {
  if (c->done) return;
  extern __shared__ float lds[];
  __shared__ float red[kThreads / 64];
  const int cnt = (int)c->count[q];
  const int nf = (int)c->nflag[q];
  if (cnt > 0) {
    for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
      visit_tile<TW, TH, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, slot, list[slot], tiles_x, outbuf,
                                                    tchange, flag, max_inner, tol_inner, &c->updates, lds, red);
  } else if (nf > 0) {
    // flagged tiles exist but none is in the band: move the band up to the smallest flagged key
    if (blockIdx.x == 0 && threadIdx.x == 0) c->bound = __float_as_uint(__uint_as_float(c->kmin[q]) + window);
  } else {
    // nothing flagged: check sweep, one Jacobi iteration of every tile
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      visit_tile<TW, TH, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, t, t, tiles_x, outbuf, tchange,
                                                    flag, 1, 0.0f, &c->updates, lds, red);
  }
}

__global__ __launch_bounds__(kThreads) void tilectl_commit_kernel(const int* __restrict__ list, int tw, int th,
                                                                  int tiles_x, int tiles_y, int n,
                                                                  const float* __restrict__ outbuf,
                                                                  const float* __restrict__ tchange, float act,
                                                                  const uint8_t* __restrict__ cls,
                                                                  float* __restrict__ w, uint8_t* __restrict__ flag,
                                                                  int q, TileCtl* __restrict__ c) {
  if (c->done) return;
  const int cnt = (int)c->count[q];
  const int nf = (int)c->nflag[q];
  const int tiles = tiles_x * tiles_y;
  if (cnt > 0) {
    for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
      commit_tile(slot, list[slot], tw, th, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag, nullptr);
  } else if (nf == 0) {
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      commit_tile(t, t, tw, th, tiles_x, tiles_y, n, outbuf, tchange, act, cls, w, flag, &c->resid);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (cnt > 0 || nf == 0) c->passes += 1u;
    c->checked = (cnt == 0 && nf == 0) ? 1u : 0u;
    // the other parity's counters serve the next pass; they were last read by the previous pass
    c->count[q ^ 1] = 0u;
    c->nflag[q ^ 1] = 0u;
    c->kmin[q ^ 1] = 0x7f800000u;
  }
}

static_assert(offsetof(TileCtl, resid) == 7 * 4 && offsetof(TileCtl, done) == 9 * 4 &&
                  offsetof(TileCtl, passes) == 10 * 4 && offsetof(TileCtl, updates) == 12 * 4,
              "host reads these words");
size_t tilectl_bytes() { return sizeof(TileCtl); }

hipError_t launch_tilectl_init(void* ctl, hipStream_t s) {
  tilectl_init_kernel<<<1, 1, 0, s>>>((TileCtl*)ctl);
  return hipGetLastError();
}

template <int TW, int TH>
static void launch_tilectl_pass_shape(const SweepArgs& a, int diffusion, int scheme, int path, bool indep,
                                      const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                      float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                      float act, float window, float tol, int q, TileCtl* c, int grid,
                                      hipEvent_t ev_before, hipEvent_t ev_after, hipStream_t s) {
  const int tiles = tiles_x * tiles_y;
  tilectl_select_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(flag, key, tiles, tol, q, list, c);
  const size_t lds = tile_pass_lds_bytes(TW, TH, a.halo, indep);
  if (ev_before) hipEventRecord(ev_before, s);
#define SLHJB_TV(D, S, PA, IN)                                                                                     \
  tilectl_visit_kernel<TW, TH, D, S, PA, IN><<<grid, kThreads, lds, s>>>(a, a.w_in, a.speed, a.cls, a.ctrl, label, \
                                                                         list, tiles_x, tiles, outbuf, tchange,    \
                                                                         flag, max_inner, tol_inner, window, q, c)
#define SLHJB_TV_S(D, PA, IN)                      \
  do {                                             \
    if (scheme == kSL2) SLHJB_TV(D, kSL2, PA, IN); \
    else SLHJB_TV(D, kSL3, PA, IN);                \
  } while (0)
#define SLHJB_TV_I(D, PA)               \
  do {                                  \
    if (indep) SLHJB_TV_S(D, PA, true); \
    else SLHJB_TV_S(D, PA, false);      \
  } while (0)
  if (path == 1) SLHJB_TV_I(kDiffNone, 1);
  else if (diffusion == kDiffNone) SLHJB_TV_I(kDiffNone, 0);
  else if (diffusion == kDiffIso) SLHJB_TV_I(kDiffIso, 0);
  else SLHJB_TV_I(kDiffRank1, 0);
#undef SLHJB_TV_I
#undef SLHJB_TV_S
#undef SLHJB_TV
  if (ev_after) hipEventRecord(ev_after, s);
  tilectl_commit_kernel<<<grid, kThreads, 0, s>>>(list, TW, TH, tiles_x, tiles_y, a.n, outbuf, tchange, act, a.cls,
                                                  const_cast<float*>(a.w_in), flag, q, c);
}

hipError_t launch_tilectl_pass(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                               const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                               float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner, float act,
                               float window, float tol, int q, void* ctl, int grid, hipEvent_t ev_before,
                               hipEvent_t ev_after, hipStream_t s) {
  if (shape == 2)
    launch_tilectl_pass_shape<8, 8>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                    tchange, flag, max_inner, tol_inner, act, window, tol, q, (TileCtl*)ctl, grid, ev_before,
                                    ev_after, s);
  else if (shape == 1)
    launch_tilectl_pass_shape<16, 16>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                      tchange, flag, max_inner, tol_inner, act, window, tol, q, (TileCtl*)ctl, grid, ev_before,
                                    ev_after, s);
  else
    launch_tilectl_pass_shape<32, 16>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf,
                                      tchange, flag, max_inner, tol_inner, act, window, tol, q, (TileCtl*)ctl, grid, ev_before,
                                    ev_after, s);
  return hipGetLastError();
}

}  // namespace slhjb
