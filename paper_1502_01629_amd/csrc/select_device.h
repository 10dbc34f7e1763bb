// Band selection of flagged tiles, shared by the tile solver and the labeler.
#pragma once

#include "internal.h"

namespace slhjb {

constexpr int kSelectThreads = 1024;

// An empty asm statement that takes the values as operands ("+s" for uniform ones, "+v" for
// per-lane ones): the loads that produce them must be complete at this point, so loads written
// above it are in flight at the same time instead of each being moved down to its first use
// behind a branch (one memory latency instead of several at the start of a short kernel).
#define SLHJB_ISSUE_TOGETHER(...) asm volatile("" : __VA_ARGS__)

// Neighbours of a tile that read node (lx, ly) of it in their halo: the node lies within the
// dependence radius d of the tile's side or corner facing them. Bit (dy + 1) * 3 + (dx + 1) stands
// for the neighbour at tile offset (dx, dy).
__host__ __device__ inline unsigned near_sides(int lx, int ly, int tw, int th, int d) {
  const bool w = lx < d, e = lx >= tw - d, s = ly < d, nn = ly >= th - d;
  return (w ? 1u << 3 : 0u) | (e ? 1u << 5 : 0u) | (s ? 1u << 1 : 0u) | (nn ? 1u << 7 : 0u) |
         (w && s ? 1u << 0 : 0u) | (e && s ? 1u << 2 : 0u) | (w && nn ? 1u << 6 : 0u) | (e && nn ? 1u << 8 : 0u);
}

__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

// One tile per thread of a kSelectThreads workgroup: `fl` says the tile is flagged, `on` that it is
// selected, `k` is its key (+inf when not flagged or unkeyed). The workgroup adds its flagged and
// selected counts to *nflag and *count and lowers *kmin with one atomic each (device-scope atomics
// on one word from every workgroup of the grid are what made a per-wavefront version slow), then
// writes its selected tiles to list at the offset the count atomic returned. Every thread of the
// workgroup must call it. The order of the list depends on timing, its contents do not.
__device__ __forceinline__ void block_select(int t, bool fl, bool on, float k, bool keyed, unsigned* count,
                                             unsigned* nflag, unsigned* kmin, int* list) {
  constexpr int W = kSelectThreads / 64;
  __shared__ unsigned s_on[W], s_fl[W];
  __shared__ float s_k[W];
  __shared__ unsigned s_base;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long fmask = __ballot(fl), mask = __ballot(on);
  if (keyed) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) k = fminf(k, __shfl_xor(k, off, 64));
  }
  if (lane == 0) {
    s_on[wave] = (unsigned)__popcll(mask);
    s_fl[wave] = (unsigned)__popcll(fmask);
    s_k[wave] = k;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned total = 0u, nf = 0u;
    float km = INFINITY;
    const int waves = (int)(blockDim.x >> 6);
    for (int w = 0; w < waves; ++w) {
      const unsigned c = s_on[w];
      s_on[w] = total;  // exclusive prefix over the wavefronts
      total += c;
      nf += s_fl[w];
      km = fminf(km, s_k[w]);
    }
    if (nf) atomicAdd(nflag, nf);
    if (keyed && km < INFINITY) atomicMin(kmin, __float_as_uint(km));
    s_base = total ? atomicAdd(count, total) : 0u;
  }
  __syncthreads();
  if (on) list[s_base + s_on[wave] + (unsigned)__popcll(mask & ((1ull << lane) - 1ull))] = t;
}

}  // namespace slhjb
