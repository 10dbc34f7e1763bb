// Active-tile solver: the GPU form of the paper's per-patch computation with a fast-marching-like
// order (Section 4.2 "The role of causality", Section 4.3 computation step).
//
// The grid is cut into tiles (32 x 16, 16 x 16 or 8 x 8 nodes). A pass takes a list of tiles; each workgroup stages
// its tile and an interpolation halo in LDS and runs Jacobi iterations of the scheme on the
// tile's FREE nodes, with the halo frozen, until no node moves by more than tol_inner (or
// max_inner iterations). Every tile of a pass reads the iterate as it was before the pass, so the
// outcome does not depend on scheduling. The graph-driven and batched passes keep the iterate in
// two arrays: a visit writes its tile into the array that does not hold the tile's current values
// and flags, for the next pass, each of the 8 neighbours whose halo holds a node that moved by
// more than the activation threshold (the tile's strip of the dependence radius on that side), and
// the tile itself when its visit stopped unsettled. The cooperative driver stages the results
// instead and writes them back, and flags, in a commit step. The next pass takes the flagged tiles; with keys
// (the arrival time of u_hat, min over the tile) only a band of them: those whose key is within
// a window of the smallest flagged key. That is the order "by increasing u_hat" of the paper at
// tile granularity, bucketed so that a whole ring of tiles runs at once, and it keeps tiles
// whose upwind values are still moving from being iterated to convergence against stale halos.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_ext.h>
#include <cstring>
#include <cstddef>

#include "select_device.h"
#include "sweep_device.h"

namespace slhjb {

// Visit of a T x T tile by T*T*S threads: lane = node, S groups of wavefronts each walk one S-th
// of the controls (whole quadrants on the first-ring path, a contiguous slice of the list
// otherwise) for all nodes of the tile. Per inner iteration the S partial optima go through LDS
// and the first group combines them in a fixed order, so the result does not depend on timing.
// Splitting the controls shortens one inner iteration S times, which is what bounds a pass when
// few tiles are selected.
//
// Modified policy iteration (pe > 0): after every full iteration, pe policy-evaluation
// iterations apply each node's maximising control of that full iteration only (one candidate,
// no search); the fixed point is the same, and only full iterations decide that a tile settled.
// Their node updates are counted apart in pe_acc. The counts go to thread 0's `acc` and `pe_acc`,
// which the caller accumulates over its visits and publishes once (same-word device atomics from
// every visit of a pass cost the pass about 1.5 us).
// How far a tile's values reach into its neighbours' updates: one cell on the first-ring path
// (the 3 x 3 stencil), the interpolation halo otherwise.
template <int PATH>
__device__ __forceinline__ int dependence_radius(const SweepArgs& a) {
  return PATH == 1 ? 1 : a.halo;
}

// Direct write-back (graph-driven and batched passes). The iterate lives in two n x n arrays; word[t] holds
// (p << 1) | a, where a names the array with tile t's current values and p the pass that wrote
// them there. A visit in pass `seq` reads every node from the array that held it before the pass:
// a word already stamped with `seq` belongs to a tile written in this pass, whose earlier values
// are in the other array, which no visit of the pass writes. It then writes its own tile to the
// array its word does not name and stamps the word. Words start at 0 and passes count from 1.
struct TileDirect {
  float* wa;       // the caller's iterate
  float* wb;       // the second array, same layout
  unsigned* word;  // [tiles]
  int tiles_y;
};

__device__ __forceinline__ float direct_load(const TileDirect& D, size_t idx, int tile, unsigned seq) {
  // the three loads are independent: the word decides which value is kept
  const unsigned wd = D.word[tile];
  const float va = D.wa[idx], vb = D.wb[idx];
  const unsigned arr = (wd >> 1) == seq ? (wd & 1u) ^ 1u : (wd & 1u);
  return arr ? vb : va;
}

// Lane b (0..8, b = (dy + 1) * 3 + dx + 1) flags the tile at offset (dx, dy) from tile tid if bit
// b of `sides` is set, or, for the tile itself, if `self`. Nine lanes store at once: one thread
// walking the nine made the 2049^2 step 0.2 ms slower.
__device__ __forceinline__ void flag_lane(int b, int tid, int tiles_x, int tiles_y, unsigned sides, bool self,
                                          uint8_t* __restrict__ flag) {
  const int dx = b % 3 - 1, dy = b / 3 - 1;
  const int nx = tid % tiles_x + dx, ny = tid / tiles_x + dy;
  const bool take = b == 4 ? self : ((sides >> b) & 1u) != 0u;
  if (take && nx >= 0 && ny >= 0 && nx < tiles_x && ny < tiles_y) flag[ny * tiles_x + nx] = 1;
}

template <int T, int S, int DIFF, int SCHEME, int PATH, bool INDEP, bool DIRECT>
__device__ __forceinline__ void visit_tile_split(const SweepArgs& a, const float* __restrict__ w,
                                                 const float* __restrict__ speed, const uint8_t* __restrict__ cls,
                                                 const float4* __restrict__ ctrl, const int16_t* __restrict__ label,
                                                 int slot, int tid, int tiles_x, float* __restrict__ outbuf,
                                                 float* __restrict__ tchange, uint8_t* __restrict__ flag, int max_inner,
                                                 float tol_inner, float act, unsigned* __restrict__ tsides,
                                                 unsigned long long& acc, float* lds, float* red, int pe,
                                                 unsigned long long& pe_acc, const TileDirect& D, unsigned seq,
                                                 float& tmax) {
  constexpr int TT = T * T, NT = TT * S;
  __shared__ unsigned sides_red[NT / 64];
  static_assert(TT % 64 == 0 && (S == 2 || S == 4), "split tile shape");
  const int R = a.halo;
  const int LW = T + 2 * R, span = LW * LW;
  float* bufA = lds;
  float* bufB = lds + span;
  float* pn = lds + 2 * span;
  float* pd = pn + NT;
  int* pix = (int*)(pd + NT);
  int16_t* labs = (int16_t*)(pix + NT);
  const int n = a.n;
  // TT is a multiple of 64, so a wavefront lies in one part: readfirstlane states that, and the
  // control loops get wavefront-uniform bounds (scalar loads of the control table, no per-lane
  // loop exit)
  const int node = threadIdx.x % TT, part = __builtin_amdgcn_readfirstlane(threadIdx.x / TT);
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  const int x0 = tx * T, y0 = ty * T;
  // direct write-back: the array holding this tile's values (its word is not stamped with this pass)
  const unsigned own = DIRECT ? (D.word[tid] & 1u) : 0u;
  if (!DIRECT && threadIdx.x == 0) flag[tid] = 0;  // direct: the selection cleared it
  for (int e = threadIdx.x; e < span; e += NT) {
    const int ly = e / LW, lx = e - ly * LW;
    const int gx = x0 - R + lx, gy = y0 - R + ly;
    const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n;
    float val = 0.0f;
    if (in) {
      if (DIRECT) val = direct_load(D, (size_t)gy * n + gx, (gy / T) * tiles_x + gx / T, seq);
      else val = w[(size_t)gy * n + gx];
    }
    bufA[e] = val;
    bufB[e] = val;
    if (INDEP) labs[e] = in ? label[(size_t)gy * n + gx] : (int16_t)-32768;
  }
  const int lx = node % T, ly = node / T;
  const int gi = x0 + lx, gj = y0 + ly;
  const int li = (ly + R) * LW + lx + R;
  bool fr = false;
  float kk = 0.0f, w0 = 0.0f;  // w0: the node's value before the visit, for the move it reports
  float qn = 0.0f, dn = 0.0f;  // path 2: the node's cost term and noise offset
  constexpr bool GEN = PATH == 2;
  if (gi < n && gj < n) {
    const size_t idx = (size_t)gj * n + gi;
    fr = cls[idx] == kFree;
    if (fr) kk = a.r * (speed ? speed[idx] : a.speed_const);
    if (GEN && fr) {
      qn = node_cost(a, idx);
      dn = node_noise(a, idx);
    }
  }
  const bool interior = x0 >= 1 && x0 + T - 1 <= n - 2 && y0 >= 1 && y0 + T - 1 <= n - 2;
  // general path: the node's drift offset k d(x), loaded once for the whole visit (the same
  // expressions as general_partial's own load, so the same bits)
  float2 kd = make_float2(0.0f, 0.0f);
  if (PATH != 1 && a.drift && fr) {
    const float2 dv = a.drift[(size_t)gj * n + gi];
    kd = make_float2(kk * dv.x, kk * dv.y);
  }
  const int slice = a.n_controls / S;  // the padded list length is a multiple of 4
  constexpr int QP = 4 / S;            // quadrants per part on the first-ring path
  __syncthreads();
  if (gi < n && gj < n) w0 = bufA[li];  // the staged value
  float* cur = bufA;
  float* nxt = bufB;
  int it = 0, evals = 0;
  int pol = 0;  // maximising control of the last full iteration (part 0)
  PolicyEval64 pv64{};  // first-ring path: that control's FP64 evaluation (part 0)
  for (;;) {
    if (fr) {
      float num, den;
      int mi = 0;
      if (PATH == 1) {
        // the maximiser is always tracked: its value is recomputed in FP64 (policy_apply64)
        const float* Tp = cur + li;
        const int16_t* L = INDEP ? labs + li : nullptr;
        if (interior)
          ring1_partial<SCHEME, false, INDEP, true>(Tp, LW, kk, ctrl, a, false, false, false, false, L, part * QP,
                                                    part * QP + QP, num, den, &mi);
        else
          ring1_partial<SCHEME, true, INDEP, true>(Tp, LW, kk, ctrl, a, gi == 0, gi == n - 1, gj == 0, gj == n - 1,
                                                   L, part * QP, part * QP + QP, num, den, &mi);
      } else {
        if (pe > 0)
          general_partial<DIFF, SCHEME, INDEP, true, GEN>(cur, LW, li, gi, gj, kk, cur[li], ctrl, a,
                                                          INDEP ? labs : nullptr, INDEP ? labs[li] : 0, part * slice,
                                                          (part + 1) * slice, num, den, &mi, &kd, nullptr, qn, dn);
        else
          general_partial<DIFF, SCHEME, INDEP, false, GEN>(cur, LW, li, gi, gj, kk, cur[li], ctrl, a,
                                                           INDEP ? labs : nullptr, INDEP ? labs[li] : 0, part * slice,
                                                           (part + 1) * slice, num, den, nullptr, &kd, nullptr, qn, dn);
      }
      pn[part * TT + node] = num;
      pd[part * TT + node] = den;
      pix[part * TT + node] = mi;
    }
    __syncthreads();
    float lmax = 0.0f;
    if (part == 0 && fr) {
      float v;
      int bi = pix[node];
      if (SCHEME == kSL2) {
        float m = pn[node];
#pragma unroll
        for (int q = 1; q < S; ++q) {
          const float qm = pn[q * TT + node];
          if (qm > m) {
            m = qm;
            bi = pix[q * TT + node];
          }
        }
        constexpr int K = Feet<DIFF>::K;
        v = PATH == 1 ? a.beta * (cur[li] + m) : a.beta * m * (1.0f / (float)K);
      } else {
        float bn = pn[node], bd = pd[node];
#pragma unroll
        for (int q = 1; q < S; ++q) {
          const float qn = pn[q * TT + node], qd = pd[q * TT + node];
          if (qn * bd > bn * qd) {
            bn = qn;
            bd = qd;
            bi = pix[q * TT + node];
          }
        }
        // through the reciprocal, as the policy evaluation of the first-ring path divides
        v = (a.beta * bn) * (1.0f / bd);
      }
      if (PATH == 1) {
        // the winner's value in FP64 (the same function as the policy evaluations below)
        pv64 = policy_prepare64<SCHEME>(LW, kk, ctrl[bi], a, gi == 0, gi == n - 1, gj == 0, gj == n - 1);
        v = policy_apply64<SCHEME, INDEP>(cur + li, pv64, a, INDEP ? labs + li : nullptr);
      }
      pol = bi;
      nxt[li] = v;
      lmax = fabsf(v - cur[li]);
    }
    const int moving = __syncthreads_or(lmax > tol_inner);
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
    ++it;
    if (!moving || it >= max_inner) break;
    // policy evaluation: the last full iteration's maximising control of every node, one
    // candidate each; leaves room for the full iteration that must end the visit
    if (pe > 0) {
      const float4 cm = ctrl[pol];
      for (int e = 0; e < pe && it < max_inner - 1; ++e) {
        if (part == 0 && fr) {
          if (PATH == 1) {
            nxt[li] = policy_apply64<SCHEME, INDEP>(cur + li, pv64, a, INDEP ? labs + li : nullptr);
          } else {
            float num, den;
            general_partial<DIFF, SCHEME, INDEP, false, GEN>(cur, LW, li, gi, gj, kk, cur[li], ctrl, a,
                                                             INDEP ? labs : nullptr, INDEP ? labs[li] : 0, pol, pol + 1,
                                                             num, den, nullptr, &kd, &cm, qn, dn);
            constexpr int K = Feet<DIFF>::K;
            nxt[li] = SCHEME == kSL2 ? a.beta * num * (1.0f / (float)K) : (a.beta * num) * (1.0f / den);
          }
        }
        __syncthreads();
        float* t2 = cur;
        cur = nxt;
        nxt = t2;
        ++it;
        ++evals;
      }
    }
  }
  float moved = 0.0f;
  unsigned sides = 0u;
  if (part == 0) {
    if (DIRECT) {
      if (gi < n && gj < n) (own ? D.wa : D.wb)[(size_t)gj * n + gi] = cur[li];
    } else {
      outbuf[(size_t)slot * TT + node] = cur[li];
    }
    if (fr) moved = fabsf(cur[li] - w0);
    if (moved > act) sides = near_sides(lx, ly, T, T, dependence_radius<PATH>(a));
  }
  moved = wave_max(moved);
  sides = wave_or(sides);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = moved;
    sides_red[threadIdx.x >> 6] = sides;
  }
  const int free_total = __syncthreads_count(part == 0 && fr);
  if (threadIdx.x < (DIRECT ? 9 : 1)) {
    float m = red[0];
    unsigned sd = sides_red[0];
#pragma unroll
    for (int k = 1; k < TT / 64; ++k) {
      m = fmaxf(m, red[k]);
      sd |= sides_red[k];
    }
    // a visit that stopped at max_inner while still moving is marked by a negative sign; after a
    // single iteration (the check sweeps) that is a move beyond the activation threshold
    const bool unsettled = it >= max_inner && (max_inner > 1 || m > act);
    if (DIRECT) {
      // what the commit step does with the staged move and sides
      const float mm = unsettled ? fmaxf(m, 1e-30f) : m;
      if (mm > act) flag_lane(threadIdx.x, tid, tiles_x, D.tiles_y, sd, unsettled, flag);
      if (threadIdx.x == 0) {
        tmax = fmaxf(tmax, mm);
        D.word[tid] = (seq << 1) | (own ^ 1u);
      }
    } else {
      tchange[slot] = unsettled ? -fmaxf(m, 1e-30f) : m;
      tsides[slot] = sd;
    }
  }
  if (threadIdx.x == 0) {
    acc += (unsigned long long)(it - evals) * (unsigned long long)free_total;
    pe_acc += (unsigned long long)evals * (unsigned long long)free_total;
  }
  __syncthreads();
}

// One visit of tile `tid`, written directly (DIRECT) or staged into slot `slot` of outbuf/tchange:
// Jacobi iterations in LDS
// against the frozen halo until no node moves by more than tol_inner (or max_inner).
template <int TW, int TH, int S, int DIFF, int SCHEME, int PATH, bool INDEP, bool DIRECT = false>
__device__ __forceinline__ void visit_tile(const SweepArgs& a, const float* __restrict__ w,
                                           const float* __restrict__ speed, const uint8_t* __restrict__ cls,
                                           const float4* __restrict__ ctrl, const int16_t* __restrict__ label,
                                           int slot, int tid, int tiles_x, float* __restrict__ outbuf,
                                           float* __restrict__ tchange, uint8_t* __restrict__ flag, int max_inner,
                                           float tol_inner, float act, unsigned* __restrict__ tsides,
                                           unsigned long long& acc, float* lds, float* red, int pe,
                                           unsigned long long& pe_acc, const TileDirect& D = TileDirect{},
                                           unsigned seq = 0u, float* tmax = nullptr) {
  float tmax_unused = 0.0f;
  float& tm = tmax ? *tmax : tmax_unused;
  if constexpr (S > 1) {
    static_assert(TW == TH, "split tiles are square");
    visit_tile_split<TW, S, DIFF, SCHEME, PATH, INDEP, DIRECT>(a, w, speed, cls, ctrl, label, slot, tid, tiles_x,
                                                               outbuf, tchange, flag, max_inner, tol_inner, act,
                                                               tsides, acc, lds, red, pe, pe_acc, D, seq, tm);
    return;
  } else {
  (void)pe;
  (void)pe_acc;
  constexpr int kTW = TW, kTH = TH, kTN = TW * TH, NPT = kTN / kThreads;  // NPT nodes per thread
  __shared__ unsigned sides_red[kThreads / 64];
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
    const unsigned own = DIRECT ? (D.word[tid] & 1u) : 0u;
    if (!DIRECT && threadIdx.x == 0) flag[tid] = 0;
    for (int e = threadIdx.x; e < span; e += kThreads) {
      const int ly = e / LW, lx = e - ly * LW;
      const int gx = x0 - R + lx, gy = y0 - R + ly;
      const bool in = gx >= 0 && gx < n && gy >= 0 && gy < n;
      float val = 0.0f;
      if (in) {
        if (DIRECT) val = direct_load(D, (size_t)gy * n + gx, (gy / kTH) * tiles_x + gx / kTW, seq);
        else val = w[(size_t)gy * n + gx];
      }
      bufA[e] = val;
      bufB[e] = val;
      if (INDEP) labs[e] = in ? label[(size_t)gy * n + gx] : (int16_t)-32768;
    }
    // the NPT nodes of this thread
    int li[NPT], gi[NPT], gj[NPT];
    bool fr[NPT];
    float kk[NPT], w0[NPT], qn[NPT], dn[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const int lx = q & (kTW - 1), ly = q / kTW;
      gi[r] = x0 + lx;
      gj[r] = y0 + ly;
      li[r] = (ly + R) * LW + lx + R;
      fr[r] = false;
      kk[r] = 0.0f;
      w0[r] = 0.0f;
      qn[r] = 0.0f;
      dn[r] = 0.0f;
      if (gi[r] < n && gj[r] < n) {
        const size_t idx = (size_t)gj[r] * n + gi[r];
        fr[r] = cls[idx] == kFree;
        if (fr[r]) kk[r] = a.r * (speed ? speed[idx] : a.speed_const);
        if (PATH == 2 && fr[r]) {
          qn[r] = node_cost(a, idx);
          dn[r] = node_noise(a, idx);
        }
      }
    }
    __syncthreads();  // tile staged
#pragma unroll
    for (int r = 0; r < NPT; ++r)
      if (gi[r] < n && gj[r] < n) w0[r] = bufA[li[r]];
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
            v = general_update<DIFF, SCHEME, INDEP, PATH == 2>(cur, LW, li[r], gi[r], gj[r], kk[r], cur[li[r]], ctrl,
                                                               a, INDEP ? labs : nullptr, INDEP ? labs[li[r]] : 0, qn[r],
                                                               dn[r]);
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
    unsigned sides = 0u;
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
      const int q = threadIdx.x + r * kThreads;
      const float v = cur[li[r]];
      if (DIRECT) {
        if (gi[r] < n && gj[r] < n) (own ? D.wa : D.wb)[(size_t)gj[r] * n + gi[r]] = v;
      } else {
        outbuf[(size_t)slot * kTN + q] = v;
      }
      const float mv = fr[r] ? fabsf(v - w0[r]) : 0.0f;
      moved = fmaxf(moved, mv);
      if (mv > act) sides |= near_sides(q & (kTW - 1), q / kTW, kTW, kTH, dependence_radius<PATH>(a));
    }
    moved = wave_max(moved);
    sides = wave_or(sides);
    if ((threadIdx.x & 63) == 0) {
      red[wave] = moved;
      sides_red[wave] = sides;
    }
    int nf = 0;
#pragma unroll
    for (int r = 0; r < NPT; ++r) nf += fr[r] ? 1 : 0;
    const int free_total = __syncthreads_count(nf >= 1) + (NPT > 1 ? __syncthreads_count(nf >= 2) : 0);
    if (threadIdx.x < (DIRECT ? 9 : 1)) {
      float m = red[0];
      unsigned sd = sides_red[0];
#pragma unroll
      for (int k = 1; k < kThreads / 64; ++k) {
        m = fmaxf(m, red[k]);
        sd |= sides_red[k];
      }
      // a visit that stopped at max_inner while still moving is marked by a negative sign; after a
      // single iteration (the check sweeps) that is a move beyond the activation threshold
      const bool unsettled = it >= max_inner && (max_inner > 1 || m > act);
      if (DIRECT) {
        const float mm = unsettled ? fmaxf(m, 1e-30f) : m;
        if (mm > act) flag_lane(threadIdx.x, tid, tiles_x, D.tiles_y, sd, unsettled, flag);
        if (threadIdx.x == 0) {
          tm = fmaxf(tm, mm);
          D.word[tid] = (seq << 1) | (own ^ 1u);
        }
      } else {
        tchange[slot] = unsettled ? -fmaxf(m, 1e-30f) : m;
        tsides[slot] = sd;
      }
    }
    if (threadIdx.x == 0) {
      acc += (unsigned long long)it * (unsigned long long)free_total;
    }
    __syncthreads();
  }
  }
}

// Write staged tile `tid` (slot `slot`) back and flag the neighbours in `sides` (the visit found a
// node that moved by more than `act` in the strip they read); the tile itself is flagged again only
// if its visit stopped before settling. `tc` is the visit's move of the tile, tchange[slot].
__device__ __forceinline__ void commit_tile(int slot, int tid, int tw, int th, int tiles_x, int tiles_y, int n,
                                            const float* __restrict__ outbuf, float tc, unsigned sides, float act,
                                            const uint8_t* __restrict__ cls, float* __restrict__ w,
                                            uint8_t* __restrict__ flag, float& tmax) {
  // tmax: thread 0 keeps the largest move of the tiles it committed (the check sweep's residual)
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  const int tn = tw * th;
  for (int q = threadIdx.x; q < tn; q += kThreads) {
    const int gx = tx * tw + q % tw, gy = ty * th + q / tw;
    if (gx < n && gy < n) {
      const size_t idx = (size_t)gy * n + gx;
      if (cls[idx] == kFree) w[idx] = outbuf[(size_t)slot * tn + q];
    }
  }
  if (threadIdx.x < 9) {
    const float m = fabsf(tc);
    if (threadIdx.x == 0) tmax = fmaxf(tmax, m);
    if (m > act) flag_lane(threadIdx.x, tid, tiles_x, tiles_y, sides, tc < 0.0f, flag);
  }
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
      // the arrival time of the start: T = -ln(w / V*) / lambda (Kruzkov), or v = V* - w itself
      // in the undiscounted form (lambda = 0)
      if (cls[idx] == kFree) {
        if (lambda == 0.0f) best = fminf(best, vstar - ww);
        else if (ww > 0.0f) best = fminf(best, -logf(ww / vstar) / lambda);
      }
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

size_t tile_pass_lds_bytes(const TileShape& sh, int halo, bool indep) {
  const size_t span = (size_t)(sh.tw + 2 * halo) * (sh.th + 2 * halo);
  // split shapes: per thread a partial numerator, denominator and control index
  const size_t partials = sh.split > 1 ? 3 * (size_t)sh.threads * sizeof(float) : 0;
  return 2 * span * sizeof(float) + partials + (indep ? span * sizeof(int16_t) : 0);
}

TileShape tile_shape_of(int shape) {
  switch (shape) {
    case 0: return {32, 16, 1, kThreads};
    case 1: return {16, 16, 1, kThreads};
    case 2: return {8, 8, 4, 256};
    case 3: return {16, 16, 4, 1024};
    default: return {16, 16, 2, 512};
  }
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
  unsigned long long pe_updates;
};
static_assert(offsetof(CoopState, updates) == 6 * 4 && offsetof(CoopState, pe_updates) == 8 * 4 &&
                  sizeof(CoopState) <= 64,
              "host reads these words");

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

template <int TW, int TH, int SPL, int DIFF, int SCHEME, int PATH, bool INDEP,
          int NT = (SPL == 1 ? kThreads : TW * TH * SPL)>
__global__ __launch_bounds__(NT) void tile_solve_coop_kernel(
    SweepArgs a, float* __restrict__ w, const float* __restrict__ speed, const uint8_t* __restrict__ cls,
    const float4* __restrict__ ctrl, const int16_t* __restrict__ label, const float* __restrict__ key,
    int* __restrict__ list, int tiles_x, int tiles_y, float* __restrict__ outbuf, float* __restrict__ tchange,
    uint8_t* __restrict__ flag, int max_inner, float tol_inner, float act, float window, float tol, int max_passes,
    CoopState* __restrict__ st, int pe) {
  extern __shared__ float lds[];
  __shared__ float red[NT / 64];
  cooperative_groups::grid_group g = cooperative_groups::this_grid();
  const int tiles = tiles_x * tiles_y;
  unsigned* tsides = reinterpret_cast<unsigned*>(tchange + tiles);
  const int n = a.n;
  const bool keyed = key != nullptr;
  int passes = 0;
  unsigned final_status = 2;
  unsigned long long acc = 0ull, pe_acc = 0ull;  // this workgroup's node updates (thread 0)
  while (passes < max_passes) {
    // (1) smallest flagged key
    if (keyed) {
      for (int base = blockIdx.x * NT; base < tiles; base += gridDim.x * NT) {
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
    for (int base = blockIdx.x * NT; base < tiles; base += gridDim.x * NT) {
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
        visit_tile<TW, TH, SPL, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, slot, list[slot], tiles_x, outbuf,
                                                      tchange, flag, max_inner, tol_inner, act, tsides, acc, lds, red,
                                                      pe, pe_acc);
      grid_barrier(g);
      // (4) commits; workgroup 0 resets the selection state for the next pass
      float unused = 0.0f;
      for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
        commit_tile(slot, list[slot], TW, TH, tiles_x, tiles_y, n, outbuf, tchange[slot], tsides[slot], act, cls, w,
                    flag, unused);
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
      visit_tile<TW, TH, SPL, DIFF, SCHEME, PATH, INDEP>(a, w, speed, cls, ctrl, label, t, t, tiles_x, outbuf, tchange,
                                                    flag, 1, 0.0f, act, tsides, acc, lds, red, 0, pe_acc);
    grid_barrier(g);
    float tmax = 0.0f;  // largest move of this workgroup's tiles (thread 0)
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      commit_tile(t, t, TW, TH, tiles_x, tiles_y, n, outbuf, tchange[t], tsides[t], act, cls, w, flag, tmax);
    if (threadIdx.x == 0 && tmax > 0.0f) atomicMax(&st->resid, __float_as_uint(tmax));  // one per workgroup
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
  if (threadIdx.x == 0) {
    if (acc) atomicAdd(&st->updates, acc);
    if (pe_acc) atomicAdd(&st->pe_updates, pe_acc);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st_agent(&st->passes, (unsigned)passes);
    st_agent(&st->status, final_status);
  }
}

template <int TW, int TH, int SPL, int DIFF, int SCHEME, int PATH, bool INDEP>
static hipError_t launch_coop_one(const SweepArgs& a, const int16_t* label, const float* key, int* list, int tiles_x,
                                  int tiles_y, float* outbuf, float* tchange, uint8_t* flag, int max_inner,
                                  float tol_inner, float act, float window, float tol, int max_passes, CoopState* st,
                                  int max_grid, int* grid_used, int pe, hipStream_t s) {
  auto kern = tile_solve_coop_kernel<TW, TH, SPL, DIFF, SCHEME, PATH, INDEP>;
  const TileShape sh{TW, TH, SPL, SPL == 1 ? kThreads : TW * TH * SPL};
  const size_t lds = tile_pass_lds_bytes(sh, a.halo, INDEP);
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, sh.threads, lds);
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
                  &tchange, &flag, &max_inner, &tol_inner, &act, &window, &tol, &max_passes, &st, &pe};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(sh.threads), args, (unsigned)lds, s);
}

template <int TW, int TH, int SPL>
static hipError_t launch_coop_shape(const SweepArgs& a, int diffusion, int scheme, int path, bool indep,
                                    const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                    float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                    float act, float window, float tol, int max_passes, CoopState* st, int max_grid,
                                    int* grid_used, int pe, hipStream_t s) {
#define SLHJB_CO(D, S, PA, IN)                                                                                        \
  return launch_coop_one<TW, TH, SPL, D, S, PA, IN>(a, label, key, list, tiles_x, tiles_y, outbuf, tchange, flag,     \
                                                    max_inner, tol_inner, act, window, tol, max_passes, st, max_grid, \
                                                    grid_used, pe, s)
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
  if (path == 2) return hipErrorNotSupported;  // checked by the caller
  if (diffusion == kDiffNone) SLHJB_CO_I(kDiffNone, 0);
  if (diffusion == kDiffIso) SLHJB_CO_I(kDiffIso, 0);
  SLHJB_CO_I(kDiffRank1, 0);
#undef SLHJB_CO_I
#undef SLHJB_CO_S
#undef SLHJB_CO
}

#define SLHJB_FOR_SHAPE(shape, CALL) \
  switch (shape) {                   \
    case 0: CALL(32, 16, 1);         \
    case 1: CALL(16, 16, 1);         \
    case 2: CALL(8, 8, 4);           \
    case 3: CALL(16, 16, 4);         \
    default: CALL(16, 16, 2);        \
  }

hipError_t launch_tile_solve_coop(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                                  const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                  float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                  float act, float window, float tol, int max_passes, void* state, int max_grid,
                                  int* grid_used, int pe, hipStream_t s) {
  CoopState* st = (CoopState*)state;
#define SLHJB_COOP_CALL(TW, TH, SPL)                                                                                  \
  return launch_coop_shape<TW, TH, SPL>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, outbuf, \
                                        tchange, flag, max_inner, tol_inner, act, window, tol, max_passes, st,       \
                                        max_grid, grid_used, pe, s)
  SLHJB_FOR_SHAPE(shape, SLHJB_COOP_CALL)
#undef SLHJB_COOP_CALL
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
  st->pe_updates = 0ull;
}

hipError_t launch_coop_state_init(void* state, hipStream_t s) {
  coop_state_init_kernel<<<1, 1, 0, s>>>((CoopState*)state);
  return hipGetLastError();
}


// ---- device-driven passes for graph capture ---------------------------------------------------
// A pass is two launches with fixed arguments (parity q alternates between passes), so a batch
// of passes can be captured once into a graph and replayed: select -> visit. The visits write
// their tiles directly (TileDirect) and flag the next pass's tiles themselves. The band bound, the
// "nothing selected" jump, the check sweep when nothing is flagged and the final decision all
// happen on the device; the host only reads `done` between replays.
//
// Who writes which word, so that no launch reads a word another workgroup of it writes:
//   select p: done and resid (when pass p - 1 was a check sweep that met tol), seq (+1), its own
//             count/nflag/kmin[q] (accumulated), the flags of the tiles it takes (cleared);
//   visit p:  count/nflag/kmin/racc[q ^ 1] (reset for pass p + 1), passes, checks, checked,
//             bound (band move), racc[q] (check sweep: one atomic max per workgroup).
struct TileCtl {
  unsigned count[2];   // selected tiles of the pass with parity q
  unsigned nflag[2];   // flagged tiles seen by that selection
  unsigned kmin[2];    // bits of their smallest key
  unsigned bound;      // bits of the band bound B (-inf at start)
  unsigned resid;      // bits of the residual of the check sweep that ended the solve
  unsigned checked;    // 1 if the last pass was a check sweep
  unsigned done;       // 1 once a check sweep met tol
  unsigned passes;     // passes that did work (check sweeps included)
  unsigned checks;     // check sweeps among them
  unsigned long long updates;
  unsigned long long pe_updates;  // policy-evaluation node updates
  unsigned seq;        // number of the current pass (from 1), stamped into the tile words
  unsigned racc[2];    // bits of the largest move of a check sweep with parity q
  unsigned pad;
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
  c->checks = 0u;
  c->updates = 0ull;
  c->pe_updates = 0ull;
  c->seq = 0u;
  c->racc[0] = c->racc[1] = 0u;
  c->pad = 0u;
}

// The outcome of the last pass (checked, racc) is written by the visit launches only, so every
// thread of this launch reads the same values and a workgroup takes one branch as a whole.
__global__ __launch_bounds__(kSelectThreads) void tilectl_select_kernel(uint8_t* __restrict__ flag,
                                                                        const float* __restrict__ key, int tiles,
                                                                        float tol, int q, int* __restrict__ list,
                                                                        TileCtl* __restrict__ c) {
  // the tile's flag and key do not depend on the pass words: all their loads go out together
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int tt = t < tiles ? t : tiles - 1;
  unsigned done = c->done, checked = c->checked, resid = c->racc[q ^ 1], bound = c->bound;
  unsigned fb = flag[tt];
  float kt = key ? key[tt] : INFINITY;
  SLHJB_ISSUE_TOGETHER("+s"(done), "+s"(checked), "+s"(resid), "+s"(bound), "+v"(fb), "+v"(kt));
  if (done) return;
  if (checked && __uint_as_float(resid) <= tol) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->resid = resid;
      c->done = 1u;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) c->seq += 1u;
  const bool fl = t < tiles && fb != 0u;
  const float B = key ? __uint_as_float(bound) : INFINITY;
  const float k = fl ? kt : INFINITY;
  const bool on = fl && (!key || k <= B);
  block_select(t, fl, on, k, key != nullptr, &c->count[q], &c->nflag[q], &c->kmin[q], list);
  if (on) flag[t] = 0;  // the visit may flag it again
}

// Three workgroups per CU (the grid the drivers launch) need 3 NT / 256 waves per SIMD: for the
// 512-thread visits at most 80 VGPRs, which the general path's direct write-back exceeds unless
// asked (86: two workgroups per CU, the eps > 0 solves 8% slower; asked, 4 VGPRs spill and they
// are 2-3% faster than with the staged write-back). The independent mode's general visits need
// 100-235 VGPRs and would spill heavily: they keep the compiler's own allocation.
template <int NT, bool INDEP = false>
constexpr int kVisitWavesPerEU = NT == 512 && !INDEP ? 6 : 1;

template <int TW, int TH, int SPL, int DIFF, int SCHEME, int PATH, bool INDEP,
          int NT = (SPL == 1 ? kThreads : TW * TH * SPL)>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kVisitWavesPerEU<NT, INDEP>))) void tilectl_visit_kernel(
    SweepArgs a, const float* __restrict__ speed, const uint8_t* __restrict__ cls, const float4* __restrict__ ctrl,
    const int16_t* __restrict__ label, const int* __restrict__ list, int tiles_x, int tiles, TileDirect D,
    uint8_t* __restrict__ flag, int max_inner, float tol_inner, float act, float window, int q,
    TileCtl* __restrict__ c, int pe, unsigned long long* __restrict__ wg_acc) {
  // The first slot's tile is read with the pass words, so that the loads overlap: the grid has at
  // most `tiles` workgroups and the list `tiles` entries, and the value is used only if the slot
  // is taken.
  // The workgroup's update counters (wg_acc[2 b], wg_acc[2 b + 1], touched only by workgroup b of
  // each launch) are read here too and written once at the end.
  unsigned done = c->done, ucnt = c->count[q], unf = c->nflag[q], seq = c->seq;
  int first = list[blockIdx.x];
  unsigned long long acc0 = wg_acc[2 * blockIdx.x], pe_acc0 = wg_acc[2 * blockIdx.x + 1];
  SLHJB_ISSUE_TOGETHER("+s"(done), "+s"(ucnt), "+s"(unf), "+s"(seq), "+s"(first), "+s"(acc0), "+s"(pe_acc0));
  if (done) return;
  extern __shared__ float lds[];
  __shared__ float red[NT / 64];
  unsigned long long acc = 0ull, pe_acc = 0ull;
  float tmax = 0.0f;  // thread 0: largest move of this workgroup's tiles (the check sweep's residual)
  const int cnt = (int)ucnt;
  const int nf = (int)unf;
  const bool check = cnt == 0 && nf == 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the other parity's words serve the next pass; the previous pass's launches have read them
    c->count[q ^ 1] = 0u;
    c->nflag[q ^ 1] = 0u;
    c->kmin[q ^ 1] = 0x7f800000u;
    c->racc[q ^ 1] = 0u;
    if (cnt > 0 || check) c->passes += 1u;
    if (check) c->checks += 1u;
    c->checked = check ? 1u : 0u;
  }
  if (cnt > 0) {
    for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x)
      visit_tile<TW, TH, SPL, DIFF, SCHEME, PATH, INDEP, true>(
          a, nullptr, speed, cls, ctrl, label, slot, slot == (int)blockIdx.x ? first : list[slot], tiles_x, nullptr,
          nullptr, flag, max_inner, tol_inner, act, nullptr, acc, lds, red, pe, pe_acc, D, seq, &tmax);
  } else if (nf > 0) {
    // flagged tiles exist but none is in the band: move the band up to the smallest flagged key
    if (blockIdx.x == 0 && threadIdx.x == 0) c->bound = __float_as_uint(__uint_as_float(c->kmin[q]) + window);
  } else {
    // nothing flagged: check sweep, one Jacobi iteration of every tile
    for (int t = blockIdx.x; t < tiles; t += gridDim.x)
      visit_tile<TW, TH, SPL, DIFF, SCHEME, PATH, INDEP, true>(a, nullptr, speed, cls, ctrl, label, t, t, tiles_x,
                                                               nullptr, nullptr, flag, 1, 0.0f, act, nullptr, acc, lds,
                                                               red, 0, pe_acc, D, seq, &tmax);
    if (threadIdx.x == 0 && tmax > 0.0f) atomicMax(&c->racc[q], __float_as_uint(tmax));  // one per workgroup
  }
  if (threadIdx.x == 0 && (acc | pe_acc) != 0ull) {
    wg_acc[2 * blockIdx.x] = acc0 + acc;
    wg_acc[2 * blockIdx.x + 1] = pe_acc0 + pe_acc;
  }
}

// The update counters of the visit workgroups into the pass state (one workgroup).
__global__ __launch_bounds__(256) void tilectl_sum_kernel(const unsigned long long* __restrict__ wg_acc, int groups,
                                                          TileCtl* __restrict__ c) {
  __shared__ unsigned long long s[2][256];
  unsigned long long u = 0ull, p = 0ull;
  for (int b = threadIdx.x; b < groups; b += 256) {
    u += wg_acc[2 * b];
    p += wg_acc[2 * b + 1];
  }
  s[0][threadIdx.x] = u;
  s[1][threadIdx.x] = p;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s[0][threadIdx.x] += s[0][threadIdx.x + h];
      s[1][threadIdx.x] += s[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    c->updates = s[0][0];
    c->pe_updates = s[1][0];
  }
}

static_assert(offsetof(TileCtl, resid) == 7 * 4 && offsetof(TileCtl, done) == 9 * 4 &&
                  offsetof(TileCtl, passes) == 10 * 4 && offsetof(TileCtl, checks) == 11 * 4 &&
                  offsetof(TileCtl, checked) == 8 * 4 && offsetof(TileCtl, updates) == 12 * 4 &&
                  offsetof(TileCtl, pe_updates) == 14 * 4 && sizeof(TileCtl) <= kTileCtlHostBytes,
              "host reads these words");
size_t tilectl_bytes() { return sizeof(TileCtl); }

hipError_t launch_tilectl_sum(const unsigned long long* wg_acc, int groups, void* ctl, hipStream_t s) {
  tilectl_sum_kernel<<<1, 256, 0, s>>>(wg_acc, groups, (TileCtl*)ctl);
  return hipGetLastError();
}

hipError_t launch_tilectl_init(void* ctl, hipStream_t s) {
  tilectl_init_kernel<<<1, 1, 0, s>>>((TileCtl*)ctl);
  return hipGetLastError();
}

template <int TW, int TH, int SPL>
static void launch_tilectl_pass_shape(const SweepArgs& a, int diffusion, int scheme, int path, bool indep,
                                      const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                      const TileDirect& D, uint8_t* flag, int max_inner, float tol_inner, float act,
                                      float window, float tol, int q, TileCtl* c, int grid, hipEvent_t ev_before,
                                      hipEvent_t ev_after, int pe, unsigned long long* wg_acc, hipStream_t s) {
  const int tiles = tiles_x * tiles_y;
  tilectl_select_kernel<<<(tiles + kSelectThreads - 1) / kSelectThreads, kSelectThreads, 0, s>>>(flag, key, tiles,
                                                                                             tol, q, list, c);
  const TileShape sh{TW, TH, SPL, SPL == 1 ? kThreads : TW * TH * SPL};
  const size_t lds = tile_pass_lds_bytes(sh, a.halo, indep);
  // With events the visit goes through hipExtLaunchKernel, which stamps them at the kernel's own
  // start and end (as a profiler measures it), not around the launch on the stream.
#define SLHJB_TV(D_, S, PA, IN)                                                                                  \
  do {                                                                                                           \
    if (ev_before)                                                                                               \
      hipExtLaunchKernelGGL((tilectl_visit_kernel<TW, TH, SPL, D_, S, PA, IN>), dim3(grid), dim3(sh.threads),    \
                            (std::uint32_t)lds, s, ev_before, ev_after, 0u, a, a.speed, a.cls, a.ctrl, label,    \
                            (const int*)list, tiles_x, tiles, D, flag, max_inner, tol_inner, act, window, q, c,  \
                            pe, wg_acc);                                                                         \
    else                                                                                                         \
      tilectl_visit_kernel<TW, TH, SPL, D_, S, PA, IN><<<grid, sh.threads, lds, s>>>(                            \
          a, a.speed, a.cls, a.ctrl, label, list, tiles_x, tiles, D, flag, max_inner, tol_inner, act, window, q, \
          c, pe, wg_acc);                                                                                        \
  } while (0)
#define SLHJB_TV_S(D_, PA, IN)                      \
  do {                                              \
    if (scheme == kSL2) SLHJB_TV(D_, kSL2, PA, IN); \
    else SLHJB_TV(D_, kSL3, PA, IN);                \
  } while (0)
#define SLHJB_TV_I(D_, PA)               \
  do {                                   \
    if (indep) SLHJB_TV_S(D_, PA, true); \
    else SLHJB_TV_S(D_, PA, false);      \
  } while (0)
  if (path == 1) SLHJB_TV_I(kDiffNone, 1);
  else if (path == 2) {
    // varying costs / no discount / diffusion field: transmission mode only (checked by the caller)
    if (diffusion == kDiffNone) SLHJB_TV_S(kDiffNone, 2, false);
    else if (diffusion == kDiffIso) SLHJB_TV_S(kDiffIso, 2, false);
    else SLHJB_TV_S(kDiffRank1, 2, false);
  } else if (diffusion == kDiffNone) SLHJB_TV_I(kDiffNone, 0);
  else if (diffusion == kDiffIso) SLHJB_TV_I(kDiffIso, 0);
  else SLHJB_TV_I(kDiffRank1, 0);
#undef SLHJB_TV_I
#undef SLHJB_TV_S
#undef SLHJB_TV
}

hipError_t launch_tilectl_pass(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                               const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                               float* w2, unsigned* tile_word, uint8_t* flag, int max_inner, float tol_inner,
                               float act, float window, float tol, int q, void* ctl, int grid, hipEvent_t ev_before,
                               hipEvent_t ev_after, int pe, unsigned long long* wg_acc, hipStream_t s) {
  // the visit launch reads list[blockIdx.x] unconditionally
  if (grid < 1 || grid > tiles_x * tiles_y) return hipErrorInvalidValue;
  const TileDirect D{const_cast<float*>(a.w_in), w2, tile_word, tiles_y};
#define SLHJB_CTL_CALL(TW, TH, SPL)                                                                                  \
  launch_tilectl_pass_shape<TW, TH, SPL>(a, diffusion, scheme, path, indep, label, key, list, tiles_x, tiles_y, D,   \
                                         flag, max_inner, tol_inner, act, window, tol, q, (TileCtl*)ctl, grid,       \
                                         ev_before, ev_after, pe, wg_acc, s);                                        \
  break
  SLHJB_FOR_SHAPE(shape, SLHJB_CTL_CALL)
#undef SLHJB_CTL_CALL
  return hipGetLastError();
}

// After the passes: the tiles whose current values are in the second array are copied back.
__global__ __launch_bounds__(kThreads) void tile_gather_kernel(float* __restrict__ w, const float* __restrict__ w2,
                                                               const unsigned* __restrict__ tile_word, int n, int tw,
                                                               int th, int tiles_x) {
  const int64_t N = (int64_t)n * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N; i += (int64_t)gridDim.x * kThreads) {
    const int gy = (int)(i / n), gx = (int)(i - (int64_t)gy * n);
    if (tile_word[(gy / th) * tiles_x + gx / tw] & 1u) w[i] = w2[i];
  }
}

hipError_t launch_tile_gather(float* w, const float* w2, const unsigned* tile_word, int n, int shape, hipStream_t s) {
  const TileShape sh = tile_shape_of(shape);
  const int64_t N = (int64_t)n * n;
  const int blocks = (int)std::min<int64_t>((N + kThreads - 1) / kThreads, 4096);
  tile_gather_kernel<<<std::max(blocks, 1), kThreads, 0, s>>>(w, w2, tile_word, n, sh.tw, sh.th,
                                                              (n + sh.tw - 1) / sh.tw);
  return hipGetLastError();
}

// ---- the active-tile solver over a batch of independent instances ---------------------------
// Every instance runs exactly its own sequence of passes (selection in its band, visits, band
// moves and check sweeps, decided from its own pass words), so its result is that of the
// single-instance solve; the passes of all instances still iterating share three launches:
//   select  one workgroup per (instance, 1024 tiles): flagged tiles in the instance's band join
//           one combined work list (per-instance counts, smallest key and flagged count kept);
//           their flags are cleared;
//   plan    one workgroup: per instance the decision the single-instance visit launch takes
//           (visits, band move, check sweep, stop) and its pass bookkeeping, the offsets of the
//           check sweeps' tiles after the selected ones, and the pass number;
//   visit   the items of the pass: the selected tiles, then every tile of each instance that
//           makes a check sweep (one iteration); each writes its tile directly (TileDirect: the
//           instance's w and its second array, one word per tile), flags its neighbours and, in
//           a check sweep, raises the instance's residual.
// Global tile g belongs to instance tile_inst[g] as its tile g - tile0; flags, keys, the list and
// the tile words are indexed by g.
struct TBInst {
  SweepArgs a;       // w_in: the instance's iterate w; ctrl: its padded control table
  float* w2;         // the instance's second array (n * n)
  unsigned* word;    // its tile words (tiles)
  const float* key;  // [tiles] (u_hat order) or NULL
  int tiles_x, tiles_y, tiles, tile0;
  int max_inner, pe;
  float tol_inner, act, window, tol;
  long long max_passes;
};
struct TBState {
  unsigned count[2], nflag[2], kmin[2];  // of the selection with parity q
  unsigned bound, resid, checked, done, passes, checks;
  unsigned mode;  // this pass: 0 nothing, 1 visits of the selected tiles, 2 check sweep
  unsigned stop;  // 1 once done or out of passes
  unsigned long long updates, pe_updates;
};
struct TBCtl {
  unsigned count[2];  // combined list length of the pass with parity q
  unsigned checks;    // tiles of this pass's check sweeps (after the selected ones)
  unsigned nchk;      // instances making a check sweep this pass
  unsigned active;    // instances still iterating after this pass's decisions
  unsigned seq;       // number of the current pass (from 1), stamped into the tile words
  unsigned pad[2];
};

__global__ void tb_init_kernel(TBState* st, int count, TBCtl* ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctl->count[0] = ctl->count[1] = 0u;
    ctl->checks = ctl->nchk = 0u;
    ctl->active = (unsigned)count;
    ctl->seq = 0u;
  }
  if (i >= count) return;
  TBState& s = st[i];
  s.count[0] = s.count[1] = 0u;
  s.nflag[0] = s.nflag[1] = 0u;
  s.kmin[0] = s.kmin[1] = 0x7f800000u;
  s.bound = 0xff800000u;
  s.resid = 0u;
  s.checked = 0u;
  s.done = 0u;
  s.passes = 0u;
  s.checks = 0u;
  s.mode = 0u;
  s.stop = 0u;
  s.updates = 0ull;
  s.pe_updates = 0ull;
}

__global__ __launch_bounds__(kSelectThreads) void tb_select_kernel(const TBInst* __restrict__ inst,
                                                                   TBState* __restrict__ st,
                                                                   uint8_t* __restrict__ flag, int q,
                                                                   int* __restrict__ list, TBCtl* __restrict__ ctl) {
  constexpr int W = kSelectThreads / 64;
  __shared__ unsigned s_on[W], s_fl[W];
  __shared__ float s_k[W];
  __shared__ unsigned s_base;
  const int i = blockIdx.y;
  const int tiles = inst[i].tiles, tile0 = inst[i].tile0;
  const float* key = inst[i].key;
  TBState& s = st[i];
  if ((int)(blockIdx.x * kSelectThreads) >= tiles) return;
  const unsigned stop = s.stop, checked = s.checked, resid = s.resid, bound = s.bound;
  if (stop || (long long)s.passes >= inst[i].max_passes) return;
  if (checked && __uint_as_float(resid) <= inst[i].tol) return;  // the plan launch ends it
  const int t = blockIdx.x * kSelectThreads + threadIdx.x;
  const bool fl = t < tiles && flag[tile0 + t] != 0u;
  const float B = key ? __uint_as_float(bound) : INFINITY;
  float k = fl && key ? key[t] : INFINITY;
  const bool on = fl && (!key || k <= B);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long fmask = __ballot(fl), mask = __ballot(on);
  if (key) {
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
    for (int w = 0; w < W; ++w) {
      const unsigned c = s_on[w];
      s_on[w] = total;
      total += c;
      nf += s_fl[w];
      km = fminf(km, s_k[w]);
    }
    if (nf) atomicAdd(&s.nflag[q], nf);
    if (key && km < INFINITY) atomicMin(&s.kmin[q], __float_as_uint(km));
    if (total) atomicAdd(&s.count[q], total);
    s_base = total ? atomicAdd(&ctl->count[q], total) : 0u;
  }
  __syncthreads();
  if (on) {
    list[s_base + s_on[wave] + (unsigned)__popcll(mask & ((1ull << lane) - 1ull))] = tile0 + t;
    flag[tile0 + t] = 0;  // the visit may flag it again
  }
}

// One workgroup of 1024 threads; instance i is handled by thread i % 1024 (in order of i).
__global__ __launch_bounds__(1024) void tb_plan_kernel(const TBInst* __restrict__ inst, TBState* __restrict__ st,
                                                       int count, int q, int* __restrict__ chk_inst,
                                                       unsigned* __restrict__ chk_off, TBCtl* __restrict__ ctl) {
  __shared__ unsigned s_sum[1024];
  __shared__ unsigned s_n[1024];
  constexpr int PER = 4;  // instances per thread (count <= 4096)
  unsigned my_tiles = 0u, my_n = 0u, my_active = 0u;
  for (int r = 0; r < PER; ++r) {
    const int i = threadIdx.x * PER + r;
    if (i >= count) break;
    TBState& s = st[i];
    const TBInst& I = inst[i];
    unsigned mode = 0u;
    if (!s.stop) {
      if (s.checked && __uint_as_float(s.resid) <= I.tol) {
        s.done = 1u;
        s.stop = 1u;
      } else if ((long long)s.passes >= I.max_passes) {
        s.stop = 1u;
      } else {
        const unsigned cnt = s.count[q], nf = s.nflag[q];
        if (cnt > 0u) {
          mode = 1u;
        } else if (nf > 0u) {
          s.bound = __float_as_uint(__uint_as_float(s.kmin[q]) + I.window);  // move the band
        } else {
          mode = 2u;  // check sweep: its visits raise resid
          s.resid = 0u;
          my_tiles += (unsigned)I.tiles;
          my_n += 1u;
        }
        if (cnt > 0u || nf == 0u) s.passes += 1u;
        if (cnt == 0u && nf == 0u) s.checks += 1u;
        s.checked = (cnt == 0u && nf == 0u) ? 1u : 0u;
      }
    }
    s.mode = mode;
    s.count[q ^ 1] = 0u;
    s.nflag[q ^ 1] = 0u;
    s.kmin[q ^ 1] = 0x7f800000u;
    my_active += s.stop ? 0u : 1u;
  }
  // exclusive prefix of the check sweeps' tiles and instances over the threads, in order of i
  s_sum[threadIdx.x] = my_tiles;
  s_n[threadIdx.x] = my_n;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned a = threadIdx.x >= (unsigned)off ? s_sum[threadIdx.x - off] : 0u;
    const unsigned b = threadIdx.x >= (unsigned)off ? s_n[threadIdx.x - off] : 0u;
    __syncthreads();
    s_sum[threadIdx.x] += a;
    s_n[threadIdx.x] += b;
    __syncthreads();
  }
  if (threadIdx.x == 1023) {
    ctl->checks = s_sum[1023];
    ctl->nchk = s_n[1023];
  }
  unsigned off_t = s_sum[threadIdx.x] - my_tiles, off_n = s_n[threadIdx.x] - my_n;
  for (int r = 0; r < PER; ++r) {
    const int i = threadIdx.x * PER + r;
    if (i >= count) break;
    if (st[i].mode == 2u) {
      chk_inst[off_n] = i;
      chk_off[off_n] = off_t;
      off_t += (unsigned)inst[i].tiles;
      off_n += 1u;
    }
  }
  // the active count: a block sum
  __syncthreads();
  s_n[threadIdx.x] = my_active;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (threadIdx.x < (unsigned)h) s_n[threadIdx.x] += s_n[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctl->active = s_n[0];
    ctl->count[q ^ 1] = 0u;
    ctl->seq += 1u;
  }
}

// item j of the pass -> instance, its tile, and whether the item is a check-sweep tile
__device__ __forceinline__ void tb_item(int j, int cnt, const int* __restrict__ list, const int* __restrict__ tile_inst,
                                        const TBInst* __restrict__ inst, const int* __restrict__ chk_inst,
                                        const unsigned* __restrict__ chk_off, int nchk, int& i, int& tid, bool& check) {
  if (j < cnt) {
    const int g = list[j];
    i = tile_inst[g];
    tid = g - inst[i].tile0;
    check = false;
  } else {
    const unsigned jj = (unsigned)(j - cnt);
    int lo = 0, hi = nchk - 1;  // last r with chk_off[r] <= jj
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (chk_off[mid] <= jj) lo = mid;
      else hi = mid - 1;
    }
    i = chk_inst[lo];
    tid = (int)(jj - chk_off[lo]);
    check = true;
  }
}

template <int TW, int TH, int SPL, int DIFF, int SCHEME, int PATH, int NT = (SPL == 1 ? kThreads : TW * TH * SPL)>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(kVisitWavesPerEU<NT>))) void tb_visit_kernel(const TBInst* __restrict__ inst, TBState* __restrict__ st,
                                                      const int* __restrict__ list,
                                                      const int* __restrict__ tile_inst,
                                                      const int* __restrict__ chk_inst,
                                                      const unsigned* __restrict__ chk_off, int q,
                                                      const TBCtl* __restrict__ ctl, uint8_t* __restrict__ flag) {
  const int cnt = (int)ctl->count[q];
  const int items = cnt + (int)ctl->checks;
  const int nchk = (int)ctl->nchk;
  const unsigned seq = ctl->seq;
  extern __shared__ float lds[];
  __shared__ float red[NT / 64];
  for (int j = blockIdx.x; j < items; j += gridDim.x) {
    int i, tid;
    bool check;
    tb_item(j, cnt, list, tile_inst, inst, chk_inst, chk_off, nchk, i, tid, check);
    i = __builtin_amdgcn_readfirstlane(i);
    tid = __builtin_amdgcn_readfirstlane(tid);
    const TBInst& I = inst[i];
    const SweepArgs a = I.a;
    const TileDirect D{const_cast<float*>(a.w_in), I.w2, I.word, I.tiles_y};
    unsigned long long acc = 0ull, pe_acc = 0ull;
    float tmax = 0.0f;
    visit_tile<TW, TH, SPL, DIFF, SCHEME, PATH, false, true>(
        a, nullptr, a.speed, a.cls, a.ctrl, nullptr, j, tid, I.tiles_x, nullptr, nullptr, flag + I.tile0,
        check ? 1 : I.max_inner, check ? 0.0f : I.tol_inner, I.act, nullptr, acc, lds, red, check ? 0 : I.pe, pe_acc,
        D, seq, &tmax);
    if (threadIdx.x == 0) {
      if (acc) atomicAdd(&st[i].updates, acc);
      if (pe_acc) atomicAdd(&st[i].pe_updates, pe_acc);
      if (check && tmax > 0.0f) atomicMax(&st[i].resid, __float_as_uint(tmax));
    }
  }
}

size_t tb_inst_bytes() { return sizeof(TBInst); }
size_t tb_state_bytes() { return sizeof(TBState); }
size_t tb_ctl_bytes() { return sizeof(TBCtl); }

void tb_fill_inst(void* dst, const SweepArgs& a, float* w2, unsigned* word, const float* key, int tiles_x,
                  int tiles_y, int tile0, int max_inner, int pe, float tol_inner, float act, float window, float tol,
                  long long max_passes) {
  TBInst I;
  memset(&I, 0, sizeof(I));
  I.a = a;
  I.w2 = w2;
  I.word = word;
  I.key = key;
  I.tiles_x = tiles_x;
  I.tiles_y = tiles_y;
  I.tiles = tiles_x * tiles_y;
  I.tile0 = tile0;
  I.max_inner = max_inner;
  I.pe = pe;
  I.tol_inner = tol_inner;
  I.act = act;
  I.window = window;
  I.tol = tol;
  I.max_passes = max_passes;
  memcpy(dst, &I, sizeof(I));
}

void tb_read_state(const void* src, int i, TBResult* out) {
  TBState s;
  memcpy(&s, static_cast<const char*>(src) + (size_t)i * sizeof(TBState), sizeof(s));
  out->done = s.done;
  out->passes = s.passes;
  out->checks = s.checks;
  memcpy(&out->resid, &s.resid, sizeof(float));
  out->updates = s.updates;
  out->pe_updates = s.pe_updates;
}

hipError_t launch_tb_init(void* st, int count, void* ctl, hipStream_t s) {
  tb_init_kernel<<<(count + 255) / 256, 256, 0, s>>>((TBState*)st, count, (TBCtl*)ctl);
  return hipGetLastError();
}

template <int TW, int TH, int SPL>
static hipError_t launch_tb_pass_shape(const void* inst, void* st, int count, int max_chunks, uint8_t* flag, int* list,
                                       const int* tile_inst, int* chk_inst, unsigned* chk_off, void* ctl,
                                       int diffusion, int scheme, int path, int q, int grid, size_t lds,
                                       hipStream_t s) {
  const TBInst* I = (const TBInst*)inst;
  TBState* S = (TBState*)st;
  TBCtl* C = (TBCtl*)ctl;
  static_assert(offsetof(TBCtl, active) == kTBCtlActive * 4, "host reads this word");
  tb_select_kernel<<<dim3(max_chunks, count), kSelectThreads, 0, s>>>(I, S, flag, q, list, C);
  tb_plan_kernel<<<1, 1024, 0, s>>>(I, S, count, q, chk_inst, chk_off, C);
  constexpr int NT = SPL == 1 ? kThreads : TW * TH * SPL;
#define SLHJB_TBV(D, SC, PA)                                                                                   \
  tb_visit_kernel<TW, TH, SPL, D, SC, PA><<<grid, NT, lds, s>>>(I, S, list, tile_inst, chk_inst, chk_off, q, C, flag)
#define SLHJB_TBV_S(D, PA)             \
  do {                                 \
    if (scheme == kSL2) SLHJB_TBV(D, kSL2, PA); \
    else SLHJB_TBV(D, kSL3, PA);       \
  } while (0)
  if (path == 1) SLHJB_TBV_S(kDiffNone, 1);
  else if (path != 0) return hipErrorInvalidValue;
  else if (diffusion == kDiffNone) SLHJB_TBV_S(kDiffNone, 0);
  else if (diffusion == kDiffIso) SLHJB_TBV_S(kDiffIso, 0);
  else SLHJB_TBV_S(kDiffRank1, 0);
#undef SLHJB_TBV_S
#undef SLHJB_TBV
  return hipGetLastError();
}

hipError_t launch_tb_pass(int shape, const void* inst, void* st, int count, int max_chunks, uint8_t* flag, int* list,
                          const int* tile_inst, int* chk_inst, unsigned* chk_off, void* ctl, int diffusion, int scheme,
                          int path, int q, int grid, size_t lds, hipStream_t s) {
  if (count < 1 || count > 4096 || grid < 1 || max_chunks < 1) return hipErrorInvalidValue;
#define SLHJB_TB_CALL(TW, TH, SPL)                                                                                \
  return launch_tb_pass_shape<TW, TH, SPL>(inst, st, count, max_chunks, flag, list, tile_inst, chk_inst, chk_off, \
                                           ctl, diffusion, scheme, path, q, grid, lds, s)
  SLHJB_FOR_SHAPE(shape, SLHJB_TB_CALL)
#undef SLHJB_TB_CALL
}

}  // namespace slhjb
