// Device-side building blocks of the sweep: the feet of a control, the Bellman update of a node
// from an LDS tile (any reach), and the first-ring update (sigma = 0, feet inside the cells
// around the node). Shared by the Jacobi sweep kernels and the active-tile solver.
#pragma once

#include "internal.h"

namespace slhjb {

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ void block_reduce_and_publish(float local, bool bad, unsigned* __restrict__ resid,
                                                         unsigned* __restrict__ flags) {
  __shared__ float red[kThreads / 64];
  __shared__ int anybad;
  if (threadIdx.x == 0) anybad = 0;
  __syncthreads();
  if (resid) {
    const float wm = wave_max(local);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = wm;
  }
  if (bad) anybad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (resid) {
      float m = red[0];
#pragma unroll
      for (int k = 1; k < kThreads / 64; ++k) m = fmaxf(m, red[k]);
      // residuals are >= 0, so the float order equals the unsigned order of the bits
      atomicMax(resid, __float_as_uint(m));
    }
    if (anybad) atomicOr(flags, 1u);
  }
}

template <int DIFF>
struct Feet;
template <>
struct Feet<kDiffNone> {
  static constexpr int K = 1;
  __device__ static __forceinline__ void get(int, float bx, float by, float, float, float, float& fx, float& fy) {
    fx = bx;
    fy = by;
  }
};
template <>
struct Feet<kDiffIso> {
  static constexpr int K = 4;
  __device__ static __forceinline__ void get(int f, float bx, float by, float, float, float d, float& fx, float& fy) {
    fx = bx + (f == 0 ? d : (f == 1 ? -d : 0.0f));
    fy = by + (f == 2 ? d : (f == 3 ? -d : 0.0f));
  }
};
template <>
struct Feet<kDiffRank1> {
  static constexpr int K = 2;
  __device__ static __forceinline__ void get(int f, float bx, float by, float ax, float ay, float d, float& fx,
                                             float& fy) {
    const float s = f == 0 ? d : -d;
    fx = __builtin_fmaf(s, ax, bx);
    fy = __builtin_fmaf(s, ay, by);
  }
};

// Bellman update of one FREE node from the LDS tile (general kernel). Feet are handled as
// offsets from the node in cell units, so positions keep full precision on large grids.
// `node_li` is the node's index in the tile.
// With INDEP, a corner whose patch label (`lab`, same layout as `tile`) differs from the node's
// label `mylab` reads w_outside: every patch is solved as a domain of its own with state
// constraints at its interfaces.
// GEN: the problem has varying costs, no discount or a diffusion-coefficient field (kernel path
// 2); then qn is the node's part of the cost term (node_cost) and dn its noise offset in cells
// (node_noise). Without GEN the update is the homogeneous one with the constant offset a.d.
template <int DIFF, int SCHEME, bool INDEP = false, bool GEN = false>
__device__ __forceinline__ float general_update(const float* __restrict__ tile, int LW, int node_li, int i, int j,
                                                float k, float wself, const float4* __restrict__ ctrl,
                                                const SweepArgs& a, const int16_t* __restrict__ lab = nullptr,
                                                int mylab = 0, float qn = 0.0f, float dn = 0.0f) {
  using F = Feet<DIFF>;
  const float dd = GEN ? dn : a.d;
  (void)wself;  // SL3 leaves the node's own value out instead of subtracting it
  const float fi = (float)i, fj = (float)j;
  const float nm1 = (float)(a.n - 1);
  const float nm2 = (float)(a.n - 2);
  // offsets that stay inside the closed box, and the largest cell offset (cell n-2)
  const float lox = -fi, hix = nm1 - fi, loy = -fj, hiy = nm1 - fj;
  const float cmx = nm2 - fi, cmy = nm2 - fj;
  const float LWf = (float)LW;
  // drift part of the feet, the same for every control: k d(x) (0 without a drift, and then
  // fma(k, a, 0) is the product k a bit for bit)
  float kdx = 0.0f, kdy = 0.0f;
  if (a.drift) {
    const float2 dv = a.drift[(size_t)j * a.n + i];
    kdx = k * dv.x;
    kdy = k * dv.y;
  }
  // SL2: max over controls of the feet sum; SL3: best quotient num / den (den > 0). Without the
  // cost term every candidate is >= 0, and the start values 0 and -1 (inline constants) keep the
  // register count of the default kernels; with it candidates can be negative.
  float best2 = GEN ? -INFINITY : 0.0f;
  float bnum = GEN ? -INFINITY : -1.0f, bden = 1.0f;
  const float4* __restrict__ ctab = (const float4*)__builtin_assume_aligned(ctrl, 64);
  // the host pads the control list to a multiple of 4 with repeats of its last control
#pragma unroll 4
  for (int m = 0; m < a.n_controls; ++m) {
    const float4 cm = ctab[m];
    const float bx = __builtin_fmaf(k, cm.x, kdx);
    const float by = __builtin_fmaf(k, cm.y, kdy);
    float acc = 0.0f, lam0 = 0.0f;
#pragma unroll
    for (int f = 0; f < F::K; ++f) {
      float ox, oy;
      F::get(f, bx, by, cm.x, cm.y, dd, ox, oy);
      const bool inside = (ox >= lox) & (ox <= hix) & (oy >= loy) & (oy <= hiy);
      const float cx = fminf(fmaxf(ox, lox), hix);
      const float cy = fminf(fmaxf(oy, loy), hiy);
      const float flx = fminf(floorf(cx), cmx);
      const float fly = fminf(floorf(cy), cmy);
      const float s = cx - flx;
      const float t = cy - fly;
      const int li = node_li + (int)__builtin_fmaf(fly, LWf, flx);
      float v00 = tile[li], v10 = tile[li + 1];
      float v01 = tile[li + LW], v11 = tile[li + LW + 1];
      if (INDEP) {
        v00 = lab[li] == mylab ? v00 : a.w_outside;
        v10 = lab[li + 1] == mylab ? v10 : a.w_outside;
        v01 = lab[li + LW] == mylab ? v01 : a.w_outside;
        v11 = lab[li + LW + 1] == mylab ? v11 : a.w_outside;
      }
      if (SCHEME == kSL3) {
        // eq. SLscheme3 leaves the node's own value out of Lambda1: the corner that is the node
        // reads 0, so the update does not read the node at all, not even through rounding
        // (subtracting lam0 w_i afterwards would leave it there at the ulp level, and the FP32
        // iteration could then cycle instead of settling). The node is a corner only of the
        // four cells around it (|offset| < 1 on both axes); a wavefront in which no foot lies
        // there skips the test.
        if (__any((fabsf(cx) < 1.0f) & (fabsf(cy) < 1.0f))) {
          const int self = node_li - li;
          v00 = self == 0 ? 0.0f : v00;
          v10 = self == 1 ? 0.0f : v10;
          v01 = self == LW ? 0.0f : v01;
          v11 = self == LW + 1 ? 0.0f : v11;
        }
      }
      const float lo = __builtin_fmaf(s, v10 - v00, v00);
      const float hi = __builtin_fmaf(s, v11 - v01, v01);
      const float val = __builtin_fmaf(t, hi - lo, lo);
      acc += inside ? val : a.w_outside;
      if (SCHEME == kSL3) {
        const float hx = fmaxf(0.0f, 1.0f - fabsf(cx));
        const float hy = fmaxf(0.0f, 1.0f - fabsf(cy));
        lam0 += inside ? hx * hy : 0.0f;
      }
    }
    // the cost term (cm.w holds the control's part on the general path)
    if (GEN) acc -= qn + cm.w;
    if (SCHEME == kSL2) {
      best2 = fmaxf(best2, acc);
    } else {
      const float num = acc;  // the node's own weight is already out (see above)
      const float den = __builtin_fmaf(-a.beta, lam0, (float)F::K);
      if (num * bden > bnum * den) {
        bnum = num;
        bden = den;
      }
    }
  }
  if (SCHEME == kSL2) return a.beta * best2 * (1.0f / (float)F::K);
  return a.beta * bnum / bden;
}

// The value of a node under one control in FP64 from the FP32 iterate, rounded once to FP32: the
// bilinear weights of the foot's cell, s(1-t), (1-s)t, st and (1-s)(1-t) with s = k|a_x|,
// t = k|a_y|, beta and (SL3) the implicit denominator 1 - beta (1-s)(1-t) folded in. The split
// visits of the first-ring path choose the maximising control in FP32, then take its value from
// here, in the full iterations and in the policy evaluations alike (the same bits for the same
// control). Taking the maximum of 64 FP32-rounded candidates biases the value upward by about
// their rounding error, at every step along a characteristic; recomputing the winner removes that
// bias, which at 2049^2 had put the FP32 fixed point 1.6e-5 from the FP64 one.
struct PolicyEval64 {
  int ox, oy;              // LDS offsets of the east/west and north/south corners
  double gX, gY, gXY, g0;  // weights of the corners X, Y, XY and of the node itself (SL2)
  bool out;                // the foot leaves the box: beta w_outside
};
template <int SCHEME>
__device__ __forceinline__ PolicyEval64 policy_prepare64(int LW, float k, float4 cm, const SweepArgs& a, bool lft,
                                                         bool rgt, bool bot, bool top) {
  PolicyEval64 p;
  p.ox = cm.x >= 0.0f ? 1 : -1;
  p.oy = cm.y >= 0.0f ? LW : -LW;
  p.out = (lft & (cm.x < 0.0f)) | (rgt & (cm.x > 0.0f)) | (bot & (cm.y < 0.0f)) | (top & (cm.y > 0.0f));
  const double s = (double)k * fabs((double)cm.x), t = (double)k * fabs((double)cm.y);
  const double b = (double)a.beta;
  const double cX = s * (1.0 - t), cY = (1.0 - s) * t, cXY = s * t, c0 = (1.0 - s) * (1.0 - t);
  if (SCHEME == kSL3) {
    const double g = b / (1.0 - b * c0);
    p.gX = g * cX;
    p.gY = g * cY;
    p.gXY = g * cXY;
    p.g0 = 0.0;
  } else {
    p.gX = b * cX;
    p.gY = b * cY;
    p.gXY = b * cXY;
    p.g0 = b * c0;
  }
  return p;
}
template <int SCHEME, bool INDEP>
__device__ __forceinline__ float policy_apply64(const float* __restrict__ T, const PolicyEval64& p, const SweepArgs& a,
                                                const int16_t* __restrict__ L) {
  if (p.out) return (float)((double)a.beta * (double)a.w_outside);
  float wX = T[p.ox], wY = T[p.oy], wXY = T[p.ox + p.oy];
  if (INDEP) {
    const int me = L[0];
    wX = L[p.ox] == me ? wX : a.w_outside;
    wY = L[p.oy] == me ? wY : a.w_outside;
    wXY = L[p.ox + p.oy] == me ? wXY : a.w_outside;
  }
  double v = __builtin_fma(p.gXY, (double)wXY, __builtin_fma(p.gY, (double)wY, p.gX * (double)wX));
  if (SCHEME == kSL2) v = __builtin_fma(p.g0, (double)T[0], v);
  return (float)v;
}

// First-ring update of one node. T points at the node in the LDS tile. EDGE adds the test for
// feet that leave the box, which only happens on the outermost nodes.
template <int SCHEME, bool EDGE, bool INDEP = false>
__device__ __forceinline__ float ring1_update(const float* __restrict__ T, int LW, float k,
                                              const float4* __restrict__ ctrl, const SweepArgs& a, bool lft, bool rgt,
                                              bool bot, bool top, const int16_t* __restrict__ L = nullptr) {
  const float w00 = T[0];
  float wE = T[1], wW = T[-1], wN = T[LW], wS = T[-LW];
  float wNE = T[LW + 1], wNW = T[LW - 1], wSE = T[-LW + 1], wSW = T[-LW - 1];
  if (INDEP) {
    // neighbours of another patch read w_outside (state constraint at the interface)
    const int me = L[0];
    const float wo = a.w_outside;
    wE = L[1] == me ? wE : wo;
    wW = L[-1] == me ? wW : wo;
    wN = L[LW] == me ? wN : wo;
    wS = L[-LW] == me ? wS : wo;
    wNE = L[LW + 1] == me ? wNE : wo;
    wNW = L[LW - 1] == me ? wNW : wo;
    wSE = L[-LW + 1] == me ? wSE : wo;
    wSW = L[-LW - 1] == me ? wSW : wo;
  }
  const float k2 = k * k;
  // quadrant order: (+x,+y), (-x,+y), (-x,-y), (+x,-y)
  const float wX[4] = {wE, wW, wW, wE};
  const float wY[4] = {wN, wN, wS, wS};
  const float wXY[4] = {wNE, wNW, wSW, wSE};
  const float sx[4] = {1.0f, -1.0f, -1.0f, 1.0f};
  const float sy[4] = {1.0f, 1.0f, -1.0f, -1.0f};
  float best2 = -INFINITY;
  float bnum = -1.0f, bden = 1.0f;
  int bidx = 0;  // the maximiser, whose value is then taken in FP64
  // SL3 denominator 1 - beta (1 - k|a_x|)(1 - k|a_y|) = (1 - beta) + beta k (|a_x|+|a_y|) - beta k^2 |a_x a_y|
  const float omb = 1.0f - a.beta, bk = a.beta * k, bk2 = -(a.beta * k2);
  const float4* __restrict__ ctab = (const float4*)__builtin_assume_aligned(ctrl, 64);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float B, C, D;
    if (SCHEME == kSL2) {
      // I = w00 + a_x B + a_y C + a_x a_y D over the quadrant's cell
      B = k * sx[q] * (wX[q] - w00);
      C = k * sy[q] * (wY[q] - w00);
      D = k2 * (sx[q] * sy[q]) * ((wXY[q] - wX[q]) - (wY[q] - w00));
    } else {
      // I - (1-s)(1-t) w00 = a_x B + a_y C + a_x a_y D  (self weight removed)
      B = k * sx[q] * wX[q];
      C = k * sy[q] * wY[q];
      D = k2 * (sx[q] * sy[q]) * (wXY[q] - wX[q] - wY[q]);
    }
    // the host pads every quadrant's list to a multiple of 4 with repeats of its last control
    for (int m0 = a.quad[q]; m0 < a.quad[q + 1]; m0 += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 cm = ctab[m0 + u];
        float val = __builtin_fmaf(cm.z, D, __builtin_fmaf(cm.y, C, cm.x * B));
        bool out = false;
        if (EDGE) {
          out = (lft & (cm.x < 0.0f)) | (rgt & (cm.x > 0.0f)) | (bot & (cm.y < 0.0f)) | (top & (cm.y > 0.0f));
          // computed on every lane: otherwise the compiler moves the control's loads and the
          // arithmetic into a branch per control (one scalar-load wait per control)
          asm volatile("" : "+v"(val));
        }
        if (SCHEME == kSL2) {
          if (EDGE) val = out ? a.w_outside - w00 : val;
          if (val > best2) {
            best2 = val;
            bidx = m0 + u;
          }
        } else {
          float den = __builtin_fmaf(bk2, fabsf(cm.z), __builtin_fmaf(bk, cm.w, omb));
          if (EDGE) {
            asm volatile("" : "+v"(den));
            val = out ? a.w_outside : val;
            den = out ? 1.0f : den;
          }
          if (val * bden > bnum * den) {
            bnum = val;
            bden = den;
            bidx = m0 + u;
          }
        }
      }
    }
  }
  const PolicyEval64 p = policy_prepare64<SCHEME>(LW, k, ctab[bidx], a, lft, rgt, bot, top);
  return policy_apply64<SCHEME, INDEP>(T, p, a, L);
}


// ---- partial updates over a subset of the controls ---------------------------------------------
// The split-tile visits give each group of wavefronts one part of the control set for the same
// nodes; the partial results are combined through LDS. For the first-ring path a part is a range
// of whole quadrants [q_lo, q_hi), for the general path a contiguous slice of the (padded)
// control list, so every wavefront still walks a uniform control range with scalar loads.
// Partial of SL2 (first ring): max over the range of I - w00; of SL2 (general): max of the feet
// sum; of SL3: the best quotient as (num, den).
template <int SCHEME, bool EDGE, bool INDEP, bool TRACK = false>
__device__ __forceinline__ void ring1_partial(const float* __restrict__ T, int LW, float k,
                                              const float4* __restrict__ ctrl, const SweepArgs& a, bool lft, bool rgt,
                                              bool bot, bool top, const int16_t* __restrict__ L, int q_lo,
                                              int q_hi, float& pnum, float& pden, int* pidx = nullptr) {
  const float w00 = T[0];
  float wE = T[1], wW = T[-1], wN = T[LW], wS = T[-LW];
  float wNE = T[LW + 1], wNW = T[LW - 1], wSE = T[-LW + 1], wSW = T[-LW - 1];
  if (INDEP) {
    const int me = L[0];
    const float wo = a.w_outside;
    wE = L[1] == me ? wE : wo;
    wW = L[-1] == me ? wW : wo;
    wN = L[LW] == me ? wN : wo;
    wS = L[-LW] == me ? wS : wo;
    wNE = L[LW + 1] == me ? wNE : wo;
    wNW = L[LW - 1] == me ? wNW : wo;
    wSE = L[-LW + 1] == me ? wSE : wo;
    wSW = L[-LW - 1] == me ? wSW : wo;
  }
  const float k2 = k * k;
  const float wX[4] = {wE, wW, wW, wE};
  const float wY[4] = {wN, wN, wS, wS};
  const float wXY[4] = {wNE, wNW, wSW, wSE};
  const float sx[4] = {1.0f, -1.0f, -1.0f, 1.0f};
  const float sy[4] = {1.0f, 1.0f, -1.0f, -1.0f};
  float best2 = -INFINITY;
  float bnum = -1.0f, bden = 1.0f;
  int bidx = 0;
  const float omb = 1.0f - a.beta, bk = a.beta * k, bk2 = -(a.beta * k2);
  const float4* __restrict__ ctab = (const float4*)__builtin_assume_aligned(ctrl, 64);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < q_lo || q >= q_hi) continue;  // uniform across the wavefront
    float B, C, D;
    if (SCHEME == kSL2) {
      B = k * sx[q] * (wX[q] - w00);
      C = k * sy[q] * (wY[q] - w00);
      D = k2 * (sx[q] * sy[q]) * ((wXY[q] - wX[q]) - (wY[q] - w00));
    } else {
      B = k * sx[q] * wX[q];
      C = k * sy[q] * wY[q];
      D = k2 * (sx[q] * sy[q]) * (wXY[q] - wX[q] - wY[q]);
    }
    for (int m0 = a.quad[q]; m0 < a.quad[q + 1]; m0 += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 cm = ctab[m0 + u];
        float val = __builtin_fmaf(cm.z, D, __builtin_fmaf(cm.y, C, cm.x * B));
        bool out = false;
        if (EDGE) {
          out = (lft & (cm.x < 0.0f)) | (rgt & (cm.x > 0.0f)) | (bot & (cm.y < 0.0f)) | (top & (cm.y > 0.0f));
          // computed on every lane: otherwise the compiler moves the control's loads and the
          // arithmetic into a branch per control (one scalar-load wait per control)
          asm volatile("" : "+v"(val));
        }
        if (SCHEME == kSL2) {
          if (EDGE) val = out ? a.w_outside - w00 : val;
          if (TRACK) {
            if (val > best2) {
              best2 = val;
              bidx = m0 + u;
            }
          } else {
            best2 = fmaxf(best2, val);
          }
        } else {
          float den = __builtin_fmaf(bk2, fabsf(cm.z), __builtin_fmaf(bk, cm.w, omb));
          if (EDGE) {
            asm volatile("" : "+v"(den));
            val = out ? a.w_outside : val;
            den = out ? 1.0f : den;
          }
          if (val * bden > bnum * den) {
            bnum = val;
            bden = den;
            if (TRACK) bidx = m0 + u;
          }
        }
      }
    }
  }
  if (SCHEME == kSL2) {
    pnum = best2;
    pden = 1.0f;
  } else {
    pnum = bnum;
    pden = bden;
  }
  if (TRACK) *pidx = bidx;
}

// Policy evaluation on the first ring (modified policy iteration): the update of a node for one
// fixed control, with the quadrant taken from the signs of (a_x, a_y) as the host groups the
// table. Everything that does not depend on the iterate is computed once per node after each full
// iteration (policy_prepare64), and the full iteration takes the value of its maximiser from the
// same function (policy_apply64), so that a node whose control is still the maximiser gets bit for
// bit the value a full iteration would give it. (Otherwise the two maps would have fixed points a
// few ulp apart, and a tolerance near the FP32 resolution could never be met.)

template <int DIFF, int SCHEME, bool INDEP, bool TRACK = false, bool GEN = false>
__device__ __forceinline__ void general_partial(const float* __restrict__ tile, int LW, int node_li, int i, int j,
                                                float k, float wself, const float4* __restrict__ ctrl,
                                                const SweepArgs& a, const int16_t* __restrict__ lab, int mylab,
                                                int m_lo, int m_hi, float& pnum, float& pden, int* pidx = nullptr,
                                                const float2* kd_pre = nullptr, const float4* cm_pre = nullptr,
                                                float qn = 0.0f, float dn = 0.0f) {
  // kd_pre: the node's drift offset k d(x), computed by the caller as below (saves its load);
  // cm_pre: the one control m_lo, already loaded (policy evaluation: m_hi = m_lo + 1);
  // GEN, qn, dn: the cost term and the node's noise offset (see general_update)
  using F = Feet<DIFF>;
  const float dd = GEN ? dn : a.d;
  (void)wself;  // SL3 leaves the node's own value out instead of subtracting it
  const float fi = (float)i, fj = (float)j;
  const float nm1 = (float)(a.n - 1);
  const float nm2 = (float)(a.n - 2);
  const float lox = -fi, hix = nm1 - fi, loy = -fj, hiy = nm1 - fj;
  const float cmx = nm2 - fi, cmy = nm2 - fj;
  const float LWf = (float)LW;
  // drift part of the feet, the same for every control: k d(x) (0 without a drift, and then
  // fma(k, a, 0) is the product k a bit for bit)
  float kdx = 0.0f, kdy = 0.0f;
  if (kd_pre) {
    kdx = kd_pre->x;
    kdy = kd_pre->y;
  } else if (a.drift) {
    const float2 dv = a.drift[(size_t)j * a.n + i];
    kdx = k * dv.x;
    kdy = k * dv.y;
  }
  float best2 = -INFINITY;
  float bnum = GEN ? -INFINITY : -1.0f, bden = 1.0f;  // without the cost term candidates are >= 0
  int bidx = m_lo;
  const float4* __restrict__ ctab = (const float4*)__builtin_assume_aligned(ctrl, 64);
#pragma unroll 4
  for (int m = m_lo; m < m_hi; ++m) {
    const float4 cm = cm_pre ? *cm_pre : ctab[m];
    const float bx = __builtin_fmaf(k, cm.x, kdx);
    const float by = __builtin_fmaf(k, cm.y, kdy);
    float acc = 0.0f, lam0 = 0.0f;
#pragma unroll
    for (int f = 0; f < F::K; ++f) {
      float ox, oy;
      F::get(f, bx, by, cm.x, cm.y, dd, ox, oy);
      const bool inside = (ox >= lox) & (ox <= hix) & (oy >= loy) & (oy <= hiy);
      const float cx = fminf(fmaxf(ox, lox), hix);
      const float cy = fminf(fmaxf(oy, loy), hiy);
      const float flx = fminf(floorf(cx), cmx);
      const float fly = fminf(floorf(cy), cmy);
      const float s = cx - flx;
      const float t = cy - fly;
      const int li = node_li + (int)__builtin_fmaf(fly, LWf, flx);
      float v00 = tile[li], v10 = tile[li + 1];
      float v01 = tile[li + LW], v11 = tile[li + LW + 1];
      if (INDEP) {
        v00 = lab[li] == mylab ? v00 : a.w_outside;
        v10 = lab[li + 1] == mylab ? v10 : a.w_outside;
        v01 = lab[li + LW] == mylab ? v01 : a.w_outside;
        v11 = lab[li + LW + 1] == mylab ? v11 : a.w_outside;
      }
      if (SCHEME == kSL3) {
        // eq. SLscheme3 leaves the node's own value out of Lambda1: the corner that is the node
        // reads 0, so the update does not read the node at all, not even through rounding
        // (subtracting lam0 w_i afterwards would leave it there at the ulp level, and the FP32
        // iteration could then cycle instead of settling). The node is a corner only of the
        // four cells around it (|offset| < 1 on both axes); a wavefront in which no foot lies
        // there skips the test.
        if (__any((fabsf(cx) < 1.0f) & (fabsf(cy) < 1.0f))) {
          const int self = node_li - li;
          v00 = self == 0 ? 0.0f : v00;
          v10 = self == 1 ? 0.0f : v10;
          v01 = self == LW ? 0.0f : v01;
          v11 = self == LW + 1 ? 0.0f : v11;
        }
      }
      const float lo = __builtin_fmaf(s, v10 - v00, v00);
      const float hi = __builtin_fmaf(s, v11 - v01, v01);
      const float val = __builtin_fmaf(t, hi - lo, lo);
      acc += inside ? val : a.w_outside;
      if (SCHEME == kSL3) {
        const float hx = fmaxf(0.0f, 1.0f - fabsf(cx));
        const float hy = fmaxf(0.0f, 1.0f - fabsf(cy));
        lam0 += inside ? hx * hy : 0.0f;
      }
    }
    if (GEN) acc -= qn + cm.w;
    if (SCHEME == kSL2) {
      if (TRACK) {
        if (acc > best2) {
          best2 = acc;
          bidx = m;
        }
      } else {
        best2 = fmaxf(best2, acc);
      }
    } else {
      const float num = acc;  // the node's own weight is already out (see above)
      const float den = __builtin_fmaf(-a.beta, lam0, (float)F::K);
      if (num * bden > bnum * den) {
        bnum = num;
        bden = den;
        if (TRACK) bidx = m;
      }
    }
  }
  if (SCHEME == kSL2) {
    pnum = best2;
    pden = 1.0f;
  } else {
    pnum = bnum;
    pden = bden;
  }
  if (TRACK) *pidx = bidx;
}
}  // namespace slhjb
