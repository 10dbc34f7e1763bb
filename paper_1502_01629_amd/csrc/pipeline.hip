// Pre-computation kernels of the patchy method (Section 4.3): bilinear upsampling of the
// coarse solution, discrete synthesis of the feedback control, and the integer form of the
// patch construction (eq. discrete-advection followed by the argmax that turns the fuzzy
// indicators into patches).
#include "internal.h"
#include "select_device.h"

namespace slhjb {

// ---- u_hat: bilinear interpolation of the coarse solution on the fine grid -------------
// Fine node i sits at coarse coordinate i (n_c - 1) / (n_f - 1): the cell index and the
// fraction are taken from the exact integer quotient and remainder.
__global__ void upsample_bilinear_kernel(const float* __restrict__ vc, int nc, float* __restrict__ vf, int nf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nf || j >= nf) return;
  const int64_t den = nf - 1;
  const int64_t pi = (int64_t)i * (nc - 1), pj = (int64_t)j * (nc - 1);
  int ci = (int)(pi / den), cj = (int)(pj / den);
  float s = (float)(pi - (int64_t)ci * den) / (float)den;
  float t = (float)(pj - (int64_t)cj * den) / (float)den;
  if (ci > nc - 2) { ci = nc - 2; s = 1.0f; }
  if (cj > nc - 2) { cj = nc - 2; t = 1.0f; }
  const float* r0 = vc + (size_t)cj * nc + ci;
  const float* r1 = r0 + nc;
  // (1-s) a + s b reproduces both end values exactly, so coarse nodes (and the clamped upper
  // edge) are copied bit for bit
  const float lo = __builtin_fmaf(s, r0[1], (1.0f - s) * r0[0]);
  const float hi = __builtin_fmaf(s, r1[1], (1.0f - s) * r1[0]);
  vf[(size_t)j * nf + i] = __builtin_fmaf(t, hi, (1.0f - t) * lo);
}

hipError_t launch_upsample(const float* vc, int nc, float* vf, int nf, hipStream_t s) {
  dim3 grid((nf + 255) / 256, nf);
  upsample_bilinear_kernel<<<grid, 256, 0, s>>>(vc, nc, vf, nf);
  return hipGetLastError();
}

// ---- bicubic u_hat (the warm-start network's input feature) -----------------------------
// Keys' cubic convolution kernel, a = -1/2: W(x) = 1.5|x|^3 - 2.5|x|^2 + 1 on [0, 1],
// -0.5|x|^3 + 2.5|x|^2 - 4|x| + 2 on (1, 2). For a fraction t in [0, 1) the weights of the
// coarse nodes c-1, c, c+1, c+2 are W(t+1), W(t), W(1-t), W(2-t).
__device__ __forceinline__ void keys_weights(float t, float w[4]) {
  const float u = 1.0f - t;
  w[0] = ((-0.5f * t + 1.0f) * t - 0.5f) * t;            // W(1 + t) = -0.5 t^3 + t^2 - 0.5 t
  w[1] = (1.5f * t - 2.5f) * t * t + 1.0f;              // W(t)
  w[2] = (1.5f * u - 2.5f) * u * u + 1.0f;              // W(1 - t)
  w[3] = ((-0.5f * u + 1.0f) * u - 0.5f) * u;            // W(2 - t)
}

// Fine node i at coarse coordinate i (n_c - 1) / (n_f - 1) (exact integer quotient and remainder,
// as the bilinear kernel), 4 x 4 coarse nodes with indices clamped to the grid.
__global__ void upsample_bicubic_kernel(const float* __restrict__ vc, int nc, float* __restrict__ vf, int nf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nf || j >= nf) return;
  const int64_t den = nf - 1;
  const int64_t pi = (int64_t)i * (nc - 1), pj = (int64_t)j * (nc - 1);
  int ci = (int)(pi / den), cj = (int)(pj / den);
  float s = (float)(pi - (int64_t)ci * den) / (float)den;
  float t = (float)(pj - (int64_t)cj * den) / (float)den;
  if (ci > nc - 2) { ci = nc - 2; s = 1.0f; }
  if (cj > nc - 2) { cj = nc - 2; t = 1.0f; }
  float wx[4], wy[4];
  keys_weights(s, wx);
  keys_weights(t, wy);
  int xs[4], ys[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    xs[m] = min(max(ci + m - 1, 0), nc - 1);
    ys[m] = min(max(cj + m - 1, 0), nc - 1);
  }
  float acc = 0.0f;
#pragma unroll
  for (int my = 0; my < 4; ++my) {
    const float* row = vc + (size_t)ys[my] * nc;
    float r = 0.0f;
#pragma unroll
    for (int mx = 0; mx < 4; ++mx) r = __builtin_fmaf(wx[mx], row[xs[mx]], r);
    acc = __builtin_fmaf(wy[my], r, acc);
  }
  vf[(size_t)j * nf + i] = acc;
}

hipError_t launch_upsample_bicubic(const float* vc, int nc, float* vf, int nf, hipStream_t s) {
  dim3 grid((nf + 255) / 256, nf);
  upsample_bicubic_kernel<<<grid, 256, 0, s>>>(vc, nc, vf, nf);
  return hipGetLastError();
}

// ---- discrete synthesis (eq. discrete-synthesis, sigma = 0) ------------------------------
// ctrl[i] = argmin_m I[v_hat](x_i + h c_i a_m) for FREE nodes (first minimum in the caller's
// control order), -1 elsewhere. Feet outside the closed box read v_out.
__global__ __launch_bounds__(256) void synthesize_kernel(const float* __restrict__ vhat, const float* __restrict__ speed,
                                                          const uint8_t* __restrict__ cls,
                                                          const float2* __restrict__ ctrl, int n_controls, int n,
                                                          float r, float speed_const, float v_out,
                                                          int16_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const size_t idx = (size_t)j * n + i;
  if (cls[idx] != kFree) {
    out[idx] = -1;
    return;
  }
  const float k = r * (speed ? speed[idx] : speed_const);
  const float fi = (float)i, fj = (float)j, nm1 = (float)(n - 1), nm2 = (float)(n - 2);
  const float lox = -fi, hix = nm1 - fi, loy = -fj, hiy = nm1 - fj, cmx = nm2 - fi, cmy = nm2 - fj;
  float best = INFINITY;
  int bm = 0;
  for (int m = 0; m < n_controls; ++m) {
    const float2 a = ctrl[m];
    const float ox = k * a.x, oy = k * a.y;
    float val;
    if ((ox >= lox) & (ox <= hix) & (oy >= loy) & (oy <= hiy)) {
      const float flx = fminf(floorf(ox), cmx), fly = fminf(floorf(oy), cmy);
      const float s = ox - flx, t = oy - fly;
      const float* r0 = vhat + (size_t)(j + (int)fly) * n + (i + (int)flx);
      const float* r1 = r0 + n;
      const float lo = __builtin_fmaf(s, r0[1] - r0[0], r0[0]);
      const float hi = __builtin_fmaf(s, r1[1] - r1[0], r1[0]);
      val = __builtin_fmaf(t, hi - lo, lo);
    } else {
      val = v_out;
    }
    if (val < best) {
      best = val;
      bm = m;
    }
  }
  out[idx] = (int16_t)bm;
}

hipError_t launch_synthesize(const float* vhat, const float* speed, const uint8_t* cls, const float2* ctrl,
                             int n_controls, int n, float r, float speed_const, float v_out, int16_t* out,
                             hipStream_t s) {
  dim3 grid((n + 255) / 256, n);
  synthesize_kernel<<<grid, 256, 0, s>>>(vhat, speed, cls, ctrl, n_controls, n, r, speed_const, v_out, out);
  return hipGetLastError();
}

// ---- integer patch labeling --------------------------------------------------------------
// phi_p(x) in [0, 2^15] per node and patch, two patches per uint32 word, stored word-planar:
// phi32[q * N + node] holds patches 2q (low half) and 2q + 1 (high half), so a plane of one word
// is contiguous over the nodes. Each labeler tile keeps a mask of the words that are nonzero
// somewhere in it (it only grows, as the values do).
// A FREE node takes the Q.8 bilinear value of phi_p at its synthesized foot,
//   D = round_half_even(256 fl(fl(r c) a))  per axis (r = fl(h/dx)),
//   corner (i + (D_x >> 8), j + (D_y >> 8)), weights (256 - f or f) per axis, f = D & 255,
//   phi' = (sum_c W_c phi(c) + 2^15) >> 16.
// The map is monotone and the start lies below its image, so updates in any order, in place
// and concurrently, climb to the same least fixed point: the kernels below update in place
// and iterate until nothing changes.

// One thread per uint32 word (two patches) of phi, plane by plane, so the stores are contiguous.
__global__ void label_init_kernel(const uint8_t* __restrict__ cls, const int16_t* __restrict__ src, int64_t count,
                                  int half, uint32_t* __restrict__ phi32) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count * half) return;
  const int q = (int)(t / count);
  const int64_t node = t - (int64_t)q * count;
  uint32_t v = 0u;
  if (cls[node] == kTarget) {
    const int p = src[node];
    if ((p >> 1) == q) v = (p & 1) ? (1u << 31) : (1u << 15);
  }
  phi32[t] = v;
}

// The word masks of the labeler tiles at the start: the words of the sources (zeroed before).
__global__ void label_mask_init_kernel(const uint8_t* __restrict__ cls, const int16_t* __restrict__ src, int n,
                                       int tiles_x, int tile, unsigned* __restrict__ mask) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  if (cls[t] != kTarget) return;
  const int p = src[t];
  if (p < 0) return;
  const int x = (int)(t % n), y = (int)(t / n);
  atomicOr(&mask[(y / tile) * tiles_x + x / tile], 1u << (p >> 1));
}

constexpr int kLabTile = 16;  // 16 x 16 nodes per tile
constexpr int kLabSub = 4;    // in-place sweeps of a tile per barrier
constexpr int kLabHalo = 2;
constexpr int kLabSpan = kLabTile + 2 * kLabHalo;

// Labeler pass control, driven on the device (as the solver's passes): `select` takes the flagged
// tiles whose u_hat key is within the band, `visit` runs them; an empty band with flagged tiles
// left moves the band up to their smallest key, and no flagged tile at all ends the iteration.
struct LabCtl {
  unsigned count[2];
  unsigned nflag[2];
  unsigned kmin[2];
  unsigned bound;
  unsigned done;
  unsigned passes;
  unsigned pad;
};

__global__ void labctl_init_kernel(LabCtl* c) {
  c->count[0] = c->count[1] = 0u;
  c->nflag[0] = c->nflag[1] = 0u;
  c->kmin[0] = c->kmin[1] = 0x7f800000u;
  c->bound = 0xff800000u;
  c->done = 0u;
  c->passes = 0u;
  c->pad = 0u;
}

// A selected tile's flag is cleared here, not in the visit kernel: visits set the flags of
// their neighbours, and a clear in the same launch could erase a neighbour's request.
__global__ __launch_bounds__(kSelectThreads) void labctl_select_kernel(uint8_t* __restrict__ flag,
                                                                       const float* __restrict__ key, int tiles, int q,
                                                                       int* __restrict__ list, LabCtl* __restrict__ c) {
  // the tile's flag and key do not depend on the pass words: all their loads go out together
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int tt = t < tiles ? t : tiles - 1;
  unsigned done = c->done, bound = c->bound;
  unsigned fb = flag[tt];
  float kt = key ? key[tt] : INFINITY;
  SLHJB_ISSUE_TOGETHER("+s"(done), "+s"(bound), "+v"(fb), "+v"(kt));
  if (done) return;
  const bool fl = t < tiles && fb != 0u;
  const float B = key ? __uint_as_float(bound) : INFINITY;
  const float k = fl ? kt : INFINITY;
  const bool on = fl && (!key || k <= B);
  block_select(t, fl, on, k, key != nullptr, &c->count[q], &c->nflag[q], &c->kmin[q], list);
  if (on) flag[t] = 0;
}

// One visit per selected tile: stage phi of the tile and a halo in LDS, iterate the in-place
// update on the tile's FREE nodes until nothing changes (or max_inner), write the changed nodes
// back and flag each neighbour whose halo holds one of them (the strip of kLabHalo nodes on its
// side), and the tile itself if it did not settle. Only the
// words (patch pairs) that are nonzero somewhere in the staged region can become nonzero, so the
// iteration walks those words only. P <= 64, even.
// LDS holds one plane per word, tile[qw * kLabPlane + node]: the 64 lanes of a wavefront update 64
// neighbouring nodes of one word and read neighbouring addresses. The odd plane stride spreads the
// banks when the staging loop writes the words of one node.
constexpr int kLabPlane = kLabSpan * kLabSpan + 1;
__global__ __launch_bounds__(256) void label_visit_kernel(uint32_t* __restrict__ phi32, const uint8_t* __restrict__ cls,
                                                          const int16_t* __restrict__ ctrl,
                                                          const float* __restrict__ speed, float speed_const,
                                                          const float2* __restrict__ ctab, float r, int n, int P,
                                                          const int* __restrict__ list, int tiles_x, int tiles_y,
                                                          uint8_t* __restrict__ flag, unsigned* __restrict__ wmask,
                                                          int max_inner, float window, int q, LabCtl* __restrict__ c) {
  // the first slot's tile is read with the pass words (the grid and the list have at most `tiles`
  // entries; the value is used only if the slot is taken)
  unsigned done = c->done, ucnt = c->count[q], unf = c->nflag[q];
  int first = list[blockIdx.x];
  SLHJB_ISSUE_TOGETHER("+s"(done), "+s"(ucnt), "+s"(unf), "+s"(first));
  if (done) return;
  extern __shared__ uint32_t lds[];
  __shared__ unsigned omask, osides;
  __shared__ int act[32];
  __shared__ int nact;
  const int cnt = (int)ucnt;
  const int nf = (int)unf;
  if (cnt == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (nf > 0) c->bound = __float_as_uint(__uint_as_float(c->kmin[q]) + window);
      else c->done = 1u;
      c->count[q ^ 1] = 0u;
      c->nflag[q ^ 1] = 0u;
      c->kmin[q ^ 1] = 0x7f800000u;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c->passes += 1u;
    c->count[q ^ 1] = 0u;
    c->nflag[q ^ 1] = 0u;
    c->kmin[q ^ 1] = 0x7f800000u;
  }
  const int half = P >> 1;
  const size_t N = (size_t)n * n;
  uint32_t* tile = lds;  // half planes of kLabPlane words
  // the node of this thread (256 threads = 256 tile nodes)
  const int lx = threadIdx.x & (kLabTile - 1), ly = threadIdx.x >> 4;
  const int self = (ly + kLabHalo) * kLabSpan + lx + kLabHalo;
  for (int slot = blockIdx.x; slot < cnt; slot += gridDim.x) {
    const int tid = slot == (int)blockIdx.x ? first : list[slot];
    const int tx = tid % tiles_x, ty = tid / tiles_x;
    const int x0 = tx * kLabTile - kLabHalo, y0 = ty * kLabTile - kLabHalo;
    // wavefront 0: the words that can be nonzero in the staged region, the union of the masks of
    // the tile and its 8 neighbours (the halo of 2 nodes lies in them), as a list of planes
    if (threadIdx.x < 64) {
      unsigned m = 0u;
      if (threadIdx.x < 9) {
        const int nx = tx + threadIdx.x % 3 - 1, ny = ty + threadIdx.x / 3 - 1;
        if (nx >= 0 && ny >= 0 && nx < tiles_x && ny < tiles_y) m = wmask[ny * tiles_x + nx];
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) m |= __shfl_xor(m, off, 64);
      if (threadIdx.x == 0) {
        int k = 0;
        for (int b = 0; b < half; ++b)
          if (m & (1u << b)) act[k++] = b;
        nact = k;
        if (k & 1) act[k] = act[k - 1];  // the sweeps take the words in pairs (k <= 31 here)
        omask = 0u;
        osides = 0u;
      }
    }
    // foot of this thread's node, if FREE: corner cell and Q.8 fractions (its loads overlap the
    // mask reads above)
    const int gx = tx * kLabTile + lx, gy = ty * kLabTile + ly;
    int base = -1;
    uint32_t w00 = 0u, w10 = 0u, w01 = 0u, w11 = 0u;
    if (gx < n && gy < n) {
      const size_t idx = (size_t)gy * n + gx;
      const int m = ctrl[idx];
      if (cls[idx] == kFree && m >= 0) {
        const float k = r * (speed ? speed[idx] : speed_const);
        const float2 a = ctab[m];
        const float px = k * a.x, py = k * a.y;
        // |D| <= 256 for every first-ring foot (the host rejects larger reaches); the clamp only
        // keeps the LDS reads inside the tile if that contract is broken
        const int Dx = min(256, max(-256, (int)rintf(256.0f * px)));
        const int Dy = min(256, max(-256, (int)rintf(256.0f * py)));
        base = (ly + kLabHalo + (Dy >> 8)) * kLabSpan + lx + kLabHalo + (Dx >> 8);
        const uint32_t fx = (uint32_t)(Dx & 255), fy = (uint32_t)(Dy & 255);
        w00 = (256u - fx) * (256u - fy);
        w10 = fx * (256u - fy);
        w01 = (256u - fx) * fy;
        w11 = fx * fy;
      }
    }
    __syncthreads();
    const int A = nact;
    // stage those words of the tile and its halo (nodes outside the grid read 0): this thread's
    // two staged nodes (the region has kLabSpan^2 <= 2 * 256), two planes at a time so that four
    // loads are in flight
    static_assert(kLabSpan * kLabSpan <= 2 * 256, "two staged nodes per thread");
    {
      const int e0 = threadIdx.x, e1 = threadIdx.x + 256;
      const int sy0 = e0 / kLabSpan, sx0 = e0 - sy0 * kLabSpan;
      const int sy1 = e1 / kLabSpan, sx1 = e1 - sy1 * kLabSpan;
      const int gx0 = x0 + sx0, gy0 = y0 + sy0, gx1 = x0 + sx1, gy1 = y0 + sy1;
      const bool in0 = gx0 >= 0 && gx0 < n && gy0 >= 0 && gy0 < n;
      const bool in1 = e1 < kLabSpan * kLabSpan && gx1 >= 0 && gx1 < n && gy1 >= 0 && gy1 < n;
      const bool st1 = e1 < kLabSpan * kLabSpan;
      const size_t o0 = in0 ? (size_t)gy0 * n + gx0 : 0, o1 = in1 ? (size_t)gy1 * n + gx1 : 0;
      for (int qi = 0; qi < A; qi += 2) {
        const int qa = act[qi], qb = act[qi + 1];  // qb == qa for the padding of an odd count
        const uint32_t va0 = in0 ? phi32[(size_t)qa * N + o0] : 0u, va1 = in1 ? phi32[(size_t)qa * N + o1] : 0u;
        const uint32_t vb0 = in0 ? phi32[(size_t)qb * N + o0] : 0u, vb1 = in1 ? phi32[(size_t)qb * N + o1] : 0u;
        tile[qa * kLabPlane + e0] = va0;
        tile[qb * kLabPlane + e0] = vb0;
        if (st1) {
          tile[qa * kLabPlane + e1] = va1;
          tile[qb * kLabPlane + e1] = vb1;
        }
      }
    }
    __syncthreads();
    int it = 0, last = 0, ever = 0;
    bool mine_changed = false;  // this thread's node changed during the visit
    if (A > 0) {
      for (;;) {
        // a round of kLabSub in-place sweeps of the tile under one barrier: values only grow, so
        // any interleaving of the wavefronts climbs to the same least fixed point, and a round in
        // which no thread changed anything read final values everywhere (the tile is settled)
        // A word's update reads only its own plane, so the words are independent: they go in
        // pairs with all ten reads issued before either write (the padding of an odd count
        // repeats the last word, which then gets the same value written twice).
        int ch = 0;
        auto interp = [&](uint32_t c00, uint32_t c10, uint32_t c01, uint32_t c11) -> uint32_t {
          const uint32_t lo = ((w00 * (c00 & 0xffffu) + w10 * (c10 & 0xffffu) + w01 * (c01 & 0xffffu) +
                                w11 * (c11 & 0xffffu) + 32768u) >> 16);
          const uint32_t hi = ((w00 * (c00 >> 16) + w10 * (c10 >> 16) + w01 * (c01 >> 16) + w11 * (c11 >> 16) +
                                32768u) >> 16);
          return lo | (hi << 16);
        };
        for (int sub = 0; sub < kLabSub; ++sub) {
          if (base >= 0) {
            for (int qi = 0; qi < A; qi += 2) {
              uint32_t* pa = tile + act[qi] * kLabPlane;
              uint32_t* pb = tile + act[qi + 1] * kLabPlane;
              const uint32_t a00 = pa[base], a10 = pa[base + 1], a01 = pa[base + kLabSpan],
                             a11 = pa[base + kLabSpan + 1], am = pa[self];
              const uint32_t b00 = pb[base], b10 = pb[base + 1], b01 = pb[base + kLabSpan],
                             b11 = pb[base + kLabSpan + 1], bm = pb[self];
              const uint32_t na = interp(a00, a10, a01, a11), nb = interp(b00, b10, b01, b11);
              if (na != am) {
                pa[self] = na;
                ch = 1;
              }
              if (nb != bm) {
                pb[self] = nb;
                ch = 1;
              }
            }
          }
        }
        mine_changed |= ch != 0;
        last = __syncthreads_or(ch);  // barrier + block-wide OR
        ever |= last;
        it += kLabSub;
        if (!last || it >= max_inner) break;
      }
    }
    const bool converged_here = (last == 0);
    // write back the words that can have changed of the nodes that changed (a node that did not
    // change holds what phi32 holds, and its nonzero words are in the mask since they were
    // written), note their nonzero words and the neighbours that read them
    if (ever) {
      unsigned sides = 0u;
      if (mine_changed) {  // only FREE nodes inside the grid are ever written
        unsigned mine = 0u;
        for (int qi = 0; qi < A; ++qi) {
          const int qw = act[qi];
          const uint32_t val = tile[qw * kLabPlane + self];
          phi32[(size_t)qw * N + (size_t)gy * n + gx] = val;
          mine |= (val != 0u ? 1u : 0u) << qw;
        }
        if (mine) atomicOr(&omask, mine);
        sides = near_sides(lx, ly, kLabTile, kLabTile, kLabHalo);
      }
      sides = wave_or(sides);
      if ((threadIdx.x & 63) == 0 && sides) atomicOr(&osides, sides);
      __syncthreads();  // uniform: `ever` is a block-wide OR
    }
    if (threadIdx.x < 9 && ever) {
      if (threadIdx.x == 0 && omask) atomicOr(&wmask[tid], omask);
      // neighbours read this tile as their halo; the tile itself continues if it did not settle.
      // Lane b = (dy + 1) * 3 + dx + 1 flags the tile at offset (dx, dy): nine stores at once.
      const unsigned sd = osides;
      const int b = threadIdx.x, dx = b % 3 - 1, dy = b / 3 - 1;
      const int nx = tx + dx, ny = ty + dy;
      const bool take = b == 4 ? !converged_here : ((sd >> b) & 1u) != 0u;
      if (take && nx >= 0 && ny >= 0 && nx < tiles_x && ny < tiles_y) flag[ny * tiles_x + nx] = 1;
    }
    __syncthreads();
  }
}

// u_hat key of a labeler tile: the smallest arrival time -ln(1 - v/V*)/lambda over its FREE nodes.
__global__ __launch_bounds__(256) void label_keys_kernel(const float* __restrict__ vhat, const uint8_t* __restrict__ cls,
                                                         int n, int tiles_x, float vstar, float lambda,
                                                         float* __restrict__ key) {
  __shared__ float red[4];
  const int tid = blockIdx.x;
  const int tx = tid % tiles_x, ty = tid / tiles_x;
  const int gx = tx * kLabTile + (threadIdx.x & (kLabTile - 1)), gy = ty * kLabTile + (threadIdx.x >> 4);
  float best = INFINITY;
  if (gx < n && gy < n) {
    const size_t idx = (size_t)gy * n + gx;
    const float w = vstar - vhat[idx];
    if (cls[idx] == kFree) {
      if (lambda == 0.0f) best = vhat[idx];  // undiscounted: v is the arrival time itself
      else if (w > 0.0f) best = -logf(w / vstar) / lambda;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = fminf(best, __shfl_xor(best, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) key[tid] = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
}

size_t labctl_bytes() { return sizeof(LabCtl); }

hipError_t launch_labctl_init(void* c, hipStream_t s) {
  labctl_init_kernel<<<1, 1, 0, s>>>((LabCtl*)c);
  return hipGetLastError();
}

hipError_t launch_label_keys(const float* vhat, const uint8_t* cls, int n, int tiles_x, int tiles_y, float vstar,
                             float lambda, float* key, hipStream_t s) {
  label_keys_kernel<<<tiles_x * tiles_y, 256, 0, s>>>(vhat, cls, n, tiles_x, vstar, lambda, key);
  return hipGetLastError();
}

hipError_t launch_label_pass2(uint32_t* phi32, const uint8_t* cls, const int16_t* ctrl, const float* speed,
                              float speed_const, const float2* ctab, float r, int n, int P, const float* key, int* list,
                              int tiles_x, int tiles_y, uint8_t* flag, unsigned* wmask, int max_inner, float window,
                              int q, void* ctl, int grid, hipStream_t s) {
  const int tiles = tiles_x * tiles_y;
  if (grid < 1 || grid > tiles) return hipErrorInvalidValue;  // the visit reads list[blockIdx.x]
  labctl_select_kernel<<<(tiles + kSelectThreads - 1) / kSelectThreads, kSelectThreads, 0, s>>>(flag, key, tiles, q,
                                                                                            list, (LabCtl*)ctl);
  label_visit_kernel<<<grid, 256, label_pass_lds_bytes(P), s>>>(phi32, cls, ctrl, speed, speed_const, ctab, r, n, P,
                                                                list, tiles_x, tiles_y, flag, wmask, max_inner, window,
                                                                q, (LabCtl*)ctl);
  return hipGetLastError();
}

// One thread per node: the planes of phi in order, keeping the larger value and, on ties, the
// lower p (reads of a plane are contiguous over the threads); the overlap bits where phi_p >= tau.
__global__ __launch_bounds__(256) void label_argmax_kernel(const uint32_t* __restrict__ phi32, int64_t count, int P,
                                                           int16_t* __restrict__ label, uint64_t* __restrict__ overlap,
                                                           uint16_t tau) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= count) return;
  const int half = P >> 1;
  uint32_t bv = 0u;
  int bp = -1;
  uint64_t ov = 0ull;
  for (int q = 0; q < half; ++q) {
    const uint32_t word = phi32[(size_t)q * count + node];
    const uint32_t v0 = word & 0xffffu, v1 = word >> 16;
    if (v0 > bv) {
      bv = v0;
      bp = 2 * q;
    }
    if (v1 > bv) {
      bv = v1;
      bp = 2 * q + 1;
    }
    if (tau > 0) ov |= (uint64_t)((v0 >= tau ? 1u : 0u) | (v1 >= tau ? 2u : 0u)) << (2 * q);
  }
  label[node] = (int16_t)bp;
  if (overlap) overlap[node] = ov;
}

// phi in the caller's layout: out[node * n_patches + p], uint16
__global__ void label_phi_out_kernel(const uint32_t* __restrict__ phi32, int64_t count, int n_patches,
                                     uint16_t* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count * n_patches) return;
  const int64_t node = t / n_patches;
  const int p = (int)(t - node * n_patches);
  const uint32_t word = phi32[(size_t)(p >> 1) * count + node];
  out[t] = (uint16_t)((p & 1) ? (word >> 16) : (word & 0xffffu));
}

hipError_t launch_label_init(const uint8_t* cls, const int16_t* src, int64_t count, int P, uint32_t* phi32,
                             hipStream_t s) {
  const int64_t words = count * (P >> 1);
  label_init_kernel<<<(unsigned)((words + 255) / 256), 256, 0, s>>>(cls, src, count, P >> 1, phi32);
  return hipGetLastError();
}

hipError_t launch_label_mask_init(const uint8_t* cls, const int16_t* src, int n, int tiles_x, unsigned* mask,
                                  hipStream_t s) {
  hipError_t e = launch_fill_u32(mask, 0u, tiles_x * tiles_x, s);
  if (e != hipSuccess) return e;
  const int64_t count = (int64_t)n * n;
  label_mask_init_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(cls, src, n, tiles_x, kLabTile, mask);
  return hipGetLastError();
}

hipError_t launch_label_phi_out(const uint32_t* phi32, int64_t count, int n_patches, uint16_t* out, hipStream_t s) {
  const int64_t total = count * n_patches;
  label_phi_out_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(phi32, count, n_patches, out);
  return hipGetLastError();
}

size_t label_pass_lds_bytes(int P) { return sizeof(uint32_t) * (size_t)kLabPlane * (P / 2); }

hipError_t launch_label_argmax(const uint16_t* phi, int64_t count, int P, int16_t* label, uint64_t* overlap,
                               uint16_t tau, hipStream_t s) {
  label_argmax_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>((const uint32_t*)phi, count, P, label, overlap,
                                                                      tau);
  return hipGetLastError();
}

__global__ void fill_u8_kernel(uint8_t* p, uint8_t v, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) p[t] = v;
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int count, hipStream_t s) {
  fill_u8_kernel<<<(count + 255) / 256, 256, 0, s>>>(p, v, count);
  return hipGetLastError();
}

}  // namespace slhjb
