// Pre-computation kernels of the patchy method (Section 4.3): bilinear upsampling of the
// coarse solution, discrete synthesis of the feedback control, and the integer form of the
// patch construction (eq. discrete-advection followed by the argmax that turns the fuzzy
// indicators into patches).
#include "internal.h"

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
// phi_p(x) in [0, 2^15] per node and patch, stored node-major: phi[node * P + p], uint16.
// A FREE node takes the Q.8 bilinear value of phi_p at its synthesized foot,
//   D = round_half_even(256 fl(fl(r c) a))  per axis (r = fl(h/dx)),
//   corner (i + (D_x >> 8), j + (D_y >> 8)), weights (256 - f or f) per axis, f = D & 255,
//   phi' = (sum_c W_c phi(c) + 2^15) >> 16.
// The map is monotone and the start lies below its image, so updates in any order, in place
// and concurrently, climb to the same least fixed point: the kernels below update in place
// and iterate until nothing changes.

__global__ void label_init_kernel(const uint8_t* __restrict__ cls, const int16_t* __restrict__ src, int64_t count,
                                  int P, uint32_t* __restrict__ phi32) {
  // one thread per node; P even, so a node is P/2 uint32 words
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int half = P >> 1;
  uint32_t* row = phi32 + t * half;
  for (int q = 0; q < half; ++q) row[q] = 0u;
  if (cls[t] == kTarget) {
    const int p = src[t];
    if (p >= 0 && p < P) row[p >> 1] = (p & 1) ? (1u << 31) : (1u << 15);
  }
}

constexpr int kLabTile = 16;  // 16 x 16 nodes per tile
constexpr int kLabHalo = 2;
constexpr int kLabSpan = kLabTile + 2 * kLabHalo;

// One pass over the active tiles of the labeler. Each workgroup loads its tile plus a halo of
// phi into LDS, iterates the in-place update on its FREE nodes until nothing changes (or
// max_inner iterations), writes the tile back, and flags itself and its neighbours for the next
// pass if anything changed. P <= 64 and even.
__global__ __launch_bounds__(256) void label_pass_kernel(uint32_t* __restrict__ phi32, const uint8_t* __restrict__ cls,
                                                         const int16_t* __restrict__ ctrl,
                                                         const float* __restrict__ speed, float speed_const,
                                                         const float2* __restrict__ ctab, float r, int n, int P,
                                                         const int* __restrict__ list, const int* __restrict__ count,
                                                         int tiles_x, int tiles_y, uint8_t* __restrict__ next_flag,
                                                         int max_inner, unsigned* __restrict__ changed_any) {
  extern __shared__ uint32_t lds[];
  const int half = P >> 1;
  uint32_t* tile = lds;                                               // kLabSpan^2 * half words
  int* fbase = (int*)(lds + kLabSpan * kLabSpan * half);              // 256 ints
  uint32_t* fw = (uint32_t*)(fbase + kLabTile * kLabTile);            // 256 packed (fx | fy << 16)
  const int total = *count;
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int tid = list[slot];
    const int tx = tid % tiles_x, ty = tid / tiles_x;
    const int x0 = tx * kLabTile - kLabHalo, y0 = ty * kLabTile - kLabHalo;
    // stage phi of the tile and its halo; nodes outside the grid read 0
    for (int w = threadIdx.x; w < kLabSpan * kLabSpan * half; w += blockDim.x) {
      const int node = w / half, q = w - node * half;
      const int ly = node / kLabSpan, lx = node - ly * kLabSpan;
      const int gx = x0 + lx, gy = y0 + ly;
      uint32_t val = 0u;
      if (gx >= 0 && gx < n && gy >= 0 && gy < n) val = phi32[((size_t)gy * n + gx) * half + q];
      tile[w] = val;
    }
    // feet of the tile's FREE nodes
    {
      const int ln = threadIdx.x;  // 256 threads = 256 tile nodes
      const int lx = ln & (kLabTile - 1), ly = ln >> 4;
      const int gx = tx * kLabTile + lx, gy = ty * kLabTile + ly;
      int base = -1;
      uint32_t packed = 0u;
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
          const int cx = lx + kLabHalo + (Dx >> 8), cy = ly + kLabHalo + (Dy >> 8);
          base = cy * kLabSpan + cx;
          packed = (uint32_t)(Dx & 255) | ((uint32_t)(Dy & 255) << 16);
        }
      }
      fbase[ln] = base;
      fw[ln] = packed;
    }
    __syncthreads();
    // in-place iteration: thread -> (node, word); the block covers blockDim/half nodes per step
    const int per_step = blockDim.x / half;
    const int q = threadIdx.x % half;
    int it = 0, last = 0, ever = 0;
    for (;;) {
      int ch = 0;
      for (int ln = threadIdx.x / half; ln < kLabTile * kLabTile; ln += per_step) {
        const int base = fbase[ln];
        if (base < 0) continue;
        const uint32_t pk = fw[ln];
        const uint32_t fx = pk & 0xffffu, fy = pk >> 16;
        const uint32_t w00 = (256u - fx) * (256u - fy), w10 = fx * (256u - fy);
        const uint32_t w01 = (256u - fx) * fy, w11 = fx * fy;
        const uint32_t c00 = tile[base * half + q], c10 = tile[(base + 1) * half + q];
        const uint32_t c01 = tile[(base + kLabSpan) * half + q], c11 = tile[(base + kLabSpan + 1) * half + q];
        const uint32_t lo = ((w00 * (c00 & 0xffffu) + w10 * (c10 & 0xffffu) + w01 * (c01 & 0xffffu) +
                              w11 * (c11 & 0xffffu) + 32768u) >> 16);
        const uint32_t hi = ((w00 * (c00 >> 16) + w10 * (c10 >> 16) + w01 * (c01 >> 16) + w11 * (c11 >> 16) +
                              32768u) >> 16);
        const uint32_t nv = lo | (hi << 16);
        const int ly = ln >> 4, lx = ln & (kLabTile - 1);
        const int self = ((ly + kLabHalo) * kLabSpan + lx + kLabHalo) * half + q;
        if (nv != tile[self]) {
          tile[self] = nv;
          ch = 1;
        }
      }
      last = __syncthreads_or(ch);  // barrier + block-wide OR
      ever |= last;
      ++it;
      if (!last || it >= max_inner) break;
    }
    const bool converged_here = (last == 0);
    // write the tile back (interior nodes only)
    for (int w = threadIdx.x; w < kLabTile * kLabTile * half; w += blockDim.x) {
      const int node = w / half, q = w - node * half;
      const int ly = node / kLabTile, lx = node - ly * kLabTile;
      const int gx = tx * kLabTile + lx, gy = ty * kLabTile + ly;
      if (gx < n && gy < n)
        phi32[((size_t)gy * n + gx) * half + q] = tile[((ly + kLabHalo) * kLabSpan + lx + kLabHalo) * half + q];
    }
    if (threadIdx.x == 0) {
      if (ever) {
        // neighbours read this tile as their halo; the tile itself continues if it did not settle
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int nx = tx + dx, ny = ty + dy;
            if (nx < 0 || ny < 0 || nx >= tiles_x || ny >= tiles_y) continue;
            if (dx == 0 && dy == 0 && converged_here) continue;
            next_flag[ny * tiles_x + nx] = 1;
          }
        atomicOr(changed_any, 1u);
      }
    }
    __syncthreads();
  }
}

// Compact the flagged tiles into a list (order irrelevant: the fixed point does not depend on
// it), clearing the flags.
__global__ void compact_flags_kernel(uint8_t* __restrict__ flag, int count, int* __restrict__ list,
                                     int* __restrict__ out_count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  bool on = false;
  if (t < count) {
    on = flag[t] != 0;
    if (on) flag[t] = 0;
  }
  const unsigned long long mask = __ballot(on);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0 && mask) base = atomicAdd(out_count, __popcll(mask));
  base = __shfl(base, 0, 64);
  if (on) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = t;
}

__global__ void label_argmax_kernel(const uint16_t* __restrict__ phi, int64_t count, int P, int16_t* __restrict__ label,
                                    uint64_t* __restrict__ overlap, uint16_t tau) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint16_t* row = phi + t * P;
  int best = -1;
  uint32_t bv = 0;
  uint64_t ov = 0;
  for (int p = 0; p < P; ++p) {
    const uint32_t v = row[p];
    if (v > bv) {
      bv = v;
      best = p;
    }
    if (tau > 0 && v >= tau) ov |= 1ull << p;
  }
  label[t] = (int16_t)best;
  if (overlap) overlap[t] = ov;
}

hipError_t launch_label_init(const uint8_t* cls, const int16_t* src, int64_t count, int P, uint32_t* phi32,
                             hipStream_t s) {
  label_init_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(cls, src, count, P, phi32);
  return hipGetLastError();
}

size_t label_pass_lds_bytes(int P) {
  return sizeof(uint32_t) * (size_t)kLabSpan * kLabSpan * (P / 2) + sizeof(int) * 256 + sizeof(uint32_t) * 256;
}

hipError_t launch_label_pass(uint32_t* phi32, const uint8_t* cls, const int16_t* ctrl, const float* speed,
                             float speed_const, const float2* ctab, float r, int n, int P, const int* list,
                             const int* count, int tiles_x, int tiles_y, uint8_t* next_flag, int max_inner,
                             unsigned* changed_any, int grid, hipStream_t s) {
  label_pass_kernel<<<grid, 256, label_pass_lds_bytes(P), s>>>(phi32, cls, ctrl, speed, speed_const, ctab, r, n, P,
                                                               list, count, tiles_x, tiles_y, next_flag, max_inner,
                                                               changed_any);
  return hipGetLastError();
}

hipError_t launch_compact_flags(uint8_t* flag, int count, int* list, int* out_count, hipStream_t s) {
  compact_flags_kernel<<<(count + 255) / 256, 256, 0, s>>>(flag, count, list, out_count);
  return hipGetLastError();
}

hipError_t launch_label_argmax(const uint16_t* phi, int64_t count, int P, int16_t* label, uint64_t* overlap,
                               uint16_t tau, hipStream_t s) {
  label_argmax_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(phi, count, P, label, overlap, tau);
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
