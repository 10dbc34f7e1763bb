// Batched Jacobi value iteration of many independent instances (serving-style solve).
//
// All instances still iterating share every sweep launch: a device work list holds one item per
// (instance, tile); a workgroup takes an item, loads that instance's parameters (uniform, so
// scalar loads), stages the tile and its halo in LDS and applies the same per-node update as the
// single-instance sweep kernels (ring1_update / general_update), so every value is bit-identical
// to the single-instance iteration whatever the tile shape. After each batch of check_every
// sweeps a single-workgroup check kernel reads the per-instance residual of the batch's last
// sweep, retires the instances that converged, failed or ran out of sweeps, and rebuilds the work
// list. The launches of several batches are captured in one graph; the host only reads the
// number of instances left between replays.
#include "sweep_device.h"

namespace slhjb {

struct BatchCtl {
  unsigned items;        // work items of the current batch
  unsigned active;       // instances still iterating
  unsigned batch_len;    // sweeps of the current batch
  unsigned pad;
  long long sweeps;      // sweeps completed by every instance still iterating
  long long max_sweeps;
  int check_every;
  int pad2;
  unsigned long long node_updates;
  unsigned long long tiles_swept;
  double tol;             // compared in double, as the single-instance solve does
};
static_assert(offsetof(BatchCtl, active) == kBatchCtlActive * 4 && offsetof(BatchCtl, sweeps) == kBatchCtlSweeps * 4 &&
                  offsetof(BatchCtl, node_updates) == kBatchCtlUpdates * 4 &&
                  offsetof(BatchCtl, tiles_swept) == kBatchCtlTiles * 4,
              "host reads these words");

// One sweep of every work item. `b` is the launch's index within its batch: launches beyond the
// batch's length (the last, shorter batch) do nothing. The iterate of sweep s is read from pool
// (s & 1) and written to pool (s & 1) ^ 1.
template <int SCHEME>
__global__ __launch_bounds__(kThreads) void batch_sweep_kernel(const BatchInst* __restrict__ inst,
                                                               const int2* __restrict__ work,
                                                               const float4* __restrict__ ctrl_all,
                                                               float* __restrict__ pool0, float* __restrict__ pool1,
                                                               unsigned* __restrict__ resid,
                                                               unsigned* __restrict__ flags, int b,
                                                               BatchCtl* __restrict__ c) {
  extern __shared__ float tile[];
  const int blen = (int)c->batch_len;
  if (b >= blen) return;
  const int items = (int)c->items;
  const int par = (int)((c->sweeps + b) & 1);
  const float* __restrict__ src = par ? pool1 : pool0;
  float* __restrict__ dst = par ? pool0 : pool1;
  const bool publish = b == blen - 1;
  for (int wi = blockIdx.x; wi < items; wi += gridDim.x) {
    const int2 it = work[wi];
    const BatchInst& I = inst[it.x];
    SweepArgs a = I.a;
    const int n = a.n, R = a.halo;
    const int twl = I.tw_log2, TW = 1 << twl, TH = I.th;
    const int tx0 = (it.y % I.tiles_x) * TW, ty0 = (it.y / I.tiles_x) * TH;
    const int LW = TW + 2 * R, LH = TH + 2 * R;
    const float* __restrict__ w_in = src + I.offset;
    float* __restrict__ w_out = dst + I.offset;
    const float4* __restrict__ ctrl = ctrl_all + I.ctrl_offset;
    const float* __restrict__ speed = a.speed;
    const uint8_t* __restrict__ cls = a.cls;
    for (int t = threadIdx.x; t < LW * LH; t += kThreads) {
      const int ly = t / LW, lx = t - ly * LW;
      const int gx = tx0 - R + lx, gy = ty0 - R + ly;
      float val = 0.0f;
      if (gx >= 0 && gx < n && gy >= 0 && gy < n) val = w_in[(size_t)gy * n + gx];
      tile[t] = val;
    }
    __syncthreads();
    float local = 0.0f;
    bool bad = false;
    for (int q = threadIdx.x; q < TW * TH; q += kThreads) {
      const int lx = q & (TW - 1), ly = q >> twl;
      const int i = tx0 + lx, j = ty0 + ly;
      if (i >= n || j >= n) continue;
      const size_t idx = (size_t)j * n + i;
      const int cl = cls[idx];
      float wn;
      if (cl == kFree) {
        const float k = a.r * (speed ? speed[idx] : a.speed_const);
        const int li = (ly + R) * LW + lx + R;
        if (I.path == 1) {
          const float* T = tile + li;
          // the wavefront's rows: 64 consecutive q
          const int q0 = q & ~63;
          const int r0 = ty0 + (q0 >> twl), r1 = ty0 + ((q0 + 63) >> twl);
          const bool interior = tx0 >= 1 && tx0 + TW - 1 <= n - 2 && r0 >= 1 && r1 <= n - 2;
          if (interior)
            wn = ring1_update<SCHEME, false>(T, LW, k, ctrl, a, false, false, false, false);
          else
            wn = ring1_update<SCHEME, true>(T, LW, k, ctrl, a, i == 0, i == n - 1, j == 0, j == n - 1);
        } else if (I.diffusion == kDiffIso) {
          wn = general_update<kDiffIso, SCHEME>(tile, LW, li, i, j, k, tile[li], ctrl, a);
        } else if (I.diffusion == kDiffRank1) {
          wn = general_update<kDiffRank1, SCHEME>(tile, LW, li, i, j, k, tile[li], ctrl, a);
        } else {
          wn = general_update<kDiffNone, SCHEME>(tile, LW, li, i, j, k, tile[li], ctrl, a);
        }
        local = fmaxf(local, fabsf(wn - tile[li]));
        bad |= !isfinite(wn);
      } else {
        wn = cl == kTarget ? a.w_target : a.w_obstacle;
      }
      w_out[idx] = wn;
    }
    block_reduce_and_publish(local, bad, publish ? resid + it.x : nullptr, flags + it.x);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&c->tiles_swept, (unsigned long long)items);
}

// End of a batch (one workgroup): every instance that iterated in it has done batch_len more
// sweeps; retire it when the residual of the batch's last sweep is <= tol (converged), when it
// produced a non-finite value, or when it reached max_sweeps; clear the per-instance words; then
// size the next batch and rebuild the work list of the instances left, in instance order.
// state[i]: 0 iterating, 1 converged, 2 out of sweeps, 3 non-finite. done_at[i]: sweeps at exit.
__global__ __launch_bounds__(1024) void batch_check_kernel(const BatchInst* __restrict__ inst, int count,
                                                           unsigned* __restrict__ resid,
                                                           unsigned* __restrict__ flags, int* __restrict__ state,
                                                           long long* __restrict__ done_at,
                                                           float* __restrict__ last_resid,
                                                           int2* __restrict__ work, BatchCtl* __restrict__ c) {
  __shared__ int scan[1024];
  __shared__ int ntile[1024];
  __shared__ int base_s;
  if (c->active == 0u) return;
  const int blen = (int)c->batch_len;
  const long long sweeps = c->sweeps + blen;
  const double tol = c->tol;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  unsigned long long upd = 0;
  for (int i0 = 0; i0 < count; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    int tiles_i = 0;
    if (i < count && state[i] == 0) {
      upd += (unsigned long long)blen * (unsigned long long)inst[i].free_nodes;
      const float r = __uint_as_float(resid[i]);
      last_resid[i] = r;
      int s = 0;
      if (flags[i] & 1u) s = 3;
      else if ((double)r <= tol) s = 1;
      else if (sweeps >= c->max_sweeps) s = 2;
      if (s != 0) {
        state[i] = s;
        done_at[i] = sweeps;
      } else {
        tiles_i = inst[i].tiles;
      }
      resid[i] = 0u;
      flags[i] = 0u;
    }
    // inclusive scan of the tile counts of this chunk
    ntile[threadIdx.x] = tiles_i;
    scan[threadIdx.x] = tiles_i;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
      const int v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    const int start = base_s + scan[threadIdx.x] - tiles_i;
    const int chunk_total = scan[blockDim.x - 1];
    __syncthreads();
    scan[threadIdx.x] = start;  // first item of each instance of the chunk
    if (threadIdx.x == 0) base_s += chunk_total;
    __syncthreads();
    // all threads write the items of one instance after the other
    const int in_chunk = min((int)blockDim.x, count - i0);
    for (int k = 0; k < in_chunk; ++k) {
      const int nt = ntile[k];
      if (nt == 0) continue;
      const int st0 = scan[k];
      for (int t = threadIdx.x; t < nt; t += blockDim.x) work[st0 + t] = make_int2(i0 + k, t);
    }
    __syncthreads();
  }
  // active count and the next batch
  __shared__ unsigned act_s;
  if (threadIdx.x == 0) act_s = 0u;
  __syncthreads();
  unsigned mine = 0u;
  for (int i = threadIdx.x; i < count; i += blockDim.x) mine += state[i] == 0 ? 1u : 0u;
  if (mine) atomicAdd(&act_s, mine);
  if (upd) atomicAdd(&c->node_updates, upd);
  __syncthreads();
  if (threadIdx.x == 0) {
    c->active = act_s;
    c->items = (unsigned)base_s;
    c->sweeps = sweeps;
    const long long left = c->max_sweeps - sweeps;
    c->batch_len = (unsigned)(left < (long long)c->check_every ? (left > 0 ? left : 0) : c->check_every);
  }
}

__global__ void batch_init_kernel(const BatchInst* __restrict__ inst, int count, int* __restrict__ state,
                                  long long* __restrict__ done_at, float* __restrict__ last_resid,
                                  unsigned* __restrict__ resid, unsigned* __restrict__ flags, int2* __restrict__ work,
                                  const int* __restrict__ first_item, BatchCtl* __restrict__ c, long long max_sweeps,
                                  int check_every, double tol, unsigned items) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const int nt = inst[i].tiles, st0 = first_item[i];
  for (int t = threadIdx.x; t < nt; t += blockDim.x) work[st0 + t] = make_int2(i, t);
  if (threadIdx.x == 0) {
    state[i] = 0;
    done_at[i] = 0;
    last_resid[i] = INFINITY;
    resid[i] = 0u;
    flags[i] = 0u;
    if (i == 0) {
      c->items = items;
      c->active = (unsigned)count;
      c->batch_len = (unsigned)(max_sweeps < check_every ? max_sweeps : check_every);
      c->pad = 0u;
      c->sweeps = 0;
      c->max_sweeps = max_sweeps;
      c->check_every = check_every;
      c->pad2 = 0;
      c->tol = tol;
      c->node_updates = 0ull;
      c->tiles_swept = 0ull;
    }
  }
}

size_t batchctl_bytes() { return sizeof(BatchCtl); }

hipError_t launch_batch_init(const BatchInst* inst, int count, int* state, long long* done_at, float* last_resid,
                             unsigned* resid, unsigned* flags, int2* work, const int* first_item, void* ctl,
                             long long max_sweeps, int check_every, double tol, unsigned items, hipStream_t s) {
  batch_init_kernel<<<count, 256, 0, s>>>(inst, count, state, done_at, last_resid, resid, flags, work, first_item,
                                          (BatchCtl*)ctl, max_sweeps, check_every, tol, items);
  return hipGetLastError();
}

hipError_t launch_batch_round(const BatchInst* inst, int count, const float4* ctrl_all, float* pool0, float* pool1,
                              unsigned* resid, unsigned* flags, int* state, long long* done_at, float* last_resid,
                              int2* work, void* ctl, int scheme, int check_every, int grid, size_t lds,
                              hipStream_t s) {
  BatchCtl* c = (BatchCtl*)ctl;
  for (int b = 0; b < check_every; ++b) {
    if (scheme == kSL2)
      batch_sweep_kernel<kSL2><<<grid, kThreads, lds, s>>>(inst, work, ctrl_all, pool0, pool1, resid, flags, b, c);
    else
      batch_sweep_kernel<kSL3><<<grid, kThreads, lds, s>>>(inst, work, ctrl_all, pool0, pool1, resid, flags, b, c);
  }
  batch_check_kernel<<<1, 1024, 0, s>>>(inst, count, resid, flags, state, done_at, last_resid, work, c);
  return hipGetLastError();
}

}  // namespace slhjb
