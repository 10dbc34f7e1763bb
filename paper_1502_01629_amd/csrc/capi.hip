// C-ABI of libslhjb: argument validation, context and scratch management, the Jacobi
// value-iteration driver, and the host-side parameter theory of Section 4.1.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <mutex>
#include <thread>
#include <memory>
#include <vector>

#include "../../include/slhjb.h"
#include "internal.h"

using namespace slhjb;

namespace {

// Instantiated graphs of device-driven pass batches, kept by the bytes of every launch argument
// they were captured with: a later solve with the same arguments (same problem, buffers,
// tolerances) replays the graph without capturing and instantiating it again. Least recently used
// entries are dropped. One cache per user (the tile solver, the labeler), each used from one
// host thread at a time.
struct GraphKey {
  std::vector<unsigned char> b;
  template <class T>
  GraphKey& add(const T& v) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
    b.insert(b.end(), p, p + sizeof(T));
    return *this;
  }
};

struct GraphCache {
  struct Entry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  static constexpr int kEntries = 4;
  Entry e[kEntries];
  uint64_t clock = 0;
  hipGraphExec_t find(const GraphKey& k) {
    for (auto& x : e)
      if (x.exec && x.key == k.b) {
        x.used = ++clock;
        return x.exec;
      }
    return nullptr;
  }
  void insert(GraphKey&& k, hipGraphExec_t exec) {
    Entry* v = &e[0];
    for (auto& x : e) {
      if (!x.exec) {
        v = &x;
        break;
      }
      if (x.used < v->used) v = &x;
    }
    if (v->exec) hipGraphExecDestroy(v->exec);
    v->key = std::move(k.b);
    v->exec = exec;
    v->used = ++clock;
  }
  void clear() {
    for (auto& x : e) {
      if (x.exec) hipGraphExecDestroy(x.exec);
      x.exec = nullptr;
      x.key.clear();
    }
  }
};

}  // namespace

struct slhjb_ctx {
  int device = 0;
  int cus = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  int last_hip = 0;
  std::string last_msg;
  // scratch
  float* buf = nullptr;          // second iterate buffer
  size_t buf_elems = 0;
  float* uhat = nullptr;         // pipeline: copy of u_hat read by the synthesis and the labeler
  size_t uhat_elems = 0;
  float* vbuf[2] = {nullptr, nullptr};  // single-sweep staging buffers
  size_t vbuf_elems = 0;
  unsigned* small = nullptr;     // [0] residual bits, [1] flags, [2..4] speed stats
  unsigned* small_host = nullptr;  // pinned mirror
  float4* ctrl = nullptr;
  int ctrl_cap = 0;
  float2* ctrl2 = nullptr;        // controls in the caller's order (synthesis, labeling)
  // labeler scratch
  uint32_t* phi = nullptr;
  size_t phi_words = 0;
  uint8_t* tflag = nullptr;       // per-tile flags
  int* tlist = nullptr;           // compacted tile list
  int* tcount = nullptr;          // [0] list length
  int* tcount_host = nullptr;
  size_t tiles_cap = 0;
  // active-tile solver scratch
  float* tkey = nullptr;
  float* tchange = nullptr;
  size_t stiles_cap = 0;
  void* coop = nullptr;           // persistent-solver state (device)
  unsigned* coop_host = nullptr;  // pinned mirror
  void* tctl = nullptr;           // device-driven pass state
  unsigned long long* tacc = nullptr;  // update counters of the visit workgroups (2 per workgroup)
  void* lctl = nullptr;           // labeler pass state
  unsigned* lctl_host = nullptr;
  unsigned* lctl_host2 = nullptr;
  unsigned* tctl_host = nullptr;
  unsigned* tctl_host2 = nullptr;    // second pinned copy (two graph replays in flight)
  hipEvent_t tdone[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  GraphCache tile_graphs;            // tile-solver pass batches
  GraphCache label_graphs;           // labeler pass batches
  hipStream_t lcap_stream = nullptr; // capture stream of the labeler
  hipEvent_t ldone[2] = {nullptr, nullptr};
  // labeler buffers of its own, so that it can run beside the tile solver (patchy pipeline)
  hipStream_t aux_stream = nullptr;
  uint8_t* lflag = nullptr;
  int* llist = nullptr;
  float* lkey = nullptr;
  size_t ltiles_cap = 0;
  float2* lctab = nullptr;        // controls in the caller's order, for the labeler's feet
  unsigned* lmask = nullptr;      // word masks of the labeler tiles
  size_t lmask_cap = 0;
  hipEvent_t tev[32] = {};           // visit-kernel timing events of one captured batch
  unsigned* tchk_host = nullptr;     // check-sweep count after each pass of a timed batch (pinned)
  float* pipe_vc = nullptr;          // patchy pipeline: coarse iterate
  size_t pipe_vc_cap = 0;
  int16_t* pipe_ctrl = nullptr;      // patchy pipeline: synthesized control, labels
  int16_t* pipe_lab = nullptr;
  size_t pipe_cap = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, eva = nullptr, evb = nullptr;
};

namespace {

constexpr int kSmallWords = 16;
constexpr int kCtrlCap = 256 + 16;  // padded control table entries

int fail(slhjb_ctx* ctx, int status, const std::string& msg) {
  if (ctx) ctx->last_msg = msg;
  return status;
}

int hip_fail(slhjb_ctx* ctx, hipError_t e, const char* what) {
  if (ctx) {
    ctx->last_hip = (int)e;
    ctx->last_msg = std::string(what) + ": " + hipGetErrorString(e);
  }
  return SLHJB_E_HIP;
}

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #expr); \
  } while (0)

// Everything a sweep launch needs, derived once per call from a validated problem.
struct Prepared {
  SweepArgs args{};
  int diffusion = 0, scheme = 0, path = 0;
  float vstar = 1.0f;
  double reach = 0.0;
  int64_t free_nodes = 0;
  float speed_min = 0.0f, speed_max = 0.0f;  // over the nodes (speed_const without a field)
};

int validate(slhjb_ctx* ctx, const slhjb_problem* p) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!p) return fail(ctx, SLHJB_E_INVALID_ARG, "problem is NULL");
  if (p->n < 3 || p->n > 32769) return fail(ctx, SLHJB_E_INVALID_ARG, "n must be in [3, 32769]");
  if (!(isfinite(p->x_lo) && isfinite(p->x_hi) && p->x_lo < p->x_hi))
    return fail(ctx, SLHJB_E_INVALID_ARG, "need finite x_lo < x_hi");
  if (!(p->h > 0.0f) || !isfinite(p->h)) return fail(ctx, SLHJB_E_INVALID_ARG, "h must be finite and > 0");
  if (!(p->lambda >= 0.0f) || !isfinite(p->lambda))
    return fail(ctx, SLHJB_E_INVALID_ARG, "lambda must be finite and >= 0");
  if (!(p->eps >= 0.0f) || !isfinite(p->eps)) return fail(ctx, SLHJB_E_INVALID_ARG, "eps must be finite and >= 0");
  if (p->diffusion < 0 || p->diffusion > 2) return fail(ctx, SLHJB_E_INVALID_ARG, "unknown diffusion kind");
  if (p->scheme < 0 || p->scheme > 1) return fail(ctx, SLHJB_E_INVALID_ARG, "unknown scheme");
  if (p->n_controls < 1 || p->n_controls > 256) return fail(ctx, SLHJB_E_INVALID_ARG, "n_controls must be in [1, 256]");
  if (!p->controls) return fail(ctx, SLHJB_E_INVALID_ARG, "controls is NULL");
  for (int m = 0; m < 2 * p->n_controls; ++m)
    if (!isfinite(p->controls[m])) return fail(ctx, SLHJB_E_INVALID_ARG, "non-finite control");
  if (!p->speed && (!(p->speed_const > 0.0f) || !isfinite(p->speed_const)))
    return fail(ctx, SLHJB_E_INVALID_ARG, "speed_const must be finite and > 0");
  if (!(p->running_cost > 0.0f) || !isfinite(p->running_cost))
    return fail(ctx, SLHJB_E_INVALID_ARG, "running_cost must be finite and > 0");
  if (p->control_cost)
    for (int m = 0; m < p->n_controls; ++m)
      if (!(p->control_cost[m] >= 0.0f) || !isfinite(p->control_cost[m]))
        return fail(ctx, SLHJB_E_INVALID_ARG, "control_cost must be finite and >= 0");
  if (!p->node_class) return fail(ctx, SLHJB_E_INVALID_ARG, "node_class is NULL");
  if (!isfinite(p->target_value) || !isfinite(p->v_out))
    return fail(ctx, SLHJB_E_INVALID_ARG, "target_value and v_out must be finite");
  return SLHJB_OK;
}

double grid_dx(const slhjb_problem* p) { return ((double)p->x_hi - (double)p->x_lo) / (double)(p->n - 1); }

// A problem the first-ring and batched kernels do not take: varying costs, the undiscounted form
// or a diffusion coefficient field (the general kernels carry the cost term and per-node noise).
bool has_general_terms(const slhjb_problem* p) {
  return p->lambda == 0.0f || p->running_cost_field || p->control_cost || p->eps_field;
}

double reach_for(const slhjb_problem* p, double speed_max, double eps_max) {
  // distance in cells along either axis between a node and its farthest foot
  const float dx32 = (p->x_hi - p->x_lo) / (float)(p->n - 1);
  const double r = (double)(p->h / dx32);
  const double k = r * speed_max;
  double amax = 0.0;
  for (int m = 0; m < 2 * p->n_controls; ++m) amax = std::max(amax, fabs((double)p->controls[m]));
  const double d = p->diffusion == SLHJB_DIFF_NONE ? 0.0 : sqrt(2.0 * eps_max * (double)p->h) / grid_dx(p);
  if (p->diffusion == SLHJB_DIFF_RANK1) return (k + d) * amax;
  return k * amax + d;
}

// The start of a cold solve: the Kruzkov "+infinity" v = l / lambda (the time to reach the target
// is infinite), or v = 0 without discount, where the iteration then climbs to the exit times.
float cold_start_value(const slhjb_problem* p) {
  return p->lambda == 0.0f ? 0.0f : (float)((double)p->running_cost / (double)p->lambda);
}

int ensure_small(slhjb_ctx* ctx) {
  if (!ctx->small) {
    HIP_TRY(ctx, hipMalloc(&ctx->small, sizeof(unsigned) * kSmallWords));
    HIP_TRY(ctx, hipHostMalloc(&ctx->small_host, sizeof(unsigned) * kSmallWords, hipHostMallocDefault));
  }
  return SLHJB_OK;
}

// Device and host memory that preparing a problem writes: `dw` device words ([0] residual bits,
// [1] flags, [2..8] problem statistics), `hw` host words (the statistics are read back there),
// the padded control table and the controls in the caller's order (nullable).
struct PrepMem {
  unsigned* dw;
  unsigned* hw;
  float4* ctrl;
  float2* ctrl2;
};

int prepare_with(slhjb_ctx* ctx, const slhjb_problem* p, Prepared* out, const PrepMem& M) {
  int st = validate(ctx, p);
  if (st != SLHJB_OK) return st;
  const int n = p->n;
  const int64_t N = (int64_t)n * n;
  // speed bounds, FREE count, class validity and the drift's reach (one device pass, one read-back)
  if (p->drift && (reinterpret_cast<uintptr_t>(p->drift) & 7u))
    return fail(ctx, SLHJB_E_INVALID_ARG, "drift must be 8-byte aligned");
  HIP_TRY(ctx, launch_fill_u32(M.dw + 2, 0x7f7fffffu, 1, ctx->stream));
  HIP_TRY(ctx, launch_fill_u32(M.dw + 3, 0u, 10, ctx->stream));
  HIP_TRY(ctx, launch_problem_stats(p->speed, p->node_class, reinterpret_cast<const float2*>(p->drift),
                                    p->speed_const, N, M.dw + 2, ctx->stream));
  // [9..10] running-cost field max / bad, [11..12] diffusion-coefficient field max / bad
  if (p->running_cost_field) HIP_TRY(ctx, launch_field_stats(p->running_cost_field, N, 1, M.dw + 9, ctx->stream));
  if (p->eps_field) HIP_TRY(ctx, launch_field_stats(p->eps_field, N, 0, M.dw + 11, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(M.hw + 2, M.dw + 2, sizeof(unsigned) * 11, hipMemcpyDeviceToHost,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (M.hw[4]) return fail(ctx, SLHJB_E_INVALID_ARG, "speed has a non-finite or non-positive value");
  if (M.hw[6]) return fail(ctx, SLHJB_E_INVALID_ARG, "node_class has a value other than 0, 1, 2");
  if (M.hw[8]) return fail(ctx, SLHJB_E_INVALID_ARG, "drift has a non-finite value");
  if (M.hw[10]) return fail(ctx, SLHJB_E_INVALID_ARG, "running_cost_field has a non-finite or non-positive value");
  if (M.hw[12]) return fail(ctx, SLHJB_E_INVALID_ARG, "eps_field has a non-finite or negative value");
  float lx_max = p->running_cost, eps_max = p->eps;
  if (p->running_cost_field) memcpy(&lx_max, &M.hw[9], sizeof(float));
  if (p->eps_field) memcpy(&eps_max, &M.hw[11], sizeof(float));
  double speed_max = p->speed_const;
  if (p->speed) {
    float hi;
    memcpy(&hi, &M.hw[3], sizeof(float));
    speed_max = hi;
  }
  const int64_t free_nodes = M.hw[5];
  double reach = reach_for(p, speed_max, eps_max);
  if (p->drift) {
    // the drift moves every foot of a node by h c d / dx
    float dmax;
    memcpy(&dmax, &M.hw[7], sizeof(float));
    const float dx32 = (p->x_hi - p->x_lo) / (float)(p->n - 1);
    reach += (double)(p->h / dx32) * (double)dmax;
  }
  Prepared P;
  P.speed_max = (float)speed_max;
  P.speed_min = p->speed_const;
  if (p->speed) memcpy(&P.speed_min, &M.hw[2], sizeof(float));
  P.diffusion = eps_max > 0.0f ? p->diffusion : SLHJB_DIFF_NONE;
  P.scheme = p->scheme;
  P.reach = reach;
  P.free_nodes = free_nodes;
  // the first-ring kernels take a foot's quadrant from the signs of the control: no drift; they
  // carry no cost term
  if (P.diffusion == SLHJB_DIFF_NONE && reach <= 1.0 + 1e-6 && !p->drift && !has_general_terms(p)) {
    P.path = 1;
  } else {
    P.path = has_general_terms(p) ? 2 : 0;  // 2: the general kernels with the cost term and noise field
  }
  const int halo = P.path == 1 ? 2 : (int)floor(reach * (1.0 + 1e-6) + 1e-6) + 1;
  if (halo > kMaxHalo)
    return fail(ctx, SLHJB_E_UNSUPPORTED,
                "feet reach more than " + std::to_string(kMaxHalo - 1) + " cells; reduce h or eps");
  // control table, grouped by quadrant for the first-ring kernel (fixed-size host arrays: the
  // no-allocation entry point prepares its problem here too)
  int order[256];
  for (int m = 0; m < p->n_controls; ++m) order[m] = m;
  int quad[5] = {0, 0, 0, 0, 0};
  if (P.path == 1) {
    auto qof = [&](int m) {
      const float ax = p->controls[2 * m], ay = p->controls[2 * m + 1];
      if (ay >= 0.0f) return ax >= 0.0f ? 0 : 1;
      return ax < 0.0f ? 2 : 3;
    };
    std::stable_sort(order, order + p->n_controls, [&](int a, int b) { return qof(a) < qof(b); });
    int q = 0;
    for (int t = 0; t < p->n_controls; ++t)
      while (q < qof(order[t])) quad[++q] = t;
    while (q < 4) quad[++q] = p->n_controls;
  } else {
    quad[4] = p->n_controls;
  }
  // Pad every quadrant's list (or the whole list for the general kernel) to a multiple of 4 by
  // repeating its last control: a repeat cannot change a max, and the kernels then fetch the
  // table four entries at a time.
  float4 tab[kCtrlCap];
  int ntab = 0;
  int pquad[5] = {0, 0, 0, 0, 0};
  // Cost term of the general kernels (see SweepArgs): the iterate is w = C - v with C = l / lambda
  // (the largest running cost over lambda when it varies) or C = 0 without discount; then
  // q = (K / beta) (fac l(x,a) - (1 - beta) C), fac = (1 - beta) / lambda or h, is 0 for a
  // constant cost with lambda > 0 and the update stays homogeneous.
  const int K = P.diffusion == SLHJB_DIFF_ISO ? 4 : (P.diffusion == SLHJB_DIFF_RANK1 ? 2 : 1);
  const double beta_d = (double)(float)exp(-(double)p->lambda * (double)p->h);
  double la_max = 0.0;
  if (p->control_cost)
    for (int m = 0; m < p->n_controls; ++m) la_max = std::max(la_max, (double)p->control_cost[m]);
  const bool varying = p->running_cost_field || p->control_cost;
  const double Cd = p->lambda == 0.0f ? 0.0
                                      : (varying ? ((double)lx_max + la_max) : (double)p->running_cost) / p->lambda;
  const double fac = p->lambda == 0.0f ? (double)p->h : (1.0 - beta_d) / (double)p->lambda;
  const bool cost = p->lambda == 0.0f || varying;
  const double kq = cost ? K / beta_d * fac : 0.0;
  const double kc = cost ? K / beta_d * (1.0 - beta_d) * Cd : 0.0;
  for (int q = 0; q < 4; ++q) {
    pquad[q] = ntab;
    for (int t = quad[q]; t < quad[q + 1]; ++t) {
      const float ax = p->controls[2 * order[t]], ay = p->controls[2 * order[t] + 1];
      // .w: |a_x| + |a_y| for the first-ring kernels, the control's cost part kq l_a for the general ones
      const float wv = P.path == 1 ? fabsf(ax) + fabsf(ay)
                                   : (float)(p->control_cost ? kq * (double)p->control_cost[order[t]] : 0.0);
      tab[ntab++] = make_float4(ax, ay, ax * ay, wv);
    }
    while (ntab % 4 != 0) {
      tab[ntab] = tab[ntab - 1];
      ++ntab;
    }
  }
  pquad[4] = ntab;
  for (int q = 0; q < 5; ++q) quad[q] = pquad[q];
  HIP_TRY(ctx, hipMemcpyAsync(M.ctrl, tab, sizeof(float4) * ntab, hipMemcpyHostToDevice, ctx->stream));
  if (M.ctrl2)
    HIP_TRY(ctx, hipMemcpyAsync(M.ctrl2, p->controls, sizeof(float2) * p->n_controls, hipMemcpyHostToDevice,
                                ctx->stream));
  // The copy reads `tab` asynchronously from pageable memory; make it complete before `tab` dies.
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));

  const double dx = grid_dx(p);
  // h/dx in float arithmetic, exactly as the foot displacements of the labeler are defined
  const float dx32 = (p->x_hi - p->x_lo) / (float)(p->n - 1);
  const float vstar = (float)Cd;
  SweepArgs& a = P.args;
  a.speed = p->speed;
  a.cls = p->node_class;
  a.ctrl = M.ctrl;
  a.resid = nullptr;
  a.flags = M.dw + 1;
  a.n = n;
  a.n_controls = quad[4];
  a.halo = halo;
  for (int q = 0; q < 5; ++q) a.quad[q] = quad[q];
  a.r = p->h / dx32;
  a.speed_const = p->speed_const;
  a.d = P.diffusion == SLHJB_DIFF_NONE ? 0.0f : (float)(sqrt(2.0 * (double)p->eps * (double)p->h) / dx);
  a.beta = (float)exp(-(double)p->lambda * (double)p->h);
  a.w_outside = vstar - p->v_out;
  a.drift = reinterpret_cast<const float2*>(p->drift);
  a.w_target = vstar - p->target_value;
  a.w_obstacle = vstar - p->v_out;
  a.cost = cost ? 1 : 0;
  a.lx = p->running_cost_field;
  a.lconst = p->running_cost;
  a.kq = (float)kq;
  a.kc = (float)kc;
  a.epsf = P.diffusion == SLHJB_DIFF_NONE ? nullptr : p->eps_field;
  a.d2 = (float)(2.0 * (double)p->h / (dx * dx));
  P.vstar = vstar;
  *out = P;
  return SLHJB_OK;
}

int prepare(slhjb_ctx* ctx, const slhjb_problem* p, Prepared* out) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  int st = ensure_small(ctx);
  if (st != SLHJB_OK) return st;
  if (!ctx->ctrl) {
    HIP_TRY(ctx, hipMalloc(&ctx->ctrl, sizeof(float4) * kCtrlCap));
    ctx->ctrl_cap = kCtrlCap;
  }
  if (!ctx->ctrl2) HIP_TRY(ctx, hipMalloc(&ctx->ctrl2, sizeof(float2) * 256));
  return prepare_with(ctx, p, out, PrepMem{ctx->small, ctx->small_host, ctx->ctrl, ctx->ctrl2});
}

int ensure_buf(slhjb_ctx* ctx, float** b, size_t* cap, size_t elems) {
  if (*cap >= elems) return SLHJB_OK;
  if (*b) hipFree(*b);
  *b = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(b, sizeof(float) * elems);
  if (e == hipErrorOutOfMemory) return fail(ctx, SLHJB_E_NOMEM, "scratch allocation failed");
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
  *cap = elems;
  return SLHJB_OK;
}

// Scratch of the patchy pipeline: the coarse iterate, the synthesized control and the labels.
int ensure_pipe(slhjb_ctx* ctx, size_t coarse_nodes, size_t fine_nodes) {
  if (ctx->pipe_vc_cap < coarse_nodes) {
    if (ctx->pipe_vc) hipFree(ctx->pipe_vc);
    ctx->pipe_vc = nullptr;
    ctx->pipe_vc_cap = 0;
    hipError_t e = hipMalloc(&ctx->pipe_vc, sizeof(float) * coarse_nodes);
    if (e != hipSuccess) return hip_fail(ctx, e, "pipeline scratch");
    ctx->pipe_vc_cap = coarse_nodes;
  }
  if (ctx->pipe_cap < fine_nodes) {
    if (ctx->pipe_ctrl) hipFree(ctx->pipe_ctrl);
    if (ctx->pipe_lab) hipFree(ctx->pipe_lab);
    ctx->pipe_ctrl = ctx->pipe_lab = nullptr;
    ctx->pipe_cap = 0;
    hipError_t e = hipMalloc(&ctx->pipe_ctrl, sizeof(int16_t) * fine_nodes);
    if (e == hipSuccess) e = hipMalloc(&ctx->pipe_lab, sizeof(int16_t) * fine_nodes);
    if (e != hipSuccess) return hip_fail(ctx, e, "pipeline scratch");
    ctx->pipe_cap = fine_nodes;
  }
  return SLHJB_OK;
}

int ensure_tiles(slhjb_ctx* ctx, size_t tiles) {
  if (!ctx->tcount) {
    HIP_TRY(ctx, hipMalloc(&ctx->tcount, sizeof(int) * 4));
    HIP_TRY(ctx, hipHostMalloc(&ctx->tcount_host, sizeof(int) * 4, hipHostMallocDefault));
  }
  if (ctx->tiles_cap >= tiles) return SLHJB_OK;
  if (ctx->tflag) hipFree(ctx->tflag);
  if (ctx->tlist) hipFree(ctx->tlist);
  ctx->tflag = nullptr;
  ctx->tlist = nullptr;
  ctx->tiles_cap = 0;
  HIP_TRY(ctx, hipMalloc(&ctx->tflag, tiles));
  HIP_TRY(ctx, hipMalloc(&ctx->tlist, sizeof(int) * tiles));
  ctx->tiles_cap = tiles;
  return SLHJB_OK;
}

}  // namespace

namespace slhjb {
// accessors for the other translation units of the library (network entry points)
hipStream_t ctx_stream(slhjb_ctx* ctx) { return ctx->stream; }
int ctx_device(slhjb_ctx* ctx) { return ctx->device; }
int ctx_fail(slhjb_ctx* ctx, int status, const std::string& msg) { return fail(ctx, status, msg); }
int ctx_hip_fail(slhjb_ctx* ctx, hipError_t e, const char* what) { return hip_fail(ctx, e, what); }
int ctx_validate(slhjb_ctx* ctx, const slhjb_problem* p) { return validate(ctx, p); }
}  // namespace slhjb

namespace {
// Jacobi value iteration from v (device, overwritten) with `other` as the second iterate buffer,
// `dw` as the device residual / flag words and `hw` as their host mirror.
int jacobi_run(slhjb_ctx* ctx, const slhjb_problem* problem, const Prepared& P, float* v, float* other,
               unsigned* dw, unsigned* hw, double tol, int64_t max_sweeps, int32_t check_every, slhjb_stats* stats) {
  const int64_t N = (int64_t)problem->n * problem->n;
  if (check_every == 0) check_every = N >= (1 << 20) ? 8 : 16;

  HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  // the caller's array holds w during the iteration
  HIP_TRY(ctx, launch_v_to_w(v, v, problem->node_class, N, P.vstar, P.args.w_target, P.args.w_obstacle, ctx->stream));
  float* cur = v;
  float* nxt = other;
  int64_t sweeps = 0, converged = -1;
  double resid = INFINITY, sweep_sec = 0.0;
  int status = SLHJB_NOT_CONVERGED;
  while (sweeps < max_sweeps) {
    const int64_t batch = std::min<int64_t>(check_every, max_sweeps - sweeps);
    HIP_TRY(ctx, launch_fill_u32(dw, 0u, 2, ctx->stream));
    HIP_TRY(ctx, hipEventRecord(ctx->eva, ctx->stream));
    for (int64_t b = 0; b < batch; ++b) {
      SweepArgs a = P.args;
      a.w_in = cur;
      a.w_out = nxt;
      a.resid = b == batch - 1 ? dw : nullptr;
      HIP_TRY(ctx, launch_sweep(a, P.diffusion, P.scheme, P.path, ctx->stream));
      std::swap(cur, nxt);
    }
    sweeps += batch;
    HIP_TRY(ctx, hipEventRecord(ctx->evb, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(hw, dw, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    float bms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&bms, ctx->eva, ctx->evb));
    sweep_sec += bms * 1e-3;
    float r;
    memcpy(&r, &hw[0], sizeof(float));
    resid = r;
    if (hw[1] & 1u) {
      status = SLHJB_E_NONFINITE;
      break;
    }
    if (resid <= tol) {
      converged = sweeps;
      status = SLHJB_OK;
      break;
    }
  }
  if (cur != v) HIP_TRY(ctx, hipMemcpyAsync(v, cur, sizeof(float) * N, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(ctx, launch_w_to_v(v, v, N, P.vstar, ctx->stream));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev1));
  float ms = 0.0f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  if (stats) {
    stats->sweeps = sweeps;
    stats->converged_sweep = converged;
    stats->node_updates = sweeps * P.free_nodes;
    stats->residual = resid;
    stats->seconds = ms * 1e-3;
    stats->sweep_seconds = sweep_sec;
    stats->sweep_launches = sweeps;
    stats->status = status;
    stats->kernel_path = P.path;
    stats->halo = P.args.halo;
    stats->pad = 0;
    stats->policy_updates = 0;
    stats->check_sweeps = 0;
    stats->check_seconds = 0.0;
  }
  if (status == SLHJB_E_NONFINITE) return fail(ctx, status, "sweep produced a non-finite value");
  return status;
}

}  // namespace

extern "C" {

const char* slhjb_status_string(int status) {
  switch (status) {
  case SLHJB_OK: return "ok";
  case SLHJB_NOT_CONVERGED: return "not converged (valid iterate returned)";
  case SLHJB_E_INVALID_ARG: return "invalid argument";
  case SLHJB_E_UNSUPPORTED: return "unsupported configuration";
  case SLHJB_E_HIP: return "HIP runtime error";
  case SLHJB_E_NOMEM: return "out of device memory";
  case SLHJB_E_NONFINITE: return "non-finite value in the iterate";
  default: return "unknown status";
  }
}

int slhjb_version(void) { return 4; }

#ifndef SLHJB_SOURCE_HASH
#define SLHJB_SOURCE_HASH "unknown"
#endif
const char* slhjb_source_hash(void) { return SLHJB_SOURCE_HASH; }

int slhjb_ctx_create(slhjb_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return SLHJB_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return SLHJB_E_INVALID_ARG;
  slhjb_ctx* ctx = new (std::nothrow) slhjb_ctx();
  if (!ctx) return SLHJB_E_NOMEM;
  ctx->device = hip_device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(hip_device) != hipSuccess || hipEventCreate(&ctx->ev0) != hipSuccess ||
      hipEventCreate(&ctx->ev1) != hipSuccess || hipEventCreate(&ctx->eva) != hipSuccess ||
      hipEventCreate(&ctx->evb) != hipSuccess ||
      hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess) {
    slhjb_ctx_destroy(ctx);
    return SLHJB_E_HIP;
  }
  *out = ctx;
  return SLHJB_OK;
}

int slhjb_ctx_destroy(slhjb_ctx* ctx) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  else hipDeviceSynchronize();
  if (ctx->buf) hipFree(ctx->buf);
  if (ctx->uhat) hipFree(ctx->uhat);
  for (auto* b : ctx->vbuf)
    if (b) hipFree(b);
  if (ctx->small) hipFree(ctx->small);
  if (ctx->small_host) hipHostFree(ctx->small_host);
  if (ctx->ctrl) hipFree(ctx->ctrl);
  if (ctx->ctrl2) hipFree(ctx->ctrl2);
  if (ctx->phi) hipFree(ctx->phi);
  if (ctx->tflag) hipFree(ctx->tflag);
  if (ctx->tlist) hipFree(ctx->tlist);
  if (ctx->tcount) hipFree(ctx->tcount);
  if (ctx->tcount_host) hipHostFree(ctx->tcount_host);
  if (ctx->tkey) hipFree(ctx->tkey);
  if (ctx->tchange) hipFree(ctx->tchange);
  if (ctx->coop) hipFree(ctx->coop);
  if (ctx->tctl) hipFree(ctx->tctl);
  if (ctx->tchk_host) hipHostFree(ctx->tchk_host);
  if (ctx->pipe_vc) hipFree(ctx->pipe_vc);
  if (ctx->pipe_ctrl) hipFree(ctx->pipe_ctrl);
  if (ctx->pipe_lab) hipFree(ctx->pipe_lab);
  if (ctx->tacc) hipFree(ctx->tacc);
  if (ctx->lctl) hipFree(ctx->lctl);
  if (ctx->lctl_host) hipHostFree(ctx->lctl_host);
  if (ctx->lctl_host2) hipHostFree(ctx->lctl_host2);
  if (ctx->tctl_host) hipHostFree(ctx->tctl_host);
  if (ctx->tctl_host2) hipHostFree(ctx->tctl_host2);
  for (auto& e : ctx->tdone)
    if (e) hipEventDestroy(e);
  ctx->tile_graphs.clear();
  ctx->label_graphs.clear();
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  if (ctx->lcap_stream) hipStreamDestroy(ctx->lcap_stream);
  for (auto& e : ctx->ldone)
    if (e) hipEventDestroy(e);
  if (ctx->aux_stream) hipStreamDestroy(ctx->aux_stream);
  if (ctx->lflag) hipFree(ctx->lflag);
  if (ctx->llist) hipFree(ctx->llist);
  if (ctx->lkey) hipFree(ctx->lkey);
  if (ctx->lctab) hipFree(ctx->lctab);
  if (ctx->lmask) hipFree(ctx->lmask);
  for (auto& e : ctx->tev)
    if (e) hipEventDestroy(e);
  if (ctx->coop_host) hipHostFree(ctx->coop_host);
  if (ctx->ev0) hipEventDestroy(ctx->ev0);
  if (ctx->ev1) hipEventDestroy(ctx->ev1);
  if (ctx->eva) hipEventDestroy(ctx->eva);
  if (ctx->evb) hipEventDestroy(ctx->evb);
  delete ctx;
  return SLHJB_OK;
}

int slhjb_last_hip_error(const slhjb_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

const char* slhjb_last_error_message(const slhjb_ctx* ctx) { return ctx ? ctx->last_msg.c_str() : ""; }

int slhjb_sweep(slhjb_ctx* ctx, const slhjb_problem* problem, const float* v_in, float* v_out,
                double* residual_host) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!v_in || !v_out || v_in == v_out) return fail(ctx, SLHJB_E_INVALID_ARG, "v_in and v_out must be distinct non-NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Prepared P;
  int st = prepare(ctx, problem, &P);
  if (st != SLHJB_OK) return st;
  const int64_t N = (int64_t)problem->n * problem->n;
  st = ensure_buf(ctx, &ctx->vbuf[0], &ctx->vbuf_elems, (size_t)N);
  if (st != SLHJB_OK) return st;
  if (!ctx->vbuf[1] || ctx->vbuf_elems < (size_t)N) {
    if (ctx->vbuf[1]) hipFree(ctx->vbuf[1]);
    ctx->vbuf[1] = nullptr;
    hipError_t e = hipMalloc(&ctx->vbuf[1], sizeof(float) * ctx->vbuf_elems);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
  }
  HIP_TRY(ctx, launch_fill_u32(ctx->small, 0u, 2, ctx->stream));
  HIP_TRY(ctx, launch_v_to_w(v_in, ctx->vbuf[0], problem->node_class, N, P.vstar, P.args.w_target,
                             P.args.w_obstacle, ctx->stream));
  SweepArgs a = P.args;
  a.w_in = ctx->vbuf[0];
  a.w_out = ctx->vbuf[1];
  a.resid = ctx->small;
  HIP_TRY(ctx, launch_sweep(a, P.diffusion, P.scheme, P.path, ctx->stream));
  HIP_TRY(ctx, launch_w_to_v(ctx->vbuf[1], v_out, N, P.vstar, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->small_host, ctx->small, sizeof(unsigned) * 2, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->small_host[1] & 1u) return fail(ctx, SLHJB_E_NONFINITE, "sweep produced a non-finite value");
  if (residual_host) {
    float r;
    memcpy(&r, &ctx->small_host[0], sizeof(float));
    *residual_host = r;
  }
  return SLHJB_OK;
}

int slhjb_solve(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_sweeps,
                int32_t check_every, slhjb_stats* stats) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!v) return fail(ctx, SLHJB_E_INVALID_ARG, "v is NULL");
  if (!(tol >= 0.0) || max_sweeps < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol >= 0 and max_sweeps >= 1");
  if (check_every < 0 || check_every > 256) return fail(ctx, SLHJB_E_INVALID_ARG, "check_every must be in [0, 256]");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Prepared P;
  int st = prepare(ctx, problem, &P);
  if (st != SLHJB_OK) return st;
  const int64_t N = (int64_t)problem->n * problem->n;
  st = ensure_buf(ctx, &ctx->buf, &ctx->buf_elems, (size_t)N);
  if (st != SLHJB_OK) return st;
  return jacobi_run(ctx, problem, P, v, ctx->buf, ctx->small, ctx->small_host, tol, max_sweeps, check_every, stats);
}

}  // extern "C"

// ---- the Jacobi solve without allocation ---------------------------------------------------------
// Scratch of slhjb_solve_noalloc in a file-scope device array, one copy per device: the second
// iterate (up to kNoAllocMaxNodes nodes), the padded control table and the residual / statistics
// words. Host code reaches it only through the address hipGetSymbolAddress returns for the device.
namespace {
constexpr int64_t kNoAllocMaxNodes = (int64_t)SLHJB_NOALLOC_MAX_N * SLHJB_NOALLOC_MAX_N;
constexpr size_t kNoAllocIterBytes = ((sizeof(float) * kNoAllocMaxNodes + 255) / 256) * 256;
constexpr size_t kNoAllocCtrlBytes = ((sizeof(float4) * kCtrlCap + 255) / 256) * 256;
constexpr size_t kNoAllocWordBytes = 256;
constexpr size_t kNoAllocBytes = kNoAllocIterBytes + kNoAllocCtrlBytes + kNoAllocWordBytes;
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kNoAllocMaxDevices] = {};
}  // namespace

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// The device address of `scratch` on `device` (which must be current), looked up once per device.
hipError_t noalloc_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}
}  // namespace

extern "C" {

int slhjb_solve_noalloc(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_sweeps,
                        int32_t check_every, slhjb_stats* stats) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!v) return fail(ctx, SLHJB_E_INVALID_ARG, "v is NULL");
  if (!(tol >= 0.0) || max_sweeps < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol >= 0 and max_sweeps >= 1");
  if (check_every < 0 || check_every > 256) return fail(ctx, SLHJB_E_INVALID_ARG, "check_every must be in [0, 256]");
  if (problem && (int64_t)problem->n * problem->n > kNoAllocMaxNodes)
    return fail(ctx, SLHJB_E_INVALID_ARG,
                "slhjb_solve_noalloc takes grids of at most " + std::to_string(SLHJB_NOALLOC_MAX_N) + "^2 nodes");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  unsigned char* base = nullptr;
  HIP_TRY(ctx, noalloc_scratch(ctx->device, &base));
  float* other = reinterpret_cast<float*>(base);
  float4* ctrl = reinterpret_cast<float4*>(base + kNoAllocIterBytes);
  unsigned* words = reinterpret_cast<unsigned*>(base + kNoAllocIterBytes + kNoAllocCtrlBytes);
  unsigned host_words[kSmallWords] = {};
  Prepared P;
  int st = prepare_with(ctx, problem, &P, PrepMem{words, host_words, ctrl, nullptr});
  if (st != SLHJB_OK) return st;
  return jacobi_run(ctx, problem, P, v, other, words, host_words, tol, max_sweeps, check_every, stats);
}

}  // extern "C"



namespace {

// Everything one run of the labeler needs, decided and validated beforehand; the run itself only
// enqueues on its stream and reads the pass state back.
struct LabelJob {
  int n = 0, Ppad = 2, n_patches = 1, tiles_x = 0;
  const int16_t* ctrl = nullptr;
  const float* v_hat = nullptr;
  const int16_t* source_patch = nullptr;
  const uint8_t* cls = nullptr;
  const float* speed = nullptr;
  float speed_const = 1.0f, r = 0.0f, vstar = 1.0f, lambda = 1.0f, window = INFINITY;
  uint16_t tau = 0;
  int16_t* label_out = nullptr;
  uint64_t* overlap_out = nullptr;
  uint16_t* phi_out = nullptr;
  // scratch
  uint32_t* phi = nullptr;
  uint8_t* flag = nullptr;
  int* list = nullptr;
  float* key = nullptr;
  void* lctl = nullptr;
  unsigned* lctl_host = nullptr;
  unsigned* lctl_host2 = nullptr;
  const float2* ctab = nullptr;
  unsigned* wmask = nullptr;
  bool keys_ready = false;  // the caller already computed the u_hat keys into `key`
  GraphCache* graphs = nullptr;  // the context's labeler graphs, capture stream and events
  hipStream_t cap = nullptr;
  hipEvent_t* done = nullptr;
};

// Validation and parameters of a labeling of `problem` (after prepare(): speed bounds in
// small_host), the phi scratch and the pass state; the tile buffers are the caller's choice.
int label_setup(slhjb_ctx* ctx, const slhjb_problem* problem, const Prepared& P, const int16_t* ctrl,
                const float* v_hat, const int16_t* source_patch, int32_t n_patches, uint16_t tau_q15,
                int16_t* label_out, uint64_t* overlap_out, uint16_t* phi_out, LabelJob* J) {
  if (!ctrl || !source_patch || !label_out) return fail(ctx, SLHJB_E_INVALID_ARG, "ctrl, source_patch, label_out must be non-NULL");
  if (problem->drift) return fail(ctx, SLHJB_E_UNSUPPORTED, "patch labels take no drift");
  if (problem->control_cost) return fail(ctx, SLHJB_E_UNSUPPORTED, "patch labels take no control cost");
  if (n_patches < 1 || n_patches > 64) return fail(ctx, SLHJB_E_INVALID_ARG, "n_patches must be in [1, 64]");
  if (tau_q15 > (1u << 15)) return fail(ctx, SLHJB_E_INVALID_ARG, "tau_q15 must be <= 2^15");
  // the labeler advects along sigma = 0 feet, which must lie in the first ring of cells
  slhjb_problem p0 = *problem;
  p0.diffusion = SLHJB_DIFF_NONE;
  const float speed_max = P.speed_max;
  if (reach_for(&p0, speed_max, 0.0) > 1.0 + 1e-6)
    return fail(ctx, SLHJB_E_UNSUPPORTED, "patch labeling needs h c |a| <= dx (feet in the first ring of cells)");
  const int n = problem->n;
  const int64_t N = (int64_t)n * n;
  int Ppad = 2;
  while (Ppad < n_patches) Ppad *= 2;
  const size_t words = (size_t)N * (Ppad / 2);
  if (ctx->phi_words < words) {
    if (ctx->phi) hipFree(ctx->phi);
    ctx->phi = nullptr;
    ctx->phi_words = 0;
    hipError_t e = hipMalloc(&ctx->phi, sizeof(uint32_t) * words);
    if (e == hipErrorOutOfMemory) return fail(ctx, SLHJB_E_NOMEM, "labeler scratch allocation failed");
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
    ctx->phi_words = words;
  }
  if (!ctx->lctl) {
    HIP_TRY(ctx, hipMalloc(&ctx->lctl, labctl_bytes()));
    HIP_TRY(ctx, hipHostMalloc(&ctx->lctl_host, 64, hipHostMallocDefault));
    HIP_TRY(ctx, hipHostMalloc(&ctx->lctl_host2, 64, hipHostMallocDefault));
  }
  const int ltx = (n + kLabelTile - 1) / kLabelTile;
  if (ctx->lmask_cap < (size_t)ltx * ltx) {
    if (ctx->lmask) hipFree(ctx->lmask);
    ctx->lmask = nullptr;
    ctx->lmask_cap = 0;
    HIP_TRY(ctx, hipMalloc(&ctx->lmask, sizeof(unsigned) * ltx * ltx));
    ctx->lmask_cap = (size_t)ltx * ltx;
  }
  J->wmask = ctx->lmask;
  J->n = n;
  J->Ppad = Ppad;
  J->n_patches = n_patches;
  J->tiles_x = (n + kLabelTile - 1) / kLabelTile;
  J->ctrl = ctrl;
  J->v_hat = v_hat;
  J->source_patch = source_patch;
  J->cls = problem->node_class;
  J->speed = problem->speed;
  J->speed_const = problem->speed_const;
  J->r = P.args.r;
  J->vstar = P.vstar;
  J->lambda = problem->lambda;
  J->window = v_hat ? (float)(std::max(16.0, (n - 1) / 16.0) * grid_dx(problem) / speed_max) : INFINITY;
  J->tau = tau_q15;
  J->label_out = label_out;
  J->overlap_out = overlap_out;
  J->phi_out = phi_out;
  J->phi = ctx->phi;
  J->lctl = ctx->lctl;
  J->lctl_host = ctx->lctl_host;
  J->lctl_host2 = ctx->lctl_host2;
  if (!ctx->lcap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->lcap_stream, hipStreamNonBlocking));
  if (!ctx->ldone[0]) {
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ldone[0], hipEventDisableTiming));
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->ldone[1], hipEventDisableTiming));
  }
  J->graphs = &ctx->label_graphs;
  J->cap = ctx->lcap_stream;
  J->done = ctx->ldone;
  return SLHJB_OK;
}

// Enqueue the labeling on stream s and run its pass loop (host reads of the pass state every 16
// passes) to the end. Touches only the job's buffers. Returns hipSuccess or the first error, and
// a status for a labeler that did not settle.
hipError_t label_run(const LabelJob& J, hipStream_t s, int64_t* passes_out, int* status) {
  *status = SLHJB_OK;
  const int n = J.n;
  const int64_t N = (int64_t)n * n;
  const int tiles = J.tiles_x * J.tiles_x;
  hipError_t e = launch_label_init(J.cls, J.source_patch, N, J.Ppad, J.phi, s);
  if (e == hipSuccess) e = launch_label_mask_init(J.cls, J.source_patch, n, J.tiles_x, J.wmask, s);
  if (e == hipSuccess) e = launch_fill_u8(J.flag, 1, tiles, s);
  if (e == hipSuccess) e = launch_labctl_init(J.lctl, s);
  if (e == hipSuccess && J.v_hat && !J.keys_ready)
    e = launch_label_keys(J.v_hat, J.cls, n, J.tiles_x, J.tiles_x, J.vstar, J.lambda, J.key, s);
  if (e != hipSuccess) return e;
  const int grid = std::min(tiles, 1024);
  // sweeps per visit: 2 kLabelTile (the 2049^2 labels: 9.7 ms, against 10.3 ms at 4 kLabelTile
  // and 10.9 ms at kLabelTile)
  const int max_inner = 2 * kLabelTile;
  // The iteration is monotone and bounded, so it stops; fields that are far from causal (random
  // ones) can creep for thousands of passes. The cap only guards against a broken invariant.
  const int64_t max_passes = 4000000;
  // 16 passes captured in a graph (kept in the context's cache); two replays in flight, so the GPU
  // never waits for the host's check of the pass state (a replay after the end is all no-ops)
  const float* keyp = J.v_hat ? J.key : nullptr;
  GraphKey gk;
  gk.add(J.phi).add(J.cls).add(J.ctrl).add(J.speed).add(J.speed_const).add(J.ctab).add(J.r).add(n).add(J.Ppad)
      .add(keyp).add(J.list).add(J.tiles_x).add(J.flag).add(J.wmask).add(max_inner).add(J.window).add(J.lctl)
      .add(grid);
  hipGraphExec_t exec = J.graphs->find(gk);
  if (!exec) {
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(J.cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ce = hipSuccess;
      for (int b = 0; b < 16 && ce == hipSuccess; ++b)
        ce = launch_label_pass2(J.phi, J.cls, J.ctrl, J.speed, J.speed_const, J.ctab, J.r, n, J.Ppad, keyp, J.list,
                                J.tiles_x, J.tiles_x, J.flag, J.wmask, max_inner, J.window, b & 1, J.lctl, grid, J.cap);
      e = hipStreamEndCapture(J.cap, &graph);
      if (ce != hipSuccess) e = ce;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    J.graphs->insert(std::move(gk), exec);
  }
  hipEvent_t* ev = J.done;
  unsigned* hb[2] = {J.lctl_host, J.lctl_host2};
  auto replay = [&](int k) -> hipError_t {
    hipError_t r = hipGraphLaunch(exec, s);
    if (r == hipSuccess) r = hipMemcpyAsync(hb[k & 1], J.lctl, labctl_bytes(), hipMemcpyDeviceToHost, s);
    if (r == hipSuccess) r = hipEventRecord(ev[k & 1], s);
    return r;
  };
  if (e == hipSuccess) e = replay(0);
  for (int k = 0; e == hipSuccess; ++k) {
    e = replay(k + 1);
    if (e == hipSuccess) e = hipEventSynchronize(ev[k & 1]);
    if (e != hipSuccess) break;
    if (hb[k & 1][7]) break;  // done
    if ((int64_t)(k + 1) * 16 > max_passes) {
      *status = SLHJB_E_HIP;
      break;
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(J.lctl_host, J.lctl, labctl_bytes(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || *status != SLHJB_OK) return e;
  *passes_out = J.lctl_host[8];
  e = launch_label_argmax((const uint16_t*)J.phi, N, J.Ppad, J.label_out, J.overlap_out, J.tau, s);
  if (e == hipSuccess && J.phi_out) e = launch_label_phi_out(J.phi, N, J.n_patches, J.phi_out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

int solve_tiles_impl(slhjb_ctx* ctx, const slhjb_problem* problem, const Prepared& P, float* v, double tol,
                     int64_t max_passes, const slhjb_tile_opts* opts, slhjb_stats* stats);

}  // namespace

extern "C" {

int slhjb_solve_patchy(slhjb_ctx* ctx, const slhjb_problem* fine, const slhjb_problem* coarse,
                       const slhjb_patchy_opts* opts, float* v, int16_t* label_out, slhjb_patchy_stats* stats) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!fine || !opts || !v) return fail(ctx, SLHJB_E_INVALID_ARG, "fine, opts and v must be non-NULL");
  if (opts->mode < 0 || opts->mode > 2) return fail(ctx, SLHJB_E_INVALID_ARG, "unknown patchy mode");
  if (!(opts->tol > 0.0) || opts->max_passes < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol > 0, max_passes >= 1");
  if (opts->policy_sweeps < 0 || opts->policy_sweeps > 64)
    return fail(ctx, SLHJB_E_INVALID_ARG, "policy_sweeps must be in [0, 64]");
  const bool pdd = opts->mode != SLHJB_PATCHY_STATIC;
  const bool need_labels = opts->mode == SLHJB_PATCHY_INDEPENDENT || label_out;
  if (pdd && need_labels && fine->control_cost)
    return fail(ctx, SLHJB_E_UNSUPPORTED, "patch labels take no control cost (transmission mode without labels does)");
  if (pdd && need_labels && fine->drift)
    return fail(ctx, SLHJB_E_UNSUPPORTED, "patch labels take no drift (transmission mode without labels does)");
  if (pdd) {
    if (!coarse) return fail(ctx, SLHJB_E_INVALID_ARG, "the patchy modes need a coarse problem");
    if (coarse->x_lo != fine->x_lo || coarse->x_hi != fine->x_hi)
      return fail(ctx, SLHJB_E_INVALID_ARG, "coarse and fine grids must cover the same box");
    if (!(opts->tol_coarse > 0.0)) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol_coarse > 0");
    if (need_labels && (!opts->source_patch || opts->n_patches < 1))
      return fail(ctx, SLHJB_E_INVALID_ARG, "labels need source_patch and n_patches >= 1");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int n = fine->n;
  const int64_t N = (int64_t)n * n;
  slhjb_patchy_stats S;
  memset(&S, 0, sizeof(S));
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  auto lap = [&](double* slot) -> hipError_t {
    hipError_t er = hipEventRecord(e1, ctx->stream);
    if (er != hipSuccess) return er;
    er = hipEventSynchronize(e1);
    if (er != hipSuccess) return er;
    float ms = 0.0f;
    er = hipEventElapsedTime(&ms, e0, e1);
    if (er != hipSuccess) return er;
    *slot = ms * 1e-3;
    return hipEventRecord(e0, ctx->stream);
  };
  int st = SLHJB_OK;
  hipError_t he = hipEventRecord(e0, ctx->stream);
  hipEvent_t t0 = nullptr;
  if (he == hipSuccess) he = hipEventCreate(&t0);
  if (he == hipSuccess) he = hipEventRecord(t0, ctx->stream);
  slhjb_tile_opts to;
  memset(&to, 0, sizeof(to));
  to.tile_shape = opts->tile_shape;
  to.key_slack = opts->key_window;
  to.collect_kernel_time = opts->collect_kernel_time;
  to.policy_sweeps = opts->policy_sweeps;
  slhjb_stats ts;
  int16_t* ctrl = nullptr;
  float* vc = nullptr;
  int16_t* lab = label_out;
  // In the transmission mode the fine solve does not read the labels: the labeler then runs on a
  // stream of its own, in a host thread of its own, beside the fine solve (buffers of its own:
  // phi, tile flags / list / keys, pass state and control table).
  const bool overlap_labels = pdd && need_labels && opts->mode == SLHJB_PATCHY_TRANSMISSION;
  std::thread labeler;
  int64_t lab_passes = 0;
  int lab_status = SLHJB_OK;
  hipError_t lab_err = hipSuccess;
  double lab_seconds = 0.0, syn_seconds = 0.0;
  LabelJob J;
  // Overlapped labels: u_hat is copied, the fine problem prepared once, and the labeler stream
  // gets the synthesis, the keys and the labeling of the copy while the fine solve overwrites v.
  auto start_labels = [&](const Prepared& Pf) -> int {
    int r = ensure_buf(ctx, &ctx->uhat, &ctx->uhat_elems, (size_t)N);
    if (r != SLHJB_OK) return r;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->uhat, v, sizeof(float) * N, hipMemcpyDeviceToDevice, ctx->stream));
    r = label_setup(ctx, fine, Pf, ctrl, ctx->uhat, opts->source_patch, opts->n_patches, 0, lab, nullptr, nullptr, &J);
    if (r != SLHJB_OK) return r;
    const size_t tiles = (size_t)J.tiles_x * J.tiles_x;
    if (ctx->ltiles_cap < tiles) {
      if (ctx->lflag) hipFree(ctx->lflag);
      if (ctx->llist) hipFree(ctx->llist);
      if (ctx->lkey) hipFree(ctx->lkey);
      ctx->lflag = nullptr;
      ctx->llist = nullptr;
      ctx->lkey = nullptr;
      ctx->ltiles_cap = 0;
      HIP_TRY(ctx, hipMalloc(&ctx->lflag, tiles));
      HIP_TRY(ctx, hipMalloc(&ctx->llist, sizeof(int) * tiles));
      HIP_TRY(ctx, hipMalloc(&ctx->lkey, sizeof(float) * tiles));
      ctx->ltiles_cap = tiles;
    }
    if (!ctx->lctab) HIP_TRY(ctx, hipMalloc(&ctx->lctab, sizeof(float2) * 256));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->lctab, fine->controls, sizeof(float2) * fine->n_controls, hipMemcpyHostToDevice,
                                ctx->stream));
    J.flag = ctx->lflag;
    J.list = ctx->llist;
    J.key = ctx->lkey;
    J.ctab = ctx->lctab;
    J.keys_ready = false;  // computed on the labeler stream, from the copy
    if (!ctx->aux_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux_stream, hipStreamNonBlocking));
    HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux_stream, e1, 0));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the host control array is pageable
    const int dev = ctx->device;
    hipStream_t aux = ctx->aux_stream;
    const float r_h = Pf.args.r;
    labeler = std::thread([&J, aux, dev, fine, ctrl, r_h, &lab_passes, &lab_status, &lab_err, &lab_seconds,
                           &syn_seconds]() {
      hipError_t e = hipSetDevice(dev);
      hipEvent_t a = nullptr, m = nullptr, b = nullptr;
      if (e == hipSuccess) e = hipEventCreate(&a);
      if (e == hipSuccess) e = hipEventCreate(&m);
      if (e == hipSuccess) e = hipEventCreate(&b);
      if (e == hipSuccess) e = hipEventRecord(a, aux);
      if (e == hipSuccess)
        e = launch_synthesize(J.v_hat, fine->speed, fine->node_class, J.ctab, fine->n_controls, fine->n, r_h,
                              fine->speed_const, fine->v_out, ctrl, aux);
      if (e == hipSuccess) e = hipEventRecord(m, aux);
      if (e == hipSuccess) e = label_run(J, aux, &lab_passes, &lab_status);
      if (e == hipSuccess) e = hipEventRecord(b, aux);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, m);
      syn_seconds = ms * 1e-3;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, m, b);
      lab_seconds = ms * 1e-3;
      if (a) hipEventDestroy(a);
      if (m) hipEventDestroy(m);
      if (b) hipEventDestroy(b);
      lab_err = e;
    });
    return SLHJB_OK;
  };
  if (he != hipSuccess) {
    st = hip_fail(ctx, he, "event");
  } else if (pdd) {
    // (1) coarse solve with sigma = 0, from v = 1 (the Kruzkov "+infinity")
    const int64_t Nc = (int64_t)coarse->n * coarse->n;
    // context-owned scratch, grown only when a larger problem comes: a repeated solve allocates
    // nothing (and its cached pass graphs, keyed by these addresses, stay valid)
    st = ensure_pipe(ctx, (size_t)Nc, (size_t)N);
    if (st == SLHJB_OK) {
      vc = ctx->pipe_vc;
      ctrl = ctx->pipe_ctrl;
      if (need_labels && !lab) lab = ctx->pipe_lab;
    }
    if (st == SLHJB_OK) {
      // start value V* on every node; the solver overwrites TARGET and OBSTACLE nodes
      const float vstar = cold_start_value(coarse);
      unsigned bits;
      memcpy(&bits, &vstar, sizeof(bits));
      he = launch_fill_u32((unsigned*)vc, bits, (int)Nc, ctx->stream);
      if (he != hipSuccess) st = hip_fail(ctx, he, "coarse start");
    }
    if (st == SLHJB_OK) {
      slhjb_problem pc = *coarse;
      pc.diffusion = SLHJB_DIFF_NONE;
      pc.eps = 0.0f;
      slhjb_tile_opts co;
      memset(&co, 0, sizeof(co));
      co.tile_shape = 2;
      co.policy_sweeps = opts->policy_sweeps;
      // the 129^2 coarse solve's best visit length: with policy evaluation 48 iterations (3 (tw + th)
      // of the 8 x 8 tiles) take 0.98-1.05 ms, 32 take 1.12-1.15 ms, 64 1.13 ms, 96 1.25 ms;
      // without it 2 (tw + th)
      co.max_inner = opts->policy_sweeps > 0 ? 48 : 32;
      // A sigma = 0 coarse problem settles within a few passes per tile row; the cap bounds a
      // coarse solve whose tolerance lies below what its FP32 iterate can resolve (the general
      // kernels, taken with a drift, settle into changes of a few 1e-7).
      const int64_t coarse_passes = std::min<int64_t>(opts->max_passes, 16 * (int64_t)coarse->n);
      st = slhjb_solve_tiles(ctx, &pc, vc, opts->tol_coarse, coarse_passes, &co, &ts);
      if (st == SLHJB_NOT_CONVERGED) st = SLHJB_OK;  // a rough coarse solution is still a valid start
      S.coarse_passes = ts.sweeps;
      S.node_updates_coarse = ts.node_updates;
    }
    if (st == SLHJB_OK && (he = lap(&S.t_coarse)) != hipSuccess) st = hip_fail(ctx, he, "event");
    // (2) u_hat on the fine grid
    if (st == SLHJB_OK) st = slhjb_upsample(ctx, coarse->n, vc, n, v);
    if (st == SLHJB_OK && (he = lap(&S.t_upsample)) != hipSuccess) st = hip_fail(ctx, he, "event");
    // the fine problem, prepared once for the synthesis, the labels and the solve (after the
    // coarse solve, which loaded the coarse problem's control table)
    Prepared Pf;
    if (st == SLHJB_OK) st = prepare(ctx, fine, &Pf);
    // (3) synthesis of the control and (4) patch labels
    if (st == SLHJB_OK && need_labels && !overlap_labels) {
      he = launch_synthesize(v, fine->speed, fine->node_class, ctx->ctrl2, fine->n_controls, n, Pf.args.r,
                             fine->speed_const, fine->v_out, ctrl, ctx->stream);
      if (he != hipSuccess) st = hip_fail(ctx, he, "synthesis");
      if (st == SLHJB_OK && (he = lap(&S.t_synthesize)) != hipSuccess) st = hip_fail(ctx, he, "event");
      if (st == SLHJB_OK) {
        int64_t lp = 0;
        st = slhjb_label(ctx, fine, ctrl, v, opts->source_patch, opts->n_patches, 0, lab, nullptr, nullptr, &lp);
        S.label_passes = lp;
        if (st == SLHJB_OK && (he = lap(&S.t_label)) != hipSuccess) st = hip_fail(ctx, he, "event");
      }
      // slhjb_label prepared the problem again: same tables, same statistics
    }
    if (st == SLHJB_OK && overlap_labels) st = start_labels(Pf);
    // (5) computation: tiles by increasing u_hat, from u_hat
    if (st == SLHJB_OK) {
      to.order = SLHJB_ORDER_KEYS;
      to.mode = opts->mode == SLHJB_PATCHY_INDEPENDENT ? SLHJB_MODE_INDEPENDENT : SLHJB_MODE_TRANSMISSION;
      to.label = opts->mode == SLHJB_PATCHY_INDEPENDENT ? lab : nullptr;
      st = solve_tiles_impl(ctx, fine, Pf, v, opts->tol, opts->max_passes, &to, &ts);
    }
    if (labeler.joinable()) {
      labeler.join();
      S.label_passes = lab_passes;
      S.t_label = lab_seconds;
      S.t_synthesize = syn_seconds;
      if (lab_err != hipSuccess && st == SLHJB_OK) st = hip_fail(ctx, lab_err, "patch labels");
      else if (lab_status != SLHJB_OK && st == SLHJB_OK) st = fail(ctx, lab_status, "labeler did not settle (internal error)");
    }
  } else {
    // static decomposition: no pre-computation, tiles in their fixed order, from v = 1
    const float vstar = cold_start_value(fine);
    unsigned bits;
    memcpy(&bits, &vstar, sizeof(bits));
    he = launch_fill_u32((unsigned*)v, bits, (int)N, ctx->stream);
    if (he != hipSuccess) st = hip_fail(ctx, he, "static start");
    if (st == SLHJB_OK && (he = lap(&S.t_coarse)) != hipSuccess) st = hip_fail(ctx, he, "event");
    if (st == SLHJB_OK) {
      to.order = SLHJB_ORDER_NONE;
      to.mode = SLHJB_MODE_TRANSMISSION;
      // from the cold start, in a fixed order, longer visits pay (2049^2: 20.3 ms at 2 (tw + th)
      // against 21.3 ms at tw + th)
      if (!(fine->eps > 0.0f && fine->diffusion != SLHJB_DIFF_NONE)) {
        const TileShape sh = tile_shape_of(opts->tile_shape);
        to.max_inner = 2 * (sh.tw + sh.th);
      }
      st = slhjb_solve_tiles(ctx, fine, v, opts->tol, opts->max_passes, &to, &ts);
    }
  }
  if (st == SLHJB_OK || st == SLHJB_NOT_CONVERGED) {
    S.passes = ts.sweeps;
    S.check_sweeps = ts.check_sweeps;
    S.t_check_visit = ts.check_seconds;
    S.node_updates = ts.node_updates;
    S.policy_updates = ts.policy_updates;
    S.residual = ts.residual;
    S.t_solve = ts.seconds;
    S.t_visit = ts.sweep_seconds;
    float ms = 0.0f;
    hipEventRecord(e1, ctx->stream);
    hipEventSynchronize(e1);
    hipEventElapsedTime(&ms, t0, e1);
    S.t_total = ms * 1e-3;
  }
  S.status = st;
  if (stats) *stats = S;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (t0) hipEventDestroy(t0);
  return st;
}

int slhjb_upsample(slhjb_ctx* ctx, int32_t n_c, const float* v_c, int32_t n_f, float* v_f) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (n_c < 3 || n_f < 3 || n_c > 32769 || n_f > 32769 || !v_c || !v_f)
    return fail(ctx, SLHJB_E_INVALID_ARG, "need 3 <= n_c, n_f <= 32769 and non-NULL arrays");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_upsample(v_c, n_c, v_f, n_f, ctx->stream));
  return SLHJB_OK;
}

int slhjb_upsample_bicubic(slhjb_ctx* ctx, int32_t n_c, const float* v_c, int32_t n_f, float* v_f) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (n_c < 3 || n_f < 3 || n_c > 32769 || n_f > 32769 || !v_c || !v_f)
    return fail(ctx, SLHJB_E_INVALID_ARG, "need 3 <= n_c, n_f <= 32769 and non-NULL arrays");
  if (v_c == v_f) return fail(ctx, SLHJB_E_INVALID_ARG, "v_c and v_f must be distinct");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, launch_upsample_bicubic(v_c, n_c, v_f, n_f, ctx->stream));
  return SLHJB_OK;
}

int slhjb_synthesize(slhjb_ctx* ctx, const slhjb_problem* problem, const float* v_hat, int16_t* ctrl_out) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!v_hat || !ctrl_out) return fail(ctx, SLHJB_E_INVALID_ARG, "v_hat and ctrl_out must be non-NULL");
  if (problem && problem->drift) return fail(ctx, SLHJB_E_UNSUPPORTED, "the synthesis takes no drift");
  if (problem && problem->control_cost) return fail(ctx, SLHJB_E_UNSUPPORTED, "the synthesis takes no control cost");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Prepared P;
  int st = prepare(ctx, problem, &P);
  if (st != SLHJB_OK) return st;
  HIP_TRY(ctx, launch_synthesize(v_hat, problem->speed, problem->node_class, ctx->ctrl2, problem->n_controls,
                                 problem->n, P.args.r, problem->speed_const, problem->v_out, ctrl_out, ctx->stream));
  return SLHJB_OK;
}

int slhjb_label(slhjb_ctx* ctx, const slhjb_problem* problem, const int16_t* ctrl, const float* v_hat,
                const int16_t* source_patch, int32_t n_patches, uint16_t tau_q15, int16_t* label_out,
                uint64_t* overlap_out, uint16_t* phi_out, int64_t* passes_out) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Prepared P;
  int st = prepare(ctx, problem, &P);
  if (st != SLHJB_OK) return st;
  LabelJob J;
  st = label_setup(ctx, problem, P, ctrl, v_hat, source_patch, n_patches, tau_q15, label_out, overlap_out, phi_out, &J);
  if (st != SLHJB_OK) return st;
  const int tiles = J.tiles_x * J.tiles_x;
  st = ensure_tiles(ctx, (size_t)tiles);
  if (st != SLHJB_OK) return st;
  if (v_hat && ctx->stiles_cap < (size_t)tiles) {
    if (ctx->tkey) hipFree(ctx->tkey);
    if (ctx->tchange) hipFree(ctx->tchange);
    ctx->tkey = ctx->tchange = nullptr;
    ctx->stiles_cap = 0;
    HIP_TRY(ctx, hipMalloc(&ctx->tkey, sizeof(float) * tiles));
    HIP_TRY(ctx, hipMalloc(&ctx->tchange, 2 * sizeof(float) * tiles));  // moves, then sides
    ctx->stiles_cap = tiles;
  }
  J.flag = ctx->tflag;
  J.list = ctx->tlist;
  J.key = ctx->tkey;
  J.ctab = ctx->ctrl2;
  int64_t passes = 0;
  int lst = SLHJB_OK;
  HIP_TRY(ctx, label_run(J, ctx->stream, &passes, &lst));
  if (lst != SLHJB_OK) return fail(ctx, lst, "labeler did not settle (internal error)");
  if (passes_out) *passes_out = passes;
  return SLHJB_OK;
}

}  // extern "C"

namespace {

// The tile solver on a problem already prepared (validated, its statistics read back and its
// control table on the device): the pipeline prepares each problem once.
int solve_tiles_impl(slhjb_ctx* ctx, const slhjb_problem* problem, const Prepared& P, float* v, double tol,
                     int64_t max_passes, const slhjb_tile_opts* opts, slhjb_stats* stats) {
  int st = SLHJB_OK;
  const int n = problem->n;
  const int64_t N = (int64_t)n * n;
  const int shape = opts->tile_shape;
  const TileShape sh = tile_shape_of(shape);
  const int tw = sh.tw, th = sh.th;
  const int tiles_x = (n + tw - 1) / tw, tiles_y = (n + th - 1) / th;
  const int tiles = tiles_x * tiles_y;
  st = ensure_buf(ctx, &ctx->buf, &ctx->buf_elems, (size_t)tiles * tw * th);
  if (st != SLHJB_OK) return st;
  st = ensure_tiles(ctx, (size_t)tiles);
  if (st != SLHJB_OK) return st;
  if (ctx->stiles_cap < (size_t)tiles) {
    if (ctx->tkey) hipFree(ctx->tkey);
    if (ctx->tchange) hipFree(ctx->tchange);
    ctx->tkey = ctx->tchange = nullptr;
    ctx->stiles_cap = 0;
    HIP_TRY(ctx, hipMalloc(&ctx->tkey, sizeof(float) * tiles));
    HIP_TRY(ctx, hipMalloc(&ctx->tchange, 2 * sizeof(float) * tiles));  // moves, then sides
    ctx->stiles_cap = tiles;
  }
  const bool indep = opts->mode == SLHJB_MODE_INDEPENDENT;
  if (P.path == 2 && (indep || opts->persistent))
    return fail(ctx, SLHJB_E_UNSUPPORTED,
                "varying costs, lambda = 0 or an eps field: transmission mode with the host-driven passes only");
  const bool keyed = opts->order == SLHJB_ORDER_KEYS;
  // Without diffusion a tile is a transport problem: iterating it to its own fixed point against
  // the frozen halo carries the values across it in one visit. With diffusion every node depends
  // on the halo through the noise feet and a settled tile is settled only once its neighbours are:
  // a few iterations per visit waste the least work.
  // (with policy-evaluation iterations: one full iteration and the policy sweeps per visit; without
  // diffusion they carry values along too, and tw + th iterations per visit do: the 2049^2
  // sigma = 0 fine solve takes 11.2 ms at tw + th against 12.0 ms at 2 (tw + th))
  const int max_inner = opts->max_inner > 0
                            ? opts->max_inner
                            : (P.diffusion == SLHJB_DIFF_NONE
                                   ? (opts->policy_sweeps > 0 ? tw + th : 2 * (tw + th))
                                   : (opts->policy_sweeps > 0 ? opts->policy_sweeps + 1 : 2));
  const float tol_inner = (float)(0.5 * tol), act = (float)(0.5 * tol);
  // band width of arrival times: the time to cross 1/16 of the box (at least 16 cells) at the
  // fastest speed
  const float window = opts->key_slack >= 0.0f
                           ? opts->key_slack
                           : (float)(std::max(16.0, (n - 1) / 16.0) * grid_dx(problem) / P.speed_max);
  // Three workgroups per CU: the band passes of the 2049^2 solves select up to several hundred
  // tiles, and workgroups beyond the selected count only read the pass words and leave; 2048
  // of them (the occupancy limit) made the 2049^2 patchy step 1.5% slower, 512 3.5% slower.
  const int grid = std::min(tiles, 3 * std::max(1, ctx->cus));
  const size_t lds = tile_pass_lds_bytes(sh, P.args.halo, indep);
  if (lds > 64 * 1024) return fail(ctx, SLHJB_E_UNSUPPORTED, "interpolation halo too large for the tile solver");

  HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  HIP_TRY(ctx, launch_v_to_w(v, v, problem->node_class, N, P.vstar, P.args.w_target, P.args.w_obstacle, ctx->stream));
  if (keyed)
    HIP_TRY(ctx, launch_tile_keys(v, problem->node_class, tw, th, n, tiles_x, tiles_y, P.vstar, problem->lambda,
                                  ctx->tkey, ctx->stream));
  HIP_TRY(ctx, launch_fill_u8(ctx->tflag, 1, tiles, ctx->stream));
  HIP_TRY(ctx, launch_fill_u32((unsigned*)ctx->tcount + 2, 0xff800000u, 1, ctx->stream));  // band bound -inf
  HIP_TRY(ctx, launch_fill_u32((unsigned*)ctx->tcount + 3, 0u, 1, ctx->stream));           // passes with work
  SweepArgs a = P.args;
  a.w_in = v;
  int64_t passes = 0, converged = -1;
  double resid = INFINITY;
  int status = SLHJB_NOT_CONVERGED;
  int64_t updates = 0, pe_updates = 0, checks = -1;
  double visit_sec = 0.0, check_sec = 0.0;
  if (opts->persistent) {
    if (!ctx->coop) {
      HIP_TRY(ctx, hipMalloc(&ctx->coop, coop_state_bytes()));
      HIP_TRY(ctx, hipHostMalloc(&ctx->coop_host, 64, hipHostMallocDefault));
    }
    HIP_TRY(ctx, launch_coop_state_init(ctx->coop, ctx->stream));
    const int mp = (int)std::min<int64_t>(max_passes, 1 << 30);
    int grid_used = 0;
    HIP_TRY(ctx, launch_tile_solve_coop(a, shape, P.diffusion, P.scheme, P.path, indep, opts->label,
                                        keyed ? ctx->tkey : nullptr, ctx->tlist, tiles_x, tiles_y, ctx->buf,
                                        ctx->tchange, ctx->tflag, max_inner, tol_inner, act, window, (float)tol, mp,
                                        ctx->coop, opts->max_workgroups > 0 ? opts->max_workgroups : 1024, &grid_used,
                                        opts->policy_sweeps, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->coop_host, ctx->coop, coop_state_bytes(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const unsigned* cs = ctx->coop_host;
    float r;
    memcpy(&r, &cs[3], sizeof(float));
    passes = cs[4];
    resid = cs[5] == 1 ? (double)r : (r > 0.0f ? (double)r : INFINITY);
    if (cs[5] == 1) {
      status = SLHJB_OK;
      converged = passes;
    }
    unsigned long long u, pu;
    memcpy(&u, &cs[6], sizeof(u));
    memcpy(&pu, &cs[8], sizeof(pu));
    updates = (int64_t)u;
    pe_updates = (int64_t)pu;
  }
  if (!opts->persistent) {
    // device-driven passes, captured once into a graph of kBatch passes and replayed; on small
    // grids a pass takes ~17 us and the no-op passes of the replays in flight after convergence
    // are a tenth of the solve, so their graphs hold fewer passes (129^2 coarse solve 1.13 ->
    // 1.08 ms at 8; the 2049^2 solve is faster at 16)
    const int kBatch = tiles <= 1024 ? 8 : 16;
    if (!ctx->tctl) {
      HIP_TRY(ctx, hipMalloc(&ctx->tctl, tilectl_bytes()));
      HIP_TRY(ctx, hipHostMalloc(&ctx->tctl_host, kTileCtlHostBytes, hipHostMallocDefault));
      // grid <= 3 * cus (above)
      HIP_TRY(ctx, hipMalloc(&ctx->tacc, sizeof(unsigned long long) * 2 * 3 * std::max(1, ctx->cus)));
    }
    if (!ctx->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_TRY(ctx, launch_tilectl_init(ctx->tctl, ctx->stream));
    HIP_TRY(ctx, launch_fill_u32((unsigned*)ctx->tacc, 0u, 4 * grid, ctx->stream));
    // the passes' second array is the staging buffer (tiles * tw * th >= n * n floats) and the
    // tile words the first `tiles` words of tchange; every tile starts in v
    unsigned* tile_word = reinterpret_cast<unsigned*>(ctx->tchange);
    HIP_TRY(ctx, launch_fill_u32(tile_word, 0u, tiles, ctx->stream));
    const bool timing = opts->collect_kernel_time != 0;
    if (timing && !ctx->tev[0])
      for (auto& e : ctx->tev) HIP_TRY(ctx, hipEventCreate(&e));
    if (timing && !ctx->tchk_host) HIP_TRY(ctx, hipHostMalloc(&ctx->tchk_host, sizeof(unsigned) * 16, hipHostMallocDefault));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // With kernel timing the same passes are launched directly on the context stream with events
    // around every visit launch (events recorded inside a captured graph cannot be timed).
    // With events, the check-sweep count (word 11) is copied after every pass, so that the host
    // can tell which timed visit launches were check sweeps.
    auto enqueue_batch = [&](hipStream_t s, bool ev) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int b = 0; b < kBatch && e == hipSuccess; ++b) {
        e = launch_tilectl_pass(a, shape, P.diffusion, P.scheme, P.path, indep, opts->label,
                                keyed ? ctx->tkey : nullptr, ctx->tlist, tiles_x, tiles_y, ctx->buf, tile_word,
                                ctx->tflag, max_inner, tol_inner, act, window, (float)tol, b & 1, ctx->tctl, grid,
                                ev ? ctx->tev[2 * b] : nullptr, ev ? ctx->tev[2 * b + 1] : nullptr,
                                opts->policy_sweeps, ctx->tacc, s);
        if (ev && e == hipSuccess)
          e = hipMemcpyAsync(ctx->tchk_host + b, static_cast<unsigned*>(ctx->tctl) + 11, sizeof(unsigned),
                             hipMemcpyDeviceToHost, s);
      }
      return e;
    };
    if (!timing) {
      // every argument of the captured launches (the parity and the events are fixed per position)
      GraphKey gk;
      gk.add(a).add(shape).add(P.diffusion).add(P.scheme).add(P.path).add(indep).add(opts->label)
          .add(keyed ? ctx->tkey : nullptr).add(ctx->tlist).add(tiles_x).add(tiles_y).add(ctx->buf)
          .add(ctx->tchange).add(ctx->tflag).add(max_inner).add(tol_inner).add(act).add(window).add((float)tol)
          .add(ctx->tctl).add(grid).add(opts->policy_sweeps).add(ctx->tacc);
      exec = ctx->tile_graphs.find(gk);
      if (!exec) {
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t ce = enqueue_batch(ctx->cap_stream, false);
        hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (ce != hipSuccess) return hip_fail(ctx, ce, "capture of the tile passes");
        if (ee != hipSuccess) return hip_fail(ctx, ee, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        graph = nullptr;
        if (ie != hipSuccess) return hip_fail(ctx, ie, "hipGraphInstantiate");
        ctx->tile_graphs.insert(std::move(gk), exec);
      }
    }
    hipError_t le = hipSuccess;
    unsigned done = 0, dev_passes = 0;
    if (timing) {
      unsigned checks_seen = 0;
      while (true) {
        le = enqueue_batch(ctx->stream, true);
        if (le == hipSuccess)
          le = hipMemcpyAsync(ctx->tctl_host, ctx->tctl, tilectl_bytes(), hipMemcpyDeviceToHost, ctx->stream);
        if (le == hipSuccess) le = hipStreamSynchronize(ctx->stream);
        for (int b = 0; b < kBatch && le == hipSuccess; ++b) {
          float ms = 0.0f;
          le = hipEventElapsedTime(&ms, ctx->tev[2 * b], ctx->tev[2 * b + 1]);
          visit_sec += ms * 1e-3;
          if (ctx->tchk_host[b] != checks_seen) check_sec += ms * 1e-3;  // this pass was a check sweep
          checks_seen = ctx->tchk_host[b];
        }
        if (le != hipSuccess) break;
        done = ctx->tctl_host[9];
        dev_passes = ctx->tctl_host[10];
        if (done || (int64_t)dev_passes >= max_passes) break;
      }
    } else {
      // Two replays in flight: the host reads the state copied after replay k while replay k + 1
      // runs, so the GPU never waits for the host; a replay after convergence is all no-ops.
      if (!ctx->tctl_host2) HIP_TRY(ctx, hipHostMalloc(&ctx->tctl_host2, kTileCtlHostBytes, hipHostMallocDefault));
      if (!ctx->tdone[0]) {
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->tdone[0], hipEventDisableTiming));
        HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->tdone[1], hipEventDisableTiming));
      }
      unsigned* hb[2] = {ctx->tctl_host, ctx->tctl_host2};
      auto replay = [&](int k) -> hipError_t {
        hipError_t e = hipGraphLaunch(exec, ctx->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hb[k & 1], ctx->tctl, tilectl_bytes(), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipEventRecord(ctx->tdone[k & 1], ctx->stream);
        return e;
      };
      le = replay(0);
      for (int k = 0; le == hipSuccess; ++k) {
        le = replay(k + 1);
        if (le == hipSuccess) le = hipEventSynchronize(ctx->tdone[k & 1]);
        if (le != hipSuccess) break;
        if (hb[k & 1][9] || (int64_t)hb[k & 1][10] >= max_passes) break;
      }
    }
    // the state after everything that ran (a replay in flight included), with the update counts
    // of the visit workgroups summed into it; the tiles last written to the second array back in v
    if (le == hipSuccess) le = launch_tile_gather(v, ctx->buf, tile_word, n, shape, ctx->stream);
    if (le == hipSuccess) le = launch_tilectl_sum(ctx->tacc, grid, ctx->tctl, ctx->stream);
    if (le == hipSuccess)
      le = hipMemcpyAsync(ctx->tctl_host, ctx->tctl, tilectl_bytes(), hipMemcpyDeviceToHost, ctx->stream);
    if (le == hipSuccess) le = hipStreamSynchronize(ctx->stream);
    done = ctx->tctl_host[9];
    dev_passes = ctx->tctl_host[10];
    // the instantiated graph stays in the context's cache
    if (le != hipSuccess) return hip_fail(ctx, le, "tile pass graph");
    passes = dev_passes;
    float r;
    memcpy(&r, &ctx->tctl_host[7], sizeof(float));
    if (done) {
      status = SLHJB_OK;
      converged = passes;
      resid = r;
    }
    unsigned long long u, pu;
    memcpy(&u, &ctx->tctl_host[12], sizeof(u));
    memcpy(&pu, &ctx->tctl_host[14], sizeof(pu));
    updates = (int64_t)u;
    pe_updates = (int64_t)pu;
    checks = ctx->tctl_host[11];
  }
  HIP_TRY(ctx, launch_w_to_v(v, v, N, P.vstar, ctx->stream));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev1));
  float ms = 0.0f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->sweeps = passes;
    stats->converged_sweep = converged;
    stats->node_updates = updates;
    stats->residual = resid;
    stats->seconds = ms * 1e-3;
    stats->status = status;
    stats->kernel_path = P.path;
    stats->halo = P.args.halo;
    stats->sweep_seconds = visit_sec;
    stats->sweep_launches = visit_sec > 0.0 ? passes : 0;
    stats->policy_updates = pe_updates;
    stats->check_sweeps = checks;
    stats->check_seconds = check_sec;
  }
  return status;
}

}  // namespace

// A batched active-tile solve: per-instance parameters prepared once, device buffers, and the
// captured graph of kTilesBatchPasses passes (slhjb_tiles_batch_*).
constexpr int kTilesBatchPasses = 16;
struct slhjb_tiles_batch {
  slhjb_ctx* ctx = nullptr;
  int count = 0, shape = 0, pe = 0, total_tiles = 0, grid = 1;
  bool keyed = false;
  size_t lds = 0;
  std::vector<Prepared> prep;
  std::vector<int> tile0, tiles_x, tiles_y, max_inner, n;
  std::vector<float> window, lambda;
  std::vector<const uint8_t*> cls;
  std::vector<float*> v;
  float4* d_ctrl = nullptr;
  char* d_inst = nullptr;
  char* d_state = nullptr;
  void* d_ctl = nullptr;
  float *d_key = nullptr, *d_w2 = nullptr;  // d_w2: the instances' second arrays, instance i at tile0[i] * tw * th
  unsigned* d_word = nullptr;                // tile words, by global tile
  uint8_t* d_flag = nullptr;
  int *d_list = nullptr, *d_tile_inst = nullptr, *d_chk_inst = nullptr;
  unsigned* d_chk_off = nullptr;
  unsigned* h_ctl = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
void tiles_batch_free(slhjb_tiles_batch& b) {
  hipStreamSynchronize(b.ctx->stream);
  if (b.exec) hipGraphExecDestroy(b.exec);
  b.exec = nullptr;
  for (void* q : {(void*)b.d_ctrl, (void*)b.d_inst, (void*)b.d_state, b.d_ctl, (void*)b.d_key, (void*)b.d_word,
                  (void*)b.d_w2, (void*)b.d_flag, (void*)b.d_list, (void*)b.d_tile_inst, (void*)b.d_chk_inst,
                  (void*)b.d_chk_off})
    if (q) hipFree(q);
  b.d_ctrl = nullptr;
  b.d_inst = b.d_state = nullptr;
  b.d_ctl = nullptr;
  b.d_key = b.d_w2 = nullptr;
  b.d_word = nullptr;
  b.d_flag = nullptr;
  b.d_list = b.d_tile_inst = b.d_chk_inst = nullptr;
  b.d_chk_off = nullptr;
  if (b.h_ctl) hipHostFree(b.h_ctl);
  b.h_ctl = nullptr;
}
}  // namespace

extern "C" {

int slhjb_solve_tiles(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_passes,
                      const slhjb_tile_opts* opts, slhjb_stats* stats) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!v || !opts) return fail(ctx, SLHJB_E_INVALID_ARG, "v and opts must be non-NULL");
  if (!(tol > 0.0) || max_passes < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol > 0 and max_passes >= 1");
  if (opts->order < 0 || opts->order > 1 || opts->mode < 0 || opts->mode > 1 || opts->max_inner < 0 ||
      opts->tile_shape < 0 || opts->tile_shape >= kTileShapes || opts->persistent < 0 || opts->persistent > 1 ||
      opts->max_workgroups < 0 || opts->collect_kernel_time < 0 || opts->collect_kernel_time > 1 ||
      opts->policy_sweeps < 0 || opts->policy_sweeps > 64)
    return fail(ctx, SLHJB_E_INVALID_ARG, "invalid tile options");
  if (opts->mode == SLHJB_MODE_INDEPENDENT && !opts->label)
    return fail(ctx, SLHJB_E_INVALID_ARG, "independent mode needs patch labels");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Prepared P;
  const int st = prepare(ctx, problem, &P);
  if (st != SLHJB_OK) return st;
  return solve_tiles_impl(ctx, problem, P, v, tol, max_passes, opts, stats);
}

int slhjb_tiles_batch_create(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v,
                             const slhjb_tile_opts* opts, slhjb_tiles_batch** out) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!out) return fail(ctx, SLHJB_E_INVALID_ARG, "out must be non-NULL");
  *out = nullptr;
  if (!problems || !v || !opts || count < 1 || count > 4096)
    return fail(ctx, SLHJB_E_INVALID_ARG, "need problems, v, opts and 1 <= count <= 4096");
  if (opts->order < 0 || opts->order > 1 || opts->max_inner < 0 || opts->tile_shape < 0 ||
      opts->tile_shape >= kTileShapes || opts->policy_sweeps < 0 || opts->policy_sweeps > 64)
    return fail(ctx, SLHJB_E_INVALID_ARG, "invalid tile options");
  if (opts->mode != SLHJB_MODE_TRANSMISSION || opts->persistent != 0)
    return fail(ctx, SLHJB_E_UNSUPPORTED, "the batched active-tile solve runs the transmission mode, pass by pass");
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(ctx, SLHJB_E_INVALID_ARG, "v[" + std::to_string(i) + "] is NULL");
    if (problems[i].drift) return fail(ctx, SLHJB_E_UNSUPPORTED, "batched solves take no drift");
    if (has_general_terms(&problems[i]))
      return fail(ctx, SLHJB_E_UNSUPPORTED,
                  "batched solves take lambda > 0, a constant running cost and a constant eps");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  std::unique_ptr<slhjb_tiles_batch> B(new slhjb_tiles_batch());
  slhjb_tiles_batch& b = *B;
  b.ctx = ctx;
  b.count = count;
  b.shape = opts->tile_shape;
  b.keyed = opts->order == SLHJB_ORDER_KEYS;
  b.pe = opts->policy_sweeps;
  const TileShape sh = tile_shape_of(b.shape);
#define TB_TRY(expr)                                                                                         \
  do {                                                                                                       \
    hipError_t _e = (expr);                                                                                  \
    if (_e != hipSuccess) {                                                                                  \
      tiles_batch_free(b);                                                                                   \
      if (_e == hipErrorOutOfMemory) return fail(ctx, SLHJB_E_NOMEM, std::string(#expr) + ": out of device memory"); \
      return hip_fail(ctx, _e, #expr);                                                                       \
    }                                                                                                        \
  } while (0)
  TB_TRY(hipMalloc(&b.d_ctrl, sizeof(float4) * kCtrlCap * count));
  // per-instance parameters, exactly as slhjb_solve_tiles derives them
  b.prep.resize(count);
  b.tile0.resize(count);
  b.tiles_x.resize(count);
  b.tiles_y.resize(count);
  b.max_inner.resize(count);
  b.window.resize(count);
  b.n.resize(count);
  b.cls.resize(count);
  b.lambda.resize(count);
  b.v.assign(v, v + count);
  int max_tiles = 0;
  for (int i = 0; i < count; ++i) {
    const int st = prepare(ctx, &problems[i], &b.prep[i]);
    if (st != SLHJB_OK) {
      tiles_batch_free(b);
      ctx->last_msg = "instance " + std::to_string(i) + ": " + ctx->last_msg;
      return st;
    }
    const Prepared& P = b.prep[i];
    if (P.path != b.prep[0].path || P.diffusion != b.prep[0].diffusion || P.scheme != b.prep[0].scheme) {
      tiles_batch_free(b);
      return fail(ctx, SLHJB_E_UNSUPPORTED,
                  "all instances of a batched active-tile solve need the same scheme, diffusion kind and kernel path "
                  "(instance " + std::to_string(i) + " differs from instance 0)");
    }
    // prepare() leaves the instance's padded control table in ctx->ctrl (stream-ordered copy)
    TB_TRY(hipMemcpyAsync(b.d_ctrl + (size_t)kCtrlCap * i, ctx->ctrl, sizeof(float4) * P.args.n_controls,
                          hipMemcpyDeviceToDevice, ctx->stream));
    const int n = problems[i].n;
    b.n[i] = n;
    b.cls[i] = problems[i].node_class;
    b.lambda[i] = problems[i].lambda;
    b.tiles_x[i] = (n + sh.tw - 1) / sh.tw;
    b.tiles_y[i] = (n + sh.th - 1) / sh.th;
    b.tile0[i] = b.total_tiles;
    b.total_tiles += b.tiles_x[i] * b.tiles_y[i];
    max_tiles = std::max(max_tiles, b.tiles_x[i] * b.tiles_y[i]);
    b.max_inner[i] = opts->max_inner > 0 ? opts->max_inner
                                         : (P.diffusion == SLHJB_DIFF_NONE
                                                ? (b.pe > 0 ? sh.tw + sh.th : 2 * (sh.tw + sh.th))
                                                : (b.pe > 0 ? b.pe + 1 : 2));
    b.window[i] = opts->key_slack >= 0.0f
                      ? opts->key_slack
                      : (float)(std::max(16.0, (n - 1) / 16.0) * grid_dx(&problems[i]) / P.speed_max);
    b.lds = std::max(b.lds, tile_pass_lds_bytes(sh, P.args.halo, false));
  }
  if (b.lds > 64 * 1024) {
    tiles_batch_free(b);
    return fail(ctx, SLHJB_E_UNSUPPORTED, "interpolation halo too large for the tile solver");
  }
  const size_t tn = (size_t)sh.tw * sh.th;
  const int T = b.total_tiles;
  TB_TRY(hipMalloc(&b.d_inst, tb_inst_bytes() * count));
  TB_TRY(hipMalloc(&b.d_state, tb_state_bytes() * count));
  TB_TRY(hipMalloc(&b.d_ctl, tb_ctl_bytes()));
  TB_TRY(hipMalloc(&b.d_key, sizeof(float) * T));
  TB_TRY(hipMalloc(&b.d_word, sizeof(unsigned) * T));
  TB_TRY(hipMalloc(&b.d_w2, sizeof(float) * tn * T));  // instance i's tiles * tw * th >= n * n floats
  TB_TRY(hipMalloc(&b.d_flag, T));
  TB_TRY(hipMalloc(&b.d_list, sizeof(int) * T));
  TB_TRY(hipMalloc(&b.d_tile_inst, sizeof(int) * T));
  TB_TRY(hipMalloc(&b.d_chk_inst, sizeof(int) * count));
  TB_TRY(hipMalloc(&b.d_chk_off, sizeof(unsigned) * count));
  TB_TRY(hipHostMalloc(&b.h_ctl, 64, hipHostMallocDefault));
  std::vector<int> h_tile_inst(T);
  for (int i = 0; i < count; ++i)
    for (int t = 0; t < b.tiles_x[i] * b.tiles_y[i]; ++t) h_tile_inst[b.tile0[i] + t] = i;
  TB_TRY(hipMemcpyAsync(b.d_tile_inst, h_tile_inst.data(), sizeof(int) * T, hipMemcpyHostToDevice, ctx->stream));
  TB_TRY(hipStreamSynchronize(ctx->stream));  // the host vector is pageable
  // the passes: captured once; they read every per-call value (tolerances, max_passes) from the
  // descriptors, which run() rewrites
  b.grid = std::min(T, 3 * std::max(1, ctx->cus));
  const int max_chunks = (max_tiles + 1023) / 1024;
  if (!ctx->cap_stream) TB_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  TB_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t ce = hipSuccess;
  for (int p = 0; p < kTilesBatchPasses && ce == hipSuccess; ++p)
    ce = launch_tb_pass(b.shape, b.d_inst, b.d_state, count, max_chunks, b.d_flag, b.d_list, b.d_tile_inst,
                        b.d_chk_inst, b.d_chk_off, b.d_ctl, b.prep[0].diffusion, b.prep[0].scheme, b.prep[0].path,
                        p & 1, b.grid, b.lds, ctx->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (ce == hipSuccess && ee == hipSuccess) ce = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
  if (graph) hipGraphDestroy(graph);
  TB_TRY(ce != hipSuccess ? ce : ee);
#undef TB_TRY
  *out = B.release();
  return SLHJB_OK;
}

int slhjb_tiles_batch_run(slhjb_tiles_batch* b, double tol, int64_t max_passes, slhjb_stats* stats,
                          slhjb_batch_stats* total) {
  if (!b) return SLHJB_E_INVALID_ARG;
  slhjb_ctx* ctx = b->ctx;
  if (!(tol > 0.0) || max_passes < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol > 0 and max_passes >= 1");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int count = b->count;
  const TileShape sh = tile_shape_of(b->shape);
  const float act = (float)(0.5 * tol), tol_inner = (float)(0.5 * tol);
  std::vector<char> h_inst(tb_inst_bytes() * count);
  for (int i = 0; i < count; ++i) {
    SweepArgs a = b->prep[i].args;
    a.w_in = b->v[i];  // the iterate w = V* - v, in place as in the single-instance solve
    a.w_out = nullptr;
    a.resid = nullptr;
    a.flags = nullptr;
    a.ctrl = b->d_ctrl + (size_t)kCtrlCap * i;
    tb_fill_inst(h_inst.data() + tb_inst_bytes() * i, a, b->d_w2 + (size_t)b->tile0[i] * sh.tw * sh.th,
                 b->d_word + b->tile0[i], b->keyed ? b->d_key + b->tile0[i] : nullptr, b->tiles_x[i], b->tiles_y[i],
                 b->tile0[i], b->max_inner[i], b->pe, tol_inner, act, b->window[i], (float)tol,
                 (long long)max_passes);
  }
  HIP_TRY(ctx, hipMemcpyAsync(b->d_inst, h_inst.data(), h_inst.size(), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));  // the host vector is pageable
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  for (int i = 0; i < count; ++i) {
    const Prepared& P = b->prep[i];
    const int64_t N = (int64_t)b->n[i] * b->n[i];
    HIP_TRY(ctx, launch_v_to_w(b->v[i], b->v[i], b->cls[i], N, P.vstar, P.args.w_target, P.args.w_obstacle,
                               ctx->stream));
    if (b->keyed)
      HIP_TRY(ctx, launch_tile_keys(b->v[i], b->cls[i], sh.tw, sh.th, b->n[i], b->tiles_x[i], b->tiles_y[i], P.vstar,
                                    b->lambda[i], b->d_key + b->tile0[i], ctx->stream));
  }
  HIP_TRY(ctx, launch_fill_u8(b->d_flag, 1, b->total_tiles, ctx->stream));
  HIP_TRY(ctx, launch_fill_u32(b->d_word, 0u, b->total_tiles, ctx->stream));  // every tile starts in v
  HIP_TRY(ctx, launch_tb_init(b->d_state, count, b->d_ctl, ctx->stream));
  int64_t replays = 0;
  // every replay advances each instance still iterating by up to kTilesBatchPasses passes; an
  // instance stops after max_passes passes that did work (at most every other pass is a band
  // move that does none), so the loop ends
  while (true) {
    HIP_TRY(ctx, hipGraphLaunch(b->exec, ctx->stream));
    ++replays;
    HIP_TRY(ctx, hipMemcpyAsync(b->h_ctl, b->d_ctl, tb_ctl_bytes(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (b->h_ctl[kTBCtlActive] == 0u) break;
  }
  for (int i = 0; i < count; ++i) {
    // the tiles last written to the second array back in v, then v from w
    HIP_TRY(ctx, launch_tile_gather(b->v[i], b->d_w2 + (size_t)b->tile0[i] * sh.tw * sh.th, b->d_word + b->tile0[i],
                                    b->n[i], b->shape, ctx->stream));
    HIP_TRY(ctx, launch_w_to_v(b->v[i], b->v[i], (int64_t)b->n[i] * b->n[i], b->prep[i].vstar, ctx->stream));
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(ctx->ev1));
  float ms = 0.0f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  std::vector<char> h_state(tb_state_bytes() * count);
  HIP_TRY(ctx, hipMemcpy(h_state.data(), b->d_state, h_state.size(), hipMemcpyDeviceToHost));
  int status = SLHJB_OK, converged = 0;
  int64_t all_passes = 0, all_updates = 0;
  for (int i = 0; i < count; ++i) {
    TBResult r;
    tb_read_state(h_state.data(), i, &r);
    const int si = r.done ? SLHJB_OK : SLHJB_NOT_CONVERGED;
    if (si != SLHJB_OK) status = SLHJB_NOT_CONVERGED;
    converged += r.done ? 1 : 0;
    all_passes += r.passes;
    all_updates += (int64_t)r.updates;
    if (stats) {
      slhjb_stats& t = stats[i];
      memset(&t, 0, sizeof(t));
      t.sweeps = r.passes;
      t.converged_sweep = r.done ? (int64_t)r.passes : -1;
      t.node_updates = (int64_t)r.updates;
      t.residual = r.done ? (double)r.resid : INFINITY;
      t.seconds = ms * 1e-3;
      t.status = si;
      t.kernel_path = b->prep[i].path;
      t.halo = b->prep[i].args.halo;
      t.policy_updates = (int64_t)r.pe_updates;
      t.check_sweeps = r.checks;
    }
  }
  if (total) {
    memset(total, 0, sizeof(*total));
    total->sweeps = all_passes;
    total->node_updates = all_updates;
    total->replays = replays;
    total->seconds = ms * 1e-3;
    total->converged = converged;
    total->status = status;
  }
  return status;
}

int slhjb_tiles_batch_destroy(slhjb_tiles_batch* b) {
  if (!b) return SLHJB_E_INVALID_ARG;
  hipSetDevice(b->ctx->device);
  hipStreamSynchronize(b->ctx->stream);
  tiles_batch_free(*b);
  delete b;
  return SLHJB_OK;
}

int slhjb_solve_tiles_batch(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v,
                            double tol, int64_t max_passes, const slhjb_tile_opts* opts, slhjb_stats* stats,
                            slhjb_batch_stats* total) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!(tol > 0.0) || max_passes < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol > 0 and max_passes >= 1");
  slhjb_tiles_batch* b = nullptr;
  int st = slhjb_tiles_batch_create(ctx, problems, count, v, opts, &b);
  if (st != SLHJB_OK) return st;
  st = slhjb_tiles_batch_run(b, tol, max_passes, stats, total);
  slhjb_tiles_batch_destroy(b);
  return st;
}

int slhjb_solve_batch(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v, double tol,
                      int64_t max_sweeps, const slhjb_batch_opts* opts, slhjb_stats* stats,
                      slhjb_batch_stats* total) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!problems || !v || count < 1 || count > 4096)
    return fail(ctx, SLHJB_E_INVALID_ARG, "need problems, v and 1 <= count <= 4096");
  if (!(tol >= 0.0) || max_sweeps < 1) return fail(ctx, SLHJB_E_INVALID_ARG, "need tol >= 0 and max_sweeps >= 1");
  slhjb_batch_opts o;
  memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (o.check_every < 0 || o.check_every > 256 || o.batches_per_graph < 0 || o.batches_per_graph > 64 ||
      o.max_workgroups < 0)
    return fail(ctx, SLHJB_E_INVALID_ARG, "invalid batch options");
  const int check_every = o.check_every > 0 ? o.check_every : 16;
  const int per_graph = o.batches_per_graph > 0 ? o.batches_per_graph : 4;
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(ctx, SLHJB_E_INVALID_ARG, "v[" + std::to_string(i) + "] is NULL");
    if (o.tile_shapes && (o.tile_shapes[i] < 0 || o.tile_shapes[i] > 3))
      return fail(ctx, SLHJB_E_INVALID_ARG, "tile_shapes[" + std::to_string(i) + "] out of range");
    if (problems[i].scheme != problems[0].scheme)
      return fail(ctx, SLHJB_E_INVALID_ARG, "all instances of a batch must use the same scheme");
    if (problems[i].drift) return fail(ctx, SLHJB_E_UNSUPPORTED, "batched solves take no drift");
    if (has_general_terms(&problems[i]))
      return fail(ctx, SLHJB_E_UNSUPPORTED,
                  "batched solves take lambda > 0, a constant running cost and a constant eps");
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // device scratch of this call
  BatchInst* d_inst = nullptr;
  float4* d_ctrl = nullptr;
  float *pool0 = nullptr, *pool1 = nullptr, *d_last = nullptr;
  unsigned *d_resid = nullptr, *d_flags = nullptr;
  int *d_state = nullptr, *d_first = nullptr;
  long long* d_done = nullptr;
  int2* d_work = nullptr;
  void* d_ctl = nullptr;
  unsigned* h_ctl = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int status = SLHJB_OK;
  auto cleanup = [&]() {
    hipStreamSynchronize(ctx->stream);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    for (void* q : {(void*)d_inst, (void*)d_ctrl, (void*)pool0, (void*)pool1, (void*)d_last, (void*)d_resid,
                    (void*)d_flags, (void*)d_state, (void*)d_first, (void*)d_done, (void*)d_work, d_ctl})
      if (q) hipFree(q);
    if (h_ctl) hipHostFree(h_ctl);
  };
  auto bail = [&](hipError_t e, const char* what) {
    cleanup();
    if (e == hipErrorOutOfMemory) return fail(ctx, SLHJB_E_NOMEM, std::string(what) + ": out of device memory");
    return hip_fail(ctx, e, what);
  };
#define BATCH_TRY(expr)                       \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return bail(_e, #expr); \
  } while (0)
  BATCH_TRY(hipMalloc(&d_ctrl, sizeof(float4) * kCtrlCap * count));
  // per-instance parameters, exactly as the single-instance solve derives them
  std::vector<BatchInst> inst(count);
  std::vector<int> first_item(count);
  std::vector<float> vstar(count);
  long long nodes = 0;
  int ctrl_total = 0, items = 0;
  size_t lds = 0;
  for (int i = 0; i < count; ++i) {
    Prepared P;
    int st = prepare(ctx, &problems[i], &P);
    if (st != SLHJB_OK) {
      cleanup();
      ctx->last_msg = "instance " + std::to_string(i) + ": " + ctx->last_msg;
      return st;
    }
    // prepare() leaves the instance's padded control table in ctx->ctrl (stream-ordered copy)
    BATCH_TRY(hipMemcpyAsync(d_ctrl + ctrl_total, ctx->ctrl, sizeof(float4) * P.args.n_controls,
                             hipMemcpyDeviceToDevice, ctx->stream));
    BatchInst& b = inst[i];
    memset(&b, 0, sizeof(b));
    b.a = P.args;
    b.a.w_in = nullptr;
    b.a.w_out = nullptr;
    b.a.resid = nullptr;
    b.a.flags = nullptr;
    b.a.ctrl = nullptr;
    const int shape = o.tile_shapes ? o.tile_shapes[i] : SLHJB_BATCH_TILE_64x16;
    b.tw_log2 = (shape == SLHJB_BATCH_TILE_32x16 || shape == SLHJB_BATCH_TILE_32x8) ? 5 : 6;
    b.th = (shape == SLHJB_BATCH_TILE_64x8 || shape == SLHJB_BATCH_TILE_32x8) ? 8 : 16;
    const int n = problems[i].n, TW = 1 << b.tw_log2;
    b.tiles_x = (n + TW - 1) / TW;
    b.tiles = b.tiles_x * ((n + b.th - 1) / b.th);
    b.offset = nodes;
    nodes += ((long long)n * n + 63) / 64 * 64;
    b.free_nodes = P.free_nodes;
    b.path = P.path;
    b.diffusion = P.diffusion;
    b.ctrl_offset = ctrl_total;
    first_item[i] = items;
    items += b.tiles;
    vstar[i] = P.vstar;
    lds = std::max(lds, sizeof(float) * (size_t)(TW + 2 * P.args.halo) * (size_t)(b.th + 2 * P.args.halo));
    ctrl_total += P.args.n_controls;
  }
  BATCH_TRY(hipMalloc(&d_inst, sizeof(BatchInst) * count));
  BATCH_TRY(hipMalloc(&pool0, sizeof(float) * nodes));
  BATCH_TRY(hipMalloc(&pool1, sizeof(float) * nodes));
  BATCH_TRY(hipMalloc(&d_last, sizeof(float) * count));
  BATCH_TRY(hipMalloc(&d_resid, sizeof(unsigned) * count));
  BATCH_TRY(hipMalloc(&d_flags, sizeof(unsigned) * count));
  BATCH_TRY(hipMalloc(&d_state, sizeof(int) * count));
  BATCH_TRY(hipMalloc(&d_first, sizeof(int) * count));
  BATCH_TRY(hipMalloc(&d_done, sizeof(long long) * count));
  BATCH_TRY(hipMalloc(&d_work, sizeof(int2) * items));
  BATCH_TRY(hipMalloc(&d_ctl, batchctl_bytes()));
  BATCH_TRY(hipHostMalloc(&h_ctl, 128, hipHostMallocDefault));
  BATCH_TRY(hipMemcpyAsync(d_inst, inst.data(), sizeof(BatchInst) * count, hipMemcpyHostToDevice, ctx->stream));
  BATCH_TRY(hipMemcpyAsync(d_first, first_item.data(), sizeof(int) * count, hipMemcpyHostToDevice, ctx->stream));
  BATCH_TRY(hipStreamSynchronize(ctx->stream));  // the host vectors are pageable
  BATCH_TRY(hipEventRecord(ctx->ev0, ctx->stream));
  for (int i = 0; i < count; ++i) {
    const int64_t N = (int64_t)problems[i].n * problems[i].n;
    BATCH_TRY(launch_v_to_w(v[i], pool0 + inst[i].offset, problems[i].node_class, N, vstar[i], inst[i].a.w_target,
                            inst[i].a.w_obstacle, ctx->stream));
  }
  BATCH_TRY(launch_batch_init(d_inst, count, d_state, d_done, d_last, d_resid, d_flags, d_work, d_first, d_ctl,
                              (long long)max_sweeps, check_every, tol, (unsigned)items, ctx->stream));
  const int grid = std::min(items, o.max_workgroups > 0 ? o.max_workgroups : 4096);
  if (!ctx->cap_stream) BATCH_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  BATCH_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t ce = hipSuccess;
  for (int r = 0; r < per_graph && ce == hipSuccess; ++r)
    ce = launch_batch_round(d_inst, count, d_ctrl, pool0, pool1, d_resid, d_flags, d_state, d_done, d_last, d_work,
                            d_ctl, problems[0].scheme, check_every, grid, lds, ctx->cap_stream);
  hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (ce != hipSuccess) return bail(ce, "capture of the batched sweeps");
  if (ee != hipSuccess) return bail(ee, "hipStreamEndCapture");
  BATCH_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  int64_t replays = 0;
  while (true) {
    BATCH_TRY(hipGraphLaunch(exec, ctx->stream));
    ++replays;
    BATCH_TRY(hipMemcpyAsync(h_ctl, d_ctl, batchctl_bytes(), hipMemcpyDeviceToHost, ctx->stream));
    BATCH_TRY(hipStreamSynchronize(ctx->stream));
    if (h_ctl[kBatchCtlActive] == 0u) break;
  }
  // results: the iterate of an instance that stopped after S sweeps is in pool (S & 1)
  std::vector<int> state(count);
  std::vector<long long> done(count);
  std::vector<float> last(count);
  BATCH_TRY(hipMemcpy(state.data(), d_state, sizeof(int) * count, hipMemcpyDeviceToHost));
  BATCH_TRY(hipMemcpy(done.data(), d_done, sizeof(long long) * count, hipMemcpyDeviceToHost));
  BATCH_TRY(hipMemcpy(last.data(), d_last, sizeof(float) * count, hipMemcpyDeviceToHost));
  for (int i = 0; i < count; ++i) {
    const int64_t N = (int64_t)problems[i].n * problems[i].n;
    const float* src = ((done[i] & 1) ? pool1 : pool0) + inst[i].offset;
    BATCH_TRY(launch_w_to_v(src, v[i], N, vstar[i], ctx->stream));
  }
  BATCH_TRY(hipEventRecord(ctx->ev1, ctx->stream));
  BATCH_TRY(hipEventSynchronize(ctx->ev1));
  float ms = 0.0f;
  BATCH_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  int converged = 0;
  for (int i = 0; i < count; ++i) {
    const int si = state[i] == 1 ? SLHJB_OK : (state[i] == 3 ? SLHJB_E_NONFINITE : SLHJB_NOT_CONVERGED);
    converged += state[i] == 1 ? 1 : 0;
    if (si == SLHJB_E_NONFINITE) status = SLHJB_E_NONFINITE;
    else if (si == SLHJB_NOT_CONVERGED && status == SLHJB_OK) status = SLHJB_NOT_CONVERGED;
    if (stats) {
      slhjb_stats& t = stats[i];
      memset(&t, 0, sizeof(t));
      t.sweeps = done[i];
      t.converged_sweep = state[i] == 1 ? done[i] : -1;
      t.node_updates = done[i] * inst[i].free_nodes;
      t.residual = last[i];
      t.seconds = ms * 1e-3;
      t.status = si;
      t.kernel_path = inst[i].path;
      t.halo = inst[i].a.halo;
    }
  }
  if (total) {
    memset(total, 0, sizeof(*total));
    long long sw;
    unsigned long long u, tv;
    memcpy(&sw, &h_ctl[kBatchCtlSweeps], sizeof(sw));
    memcpy(&u, &h_ctl[kBatchCtlUpdates], sizeof(u));
    memcpy(&tv, &h_ctl[kBatchCtlTiles], sizeof(tv));
    total->sweeps = sw;
    total->node_updates = (int64_t)u;
    total->tiles_swept = (int64_t)tv;
    total->replays = replays;
    total->seconds = ms * 1e-3;
    total->converged = converged;
    total->status = status;
  }
  cleanup();
#undef BATCH_TRY
  if (status == SLHJB_E_NONFINITE) return fail(ctx, status, "an instance produced a non-finite value");
  return status;
}

}  // extern "C"

namespace {
// 4-connected TARGET components, numbered in raster order of their first node: comp[v] (-1 off
// the targets), node count and the sums of i and j of each
void target_components(int n, const uint8_t* node_class, std::vector<int32_t>& comp, std::vector<int64_t>& cnt,
                       std::vector<int64_t>& si, std::vector<int64_t>& sj) {
  const int64_t N = (int64_t)n * n;
  comp.assign(N, -1);
  cnt.clear();
  si.clear();
  sj.clear();
  std::vector<int64_t> stack;
  for (int64_t start = 0; start < N; ++start) {
    if (node_class[start] != SLHJB_TARGET || comp[start] >= 0) continue;
    const int32_t id = (int32_t)cnt.size();
    cnt.push_back(0);
    si.push_back(0);
    sj.push_back(0);
    comp[start] = id;
    stack.assign(1, start);
    while (!stack.empty()) {
      const int64_t v = stack.back();
      stack.pop_back();
      const int64_t i = v % n, j = v / n;
      cnt[id] += 1;
      si[id] += i;
      sj[id] += j;
      const int64_t nb[4] = {i > 0 ? v - 1 : -1, i < n - 1 ? v + 1 : -1, j > 0 ? v - n : -1, j < n - 1 ? v + n : -1};
      for (int64_t u : nb)
        if (u >= 0 && node_class[u] == SLHJB_TARGET && comp[u] < 0) {
          comp[u] = id;
          stack.push_back(u);
        }
    }
  }
}
}  // namespace

extern "C" {

int slhjb_partition_sources(int32_t n, const uint8_t* node_class, int32_t n_patches, int16_t* source_patch,
                            int32_t* n_targets_out) {
  if (n < 3 || n > 32769 || !node_class || !source_patch || n_patches < 1 || n_patches > 32767)
    return SLHJB_E_INVALID_ARG;
  const int64_t N = (int64_t)n * n;
  std::vector<int32_t> comp;
  std::vector<int64_t> cnt, si, sj;
  target_components(n, node_class, comp, cnt, si, sj);
  const int T = (int)cnt.size();
  if (n_targets_out) *n_targets_out = T;
  for (int64_t v = 0; v < N; ++v) source_patch[v] = -1;
  if (T == 0) return SLHJB_OK;
  if (n_patches < T) return SLHJB_E_INVALID_ARG;
  // one patch per target, the remaining n_patches - T apportioned by node count (largest remainder)
  int64_t total = 0;
  for (int t = 0; t < T; ++t) total += cnt[t];
  const int extra = n_patches - T;
  std::vector<int> share(T);
  std::vector<std::pair<double, int>> rem(T);
  int given = 0;
  for (int t = 0; t < T; ++t) {
    const double quota = (double)extra * (double)cnt[t] / (double)total;
    share[t] = (int)floor(quota);
    given += share[t];
    rem[t] = {quota - share[t], t};
  }
  std::stable_sort(rem.begin(), rem.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first > b.first;
  });
  for (int k = 0; k < extra - given; ++k) share[rem[k].second] += 1;
  std::vector<int> offset(T + 1, 0);
  for (int t = 0; t < T; ++t) offset[t + 1] = offset[t] + 1 + share[t];
  // within a target: equal angular sectors around its centroid, in grid units
  const double two_pi = 2.0 * M_PI;
  for (int64_t v = 0; v < N; ++v) {
    const int32_t t = comp[v];
    if (t < 0) continue;
    const int Pt = offset[t + 1] - offset[t];
    const double ci = (double)si[t] / (double)cnt[t], cj = (double)sj[t] / (double)cnt[t];
    const double th = atan2((double)(v / n) - cj, (double)(v % n) - ci);
    int sec = (int)floor((double)Pt * (th + M_PI) / two_pi);
    if (sec > Pt - 1) sec = Pt - 1;
    if (sec < 0) sec = 0;
    source_patch[v] = (int16_t)(offset[t] + sec);
  }
  return SLHJB_OK;
}

int slhjb_balance_sources(slhjb_ctx* ctx, const slhjb_problem* problem, const int16_t* ctrl, const float* v_hat,
                          int32_t n_patches, int32_t iterations, int16_t* source_patch, int64_t* sizes_out,
                          int16_t* label_out, int32_t* best_round_out) {
  if (!ctx) return SLHJB_E_INVALID_ARG;
  if (!problem || !ctrl || !source_patch)
    return fail(ctx, SLHJB_E_INVALID_ARG, "problem, ctrl and source_patch must be non-NULL");
  if (n_patches < 1 || n_patches > 64) return fail(ctx, SLHJB_E_INVALID_ARG, "n_patches must be in [1, 64]");
  if (iterations < 0 || iterations > 64) return fail(ctx, SLHJB_E_INVALID_ARG, "iterations must be in [0, 64]");
  const int st0 = validate(ctx, problem);
  if (st0 != SLHJB_OK) return st0;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int n = problem->n;
  const int64_t N = (int64_t)n * n;
  std::vector<uint8_t> cls(N);
  HIP_TRY(ctx, hipMemcpy(cls.data(), problem->node_class, N, hipMemcpyDeviceToHost));
  std::vector<int32_t> comp;
  std::vector<int64_t> cnt, si, sj;
  target_components(n, cls.data(), comp, cnt, si, sj);
  const int T = (int)cnt.size();
  if (T > n_patches) return fail(ctx, SLHJB_E_INVALID_ARG, "fewer patches than target components");
  // the sources of every component in angular order around its centroid, exactly: direction
  // (i cnt - sum_i, j cnt - sum_j) by half-plane and integer cross product (the order of atan2 on
  // (-pi, pi]), ties by node index
  std::vector<std::vector<int64_t>> nodes(T);
  for (int64_t v = 0; v < N; ++v)
    if (comp[v] >= 0) nodes[comp[v]].push_back(v);
  for (int t = 0; t < T; ++t) {
    const int64_t c = cnt[t], ci = si[t], cj = sj[t];
    auto half = [](int64_t dx, int64_t dy) { return dy < 0 ? 0 : (dy == 0 && dx >= 0 ? 1 : (dy > 0 ? 2 : 3)); };
    std::stable_sort(nodes[t].begin(), nodes[t].end(), [&](int64_t a, int64_t b) {
      const int64_t ax = (a % n) * c - ci, ay = (a / n) * c - cj;
      const int64_t bx = (b % n) * c - ci, by = (b / n) * c - cj;
      const int ha = half(ax, ay), hb = half(bx, by);
      if (ha != hb) return ha < hb;
      if (ha == 0 || ha == 2) {
        const __int128 cross = (__int128)ax * by - (__int128)ay * bx;
        if (cross != 0) return cross > 0;
      }
      return a < b;
    });
  }
  // the labels of every round go to a scratch buffer; those of the best round also to label_out
  int16_t* lab = nullptr;
  int16_t* own_lab = nullptr;
  HIP_TRY(ctx, hipMalloc(&own_lab, sizeof(int16_t) * N));
  lab = own_lab;
  std::vector<int16_t> src(N), labels(N), best_src;
  std::vector<int64_t> best_sizes;
  int best_round = -1;
  int status = SLHJB_OK;
  {
    hipError_t e = hipMemcpy(src.data(), source_patch, sizeof(int16_t) * N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      if (own_lab) hipFree(own_lab);
      return hip_fail(ctx, e, "balance: read-back");
    }
    for (int64_t v = 0; v < N; ++v)
      if ((cls[v] == SLHJB_TARGET) != (src[v] >= 0) || src[v] >= n_patches) {
        if (own_lab) hipFree(own_lab);
        return fail(ctx, SLHJB_E_INVALID_ARG,
                    "source_patch must give every TARGET node a patch in [0, n_patches) and -1 elsewhere");
      }
  }
  for (int k = 0; k <= iterations && status == SLHJB_OK; ++k) {
    status = slhjb_label(ctx, problem, ctrl, v_hat, source_patch, n_patches, 0, lab, nullptr, nullptr, nullptr);
    if (status != SLHJB_OK) break;
    hipError_t e = hipMemcpy(labels.data(), lab, sizeof(int16_t) * N, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(src.data(), source_patch, sizeof(int16_t) * N, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      status = hip_fail(ctx, e, "balance: read-back");
      break;
    }
    std::vector<int64_t> sizes(n_patches, 0), members(n_patches, 0);
    for (int64_t v = 0; v < N; ++v) {
      if (labels[v] >= 0 && labels[v] < n_patches) sizes[labels[v]] += 1;
      if (src[v] >= 0 && src[v] < n_patches) members[src[v]] += 1;
    }
    if (sizes_out) std::copy(sizes.begin(), sizes.end(), sizes_out + (int64_t)k * n_patches);
    // keep the best balanced subdivision: smaller largest-over-mean size, compared exactly
    // (max_k sum_best < max_best sum_k); the earliest on ties
    bool better = best_round < 0;
    if (!better) {
      int64_t mk = 0, sk = 0, mb = 0, sb = 0;
      for (int p = 0; p < n_patches; ++p) {
        mk = std::max(mk, sizes[p]);
        sk += sizes[p];
        mb = std::max(mb, best_sizes[p]);
        sb += best_sizes[p];
      }
      better = (__int128)mk * sb < (__int128)mb * sk;
    }
    if (better) {
      best_round = k;
      best_src = src;
      best_sizes = sizes;
      if (label_out) {
        e = hipMemcpy(label_out, lab, sizeof(int16_t) * N, hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
          status = hip_fail(ctx, e, "balance: labels");
          break;
        }
      }
    }
    if (k == iterations || T == 0) break;
    // patches per component by total size (one each, the rest by largest remainder)
    std::vector<int64_t> weight(T, 0);
    std::vector<int> seen(n_patches, 0);
    for (int64_t v = 0; v < N; ++v) {
      const int p = src[v];
      if (comp[v] >= 0 && p >= 0 && p < n_patches && !seen[p]) {
        seen[p] = 1;
        weight[comp[v]] += sizes[p];
      }
    }
    int64_t total = 0, total_cnt = 0;
    for (int t = 0; t < T; ++t) {
      total += weight[t];
      total_cnt += cnt[t];
    }
    const int extra = n_patches - T;
    std::vector<int> share(T);
    std::vector<std::pair<double, int>> rem(T);
    int given = 0;
    for (int t = 0; t < T; ++t) {
      const double quota = total > 0 ? (double)extra * (double)weight[t] / (double)total
                                     : (double)extra * (double)cnt[t] / (double)total_cnt;
      share[t] = (int)floor(quota);
      given += share[t];
      rem[t] = {quota - share[t], t};
    }
    std::stable_sort(rem.begin(), rem.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
      return a.first > b.first;
    });
    for (int q = 0; q < extra - given; ++q) share[rem[q].second] += 1;
    std::vector<int> offset(T + 1, 0);
    for (int t = 0; t < T; ++t) offset[t + 1] = offset[t] + 1 + share[t];
    // within a component: runs of equal total weight in angular order; a source's weight is its
    // patch's size shared out over the patch's sources
    std::vector<int16_t> next(N, (int16_t)-1);
    for (int t = 0; t < T; ++t) {
      const int Pt = offset[t + 1] - offset[t];
      const std::vector<int64_t>& nd = nodes[t];
      std::vector<double> w(nd.size());
      double wt = 0.0;
      for (size_t r = 0; r < nd.size(); ++r) {
        const int p = src[nd[r]];
        w[r] = (double)sizes[p] / (double)members[p];
        wt += w[r];
      }
      double cum = 0.0;
      for (size_t r = 0; r < nd.size(); ++r) {
        int64_t sec = wt > 0.0 ? (int64_t)floor((double)Pt * (cum + w[r] / 2) / wt)
                               : ((int64_t)Pt * (int64_t)r) / (int64_t)nd.size();
        sec = std::min<int64_t>(std::max<int64_t>(sec, 0), Pt - 1);
        next[nd[r]] = (int16_t)(offset[t] + sec);
        cum += w[r];
      }
    }
    e = hipMemcpy(source_patch, next.data(), sizeof(int16_t) * N, hipMemcpyHostToDevice);
    if (e != hipSuccess) status = hip_fail(ctx, e, "balance: upload");
  }
  if (status == SLHJB_OK && best_round >= 0) {
    const hipError_t e = hipMemcpy(source_patch, best_src.data(), sizeof(int16_t) * N, hipMemcpyHostToDevice);
    if (e != hipSuccess) status = hip_fail(ctx, e, "balance: upload");
  }
  if (best_round_out) *best_round_out = best_round;
  if (own_lab) hipFree(own_lab);
  return status;
}


int slhjb_regime_analyze(double f_min, double f_max, double sigma_inf, double dx, slhjb_regime* out) {
  if (!out || !(f_min > 0.0) || !(f_max >= f_min) || !(sigma_inf >= 0.0) || !(dx > 0.0) || !isfinite(f_max) ||
      !isfinite(sigma_inf) || !isfinite(dx))
    return SLHJB_E_INVALID_ARG;
  slhjb_regime r;
  memset(&r, 0, sizeof(r));
  r.upsilon = f_max / f_min;
  r.alpha_opt = 1.0 / (1.0 + r.upsilon);
  r.tau_dx = dx / (1.0 + r.upsilon);
  if (sigma_inf > 0.0) {
    r.omega = f_min / (sigma_inf * sigma_inf);
    const double od = r.omega * dx;
    r.alpha_lower = 1.0 / od;
    r.alpha_upper = 1.0 / r.upsilon - (sqrt(1.0 + 4.0 * od * r.upsilon) - 1.0) / (2.0 * od * r.upsilon * r.upsilon);
    r.hyperbolic = (1.0 / r.omega < r.tau_dx) ? 1 : 0;
  } else {
    r.omega = INFINITY;
    r.alpha_lower = 0.0;
    r.alpha_upper = 1.0 / r.upsilon;
    r.hyperbolic = 1;
  }
  r.h_alpha = r.alpha_opt * dx / f_min;
  // largest h with h f_max + sqrt(h) sigma_inf <= dx: a quadratic in sqrt(h)
  const double b = sigma_inf;
  const double sq = (-b + sqrt(b * b + 4.0 * f_max * dx)) / (2.0 * f_max);
  r.h_upper = sq * sq;
  *out = r;
  return SLHJB_OK;
}

double slhjb_foot_reach(const slhjb_problem* problem, float speed_max) {
  if (!problem || problem->n < 3 || !(problem->x_hi > problem->x_lo) || !problem->controls ||
      problem->n_controls < 1 || !(speed_max > 0.0f))
    return -1.0;
  slhjb_problem p = *problem;
  if (!(p.eps > 0.0f)) p.diffusion = SLHJB_DIFF_NONE;
  return reach_for(&p, speed_max, (double)p.eps);
}

}  // extern "C"
