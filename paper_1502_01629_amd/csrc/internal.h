// Internal declarations shared by the HIP kernels and the C-ABI host code of libslhjb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slhjb {

enum : int { kFree = 0, kTarget = 1, kObstacle = 2 };
enum : int { kDiffNone = 0, kDiffIso = 1, kDiffRank1 = 2 };
enum : int { kSL2 = 0, kSL3 = 1 };

// Tile of the sweep kernels: one wavefront spans 64 consecutive nodes of a row, four
// wavefronts per workgroup, each wavefront walks kTileH / 4 rows.
constexpr int kTileW = 64;
constexpr int kTileH = 16;
constexpr int kThreads = 256;
constexpr int kMaxHalo = 12;  // largest interpolation halo the general kernel accepts

// Per-control constants, precomputed on the host: (a_x, a_y, a_x a_y, |a_x| + |a_y|).
// The iterate is held as w = V* - v with V* = l / lambda, so that the update is the
// homogeneous w_i = beta max_a mean_feet I[w](y) (SL2) or its self-weight-free quotient (SL3).
struct SweepArgs {
  const float* w_in;
  float* w_out;
  const float* speed;      // nullable: speed_const then
  const uint8_t* cls;
  const float4* ctrl;      // [n_controls]
  unsigned* resid;         // nullable: float bits of max |w_out - w_in| over FREE nodes
  unsigned* flags;         // bit 0: non-finite value produced
  int n;
  int n_controls;
  int halo;                // interpolation halo radius of the LDS tile (cells)
  int quad[5];             // first-ring kernel: controls [quad[q], quad[q+1]) lie in quadrant q
  float r;                 // h / dx
  float speed_const;
  float d;                 // sqrt(2 eps h) / dx
  float beta;
  float w_outside;         // w at feet outside the closed box
  float w_target;
  float w_obstacle;
  const float2* drift;     // nullable: f(x,a) = c(x) (drift(x) + a), general kernels only
  // Varying costs and undiscounted problems (general kernels only). With the iterate w = C - v
  // the update of control a at node i subtracts q = qn_i + qa_a from the feet sum before the
  // quotient (SL3) or the max (SL2): qn_i = kq l_x(x_i) - kc with kq = (K / beta) fac,
  // kc = (K / beta) (1 - beta) C, fac = (1 - beta) / lambda (or h for lambda = 0), and
  // qa_a = kq l_a(a) in the .w component of the control table. cost == 0: q = 0 everywhere.
  int cost;
  const float* lx;         // nullable: l_x per node, else lconst
  float lconst;
  float kq, kc;
  const float* epsf;       // nullable: eps(x) per node; the noise offset is then sqrt(d2 eps(x))
  float d2;                // 2 h / dx^2
};

// Per-node parts of the general update: the cost term qn and the noise offset (cells).
__device__ __forceinline__ float node_cost(const SweepArgs& a, size_t idx) {
  if (!a.cost) return 0.0f;
  const float l = a.lx ? a.lx[idx] : a.lconst;
  return __builtin_fmaf(a.kq, l, -a.kc);
}
__device__ __forceinline__ float node_noise(const SweepArgs& a, size_t idx) {
  return a.epsf ? __builtin_sqrtf(a.d2 * a.epsf[idx]) : a.d;
}

// Launchers (sweep.hip). `path` 0 = general halo tile, 1 = first-ring register stencil.
hipError_t launch_sweep(const SweepArgs& a, int diffusion, int scheme, int path, hipStream_t s);
hipError_t launch_v_to_w(const float* v, float* w, const uint8_t* cls, int64_t count, float vstar,
                         float w_target, float w_obstacle, hipStream_t s);
hipError_t launch_w_to_v(const float* w, float* v, int64_t count, float vstar, hipStream_t s);
// out[0] min speed, [1] max speed (float bits), [2] bad speed, [3] FREE count, [4] bad class,
// [5] max over nodes of c |drift|_inf (float bits), [6] bad drift (drift may be NULL)
hipError_t launch_problem_stats(const float* speed, const uint8_t* cls, const float2* drift, float speed_const,
                                int64_t count, unsigned* out, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, unsigned value, int count, hipStream_t s);
// out[0]: max of f (float bits, f >= 0), out[1]: 1 if some value is non-finite, negative, or (with
// positive = 1) zero. The caller clears both words first.
hipError_t launch_field_stats(const float* f, int64_t count, int positive, unsigned* out, hipStream_t s);

// Pre-computation kernels (pipeline.hip).
hipError_t launch_upsample(const float* vc, int nc, float* vf, int nf, hipStream_t s);
hipError_t launch_upsample_bicubic(const float* vc, int nc, float* vf, int nf, hipStream_t s);
hipError_t launch_synthesize(const float* vhat, const float* speed, const uint8_t* cls, const float2* ctrl,
                             int n_controls, int n, float r, float speed_const, float v_out, int16_t* out,
                             hipStream_t s);
hipError_t launch_label_init(const uint8_t* cls, const int16_t* src, int64_t count, int P, uint32_t* phi32,
                             hipStream_t s);
size_t label_pass_lds_bytes(int P);
size_t labctl_bytes();
hipError_t launch_labctl_init(void* c, hipStream_t s);
hipError_t launch_label_keys(const float* vhat, const uint8_t* cls, int n, int tiles_x, int tiles_y, float vstar,
                             float lambda, float* key, hipStream_t s);
hipError_t launch_label_pass2(uint32_t* phi32, const uint8_t* cls, const int16_t* ctrl, const float* speed,
                              float speed_const, const float2* ctab, float r, int n, int P, const float* key, int* list,
                              int tiles_x, int tiles_y, uint8_t* flag, unsigned* wmask, int max_inner, float window,
                              int q, void* ctl, int grid, hipStream_t s);
// word masks of the labeler tiles (uint32 each); phi in the caller's node-major layout
hipError_t launch_label_mask_init(const uint8_t* cls, const int16_t* src, int n, int tiles_x, unsigned* mask,
                                  hipStream_t s);
hipError_t launch_label_phi_out(const uint32_t* phi32, int64_t count, int n_patches, uint16_t* out, hipStream_t s);
hipError_t launch_label_argmax(const uint16_t* phi, int64_t count, int P, int16_t* label, uint64_t* overlap,
                               uint16_t tau, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int count, hipStream_t s);
constexpr int kLabelTile = 16;

// Active-tile solver (tiles.hip). Tile shapes: 0 = 32 x 16 nodes, 1 = 16 x 16 nodes (one node
// per lane, 256 threads), 2 = 8 x 8 nodes with the controls split over 4 groups of wavefronts
// (256 threads), 3 = 16 x 16 split over 4 (1024 threads), 4 = 16 x 16 split over 2 (512 threads).
struct TileShape {
  int tw, th, split, threads;
};
constexpr int kTileShapes = 5;
TileShape tile_shape_of(int shape);
size_t tile_pass_lds_bytes(const TileShape& sh, int halo, bool indep);
hipError_t launch_tile_keys(const float* w, const uint8_t* cls, int tw, int th, int n, int tiles_x, int tiles_y,
                            float vstar, float lambda, float* key, hipStream_t s);
// The whole iteration in one cooperative launch; `state` is device memory of coop_state_bytes(),
// initialised by the caller: {count 0, kmin +inf, bound -inf, resid 0, passes 0, status 0, updates 0}.
size_t coop_state_bytes();
hipError_t launch_coop_state_init(void* state, hipStream_t s);
// `tchange` of the tile-solver launches holds 2 * tiles words: the move of each staged slot
// (float, negative when its visit stopped unsettled), then the neighbour sides it flags (uint32,
// bit (dy + 1) * 3 + dx + 1 for the neighbour at tile offset (dx, dy)).
// Device-driven passes (graph-capturable): `ctl` is device memory of tilectl_bytes() (at most
// kTileCtlHostBytes, the size of the host copies). Layout of the words the host reads: [9] done,
// [10] passes, [11] check sweeps, [7] resid bits, [12..13] updates, [14..15] policy-evaluation
// updates. `pe`: policy-evaluation iterations after each full one (split tile shapes only). The
// cooperative state: [6..7] updates, [8..9] policy updates.
// The passes keep the iterate in two arrays: a.w_in and w2 (n * n floats each), with one word per
// tile (tile_word, zeroed by the caller before the first pass) naming the array that holds the
// tile's current values; launch_tile_gather copies the tiles held in w2 back to w_in afterwards.
constexpr size_t kTileCtlHostBytes = 128;
size_t tilectl_bytes();
hipError_t launch_tilectl_init(void* ctl, hipStream_t s);
hipError_t launch_tilectl_pass(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                               const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                               float* w2, unsigned* tile_word, uint8_t* flag, int max_inner, float tol_inner,
                               float act, float window, float tol, int q, void* ctl, int grid, hipEvent_t ev_before,
                               hipEvent_t ev_after, int pe, unsigned long long* wg_acc, hipStream_t s);
hipError_t launch_tile_gather(float* w, const float* w2, const unsigned* tile_word, int n, int shape, hipStream_t s);
// `wg_acc`: 2 * grid counters (node updates, policy-evaluation updates per visit workgroup), zeroed
// by the caller before the first pass; launch_tilectl_sum writes their totals to the pass state.
hipError_t launch_tilectl_sum(const unsigned long long* wg_acc, int groups, void* ctl, hipStream_t s);
// The active-tile solver over a batch of instances (tiles.hip): per-instance descriptors
// (tb_inst_bytes each, filled by tb_fill_inst) and pass states (tb_state_bytes each), one control
// block (tb_ctl_bytes; word kTBCtlActive = instances still iterating). A pass is three launches.
// Each instance has a second array w2 (n * n floats) and one word per tile, as the single-instance
// passes (launch_tilectl_pass); the caller zeroes the words before the first pass and gathers
// each instance with launch_tile_gather after the last.
struct TBResult {
  unsigned done, passes, checks;
  float resid;
  unsigned long long updates, pe_updates;
};
constexpr int kTBCtlActive = 4;
size_t tb_inst_bytes();
size_t tb_state_bytes();
size_t tb_ctl_bytes();
void tb_fill_inst(void* dst, const SweepArgs& a, float* w2, unsigned* word, const float* key, int tiles_x,
                  int tiles_y, int tile0, int max_inner, int pe, float tol_inner, float act, float window, float tol,
                  long long max_passes);
void tb_read_state(const void* src, int i, TBResult* out);
hipError_t launch_tb_init(void* st, int count, void* ctl, hipStream_t s);
hipError_t launch_tb_pass(int shape, const void* inst, void* st, int count, int max_chunks, uint8_t* flag, int* list,
                          const int* tile_inst, int* chk_inst, unsigned* chk_off, void* ctl, int diffusion, int scheme,
                          int path, int q, int grid, size_t lds, hipStream_t s);
hipError_t launch_tile_solve_coop(const SweepArgs& a, int shape, int diffusion, int scheme, int path, bool indep,
                                  const int16_t* label, const float* key, int* list, int tiles_x, int tiles_y,
                                  float* outbuf, float* tchange, uint8_t* flag, int max_inner, float tol_inner,
                                  float act, float window, float tol, int max_passes, void* state, int max_grid,
                                  int* grid_used, int pe, hipStream_t s);

// Batched solve (batch.hip). One entry per instance; `a` carries the instance's parameters as for
// the single-instance sweep (its pointers w_in/w_out/resid/flags are not used: the iterates live in
// two pools at `offset`, the control table in one array at `ctrl_offset`).
struct BatchInst {
  SweepArgs a;
  long long offset;        // first node of the instance in the pools
  long long free_nodes;
  int ctrl_offset;
  int tiles_x;
  int tiles;
  int tw_log2;             // tile width 1 << tw_log2 (32 or 64)
  int th;                  // tile height (8 or 16)
  int path;                // 1 first-ring kernel path, 0 general
  int diffusion;
  int pad;
};
size_t batchctl_bytes();
hipError_t launch_batch_init(const BatchInst* inst, int count, int* state, long long* done_at, float* last_resid,
                             unsigned* resid, unsigned* flags, int2* work, const int* first_item, void* ctl,
                             long long max_sweeps, int check_every, double tol, unsigned items, hipStream_t s);
hipError_t launch_batch_round(const BatchInst* inst, int count, const float4* ctrl_all, float* pool0, float* pool1,
                              unsigned* resid, unsigned* flags, int* state, long long* done_at, float* last_resid,
                              int2* work, void* ctl, int scheme, int check_every, int grid, size_t lds,
                              hipStream_t s);
// Host-readable words of the batch control block: [1] active, [4..5] sweeps, [10..11] node
// updates, [12..13] tile visits.
constexpr int kBatchCtlActive = 1, kBatchCtlSweeps = 4, kBatchCtlUpdates = 10, kBatchCtlTiles = 12;

// Context accessors (capi.hip) for the network entry points (net.hip).
}  // namespace slhjb
struct slhjb_ctx;
#include <string>
namespace slhjb {
hipStream_t ctx_stream(slhjb_ctx* ctx);
int ctx_device(slhjb_ctx* ctx);
int ctx_fail(slhjb_ctx* ctx, int status, const std::string& msg);
int ctx_hip_fail(slhjb_ctx* ctx, hipError_t e, const char* what);

// Learned warm start (cnn.hip): NHWC bfloat16 activations, FP32 master parameters.
hipError_t launch_conv3x3(int cin, int cout, int mode, const uint16_t* in, const uint16_t* w, const float* bias,
                          const uint16_t* gate, int images, int H, int W, int dil, int relu, uint16_t* out,
                          hipStream_t s);
// weight and bias gradients, accumulated into dw and db; `work` is device scratch of
// kWgradWorkFloats floats (the per-workgroup partial sums)
constexpr long long kWgradWorkFloats = 512LL * (9 * 64 * 32 + 64);
hipError_t launch_conv3x3_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dy, int images, int H, int W,
                                int dil, float* dw, float* db, float* work, hipStream_t s);
hipError_t launch_head_fwd(int c, const uint16_t* h, const float* hw, const float* hb, long long total, float* delta,
                           hipStream_t s);
hipError_t launch_loss_head_bwd(int c, const float* delta, const float* uhat, const float* vstar, const uint8_t* mask,
                                long long total, float inv_n, const uint16_t* h, const float* hw, uint16_t* dh,
                                float* dhw, float* dhb, float* loss_acc, hipStream_t s);
struct CropSrc {
  const float* uhat;
  const float* vstar;
  const float* speed;
  const uint8_t* cls;
  float speed_const;
  float leps;
  int n, x0, y0;
};
hipError_t launch_crops(int cin, const CropSrc* src, int images, int S, int margin, uint16_t* feat, float* uhat,
                        float* vstar, uint8_t* mask, hipStream_t s);
hipError_t launch_project(const float* uhat, const float* delta, const uint8_t* cls, int n, int pitch,
                          float target_value, float v_out, float* v, hipStream_t s);
hipError_t launch_pool2(const uint16_t* in, int images, int H, int W, int C, uint16_t* out, hipStream_t s);
hipError_t launch_upcat(const uint16_t* low, const uint16_t* skip, int images, int H, int W, int Cu, int Cs,
                        uint16_t* out, hipStream_t s);
hipError_t launch_upcat_bwd(const uint16_t* g, int images, int H, int W, int Cu, int Cs, uint16_t* glow,
                            hipStream_t s);
hipError_t launch_skip_combine(const uint16_t* e_act, const uint16_t* gcat, int Cu, const uint16_t* gpool, int images,
                               int H, int W, int C, uint16_t* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long count, float lr_t, float b1, float b2,
                       float eps_t, hipStream_t s);
hipError_t launch_pack_weights(const float* w, int cout, int cin, uint16_t* wt, uint16_t* wtt, hipStream_t s);
hipError_t launch_zero_f32(float* p, long long count, hipStream_t s);
hipError_t launch_scale_f32(float* p, long long count, float a, hipStream_t s);
hipError_t launch_count_nonzero_u8(const uint8_t* m, long long count, unsigned* out, hipStream_t s);

}  // namespace slhjb
