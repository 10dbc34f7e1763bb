/*
 * slhjb — semi-Lagrangian solver for second order HJB equations on MI355X (gfx950).
 *
 * The method is the semi-Lagrangian Markov-chain scheme of Cacace & Falcone, "A dynamic
 * domain decomposition for a class of second order semi-linear equations" (arXiv
 * 1502.01629), Section 3, eqs. SLscheme2 and SLscheme3, in a discounted (Kruzkov) form:
 *
 *   feet    y = x_i + h f(x_i,a) + s sqrt(h) sigma_k(x_i,a),   s = +-1, k = 1..d,  f = c(x) a
 *   SL2     v_i = min_a [ beta (1/2d) sum_{k,s} I[v](y) + rho ]
 *   SL3     v_i = min_a (beta Lambda1(a) + rho) / (1 - beta Lambda0(a))
 *
 * with beta = exp(-lambda h) rounded to float, rho = (1 - beta) l / lambda, I[.] the
 * bilinear reconstruction on the grid (v_out outside the closed box), Lambda0 the node's own
 * interpolation weight averaged over the feet and Lambda1 the rest (eq. SLimplicit). With
 * lambda = 0 the scheme is the undiscounted one exactly as Section 3 prints it: beta = 1,
 * rho = h l. The running cost may depend on the state and the control, l(x,a) = l_x(x) + l_a(a),
 * and the diffusion coefficient on the state, eps(x) (Sections 5.2-5.3).
 *
 * Conventions for every entry point:
 *  - Grids are n x n nodes on [x_lo, x_hi]^2, node (i,j) at (x_lo + i dx, x_lo + j dx),
 *    dx = (x_hi - x_lo)/(n-1), stored row-major at j*n + i (x1 fastest).
 *  - Arrays named "device" are HIP device pointers owned by the caller; the library never
 *    frees or keeps them beyond the call (except where a call says otherwise). Arrays named
 *    "host" are read during the call only.
 *  - All work is enqueued on the context's stream. Calls that return host results
 *    synchronise that stream once before returning.
 *  - Every argument is validated before anything is launched; on error nothing is
 *    launched and the function returns SLHJB_E_INVALID_ARG (or another negative status).
 *    No C++ exception ever crosses this interface.
 *  - A context is used by one host thread at a time.
 */
#ifndef SLHJB_H
#define SLHJB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------------------- */
enum {
    SLHJB_OK = 0,
    SLHJB_NOT_CONVERGED = 1,   /* soft: the result is a valid iterate, tolerance not met   */
    SLHJB_E_INVALID_ARG = -1,
    SLHJB_E_UNSUPPORTED = -2,
    SLHJB_E_HIP = -3,          /* a HIP runtime call failed; see slhjb_last_hip_error      */
    SLHJB_E_NOMEM = -4,
    SLHJB_E_NONFINITE = -5     /* a NaN or infinity appeared in the iterate                */
};

/* Static description of a status code. Never NULL. */
const char* slhjb_status_string(int status);
/* Interface version (increments on any change of a declaration in this header). */
int slhjb_version(void);
/* Identity of the build: the first 16 hex digits of the SHA-256 of the sources the library was
 * compiled from (so that a caller can refuse a library older than its sources). Never NULL. */
const char* slhjb_source_hash(void);

/* ---- context ------------------------------------------------------------------------ */
typedef struct slhjb_ctx slhjb_ctx;

/* Create a context on HIP device `hip_device` that enqueues on `hip_stream` (a hipStream_t,
 * NULL = the device's null stream). The context owns its scratch memory (iterate buffers,
 * residual slots, control tables) and frees it in slhjb_ctx_destroy. */
int slhjb_ctx_create(slhjb_ctx** out, int hip_device, void* hip_stream);
int slhjb_ctx_destroy(slhjb_ctx* ctx);
/* Raw hipError_t behind the last SLHJB_E_HIP returned on this context (0 if none). */
int slhjb_last_hip_error(const slhjb_ctx* ctx);
/* Human-readable detail of the last error on this context ("" if none). Never NULL. */
const char* slhjb_last_error_message(const slhjb_ctx* ctx);

/* ---- problem -------------------------------------------------------------------------- */
enum { SLHJB_DIFF_NONE = 0,   /* sigma = 0: one foot per control (Section 4.3)                  */
       SLHJB_DIFF_ISO = 1,    /* sigma = sqrt(2 eps) I: 4 feet x + h f +- sqrt(2 eps h) e_k (4.1) */
       SLHJB_DIFF_RANK1 = 2   /* sigma = sqrt(2 eps) a: 2 feet x + h f +- sqrt(2 eps h) a (5.3)  */ };
enum { SLHJB_SCHEME_SL2 = 0,  /* eq. SLscheme2                                                  */
       SLHJB_SCHEME_SL3 = 1   /* eq. SLscheme3: the node's dependence on itself removed          */ };
enum { SLHJB_FREE = 0, SLHJB_TARGET = 1, SLHJB_OBSTACLE = 2 };

/* The discrete problem (Section 3: domain, dynamics, diffusion, cost, control set, h, dx;
 * plus the discount lambda of the Kruzkov form). */
typedef struct {
    int32_t n;                  /* nodes per side, 3 <= n <= 32769                             */
    float x_lo, x_hi;           /* the box [x_lo, x_hi]^2, x_lo < x_hi                           */
    float h;                    /* time step, > 0                                                */
    float lambda;               /* discount rate, >= 0 (1 = Kruzkov minimum time; 0 = the
                                   undiscounted scheme of Section 3: beta = 1, rho = h l)        */
    float eps;                  /* diffusion coefficient, >= 0 (ignored for SLHJB_DIFF_NONE and
                                   where eps_field is given)                                     */
    int32_t diffusion;          /* SLHJB_DIFF_*                                                  */
    int32_t scheme;             /* SLHJB_SCHEME_*                                                */
    int32_t n_controls;         /* 1 <= N_A <= 256                                               */
    const float* controls;      /* host float[2*N_A]: a_m = (controls[2m], controls[2m+1])       */
    const float* speed;         /* device float[n*n], c(x_i) > 0 finite; NULL = speed_const      */
    float speed_const;          /* c when speed == NULL, > 0                                     */
    float running_cost;         /* l > 0 where running_cost_field is NULL                        */
    const uint8_t* node_class;  /* device uint8[n*n] of SLHJB_FREE / _TARGET / _OBSTACLE         */
    float target_value;         /* g on TARGET nodes                                             */
    float v_out;                /* value at feet outside the closed box and on OBSTACLE nodes    */
    const float* drift;         /* device float[2*n*n], (d_1, d_2) per node, row-major, finite, or
                                 * NULL. With a drift the dynamics is f(x,a) = c(x) (d(x) + a):
                                 * the advection (A) and Zermelo (C) examples of Section 5 (for C,
                                 * c = 1/(1+|x|^2), d = R_theta x/|x| and the controls carry the
                                 * factor eta/2). The feet then go through the general kernels;
                                 * slhjb_synthesize, slhjb_label, patch labels in
                                 * slhjb_solve_patchy and slhjb_solve_batch reject a drift
                                 * (SLHJB_E_UNSUPPORTED). NULL: f(x,a) = c(x) a.            */
    /* Costs and diffusion that vary (Sections 5.2 "Degenerate diffusion" and 5.3 "General
     * nonlinear problems"). Any of them, and lambda = 0, take the general kernels (kernel path 2);
     * the batched solve rejects them, the active-tile solver takes them in the transmission mode
     * with host-driven passes only, and slhjb_synthesize / slhjb_label (patch labels) reject a
     * control cost (SLHJB_E_UNSUPPORTED).                                                        */
    const float* running_cost_field; /* device float[n*n]: l_x(x_i) > 0 finite per node, replacing
                                        running_cost; or NULL                                     */
    const float* control_cost;       /* host float[N_A]: l_a(a_m) >= 0 finite added to the running
                                        cost under control m; or NULL (0)                          */
    const float* eps_field;          /* device float[n*n]: eps(x_i) >= 0 finite per node, replacing
                                        eps (degenerate diffusion where it is 0); or NULL          */
} slhjb_problem;

typedef struct {
    int64_t sweeps;             /* sweeps performed                                              */
    int64_t converged_sweep;    /* first sweep whose residual was <= tol (-1 if none)            */
    int64_t node_updates;       /* FREE-node Bellman updates performed                           */
    double residual;            /* sup-norm change of the last sweep                              */
    double seconds;             /* device time of the whole call (HIP events on the ctx stream)   */
    double sweep_seconds;       /* device time spent in the batches of sweep kernels              */
    int64_t sweep_launches;     /* sweep kernel launches inside sweep_seconds                     */
    int32_t status;             /* SLHJB_OK / SLHJB_NOT_CONVERGED / error                         */
    int32_t kernel_path;        /* 0 general halo-tile kernel, 1 first-ring register kernel,
                                   2 general kernel with the cost term and per-node noise (varying
                                   costs, lambda = 0 or an eps field)                               */
    int32_t halo;               /* interpolation halo of the LDS tile, in cells                   */
    int32_t pad;
    int64_t policy_updates;     /* node updates of policy-evaluation iterations (one control each;
                                   active-tile solver with policy_sweeps > 0), not in node_updates */
    int64_t check_sweeps;       /* active-tile solver: passes that were full check sweeps (every
                                   tile, one iteration), counted in sweeps; -1 = not counted
                                   (persistent launch); 0 for the Jacobi solves                     */
    double check_seconds;       /* active-tile solver with collect_kernel_time: the part of
                                   sweep_seconds spent in check-sweep visit launches               */
} slhjb_stats;

/* One Jacobi sweep of the scheme (eq. SLscheme2 or SLscheme3 per problem->scheme):
 * v_out = T(v_in) on FREE nodes; TARGET nodes get target_value, OBSTACLE nodes v_out.
 * v_in, v_out: device float[n*n], distinct. residual_host (nullable): receives
 * max over FREE nodes of |v_out - v_in|. Synchronises the stream. */
int slhjb_sweep(slhjb_ctx* ctx, const slhjb_problem* problem, const float* v_in, float* v_out,
                double* residual_host);

/* Jacobi value iteration from the guess in v (device float[n*n], overwritten with the result)
 * until the sup-norm change of a sweep is <= tol, or max_sweeps. The residual is read back
 * every `check_every` sweeps (1..256, 0 = automatic), so up to check_every-1 sweeps may run
 * past the converged one; stats->converged_sweep reports the first converged sweep.
 * Returns SLHJB_OK, SLHJB_NOT_CONVERGED (v holds the last iterate) or an error.
 * stats (nullable) is filled in every case where the call got past validation. */
int slhjb_solve(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_sweeps,
                int32_t check_every, slhjb_stats* stats);

/* Largest grid side slhjb_solve_noalloc accepts. */
#define SLHJB_NOALLOC_MAX_N 1025

/* slhjb_solve for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same arguments, arithmetic, check cadence,
 * stopping rule, statistics and results as slhjb_solve, bit for bit, with no hipMalloc / hipFree
 * or other allocating call. Its scratch (the second iterate of up to SLHJB_NOALLOC_MAX_N^2 nodes,
 * the padded control table and the residual words, 4.21 MB) is a static device array of the
 * library: one copy per device, held until the process ends, and shared by every call on that
 * device, which leaves in it what the last call wrote (each call clears the words it needs first).
 * Calls that overlap on one device (two host threads, or two contexts on different streams) race
 * on it and must not be made. ctx must exist already (slhjb_ctx_create allocates its events).
 * n * n > SLHJB_NOALLOC_MAX_N^2: SLHJB_E_INVALID_ARG, nothing launched. */
int slhjb_solve_noalloc(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_sweeps,
                        int32_t check_every, slhjb_stats* stats);

/* ---- active-tile solve (Sections 4.2-4.3, computation step) ----------------------------- */
enum { SLHJB_ORDER_NONE = 0,   /* every flagged tile each pass (static order)                     */
       SLHJB_ORDER_KEYS = 1    /* frontier by the arrival time of the start (u_hat order)         */ };
enum { SLHJB_MODE_TRANSMISSION = 0,  /* one shared iterate: sharp interfaces, transmission by the
                                        shared values (Section 4.3)                               */
       SLHJB_MODE_INDEPENDENT = 1    /* each patch alone: a node reads grid values of other patches
                                        as v_out (state constraints at the interfaces, Section 2) */ };
typedef struct {
    int32_t order;              /* SLHJB_ORDER_*                                                  */
    int32_t mode;               /* SLHJB_MODE_*                                                   */
    const int16_t* label;       /* device int16[n*n] patch labels; needed for INDEPENDENT         */
    float key_slack;            /* band width of arrival times (ORDER_KEYS); < 0 = the time to
                                   cross max(16, (n-1)/16) cells at the fastest speed             */
    int32_t max_inner;          /* Jacobi iterations per tile visit at most; 0 = without diffusion
                                   2 (tile width + height), or tile width + height with
                                   policy_sweeps > 0; with diffusion (eps > 0) 2, or
                                   policy_sweeps + 1 with policy_sweeps > 0                        */
    int32_t tile_shape;         /* 0: 32x16 nodes, 1: 16x16 nodes (one node per thread, 256
                                   threads); 2: 8x8 nodes with the control set split over four
                                   groups of wavefronts (256 threads); 3: 16x16 split over four
                                   (1024 threads); 4: 16x16 split over two (512 threads)      */
    int32_t persistent;         /* 1: the whole iteration in one cooperative launch (grid barriers
                                   between phases); 0: one launch per phase, driven by the host   */
    int32_t max_workgroups;     /* persistent launch: cap on co-resident workgroups; 0 = 1024     */
    int32_t collect_kernel_time;/* 1: time every visit launch with events (stats->sweep_seconds,
                                   sweep_launches = passes); graph driver only                    */
    int32_t policy_sweeps;      /* 0..64 (tile shapes 2-4): after each full iteration of a visit,
                                   this many iterations that apply every node's maximising control
                                   of that iteration only (modified policy iteration; the fixed point
                                   is the same, only full iterations decide that a tile settled)  */
} slhjb_tile_opts;

/* Solve from the guess in v (device float[n*n], overwritten) with the active-tile method: the
 * grid is cut into tiles (opts->tile_shape); a pass iterates each selected tile in LDS against its frozen
 * halo until no node moves by more than tol/2, writes it back (every tile of a pass reads the
 * values from before the pass; the library keeps a second n*n array for that), and flags the tile
 * and its neighbours when it moved by more than tol/2. The first pass takes every tile; with SLHJB_ORDER_KEYS a
 * pass takes only the flagged tiles whose key (minimum arrival time -ln(1 - v/V*)/lambda of the
 * start over the tile's FREE nodes, V* = l/lambda) is within key_slack of the smallest flagged
 * key: the nodes are processed by increasing u_hat, as the paper prescribes, in bands of tiles.
 * When no tile is flagged, one Jacobi sweep of the whole grid checks the sup-norm change; the
 * call returns SLHJB_OK when it is <= tol (stats->residual), else continues.
 * stats->sweeps counts passes (the checks included), stats->node_updates the FREE-node Bellman
 * updates actually performed. In INDEPENDENT mode the fixed point is that of the per-patch
 * problems (the decomposition error is its distance to the global solution). */
int slhjb_solve_tiles(slhjb_ctx* ctx, const slhjb_problem* problem, float* v, double tol, int64_t max_passes,
                      const slhjb_tile_opts* opts, slhjb_stats* stats);

/* ---- batched solve of many independent instances ------------------------------------------ */
enum { SLHJB_BATCH_TILE_64x16 = 0, SLHJB_BATCH_TILE_64x8 = 1, SLHJB_BATCH_TILE_32x16 = 2, SLHJB_BATCH_TILE_32x8 = 3 };
typedef struct {
    int32_t check_every;        /* sweeps between residual checks, 1..256; 0 = 16. (slhjb_solve's
                                   automatic value depends on the grid size: give both calls the
                                   same explicit value to compare them.)                           */
    int32_t batches_per_graph;  /* check batches captured in one graph replay, 1..64; 0 = 4         */
    const int8_t* tile_shapes;  /* host int8[count] of SLHJB_BATCH_TILE_* per instance, nullable
                                   (= SLHJB_BATCH_TILE_64x16 for all)                             */
    int32_t max_workgroups;     /* grid of the sweep launches; 0 = 4096                             */
    int32_t pad;
} slhjb_batch_opts;
typedef struct {
    int64_t sweeps;             /* sweep launches (each covers every instance still iterating)      */
    int64_t node_updates;       /* FREE-node Bellman updates over all instances                      */
    int64_t tiles_swept;        /* tile visits over all sweeps                                       */
    int64_t replays;            /* graph replays                                                     */
    double seconds;             /* device time of the call (HIP events), conversions included        */
    int32_t converged;          /* instances that met tol                                            */
    int32_t status;             /* worst status over the instances                                    */
} slhjb_batch_stats;
/* Jacobi value iteration (as slhjb_solve) of `count` independent problems at once (1 <= count
 * <= 4096, all with the same scheme). v[i]: device float[n_i*n_i], the start, overwritten with the
 * result. Every instance gets exactly the arithmetic, the check cadence (residual of the last sweep
 * of each batch of check_every sweeps) and the stopping rule of slhjb_solve(problems[i], v[i], tol,
 * max_sweeps, check_every): the results, stats[i].sweeps and stats[i].converged_sweep are
 * bit-for-bit those of the single-instance calls. The sweeps of all instances still iterating run
 * in the same launches, over one device work list of (instance, tile) items rebuilt after every
 * check; an instance leaves it when it converges, fails (non-finite value) or reaches max_sweeps.
 * The launches of batches_per_graph checks are captured in one HIP graph and replayed until no
 * instance is left. The tile shape of an instance changes the schedule, never the values.
 * stats (nullable): slhjb_stats[count] (seconds = the whole call); total (nullable).
 * Returns SLHJB_OK if every instance converged, SLHJB_NOT_CONVERGED if some reached max_sweeps, a
 * negative status on an error (for SLHJB_E_NONFINITE, stats[i].status names the instance).
 * Needs device memory for two FP32 copies of all the grids. Synchronises. */
int slhjb_solve_batch(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v, double tol,
                      int64_t max_sweeps, const slhjb_batch_opts* opts, slhjb_stats* stats,
                      slhjb_batch_stats* total);

/* The active-tile solve (as slhjb_solve_tiles, transmission mode, pass by pass) of `count`
 * independent problems at once (1 <= count <= 4096; all with the same scheme, diffusion kind and
 * kernel path; lambda > 0, constant running cost and eps, no drift). v[i]: device float[n_i*n_i],
 * the start, overwritten with the result. Every instance runs exactly the passes of
 * slhjb_solve_tiles(problems[i], v[i], tol, max_passes, opts): its own band of u_hat keys, flags,
 * band moves and check sweeps, so a converged instance's values, stats[i].sweeps (passes) and
 * node_updates are bit-for-bit those of the single-instance call. The passes of all instances
 * still iterating share three launches (selection into one work list of (instance, tile) items,
 * per-instance decisions, visits that write their tiles back), captured 16 at a time in a HIP
 * graph and replayed
 * until every instance has converged or made max_passes passes (the single-instance call checks
 * max_passes only between its graph replays, so an instance that does not converge may stop a few
 * passes apart). opts: order, max_inner, key_slack, tile_shape and policy_sweeps as for
 * slhjb_solve_tiles; mode must be SLHJB_MODE_TRANSMISSION and persistent 0 (SLHJB_E_UNSUPPORTED
 * otherwise); collect_kernel_time is ignored. stats (nullable): slhjb_stats[count] (seconds = the
 * whole call); total (nullable): sweeps = passes over all instances, node_updates, replays,
 * seconds, converged. Returns SLHJB_OK if every instance converged, SLHJB_NOT_CONVERGED otherwise.
 * Needs device memory for a second copy of every instance's iterate (tiles * tile nodes floats per
 * instance) and per-tile state. Synchronises. */
int slhjb_solve_tiles_batch(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v,
                            double tol, int64_t max_passes, const slhjb_tile_opts* opts, slhjb_stats* stats,
                            slhjb_batch_stats* total);

/* The same batched active-tile solve as a reusable object, for callers that solve the same set of
 * instances (same problems, same iterate buffers) again and again: create prepares every
 * instance (statistics, control tables, tile layout), allocates the device buffers and captures
 * the graph of 16 passes once; run starts from whatever v[i] holds, solves to tol in at most
 * max_passes passes per instance and overwrites v[i] (same values and statistics as
 * slhjb_solve_tiles_batch); destroy frees everything. The object keeps the problems' device
 * arrays (speed, node_class) and the v pointers: they must stay valid and unchanged in shape until
 * destroy (their contents may change between runs). The object belongs to ctx and uses its
 * stream; runs of one object must not overlap. Errors as slhjb_solve_tiles_batch; *out is NULL
 * on failure. */
typedef struct slhjb_tiles_batch slhjb_tiles_batch;
int slhjb_tiles_batch_create(slhjb_ctx* ctx, const slhjb_problem* problems, int32_t count, float* const* v,
                             const slhjb_tile_opts* opts, slhjb_tiles_batch** out);
int slhjb_tiles_batch_run(slhjb_tiles_batch* batch, double tol, int64_t max_passes, slhjb_stats* stats,
                          slhjb_batch_stats* total);
int slhjb_tiles_batch_destroy(slhjb_tiles_batch* batch);

/* ---- the patchy method end to end (Section 4.3) ------------------------------------------- */
enum { SLHJB_PATCHY_TRANSMISSION = 0,  /* patchy decomposition, one shared iterate             */
       SLHJB_PATCHY_INDEPENDENT = 1,   /* patchy decomposition, state constraints at interfaces */
       SLHJB_PATCHY_STATIC = 2         /* static decomposition: no pre-computation, fixed tile
                                          order, cold start (the comparison of Section 5.4)     */ };
typedef struct {
    int32_t mode;                 /* SLHJB_PATCHY_*                                               */
    int32_t n_patches;            /* N_P (labels only)                                            */
    const int16_t* source_patch;  /* device int16[n*n] from slhjb_partition_sources (labels only) */
    double tol;                   /* fine tolerance (sup-norm change of a full sweep)             */
    double tol_coarse;            /* coarse tolerance                                             */
    int64_t max_passes;           /* per solve                                                    */
    float key_window;             /* band width of the u_hat order, < 0 = automatic               */
    int32_t tile_shape;           /* as slhjb_tile_opts.tile_shape                                */
    int32_t collect_kernel_time;  /* as slhjb_tile_opts.collect_kernel_time (fine solve)          */
    int32_t policy_sweeps;        /* as slhjb_tile_opts.policy_sweeps (coarse and fine solves)    */
} slhjb_patchy_opts;

typedef struct {
    double t_coarse, t_upsample, t_synthesize, t_label, t_solve, t_total;  /* seconds (events)    */
    double t_visit;               /* fine solve: time inside the tile-visit kernels (if collected)*/
    int64_t coarse_passes, node_updates_coarse, label_passes, passes, node_updates;
    int64_t policy_updates;       /* fine solve: policy-evaluation node updates                    */
    double residual;              /* of the final check sweep on the fine grid                    */
    int32_t status;
    int32_t pad;
    int64_t check_sweeps;         /* fine solve: passes that were full check sweeps               */
    double t_check_visit;         /* fine solve: part of t_visit in check-sweep visits (if timed)  */
} slhjb_patchy_stats;

/* The algorithm of Section 4.3 on one GPU. Patchy modes: (1) coarse solve of `coarse` with
 * sigma = 0 from v = V* (the Kruzkov "+infinity") to tol_coarse by the active-tile solver, for
 * at most min(max_passes, 16 n_coarse) passes (a coarse solution short of tol_coarse is still a
 * valid start);
 * (2) u_hat = bilinear interpolation on the fine grid, written to v; (3) synthesis of the
 * feedback control from u_hat and (4) integer patch labels (when label_out is given or the mode
 * is INDEPENDENT); (5) the fine solve from u_hat, tiles by increasing u_hat
 * (SLHJB_ORDER_KEYS), sharing one iterate (TRANSMISSION) or with state constraints at the patch
 * interfaces (INDEPENDENT). STATIC: the fine solve from v = V* with every flagged tile each pass.
 * v: device float[n*n] output; label_out (nullable): device int16[n*n].
 * `coarse` must cover the same box; its eps/diffusion are ignored (sigma = 0). Synchronises. */
int slhjb_solve_patchy(slhjb_ctx* ctx, const slhjb_problem* fine, const slhjb_problem* coarse,
                       const slhjb_patchy_opts* opts, float* v, int16_t* label_out, slhjb_patchy_stats* stats);

/* ---- pre-computation of the patchy method (Section 4.3) --------------------------------- */

/* u_hat: bilinear interpolation of a coarse grid solution onto a fine grid of the same box
 * (Section 4.3, pre-computation step: the coarse solution carried to the fine grid). v_c: device float[n_c*n_c],
 * v_f: device float[n_f*n_f]. Fine node i lies at coarse coordinate i (n_c-1)/(n_f-1); the
 * grids need not be nested. Enqueued only (no synchronisation). */
int slhjb_upsample(slhjb_ctx* ctx, int32_t n_c, const float* v_c, int32_t n_f, float* v_f);

/* Bicubic interpolation of a coarse grid solution onto a fine grid of the same box: the smooth
 * input feature of the learned warm start (the coarse solution of Section 4.3's pre-computation,
 * carried over with a third-order kernel). Keys' cubic convolution kernel with a = -1/2 over the
 * 4 x 4 coarse nodes around each fine node, coarse indices clamped to the grid (edge
 * replication); fine node i at coarse coordinate i (n_c-1)/(n_f-1); coarse nodes are copied
 * exactly. v_c: device float[n_c*n_c], v_f: device float[n_f*n_f], distinct. Enqueued only. */
int slhjb_upsample_bicubic(slhjb_ctx* ctx, int32_t n_c, const float* v_c, int32_t n_f, float* v_f);

/* Discrete synthesis of the feedback control (eq. discrete-synthesis) with sigma = 0 and a
 * constant running cost: for every FREE node, the index m of the control minimising
 * I[v_hat](x_i + h c(x_i) a_m) (feet outside the box read v_out; the first minimum in the
 * caller's control order wins). v_hat: device float[n*n]; ctrl_out: device int16[n*n], -1 on
 * TARGET and OBSTACLE nodes. Enqueued after one synchronising validation pass. */
int slhjb_synthesize(slhjb_ctx* ctx, const slhjb_problem* problem, const float* v_hat, int16_t* ctrl_out);

/* Split the TARGET nodes (the sources of information in a target problem, standing in for the
 * boundary nodes that Section 4.3's pre-computation step splits into one set per patch) into
 * n_patches sets. Host-only. Targets are the 4-connected components of TARGET nodes, numbered
 * in row-major order of their first node; each gets one patch plus a largest-remainder share
 * (by node count, ties to the lower component) of the remaining n_patches - T; within a
 * component, patch = floor(P_t (atan2(j - cj, i - ci) + pi) / 2 pi) with (ci, cj) the
 * component's centroid in grid units. node_class: host uint8[n*n]; source_patch: host
 * int16[n*n] (patch id on TARGET nodes, -1 elsewhere). Needs n_patches >= number of targets. */
int slhjb_partition_sources(int32_t n, const uint8_t* node_class, int32_t n_patches, int16_t* source_patch,
                            int32_t* n_targets_out);

/* Balanced patches (Section 2 on the relative sizes of the patches, Section 4.3 closing remarks:
 * equal sub-sets of the sources can give very unequal patches, and the paper proposes to optimise
 * the subdivision iteratively so that the patches come out about equal, without giving a method).
 * This is one such method, `iterations` rounds of:
 *   1. label the patches of the current subdivision (as slhjb_label, tau = 0);
 *   2. size of patch p = the nodes labelled p; weight of a source node = its patch's size
 *      divided by its patch's number of source nodes;
 *   3. across the target components (4-connected, numbered in raster order of their first node):
 *      one patch each, the rest by the components' total size, largest remainder (ties: lower
 *      component; no size at all: by node count);
 *   4. within a component: its sources in angular order around the centroid (exact: direction
 *      (i cnt - sum_i, j cnt - sum_j) by half-plane and integer cross product, the order of atan2
 *      on (-pi, pi], ties by node index) cut into consecutive runs of equal total weight: source r
 *      with weight w_r goes to run floor(P_t (W_<r + w_r / 2) / W), clamped to [0, P_t - 1]
 *      (W: the component's total; without weight, equal counts), FP64 sums in that order.
 * problem, ctrl, v_hat as for slhjb_label (v_hat only orders the work); n_patches 1..64.
 * source_patch: device int16[n*n], in: a subdivision (every TARGET node in [0, n_patches), -1
 * elsewhere; e.g. from slhjb_partition_sources), out: the subdivision kept after `iterations`
 * (0..64) rounds. The rounds do not converge in general (a patch's territory is an argmax of fuzzy
 * indicators and can jump when its sources change), so the output is the best balanced
 * subdivision visited, the start included: the smallest largest-over-mean patch size, compared
 * exactly (max_k sum_b < max_b sum_k), the earliest on ties. sizes_out (nullable): host
 * int64[(iterations + 1) * n_patches], the patch sizes of every subdivision visited (round 0 is
 * the start). label_out (nullable): device int16[n*n], the labels of the output subdivision.
 * best_round_out (nullable): the round of the output. Synchronises. */
int slhjb_balance_sources(slhjb_ctx* ctx, const slhjb_problem* problem, const int16_t* ctrl, const float* v_hat,
                          int32_t n_patches, int32_t iterations, int16_t* source_patch, int64_t* sizes_out,
                          int16_t* label_out, int32_t* best_round_out);

/* Patch construction (eq. discrete-advection iterated to its fixed point, then the argmax that
 * turns the fuzzy indicators into patches), in exact integer arithmetic:
 *   phi_p in [0, 2^15]; 2^15 on TARGET nodes whose source_patch is p, 0 on other TARGET
 *   nodes, OBSTACLE nodes and outside the grid; a FREE node takes the bilinear value of phi_p
 *   at its synthesized foot x + h c(x) a_ctrl(x), with the foot offset quantised per axis to
 *   D = round_half_even(256 fl(fl(h/dx32) c) a) (dx32 = fl((x_hi-x_lo)/(n-1)), float
 *   arithmetic), cell offset D >> 8, weights (256 - f or f), f = D & 255, and
 *   phi' = (sum_c W_c phi(c) + 2^15) >> 16.
 * The map is monotone, so the iteration (in place, any order) stops at its least fixed point
 * above the start: the result is exact and does not depend on the schedule.
 * label_out[x] = argmax_p phi_p(x) (lowest p on ties), -1 where every phi_p is 0.
 * overlap_out (nullable) bit p set where phi_p >= tau_q15 (0 = no bits: sharp interfaces).
 * ctrl: device int16[n*n] from slhjb_synthesize (or any field, -1 = not advected);
 * v_hat (nullable): device float[n*n] u_hat; when given, 16x16-node tiles are visited in bands of
 * increasing arrival time of u_hat (the result does not depend on it, only the work);
 * source_patch: device int16[n*n]; phi_out (nullable): device uint16[n*n*n_patches].
 * Needs sigma = 0 feet inside the first ring of cells (h c_max |a| <= dx), else
 * SLHJB_E_UNSUPPORTED; 1 <= n_patches <= 64. Synchronises. */
int slhjb_label(slhjb_ctx* ctx, const slhjb_problem* problem, const int16_t* ctrl, const float* v_hat,
                const int16_t* source_patch, int32_t n_patches, uint16_t tau_q15, int16_t* label_out,
                uint64_t* overlap_out, uint16_t* phi_out, int64_t* passes_out);

/* ---- learned warm start ------------------------------------------------------------------ */
/* A convolutional network (the 4-level U-Net of slhjb_net_config arch 1, or the dilated network
 * of arch 0) that maps [u_hat, c, target mask, log10(eps) + 3,
 * 1 / (1 + d / 4)] (d: distance in cells to the nearest side of the box) on the fine grid to a
 * correction delta of u_hat; the start of the SL iteration is then
 * clamp(u_hat + delta, 0, 1) on FREE nodes (the boundary data elsewhere). The iteration
 * converges to the same fixed point from any start, so the network can only change the work,
 * never the result. (A serving addition beside the u_hat start of Section 4.3; the paper has no
 * network.)
 * Architecture: `layers` 3 x 3 convolutions with ReLU, the first from 16 input channels (5 used,
 * 11 zero) to `channels`, the others channels -> channels, with per-layer dilation, then a 1 x 1
 * head channels -> 1. Zero padding at image borders. Activations and conv weights in bfloat16
 * on the matrix cores with FP32 accumulation; head, loss, gradients and Adam in FP32.
 * Parameters (FP32, flat): per layer l, W_l[9][channels][cin_l] (tap-major, taps row-major over
 * dy, dx in {-1,0,1} x dilation) then b_l[channels]; then the head w[channels], b[1]. */
typedef struct slhjb_net slhjb_net;
typedef struct {
    int32_t layers;             /* 1..12 (arch 0)                                                  */
    int32_t channels;           /* 32 (arch 0)                                                     */
    int32_t dilation[12];       /* per layer, 1..32 (arch 0)                                       */
    int32_t arch;               /* 0: the dilated CNN above; 1: a 4-level U-Net: two 3 x 3
                                   convolutions (ReLU) per level with 32, 64, 128 and 128 channels,
                                   2 x 2 average pooling down, nearest x2 upsampling concatenated
                                   with the level's skip (upsampled first) up, the same 1 x 1 head;
                                   layers / channels / dilation are ignored. Its 14 convolutions, in
                                   parameter order: 16->32, 32->32 | 32->64, 64->64 | 64->128,
                                   128->128 | 128->128, 128->128 (bottom) | 256->128, 128->128 |
                                   192->64, 64->64 | 96->32, 32->32. Crops must be a multiple of 8
                                   pixels; the loss mask keeps 48 pixels (the receptive-field
                                   radius) from crop edges inside the frame, and the warm start
                                   pads the frame to a multiple of 8 by edge replication.        */
} slhjb_net_config;
/* One training or evaluation frame: the crop [x0, x0+crop) x [y0, y0+crop) of an n x n problem. */
typedef struct {
    const float* v_hat;         /* device float[n*n]: u_hat, the upsampled coarse solution         */
    const float* v_star;        /* device float[n*n]: the converged solution (target), nullable for
                                   inference                                                       */
    const float* speed;         /* device float[n*n], NULL = speed_const                           */
    const uint8_t* node_class;  /* device uint8[n*n]                                               */
    float speed_const;
    float eps;                  /* diffusion coefficient of the problem (> 0; feature log10(eps)+3) */
    int32_t n;
    int32_t x0, y0;
} slhjb_net_sample;
/* Create a network with zero parameters (set them with slhjb_net_set_params). The network owns
 * its device memory (parameters, gradients, Adam moments, activations) and uses ctx's stream. */
int slhjb_net_create(slhjb_ctx* ctx, const slhjb_net_config* cfg, slhjb_net** out);
int slhjb_net_destroy(slhjb_net* net);
/* Number of FP32 parameters (the length of the flat vectors below). */
int64_t slhjb_net_param_count(const slhjb_net* net);
/* Copy parameters from / to host float[param_count]; set also resets the Adam moments and step. */
int slhjb_net_set_params(slhjb_net* net, const float* host);
int slhjb_net_get_params(slhjb_net* net, float* host);
/* Gradients of the last slhjb_net_loss_grad call, host float[param_count]. */
int slhjb_net_get_grads(slhjb_net* net, float* host);
/* Forward pass on `count` crops of side `crop` (1 <= count <= 256, 1 <= crop <= 4096, crop
 * inside each frame): delta_out device float[count*crop*crop] (row-major per crop). */
int slhjb_net_forward(slhjb_net* net, const slhjb_net_sample* samples, int32_t count, int32_t crop,
                      float* delta_out);
/* Loss and gradients on `count` crops: L = mean of (u_hat + delta - v*)^2 over the FREE nodes at
 * least R = sum of the dilations (the receptive-field radius) away from every crop edge that lies
 * inside the frame (there the zero padding is not the box boundary), into the network's gradient
 * buffer (zeroed first). loss_out: host, nullable. */
int slhjb_net_loss_grad(slhjb_net* net, const slhjb_net_sample* samples, int32_t count, int32_t crop,
                        double* loss_out);
/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8, bias-corrected) with learning rate lr on
 * the current gradients. */
int slhjb_net_adam_step(slhjb_net* net, float lr);
/* Start of the SL iteration for `problem` from u_hat: v_out = clamp(v_hat + delta, 0, 1) on FREE
 * nodes, target_value on TARGET, v_out on OBSTACLE (device float[n*n]; v_hat and v_out may be the
 * same array). Needs problem->eps > 0 for the feature. */
int slhjb_net_warm_start(slhjb_net* net, const slhjb_problem* problem, const float* v_hat, float* v_out);

/* ---- parameter theory (host only, no GPU needed) --------------------------------------- */
/* The upwind diffusion ball analysis of Section 4.1 for dynamics bounded by f_min <= |f| <= f_max
 * and diffusion rows of length at most sigma_inf (eq. upper-bound, lower-bound, upper-alpha,
 * lower-alpha, hyperbolicity). */
typedef struct {
    double omega;               /* f_min / sigma_inf^2 (= f_min / 2 eps for sigma = sqrt(2 eps) I) */
    double upsilon;             /* f_max / f_min                                                 */
    double alpha_lower;         /* 1 / (omega dx)                       (eq. lower-alpha)         */
    double alpha_upper;         /* 1/Upsilon - (sqrt(1+4 omega dx Upsilon)-1)/(2 omega dx Upsilon^2) */
    double alpha_opt;           /* 1 / (1 + Upsilon)                                              */
    double tau_dx;              /* dx / (1 + Upsilon): the threshold on 1/omega                   */
    double h_alpha;             /* alpha_opt dx / f_min                                           */
    double h_upper;             /* the largest h with h f_max + sqrt(h) sigma_inf <= dx           */
    int32_t hyperbolic;         /* 1 if 1/omega < dx/(1+Upsilon)        (eq. hyperbolicity)       */
    int32_t pad;
} slhjb_regime;

int slhjb_regime_analyze(double f_min, double f_max, double sigma_inf, double dx, slhjb_regime* out);

/* Largest distance, in cells along either axis, between a FREE node and any of its feet, for
 * speeds bounded by speed_max (host computation). Used to size the interpolation halo. A drift
 * and a diffusion-coefficient field (device data) are not included: the solvers add
 * max_x h c(x) |d(x)|_inf / dx and take the largest eps(x) from a device pass. */
double slhjb_foot_reach(const slhjb_problem* problem, float speed_max);

#ifdef __cplusplus
}
#endif
#endif /* SLHJB_H */
