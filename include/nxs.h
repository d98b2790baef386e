/*
 * nxs.h -- C ABI of the non-exponential Gaussian splatting renderer for
 * AMD Instinct MI355X (gfx950).
 *
 * The library renders images of 3D Gaussians by compositing them front to
 * back with a pluggable transmittance operator: the generalized image
 * formation of Sec. 4 of "Generalized non-exponential Gaussian splatting"
 * (eq. generalized_gaussian with the discrete extinction of eq. nexp_p and
 * the operators of Table 1).  Each call runs, on the caller's HIP stream:
 * EWA projection, depth sort, tile binning, a stable tile sort, tile ranges,
 * and a per-tile composite that gathers each tile's splats in sorted order
 * batch by batch into on-chip memory.
 *
 * Conventions common to every entry point
 *   - Array pointers are DEVICE pointers of the context's device, unless the
 *     argument says "host".  Structs passed by pointer are HOST memory, read
 *     during the call only.
 *   - The caller owns every input and output buffer.  Inputs must stay
 *     unmodified and alive until the stream has passed the call's work.
 *     Outputs are fully overwritten; they need no clearing.
 *   - The context owns its workspace: device memory grown on demand, in
 *     stream order, from the caller's allocator (nxs_create) or, without
 *     one, from a memory pool of the library's own, and kept until
 *     nxs_destroy or nxs_release_workspace; and a small pinned host buffer.
 *     A forward that keeps backward state hands the buffers the backward
 *     needs to an nxs_fwd_state, which owns them until nxs_state_release.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     nxs_render_forward waits once on the host, after projection, for the
 *     number of tile instances that sizes the workspace, unless the render
 *     is deferred (NXS_FLAG_DEFERRED): it then waits for nothing and a
 *     render that outgrew the workspace is reported by
 *     nxs_forward_status.  Calls return once their work is enqueued.
 *   - No exception crosses the ABI.  Every call returns an nxs_status; for
 *     a non-OK status nxs_last_error() gives a message.  Arguments are
 *     checked before any launch, so NXS_EINVAL leaves outputs untouched.
 *   - A context is used by one host thread at a time.  Calls on the same
 *     context are serialised by the caller; they may use different streams.
 */
#ifndef NXS_H
#define NXS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NXS_OK = 0,
  NXS_EINVAL = -1,       /* bad argument; nothing was launched */
  NXS_ENOMEM = -2,       /* workspace allocation failed */
  NXS_EHIP = -3,         /* a HIP runtime call failed; see nxs_last_error */
  NXS_ECAPACITY = -4,    /* more than 2^32 - 1 tile instances, more workspace
                            than the context's limit (or the no-alloc entry
                            point's scratch) allows, or a deferred render
                            that outgrew the workspace (outputs undefined;
                            retry, with fewer views where the limit is the
                            cause) */
  NXS_EUNSUPPORTED = -5  /* operation not supported for these arguments (e.g. a
                            backward of a model that has none) */
} nxs_status;

/* Transmittance models (Table 1 and Sec. 5 of the paper).
 *   EXPONENTIAL       T = exp(-tau):  p_i = a_i prod_{j<i} (1 - a_j)  (classic 3DGS)
 *   LINEAR            T = [1 - tau]_+:  p_i = a_i
 *   QUAD_SUBLINEAR    T = [1 - tau - c tau^2 / 2]_+ with c = -0.5: p_i = a_i (1 + c tau_i)
 *   QUAD_SUPERLINEAR  the same with c = +0.5
 * For every model the splat whose p would take sum p to >= 1 gets the remainder
 * 1 - sum_{j<k} p_j, the transmittance becomes exactly 0 and compositing stops
 * (eq. nexp_p). */
typedef enum {
  NXS_EXPONENTIAL = 0,
  NXS_LINEAR = 1,
  NXS_QUAD_SUBLINEAR = 2,
  NXS_QUAD_SUPERLINEAR = 3,
  /* The remaining operators of Table 1, with their parameter in opts.param:
   *   QUADRATIC   T = [1 - tau - c tau^2 / 2]_+, c = param >= -0.5
   *   BLENDED     T = [lerp(1 - tau, exp(-tau), gamma)]_+:
   *               p_i = a_i (1 - gamma + gamma prod_{j<i} (1 - a_j)), gamma = param in [0, 1]
   *   VICINI      lerp of the complete linear and exponential operators, each
   *               saturating / stopping on its own (the exponential part obeys
   *               t_eps), gamma = param in [0, 1]
   *   POWER_LAW   T = [(1 + v tau)^(-1/v)]_+: p_i = a_i (1 + v tau_i)^(-(1+v)/v),
   *               v = param != 0; where 1 + v tau_i <= 0 the splat saturates */
  NXS_QUADRATIC = 4,
  NXS_BLENDED = 5,
  NXS_VICINI = 6,
  NXS_POWER_LAW = 7
} nxs_model;

/* Gaussians (Sec. 3: centre, covariance, opacity aleph, directional emission).
 *   means      [n,3]  world-space centres
 *   scales     [n,3]  per-axis standard deviations (> 0)
 *   quats      [n,4]  rotation as (w, x, y, z), normalised by the library;
 *                     an all-zero quaternion culls that Gaussian
 *   opacities  [n]    aleph in [0, 1] (values above 1 make the tile
 *                     bounds non-conservative)
 *   sh         [n, (sh_degree+1)^2, 3]  real SH coefficients per channel,
 *                     index l*l + l + m; colour = max(0, sum c_lm Y_lm(d) + 1/2)
 *                     with d the unit vector camera centre -> mean
 * All float32, C-contiguous. */
typedef struct {
  int32_t n;
  int32_t sh_degree; /* 0..3 */
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
} nxs_gaussians;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).
 * p_cam = R p_world + t with R row-major; pixel (x, y) is sampled at its
 * centre (x + 1/2, y + 1/2); u = fx x/z + cx, v = fy y/z + cy.
 * Gaussians with camera-space z <= znear are culled. */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float znear;
  int32_t width, height;
} nxs_camera;

/* Render options.  Zero-initialised fields take the defaults noted. */
typedef struct {
  int32_t model;          /* nxs_model */
  float background[3];    /* L_b of eq. generalized_gaussian (default 0) */
  float alpha_min;        /* splats with alpha < alpha_min are skipped;
                             0 -> 1e-3 */
  float t_eps;            /* exponential (and Vicini's exponential part): stop
                             after the first splat that leaves T < t_eps;
                             0 -> 1e-4, < 0 -> only once T falls below the
                             smallest normal float32 (1.2e-38) */
  int32_t tile_w, tile_h; /* 8x8, 16x16 or 32x8; 0 -> 16x16 */
  int32_t lds_batch;      /* sorted-list entries each wave of the composite
                             gathers into LDS per round, culls against its
                             8x8 block and then composites: 64, 128 or 256;
                             0 -> 64 */
  float param;            /* operator parameter of models 4..7 (c, gamma or v) */
  int32_t flags;          /* NXS_FLAG_* */
  int32_t schedule;       /* nxs_schedule of the composite; 0 -> NXS_SCHED_QUEUE */
  float instance_hint;    /* deferred renders: the tile instances the caller
                             expects (0 -> the context's last count); sizes the
                             tile sort's launches, never the result */
  int32_t sort_order;     /* nxs_sort_order; 0 -> NXS_SORT_AUTO */
} nxs_render_opts;

/* How the per-tile front-to-back lists are built (bitwise the same lists,
 * ordered by tile, float32 depth bits, Gaussian index):
 *   DEPTH_FIRST  sort all projected Gaussians by depth, emit their tile
 *                instances in that order, sort the instances stably by tile
 *   TILE_FIRST   emit instances in Gaussian order, sort them stably by tile,
 *                then sort each tile's list by depth in on-chip memory (a list
 *                longer than 4,096 entries is sorted through device memory)
 *   AUTO         TILE_FIRST when the expected instances per tile (the
 *                caller's instance_hint, else the context's last count) are
 *                at most 1,024 on average, else DEPTH_FIRST */
typedef enum {
  NXS_SORT_AUTO = 0,
  NXS_SORT_DEPTH_FIRST = 1,
  NXS_SORT_TILE_FIRST = 2
} nxs_sort_order;

/* opts.flags
 *   NXS_FLAG_DEFERRED  the forward does not wait on the host for the
 *       instance count: the instance buffers and the grids of the tile sort
 *       are sized from the context's current capacity (what earlier renders
 *       needed, with headroom).  A render that needs more instances than that
 *       (or a depth sort of more passes than the context planned) is detected
 *       on the device, does no work after the emission (its outputs are the
 *       background) and is reported by the next nxs_forward_status, which
 *       also grows the capacity so that repeating the render succeeds.
 *       Results are bitwise those of a render that waits. */
#define NXS_FLAG_DEFERRED 1

/* How the composite's work is laid onto the GPU (results are bitwise the same
 * under all four; only the time differs):
 *   TILES       one work-group per tile, one wave per 8x8 block of it
 *   BLOCKS      one single-wave work-group per 8x8 block
 *   QUEUE       all views' tiles in one queue ordered by decreasing
 *               tile-list length, consumed in order by the hardware
 *               dispatcher (single-wave work-groups, one per 8x8 block)
 *   PERSISTENT  a fixed grid of single-wave work-groups taking whole tiles
 *               of that order from atomic counters (one per XCD) */
typedef enum {
  NXS_SCHED_TILES = 1,
  NXS_SCHED_BLOCKS = 2,
  NXS_SCHED_QUEUE = 3,
  NXS_SCHED_PERSISTENT = 4
} nxs_schedule;

/* Per-view outputs (device pointers), row-major:
 *   rgb       [H, W, 3] float32   pixel value L0
 *   trans     [H, W]    float32   final transmittance T_{N+1}
 *   overdraw  [H, W]    int32     composited splats (terminating one included);
 *                                 may be NULL */
typedef struct {
  float* rgb;
  float* trans;
  int32_t* overdraw;
} nxs_image;

typedef struct nxs_context nxs_context;

/* What a forward keeps for its backward (appendix "Adjoints": the per-pixel
 * final values and the sorted splat lists the path replay re-walks). */
typedef struct nxs_fwd_state nxs_fwd_state;

/* Device allocator of the caller (e.g. a framework's caching allocator).
 *   alloc(bytes, stream, user): device memory of at least `bytes` bytes on
 *       the context's device, aligned to 256 bytes, usable by work enqueued
 *       on `stream` after the call; NULL on failure (the render then fails
 *       with NXS_ENOMEM; a block that is not aligned is given back and the
 *       render fails with NXS_EINVAL).
 *   free(ptr, stream, user): gives back a block from alloc.  Work enqueued
 *       on `stream` before the call may still use it, and all other work
 *       that used it is ordered before that point of `stream`: the
 *       allocator must not hand the block to work that can run earlier
 *       (a stream-ordered free).
 * Both are called from inside nxs_* calls on the calling thread. */
typedef void* (*nxs_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*nxs_free_fn)(void* ptr, void* stream, void* user);

/* Creates a context on HIP device `device`; *ctx receives the handle.
 * alloc and free: the caller's allocator (both or neither; `user` is passed
 * back to them).  Without them the workspace comes from a stream-ordered
 * memory pool the context creates (hipMallocFromPoolAsync / hipFreeAsync),
 * so that growing it never waits for the device. */
nxs_status nxs_create(nxs_context** ctx, int device, nxs_alloc_fn alloc, nxs_free_fn free,
                      void* user);

/* Waits for the context's work, then frees the workspace and the context.
 * States the caller has not released stay valid until it releases them. */
nxs_status nxs_destroy(nxs_context* ctx);

/* Renders n_views >= 1 views of the same Gaussians (Sec. 4, eq.
 * generalized_gaussian with the operator of opts.model).
 *   cams [n_views] host array; out [n_views] host array of device outputs.
 * Views may differ in size; all share opts.  n = 0 renders background.
 *   state  NULL: nothing is kept for a backward.  Otherwise *state receives
 *          a new nxs_fwd_state holding what nxs_render_backward needs (the
 *          sorted splat lists and records, the tile ranges and order, 12
 *          floats per pixel); the caller releases it with nxs_state_release.
 *          Models 0..4 only (NXS_EUNSUPPORTED otherwise).  On failure
 *          *state is NULL. */
nxs_status nxs_render_forward(nxs_context* ctx, const nxs_gaussians* g,
                              const nxs_camera* cams, int32_t n_views,
                              const nxs_render_opts* opts, const nxs_image* out,
                              nxs_fwd_state** state, void* stream);

/* nxs_render_forward for callers that cannot allocate device memory (code
 * under HIP graph capture set-up, tight serving loops, harnesses that forbid
 * hipMalloc): the same render, bitwise, with every buffer of the workspace
 * carved from a fixed scratch array of 64 MiB per device that the library
 * holds until the process ends; nothing is allocated, on the device or in
 * pinned host memory, and no state is kept.
 *   Arguments as for nxs_render_forward; opts.flags must be 0.
 *   Size limit: the render's workspace must fit the 64 MiB -- about 90
 *   bytes per Gaussian per view, 16 per tile instance, 16 per tile, plus the
 *   sort's digit counts (e.g. 150,000 Gaussians at 1920x1080 with about a
 *   million instances).  A render beyond it fails with NXS_ECAPACITY and a
 *   message naming the limit, before its composite writes any output.
 *   The call waits on the host for the instance count, like a waiting
 *   nxs_render_forward.  Every call on one GPU shares that GPU's scratch:
 *   calls that overlap on the device (another stream, another thread or
 *   context) race and give undefined results; calls on one stream are
 *   ordered.  Work is ordered after the context's earlier calls. */
nxs_status nxs_render_forward_noalloc(nxs_context* ctx, const nxs_gaussians* g,
                                      const nxs_camera* cams, int32_t n_views,
                                      const nxs_render_opts* opts, const nxs_image* out,
                                      void* stream);

/* Outcome of the deferred forwards (NXS_FLAG_DEFERRED) on the context since
 * the last call: waits for the context's last render, then returns NXS_OK,
 * or NXS_ECAPACITY if any of them outgrew the workspace (their outputs are
 * the background; their states, if any, hold no lists).  Before returning
 * NXS_ECAPACITY it grows the instance capacity to the largest count
 * needed (within the workspace limit), so repeating those renders succeeds.
 * needed (may be NULL): the largest instance count any of them needed. */
nxs_status nxs_forward_status(nxs_context* ctx, int64_t* needed);

/* Gradients of the Gaussians' parameters, device arrays shaped like the
 * inputs of nxs_gaussians (means [n,3], scales [n,3], quats [n,4],
 * opacities [n], sh [n,K,3]); overwritten by nxs_render_backward. */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
} nxs_gaussians_grad;

/* Path-replay backward of the forward that made `state` (appendix
 * "Adjoints": the linear and quadratic recursions; the front-to-back form
 * for the exponential).
 *   state     from nxs_render_forward on this context, not yet released
 *   dL_drgb   [n_views] host array of device [H,W,3] upstream gradients
 *   dL_dtrans [n_views] host array of device [H,W] gradients, or NULL (the
 *             array itself, or any entry, may be NULL for "zero")
 *   grads     device outputs, overwritten (sum over all views); per-Gaussian
 *             sums are accumulated with float atomics, so repeated calls agree
 *             to float32 rounding, not bitwise
 * Each tile's splats are re-walked front to back, rebuilding every pixel's
 * state from the start with the same float32 decisions as the forward;
 * nothing is stored per splat, only 12 floats per pixel.  The Gaussians of
 * the forward must be unchanged.  Any number of backwards may use one state,
 * and other forwards may run between its forward and its backward.
 * NXS_EINVAL on a NULL state, dL_drgb entry or gradient array, or a state
 * of another context; NXS_ECAPACITY for the state of a deferred forward that
 * outgrew the workspace.  Enqueued on `stream` after the context's earlier
 * calls; the gradients are complete when the stream reaches this point. */
nxs_status nxs_render_backward(nxs_context* ctx, const nxs_fwd_state* state,
                               const float* const* dL_drgb, const float* const* dL_dtrans,
                               const nxs_gaussians_grad* grads, void* stream);

/* Frees a state (stream-ordered on `stream`, after every call that used it).
 * NULL state: nothing. */
nxs_status nxs_state_release(nxs_context* ctx, nxs_fwd_state* state, void* stream);

/* Measured choice of tile shape, composite schedule and LDS batch for one
 * workload. */
typedef struct {
  int32_t tile_w, tile_h;
  int32_t schedule;       /* nxs_schedule */
  int32_t lds_batch;      /* list entries gathered per round (64, 128, 256) */
  int32_t sort_order;     /* nxs_sort_order (DEPTH_FIRST or TILE_FIRST) */
  float ms;               /* GPU time per render of the choice when measured */
} nxs_tuning;

/* Autotuner: the tile shape (8x8, 16x16, 32x8), composite schedule, LDS
 * batch (64, 128, 256 list entries per round) and sort order with the lowest
 * GPU time of a whole nxs_render_forward on this workload: every tile
 * shape and schedule at a batch of 64 and the automatic sort order, then
 * the other batches, then both sort orders, at the best so far.  A
 * candidate's time is that of `reps` deferred renders enqueued back to back
 * (no host wait inside the timed span) over their number.
 * The result is cached per (GPU architecture, CU count, n, SH degree, model,
 * number and sizes of the views): first in the context, then, if cache_path
 * is not NULL, in that text file (one line per workload; read on a miss,
 * appended after a sweep).  On a cache hit nothing is rendered.  On a miss
 * every candidate is rendered once untimed (waiting) and `reps` times
 * (0 -> 5) timed with events on `stream` (deferred; timed again if they
 * outgrew the context), writing `out` (the outputs are those of the last
 * candidate) and synchronising the stream.  Other fields of `opts` are used
 * as given; its tile, schedule, lds_batch and sort_order fields are ignored.  Errors as
 * for nxs_render_forward; an unreadable or unwritable cache file is
 * ignored. */
nxs_status nxs_autotune(nxs_context* ctx, const nxs_gaussians* g, const nxs_camera* cams,
                        int32_t n_views, const nxs_render_opts* opts, const nxs_image* out,
                        const char* cache_path, int32_t reps, nxs_tuning* result,
                        void* stream);

/* Workspace: the device memory a context keeps between renders (sort
 * buffers, per-slot and per-instance records), grown on demand and never
 * shrunk; states hold their own buffers and are not counted.  With a limit
 * set (bytes; 0 = none), a render that would grow it past the limit returns
 * NXS_ECAPACITY.  nxs_release_workspace waits for the context's work and
 * frees all of it (states stay valid). */
nxs_status nxs_set_workspace_limit(nxs_context* ctx, size_t bytes);
nxs_status nxs_workspace_bytes(const nxs_context* ctx, size_t* bytes);
nxs_status nxs_release_workspace(nxs_context* ctx);

/* ---------------------------------------------------------------------------
 * Serving: resident scenes, continuous batching under a workspace budget, and
 * several batches in flight.  A server has n_slots slots (0 -> 2, at most 16),
 * each a context on `device` with its own stream and workspace_budget /
 * n_slots bytes of workspace (budget 0 = no limit).  Scenes are caller-owned
 * device arrays that must stay unchanged and alive while the server uses them.
 * Requests queue in submission order.  A batch is the oldest pending request
 * together with later pending requests for the same scene with identical
 * options (up to max_batch_views, 0 -> 16, while the estimated workspace fits a
 * slot's share), rendered as one multi-view nxs_render_forward.
 * nxs_server_step collects the batches that have finished, starts a batch on
 * every free slot, and returns: batches on different slots overlap on the
 * device, and requests submitted meanwhile join later batches.  Results are
 * bitwise those of rendering each request alone with the same options.  A
 * request whose options are invalid, or that alone exceeds a slot's workspace
 * (NXS_ECAPACITY), is completed with that status without blocking the others.
 * A server is used from one host thread; outputs of a request may be read once
 * a step has reported it.
 * ------------------------------------------------------------------------- */
typedef struct nxs_server nxs_server;

nxs_status nxs_server_create(int device, size_t workspace_budget, int32_t max_batch_views,
                             int32_t n_slots, nxs_server** out);
/* Waits for every batch in flight, then frees the server. */
nxs_status nxs_server_destroy(nxs_server* server);
nxs_status nxs_server_add_scene(nxs_server* server, const nxs_gaussians* g,
                                int32_t* scene_id);
/* Queue one view of a scene; `out` (device images, caller-owned) is written
 * before a step reports the request.  Served renders keep no backward state;
 * opts.flags must be 0 (the server defers every batch itself: a batch that
 * outgrows its slot's workspace is detected when it completes and rendered
 * again, after the slot has grown or the batch has been split). */
nxs_status nxs_server_submit(nxs_server* server, int32_t scene_id, const nxs_camera* cam,
                             const nxs_render_opts* opts, const nxs_image* out, int64_t tag);
/* One scheduling step.  tags / status: host arrays of `capacity` entries
 * (capacity >= max_batch_views + n_slots); the first *n_done are filled with
 * completed requests, oldest batch first.  wait != 0: if nothing has completed,
 * block until the oldest batch in flight does.  Returns an error only if a
 * stream fails. */
nxs_status nxs_server_step(nxs_server* server, int32_t wait, int64_t* tags, int32_t* status,
                           int32_t capacity, int32_t* n_done);
/* Requests queued and not yet started; requests in flight on the slots. */
int32_t nxs_server_pending(const nxs_server* server);
int32_t nxs_server_in_flight(const nxs_server* server);
/* Workspace currently held by all slots (bytes). */
nxs_status nxs_server_workspace_bytes(const nxs_server* server, size_t* bytes);
const char* nxs_server_last_error(const nxs_server* server);

/* ---------------------------------------------------------------------------
 * Pipelined renders (for callers that enqueue many independent renders back
 * to back and want them to overlap on the device, from one object and one
 * stream).  A pipeline holds `lanes` contexts, each with a stream of its own,
 * and deals consecutive renders to them in turn: one render's latency-bound
 * sort kernels then run beside another's projection or composite.  Images
 * are those nxs_render_forward renders (Sec. 4), bitwise.
 *
 *   nxs_pipeline_create: lanes in 1..8; alloc / free / user as for nxs_create
 *     (every lane's workspace comes from them; both NULL: each lane's own
 *     stream-ordered pool).  The streams are created at the default priority.
 *   nxs_pipeline_render: as nxs_render_forward without backward state.  The
 *     render waits for the work already enqueued on `stream` (an event) and
 *     runs on the next lane's stream; `stream` itself does not wait for it.
 *     The outputs are complete, and the inputs may be changed or freed, only
 *     after nxs_pipeline_join has made a stream wait for the lanes (and that
 *     stream has reached the join).  Renders in flight at the same time must
 *     write distinct outputs.  With NXS_FLAG_DEFERRED no call waits on the
 *     host; nxs_pipeline_status then reports renders that outgrew their lane.
 *     Errors as nxs_render_forward (message: nxs_pipeline_last_error); a lane
 *     that fails is used again by the next call.
 *   nxs_pipeline_join: makes `stream` wait for every render enqueued so far
 *     (nothing waits on the host).
 *   nxs_pipeline_status: nxs_forward_status of every lane (waits for them on
 *     the host): NXS_OK, or NXS_ECAPACITY if a deferred render outgrew its
 *     lane's workspace; every lane has then grown to the largest count
 *     needed (within its workspace limit), so rendering it again succeeds on
 *     any lane.  (A render that needed a four-pass depth sort where three
 *     were launched is reported the same way; each lane then launches four
 *     once one of its own renders has needed them.)  needed (may be NULL):
 *     the largest instance count needed.
 *   nxs_pipeline_destroy: waits for the lanes, then frees them.
 * A pipeline is used by one host thread at a time.
 * ------------------------------------------------------------------------- */
typedef struct nxs_pipeline nxs_pipeline;

nxs_status nxs_pipeline_create(nxs_pipeline** pipeline, int device, int32_t lanes,
                               nxs_alloc_fn alloc, nxs_free_fn free, void* user);
nxs_status nxs_pipeline_destroy(nxs_pipeline* pipeline);
nxs_status nxs_pipeline_render(nxs_pipeline* pipeline, const nxs_gaussians* g,
                               const nxs_camera* cams, int32_t n_views,
                               const nxs_render_opts* opts, const nxs_image* out,
                               void* stream);
nxs_status nxs_pipeline_join(nxs_pipeline* pipeline, void* stream);
nxs_status nxs_pipeline_status(nxs_pipeline* pipeline, int64_t* needed);
const char* nxs_pipeline_last_error(const nxs_pipeline* pipeline);

/* Message for the last non-OK status returned on this context ("" if none).
 * The pointer stays valid until the next call on the context. */
const char* nxs_last_error(const nxs_context* ctx);

/* ---------------------------------------------------------------------------
 * Inspection of the last nxs_render_forward on a context (for testing).
 * Each call synchronises the stream of that render and copies into HOST
 * buffers the caller provides.
 * ------------------------------------------------------------------------- */

/* Measured peaks of the context's GPU, to report kernels against what this
 * build reaches as well as against the datasheet: *fp32_fma_tflops from
 * independent FP32 FMA chains (8 waves per SIMD; an FMA counts 2 flops;
 * packed FP32 is disabled in every kernel of the library, so this is the
 * non-packed rate), *copy_gbs from the best of three device-to-device copies
 * of 512 MiB (bytes read + written over time).  Takes 1 GiB of workspace
 * for the call (from the context's allocator, freed stream-ordered before
 * returning) and a few tens of milliseconds; enqueues on `stream` and
 * synchronises it.  Errors: NXS_EINVAL (null argument), NXS_ENOMEM, NXS_EHIP. */
nxs_status nxs_measure_peaks(nxs_context* ctx, double* fp32_fma_tflops, double* copy_gbs,
                             void* stream);

/* Per-stage GPU timing.  With timing enabled, each render records hipEvents
 * on its stream between its stages; nxs_inspect_stage_times then returns the
 * milliseconds of the last render's stages, in this order:
 *   0 projection, 1 depth sort, 2 instance emission, 3 tile sort,
 *   4 tile ranges (and the tile order of the queue schedules), 5 composite
 *   (with the gather of the splats it reaches).
 * ms_host has n >= NXS_N_STAGES entries.  Waits for the last render. */
#define NXS_N_STAGES 6
nxs_status nxs_set_timing(nxs_context* ctx, int32_t enable);
nxs_status nxs_inspect_stage_times(nxs_context* ctx, float* ms_host, int32_t n);

/* Number of tile instances M and of global tiles of the last render; after a
 * render that failed with NXS_ECAPACITY once M was known, the M it needed. */
nxs_status nxs_inspect_counts(nxs_context* ctx, int64_t* n_instances,
                              int64_t* n_tiles);

/* The sorted instance list: for instance j, keys_host[j] =
 * (global_tile << 32) | float32 bits of the Gaussian's camera-space depth,
 * ids_host[j] = Gaussian index; sorted by key, then index.  Global tile =
 * first tile of the view + ty * tiles_x + tx.  `capacity` is the length of
 * both host arrays; NXS_EINVAL if it is below the instance count. */
nxs_status nxs_inspect_instances(nxs_context* ctx, uint64_t* keys_host,
                                 int32_t* ids_host, int64_t capacity);

/* Per global tile [start, end) into the sorted list: ranges_host[2*t], [2*t+1]. */
nxs_status nxs_inspect_ranges(nxs_context* ctx, int32_t* ranges_host,
                              int64_t capacity);

/* Per Gaussian of view `view`: float32 depth bits (0 if culled) and the
 * covered tile rectangle (tx0, tx1, ty0, ty1) inclusive, or all -1 if culled.
 * depth_bits_host [n], rect_host [n*4]. */
nxs_status nxs_inspect_projection(nxs_context* ctx, int32_t view,
                                  uint32_t* depth_bits_host, int32_t* rect_host,
                                  int64_t capacity);

/* Per-slot sums of the last nxs_render_backward on this context, before the
 * projection's chain rule (slot = view * n + Gaussian): for each slot, 9
 * floats dLoss/d(aleph, u, v, A, B, C, r, g, b) -- the opacity aleph, the
 * image-plane centre (u, v), the conic (A, B, C) of alpha = aleph exp(-q/2)
 * with q = A dx^2 + 2 B dx dy + C dy^2, and the emission -- each summed over
 * the pixels that composited the splat (appendix "Adjoints": dL/dalpha_i and
 * dL/dE_i per pixel, chained through alpha_i).  slot_grads_host [capacity]
 * with capacity >= 9 * n * n_views.  Waits for the backward. */
nxs_status nxs_inspect_slot_grads(nxs_context* ctx, float* slot_grads_host, int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* NXS_H */
