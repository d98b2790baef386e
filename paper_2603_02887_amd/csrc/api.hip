// Host side of the C ABI declared in include/nxs.h: argument checks,
// workspace management, forward states and the launch sequence of one
// forward render and its backward.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "nxs.h"
#include "nxs_internal.h"

using namespace nxs;

// Workspace of nxs_render_forward_noalloc: one array per device, kept until
// the process ends.  Host code never names it after set-up: it uses the
// device address hipGetSymbolAddress returned on that device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// NXS_SORT_AUTO takes the tile-first order up to this many expected
// instances per tile on average (0: never)
constexpr double kAutoTileFirstPerTile = 0.0;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Where the device memory of a context comes from: the caller's callbacks,
// a stream-ordered pool of the context's own, or (the no-alloc entry point)
// a fixed region carved front to back for one call.
struct Allocator {
  nxs_alloc_fn alloc = nullptr;
  nxs_free_fn free = nullptr;
  void* user = nullptr;
  hipMemPool_t pool = nullptr;
  char* region = nullptr;
  size_t region_size = 0, region_used = 0;
};

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct nxs_fwd_state {
  nxs_context* owner = nullptr;
  // device buffers handed over by the forward (owned)
  DevBuf prec, list, ranges, order, pstate;
  hipEvent_t used = nullptr;   // after the last call that used the state
  nxs_gaussians g{};
  int model = 0, tw = 16, th = 16;
  CompositeParams cp{};
  std::vector<ViewDev> views;
  int64_t n_tiles = 0;
  bool has_order = false;
};

struct nxs_context {
  int device = 0;
  std::string err;
  Allocator al;
  char* scratch = nullptr;   // this device's scratch (nxs_render_forward_noalloc)
  bool noalloc = false;   // the no-alloc entry point: no events, no pinned memory
  // workspace
  DevBuf views, counters, partials, status;
  DevBuf depth_key, dsort_a, dsort_b, slot_a, slot_b, trect, nt_sorted, rect_sorted, prec;
  DevBuf scan_local, block_sums, counts;
  DevBuf inst_tile, inst_tile_alt, inst_val, inst_val_alt;
  DevBuf ranges, pstate, gslot, order;
  int n_cu = 256;
  std::string arch;
  size_t ws_limit = 0;   // 0: no limit on the workspace
  size_t ws_total = 0;   // bytes currently allocated for the workspace
  std::map<std::string, nxs_tuning> tuned;   // autotuner results of this process
  Counters* host_counters = nullptr;  // pinned, written by the fold kernel (no-alloc: pageable)
  // pinned copy of the deferred-render status, written by each deferred
  // render's projection (complete once `done` has fired)
  DeferredStatus* host_status = nullptr;
  bool last_deferred = false;
  bool last_failed = false;   // the last render was deferred and failed
  // view tables, pinned: a ring, so that a call fills one while the copies
  // of up to kViewRing - 1 earlier calls may still be pending (no-alloc: one
  // pageable table)
  static constexpr int kViewRing = 8;
  ViewDev* host_views[kViewRing] = {};
  hipEvent_t views_copied[kViewRing] = {};
  bool views_pending[kViewRing] = {};
  int views_next = 0;
  int host_views_cap = 0;
  hipEvent_t done = nullptr;           // recorded at the end of each call
  hipEvent_t counted = nullptr;        // the instance count has reached the host
  bool has_done = false;
  bool status_clear = false;           // the deferred-status word has been zeroed
  // optional per-stage timing (hipEvents on the render's stream)
  bool timing = false;
  hipEvent_t ev[8] = {};
  bool ev_valid = false;
  std::set<nxs_fwd_state*> states;     // states of this context not yet released
  // the last render, for inspection (last_m < 0: a deferred render whose
  // count is read from the device on demand)
  int64_t last_m = 0, last_tiles = 0, last_slots = 0;
  // first depth-sort pass to launch: 1 while the last render's plan left
  // pass 0 inactive (at most 27 varying depth bits), else 0
  int depth_first = 0;
  int32_t last_n = 0, last_views = 0;
  uint32_t* last_inst_tile = nullptr;
  uint32_t* last_inst_val = nullptr;
  const nxs_fwd_state* last_state = nullptr;   // holds last_inst_val, if any
  // instances of the context's last known render: a deferred render's tile
  // sort and ranges are launched for about this many (and loop beyond it)
  uint64_t m_hint = 0;
  int64_t last_bwd_slots = -1;   // slots of the last backward (inspection)
};

namespace {

nxs_status fail(nxs_context* ctx, nxs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, NXS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

// Device memory from the context's allocator, usable by work on `s` after
// the call.
nxs_status dev_alloc(nxs_context* ctx, size_t bytes, hipStream_t s, void** p) {
  Allocator& a = ctx->al;
  *p = nullptr;
  if (a.region) {
    if (a.region_used + bytes > a.region_size)
      return fail(ctx, NXS_ECAPACITY,
                  "the render needs more than the %zu bytes of the no-alloc scratch",
                  a.region_size);
    *p = a.region + a.region_used;
    a.region_used += bytes;
    return NXS_OK;
  }
  if (a.alloc) {
    *p = a.alloc(bytes, (void*)s, a.user);
    if (!*p) return fail(ctx, NXS_ENOMEM, "the caller's allocator failed for %zu bytes", bytes);
    if (reinterpret_cast<uintptr_t>(*p) & 255u) {
      a.free(*p, (void*)s, a.user);
      *p = nullptr;
      return fail(ctx, NXS_EINVAL, "the caller's allocator returned a block not aligned to "
                  "256 bytes");
    }
    return NXS_OK;
  }
  if (hipMallocFromPoolAsync(p, bytes, a.pool, s) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(ctx, NXS_ENOMEM, "hipMallocFromPoolAsync(%zu bytes) failed", bytes);
  }
  return NXS_OK;
}

// Gives memory back, stream-ordered after the work enqueued on `s` (all
// earlier work of the context is ordered before that point).
void dev_free(nxs_context* ctx, void* p, hipStream_t s) {
  Allocator& a = ctx->al;
  if (!p || a.region) return;
  if (a.free)
    a.free(p, (void*)s, a.user);
  else if (hipFreeAsync(p, s) != hipSuccess)
    (void)hipGetLastError();
}

void drop(nxs_context* ctx, DevBuf& b, hipStream_t s, bool workspace) {
  if (b.p) {
    dev_free(ctx, b.p, s);
    if (workspace) ctx->ws_total -= b.cap;
  }
  b.p = nullptr;
  b.cap = 0;
}

// Grow buffer b to at least `bytes` (with 25% headroom when the workspace
// limit allows it); never shrinks.  Beyond the context's workspace limit the
// call fails with NXS_ECAPACITY before freeing anything.  The old block is
// freed in stream order on `s`, so growing never waits for the device.
nxs_status ensure(nxs_context* ctx, DevBuf& b, size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return NXS_OK;
  size_t want = ctx->al.region ? round256(bytes) : round256(bytes + bytes / 4);
  if (ctx->ws_limit) {
    const size_t others = ctx->ws_total - b.cap;
    if (others + want > ctx->ws_limit) want = round256(bytes);
    if (others + want > ctx->ws_limit)
      return fail(ctx, NXS_ECAPACITY, "workspace limit: %zu bytes needed, %zu allowed",
                  others + want, ctx->ws_limit);
  }
  drop(ctx, b, s, true);
  void* p = nullptr;
  nxs_status st = dev_alloc(ctx, want, s, &p);
  if (st != NXS_OK) return st;
  b.p = p;
  b.cap = want;
  ctx->ws_total += want;
  return NXS_OK;
}

void free_workspace(nxs_context* ctx, hipStream_t s) {
  DevBuf* list[] = {&ctx->views,      &ctx->counters,  &ctx->partials,      &ctx->status,
                    &ctx->depth_key,  &ctx->dsort_a,   &ctx->dsort_b,       &ctx->slot_a,
                    &ctx->slot_b,     &ctx->trect,     &ctx->nt_sorted,     &ctx->rect_sorted,
                    &ctx->prec,       &ctx->scan_local, &ctx->block_sums,   &ctx->counts,
                    &ctx->inst_tile,  &ctx->inst_tile_alt, &ctx->inst_val,  &ctx->inst_val_alt,
                    &ctx->ranges,     &ctx->pstate,    &ctx->gslot,         &ctx->order};
  for (DevBuf* b : list) drop(ctx, *b, s, true);
  ctx->ws_total = 0;
  ctx->status_clear = false;
}

int bit_length(uint64_t x) {
  int b = 0;
  while (x) {
    ++b;
    x >>= 1;
  }
  return b;
}

template <typename T>
T* P(DevBuf& b) {
  return static_cast<T*>(b.p);
}

// Instances the context's buffers hold without growing.
uint64_t instance_capacity(const nxs_context* ctx) {
  const size_t c = std::min(std::min(ctx->inst_tile.cap, ctx->inst_tile_alt.cap),
                            std::min(ctx->inst_val.cap, ctx->inst_val_alt.cap));
  return std::min<uint64_t>(c / 4, 0xFFFFFFFEull);
}

nxs_status grow_instances(nxs_context* ctx, uint64_t m, int64_t S, hipStream_t s) {
  nxs_status st;
  if ((st = ensure(ctx, ctx->counts, 4 * radix_counts_words(std::max<int64_t>(S, (int64_t)m)),
                   s)) ||
      (st = ensure(ctx, ctx->inst_tile, 4 * m, s)) ||
      (st = ensure(ctx, ctx->inst_tile_alt, 4 * m, s)) ||
      (st = ensure(ctx, ctx->inst_val, 4 * m, s)) ||
      (st = ensure(ctx, ctx->inst_val_alt, 4 * m, s)))
    return st;
  return NXS_OK;
}

}  // namespace

// After the context's work: instance buffers for `need` instances (a pipeline
// grows every lane to what one of them needed).
nxs_status nxs::grow_instance_capacity(nxs_context* ctx, uint64_t need) {
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_done) HIP_TRY(hipEventSynchronize(ctx->done));
  if (need == 0 || need >= 0xFFFFFFFFull || need <= instance_capacity(ctx)) return NXS_OK;
  return grow_instances(ctx, need, ctx->last_slots, nullptr);
}

namespace {

// Records ctx->done on `s` when it goes out of scope once work has been
// enqueued (so that the next call on any stream orders after a failed one).
struct DoneGuard {
  nxs_context* ctx;
  hipStream_t s;
  bool armed = false;
  ~DoneGuard() {
    if (!armed || ctx->noalloc) return;
    if (hipEventRecord(ctx->done, s) == hipSuccess)
      ctx->has_done = true;
    else
      (void)hipGetLastError();
  }
};

void release_state(nxs_context* ctx, nxs_fwd_state* st, hipStream_t s) {
  DevBuf* bufs[] = {&st->prec, &st->list, &st->ranges, &st->order, &st->pstate};
  for (DevBuf* b : bufs) drop(ctx, *b, s, false);
  if (st->used) (void)hipEventDestroy(st->used);
  if (ctx->last_state == st) {
    ctx->last_state = nullptr;
    ctx->last_inst_val = nullptr;
    ctx->last_inst_tile = nullptr;
  }
  ctx->states.erase(st);
  delete st;
}

}  // namespace

namespace {

std::string tuning_key(const nxs_context* ctx, const nxs_gaussians* g, const nxs_camera* cams,
                       int32_t n_views, const nxs_render_opts* opts) {
  char buf[160];
  snprintf(buf, sizeof(buf), "%s|cu%d|n%d|sh%d|m%d|p%.6g|v%d", ctx->arch.c_str(), ctx->n_cu,
           g->n, g->sh_degree, opts->model, (double)opts->param, n_views);
  std::string k = buf;
  for (int v = 0; v < n_views; ++v) {
    snprintf(buf, sizeof(buf), "|%dx%d", cams[v].width, cams[v].height);
    k += buf;
  }
  return k;
}

bool read_cache(const char* path, const std::string& key, nxs_tuning* t) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[4000];
    nxs_tuning r{};
    if (sscanf(line, "%3999s %d %d %d %d %d %f", k, &r.tile_w, &r.tile_h, &r.schedule,
               &r.lds_batch, &r.sort_order, &r.ms) == 7 &&
        key == k) {
      *t = r;   // the last line for a key wins
      found = true;
    }
  }
  fclose(f);
  return found;
}

void append_cache(const char* path, const std::string& key, const nxs_tuning& t) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %d %d %.5f\n", key.c_str(), t.tile_w, t.tile_h, t.schedule,
          t.lds_batch, t.sort_order, (double)t.ms);
  fclose(f);
}

// Everything a render needs, checked, before anything is launched.
struct Checked {
  int tw, th, sched, batch, sort_order;
  float alpha_min, t_eps, param;
  int64_t total_tiles, S;
  bool deferred;
};

nxs_status check_args(nxs_context* ctx, const nxs_gaussians* g, const nxs_camera* cams,
                      int32_t n_views, const nxs_render_opts* opts, const nxs_image* out,
                      Checked* c) {
  if (!g || !cams || !opts || !out) return fail(ctx, NXS_EINVAL, "null argument");
  if (n_views < 1) return fail(ctx, NXS_EINVAL, "n_views must be >= 1");
  if (g->n < 0) return fail(ctx, NXS_EINVAL, "n must be >= 0");
  if (g->sh_degree < 0 || g->sh_degree > 3)
    return fail(ctx, NXS_EINVAL, "sh_degree must be 0..3");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
    return fail(ctx, NXS_EINVAL, "null Gaussian array");
  if (opts->model < 0 || opts->model > 7) return fail(ctx, NXS_EINVAL, "unknown model %d", opts->model);
  const float param = opts->param;
  if (opts->model == NXS_QUADRATIC && !(param >= -0.5f))
    return fail(ctx, NXS_EINVAL, "quadratic c must be >= -0.5");
  if ((opts->model == NXS_BLENDED || opts->model == NXS_VICINI) &&
      !(param >= 0.0f && param <= 1.0f))
    return fail(ctx, NXS_EINVAL, "gamma must be in [0, 1]");
  if (opts->model == NXS_POWER_LAW && !(param != 0.0f && std::isfinite(param)))
    return fail(ctx, NXS_EINVAL, "power-law v must be finite and non-zero");
  if (opts->flags & ~NXS_FLAG_DEFERRED)
    return fail(ctx, NXS_EINVAL, "unknown flags 0x%x", (unsigned)opts->flags);
  c->tw = opts->tile_w ? opts->tile_w : 16;
  c->th = opts->tile_h ? opts->tile_h : 16;
  if (!((c->tw == 8 && c->th == 8) || (c->tw == 16 && c->th == 16) ||
        (c->tw == 32 && c->th == 8)))
    return fail(ctx, NXS_EINVAL, "tile size %dx%d not supported (8x8, 16x16, 32x8)", c->tw,
                c->th);
  c->sched = opts->schedule ? opts->schedule : NXS_SCHED_QUEUE;
  if (c->sched < NXS_SCHED_TILES || c->sched > NXS_SCHED_PERSISTENT)
    return fail(ctx, NXS_EINVAL, "schedule %d not supported (0..4)", opts->schedule);
  c->batch = opts->lds_batch ? opts->lds_batch : 64;
  if (c->batch != 64 && c->batch != 128 && c->batch != 256)
    return fail(ctx, NXS_EINVAL, "lds_batch must be 0, 64, 128 or 256");
  c->sort_order = opts->sort_order;
  if (c->sort_order < NXS_SORT_AUTO || c->sort_order > NXS_SORT_TILE_FIRST)
    return fail(ctx, NXS_EINVAL, "sort_order %d not supported (0..2)", opts->sort_order);
  c->alpha_min = opts->alpha_min > 0.0f ? opts->alpha_min : 1e-3f;
  if (!(c->alpha_min < 1.0f)) return fail(ctx, NXS_EINVAL, "alpha_min must be in (0, 1)");
  c->t_eps = opts->t_eps == 0.0f ? 1e-4f : opts->t_eps;
  c->param = param;
  c->total_tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    const nxs_camera& cm = cams[v];
    if (cm.width <= 0 || cm.height <= 0 || cm.width > 32768 || cm.height > 32768)
      return fail(ctx, NXS_EINVAL, "view %d: bad size %dx%d", v, cm.width, cm.height);
    if (!out[v].rgb || !out[v].trans) return fail(ctx, NXS_EINVAL, "view %d: null output", v);
    if (!(cm.fx > 0.0f) || !(cm.fy > 0.0f)) return fail(ctx, NXS_EINVAL, "view %d: bad focal", v);
    c->total_tiles += (int64_t)((cm.width + c->tw - 1) / c->tw) * ((cm.height + c->th - 1) / c->th);
  }
  if (c->total_tiles >= (int64_t)1 << 31) return fail(ctx, NXS_EINVAL, "too many tiles");
  c->S = (int64_t)g->n * n_views;
  if (c->S >= ((int64_t)1 << 32) - 1) return fail(ctx, NXS_EINVAL, "n * n_views too large");
  c->deferred = (opts->flags & NXS_FLAG_DEFERRED) != 0;
  return NXS_OK;
}

// The forward of include/nxs.h, arguments already checked.
nxs_status forward(nxs_context* ctx, const nxs_gaussians* g, const nxs_camera* cams,
                   int32_t n_views, const nxs_render_opts* opts, const nxs_image* out,
                   const Checked& c, nxs_fwd_state** state_out, hipStream_t s) {
  const int tw = c.tw, th = c.th, sched = c.sched;
  const int64_t total_tiles = c.total_tiles, S = c.S;
  HIP_TRY(hipSetDevice(ctx->device));
  // the workspace is shared by all calls on this context: order after the last one
  if (ctx->has_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
  ctx->last_inst_tile = ctx->last_inst_val = nullptr;
  ctx->last_state = nullptr;
  ctx->last_m = 0;
  ctx->last_deferred = false;
  ctx->last_failed = false;

  // ---- view table -----------------------------------------------------------
  // Up to kArgViews views reach the projection as a kernel argument, which
  // writes the device table.  More views are copied from a pinned table of
  // the ring whose last copy has completed (the copy is asynchronous, so a
  // table is not reused before its event has fired).
  const bool by_arg = g->n > 0 && n_views <= kArgViews;
  std::vector<ViewDev> arg_views(by_arg ? n_views : 0);
  int ring = 0;
  if (!ctx->noalloc && !by_arg) {
    if (ctx->host_views_cap < n_views) {
      for (int k = 0; k < nxs_context::kViewRing; ++k) {
        if (ctx->views_pending[k]) HIP_TRY(hipEventSynchronize(ctx->views_copied[k]));
        ctx->views_pending[k] = false;
        if (ctx->host_views[k]) (void)hipHostFree(ctx->host_views[k]);
        ctx->host_views[k] = nullptr;
      }
      ctx->host_views_cap = 0;
      for (int k = 0; k < nxs_context::kViewRing; ++k)
        HIP_TRY(hipHostMalloc((void**)&ctx->host_views[k], sizeof(ViewDev) * n_views,
                              hipHostMallocDefault));
      ctx->host_views_cap = n_views;
    }
    ring = ctx->views_next;
    ctx->views_next = (ring + 1) % nxs_context::kViewRing;
    if (ctx->views_pending[ring]) {
      HIP_TRY(hipEventSynchronize(ctx->views_copied[ring]));
      ctx->views_pending[ring] = false;
    }
  }
  ViewDev* host_views = by_arg ? arg_views.data() : ctx->host_views[ring];
  int64_t off = 0, pix_off = 0;
  for (int v = 0; v < n_views; ++v) {
    const nxs_camera& cm = cams[v];
    ViewDev& d = host_views[v];
    std::memset(&d, 0, sizeof(d));
    std::memcpy(d.R, cm.R, sizeof(d.R));
    std::memcpy(d.t, cm.t, sizeof(d.t));
    d.fx = cm.fx; d.fy = cm.fy; d.cx = cm.cx; d.cy = cm.cy; d.znear = cm.znear;
    for (int k = 0; k < 3; ++k)
      d.campos[k] = (float)-((double)cm.R[k] * cm.t[0] + (double)cm.R[3 + k] * cm.t[1] +
                             (double)cm.R[6 + k] * cm.t[2]);
    d.width = cm.width; d.height = cm.height;
    d.tiles_x = (cm.width + tw - 1) / tw;
    d.tiles_y = (cm.height + th - 1) / th;
    d.tile_off = (int32_t)off;
    off += (int64_t)d.tiles_x * d.tiles_y;
    d.pix_off = pix_off;
    pix_off += (int64_t)cm.width * cm.height;
    d.rgb = out[v].rgb; d.trans = out[v].trans; d.od = out[v].overdraw;
  }
  // a deferred render needs instance buffers sized by an earlier render;
  // until then it waits for the count like any other
  const bool deferred = c.deferred && !ctx->noalloc && instance_capacity(ctx) > 0;
  DoneGuard guard{ctx, s};
  nxs_status st;
  if ((st = ensure(ctx, ctx->views, sizeof(ViewDev) * n_views, s))) return st;
  if ((st = ensure(ctx, ctx->counters, sizeof(Counters), s))) return st;
  if ((st = ensure(ctx, ctx->partials, sizeof(uint4) * project_partials_size(g->n), s)))
    return st;
  guard.armed = true;
  if (!by_arg) {
    HIP_TRY(hipMemcpyAsync(ctx->views.p, host_views, sizeof(ViewDev) * n_views,
                           hipMemcpyHostToDevice, s));
    if (!ctx->noalloc) {
      HIP_TRY(hipEventRecord(ctx->views_copied[ring], s));
      ctx->views_pending[ring] = true;
    }
  }
  const ViewDev* dviews = P<ViewDev>(ctx->views);

  // ---- per-slot buffers and projection ----------------------------------------
  if ((st = ensure(ctx, ctx->depth_key, 4 * S, s)) || (st = ensure(ctx, ctx->dsort_a, 4 * S, s)) ||
      (st = ensure(ctx, ctx->dsort_b, 4 * S, s)) ||
      (st = ensure(ctx, ctx->slot_a, 4 * S, s)) || (st = ensure(ctx, ctx->slot_b, 4 * S, s)) ||
      (st = ensure(ctx, ctx->trect, 8 * S, s)) || (st = ensure(ctx, ctx->nt_sorted, 4 * S, s)) ||
      (st = ensure(ctx, ctx->rect_sorted, 8 * S, s)) ||
      (st = ensure(ctx, ctx->prec, 48 * S, s)) || (st = ensure(ctx, ctx->scan_local, 4 * S, s)) ||
      (st = ensure(ctx, ctx->block_sums, 4 * scan_blocks_size(S), s)) ||
      (st = ensure(ctx, ctx->counts, 4 * radix_counts_words(S), s)) ||
      (st = ensure(ctx, ctx->ranges, 8 * total_tiles + 4 * kSchedCounters, s)))
    return st;
  uint64_t icap = 0;   // deferred: the instances this render may use
  if (deferred) {
    if ((st = ensure(ctx, ctx->status, sizeof(DeferredStatus), s))) return st;
    if (!ctx->status_clear) {
      launch_fill_u32(P<uint32_t>(ctx->status), sizeof(DeferredStatus) / 4, 0u, s);
      ctx->status_clear = true;
    }
    icap = instance_capacity(ctx);
    // (the count of the latest deferred render whose status has landed)
    if (ctx->host_status->last) ctx->m_hint = ctx->host_status->last;
    if ((st = ensure(ctx, ctx->counts, 4 * radix_counts_words(std::max<int64_t>(S, icap)), s)))
      return st;
  }
  ProjDev proj{P<uint32_t>(ctx->depth_key), P<uint2>(ctx->trect), P<float4>(ctx->prec)};
  GaussDev gd{g->means, g->scales, g->quats, g->opacities, g->sh, g->n, g->sh_degree};
  Counters* dcount = P<Counters>(ctx->counters);
  const float kappa2 = (float)(2.0 * std::log(1.0 / (double)c.alpha_min));
  auto mark = [&](int k) -> hipError_t {
    return ctx->timing ? hipEventRecord(ctx->ev[k], s) : hipSuccess;
  };
  ctx->ev_valid = false;
  HIP_TRY(mark(0));
  // the list order: the caller's, else by the expected instances per tile
  // (the hint, else the context's last count; unknown: depth first)
  bool tile_first = c.sort_order == NXS_SORT_TILE_FIRST;
  if (c.sort_order == NXS_SORT_AUTO) {
    const double expect = opts->instance_hint > 0.0f ? (double)opts->instance_hint
                                                     : (double)ctx->m_hint;
    tile_first = expect > 0.0 && expect <= kAutoTileFirstPerTile * (double)total_tiles;
  }
  const int depth_first = (ctx->noalloc || tile_first) ? 0 : ctx->depth_first;
  // (the fold writes the counters, or a deferred render's status, straight
  // into the context's pinned memory; the no-alloc call copies them)
  DeferCheck chk{~0ull, 0, nullptr, nullptr, ctx->noalloc ? nullptr : ctx->host_counters};
  if (deferred)
    chk = DeferCheck{icap, depth_first, P<DeferredStatus>(ctx->status), ctx->host_status,
                     nullptr};
  // (also clears the tile ranges and, after them, the composite schedules'
  // counters)
  if (!launch_project(gd, P<ViewDev>(ctx->views), by_arg ? host_views : nullptr, n_views,
                      kappa2, c.alpha_min, tw, th, proj, P<uint4>(ctx->partials), dcount, chk,
                      P<uint32_t>(ctx->ranges), 2 * total_tiles + kSchedCounters, s))
    return fail(ctx, NXS_EHIP, "the view table could not be passed to the projection");
  HIP_TRY(hipGetLastError());
  HIP_TRY(mark(1));
  // The instance count M is read by the host only where it sizes buffers and
  // grids: the depth sort (its digits planned on the device) and the emission
  // (total read on the device, writes bounded by the current capacity) are
  // enqueued first, so the GPU keeps working while the host waits.  (Copying
  // the counters on a second stream, beside the depth sort, was measured
  // slower: the cross-stream wait costs more than the copy.)  A deferred
  // render reads nothing.
  if (!deferred) {
    if (ctx->noalloc)
      HIP_TRY(hipMemcpyAsync(ctx->host_counters, dcount, sizeof(Counters),
                             hipMemcpyDeviceToHost, s));
    else
      HIP_TRY(hipEventRecord(ctx->counted, s));
  }
  HIP_TRY(mark(2));
  // 1. depth sort of the slots (values: the slots 0..S-1)
  //    (its last pass also lays out the slots' tile counts and rectangles in
  //    that order, so that the emission reads them coalesced)
  //    (launched from the pass the last render's plan needed; checked below,
  //    or on the device for a deferred render)
  auto depth_sort = [&](int first) {
    return radix_sort_planned(P<uint32_t>(ctx->depth_key), nullptr, P<uint32_t>(ctx->dsort_a),
                              P<uint32_t>(ctx->slot_a), P<uint32_t>(ctx->dsort_b),
                              P<uint32_t>(ctx->slot_b), S, dcount->plan, first,
                              P<uint32_t>(ctx->counts), proj.trect,
                              P<uint32_t>(ctx->nt_sorted), P<uint2>(ctx->rect_sorted), s);
  };
  // (tile first: no depth sort; the slots are emitted in their own order)
  uint32_t* sorted_slots = nullptr;
  if (!tile_first) {
    const int wd = depth_sort(depth_first);
    sorted_slots = wd ? P<uint32_t>(ctx->slot_b) : P<uint32_t>(ctx->slot_a);
  }
  const uint32_t* nt_in = tile_first ? nullptr : P<uint32_t>(ctx->nt_sorted);
  const uint2* rect_in = tile_first ? nullptr : P<uint2>(ctx->rect_sorted);
  HIP_TRY(mark(3));
  // 2. emission (in depth order, or in slot order), into the buffers as they are
  launch_emit_scan(nt_in, proj.trect, S, P<uint32_t>(ctx->scan_local),
                   P<uint32_t>(ctx->block_sums), s);
  const uint32_t cap32 = (uint32_t)instance_capacity(ctx);
  if (cap32 > 0)
    launch_emit_write(sorted_slots, rect_in, proj.trect, S, g->n, dviews,
                      P<uint32_t>(ctx->scan_local), P<uint32_t>(ctx->block_sums), cap32,
                      P<uint32_t>(ctx->inst_tile), P<uint32_t>(ctx->inst_val), s);
  HIP_TRY(hipGetLastError());
  uint64_t M = 0;          // instances (deferred: their upper bound)
  if (!deferred) {
    if (ctx->noalloc)
      HIP_TRY(hipStreamSynchronize(s));
    else
      HIP_TRY(hipEventSynchronize(ctx->counted));
    M = ctx->host_counters->total;
    // (every earlier render has completed, its status copy included: this
    // count is now the newest one)
    ctx->m_hint = M;
    if (!ctx->noalloc) ctx->host_status->last = 0;
    // the depth sort skipped pass 0 but this render's plan needs it: sort and
    // emit again below (the depth keys are intact)
    const bool pass0 = (ctx->host_counters->plan[0] & kPassActive) != 0;
    const bool resort = !tile_first && S > 0 && depth_first == 1 && pass0;
    if (!ctx->noalloc) ctx->depth_first = pass0 ? 0 : 1;
    // what this render needs, visible through nxs_inspect_counts even if it fails
    ctx->last_m = (int64_t)M;
    ctx->last_tiles = total_tiles;
    if (M >= 0xFFFFFFFFull)
      return fail(ctx, NXS_ECAPACITY, "%llu tile instances exceed the 32-bit range",
                  (unsigned long long)M);
    // ---- instance buffers (growing them is stream-ordered) -------------------
    if ((st = grow_instances(ctx, M, S, s))) return st;
    if (resort) {
      (void)depth_sort(0);
      launch_emit_scan(nt_in, proj.trect, S, P<uint32_t>(ctx->scan_local),
                       P<uint32_t>(ctx->block_sums), s);
    }
    if (resort || M > cap32)   // emit (again) into the grown buffers
      launch_emit_write(sorted_slots, rect_in, proj.trect, S, g->n, dviews,
                        P<uint32_t>(ctx->scan_local), P<uint32_t>(ctx->block_sums),
                        (uint32_t)M, P<uint32_t>(ctx->inst_tile), P<uint32_t>(ctx->inst_val),
                        s);
  } else {
    M = icap;
    ctx->last_m = -1;
    ctx->last_tiles = total_tiles;
  }
  const Counters* dn = deferred ? dcount : nullptr;
  // deferred: grids for the expected count (the caller's hint, else the
  // context's last count), not the capacity
  const uint64_t expect = opts->instance_hint > 0.0f && std::isfinite(opts->instance_hint)
                              ? (uint64_t)std::min(opts->instance_hint, 4.0e9f)
                              : ctx->m_hint;
  const int64_t m_plan =
      deferred ? (int64_t)std::min<uint64_t>(M, expect + expect / 4 + 4096) : (int64_t)M;
  uint32_t* inst_tile = P<uint32_t>(ctx->inst_tile);
  uint32_t* inst_val = P<uint32_t>(ctx->inst_val);
  bool list_alt = false;
  HIP_TRY(mark(4));
  if (M > 0) {
    // 3. stable sort by global tile
    const int tbits = bit_length((uint64_t)(total_tiles - 1));
    const int wt = radix_sort(inst_tile, inst_val, P<uint32_t>(ctx->inst_tile_alt),
                              P<uint32_t>(ctx->inst_val_alt), inst_tile, inst_val, (int64_t)M,
                              tbits, P<uint32_t>(ctx->counts), s, dn, m_plan);
    if (wt == 0) {
      inst_tile = P<uint32_t>(ctx->inst_tile_alt);
      inst_val = P<uint32_t>(ctx->inst_val_alt);
      list_alt = true;
    }
    HIP_TRY(mark(5));
    // 4. tile ranges
    launch_ranges(inst_tile, (int64_t)M, P<uint2>(ctx->ranges), s, dn, m_plan);
    // 4a. tile first: each tile's list (in slot order) by depth, through the
    //     buffer the tile sort left free
    if (tile_first)
      launch_tile_depth_sort(P<uint2>(ctx->ranges), total_tiles, P<uint32_t>(ctx->depth_key),
                             dcount, inst_val,
                             list_alt ? P<uint32_t>(ctx->inst_val) : P<uint32_t>(ctx->inst_val_alt),
                             s);
  } else {
    HIP_TRY(mark(5));
  }
  // 4b. the tile order of the queue schedules (longest tile lists first)
  // (the composite gathers the records of the sorted slots batch by batch)
  CompositeLaunch cl{sched, tw, th, total_tiles, dviews, n_views, P<uint2>(ctx->ranges),
                     inst_val, proj.rec, nullptr, nullptr, ctx->n_cu};
  if (sched == NXS_SCHED_QUEUE || sched == NXS_SCHED_PERSISTENT) {
    if ((st = ensure(ctx, ctx->order, 8 * (size_t)total_tiles, s))) return st;
    cl.order = P<uint32_t>(ctx->order);
    cl.sched_counters = P<uint32_t>(ctx->ranges) + 2 * total_tiles;
    launch_composite_order(cl, s);
  }
  float4* pstate = nullptr;
  if (state_out) {
    if ((st = ensure(ctx, ctx->pstate, 48 * (size_t)pix_off, s))) return st;
    pstate = P<float4>(ctx->pstate);
  }
  CompositeParams cp;
  cp.log2_alpha_min = (float)std::log2((double)c.alpha_min);
  // the exponential parts stop once T < cp.t_eps; "never" is the smallest
  // normal float, below which the float32 product would underflow
  cp.t_eps = (opts->model == NXS_EXPONENTIAL || opts->model == NXS_VICINI)
                 ? (c.t_eps > 0.0f ? c.t_eps : 1.17549435e-38f)
                 : 0.0f;
  cp.param = c.param;
  for (int k = 0; k < 3; ++k) cp.bg[k] = opts->background[k];
  cp.lds_batch = c.batch;
  HIP_TRY(mark(6));
  // 5. composite (also writes the background where no splat lands)
  launch_composite(opts->model, cl, cp, pstate, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(mark(7));
  ctx->ev_valid = ctx->timing;
  ctx->last_deferred = deferred;

  ctx->last_slots = S;
  ctx->last_n = g->n;
  ctx->last_views = n_views;
  ctx->last_inst_tile = inst_tile;
  ctx->last_inst_val = inst_val;

  if (state_out) {
    // hand the buffers the backward re-reads to a new state; the context
    // allocates fresh ones for its next render
    nxs_fwd_state* fs = new (std::nothrow) nxs_fwd_state();
    if (!fs) return fail(ctx, NXS_ENOMEM, "out of host memory");
    if (hipEventCreateWithFlags(&fs->used, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      delete fs;
      return fail(ctx, NXS_EHIP, "hipEventCreate failed");
    }
    fs->owner = ctx;
    auto take = [&](DevBuf& from, DevBuf& to) {
      to = from;
      ctx->ws_total -= from.cap;
      from = DevBuf{};
    };
    take(ctx->prec, fs->prec);
    take(list_alt ? ctx->inst_val_alt : ctx->inst_val, fs->list);
    take(ctx->ranges, fs->ranges);
    take(ctx->pstate, fs->pstate);
    fs->has_order = cl.order != nullptr;
    if (fs->has_order) take(ctx->order, fs->order);
    fs->g = *g;
    fs->model = opts->model;
    fs->tw = tw;
    fs->th = th;
    fs->cp = cp;
    fs->n_tiles = total_tiles;
    fs->views.assign(host_views, host_views + n_views);
    HIP_TRY(hipEventRecord(fs->used, s));
    ctx->states.insert(fs);
    ctx->last_state = fs;
    *state_out = fs;
  }
  return NXS_OK;   // (the guard records `done` on the stream)
}

}  // namespace

extern "C" {

nxs_status nxs_create(nxs_context** out, int device, nxs_alloc_fn alloc, nxs_free_fn free_fn,
                      void* user) {
  if (!out) return NXS_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return NXS_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return NXS_EINVAL;
  nxs_context* ctx = new (std::nothrow) nxs_context();
  if (!ctx) return NXS_ENOMEM;
  ctx->device = device;
  ctx->al.alloc = alloc;
  ctx->al.free = free_fn;
  ctx->al.user = user;
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipHostMalloc((void**)&ctx->host_counters, sizeof(Counters),
                          hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&ctx->host_status, sizeof(DeferredStatus),
                          hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->counted, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < nxs_context::kViewRing && ok; ++k)
    ok = hipEventCreateWithFlags(&ctx->views_copied[k], hipEventDisableTiming) == hipSuccess;
  if (ok && !alloc) {
    // a pool of the context's own that keeps freed memory for reuse (no
    // release threshold), so that stream-ordered frees and allocations
    // recycle blocks without returning them to the driver
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    ok = hipMemPoolCreate(&ctx->al.pool, &props) == hipSuccess;
    if (ok) {
      uint64_t keep = ~0ull;
      ok = hipMemPoolSetAttribute(ctx->al.pool, hipMemPoolAttrReleaseThreshold, &keep) ==
           hipSuccess;
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
    if (ctx->host_status) (void)hipHostFree(ctx->host_status);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->counted) (void)hipEventDestroy(ctx->counted);
    for (int k = 0; k < nxs_context::kViewRing; ++k)
      if (ctx->views_copied[k]) (void)hipEventDestroy(ctx->views_copied[k]);
    if (ctx->al.pool) (void)hipMemPoolDestroy(ctx->al.pool);
    delete ctx;
    return NXS_EHIP;
  }
  // the scratch of the allocation-free forward: its address on this device,
  // looked up once per device with the device current
  if (ok) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (device < kMaxDevices && !g_scratch[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
        g_scratch[device] = static_cast<char*>(p);
      else
        (void)hipGetLastError();
    }
    ctx->scratch = device < kMaxDevices ? g_scratch[device] : nullptr;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->arch = prop.gcnArchName;
  }
  *out = ctx;
  return NXS_OK;
}

nxs_status nxs_destroy(nxs_context* ctx) {
  if (!ctx) return NXS_EINVAL;
  (void)hipSetDevice(ctx->device);
  if (ctx->has_done) (void)hipEventSynchronize(ctx->done);
  while (!ctx->states.empty()) {
    nxs_fwd_state* st = *ctx->states.begin();
    if (st->used) (void)hipEventSynchronize(st->used);
    release_state(ctx, st, nullptr);
  }
  free_workspace(ctx, nullptr);
  if (ctx->al.pool) {
    (void)hipDeviceSynchronize();   // the frees above complete before the pool goes
    (void)hipMemPoolDestroy(ctx->al.pool);
  }
  if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
  if (ctx->host_status) (void)hipHostFree(ctx->host_status);
  for (int k = 0; k < nxs_context::kViewRing; ++k) {
    if (ctx->host_views[k]) (void)hipHostFree(ctx->host_views[k]);
    if (ctx->views_copied[k]) (void)hipEventDestroy(ctx->views_copied[k]);
  }
  if (ctx->done) (void)hipEventDestroy(ctx->done);
  if (ctx->counted) (void)hipEventDestroy(ctx->counted);
  for (int k = 0; k < 8; ++k)
    if (ctx->ev[k]) (void)hipEventDestroy(ctx->ev[k]);
  delete ctx;
  return NXS_OK;
}

const char* nxs_last_error(const nxs_context* ctx) { return ctx ? ctx->err.c_str() : ""; }

nxs_status nxs_render_forward(nxs_context* ctx, const nxs_gaussians* g,
                              const nxs_camera* cams, int32_t n_views,
                              const nxs_render_opts* opts, const nxs_image* out,
                              nxs_fwd_state** state, void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (state) *state = nullptr;
  Checked c;
  nxs_status st = check_args(ctx, g, cams, n_views, opts, out, &c);
  if (st != NXS_OK) return st;
  if (state && opts->model > NXS_QUADRATIC)
    return fail(ctx, NXS_EUNSUPPORTED, "backward state: models 0..4, not %d", opts->model);
  return forward(ctx, g, cams, n_views, opts, out, c, state, (hipStream_t)stream);
}

nxs_status nxs_render_forward_noalloc(nxs_context* ctx, const nxs_gaussians* g,
                                      const nxs_camera* cams, int32_t n_views,
                                      const nxs_render_opts* opts, const nxs_image* out,
                                      void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  Checked c;
  nxs_status st = check_args(ctx, g, cams, n_views, opts, out, &c);
  if (st != NXS_OK) return st;
  if (opts->flags) return fail(ctx, NXS_EINVAL, "the no-alloc forward takes no flags");
  if (!ctx->scratch)
    return fail(ctx, NXS_EHIP, "no scratch address for device %d", ctx->device);
  // a context of this call only: its buffers are carved from the scratch,
  // its host tables are ordinary memory, and it records no events
  nxs_context tmp;
  tmp.device = ctx->device;
  tmp.noalloc = true;
  tmp.n_cu = ctx->n_cu;
  tmp.al.region = ctx->scratch;
  tmp.al.region_size = kScratchBytes;
  Counters counters{};
  std::vector<ViewDev> views(n_views);
  tmp.host_counters = &counters;
  tmp.host_views[0] = views.data();
  tmp.host_views_cap = n_views;
  hipStream_t s = (hipStream_t)stream;
  // ordered after the context's own calls (the scratch is not theirs, but
  // the caller's inputs and outputs may be)
  if (ctx->has_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
  st = forward(&tmp, g, cams, n_views, opts, out, c, nullptr, s);
  if (st != NXS_OK) {
    ctx->err = tmp.err;
    return st;
  }
  return NXS_OK;
}

nxs_status nxs_forward_status(nxs_context* ctx, int64_t* needed) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (needed) *needed = 0;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_done) HIP_TRY(hipEventSynchronize(ctx->done));
  if (!ctx->status.p || !ctx->status_clear) return NXS_OK;
  // (the last deferred render copied the status here before `done`)
  const DeferredStatus ds = *ctx->host_status;
  if (ds.count == 0) return NXS_OK;
  DeferredStatus zero{};
  zero.last = ds.last;
  zero.last_fail = ds.last_fail;
  HIP_TRY(hipMemcpy(ctx->status.p, &zero, sizeof(zero), hipMemcpyHostToDevice));
  *ctx->host_status = zero;
  if (needed) *needed = (int64_t)ds.need;
  if (ds.fail & kFailPlan) ctx->depth_first = 0;
  if (ds.need >= 0xFFFFFFFFull)
    return fail(ctx, NXS_ECAPACITY, "%u deferred render(s) failed: %llu tile instances exceed "
                "the 32-bit range", ds.count, (unsigned long long)ds.need);
  if ((ds.fail & kFailCapacity) && ds.need > instance_capacity(ctx)) {
    // all of the context's work has completed: grow on the null stream
    nxs_status st = grow_instances(ctx, ds.need, ctx->last_slots, nullptr);
    if (st != NXS_OK) {
      const std::string why = ctx->err;
      return fail(ctx, NXS_ECAPACITY, "%u deferred render(s) failed; growing to %llu "
                  "instances failed too: %s", ds.count, (unsigned long long)ds.need,
                  why.c_str());
    }
  }
  if (!(ds.fail & kFailCapacity))
    return fail(ctx, NXS_ECAPACITY, "%u deferred render(s) needed a four-pass depth sort "
                "where the context launched three; it now launches four: render them again",
                ds.count);
  return fail(ctx, NXS_ECAPACITY, "%u deferred render(s) outgrew the workspace (%llu "
              "instances needed); the context has grown: render them again", ds.count,
              (unsigned long long)ds.need);
}

nxs_status nxs_render_backward(nxs_context* ctx, const nxs_fwd_state* state,
                               const float* const* dL_drgb, const float* const* dL_dtrans,
                               const nxs_gaussians_grad* grads, void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (!state) return fail(ctx, NXS_EINVAL, "null state");
  nxs_fwd_state* fs = const_cast<nxs_fwd_state*>(state);
  if (fs->owner != ctx || !ctx->states.count(fs))
    return fail(ctx, NXS_EINVAL, "the state is not a live state of this context");
  if (!dL_drgb || !grads) return fail(ctx, NXS_EINVAL, "null argument");
  const nxs_gaussians& g = fs->g;
  if (g.n > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacities ||
                  !grads->sh))
    return fail(ctx, NXS_EINVAL, "null gradient array");
  const int n_views = (int)fs->views.size();
  std::vector<ViewDev> views = fs->views;
  for (int v = 0; v < n_views; ++v) {
    if (!dL_drgb[v]) return fail(ctx, NXS_EINVAL, "view %d: null dL_drgb", v);
    views[v].g_rgb = dL_drgb[v];
    views[v].g_trans = dL_dtrans ? dL_dtrans[v] : nullptr;
  }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
  HIP_TRY(hipStreamWaitEvent(s, fs->used, 0));
  DoneGuard guard{ctx, s};
  nxs_status st;
  const int64_t S = (int64_t)g.n * n_views;
  if ((st = ensure(ctx, ctx->gslot, 36 * (size_t)S, s))) return st;
  if ((st = ensure(ctx, ctx->views, sizeof(ViewDev) * n_views, s))) return st;
  guard.armed = true;
  // pageable source: the copy has consumed `views` when the call returns
  HIP_TRY(hipMemcpyAsync(ctx->views.p, views.data(), sizeof(ViewDev) * n_views,
                         hipMemcpyHostToDevice, s));
  launch_fill_u32(P<uint32_t>(ctx->gslot), 9 * S, 0u, s);
  launch_composite_bwd(fs->model, fs->tw, fs->th, fs->n_tiles, P<ViewDev>(ctx->views), n_views,
                       P<uint2>(fs->ranges), P<uint32_t>(fs->list), P<float4>(fs->prec),
                       fs->cp, P<float4>(fs->pstate), P<float>(ctx->gslot),
                       fs->has_order ? P<uint32_t>(fs->order) : nullptr, s);
  GaussDev gd{g.means, g.scales, g.quats, g.opacities, g.sh, g.n, g.sh_degree};
  GaussGradDev gg{grads->means, grads->scales, grads->quats, grads->opacities, grads->sh};
  launch_project_bwd(gd, P<ViewDev>(ctx->views), n_views, P<float>(ctx->gslot), gg, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(fs->used, s));
  ctx->last_bwd_slots = S;
  return NXS_OK;
}

nxs_status nxs_state_release(nxs_context* ctx, nxs_fwd_state* state, void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (!state) return NXS_OK;
  if (state->owner != ctx || !ctx->states.count(state))
    return fail(ctx, NXS_EINVAL, "the state is not a live state of this context");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamWaitEvent(s, state->used, 0));
  release_state(ctx, state, s);
  return NXS_OK;
}

nxs_status nxs_autotune(nxs_context* ctx, const nxs_gaussians* g, const nxs_camera* cams,
                        int32_t n_views, const nxs_render_opts* opts, const nxs_image* out,
                        const char* cache_path, int32_t reps, nxs_tuning* result,
                        void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (!g || !cams || !opts || !out || !result || n_views <= 0 || reps < 0)
    return fail(ctx, NXS_EINVAL, "bad autotune argument");
  const std::string key = tuning_key(ctx, g, cams, n_views, opts);
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    *result = it->second;
    return NXS_OK;
  }
  nxs_tuning t{};
  if (read_cache(cache_path, key, &t)) {
    ctx->tuned[key] = t;
    *result = t;
    return NXS_OK;
  }
  if (reps == 0) reps = 5;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, NXS_EHIP, "hipEventCreate failed");
  }
  nxs_status st = NXS_OK;
  // GPU time per render: one waiting render (it sizes the buffers), then
  // `reps` deferred renders back to back on the stream between two events, so
  // that no host wait sits inside the timed span; renders that outgrew the
  // context (the device's flag, read by nxs_forward_status, which also grows
  // it) are timed again
  auto measure = [&](const nxs_render_opts& o, float* per_render) -> nxs_status {
    nxs_status rs = nxs_render_forward(ctx, g, cams, n_views, &o, out, nullptr, stream);
    if (rs != NXS_OK) return rs;
    nxs_render_opts od = o;
    od.flags |= NXS_FLAG_DEFERRED;
    for (int attempt = 0; attempt < 3; ++attempt) {
      if (hipEventRecord(e0, s) != hipSuccess) return fail(ctx, NXS_EHIP, "event record");
      for (int r = 0; r < reps; ++r) {
        rs = nxs_render_forward(ctx, g, cams, n_views, &od, out, nullptr, stream);
        if (rs != NXS_OK) return rs;
      }
      float t_ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess)
        return fail(ctx, NXS_EHIP, "autotune timing failed");
      rs = nxs_forward_status(ctx, nullptr);
      if (rs == NXS_OK) {
        *per_render = t_ms / (float)reps;
        return NXS_OK;
      }
      if (rs != NXS_ECAPACITY) return rs;
      ctx->err.clear();
    }
    return fail(ctx, NXS_ECAPACITY, "autotune: deferred renders kept outgrowing the context");
  };
  const int shapes[3][2] = {{8, 8}, {16, 16}, {32, 8}};
  nxs_tuning best{0, 0, 0, 64, NXS_SORT_AUTO, 0.0f};
  nxs_render_opts o = *opts;
  o.flags = 0;
  auto apply = [&](const nxs_tuning& t) {
    o.tile_w = t.tile_w;
    o.tile_h = t.tile_h;
    o.schedule = t.schedule;
    o.lds_batch = t.lds_batch;
    o.sort_order = t.sort_order;
  };
  auto consider = [&](const nxs_tuning& t) {
    apply(t);
    float med = 0.0f;
    st = measure(o, &med);
    if (st == NXS_OK && (best.schedule == 0 || med < best.ms)) {
      best = t;
      best.ms = med;
    }
  };
  // every tile shape and schedule at a batch of 64 list entries
  for (int sh = 0; sh < 3 && st == NXS_OK; ++sh)
    for (int sc = NXS_SCHED_TILES; sc <= NXS_SCHED_PERSISTENT && st == NXS_OK; ++sc)
      consider({shapes[sh][0], shapes[sh][1], sc, 64, NXS_SORT_AUTO, 0.0f});
  // then the larger batches, then both sort orders, at the best so far
  for (int b = 128; b <= 256 && st == NXS_OK; b *= 2) {
    nxs_tuning t = best;
    t.lds_batch = b;
    consider(t);
  }
  // both sort orders explicitly (the automatic one is one of them); the
  // result names the faster
  float m_order[2] = {0.0f, 0.0f};
  for (int k = 0; k < 2 && st == NXS_OK; ++k) {
    nxs_tuning t = best;
    t.sort_order = NXS_SORT_DEPTH_FIRST + k;
    apply(t);
    st = measure(o, &m_order[k]);
  }
  if (st == NXS_OK) {
    const int k = m_order[0] <= m_order[1] ? 0 : 1;
    best.sort_order = NXS_SORT_DEPTH_FIRST + k;
    best.ms = std::min(best.ms, m_order[k]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != NXS_OK) return st;
  ctx->tuned[key] = best;
  append_cache(cache_path, key, best);
  *result = best;
  return NXS_OK;
}

nxs_status nxs_set_workspace_limit(nxs_context* ctx, size_t bytes) {
  if (!ctx) return NXS_EINVAL;
  ctx->ws_limit = bytes;
  return NXS_OK;
}

nxs_status nxs_release_workspace(nxs_context* ctx) {
  if (!ctx) return NXS_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_done) HIP_TRY(hipEventSynchronize(ctx->done));
  free_workspace(ctx, nullptr);
  ctx->last_bwd_slots = -1;
  if (!ctx->last_state) {
    ctx->last_inst_tile = ctx->last_inst_val = nullptr;
    ctx->last_m = ctx->last_tiles = ctx->last_slots = 0;
  } else {
    ctx->last_inst_tile = nullptr;   // the tile keys were workspace
  }
  return NXS_OK;
}

nxs_status nxs_workspace_bytes(const nxs_context* ctx, size_t* bytes) {
  if (!ctx || !bytes) return NXS_EINVAL;
  *bytes = ctx->ws_total;
  return NXS_OK;
}

nxs_status nxs_measure_peaks(nxs_context* ctx, double* fp32_fma_tflops, double* copy_gbs,
                             void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (!fp32_fma_tflops || !copy_gbs) return fail(ctx, NXS_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const int groups = 8 * ctx->n_cu;              // 8 waves per SIMD
  const int iters = 20000;
  const size_t copy_bytes = size_t(512) << 20;   // read, and again written
  void* out = nullptr;
  void* src = nullptr;
  void* dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  nxs_status st = NXS_OK;
  float fma_ms = 0.0f, copy_ms = 0.0f;
  auto hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == NXS_OK)
      st = fail(ctx, NXS_EHIP, "%s failed: %s", what, hipGetErrorString(e));
    return st == NXS_OK;
  };
  auto timed = [&](auto&& launch, float* ms) {
    if (!hip(hipEventRecord(e0, s), "hipEventRecord")) return false;
    launch();
    if (!hip(hipGetLastError(), "peak kernel launch") || !hip(hipEventRecord(e1, s), "hipEventRecord") ||
        !hip(hipEventSynchronize(e1), "hipEventSynchronize") ||
        !hip(hipEventElapsedTime(ms, e0, e1), "hipEventElapsedTime"))
      return false;
    return true;
  };
  if ((st = dev_alloc(ctx, 4 * peak_fma_out_floats(groups), s, &out)) == NXS_OK &&
      (st = dev_alloc(ctx, copy_bytes, s, &src)) == NXS_OK &&
      (st = dev_alloc(ctx, copy_bytes, s, &dst)) == NXS_OK &&
      hip(hipEventCreate(&e0), "hipEventCreate") && hip(hipEventCreate(&e1), "hipEventCreate")) {
    // FP32 FMA chains: one warm-up launch, then the timed one
    auto fma = [&]() { launch_peak_fma(static_cast<float*>(out), groups, iters, s); };
    fma();
    if (timed(fma, &fma_ms)) {
      // copy: the source set first, one warm-up, then the best of three
      const int64_t n4 = (int64_t)(copy_bytes / 16);
      auto copy = [&]() {
        launch_peak_copy(static_cast<const float4*>(src), static_cast<float4*>(dst), n4, s);
      };
      if (hip(hipMemsetAsync(src, 0, copy_bytes, s), "hipMemsetAsync")) {
        copy();
        copy_ms = 1e30f;
        for (int r = 0; r < 3 && st == NXS_OK; ++r) {
          float ms = 0.0f;
          if (timed(copy, &ms)) copy_ms = std::min(copy_ms, ms);
        }
      }
    }
  }
  if (out) dev_free(ctx, out, s);
  if (src) dev_free(ctx, src, s);
  if (dst) dev_free(ctx, dst, s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != NXS_OK) return st;
  if (!(fma_ms > 0.0f) || !(copy_ms > 0.0f))
    return fail(ctx, NXS_EHIP, "peak timing gave no duration");
  *fp32_fma_tflops = (double)peak_fma_flops(groups, iters) / (fma_ms * 1e-3) / 1e12;
  *copy_gbs = 2.0 * (double)copy_bytes / (copy_ms * 1e-3) / 1e9;
  return NXS_OK;
}

nxs_status nxs_set_timing(nxs_context* ctx, int32_t enable) {
  if (!ctx) return NXS_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  if (enable && !ctx->ev[0])
    for (int k = 0; k < 8; ++k) HIP_TRY(hipEventCreate(&ctx->ev[k]));
  ctx->timing = enable != 0;
  ctx->ev_valid = false;
  return NXS_OK;
}

nxs_status nxs_inspect_stage_times(nxs_context* ctx, float* ms_host, int32_t n) {
  if (!ctx || !ms_host || n < NXS_N_STAGES) return NXS_EINVAL;
  if (!ctx->ev_valid) return fail(ctx, NXS_EINVAL, "no timed render on this context");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->ev[7]));
  // project, depth sort (incl. ranges clear), emit, tile sort, ranges, composite
  const int from[NXS_N_STAGES] = {0, 2, 3, 4, 5, 6};
  const int to[NXS_N_STAGES] = {1, 3, 4, 5, 6, 7};
  for (int k = 0; k < NXS_N_STAGES; ++k)
    HIP_TRY(hipEventElapsedTime(&ms_host[k], ctx->ev[from[k]], ctx->ev[to[k]]));
  return NXS_OK;
}

}  // extern "C"

namespace {

// The instance count of the last render; a deferred one's is read from the
// device (its needed count if it failed).  Returns false if unknown.
nxs_status resolve_last_m(nxs_context* ctx, bool* failed) {
  *failed = ctx->last_failed;
  if (ctx->last_m >= 0) return NXS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->has_done) HIP_TRY(hipEventSynchronize(ctx->done));
  // the deferred render copied its count and fail bits to the pinned status
  // before `done`
  ctx->last_m = (int64_t)ctx->host_status->last;
  ctx->last_failed = ctx->host_status->last_fail != 0;
  *failed = ctx->last_failed;
  return NXS_OK;
}

}  // namespace

extern "C" {

nxs_status nxs_inspect_counts(nxs_context* ctx, int64_t* n_instances, int64_t* n_tiles) {
  if (!ctx || !n_instances || !n_tiles) return NXS_EINVAL;
  bool failed = false;
  nxs_status st = resolve_last_m(ctx, &failed);
  if (st != NXS_OK) return st;
  *n_instances = ctx->last_m;
  *n_tiles = ctx->last_tiles;
  return NXS_OK;
}

nxs_status nxs_inspect_instances(nxs_context* ctx, uint64_t* keys_host, int32_t* ids_host,
                                 int64_t capacity) {
  if (!ctx) return NXS_EINVAL;
  bool failed = false;
  nxs_status st = resolve_last_m(ctx, &failed);
  if (st != NXS_OK) return st;
  if ((!keys_host && ctx->last_m) || (!ids_host && ctx->last_m)) return NXS_EINVAL;
  if (capacity < ctx->last_m) return fail(ctx, NXS_EINVAL, "capacity below instance count");
  if (ctx->last_m == 0) return NXS_OK;
  if (failed || !ctx->last_inst_tile || !ctx->last_inst_val)
    return fail(ctx, NXS_EINVAL, "the last render did not complete");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->done));
  std::vector<uint32_t> tile(ctx->last_m), val(ctx->last_m), dk(ctx->last_slots);
  HIP_TRY(hipMemcpy(tile.data(), ctx->last_inst_tile, 4 * ctx->last_m, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(val.data(), ctx->last_inst_val, 4 * ctx->last_m, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(dk.data(), ctx->depth_key.p, 4 * ctx->last_slots, hipMemcpyDeviceToHost));
  for (int64_t j = 0; j < ctx->last_m; ++j) {
    keys_host[j] = ((uint64_t)tile[j] << 32) | dk[val[j]];
    ids_host[j] = (int32_t)(val[j] % (uint32_t)ctx->last_n);
  }
  return NXS_OK;
}

nxs_status nxs_inspect_ranges(nxs_context* ctx, int32_t* ranges_host, int64_t capacity) {
  if (!ctx || !ranges_host) return NXS_EINVAL;
  if (capacity < 2 * ctx->last_tiles) return fail(ctx, NXS_EINVAL, "capacity below 2 * tiles");
  const void* src = ctx->last_state ? ctx->last_state->ranges.p : ctx->ranges.p;
  if (!src) return fail(ctx, NXS_EINVAL, "no render on this context");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->done));
  HIP_TRY(hipMemcpy(ranges_host, src, 8 * ctx->last_tiles, hipMemcpyDeviceToHost));
  return NXS_OK;
}

nxs_status nxs_inspect_slot_grads(nxs_context* ctx, float* slot_grads_host, int64_t capacity) {
  if (!ctx || !slot_grads_host) return NXS_EINVAL;
  if (ctx->last_bwd_slots < 0 || !ctx->gslot.p)
    return fail(ctx, NXS_EINVAL, "no backward on this context");
  if (capacity < 9 * ctx->last_bwd_slots) return fail(ctx, NXS_EINVAL, "capacity below 9 * slots");
  if (ctx->last_bwd_slots == 0) return NXS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->done));
  HIP_TRY(hipMemcpy(slot_grads_host, ctx->gslot.p, 36 * ctx->last_bwd_slots,
                    hipMemcpyDeviceToHost));
  return NXS_OK;
}

nxs_status nxs_inspect_projection(nxs_context* ctx, int32_t view, uint32_t* depth_bits_host,
                                  int32_t* rect_host, int64_t capacity) {
  if (!ctx || !depth_bits_host || !rect_host) return NXS_EINVAL;
  if (view < 0 || view >= ctx->last_views) return fail(ctx, NXS_EINVAL, "bad view");
  const int64_t n = ctx->last_n;
  if (capacity < n) return fail(ctx, NXS_EINVAL, "capacity below n");
  if (n == 0) return NXS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->done));
  std::vector<uint2> rect(n);
  HIP_TRY(hipMemcpy(depth_bits_host, (uint32_t*)ctx->depth_key.p + view * n, 4 * n,
                    hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rect.data(), (uint2*)ctx->trect.p + view * n, 8 * n,
                    hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) {
    if (rect[i].x == 0xFFFFFFFFu) {
      depth_bits_host[i] = 0;
      for (int k = 0; k < 4; ++k) rect_host[4 * i + k] = -1;
    } else {
      rect_host[4 * i + 0] = (int32_t)(rect[i].x & 0xFFFF);
      rect_host[4 * i + 1] = (int32_t)(rect[i].x >> 16);
      rect_host[4 * i + 2] = (int32_t)(rect[i].y & 0xFFFF);
      rect_host[4 * i + 3] = (int32_t)(rect[i].y >> 16);
    }
  }
  return NXS_OK;
}

}  // extern "C"
