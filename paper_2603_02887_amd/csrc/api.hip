// Host side of the C ABI declared in include/nxs.h: argument checks,
// workspace management and the launch sequence of one forward render.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "nxs.h"
#include "nxs_internal.h"

using namespace nxs;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct nxs_context {
  int device = 0;
  std::string err;
  // workspace
  DevBuf views, counters, partials;
  DevBuf depth_key, dsort_a, dsort_b, slot_a, slot_b, tinfo, nt_sorted, rect_sorted, prec;
  DevBuf scan_local, block_sums, counts;
  DevBuf inst_tile, inst_tile_alt, inst_val, inst_val_alt;
  DevBuf ranges, pstate, gslot, order;
  int n_cu = 256;
  std::string arch;
  size_t ws_limit = 0;   // 0: no limit on the workspace
  size_t ws_total = 0;   // bytes currently allocated for the workspace
  std::map<std::string, nxs_tuning> tuned;   // autotuner results of this process
  Counters* host_counters = nullptr;  // pinned
  ViewDev* host_views = nullptr;      // pinned
  int host_views_cap = 0;
  hipEvent_t done = nullptr;           // recorded at the end of each render
  hipEvent_t counted = nullptr;        // the instance count has reached the host
  bool has_done = false;
  // optional per-stage timing (hipEvents on the render's stream)
  bool timing = false;
  hipEvent_t ev[8] = {};
  bool ev_valid = false;
  // what the backward of the last render needs
  bool bwd_valid = false;
  nxs_gaussians bwd_g{};
  int bwd_model = 0, bwd_tw = 16, bwd_th = 16;
  CompositeParams bwd_cp{};
  std::vector<ViewDev> bwd_views;
  // state of the last render, for inspection
  int64_t last_m = 0, last_tiles = 0, last_slots = 0;
  // first depth-sort pass to launch: 1 while the last render's plan left
  // pass 0 inactive (at most 27 varying depth bits), else 0
  int depth_first = 0;
  const uint32_t* bwd_order = nullptr;
  int32_t last_n = 0, last_views = 0;
  uint32_t* last_inst_tile = nullptr;
  uint32_t* last_inst_val = nullptr;
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

// Grow buffer b to at least `bytes` (with 25% headroom when the workspace
// limit allows it); never shrinks.  Beyond the context's workspace limit the
// call fails with NXS_ECAPACITY before freeing anything.
nxs_status ensure(nxs_context* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return NXS_OK;
  size_t want = bytes + bytes / 4;
  want = (want + 255) & ~(size_t)255;
  if (ctx->ws_limit) {
    const size_t others = ctx->ws_total - b.cap;
    if (others + want > ctx->ws_limit) want = (bytes + 255) & ~(size_t)255;
    if (others + want > ctx->ws_limit)
      return fail(ctx, NXS_ECAPACITY, "workspace limit: %zu bytes needed, %zu allowed",
                  others + want, ctx->ws_limit);
  }
  if (b.p) {
    // kernels enqueued earlier (this render's included) may still use the
    // buffer: wait for the device before freeing it (growth is rare)
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(b.p);
    ctx->ws_total -= b.cap;
    b.p = nullptr;
    b.cap = 0;
    if (e != hipSuccess) return fail(ctx, NXS_EHIP, "hipFree: %s", hipGetErrorString(e));
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, NXS_ENOMEM, "hipMalloc(%zu bytes) failed", want);
  }
  b.cap = want;
  ctx->ws_total += want;
  return NXS_OK;
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
    if (sscanf(line, "%3999s %d %d %d %f", k, &r.tile_w, &r.tile_h, &r.schedule, &r.ms) == 5 &&
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
  fprintf(f, "%s %d %d %d %.5f\n", key.c_str(), t.tile_w, t.tile_h, t.schedule, (double)t.ms);
  fclose(f);
}

}  // namespace

extern "C" {

nxs_status nxs_create(nxs_context** out, int device) {
  if (!out) return NXS_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return NXS_EINVAL;
  nxs_context* ctx = new (std::nothrow) nxs_context();
  if (!ctx) return NXS_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&ctx->host_counters, sizeof(Counters), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->counted, hipEventDisableTiming) != hipSuccess) {
    if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->counted) (void)hipEventDestroy(ctx->counted);
    delete ctx;
    return NXS_EHIP;
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
  (void)hipDeviceSynchronize();
  DevBuf* all[] = {&ctx->views,      &ctx->counters,      &ctx->partials,      &ctx->depth_key, &ctx->dsort_a, &ctx->dsort_b,
                   &ctx->slot_a,     &ctx->slot_b,        &ctx->tinfo,     &ctx->nt_sorted,     &ctx->rect_sorted,
                   &ctx->prec,       &ctx->scan_local,
                   &ctx->block_sums, &ctx->counts,        &ctx->inst_tile, &ctx->inst_tile_alt,
                   &ctx->inst_val,   &ctx->inst_val_alt,  &ctx->ranges,
                   &ctx->pstate,     &ctx->gslot,         &ctx->order};
  for (DevBuf* b : all)
    if (b->p) (void)hipFree(b->p);
  if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
  if (ctx->host_views) (void)hipHostFree(ctx->host_views);
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
                              void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  ctx->bwd_valid = false;   // any forward, even a failed one, ends the kept state
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
  int tw = opts->tile_w ? opts->tile_w : 16, th = opts->tile_h ? opts->tile_h : 16;
  if (!((tw == 8 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 8)))
    return fail(ctx, NXS_EINVAL, "tile size %dx%d not supported (8x8, 16x16, 32x8)", tw, th);
  const int sched = opts->schedule ? opts->schedule : NXS_SCHED_QUEUE;
  if (sched < NXS_SCHED_TILES || sched > NXS_SCHED_PERSISTENT)
    return fail(ctx, NXS_EINVAL, "schedule %d not supported (0..4)", opts->schedule);
  int batch = opts->lds_batch ? opts->lds_batch : 256;
  if (batch != 128 && batch != 256 && batch != 512)
    return fail(ctx, NXS_EINVAL, "lds_batch must be 0, 128, 256 or 512");
  float alpha_min = opts->alpha_min > 0.0f ? opts->alpha_min : 1e-3f;
  if (!(alpha_min < 1.0f)) return fail(ctx, NXS_EINVAL, "alpha_min must be in (0, 1)");
  float t_eps = opts->t_eps == 0.0f ? 1e-4f : opts->t_eps;
  int64_t total_tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    const nxs_camera& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768)
      return fail(ctx, NXS_EINVAL, "view %d: bad size %dx%d", v, c.width, c.height);
    if (!out[v].rgb || !out[v].trans) return fail(ctx, NXS_EINVAL, "view %d: null output", v);
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f)) return fail(ctx, NXS_EINVAL, "view %d: bad focal", v);
    total_tiles += (int64_t)((c.width + tw - 1) / tw) * ((c.height + th - 1) / th);
  }
  if (total_tiles >= (int64_t)1 << 31) return fail(ctx, NXS_EINVAL, "too many tiles");
  const int64_t n = g->n;
  const int64_t S = n * n_views;
  if (S >= ((int64_t)1 << 32) - 1) return fail(ctx, NXS_EINVAL, "n * n_views too large");

  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  // the workspace is shared by all calls on this context: order after the last one
  if (ctx->has_done) HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));

  // ---- view table -----------------------------------------------------------
  if (ctx->host_views_cap < n_views) {
    if (ctx->host_views) (void)hipHostFree(ctx->host_views);
    ctx->host_views = nullptr;
    ctx->host_views_cap = 0;
    HIP_TRY(hipHostMalloc((void**)&ctx->host_views, sizeof(ViewDev) * n_views,
                          hipHostMallocDefault));
    ctx->host_views_cap = n_views;
  }
  // (the previous call's copy out of host_views finished before it returned:
  // it synchronised its stream after the projection)
  int64_t off = 0, pix_off = 0;
  for (int v = 0; v < n_views; ++v) {
    const nxs_camera& c = cams[v];
    ViewDev& d = ctx->host_views[v];
    std::memset(&d, 0, sizeof(d));
    std::memcpy(d.R, c.R, sizeof(d.R));
    std::memcpy(d.t, c.t, sizeof(d.t));
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy; d.znear = c.znear;
    for (int k = 0; k < 3; ++k)
      d.campos[k] = (float)-((double)c.R[k] * c.t[0] + (double)c.R[3 + k] * c.t[1] +
                             (double)c.R[6 + k] * c.t[2]);
    d.width = c.width; d.height = c.height;
    d.tiles_x = (c.width + tw - 1) / tw;
    d.tiles_y = (c.height + th - 1) / th;
    d.tile_off = (int32_t)off;
    off += (int64_t)d.tiles_x * d.tiles_y;
    d.pix_off = pix_off;
    pix_off += (int64_t)c.width * c.height;
    d.rgb = out[v].rgb; d.trans = out[v].trans; d.od = out[v].overdraw;
  }
  nxs_status st;
  if ((st = ensure(ctx, ctx->views, sizeof(ViewDev) * n_views))) return st;
  if ((st = ensure(ctx, ctx->counters, sizeof(Counters)))) return st;
  if ((st = ensure(ctx, ctx->partials, sizeof(uint4) * project_partials_size(g->n)))) return st;
  HIP_TRY(hipMemcpyAsync(ctx->views.p, ctx->host_views, sizeof(ViewDev) * n_views,
                         hipMemcpyHostToDevice, s));
  const ViewDev* dviews = P<ViewDev>(ctx->views);

  // ---- per-slot buffers and projection ----------------------------------------
  if ((st = ensure(ctx, ctx->depth_key, 4 * S)) || (st = ensure(ctx, ctx->dsort_a, 4 * S)) ||
      (st = ensure(ctx, ctx->dsort_b, 4 * S)) ||
      (st = ensure(ctx, ctx->slot_a, 4 * S)) || (st = ensure(ctx, ctx->slot_b, 4 * S)) ||
      (st = ensure(ctx, ctx->tinfo, 16 * S)) || (st = ensure(ctx, ctx->nt_sorted, 4 * S)) ||
      (st = ensure(ctx, ctx->rect_sorted, 8 * S)) ||
      (st = ensure(ctx, ctx->prec, 48 * S)) || (st = ensure(ctx, ctx->scan_local, 4 * S)) ||
      (st = ensure(ctx, ctx->block_sums, 4 * scan_blocks_size(S))) ||
      (st = ensure(ctx, ctx->counts, 4 * radix_counts_words(S))) ||
      (st = ensure(ctx, ctx->ranges, 8 * total_tiles + 4 * kSchedCounters)))
    return st;
  ProjDev proj{P<uint32_t>(ctx->depth_key), P<uint4>(ctx->tinfo), P<float4>(ctx->prec)};
  GaussDev gd{g->means, g->scales, g->quats, g->opacities, g->sh, g->n, g->sh_degree};
  Counters* dcount = P<Counters>(ctx->counters);
  const float kappa2 = (float)(2.0 * std::log(1.0 / (double)alpha_min));
  auto mark = [&](int k) -> hipError_t {
    return ctx->timing ? hipEventRecord(ctx->ev[k], s) : hipSuccess;
  };
  ctx->ev_valid = false;
  HIP_TRY(mark(0));
  // (also clears the tile ranges and, after them, the composite schedules'
  // counters)
  launch_project(gd, dviews, n_views, kappa2, alpha_min, tw, th, proj,
                 P<uint4>(ctx->partials), dcount, P<uint32_t>(ctx->ranges),
                 2 * total_tiles + kSchedCounters, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(mark(1));
  // The instance count M is read by the host only where it sizes buffers and
  // grids: the depth sort (its digits planned on the device) and the emission
  // (total read on the device, writes bounded by the current capacity) are
  // enqueued first, so the GPU keeps working while the host waits.  (Copying
  // the counters on a second stream, beside the depth sort, was measured
  // slower: the cross-stream wait costs more than the copy.)
  HIP_TRY(hipMemcpyAsync(ctx->host_counters, dcount, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipEventRecord(ctx->counted, s));
  HIP_TRY(mark(2));
  // 1. depth sort of the slots (values: the slots 0..S-1)
  //    (its last pass also lays out the slots' tile counts and rectangles in
  //    that order, so that the emission reads them coalesced)
  //    (launched from the pass the last render's plan needed; checked below)
  const int depth_first = ctx->depth_first;
  auto depth_sort = [&](int first) {
    return radix_sort_planned(P<uint32_t>(ctx->depth_key), nullptr, P<uint32_t>(ctx->dsort_a),
                              P<uint32_t>(ctx->slot_a), P<uint32_t>(ctx->dsort_b),
                              P<uint32_t>(ctx->slot_b), S, dcount->plan, first,
                              P<uint32_t>(ctx->counts), proj.tinfo,
                              P<uint32_t>(ctx->nt_sorted), P<uint2>(ctx->rect_sorted), s);
  };
  const int wd = depth_sort(depth_first);
  uint32_t* sorted_slots = wd ? P<uint32_t>(ctx->slot_b) : P<uint32_t>(ctx->slot_a);
  HIP_TRY(mark(3));
  // 2. emission in depth order, into the buffers as they are
  launch_emit_scan(P<uint32_t>(ctx->nt_sorted), S, P<uint32_t>(ctx->scan_local),
                   P<uint32_t>(ctx->block_sums), s);
  const size_t cap = std::min(ctx->inst_tile.cap, ctx->inst_val.cap) / 4;
  const uint32_t cap32 = (uint32_t)std::min<size_t>(cap, 0xFFFFFFFFu);
  if (cap32 > 0)
    launch_emit_write(sorted_slots, P<uint2>(ctx->rect_sorted), S, g->n, dviews,
                      P<uint32_t>(ctx->scan_local), P<uint32_t>(ctx->block_sums), cap32,
                      P<uint32_t>(ctx->inst_tile), P<uint32_t>(ctx->inst_val), s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventSynchronize(ctx->counted));
  const uint64_t M = ctx->host_counters->total;
  // the depth sort skipped pass 0 but this render's plan needs it: sort and
  // emit again below (the depth keys are intact)
  const bool pass0 = (ctx->host_counters->plan[0] & kPassActive) != 0;
  const bool resort = S > 0 && depth_first == 1 && pass0;
  ctx->depth_first = pass0 ? 0 : 1;
  // what this render needs, visible through nxs_inspect_counts even if it fails
  ctx->last_m = (int64_t)M;
  ctx->last_tiles = total_tiles;
  ctx->last_inst_tile = ctx->last_inst_val = nullptr;
  if (M >= 0xFFFFFFFFull)
    return fail(ctx, NXS_ECAPACITY, "%llu tile instances exceed the 32-bit range",
                (unsigned long long)M);

  // ---- instance buffers (growing them waits for the work above) ------------------
  const int tbits = bit_length((uint64_t)(total_tiles - 1));
  if ((st = ensure(ctx, ctx->counts, 4 * radix_counts_words(std::max<int64_t>(S, M)))) ||
      (st = ensure(ctx, ctx->inst_tile, 4 * M)) || (st = ensure(ctx, ctx->inst_tile_alt, 4 * M)) ||
      (st = ensure(ctx, ctx->inst_val, 4 * M)) || (st = ensure(ctx, ctx->inst_val_alt, 4 * M)))
    return st;
  uint32_t* inst_tile = P<uint32_t>(ctx->inst_tile);
  uint32_t* inst_val = P<uint32_t>(ctx->inst_val);
  if (resort) {
    (void)depth_sort(0);
    launch_emit_scan(P<uint32_t>(ctx->nt_sorted), S, P<uint32_t>(ctx->scan_local),
                     P<uint32_t>(ctx->block_sums), s);
  }
  if (resort || M > cap32)   // emit (again) into the grown buffers
    launch_emit_write(sorted_slots, P<uint2>(ctx->rect_sorted), S, g->n, dviews,
                      P<uint32_t>(ctx->scan_local), P<uint32_t>(ctx->block_sums), (uint32_t)M,
                      inst_tile, inst_val, s);
  HIP_TRY(mark(4));
  if (M > 0) {
    // 3. stable sort by global tile
    const int wt = radix_sort(inst_tile, inst_val, P<uint32_t>(ctx->inst_tile_alt),
                              P<uint32_t>(ctx->inst_val_alt), inst_tile, inst_val, (int64_t)M,
                              tbits, P<uint32_t>(ctx->counts), s);
    if (wt == 0) {
      inst_tile = P<uint32_t>(ctx->inst_tile_alt);
      inst_val = P<uint32_t>(ctx->inst_val_alt);
    }
    HIP_TRY(mark(5));
    // 4. tile ranges
    launch_ranges(inst_tile, (int64_t)M, P<uint2>(ctx->ranges), s);
  } else {
    HIP_TRY(mark(5));
  }
  // 4b. the tile order of the queue schedules (longest tile lists first)
  // (the composite gathers the records of the sorted slots batch by batch)
  CompositeLaunch cl{sched, tw, th, total_tiles, dviews, n_views, P<uint2>(ctx->ranges),
                     inst_val, proj.rec, nullptr, nullptr, ctx->n_cu};
  if (sched == NXS_SCHED_QUEUE || sched == NXS_SCHED_PERSISTENT) {
    if ((st = ensure(ctx, ctx->order, 8 * (size_t)total_tiles))) return st;
    cl.order = P<uint32_t>(ctx->order);
    cl.sched_counters = P<uint32_t>(ctx->ranges) + 2 * total_tiles;
    launch_composite_order(cl, s);
  }
  float4* pstate = nullptr;
  if (opts->keep_state) {
    if ((st = ensure(ctx, ctx->pstate, 48 * (size_t)pix_off))) return st;
    pstate = P<float4>(ctx->pstate);
  }
  CompositeParams cp;
  cp.log2_alpha_min = (float)std::log2((double)alpha_min);
  // the exponential parts stop once T < cp.t_eps; "never" is the smallest
  // normal float, below which the float32 product would underflow
  cp.t_eps = (opts->model == NXS_EXPONENTIAL || opts->model == NXS_VICINI)
                 ? (t_eps > 0.0f ? t_eps : 1.17549435e-38f)
                 : 0.0f;
  cp.param = param;
  for (int k = 0; k < 3; ++k) cp.bg[k] = opts->background[k];
  cp.lds_batch = batch;
  HIP_TRY(mark(6));
  // 5. composite (also writes the background where no splat lands)
  launch_composite(opts->model, cl, cp, pstate, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(mark(7));
  HIP_TRY(hipEventRecord(ctx->done, s));
  ctx->has_done = true;
  if (opts->keep_state) {
    ctx->bwd_valid = true;
    ctx->bwd_g = *g;
    ctx->bwd_model = opts->model;
    ctx->bwd_tw = tw;
    ctx->bwd_th = th;
    ctx->bwd_cp = cp;
    ctx->bwd_order = cl.order;   // the tile order, if the schedule made one
    ctx->bwd_views.assign(ctx->host_views, ctx->host_views + n_views);
  }
  ctx->ev_valid = ctx->timing;

  ctx->last_m = (int64_t)M;
  ctx->last_tiles = total_tiles;
  ctx->last_slots = S;
  ctx->last_n = g->n;
  ctx->last_views = n_views;
  ctx->last_inst_tile = inst_tile;
  ctx->last_inst_val = inst_val;
  return NXS_OK;
}

nxs_status nxs_render_backward(nxs_context* ctx, const float* const* dL_drgb,
                               const float* const* dL_dtrans,
                               const nxs_gaussians_grad* grads, void* stream) {
  if (!ctx) return NXS_EINVAL;
  ctx->err.clear();
  if (!ctx->bwd_valid)
    return fail(ctx, NXS_EINVAL, "no forward with keep_state since the last forward");
  if (ctx->bwd_model > NXS_QUADRATIC)
    return fail(ctx, NXS_EUNSUPPORTED, "backward supports models 0..4, not %d", ctx->bwd_model);
  if (!dL_drgb || !grads) return fail(ctx, NXS_EINVAL, "null argument");
  const nxs_gaussians& g = ctx->bwd_g;
  if (g.n > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacities ||
                  !grads->sh))
    return fail(ctx, NXS_EINVAL, "null gradient array");
  const int n_views = (int)ctx->bwd_views.size();
  std::vector<ViewDev> views = ctx->bwd_views;
  for (int v = 0; v < n_views; ++v) {
    if (!dL_drgb[v]) return fail(ctx, NXS_EINVAL, "view %d: null dL_drgb", v);
    views[v].g_rgb = dL_drgb[v];
    views[v].g_trans = dL_dtrans ? dL_dtrans[v] : nullptr;
  }
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
  nxs_status st;
  const int64_t S = (int64_t)g.n * n_views;
  if ((st = ensure(ctx, ctx->gslot, 36 * (size_t)S))) return st;
  // pageable source: the copy has consumed `views` when the call returns
  HIP_TRY(hipMemcpyAsync(ctx->views.p, views.data(), sizeof(ViewDev) * n_views,
                         hipMemcpyHostToDevice, s));
  launch_fill_u32(P<uint32_t>(ctx->gslot), 9 * S, 0u, s);
  launch_composite_bwd(ctx->bwd_model, ctx->bwd_tw, ctx->bwd_th, ctx->last_tiles,
                       P<ViewDev>(ctx->views), n_views, P<uint2>(ctx->ranges),
                       ctx->last_inst_val, P<float4>(ctx->prec), ctx->bwd_cp,
                       P<float4>(ctx->pstate), P<float>(ctx->gslot), ctx->bwd_order, s);
  GaussDev gd{g.means, g.scales, g.quats, g.opacities, g.sh, g.n, g.sh_degree};
  GaussGradDev gg{grads->means, grads->scales, grads->quats, grads->opacities, grads->sh};
  launch_project_bwd(gd, P<ViewDev>(ctx->views), n_views, P<float>(ctx->gslot), gg, s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(ctx->done, s));
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
  const int shapes[3][2] = {{8, 8}, {16, 16}, {32, 8}};
  nxs_tuning best{0, 0, 0, 0.0f};
  nxs_status st = NXS_OK;
  for (int sh = 0; sh < 3 && st == NXS_OK; ++sh) {
    for (int sc = NXS_SCHED_TILES; sc <= NXS_SCHED_PERSISTENT && st == NXS_OK; ++sc) {
      nxs_render_opts o = *opts;
      o.tile_w = shapes[sh][0];
      o.tile_h = shapes[sh][1];
      o.schedule = sc;
      o.keep_state = 0;
      std::vector<float> ms;
      for (int r = 0; r <= reps && st == NXS_OK; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) { st = NXS_EHIP; break; }
        st = nxs_render_forward(ctx, g, cams, n_views, &o, out, stream);
        if (st != NXS_OK) break;
        float t_ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess) {
          st = fail(ctx, NXS_EHIP, "autotune timing failed");
          break;
        }
        if (r > 0) ms.push_back(t_ms);   // the first render is a warm-up
      }
      if (st != NXS_OK) break;
      std::sort(ms.begin(), ms.end());
      const float med = ms[ms.size() / 2];
      if (best.schedule == 0 || med < best.ms) best = {o.tile_w, o.tile_h, sc, med};
    }
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
  HIP_TRY(hipDeviceSynchronize());
  DevBuf* all[] = {&ctx->views,      &ctx->counters,      &ctx->partials,      &ctx->depth_key, &ctx->dsort_a, &ctx->dsort_b,
                   &ctx->slot_a,     &ctx->slot_b,        &ctx->tinfo,     &ctx->nt_sorted,     &ctx->rect_sorted,
                   &ctx->prec,       &ctx->scan_local,
                   &ctx->block_sums, &ctx->counts,        &ctx->inst_tile, &ctx->inst_tile_alt,
                   &ctx->inst_val,   &ctx->inst_val_alt,  &ctx->ranges,
                   &ctx->pstate,     &ctx->gslot,         &ctx->order};
  for (DevBuf* b : all) {
    if (b->p) HIP_TRY(hipFree(b->p));
    b->p = nullptr;
    b->cap = 0;
  }
  ctx->ws_total = 0;
  ctx->bwd_valid = false;
  ctx->last_m = ctx->last_tiles = ctx->last_slots = 0;
  ctx->last_inst_tile = ctx->last_inst_val = nullptr;
  return NXS_OK;
}

nxs_status nxs_workspace_bytes(const nxs_context* ctx, size_t* bytes) {
  if (!ctx || !bytes) return NXS_EINVAL;
  *bytes = ctx->ws_total;
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

nxs_status nxs_inspect_counts(nxs_context* ctx, int64_t* n_instances, int64_t* n_tiles) {
  if (!ctx || !n_instances || !n_tiles) return NXS_EINVAL;
  *n_instances = ctx->last_m;
  *n_tiles = ctx->last_tiles;
  return NXS_OK;
}

nxs_status nxs_inspect_instances(nxs_context* ctx, uint64_t* keys_host, int32_t* ids_host,
                                 int64_t capacity) {
  if (!ctx || (!keys_host && ctx->last_m) || (!ids_host && ctx->last_m))
    return NXS_EINVAL;
  if (capacity < ctx->last_m) return fail(ctx, NXS_EINVAL, "capacity below instance count");
  if (ctx->last_m == 0) return NXS_OK;
  if (!ctx->last_inst_tile) return fail(ctx, NXS_EINVAL, "the last render did not complete");
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
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipEventSynchronize(ctx->done));
  HIP_TRY(hipMemcpy(ranges_host, ctx->ranges.p, 8 * ctx->last_tiles, hipMemcpyDeviceToHost));
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
  std::vector<uint4> rect(n);
  HIP_TRY(hipMemcpy(depth_bits_host, (uint32_t*)ctx->depth_key.p + view * n, 4 * n,
                    hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rect.data(), (uint4*)ctx->tinfo.p + view * n, 16 * n,
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
