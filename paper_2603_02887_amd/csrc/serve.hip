// Serving loop: resident scenes, continuous batching under a workspace budget,
// several batches in flight at once.
//
// Requests (scene, camera, render options, caller-owned output images) queue in
// arrival order.  A batch is the oldest pending request together with the later
// pending requests that can share its render: same scene and identical options,
// so that one multi-view nxs_render_forward covers them all (one projection pass
// over the scene for all their cameras, one sort, one composite launch).  A batch
// grows in arrival order while its estimated workspace stays within a slot's
// share of the budget; the estimate uses the instance density that the scene's
// earlier renders produced.
//
// The server has n_slots slots, each a context with its own stream and a share
// of the budget as its workspace limit.  A step first collects the batches whose
// completion events have fired, then starts a batch on every free slot while
// requests are pending, and returns without waiting (unless asked to wait for at
// least one completion).  So batches on different slots overlap on the device:
// one slot's projection runs while another's sort or composite does, and
// requests that arrive meanwhile are admitted as slots free up.
//
// Batches are rendered deferred (NXS_FLAG_DEFERRED): starting one never waits
// on the host.  A deferred batch that outgrew its slot's instance buffers is
// found when it completes (nxs_forward_status): its requests go back to the
// front of the queue and are rendered again, waiting this time, after the
// slot has grown.  A waiting batch whose estimate was too low fails with
// NXS_ECAPACITY before allocating past the limit: the step reads the instance
// count the attempt needed, re-estimates and starts the prefix that fits
// (after one release of a fragmented workspace); a single request that
// cannot fit on its own, or one with invalid options, is completed with its
// error without blocking the queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "nxs.h"

namespace {

struct Request {
  int32_t scene;
  nxs_camera cam;
  nxs_render_opts opts;
  nxs_image out;
  int64_t tag;
  bool retry = false;   // a deferred render of it outgrew its slot: render waiting
};

struct Scene {
  nxs_gaussians g;
  double inst_per_px;   // instances per output pixel of recent renders (estimate)
};

struct Slot {
  nxs_context* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  bool deferred = false;         // the batch in flight was rendered deferred
  uint64_t seq = 0;              // start order, to report older batches first
  std::vector<int64_t> tags;     // requests in flight on this slot
  std::vector<Request> reqs;     // the same requests, to queue again on a retry
};

bool same_batch(const Request& a, const Request& b) {
  nxs_render_opts x = a.opts, y = b.opts;
  x.instance_hint = y.instance_hint = 0.0f;   // a launch size, not a result
  return a.scene == b.scene && std::memcmp(&x, &y, sizeof(nxs_render_opts)) == 0;
}

// Workspace bytes of one render (the library's per-slot, per-instance and
// per-tile buffers, without the 25% growth headroom).
double workspace_estimate(const Scene& sc, const std::vector<const Request*>& batch) {
  double pixels = 0.0, tiles = 0.0;
  for (const Request* r : batch) {
    const int tw = r->opts.tile_w ? r->opts.tile_w : 16, th = r->opts.tile_h ? r->opts.tile_h : 16;
    pixels += (double)r->cam.width * r->cam.height;
    tiles += std::ceil((double)r->cam.width / tw) * std::ceil((double)r->cam.height / th);
  }
  const double slots = (double)sc.g.n * (double)batch.size();
  const double inst = sc.inst_per_px * pixels;
  return 92.0 * slots + 20.0 * inst + 12.0 * tiles + (1 << 20);
}

double pixels_of(const std::vector<const Request*>& batch) {
  double px = 0.0;
  for (const Request* r : batch) px += (double)r->cam.width * r->cam.height;
  return px;
}

}  // namespace

struct nxs_server {
  size_t budget = 0;           // per slot
  int32_t max_views = 16;
  std::vector<Slot> slots;
  std::vector<Scene> scenes;
  std::deque<Request> pending;
  uint64_t seq = 0;
  std::string err;
};

namespace {

nxs_status sfail(nxs_server* s, nxs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  s->err = buf;
  return st;
}

void destroy_slots(nxs_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) nxs_destroy(sl.ctx);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  s->slots.clear();
}

// Start the oldest pending request's batch on slot `sl`.  A request that fails
// on its own is completed at once into (tags, status).  Returns false if the
// slot's stream failed.
bool start_batch(nxs_server* s, Slot& sl, std::vector<int64_t>& tags,
                 std::vector<int32_t>& status) {
  Scene& sc = s->scenes[s->pending.front().scene];
  std::vector<size_t> idx{0};
  std::vector<const Request*> batch{&s->pending.front()};
  for (size_t i = 1; i < s->pending.size() && (int32_t)batch.size() < s->max_views; ++i) {
    if (!same_batch(s->pending.front(), s->pending[i])) continue;
    batch.push_back(&s->pending[i]);
    if ((s->budget && workspace_estimate(sc, batch) > (double)s->budget) ||
        sc.inst_per_px * pixels_of(batch) >= 4.0e9) {
      batch.pop_back();
      break;
    }
    idx.push_back(i);
  }

  nxs_status st = NXS_OK;
  bool released = false;
  bool deferred = false;
  for (;;) {
    const int32_t V = (int32_t)idx.size();
    std::vector<nxs_camera> cams(V);
    std::vector<nxs_image> outs(V);
    std::vector<const Request*> cur;
    bool retry = false;
    for (int32_t v = 0; v < V; ++v) {
      cams[v] = s->pending[idx[v]].cam;
      outs[v] = s->pending[idx[v]].out;
      cur.push_back(&s->pending[idx[v]]);
      retry = retry || s->pending[idx[v]].retry;
    }
    const double pixels = pixels_of(cur);
    nxs_render_opts opts = s->pending[idx[0]].opts;
    deferred = !retry;
    if (deferred) {
      opts.flags |= NXS_FLAG_DEFERRED;
      opts.instance_hint = (float)(sc.inst_per_px * pixels);
    }
    st = nxs_render_forward(sl.ctx, &sc.g, cams.data(), V, &opts, outs.data(), nullptr,
                            sl.stream);
    // (a waiting render's count is known now; a deferred one's when it completes)
    int64_t m = 0, t = 0;
    if (!deferred || st != NXS_OK) nxs_inspect_counts(sl.ctx, &m, &t);
    if (st == NXS_OK) {
      // follow the scene's instance density, decaying slowly towards lighter views
      if (!deferred && pixels > 0.0)
        sc.inst_per_px = std::max((double)m / pixels, 0.9 * sc.inst_per_px);
      if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
        (void)hipGetLastError();
        s->err = "event record failed";
        return false;
      }
      break;
    }
    if (V == 1 && (st != NXS_ECAPACITY || released)) break;   // complete it with the error
    if (st != NXS_ECAPACITY) {
      idx.resize(1);             // some request of the batch is bad: the oldest alone
      continue;
    }
    // the render needed m instances: re-estimate and keep the prefix that fits
    if (m > 0 && pixels > 0.0)
      sc.inst_per_px = std::max(sc.inst_per_px, 1.05 * (double)m / pixels);
    size_t keep = 1;
    while (keep < idx.size()) {
      std::vector<const Request*> pre;
      for (size_t k = 0; k <= keep; ++k) pre.push_back(&s->pending[idx[k]]);
      if ((s->budget && workspace_estimate(sc, pre) > (double)s->budget) ||
          sc.inst_per_px * pixels_of(pre) >= 4.0e9)
        break;
      ++keep;
    }
    if (keep < idx.size()) {
      idx.resize(keep);          // serve the older part now, the rest later
    } else if (!released) {      // it should fit: the workspace is fragmented by
      released = true;           // earlier batches, so start afresh
      nxs_release_workspace(sl.ctx);
    } else {
      idx.resize((V + 1) / 2);
    }
  }
  if (st == NXS_OK) {
    sl.busy = true;
    sl.deferred = deferred;
    sl.seq = s->seq++;
    sl.tags.clear();
    sl.reqs.clear();
    for (size_t k : idx) {
      sl.tags.push_back(s->pending[k].tag);
      sl.reqs.push_back(s->pending[k]);
    }
  } else {
    tags.push_back(s->pending[idx[0]].tag);   // failed on its own: complete it now
    status.push_back(st);
    s->err = nxs_last_error(sl.ctx);
  }
  for (size_t k = idx.size(); k-- > 0;) s->pending.erase(s->pending.begin() + (long)idx[k]);
  return true;
}

}  // namespace

extern "C" {

nxs_status nxs_server_create(int device, size_t workspace_budget, int32_t max_batch_views,
                             int32_t n_slots, nxs_server** out) {
  if (!out || max_batch_views < 0 || n_slots < 0 || n_slots > 16) return NXS_EINVAL;
  *out = nullptr;
  nxs_server* s = new (std::nothrow) nxs_server();
  if (!s) return NXS_ENOMEM;
  const int32_t k = n_slots ? n_slots : 2;
  s->budget = workspace_budget / (size_t)k;
  s->max_views = max_batch_views ? max_batch_views : 16;
  s->slots.resize(k);
  for (Slot& sl : s->slots) {
    nxs_status st = nxs_create(&sl.ctx, device, nullptr, nullptr, nullptr);
    if (st == NXS_OK &&
        (hipSetDevice(device) != hipSuccess ||
         hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess))
      st = NXS_EHIP;
    if (st != NXS_OK) {
      (void)hipGetLastError();
      destroy_slots(s);
      delete s;
      return st;
    }
    nxs_set_workspace_limit(sl.ctx, s->budget);
  }
  *out = s;
  return NXS_OK;
}

nxs_status nxs_server_destroy(nxs_server* s) {
  if (!s) return NXS_EINVAL;
  destroy_slots(s);
  delete s;
  return NXS_OK;
}

nxs_status nxs_server_add_scene(nxs_server* s, const nxs_gaussians* g, int32_t* scene_id) {
  if (!s || !g || !scene_id) return NXS_EINVAL;
  s->err.clear();
  if (g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3)
    return sfail(s, NXS_EINVAL, "bad scene (n %d, SH degree %d)", g->n, g->sh_degree);
  // until a render of the scene says otherwise: 8 instances per pixel
  s->scenes.push_back({*g, 8.0});
  *scene_id = (int32_t)s->scenes.size() - 1;
  return NXS_OK;
}

nxs_status nxs_server_submit(nxs_server* s, int32_t scene_id, const nxs_camera* cam,
                             const nxs_render_opts* opts, const nxs_image* out, int64_t tag) {
  if (!s || !cam || !opts || !out) return NXS_EINVAL;
  s->err.clear();
  if (scene_id < 0 || scene_id >= (int32_t)s->scenes.size())
    return sfail(s, NXS_EINVAL, "unknown scene %d", scene_id);
  if (!out->rgb || !out->trans) return sfail(s, NXS_EINVAL, "null output");
  if (opts->flags) return sfail(s, NXS_EINVAL, "served renders take no flags");
  s->pending.push_back({scene_id, *cam, *opts, *out, tag});
  return NXS_OK;
}

int32_t nxs_server_pending(const nxs_server* s) { return s ? (int32_t)s->pending.size() : 0; }

int32_t nxs_server_in_flight(const nxs_server* s) {
  if (!s) return 0;
  int32_t n = 0;
  for (const Slot& sl : s->slots)
    if (sl.busy) n += (int32_t)sl.tags.size();
  return n;
}

nxs_status nxs_server_workspace_bytes(const nxs_server* s, size_t* bytes) {
  if (!s || !bytes) return NXS_EINVAL;
  size_t total = 0;
  for (const Slot& sl : s->slots) {
    size_t b = 0;
    nxs_workspace_bytes(sl.ctx, &b);
    total += b;
  }
  *bytes = total;
  return NXS_OK;
}

nxs_status nxs_server_step(nxs_server* s, int32_t wait, int64_t* tags, int32_t* status,
                           int32_t capacity, int32_t* n_done) {
  if (!s || !n_done || capacity < 1 || !tags || !status) return NXS_EINVAL;
  s->err.clear();
  if (capacity < s->max_views + (int32_t)s->slots.size())
    return sfail(s, NXS_EINVAL, "capacity must be at least max_batch_views + n_slots");
  *n_done = 0;
  std::vector<int64_t> t_out;
  std::vector<int32_t> s_out;
  // finished batches, oldest first, as far as `capacity` allows; with `block`,
  // wait for the oldest one in flight
  auto collect = [&](bool block) -> bool {
    for (;;) {
      Slot* best = nullptr;
      for (Slot& sl : s->slots)
        if (sl.busy && (!best || sl.seq < best->seq)) best = &sl;
      if (!best) return true;
      if (t_out.size() + best->tags.size() > (size_t)capacity) return true;
      const hipError_t q = block ? hipEventSynchronize(best->done) : hipEventQuery(best->done);
      if (q == hipErrorNotReady) return true;
      if (q != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      block = false;
      best->busy = false;
      if (best->deferred) {
        Scene& sc = s->scenes[best->reqs.front().scene];
        double pixels = 0.0;
        for (const Request& r : best->reqs) pixels += (double)r.cam.width * r.cam.height;
        int64_t need = 0;
        const nxs_status fs = nxs_forward_status(best->ctx, &need);
        if (fs == NXS_ECAPACITY) {
          // outgrew the slot: queue the requests again, in order, at the
          // front; they are rendered waiting (the slot has grown if its
          // limit allows, else the waiting render splits the batch)
          if (need > 0 && pixels > 0.0)
            sc.inst_per_px = std::max(sc.inst_per_px, 1.05 * (double)need / pixels);
          for (size_t k = best->reqs.size(); k-- > 0;) {
            Request r = best->reqs[k];
            r.retry = true;
            s->pending.push_front(r);
          }
          continue;
        }
        if (fs != NXS_OK) return false;
        int64_t m = 0, t = 0;
        if (nxs_inspect_counts(best->ctx, &m, &t) == NXS_OK && pixels > 0.0)
          sc.inst_per_px = std::max((double)m / pixels, 0.9 * sc.inst_per_px);
      }
      t_out.insert(t_out.end(), best->tags.begin(), best->tags.end());
      s_out.insert(s_out.end(), best->tags.size(), (int32_t)NXS_OK);
    }
  };
  // 1. batches that have finished
  if (!collect(false)) return sfail(s, NXS_EHIP, "a render stream failed");
  // 2. start batches on the free slots (each start completes at most one
  //    request at once, so keep room for it)
  auto start_all = [&]() -> bool {
    for (Slot& sl : s->slots) {
      if (sl.busy || s->pending.empty()) continue;
      if (t_out.size() >= (size_t)capacity) break;
      if (!start_batch(s, sl, t_out, s_out)) return false;
    }
    return true;
  };
  if (!start_all()) return sfail(s, NXS_EHIP, "%s", s->err.c_str());
  // 3. optionally wait for the oldest batch in flight, then refill its slot
  if (wait && t_out.empty()) {
    if (!collect(true)) return sfail(s, NXS_EHIP, "a render stream failed");
    if (!start_all()) return sfail(s, NXS_EHIP, "%s", s->err.c_str());
  }
  for (size_t k = 0; k < t_out.size(); ++k) {
    tags[k] = t_out[k];
    status[k] = s_out[k];
  }
  *n_done = (int32_t)t_out.size();
  return NXS_OK;
}

const char* nxs_server_last_error(const nxs_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
