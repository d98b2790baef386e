// Serving loop: resident scenes, continuous batching under a workspace budget.
//
// Requests (scene, camera, render options, caller-owned output images) queue in
// arrival order.  Each step serves the oldest pending request together with the
// later pending requests that can share its render: same scene and identical
// options, so that one multi-view nxs_render_forward covers them all (one
// projection pass over the scene for all their cameras, one sort, one composite
// launch).  A batch grows in arrival order while its estimated workspace stays
// within the budget; the estimate uses the instances per pixel that the
// scene's last render produced.  The context's workspace limit is the budget,
// so a batch whose estimate was too low fails with NXS_ECAPACITY instead of
// growing past it: the step then frees the workspace and retries, and if that
// fails too, serves the first half of the batch; a single request that cannot
// fit is completed with that status.  Requests that arrive while a batch renders
// join a later batch.  Every step synchronises its stream before returning the
// tags it completed.
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
};

struct Scene {
  nxs_gaussians g;
  double inst_per_px;   // instances per output pixel of the last render (estimate)
};

bool same_batch(const Request& a, const Request& b) {
  return a.scene == b.scene && std::memcmp(&a.opts, &b.opts, sizeof(nxs_render_opts)) == 0;
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
  return 88.0 * slots + 68.0 * inst + 12.0 * tiles + (1 << 20);
}

}  // namespace

struct nxs_server {
  nxs_context* ctx = nullptr;
  size_t budget = 0;
  int32_t max_views = 16;
  std::vector<Scene> scenes;
  std::deque<Request> pending;
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

}  // namespace

extern "C" {

nxs_status nxs_server_create(int device, size_t workspace_budget, int32_t max_batch_views,
                             nxs_server** out) {
  if (!out || max_batch_views < 0) return NXS_EINVAL;
  *out = nullptr;
  nxs_server* s = new (std::nothrow) nxs_server();
  if (!s) return NXS_ENOMEM;
  nxs_status st = nxs_create(&s->ctx, device);
  if (st != NXS_OK) {
    delete s;
    return st;
  }
  s->budget = workspace_budget;
  s->max_views = max_batch_views ? max_batch_views : 16;
  nxs_set_workspace_limit(s->ctx, workspace_budget);
  *out = s;
  return NXS_OK;
}

nxs_status nxs_server_destroy(nxs_server* s) {
  if (!s) return NXS_EINVAL;
  nxs_destroy(s->ctx);
  delete s;
  return NXS_OK;
}

nxs_context* nxs_server_context(nxs_server* s) { return s ? s->ctx : nullptr; }

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
  if (opts->keep_state) return sfail(s, NXS_EINVAL, "served renders keep no backward state");
  s->pending.push_back({scene_id, *cam, *opts, *out, tag});
  return NXS_OK;
}

int32_t nxs_server_pending(const nxs_server* s) { return s ? (int32_t)s->pending.size() : 0; }

nxs_status nxs_server_step(nxs_server* s, void* stream, int64_t* tags, int32_t* status,
                           int32_t capacity, int32_t* n_done) {
  if (!s || !n_done || (capacity > 0 && (!tags || !status))) return NXS_EINVAL;
  s->err.clear();
  *n_done = 0;
  if (s->pending.empty()) return NXS_OK;
  if (capacity < 1) return sfail(s, NXS_EINVAL, "capacity must be >= 1");
  const int32_t limit = std::min(s->max_views, capacity);
  Scene& sc = s->scenes[s->pending.front().scene];

  // oldest request, then later compatible ones while the estimate fits
  std::vector<size_t> idx{0};
  std::vector<const Request*> batch{&s->pending.front()};
  for (size_t i = 1; i < s->pending.size() && (int32_t)batch.size() < limit; ++i) {
    if (!same_batch(s->pending.front(), s->pending[i])) continue;
    batch.push_back(&s->pending[i]);
    double px = 0.0;
    for (const Request* r : batch) px += (double)r->cam.width * r->cam.height;
    if ((s->budget && workspace_estimate(sc, batch) > (double)s->budget) ||
        sc.inst_per_px * px >= 4.0e9) {
      batch.pop_back();
      break;
    }
    idx.push_back(i);
  }

  hipStream_t strm = (hipStream_t)stream;
  nxs_status st = NXS_OK;
  bool released = false;
  for (;;) {
    const int32_t V = (int32_t)idx.size();
    std::vector<nxs_camera> cams(V);
    std::vector<nxs_image> outs(V);
    double pixels = 0.0;
    for (int32_t v = 0; v < V; ++v) {
      cams[v] = s->pending[idx[v]].cam;
      outs[v] = s->pending[idx[v]].out;
      pixels += (double)cams[v].width * cams[v].height;
    }
    st = nxs_render_forward(s->ctx, &sc.g, cams.data(), V, &s->pending[idx[0]].opts,
                            outs.data(), stream);
    int64_t m = 0, t = 0;
    nxs_inspect_counts(s->ctx, &m, &t);
    if (st == NXS_OK) {
      // follow the scene's instance density, decaying slowly towards lighter views
      if (pixels > 0.0) sc.inst_per_px = std::max((double)m / pixels, 0.9 * sc.inst_per_px);
      if (hipStreamSynchronize(strm) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(s, NXS_EHIP, "stream synchronisation failed");
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
      if (workspace_estimate(sc, pre) > (double)s->budget && s->budget) break;
      double px = 0.0;
      for (const Request* r : pre) px += (double)r->cam.width * r->cam.height;
      if (sc.inst_per_px * px >= 4.0e9) break;   // the 32-bit instance range
      ++keep;
    }
    if (keep < idx.size()) {
      idx.resize(keep);          // serve the older part now, the rest later
    } else if (!released) {      // it should fit: the workspace is fragmented by
      released = true;           // earlier batches, so start afresh
      nxs_release_workspace(s->ctx);
    } else {
      idx.resize((V + 1) / 2);
    }
  }
  // complete the served requests (or the single one that failed), in order
  for (size_t k = 0; k < idx.size(); ++k) {
    tags[k] = s->pending[idx[k]].tag;
    status[k] = st;
  }
  *n_done = (int32_t)idx.size();
  if (st != NXS_OK) s->err = nxs_last_error(s->ctx);
  for (size_t k = idx.size(); k-- > 0;) s->pending.erase(s->pending.begin() + (long)idx[k]);
  return NXS_OK;
}

const char* nxs_server_last_error(const nxs_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
