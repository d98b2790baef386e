// Pipelined renders on one object: K lanes, each a context with a stream of its
// own.  Consecutive renders are dealt to the lanes in turn, so that one
// render's latency-bound sort kernels overlap another's projection (HBM) or
// composite (VALU) on the device, as renders on several contexts and streams
// do; the caller sees one object, one stream to order against and one join.
//
// A render on lane i waits (an event) for the work already enqueued on the
// caller's stream, then runs on lane i's stream; lane i's next render follows
// it on that stream, so its workspace is reused in order.  The caller's stream
// does not wait for the render: nxs_pipeline_join makes it wait for every lane.
#include "nxs_internal.h"

#include <cstdarg>
#include <cstdio>
#include <string>

namespace {

constexpr int kMaxLanes = 8;

struct Lane {
  nxs_context* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr;   // recorded on the caller's stream
  hipEvent_t done = nullptr;   // recorded on the lane's stream after each render
  bool used = false;
};

}  // namespace

struct nxs_pipeline {
  int device = 0;
  int lanes = 0;
  int next = 0;
  Lane lane[kMaxLanes];
  std::string err;
};

namespace {

nxs_status pfail(nxs_pipeline* p, nxs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  p->err = buf;
  return st;
}

nxs_status phip(nxs_pipeline* p, hipError_t e, const char* what) {
  if (e == hipSuccess) return NXS_OK;
  return pfail(p, NXS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void destroy_lanes(nxs_pipeline* p) {
  for (int i = 0; i < kMaxLanes; ++i) {
    Lane& l = p->lane[i];
    if (l.stream) (void)hipStreamSynchronize(l.stream);
    if (l.ctx) (void)nxs_destroy(l.ctx);
    if (l.fork) (void)hipEventDestroy(l.fork);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.stream) (void)hipStreamDestroy(l.stream);
    l = Lane{};
  }
}

}  // namespace

extern "C" {

nxs_status nxs_pipeline_create(nxs_pipeline** out, int device, int32_t lanes,
                               nxs_alloc_fn alloc, nxs_free_fn free, void* user) {
  if (!out) return NXS_EINVAL;
  *out = nullptr;
  if (lanes < 1 || lanes > kMaxLanes) return NXS_EINVAL;
  if ((alloc == nullptr) != (free == nullptr)) return NXS_EINVAL;
  nxs_pipeline* p = new (std::nothrow) nxs_pipeline();
  if (!p) return NXS_ENOMEM;
  p->device = device;
  p->lanes = lanes;
  if (hipSetDevice(device) != hipSuccess) {
    delete p;
    return NXS_EHIP;
  }
  for (int i = 0; i < lanes; ++i) {
    Lane& l = p->lane[i];
    const nxs_status st = nxs_create(&l.ctx, device, alloc, free, user);
    if (st != NXS_OK ||
        hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&l.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
      destroy_lanes(p);
      delete p;
      return st != NXS_OK ? st : NXS_EHIP;
    }
  }
  *out = p;
  return NXS_OK;
}

nxs_status nxs_pipeline_destroy(nxs_pipeline* p) {
  if (!p) return NXS_EINVAL;
  (void)hipSetDevice(p->device);
  destroy_lanes(p);
  delete p;
  return NXS_OK;
}

nxs_status nxs_pipeline_render(nxs_pipeline* p, const nxs_gaussians* g, const nxs_camera* cams,
                               int32_t n_views, const nxs_render_opts* opts,
                               const nxs_image* out, void* stream) {
  if (!p) return NXS_EINVAL;
  p->err.clear();
  nxs_status st = phip(p, hipSetDevice(p->device), "hipSetDevice");
  if (st != NXS_OK) return st;
  Lane& l = p->lane[p->next];
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = phip(p, hipEventRecord(l.fork, s), "hipEventRecord")) != NXS_OK ||
      (st = phip(p, hipStreamWaitEvent(l.stream, l.fork, 0), "hipStreamWaitEvent")) != NXS_OK)
    return st;
  st = nxs_render_forward(l.ctx, g, cams, n_views, opts, out, nullptr, l.stream);
  // (recorded whatever the outcome, so that a join also covers what a failed
  // call enqueued)
  const hipError_t e = hipEventRecord(l.done, l.stream);
  if (e == hipSuccess) l.used = true;
  if (st != NXS_OK) {
    p->err = nxs_last_error(l.ctx);
    return st;
  }
  if ((st = phip(p, e, "hipEventRecord")) != NXS_OK) return st;
  p->next = (p->next + 1) % p->lanes;
  return NXS_OK;
}

nxs_status nxs_pipeline_join(nxs_pipeline* p, void* stream) {
  if (!p) return NXS_EINVAL;
  p->err.clear();
  nxs_status st = phip(p, hipSetDevice(p->device), "hipSetDevice");
  if (st != NXS_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < p->lanes; ++i)
    if (p->lane[i].used &&
        (st = phip(p, hipStreamWaitEvent(s, p->lane[i].done, 0), "hipStreamWaitEvent")) != NXS_OK)
      return st;
  return NXS_OK;
}

nxs_status nxs_pipeline_status(nxs_pipeline* p, int64_t* needed) {
  if (!p) return NXS_EINVAL;
  p->err.clear();
  if (needed) *needed = 0;
  nxs_status worst = NXS_OK;
  int64_t most = 0;
  for (int i = 0; i < p->lanes; ++i) {
    int64_t need = 0;
    const nxs_status st = nxs_forward_status(p->lane[i].ctx, &need);
    most = need > most ? need : most;
    if (st != NXS_OK && worst == NXS_OK) {
      worst = st;
      p->err = nxs_last_error(p->lane[i].ctx);
    }
  }
  // a render dealt again goes to the next lane: every lane grows to what the
  // largest one needed (the lanes' work has completed)
  if (worst == NXS_ECAPACITY && most > 0)
    for (int i = 0; i < p->lanes; ++i) {
      const nxs_status st = nxs::grow_instance_capacity(p->lane[i].ctx, (uint64_t)most);
      if (st != NXS_OK) {
        p->err += std::string("; growing a lane failed too: ") + nxs_last_error(p->lane[i].ctx);
        break;
      }
    }
  if (needed) *needed = most;
  return worst;
}

const char* nxs_pipeline_last_error(const nxs_pipeline* p) {
  return p ? p->err.c_str() : "null pipeline";
}

}  // extern "C"
