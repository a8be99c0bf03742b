// serve.cpp - multi-volume serving: per-stream frame requests, HBM admission
// by device footprint, eviction to host snapshots, completion timestamps.
//
// Each stream owns one probe volume (its own scene, grid and budget). A
// request asks for the stream's next frame with that frame's light
// positions. The server keeps at most one frame of a stream in flight (a
// stream's frames are sequential) and at most max_inflight frames in total,
// dispatching the waiting requests of resident streams in arrival order. A
// stream whose volume is not resident is admitted when its device footprint
// fits the HBM budget after evicting idle resident streams with no request
// waiting (least recently used first). A request that has waited over
// kMaxWaitNs may also evict idle streams that have work waiting, but only
// ones resident for at least kMinResidencyNs, so a working set stays resident
// instead of volumes being traded per request. Eviction saves the volume's
// temporal state to host memory and frees every device byte; admission
// re-creates the volume, installs the scene from the BVH built once when the
// stream was added, and restores the state, so a stream's results do not
// depend on the mix it runs in. Frames run on server-owned lanes (one stream
// per in-flight slot); a frame's completion is an event recorded behind it,
// polled by the dispatcher, which stamps the time it sees the event done.
// Eviction and admission enqueue their copies and return: an evicted volume
// keeps its memory until its state copy has landed.
#include <hip/hip_runtime.h>

#include <execinfo.h>
#include <signal.h>
#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "../../include/adgi.h"
#include "adgi_internal.hpp"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

thread_local char g_serve_err[512];

// A request waiting longer than kMaxWaitNs is admitted even if that evicts
// streams that have work waiting, provided they have been resident for
// kMinResidencyNs.
constexpr int64_t kMaxWaitNs = 250'000'000;
constexpr int64_t kMinResidencyNs = 500'000'000;

adgi_status sfail(adgi_status st, const char* msg) {
  std::snprintf(g_serve_err, sizeof(g_serve_err), "%s", msg);
  return st;
}

// A volume call's failure, with the volume's message.
adgi_status pass(adgi_status e) {
  if (e != ADGI_OK) std::snprintf(g_serve_err, sizeof(g_serve_err), "%s", adgi_last_error());
  return e;
}

// Device memory for the server's volumes when the caller gives no allocator:
// freed blocks are kept by exact size and handed out again, so evicting and
// re-admitting a stream allocates and frees nothing on the device (hipFree
// would wait for every stream on the GPU).
struct Pool {
  std::multimap<size_t, void*> free_blocks;
  std::map<void*, size_t> size_of;
  int64_t held = 0;
};

// With ADGI_CRASH_TRACE set in the environment, a segmentation fault in a
// process that created a server prints the native stack (symbols, or offsets
// into the library for addr2line) to stderr, then hands the signal to the
// handler installed before (Python's faulthandler, or the default action).
struct sigaction g_prev_segv;

void crash_trace(int sig, siginfo_t*, void*) {
  void* frames[64];
  const int n = backtrace(frames, 64);
  static const char msg[] = "adgi: native stack at the fault:\n";
  if (write(2, msg, sizeof(msg) - 1) < 0) {
  }
  backtrace_symbols_fd(frames, n, 2);
  sigaction(SIGSEGV, &g_prev_segv, nullptr);
  raise(sig);
}

void install_crash_trace() {
  static std::once_flag once;
  std::call_once(once, [] {
    if (!std::getenv("ADGI_CRASH_TRACE")) return;
    void* warm[1];
    (void)backtrace(warm, 1);  // loads the unwinder now, not inside the handler
    struct sigaction sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.sa_sigaction = crash_trace;
    sa.sa_flags = SA_SIGINFO;
    sigemptyset(&sa.sa_mask);
    sigaction(SIGSEGV, &sa, &g_prev_segv);
  });
}

void* pool_alloc(size_t bytes, void* ctx) {
  Pool* p = static_cast<Pool*>(ctx);
  auto it = p->free_blocks.find(bytes);
  if (it != p->free_blocks.end()) {
    void* ptr = it->second;
    p->free_blocks.erase(it);
    return ptr;
  }
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes) != hipSuccess) return nullptr;
  p->size_of[ptr] = bytes;
  p->held += (int64_t)bytes;
  return ptr;
}

void pool_free(void* ptr, void* ctx) {
  Pool* p = static_cast<Pool*>(ctx);
  auto it = p->size_of.find(ptr);
  if (it != p->size_of.end()) p->free_blocks.insert({it->second, ptr});
}

struct Request {
  int32_t stream = 0;
  int32_t frame = 0;
  float lights[ADGI_MAX_LIGHTS][3] = {};
  int64_t arrival_ns = 0, dispatch_ns = 0;
  int64_t done_ns = 0;  // when the dispatcher saw the frame done
  bool completed = false;
};

struct Stream {
  adgi_volume_desc vdesc{};
  std::vector<float> positions, albedo, light_int;
  std::vector<int32_t> indices;
  float sky[3] = {0.f, 0.f, 0.f};
  int32_t num_lights = 0;
  adgi::BuiltScene built;
  adgi_update_params params{};
  int64_t footprint = 0;
  adgi_volume* vol = nullptr;
  // temporal state while evicted, in pinned host memory sized when the
  // stream is added (state_len 0: fresh), so eviction and admission copy at
  // full PCIe rate
  uint8_t* state_buf = nullptr;
  size_t state_cap = 0, state_len = 0;
  // an evicted volume whose state copy is still in flight: it keeps its
  // device memory (and its share of the budget) until retire_ev completes
  adgi_volume* retiring = nullptr;
  hipEvent_t retire_ev = nullptr;
  hipEvent_t start_ev = nullptr; // recorded on the lane before the frame in flight
  hipEvent_t done_ev = nullptr;  // recorded behind the frame in flight
  int32_t lane = -1;             // server lane of the frame in flight
  int32_t next_frame = 0;
  std::deque<int64_t> pending;  // request ids not yet dispatched, in order
  int64_t inflight = -1;
  int64_t last_use_ns = 0;
  int64_t admitted_ns = 0;

  Stream() = default;
  Stream(const Stream&) = delete;
  Stream& operator=(const Stream&) = delete;
  ~Stream() {
    if (retire_ev) (void)hipEventDestroy(retire_ev);
    if (start_ev) (void)hipEventDestroy(start_ev);
    if (done_ev) (void)hipEventDestroy(done_ev);
    if (state_buf) (void)hipHostFree(state_buf);
    adgi::unpin_scene(built);
  }

  adgi_scene_desc scene(int32_t mode, const float* lights) const {
    adgi_scene_desc d{};
    d.positions = positions.data();
    d.num_vertices = (int32_t)(positions.size() / 3);
    d.indices = indices.data();
    d.num_triangles = (int32_t)(indices.size() / 3);
    d.albedo = albedo.data();
    d.light_pos = lights;
    d.light_intensity = light_int.data();
    d.num_lights = num_lights;
    for (int a = 0; a < 3; ++a) d.sky[a] = sky[a];
    d.mode = mode;
    d.refit_vertex_begin = 0;
    d.refit_vertex_end = 0;
    return d;
  }
};


}  // namespace

struct adgi_server {
  adgi_allocator alloc{};
  Pool pool;
  int64_t budget = 0;
  int32_t max_inflight = 4;
  // Frames run on a few server-owned streams ("lanes"), created in a row so
  // the runtime spreads them over its hardware queues: a hardware queue
  // runs its work in order, and streams created one volume at a time can
  // all land on the same queue, serialising every stream's frames.
  // The runtime gives a new stream the queue with the fewest streams, so
  // lanes created after other streams crowd onto the emptiest queues first;
  // there are twice as many lanes as in-flight slots and frames take them in
  // rotation (least loaded first), which spreads them over every queue.
  std::vector<hipStream_t> lanes;
  std::vector<int32_t> lane_load;
  size_t next_lane = 0;
  std::vector<std::unique_ptr<Stream>> streams;
  std::deque<Request> reqs;     // stable addresses for the completion callbacks
  std::deque<int64_t> waiting;  // undispatched request ids, arrival order
  int32_t inflight = 0;
  int64_t resident = 0, peak_resident = 0;
  int64_t retiring_bytes = 0;  // part of `resident` held by retiring volumes
  int64_t admissions = 0, evictions = 0, completed = 0, rays = 0;
  int64_t first_arrival_ns = 0, last_done_ns = 0;
  double admit_ms = 0.0, evict_ms = 0.0;
  double busy_ms = 0.0;  // sum over completed frames of start -> done on the device
  std::vector<double> latency_ms;
};

namespace {

// Eviction enqueues the state copy behind the stream's last frame and
// retires the volume; its memory is released once the copy has landed
// (finish_retire), so the dispatcher never waits on the transfer.
adgi_status evict(adgi_server* s, Stream& st) {
  auto t0 = now_ns();
  const size_t n = adgi_state_size(st.vol);
  if (!st.state_buf || n > st.state_cap) return sfail(ADGI_ERR_DEVICE, "stream state outgrew its host buffer");
  // idle: the copy goes on the volume's own stream, not behind a lane
  adgi_status e = adgi::bind_streams(st.vol, nullptr);
  if (e != ADGI_OK) return pass(e);
  e = adgi::save_state_impl(st.vol, st.state_buf, n, true);
  if (e != ADGI_OK) return pass(e);
  if (hipEventRecord(st.retire_ev, adgi::volume_stream(st.vol)) != hipSuccess)
    return sfail(ADGI_ERR_DEVICE, "hipEventRecord failed");
  st.state_len = n;
  st.retiring = st.vol;
  st.vol = nullptr;
  s->retiring_bytes += st.footprint;
  ++s->evictions;
  s->evict_ms += (now_ns() - t0) * 1e-6;
  return ADGI_OK;
}

// Releases a retired volume once its state copy is done (or, with `wait`,
// after waiting for it); true if the volume was released.
bool finish_retire(adgi_server* s, Stream& st, bool wait) {
  if (!st.retiring) return false;
  if (wait) {
    if (hipEventSynchronize(st.retire_ev) != hipSuccess) return false;
  } else if (hipEventQuery(st.retire_ev) != hipSuccess) {
    return false;
  }
  auto t0 = now_ns();
  adgi_destroy_volume(st.retiring);
  st.retiring = nullptr;
  s->resident -= st.footprint;
  s->retiring_bytes -= st.footprint;
  s->evict_ms += (now_ns() - t0) * 1e-6;
  return true;
}

// Releases every retired volume whose copy is done, except `keep`'s.
void reap(adgi_server* s, const Stream* keep = nullptr) {
  if (!s->retiring_bytes) return;
  for (auto& p : s->streams)
    if (p.get() != keep) finish_retire(s, *p, false);
}

adgi_status make_resident(adgi_server* s, Stream& st) {
  auto t0 = now_ns();
  if (st.retiring) {
    // re-admitted before its eviction finished: the volume still holds the
    // live state, and the copy in flight ahead of the next frame is harmless
    st.vol = st.retiring;
    st.retiring = nullptr;
    s->retiring_bytes -= st.footprint;
    st.admitted_ns = now_ns();
    ++s->admissions;
    s->admit_ms += (now_ns() - t0) * 1e-6;
    return ADGI_OK;
  }
  adgi_volume* vol = nullptr;
  adgi_status e = adgi_create_volume(&st.vdesc, &s->alloc, nullptr, &vol);
  if (e != ADGI_OK) return pass(e);
  std::vector<float> lp(3 * (size_t)std::max(st.num_lights, 1), 0.f);
  adgi_scene_desc sd = st.scene(ADGI_SCENE_REBUILD, lp.data());
  e = adgi::update_scene_impl(vol, &sd, &st.built);
  // the state copy is enqueued on the volume's stream: state_buf is next
  // written by this stream's eviction, which first waits for that stream
  if (e == ADGI_OK && st.state_len > st.state_cap) e = sfail(ADGI_ERR_DEVICE, "stream state larger than its host buffer");
  if (e == ADGI_OK && st.state_len) e = adgi::restore_state_impl(vol, st.state_buf, st.state_len, true);
  if (e != ADGI_OK) {
    pass(e);
    adgi_destroy_volume(vol);
    return e;
  }
  st.vol = vol;
  st.admitted_ns = now_ns();
  s->resident += st.footprint;
  s->peak_resident = std::max(s->peak_resident, s->resident);
  ++s->admissions;
  s->admit_ms += (now_ns() - t0) * 1e-6;
  return ADGI_OK;
}

// Makes room to admit `target`: evicts idle streams until it fits once
// every retiring copy has landed; false if it cannot yet. A target whose
// own volume is still retiring needs no room (it is revived, and keeps its
// share of the budget). gentle: only streams with no request waiting are
// evicted. block: wait for retiring copies instead of returning false while
// they are in flight.
bool make_room(adgi_server* s, const Stream& target, bool gentle, bool block, adgi_status* err) {
  const int64_t need = target.retiring ? 0 : target.footprint;
  reap(s, &target);
  while (s->resident - s->retiring_bytes + need > s->budget) {
    Stream* victim = nullptr;
    for (auto& p : s->streams) {
      Stream& c = *p;
      if (!c.vol || c.inflight >= 0) continue;
      if (!c.pending.empty() && (gentle || now_ns() - c.admitted_ns < kMinResidencyNs)) continue;
      if (!victim) {
        victim = &c;
        continue;
      }
      const bool cw = !c.pending.empty(), vw = !victim->pending.empty();
      if (cw != vw ? !cw : c.last_use_ns < victim->last_use_ns) victim = &c;
    }
    if (!victim) return false;
    if ((*err = evict(s, *victim)) != ADGI_OK) return false;
  }
  if (s->resident + need <= s->budget) return true;
  if (!block) {
    reap(s, &target);
    return s->resident + need <= s->budget;
  }
  for (auto& p : s->streams) {
    if (s->resident + need <= s->budget) break;
    if (p.get() != &target) finish_retire(s, *p, true);
  }
  return s->resident + need <= s->budget;
}

adgi_status dispatch(adgi_server* s, Stream& st, int64_t id) {
  if (id < 0 || id >= (int64_t)s->reqs.size()) return sfail(ADGI_ERR_INVALID_ARG, "request id out of range");
  if (!st.vol || st.inflight >= 0) return sfail(ADGI_ERR_INVALID_ARG, "stream not idle and resident");
  Request& r = s->reqs[id];
  // the stream is idle: its last frame is done, so it may change lanes
  const size_t nl = s->lanes.size();
  if (nl == 0 || s->lane_load.size() != nl) return sfail(ADGI_ERR_DEVICE, "server has no lanes");
  size_t k = s->next_lane % nl;
  for (size_t a = 1; a < nl; ++a) {
    const size_t j = (s->next_lane + a) % nl;
    if (s->lane_load[j] < s->lane_load[k]) k = j;
  }
  adgi_status e = adgi::bind_streams(st.vol, s->lanes[k]);
  if (e != ADGI_OK) return pass(e);
  if (hipEventRecord(st.start_ev, s->lanes[k]) != hipSuccess) return sfail(ADGI_ERR_DEVICE, "hipEventRecord failed");
  adgi_scene_desc sd = st.scene(ADGI_SCENE_REFIT, &r.lights[0][0]);
  e = adgi_update_scene(st.vol, &sd);
  if (e != ADGI_OK) return pass(e);
  adgi_update_params p = st.params;
  p.frame = st.next_frame;
  p.sync = 0;
  if ((e = adgi_update_probes(st.vol, &p, nullptr)) != ADGI_OK) return pass(e);
  if (hipEventRecord(st.done_ev, adgi::volume_stream(st.vol)) != hipSuccess)
    return sfail(ADGI_ERR_DEVICE, "hipEventRecord failed");
  r.frame = st.next_frame++;
  r.dispatch_ns = now_ns();
  st.lane = (int32_t)k;
  ++s->lane_load[k];
  s->next_lane = k + 1;
  st.inflight = id;
  st.pending.pop_front();
  ++s->inflight;
  return ADGI_OK;
}

adgi_status progress_once(adgi_server* s, int32_t* done_now) {
  int32_t done = 0;
  for (auto& p : s->streams) {
    Stream& st = *p;
    if (st.inflight < 0) continue;
    if (st.inflight >= (int64_t)s->reqs.size() || st.lane < 0 || st.lane >= (int32_t)s->lanes.size())
      return sfail(ADGI_ERR_DEVICE, "in-flight bookkeeping out of range");
    Request& r = s->reqs[st.inflight];
    if (hipEventQuery(st.done_ev) != hipSuccess) continue;
    const int64_t t = now_ns();
    float span_ms = 0.f;
    if (hipEventElapsedTime(&span_ms, st.start_ev, st.done_ev) == hipSuccess) s->busy_ms += span_ms;
    r.done_ns = t;
    r.completed = true;
    s->latency_ms.push_back((t - r.arrival_ns) * 1e-6);
    s->rays += st.params.budget;
    s->last_done_ns = std::max(s->last_done_ns, t);
    st.last_use_ns = t;
    st.inflight = -1;
    --s->lane_load[st.lane];
    st.lane = -1;
    --s->inflight;
    ++s->completed;
    ++done;
  }
  // (1) a request that has waited too long goes first, evicting whatever idle
  //     stream it must (bounds the wait of streams that are not resident)
  if (!s->waiting.empty() && s->inflight < s->max_inflight) {
    const int64_t id = s->waiting.front();
    Stream& st = *s->streams[s->reqs[id].stream];
    if (!st.vol && st.inflight < 0 && st.pending.front() == id &&
        now_ns() - s->reqs[id].arrival_ns > kMaxWaitNs) {
      adgi_status err = ADGI_OK;
      if (make_room(s, st, /*gentle=*/false, /*block=*/false, &err)) {
        if ((err = make_resident(s, st)) != ADGI_OK) return err;
        // dispatched by (2) once its setup copies have landed
      } else if (err != ADGI_OK) {
        return err;
      }
    }
  }
  // (2) resident streams, in arrival order
  for (size_t k = 0; k < s->waiting.size() && s->inflight < s->max_inflight;) {
    const int64_t id = s->waiting[k];
    Stream& st = *s->streams[s->reqs[id].stream];
    // a volume just admitted waits until its uploads and state copy have
    // landed: a lane made to wait for them would hold up every frame behind
    if (!st.vol || st.inflight >= 0 || st.pending.front() != id || !adgi::volume_settled(st.vol)) {
      ++k;
      continue;
    }
    adgi_status e = dispatch(s, st, id);
    if (e != ADGI_OK) return e;
    s->waiting.erase(s->waiting.begin() + (std::ptrdiff_t)k);
  }
  // (3) admissions, in arrival order, evicting only idle streams with nothing
  //     waiting (after (2) every idle resident stream is one, unless the
  //     in-flight limit stopped (2), in which case this loop does not run)
  for (size_t k = 0; k < s->waiting.size() && s->inflight < s->max_inflight;) {
    const int64_t id = s->waiting[k];
    Stream& st = *s->streams[s->reqs[id].stream];
    if (st.vol || st.inflight >= 0 || st.pending.front() != id) {
      ++k;
      continue;
    }
    adgi_status err = ADGI_OK;
    if (!make_room(s, st, /*gentle=*/true, /*block=*/false, &err)) {
      if (err != ADGI_OK) return err;
      break;  // the budget is held by streams in flight or with work waiting
    }
    if ((err = make_resident(s, st)) != ADGI_OK) return err;
    if (adgi::volume_settled(st.vol)) {
      if ((err = dispatch(s, st, id)) != ADGI_OK) return err;
      s->waiting.erase(s->waiting.begin() + (std::ptrdiff_t)k);
    } else {
      ++k;  // dispatched by (2) on a later pass
    }
  }
  if (done_now) *done_now = done;
  return ADGI_OK;
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q / 100.0 * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

extern "C" {

int64_t adgi_server_now_ns(void) { return now_ns(); }

const char* adgi_server_last_error(void) { return g_serve_err; }

adgi_status adgi_server_create(const adgi_server_desc* desc, const adgi_allocator* alloc, adgi_server** out) {
  install_crash_trace();
  if (!desc || !out) return sfail(ADGI_ERR_INVALID_ARG, "desc and out must not be NULL");
  if (desc->hbm_budget_bytes <= 0 || desc->max_inflight < 1 || desc->max_inflight > 64)
    return sfail(ADGI_ERR_INVALID_ARG, "need hbm_budget_bytes > 0 and max_inflight in [1, 64]");
  auto* s = new adgi_server();
  s->budget = desc->hbm_budget_bytes;
  s->max_inflight = desc->max_inflight;
  if (alloc && (!alloc->alloc || !alloc->free)) {
    delete s;
    return sfail(ADGI_ERR_INVALID_ARG, "allocator callbacks must not be NULL");
  }
  s->alloc = alloc ? *alloc : adgi_allocator{pool_alloc, pool_free, &s->pool};
  const int nl = std::min(2 * desc->max_inflight, 16);
  for (int k = 0; k < nl; ++k) {
    hipStream_t l = nullptr;
    if (hipStreamCreateWithFlags(&l, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->lanes) (void)hipStreamDestroy(x);
      delete s;
      return sfail(ADGI_ERR_DEVICE, "hipStreamCreate failed");
    }
    s->lanes.push_back(l);
  }
  s->lane_load.assign(s->lanes.size(), 0);
  *out = s;
  return ADGI_OK;
}

adgi_status adgi_server_set_budget(adgi_server* s, int64_t hbm_budget_bytes) {
  if (!s || hbm_budget_bytes <= 0) return sfail(ADGI_ERR_INVALID_ARG, "bad server or budget");
  for (auto& p : s->streams)
    if (p->footprint > hbm_budget_bytes) return sfail(ADGI_ERR_OUT_OF_MEMORY, "a stream exceeds the budget");
  s->budget = hbm_budget_bytes;
  return ADGI_OK;
}

adgi_status adgi_server_add_stream(adgi_server* s, const adgi_stream_desc* d, int32_t* id) {
  if (!s || !d || !id) return sfail(ADGI_ERR_INVALID_ARG, "server, desc and id must not be NULL");
  const adgi_scene_desc& sc = d->scene;
  if (sc.num_lights < 0 || sc.num_lights > ADGI_MAX_LIGHTS || sc.num_vertices <= 0 || sc.num_triangles <= 0 ||
      !sc.positions || !sc.indices || !sc.albedo || (sc.num_lights > 0 && !sc.light_intensity))
    return sfail(ADGI_ERR_INVALID_ARG, "stream scene needs vertices, triangles, albedo and light intensities");
  if (d->params.adaptive != 1) return sfail(ADGI_ERR_INVALID_ARG, "serving streams run adaptive frames");
  auto st = std::make_unique<Stream>();
  st->vdesc = d->volume;
  st->positions.assign(sc.positions, sc.positions + 3 * (size_t)sc.num_vertices);
  st->indices.assign(sc.indices, sc.indices + 3 * (size_t)sc.num_triangles);
  st->albedo.assign(sc.albedo, sc.albedo + 3 * (size_t)sc.num_triangles);
  st->light_int.assign(3 * (size_t)std::max(sc.num_lights, 1), 0.f);
  if (sc.num_lights > 0) std::memcpy(st->light_int.data(), sc.light_intensity, 12 * (size_t)sc.num_lights);
  for (int a = 0; a < 3; ++a) st->sky[a] = sc.sky[a];
  st->num_lights = sc.num_lights;
  st->params = d->params;
  // the padding term depends on the light positions given here
  adgi_scene_desc bd = st->scene(ADGI_SCENE_REBUILD, sc.light_pos);
  const char* err = "";
  if (!adgi::build_scene(st->vdesc, &bd, st->built, &err)) return sfail(ADGI_ERR_INVALID_ARG, err);
  // a pinned image of the uploaded arrays lets every admission enqueue them
  // and return; without one (pinned memory refused) admission copies
  // synchronously
  (void)adgi::pin_scene(st->built, &bd);
  // footprint: build the volume once, measure, release
  adgi_volume* vol = nullptr;
  adgi_status e = adgi_create_volume(&st->vdesc, &s->alloc, nullptr, &vol);
  if (e != ADGI_OK) return pass(e);
  e = adgi::update_scene_impl(vol, &bd, &st->built);
  if (e == ADGI_OK) {
    adgi_update_params p = st->params;
    p.frame = 0;
    p.sync = 1;
    // a dry frame validates the parameters; the stream still starts from zero state
    e = adgi_update_probes(vol, &p, nullptr);
  }
  st->footprint = (int64_t)adgi_device_bytes(vol);
  st->state_cap = adgi_state_size(vol);
  if (e != ADGI_OK) pass(e);
  adgi_destroy_volume(vol);
  if (e != ADGI_OK) return e;
  if (hipHostMalloc((void**)&st->state_buf, std::max<size_t>(st->state_cap, 1), hipHostMallocDefault) != hipSuccess)
    return sfail(ADGI_ERR_OUT_OF_MEMORY, "pinned host buffer for the stream state");
  if (hipEventCreateWithFlags(&st->retire_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&st->start_ev) != hipSuccess || hipEventCreate(&st->done_ev) != hipSuccess)
    return sfail(ADGI_ERR_DEVICE, "hipEventCreate failed");
  if (st->footprint > s->budget) return sfail(ADGI_ERR_OUT_OF_MEMORY, "stream footprint exceeds the HBM budget");
  *id = (int32_t)s->streams.size();
  s->streams.push_back(std::move(st));
  return ADGI_OK;
}

adgi_status adgi_server_stream_info(const adgi_server* s, int32_t id, int64_t* footprint_bytes,
                                    int32_t* resident, int32_t* frames_done) {
  if (!s || id < 0 || id >= (int32_t)s->streams.size()) return sfail(ADGI_ERR_INVALID_ARG, "bad stream id");
  const Stream& st = *s->streams[id];
  if (footprint_bytes) *footprint_bytes = st.footprint;
  if (resident) *resident = st.vol ? 1 : 0;
  if (frames_done) *frames_done = st.next_frame - (st.inflight >= 0 ? 1 : 0);
  return ADGI_OK;
}

adgi_status adgi_server_submit(adgi_server* s, int32_t id, const float* light_pos, int64_t arrival_ns) {
  if (!s || id < 0 || id >= (int32_t)s->streams.size()) return sfail(ADGI_ERR_INVALID_ARG, "bad stream id");
  Stream& st = *s->streams[id];
  if (st.num_lights > 0 && !light_pos) return sfail(ADGI_ERR_INVALID_ARG, "light_pos is NULL");
  s->reqs.emplace_back();
  Request& r = s->reqs.back();
  r.stream = id;
  r.arrival_ns = arrival_ns;
  if (st.num_lights > 0) std::memcpy(r.lights, light_pos, 12 * (size_t)st.num_lights);
  const int64_t rid = (int64_t)s->reqs.size() - 1;
  if (s->reqs.size() == 1) s->first_arrival_ns = arrival_ns;
  st.pending.push_back(rid);
  s->waiting.push_back(rid);
  return ADGI_OK;
}

adgi_status adgi_server_progress(adgi_server* s, int32_t* completed_now) {
  if (!s) return sfail(ADGI_ERR_INVALID_ARG, "server is NULL");
  return progress_once(s, completed_now);
}

adgi_status adgi_server_drain(adgi_server* s) {
  if (!s) return sfail(ADGI_ERR_INVALID_ARG, "server is NULL");
  for (;;) {
    adgi_status e = progress_once(s, nullptr);
    if (e != ADGI_OK) return e;
    if (s->waiting.empty() && s->inflight == 0) return ADGI_OK;
    if (s->inflight > 0) {
      // wait for the oldest frame in flight instead of spinning
      for (auto& p : s->streams)
        if (p->inflight >= 0) {
          if (hipStreamSynchronize(adgi::volume_stream(p->vol)) != hipSuccess)
            return sfail(ADGI_ERR_DEVICE, "hipStreamSynchronize failed");
          break;
        }
    } else if (s->retiring_bytes) {
      // admissions wait for a state copy to land
      for (auto& p : s->streams)
        if (finish_retire(s, *p, true)) break;
    }
  }
}

adgi_status adgi_server_get_stats(const adgi_server* s, adgi_server_stats* out) {
  if (!s || !out) return sfail(ADGI_ERR_INVALID_ARG, "server and out must not be NULL");
  std::memset(out, 0, sizeof(*out));
  out->submitted = (int64_t)s->reqs.size();
  out->completed = s->completed;
  out->admissions = s->admissions;
  out->evictions = s->evictions;
  out->primary_rays = s->rays;
  out->resident_bytes = s->resident;
  out->peak_resident_bytes = s->peak_resident;
  out->p50_ms = percentile(s->latency_ms, 50.0);
  out->p99_ms = percentile(s->latency_ms, 99.0);
  out->max_ms = s->latency_ms.empty() ? 0.0 : *std::max_element(s->latency_ms.begin(), s->latency_ms.end());
  double sum = 0.0;
  for (double x : s->latency_ms) sum += x;
  out->mean_ms = s->latency_ms.empty() ? 0.0 : sum / (double)s->latency_ms.size();
  out->span_s = s->completed ? (s->last_done_ns - s->first_arrival_ns) * 1e-9 : 0.0;
  out->admit_ms = s->admit_ms;
  out->evict_ms = s->evict_ms;
  out->device_busy_ms = s->busy_ms;
  return ADGI_OK;
}

adgi_status adgi_server_latencies(const adgi_server* s, double* out_ms, int64_t capacity, int64_t* count) {
  if (!s || !count) return sfail(ADGI_ERR_INVALID_ARG, "server and count must not be NULL");
  *count = (int64_t)s->latency_ms.size();
  if (out_ms)
    std::memcpy(out_ms, s->latency_ms.data(), sizeof(double) * (size_t)std::min<int64_t>(capacity, *count));
  return ADGI_OK;
}

adgi_status adgi_server_read_stream(adgi_server* s, int32_t id, adgi_probe_readback* rb) {
  if (!s || !rb || id < 0 || id >= (int32_t)s->streams.size()) return sfail(ADGI_ERR_INVALID_ARG, "bad arguments");
  Stream& st = *s->streams[id];
  if (st.inflight >= 0 || !st.pending.empty()) return sfail(ADGI_ERR_INVALID_ARG, "stream has frames outstanding");
  if (!st.vol) {
    adgi_status err = ADGI_OK;
    if (!make_room(s, st, false, true, &err))
      return err != ADGI_OK ? err : sfail(ADGI_ERR_OUT_OF_MEMORY, "no room to admit the stream");
    if ((err = make_resident(s, st)) != ADGI_OK) return err;
  }
  // idle: read on the volume's own stream rather than behind a lane
  adgi_status e = adgi::bind_streams(st.vol, nullptr);
  if (e != ADGI_OK) return pass(e);
  return pass(adgi_read_probes(st.vol, rb));
}

void adgi_server_destroy(adgi_server* s) {
  if (!s) return;
  for (auto& p : s->streams) {
    if (p->vol) {
      (void)hipStreamSynchronize(adgi::volume_stream(p->vol));
      (void)adgi::bind_streams(p->vol, nullptr);
      adgi_destroy_volume(p->vol);
    }
    if (p->retiring) adgi_destroy_volume(p->retiring);
  }
  for (auto& kv : s->pool.size_of) (void)hipFree(kv.first);
  for (hipStream_t l : s->lanes) (void)hipStreamDestroy(l);
  delete s;
}

}  // extern "C"
