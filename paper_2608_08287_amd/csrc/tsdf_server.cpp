// Host half of the serving calls of include/tsdf.h (tsdf_server_*): session
// admission against a device budget, the frame queue, continuous batching
// through tsdf_batch_fuse, per-session failure marking, and a real-time
// replay driver for arrival traces.
//
// Ordering: a server has max_inflight streams: the one given at creation and
// max_inflight - 1 of its own (default priority).  Volume initialisation and
// the plain launches of a replay go to the first; each fusion launch (its work
// list copy, kernels and status gather) goes to a stream that has no launch
// running, so launches overlap on the device and a frame that arrives while
// others are being fused starts at once.  Launches may finish out of order;
// one event per launch tells when its frames are fused.  A session's volume is
// initialised on the first stream, and the other streams wait for an event
// recorded behind that before any launch can reach the volume.  Launches into
// one volume may run at once on different streams: fusion is a sum, and every
// update the kernels make is an atomic one.

#include <chrono>
#include <deque>
#include <new>
#include <vector>

#include "tsdf_host.h"

using namespace tsdf_host;

namespace {

constexpr uint32_t kMaxSessions = 65536;
constexpr uint32_t kMaxInflight = 4;  // one stream per launch; within the device's hardware queues
constexpr uint32_t kMaxQueue = 1u << 24;

struct Session {
  bool open = false;
  tsdf_volume* vol = nullptr;
  void* arena = nullptr;
  int32_t failure = TSDF_OK;
  uint32_t inflight = 0;     // frames in launches not yet retired
  uint64_t opened_at = 0;    // sequence number of the first launch after opening
};

struct Pending {
  uint32_t session;
  const float* depth;
  tsdf_camera cam;
  uint64_t tag;
};

// One launch: its frames complete at `done`; the status copy behind it
// completes at `gathered`.  Frames are handed back as soon as `done` has
// passed, so the status copy stays off the frames' latency.
struct Launch {
  uint64_t seq;
  uint32_t stream;  // index into the server's streams
  hipEvent_t done;
  hipEvent_t gathered;
  bool frames_retired = false;
  std::vector<uint32_t> sessions;  // one entry per frame
  std::vector<uint64_t> tags;
};

bool valid_params(const tsdf_server_params* p) {
  return p && p->max_sessions >= 1 && p->max_sessions <= kMaxSessions && p->max_batch >= 1 &&
         p->max_batch <= TSDF_BATCH_MAX_ITEMS && p->max_inflight >= 1 &&
         p->max_inflight <= kMaxInflight && p->max_queue >= p->max_batch &&
         p->max_queue <= kMaxQueue;
}

int32_t failure_of(uint32_t bits) {
  if (bits & TSDF_FLAG_INTERNAL) return TSDF_ERR_INTERNAL;
  if (bits & TSDF_FLAG_TABLE_FULL) return TSDF_ERR_TABLE_FULL;
  if (bits & TSDF_FLAG_POOL_EXHAUSTED) return TSDF_ERR_POOL_EXHAUSTED;
  return TSDF_OK;
}

double now_ns() {
  return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct tsdf_server {
  tsdf_server_params p;
  hipStream_t stream = nullptr;        // the caller's: streams[0]
  std::vector<hipStream_t> streams;    // one per launch in flight
  std::vector<bool> stream_busy;
  hipEvent_t opened = nullptr;         // behind the latest volume initialisation
  tsdf_batch* batch = nullptr;
  tsdf_region* region = nullptr;
  std::vector<Session> sessions;
  uint32_t n_open = 0;
  std::deque<Pending> queue;
  std::deque<Launch> inflight;
  uint32_t running = 0;  // launches whose frames have not completed
  std::vector<hipEvent_t> spare_events;
  std::deque<std::pair<uint64_t, int32_t>> done;
  uint64_t next_seq = 0;
  uint32_t inflight_frames = 0;
  // pinned, device-mapped mirrors: counters pointer per session (read by the
  // gather kernel) and the sticky status it copies out, one row of
  // max_sessions words per stream, so that a gather running late on one stream
  // never overwrites what a later gather on another stream wrote
  tsdf::DevCounters** ctr_host = nullptr;
  tsdf::DevCounters** ctr_dev = nullptr;
  unsigned* status_host = nullptr;
  unsigned* status_dev = nullptr;
  std::vector<tsdf_fuse_item> items;  // per-launch scratch
};

namespace {

void release_session(tsdf_server* s, uint32_t id) {
  Session& ss = s->sessions[id];
  if (ss.vol) (void)tsdf_destroy_volume(ss.vol);
  if (ss.arena) (void)tsdf_region_free(s->region, ss.arena);
  s->ctr_host[id] = nullptr;
  ss = Session();
  --s->n_open;
}

hipError_t poll(hipEvent_t ev, bool wait) {
  return wait ? hipEventSynchronize(ev) : hipEventQuery(ev);
}

// Hand back the frames of launches that have finished, and read the status
// words of those whose status copy has finished.  Launches on different
// streams finish in any order.  Non-blocking unless `wait_all`.
tsdf_status retire(tsdf_server* s, bool wait_all) {
  for (Launch& L : s->inflight) {
    if (L.frames_retired) continue;
    const hipError_t e = poll(L.done, wait_all);
    if (e == hipErrorNotReady) continue;
    if (e != hipSuccess) return TSDF_ERR_HIP;
    for (size_t i = 0; i < L.tags.size(); ++i) {
      s->done.emplace_back(L.tags[i], (int32_t)TSDF_OK);
      --s->sessions[L.sessions[i]].inflight;
    }
    s->inflight_frames -= (uint32_t)L.tags.size();
    L.frames_retired = true;
    --s->running;
    // a new launch on this stream queues behind the small status copy only
    s->stream_busy[L.stream] = false;
  }
  for (auto it = s->inflight.begin(); it != s->inflight.end();) {
    Launch& L = *it;
    if (!L.frames_retired) {
      ++it;
      continue;
    }
    const hipError_t e = poll(L.gathered, wait_all);
    if (e == hipErrorNotReady) {
      ++it;
      continue;
    }
    if (e != hipSuccess) return TSDF_ERR_HIP;
    // statuses copied behind this launch, or behind a later one on its stream,
    // are current for sessions opened before it was made (status bits are only
    // ever set while a session is open)
    const unsigned* row = s->status_host + (size_t)L.stream * s->p.max_sessions;
    for (uint32_t id = 0; id < s->p.max_sessions; ++id) {
      Session& ss = s->sessions[id];
      if (!ss.open || ss.failure != TSDF_OK || L.seq < ss.opened_at) continue;
      ss.failure = failure_of(__atomic_load_n(&row[id], __ATOMIC_ACQUIRE));
    }
    s->spare_events.push_back(L.done);
    s->spare_events.push_back(L.gathered);
    it = s->inflight.erase(it);
  }
  return TSDF_OK;
}

bool take_event(tsdf_server* s, hipEvent_t* ev) {
  if (s->spare_events.empty()) {
    if (hipEventCreateWithFlags(ev, hipEventDisableTiming) != hipSuccess) return false;
    return true;
  }
  *ev = s->spare_events.back();
  s->spare_events.pop_back();
  return true;
}

tsdf_status launch_one(tsdf_server* s, uint32_t* launched) {
  s->items.clear();
  Launch L;
  while (!s->queue.empty() && s->items.size() < s->p.max_batch) {
    const Pending q = s->queue.front();
    s->queue.pop_front();
    Session& ss = s->sessions[q.session];
    if (ss.failure != TSDF_OK) {
      s->done.emplace_back(q.tag, ss.failure);
      continue;
    }
    s->items.push_back(tsdf_fuse_item{ss.vol, q.depth, nullptr, q.cam});
    L.sessions.push_back(q.session);
    L.tags.push_back(q.tag);
  }
  if (s->items.empty()) return TSDF_OK;
  uint32_t k = 0;
  while (k < s->streams.size() && s->stream_busy[k]) ++k;
  if (k == s->streams.size()) return TSDF_ERR_INTERNAL;  // the caller checked for room
  hipStream_t st_k = s->streams[k];
  L.stream = k;
  if (!take_event(s, &L.done)) return TSDF_ERR_HIP;
  if (!take_event(s, &L.gathered)) {
    s->spare_events.push_back(L.done);
    return TSDF_ERR_HIP;
  }
  // A lone frame takes the one-volume kernel: no work list to copy, no tile
  // search.  Several frames share one persistent launch.
  const tsdf_fuse_item& one = s->items[0];
  tsdf_status st = s->items.size() == 1
                       ? tsdf_fuse_frame(one.volume, one.depth_dev, &one.camera, st_k)
                       : tsdf_batch_fuse(s->batch, s->items.data(), (uint32_t)s->items.size(), 0,
                                         st_k);
  if (st == TSDF_OK) st = hip_status(hipEventRecord(L.done, st_k));
  if (st == TSDF_OK)
    st = hip_status(tsdf::launch_gather_status(
        s->ctr_dev, s->p.max_sessions, s->status_dev + (size_t)k * s->p.max_sessions, st_k));
  if (st == TSDF_OK) st = hip_status(hipEventRecord(L.gathered, st_k));
  if (st != TSDF_OK) {
    s->spare_events.push_back(L.done);
    s->spare_events.push_back(L.gathered);
    return st;
  }
  L.seq = s->next_seq++;
  s->stream_busy[k] = true;
  for (uint32_t id : L.sessions) ++s->sessions[id].inflight;
  s->inflight_frames += (uint32_t)L.tags.size();
  ++s->running;
  if (launched) *launched = (uint32_t)L.tags.size();
  s->inflight.push_back(std::move(L));
  return TSDF_OK;
}

void free_server(tsdf_server* s) {
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (uint32_t id = 0; id < s->sessions.size(); ++id)
    if (s->sessions[id].open) release_session(s, id);
  for (Launch& L : s->inflight) {
    s->spare_events.push_back(L.done);
    s->spare_events.push_back(L.gathered);
  }
  for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
  if (s->opened) (void)hipEventDestroy(s->opened);
  for (size_t k = 1; k < s->streams.size(); ++k) (void)hipStreamDestroy(s->streams[k]);
  if (s->batch) (void)tsdf_batch_destroy(s->batch);
  if (s->region) (void)tsdf_region_destroy(s->region);
  if (s->ctr_host) (void)hipHostFree(s->ctr_host);
  if (s->status_host) (void)hipHostFree(s->status_host);
  delete s;
}

}  // namespace

extern "C" {

size_t tsdf_server_workspace_bytes(const tsdf_server_params* params) {
  if (!valid_params(params)) return 0;
  return tsdf_batch_workspace_bytes(params->max_batch);
}

tsdf_status tsdf_server_create(const tsdf_server_params* params, void* workspace_dev,
                               size_t workspace_bytes, void* session_region_dev,
                               uint64_t budget_bytes, void* hip_stream, tsdf_server** out) {
  if (!out) return TSDF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!valid_params(params) || !workspace_dev || !session_region_dev || budget_bytes == 0)
    return TSDF_ERR_INVALID_ARGUMENT;
  if (workspace_bytes < tsdf_server_workspace_bytes(params)) return TSDF_ERR_BUFFER_TOO_SMALL;
  tsdf_server* s = new (std::nothrow) tsdf_server();
  if (!s) return TSDF_ERR_INTERNAL;
  s->p = *params;
  s->stream = as_stream(hip_stream);
  s->streams.push_back(s->stream);
  tsdf_status st = TSDF_OK;
  for (uint32_t k = 1; k < params->max_inflight && st == TSDF_OK; ++k) {
    hipStream_t extra = nullptr;
    st = hip_status(hipStreamCreateWithFlags(&extra, hipStreamNonBlocking));
    if (st == TSDF_OK) s->streams.push_back(extra);
  }
  s->stream_busy.assign(s->streams.size(), false);
  if (st == TSDF_OK) st = hip_status(hipEventCreateWithFlags(&s->opened, hipEventDisableTiming));
  if (st == TSDF_OK) st = tsdf_region_create(session_region_dev, budget_bytes, &s->region);
  if (st == TSDF_OK)
    st = tsdf_batch_create(params->max_batch, workspace_dev, workspace_bytes, &s->batch);
  const size_t n = params->max_sessions;
  if (st == TSDF_OK)
    st = hip_status(hipHostMalloc(reinterpret_cast<void**>(&s->ctr_host), n * sizeof(void*),
                                  hipHostMallocMapped));
  if (st == TSDF_OK)
    st = hip_status(hipHostMalloc(reinterpret_cast<void**>(&s->status_host),
                                  n * s->streams.size() * sizeof(unsigned), hipHostMallocMapped));
  if (st == TSDF_OK)
    st = hip_status(hipHostGetDevicePointer(reinterpret_cast<void**>(&s->ctr_dev), s->ctr_host, 0));
  if (st == TSDF_OK)
    st = hip_status(
        hipHostGetDevicePointer(reinterpret_cast<void**>(&s->status_dev), s->status_host, 0));
  if (st != TSDF_OK) {
    free_server(s);
    return st;
  }
  for (size_t i = 0; i < n; ++i) s->ctr_host[i] = nullptr;
  for (size_t i = 0; i < n * s->streams.size(); ++i) s->status_host[i] = 0;
  s->sessions.resize(n);
  s->items.reserve(params->max_batch);
  *out = s;
  return TSDF_OK;
}

tsdf_status tsdf_server_destroy(tsdf_server* server) {
  if (!server) return TSDF_ERR_INVALID_ARGUMENT;
  free_server(server);
  return TSDF_OK;
}

tsdf_status tsdf_server_open(tsdf_server* s, const tsdf_volume_params* params,
                             uint32_t* session_out) {
  if (!s || !session_out) return TSDF_ERR_INVALID_ARGUMENT;
  const size_t bytes = tsdf_volume_bytes(params);
  if (bytes == 0 || (params->flags & TSDF_VOLUME_COLOUR)) return TSDF_ERR_INVALID_ARGUMENT;
  uint32_t id = 0;
  while (id < s->p.max_sessions && s->sessions[id].open) ++id;
  if (id == s->p.max_sessions) return TSDF_ERR_BUDGET;
  void* arena = nullptr;
  tsdf_status st = tsdf_region_alloc(s->region, bytes, &arena);
  if (st != TSDF_OK) return st;
  tsdf_volume* vol = nullptr;
  st = tsdf_create_volume(params, arena, bytes, s->stream, &vol);
  // the other streams reach the volume only after its initialisation
  if (st == TSDF_OK) st = hip_status(hipEventRecord(s->opened, s->stream));
  for (size_t k = 1; k < s->streams.size() && st == TSDF_OK; ++k)
    st = hip_status(hipStreamWaitEvent(s->streams[k], s->opened, 0));
  if (st != TSDF_OK) {
    if (vol) (void)tsdf_destroy_volume(vol);
    (void)tsdf_region_free(s->region, arena);
    return st;
  }
  Session& ss = s->sessions[id];
  ss = Session();
  ss.open = true;
  ss.vol = vol;
  ss.arena = arena;
  ss.opened_at = s->next_seq;
  s->ctr_host[id] = vol->dev.ctr;
  ++s->n_open;
  *session_out = id;
  return TSDF_OK;
}

tsdf_status tsdf_server_close(tsdf_server* s, uint32_t session) {
  if (!s || session >= s->p.max_sessions || !s->sessions[session].open)
    return TSDF_ERR_INVALID_ARGUMENT;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (it->session == session) {
      s->done.emplace_back(it->tag, (int32_t)TSDF_ERR_INVALID_ARGUMENT);
      it = s->queue.erase(it);
    } else {
      ++it;
    }
  }
  if (s->sessions[session].inflight > 0) {
    const tsdf_status st = retire(s, true);
    if (st != TSDF_OK) return st;
  }
  release_session(s, session);
  return TSDF_OK;
}

tsdf_status tsdf_server_submit(tsdf_server* s, uint32_t session, const float* depth_dev,
                               const tsdf_camera* camera, uint64_t tag) {
  if (!s || session >= s->p.max_sessions || !s->sessions[session].open ||
      !valid_camera(camera))
    return TSDF_ERR_INVALID_ARGUMENT;
  if ((uint64_t)camera->width * camera->height > 0 && !depth_dev) return TSDF_ERR_INVALID_ARGUMENT;
  if (s->sessions[session].failure != TSDF_OK) return (tsdf_status)s->sessions[session].failure;
  if (s->queue.size() >= s->p.max_queue) return TSDF_ERR_BUDGET;
  s->queue.push_back(Pending{session, depth_dev, *camera, tag});
  return TSDF_OK;
}

tsdf_status tsdf_server_step(tsdf_server* s, uint32_t* launched) {
  if (!s) return TSDF_ERR_INVALID_ARGUMENT;
  if (launched) *launched = 0;
  tsdf_status st = retire(s, false);
  if (st != TSDF_OK) return st;
  if (s->running < s->p.max_inflight && !s->queue.empty()) st = launch_one(s, launched);
  return st;
}

tsdf_status tsdf_server_completions(tsdf_server* s, uint64_t* tags, int32_t* statuses,
                                    uint32_t max, uint32_t* n_out) {
  if (!s || !n_out) return TSDF_ERR_INVALID_ARGUMENT;
  uint32_t n = 0;
  while (n < max && !s->done.empty()) {
    if (tags) tags[n] = s->done.front().first;
    if (statuses) statuses[n] = s->done.front().second;
    s->done.pop_front();
    ++n;
  }
  *n_out = n;
  return TSDF_OK;
}

tsdf_status tsdf_server_session(tsdf_server* s, uint32_t session, tsdf_volume** volume,
                                int32_t* failure) {
  if (!s || session >= s->p.max_sessions || !s->sessions[session].open)
    return TSDF_ERR_INVALID_ARGUMENT;
  if (volume) *volume = s->sessions[session].vol;
  if (failure) *failure = s->sessions[session].failure;
  return TSDF_OK;
}

tsdf_status tsdf_server_batch(tsdf_server* s, tsdf_batch** out) {
  if (!s || !out) return TSDF_ERR_INVALID_ARGUMENT;
  *out = s->batch;
  return TSDF_OK;
}

tsdf_status tsdf_server_load(tsdf_server* s, uint32_t* queued, uint32_t* inflight_frames,
                             uint32_t* inflight_launches, uint32_t* sessions,
                             uint64_t* budget_used) {
  if (!s) return TSDF_ERR_INVALID_ARGUMENT;
  if (queued) *queued = (uint32_t)s->queue.size();
  if (inflight_frames) *inflight_frames = s->inflight_frames;
  if (inflight_launches) *inflight_launches = s->running;
  if (sessions) *sessions = s->n_open;
  if (budget_used) return tsdf_region_usage(s->region, nullptr, budget_used, nullptr, nullptr);
  return TSDF_OK;
}

tsdf_status tsdf_server_replay(tsdf_server* s, const tsdf_request* reqs, uint32_t n,
                               uint32_t mode, double* latency_ns, double* elapsed_ns) {
  if (!s || (n > 0 && (!reqs || !latency_ns)) || mode > TSDF_REPLAY_PLAIN)
    return TSDF_ERR_INVALID_ARGUMENT;
  for (uint32_t i = 0; i < n; ++i) {
    if (i > 0 && reqs[i].arrival_ns < reqs[i - 1].arrival_ns) return TSDF_ERR_INVALID_ARGUMENT;
    if (reqs[i].session >= s->p.max_sessions || !s->sessions[reqs[i].session].open)
      return TSDF_ERR_INVALID_ARGUMENT;
    if (!valid_camera(&reqs[i].camera)) return TSDF_ERR_INVALID_ARGUMENT;
  }
  // the replay owns the server while it runs: nothing may be queued or
  // waiting to be collected; launches still finishing are waited for
  if (!s->queue.empty() || s->running > 0 || !s->done.empty()) return TSDF_ERR_INVALID_ARGUMENT;
  const tsdf_status pre = retire(s, true);
  if (pre != TSDF_OK) return pre;
  for (uint32_t i = 0; i < n; ++i) latency_ns[i] = -1.0;
  const double t0 = now_ns();
  double last = t0;
  uint32_t next = 0, finished = 0;
  if (mode == TSDF_REPLAY_SERVED) {
    uint64_t tags[256];
    int32_t sts[256];
    while (finished < n) {
      double t = now_ns();
      while (next < n && (double)reqs[next].arrival_ns <= t - t0) {
        const tsdf_request& r = reqs[next];
        const tsdf_status st = tsdf_server_submit(s, r.session, r.depth_dev, &r.camera, next);
        if (st == TSDF_ERR_BUDGET) break;  // queue full: try again after a launch
        if (st != TSDF_OK) ++finished;     // refused: latency stays -1
        ++next;
      }
      tsdf_status st = tsdf_server_step(s, nullptr);
      if (st != TSDF_OK) return st;
      uint32_t k = 0;
      tsdf_server_completions(s, tags, sts, 256, &k);
      if (k) {
        t = now_ns();
        for (uint32_t j = 0; j < k; ++j) {
          if (sts[j] == TSDF_OK) latency_ns[tags[j]] = t - t0 - (double)reqs[tags[j]].arrival_ns;
          ++finished;
        }
        last = t;
      }
    }
  } else {
    std::deque<std::pair<uint32_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> spare;
    tsdf_status result = TSDF_OK;
    while (finished < n && result == TSDF_OK) {
      double t = now_ns();
      while (next < n && (double)reqs[next].arrival_ns <= t - t0) {
        const tsdf_request& r = reqs[next];
        hipEvent_t ev;
        if (!spare.empty()) {
          ev = spare.back();
          spare.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
          result = TSDF_ERR_HIP;
          break;
        }
        tsdf_status st = tsdf_fuse_frame(s->sessions[r.session].vol, r.depth_dev, &r.camera,
                                         s->stream);
        if (st == TSDF_OK) st = hip_status(hipEventRecord(ev, s->stream));
        if (st != TSDF_OK) {
          spare.push_back(ev);
          result = st;
          break;
        }
        pending.emplace_back(next, ev);
        ++next;
      }
      while (!pending.empty()) {
        const hipError_t e = hipEventQuery(pending.front().second);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) {
          result = TSDF_ERR_HIP;
          break;
        }
        t = now_ns();
        const uint32_t i = pending.front().first;
        latency_ns[i] = t - t0 - (double)reqs[i].arrival_ns;
        spare.push_back(pending.front().second);
        pending.pop_front();
        ++finished;
        last = t;
      }
    }
    (void)hipStreamSynchronize(s->stream);
    for (auto& pe : pending) spare.push_back(pe.second);
    for (hipEvent_t ev : spare) (void)hipEventDestroy(ev);
    if (result != TSDF_OK) return result;
  }
  if (elapsed_ns) *elapsed_ns = last - t0;
  return TSDF_OK;
}

}  // extern "C"
