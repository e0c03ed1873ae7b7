// Serving form: many model-building sessions share one device arena and a few
// streams.  Client threads submit node creation, Connect, Calibrate and Close
// requests; one scheduler thread admits them in arrival order (each session's
// requests in its own order) as memory in the shared arena allows, packs the
// admitted Connect calls of all sessions on a stream into a single generation
// launch, and runs calibrations on their sessions' streams, so the work of
// different sessions overlaps on the device.  Every request carries its
// arrival, admission and completion times (host steady clock).
//
// Locking: the API side (submit, open, wait, stats) touches only the shared
// part of the server under `mu` for a few instructions.  The scheduler takes
// the new submissions at the start of a round, does all device work on
// private state without the lock, and publishes the requests it finished
// (and its counters) under the lock at the end of the round, so a client is
// never held up by the scheduler's device calls.
//
// Arithmetic is unchanged: a session's result equals the same calls issued on
// a context of its own (same seed, same call order).
#include <sys/prctl.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <thread>
#include <unordered_map>

#include "ng_rt.h"

using namespace ngrt;

namespace {

int64_t now_ns(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
}

// An event shared by every request finished by the same launch.
struct EventBox {
  hipEvent_t ev = nullptr;
  ~EventBox() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

enum ReqKind { REQ_CREATE_NODES = 0, REQ_CONNECT = 1, REQ_CALIBRATE = 2, REQ_CLOSE = 3 };

struct Request {
  uint64_t ticket = 0;
  ng_session* sess = nullptr;
  int kind = REQ_CONNECT;
  uint32_t n_nodes = 0;
  ng_range src{}, tgt{};
  ng_conn_spec conn{};
  ng_syn_spec syn{};
  int64_t arrival_ns = 0, admit_ns = 0, done_ns = 0;
  int32_t status = NG_OK;
  uint64_t n_conns = 0;
  std::string msg;
  bool done = false;
};

// Pinned upload region for one packed launch; reusable once its copy ran.
// Each stream starts with kStagesPerStream of kStageBytes, allocated with the
// server: pinning host memory takes far longer than a launch, so a burst of
// launches must not pay for it.
constexpr int kStagesPerStream = 16;
constexpr uint64_t kStageBytes = 64 << 10;
struct Stage {
  char* p = nullptr;
  uint64_t cap = 0;
  std::shared_ptr<EventBox> busy;  // event after the upload that reads it
};

}  // namespace

struct ng_session {
  ng_server* server = nullptr;
  ng_ctx* ctx = nullptr;
  int stream = 0;
  uint32_t client_nodes = 0;   // node count as the client sees it (ranges returned at submit)
  std::deque<Request*> queue;  // scheduler: taken over, not yet admitted, in order
  bool close_submitted = false;  // under mu
  uint32_t pending = 0;          // under mu: submitted and not yet finished
  uint64_t blocked_round = 0;    // scheduler: head request must wait in this round
  uint64_t base_held = 0;      // arena bytes of an empty session (tables)
};

struct ng_server {
  ng_server_config cfg{};
  int log2B = 24;
  Arena arena;  // thread-safe on its own
  std::vector<hipStream_t> streams;
  std::vector<std::vector<Stage>> stages;
  int device = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  // shared with the API side, under mu
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread thr;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t next_stream = 0;                       // sessions are spread over the streams in turn
  std::vector<Request*> incoming;                 // submitted, not yet taken by the scheduler
  std::vector<ng_session*> new_sessions;          // opened, not yet taken by the scheduler
  std::unordered_map<uint64_t, Request*> tickets;  // not yet collected by ng_wait
  ng_server_stats stats{};

  // scheduler thread only
  std::vector<ng_session*> sessions;  // open sessions
  std::deque<Request*> arrivals;      // global arrival order, not yet admitted
  // launched requests, per stream in launch order: the events of a stream
  // complete in order, so only the oldest group of each is queried
  struct Group {
    std::shared_ptr<EventBox> ev;
    std::vector<Request*> reqs;
  };
  std::vector<std::deque<Group>> inflight;
  size_t n_inflight = 0;
  uint64_t round = 0;                 // scheduling rounds (blocked-session marks)
  std::vector<Request*> finished;     // finished this round, published under mu
  std::vector<ng_session*> closed;    // deleted once all their requests are published
  ng_server_stats sched{};            // scheduler-owned counters

  void run();
  // Record a request's result; it becomes visible to ng_wait when published.
  void finish(Request* r, int32_t status, const std::string& msg = "");
  // Under mu: make this round's finished requests and counters visible.
  void publish();
  // Copy host bytes to device memory on stream k through the stream's pinned
  // stages (allocated once, reused once their last copy ran; the scheduler
  // never frees pinned memory, which would wait for the whole device).
  // A second piece (src2, n2 bytes) may follow at offset off2 of the same
  // copy.
  int upload(int k, void* d, const void* src, uint64_t nb, const void* src2 = nullptr, uint64_t off2 = 0,
             uint64_t n2 = 0);
  // Calibrate the collected requests' sessions together (one packed
  // calibration); if that fails, one by one, where a request that does not
  // fit stays queued (and joins oom_wait) unless hopeless(session).
  // Admitted requests leave the queues.  Returns whether any was admitted.
  bool run_calibrations(const std::vector<Request*>& batch, const std::function<bool(ng_session*)>& hopeless,
                        std::vector<Request*>& oom_wait);
  void admit_calibration(Request* r);
  // r is its session's head request: remove it from the queues
  void dequeue(Request* r);
};

void ng_server::dequeue(Request* r) {
  r->sess->queue.pop_front();
  arrivals.erase(std::find(arrivals.begin(), arrivals.end(), r));
}

void ng_server::admit_calibration(Request* r) {
  ng_ctx* c = r->sess->ctx;
  r->admit_ns = now_ns(t0);
  r->n_conns = c->n_conns;
  dequeue(r);
  auto box = std::make_shared<EventBox>();
  if (hipEventCreateWithFlags(&box->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(box->ev, streams[r->sess->stream]) != hipSuccess) {
    finish(r, NG_ERR_DEVICE, "event");
    return;
  }
  inflight[r->sess->stream].push_back({box, {r}});
  n_inflight++;
  sched.calibrations++;
}

bool ng_server::run_calibrations(const std::vector<Request*>& batch,
                                 const std::function<bool(ng_session*)>& hopeless,
                                 std::vector<Request*>& oom_wait) {
  // every session's pending connects were flushed to its stream before this
  if (batch.size() > 1) {
    std::vector<ng_ctx*> ctxs;
    for (Request* r : batch) ctxs.push_back(r->sess->ctx);
    const Uploader up = [&](hipStream_t st, void* d, const void* src, uint64_t nb) {
      for (size_t k = 0; k < streams.size(); ++k)
        if (streams[k] == st) return upload((int)k, d, src, nb);
      return (int)NG_ERR_STATE;
    };
    if (calibrate_many(ctxs.data(), (uint32_t)ctxs.size(), &up) == NG_OK) {
      sched.calibrate_packs++;
      if (batch.size() > sched.max_sessions_per_pack) sched.max_sessions_per_pack = batch.size();
      for (Request* r : batch) admit_calibration(r);
      return true;
    }
  }
  bool any = false;
  for (Request* r : batch) {
    const int rc = ng_calibrate(r->sess->ctx);
    if (rc == NG_ERR_OOM && !hopeless(r->sess)) {  // waits for memory
      oom_wait.push_back(r);
      continue;
    }
    any = true;
    if (rc != NG_OK) {
      r->admit_ns = now_ns(t0);
      dequeue(r);
      finish(r, rc, ng_last_error());
      continue;
    }
    admit_calibration(r);
  }
  return any;
}

void ng_server::finish(Request* r, int32_t status, const std::string& msg) {
  r->status = status;
  r->msg = msg;
  r->done_ns = now_ns(t0);
  finished.push_back(r);
}

void ng_server::publish() {
  for (Request* r : finished) {
    r->sess->pending--;
    r->done = true;  // from here on ng_wait may delete r
  }
  const bool any = !finished.empty();
  finished.clear();
  for (size_t i = 0; i < closed.size();) {
    if (closed[i]->pending == 0) {
      delete closed[i];
      closed[i] = closed.back();
      closed.pop_back();
    } else {
      ++i;
    }
  }
  stats.launches = sched.launches;
  stats.packed_calls = sched.packed_calls;
  stats.max_calls_per_launch = sched.max_calls_per_launch;
  stats.calibrations = sched.calibrations;
  stats.peak_arena_bytes = sched.peak_arena_bytes;
  stats.calibrate_packs = sched.calibrate_packs;
  stats.max_sessions_per_pack = sched.max_sessions_per_pack;
  stats.scheduler_busy_ns = sched.scheduler_busy_ns;
  stats.host_launch_ns = sched.host_launch_ns;
  stats.host_calibrate_ns = sched.host_calibrate_ns;
  if (any) cv_done.notify_all();
}

// Copy descriptors to the device through a pinned stage of stream k.
int ng_server::upload(int k, void* d, const void* src, uint64_t nb, const void* src2, uint64_t off2, uint64_t n2) {
  const uint64_t total = src2 ? off2 + n2 : nb;
  Stage* st = nullptr;
  for (auto& s : stages[k])
    if (s.cap >= total && (!s.busy || hipEventQuery(s.busy->ev) == hipSuccess)) {
      st = &s;
      break;
    }
  if (!st) {
    Stage s;
    s.cap = std::max<uint64_t>(total, kStageBytes);
    if (hipHostMalloc((void**)&s.p, s.cap, hipHostMallocDefault) != hipSuccess) return NG_ERR_DEVICE;
    stages[k].push_back(s);
    st = &stages[k].back();
  }
  memcpy(st->p, src, nb);
  if (src2) memcpy(st->p + off2, src2, n2);
  if (hipMemcpyAsync(d, st->p, total, hipMemcpyHostToDevice, streams[k]) != hipSuccess) return NG_ERR_DEVICE;
  auto box = std::make_shared<EventBox>();
  if (hipEventCreateWithFlags(&box->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(box->ev, streams[k]) != hipSuccess)
    return NG_ERR_DEVICE;
  st->busy = box;
  return NG_OK;
}

void ng_server::run() {
  (void)hipSetDevice(device);
  // The completion poll below sleeps 10 us at a time; with the default 50 us
  // timer slack of a thread each of those sleeps would last about 60 us and
  // add that much to a request's latency.
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  const int ns = (int)streams.size();
  bool progress = true;
  for (;;) {
    bool stopping;
    {
      std::unique_lock<std::mutex> lk(mu);
      publish();
      // Sleep until something can change: new requests, or (polling every
      // 10 us) device work or memory releases still pending.
      auto news = [&] { return stop || !incoming.empty() || !new_sessions.empty(); };
      const bool pending = n_inflight != 0 || arena.deferred_bytes() != 0;
      if (!pending && !progress)
        cv_work.wait(lk, news);
      else if (pending)
        cv_work.wait_for(lk, std::chrono::microseconds(10), news);
      for (ng_session* ss : new_sessions) sessions.push_back(ss);
      new_sessions.clear();
      for (Request* r : incoming) {
        arrivals.push_back(r);
        r->sess->queue.push_back(r);
      }
      incoming.clear();
      stopping = stop;
    }
    if (stopping && arrivals.empty() && n_inflight == 0) break;
    const auto busy0 = std::chrono::steady_clock::now();
    ++round;

    // completions
    size_t completed = 0;
    for (auto& q : inflight) {
      while (!q.empty() && hipEventQuery(q.front().ev->ev) == hipSuccess) {
        for (Request* r : q.front().reqs) finish(r, NG_OK);
        completed += q.front().reqs.size();
        q.pop_front();
      }
    }
    n_inflight -= completed;

    // admission, in arrival order; a session whose head request must wait
    // blocks its later requests (per-session order is kept)
    std::vector<std::vector<ng::GenDesc>> descs(ns);
    std::vector<std::vector<Request*>> packed(ns);
    auto is_blocked = [&](ng_session* s) { return s->blocked_round == round; };
    auto flush = [&](int k) {
      if (descs[k].empty()) return;
      const auto f0 = std::chrono::steady_clock::now();
      uint64_t groups = 0;
      for (auto& d : descs[k]) {
        d.group0 = groups;
        groups += ((uint64_t)d.n_new + 3) / 4;
      }
      int rc = check_descs(descs[k]);
      // The sessions' new block-table entries are written by one launch; they
      // travel in the same upload as the descriptors, behind them (or, without
      // arena room for both, each context writes its own).
      std::vector<ng::TabEntry> entries;
      std::vector<std::pair<ng_ctx*, uint32_t>> synced;
      for (Request* r : packed[k]) {
        ng_ctx* c = r->sess->ctx;
        if (c->tab_synced < c->blocks.size()) {
          synced.emplace_back(c, c->tab_synced);
          take_table_entries(c, entries);
        }
      }
      auto unsync = [&] {  // the entries were not written
        for (auto& cs : synced) cs.first->tab_synced = cs.second;
        synced.clear();
        entries.clear();
      };
      const uint64_t nd = descs[k].size() * sizeof(ng::GenDesc);
      const uint64_t eoff = (nd + 255) / 256 * 256;
      uint64_t nb = entries.empty() ? nd : eoff + entries.size() * sizeof(ng::TabEntry);
      char* d = nullptr;
      hipError_t e = hipSuccess;
      if (rc == NG_OK) {
        d = arena.alloc(nb);
        if (!d && !entries.empty()) {
          unsync();
          for (auto& cs : synced)
            if (rc == NG_OK) rc = sync_table(cs.first);
          nb = nd;
          if (rc == NG_OK) d = arena.alloc(nb);
        }
        if (rc == NG_OK && !d) rc = NG_ERR_OOM;
      }
      if (rc == NG_OK) {
        rc = entries.empty() ? upload(k, d, descs[k].data(), nd)
                             : upload(k, d, descs[k].data(), nd, entries.data(), eoff,
                                      entries.size() * sizeof(ng::TabEntry));
        if (rc != NG_OK) {
          arena.release(d, nb);
          d = nullptr;
        }
      }
      if (rc != NG_OK) unsync();
      if (rc == NG_OK && !entries.empty())
        e = ng::launch_set_entries((const ng::TabEntry*)(d + eoff), (uint32_t)entries.size(), streams[k]);
      ng::GenDesc* d_descs = (ng::GenDesc*)d;
      std::shared_ptr<EventBox> box;
      if (rc == NG_OK && e == hipSuccess) {
        e = ng::launch_generate_batch(d_descs, (uint32_t)descs[k].size(), groups, log2B, streams[k]);
        box = std::make_shared<EventBox>();
        if (e == hipSuccess) e = hipEventCreateWithFlags(&box->ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(box->ev, streams[k]);
        sched.launches++;
        sched.packed_calls += descs[k].size();
        if (descs[k].size() > sched.max_calls_per_launch) sched.max_calls_per_launch = descs[k].size();
      }
      if (d) {  // descriptors and entries return to the arena after the launches
        hipEvent_t fe = nullptr;
        if (hipEventCreateWithFlags(&fe, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(fe, streams[k]) == hipSuccess) {
          Arena::Ranges rs;
          rs.emplace_back(d, nb);
          arena.release_after(streams[k], std::move(rs), fe);
        } else {
          if (fe) (void)hipEventDestroy(fe);
          (void)hipStreamSynchronize(streams[k]);
          arena.release(d, nb);
        }
      }
      if (rc != NG_OK || e != hipSuccess) {
        for (Request* r : packed[k]) finish(r, NG_ERR_DEVICE, "packed generation launch failed");
      } else {
        inflight[k].push_back({box, packed[k]});
        n_inflight += packed[k].size();
      }
      descs[k].clear();
      packed[k].clear();
      sched.host_launch_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                                  std::chrono::steady_clock::now() - f0).count();
    };
    // A request that does not fit waits for memory to come back (another
    // session's release or close).  It fails at once if it would not fit even
    // with every other session gone (hopeless).  If no request can move and
    // every session that could give memory back is itself waiting on the
    // server (a deadlock), the latest such request fails; see below.
    bool admitted_any = false;
    std::vector<Request*> oom_wait;
    auto hopeless = [&](ng_session* me) {
      return me->ctx->need > arena.size() - std::min(arena.size(), me->ctx->held);
    };
    std::vector<Request*> cal_batch;
    for (auto it = arrivals.begin(); it != arrivals.end();) {
      Request* r = *it;
      ng_session* s = r->sess;
      if (is_blocked(s) || s->queue.empty() || s->queue.front() != r) {
        ++it;
        continue;
      }
      ng_ctx* c = s->ctx;
      const int k = s->stream;
      bool admitted = true;
      switch (r->kind) {
        case REQ_CREATE_NODES: {
          ng_range out;
          const int rc = ng_create_nodes(c, r->n_nodes, &out);
          r->admit_ns = now_ns(t0);
          finish(r, rc, rc ? ng_last_error() : "");
          break;
        }
        case REQ_CONNECT: {
          ng::GenDesc d;
          uint64_t n = 0;
          const int rc = connect_prepare(c, r->src, r->tgt, &r->conn, &r->syn, &d, &n);
          if (rc == NG_ERR_OOM && !hopeless(s)) {
            admitted = false;  // wait for memory to come back
            oom_wait.push_back(r);
            break;
          }
          r->admit_ns = now_ns(t0);
          if (rc != NG_OK) {
            finish(r, rc, ng_last_error());
            break;
          }
          connect_commit(c, d, d.max_delay);
          r->n_conns = n;
          if (n == 0) {
            finish(r, NG_OK);
          } else {
            descs[k].push_back(d);
            packed[k].push_back(r);
          }
          break;
        }
        case REQ_CALIBRATE:
          // collected: the calibrations of this round run together below; the
          // session's later requests wait for the next round
          cal_batch.push_back(r);
          admitted = false;
          break;
        case REQ_CLOSE: {
          flush(k);
          r->admit_ns = now_ns(t0);
          ctx_destroy_release(c);  // frees wait for the stream's pending work
          s->ctx = nullptr;
          finish(r, NG_OK);
          break;
        }
      }
      if (!admitted) {
        s->blocked_round = round;
        ++it;
        continue;
      }
      admitted_any = true;
      s->queue.pop_front();
      it = arrivals.erase(it);
      if (r->kind == REQ_CLOSE) {
        sessions.erase(std::find(sessions.begin(), sessions.end(), s));
        closed.push_back(s);  // deleted once its requests are published
      }
    }
    for (int k = 0; k < ns; ++k) flush(k);
    if (!cal_batch.empty()) {
      const auto c0 = std::chrono::steady_clock::now();
      if (run_calibrations(cal_batch, hopeless, oom_wait)) admitted_any = true;
      sched.host_calibrate_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now() - c0).count();
    }
    if (!oom_wait.empty() && !admitted_any && n_inflight == 0 && arena.deferred_bytes() == 0) {
      // Nothing runs and nothing is pending release.  Memory can still come
      // back from a session that holds connections and has no request queued
      // (its client may close it); if there is none, break the deadlock by
      // failing the latest waiting request.
      bool can_wait = false;
      for (ng_session* o : sessions)
        if (o->ctx && o->ctx->held > o->base_held && o->queue.empty()) can_wait = true;
      if (!can_wait) {
        Request* victim = oom_wait[0];
        for (Request* r : oom_wait)
          if (r->ticket > victim->ticket) victim = r;
        victim->admit_ns = now_ns(t0);
        dequeue(victim);
        finish(victim, NG_ERR_OOM, "arena exhausted: every session holding memory waits for more");
        admitted_any = true;
      }
    }
    progress = admitted_any || completed != 0;
    if (stopping && !progress && n_inflight == 0 && arena.deferred_bytes() == 0) {
      // shutting down with requests that can never be admitted
      for (Request* r : arrivals) {
        r->admit_ns = now_ns(t0);
        finish(r, NG_ERR_STATE, "server shut down before the request could run");
        if (r->sess) r->sess->queue.clear();
      }
      arrivals.clear();
      break;
    }
    const uint64_t used = arena.used();
    if (used > sched.peak_arena_bytes) sched.peak_arena_bytes = used;
    sched.scheduler_busy_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                                   std::chrono::steady_clock::now() - busy0).count();
  }
  std::lock_guard<std::mutex> lk(mu);
  publish();
}

extern "C" {

int ng_server_create(const ng_server_config* cfg, void* arena, uint64_t arena_bytes, void* const* streams,
                     int n_streams, ng_server** out) {
  if (!cfg || !out || !arena || n_streams < 1 || n_streams > 64 || !streams)
    return fail(NG_ERR_INVALID_ARG, "bad server arguments");
  if ((uintptr_t)arena % kAlign) return fail(NG_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  for (int i = 0; i < n_streams; ++i)
    if (!streams[i]) return fail(NG_ERR_INVALID_ARG, "server streams must not be the null stream");
  ng_server* s = new ng_server();
  s->cfg = *cfg;
  s->arena.init((char*)arena, arena_bytes);
  for (int i = 0; i < n_streams; ++i) s->streams.push_back((hipStream_t)streams[i]);
  s->stages.resize(n_streams);
  s->inflight.resize(n_streams);
  for (auto& v : s->stages)
    for (int i = 0; i < kStagesPerStream; ++i) {
      Stage st;
      st.cap = kStageBytes;
      if (hipHostMalloc((void**)&st.p, st.cap, hipHostMallocDefault) != hipSuccess) {
        for (auto& w : s->stages)
          for (auto& x : w) (void)hipHostFree(x.p);
        delete s;
        return fail(NG_ERR_DEVICE, "hipHostMalloc of the upload stages failed");
      }
      v.push_back(st);
    }
  const uint64_t B = cfg->block_size ? cfg->block_size : (1ull << 24);
  if (B & (B - 1) || B < (1ull << 16) || B > (1ull << 30)) {
    delete s;
    return fail(NG_ERR_INVALID_ARG, "block_size must be a power of two in [2^16, 2^30]");
  }
  s->log2B = bitwidth(B) - 1;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(NG_ERR_DEVICE, "no HIP device");
  }
  s->thr = std::thread([s] { s->run(); });
  *out = s;
  return NG_OK;
}

int ng_server_destroy(ng_server* s) {
  if (!s) return NG_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->thr.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (auto* list : {&s->sessions, &s->new_sessions}) {  // sessions never closed
    for (ng_session* ss : *list) {
      ctx_destroy_release(ss->ctx);
      delete ss;
    }
  }
  for (ng_session* ss : s->closed) delete ss;
  for (auto& kv : s->tickets) delete kv.second;
  for (auto& v : s->stages)
    for (auto& st : v) (void)hipHostFree(st.p);
  delete s;
  return NG_OK;
}

int ng_session_open(ng_server* s, uint64_t seed, ng_session** out) {
  if (!s || !out) return fail(NG_ERR_INVALID_ARG, "null argument");
  ng_config cfg{};
  cfg.block_size = s->cfg.block_size;
  cfg.seed = seed;
  cfg.h_ms = s->cfg.h_ms;
  int k = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    k = (int)(s->next_stream++ % s->streams.size());
  }
  // The context is made without the server's lock (its events, tables in the
  // shared arena, which locks itself, and two small launches on stream k), so
  // the scheduler is not held up; the scheduler first sees the session when
  // it is registered below.
  ng_ctx* c = nullptr;
  if (int rc = ctx_create_shared(&cfg, &s->arena, s->streams[k], &c)) return rc;
  if (s->cfg.radix_bits)
    (void)ng_set_tuning(c, s->cfg.radix_bits, s->cfg.sort_ranges ? s->cfg.sort_ranges : 1024);
  ng_session* ss = new ng_session();
  ss->server = s;
  ss->ctx = c;
  ss->base_held = c->held;
  ss->stream = k;
  std::lock_guard<std::mutex> lk(s->mu);
  s->new_sessions.push_back(ss);
  s->stats.sessions_opened++;
  *out = ss;
  return NG_OK;
}

static int submit(ng_session* ss, Request* r, uint64_t* ticket) {
  ng_server* s = ss->server;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (ss->close_submitted) {
      delete r;
      return fail(NG_ERR_STATE, "session is closing");
    }
    r->ticket = s->next_ticket++;
    r->sess = ss;
    r->arrival_ns = now_ns(s->t0);
    if (r->kind == REQ_CLOSE) ss->close_submitted = true;
    s->incoming.push_back(r);
    s->tickets[r->ticket] = r;
    s->stats.submitted++;
    ss->pending++;
    if (ticket) *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return NG_OK;
}

int ng_submit_create_nodes(ng_session* ss, uint32_t n, ng_range* out, uint64_t* ticket) {
  if (!ss) return fail(NG_ERR_INVALID_ARG, "null session");
  Request* r = new Request();
  r->kind = REQ_CREATE_NODES;
  r->n_nodes = n;
  {
    std::lock_guard<std::mutex> lk(ss->server->mu);
    if ((uint64_t)ss->client_nodes + n > 0xFFFFFFFFull) {
      delete r;
      return fail(NG_ERR_TOO_LARGE, "too many nodes");
    }
    if (out) *out = ng_range{ss->client_nodes, n};
    ss->client_nodes += n;
  }
  return submit(ss, r, ticket);
}

int ng_submit_connect(ng_session* ss, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                      const ng_syn_spec* syn, uint64_t* ticket) {
  if (!ss || !conn || !syn) return fail(NG_ERR_INVALID_ARG, "null argument");
  Request* r = new Request();
  r->kind = REQ_CONNECT;
  r->src = src;
  r->tgt = tgt;
  r->conn = *conn;
  r->syn = *syn;
  return submit(ss, r, ticket);
}

int ng_submit_calibrate(ng_session* ss, uint64_t* ticket) {
  if (!ss) return fail(NG_ERR_INVALID_ARG, "null session");
  Request* r = new Request();
  r->kind = REQ_CALIBRATE;
  return submit(ss, r, ticket);
}

int ng_submit_close(ng_session* ss, uint64_t* ticket) {
  if (!ss) return fail(NG_ERR_INVALID_ARG, "null session");
  Request* r = new Request();
  r->kind = REQ_CLOSE;
  return submit(ss, r, ticket);
}

int ng_session_close(ng_session* ss) {
  if (!ss) return fail(NG_ERR_INVALID_ARG, "null session");
  ng_server* srv = ss->server;
  uint64_t t = 0;
  if (int rc = ng_submit_close(ss, &t)) return rc;
  ng_ticket_info info{};
  if (int rc = ng_wait(srv, t, -1, &info)) return rc;
  return info.status;
}

int ng_wait(ng_server* s, uint64_t ticket, int64_t timeout_ns, ng_ticket_info* out) {
  if (!s) return fail(NG_ERR_INVALID_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(NG_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  Request* r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_ns < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), pred)) {
    return fail(NG_ERR_STATE, "ticket %llu not finished yet", (unsigned long long)ticket);
  }
  if (out) {
    memset(out, 0, sizeof *out);
    out->status = r->status;
    out->kind = r->kind;
    out->n_conns = r->n_conns;
    out->arrival_ns = r->arrival_ns;
    out->admit_ns = r->admit_ns;
    out->done_ns = r->done_ns;
  }
  if (r->status != NG_OK) fail(r->status, "%s", r->msg.c_str());
  s->tickets.erase(it);
  delete r;
  return NG_OK;
}

int ng_session_context(ng_session* ss, ng_ctx** out) {
  if (!ss || !out) return fail(NG_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(ss->server->mu);
  if (ss->pending) return fail(NG_ERR_STATE, "the session has requests not yet finished");
  *out = ss->ctx;
  return NG_OK;
}

int ng_server_get_stats(ng_server* s, ng_server_stats* out) {
  if (!s || !out) return fail(NG_ERR_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->arena_used_bytes = s->arena.used();
  return NG_OK;
}

}  // extern "C"
