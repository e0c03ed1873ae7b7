// Internal: the host runtime's context and helpers, shared by the context
// API (ng_runtime.cpp) and the serving layer (ng_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ng.h"
#include "ng_internal.h"

namespace ngrt {

int fail(int code, const char* fmt, ...);

constexpr uint64_t kAlign = 256;
constexpr uint64_t kScalarBytes = 128;  // a context's device words (ng_ctx::d_scalars)
constexpr uint32_t kCheckWord = 16;     // d_scalars[16..23]: the array check's four u64 results

// First-fit sub-allocator over the caller's arena (host bookkeeping only).
// Thread-safe.  A context that owns its arena frees immediately (reuse is
// ordered by its single stream).  An arena shared by contexts on several
// streams takes frees through release_after(stream, ranges, event): the
// ranges come back once the event, recorded on that stream after their last
// use, has completed.  Events of one stream complete in order, so only the
// oldest pending release of each stream is ever queried.
class Arena {
 public:
  using Ranges = std::vector<std::pair<char*, uint64_t>>;
  ~Arena() {
    for (auto& kv : deferred_)
      for (auto& d : kv.second) (void)hipEventDestroy(d.ev);
  }
  void init(char* base, uint64_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
  }
  char* alloc(uint64_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    bytes = round_up(bytes ? bytes : 1);
    char* p = first_fit_locked(bytes);
    if (!p && deferred_bytes_) {
      reclaim_locked();
      p = first_fit_locked(bytes);
    }
    return p;
  }
  void release(char* p, uint64_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    release_locked(p, bytes);
  }
  // release the ranges once `ev` (recorded on `stream` after their last use)
  // has completed; takes the event
  void release_after(hipStream_t stream, Ranges&& ranges, hipEvent_t ev) {
    std::lock_guard<std::mutex> lk(mu_);
    uint64_t b = 0;
    for (auto& r : ranges)
      if (r.first) b += round_up(r.second ? r.second : 1);
    deferred_[stream].push_back({std::move(ranges), ev, b});
    deferred_bytes_ += b;
  }
  uint64_t deferred_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    reclaim_locked();
    return deferred_bytes_;
  }
  uint64_t size() const { return size_; }

 private:
  struct Deferred {
    Ranges ranges;
    hipEvent_t ev;
    uint64_t bytes;
  };
  char* first_fit_locked(uint64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const uint64_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > bytes) free_[off + bytes] = sz - bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return base_ + off;
      }
    }
    return nullptr;
  }
  void reclaim_locked() {
    for (auto& kv : deferred_) {
      auto& q = kv.second;
      while (!q.empty() && hipEventQuery(q.front().ev) == hipSuccess) {
        for (auto& r : q.front().ranges) release_locked(r.first, r.second);
        (void)hipEventDestroy(q.front().ev);
        deferred_bytes_ -= q.front().bytes;
        q.pop_front();
      }
    }
  }
  void release_locked(char* p, uint64_t bytes) {
    if (!p) return;
    bytes = round_up(bytes ? bytes : 1);
    uint64_t off = (uint64_t)(p - base_);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 public:
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  uint64_t largest_free() {
    std::lock_guard<std::mutex> lk(mu_);
    reclaim_locked();
    uint64_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  static uint64_t round_up(uint64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

 private:
  char* base_ = nullptr;
  uint64_t size_ = 0;
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0, peak_ = 0;
  std::mutex mu_;
  std::map<hipStream_t, std::deque<Deferred>> deferred_;
  uint64_t deferred_bytes_ = 0;
};


int bitwidth(uint64_t v);
int64_t delay_steps_f32(float ms, float h);

struct Plan {
  ng::GenDesc d{};
  uint64_t n_new = 0;
  int32_t max_delay = 1;
};

// Validate one Connect call and fill its generation descriptor (Sec. 2.1).
int plan_call(uint32_t n_nodes, ng_range src, ng_range tgt, const ng_conn_spec* conn,
              const ng_syn_spec* syn, float h, Plan* out);

}  // namespace ngrt

struct ng_ctx {
  ng_config cfg{};
  int log2B = 24;
  uint64_t B = 1ull << 24;
  hipStream_t stream = nullptr;
  int device = 0;
  ngrt::Arena own_arena;
  ngrt::Arena* arena = &own_arena;  // a server's shared arena for sessions
  bool shared_arena = false;        // frees wait for this context's stream
  ngrt::Arena::Ranges pending_frees;  // shared arena: freed, not yet handed back
  uint64_t held = 0;                // arena bytes this context holds
  uint64_t need = 0;                // bytes the last NG_ERR_OOM asked for

  uint32_t n_nodes = 0;
  uint32_t next_cid = 0;
  uint64_t n_conns = 0;
  int32_t max_delay = 1;

  std::vector<char*> blocks;      // current storage, host copy of the device table
  char** d_tab[2] = {nullptr, nullptr};
  int cur = 0;                    // d_tab[cur] describes `blocks`
  uint32_t tab_synced = 0;        // leading entries of d_tab[cur] written on the device
  uint32_t tab_cap = 0;

  bool calibrated = false;
  uint32_t* d_group_ptr = nullptr;
  uint64_t group_ptr_bytes = 0;
  uint32_t* d_group_start = nullptr;
  uint64_t group_start_bytes = 0;
  // spike buffers over the calibrated connections (one allocation; released with the index)
  char* d_spikes = nullptr;
  uint64_t spikes_bytes = 0;
  ng::SpikeState spikes{};
  uint32_t spike_step = 0;  // steps since ng_spikes_init (stamps the emitting nodes)
  // device words: [0] = G, [2] = spike error word, [4..5] = Philox key,
  // [12..13] = spike-array entries (even, odd steps), [16..23] = array check
  // results (4 x u64)
  uint32_t* d_scalars = nullptr;
  uint32_t check_epoch = 0;       // ng_connect_groups calls checked so far (mod 2^32)
  uint32_t* h_words = nullptr;    // pinned host words for small device-to-host reads
  uint64_t h_words_cap = 0;       // words
  uint32_t gi_nodes = 0;          // n_nodes the index was built for

  int radix_bits = 9;  // widest digit: the fewest passes
  uint32_t sort_ranges = 1024;  // static ranges (= workgroups) of each sort pass
  int calib_mode = 0;           // NG_CALIB_RADIX, _COPASS, _RADIX_LSD or _RADIX_MSD
  uint32_t msd_tile = 0;        // records per tile of the MSD second scatter over packed records (0: default)
  uint32_t gen_quads = 1;       // groups of four synapses per generation lane
  int sticky = NG_OK;
  std::string sticky_msg;

  // optional per-kernel timing with HIP events on the context's stream
  struct Timed {
    const char* name;
    hipEvent_t a, b;
    uint64_t records;
  };
  struct TimeAcc {
    double ms = 0;
    uint64_t launches = 0, records = 0;
  };
  bool timing = false;
  std::string timing_only;  // with timing on: only launches of this name get events (empty: all)
  std::vector<hipEvent_t> ev_pool;
  std::vector<Timed> pending;
  std::map<std::string, TimeAcc> timing_acc;

  // graph capture: while capturing, nothing may synchronize; descriptors go
  // to a pinned region the graph owns.  A context with live graphs is frozen.
  bool capturing = false;
  bool timing_before_capture = false;
  char* cap_stage = nullptr;
  uint64_t cap_stage_cap = 0, cap_stage_used = 0;
  int frozen = 0;

  // Connect calls planned and committed whose generation is not launched yet:
  // they go out together as one batched launch when a call needs their
  // connections (flush_connects).  Groups of four synapses queued so far.
  std::vector<ng::GenDesc> queued;
  uint64_t queued_groups = 0;
  uint32_t queued_max = 256;  // calls queued before they go out (0: none)

  // pinned staging for descriptor uploads
  char* h_stage = nullptr;
  uint64_t h_stage_cap = 0;  // bytes
  hipEvent_t stage_done = nullptr;
  // orders this context's stream against another one (packed calibration)
  hipEvent_t order_ev = nullptr;
};

namespace ngrt {

// Allocate from the context's arena, counting what the context holds.
char* ctx_alloc(ng_ctx* c, uint64_t bytes);

// A set of context allocations made all-or-nothing.
struct AllocSet {
  ng_ctx* ctx;
  std::vector<std::pair<char*, uint64_t>> items;
  bool ok = true;
  uint64_t asked = 0;  // everything requested, also after a failure
  explicit AllocSet(ng_ctx* c) : ctx(c) {}
  char* get(uint64_t bytes) {
    asked += Arena::round_up(bytes ? bytes : 1);
    if (!ok) return nullptr;
    char* p = ctx_alloc(ctx, bytes);
    if (!p) {
      ok = false;
      return nullptr;
    }
    items.emplace_back(p, bytes);
    return p;
  }
  // nothing was enqueued on these yet: return them at once
  void release_all() {
    for (auto& it : items) {
      ctx->arena->release(it.first, it.second);
      ctx->held -= Arena::round_up(it.second ? it.second : 1);
    }
    items.clear();
  }
};

int dev_fail(ng_ctx* c, hipError_t e, const char* what);
hipEvent_t take_event(ng_ctx* c);
// Whether a launch of this name is bracketed by timing events.
inline bool timed_launch(const ng_ctx* c, const char* name) {
  return c->timing && (c->timing_only.empty() || c->timing_only == name);
}
void collect_timing(ng_ctx* c);
int enter(ng_ctx* c);
hipError_t set_table(char** tab, uint32_t first, const std::vector<char*>& ptrs, uint32_t from,
                     hipStream_t s);
uint32_t* key_ptr(ng_ctx* c);
uint32_t* gen_err_ptr(ng_ctx* c);
hipError_t set_seed(ng_ctx* c, uint64_t seed);
int mutable_state(ng_ctx* c);
int not_capturing(ng_ctx* c);
int reserve_blocks(ng_ctx* c, uint64_t n_new);
// Write the block-table entries not yet on the device (kernel arguments, on
// the context's stream); every launch that reads d_tab[cur] comes after.
int sync_table(ng_ctx* c);
// Hand the unwritten entries to a caller that writes many contexts' entries
// in one launch (marks them written).
void take_table_entries(ng_ctx* c, std::vector<ng::TabEntry>& out);
void release_index(ng_ctx* c);
// Return memory to the context's arena.  With a shared arena the range is
// collected and handed back by ctx_flush_frees, behind one event recorded on
// the context's stream after everything enqueued so far.
void ctx_free(ng_ctx* c, char* p, uint64_t bytes);
void ctx_flush_frees(ng_ctx* c);
// Undo an allocation that no enqueued work has used (rollback): at once.
void ctx_unalloc(ng_ctx* c, char* p, uint64_t bytes);
// A context over a shared arena on `stream` (server sessions).
int ctx_init(const ng_config* cfg, Arena* shared, char* base, uint64_t bytes, hipStream_t stream,
             ng_ctx** out);
int ctx_create_shared(const ng_config* cfg, Arena* arena, hipStream_t stream, ng_ctx** out);
// Release everything a context holds in its arena, then delete it.
void ctx_destroy_release(ng_ctx* c);
// Plan a Connect call and reserve its blocks without launching it; the
// descriptor carries the block table and key of this context.
int connect_prepare(ng_ctx* c, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                    const ng_syn_spec* syn, ng::GenDesc* out, uint64_t* out_n);
int connect_prepare_limit(ng_ctx* c, uint32_t node_limit, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                          const ng_syn_spec* syn, ng::GenDesc* out, uint64_t* out_n);
// Upload `bytes` of host data to device memory on the context's stream:
// through the graph's own pinned region while capturing, else through the
// context's pinned staging buffer (reused once its last upload completed).
int stage_upload(ng_ctx* c, void* d_dst, const void* src, uint64_t bytes);
// Pinned host buffer of at least n words for a device-to-host read that is
// synchronized before the next one; null (with the error set) on failure.
uint32_t* host_words(ng_ctx* c, uint64_t n);
// Copies host bytes to device memory, stream-ordered on the given stream.
using Uploader = std::function<int(hipStream_t, void* d_dst, const void* src, uint64_t bytes)>;
// Calibrate n distinct contexts with one sequence of launches on the first
// one's stream (each context is one segment of the sorts); the others'
// streams are ordered before and after with events.  Descriptor tables go up
// through `upload` if given, else through the first context's staging.
// Bump allocator over a fixed device region (the no-allocation calibration's
// scratch): 256-byte aligned pieces; ok turns false once a request does not fit.
struct ScratchBump {
  char* base = nullptr;
  uint64_t cap = 0, used = 0;
  bool ok = true;
  char* get(uint64_t bytes) {
    const uint64_t b = (bytes + kAlign - 1) / kAlign * kAlign;
    if (!ok || b > cap - used) {
      ok = false;
      used = cap;
      return nullptr;
    }
    char* p = base + used;
    used += b ? b : kAlign;
    return p;
  }
};

// sb: the sort and group-index scratch comes from sb instead of the arena
// (one context only); outputs still live in the context's arena.
int calibrate_many(ng_ctx* const* cs, uint32_t n, const Uploader* upload = nullptr, ScratchBump* sb = nullptr);
// The device address of the no-allocation calibration's scratch on the
// current device (looked up once per device; 0 on success).
int noalloc_scratch_init(int device);
// NG_OK if every descriptor names a block table and a key (checked on the host
// before any batched launch).
int check_descs(const std::vector<ng::GenDesc>& descs);
// Commit a prepared call: consume its call id and count its connections.
void connect_commit(ng_ctx* c, const ng::GenDesc& d, int32_t max_delay);
// Launch the queued Connect calls' generation: one batched launch whose
// descriptors come from the arena, or (batched = false, or no arena room)
// one launch per call with its descriptor as the argument.  Every entry point
// that reads the connections or orders work after them calls it first.
// NG_OK when nothing is queued.
int flush_connects(ng_ctx* c, bool batched = true);

}  // namespace ngrt

#define NG_HIP(ctx, expr, what)                 \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return dev_fail(ctx, e_, what); \
  } while (0)

// Launch `expr` on the context stream; with timing on, bracket it by events.
#define NG_LAUNCH_N(ctx, name, recs, expr)                                      \
  do {                                                                          \
    hipEvent_t a_ = nullptr;                                                    \
    if (timed_launch(ctx, name) && (a_ = take_event(ctx)) != nullptr)          \
      (void)hipEventRecord(a_, (ctx)->stream);                                  \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) return dev_fail(ctx, e_, name);                       \
    if (a_) {                                                                   \
      hipEvent_t b_ = take_event(ctx);                                          \
      if (b_) {                                                                 \
        (void)hipEventRecord(b_, (ctx)->stream);                                \
        (ctx)->pending.push_back({name, a_, b_, (uint64_t)(recs)});             \
      } else {                                                                  \
        (ctx)->ev_pool.push_back(a_);                                           \
      }                                                                         \
    }                                                                           \
  } while (0)
#define NG_LAUNCH(ctx, name, expr) NG_LAUNCH_N(ctx, name, 0, expr)
