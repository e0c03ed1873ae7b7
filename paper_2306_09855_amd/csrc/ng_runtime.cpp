// Host runtime of the connectivity builder: context, arena sub-allocator,
// Connect planning (Sec. 2.1: rule counts, Eq. (1) blocks, Eqs. (2)-(3)
// numbering) and calibration orchestration (Sec. 2.2).  All device work is
// enqueued on the caller's stream; nothing here computes connections on the
// host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ng_rt.h"

namespace ngrt {

// Connect calls with fewer synapses than this wait in the context's queue;
// the queue goes out when it holds the schedule's queued_calls calls (or
// earlier, when a call needs the connections).
constexpr uint64_t kQueuedCallMax = 1ull << 24;
constexpr uint32_t kQueuedCallsLimit = 4096;

// Scratch of ng_calibrate_noalloc: a fixed array in device memory, one copy per
// GPU at its own address, held until the process ends.  Host code never uses
// the name `scratch` as an address: the address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch_ptr;  // per device id

int noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return fail(NG_ERR_DEVICE, "bad device id");
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (g_scratch_ptr[(size_t)device]) return NG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(NG_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch_ptr[(size_t)device] = (char*)ptr;
  return NG_OK;
}

static char* noalloc_scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && (size_t)device < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)device] : nullptr;
}


thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}


int bitwidth(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

// fp32 ms -> steps, one-step minimum (Sec. 2.1)
int64_t delay_steps_f32(float ms, float h) {
  const float q = ms / h;
  const float r = std::rint(q);
  if (!(r >= 1.0f)) return 1;
  if (r > 2147483647.0f) return INT64_MAX;
  return (int64_t)r;
}

int plan_call(uint32_t n_nodes, ng_range src, ng_range tgt, const ng_conn_spec* conn,
              const ng_syn_spec* syn, float h, Plan* out) {
  if (!conn || !syn) return fail(NG_ERR_INVALID_ARG, "null connection or synapse spec");
  if ((uint64_t)src.first + src.n > n_nodes || (uint64_t)tgt.first + tgt.n > n_nodes)
    return fail(NG_ERR_INVALID_ARG, "node range [%u,+%u) or [%u,+%u) exceeds the %u created nodes",
                src.first, src.n, tgt.first, tgt.n, n_nodes);
  const uint64_t ns = src.n, nt = tgt.n, k = conn->k_or_n;
  // allow_autapses = 0 matters only where the ranges share nodes
  const uint64_t ov_lo = std::max<uint64_t>(src.first, tgt.first);
  const uint64_t ov_hi = std::min<uint64_t>((uint64_t)src.first + ns, (uint64_t)tgt.first + nt);
  const uint64_t ov = ov_hi > ov_lo ? ov_hi - ov_lo : 0;
  const bool no_self = !conn->allow_autapses && ov > 0;
  uint64_t n = 0;
  switch (conn->rule) {
    case NG_ONE_TO_ONE:
      if (ns != nt) return fail(NG_ERR_INVALID_ARG, "one_to_one needs equal ranges (%llu vs %llu)",
                                (unsigned long long)ns, (unsigned long long)nt);
      n = (no_self && src.first == tgt.first) ? 0 : ns;  // with s0 != t0 no pair is s == t
      break;
    case NG_ALL_TO_ALL: n = ns * nt - (no_self ? ov : 0); break;
    case NG_FIXED_INDEGREE:
      if (k > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "K too large");
      n = nt * k;
      if (n && ns == 0) return fail(NG_ERR_INVALID_ARG, "fixed_indegree needs a non-empty source range");
      if (n && no_self && ns == 1)
        return fail(NG_ERR_INVALID_ARG, "fixed_indegree without autapses: a target has no other source");
      if (n && !conn->allow_multapses && k > ns - (no_self ? 1 : 0))
        return fail(NG_ERR_INVALID_ARG, "fixed_indegree without multapses: K exceeds the distinct sources");
      break;
    case NG_FIXED_OUTDEGREE:
      if (k > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "K too large");
      n = ns * k;
      if (n && nt == 0) return fail(NG_ERR_INVALID_ARG, "fixed_outdegree needs a non-empty target range");
      if (n && no_self && nt == 1)
        return fail(NG_ERR_INVALID_ARG, "fixed_outdegree without autapses: a source has no other target");
      if (n && !conn->allow_multapses && k > nt - (no_self ? 1 : 0))
        return fail(NG_ERR_INVALID_ARG, "fixed_outdegree without multapses: K exceeds the distinct targets");
      break;
    case NG_FIXED_TOTAL_NUMBER:
      n = k;
      if (n && (ns == 0 || nt == 0))
        return fail(NG_ERR_INVALID_ARG, "fixed_total_number needs non-empty ranges");
      if (n && no_self && ns * nt == ov)
        return fail(NG_ERR_INVALID_ARG, "fixed_total_number without autapses: every pair is an autapse");
      if (n && !conn->allow_multapses && n > ns * nt - (no_self ? ov : 0))
        return fail(NG_ERR_INVALID_ARG, "fixed_total_number without multapses: N exceeds the distinct pairs");
      break;
    case NG_PAIRWISE_BERNOULLI:
      return fail(NG_ERR_UNSUPPORTED, "pairwise_bernoulli is taken only by ng_connect (its count needs a device pass)");
    default: return fail(NG_ERR_INVALID_ARG, "unknown rule %d", conn->rule);
  }
  if (n > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "a call may create at most 2^32-1 connections");

  ng::GenDesc d{};
  d.n_new = (uint32_t)n;
  d.rule = (uint32_t)conn->rule;
  d.k = (uint32_t)k;
  d.s0 = src.first;
  d.ns = src.n;
  d.t0 = tgt.first;
  d.nt = tgt.n;
  d.h = h;
  if (no_self && conn->rule != NG_ONE_TO_ONE) {
    d.no_self = 1;
    d.a_lo = (uint32_t)(ov_lo - src.first);  // source positions whose node is also a target
    d.a_hi = (uint32_t)(ov_hi - src.first);
  }
  if (!conn->allow_multapses && n) {  // distinct draws: a keyed permutation per call or node
    if (conn->rule == NG_FIXED_INDEGREE) d.rule = ng::kRuleIndegDistinct;
    if (conn->rule == NG_FIXED_OUTDEGREE) d.rule = ng::kRuleOutdegDistinct;
    if (conn->rule == NG_FIXED_TOTAL_NUMBER) {
      d.rule = ng::kRuleTotalDistinct;
      d.n_pairs = ns * nt - (no_self ? ov : 0);
    }
  }

  const ng_param& w = syn->weight;
  if (!std::isfinite(w.a) || !std::isfinite(w.b)) return fail(NG_ERR_INVALID_ARG, "non-finite weight parameter");
  switch (w.kind) {
    case NG_CONST: d.w_kind = ng::W_CONST; d.w_a = (float)w.a; break;
    case NG_NORMAL:
      if (w.b < 0) return fail(NG_ERR_INVALID_ARG, "normal weight needs sd >= 0");
      d.w_kind = ng::W_NORMAL; d.w_a = (float)w.a; d.w_b = (float)w.b;
      break;
    case NG_UNIFORM:
      if (w.b < w.a) return fail(NG_ERR_INVALID_ARG, "uniform weight needs a <= b");
      d.w_kind = ng::W_UNIFORM; d.w_a = (float)w.a; d.w_b = (float)(w.b - w.a);
      break;
    default: return fail(NG_ERR_INVALID_ARG, "unsupported weight distribution %d", w.kind);
  }

  const ng_param& dl = syn->delay;
  if (!std::isfinite(dl.a) || !std::isfinite(dl.b)) return fail(NG_ERR_INVALID_ARG, "non-finite delay parameter");
  int64_t maxd = 1;
  switch (dl.kind) {
    case NG_CONST: {
      const int64_t st = delay_steps_f32((float)dl.a, h);
      if (st > 32767) return fail(NG_ERR_INVALID_ARG, "delay exceeds 32767 steps");
      d.d_kind = ng::D_CONST;
      d.d_const = (int32_t)st;
      maxd = st;
      break;
    }
    case NG_UNIFORM_INT: {
      if (dl.a != std::floor(dl.a) || dl.b != std::floor(dl.b) || dl.a < 1 || dl.b < dl.a || dl.b > 32767)
        return fail(NG_ERR_INVALID_ARG, "uniform_int delay needs integers 1 <= a <= b <= 32767");
      d.d_kind = ng::D_UNIFORM_INT;
      d.d_lo = (uint32_t)dl.a;
      d.d_range = (uint32_t)(dl.b - dl.a + 1);
      maxd = (int64_t)dl.b;
      break;
    }
    case NG_UNIFORM: {
      if (dl.a < 0 || dl.b < dl.a) return fail(NG_ERR_INVALID_ARG, "uniform ms delay needs 0 <= a <= b");
      d.d_kind = ng::D_UNIFORM_MS;
      d.d_ms_lo = (float)dl.a;
      d.d_ms_width = (float)(dl.b - dl.a);
      // the largest step count is reached at u -> 1 (every fp32 step is monotone)
      maxd = delay_steps_f32(std::fmaf(d.d_ms_width, 1.0f, d.d_ms_lo), h);
      if (maxd > 32767) return fail(NG_ERR_INVALID_ARG, "delay exceeds 32767 steps");
      break;
    }
    default: return fail(NG_ERR_INVALID_ARG, "unsupported delay distribution %d", dl.kind);
  }
  out->d = d;
  out->n_new = n;
  out->max_delay = (int32_t)maxd;
  return NG_OK;
}


int dev_fail(ng_ctx* c, hipError_t e, const char* what) {
  c->sticky = NG_ERR_DEVICE;
  c->sticky_msg = std::string(what) + ": " + hipGetErrorString(e);
  return fail(NG_ERR_DEVICE, "%s", c->sticky_msg.c_str());
}

// Timing events only measure: they carry no system-scope fence (the fence
// writes back and invalidates the caches at every record and left ~10 us of
// idle GPU at each one; ~7.7 us without it).  Results reach the host through
// the synchronizing calls, which do not rely on these events.
hipEvent_t take_event(ng_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

void collect_timing(ng_ctx* c) {
  for (auto& t : c->pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      auto& acc = c->timing_acc[t.name];
      acc.ms += ms;
      acc.launches += 1;
      acc.records += t.records;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->pending.clear();
}

int enter(ng_ctx* c) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  if (c->sticky != NG_OK) return fail(c->sticky, "%s", c->sticky_msg.c_str());
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return dev_fail(c, e, "hipSetDevice");
  if (!c->capturing) ctx_flush_frees(c);  // frees left by an earlier call
  return NG_OK;
}

// Write block pointers into a device table through kernel arguments (no host
// buffer lifetime to track).
hipError_t set_table(char** tab, uint32_t first, const std::vector<char*>& ptrs, uint32_t from,
                     hipStream_t s) {
  for (uint32_t i = from; i < ptrs.size(); i += 8) {
    uint64_t v[8] = {0};
    const uint32_t cnt = std::min<uint32_t>(8, (uint32_t)ptrs.size() - i);
    for (uint32_t k = 0; k < cnt; ++k) v[k] = (uint64_t)ptrs[i + k];
    hipError_t e = ng::launch_set_ptrs(tab, first + (i - from), cnt, v, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The Philox key lives in device memory (d_scalars[4..5]) so that a captured
// graph can be replayed with another seed.
uint32_t* key_ptr(ng_ctx* c) { return c->d_scalars + 4; }

// Generation error word (d_scalars[3], sticky): bit 0 a permutation walk
// started at or above its bound, bit 1 a walk reached its step cap.
uint32_t* gen_err_ptr(ng_ctx* c) { return c->d_scalars + 3; }

hipError_t set_seed(ng_ctx* c, uint64_t seed) {
  return ng::launch_set_ptrs(reinterpret_cast<char**>(key_ptr(c)), 0, 1, &seed, c->stream);
}

int mutable_state(ng_ctx* c) {
  if (c->frozen) return fail(NG_ERR_STATE, "the context has live graphs; destroy them before changing it");
  return NG_OK;
}

int not_capturing(ng_ctx* c) {
  if (c->capturing) return fail(NG_ERR_STATE, "not allowed while a graph is being captured");
  return NG_OK;
}

// Eq. (1) plus allocation; all-or-nothing.
int reserve_blocks(ng_ctx* c, uint64_t n_new) {
  const uint64_t nb = ng_blocks_needed(c->n_conns, n_new, c->B, c->blocks.size());
  if (c->blocks.size() + nb > c->tab_cap) {
    c->need = ~0ull;  // no release elsewhere makes room in the table
    return fail(NG_ERR_OOM, "block table full");
  }
  std::vector<char*> fresh;
  for (uint64_t b = 0; b < nb; ++b) {
    char* p = ctx_alloc(c, ng::kBytesPerConn * c->B);
    if (!p) {
      for (char* q : fresh) ctx_unalloc(c, q, ng::kBytesPerConn * c->B);
      c->need = nb * Arena::round_up(ng::kBytesPerConn * c->B);
      return fail(NG_ERR_OOM, "arena cannot hold %llu more blocks of %llu connections",
                  (unsigned long long)nb, (unsigned long long)c->B);
    }
    fresh.push_back(p);
  }
  for (char* p : fresh) c->blocks.push_back(p);  // written to the device table by sync_table
  return NG_OK;
}

int sync_table(ng_ctx* c) {
  if (c->tab_synced < c->blocks.size()) {
    NG_HIP(c, set_table(c->d_tab[c->cur], c->tab_synced, c->blocks, c->tab_synced, c->stream), "block table");
    c->tab_synced = (uint32_t)c->blocks.size();
  }
  return NG_OK;
}

void take_table_entries(ng_ctx* c, std::vector<ng::TabEntry>& out) {
  for (uint32_t i = c->tab_synced; i < c->blocks.size(); ++i)
    out.push_back(ng::TabEntry{c->d_tab[c->cur], c->blocks[i], i, 0});
  c->tab_synced = (uint32_t)c->blocks.size();
}

void release_index(ng_ctx* c) {
  ctx_free(c, (char*)c->d_group_ptr, c->group_ptr_bytes);
  ctx_free(c, (char*)c->d_group_start, c->group_start_bytes);
  c->d_group_ptr = c->d_group_start = nullptr;
  c->group_ptr_bytes = c->group_start_bytes = 0;
  ctx_free(c, c->d_spikes, c->spikes_bytes);  // the spike buffers walk the index
  c->d_spikes = nullptr;
  c->spikes_bytes = 0;
}

int check_descs(const std::vector<ng::GenDesc>& descs) {
  for (const auto& d : descs)
    if (!d.blocks || !d.key || !d.err)
      return fail(NG_ERR_STATE, "internal: a generation descriptor has no block table, key or error word");
  return NG_OK;
}

// Host-side resources of a context: pinned staging, events.
void ctx_host_release(ng_ctx* c) {
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  c->h_stage = nullptr;
  if (c->h_words) (void)hipHostFree(c->h_words);
  c->h_words = nullptr;
  c->h_words_cap = 0;
  if (c->stage_done) (void)hipEventDestroy(c->stage_done);
  if (c->order_ev) (void)hipEventDestroy(c->order_ev);
  c->stage_done = c->order_ev = nullptr;
  collect_timing(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
}

char* ctx_alloc(ng_ctx* c, uint64_t bytes) {
  char* p = c->arena->alloc(bytes);
  if (p) c->held += Arena::round_up(bytes ? bytes : 1);
  return p;
}

void ctx_free(ng_ctx* c, char* p, uint64_t bytes) {
  if (!p) return;
  c->held -= Arena::round_up(bytes ? bytes : 1);
  if (!c->shared_arena) {
    c->arena->release(p, bytes);
    return;
  }
  c->pending_frees.emplace_back(p, bytes);
}

void ctx_unalloc(ng_ctx* c, char* p, uint64_t bytes) {
  if (!p) return;
  c->held -= Arena::round_up(bytes ? bytes : 1);
  c->arena->release(p, bytes);
}

void ctx_flush_frees(ng_ctx* c) {
  if (c->pending_frees.empty()) return;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
      hipEventRecord(ev, c->stream) == hipSuccess) {
    c->arena->release_after(c->stream, std::move(c->pending_frees), ev);
  } else {
    // cannot order the release: wait for the stream instead
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(c->stream);
    for (auto& r : c->pending_frees) c->arena->release(r.first, r.second);
  }
  c->pending_frees.clear();
}

// Common construction: an own arena over [base, base + bytes), or a shared one.
int ctx_init(const ng_config* cfg, Arena* shared, char* base, uint64_t bytes, hipStream_t stream,
             ng_ctx** out) {
  if (!cfg || !out) return fail(NG_ERR_INVALID_ARG, "null config or output");
  uint64_t B = cfg->block_size ? cfg->block_size : (1ull << 24);
  if (B & (B - 1) || B < (1ull << 16) || B > (1ull << 30))
    return fail(NG_ERR_INVALID_ARG, "block_size must be a power of two in [2^16, 2^30]");
  if (!(cfg->h_ms >= 0) || !std::isfinite(cfg->h_ms)) return fail(NG_ERR_INVALID_ARG, "bad time resolution");
  ng_ctx* c = new ng_ctx();
  c->cfg = *cfg;
  c->cfg.block_size = B;
  if (c->cfg.h_ms == 0) c->cfg.h_ms = 0.1f;
  c->B = B;
  c->log2B = bitwidth(B) - 1;
  c->stream = stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(NG_ERR_DEVICE, "no HIP device");
  }
  if (int rc = noalloc_scratch_init(c->device)) {  // library set-up, once per device
    delete c;
    return rc;
  }
  if (shared) {
    c->arena = shared;
    c->shared_arena = true;
    bytes = shared->size();
  } else {
    c->arena->init(base, bytes);
  }
  c->tab_cap = (uint32_t)std::min<uint64_t>(bytes / (ng::kBytesPerConn * B) + 2, 1u << 20);
  for (int t = 0; t < 2; ++t) c->d_tab[t] = (char**)ctx_alloc(c, 8ull * c->tab_cap);
  c->d_scalars = (uint32_t*)ctx_alloc(c, kScalarBytes);
  if (!c->d_tab[0] || !c->d_tab[1] || !c->d_scalars) {
    for (int t = 0; t < 2; ++t)
      if (c->d_tab[t]) c->arena->release((char*)c->d_tab[t], 8ull * c->tab_cap);
    if (c->d_scalars) c->arena->release((char*)c->d_scalars, kScalarBytes);
    delete c;
    return fail(NG_ERR_OOM, "arena too small");
  }
  if (hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) {
    ctx_host_release(c);
    delete c;
    return fail(NG_ERR_DEVICE, "hipEventCreate failed");
  }
  if (ng::launch_fill_u32(c->d_scalars, 0u, kScalarBytes / 4, c->stream) != hipSuccess ||
      set_seed(c, c->cfg.seed) != hipSuccess) {
    ctx_host_release(c);
    delete c;
    return fail(NG_ERR_DEVICE, "kernel launch failed");
  }
  *out = c;
  return NG_OK;
}

int ctx_create_shared(const ng_config* cfg, Arena* arena, hipStream_t stream, ng_ctx** out) {
  return ctx_init(cfg, arena, nullptr, 0, stream, out);
}

void ctx_destroy_release(ng_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (char* b : c->blocks) ctx_free(c, b, ng::kBytesPerConn * c->B);
  c->blocks.clear();
  release_index(c);
  for (int t = 0; t < 2; ++t) ctx_free(c, (char*)c->d_tab[t], 8ull * c->tab_cap);
  ctx_free(c, (char*)c->d_scalars, kScalarBytes);
  ctx_flush_frees(c);
  ctx_host_release(c);
  delete c;
}

int connect_prepare(ng_ctx* c, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                    const ng_syn_spec* syn, ng::GenDesc* out, uint64_t* out_n) {
  return connect_prepare_limit(c, c->n_nodes, src, tgt, conn, syn, out, out_n);
}

// node_limit bounds the ranges; a group given by an index array is planned as
// the position range [0, n), which the node count does not bound
int connect_prepare_limit(ng_ctx* c, uint32_t node_limit, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                          const ng_syn_spec* syn, ng::GenDesc* out, uint64_t* out_n) {
  if (!c->capturing) ctx_flush_frees(c);  // make this context's frees reusable
  Plan p;
  if (int rc = plan_call(node_limit, src, tgt, conn, syn, c->cfg.h_ms, &p)) return rc;
  if (c->next_cid == 0xFFFFFFFFu) return fail(NG_ERR_TOO_LARGE, "connect call ids exhausted");
  if (c->n_conns + p.n_new > 0xFFFFFFFFull)
    return fail(NG_ERR_TOO_LARGE, "a context holds at most 2^32-1 connections");
  if (int rc = reserve_blocks(c, p.n_new)) return rc;
  p.d.pos0 = c->n_conns;
  p.d.cid = c->next_cid;
  p.d.blocks = c->d_tab[c->cur];
  p.d.key = key_ptr(c);
  p.d.err = gen_err_ptr(c);
  p.d.max_delay = p.max_delay;
  *out = p.d;
  if (out_n) *out_n = p.n_new;
  return NG_OK;
}

// Pinned host words for the small results the host reads back (kept, and
// grown when needed, until the context is released); every read is followed
// by a stream synchronization before the next one.
uint32_t* host_words(ng_ctx* c, uint64_t n) {
  if (c->h_words_cap < n) {
    if (c->h_words) (void)hipHostFree(c->h_words);
    c->h_words = nullptr;
    c->h_words_cap = 0;
    if (hipHostMalloc((void**)&c->h_words, 4 * n, hipHostMallocDefault) != hipSuccess) {
      c->h_words = nullptr;
      fail(NG_ERR_DEVICE, "hipHostMalloc of %llu bytes failed", (unsigned long long)(4 * n));
      return nullptr;
    }
    c->h_words_cap = n;
  }
  return c->h_words;
}

int stage_upload(ng_ctx* c, void* d_dst, const void* src, uint64_t bytes) {
  if (bytes == 0) return NG_OK;
  if (c->capturing) {
    // the upload becomes a graph node reading this pinned region on every replay
    const uint64_t need = (bytes + 255) / 256 * 256;
    if (c->cap_stage_used + need > c->cap_stage_cap)
      return fail(NG_ERR_OOM, "graph staging region full (%llu bytes)", (unsigned long long)c->cap_stage_cap);
    char* h = c->cap_stage + c->cap_stage_used;
    c->cap_stage_used += need;
    memcpy(h, src, bytes);
    NG_HIP(c, hipMemcpyAsync(d_dst, h, bytes, hipMemcpyHostToDevice, c->stream), "upload");
    return NG_OK;
  }
  NG_HIP(c, hipEventSynchronize(c->stage_done), "stage wait");
  if (c->h_stage_cap < bytes) {
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    c->h_stage = nullptr;
    c->h_stage_cap = 0;
    NG_HIP(c, hipHostMalloc((void**)&c->h_stage, bytes, hipHostMallocDefault), "hipHostMalloc");
    c->h_stage_cap = bytes;
  }
  memcpy(c->h_stage, src, bytes);
  NG_HIP(c, hipMemcpyAsync(d_dst, c->h_stage, bytes, hipMemcpyHostToDevice, c->stream), "upload");
  NG_HIP(c, hipEventRecord(c->stage_done, c->stream), "event");
  return NG_OK;
}

namespace {

// One context's part of a (packed) calibration.
struct CalSeg {
  ng_ctx* c = nullptr;
  uint64_t N = 0;
  uint32_t nn = 0;
  int dbits = 0, passes = 1;
  uint32_t shift[32] = {0}, nbits[32] = {0};
  uint32_t tiles_per_range = 0, n_ranges = 0;
  uint64_t gi_tiles = 0, gcap = 1;
  std::unique_ptr<AllocSet> as;
  std::vector<char*> nblocks;
  uint32_t* keys[2] = {nullptr, nullptr};
  uint2* pay[2] = {nullptr, nullptr};
  uint32_t* group_src = nullptr;
  uint32_t* bitmap = nullptr;
  uint32_t* gptr = nullptr;
  uint32_t* gstart = nullptr;
  uint64_t gp_bytes = 0, gs_bytes = 0;
  int nxt = 0;
  ScratchBump* sb = nullptr;  // scratch from a fixed region instead of the arena
};

// Digit schedule and geometry (no allocation).
int cal_plan(CalSeg& g) {
  ng_ctx* c = g.c;
  g.N = c->n_conns;
  g.nn = c->n_nodes;
  const int sbits = bitwidth(g.nn > 0 ? g.nn - 1 : 0);
  g.dbits = bitwidth((uint64_t)c->max_delay);
  const int keybits = sbits + g.dbits;
  if (keybits > 32) return fail(NG_ERR_UNSUPPORTED, "source+delay keys wider than 32 bits");
  const int RB = c->radix_bits;
  g.passes = std::max(1, (keybits + RB - 1) / RB);
  const int base_bits = keybits / g.passes, extra = keybits % g.passes;
  int sh = 0;
  for (int p = 0; p < g.passes; ++p) {
    g.nbits[p] = (uint32_t)(base_bits + (p < extra ? 1 : 0));
    g.shift[p] = (uint32_t)sh;
    sh += (int)g.nbits[p];
  }
  // static ranges of consecutive tiles, one workgroup each
  const uint64_t tile = ng::sort_tile_size();
  const uint64_t n_tiles = (g.N + tile - 1) / tile;
  g.tiles_per_range = (uint32_t)std::max<uint64_t>(1, (n_tiles + c->sort_ranges - 1) / c->sort_ranges);
  g.n_ranges = (uint32_t)((n_tiles + g.tiles_per_range - 1) / g.tiles_per_range);
  g.gi_tiles = (g.N + ng::gi_tile_size() - 1) / ng::gi_tile_size();
  g.gcap = std::min<uint64_t>(g.N, (uint64_t)g.nn * (uint64_t)c->max_delay) + 1;
  const uint64_t nblk = (g.N + c->B - 1) / c->B;
  if (nblk > c->tab_cap) {
    c->need = ~0ull;  // no release elsewhere makes room in the table
    return fail(NG_ERR_OOM, "block table full");
  }
  return NG_OK;
}

// Per-context buffers, all-or-nothing.  The context is uncalibrated, so its
// old index is stale and is released first to make room.
int cal_alloc(CalSeg& g) {
  ng_ctx* c = g.c;
  g.as.reset(new AllocSet(c));
  AllocSet& as = *g.as;
  const uint64_t nblk = (g.N + c->B - 1) / c->B;
  for (uint64_t b = 0; b < nblk && as.ok; ++b) g.nblocks.push_back(as.get(ng::kBytesPerConn * c->B));
  auto sget = [&](uint64_t bytes) { return g.sb ? g.sb->get(bytes) : as.get(bytes); };
  for (int t = 0; t < std::min(g.passes - 1, 2); ++t) {
    g.keys[t] = (uint32_t*)sget(4 * std::max<uint64_t>(g.N, 1));
    g.pay[t] = (uint2*)sget(8 * std::max<uint64_t>(g.N, 1));
  }
  g.group_src = (uint32_t*)sget(4 * g.gcap);
  g.bitmap = (uint32_t*)sget(4 * ((g.N + 31) / 32 + 1));
  if (g.sb && !g.sb->ok) {
    as.release_all();
    g.nblocks.clear();
    return fail(NG_ERR_TOO_LARGE, "the calibration scratch of %llu connections exceeds the fixed %llu-byte region",
                (unsigned long long)g.N, (unsigned long long)g.sb->cap);
  }
  g.gp_bytes = 4 * (g.nn + 1ull);
  g.gs_bytes = 4 * g.gcap;
  release_index(c);
  c->calibrated = false;
  g.gptr = (uint32_t*)ctx_alloc(c, g.gp_bytes);
  g.gstart = g.gptr ? (uint32_t*)ctx_alloc(c, g.gs_bytes) : nullptr;
  if (!as.ok || !g.gptr || !g.gstart) {
    as.release_all();
    ctx_unalloc(c, (char*)g.gptr, g.gp_bytes);
    ctx_unalloc(c, (char*)g.gstart, g.gs_bytes);
    g.gptr = g.gstart = nullptr;
    g.nblocks.clear();
    c->need = as.asked + Arena::round_up(g.gp_bytes) + Arena::round_up(g.gs_bytes);
    return fail(NG_ERR_OOM, "arena cannot hold the calibration buffers (N=%llu)", (unsigned long long)g.N);
  }
  g.nxt = 1 - c->cur;
  return NG_OK;
}

void cal_release(CalSeg& g) {
  if (!g.as) return;
  g.as->release_all();
  ctx_unalloc(g.c, (char*)g.gptr, g.gp_bytes);
  ctx_unalloc(g.c, (char*)g.gstart, g.gs_bytes);
  g.gptr = g.gstart = nullptr;
  g.nblocks.clear();
  g.as.reset();
}

ng::SortSeg sort_seg(const CalSeg& g, int p) {
  ng_ctx* c = g.c;
  ng::SortSeg s{};
  s.io.log2B = c->log2B;
  s.io.dbits = (uint32_t)g.dbits;
  if (p == 0) s.io.in_blocks = c->d_tab[c->cur];
  else {
    s.io.in_keys = g.keys[(p - 1) & 1];
    s.io.in_pay = g.pay[(p - 1) & 1];
  }
  if (p == g.passes - 1) s.io.out_blocks = c->d_tab[g.nxt];
  else {
    s.io.out_keys = g.keys[p & 1];
    s.io.out_pay = g.pay[p & 1];
  }
  s.n = g.N;
  s.shift = g.shift[p];
  s.nbits = g.nbits[p];
  s.tiles_per_range = g.tiles_per_range;
  s.n_ranges = g.n_ranges;
  return s;
}

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

// COPASS in-place block sort (Appendix A) of one context, then the group
// index.  The connections stay in their blocks.  Scratch: the auxiliary
// array and one or two sort buffers of one block each (packed key + payload,
// 12 bytes per record; the first sort buffer doubles as the bounce buffer of
// the shifts), the sort counts, the partition's per-subarray words and the
// copy lists.
int calibrate_copass(ng_ctx* c) {
  if (c->capturing) return fail(NG_ERR_UNSUPPORTED, "a COPASS calibration reads partition sizes back; it cannot be captured");
  CalSeg g;
  g.c = c;
  if (int rc = cal_plan(g)) return rc;
  const uint64_t N = g.N, B = c->B;
  const uint32_t k = (uint32_t)((N + B - 1) / B);
  const uint64_t A = std::max<uint64_t>(1, std::min<uint64_t>(B, N));  // the largest block
  const int P = g.passes;
  const uint64_t tile = ng::sort_tile_size();
  const uint64_t blk_tiles = (A + tile - 1) / tile;
  // a sort of n <= A records uses ceil(tiles / ceil(tiles / sort_ranges)) <= min(sort_ranges, tiles) ranges
  const uint64_t max_ranges = std::max<uint64_t>(1, std::min<uint64_t>(c->sort_ranges, blk_tiles));
  uint32_t maxbits = 0;
  for (int p = 0; p < P; ++p) maxbits = std::max(maxbits, g.nbits[p]);
  const uint64_t counts_n = ((uint64_t)1 << maxbits) * max_ranges;
  const uint64_t seg_cap = 5ull * k + 8;  // copy pieces of one step
  // the partition results are read back through pinned words: had before
  // anything moves, so that failing to get them changes nothing
  if (k > 1 && !host_words(c, (uint64_t)k + 3)) return NG_ERR_DEVICE;

  AllocSet as(c);
  uint32_t* aux_k = (uint32_t*)as.get(4 * A);
  uint2* aux_p = (uint2*)as.get(8 * A);
  uint32_t* s_k[2] = {nullptr, nullptr};
  uint2* s_p[2] = {nullptr, nullptr};
  for (int t = 0; t < (P >= 3 ? 2 : 1); ++t) {
    s_k[t] = (uint32_t*)as.get(4 * A);
    s_p[t] = (uint2*)as.get(8 * A);
  }
  uint32_t* counts = (uint32_t*)as.get(4 * counts_n);
  const uint64_t tmp_words = std::max(ng::scan_tmp_words(counts_n), ng::scan_tmp_words(g.gi_tiles));
  uint32_t* scan_tmp = (uint32_t*)as.get(4 * tmp_words);
  uint32_t* part = (uint32_t*)as.get(4 * (7ull * std::max<uint32_t>(k, 1) + 4));
  ng::CopySeg* d_lists = (ng::CopySeg*)as.get(sizeof(ng::CopySeg) * seg_cap);
  uint32_t* tile_flags = (uint32_t*)as.get(4 * (g.gi_tiles + 1));
  g.group_src = (uint32_t*)as.get(4 * g.gcap);
  g.bitmap = (uint32_t*)as.get(4 * ((N + 31) / 32 + 1));
  g.gp_bytes = 4 * (g.nn + 1ull);
  g.gs_bytes = 4 * g.gcap;
  release_index(c);
  c->calibrated = false;
  g.gptr = (uint32_t*)ctx_alloc(c, g.gp_bytes);
  g.gstart = g.gptr ? (uint32_t*)ctx_alloc(c, g.gs_bytes) : nullptr;
  if (!as.ok || !g.gptr || !g.gstart) {
    as.release_all();
    ctx_unalloc(c, (char*)g.gptr, g.gp_bytes);
    ctx_unalloc(c, (char*)g.gstart, g.gs_bytes);
    c->need = as.asked + Arena::round_up(g.gp_bytes) + Arena::round_up(g.gs_bytes);
    return fail(NG_ERR_OOM, "arena cannot hold the COPASS scratch (block of %llu)", (unsigned long long)A);
  }
  uint32_t* d_start = part;
  uint32_t* d_len = part + k;
  uint32_t* d_lo = part + 2ull * k;
  uint32_t* d_hi = part + 3ull * k;
  uint32_t* d_mulo = part + 4ull * k;
  uint32_t* d_muhi = part + 5ull * k;
  uint32_t* d_mout = part + 6ull * k;
  uint32_t* d_status = part + 7ull * k;
  hipStream_t s = c->stream;
  char** tab = c->d_tab[c->cur];
  const ng::BlockView view{tab, c->log2B, (uint32_t)g.dbits};

  auto run = [&]() -> int {
    if (int rc = sync_table(c)) return rc;
    // sort the packed records aux[0, n) into block b
    auto sort_into = [&](uint32_t b, uint32_t n) -> int {
      const uint64_t tiles = (n + tile - 1) / tile;
      const uint32_t tpr = (uint32_t)std::max<uint64_t>(1, (tiles + c->sort_ranges - 1) / c->sort_ranges);
      const uint32_t nr = (uint32_t)((tiles + tpr - 1) / tpr);
      for (int p = 0; p < P; ++p) {
        ng::SortSeg sg{};
        sg.io.log2B = c->log2B;
        sg.io.dbits = (uint32_t)g.dbits;
        if (p == 0) {
          sg.io.in_keys = aux_k;
          sg.io.in_pay = aux_p;
        } else {
          sg.io.in_keys = s_k[(p - 1) & 1];
          sg.io.in_pay = s_p[(p - 1) & 1];
        }
        if (p == P - 1) {
          sg.io.out_blocks = tab + b;
        } else {
          sg.io.out_keys = s_k[p & 1];
          sg.io.out_pay = s_p[p & 1];
        }
        sg.n = n;
        sg.shift = g.shift[p];
        sg.nbits = g.nbits[p];
        sg.tiles_per_range = tpr;
        sg.n_ranges = nr;
        ng::SortPack pk{};
        pk.one = sg;
        pk.n_segs = 1;
        pk.total_ranges = nr;
        pk.ranges_per_xcd = (nr + 7) / 8;
        pk.max_nbits = sg.nbits;
        NG_LAUNCH(c, "upsweep", ng::launch_upsweep(pk, counts, s));
        NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(counts, counts, ((uint64_t)1 << sg.nbits) * nr, scan_tmp,
                                                        nullptr, s));
        NG_LAUNCH(c, "downsweep", ng::launch_downsweep(pk, counts, s));
      }
      return NG_OK;
    };
    auto block_len = [&](uint32_t b) -> uint32_t {
      const uint64_t a = (uint64_t)b * B;
      return (uint32_t)std::min<uint64_t>(B, N - a);
    };
    std::vector<ng::CopySeg> lists;
    // (B) every block sorted: packed into the auxiliary array, sorted back
    for (uint32_t b = 0; b < k; ++b) lists.push_back(ng::CopySeg{(uint32_t)((uint64_t)b * B), 0, block_len(b), 0});
    if (k) {
      if (int rc = stage_upload(c, d_lists, lists.data(), sizeof(ng::CopySeg) * lists.size())) return rc;
    }
    for (uint32_t b = 0; b < k; ++b) {
      NG_LAUNCH_N(c, "copass_copy", block_len(b),
                  ng::launch_copass_copy(view, ng::CopyList{d_lists + b, 1, block_len(b)}, true, aux_k, aux_p, s));
      if (int rc = sort_into(b, block_len(b))) return rc;
    }
    // the remaining region holds k sorted subarrays; block b = 0, 1, ... is
    // extracted in turn
    std::vector<uint32_t> start(k), len(k), mi(k), st(4);
    for (uint32_t i = 0; i < k; ++i) {
      start[i] = (uint32_t)((uint64_t)i * B);
      len[i] = block_len(i);
    }
    for (uint32_t b = 0; b < (k > 1 ? k : 0); ++b) {  // one block: sorted above
      const uint32_t first = (uint32_t)((uint64_t)b * B), m = block_len(b);
      const uint64_t remaining = N - first;
      if (m < remaining) {
        std::vector<uint32_t> sl(2ull * k);
        std::copy(start.begin(), start.end(), sl.begin());
        std::copy(len.begin(), len.end(), sl.begin() + k);
        if (int rc = stage_upload(c, d_start, sl.data(), 8ull * k)) return rc;
        ng::CopassPart pp{view, d_start, d_len, k, m, d_lo, d_hi, d_mulo, d_muhi, d_mout, d_status};
        NG_LAUNCH(c, "copass_partition", ng::launch_copass_partition(pp, s));
        uint32_t* h = c->h_words;  // k + 3 words, held since the calibration began
        NG_HIP(c, hipMemcpyAsync(h, d_mout, 4ull * k, hipMemcpyDeviceToHost, s), "partition sizes");
        NG_HIP(c, hipMemcpyAsync(h + k, d_status, 12, hipMemcpyDeviceToHost, s), "partition status");
        NG_HIP(c, hipStreamSynchronize(s), "partition");
        std::copy(h, h + k, mi.begin());
        std::copy(h + k, h + k + 3, st.begin());
        uint64_t sum = 0;
        bool bad = st[2] != 0 || (st[0] != 1 && st[0] != 2);
        for (uint32_t i = 0; i < k && !bad; ++i) {
          bad = mi[i] > len[i];
          sum += mi[i];
        }
        if (bad || sum != m) return dev_fail(c, hipErrorUnknown, "COPASS partition did not converge");
      } else {
        mi = len;
      }
      lists.clear();
      // (D) left partitions to the auxiliary array
      uint32_t q = 0;
      for (uint32_t i = 0; i < k; ++i)
        if (mi[i]) {
          lists.push_back(ng::CopySeg{start[i], q, mi[i], q});
          q += mi[i];
        }
      const uint32_t n_gather = (uint32_t)lists.size();
      // (E) right partitions shifted to the end, last subarray last: new
      // positions, and the moves of those that shift
      std::vector<uint32_t> nstart(k), nlen(k);
      uint64_t e = N;
      for (uint32_t i = k; i-- > 0;) {
        nlen[i] = len[i] - mi[i];
        e -= nlen[i];
        nstart[i] = (uint32_t)e;
      }
      struct Move {
        uint32_t src, dst, len;
      };
      std::vector<Move> moves;
      for (uint32_t i = 0; i < k; ++i)
        if (nlen[i] && start[i] + mi[i] != nstart[i]) moves.push_back(Move{start[i] + mi[i], nstart[i], nlen[i]});
      // chunks of at most one block, from the end: each is read into the
      // bounce buffer, then written; the sources of lower chunks lie below
      // the chunk, so no chunk overwrites what a later one reads
      struct Chunk {
        uint32_t off, n, total;
      };
      std::vector<Chunk> chunks;
      uint64_t ce = N;
      const uint64_t lo_end = (uint64_t)first + m;
      while (ce > lo_end && !moves.empty()) {
        const uint64_t cs = ce > lo_end + A ? ce - A : lo_end;
        const uint32_t off = (uint32_t)lists.size();
        uint32_t pre = 0;
        // the moves are disjoint and ascending: those meeting [cs, ce) are a contiguous run
        const auto first_mv = std::partition_point(moves.begin(), moves.end(),
                                                   [&](const Move& mv) { return (uint64_t)mv.dst + mv.len <= cs; });
        for (auto it = first_mv; it != moves.end() && it->dst < ce; ++it) {
          const Move& mv = *it;
          const uint64_t a = std::max<uint64_t>(mv.dst, cs), z = std::min<uint64_t>((uint64_t)mv.dst + mv.len, ce);
          if (a >= z) continue;
          lists.push_back(ng::CopySeg{(uint32_t)(mv.src + (a - mv.dst)), (uint32_t)(a - cs), (uint32_t)(z - a), pre});
          pre += (uint32_t)(z - a);
        }
        const uint32_t npiece = (uint32_t)lists.size() - off;
        for (uint32_t j = 0; j < npiece; ++j) {
          const ng::CopySeg& r = lists[off + j];
          lists.push_back(ng::CopySeg{r.dst, (uint32_t)(cs + r.dst), r.len, r.pre});
        }
        if (npiece) chunks.push_back(Chunk{off, npiece, pre});
        ce = cs;
      }
      if (lists.size() > seg_cap) return dev_fail(c, hipErrorUnknown, "COPASS copy list overflow");
      if (!lists.empty())
        if (int rc = stage_upload(c, d_lists, lists.data(), sizeof(ng::CopySeg) * lists.size())) return rc;
      NG_LAUNCH_N(c, "copass_copy", m,
                  ng::launch_copass_copy(view, ng::CopyList{d_lists, n_gather, m}, true, aux_k, aux_p, s));
      for (const Chunk& ch : chunks) {
        NG_LAUNCH_N(c, "copass_copy", ch.total,
                    ng::launch_copass_copy(view, ng::CopyList{d_lists + ch.off, ch.n, ch.total}, true, s_k[0],
                                           s_p[0], s));
        NG_LAUNCH_N(c, "copass_copy", ch.total,
                    ng::launch_copass_copy(view, ng::CopyList{d_lists + ch.off + ch.n, ch.n, ch.total}, false,
                                           s_k[0], s_p[0], s));
      }
      // (F) the auxiliary array sorted into block b
      if (int rc = sort_into(b, m)) return rc;
      start = nstart;
      len = nlen;
    }
    // group index over the sorted blocks
    ng::GiPack gp{};
    ng::GiSeg gs{};
    gs.blocks = tab;
    gs.n = N;
    gs.bitmap = g.bitmap;
    gs.group_start = g.gstart;
    gs.group_src = g.group_src;
    gs.group_ptr = g.gptr;
    gs.n_groups = c->d_scalars;
    gs.tile0 = 0;
    gs.n_tiles = (uint32_t)g.gi_tiles;
    gs.n_nodes = g.nn;
    gs.ptr_block0 = 0;
    gs.n_ptr_blocks = ng::gi_ptr_blocks(g.nn);
    gp.one = gs;
    gp.n_segs = 1;
    gp.total_tiles = gs.n_tiles;
    gp.total_ptr_blocks = gs.n_ptr_blocks;
    gp.log2B = c->log2B;
    NG_LAUNCH(c, "group_flags", ng::launch_group_flags(gp, tile_flags, s));
    NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(tile_flags, tile_flags, g.gi_tiles, scan_tmp,
                                                    tile_flags + g.gi_tiles, s));
    NG_LAUNCH(c, "group_write", ng::launch_group_write(gp, tile_flags, s));
    NG_LAUNCH(c, "group_ptr", ng::launch_group_ptr(gp, tile_flags, s));
    return NG_OK;
  };
  if (int rc = run()) {
    // scratch stays with the context's deferred frees; device state unknown
    for (auto& it : as.items) ctx_free(c, it.first, it.second);
    ctx_free(c, (char*)g.gptr, g.gp_bytes);
    ctx_free(c, (char*)g.gstart, g.gs_bytes);
    return rc;
  }
  for (auto& it : as.items) ctx_free(c, it.first, it.second);
  c->d_group_ptr = g.gptr;
  c->group_ptr_bytes = g.gp_bytes;
  c->d_group_start = g.gstart;
  c->group_start_bytes = g.gs_bytes;
  c->gi_nodes = g.nn;
  c->calibrated = true;
  ctx_flush_frees(c);
  return NG_OK;
}

// Digit plan of the most-significant-digit calibration (keys of at most 27
// bits, see ng_internal.h).  The last digit (pass C, in LDS) is as wide as
// keeps an average occupied sub-bucket at about half of what one LDS piece
// holds; the keys only occupy [0, n_nodes << dbits), so that range, not
// 2^keybits, sets the occupancy.  The remaining bits go to pass A alone when
// they fit one digit, else are split between A and B so that the occupied
// values of D1 and the values of D2 balance (both set the run lengths of
// their scatter).  False if the plan does not apply (the LSD sort runs).
bool msd_geometry(uint64_t N, uint32_t nn, int dbits, int log2B, uint32_t sort_ranges, ng::MsdPlan& p,
                  uint32_t msd_tile = 0) {
  const int sbits = bitwidth(nn > 0 ? nn - 1 : 0);
  const int K = sbits + dbits;
  if (N == 0 || N > 0xFFFFFFFFull || K < 2 || K > (int)ng::kMsdMaxKeyBits) return false;
  const uint32_t tbits = (uint32_t)std::max(1, sbits);
  const uint64_t keyspace = (uint64_t)nn << dbits;
  const uint64_t cap = ng::msd_cap(tbits + ng::kMsdMaxDigit <= 32);
  int b3 = 0;
  while (b3 < 9 && ((keyspace * (cap / 2)) >> (b3 + 1)) >= N) ++b3;
  b3 = std::max(b3, std::max(1, K - 18));
  b3 = std::min(b3, std::min(9, K - 1));
  const int hb = K - b3;
  int b1 = hb, b2 = 0;
  if (hb > 9) {
    uint64_t best = ~0ull;
    for (int t = std::max(1, hb - 9); t <= std::min(9, hb - 1); ++t) {
      const uint64_t occ1 = (keyspace + (1ull << (t + b3)) - 1) >> (t + b3);
      const uint64_t cost = std::max<uint64_t>(occ1, 1ull << t);
      if (cost < best) {
        best = cost;
        b2 = t;
      }
    }
    b1 = hb - b2;
  }
  p = ng::MsdPlan{};
  p.n = (uint32_t)N;
  p.keybits = (uint32_t)K;
  p.dbits = (uint32_t)dbits;
  p.tbits = tbits;
  p.b1 = (uint32_t)b1;
  p.b2 = (uint32_t)b2;
  p.b3 = (uint32_t)b3;
  p.narrow_a = (uint32_t)(b2 + b3) + tbits <= 32 ? 1u : 0u;
  p.narrow_b = (uint32_t)b3 + tbits <= 32 ? 1u : 0u;
  // packed records entering pass C hold D3 and as many D2 bits as fit
  p.cbits = (uint32_t)b3;
  if (b2 && p.narrow_a) p.cbits = (uint32_t)(b2 + b3);
  else if (b2 && p.narrow_b) p.cbits = std::min<uint32_t>((uint32_t)(b2 + b3), 32u - tbits);
  const uint64_t tile = ng::kMsdTile;
  const uint64_t ntiles = (N + tile - 1) / tile;
  p.tpr = (uint32_t)std::max<uint64_t>(1, (ntiles + sort_ranges - 1) / std::max<uint32_t>(sort_ranges, 1));
  p.ranges_a = (uint32_t)((ntiles + p.tpr - 1) / p.tpr);
  p.tile_b = p.narrow_a && msd_tile != ng::kMsdTile ? ng::kMsdTileN : ng::kMsdTile;
  // each bucket asks for ceil(its tiles x ranges_b / all tiles) ranges;
  // three times the ranges of pass A (measured on the 3e8 microcircuit's
  // second scatter: as many as pass A 1.99 ms, twice 1.69, 2.5x 1.66, three
  // times 1.60, 3.5x 1.73, four times 1.70; the 1.54e8 two-population
  // network's: 0.78 ms at three times against 0.83 at twice)
  p.ranges_b = 3 * std::max<uint32_t>(sort_ranges, 1);
  p.max_ranges_b = b2 ? (uint32_t)(p.ranges_b + (1ull << b1)) : 0u;
  // pass C: workgroups of about six LDS loads of records each (measured:
  // 3e8 microcircuit 1.90 -> 1.88 ms against eight, 1.54e8 two-population
  // network 1.10 -> 1.06 ms; two loads: no gain; sixteen: 1.97 ms), and at
  // least 1,024 (four per CU) so that short tiles of few records -- small or
  // sparse calibrations -- still spread over the chip; no more workgroups
  // than sub-buckets
  const uint64_t piece = ng::msd_cap(b2 ? p.narrow_b : p.narrow_a);
  const uint64_t nsb = 1ull << (b1 + b2);
  p.wgs_c = (uint32_t)std::min<uint64_t>(
      std::max<uint64_t>(1, std::min<uint64_t>(std::max<uint64_t>((N + 6 * piece - 1) / (6 * piece), 1024), nsb)),
      1u << 20);
  p.max_big = (uint32_t)(N / (piece + 1) + 1);
  p.n_nodes = nn;
  p.log2B = log2B;
  p.mask_words = std::max<uint32_t>(1, (1u << b3) / 32);
  return true;
}

// The default radix calibration takes the most-significant-digit form when
// (1) there are at least 2^25 connections: below, the LSD passes are faster
// (measured on MI355X: 0.94 against 1.04 ms at 3e7 connections over 77,169
// nodes, 2.9 against 2.3 ms at 1e8); (2) the sub-buckets it must visit hold
// 256 connections on average or more (fewer connections over a wide key
// leave most sub-buckets empty); and (3) the 512 keys that one LDS tile can
// tell apart hold at least half a tile of connections (n >= 10 connections
// per possible key: otherwise pass C sorts nearly empty tiles).
bool msd_pays(const ng::MsdPlan& p) {
  const uint64_t keyspace = (uint64_t)p.n_nodes << p.dbits;
  return p.n >= (1u << 25) && (uint64_t)p.n >= (256ull << (p.b1 + p.b2)) &&
         (uint64_t)p.n * 512 >= keyspace * (ng::kMsdTile / 2);
}

// Calibration of one context by the most-significant-digit sort: count and
// scatter by D1 (A), count and scatter each bucket by D2 (B), each
// sub-bucket sorted by D3 in LDS into the calibrated blocks with its groups
// (C), then group_start and group_ptr (Eq. (14)).  Every launch size is an
// upper bound computed on the host; the bucket layout stays on the device.
int calibrate_msd(CalSeg& g, const ng::MsdPlan& plan) {
  ng_ctx* c = g.c;
  ng::MsdPlan p = plan;
  const uint64_t N = g.N;
  const uint64_t nb = 1ull << p.b1, nsb = 1ull << (p.b1 + p.b2);
  AllocSet as(c);
  const uint64_t nblk = (N + c->B - 1) / c->B;
  for (uint64_t b = 0; b < nblk && as.ok; ++b) g.nblocks.push_back(as.get(ng::kBytesPerConn * c->B));
  const uint64_t first_scratch = g.nblocks.size();
  p.a_key = (uint32_t*)as.get(4 * N);
  p.a_w = (uint32_t*)as.get(4 * N);
  p.a_tgt = p.narrow_a ? nullptr : (uint32_t*)as.get(4 * N);
  if (p.b2) {
    p.b_key = (uint32_t*)as.get(4 * N);
    p.b_w = (uint32_t*)as.get(4 * N);
    p.b_tgt = p.narrow_b ? nullptr : (uint32_t*)as.get(4 * N);
    p.gslot = p.a_key;  // pass C reads B's records; A's keys are dead by then
  } else {
    p.gslot = (uint32_t*)as.get(4 * N);
  }
  const uint64_t na = nb * p.ranges_a, nbc = p.b2 ? ((uint64_t)p.max_ranges_b << p.b2) : 0;
  p.cnt_a = (uint32_t*)as.get(4 * na);
  p.cnt_b = p.b2 ? (uint32_t*)as.get(4 * nbc) : nullptr;
  uint32_t* scan_tmp =
      (uint32_t*)as.get(4 * std::max({ng::scan_tmp_words(na), ng::scan_tmp_words(nbc), ng::scan_tmp_words(nsb)}));
  p.bstart = (uint32_t*)as.get(4 * (nb + 1));
  p.rangeb0 = (uint32_t*)as.get(4 * (nb + 1));
  p.tprb = (uint32_t*)as.get(4 * nb);
  p.sbstart = (uint32_t*)as.get(4 * (nsb + 1));
  p.gcount = (uint32_t*)as.get(4 * (nsb + 1));
  p.gmask = (uint32_t*)as.get(4 * nsb * p.mask_words);
  p.wg_sb0 = (uint32_t*)as.get(4 * ((uint64_t)p.wgs_c + 1));
  p.big_count = (uint32_t*)as.get(4);
  p.big_list = (uint32_t*)as.get(4 * (uint64_t)p.max_big);
  g.gp_bytes = 4 * (g.nn + 1ull);
  g.gs_bytes = 4 * g.gcap;
  release_index(c);
  c->calibrated = false;
  g.gptr = (uint32_t*)ctx_alloc(c, g.gp_bytes);
  g.gstart = g.gptr ? (uint32_t*)ctx_alloc(c, g.gs_bytes) : nullptr;
  if (!as.ok || !g.gptr || !g.gstart) {
    as.release_all();
    ctx_unalloc(c, (char*)g.gptr, g.gp_bytes);
    ctx_unalloc(c, (char*)g.gstart, g.gs_bytes);
    g.nblocks.clear();
    c->need = as.asked + Arena::round_up(g.gp_bytes) + Arena::round_up(g.gs_bytes);
    return fail(NG_ERR_OOM, "arena cannot hold the calibration buffers (N=%llu)", (unsigned long long)N);
  }
  g.nxt = 1 - c->cur;
  p.in_blocks = c->d_tab[c->cur];
  p.out_blocks = c->d_tab[g.nxt];
  p.group_ptr = g.gptr;
  p.group_start = g.gstart;
  p.n_groups = c->d_scalars;

  hipStream_t s = c->stream;
  if (int rc = sync_table(c)) return rc;
  NG_HIP(c, set_table(c->d_tab[g.nxt], 0, g.nblocks, 0, s), "block table");
  NG_LAUNCH_N(c, "msd_count_a", N, ng::launch_msd_count_a(p, s));
  NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(p.cnt_a, p.cnt_a, na, scan_tmp, nullptr, s));
  NG_LAUNCH_N(c, "msd_scatter_a", N, ng::launch_msd_scatter_a(p, s));
  NG_LAUNCH(c, "msd_plan", ng::launch_msd_plan_b(p, s));
  if (p.b2) {
    NG_LAUNCH_N(c, "msd_count_b", N, ng::launch_msd_count_b(p, s));
    NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(p.cnt_b, p.cnt_b, nbc, scan_tmp, nullptr, s));
    NG_LAUNCH_N(c, "msd_scatter_b", N, ng::launch_msd_scatter_b(p, s));
  }
  NG_LAUNCH(c, "msd_plan", ng::launch_msd_plan_c(p, s));
  NG_LAUNCH_N(c, "msd_tiles_c", N, ng::launch_msd_tiles_c(p, s));
  NG_LAUNCH(c, "msd_big_c", ng::launch_msd_big_c(p, s));
  NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(p.gcount, p.gcount, nsb, scan_tmp, p.gcount + nsb, s));
  NG_LAUNCH(c, "msd_groups", ng::launch_msd_groups(p, s));

  // old storage and scratch return to the arena (ordered after the launches)
  for (char* b : c->blocks) ctx_free(c, b, ng::kBytesPerConn * c->B);
  for (size_t i = first_scratch; i < as.items.size(); ++i) ctx_free(c, as.items[i].first, as.items[i].second);
  c->blocks = g.nblocks;
  c->tab_synced = (uint32_t)g.nblocks.size();
  c->cur = g.nxt;
  c->d_group_ptr = g.gptr;
  c->group_ptr_bytes = g.gp_bytes;
  c->d_group_start = g.gstart;
  c->group_start_bytes = g.gs_bytes;
  c->gi_nodes = g.nn;
  c->calibrated = true;
  if (!c->capturing) ctx_flush_frees(c);
  return NG_OK;
}

}  // namespace

int calibrate_many(ng_ctx* const* cs, uint32_t n, const Uploader* upload, ScratchBump* sb) {
  if (n == 0) return NG_OK;
  if (!cs) return fail(NG_ERR_INVALID_ARG, "null context array");
  if (sb && n != 1) return fail(NG_ERR_INVALID_ARG, "internal: fixed scratch serves one context");
  for (uint32_t i = 0; i < n; ++i) {
    if (int rc = enter(cs[i])) return rc;
    if (int rc = mutable_state(cs[i])) return rc;
    for (uint32_t j = 0; j < i; ++j)
      if (cs[j] == cs[i]) return fail(NG_ERR_INVALID_ARG, "a context appears twice");
    if (n > 1) {
      if (cs[i]->capturing) return fail(NG_ERR_STATE, "packed calibration cannot be captured");
      if (cs[i]->device != cs[0]->device) return fail(NG_ERR_INVALID_ARG, "contexts on different devices");
      if (cs[i]->log2B != cs[0]->log2B) return fail(NG_ERR_INVALID_ARG, "contexts with different block sizes");
    }
  }
  // (the fixed-scratch form allocates nothing: its queued calls launch one by one)
  for (uint32_t i = 0; i < n; ++i)
    if (int rc = flush_connects(cs[i], sb == nullptr)) return rc;
  // contexts in COPASS mode, one by one
  for (uint32_t i = 0; i < n; ++i)
    if (!cs[i]->calibrated && cs[i]->calib_mode == NG_CALIB_COPASS) {
      if (hipSetDevice(cs[i]->device) != hipSuccess) return fail(NG_ERR_DEVICE, "hipSetDevice");
      if (int rc = calibrate_copass(cs[i])) return rc;
    }
  std::vector<CalSeg> segs;
  for (uint32_t i = 0; i < n; ++i)
    if (!cs[i]->calibrated) {
      segs.emplace_back();
      segs.back().c = cs[i];
    }
  if (segs.empty()) return NG_OK;
  if (hipSetDevice(segs[0].c->device) != hipSuccess) return fail(NG_ERR_DEVICE, "hipSetDevice");
  for (auto& g : segs) {
    if (int rc = cal_plan(g)) return rc;
    g.sb = sb;
  }
  // one context with its own scratch: the most-significant-digit sort when
  // its keys fit
  if (segs.size() == 1 && !sb &&
      (segs[0].c->calib_mode == NG_CALIB_RADIX || segs[0].c->calib_mode == NG_CALIB_RADIX_MSD)) {
    ng::MsdPlan mp;
    const CalSeg& g = segs[0];
    if (msd_geometry(g.N, g.nn, g.dbits, g.c->log2B, g.c->sort_ranges, mp, g.c->msd_tile) &&
        (g.c->calib_mode == NG_CALIB_RADIX_MSD || msd_pays(mp)))
      return calibrate_msd(segs[0], mp);
  }
  ng_ctx* c0 = segs[0].c;
  const bool multi = segs.size() > 1;

  // sort packs: segments with records, grouped by their number of passes
  std::map<int, std::vector<uint32_t>> packs;
  for (uint32_t k = 0; k < segs.size(); ++k)
    if (segs[k].N > 0) packs[segs[k].passes].push_back(k);
  uint64_t counts_max = 0, tables = 0;
  for (auto& pr : packs) {
    uint64_t ranges = 0;
    for (uint32_t k : pr.second) ranges += segs[k].n_ranges;
    if (ranges > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "too many sort ranges");
    for (int p = 0; p < pr.first; ++p) {
      uint64_t cn = 0;
      for (uint32_t k : pr.second) cn += ((uint64_t)1 << segs[k].nbits[p]) * segs[k].n_ranges;
      counts_max = std::max(counts_max, cn);
    }
    tables += align256(sizeof(ng::SortSeg) * pr.second.size() * pr.first) + align256(4 * ranges);
  }
  uint64_t total_tiles = 0, total_ptr_blocks = 0;
  for (auto& g : segs) {
    total_tiles += g.gi_tiles;
    total_ptr_blocks += ng::gi_ptr_blocks(g.nn);
  }
  if (total_tiles >= 0xFFFFFFFFull || total_ptr_blocks >= 0xFFFFFFFFull)
    return fail(NG_ERR_TOO_LARGE, "too many index tiles");
  tables += align256(sizeof(ng::GiSeg) * segs.size()) + align256(4 * total_tiles) + align256(4 * total_ptr_blocks);
  // block-table entries, written by one launch: the unwritten ones of each
  // current table (pass 0 reads it) and every one of each new table
  uint64_t n_entries = 0;
  for (auto& g : segs) n_entries += (g.c->blocks.size() - g.c->tab_synced) + (g.N + g.c->B - 1) / g.c->B;
  tables += align256(sizeof(ng::TabEntry) * n_entries);
  if (!multi) tables = 0;

  // allocation: per-context buffers, then the shared scratch from the first
  for (size_t k = 0; k < segs.size(); ++k) {
    if (int rc = cal_alloc(segs[k])) {
      for (size_t j = 0; j < k; ++j) cal_release(segs[j]);
      return rc;
    }
  }
  AllocSet shared(c0);
  auto sget = [&](uint64_t bytes) { return sb ? sb->get(bytes) : shared.get(bytes); };
  uint32_t* counts = (uint32_t*)sget(4 * std::max<uint64_t>(counts_max, 1));
  const uint64_t tmp_words = std::max(ng::scan_tmp_words(counts_max), ng::scan_tmp_words(total_tiles));
  uint32_t* scan_tmp = (uint32_t*)sget(4 * tmp_words);
  uint32_t* tile_flags = (uint32_t*)sget(4 * (total_tiles + 1));
  char* d_tables = tables ? shared.get(tables) : nullptr;
  if (sb && !sb->ok) {
    for (auto& g : segs) cal_release(g);
    return fail(NG_ERR_TOO_LARGE, "the calibration scratch exceeds the fixed %llu-byte region",
                (unsigned long long)sb->cap);
  }
  if (!shared.ok) {
    const uint64_t asked = shared.asked;
    shared.release_all();
    for (auto& g : segs) cal_release(g);
    c0->need = asked;
    return fail(NG_ERR_OOM, "arena cannot hold the calibration scratch");
  }

  // host images of the pack descriptors
  struct PackLaunch {
    int passes;
    std::vector<ng::SortPack> pass;
    std::vector<uint64_t> counts_n;
  };
  std::vector<PackLaunch> launches;
  std::vector<char> h_tables(tables);
  uint64_t toff = 0;
  for (auto& pr : packs) {
    const int P = pr.first;
    const std::vector<uint32_t>& ks = pr.second;
    PackLaunch pl;
    pl.passes = P;
    uint32_t total_ranges = 0;
    std::vector<uint32_t> range0(ks.size());
    for (size_t i = 0; i < ks.size(); ++i) {
      range0[i] = total_ranges;
      total_ranges += segs[ks[i]].n_ranges;
    }
    ng::SortSeg* h_segs = nullptr;
    uint32_t* h_sor = nullptr;
    const ng::SortSeg* d_segs = nullptr;
    const uint32_t* d_sor = nullptr;
    if (multi) {
      h_segs = reinterpret_cast<ng::SortSeg*>(h_tables.data() + toff);
      d_segs = reinterpret_cast<const ng::SortSeg*>(d_tables + toff);
      toff += align256(sizeof(ng::SortSeg) * ks.size() * P);
      h_sor = reinterpret_cast<uint32_t*>(h_tables.data() + toff);
      d_sor = reinterpret_cast<const uint32_t*>(d_tables + toff);
      toff += align256(4 * (uint64_t)total_ranges);
      for (size_t i = 0; i < ks.size(); ++i)
        for (uint32_t r = 0; r < segs[ks[i]].n_ranges; ++r) h_sor[range0[i] + r] = (uint32_t)i;
    }
    for (int p = 0; p < P; ++p) {
      ng::SortPack pk{};
      uint64_t cbase = 0, before = 0;
      for (size_t i = 0; i < ks.size(); ++i) {
        ng::SortSeg sg = sort_seg(segs[ks[i]], p);
        sg.range0 = range0[i];
        sg.cbase = cbase;
        sg.base = (uint32_t)before;  // mod 2^32, as the u32 scan wraps
        cbase += ((uint64_t)1 << sg.nbits) * sg.n_ranges;
        before += sg.n;
        pk.max_nbits = std::max(pk.max_nbits, sg.nbits);
        if (i == 0) pk.one = sg;
        if (multi) h_segs[(size_t)p * ks.size() + i] = sg;
      }
      pk.n_segs = (uint32_t)ks.size();
      pk.total_ranges = total_ranges;
      pk.ranges_per_xcd = (total_ranges + 7) / 8;
      if (multi) {
        pk.segs = d_segs + (size_t)p * ks.size();
        pk.seg_of_range = d_sor;
      }
      pl.pass.push_back(pk);
      pl.counts_n.push_back(cbase);
    }
    launches.push_back(std::move(pl));
  }
  ng::GiPack gp{};
  {
    ng::GiSeg* h_gs = nullptr;
    uint32_t *h_sot = nullptr, *h_sopb = nullptr;
    if (multi) {
      h_gs = reinterpret_cast<ng::GiSeg*>(h_tables.data() + toff);
      gp.segs = reinterpret_cast<const ng::GiSeg*>(d_tables + toff);
      toff += align256(sizeof(ng::GiSeg) * segs.size());
      h_sot = reinterpret_cast<uint32_t*>(h_tables.data() + toff);
      gp.seg_of_tile = reinterpret_cast<const uint32_t*>(d_tables + toff);
      toff += align256(4 * total_tiles);
      h_sopb = reinterpret_cast<uint32_t*>(h_tables.data() + toff);
      gp.seg_of_ptr_block = reinterpret_cast<const uint32_t*>(d_tables + toff);
      toff += align256(4 * total_ptr_blocks);
    }
    uint32_t tile0 = 0, pb0 = 0;
    for (size_t k = 0; k < segs.size(); ++k) {
      const CalSeg& g = segs[k];
      ng::GiSeg s{};
      s.blocks = g.c->d_tab[g.nxt];
      s.n = g.N;
      s.bitmap = g.bitmap;
      s.group_start = g.gstart;
      s.group_src = g.group_src;
      s.group_ptr = g.gptr;
      s.n_groups = g.c->d_scalars;
      s.tile0 = tile0;
      s.n_tiles = (uint32_t)g.gi_tiles;
      s.n_nodes = g.nn;
      s.ptr_block0 = pb0;
      s.n_ptr_blocks = ng::gi_ptr_blocks(g.nn);
      if (multi) {
        h_gs[k] = s;
        for (uint32_t t = 0; t < s.n_tiles; ++t) h_sot[tile0 + t] = (uint32_t)k;
        for (uint32_t b = 0; b < s.n_ptr_blocks; ++b) h_sopb[pb0 + b] = (uint32_t)k;
      }
      if (k == 0) gp.one = s;
      tile0 += s.n_tiles;
      pb0 += s.n_ptr_blocks;
    }
    gp.n_segs = (uint32_t)segs.size();
    gp.total_tiles = tile0;
    gp.total_ptr_blocks = pb0;
    gp.log2B = c0->log2B;
  }
  const ng::TabEntry* d_entries = nullptr;
  std::vector<uint32_t> synced_before;
  for (auto& g : segs) synced_before.push_back(g.c->tab_synced);
  if (multi) {
    std::vector<ng::TabEntry> entries;
    for (auto& g : segs) {
      take_table_entries(g.c, entries);
      for (uint32_t b = 0; b < g.nblocks.size(); ++b)
        entries.push_back(ng::TabEntry{g.c->d_tab[g.nxt], g.nblocks[b], b, 0});
    }
    memcpy(h_tables.data() + toff, entries.data(), sizeof(ng::TabEntry) * entries.size());
    d_entries = reinterpret_cast<const ng::TabEntry*>(d_tables + toff);
    toff += align256(sizeof(ng::TabEntry) * entries.size());
    n_entries = entries.size();
  }

  // launches, all on the first context's stream
  hipStream_t s = c0->stream;
  if (multi) {
    // the other streams' pending work (the segments' connects) comes first
    int rc = NG_OK;
    for (auto& g : segs)
      if (rc == NG_OK && g.c->stream != s &&
          (hipEventRecord(g.c->order_ev, g.c->stream) != hipSuccess ||
           hipStreamWaitEvent(s, g.c->order_ev, 0) != hipSuccess))
        rc = dev_fail(c0, hipErrorUnknown, "stream ordering");
    if (rc == NG_OK)
      rc = upload ? (*upload)(s, d_tables, h_tables.data(), tables)
                  : stage_upload(c0, d_tables, h_tables.data(), tables);
    if (rc != NG_OK) {  // nothing has used the new buffers yet
      shared.release_all();
      for (size_t k = 0; k < segs.size(); ++k) segs[k].c->tab_synced = synced_before[k];
      for (auto& g : segs) cal_release(g);
      return rc == NG_ERR_DEVICE || rc == NG_ERR_OOM ? rc : fail(rc, "packed calibration upload failed");
    }
  }
  auto run = [&]() -> int {
    if (multi) {
      NG_HIP(c0, ng::launch_set_entries(d_entries, (uint32_t)n_entries, s), "block tables");
    } else {
      if (int rc = sync_table(c0)) return rc;
      NG_HIP(c0, set_table(c0->d_tab[segs[0].nxt], 0, segs[0].nblocks, 0, s), "block table");
    }
    for (auto& pl : launches)
      for (int p = 0; p < pl.passes; ++p) {
        NG_LAUNCH(c0, "upsweep", ng::launch_upsweep(pl.pass[p], counts, s));
        NG_LAUNCH(c0, "scan", ng::launch_exclusive_scan(counts, counts, pl.counts_n[p], scan_tmp, nullptr, s));
        NG_LAUNCH(c0, "downsweep", ng::launch_downsweep(pl.pass[p], counts, s));
      }
    NG_LAUNCH(c0, "group_flags", ng::launch_group_flags(gp, tile_flags, s));
    NG_LAUNCH(c0, "scan", ng::launch_exclusive_scan(tile_flags, tile_flags, total_tiles, scan_tmp,
                                                     tile_flags + total_tiles, s));
    NG_LAUNCH(c0, "group_write", ng::launch_group_write(gp, tile_flags, s));
    NG_LAUNCH(c0, "group_ptr", ng::launch_group_ptr(gp, tile_flags, s));
    if (multi) {
      NG_HIP(c0, hipEventRecord(c0->order_ev, s), "event");
      for (auto& g : segs)
        if (g.c->stream != s) NG_HIP(c0, hipStreamWaitEvent(g.c->stream, c0->order_ev, 0), "stream wait");
    }
    return NG_OK;
  };
  if (int rc = run()) {
    // device state of every context is now unknown
    for (auto& g : segs)
      if (g.c != c0 && c0->sticky != NG_OK) {
        g.c->sticky = c0->sticky;
        g.c->sticky_msg = c0->sticky_msg;
      }
    return rc;
  }

  // old storage and scratch return to the arenas (ordered after the launches)
  for (auto& g : segs) {
    ng_ctx* c = g.c;
    for (char* b : c->blocks) ctx_free(c, b, ng::kBytesPerConn * c->B);
    const size_t nblk = g.nblocks.size();
    for (size_t i = nblk; i < g.as->items.size(); ++i) ctx_free(c, g.as->items[i].first, g.as->items[i].second);
    c->blocks = g.nblocks;
    c->tab_synced = (uint32_t)g.nblocks.size();  // the new table was written above
    c->cur = g.nxt;
    c->d_group_ptr = g.gptr;
    c->group_ptr_bytes = g.gp_bytes;
    c->d_group_start = g.gstart;
    c->group_start_bytes = g.gs_bytes;
    c->gi_nodes = g.nn;
    c->calibrated = true;
  }
  for (auto& it : shared.items) ctx_free(c0, it.first, it.second);
  if (!c0->capturing)
    for (auto& g : segs) ctx_flush_frees(g.c);
  return NG_OK;
}


void connect_commit(ng_ctx* c, const ng::GenDesc& d, int32_t max_delay) {
  c->next_cid++;
  c->n_conns += d.n_new;
  c->max_delay = std::max(c->max_delay, max_delay);
  if (d.n_new) c->calibrated = false;
}

int flush_connects(ng_ctx* c, bool batched) {
  if (c->queued.empty()) return NG_OK;
  std::vector<ng::GenDesc> q;
  q.swap(c->queued);
  const uint64_t groups = c->queued_groups;
  c->queued_groups = 0;
  if (int rc = sync_table(c)) return rc;
  const uint64_t bytes = q.size() * sizeof(ng::GenDesc);
  char* d_descs = batched ? ctx_alloc(c, bytes) : nullptr;
  if (d_descs && stage_upload(c, d_descs, q.data(), bytes) != NG_OK) {
    ctx_unalloc(c, d_descs, bytes);
    d_descs = nullptr;
  }
  if (!d_descs) {  // no room for the descriptors: one launch per call, arguments by value
    for (const auto& d : q)
      NG_LAUNCH_N(c, "generate", d.n_new, ng::launch_generate(d, key_ptr(c), d.blocks, c->log2B, c->stream, c->gen_quads));
    return NG_OK;
  }
  uint64_t syn = 0;
  for (const auto& d : q) syn += d.n_new;
  NG_LAUNCH_N(c, "generate_batch", syn,
              ng::launch_generate_batch((const ng::GenDesc*)d_descs, (uint32_t)q.size(), groups, c->log2B, c->stream,
                                        c->gen_quads));
  ctx_free(c, d_descs, bytes);  // stream-ordered reuse is safe
  if (!c->capturing) ctx_flush_frees(c);
  return NG_OK;
}

}  // namespace ngrt

using namespace ngrt;

extern "C" {

const char* ng_version(void) { return "ng 0.1 gfx950"; }

const char* ng_last_error(void) { return g_err.c_str(); }

int ng_calibration_plan(uint64_t n_conns, uint32_t n_nodes, int32_t max_delay, uint32_t sort_ranges,
                        uint32_t out[8]) {
  if (!out || max_delay < 1) return fail(NG_ERR_INVALID_ARG, "null output or max_delay < 1");
  for (int i = 0; i < 8; ++i) out[i] = 0;
  ng::MsdPlan p;
  if (!msd_geometry(n_conns, n_nodes, bitwidth((uint64_t)max_delay), 24, sort_ranges ? sort_ranges : 1024, p))
    return NG_OK;
  const uint32_t v[8] = {msd_pays(p) ? 2u : 1u, p.b1, p.b2, p.b3, p.narrow_a, p.narrow_b, p.wgs_c, p.tpr};
  for (int i = 0; i < 8; ++i) out[i] = v[i];
  return NG_OK;
}

uint64_t ng_blocks_needed(uint64_t n_conns, uint64_t n_new, uint64_t block_size, uint64_t n_blocks) {
  if (block_size == 0) return 0;
  const uint64_t need = (n_conns + n_new + block_size - 1) / block_size;  // Eq. (1)
  return need > n_blocks ? need - n_blocks : 0;
}

int ng_plan_count(uint32_t n_nodes, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                  const ng_syn_spec* syn, float h_ms, uint64_t* out_n) {
  Plan p;
  const int rc = plan_call(n_nodes, src, tgt, conn, syn, h_ms > 0 ? h_ms : 0.1f, &p);
  if (rc == NG_OK && out_n) *out_n = p.n_new;
  return rc;
}

int ng_create(const ng_config* cfg, void* arena, uint64_t arena_bytes, void* stream, ng_ctx** out) {
  if (!arena || ((uintptr_t)arena % kAlign)) return fail(NG_ERR_INVALID_ARG, "arena must be 256-byte aligned");
  return ctx_init(cfg, nullptr, (char*)arena, arena_bytes, (hipStream_t)stream, out);
}

int ng_destroy(ng_ctx* c) {
  if (!c) return NG_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  ctx_host_release(c);
  delete c;
  return NG_OK;
}

int ng_create_nodes(ng_ctx* c, uint32_t n, ng_range* out) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if ((uint64_t)c->n_nodes + n > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "too many nodes");
  if (out) *out = ng_range{c->n_nodes, n};
  c->n_nodes += n;
  if (n) c->calibrated = false;  // the group index covers the old node count
  return NG_OK;
}

// pairwise_bernoulli: count the connections on the device, read the total,
// reserve exactly that many, write them.  All-or-nothing.
static int connect_pairwise(ng_ctx* c, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                            const ng_syn_spec* syn, uint32_t* out_cid, uint64_t* out_first, uint64_t* out_n) {
  if (int rc = not_capturing(c)) return rc;
  if (!(conn->p >= 0.0 && conn->p <= 1.0)) return fail(NG_ERR_INVALID_ARG, "pairwise_bernoulli needs 0 <= p <= 1");
  if (int rc = flush_connects(c)) return rc;  // the call synchronizes: queued work goes first
  // the unit counts are scanned in 32 bits: fewer than 2^32 pairs bound every count
  if ((uint64_t)src.n * tgt.n > 0xFFFFFFFFull)
    return fail(NG_ERR_TOO_LARGE, "pairwise_bernoulli takes at most 2^32-1 source-target pairs per call");
  if (!c->capturing) ctx_flush_frees(c);
  // ranges, weight and delay as for all_to_all (no connection is made here)
  ng_conn_spec a2a = *conn;
  a2a.rule = NG_ALL_TO_ALL;
  a2a.allow_multapses = 1;
  Plan pl;
  if (int rc = plan_call(c->n_nodes, src, tgt, &a2a, syn, c->cfg.h_ms, &pl)) return rc;
  if (c->next_cid == 0xFFFFFFFFu) return fail(NG_ERR_TOO_LARGE, "connect call ids exhausted");
  ng::GenDesc d = pl.d;
  d.rule = NG_PAIRWISE_BERNOULLI;
  d.p_thr = (uint64_t)std::floor(conn->p * 4294967296.0);
  d.cid = c->next_cid;
  d.no_self = !conn->allow_autapses;
  const uint64_t units = (uint64_t)src.n * ((tgt.n + ng::kPbUnit - 1) / ng::kPbUnit);
  uint64_t n = 0;
  uint32_t* counts = nullptr;
  uint64_t cbytes = 0, bits_bytes = 0;
  uint16_t* bits = nullptr;
  if (units) {
    // the count is read back through pinned words: had before any launch
    if (!host_words(c, 1)) return NG_ERR_DEVICE;
    cbytes = 4 * (units + 1);
    const uint64_t tbytes = 4 * ng::scan_tmp_words(units);
    counts = (uint32_t*)ctx_alloc(c, cbytes + tbytes);
    if (!counts) {
      c->need = Arena::round_up(cbytes + tbytes);
      return fail(NG_ERR_OOM, "arena cannot hold the pair counts");
    }
    cbytes += tbytes;
    uint32_t* tmp = counts + units + 1;
    // the decisions of the counting pass, kept for the writing pass when the
    // arena has room (one bit per pair), else evaluated again
    bits_bytes = units * (ng::kPbUnit / 8);
    bits = (uint16_t*)ctx_alloc(c, bits_bytes);
    if (!bits) bits_bytes = 0;
    NG_LAUNCH(c, "pb_count", ng::launch_pb_count(d, key_ptr(c), counts, bits, c->stream));
    NG_LAUNCH(c, "scan", ng::launch_exclusive_scan(counts, counts, units, tmp, counts + units, c->stream));
    uint32_t* h = c->h_words;  // held since before the counting pass
    NG_HIP(c, hipMemcpyAsync(h, counts + units, 4, hipMemcpyDeviceToHost, c->stream), "pair count");
    NG_HIP(c, hipStreamSynchronize(c->stream), "pair count");
    n = h[0];
  }
  if (c->n_conns + n > 0xFFFFFFFFull) {
    ctx_unalloc(c, (char*)counts, cbytes);
    ctx_unalloc(c, (char*)bits, bits_bytes);
    return fail(NG_ERR_TOO_LARGE, "a context holds at most 2^32-1 connections");
  }
  if (int rc = reserve_blocks(c, n)) {
    if (bits) {  // the decisions can be evaluated again: give their room to the blocks
      ctx_unalloc(c, (char*)bits, bits_bytes);
      bits = nullptr;
      bits_bytes = 0;
      rc = reserve_blocks(c, n);
    }
    if (rc) {
      ctx_unalloc(c, (char*)counts, cbytes);
      return rc;
    }
  }
  d.n_new = (uint32_t)n;
  d.pos0 = c->n_conns;
  if (int rc = sync_table(c)) return rc;
  if (n)
    NG_LAUNCH(c, "pb_write", ng::launch_pb_write(d, key_ptr(c), counts, bits, c->d_tab[c->cur], c->log2B, c->stream));
  ctx_free(c, (char*)counts, cbytes);
  ctx_free(c, (char*)bits, bits_bytes);
  if (out_cid) *out_cid = d.cid;
  if (out_first) *out_first = d.pos0;
  if (out_n) *out_n = n;
  connect_commit(c, d, pl.max_delay);
  return NG_OK;
}

int ng_connect(ng_ctx* c, ng_range src, ng_range tgt, const ng_conn_spec* conn, const ng_syn_spec* syn,
               uint32_t* out_cid, uint64_t* out_first, uint64_t* out_n) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (conn && conn->rule == NG_PAIRWISE_BERNOULLI) return connect_pairwise(c, src, tgt, conn, syn, out_cid, out_first, out_n);
  ng::GenDesc d;
  uint64_t n = 0;
  if (int rc = connect_prepare(c, src, tgt, conn, syn, &d, &n)) return rc;
  if (out_cid) *out_cid = d.cid;
  if (out_first) *out_first = d.pos0;
  if (out_n) *out_n = n;
  connect_commit(c, d, d.max_delay);
  // Calls below kQueuedCallMax synapses wait in the queue and go out as one
  // launch: each launch's ramp and the gaps between launches cost more than
  // a small call's work (the microcircuit's 64 calls: 1.43 ms of generation
  // in 64 launches, 1.05 ms in one).  Larger calls launch at once in the
  // kernel of their own rule, and the queue keeps waiting: each call writes
  // its own positions, so generation launches may run in any order (the
  // microcircuit: 7.19 ms per build with its 60 small calls in one launch,
  // 7.29 with the queue launched before each of its 4 large calls).  Under
  // graph capture (the graph records each launch; the queue went out when
  // the capture began) every call launches at once.
  if (n == 0) return NG_OK;
  if (!c->capturing && n < kQueuedCallMax && c->queued_max > 0) {
    d.group0 = c->queued_groups;
    c->queued_groups += (n + 3) / 4;
    c->queued.push_back(d);
    return c->queued.size() >= c->queued_max ? flush_connects(c) : NG_OK;
  }
  if (int rc = sync_table(c)) return rc;
  NG_LAUNCH_N(c, "generate", n, ng::launch_generate(d, key_ptr(c), c->d_tab[c->cur], c->log2B, c->stream, c->gen_quads));
  return NG_OK;
}

int ng_connect_groups(ng_ctx* c, ng_group src, ng_group tgt, const ng_conn_spec* conn, const ng_syn_spec* syn,
                      const float* weights, const float* delays_ms, uint32_t* out_cid, uint64_t* out_first,
                      uint64_t* out_n) {
  const ng_range rs{src.first, src.n}, rt{tgt.first, tgt.n};
  if (!src.idx && !tgt.idx && !weights && !delays_ms) return ng_connect(c, rs, rt, conn, syn, out_cid, out_first, out_n);
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  if (!conn || !syn) return fail(NG_ERR_INVALID_ARG, "null connection or synapse spec");
  if (int rc = flush_connects(c)) return rc;  // the call synchronizes: queued work goes first
  if ((src.idx && src.first) || (tgt.idx && tgt.first))
    return fail(NG_ERR_INVALID_ARG, "a group given by an index array needs first = 0");
  if ((src.idx || tgt.idx) && (!conn->allow_autapses || !conn->allow_multapses))
    return fail(NG_ERR_UNSUPPORTED, "allow_autapses = 0 or allow_multapses = 0 is not implemented for index arrays");
  // ranges of the groups without arrays are node ranges
  if ((!src.idx && (uint64_t)src.first + src.n > c->n_nodes) || (!tgt.idx && (uint64_t)tgt.first + tgt.n > c->n_nodes))
    return fail(NG_ERR_INVALID_ARG, "node range exceeds the %u created nodes", c->n_nodes);
  ng_syn_spec sy = *syn;
  if (weights) sy.weight = ng_param{NG_CONST, 0, 0.0, 0.0};
  if (delays_ms) sy.delay = ng_param{NG_CONST, 0, (double)c->cfg.h_ms, 0.0};  // one step; replaced below
  // plan without side effects, to size the arrays
  Plan pl;
  if (int rc = plan_call(0xFFFFFFFFu, rs, rt, conn, &sy, c->cfg.h_ms, &pl)) return rc;
  ng::CallArrays ca{};
  ca.src_idx = src.idx;
  ca.ns = src.idx ? src.n : 0;
  ca.tgt_idx = tgt.idx;
  ca.nt = tgt.idx ? tgt.n : 0;
  ca.w = weights;
  ca.d_ms = delays_ms;
  ca.n = (uint32_t)pl.n_new;
  ca.h = c->cfg.h_ms;
  // the arrays are checked on the device before anything changes; the four
  // results carry this call's epoch in their high words, so the maxima of
  // earlier calls lose without a clearing pass (the words start at zero and
  // are cleared again when the epoch wraps)
  uint32_t* h = host_words(c, 8);
  if (!h) return NG_ERR_DEVICE;
  uint64_t* d_chk = reinterpret_cast<uint64_t*>(c->d_scalars + kCheckWord);
  if (++c->check_epoch == 0) {
    NG_LAUNCH(c, "fill", ng::launch_fill_u32(c->d_scalars + kCheckWord, 0u, 8, c->stream));
    c->check_epoch = 1;
  }
  NG_LAUNCH(c, "check_arrays", ng::launch_check_arrays(ca, d_chk, c->check_epoch, c->stream));
  NG_HIP(c, hipMemcpyAsync(h, d_chk, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream), "array check");
  NG_HIP(c, hipStreamSynchronize(c->stream), "array check");
  uint32_t chk[4];
  for (int w = 0; w < 4; ++w)  // (low, high) words; no launch (no entries): no result of this epoch
    chk[w] = h[2 * w + 1] == c->check_epoch ? h[2 * w] : 0u;
  if (src.idx && src.n && chk[0] >= c->n_nodes)
    return fail(NG_ERR_INVALID_ARG, "source index %u is not below the %u created nodes", chk[0], c->n_nodes);
  if (tgt.idx && tgt.n && chk[1] >= c->n_nodes)
    return fail(NG_ERR_INVALID_ARG, "target index %u is not below the %u created nodes", chk[1], c->n_nodes);
  int64_t max_steps = 1;
  if (delays_ms && pl.n_new) {
    float max_ms;
    memcpy(&max_ms, &chk[2], 4);
    max_steps = delay_steps_f32(max_ms, c->cfg.h_ms);  // the conversion is monotone in the delay
    if (chk[3] || max_steps > 32767) return fail(NG_ERR_INVALID_ARG, "a delay is not finite or exceeds 32767 steps");
  }
  const ng_range ps{src.idx ? 0u : src.first, src.n}, pt{tgt.idx ? 0u : tgt.first, tgt.n};
  ng::GenDesc d;
  uint64_t n = 0;
  if (int rc = connect_prepare_limit(c, 0xFFFFFFFFu, ps, pt, conn, &sy, &d, &n)) return rc;
  if (int rc = sync_table(c)) return rc;
  // generation maps each synapse through the arrays as it stores it
  d.src_idx = src.idx;
  d.tgt_idx = tgt.idx;
  d.w_arr = weights;
  d.d_ms_arr = delays_ms;
  if (n) NG_LAUNCH_N(c, "generate", n, ng::launch_generate(d, key_ptr(c), c->d_tab[c->cur], c->log2B, c->stream, c->gen_quads));
  if (out_cid) *out_cid = d.cid;
  if (out_first) *out_first = d.pos0;
  if (out_n) *out_n = n;
  connect_commit(c, d, delays_ms ? (int32_t)max_steps : d.max_delay);
  return NG_OK;
}

int ng_connect_batch(ng_ctx* c, uint32_t n_calls, const ng_range* src, const ng_range* tgt,
                     const ng_conn_spec* conn, const ng_syn_spec* syn, uint64_t* out_first) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (n_calls == 0) return NG_OK;
  if (!src || !tgt || !conn || !syn) return fail(NG_ERR_INVALID_ARG, "null array");
  if (int rc = flush_connects(c)) return rc;
  if ((uint64_t)c->next_cid + n_calls > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "connect call ids exhausted");
  std::vector<ng::GenDesc> descs;
  descs.reserve(n_calls);
  uint64_t pos = c->n_conns, groups = 0;
  int32_t maxd = c->max_delay;
  for (uint32_t i = 0; i < n_calls; ++i) {
    Plan p;
    if (int rc = plan_call(c->n_nodes, src[i], tgt[i], &conn[i], &syn[i], c->cfg.h_ms, &p)) {
      g_err = "call " + std::to_string(i) + ": " + g_err;
      return rc;
    }
    p.d.pos0 = pos;
    p.d.cid = c->next_cid + i;
    p.d.group0 = groups;
    p.d.key = key_ptr(c);
    p.d.err = gen_err_ptr(c);
    pos += p.n_new;
    groups += (p.n_new + 3) / 4;
    maxd = std::max(maxd, p.max_delay);
    if (pos > 0xFFFFFFFFull) return fail(NG_ERR_TOO_LARGE, "a context holds at most 2^32-1 connections");
    if (out_first) out_first[i] = p.d.pos0;
    if (p.n_new) descs.push_back(p.d);
  }
  const uint64_t total = pos - c->n_conns;
  const uint64_t desc_bytes = descs.size() * sizeof(ng::GenDesc);
  char* d_descs = nullptr;
  if (!descs.empty()) {
    d_descs = ctx_alloc(c, desc_bytes);
    if (!d_descs) return fail(NG_ERR_OOM, "arena cannot hold the call descriptors");
  }
  if (int rc = reserve_blocks(c, total)) {
    ctx_unalloc(c, d_descs, desc_bytes);
    return rc;
  }
  for (auto& d : descs) d.blocks = c->d_tab[c->cur];
  if (int rc = check_descs(descs)) {
    ctx_unalloc(c, d_descs, desc_bytes);
    return rc;
  }
  if (!descs.empty()) {
    if (int rc = stage_upload(c, d_descs, descs.data(), desc_bytes)) {
      ctx_unalloc(c, d_descs, desc_bytes);
      return rc;
    }
  }
  if (int rc = sync_table(c)) return rc;
  if (!descs.empty()) {
    NG_LAUNCH_N(c, "generate_batch", total,
              ng::launch_generate_batch((const ng::GenDesc*)d_descs, (uint32_t)descs.size(), groups,
                                        c->log2B, c->stream, c->gen_quads));
    ctx_free(c, d_descs, desc_bytes);  // stream-ordered reuse is safe
    if (!c->capturing) ctx_flush_frees(c);
    c->calibrated = false;
  }
  c->next_cid += n_calls;
  c->n_conns = pos;
  c->max_delay = maxd;
  return NG_OK;
}

int ng_set_tuning(ng_ctx* c, int radix_bits, uint32_t sort_ranges) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  if (radix_bits < 4 || radix_bits > ng::sort_max_radix_bits())
    return fail(NG_ERR_INVALID_ARG, "radix_bits must be in [4, %d]", ng::sort_max_radix_bits());
  if (sort_ranges < 1 || sort_ranges > (1u << 20)) return fail(NG_ERR_INVALID_ARG, "sort_ranges in [1, 2^20]");
  c->radix_bits = radix_bits;
  c->sort_ranges = sort_ranges;
  return NG_OK;
}

int ng_set_schedule(ng_ctx* c, const ng_schedule* sc) {
  if (!c || !sc) return fail(NG_ERR_INVALID_ARG, "null context or schedule");
  const int cal = sc->calibration;
  if (cal != NG_CALIB_RADIX && cal != NG_CALIB_COPASS && cal != NG_CALIB_RADIX_LSD && cal != NG_CALIB_RADIX_MSD)
    return fail(NG_ERR_INVALID_ARG, "unknown calibration algorithm %d", cal);
  if (sc->radix_bits < 4 || sc->radix_bits > ng::sort_max_radix_bits())
    return fail(NG_ERR_INVALID_ARG, "radix_bits must be in [4, %d]", ng::sort_max_radix_bits());
  if (sc->sort_ranges < 1 || sc->sort_ranges > (1u << 20)) return fail(NG_ERR_INVALID_ARG, "sort_ranges in [1, 2^20]");
  if (sc->msd_tile != ng::kMsdTile && sc->msd_tile != ng::kMsdTileN)
    return fail(NG_ERR_INVALID_ARG, "msd_tile must be %u or %u", ng::kMsdTile, ng::kMsdTileN);
  const uint32_t spl = sc->gen_synapses_per_lane;
  if (spl != 4 && spl != 8 && spl != 16 && spl != 32)
    return fail(NG_ERR_INVALID_ARG, "gen_synapses_per_lane must be 4, 8, 16 or 32");
  if (sc->queued_calls > kQueuedCallsLimit)
    return fail(NG_ERR_INVALID_ARG, "queued_calls must be at most %u", kQueuedCallsLimit);
  if (c->queued.size() > sc->queued_calls) {  // the queue holds more than the new bound
    if (int rc = enter(c)) return rc;
    if (int rc = flush_connects(c)) return rc;
  }
  c->queued_max = sc->queued_calls;
  c->calib_mode = cal;
  c->radix_bits = sc->radix_bits;
  c->sort_ranges = sc->sort_ranges;
  c->msd_tile = sc->msd_tile;
  c->gen_quads = spl / 4;
  return NG_OK;
}

int ng_get_schedule(ng_ctx* c, ng_schedule* sc) {
  if (!c || !sc) return fail(NG_ERR_INVALID_ARG, "null context or schedule");
  sc->calibration = c->calib_mode;
  sc->radix_bits = c->radix_bits;
  sc->sort_ranges = c->sort_ranges;
  sc->msd_tile = c->msd_tile ? c->msd_tile : ng::kMsdTileN;
  sc->gen_synapses_per_lane = 4 * c->gen_quads;
  sc->queued_calls = c->queued_max;
  return NG_OK;
}

int ng_spikes_init(ng_ctx* c) {
  if (int rc = enter(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  if (!c->calibrated || !c->d_group_ptr) return fail(NG_ERR_STATE, "spike buffers need a calibrated context");
  NG_HIP(c, hipStreamSynchronize(c->stream), "spike init");
  uint32_t G = 0;
  NG_HIP(c, hipMemcpy(&G, c->d_scalars, 4, hipMemcpyDeviceToHost), "group count");
  const uint64_t N = c->gi_nodes, cap = (uint64_t)std::max<int32_t>(c->max_delay, 1) + 1;
  // time, group, multiplicity and spike-array slots per node, head, count, group delays
  const uint64_t slots = N * cap;
  const uint64_t off_entries = align256(3 * 4 * slots + 3 * 4 * N);
  const uint64_t off_gd = off_entries + align256(8 * slots);
  const uint64_t bytes = off_gd + align256(2 * (uint64_t)G + 2);
  ctx_free(c, c->d_spikes, c->spikes_bytes);
  c->d_spikes = nullptr;
  c->spikes_bytes = 0;
  char* m = ctx_alloc(c, bytes);
  if (!m) {
    c->need = Arena::round_up(bytes);
    return fail(NG_ERR_OOM, "arena cannot hold the spike buffers (%llu bytes)", (unsigned long long)bytes);
  }
  c->d_spikes = m;
  c->spikes_bytes = bytes;
  ng::SpikeState& st = c->spikes;
  st.time = (uint32_t*)m;
  st.group = st.time + slots;
  st.mult = st.group + slots;
  st.head = st.mult + slots;
  st.count = st.head + N;
  st.stamp = st.count + N;
  st.entries = (uint2*)(m + off_entries);
  st.gdelay = (int16_t*)(m + off_gd);
  st.n_entries = c->d_scalars + 12;
  st.err = c->d_scalars + 2;
  st.group_ptr = c->d_group_ptr;
  st.group_start = c->d_group_start;
  st.blocks = c->d_tab[c->cur];
  st.log2B = c->log2B;
  st.n_nodes = (uint32_t)N;
  st.cap = (uint32_t)cap;
  c->spike_step = 0;
  NG_LAUNCH(c, "spikes_init", ng::launch_spikes_init(st, G, c->stream));
  return NG_OK;
}

int ng_spikes_step(ng_ctx* c, const uint32_t* nodes, const uint32_t* mult, uint32_t n, float* input) {
  if (int rc = enter(c)) return rc;
  if (int rc = not_capturing(c)) return rc;  // each step stamps the emitting nodes with its own number
  if (!c->calibrated || !c->d_spikes) return fail(NG_ERR_STATE, "ng_spikes_init first (after calibration)");
  if ((n && !nodes) || !input) return fail(NG_ERR_INVALID_ARG, "null spike or input array");
  // stamps tell a node's second spike in one step apart; 0xFFFFFFFF marks "never"
  if (c->spike_step == 0xFFFFFFFEu) return fail(NG_ERR_STATE, "step count exhausted; ng_spikes_init again");
  NG_LAUNCH(c, "spikes_step", ng::launch_spikes_step(c->spikes, nodes, mult, n, input, c->spike_step, c->stream));
  c->spike_step++;
  return NG_OK;
}

int ng_set_calibration(ng_ctx* c, int algorithm) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  if (algorithm != NG_CALIB_RADIX && algorithm != NG_CALIB_COPASS && algorithm != NG_CALIB_RADIX_LSD &&
      algorithm != NG_CALIB_RADIX_MSD)
    return fail(NG_ERR_INVALID_ARG, "unknown calibration algorithm %d", algorithm);
  c->calib_mode = algorithm;
  return NG_OK;
}

int ng_calibrate(ng_ctx* c) { return calibrate_many(&c, 1); }

int ng_calibrate_noalloc(ng_ctx* c) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (c->calibrated) return NG_OK;
  if (c->calib_mode == NG_CALIB_COPASS)
    return fail(NG_ERR_UNSUPPORTED, "the fixed-scratch calibration is the radix sort; the context is in COPASS mode");
  if (c->shared_arena)
    return fail(NG_ERR_UNSUPPORTED, "the fixed-scratch calibration needs a context with its own arena");
  ScratchBump sb;
  sb.base = noalloc_scratch_ptr(c->device);
  sb.cap = kNoAllocScratchBytes;
  if (!sb.base) return fail(NG_ERR_STATE, "the fixed scratch of this device was not set up");
  return calibrate_many(&c, 1, nullptr, &sb);
}

uint64_t ng_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int ng_calibrate_many(ng_ctx* const* ctxs, uint32_t n) { return calibrate_many(ctxs, n); }

int ng_set_seed(ng_ctx* c, uint64_t seed) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  if (c->n_conns != 0 || c->next_cid != 0)
    return fail(NG_ERR_STATE, "the seed can change only on a context without Connect calls (after ng_reset)");
  NG_HIP(c, set_seed(c, seed), "seed");
  c->cfg.seed = seed;
  return NG_OK;
}

int ng_reset(ng_ctx* c) {
  if (int rc = enter(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  for (char* b : c->blocks) ctx_free(c, b, ng::kBytesPerConn * c->B);
  c->blocks.clear();
  c->tab_synced = 0;
  c->queued.clear();  // their connections are discarded with the blocks
  c->queued_groups = 0;
  release_index(c);
  c->n_nodes = 0;
  c->next_cid = 0;
  c->n_conns = 0;
  c->max_delay = 1;
  c->calibrated = false;
  c->gi_nodes = 0;
  return NG_OK;
}

}  // extern "C"

struct ng_graph {
  ng_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* stage = nullptr;  // pinned descriptors the graph's upload nodes read
};

extern "C" {

int ng_graph_begin(ng_ctx* c, uint64_t staging_bytes) {
  if (int rc = enter(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  if (int rc = mutable_state(c)) return rc;
  if (c->stream == nullptr) return fail(NG_ERR_STATE, "graph capture needs a non-default stream");
  if (int rc = flush_connects(c)) return rc;  // queued calls are not part of the graph
  if (staging_bytes == 0) staging_bytes = 4ull << 20;
  NG_HIP(c, hipHostMalloc((void**)&c->cap_stage, staging_bytes, hipHostMallocDefault), "hipHostMalloc");
  c->cap_stage_cap = staging_bytes;
  c->cap_stage_used = 0;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipHostFree(c->cap_stage);
    c->cap_stage = nullptr;
    return dev_fail(c, e, "hipStreamBeginCapture");
  }
  c->capturing = true;
  c->timing_before_capture = c->timing;
  c->timing = false;
  return NG_OK;
}

int ng_graph_end(ng_ctx* c, ng_graph** out) {
  if (!c || !out) return fail(NG_ERR_INVALID_ARG, "null argument");
  if (!c->capturing) return fail(NG_ERR_STATE, "no capture in progress");
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  c->capturing = false;
  c->timing = c->timing_before_capture;
  if (e != hipSuccess) {
    (void)hipHostFree(c->cap_stage);
    c->cap_stage = nullptr;
    return dev_fail(c, e, "hipStreamEndCapture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    (void)hipHostFree(c->cap_stage);
    c->cap_stage = nullptr;
    return dev_fail(c, e, "hipGraphInstantiate");
  }
  ng_graph* g = new ng_graph();
  g->ctx = c;
  g->graph = graph;
  g->exec = exec;
  g->stage = c->cap_stage;
  c->cap_stage = nullptr;
  c->frozen++;
  *out = g;
  return NG_OK;
}

int ng_graph_launch(ng_graph* g, uint64_t seed) {
  if (!g) return fail(NG_ERR_INVALID_ARG, "null graph");
  ng_ctx* c = g->ctx;
  if (int rc = enter(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  NG_HIP(c, set_seed(c, seed), "seed");
  NG_HIP(c, hipGraphLaunch(g->exec, c->stream), "hipGraphLaunch");
  c->cfg.seed = seed;
  return NG_OK;
}

int ng_graph_destroy(ng_graph* g) {
  if (!g) return NG_OK;
  ng_ctx* c = g->ctx;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  if (g->stage) (void)hipHostFree(g->stage);
  c->frozen--;
  delete g;
  return NG_OK;
}

int ng_enable_timing(ng_ctx* c, int on) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  c->timing = on != 0;
  return NG_OK;
}

int ng_time_only(ng_ctx* c, const char* name) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  if (name && strlen(name) >= sizeof(ng_kernel_time::name))
    return fail(NG_ERR_INVALID_ARG, "kernel name longer than %zu characters", sizeof(ng_kernel_time::name) - 1);
  c->timing_only = name ? name : "";
  return NG_OK;
}

int ng_read_timing(ng_ctx* c, ng_kernel_time* out, int capacity, int* count, int reset) {
  if (int rc = ng_sync(c)) return rc;
  collect_timing(c);
  int n = 0;
  for (auto& kv : c->timing_acc) {
    if (out && n < capacity) {
      memset(&out[n], 0, sizeof(out[n]));
      strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.launches;
      out[n].total_ms = kv.second.ms;
      out[n].records = kv.second.records;
    }
    ++n;
  }
  if (count) *count = n;
  if (reset) c->timing_acc.clear();
  return NG_OK;
}

int ng_sync(ng_ctx* c) {
  if (int rc = enter(c)) return rc;
  if (int rc = not_capturing(c)) return rc;
  if (int rc = flush_connects(c)) return rc;
  NG_HIP(c, hipStreamSynchronize(c->stream), "kernel execution");
  uint32_t words[2] = {0, 0};
  NG_HIP(c, hipMemcpy(words, c->d_scalars + 2, 8, hipMemcpyDeviceToHost), "read error words");
  if (words[1]) {  // generation: the connections of some call are not valid
    c->sticky = NG_ERR_DEVICE;
    c->sticky_msg = std::string("generation error:") +
                    ((words[1] & 1u) ? " a permutation walk started at or above its bound" : "") +
                    ((words[1] & 2u) ? " a permutation walk reached its step cap" : "");
    return fail(NG_ERR_DEVICE, "%s", c->sticky_msg.c_str());
  }
  const uint32_t err = words[0];
  if (err) {  // spike input the steps since the last check dropped (not sticky)
    NG_HIP(c, hipMemset(c->d_scalars + 2, 0, 4), "clear error word");
    return fail(NG_ERR_INVALID_ARG, "spike input dropped:%s%s", (err & 2) ? " a node emitted twice in one step" : "",
                (err & 4) ? " a node index not below the node count" : "");
  }
  return NG_OK;
}

int ng_get_connections(ng_ctx* c, ng_conn_view* out) {
  if (!out) return fail(NG_ERR_INVALID_ARG, "null view");
  if (int rc = ng_sync(c)) return rc;
  memset(out, 0, sizeof *out);
  out->n_conns = c->n_conns;
  out->block_size = c->B;
  out->n_nodes = c->n_nodes;
  out->n_blocks = (uint32_t)c->blocks.size();
  out->block_base = (void* const*)c->blocks.data();
  out->calibrated = c->calibrated ? 1 : 0;
  if (c->calibrated) {
    uint32_t G = 0;
    NG_HIP(c, hipMemcpy(&G, c->d_scalars, 4, hipMemcpyDeviceToHost), "read G");
    out->n_groups = G;
    out->group_ptr = c->d_group_ptr;
    out->group_start = c->d_group_start;
  }
  return NG_OK;
}

int ng_copy_connections(ng_ctx* c, uint64_t first, uint64_t count, uint32_t* src, uint32_t* tgt, float* w,
                        int16_t* delay) {
  if (int rc = ng_sync(c)) return rc;
  if (first > c->n_conns || count > c->n_conns - first)
    return fail(NG_ERR_INVALID_ARG, "range [%llu,+%llu) outside the %llu connections",
                (unsigned long long)first, (unsigned long long)count, (unsigned long long)c->n_conns);
  uint64_t done = 0;
  while (done < count) {
    const uint64_t j = first + done;
    const uint64_t b = j >> c->log2B, o = j & (c->B - 1);
    const uint64_t len = std::min(count - done, c->B - o);
    char* base = c->blocks[b];
    if (src) NG_HIP(c, hipMemcpyAsync(src + done, base + 4 * o, 4 * len, hipMemcpyDefault, c->stream), "copy");
    if (tgt) NG_HIP(c, hipMemcpyAsync(tgt + done, base + 4 * c->B + 4 * o, 4 * len, hipMemcpyDefault, c->stream), "copy");
    if (w) NG_HIP(c, hipMemcpyAsync(w + done, base + 8 * c->B + 4 * o, 4 * len, hipMemcpyDefault, c->stream), "copy");
    if (delay)
      NG_HIP(c, hipMemcpyAsync(delay + done, base + 12 * c->B + 2 * o, 2 * len, hipMemcpyDefault, c->stream), "copy");
    done += len;
  }
  NG_HIP(c, hipStreamSynchronize(c->stream), "copy");
  return NG_OK;
}

int ng_copy_group_index(ng_ctx* c, uint32_t* group_ptr, uint32_t* group_start) {
  if (int rc = ng_sync(c)) return rc;
  if (!c->calibrated) return fail(NG_ERR_STATE, "not calibrated");
  uint32_t G = 0;
  NG_HIP(c, hipMemcpy(&G, c->d_scalars, 4, hipMemcpyDeviceToHost), "read G");
  if (group_ptr)
    NG_HIP(c, hipMemcpy(group_ptr, c->d_group_ptr, 4 * (c->gi_nodes + 1ull), hipMemcpyDefault), "copy");
  if (group_start)
    NG_HIP(c, hipMemcpy(group_start, c->d_group_start, 4 * (G + 1ull), hipMemcpyDefault), "copy");
  return NG_OK;
}

int ng_memory_stats(ng_ctx* c, uint64_t* used, uint64_t* peak, uint64_t* largest_free) {
  if (!c) return fail(NG_ERR_INVALID_ARG, "null context");
  if (used) *used = c->arena->used();
  if (peak) *peak = c->arena->peak();
  if (largest_free) *largest_free = c->arena->largest_free();
  return NG_OK;
}

}  // extern "C"
