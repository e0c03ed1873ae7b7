/*
 * ng.h -- C ABI of the MI355X connectivity builder.
 *
 * Builds spiking-network connectivity directly in device memory from
 * high-level connection rules and then calibrates it, following Golosio et
 * al., "Runtime Construction of Large-Scale Spiking Neuronal Network Models
 * on GPU Devices" (arXiv 2306.09855):
 *   ng_create_nodes   node creation (Sec. 2.6, stage "node creation")
 *   ng_connect        one Connect call (Sec. 2.1: rules of Eqs. (4)-(13),
 *                     blocks of Eq. (1), connection numbering of Eqs. (2)-(3))
 *   ng_calibrate      ordering by (source, delay) and the connection-group
 *                     index of Eq. (14) (Sec. 2.2; stage "calibration")
 *   ng_calibrate_many the same for several contexts in shared launches
 *   ng_get_connections / ng_copy_connections   read the result back
 *
 * Conventions
 *   - Every call returns an ng_status; 0 is success, negative is an error.
 *     ng_last_error() gives a message for the calling thread's last error.
 *     No C++ exception crosses this boundary.
 *   - Device memory: the caller hands ng_create one device buffer (the arena);
 *     the context carves all of its device allocations out of it and never
 *     allocates device memory itself.  The arena and the stream must outlive
 *     the context.
 *   - Work is enqueued on the caller's HIP stream and is asynchronous unless a
 *     function says it synchronizes.  Errors raised by kernels are reported by
 *     the next synchronizing call as NG_ERR_DEVICE and stay sticky.
 *   - A context is not thread-safe; use one context per thread or lock.
 *
 * Random numbers (the paper uses cuRAND and notes that a change of generator
 * preserves the network only statistically, Sec. 2.7).  The contract here:
 *   Philox4x32-10 (Salmon et al., SC'11), key = (seed mod 2^32, seed >> 32).
 *   Word q of stream s of Connect call c is word (q mod 4) of the block with
 *   counter (q/4 mod 2^32, q/4 >> 32, c, s).  Synapse i of a call takes word
 *   i of stream 0 for a random source, word i of stream 2 for a random
 *   target and word i of stream 3 for a random delay, so the draws of one
 *   kind are independent of the others'.  Stream 1 holds weight draws: normal
 *   weights of synapses 2j and 2j+1 are the cosine and sine outputs of
 *   Box-Muller on words y0 = 2j, y1 = 2j+1, u1 = (y0>>8 + 1)/2^24,
 *   u2 = (y1>>8)/2^24; a uniform weight of synapse i takes word i.  Computed
 *   in fp32 and stored as fp32.  rand(N) = floor(x * N / 2^32) for a word x.
 */
#ifndef NG_H
#define NG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NG_OK = 0,
  NG_ERR_INVALID_ARG = -1, /* bad range, spec or pointer; nothing changed */
  NG_ERR_OOM = -2,         /* the arena cannot hold the request; nothing changed */
  NG_ERR_UNSUPPORTED = -3, /* valid request this library does not implement */
  NG_ERR_STATE = -4,       /* call not allowed in the current state */
  NG_ERR_TOO_LARGE = -5,   /* more than 2^32-1 connections in one context */
  NG_ERR_DEVICE = -6       /* a HIP call or kernel failed (sticky) */
} ng_status;

typedef struct ng_ctx ng_ctx;

/* A node group of consecutive indices [first, first+n) (Sec. 2.1). */
typedef struct {
  uint32_t first, n;
} ng_range;

/* Connection rules of Sec. 2.1, multapses allowed.  With allow_autapses = 0
 * (a flag the paper names as future work, Discussion) no connection joins a
 * node to itself:
 *   one_to_one       no connections if the ranges start at the same node;
 *   all_to_all       the pairs s != t, row by row, targets ascending;
 *   fixed_indegree   a target inside the source range draws from the other
 *                    N_s - 1 sources (rand(N_s - 1) from its usual word, the
 *                    target's own position skipped); fixed_outdegree likewise;
 *   fixed_total_number  a drawn pair with s == t is redrawn from words 2i,
 *                    2i+1 of stream 65536 + a for attempt a = 1, 2, ...; the
 *                    64th attempt draws the target among the others.
 * Calls that could only make autapses fail with NG_ERR_INVALID_ARG.
 * With allow_multapses = 0 (also named as future work) no two connections
 * join the same pair.  one_to_one and all_to_all never repeat a pair.
 * fixed_indegree: target t takes the sources at positions pi_t(0..K-1) of
 * its candidates (the source range, without t when autapses are
 * prohibited), pi_t a permutation of [0, M) keyed by the call and t: a
 * 4-round Feistel network on n bits, the smallest n >= 2 with 2^n >= M,
 * reapplied until the value is below M: the value is L * 2^nb + R (R the low
 * nb = n - floor(n/2) bits), rounds 0 and 2 set L ^= lowbias32(R ^ k_r) mod
 * 2^(n - nb), rounds 1 and 3 set R ^= lowbias32(L ^ k_r) mod 2^nb, with
 * k_0..k_3 the words of Philox(ctr = (t, 0, call, 131072)) and lowbias32
 * the integer hash of C. Wellons (2018).  fixed_outdegree likewise with sources and targets exchanged.
 * fixed_total_number: synapse i is the pair of index pi_0(i) in the
 * all_to_all order.  These draws take no source or target word (synapse
 * i's delay is word i of the delay stream, as for every rule).  K or N above
 * the distinct candidates is NG_ERR_INVALID_ARG. */
typedef enum {
  NG_ONE_TO_ONE = 0,         /* Eqs. (4)-(5): N_new = N_s = N_t         */
  NG_ALL_TO_ALL = 1,         /* Eqs. (6)-(7): N_new = N_s * N_t         */
  NG_FIXED_INDEGREE = 2,     /* Eqs. (10)-(11): N_new = N_t * K          */
  NG_FIXED_OUTDEGREE = 3,    /* Eqs. (8)-(9): N_new = N_s * K           */
  NG_FIXED_TOTAL_NUMBER = 4, /* Eqs. (12)-(13): N_new = N                */
  NG_PAIRWISE_BERNOULLI = 5  /* each pair with probability p (below)     */
} ng_rule;

typedef struct {
  int32_t rule;            /* ng_rule */
  int32_t allow_autapses;  /* 0: no connection from a node to itself (below) */
  int32_t allow_multapses; /* 0: no two connections join the same pair (below) */
  int32_t reserved;
  uint64_t k_or_n;         /* K for in/out-degree, N for fixed_total_number */
  double p;                /* pairwise_bernoulli: connection probability in [0, 1] */
} ng_conn_spec;

/* pairwise_bernoulli (the Discussion names it as missing: the number of
 * connections is not known before they are drawn).  Pair (s, t) -- rows of
 * sources in order, targets ascending, positions a and b in the ranges --
 * is a connection when word a * N_t + b of stream 0 is below
 * floor(p * 2^32); with allow_autapses = 0 a self-pair never is.  The
 * connections are numbered in pair order; connection j takes the delay and
 * weight words of synapse j (word j of stream 3, stream 1).  Only
 * ng_connect takes it: a counting pass over the pairs gives the exact number
 * of connections, the host reads it (ng_connect synchronizes for this rule;
 * NG_ERR_STATE under capture), reserves exactly that many, and a second pass
 * writes them (never a multapse, so allow_multapses is ignored).  The
 * batched, array and served forms return NG_ERR_UNSUPPORTED. */

/* Weight and delay specifications (Sec. 2.1, last paragraph). */
typedef enum {
  NG_CONST = 0,       /* weight: a.  delay: a in ms -> steps                    */
  NG_NORMAL = 1,      /* weight only: Normal(mean a, sd b), b >= 0               */
  NG_UNIFORM_INT = 2, /* delay only: integer steps uniform in {a..b}, 1 <= a <= b */
  NG_UNIFORM = 3      /* weight: uniform in [a, b).  delay: ms uniform in [a, b) */
} ng_dist;

typedef struct {
  int32_t kind; /* ng_dist */
  int32_t reserved;
  double a, b;
} ng_param;

typedef struct {
  ng_param weight, delay;
} ng_syn_spec;

typedef struct {
  uint64_t block_size; /* connections per block B (Eq. (1)); power of two,
                          2^16 .. 2^30; 0 selects 2^24 */
  uint64_t seed;       /* Philox key */
  float h_ms;          /* time resolution for ms -> step conversion; 0 -> 0.1 */
  int32_t reserved;
} ng_config;

/* Read-only view of the connections of a context.
 * Connection j (0 <= j < n_conns) lives in block j / block_size at offset
 * o = j % block_size.  Block b starts at device address block_base[b]:
 *   uint32_t src[B] at +0, uint32_t tgt[B] at +4B, float w[B] at +8B,
 *   int16_t delay[B] at +12B  (B = block_size, 14 bytes per connection).
 * Before calibration connections are in creation order (calls in issue order,
 * then i_newconns); after it they are ordered by (source, delay), ties in
 * creation order.  group_ptr[i] (i = 0..n_nodes) is p_i of Eq. (14); the
 * groups of source i are g = group_ptr[i] .. group_ptr[i+1]-1 and group g
 * holds connections group_start[g] .. group_start[g+1]-1.
 * All pointers are borrowed: valid until the next mutating call on the
 * context.  block_base is a host array; everything else is device memory. */
typedef struct {
  uint64_t n_conns;
  uint64_t n_groups;          /* G; 0 if not calibrated */
  uint64_t block_size;
  uint32_t n_nodes;
  uint32_t n_blocks;
  int32_t calibrated;
  int32_t reserved;
  void* const* block_base;    /* host array [n_blocks] of device pointers */
  const uint32_t* group_ptr;  /* device [n_nodes + 1]; NULL if not calibrated */
  const uint32_t* group_start;/* device [n_groups + 1]; NULL if not calibrated */
} ng_conn_view;

/* Create a context over the caller's device arena [arena, arena + bytes) on
 * the current HIP device; all work goes to `stream` (a hipStream_t, NULL =
 * null stream).  The arena must be 256-byte aligned. */
int ng_create(const ng_config* cfg, void* arena, uint64_t arena_bytes, void* stream,
              ng_ctx** out);
/* Wait for the context's work and release it (the arena stays the caller's). */
int ng_destroy(ng_ctx* ctx);

/* Append n nodes; *out = {first new index, n}.  Host only. */
int ng_create_nodes(ng_ctx* ctx, uint32_t n, ng_range* out);

/* One Connect call (Sec. 2.1).  Validates, reserves blocks by Eq. (1) and
 * queues the call's generation; returns without waiting.  All-or-nothing:
 * on error nothing changes and no call id is consumed.  The call creates
 * connections [*out_first, *out_first + *out_n) in creation order and uses
 * Philox call id *out_connect_id.  Any output pointer may be NULL.
 * Queued calls (fewer than 2^24 synapses each) go to the context's stream
 * together, as one generation launch, when a call reads or orders work after
 * the connections (ng_calibrate, ng_calibrate_many, ng_calibrate_noalloc,
 * ng_sync and every call that synchronizes, ng_connect_batch,
 * ng_connect_groups, pairwise_bernoulli, ng_graph_begin) and when the queue
 * holds ng_schedule.queued_calls calls.  A larger call, and any call under
 * graph capture, launches at once; the queue keeps waiting (each call writes
 * its own positions, so the launches may run in any order).  Work ordered on
 * the stream by other means (events, the caller's own kernels) sees a
 * Connect call's connections only after such a call: ng_sync, or
 * ng_get_connections, in between.  The arithmetic is the same either way. */
int ng_connect(ng_ctx* ctx, ng_range src, ng_range tgt, const ng_conn_spec* conn,
               const ng_syn_spec* syn, uint32_t* out_connect_id, uint64_t* out_first,
               uint64_t* out_n);

/* A node group (Sec. 2.1): the consecutive indices [first, first + n) when
 * idx is NULL; else the n node indices idx[0..n) (device memory, u32, each
 * below the node count, repeats allowed) and first must be 0. */
typedef struct {
  uint32_t first, n;
  const uint32_t* idx;
} ng_group;

/* A Connect call whose node groups may be index arrays and whose weights or
 * delays may be given per connection (Sec. 2.1, last paragraphs).  Same as
 * ng_connect, except:
 *   - a group with an index array takes its node indices from the array, at
 *     the positions the rule's formulas give (the formulas taken from 0);
 *   - weights != NULL: weights[i] (device, f32, one per connection of the
 *     call, creation order) is the weight of connection i; syn->weight is
 *     ignored and no weight words are drawn;
 *   - delays_ms != NULL: delays_ms[i] (device, f32, ms) is the delay of
 *     connection i, converted to steps like a constant delay (divided by the
 *     resolution in fp32, rounded to nearest even, at least one step);
 *     syn->delay is ignored and the connection draws no delay word, so its
 *     source and target draws are those of a constant-delay call.
 * The random words of everything else are those of ng_connect.  With any
 * array the call first checks the arrays on the device (indices below the
 * node count; delays finite and at most 32767 steps) and synchronizes:
 * NG_ERR_INVALID_ARG if a check fails (nothing changed), NG_ERR_STATE under
 * graph capture, NG_ERR_UNSUPPORTED with allow_autapses = 0.  The arrays must
 * stay valid until the context's stream has run the call's generation.  With
 * no array it is ng_connect. */
int ng_connect_groups(ng_ctx* ctx, ng_group src, ng_group tgt, const ng_conn_spec* conn,
                      const ng_syn_spec* syn, const float* weights, const float* delays_ms,
                      uint32_t* out_connect_id, uint64_t* out_first, uint64_t* out_n);

/* Many Connect calls at once, with results identical to issuing them one by
 * one with ng_connect in array order: one generation kernel for all of them.
 * out_first (may be NULL) receives each call's first connection index. */
int ng_connect_batch(ng_ctx* ctx, uint32_t n_calls, const ng_range* src, const ng_range* tgt,
                     const ng_conn_spec* conn, const ng_syn_spec* syn, uint64_t* out_first);

/* Calibration (Sec. 2.2): stable sort of all connections by (source, delay)
 * and the group index (Eq. (14)).  Asynchronous.  Connecting after a
 * calibration is allowed; the next calibration sorts everything again, with
 * the same result as a single calibration at the end. */
int ng_calibrate(ng_ctx* ctx);

/* Calibrate n contexts together (Sec. 2.2 applied to each): every context is
 * one segment of the same sort launches and of the same group-index
 * launches, so many small networks cost the launches of one.  Each context's
 * result is identical to ng_calibrate on it.  The work runs on ctxs[0]'s
 * stream; every other context's stream is ordered before it and after it
 * with events, so later work on any of the streams sees the result.
 * Contexts already calibrated are skipped.  Requirements: distinct contexts
 * on one device with one block size, none frozen by a live graph, none being
 * captured (NG_ERR_INVALID_ARG / NG_ERR_STATE otherwise).  Scratch shared by
 * the segments comes from ctxs[0]'s arena, the rest from each context's own.
 * All-or-nothing on NG_ERR_OOM: no context changes except that a context's
 * stale group index (it was uncalibrated) may have been released. */
int ng_calibrate_many(ng_ctx* const* ctxs, uint32_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): ng_calibrate with
 * its sort and group-index scratch (digit counts, scan partials, ping-pong
 * key and payload arrays, group-start bitmap and group sources) taken from a
 * fixed region of ng_noalloc_scratch_bytes() = 64 MiB in device memory that
 * the library holds on each GPU it runs on until the process ends, instead
 * of from the arena.  It calls no hipMalloc, hipFree or other allocating
 * routine (with timing off: ng_enable_timing creates events).  The outputs
 * -- the calibrated connection blocks and the group index -- live in the
 * context's arena as after ng_calibrate, and the result is identical to
 * ng_calibrate's.  The radix calibration of one context with its own arena:
 * NG_ERR_UNSUPPORTED for a context in COPASS mode or on a server's shared
 * arena.  NG_ERR_TOO_LARGE, with nothing changed, when the scratch does not
 * fit the region: 24 bytes per connection with three or more digit passes
 * (keys wider than 2 x radix bits), 12 with two, none with one, plus about
 * 4.2 bytes per connection for the group index and the counts -- so up to
 * about 2.3 million connections with wide keys.  Asynchronous on the
 * context's stream.  Every call on one GPU uses that GPU's one region:
 * calls whose work may overlap on one GPU (contexts on different streams
 * without ordering between them) race and give wrong results; serialize
 * them.  The region keeps the previous call's contents; nothing in it needs
 * to start at zero. */
int ng_calibrate_noalloc(ng_ctx* ctx);
uint64_t ng_noalloc_scratch_bytes(void);

/* Wait for all enqueued work; reports kernel errors. */
int ng_sync(ng_ctx* ctx);

/* Fill *out with a view of the connections (synchronizes). */
int ng_get_connections(ng_ctx* ctx, ng_conn_view* out);

/* Copy connections [first, first+count) into caller buffers (host or device
 * pointers, any may be NULL to skip that array).  Synchronizes. */
int ng_copy_connections(ng_ctx* ctx, uint64_t first, uint64_t count, uint32_t* src,
                        uint32_t* tgt, float* w, int16_t* delay);

/* Copy the group index into caller buffers (host or device; NULL skips):
 * group_ptr [n_nodes + 1] and group_start [n_groups + 1] of the last
 * calibration.  Synchronizes.  NG_ERR_STATE if not calibrated. */
int ng_copy_group_index(ng_ctx* ctx, uint32_t* group_ptr, uint32_t* group_start);

/* Calibration schedule: the widest radix digit in bits (4..9; default 9) --
 * the key bits are split into the fewest passes of at most that width, as
 * evenly as possible (22-bit keys: 8+7+7; 26-bit keys: 9+9+8) -- and
 * the number of static ranges (one workgroup each) a sort pass splits the
 * connections into (1..2^20; default 1024).  Results do not depend on either;
 * speed does. */
int ng_set_tuning(ng_ctx* ctx, int radix_bits, uint32_t sort_ranges);

/* The whole kernel schedule of a context, for an autotuner (results never
 * depend on it; speed does):
 *   calibration            NG_CALIB_RADIX (default), NG_CALIB_RADIX_LSD,
 *                          NG_CALIB_RADIX_MSD or NG_CALIB_COPASS (as
 *                          ng_set_calibration);
 *   radix_bits             widest digit of the LSD form, 4..9 (default 9);
 *   sort_ranges            static ranges of each scatter pass, 1..2^20
 *                          (default 1024; as ng_set_tuning; the second
 *                          scatter of the most-significant-digit form takes
 *                          twice as many);
 *   msd_tile               records per tile of the most-significant-digit
 *                          form's second scatter when its records are packed:
 *                          10240 or 16384 (default);
 *   gen_synapses_per_lane  synapses each generation lane makes in groups of
 *                          four: 4 (default), 8, 16 or 32 (fewer
 *                          workgroups per launch);
 *   queued_calls           Connect calls ng_connect queues before their
 *                          generation goes out as one launch, 0..4096
 *                          (default 256; 0: every call launches at once, one
 *                          launch per call).
 * ng_set_schedule: NG_ERR_INVALID_ARG (nothing changed) for a value outside
 * these; ng_get_schedule fills the current values.  Lowering queued_calls
 * launches what the queue holds beyond it. */
typedef struct {
  int32_t calibration;
  int32_t radix_bits;
  uint32_t sort_ranges;
  uint32_t msd_tile;
  uint32_t gen_synapses_per_lane;
  uint32_t queued_calls;
} ng_schedule;
int ng_set_schedule(ng_ctx* ctx, const ng_schedule* schedule);
int ng_get_schedule(ng_ctx* ctx, ng_schedule* schedule);

/* Spike buffers and delivery (Sec. 2.3), the consumer of the calibrated
 * connections.  ng_spikes_init (after calibration; synchronizes) gives every
 * node a queue of spikes -- (time index, connection-group index,
 * multiplicity), room for the largest delay plus one -- and empties them.
 * ng_spikes_step runs one simulation step on the context's stream: every
 * queued spike's time index grows by one; a spike whose time index equals
 * the delay of its current group (the node's groups in ascending delay) puts
 * that group in the spike array and moves to the next group, and leaves
 * after the last; every connection of every group in the spike array adds
 * weight x multiplicity to input[target] (device f32 array of n_nodes
 * entries, accumulated with atomics: the order of the additions, and so the
 * rounding, varies between runs; the caller clears it when it wants); then
 * nodes[0..n) (device u32, each at most once per step) emit spikes of
 * multiplicity mult[k] (device u32; NULL: 1) with time and group index zero.
 * A connection of delay d thus delivers d steps after its source emitted.
 * Spikes given with a node index not below the node count, or a node twice
 * in one step, are dropped; the next ng_sync returns NG_ERR_INVALID_ARG
 * once for them.  The buffers hold 20 bytes per node and queue slot, 12 per
 * node and 2 per group, and are released with the group index (a new
 * calibration, ng_reset).  NG_ERR_STATE before calibration / init and
 * under graph capture (every step numbers the spikes it takes in). */
int ng_spikes_init(ng_ctx* ctx);
int ng_spikes_step(ng_ctx* ctx, const uint32_t* nodes, const uint32_t* mult, uint32_t n, float* input);

/* Calibration algorithm of a context; the calibrated arrays and group index
 * are the same with either (stable order by (source, delay), Sec. 2.2).
 *   NG_CALIB_RADIX (default): stable radix sort of all connections into a
 *     second block set, in the most-significant-digit form (below) when one
 *     context with at least 2^25 connections is calibrated, its keys
 *     (source bits + delay bits) fit in 27 bits, its connections average at
 *     least 256 per sub-bucket and at least 10 per possible key (n_nodes x
 *     2^delay bits), else in the LSD form.
 *   NG_CALIB_RADIX_MSD: the most-significant-digit form whenever one context
 *     with keys of at most 27 bits is calibrated (else LSD): a scatter by
 *     the top digit, a scatter of each bucket by the second digit, and runs
 *     of whole sub-buckets sorted by the last digit in on-chip memory and
 *     written straight into the calibrated blocks with their connection
 *     groups; the records between passes carry only the key bits not yet
 *     applied, packed with the target into one word when they fit (peak
 *     scratch 16-24 bytes per connection).  Packed calibrations
 *     (ng_calibrate_many with several contexts) and ng_calibrate_noalloc
 *     always use the LSD form.
 *   NG_CALIB_RADIX_LSD: stable least-significant-digit radix sort (digit
 *     passes of at most 9 bits over the whole key, then a group-index pass;
 *     peak scratch ~ 38 bytes per connection).
 *   NG_CALIB_COPASS: the COPASS in-place block sort of Appendix A.  Each
 *     block is sorted, then block b = 0, 1, ... is filled with the next
 *     block-size smallest connections: a threshold partition of the sorted
 *     remainders, the left partitions gathered into an auxiliary array, the
 *     right partitions shifted toward the end, the auxiliary array sorted
 *     into block b.  The connections stay in their blocks; scratch is about
 *     36 bytes times the block size plus the group index arrays, at the cost
 *     of moving the remaining connections once per block.  Each block's
 *     partition sizes are read back to the host, so a COPASS calibration
 *     synchronizes and cannot be captured (NG_ERR_UNSUPPORTED); in
 *     ng_calibrate_many such contexts are calibrated one by one.
 * Returns NG_OK, or NG_ERR_INVALID_ARG for another value. */
enum { NG_CALIB_RADIX = 0, NG_CALIB_COPASS = 1, NG_CALIB_RADIX_LSD = 2, NG_CALIB_RADIX_MSD = 3 };
int ng_set_calibration(ng_ctx* ctx, int algorithm);

/* Arena bytes in use now, at peak, and the largest free extent. */
int ng_memory_stats(ng_ctx* ctx, uint64_t* used, uint64_t* peak, uint64_t* largest_free);

/* Drop all nodes and connections (the context and its arena stay); the
 * next call ids start at 0 again.  Asynchronous: pending work still runs. */
int ng_reset(ng_ctx* ctx);

/* Seed of the context's Philox key (key = (seed mod 2^32, seed >> 32)),
 * for a new network on the same context, e.g. the repetitions of one
 * network over several seeds that the paper's timings average (Sec. 3).
 * Only on a context that has issued no Connect call since ng_create or
 * ng_reset, and not under graph capture or with live graphs: NG_ERR_STATE
 * otherwise.  Stream-ordered on the context's stream. */
int ng_set_seed(ng_ctx* ctx, uint64_t seed);

/* Per-kernel device time: with timing on, every kernel launch of the context
 * is bracketed by HIP events on its stream.  ng_read_timing synchronizes and
 * reports, per kernel name, the number of launches, the summed time and the
 * records the launches processed where a kernel reports them (the COPASS
 * copies: records copied), else 0. */
typedef struct {
  char name[24];
  uint64_t launches;
  double total_ms;
  uint64_t records;
} ng_kernel_time;
int ng_enable_timing(ng_ctx* ctx, int on);
/* With timing on, bracket only the launches named `name` (a name that
 * ng_read_timing reports, at most 23 characters) by events; NULL or "" (the
 * default) brackets every launch.  Each event pair leaves the GPU idle for a
 * few microseconds between kernels, so a caller timing one kernel inside a
 * longer run can keep the others free of events.  Host only; applies to
 * later launches.  NG_ERR_INVALID_ARG: null context, name too long. */
int ng_time_only(ng_ctx* ctx, const char* name);
int ng_read_timing(ng_ctx* ctx, ng_kernel_time* out, int capacity, int* count, int reset);

/* --- captured graphs (batched form) -------------------------------------
 * ng_graph_begin starts capturing the context's stream (which must not be
 * the null stream); the following ng_create_nodes / ng_connect /
 * ng_connect_batch / ng_calibrate calls enqueue nothing runnable -- their
 * kernels and descriptor uploads become graph nodes.  ng_graph_end closes
 * the capture.  ng_graph_launch writes `seed` as the Philox key and replays
 * the captured work on the context stream: the same calls rebuilt for that
 * seed, results identical to issuing the calls directly with that seed
 * (Discussion: parameter scans rebuild the same structure many times).
 * While a graph exists the context is frozen: calls that change it return
 * NG_ERR_STATE; reading (ng_get_connections, ng_copy_*) is allowed.
 * During capture, calls that synchronize return NG_ERR_STATE.
 * staging_bytes: pinned host bytes for batch descriptors (0: 4 MiB). */
typedef struct ng_graph ng_graph;
int ng_graph_begin(ng_ctx* ctx, uint64_t staging_bytes);
int ng_graph_end(ng_ctx* ctx, ng_graph** out);
int ng_graph_launch(ng_graph* graph, uint64_t seed);
int ng_graph_destroy(ng_graph* graph);

/* --- serving form ----------------------------------------------------------
 * A server runs many model-building sessions over one device arena and a few
 * streams.  Client threads submit requests; ng_submit_* only enqueue and
 * return a ticket.  A scheduler thread admits requests in arrival order (each
 * session's in the order submitted) while the arena has room -- a request
 * that does not fit waits until memory comes back (another calibration's
 * scratch, another session's close) and fails with NG_ERR_OOM at once when
 * it would not fit even with every other session gone, or later when nothing
 * could bring memory back (the device is idle and no other session holds
 * arena memory).  A request can therefore wait for as long as another
 * session stays open; ng_wait's timeout bounds the client's wait.  Connect
 * calls admitted together from the sessions sharing a stream run as one
 * generation launch; calibrations admitted together run as one packed
 * calibration (ng_calibrate_many) when their memory allows, else one by one
 * on their session's stream.  The arithmetic is that
 * of a context of its own: a session's connections equal the same calls on
 * ng_connect with the same seed.  Sessions are spread over the streams
 * round-robin.  All streams must be non-null. */
typedef struct ng_server ng_server;
typedef struct ng_session ng_session;
typedef struct {
  uint64_t block_size;  /* as ng_config.block_size */
  float h_ms;           /* as ng_config.h_ms */
  int32_t radix_bits;   /* 0: default schedule, else as ng_set_tuning */
  uint32_t sort_ranges; /* as ng_set_tuning (used when radix_bits != 0) */
  uint32_t reserved;
} ng_server_config;
typedef struct {
  int32_t status;       /* the request's own result (ng_status) */
  int32_t kind;         /* 0 create_nodes, 1 connect, 2 calibrate, 3 close */
  uint64_t n_conns;     /* connect: connections created; calibrate: connections sorted */
  int64_t arrival_ns, admit_ns, done_ns;  /* host steady clock since the server started */
} ng_ticket_info;
typedef struct {
  uint64_t submitted, launches, packed_calls, max_calls_per_launch, calibrations;
  uint64_t sessions_opened, peak_arena_bytes, arena_used_bytes;
  uint64_t calibrate_packs;        /* calibrations of several sessions run together */
  uint64_t max_sessions_per_pack;
  uint64_t scheduler_busy_ns;      /* scheduler thread time outside its waits */
  uint64_t host_launch_ns;         /* of which: planning and launching packed generation */
  uint64_t host_calibrate_ns;      /* of which: planning and launching calibrations */
} ng_server_stats;
int ng_server_create(const ng_server_config* cfg, void* arena, uint64_t arena_bytes,
                     void* const* streams, int n_streams, ng_server** out);
/* Finish all submitted work, close the remaining sessions, release the server. */
int ng_server_destroy(ng_server* server);
int ng_session_open(ng_server* server, uint64_t seed, ng_session** out);
/* Node creation is ordered with the session's other requests; the range is
 * returned at once. */
int ng_submit_create_nodes(ng_session* session, uint32_t n, ng_range* out, uint64_t* ticket);
int ng_submit_connect(ng_session* session, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                      const ng_syn_spec* syn, uint64_t* ticket);
int ng_submit_calibrate(ng_session* session, uint64_t* ticket);
/* Close after the session's earlier requests; the handle is invalid afterwards. */
int ng_submit_close(ng_session* session, uint64_t* ticket);
/* The same, waiting for the close to finish: returns its status. */
int ng_session_close(ng_session* session);
/* Wait up to timeout_ns (< 0: forever) for a ticket.  NG_OK: finished, *out
 * filled (out->status is the request's result) and the ticket consumed;
 * NG_ERR_STATE: still running (the ticket stays valid). */
int ng_wait(ng_server* server, uint64_t ticket, int64_t timeout_ns, ng_ticket_info* out);
/* The session's context, for ng_get_connections / ng_copy_*; only while the
 * session has no request unfinished (NG_ERR_STATE otherwise). */
int ng_session_context(ng_session* session, ng_ctx** out);
int ng_server_get_stats(ng_server* server, ng_server_stats* out);

/* Message of the calling thread's last error ("" if none). */
const char* ng_last_error(void);

/* --- pure host helpers (no device work) ---------------------------------- */

/* Eq. (1): blocks to add so that n_conns + n_new connections fit in blocks of
 * size block_size, given n_blocks already allocated (never negative). */
uint64_t ng_blocks_needed(uint64_t n_conns, uint64_t n_new, uint64_t block_size,
                          uint64_t n_blocks);

/* Digit plan that the default calibration (NG_CALIB_RADIX) takes for one
 * context of n_conns connections over n_nodes nodes whose delays are at most
 * max_delay steps, with sort_ranges static ranges per scatter pass (the
 * ng_set_tuning value, 1024 by default).  out[0] = 2 when the default
 * calibration takes the most-significant-digit form, 1 when only
 * NG_CALIB_RADIX_MSD takes it (fewer than 2^25 connections, too few per
 * sub-bucket or per key), 0 when
 * it does not apply (keys wider than 27 bits, n_conns = 0 or >= 2^32; the
 * rest is then zero); out[1..3] = the widths b1, b2, b3
 * of the digits from the top (b2 = 0: no second scatter); out[4], out[5] =
 * 1 when the records after the first / second scatter pack the remaining
 * key bits and the target into one word; out[6] = workgroups of the
 * in-LDS pass; out[7] = tiles per range.  Returns NG_OK, or
 * NG_ERR_INVALID_ARG for a null out or max_delay < 1. */
int ng_calibration_plan(uint64_t n_conns, uint32_t n_nodes, int32_t max_delay, uint32_t sort_ranges,
                        uint32_t out[8]);

/* Validate a Connect call against n_nodes existing nodes and return the
 * number of connections it creates (Sec. 2.1). */
int ng_plan_count(uint32_t n_nodes, ng_range src, ng_range tgt, const ng_conn_spec* conn,
                  const ng_syn_spec* syn, float h_ms, uint64_t* out_n);

/* Library version string. */
const char* ng_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NG_H */
