// Internal interface between the host runtime (ng_runtime.cpp) and the HIP
// kernels (ng_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ng {

// Connection storage: fixed-size blocks of B connections (Sec. 2.1), each
// block a structure of arrays -- src u32[B] | tgt u32[B] | w f32[B] | delay i16[B].
constexpr uint64_t kBytesPerConn = 14;

// Delay and weight kinds after host-side planning.
enum : uint32_t { W_CONST = 0, W_NORMAL = 1, W_UNIFORM = 3 };
enum : uint32_t { D_CONST = 0, D_UNIFORM_INT = 2, D_UNIFORM_MS = 3 };

// One planned Connect call, as the generation kernels consume it.
// Generation rule codes beyond ng_rule's: the multapse-free draws (a keyed
// permutation instead of independent draws; no source or target words).
constexpr uint32_t kRuleIndegDistinct = 8;
constexpr uint32_t kRuleOutdegDistinct = 9;
constexpr uint32_t kRuleTotalDistinct = 10;

struct GenDesc {
  uint64_t pos0;     // creation position of synapse 0 (global connection index)
  uint32_t n_new;    // synapses in this call (< 2^32)
  uint32_t cid;      // connect call id (Philox counter word 2)
  uint32_t rule;     // ng_rule
  uint32_t k;        // K for in/out-degree (N_new < 2^32 bounds it)
  uint32_t s0, ns, t0, nt;
  uint32_t w_kind;   // W_*
  uint32_t d_kind;   // D_*
  float w_a, w_b;    // CONST: a | NORMAL: mean, sd | UNIFORM: lo, (hi - lo)
  int32_t d_const;   // D_CONST: steps
  uint32_t d_lo;     // D_UNIFORM_INT: lo steps
  uint32_t d_range;  // D_UNIFORM_INT: hi - lo + 1
  float d_ms_lo, d_ms_width, h;  // D_UNIFORM_MS
  int32_t max_delay; // largest delay this call can produce (host bookkeeping)
  uint32_t no_self;  // no connection from a node to itself, and the ranges overlap
  uint32_t a_lo, a_hi;  // all_to_all without autapses: source positions whose node is a target
  uint64_t p_thr;       // pairwise_bernoulli: a pair connects when its word is below this
  uint64_t n_pairs;     // fixed_total_number without multapses: candidate pairs
  uint64_t group0;   // batched form: index of this call's first 4-synapse group
  char* const* blocks;        // batched form: block table of the call's context
  const uint32_t* key;        // batched form: Philox key of the call's context
  uint32_t* err;              // the context's generation error word (bits: see permute_below)
  // node groups as index arrays and per-connection values (plain form only):
  // a generated source (target) position p becomes src_idx[p] (tgt_idx[p]);
  // synapse i takes weight w_arr[i] and the delay d_ms_arr[i] ms in steps
  const uint32_t* src_idx = nullptr;
  const uint32_t* tgt_idx = nullptr;
  const float* w_arr = nullptr;
  const float* d_ms_arr = nullptr;
};

// --- generation -----------------------------------------------------------
// d_key: the Philox key (seed low word, seed high word) in device memory.
hipError_t launch_generate(const GenDesc& d, const uint32_t* d_key, char* const* d_blocks, int log2B,
                           hipStream_t s,
                           uint32_t quads_per_lane = 1);
// All calls of a batch in one launch; d_descs[n_calls] device array sorted by
// group0, total_groups = sum of ceil(n_new / 4).  Each descriptor names its
// own block table and key, so one launch may serve several contexts.
hipError_t launch_generate_batch(const GenDesc* d_descs, uint32_t n_calls, uint64_t total_groups,
                                 int log2B, hipStream_t s,
                                 uint32_t quads_per_lane = 1);

// --- calibration ----------------------------------------------------------
// Input and output of one digit pass of one segment.
struct SortIO {
  // blocked SoA input (first pass) or key/payload arrays
  char* const* in_blocks;   // device block table, or nullptr
  const uint32_t* in_keys;
  const uint2* in_pay;      // (tgt, w bits)
  // blocked SoA output (last pass) or key/payload arrays
  char* const* out_blocks;
  uint32_t* out_keys;
  uint2* out_pay;
  int log2B;
  uint32_t dbits;           // key = src << dbits | delay
};

// One segment of a digit pass.  A segment is one context's independent sort;
// several segments run in one launch.  Ranges (runs of consecutive tiles, one
// workgroup each) are numbered across segments from range0, and the digit
// counts of the segments lie one after another in one array
// (counts[cbase + d * n_ranges + r]), so that one exclusive scan serves all:
// a segment's scanned offsets then start at base = the records of the
// segments before it (mod 2^32), which the downsweep subtracts.
struct SortSeg {
  SortIO io;
  uint64_t n;               // records
  uint64_t cbase;
  uint32_t shift, nbits;    // digit of this pass
  uint32_t tiles_per_range, n_ranges, range0;
  uint32_t base;
};

// A digit pass over n_segs segments that agree on in/out kind (first pass
// reads blocks, last pass writes blocks).  With one segment it travels by
// value in `one` and no device table is read.
struct SortPack {
  const SortSeg* segs;            // device [n_segs] (n_segs > 1)
  const uint32_t* seg_of_range;   // device [total_ranges] (n_segs > 1)
  uint32_t n_segs;
  uint32_t total_ranges;
  uint32_t ranges_per_xcd;        // launch = 8 * ranges_per_xcd workgroups
  uint32_t max_nbits;
  SortSeg one;
};

// Records per sort tile (a tile may straddle two blocks).
uint32_t sort_tile_size();
int sort_max_radix_bits();

// Digit counts of every range of every segment.
hipError_t launch_upsweep(const SortPack& pk, uint32_t* counts, hipStream_t s);
// One stable digit pass; offsets = exclusive scan of the counts.
hipError_t launch_downsweep(const SortPack& pk, const uint32_t* offsets, hipStream_t s);

// Exclusive scan of n u32 values (in may equal out).  tmp needs
// scan_tmp_words(n) words.  If total != nullptr the sum is written there.
uint64_t scan_tmp_words(uint64_t n);
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* tmp,
                                 uint32_t* total, hipStream_t s);

// tab[first + k] = ptrs[k] for k < count <= 8
hipError_t launch_set_ptrs(char** tab, uint32_t first, uint32_t count, const uint64_t* ptrs,
                           hipStream_t s);
// Block-table entries of several contexts in one launch: e[i].tab[e[i].idx] = e[i].ptr.
struct TabEntry {
  char** tab;
  char* ptr;
  uint32_t idx;
  uint32_t pad;
};
hipError_t launch_set_entries(const TabEntry* d_entries, uint32_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Most-significant-digit calibration (Sec. 2.2): the stable sort by key =
// src << dbits | delay (keybits <= 27) in three digits from the top, key =
// D1 (b1 bits) | D2 (b2 bits) | D3 (b3 bits), each at most 9 bits:
//   A  all records, stably by D1, into 2^b1 buckets (reads the creation-order
//      blocks);
//   B  each bucket stably by D2 into 2^b2 sub-buckets (skipped when b2 = 0);
//   C  each sub-bucket sorted by D3 in LDS and written as calibrated blocks,
//      with its groups (distinct keys) recorded for the group index.
// Records between passes: "narrow" = a u32 kt = (key mod 2^r) << tbits | tgt
// (r = the key bits below the digit already applied) plus a u32 weight, when
// r + tbits <= 32 and tbits < 32; "wide" = the full u32 key, u32 tgt and u32
// weight.  Buckets, sub-buckets and the ranges of pass B are laid out on the
// device from the counts, so no value travels back to the host.
constexpr uint32_t kMsdTile = 10240;      // records per tile of passes A and C, and of B with unpacked records
constexpr uint32_t kMsdTileN = 16384;     // records per tile of B with packed (8-byte) records
constexpr uint32_t kMsdMaxDigit = 9;      // widest digit
constexpr uint32_t kMsdMaxKeyBits = 27;   // 3 x kMsdMaxDigit

struct MsdPlan {
  uint32_t n;                       // records (n > 0)
  uint32_t keybits, dbits, tbits;   // tbits: bits of a target index (nodes - 1)
  uint32_t b1, b2, b3;
  uint32_t narrow_a, narrow_b;      // formats of the output of A and of B
  uint32_t cbits;                   // packed records entering pass C: key bits held above the target
  uint32_t tpr;                     // tiles per range (passes A and B)
  uint32_t tile_b;                  // records per tile of pass B (kMsdTileN when its input is packed)
  uint32_t ranges_a;                // ranges of pass A
  uint32_t ranges_b;                // ranges of pass B wanted (spread over the buckets by their tiles)
  uint32_t max_ranges_b;            // ranges of pass B: at most this many
  uint32_t wgs_c;                   // workgroups of pass C
  uint32_t n_nodes;
  int log2B;
  char* const* in_blocks;           // creation-order blocks
  char* const* out_blocks;          // calibrated blocks
  // records after A (= input of B) and after B (= input of C); *_tgt only wide
  uint32_t *a_key, *a_tgt, *a_w;
  uint32_t *b_key, *b_tgt, *b_w;
  uint32_t* cnt_a;                  // [2^b1 * ranges_a] digit-major counts, scanned in place
  uint32_t* cnt_b;                  // [2^b2 * max_ranges_b] (bucket, digit, range) counts, scanned
  uint32_t* bstart;                 // [2^b1 + 1] bucket starts
  uint32_t* rangeb0;                // [2^b1 + 1] first range of pass B of each bucket
  uint32_t* tprb;                   // [2^b1] tiles per range of pass B of each bucket
  uint32_t* sbstart;                // [2^(b1+b2) + 1] sub-bucket starts
  uint32_t* wg_sb0;                 // [wgs_c + 1] first sub-bucket of each workgroup of C
  uint32_t* big_count;              // sub-buckets larger than one LDS load (set by pass C)
  uint32_t* big_list;               // [max_big] their numbers
  uint32_t max_big;                 // n / (one load + 1) + 1
  uint32_t* gcount;                 // [2^(b1+b2) + 1] groups per sub-bucket, scanned in place
  uint32_t* gmask;                  // [2^(b1+b2) * mask_words] present D3 values per sub-bucket
  uint32_t* gslot;                  // [n] local group starts at sub-bucket offsets (scratch)
  uint32_t mask_words;              // max(1, 2^b3 / 32)
  uint32_t* group_ptr;              // [n_nodes + 1]
  uint32_t* group_start;            // [min(n, 2^keybits) + 1]
  uint32_t* n_groups;               // G (device word)
};

// Records pass C sorts in LDS at once: runs of whole sub-buckets up to this
// many records form one tile; a larger sub-bucket is sorted in pieces of
// this size after a counting pass.
uint32_t msd_cap(bool narrow);
hipError_t launch_msd_count_a(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_scatter_a(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_plan_b(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_count_b(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_scatter_b(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_plan_c(const MsdPlan& p, hipStream_t s);
// pass C: tiles of whole sub-buckets, then the sub-buckets larger than one load
hipError_t launch_msd_tiles_c(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_big_c(const MsdPlan& p, hipStream_t s);
hipError_t launch_msd_groups(const MsdPlan& p, hipStream_t s);

// ---------------------------------------------------------------------------
// pairwise_bernoulli: pairs (rows of sources, targets ascending) in units of
// kPbUnit consecutive targets of one row.  count: counts[u] = connections of
// unit u, and, when bits is not null, the decisions (16 per thread, one u16
// per 16 pairs: kPbUnit / 8 bytes per unit).  write: the connections of unit
// u from creation position d.pos0 + offsets[u] on, in pair order, from the
// stored decisions when bits is not null, else evaluated again.
constexpr uint32_t kPbUnit = 4096;
hipError_t launch_pb_count(const GenDesc& d, const uint32_t* d_key, uint32_t* counts, uint16_t* bits,
                           hipStream_t s);
hipError_t launch_pb_write(const GenDesc& d, const uint32_t* d_key, const uint32_t* offsets, const uint16_t* bits,
                           char* const* blocks, int log2B, hipStream_t s);

// ---------------------------------------------------------------------------
// Spike buffers and delivery (Sec. 2.3) over the calibrated connections.
struct SpikeState {
  uint32_t *time, *group, *mult;  // [n_nodes * cap] queue slots per node
  uint32_t *head, *count;         // [n_nodes]
  uint32_t* stamp;                // [n_nodes] last step a node emitted in
  uint2* entries;                 // [n_nodes * cap] spike array: (global group, multiplicity)
  uint32_t* n_entries;            // [2]: entries of the steps of even and odd number
  uint32_t* err;                  // bit 1: a node emitted into a full queue; bit 2: a node index out of range
  int16_t* gdelay;                // [G] delay of each group
  const uint32_t* group_ptr;      // [n_nodes + 1]
  const uint32_t* group_start;    // [G + 1]
  char* const* blocks;            // calibrated connections
  int log2B;
  uint32_t n_nodes, cap;
};
// group delays, empty queues
hipError_t launch_spikes_init(const SpikeState& st, uint64_t n_groups, hipStream_t s);
// one step: queued spikes advance, the reached groups are delivered
// (input[t] += w * multiplicity), then nodes[0..n) emit
hipError_t launch_spikes_step(const SpikeState& st, const uint32_t* nodes, const uint32_t* mult, uint32_t n,
                              float* input, uint32_t step, hipStream_t s);

// ---------------------------------------------------------------------------
// Node groups as index arrays and per-connection weights / delays (Sec. 2.1).
// check: the low words of out[0] = largest source index, out[1] = largest
// target index, out[2] = bits of the largest delay in ms (negative delays
// count as 0), out[3] = 1 if a delay is NaN; every workgroup raises each
// out[w] to at least (epoch << 32 | its value), so out must hold values of
// smaller epochs on entry.  Generation then applies the arrays
// (GenDesc::src_idx, tgt_idx, w_arr, d_ms_arr).
struct CallArrays {
  const uint32_t* src_idx;  // ns entries, or null
  uint32_t ns;
  const uint32_t* tgt_idx;  // nt entries, or null
  uint32_t nt;
  const float* w;           // n entries, or null
  const float* d_ms;        // n entries, or null
  uint32_t n;
  float h;
};
hipError_t launch_check_arrays(const CallArrays& a, uint64_t* out, uint32_t epoch, hipStream_t s);

// ---------------------------------------------------------------------------
// COPASS in-place block sort (Appendix A).
// Record positions index the block array: position p lives in block p >> log2B.
struct BlockView {
  char* const* blocks;  // device block table
  int log2B;
  uint32_t dbits;       // key = src << dbits | delay
};
// One piece of a copy list: len records from position src to position dst;
// pre = records of the list's pieces before this one.
struct CopySeg {
  uint32_t src, dst, len, pre;
};
struct CopyList {
  const CopySeg* segs;  // device array, pre ascending
  uint32_t n_segs;
  uint32_t total;       // sum of len
};
// Copies the listed records between the block array and packed arrays
// (key u32, payload = (tgt, weight bits)); to_packed: block array -> packed.
hipError_t launch_copass_copy(const BlockView& v, const CopyList& l, bool to_packed, uint32_t* keys, uint2* pay,
                              hipStream_t s);
// Partition of k sorted subarrays (subarray i: positions [start[i],
// start[i]+len[i]) of the block array) for a total of m, 0 < m < sum len:
// m_out[i] = size of the left partition of subarray i.  lo, hi, mu_lo, mu_hi:
// k words of scratch each.  status[0] = last step taken (1 threshold found,
// 2 brackets of width one), status[1] = iterations, status[2] = 1 if the
// iteration bound was hit.  One workgroup.
struct CopassPart {
  BlockView v;
  const uint32_t* start;
  const uint32_t* len;
  uint32_t k;
  uint32_t m;
  uint32_t *lo, *hi, *mu_lo, *mu_hi;
  uint32_t* m_out;
  uint32_t* status;
};
hipError_t launch_copass_partition(const CopassPart& p, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t s);

// Connection-group index over sorted blocked SoA (Sec. 2.2, Eq. (14)), for
// one or several segments:
//   flags      per segment a bitmap[ceil(n/32)] of group starts; per tile of
//              gi_tile_size() positions (tiles numbered across segments from
//              tile0) the number of groups starting in it -> tile_flags
//   write      with tile_base = exclusive scan of tile_flags over all tiles
//              (tile_base[total_tiles] = the grand total): group_start[g] and
//              group_src[g] of every group of every segment
//   ptr        per segment: G = its tile_base span, *n_groups = G,
//              group_start[G] = n, group_ptr[i] for i = 0..n_nodes by binary
//              search in group_src
struct GiSeg {
  char* const* blocks;      // sorted blocked SoA
  uint64_t n;
  uint32_t* bitmap;         // ceil(n/32) + 1 words
  uint32_t* group_start;    // capacity G + 1
  uint32_t* group_src;      // capacity G
  uint32_t* group_ptr;      // n_nodes + 1
  uint32_t* n_groups;       // out: G
  uint32_t tile0, n_tiles;  // gi tiles
  uint32_t n_nodes;
  uint32_t ptr_block0, n_ptr_blocks;  // workgroups of the ptr step
  uint32_t pad;
};

struct GiPack {
  const GiSeg* segs;               // device [n_segs] (n_segs > 1)
  const uint32_t* seg_of_tile;     // device [total_tiles] (n_segs > 1)
  const uint32_t* seg_of_ptr_block;// device [total_ptr_blocks] (n_segs > 1)
  uint32_t n_segs, total_tiles, total_ptr_blocks;
  int log2B;
  GiSeg one;
};

uint32_t gi_tile_size();
// workgroups of the ptr step for a segment of n_nodes nodes
uint32_t gi_ptr_blocks(uint32_t n_nodes);
hipError_t launch_group_flags(const GiPack& pk, uint32_t* tile_flags, hipStream_t s);
hipError_t launch_group_write(const GiPack& pk, const uint32_t* tile_base, hipStream_t s);
hipError_t launch_group_ptr(const GiPack& pk, const uint32_t* tile_base, hipStream_t s);

}  // namespace ng
