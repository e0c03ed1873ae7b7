// HIP kernels for gfx950 (MI355X): connection generation and calibration.
//
// Generation (Sec. 2.1 of Golosio et al.): one lane produces four
// consecutive synapses of a Connect call -- Philox4x32-10 words in
// registers, the rule's index formulas (Eqs. (4)-(13)), delay and weight
// transforms -- and stores them into the block-structured SoA storage.
//
// Calibration (Sec. 2.2): a stable LSD radix sort by key = src << dbits |
// delay, in reduce-then-scan digit passes over XCD-aware static ranges (see
// the sort section), then the connection-group index (Eq. (14)).
#include "ng_internal.h"
#include "ng_device.h"

namespace ng {
namespace {

constexpr int kGenThreads = 256;

template <int RULE, bool DRAND>
__global__ __launch_bounds__(kGenThreads) void k_generate(GenDesc d, const uint32_t* __restrict__ key,
                                                          char* const* __restrict__ blocks, int log2B) {
  const uint32_t key0 = key[0], key1 = key[1];  // the seed lives in device memory (graph replays)
  const uint32_t ngroups = (uint32_t)(((uint64_t)d.n_new + 3) >> 2);
  for (uint32_t g = blockIdx.x * kGenThreads + threadIdx.x; g < ngroups;
       g += gridDim.x * kGenThreads) {
    Quad q;
    gen_quad<RULE, DRAND>(d, g, key0, key1, q);
    const uint32_t i0 = g << 2;
    if (d.src_idx || d.tgt_idx || d.w_arr || d.d_ms_arr) apply_arrays(d, i0, q);
    store_quad(blocks, log2B, d.pos0 + i0, min(4u, d.n_new - i0), q);
  }
}

template <bool DRAND>
__device__ __forceinline__ void gen_any(const GenDesc& d, uint32_t g, uint32_t key0, uint32_t key1,
                                        Quad& q) {
  switch (d.rule) {
    case R_ONE_TO_ONE: gen_quad<R_ONE_TO_ONE, DRAND>(d, g, key0, key1, q); break;
    case R_ALL_TO_ALL: gen_quad<R_ALL_TO_ALL, DRAND>(d, g, key0, key1, q); break;
    case R_INDEG: gen_quad<R_INDEG, DRAND>(d, g, key0, key1, q); break;
    case R_OUTDEG: gen_quad<R_OUTDEG, DRAND>(d, g, key0, key1, q); break;
    case R_INDEG_D: gen_quad<R_INDEG_D, DRAND>(d, g, key0, key1, q); break;
    case R_OUTDEG_D: gen_quad<R_OUTDEG_D, DRAND>(d, g, key0, key1, q); break;
    case R_TOTAL_D: gen_quad<R_TOTAL_D, DRAND>(d, g, key0, key1, q); break;
    default: gen_quad<R_TOTAL, DRAND>(d, g, key0, key1, q); break;
  }
}

// Batched form: a grid-stride loop over the 4-synapse groups of all calls.
// A wave covers 64 consecutive groups; it finds the call of its first group
// once (scalar loads) and, when all 64 lie in that call -- nearly always --
// runs with the descriptor in scalar registers and a uniform rule.  A wave
// that straddles calls looks each lane's call up by binary search.
__global__ __launch_bounds__(kGenThreads) void k_generate_batch(const GenDesc* __restrict__ descs,
                                                                uint32_t n_calls, uint64_t total_groups,
                                                                int log2B) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform by construction
  for (uint64_t wbase = (uint64_t)blockIdx.x * kGenThreads + 64u * wave; wbase < total_groups;
       wbase += (uint64_t)gridDim.x * kGenThreads) {
    const uint64_t gg = wbase + lane;
    const uint64_t wlast = min(wbase + 63, total_groups - 1);
    uint32_t lo = 0, hi = n_calls - 1;  // last call with group0 <= wbase (uniform)
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (C(&descs[mid].group0, 0) <= wbase) lo = mid; else hi = mid - 1;
    }
    const bool one_call = lo + 1 >= n_calls || C(&descs[lo + 1].group0, 0) > wlast;
    if (one_call) {
      const GenDesc d = C_struct(descs, lo);
      if (gg < total_groups) {
        const uint32_t key0 = C(d.key, 0), key1 = C(d.key, 1);
        const uint32_t g = (uint32_t)(gg - d.group0);
        Quad q;
        if (d.d_kind == D_CONST) gen_any<false>(d, g, key0, key1, q);
        else gen_any<true>(d, g, key0, key1, q);
        const uint32_t i0 = g << 2;
        store_quad(d.blocks, log2B, d.pos0 + i0, min(4u, d.n_new - i0), q);
      }
    } else if (gg < total_groups) {
      uint32_t l = lo, h = n_calls - 1;  // this lane's call
      while (l < h) {
        const uint32_t mid = (l + h + 1) >> 1;
        if (descs[mid].group0 <= gg) l = mid; else h = mid - 1;
      }
      const GenDesc d = descs[l];
      const uint32_t key0 = G(d.key)[0], key1 = G(d.key)[1];
      const uint32_t g = (uint32_t)(gg - d.group0);
      Quad q;
      if (d.d_kind == D_CONST) gen_any<false>(d, g, key0, key1, q);
      else gen_any<true>(d, g, key0, key1, q);
      const uint32_t i0 = g << 2;
      store_quad(d.blocks, log2B, d.pos0 + i0, min(4u, d.n_new - i0), q);
    }
  }
}


// ---------------------------------------------------------------------------
// Radix sort: reduce-then-scan digit passes over static ranges of tiles.
// No workgroup waits on another inside a pass: on this chip each XCD has its
// own L2, so a chained (look-back) scan pays an agent-scope round trip per
// tile, while per-range counts cost only one extra read of the keys.
//   upsweep    range r counts the digits of its records
//   scan       exclusive scan of the digit-major count matrix -> offsets
//   downsweep  range r walks its tiles in order: stable wave64 ballot ranks,
//              LDS staging by digit (keys, then payloads, each in its own
//              buffer), runs of equal digits stored to consecutive positions;
//              stores that fill whole 128-byte lines are marked streaming.
// Tiles are large (10,240 records, 512 threads) because the cost of a pass
// is set by the length of the runs each tile writes per digit.  Ranges are
// XCD-aware: workgroup w runs on XCD w % 8, and each XCD owns a contiguous
// span of ranges, so the runs written by neighbouring ranges meet in one L2.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 512;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kItems = 20;
constexpr int kTile = kSortThreads * kItems;  // 10,240 records
constexpr int kMaxRadixBits = 9;


__device__ __forceinline__ int range_index(const SortPack& pk) {
  const uint32_t w = blockIdx.x;
  const uint32_t r = (w & 7u) * pk.ranges_per_xcd + (w >> 3);
  return r < pk.total_ranges ? (int)r : -1;
}

// Tiles of one range in 32-bit uniform arithmetic (a segment holds < 2^32
// records): n_full full tiles from `start`, then a partial tile of `tail`
// records if the range holds the segment's ragged end.  Deriving the tile
// counts once per range keeps 64-bit min/compare selects out of the tile
// loops.
struct RangeTiles {
  uint32_t start, n_full, tail;
};
__device__ __forceinline__ RangeTiles range_tiles(const SortSeg& sg, uint32_t r) {
  RangeTiles t;
  const uint32_t tpr = sg.tiles_per_range;
  t.start = r * tpr * (uint32_t)kTile;  // r < n_ranges, so start < n
  const uint32_t rem = (uint32_t)sg.n - t.start;
  const uint32_t whole = rem / (uint32_t)kTile;
  t.n_full = whole < tpr ? whole : tpr;
  t.tail = whole < tpr ? rem - whole * (uint32_t)kTile : 0u;
  return t;
}

// The segment a global range belongs to (uniform across the workgroup).
__device__ __forceinline__ SortSeg sort_seg(const SortPack& pk, uint32_t gr) {
  if (pk.n_segs == 1) return pk.one;
  const uint32_t k = __builtin_amdgcn_readfirstlane(C(pk.seg_of_range, gr));
  return C_struct(pk.segs, k);
}

// Blocked SoA source of one tile: a tile spans at most two blocks.
struct TileSrc {
  const char* blk[2];
  uint64_t first_block;
};

__device__ __forceinline__ TileSrc tile_src(const SortIO& io, uint64_t base, uint32_t cnt) {
  TileSrc t;
  t.first_block = base >> io.log2B;
  t.blk[0] = C(io.in_blocks, t.first_block);
  const uint64_t last = (base + cnt - 1) >> io.log2B;  // cnt >= 1
  t.blk[1] = last != t.first_block ? C(io.in_blocks, t.first_block + 1) : t.blk[0];
  return t;
}

__device__ __forceinline__ uint32_t load_blocked_key(const SortIO& io, const TileSrc& t, uint64_t j) {
  const uint64_t B = 1ull << io.log2B;
  const char* blk = t.blk[(j >> io.log2B) != t.first_block];
  const uint64_t o = j & (B - 1);
  return (G(reinterpret_cast<const uint32_t*>(blk))[o] << io.dbits) |
         (uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o];
}

// The histogram has kHistCopies interleaved copies (word 4d + c counts
// digit d for lanes with lane % 4 == c): lanes of one add that hold the same
// digit then mostly hit different words in different banks instead of
// serializing on one word.
constexpr int kHistCopies = 4;
static_assert(kHistCopies == 4, "word 4d + c, read back as one uint4 (16-byte aligned array)");

template <int RB, bool IN_BLOCKED>
__global__ __launch_bounds__(kSortThreads) void k_upsweep(SortPack pk, uint32_t* __restrict__ counts) {
  constexpr int NB = 1 << RB;
  __shared__ __align__(16) uint32_t hist[NB * kHistCopies];
  const int gr = range_index(pk);
  if (gr < 0) return;
  const SortSeg sg = sort_seg(pk, (uint32_t)gr);
  const SortIO& io = sg.io;
  const uint32_t r = (uint32_t)gr - sg.range0, shift = sg.shift;
  const uint32_t nd = 1u << sg.nbits, mask = nd - 1;
  const uint32_t copy = threadIdx.x & (kHistCopies - 1);
  for (uint32_t d = threadIdx.x; d < nd * kHistCopies; d += kSortThreads) hist[d] = 0;
  __syncthreads();
  const RangeTiles rt = range_tiles(sg, r);
  for (uint32_t t = 0; t < rt.n_full; ++t) {
    const uint64_t base = rt.start + t * (uint32_t)kTile;
    const uint32_t cnt = kTile;
    uint32_t key[kItems];
    // A full tile with 16-byte loads: 4 consecutive records per load (the
    // order of records does not matter to a histogram).  base is a
    // multiple of 4 records and so is every block size, so a group of 4
    // never straddles two blocks and every load is aligned.
    static_assert(kItems % 4 == 0, "vector loads of 4 records");
    if constexpr (IN_BLOCKED) {
      const TileSrc ts = tile_src(io, base, cnt);
      const uint64_t B = 1ull << io.log2B;
#pragma unroll
      for (int v = 0; v < kItems / 4; ++v) {
        const uint64_t j = base + 4ull * (v * kSortThreads + threadIdx.x);
        const char* blk = ts.blk[(j >> io.log2B) != ts.first_block];
        const uint64_t o = j & (B - 1);
        const u32x4 s4 = *(const NG_GLOBAL u32x4*)(blk + 4 * o);
        const u32x2 d4 = *(const NG_GLOBAL u32x2*)(blk + 12 * B + 2 * o);
        key[4 * v + 0] = (s4.x << io.dbits) | (d4.x & 0xFFFFu);
        key[4 * v + 1] = (s4.y << io.dbits) | (d4.x >> 16);
        key[4 * v + 2] = (s4.z << io.dbits) | (d4.y & 0xFFFFu);
        key[4 * v + 3] = (s4.w << io.dbits) | (d4.y >> 16);
      }
    } else {
#pragma unroll
      for (int v = 0; v < kItems / 4; ++v) {
        const u32x4 k4 = *(const NG_GLOBAL u32x4*)(io.in_keys + base + 4ull * (v * kSortThreads + threadIdx.x));
        key[4 * v + 0] = k4.x;
        key[4 * v + 1] = k4.y;
        key[4 * v + 2] = k4.z;
        key[4 * v + 3] = k4.w;
      }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) atomicAdd(&hist[(((key[k] >> shift) & mask) << 2) | copy], 1u);
  }
  if (rt.tail) {  // the ragged last tile of the segment
    const uint64_t base = rt.start + rt.n_full * (uint32_t)kTile;
    const uint32_t cnt = rt.tail;
    uint32_t key[kItems];
    if constexpr (IN_BLOCKED) {
      const TileSrc ts = tile_src(io, base, cnt);
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const uint32_t lj = k * kSortThreads + threadIdx.x;
        key[k] = lj < cnt ? load_blocked_key(io, ts, base + lj) : 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        const uint32_t lj = k * kSortThreads + threadIdx.x;
        key[k] = lj < cnt ? G(io.in_keys)[base + lj] : 0u;
      }
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if ((uint32_t)(k * kSortThreads + threadIdx.x) < cnt) atomicAdd(&hist[(((key[k] >> shift) & mask) << 2) | copy], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nd; d += kSortThreads) {
    const uint4 h = *reinterpret_cast<const uint4*>(&hist[d << 2]);
    counts[sg.cbase + (uint64_t)d * sg.n_ranges + r] = h.x + h.y + h.z + h.w;
  }
}

struct SortLds {
  uint32_t* key;                    // [kTile] keys staged by digit
  uint2* pay;                       // [kTile] payloads staged by digit (LDS holds both: 120 KB)
  uint32_t* wh;                     // [kSortWaves][NB]: per-wave digit counts, then each wave's
                                    // first tile position per digit
  uint4* dig;                       // [NB] per digit: x = global position of its first record
                                    // in the tile minus its tile position (mod 2^32); [y, y + z):
                                    // the global positions whose 128-byte key line the tile's
                                    // run fills completely
  uint32_t* run;                    // [NB] next global position per digit
  uint32_t* tmp;                    // [kSortWaves]
  uint32_t* sink;                   // [kSortThreads]: counting adds of lanes that lead no digit
  char** blk;                       // [kLdsBlocks]: output block table when it fits, else null
};

constexpr int kLdsBlocks = 512;  // output blocks whose pointers the last pass keeps in LDS

// Output block of a sorted position (last pass): from the LDS copy of the
// table when there is one, so that the lookup does not wait behind the
// tile's outstanding global loads.
__device__ __forceinline__ char* out_block(const SortIO& io, const SortLds& L, uint32_t dest) {
  return L.blk ? L.blk[dest >> io.log2B] : G(io.out_blocks)[dest >> io.log2B];
}

// Records of one tile into registers: wave w owns tile records
// [w*kItems*64, (w+1)*kItems*64), 64 consecutive records per item slot.
template <bool IN_BLOCKED, bool FULL>
__device__ __forceinline__ void load_keys(const SortIO& io, uint64_t base, uint32_t cnt, uint32_t (&key)[kItems]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (IN_BLOCKED) {
    const TileSrc ts = tile_src(io, base, cnt);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
      key[k] = (FULL || lj < cnt) ? load_blocked_key(io, ts, base + lj) : 0u;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
      key[k] = (FULL || lj < cnt) ? G(io.in_keys)[base + lj] : 0u;
    }
  }
}

template <bool IN_BLOCKED, bool FULL>
__device__ __forceinline__ void load_pays(const SortIO& io, uint64_t base, uint32_t cnt, uint2 (&pay)[kItems]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t B = 1ull << io.log2B;
  if constexpr (IN_BLOCKED) {
    const TileSrc ts = tile_src(io, base, cnt);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
      if (FULL || lj < cnt) {
        const uint64_t j = base + lj;
        const char* blk = ts.blk[(j >> io.log2B) != ts.first_block];
        const uint64_t o = j & (B - 1);
        pay[k] = make_uint2(G(reinterpret_cast<const uint32_t*>(blk + 4 * B))[o],
                            G(reinterpret_cast<const uint32_t*>(blk + 8 * B))[o]);
      } else {
        pay[k] = make_uint2(0, 0);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
      pay[k] = (FULL || lj < cnt) ? ld_u32x2(io.in_pay + base + lj) : make_uint2(0, 0);
    }
  }
}

template <bool IN_BLOCKED>
__device__ __forceinline__ void load_keys_any(const SortIO& io, uint64_t base, uint32_t cnt, uint32_t (&key)[kItems]) {
  if (cnt == kTile) load_keys<IN_BLOCKED, true>(io, base, cnt, key);
  else load_keys<IN_BLOCKED, false>(io, base, cnt, key);
}

// Store of one payload to its sorted position: streaming where the run fills
// the 128-byte line, cached otherwise.
template <bool OUT_BLOCKED>
__device__ __forceinline__ void store_pay(const SortIO& io, const SortLds& L, uint32_t dest, bool in, uint2 pp) {
  if constexpr (OUT_BLOCKED) {
    const uint64_t B = 1ull << io.log2B;
    char* blk = out_block(io, L, dest);
    const uint64_t o = dest & (B - 1);
    if (in) {
      st_u32_nt(blk + 4 * B + 4 * o, pp.x);
      st_u32_nt(blk + 8 * B + 4 * o, pp.y);
    } else {
      G(reinterpret_cast<uint32_t*>(blk + 4 * B))[o] = pp.x;
      G(reinterpret_cast<uint32_t*>(blk + 8 * B))[o] = pp.y;
    }
  } else {
    if (in) st_u32x2_nt(io.out_pay + dest, pp.x, pp.y);
    else st_u32x2(io.out_pay + dest, pp.x, pp.y);
  }
}

// One tile of a digit pass, its records in registers (the payloads possibly
// still arriving).  FULL: all kTile records present (no predicates).  RB
// bounds the digit width; digits are masked to nbits, so the ballots for bits
// nbits..RB-1 see all-zero bits and leave the peer masks unchanged.  Keys are
// staged by digit and stored, then payloads (the key registers are free by
// then, so the keys of the next tile (next_cnt > 0) load while this tile's
// payloads are stored).
//
// Ranking: for each item slot, the lanes holding the same digit (peers) come
// from one ballot per digit bit; a record's rank is the number of records of
// its digit in the wave's earlier slots plus its peers in lower lanes.  The
// lowest peer adds the slot's count to the wave's digit counter with an LDS
// atomic (the other lanes add to a private word), and the value it gets back
// reaches its peers through a lane permute a few slots later, so no slot
// waits on the one before it.
template <int RB, bool IN_BLOCKED, bool OUT_BLOCKED, bool FULL>
__device__ __forceinline__ void sort_tile(const SortIO& io, uint64_t base, uint32_t cnt, uint32_t shift,
                                          uint32_t nbits, const SortLds& L, uint32_t (&key)[kItems],
                                          uint2 (&pay)[kItems], uint64_t next_base, uint32_t next_cnt) {
  constexpr int NB = 1 << RB;
  constexpr int kLag = 4;  // slots between a counter add and the permute of its result
  const uint32_t nd = 1u << nbits, mask = nd - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t B = 1ull << io.log2B;

  uint32_t pos[kItems];  // rank: (peers below) | (lowest peer's lane << 8), then the rank itself
  uint32_t prv[kItems];  // counter value returned to the lowest peer
#pragma unroll
  for (int k = 0; k < kItems + kLag; ++k) {
    if (k < kItems) {
      const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
      const bool valid = FULL || lj < cnt;
      const uint32_t dg = (key[k] >> shift) & mask;
      uint32_t plo = ~0u, phi = ~0u;
      if (!FULL) {
        const uint64_t v = __ballot(valid);
        plo = (uint32_t)v;
        phi = (uint32_t)(v >> 32);
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t sb = (uint32_t)((int32_t)(dg << (31 - b)) >> 31);  // bit b, all ones or zero
        const uint64_t m = __ballot(sb != 0u);
        plo &= ~((uint32_t)m ^ sb);
        phi &= ~((uint32_t)(m >> 32) ^ sb);
      }
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
      const uint32_t tot = (uint32_t)__popc(plo) + (uint32_t)__popc(phi);
      // lowest peer (bit 63 keeps the operand nonzero; a valid lane is its own peer)
      const uint32_t lead = (uint32_t)__builtin_ctzll(((uint64_t)phi << 32) | plo | (1ull << 63));
      uint32_t* ctr = (valid && below == 0) ? &L.wh[wave * NB + dg] : &L.sink[threadIdx.x];
      prv[k] = atomicAdd(ctr, tot);
      pos[k] = below | (lead << 8);
    }
    if (k >= kLag) {
      const int q = k - kLag;
      const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((pos[q] >> 8) << 2), (int)prv[q]);
      pos[q] = prev + (pos[q] & 0xFFu);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the lag: no permute moves up to its add
  }
  lds_barrier();

  // thread d: digit d's counts over the waves become each wave's first tile
  // position; the tile's digit starts are an exclusive scan of the totals
  {
    const uint32_t d = threadIdx.x;  // NB <= kSortThreads
    uint32_t c[kSortWaves];
    uint32_t tot = 0;
#pragma unroll
    for (int v = 0; v < kSortWaves; ++v) {
      c[v] = d < nd ? L.wh[v * NB + d] : 0u;
      const uint32_t t = c[v];
      c[v] = tot;
      tot += t;
    }
    const uint32_t inc = wave_inclusive_scan(tot);
    if (lane == 63) L.tmp[wave] = inc;
    lds_barrier();
    uint32_t start = inc - tot;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w)
      if (w < wave) start += L.tmp[w];
    if (d < nd) {
#pragma unroll
      for (int v = 0; v < kSortWaves; ++v) L.wh[v * NB + d] = start + c[v];
      const uint32_t r = L.run[d];
      const uint32_t lo = (r + 31u) & ~31u, hi = (r + tot) & ~31u;
      L.dig[d] = make_uint4(r - start, lo, hi > lo ? hi - lo : 0u, 0u);
      L.run[d] = r + tot;
    }
  }
  lds_barrier();

  // phase 1: keys staged by digit, stored as runs of equal digits
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
    if (FULL || lj < cnt) {
      const uint32_t dg = (key[k] >> shift) & mask;
      pos[k] += L.wh[wave * NB + dg];
      L.key[pos[k]] = key[k];
    }
  }
  lds_barrier();
  // Records whose 128-byte lines the run fills are stored streaming; the
  // partial lines at a run's ends stay cached, so that the neighbouring
  // tile's run can complete them in L2 before they reach HBM.
  const uint32_t dmask = (1u << io.dbits) - 1;
  uint32_t dest[kItems];
  uint32_t inner = 0;  // bit k: record k lies in a completely filled line
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t lp = (uint32_t)(k * kSortThreads + threadIdx.x);
    if (FULL || lp < cnt) {
      const uint32_t kk = L.key[lp];
      const uint32_t dg = (kk >> shift) & mask;
      const uint4 di = L.dig[dg];
      dest[k] = di.x + lp;
      const bool in = dest[k] - di.y < di.z;
      inner |= (uint32_t)in << k;
      if constexpr (OUT_BLOCKED) {
        char* blk = out_block(io, L, dest[k]);
        const uint64_t o = dest[k] & (B - 1);
        if (in) st_u32_nt(blk + 4 * o, kk >> io.dbits);
        else G(reinterpret_cast<uint32_t*>(blk))[o] = kk >> io.dbits;
        G(reinterpret_cast<int16_t*>(blk + 12 * B))[o] = (int16_t)(kk & dmask);
      } else {
        if (in) st_u32_nt(io.out_keys + dest[k], kk);
        else G(io.out_keys)[dest[k]] = kk;
      }
    }
  }
  // phase 2: payloads through their own buffer (the counters are free again
  // once every wave has read its positions above)
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t lj = (uint32_t)(wave * kItems * 64 + k * 64 + lane);
    if (FULL || lj < cnt) L.pay[pos[k]] = pay[k];
  }
  for (uint32_t d = threadIdx.x; d < nd; d += kSortThreads) {
#pragma unroll
    for (int v = 0; v < kSortWaves; ++v) L.wh[v * NB + d] = 0;
  }
  lds_barrier();
  if (next_cnt) load_keys_any<IN_BLOCKED>(io, next_base, next_cnt, key);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t lp = (uint32_t)(k * kSortThreads + threadIdx.x);
    if (FULL || lp < cnt) store_pay<OUT_BLOCKED>(io, L, dest[k], (inner >> k) & 1u, L.pay[lp]);
  }
  lds_barrier();  // the buffers are reused by the next tile
}

template <int RB, bool IN_BLOCKED, bool OUT_BLOCKED>
__global__ __launch_bounds__(kSortThreads) void k_downsweep(SortPack pk, const uint32_t* __restrict__ offsets) {
  constexpr int NB = 1 << RB;
  __shared__ uint32_t s_key[kTile];
  __shared__ uint2 s_pay[kTile];
  __shared__ uint32_t s_wh[kSortWaves * NB];
  __shared__ uint4 s_dig[NB];
  __shared__ uint32_t s_run[NB];
  __shared__ uint32_t s_tmp[kSortWaves];
  __shared__ uint32_t s_sink[kSortThreads];
  __shared__ char* s_blk[OUT_BLOCKED ? kLdsBlocks : 1];
  const int gr = range_index(pk);
  if (gr < 0) return;
  const SortSeg sg = sort_seg(pk, (uint32_t)gr);
  const uint32_t r = (uint32_t)gr - sg.range0, shift = sg.shift, nbits = sg.nbits;
  const uint32_t nd = 1u << nbits;
  const uint32_t n_out_blocks = (uint32_t)((sg.n + (1ull << sg.io.log2B) - 1) >> sg.io.log2B);
  const bool lds_tab = OUT_BLOCKED && n_out_blocks <= (uint32_t)kLdsBlocks;
  if (lds_tab)
    for (uint32_t b = threadIdx.x; b < n_out_blocks; b += kSortThreads) s_blk[b] = G(sg.io.out_blocks)[b];
  const SortLds L{s_key, s_pay, s_wh, s_dig, s_run, s_tmp, s_sink, lds_tab ? s_blk : nullptr};
  for (uint32_t d = threadIdx.x; d < nd; d += kSortThreads) {
    s_run[d] = offsets[sg.cbase + (uint64_t)d * sg.n_ranges + r] - sg.base;
#pragma unroll
    for (int v = 0; v < kSortWaves; ++v) s_wh[v * NB + d] = 0;
  }
  lds_barrier();
  const RangeTiles rt = range_tiles(sg, r);
  // the keys of each tile are loaded while the tile before it stores its
  // payloads; the payloads load at the start of their tile and are first
  // needed after the ranking
  uint32_t key[kItems];
  uint2 pay[kItems];
  load_keys_any<IN_BLOCKED>(sg.io, rt.start, rt.n_full ? (uint32_t)kTile : rt.tail, key);
  for (uint32_t t = 0; t < rt.n_full; ++t) {
    const uint32_t base = rt.start + t * (uint32_t)kTile;
    const uint32_t next_cnt = t + 1 < rt.n_full ? (uint32_t)kTile : rt.tail;
    load_pays<IN_BLOCKED, true>(sg.io, base, kTile, pay);
    sort_tile<RB, IN_BLOCKED, OUT_BLOCKED, true>(sg.io, base, kTile, shift, nbits, L, key, pay,
                                                 base + (uint32_t)kTile, next_cnt);
  }
  if (rt.tail) {
    const uint32_t base = rt.start + rt.n_full * (uint32_t)kTile;
    load_pays<IN_BLOCKED, false>(sg.io, base, rt.tail, pay);
    sort_tile<RB, IN_BLOCKED, OUT_BLOCKED, false>(sg.io, base, rt.tail, shift, nbits, L, key, pay, 0, 0u);
  }
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (reduce, scan of partials, downsweep)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n,
                                                          uint32_t* __restrict__ partial) {
  __shared__ uint32_t s_tmp[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t j = base + k * kThreads + threadIdx.x;
    if (j < n) sum += in[j];
  }
  uint32_t total;
  block_exclusive_scan(sum, s_tmp, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_partials(uint32_t* __restrict__ partial, uint64_t nb,
                                                            uint32_t* __restrict__ total_out) {
  __shared__ uint32_t s_tmp[kWaves];
  uint32_t carry = 0;
  for (uint64_t base = 0; base < nb; base += kThreads) {
    const uint64_t j = base + threadIdx.x;
    const uint32_t v = j < nb ? partial[j] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, s_tmp, &total);
    if (j < nb) partial[j] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_down(const uint32_t* in, uint32_t* out, uint64_t n,
                                                        const uint32_t* __restrict__ partial) {
  __shared__ uint32_t s_tmp[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t j = base + k;
    v[k] = j < n ? in[j] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t run = partial[blockIdx.x] + block_exclusive_scan(sum, s_tmp, &total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t j = base + k;
    if (j < n) out[j] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(256) void k_set_entries(const TabEntry* __restrict__ e, uint32_t n) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const TabEntry t = e[i];
    G(t.tab)[t.idx] = t.ptr;
  }
}

__global__ void k_set_ptrs(char** tab, uint32_t first, uint32_t count, uint64_t p0, uint64_t p1,
                           uint64_t p2, uint64_t p3, uint64_t p4, uint64_t p5, uint64_t p6,
                           uint64_t p7) {
  const uint64_t v[8] = {p0, p1, p2, p3, p4, p5, p6, p7};
  const uint32_t t = threadIdx.x;
  if (t < count && t < 8) tab[first + t] = reinterpret_cast<char*>(v[t]);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint64_t n) {
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x)
    p[j] = value;
}

// ---------------------------------------------------------------------------
// Connection-group index (Sec. 2.2): a connection opens a group when its
// source or delay differs from those of the previous connection.
//   flags: coalesced reads of (src, delay) at j and j-1, one wave64 ballot
//          per 64 positions -> a bitmap of group starts and per-tile counts
//   write: one thread per 32-bit bitmap word; a workgroup scan of the word
//          popcounts places every group start in order
// ---------------------------------------------------------------------------
constexpr int kGiItems = 32;
constexpr int kGiTile = kThreads * kGiItems;  // 8,192 positions = 256 bitmap words

__device__ __forceinline__ uint64_t group_key(char* const* __restrict__ blocks, int log2B, uint64_t j) {
  const uint64_t B = 1ull << log2B;
  const char* blk = G(blocks)[j >> log2B];
  const uint64_t o = j & (B - 1);
  return ((uint64_t)G(reinterpret_cast<const uint32_t*>(blk))[o] << 16) |
         (uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o];
}

__device__ __forceinline__ GiSeg gi_seg(const GiPack& pk, const uint32_t* table, uint32_t i) {
  if (pk.n_segs == 1) return pk.one;
  const uint32_t k = __builtin_amdgcn_readfirstlane(C(table, i));
  return C_struct(pk.segs, k);
}

__global__ __launch_bounds__(kThreads) void k_group_flags(GiPack pk, uint32_t* __restrict__ tile_flags) {
  __shared__ uint32_t s_tmp[kWaves];
  const GiSeg sg = gi_seg(pk, pk.seg_of_tile, blockIdx.x);
  const int log2B = pk.log2B;
  const uint32_t n = (uint32_t)sg.n;  // a segment holds < 2^32 connections
  char* const* blocks = sg.blocks;
  NG_GLOBAL uint32_t* bitmap = G(sg.bitmap);
  const uint32_t base = (blockIdx.x - sg.tile0) * (uint32_t)kGiTile;
  const uint64_t B = 1ull << log2B;
  const char* blk = C(blocks, base >> log2B);  // kGiTile divides the block size
  const uint64_t o0 = base & (B - 1);
  const NG_GLOBAL uint32_t* src = G(reinterpret_cast<const uint32_t*>(blk)) + o0;
  const NG_GLOBAL int16_t* del = G(reinterpret_cast<const int16_t*>(blk + 12 * B)) + o0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t c = 0;
  if (n - base >= (uint32_t)kGiTile) {
    // A full tile: each lane takes 4 consecutive positions per item with
    // 16-byte (source) and 8-byte (delay) loads; the position before a
    // lane's first is the last of the lane below (a shuffle), or for lane 0
    // one more load.  A bitmap word is the flags of 8 lanes, gathered by
    // three xor-shuffles.
    static_assert(kGiItems % 4 == 0, "4 positions per lane");
#pragma unroll 2
    for (int v = 0; v < kGiItems / 4; ++v) {
      const uint32_t lj = 4u * (uint32_t)(v * kThreads + threadIdx.x);
      const u32x4 s4 = *(const NG_GLOBAL u32x4*)(src + lj);
      const u32x2 d4 = *(const NG_GLOBAL u32x2*)(del + lj);
      const uint32_t d0 = d4.x & 0xFFFFu, d1 = d4.x >> 16, d2 = d4.y & 0xFFFFu, d3 = d4.y >> 16;
      uint32_t ps = __shfl_up(s4.w, 1), pd = __shfl_up(d3, 1);
      if (lane == 0) {
        const uint32_t j = base + lj;
        if (j > 0) {
          const uint64_t k = group_key(blocks, log2B, j - 1);
          ps = (uint32_t)(k >> 16);
          pd = (uint32_t)(k & 0xFFFFu);
        } else {
          ps = ~s4.x;  // position 0 opens a group
        }
      }
      const uint32_t nib = (((s4.x != ps) | (d0 != pd)) ? 1u : 0u) | (((s4.y != s4.x) | (d1 != d0)) ? 2u : 0u) |
                           (((s4.z != s4.y) | (d2 != d1)) ? 4u : 0u) | (((s4.w != s4.z) | (d3 != d2)) ? 8u : 0u);
      c += (uint32_t)__popc(nib);
      uint32_t w = nib << (4 * (lane & 7));
      w |= __shfl_xor(w, 1);
      w |= __shfl_xor(w, 2);
      w |= __shfl_xor(w, 4);
      if ((lane & 7) == 0) bitmap[(base + lj) >> 5] = w;
    }
  } else {
#pragma unroll 8
    for (int k = 0; k < kGiItems; ++k) {
      const uint32_t lj = k * kThreads + threadIdx.x;  // 64 consecutive positions per wave
      const uint32_t j = base + lj;
      bool f = false;
      if (j < n) {
        const uint64_t key = ((uint64_t)src[lj] << 16) | (uint16_t)del[lj];
        uint64_t prev;
        if (lj > 0) prev = ((uint64_t)src[lj - 1] << 16) | (uint16_t)del[lj - 1];
        else prev = j > 0 ? group_key(blocks, log2B, j - 1) : ~0ull;
        f = key != prev;
      }
      const uint64_t m = __ballot(f);
      if (lane == 0) {
        const uint32_t w = (base + k * kThreads + wave * 64) >> 5;  // two bitmap words
        if ((w << 5) < n) bitmap[w] = (uint32_t)m;
        if (((w + 1) << 5) < n) bitmap[w + 1] = (uint32_t)(m >> 32);
      }
      c += f ? 1u : 0u;
    }
  }
  uint32_t total;
  block_exclusive_scan(c, s_tmp, &total);
  if (threadIdx.x == 0) tile_flags[blockIdx.x] = total;
}

// group_start[g]: first connection of group g; group_src[g]: its source.
// Each wave takes 2,048 consecutive positions, one bitmap word per lane, and
// writes its groups in one of two orders. Sparse groups go lane by lane:
// each lane walks its own word's bits, as many rounds as the largest word
// count; a round's addresses are consecutive only where lanes hold one group
// each. Dense groups go 64 positions at a time, the flagged lanes taking
// consecutive group numbers: one fully coalesced round per 64 positions that
// hold a group. A lane-by-lane round is priced at four of those.
__global__ __launch_bounds__(kThreads) void k_group_write(GiPack pk, const uint32_t* __restrict__ tile_base) {
  static_assert(kGiTile == kWaves * 64 * 32, "one bitmap word per lane");
  __shared__ uint32_t s_cnt[kWaves];
  const GiSeg sg = gi_seg(pk, pk.seg_of_tile, blockIdx.x);
  const uint32_t n = (uint32_t)sg.n;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t base = (blockIdx.x - sg.tile0) * (uint32_t)kGiTile;
  const uint32_t wi = ((base + wave * 2048u) >> 5) + lane;  // this lane's bitmap word
  uint32_t bits = 0;
  if (wi * 32u < n) {
    bits = G(sg.bitmap)[wi];
    if (n - wi * 32u < 32u) bits &= (1u << (n - wi * 32u)) - 1u;
  }
  const uint32_t pc = (uint32_t)__popc(bits);
  uint32_t incl = pc, mx = pc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o);
    if (lane >= (uint32_t)o) incl += t;
    mx = max(mx, (uint32_t)__shfl_xor(mx, o));
  }
  if (lane == 63) s_cnt[wave] = incl;
  __syncthreads();
  uint32_t g = tile_base[blockIdx.x] - tile_base[sg.tile0];
  for (uint32_t w = 0; w < wave; ++w) g += s_cnt[w];
  const uint64_t B = 1ull << pk.log2B;
  const char* blk = C(sg.blocks, base >> pk.log2B);  // kGiTile divides the block size
  const NG_GLOBAL uint32_t* src = G(reinterpret_cast<const uint32_t*>(blk)) + (base & (B - 1)) + wave * 2048u;
  NG_GLOBAL uint32_t* gstart = G(sg.group_start);
  NG_GLOBAL uint32_t* gsrc = G(sg.group_src);
  const uint32_t p0 = base + wave * 2048u;  // first position of this wave
  const uint64_t nz = __ballot(bits != 0);
  uint64_t chunks = (nz | (nz >> 1)) & 0x5555555555555555ull;  // bit 2i: positions 64i.. hold a group
  if (4u * __builtin_amdgcn_readfirstlane(mx) <= (uint32_t)__popcll(chunks)) {
    uint32_t gl = g + incl - pc;
    while (bits) {
      const uint32_t j = 32u * lane + (uint32_t)(__ffs(bits) - 1);
      bits &= bits - 1;
      gstart[gl] = p0 + j;
      gsrc[gl] = src[j];
      ++gl;
    }
    return;
  }
  while (chunks) {
    const uint32_t i = (uint32_t)(__ffsll((unsigned long long)chunks) - 1) >> 1;
    chunks &= chunks - 1;
    const uint32_t lo = __builtin_amdgcn_readlane(bits, 2 * i), hi = __builtin_amdgcn_readlane(bits, 2 * i + 1);
    const uint64_t m = ((uint64_t)hi << 32) | lo;
    if ((m >> lane) & 1ull) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
      gstart[g + below] = p0 + 64u * i + lane;
      gsrc[g + below] = src[64u * i + lane];
    }
    g += (uint32_t)__popcll(m);
  }
}

// Eq. (14): p_i = sum_{j<i} G_j = the number of groups whose source is below
// i, found by binary search in the sorted group sources (i = 0..n_nodes).
__global__ __launch_bounds__(kThreads) void k_group_ptr(GiPack pk, const uint32_t* __restrict__ tile_base) {
  const GiSeg sg = gi_seg(pk, pk.seg_of_ptr_block, blockIdx.x);
  const uint32_t lb = blockIdx.x - sg.ptr_block0;
  const uint32_t ng = tile_base[sg.tile0 + sg.n_tiles] - tile_base[sg.tile0];  // G
  if (lb == 0 && threadIdx.x == 0) {
    *G(sg.n_groups) = ng;
    G(sg.group_start)[ng] = (uint32_t)sg.n;  // group_start[G] = n closes the last group
  }
  const NG_GLOBAL uint32_t* group_src = G(sg.group_src);
  for (uint64_t i = (uint64_t)lb * kThreads + threadIdx.x; i <= sg.n_nodes;
       i += (uint64_t)sg.n_ptr_blocks * kThreads) {
    uint32_t lo = 0, hi = ng;  // first g with group_src[g] >= i
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (group_src[mid] < i) lo = mid + 1; else hi = mid;
    }
    G(sg.group_ptr)[i] = lo;
  }
}

template <int RB>
hipError_t upsweep_rb(const SortPack& pk, uint32_t* counts, hipStream_t s) {
  const dim3 grid(8 * pk.ranges_per_xcd);
  if (pk.one.io.in_blocks)
    hipLaunchKernelGGL((k_upsweep<RB, true>), grid, dim3(kSortThreads), 0, s, pk, counts);
  else
    hipLaunchKernelGGL((k_upsweep<RB, false>), grid, dim3(kSortThreads), 0, s, pk, counts);
  return hipGetLastError();
}

template <int RB>
hipError_t downsweep_rb(const SortPack& pk, const uint32_t* offsets, hipStream_t s) {
  const dim3 grid(8 * pk.ranges_per_xcd);
  const bool ib = pk.one.io.in_blocks != nullptr, ob = pk.one.io.out_blocks != nullptr;
  if (ib && ob)
    hipLaunchKernelGGL((k_downsweep<RB, true, true>), grid, dim3(kSortThreads), 0, s, pk, offsets);
  else if (ib)
    hipLaunchKernelGGL((k_downsweep<RB, true, false>), grid, dim3(kSortThreads), 0, s, pk, offsets);
  else if (ob)
    hipLaunchKernelGGL((k_downsweep<RB, false, true>), grid, dim3(kSortThreads), 0, s, pk, offsets);
  else
    hipLaunchKernelGGL((k_downsweep<RB, false, false>), grid, dim3(kSortThreads), 0, s, pk, offsets);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// pairwise_bernoulli: pair (a, b) connects when word a*N_t + b of stream 0 is
// below p * 2^32 (never a self-pair when those are prohibited).  A workgroup
// takes one unit of kPbUnit targets of one row, 16 consecutive pairs per
// thread; the counting pass and the writing pass evaluate the same words.
// ---------------------------------------------------------------------------
constexpr int kPbThreads = 256;
constexpr int kPbPer = kPbUnit / kPbThreads;  // 16 pairs per thread

__device__ __forceinline__ uint32_t pb_bits(const GenDesc& d, uint32_t a, uint32_t b0, uint32_t key0,
                                            uint32_t key1) {
  // bit k: pair (a, b0 + k) connects, for the pairs of this thread inside the row
  uint32_t bits = 0;
  uint64_t blk = ~0ull;
  uint32_t w4[4] = {0, 0, 0, 0};
  for (int k = 0; k < kPbPer; ++k) {
    const uint32_t b = b0 + k;
    if (b >= d.nt) break;
    const uint64_t q = (uint64_t)a * d.nt + b;
    if ((q >> 2) != blk) {
      blk = q >> 2;
      philox_block(blk, d.cid, kStreamSrc, key0, key1, w4);  // the decisions' stream
    }
    const uint32_t x = w4[0] * ((q & 3) == 0) + w4[1] * ((q & 3) == 1) + w4[2] * ((q & 3) == 2) + w4[3] * ((q & 3) == 3);
    const bool self = d.no_self && d.s0 + a == d.t0 + b;
    if (!self && (uint64_t)x < d.p_thr) bits |= 1u << k;
  }
  return bits;
}

__global__ __launch_bounds__(kPbThreads) void k_pb_count(GenDesc d, const uint32_t* __restrict__ key,
                                                         uint32_t* __restrict__ counts, uint16_t* __restrict__ dbits) {
  __shared__ uint32_t s_tmp[kPbThreads / 64];
  const uint32_t key0 = C(key, 0), key1 = C(key, 1);
  const uint32_t upr = (d.nt + kPbUnit - 1) / kPbUnit;
  const uint64_t units = (uint64_t)d.ns * upr;
  for (uint64_t u = blockIdx.x; u < units; u += gridDim.x) {
    const uint32_t a = (uint32_t)(u / upr), c = (uint32_t)(u - (uint64_t)a * upr);
    const uint32_t bits = pb_bits(d, a, c * kPbUnit + threadIdx.x * kPbPer, key0, key1);
    if (dbits) G(dbits)[u * kPbThreads + threadIdx.x] = (uint16_t)bits;
    uint32_t total;
    (void)block_exclusive_scan((uint32_t)__popc(bits), s_tmp, &total);
    if (threadIdx.x == 0) counts[u] = total;
    __syncthreads();  // s_tmp is reused by the next unit
  }
}

// Writing pass.  The unit's connections are numbered j = offsets[u] + l,
// l = 0..total-1 in pair order; their target offsets are staged in LDS, then
// each lane takes an aligned quad of connection indices: one stream-2 block
// gives the quad's delays and one stream-1 block its weights (the draws of
// synapses 4q..4q+3 of a generated call), so a block is evaluated once per
// four connections instead of once per connection.  A unit's connections
// span at most two blocks (a block holds >= 2^16 connections), whose
// addresses are read once per unit; the next unit's decisions and offset
// load while this unit is written.  A quad that is whole, inside one block
// and 4-aligned there is written with vector stores.
__global__ __launch_bounds__(kPbThreads) void k_pb_write(GenDesc d, const uint32_t* __restrict__ key,
                                                         const uint32_t* __restrict__ offsets,
                                                         const uint16_t* __restrict__ dbits,
                                                         char* const* __restrict__ blocks, int log2B) {
  __shared__ uint32_t s_tmp[kPbThreads / 64];
  __shared__ uint16_t s_b[kPbUnit];  // target offset within the unit of local connection l
  const uint32_t key0 = C(key, 0), key1 = C(key, 1);
  const uint64_t B = 1ull << log2B;
  const uint32_t upr = (d.nt + kPbUnit - 1) / kPbUnit;
  const uint64_t units = (uint64_t)d.ns * upr;
  uint64_t u = blockIdx.x;
  uint32_t bits_next = 0, off_next = 0;
  if (u < units) {
    if (dbits) bits_next = G(dbits)[u * kPbThreads + threadIdx.x];
    off_next = offsets[u];
  }
  for (; u < units; u += gridDim.x) {
    const uint32_t a = (uint32_t)(u / upr), c = (uint32_t)(u - (uint64_t)a * upr);
    uint32_t bits = dbits ? bits_next : pb_bits(d, a, c * kPbUnit + threadIdx.x * kPbPer, key0, key1);
    const uint64_t j0 = off_next;
    const uint64_t un = u + gridDim.x;
    if (un < units) {
      if (dbits) bits_next = G(dbits)[un * kPbThreads + threadIdx.x];
      off_next = offsets[un];
    }
    uint32_t total;
    uint32_t l = block_exclusive_scan((uint32_t)__popc(bits), s_tmp, &total);
    while (bits) {
      const uint32_t k = (uint32_t)(__ffs(bits) - 1);
      bits &= bits - 1;
      s_b[l++] = (uint16_t)(threadIdx.x * kPbPer + k);
    }
    __syncthreads();
    if (total) {
      const uint64_t j1 = j0 + total;  // this unit's connections [j0, j1)
      const uint64_t q0 = j0 >> 2, nq = ((j1 - 1) >> 2) - q0 + 1;
      const uint32_t src = d.s0 + a, tgt0 = d.t0 + c * kPbUnit;
      const uint64_t bA = (d.pos0 + j0) >> log2B, bZ = (d.pos0 + j1 - 1) >> log2B;  // bZ <= bA + 1
      char* const blkA = G(blocks)[bA];
      char* const blkZ = bZ != bA ? G(blocks)[bZ] : blkA;
      for (uint64_t qi = threadIdx.x; qi < nq; qi += kPbThreads) {
        const uint64_t q = q0 + qi;
        uint32_t xd[4] = {0, 0, 0, 0}, y[4] = {0, 0, 0, 0};
        if (d.d_kind != D_CONST) philox_block(q, d.cid, kStreamDelay, key0, key1, xd);
        float w[4] = {d.w_a, d.w_a, d.w_a, d.w_a};
        if (d.w_kind != W_CONST) {
          philox_block(q, d.cid, kStreamW, key0, key1, y);
          if (d.w_kind == W_NORMAL) {
            normal_pair(d, y[0], y[1], w[0], w[1]);
            normal_pair(d, y[2], y[3], w[2], w[3]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) w[r] = uniform_weight(d, y[r]);
          }
        }
        int32_t dl[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) dl[r] = d.d_kind != D_CONST ? delay_from_word(d, xd[r]) : d.d_const;
        const uint64_t p4 = d.pos0 + 4 * q;
        const bool whole = 4 * q >= j0 && 4 * q + 3 < j1;
        if (whole && (p4 & 3) == 0) {
          // p4 is 4-aligned and a block holds a multiple of 4, so the quad is in one block
          char* blk = (p4 >> log2B) == bA ? blkA : blkZ;
          const uint64_t o = p4 & (B - 1);
          const uint32_t lq = (uint32_t)(4 * q - j0);
          *(NG_GLOBAL u32x4*)(blk + 4 * o) = u32x4{src, src, src, src};
          *(NG_GLOBAL u32x4*)(blk + 4 * B + 4 * o) =
              u32x4{tgt0 + s_b[lq], tgt0 + s_b[lq + 1], tgt0 + s_b[lq + 2], tgt0 + s_b[lq + 3]};
          *(NG_GLOBAL u32x4*)(blk + 8 * B + 4 * o) =
              u32x4{__float_as_uint(w[0]), __float_as_uint(w[1]), __float_as_uint(w[2]), __float_as_uint(w[3])};
          *(NG_GLOBAL u32x2*)(blk + 12 * B + 2 * o) =
              u32x2{((uint32_t)dl[0] & 0xFFFFu) | ((uint32_t)dl[1] << 16), ((uint32_t)dl[2] & 0xFFFFu) | ((uint32_t)dl[3] << 16)};
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint64_t j = 4 * q + r;
            if (j < j0 || j >= j1) continue;
            const uint64_t p = d.pos0 + j;
            char* blk = (p >> log2B) == bA ? blkA : blkZ;
            const uint64_t o = p & (B - 1);
            G(reinterpret_cast<uint32_t*>(blk))[o] = src;
            G(reinterpret_cast<uint32_t*>(blk + 4 * B))[o] = tgt0 + s_b[j - j0];
            G(reinterpret_cast<float*>(blk + 8 * B))[o] = w[r];
            G(reinterpret_cast<int16_t*>(blk + 12 * B))[o] = (int16_t)dl[r];
          }
        }
      }
    }
    __syncthreads();  // s_b and s_tmp are reused by the next unit
  }
}

// ---------------------------------------------------------------------------
// Spike buffers and delivery (Sec. 2.3).  Each node holds a ring of `cap`
// spike slots (time index, group index within the node, multiplicity).  A
// step advances every queued spike; a spike whose time index reaches its
// group's delay enters the spike array and moves to the next group (a node's
// groups are in ascending delay); finished spikes leave the front of the
// ring.  Delivery gives one wave to each spike-array entry, a lane to each of
// the group's connections.  Then the emitting nodes push new spikes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spikes_init(SpikeState st, uint64_t n_groups) {
  const uint64_t B = 1ull << st.log2B;
  const uint64_t n = max((uint64_t)st.n_nodes, n_groups);
  for (uint64_t j = blockIdx.x * 256ull + threadIdx.x; j < n; j += gridDim.x * 256ull) {
    if (j < n_groups) {
      const uint32_t p = G(st.group_start)[j];
      const char* blk = G(st.blocks)[p >> st.log2B];
      G(st.gdelay)[j] = G(reinterpret_cast<const int16_t*>(blk + 12 * B))[p & (B - 1)];
    }
    if (j < st.n_nodes) {
      G(st.head)[j] = 0;
      G(st.count)[j] = 0;
      G(st.stamp)[j] = 0xFFFFFFFFu;
    }
  }
}

// The spike-array entries of step k are counted in n_entries[k & 1]; the
// advance of step k clears the other word for step k + 1 (its last reader, the
// delivery of step k - 1, has finished), so no launch clears the counter.
constexpr int kAdvThreads = 1024;

__global__ __launch_bounds__(kAdvThreads) void k_spikes_advance(SpikeState st, uint32_t step) {
  constexpr uint32_t kFast = 4;  // queued spikes a node keeps in registers
  __shared__ uint32_t s_wave[kAdvThreads / 64 + 1];
  const uint32_t i = blockIdx.x * kAdvThreads + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (i == 0) G(st.n_entries)[(step + 1) & 1] = 0;
  uint32_t cnt = 0, h = 0, base = 0, gi = 0;
  if (i < st.n_nodes) {
    cnt = G(st.count)[i];
    h = G(st.head)[i];
    base = G(st.group_ptr)[i];
    gi = G(st.group_ptr)[i + 1] - base;
  }
  const uint64_t q0 = (uint64_t)i * st.cap;
  // time indices grow by one; count the spikes that reach their group's delay.
  // Up to kFast spikes (almost every node at biological rates) are read once
  // and kept in registers; a longer queue is walked in global memory.
  const bool fast = cnt <= kFast;
  uint32_t sl[kFast], t[kFast], g[kFast];
  uint32_t hit_mask = 0, hits = 0;
  if (fast) {
    uint32_t r = h;
#pragma unroll
    for (uint32_t e = 0; e < kFast; ++e) {
      sl[e] = r;
      r = r + 1 == st.cap ? 0 : r + 1;
      t[e] = 0;
      g[e] = 0;
      if (e < cnt) {
        t[e] = G(st.time)[q0 + sl[e]] + 1;
        g[e] = G(st.group)[q0 + sl[e]];
      }
    }
#pragma unroll
    for (uint32_t e = 0; e < kFast; ++e)
      if (e < cnt && (int32_t)t[e] == G(st.gdelay)[base + g[e]]) hit_mask |= 1u << e;
    hits = (uint32_t)__popc(hit_mask);
  } else {
    for (uint32_t e = 0; e < cnt; ++e) {
      const uint64_t q = q0 + (h + e) % st.cap;
      const uint32_t tt = G(st.time)[q] + 1;
      G(st.time)[q] = tt;
      if ((int32_t)tt == G(st.gdelay)[base + G(st.group)[q]]) ++hits;
    }
  }
  // one counter update per workgroup (the grid's updates of one word serialize)
  uint32_t incl = hits;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o);
    if (lane >= (uint32_t)o) incl += v;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < kAdvThreads / 64; ++w) {
      const uint32_t c = s_wave[w];
      s_wave[w] = run;
      run += c;
    }
    s_wave[kAdvThreads / 64] = run ? atomicAdd(st.n_entries + (step & 1), run) : 0u;
  }
  __syncthreads();
  uint32_t pos = s_wave[kAdvThreads / 64] + s_wave[wave] + incl - hits;
  if (fast) {
#pragma unroll
    for (uint32_t e = 0; e < kFast; ++e) {
      if (e >= cnt) break;
      const uint64_t q = q0 + sl[e];
      G(st.time)[q] = t[e];
      if ((hit_mask >> e) & 1u) {
        st_u32x2(st.entries + pos++, base + g[e], G(st.mult)[q]);
        G(st.group)[q] = ++g[e];
      }
    }
    // the oldest spikes finish first (a node's spikes pass the same delays in
    // emission order): drop the finished ones from the front
    uint32_t fin = 0;
#pragma unroll
    for (uint32_t e = 0; e < kFast; ++e)
      if (e < cnt && fin == e && g[e] == gi) ++fin;
    if (fin) h = sl[fin - 1] + 1 == st.cap ? 0 : sl[fin - 1] + 1;
    cnt -= fin;
  } else {
    for (uint32_t e = 0; e < cnt && hits; ++e) {
      const uint64_t q = q0 + (h + e) % st.cap;
      const uint32_t gg = G(st.group)[q];
      if ((int32_t)G(st.time)[q] == G(st.gdelay)[base + gg]) {
        st_u32x2(st.entries + pos++, base + gg, G(st.mult)[q]);
        G(st.group)[q] = gg + 1;
      }
    }
    while (cnt && G(st.group)[q0 + h] == gi) {
      h = h + 1 == st.cap ? 0 : h + 1;
      --cnt;
    }
  }
  if (i < st.n_nodes) {
    G(st.head)[i] = h;
    G(st.count)[i] = cnt;
  }
}

__global__ __launch_bounds__(256) void k_spikes_deliver(SpikeState st, float* __restrict__ input, uint32_t step) {
  const uint64_t B = 1ull << st.log2B;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_e = __builtin_amdgcn_readfirstlane(G(st.n_entries)[step & 1]);
  const uint32_t waves = gridDim.x * 4;
  for (uint32_t e = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); e < n_e; e += waves) {
    const uint2 en = ld_u32x2(st.entries + e);
    const uint32_t a = G(st.group_start)[en.x], b = G(st.group_start)[en.x + 1];
    const float m = (float)en.y;
    // the group's connections are consecutive: the block of its first one is
    // read once per entry, any other block only where the group reaches it
    const uint32_t ba = a >> st.log2B;
    const char* const blk_a = G(st.blocks)[ba];
    for (uint32_t j = a + lane; j < b; j += 64) {
      const char* blk = (j >> st.log2B) == ba ? blk_a : G(st.blocks)[j >> st.log2B];
      const uint64_t o = j & (B - 1);
      const uint32_t t = G(reinterpret_cast<const uint32_t*>(blk + 4 * B))[o];
      const float w = G(reinterpret_cast<const float*>(blk + 8 * B))[o];
      unsafeAtomicAdd(input + t, w * m);
    }
  }
}

__global__ __launch_bounds__(256) void k_spikes_push(SpikeState st, const uint32_t* __restrict__ nodes,
                                                     const uint32_t* __restrict__ mult, uint32_t n, uint32_t step) {
  for (uint64_t k = blockIdx.x * 256ull + threadIdx.x; k < n; k += gridDim.x * 256ull) {
    const uint32_t i = G(nodes)[k];
    if (i >= st.n_nodes) {
      atomicOr(st.err, 4u);
      continue;
    }
    if (atomicExch(st.stamp + i, step) == step) {  // the node already emitted in this step
      atomicOr(st.err, 2u);
      continue;
    }
    if (G(st.group_ptr)[i + 1] == G(st.group_ptr)[i]) continue;  // no outgoing connections
    const uint32_t c = atomicAdd(st.count + i, 1u);
    if (c >= st.cap) {  // cannot happen with one spike per node and step; never write past the ring
      atomicSub(st.count + i, 1u);
      atomicOr(st.err, 2u);
      continue;
    }
    const uint64_t sl = (uint64_t)i * st.cap + (G(st.head)[i] + c) % st.cap;
    G(st.time)[sl] = 0;
    G(st.group)[sl] = 0;
    G(st.mult)[sl] = mult ? G(mult)[k] : 1u;
  }
}

// ---------------------------------------------------------------------------
// Node groups as index arrays and per-connection weights and delays
// (Sec. 2.1): before a call changes anything, one pass finds the largest
// source and target index, the largest delay (its fp32 bits, delays being
// non-negative) and whether a delay is not finite.  Generation then runs with
// the groups as position ranges from 0 and maps each synapse through the
// arrays as it stores it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_check_arrays(CallArrays a, unsigned long long* out, uint32_t epoch) {
  constexpr int U = 8;  // independent loads in flight per thread and round
  uint32_t ms = 0, mt = 0, md = 0, bad = 0;
  const uint64_t n = max(max(a.ns, a.nt), a.n);
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t j0 = blockIdx.x * 256ull + threadIdx.x; j0 < n; j0 += U * stride) {
    uint32_t vs[U], vt[U];
    float vd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t j = j0 + u * stride;
      vs[u] = a.src_idx && j < a.ns ? G(a.src_idx)[j] : 0u;
      vt[u] = a.tgt_idx && j < a.nt ? G(a.tgt_idx)[j] : 0u;
      vd[u] = a.d_ms && j < a.n ? G(a.d_ms)[j] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ms = max(ms, vs[u]);
      mt = max(mt, vt[u]);
      // the step count is monotone in the delay: the largest delay in ms
      // (bits of a non-negative float order like the float) is converted once
      if (vd[u] != vd[u]) bad = 1;
      else md = max(md, __float_as_uint(fmaxf(vd[u], 0.0f)));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ms = max(ms, (uint32_t)__shfl_xor(ms, o));
    mt = max(mt, (uint32_t)__shfl_xor(mt, o));
    md = max(md, (uint32_t)__shfl_xor(md, o));
    bad |= (uint32_t)__shfl_xor(bad, o);
  }
  // one atomic per workgroup and word: the four words are shared by the whole grid
  __shared__ uint32_t red[4][4];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ms;
    red[1][threadIdx.x >> 6] = mt;
    red[2][threadIdx.x >> 6] = md;
    red[3][threadIdx.x >> 6] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    uint32_t v = red[threadIdx.x][0];
    for (int w = 1; w < 4; ++w) v = threadIdx.x == 3 ? (v | red[3][w]) : max(v, red[threadIdx.x][w]);
    // the epoch in the high word: values left by earlier calls are smaller
    atomicMax(out + threadIdx.x, ((unsigned long long)epoch << 32) | v);
  }
}


// ---------------------------------------------------------------------------
// COPASS in-place block sort (Appendix A): the copies of left partitions to
// the auxiliary array and of right partitions through a bounce buffer, and
// the partition search.
// ---------------------------------------------------------------------------
constexpr int kCopyThreads = 256;
constexpr int kCopyItems = 8;

__device__ __forceinline__ uint32_t view_key(const BlockView& v, uint32_t p) {
  const uint64_t B = 1ull << v.log2B;
  const char* blk = G(v.blocks)[p >> v.log2B];
  const uint64_t o = p & (B - 1);
  return (G(reinterpret_cast<const uint32_t*>(blk))[o] << v.dbits) |
         (uint32_t)(uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o];
}

// Each workgroup copies kCopyThreads * kCopyItems consecutive records of the
// list; a record finds its piece by walking forward from the piece of the
// workgroup's first record (pieces are long, so the walk is short).
template <bool TO_PACKED>
__global__ __launch_bounds__(kCopyThreads) void k_copass_copy(BlockView v, CopyList l, uint32_t* __restrict__ keys,
                                                              uint2* __restrict__ pay) {
  const uint64_t B = 1ull << v.log2B;
  const uint64_t per = kCopyThreads * kCopyItems;
  for (uint64_t base = blockIdx.x * per; base < l.total; base += gridDim.x * per) {
    uint32_t a = 0, b = l.n_segs;  // last piece with pre <= base
    while (b - a > 1) {
      const uint32_t mid = (a + b) / 2;
      if (G(l.segs)[mid].pre <= base) a = mid;
      else b = mid;
    }
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(a);
#pragma unroll
    for (int j = 0; j < kCopyItems; ++j) {
      const uint64_t r = base + j * kCopyThreads + threadIdx.x;
      if (r >= l.total) break;
      uint32_t sg = s0;
      while (sg + 1 < l.n_segs && G(l.segs)[sg + 1].pre <= r) ++sg;
      const u32x4 sq = *(const NG_GLOBAL u32x4*)(const void*)(l.segs + sg);  // (src, dst, len, pre)
      const CopySeg cs{sq.x, sq.y, sq.z, sq.w};
      const uint32_t o = (uint32_t)r - cs.pre;
      if constexpr (TO_PACKED) {
        const uint32_t p = cs.src + o;
        const char* blk = G(v.blocks)[p >> v.log2B];
        const uint64_t q = p & (B - 1);
        const uint32_t src = G(reinterpret_cast<const uint32_t*>(blk))[q];
        const uint32_t tgt = G(reinterpret_cast<const uint32_t*>(blk + 4 * B))[q];
        const uint32_t w = G(reinterpret_cast<const uint32_t*>(blk + 8 * B))[q];
        const uint32_t d = (uint32_t)(uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[q];
        G(keys)[cs.dst + o] = (src << v.dbits) | d;
        st_u32x2(pay + cs.dst + o, tgt, w);
      } else {
        const uint32_t kk = G(keys)[cs.src + o];
        const uint2 pp = ld_u32x2(pay + cs.src + o);
        const uint32_t p = cs.dst + o;
        char* blk = G(v.blocks)[p >> v.log2B];
        const uint64_t q = p & (B - 1);
        G(reinterpret_cast<uint32_t*>(blk))[q] = kk >> v.dbits;
        G(reinterpret_cast<uint32_t*>(blk + 4 * B))[q] = pp.x;
        G(reinterpret_cast<uint32_t*>(blk + 8 * B))[q] = pp.y;
        G(reinterpret_cast<int16_t*>(blk + 12 * B))[q] = (int16_t)(kk & ((1u << v.dbits) - 1u));
      }
    }
  }
}

constexpr int kPartThreads = 1024;
constexpr int kPartWaves = kPartThreads / 64;

__device__ __forceinline__ uint64_t part_sum(uint64_t x, uint64_t* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  uint64_t t = 0;
#pragma unroll
  for (int w = 0; w < kPartWaves; ++w) t += red[w];
  return t;
}

// exclusive prefix of x over the threads in order
__device__ __forceinline__ uint64_t part_excl(uint64_t x, uint64_t* red) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t n = __shfl_up(inc, o);
    if (lane >= (uint32_t)o) inc += n;
  }
  __syncthreads();
  if (lane == 63) red[wave] = inc;
  __syncthreads();
  uint64_t before = 0;
  for (uint32_t w = 0; w < wave; ++w) before += red[w];
  return before + inc - x;
}

// number of keys of subarray (at position st) with index in [a, b) that are
// <= t (le) or < t (!le), plus a; the answer is known to lie in [a, b] and
// the keys ascend.  One wave, all lanes active with the same arguments: each
// step probes 64 evenly spaced keys and keeps the slice between the last
// probe that passes and the first that fails (a 65-ary search: a bracket of
// 2^24 keys takes 4 steps and a final probe of <= 64 keys).
__device__ __forceinline__ uint32_t part_count(const BlockView& v, uint32_t st, uint32_t a, uint32_t b, uint32_t t,
                                               bool le) {
  const uint32_t lane = threadIdx.x & 63;
  while (b - a > 64) {
    const uint64_t span = b - a;  // >= 65: the probes a + floor(span (j+1) / 65) ascend strictly inside (a, b)
    const uint32_t x = view_key(v, st + a + (uint32_t)(span * (lane + 1) / 65));
    const uint32_t c = (uint32_t)__popcll(__ballot(le ? x <= t : x < t));  // the passing probes are 0..c-1
    const uint32_t na = c ? a + (uint32_t)(span * c / 65) + 1 : a;
    const uint32_t nb = c < 64 ? a + (uint32_t)(span * (c + 1) / 65) : b;
    a = na;
    b = nb;
  }
  const bool in = lane < b - a;
  const uint32_t x = in ? view_key(v, st + a + lane) : 0u;
  return a + (uint32_t)__popcll(__ballot(in && (le ? x <= t : x < t)));
}

// The partition search of the appendix.  Brackets [lo_i, hi_i]: lo_i counts
// the keys <= the lower threshold, hi_i those < the upper one.  Each round
// bisects the widest bracket (lowest i on ties), takes its middle key as the
// trial threshold t and counts every subarray's keys < t and <= t; if m lies
// between the sums, t is the threshold, else the bracket side that keeps m
// inside moves to t.  When every bracket has width <= 1, the subarrays of
// width one offer their next key and the smallest offers, by (key, i), fill
// the rest.  Thread t owns the brackets of subarrays [t*C, (t+1)*C); the
// counting searches of a round are spread over the waves.
__global__ __launch_bounds__(kPartThreads) void k_copass_partition(CopassPart p) {
  __shared__ uint64_t red[kPartWaves];
  __shared__ uint32_t s_w[kPartWaves], s_i[kPartWaves];
  const uint32_t k = p.k, m = p.m;
  const uint32_t C = (k + kPartThreads - 1) / kPartThreads;
  const uint32_t i0 = min(threadIdx.x * C, k), i1 = min(i0 + C, k);
  for (uint32_t i = i0; i < i1; ++i) {
    p.lo[i] = 0;
    p.hi[i] = p.len[i];
  }
  const uint32_t cap = 33u * (k + 1u);  // each round shrinks one bracket of < 2^32 to at most half
  uint32_t iter = 0, path = 0, err = 0;
  for (;;) {
    uint32_t bw = 0, bi = 0;
    for (uint32_t i = i0; i < i1; ++i) {
      const uint32_t w = p.hi[i] - p.lo[i];
      if (w > bw) {
        bw = w;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t ow = __shfl_xor(bw, o), oi = __shfl_xor(bi, o);
      if (ow > bw || (ow == bw && oi < bi)) {
        bw = ow;
        bi = oi;
      }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      s_w[threadIdx.x >> 6] = bw;
      s_i[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    bw = s_w[0];
    bi = s_i[0];
    for (int w = 1; w < kPartWaves; ++w)
      if (s_w[w] > bw || (s_w[w] == bw && s_i[w] < bi)) {
        bw = s_w[w];
        bi = s_i[w];
      }
    if (bw <= 1) break;
    if (++iter > cap) {
      err = 1;
      break;
    }
    const uint32_t t = view_key(p.v, p.start[bi] + (p.lo[bi] + p.hi[bi]) / 2);
    // counts at t: wave w searches subarrays w, w + kPartWaves, ... (the
    // brackets were last written before the barriers above)
    for (uint32_t i = threadIdx.x >> 6; i < k; i += kPartWaves) {
      const uint32_t st = p.start[i], lo = p.lo[i], hi = p.hi[i];
      const uint32_t mh = part_count(p.v, st, lo, hi, t, true);
      const uint32_t ml = part_count(p.v, st, lo, mh, t, false);
      if ((threadIdx.x & 63) == 0) {
        p.mu_hi[i] = mh;
        p.mu_lo[i] = ml;
      }
    }
    __syncthreads();
    uint64_t slo = 0, shi = 0;
    for (uint32_t i = i0; i < i1; ++i) {
      slo += p.mu_lo[i];
      shi += p.mu_hi[i];
    }
    slo = part_sum(slo, red);
    shi = part_sum(shi, red);
    if (slo <= m && m <= shi) {
      // t is the threshold: the keys equal to t fill d = m - sum mu_lo,
      // subarray by subarray in ascending i
      const uint64_t d = m - slo;
      uint64_t mine = 0;
      for (uint32_t i = i0; i < i1; ++i) mine += p.mu_hi[i] - p.mu_lo[i];
      uint64_t pre = part_excl(mine, red);
      for (uint32_t i = i0; i < i1; ++i) {
        const uint64_t cnt = p.mu_hi[i] - p.mu_lo[i];
        const uint64_t take = pre >= d ? 0 : (d - pre < cnt ? d - pre : cnt);
        p.m_out[i] = p.mu_lo[i] + (uint32_t)take;
        pre += cnt;
      }
      path = 1;
      break;
    }
    if (m < slo) {
      for (uint32_t i = i0; i < i1; ++i) p.hi[i] = p.mu_lo[i];
    } else {
      for (uint32_t i = i0; i < i1; ++i) p.lo[i] = p.mu_hi[i];
    }
  }
  if (!path && !err) {
    // brackets of width <= 1: offers of the width-one subarrays (their keys
    // kept in mu_lo); the d smallest by (key, i) go left
    uint64_t s = 0;
    for (uint32_t i = i0; i < i1; ++i) {
      s += p.lo[i];
      if (p.hi[i] == p.lo[i] + 1) p.mu_lo[i] = view_key(p.v, p.start[i] + p.lo[i]);
    }
    s = part_sum(s, red);
    const uint64_t d = m - s;
    // smallest key V with #{offers <= V} >= d
    uint32_t va = 0, vb = 0xFFFFFFFFu;
    while (va < vb) {
      const uint32_t mid = va + (vb - va) / 2;
      uint64_t c = 0;
      for (uint32_t i = i0; i < i1; ++i) c += (p.hi[i] == p.lo[i] + 1 && p.mu_lo[i] <= mid) ? 1u : 0u;
      c = part_sum(c, red);
      if (c >= d) vb = mid;
      else va = mid + 1;
    }
    uint64_t less = 0, eq = 0;
    for (uint32_t i = i0; i < i1; ++i)
      if (p.hi[i] == p.lo[i] + 1) {
        less += p.mu_lo[i] < va ? 1u : 0u;
        eq += p.mu_lo[i] == va ? 1u : 0u;
      }
    less = part_sum(less, red);
    const uint64_t need = d - less;  // offers equal to V that go left, lowest i first
    uint64_t pre = part_excl(eq, red);
    for (uint32_t i = i0; i < i1; ++i) {
      uint32_t add = 0;
      if (p.hi[i] == p.lo[i] + 1) {
        if (p.mu_lo[i] < va) add = 1;
        else if (p.mu_lo[i] == va) add = pre++ < need ? 1u : 0u;
      }
      p.m_out[i] = p.lo[i] + add;
    }
    path = 2;
  }
  if (threadIdx.x == 0) {
    p.status[0] = path;
    p.status[1] = iter;
    p.status[2] = err;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <int RULE>
static void gen_launch(const GenDesc& d, const uint32_t* key, char* const* blocks, int log2B, dim3 grid,
                       hipStream_t s) {
  if (d.d_kind == D_CONST)
    hipLaunchKernelGGL((k_generate<RULE, false>), grid, dim3(kGenThreads), 0, s, d, key, blocks, log2B);
  else
    hipLaunchKernelGGL((k_generate<RULE, true>), grid, dim3(kGenThreads), 0, s, d, key, blocks, log2B);
}

// Workgroups of a generation launch: each lane makes about quads_per_lane
// groups of four synapses (the kernels loop over their groups), at most
// 16,384 workgroups.
static uint32_t gen_grid(uint64_t groups, uint32_t quads_per_lane) {
  const uint64_t per_wg = (uint64_t)kGenThreads * (quads_per_lane ? quads_per_lane : 1);
  const uint64_t need = (groups + per_wg - 1) / per_wg;
  return (uint32_t)(need < 16384 ? (need ? need : 1) : 16384);
}

hipError_t launch_generate(const GenDesc& d, const uint32_t* d_key, char* const* d_blocks, int log2B,
                           hipStream_t s, uint32_t quads_per_lane) {
  if (d.n_new == 0) return hipSuccess;
  const dim3 grid(gen_grid(((uint64_t)d.n_new + 3) / 4, quads_per_lane));
  switch (d.rule) {
    case R_ONE_TO_ONE: gen_launch<R_ONE_TO_ONE>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_ALL_TO_ALL: gen_launch<R_ALL_TO_ALL>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_INDEG: gen_launch<R_INDEG>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_OUTDEG: gen_launch<R_OUTDEG>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_TOTAL: gen_launch<R_TOTAL>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_INDEG_D: gen_launch<R_INDEG_D>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_OUTDEG_D: gen_launch<R_OUTDEG_D>(d, d_key, d_blocks, log2B, grid, s); break;
    case R_TOTAL_D: gen_launch<R_TOTAL_D>(d, d_key, d_blocks, log2B, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_generate_batch(const GenDesc* d_descs, uint32_t n_calls, uint64_t total_groups,
                                 int log2B, hipStream_t s, uint32_t quads_per_lane) {
  if (n_calls == 0 || total_groups == 0) return hipSuccess;
  const dim3 grid(gen_grid(total_groups, quads_per_lane));
  hipLaunchKernelGGL(k_generate_batch, grid, dim3(kGenThreads), 0, s, d_descs, n_calls, total_groups, log2B);
  return hipGetLastError();
}

uint32_t sort_tile_size() { return kTile; }
int sort_max_radix_bits() { return kMaxRadixBits; }

hipError_t launch_upsweep(const SortPack& pk, uint32_t* counts, hipStream_t s) {
  if (pk.total_ranges == 0) return hipSuccess;
  if (pk.max_nbits > (uint32_t)kMaxRadixBits) return hipErrorInvalidValue;
  return pk.max_nbits <= 8 ? upsweep_rb<8>(pk, counts, s) : upsweep_rb<9>(pk, counts, s);
}

hipError_t launch_downsweep(const SortPack& pk, const uint32_t* offsets, hipStream_t s) {
  if (pk.total_ranges == 0) return hipSuccess;
  if (pk.max_nbits > (uint32_t)kMaxRadixBits) return hipErrorInvalidValue;
  return pk.max_nbits <= 8 ? downsweep_rb<8>(pk, offsets, s) : downsweep_rb<9>(pk, offsets, s);
}

uint64_t scan_tmp_words(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* tmp,
                                 uint32_t* total, hipStream_t s) {
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, total, 0u, (uint64_t)1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(kThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, tmp, nb, total);
  hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)nb), dim3(kThreads), 0, s, in, out, n, tmp);
  return hipGetLastError();
}

hipError_t launch_set_ptrs(char** tab, uint32_t first, uint32_t count, const uint64_t* v,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(64), 0, s, tab, first, count, v[0], v[1], v[2], v[3],
                     v[4], v[5], v[6], v[7]);
  return hipGetLastError();
}

hipError_t launch_pb_count(const GenDesc& d, const uint32_t* d_key, uint32_t* counts, uint16_t* bits,
                           hipStream_t s) {
  const uint64_t units = (uint64_t)d.ns * ((d.nt + kPbUnit - 1) / kPbUnit);
  if (units == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_count, dim3((uint32_t)std::min<uint64_t>(units, 65536)), dim3(kPbThreads), 0, s, d, d_key,
                     counts, bits);
  return hipGetLastError();
}

hipError_t launch_pb_write(const GenDesc& d, const uint32_t* d_key, const uint32_t* offsets, const uint16_t* bits,
                           char* const* blocks, int log2B, hipStream_t s) {
  const uint64_t units = (uint64_t)d.ns * ((d.nt + kPbUnit - 1) / kPbUnit);
  if (units == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_write, dim3((uint32_t)std::min<uint64_t>(units, 65536)), dim3(kPbThreads), 0, s, d, d_key,
                     offsets, bits, blocks, log2B);
  return hipGetLastError();
}

hipError_t launch_spikes_init(const SpikeState& st, uint64_t n_groups, hipStream_t s) {
  hipError_t e = launch_fill_u32(st.n_entries, 0u, 2, s);  // both step parities' entry counters
  if (e != hipSuccess) return e;
  const uint64_t n = std::max<uint64_t>(st.n_nodes, n_groups);
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_spikes_init, dim3(grid), dim3(256), 0, s, st, n_groups);
  return hipGetLastError();
}

hipError_t launch_spikes_step(const SpikeState& st, const uint32_t* nodes, const uint32_t* mult, uint32_t n,
                              float* input, uint32_t step, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (st.n_nodes) {
    hipLaunchKernelGGL(k_spikes_advance, dim3((st.n_nodes + kAdvThreads - 1) / kAdvThreads), dim3(kAdvThreads), 0, s,
                       st, step);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_spikes_deliver, dim3(2048), dim3(256), 0, s, st, input, step);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (n) {
    hipLaunchKernelGGL(k_spikes_push, dim3(std::min<uint32_t>((n + 255) / 256, 4096u)), dim3(256), 0, s, st, nodes,
                       mult, n, step);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_check_arrays(const CallArrays& a, uint64_t* out, uint32_t epoch, hipStream_t s) {
  const uint32_t n = std::max(std::max(a.ns, a.nt), a.n);
  if (n == 0) return hipSuccess;
  // each workgroup ends in one atomic per word; all of them share the four words
  const uint32_t grid = std::min<uint32_t>((n + 2047) / 2048, 512u);
  hipLaunchKernelGGL(k_check_arrays, dim3(grid), dim3(256), 0, s, a, reinterpret_cast<unsigned long long*>(out),
                     epoch);
  return hipGetLastError();
}


hipError_t launch_copass_copy(const BlockView& v, const CopyList& l, bool to_packed, uint32_t* keys, uint2* pay,
                              hipStream_t s) {
  if (l.total == 0) return hipSuccess;
  const uint32_t per = kCopyThreads * kCopyItems;
  const uint32_t grid = std::min<uint32_t>((l.total + per - 1) / per, 4096u);
  if (to_packed)
    hipLaunchKernelGGL(k_copass_copy<true>, dim3(grid), dim3(kCopyThreads), 0, s, v, l, keys, pay);
  else
    hipLaunchKernelGGL(k_copass_copy<false>, dim3(grid), dim3(kCopyThreads), 0, s, v, l, keys, pay);
  return hipGetLastError();
}

hipError_t launch_copass_partition(const CopassPart& p, hipStream_t s) {
  hipLaunchKernelGGL(k_copass_partition, dim3(1), dim3(kPartThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_set_entries(const TabEntry* d_entries, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_entries, dim3((n + 255) / 256), dim3(256), 0, s, d_entries, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

uint32_t gi_tile_size() { return kGiTile; }

uint32_t gi_ptr_blocks(uint32_t n_nodes) {
  const uint64_t b = ((uint64_t)n_nodes + 1 + kThreads - 1) / kThreads;
  return (uint32_t)(b < 4096 ? b : 4096);
}

hipError_t launch_group_flags(const GiPack& pk, uint32_t* tile_flags, hipStream_t s) {
  if (pk.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_flags, dim3(pk.total_tiles), dim3(kThreads), 0, s, pk, tile_flags);
  return hipGetLastError();
}

hipError_t launch_group_write(const GiPack& pk, const uint32_t* tile_base, hipStream_t s) {
  if (pk.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_write, dim3(pk.total_tiles), dim3(kThreads), 0, s, pk, tile_base);
  return hipGetLastError();
}

hipError_t launch_group_ptr(const GiPack& pk, const uint32_t* tile_base, hipStream_t s) {
  if (pk.total_ptr_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_ptr, dim3(pk.total_ptr_blocks), dim3(kThreads), 0, s, pk, tile_base);
  return hipGetLastError();
}

}  // namespace ng
