// Calibration (Sec. 2.2 of Golosio et al.) as a most-significant-digit sort,
// for gfx950 (MI355X).
//
// The connections are ordered stably by key = src << dbits | delay, and the
// group index of Eq. (14) is built.  The key is split into three digits from
// the top, key = D1 | D2 | D3:
//   A  every record, in creation order, goes to the bucket of its D1;
//   B  the records of each bucket go to the sub-bucket of their D2;
//   C  each sub-bucket -- a few thousand records -- is sorted by D3 in LDS
//      and written, contiguous and fully coalesced, as calibrated blocks; the
//      distinct keys it holds are the connection groups (Sec. 2.2), recorded
//      here and turned into group_start and group_ptr by one scan.
// A and B are stable scatter passes over tiles of 10,240 records: wave64
// ballot ranks, LDS staging by digit, runs of equal digits written to their
// scanned positions.  Each pass narrows the record: after A, a record holds
// only the key bits below D1 next to its target in one 32-bit word when they
// fit, so B and C move 8 bytes per record instead of 12.  With no pass over
// the creation-order keys after A and the group starts found inside C, the
// path moves the creation-order record once, the narrow record twice and
// the calibrated record once.
//
// Buckets, sub-buckets and the ranges of pass B live on the device: small
// kernels turn the scanned counts into start tables, and every launch size
// is an upper bound, so the calibration needs no value from the device and
// can be captured in a graph.
#include "ng_internal.h"
#include "ng_device.h"

namespace ng {
namespace {

constexpr int kMThreads = 512;
// The counting passes run 1,024 threads (more loads in flight per CU: on the
// 3e8 microcircuit 0.30 -> 0.295 ms for the first count, 0.254 -> 0.239 ms
// for the second, against 512).
constexpr int kCntThreads = 1024;
constexpr int kMWaves = kMThreads / 64;
constexpr int kMItems = (int)kMsdTile / kMThreads;   // tile of pass A and of unpacked records
constexpr int kMItemsN = (int)kMsdTileN / kMThreads;  // tile of packed records (passes B and C)
static_assert(kMThreads * kMItems == (int)kMsdTile, "tile of unpacked records");
static_assert(kMThreads * kMItemsN == (int)kMsdTileN, "tile of packed records");
constexpr int kMNB = 1 << kMsdMaxDigit;  // 512 digit values at most
static_assert(kMThreads >= kMNB, "one thread per digit value");
static_assert(kMWaves % 2 == 0, "wave counters come in pairs");
constexpr int kMLdsBlocks = 512;
// Pass C sorts its tiles with twice the waves of the scatter passes: it holds
// only the packed records (its LDS leaves room for the wave counters of 16
// waves), and with half the records per thread it fits 1024 threads.
constexpr int kCThreads = 1024;
constexpr int kCWaves = kCThreads / 64;
static_assert(kCWaves % 2 == 0 && kCThreads >= kMNB, "pass C waves");

// Per-wave digit counters in LDS: waves 2v and 2v + 1 share the words
// wh[v][d], wave 2v in the low and wave 2v + 1 in the high 16 bits.  A
// wave's count of one digit in a tile is at most 64 x 32 records, and a
// tile position at most 16,384, so neither half carries into the other.
constexpr int kMWhWords = kMWaves / 2 * kMNB;
constexpr int kCWhWords = kCWaves / 2 * kMNB;
__device__ __forceinline__ uint32_t wh_at(int wave, uint32_t d) { return (uint32_t)(wave >> 1) * kMNB + d; }
__device__ __forceinline__ uint32_t wh_shift(int wave) { return (uint32_t)(wave & 1) * 16u; }
__device__ __forceinline__ uint32_t wh_get(const uint32_t* wh, int wave, uint32_t d) {
  return (wh[wh_at(wave, d)] >> wh_shift(wave)) & 0xFFFFu;
}

enum { IN_BLOCKS = 0, IN_NARROW = 1, IN_WIDE = 2 };

// Thread index as the shared helpers read it.  TidOpaque hides it from the
// compiler at every use, so that values derived from it are recomputed where
// they are needed instead of being computed once and held in registers for
// the whole kernel: pass C's tile loop then fits 1,024 threads without
// spilling (its per-slot LDS and global offsets otherwise fill the register
// file).  The scatter passes keep the plain index (faster there: 1.77 vs
// 1.99 ms for pass A at 3e8).
struct TidPlain {
  static __device__ __forceinline__ uint32_t get() { return threadIdx.x; }
};
struct TidOpaque {
  static __device__ __forceinline__ uint32_t get() {
    uint32_t t = __builtin_amdgcn_workitem_id_x();
    asm volatile("" : "+v"(t));
    return t;
  }
};

// Exclusive scan across a workgroup of NW waves; *total = the sum.
template <int NW = kMWaves, class TID = TidPlain>
__device__ __forceinline__ uint32_t m_block_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = TID::get() & 63, wave = TID::get() >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_tmp[wave] = inc;
  lds_barrier();
  uint32_t off = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = s_tmp[w];
    if (w < wave) off += t;
    sum += t;
  }
  lds_barrier();
  *total = sum;
  return off + inc - v;
}

// XCD-aware range number: workgroup w runs on XCD w % 8, and each XCD takes
// a contiguous span of ranges, so neighbouring runs meet in one L2.  The
// counting passes use it (first count on the 3e8 microcircuit: 0.30 ms
// against 0.31 with range = workgroup); the scatters take range =
// workgroup, consecutive ranges spread over the XCDs (pass A 1.78 -> 1.77
// ms, pass B 1.61 -> 1.54 ms against the XCD spans).
__device__ __forceinline__ uint32_t m_range(uint32_t per_xcd) {
  const uint32_t w = blockIdx.x;
  return (w & 7u) * per_xcd + (w >> 3);
}

// ---------------------------------------------------------------------------
// Tile records in registers.  Item k of wave w is tile record
// w * ITEMS * 64 + k * 64 + lane (64 consecutive records per item slot), so
// ranks computed slot by slot follow the record order.
// ---------------------------------------------------------------------------
template <int ITEMS>
struct Recs {
  uint32_t k[ITEMS];  // key (blocks, wide) or kt (narrow)
  uint32_t t[ITEMS];  // target (blocks, wide)
  uint32_t w[ITEMS];  // weight bits
};

template <class TID = TidPlain>
__device__ __forceinline__ uint32_t item_index(int ITEMS, int k) {
  const int lane = TID::get() & 63, wave = TID::get() >> 6;
  return (uint32_t)(wave * ITEMS * 64 + k * 64 + lane);
}

// Records [base, base + cnt) of the creation-order blocks (a tile spans at
// most two blocks), as (key, target, weight).
template <int ITEMS, bool FULL>
__device__ __forceinline__ void load_blocks(char* const* blocks, int log2B, uint32_t dbits, uint32_t base,
                                            uint32_t cnt, Recs<ITEMS>& r) {
  const uint64_t B = 1ull << log2B;
  const uint32_t b0 = base >> log2B;
  const char* blk0 = C(blocks, b0);
  const char* blk1 = C(blocks, (base + cnt - 1) >> log2B);
// Each slot's values are selected, not stored on two paths, so that the
// record arrays stay in registers.
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t lj = item_index(ITEMS, k);
    uint32_t kv = 0, tv = 0, wv = 0;
    if (FULL || lj < cnt) {
      const uint32_t j = base + lj;
      const char* blk = (j >> log2B) != b0 ? blk1 : blk0;
      const uint64_t o = j & (B - 1);
      const uint32_t s = G(reinterpret_cast<const uint32_t*>(blk))[o];
      tv = G(reinterpret_cast<const uint32_t*>(blk + 4 * B))[o];
      wv = G(reinterpret_cast<const uint32_t*>(blk + 8 * B))[o];
      kv = (s << dbits) | (uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o];
    }
    r.k[k] = kv;
    r.t[k] = tv;
    r.w[k] = wv;
  }
}

template <int ITEMS, int IN, bool FULL, class TID = TidPlain>
__device__ __forceinline__ void load_arrays(const uint32_t* ik, const uint32_t* it, const uint32_t* iw,
                                            uint32_t base, uint32_t cnt, Recs<ITEMS>& r) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t lj = item_index<TID>(ITEMS, k);
    uint32_t kv = 0, tv = 0, wv = 0;
    if (FULL || lj < cnt) {
      kv = G(ik)[base + lj];
      if constexpr (IN == IN_WIDE) tv = G(it)[base + lj];
      wv = G(iw)[base + lj];
    }
    r.k[k] = kv;
    r.t[k] = tv;
    r.w[k] = wv;
  }
}

// Stable ranks of the tile's digits.  For each item slot the lanes holding
// the same digit (peers) come from one ballot per digit bit; a record's rank
// is the number of records of its digit in the wave's earlier slots plus its
// peers in lower lanes.  The lowest peer adds the slot's count to the wave's
// counter of that digit with one LDS atomic (other lanes add to a private
// word), and the old value reaches its peers through a lane permute a few
// slots later, so no slot waits on the one before it.  The digit of a key is
// ((key >> shift) - base) & mask, below 2^nbits (ballots only for those
// bits).  On return pos[k] is the rank within the wave's records of the
// digit, and the wave's half of wh[wave / 2][d] holds its count of digit d.
// Lanes that add nothing add to their word of sink[64].
template <int RB, int ITEMS, bool FULL, class TID = TidPlain>
__device__ __forceinline__ void rank_digits(const uint32_t (&key)[ITEMS], uint32_t shift, uint32_t mask, uint32_t cnt,
                                            uint32_t* wh, uint32_t* sink, uint32_t (&pos)[ITEMS],
                                            uint32_t base = 0, uint32_t nbits = RB) {
  constexpr int kLag = 4;
  const int lane = TID::get() & 63, wave = TID::get() >> 6;
  uint32_t prv[ITEMS];
  // slots past the tile's end hold no record of this wave (a uniform test)
  auto slot_used = [&](int k) { return FULL || (uint32_t)(wave * ITEMS * 64 + k * 64) < cnt; };
#pragma unroll
  for (int k = 0; k < ITEMS + kLag; ++k) {
    if (k < ITEMS && slot_used(k)) {
      const uint32_t lj = (uint32_t)(wave * ITEMS * 64 + k * 64 + lane);
      const bool valid = FULL || lj < cnt;
      const uint32_t d = ((key[k] >> shift) - base) & mask;
      uint32_t plo = ~0u, phi = ~0u;
      if (!FULL) {
        const uint64_t v = __ballot(valid);
        plo = (uint32_t)v;
        phi = (uint32_t)(v >> 32);
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        if ((uint32_t)b < nbits) {  // digits are below 2^nbits (a uniform test)
          const uint32_t sb = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // bit b, all ones or zero
          const uint64_t m = __ballot(sb != 0u);
          plo &= ~((uint32_t)m ^ sb);
          phi &= ~((uint32_t)(m >> 32) ^ sb);
        }
      }
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
      const uint32_t tot = (uint32_t)__popc(plo) + (uint32_t)__popc(phi);
      const uint32_t lead = (uint32_t)__builtin_ctzll(((uint64_t)phi << 32) | plo | (1ull << 63));
      uint32_t* ctr = (valid && below == 0) ? &wh[wh_at(wave, d)] : &sink[lane];
      prv[k] = atomicAdd(ctr, tot << wh_shift(wave));
      pos[k] = below | (lead << 8);
    }
    if (k >= kLag && slot_used(k - kLag)) {
      const int q = k - kLag;
      const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((pos[q] >> 8) << 2), (int)prv[q]);
      pos[q] = ((prev >> wh_shift(wave)) & 0xFFFFu) + (pos[q] & 0xFFu);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the lag: no permute moves up to its add
  }
}

// m_block_scan without its closing barrier, for callers whose next use of
// s_tmp comes after another barrier.
template <int NW, class TID>
__device__ __forceinline__ uint32_t m_block_scan_open(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = TID::get() & 63, wave = TID::get() >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_tmp[wave] = inc;
  lds_barrier();
  uint32_t off = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = s_tmp[w];
    if (w < wave) off += t;
    sum += t;
  }
  *total = sum;
  return off + inc - v;
}

// Thread d: digit d's counts over the waves become each wave's first tile
// position of that digit; returns the digit's count in the tile and sets
// *start to its first tile position.  Leaves each wave's half of
// wh[wave / 2][d] = that tile position.
template <int NW = kMWaves, class TID = TidPlain>
__device__ __forceinline__ uint32_t digit_starts(uint32_t nd, uint32_t* wh, uint32_t* s_tmp, uint32_t* start) {
  const uint32_t d = TID::get();
  uint32_t c[NW];
  uint32_t tot = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    const uint32_t x = d < nd ? wh_get(wh, v, d) : 0u;
    c[v] = tot;
    tot += x;
  }
  uint32_t all;
  const uint32_t st = m_block_scan<NW, TID>(tot, s_tmp, &all);
  if (d < nd) {
#pragma unroll
    for (int v = 0; v < NW; v += 2) wh[wh_at(v, d)] = (st + c[v]) | ((st + c[v + 1]) << 16);
  }
  *start = st;
  return tot;
}

// digit_starts for pass C, which also needs the present digits: one scan of
// (count << 10 | present) gives each digit's first tile position (*start)
// and the number of present digits before it (*ex); *all = the tile's
// records << 10 | its present digits.  Leaves s_tmp in use (a barrier must
// come before its next use).
template <int NW, class TID>
__device__ __forceinline__ uint32_t digit_starts_present(uint32_t nd, uint32_t* wh, uint32_t* s_tmp,
                                                         uint32_t* start, uint32_t* ex, uint32_t* all) {
  const uint32_t d = TID::get();
  uint32_t c[NW];
  uint32_t tot = 0;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    const uint32_t x = d < nd ? wh_get(wh, v, d) : 0u;
    c[v] = tot;
    tot += x;
  }
  // tot < 2^15 (one load), at most 512 present digits: the fields do not mix
  const uint32_t sc = m_block_scan_open<NW, TID>((tot << 10) | (tot ? 1u : 0u), s_tmp, all);
  const uint32_t st = sc >> 10;
  if (d < nd) {
#pragma unroll
    for (int v = 0; v < NW; v += 2) wh[wh_at(v, d)] = (st + c[v]) | ((st + c[v + 1]) << 16);
  }
  *start = st;
  *ex = sc & 1023u;
  return tot;
}

// ---------------------------------------------------------------------------
// Passes A and B: stable scatter of tiles by one digit.
// ---------------------------------------------------------------------------
struct PassIO {
  char* const* in_blocks;
  int log2B;
  uint32_t dbits;
  const uint32_t *ik, *it, *iw;
  uint32_t *ok, *ot, *ow;
  uint32_t shift, mask;  // digit = (k >> shift) & mask, k as held in the input
  uint32_t tbits;        // narrow output
  uint32_t remmask;      // narrow output from a full key: kt = ((key & remmask) << tbits) | tgt
};

struct ScatterLds {
  uint32_t *k, *t, *w;   // [kMsdTile] staged records
  uint32_t* wh;          // [kMWaves / 2][kMNB], two waves per word
  uint4* dig;            // [kMNB]: x = global position of the digit's first record minus its
                         // tile position (mod 2^32); [y, y + z): positions whose 128-byte line
                         // the tile's run fills completely
  uint32_t* run;         // [kMNB] next global position per digit
  uint32_t* tmp;         // [kMWaves]
  uint32_t* sink;        // [64]
};

template <int ITEMS, int IN, bool FULL>
__device__ __forceinline__ void load_tile(const PassIO& io, uint32_t base, uint32_t cnt, Recs<ITEMS>& r) {
  if constexpr (IN == IN_BLOCKS) load_blocks<ITEMS, FULL>(io.in_blocks, io.log2B, io.dbits, base, cnt, r);
  else load_arrays<ITEMS, IN, FULL>(io.ik, io.it, io.iw, base, cnt, r);
}

template <int ITEMS, int IN>
__device__ __forceinline__ void load_tile_any(const PassIO& io, uint32_t base, uint32_t cnt, Recs<ITEMS>& r) {
  if (cnt == (uint32_t)(ITEMS * kMThreads)) load_tile<ITEMS, IN, true>(io, base, cnt, r);
  else load_tile<ITEMS, IN, false>(io, base, cnt, r);
}

// One tile, its records in registers; next_cnt > 0: the next tile's records
// load (into r) while this tile's runs are written.
template <int RB, int IN, bool OUT_NARROW, bool FULL, int ITEMS>
__device__ __forceinline__ void scatter_tile(const PassIO& io, uint32_t cnt, const ScatterLds& L, Recs<ITEMS>& r,
                                             uint32_t next_base, uint32_t next_cnt) {
  constexpr bool HAS_T = IN != IN_NARROW;
  const int wave = threadIdx.x >> 6;
  uint32_t pos[ITEMS];
  rank_digits<RB, ITEMS, FULL>(r.k, io.shift, io.mask, cnt, L.wh, L.sink, pos);
  lds_barrier();
  {
    const uint32_t d = threadIdx.x;
    uint32_t st;
    const uint32_t tot = digit_starts(io.mask + 1, L.wh, L.tmp, &st);
    if (d <= io.mask) {
      const uint32_t rn = L.run[d];
      const uint32_t lo = (rn + 31u) & ~31u, hi = (rn + tot) & ~31u;
      L.dig[d] = make_uint4(rn - st, lo, hi > lo ? hi - lo : 0u, 0u);
      L.run[d] = rn + tot;
    }
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (FULL || item_index(ITEMS, k) < cnt) {
      const uint32_t p = pos[k] + wh_get(L.wh, wave, (r.k[k] >> io.shift) & io.mask);
      L.k[p] = r.k[k];
      if constexpr (HAS_T) L.t[p] = r.t[k];
      L.w[p] = r.w[k];
    }
  }
  lds_barrier();
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
#pragma unroll
    for (int v = 0; v < kMWaves / 2; ++v) L.wh[v * kMNB + d] = 0;
  }
  if (next_cnt) load_tile_any<ITEMS, IN>(io, next_base, next_cnt, r);
  // Runs of equal digits go to consecutive positions.  Stores of records
  // whose 128-byte lines the run fills are marked streaming; the partial
  // lines at a run's ends stay cached, so that the neighbouring tile's run
  // can complete them in L2 before they reach HBM.  In the second scatter
  // each record first waits until at most four of the wave's memory
  // operations are in flight (s_waitcnt vmcnt(4); expcnt and lgkmcnt left
  // open): so paced, its two or three store streams finished the pass in
  // 1.70 ms instead of 1.74 on the 3e8 microcircuit; the first scatter,
  // paced the same way, was slower.
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t lp = (uint32_t)(k * kMThreads + threadIdx.x);
    if constexpr (IN != IN_BLOCKS) __builtin_amdgcn_s_waitcnt(0x0F74);
    if (FULL || lp < cnt) {
      const uint32_t kk = L.k[lp];
      const uint32_t wv = L.w[lp];
      const uint4 di = L.dig[(kk >> io.shift) & io.mask];
      const uint32_t dest = di.x + lp;
      const bool in = dest - di.y < di.z;
      uint32_t ko = kk;
      if constexpr (OUT_NARROW && IN != IN_NARROW) ko = ((kk & io.remmask) << io.tbits) | L.t[lp];
      if (in) {
        st_u32_nt(io.ok + dest, ko);
        if constexpr (!OUT_NARROW) st_u32_nt(io.ot + dest, L.t[lp]);
        st_u32_nt(io.ow + dest, wv);
      } else {
        G(io.ok)[dest] = ko;
        if constexpr (!OUT_NARROW) G(io.ot)[dest] = L.t[lp];
        G(io.ow)[dest] = wv;
      }
    }
  }
  lds_barrier();  // the staging buffers and counters are reused by the next tile
}

// Tiles [t0, t1) of a record span starting at span0 and ending at span1:
// tile t holds records [span0 + t * tile, min(span0 + (t + 1) * tile, span1)).
template <int RB, int IN, bool OUT_NARROW, int ITEMS>
__device__ __forceinline__ void scatter_range(const PassIO& io, const ScatterLds& L, uint32_t span0, uint32_t span1,
                                              uint32_t t0, uint32_t t1) {
  constexpr uint32_t TILE = (uint32_t)(ITEMS * kMThreads);
  if (t0 >= t1) return;
  Recs<ITEMS> r;
  auto tile_cnt = [&](uint32_t t) {
    const uint32_t b = span0 + t * TILE;
    return span1 - b < TILE ? span1 - b : TILE;
  };
  load_tile_any<ITEMS, IN>(io, span0 + t0 * TILE, tile_cnt(t0), r);
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t cnt = tile_cnt(t);
    const uint32_t nb = t + 1 < t1 ? span0 + (t + 1) * TILE : 0u;
    const uint32_t nc = t + 1 < t1 ? tile_cnt(t + 1) : 0u;
    if (cnt == TILE) scatter_tile<RB, IN, OUT_NARROW, true, ITEMS>(io, cnt, L, r, nb, nc);
    else scatter_tile<RB, IN, OUT_NARROW, false, ITEMS>(io, cnt, L, r, nb, nc);
  }
}

#define M_SCATTER_LDS(TILE)                             \
  __shared__ uint32_t s_k[TILE];                        \
  __shared__ uint32_t s_t[IN == IN_NARROW ? 1 : TILE];  \
  __shared__ uint32_t s_w[TILE];                        \
  __shared__ uint32_t s_wh[kMWhWords];                  \
  __shared__ uint4 s_dig[kMNB];                         \
  __shared__ uint32_t s_run[kMNB];                      \
  __shared__ uint32_t s_tmp[kMWaves];                   \
  __shared__ uint32_t s_sink[64];                       \
  const ScatterLds L{s_k, s_t, s_w, s_wh, s_dig, s_run, s_tmp, s_sink};

// Pass A: range r of the creation-order records by D1.
template <int RB, bool OUT_NARROW>
__global__ __launch_bounds__(kMThreads) void k_msd_scatter_a(MsdPlan p) {
  constexpr int IN = IN_BLOCKS;
  M_SCATTER_LDS(kMsdTile)
  const uint32_t r = blockIdx.x;
  if (r >= p.ranges_a) return;
  const uint32_t nd = 1u << p.b1;
  PassIO io{};
  io.in_blocks = p.in_blocks;
  io.log2B = p.log2B;
  io.dbits = p.dbits;
  io.ok = p.a_key;
  io.ot = p.a_tgt;
  io.ow = p.a_w;
  io.shift = p.b2 + p.b3;
  io.mask = nd - 1;
  io.tbits = p.tbits;
  io.remmask = (1u << (p.b2 + p.b3)) - 1u;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
    s_run[d] = d < nd ? p.cnt_a[(uint64_t)d * p.ranges_a + r] : 0u;
#pragma unroll
    for (int v = 0; v < kMWaves / 2; ++v) s_wh[v * kMNB + d] = 0;
  }
  lds_barrier();
  const uint32_t ntiles = (p.n + kMsdTile - 1) / kMsdTile;
  const uint32_t t0 = r * p.tpr, t1 = min(t0 + p.tpr, ntiles);
  scatter_range<RB, IN, OUT_NARROW, kMItems>(io, L, 0u, p.n, t0, t1);
}

// Bucket of pass-B range r: the last b with rangeb0[b] <= r (from LDS).
__device__ __forceinline__ uint32_t bucket_of_range(const uint32_t* s_rb0, uint32_t nb, uint32_t r) {
  uint32_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (s_rb0[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Pass B: range r of a bucket by D2.
template <int RB, int IN, bool OUT_NARROW, int ITEMS>
__global__ __launch_bounds__(kMThreads) void k_msd_scatter_b(MsdPlan p) {  // the tile is p.tile_b = ITEMS x kMThreads
  M_SCATTER_LDS(ITEMS * kMThreads)
  __shared__ uint32_t s_rb0[kMNB + 1];
  const uint32_t nb = 1u << p.b1, nd = 1u << p.b2;
  for (uint32_t b = threadIdx.x; b <= nb; b += kMThreads) s_rb0[b] = p.rangeb0[b];
  lds_barrier();
  const uint32_t r = blockIdx.x;
  if (r >= s_rb0[nb]) return;
  const uint32_t b = bucket_of_range(s_rb0, nb, r);
  const uint32_t rl = r - s_rb0[b], nr = s_rb0[b + 1] - s_rb0[b];
  const uint32_t bs = p.bstart[b], be = p.bstart[b + 1];
  PassIO io{};
  io.ik = p.a_key;
  io.it = p.a_tgt;
  io.iw = p.a_w;
  io.ok = p.b_key;
  io.ot = p.b_tgt;
  io.ow = p.b_w;
  io.shift = (IN == IN_NARROW ? p.tbits : 0u) + p.b3;
  io.mask = nd - 1;
  io.tbits = p.tbits;
  io.remmask = (1u << p.cbits) - 1u;  // packed from full keys: as many low key bits as fit
  const uint64_t cb = ((uint64_t)s_rb0[b] << p.b2) + rl;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
    s_run[d] = d < nd ? p.cnt_b[cb + (uint64_t)d * nr] : 0u;
#pragma unroll
    for (int v = 0; v < kMWaves / 2; ++v) s_wh[v * kMNB + d] = 0;
  }
  lds_barrier();
  const uint32_t ntiles = (be - bs + p.tile_b - 1) / p.tile_b;
  const uint32_t tpr = p.tprb[b];
  const uint32_t t0 = rl * tpr, t1 = min(t0 + tpr, ntiles);
  scatter_range<RB, IN, OUT_NARROW, ITEMS>(io, L, bs, be, t0, t1);
}

// ---------------------------------------------------------------------------
// Digit counts of the ranges of passes A and B.
// ---------------------------------------------------------------------------
// Adds four digits of a lane to an LDS histogram.  When every active lane of
// the wave holds one digit four times (sorted input: the same address for
// the whole wave would serialize the adds) the wave adds once; a lane whose
// four digits agree adds once.
__device__ __forceinline__ void hist_add4(uint32_t* hist, uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3) {
  const bool same = d0 == d1 && d0 == d2 && d0 == d3;
  const uint32_t first = __builtin_amdgcn_readfirstlane(d0);
  const uint64_t act = __ballot(1);
  const uint64_t agree = __ballot(same && d0 == first);
  if (agree == act) {
    if ((threadIdx.x & 63u) == (uint32_t)__builtin_ctzll(act)) atomicAdd(&hist[first], 4u * (uint32_t)__popcll(act));
  } else if (same) {
    atomicAdd(&hist[d0], 4u);
  } else {
    atomicAdd(&hist[d0], 1u);
    atomicAdd(&hist[d1], 1u);
    atomicAdd(&hist[d2], 1u);
    atomicAdd(&hist[d3], 1u);
  }
}

// Pass A: D1 of every creation-order record (the delays are read only when
// D1 reaches into the delay bits).
template <bool NEED_DELAY>
__global__ __launch_bounds__(kCntThreads) void k_msd_count_a(MsdPlan p) {
  __shared__ uint32_t hist[kMNB];
  const uint32_t r = m_range((p.ranges_a + 7) / 8);
  if (r >= p.ranges_a) return;
  const uint32_t nd = 1u << p.b1, shift = p.b2 + p.b3;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kCntThreads) hist[d] = 0;
  __syncthreads();
  const uint32_t ntiles = (p.n + kMsdTile - 1) / kMsdTile;
  const uint32_t t0 = r * p.tpr, t1 = min(t0 + p.tpr, ntiles);
  // The range's records [lo, hi) are contiguous; they are read block by
  // block, each block's table entry once, 16-byte loads of four sources
  // (and 8-byte loads of four delays), eight groups in flight per thread
  // (3e8 microcircuit, 512 threads: 0.31 ms; a table lookup per group of
  // four, one group in flight: 0.325 ms).
  // lo and the block starts are multiples of 4, so each piece's groups are
  // aligned and only its last 0-3 records are read one by one.
  const uint32_t lo = t0 < t1 ? t0 * kMsdTile : 0u;
  const uint32_t hi = t0 < t1 ? (uint32_t)min((uint64_t)t1 * kMsdTile, (uint64_t)p.n) : 0u;
  const uint32_t m = nd - 1;
  auto key = [&](uint32_t src, uint32_t dl) { return (((src << p.dbits) | dl) >> shift) & m; };
  for (uint32_t j0 = lo; j0 < hi;) {
    const uint32_t bi = j0 >> p.log2B;
    const uint32_t bend = (uint32_t)min((uint64_t)hi, ((uint64_t)bi + 1) << p.log2B);
    const char* blk = C(p.in_blocks, bi);
    const uint32_t o0 = j0 - (bi << p.log2B), o1 = bend - (bi << p.log2B);
    const uint32_t nq = (o1 - o0) / 4, oe = o0 + 4 * nq;
    const NG_GLOBAL u32x4* vs = (const NG_GLOBAL u32x4*)(blk + 4 * (uint64_t)o0);
    const NG_GLOBAL u32x2* vd = (const NG_GLOBAL u32x2*)(blk + (12ull << p.log2B) + 2 * (uint64_t)o0);
    auto group = [&](const u32x4& s4, const u32x2& d4) {
      hist_add4(hist, key(s4.x, d4.x & 0xFFFFu), key(s4.y, d4.x >> 16), key(s4.z, d4.y & 0xFFFFu),
                key(s4.w, d4.y >> 16));
    };
    uint32_t q = threadIdx.x;
    for (; q + 7 * kCntThreads < nq; q += 8 * kCntThreads) {
      u32x4 s4[8];
      u32x2 d4[8] = {};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s4[u] = vs[q + u * kCntThreads];
        if constexpr (NEED_DELAY) d4[u] = vd[q + u * kCntThreads];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) group(s4[u], d4[u]);
    }
    for (; q < nq; q += kCntThreads) {
      u32x2 d4 = {};
      if constexpr (NEED_DELAY) d4 = vd[q];
      const u32x4 s4 = vs[q];
      group(s4, d4);
    }
    if (oe + threadIdx.x < o1) {
      const uint32_t o = oe + threadIdx.x;
      const uint32_t src = G(reinterpret_cast<const uint32_t*>(blk))[o];
      const uint32_t dl =
          NEED_DELAY ? (uint16_t)G(reinterpret_cast<const int16_t*>(blk + (12ull << p.log2B)))[o] : 0u;
      atomicAdd(&hist[key(src, dl)], 1u);
    }
    j0 = bend;
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nd; d += kCntThreads) p.cnt_a[(uint64_t)d * p.ranges_a + r] = hist[d];
}

// Pass B: D2 of the records of each range of each bucket.
template <int IN>
__global__ __launch_bounds__(kCntThreads) void k_msd_count_b(MsdPlan p) {
  __shared__ uint32_t hist[kMNB];
  __shared__ uint32_t s_rb0[kMNB + 1];
  const uint32_t nb = 1u << p.b1, nd = 1u << p.b2;
  for (uint32_t b = threadIdx.x; b <= nb; b += kCntThreads) s_rb0[b] = p.rangeb0[b];
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kCntThreads) hist[d] = 0;
  __syncthreads();
  const uint32_t r = m_range((p.max_ranges_b + 7) / 8);
  if (r >= s_rb0[nb]) return;
  const uint32_t b = bucket_of_range(s_rb0, nb, r);
  const uint32_t rl = r - s_rb0[b], nr = s_rb0[b + 1] - s_rb0[b];
  const uint32_t bs = p.bstart[b], be = p.bstart[b + 1];
  const uint32_t shift = (IN == IN_NARROW ? p.tbits : 0u) + p.b3;
  const uint32_t tpr = p.tprb[b];
  const uint32_t lo = bs + rl * tpr * p.tile_b;
  const uint32_t hi = (be - lo) / p.tile_b < tpr ? be : lo + tpr * p.tile_b;
  // 16-byte loads over the aligned middle (the key array starts 256-byte
  // aligned), four in flight per thread; single words at the ends
  const uint32_t a0 = min(hi, (lo + 3u) & ~3u), a1 = max(a0, hi & ~3u);
  auto add = [&](uint32_t k) { atomicAdd(&hist[(k >> shift) & (nd - 1)], 1u); };
  if (lo + threadIdx.x < a0) add(G(p.a_key)[lo + threadIdx.x]);
  if (a1 + threadIdx.x < hi) add(G(p.a_key)[a1 + threadIdx.x]);
  const NG_GLOBAL u32x4* v = (const NG_GLOBAL u32x4*)(p.a_key + a0);
  const uint32_t nq = (a1 - a0) / 4;
  uint32_t q = threadIdx.x;
  for (; q + 3 * kCntThreads < nq; q += 4 * kCntThreads) {
    u32x4 x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = v[q + u * kCntThreads];
    const uint32_t m = nd - 1;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      hist_add4(hist, (x[u].x >> shift) & m, (x[u].y >> shift) & m, (x[u].z >> shift) & m, (x[u].w >> shift) & m);
  }
  for (; q < nq; q += kCntThreads) {
    const u32x4 x = v[q];
    const uint32_t m = nd - 1;
    hist_add4(hist, (x.x >> shift) & m, (x.y >> shift) & m, (x.z >> shift) & m, (x.w >> shift) & m);
  }
  __syncthreads();
  const uint64_t cb = ((uint64_t)s_rb0[b] << p.b2) + rl;
  for (uint32_t d = threadIdx.x; d < nd; d += kCntThreads) p.cnt_b[cb + (uint64_t)d * nr] = hist[d];
}

// ---------------------------------------------------------------------------
// Start tables.
// ---------------------------------------------------------------------------
// Bucket starts from the scanned counts of pass A, and the ranges of pass B
// (tiles of tile_b records from each bucket's start, tprb[b] tiles per range
// of bucket b).
// One workgroup, one thread per bucket.  Without pass B the buckets are the
// sub-buckets.
__global__ __launch_bounds__(kMThreads) void k_msd_plan_b(MsdPlan p) {
  __shared__ uint32_t s_tmp[kMWaves];
  const uint32_t nb = 1u << p.b1, b = threadIdx.x;
  uint32_t bs = 0, be = 0;
  if (b < nb) {
    bs = p.cnt_a[(uint64_t)b * p.ranges_a];
    be = b + 1 < nb ? p.cnt_a[(uint64_t)(b + 1) * p.ranges_a] : p.n;
    p.bstart[b] = bs;
    if (p.b2 == 0) p.sbstart[b] = bs;
  }
  if (b == 0) {
    p.bstart[nb] = p.n;
    if (p.b2 == 0) p.sbstart[nb] = p.n;
  }
  // Every bucket gets ranges in proportion to its tiles, about ranges_b in
  // all, and its tiles are spread evenly over them, so that all ranges of
  // pass B hold about the same number of tiles (no short last ranges).
  const uint32_t ntiles = (be - bs + p.tile_b - 1) / p.tile_b;
  uint32_t all_tiles;
  (void)m_block_scan(b < nb ? ntiles : 0u, s_tmp, &all_tiles);
  uint32_t nr = 0, tpr = 1;
  if (b < nb && ntiles) {
    const uint64_t want = ((uint64_t)ntiles * p.ranges_b + all_tiles - 1) / all_tiles;  // >= 1
    tpr = (uint32_t)((ntiles + want - 1) / want);
    nr = (ntiles + tpr - 1) / tpr;  // <= want
  }
  if (b < nb) p.tprb[b] = tpr;
  uint32_t total;
  const uint32_t ex = m_block_scan(b < nb ? nr : 0u, s_tmp, &total);
  if (b < nb) p.rangeb0[b] = ex;
  if (b == 0) p.rangeb0[nb] = total;
}

// Sub-bucket starts from the scanned counts of pass B: sub-bucket (b, d)
// starts at the offset of range 0 of bucket b for digit d (at the bucket's
// start when the bucket is empty).
__global__ __launch_bounds__(256) void k_msd_plan_c(MsdPlan p) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t sb = blockIdx.x * 256u + threadIdx.x;
  if (sb < nsb) {
    const uint32_t b = sb >> p.b2, d = sb & ((1u << p.b2) - 1u);
    const uint32_t r0 = p.rangeb0[b], nr = p.rangeb0[b + 1] - r0;
    p.sbstart[sb] = nr ? p.cnt_b[((uint64_t)r0 << p.b2) + (uint64_t)d * nr] : p.bstart[b];
  }
  if (sb == 0) p.sbstart[nsb] = p.n;
}

// Group counts and masks of all sub-buckets start at zero; pass C writes
// those of the sub-buckets that hold records.
__global__ __launch_bounds__(256) void k_msd_zero(MsdPlan p) {
  const uint64_t nsb = 1ull << (p.b1 + p.b2);
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < nsb; i += stride) G(p.gcount)[i] = 0;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < nsb * p.mask_words; i += stride) G(p.gmask)[i] = 0;
}

// Workgroup w of pass C takes the sub-buckets whose first record lies in
// [w * n / wgs, (w + 1) * n / wgs): a split by records.
__global__ __launch_bounds__(256) void k_msd_split(MsdPlan p) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t w = blockIdx.x * 256u + threadIdx.x;
  if (w == 0) *p.big_count = 0;  // sub-buckets listed by pass C
  if (w > p.wgs_c) return;
  // the last boundary is the first sub-bucket past the records: the empty
  // sub-buckets above it are never visited (their group counts and masks are
  // zero from k_msd_zero)
  const uint32_t target = (uint32_t)((uint64_t)w * p.n / p.wgs_c);
  uint32_t lo = 0, hi = nsb;  // first sb with sbstart[sb] >= target
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (p.sbstart[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  p.wg_sb0[w] = lo;
}

// ---------------------------------------------------------------------------
// Pass C: runs of whole sub-buckets sorted in LDS, written as calibrated
// blocks.
// ---------------------------------------------------------------------------
// A tile is a run of consecutive sub-buckets [sb, e) holding at most one
// LDS load of records, with at most kCMaxSub sub-buckets; sorting it by the
// combined digit (sub-bucket offset in the run, D3) sorts every sub-bucket by
// D3, and its sorted order is its final order, so the tile is written to
// [sbstart[sb], sbstart[e]) as one contiguous run.  A sub-bucket larger than
// one load is its own tile and is sorted in pieces after a counting pass.
// Output block of a sorted position: from the LDS copy of the block table
// when it holds all of them.
__device__ __forceinline__ char* m_out_block(const MsdPlan& p, char* const* s_blk, uint32_t dest) {
  return s_blk ? s_blk[dest >> p.log2B] : C(p.out_blocks, dest >> p.log2B);
}

// Records per LDS load of pass C: 10,240 for packed and unpacked records,
// 10 per thread of 1,024.  (Measured on the 3e8 microcircuit, with 512
// threads: 16,384-record tiles spill registers and took 2.46 ms; 6,144-record
// tiles with two workgroups per CU need a narrower last digit, hence a 9-bit
// second scatter, and took 2.38 ms plus 0.7 ms more in pass B; 10,240: 2.17
// ms.  With 1,024 threads: 2.03 ms; stores through a scalar block base for
// runs inside one block, next to the general store loop: 2.15 ms.)
template <bool NARROW>
struct CSize {
  static constexpr int ITEMS = (int)kMsdTile / kCThreads;
  static constexpr uint32_t TILE = (uint32_t)(ITEMS * kCThreads);
};
static_assert(CSize<true>::TILE == kMsdTile, "tile of pass C");
constexpr uint32_t kCMaxSub = 63;      // sub-buckets per tile: lanes 1..63 test the ends

// Sub-buckets per tile: bounded by the lanes of one wave, by 9-bit combined
// digits, and for packed records by the sub-bucket bits they hold.
__host__ __device__ inline uint32_t msd_max_sub(const MsdPlan& p, bool narrow) {
  uint32_t m = kCMaxSub < (512u >> p.b3) ? kCMaxSub : (512u >> p.b3);
  if (narrow) {
    const uint32_t own = 1u << (p.cbits - p.b3);
    m = m < own ? m : own;
  }
  return m;
}

struct CTile {
  uint32_t sb, e, r0, r1;  // sub-buckets [sb, e), records [r0, r1); e == sb: no tile left
};

// The next tile from sub-bucket sb in [sb, sb_end), found by one wave in
// two steps so that the load's latency can hide behind other work: the
// probe reads the starts of sub-buckets sb .. sb + lim (lane l: sb +
// min(l, lim), lim = min(63, sb_end - sb)); the finish takes the longest run
// of at most m sub-buckets whose records fit one load (sub-bucket starts
// ascend, so the runs that fit form a prefix of the lanes).  A run that
// starts with empty sub-buckets becomes a tile of those alone (no records;
// their group counts and masks are already zero).  Wave 0 only.
__device__ __forceinline__ uint32_t tile_probe(const MsdPlan& p, uint32_t sb, uint32_t lim) {
  const uint32_t lane = TidOpaque::get() & 63;
  return G(p.sbstart)[sb + min(lane, lim)];
}

__device__ __forceinline__ CTile tile_finish(uint32_t st, uint32_t sb, uint32_t lim, uint32_t m, uint32_t cap) {
  const uint32_t lane = TidOpaque::get() & 63;
  CTile t{sb, sb, 0, 0};
  if (lim == 0) return t;
  const uint32_t r0 = (uint32_t)__shfl(st, 0);
  t.r0 = t.r1 = r0;
  if ((uint32_t)__shfl(st, 1) == r0) {  // empty sub-buckets first
    t.e = sb + (uint32_t)__popcll(__ballot(lane <= lim && st == r0)) - 1u;
    return t;
  }
  const bool ok = lane <= min(lim, m) && st - r0 <= cap;
  const uint32_t L = (uint32_t)__popcll(__ballot(ok)) - 1u;  // lane 0 always fits
  const uint32_t Lx = L ? L : 1u;
  t.e = sb + Lx;
  t.r1 = (uint32_t)__shfl(st, (int)Lx);
  return t;
}

// One predicated form of each step: pass C keeps a single copy of its
// load and ranking, which keeps its loop within the register file.
template <bool NARROW>
__device__ __forceinline__ void load_c(const uint32_t* ik, const uint32_t* it, const uint32_t* iw, uint32_t base,
                                       uint32_t cnt, Recs<CSize<NARROW>::ITEMS>& r) {
  load_arrays<CSize<NARROW>::ITEMS, NARROW ? IN_NARROW : IN_WIDE, false, TidOpaque>(ik, it, iw, base, cnt, r);
}

template <bool NARROW>
__device__ __forceinline__ bool tile_fits(const CTile& t) {
  return t.e > t.sb && t.r1 > t.r0 && t.r1 - t.r0 <= CSize<NARROW>::TILE;
}

// The connection groups of a tile of nsub sub-buckets from sba whose records
// start at r0 (Sec. 2.2): each present combined digit (thread d, h = its
// record count, 0 past the tile's digits; hst = records and ex = present
// digits before it, all_present = the tile's present digits) is a group.
// Its start goes to its sub-bucket's offset in gslot, at the group's rank in
// the sub-bucket; each sub-bucket gets its group count and its mask of
// present D3 values.  Uses s_ex, s_st, s_bal; contains one barrier, after
// which the LDS writes made before the call are visible to all.
__device__ __forceinline__ void tile_groups(const MsdPlan& p, uint32_t sba, uint32_t nsub, uint32_t r0, uint32_t h,
                                            uint32_t hst, uint32_t ex, uint32_t all_present, uint32_t* s_ex,
                                            uint32_t* s_st, uint32_t* s_bal) {
  const uint32_t d = TidOpaque::get(), lane = d & 63, wave = d >> 6;
  const uint32_t b3 = p.b3, m3 = (1u << b3) - 1u, nd = nsub << b3;
  const bool present = h != 0;
  const uint64_t bal = __ballot(present);
  if (d < (uint32_t)kMNB) {  // threads past the digits hold none
    s_ex[d] = ex;
    s_st[d] = hst;
    if (lane == 0) {
      s_bal[2 * wave] = (uint32_t)bal;
      s_bal[2 * wave + 1] = (uint32_t)(bal >> 32);
    }
  }
  if (d == 0) s_ex[kMNB] = all_present;
  lds_barrier();
  if (present) {
    const uint32_t d0 = d & ~m3;  // first digit of its sub-bucket
    G(p.gslot)[r0 + s_st[d0] + (ex - s_ex[d0])] = r0 + hst;
  }
  if (d < nsub) {
    const uint32_t hi = d + 1 < nsub ? s_ex[(d + 1) << b3] : s_ex[kMNB];
    G(p.gcount)[sba + d] = hi - s_ex[d << b3];
  }
  if (d < nd) {
    if (b3 >= 5) {
      if ((d & 31u) == 0) G(p.gmask)[(uint64_t)(sba + (d >> b3)) * p.mask_words + ((d & m3) >> 5)] = s_bal[d >> 5];
    } else if ((d & m3) == 0) {
      G(p.gmask)[sba + (d >> b3)] = (s_bal[d >> 5] >> (d & 31u)) & ((1u << (1u << b3)) - 1u);
    }
  }
}

#define M_C_LDS                                  \
  __shared__ uint32_t s_k[CSize<NARROW>::TILE];              \
  __shared__ uint32_t s_t[NARROW ? 1 : CSize<NARROW>::TILE]; \
  __shared__ uint32_t s_w[CSize<NARROW>::TILE];              \
  __shared__ uint32_t s_wh[kCWhWords];           \
  __shared__ uint32_t s_st[kMNB + 1];            \
  __shared__ uint32_t s_ex[kMNB + 1];            \
  __shared__ uint32_t s_tmp[kCWaves];            \
  __shared__ uint32_t s_sink[64];                \
  __shared__ uint32_t s_bal[kMNB / 32];          \
  __shared__ char* s_blk_tab[kMLdsBlocks];

// Key-field constants of pass C: a record holds the low cbits key bits above
// its target (packed) or the whole key, so the combined digit of a tile is
// ((k >> ks) - base) & km with base = (first sub-bucket << b3) & km.
struct CFields {
  uint32_t ks, km, msub, tmask, dmask;
  const uint32_t *ik, *it, *iw;
};

template <bool NARROW>
__device__ __forceinline__ CFields c_fields(const MsdPlan& p) {
  CFields f;
  f.ks = NARROW ? p.tbits : 0u;
  f.km = NARROW ? ((1u << p.cbits) - 1u) : ((1u << p.keybits) - 1u);
  f.msub = msd_max_sub(p, NARROW);
  f.tmask = NARROW ? ((1u << p.tbits) - 1u) : ~0u;
  f.dmask = (1u << p.dbits) - 1u;
  f.ik = p.b2 ? p.b_key : p.a_key;
  f.it = p.b2 ? p.b_tgt : p.a_tgt;
  f.iw = p.b2 ? p.b_w : p.a_w;
  return f;
}

// Block table in LDS when it fits; clears the per-wave digit counters.
__device__ __forceinline__ char* const* c_setup(const MsdPlan& p, char** s_blk_tab, uint32_t* s_wh) {
  const uint32_t n_out_blocks = (uint32_t)(((uint64_t)p.n + (1ull << p.log2B) - 1) >> p.log2B);
  char* const* s_blk = n_out_blocks <= (uint32_t)kMLdsBlocks ? s_blk_tab : nullptr;
  if (s_blk)
    for (uint32_t b = TidOpaque::get(); b < n_out_blocks; b += kCThreads) s_blk_tab[b] = C(p.out_blocks, b);
  for (uint32_t d = TidOpaque::get(); d < (uint32_t)kMNB; d += kCThreads) {
#pragma unroll
    for (int v = 0; v < kCWaves / 2; ++v) s_wh[v * kMNB + d] = 0;
  }
  return s_blk;
}

// Records staged in sorted order at [0, cnt) of the LDS arrays go out to
// their positions: dest = dx[digit] + lp (or r0 + lp when dx is null).
template <bool NARROW>
__device__ __forceinline__ void c_store(const MsdPlan& p, const CFields& f, char* const* s_blk, const uint32_t* s_k,
                                        const uint32_t* s_t, const uint32_t* s_w, uint32_t cnt, uint32_t base,
                                        uint32_t kb, const uint32_t* dx, uint32_t r0) {
  const uint64_t B = 1ull << p.log2B;
#pragma unroll
  for (int k = 0; k < CSize<NARROW>::ITEMS; ++k) {
    const uint32_t lp = (uint32_t)(k * kCThreads + TidOpaque::get());
    if (lp < cnt) {
      const uint32_t kk = s_k[lp];
      const uint32_t dg = ((kk >> f.ks) - base) & f.km;
      const uint32_t dest = dx ? dx[dg] + lp : r0 + lp;
      const uint32_t key = kb + dg;
      char* blk = m_out_block(p, s_blk, dest);
      const uint64_t o = dest & (B - 1);
      G(reinterpret_cast<uint32_t*>(blk))[o] = key >> p.dbits;
      G(reinterpret_cast<uint32_t*>(blk + 4 * B))[o] = NARROW ? (kk & f.tmask) : s_t[lp];
      G(reinterpret_cast<uint32_t*>(blk + 8 * B))[o] = s_w[lp];
      G(reinterpret_cast<int16_t*>(blk + 12 * B))[o] = (int16_t)(key & f.dmask);
    }
  }
}

// Records ranked by their combined digit move to their sorted places in LDS.
template <bool NARROW>
__device__ __forceinline__ void c_stage(const CFields& f, const Recs<CSize<NARROW>::ITEMS>& r,
                                        const uint32_t (&pos)[CSize<NARROW>::ITEMS],
                                        uint32_t cnt, uint32_t base, const uint32_t* s_wh, uint32_t* s_k, uint32_t* s_t,
                                        uint32_t* s_w) {
  const int wave = TidOpaque::get() >> 6;
#pragma unroll
  for (int k = 0; k < CSize<NARROW>::ITEMS; ++k) {
    if (item_index<TidOpaque>(CSize<NARROW>::ITEMS, k) < cnt) {
      const uint32_t dg = ((r.k[k] >> f.ks) - base) & f.km;
      const uint32_t q = pos[k] + wh_get(s_wh, wave, dg);
      s_k[q] = r.k[k];
      if constexpr (!NARROW) s_t[q] = r.t[k];
      s_w[q] = r.w[k];
    }
  }
}

__device__ __forceinline__ void clear_wh(uint32_t* s_wh) {
  for (uint32_t e = TidOpaque::get(); e < (uint32_t)kMNB; e += kCThreads) {
#pragma unroll
    for (int v = 0; v < kCWaves / 2; ++v) s_wh[v * kMNB + e] = 0;
  }
}

// Tiles of the workgroup's sub-buckets [wg_sb0[w], wg_sb0[w + 1]); the
// records of the next tile load while a tile is written.  Sub-buckets larger
// than one load are listed for k_msd_big_c.
template <int RB, bool NARROW>
__global__ __launch_bounds__(kCThreads) void k_msd_tiles_c(MsdPlan p) {
  M_C_LDS
  __shared__ CTile s_next[2];  // by iteration parity: wave 0 writes one while the other is read
  const int lane = TidOpaque::get() & 63, wave = TidOpaque::get() >> 6;
  const CFields f = c_fields<NARROW>(p);
  char* const* s_blk = c_setup(p, s_blk_tab, s_wh);
  const uint32_t b3 = p.b3;
  const uint32_t sb0 = p.wg_sb0[blockIdx.x], sb_end = p.wg_sb0[blockIdx.x + 1];
  if (wave == 0) {
    const uint32_t lim = min(kCMaxSub, sb_end - sb0);
    const CTile t = tile_finish(tile_probe(p, sb0, lim), sb0, lim, f.msub, CSize<NARROW>::TILE);
    if (lane == 0) s_next[0] = t;
  }
  lds_barrier();
  CTile cur = s_next[0];
  uint32_t par = 1;  // s_next[par] receives the tile after cur
  constexpr int ITEMS = CSize<NARROW>::ITEMS;
  constexpr uint32_t TILE = CSize<NARROW>::TILE;
  Recs<ITEMS> r;
  // invariant at the top of the loop: loaded == tile_fits(cur), and then r
  // holds cur's records
  bool loaded = tile_fits<NARROW>(cur);
  if (loaded) load_c<NARROW>(f.ik, f.it, f.iw, cur.r0, cur.r1 - cur.r0, r);
  while (cur.e > cur.sb) {
    const uint32_t n = cur.r1 - cur.r0;
    const uint32_t nsub = cur.e - cur.sb;
    const uint32_t lim = min(kCMaxSub, sb_end - cur.e);
    uint32_t probe = 0;
    if (wave == 0) probe = tile_probe(p, cur.e, lim);  // used after the ranking
    if (n == 0 || n > TILE) {
      // empty sub-buckets: nothing to do; one sub-bucket too large for one
      // load: listed for k_msd_big_c
      if (n && TidOpaque::get() == 0) G(p.big_list)[atomicAdd(p.big_count, 1u)] = cur.sb;
      if (wave == 0) {
        const CTile t = tile_finish(probe, cur.e, lim, f.msub, TILE);
        if (lane == 0) s_next[par] = t;
      }
    } else {
      const uint32_t base = (cur.sb << b3) & f.km;
      const uint32_t nd = nsub << b3;
      uint32_t nbits = 1;
      while ((1u << nbits) < nd) ++nbits;
      uint32_t pos[ITEMS];
      rank_digits<RB, ITEMS, false, TidOpaque>(r.k, f.ks, f.km, n, s_wh, s_sink, pos, base, nbits);
      if (wave == 0) {
        const CTile t = tile_finish(probe, cur.e, lim, f.msub, TILE);
        if (lane == 0) s_next[par] = t;
      }
      lds_barrier();
      uint32_t st, ex, all;
      const uint32_t d = TidOpaque::get();
      const uint32_t tot = digit_starts_present<kCWaves, TidOpaque>(nd, s_wh, s_tmp, &st, &ex, &all);
      tile_groups(p, cur.sb, nsub, cur.r0, d < nd ? tot : 0u, st, ex, all & 1023u, s_ex, s_st, s_bal);
      c_stage<NARROW>(f, r, pos, n, base, s_wh, s_k, s_t, s_w);
      lds_barrier();
      clear_wh(s_wh);
      const CTile nx = s_next[par];
      loaded = tile_fits<NARROW>(nx);
      if (loaded) load_c<NARROW>(f.ik, f.it, f.iw, nx.r0, nx.r1 - nx.r0, r);
      c_store<NARROW>(p, f, s_blk, s_k, s_t, s_w, n, base, cur.sb << b3, nullptr, cur.r0);
    }
    lds_barrier();  // s_next[par] is complete; the tile's LDS is free
    const CTile nx = s_next[par];
    if (!loaded && tile_fits<NARROW>(nx)) {
      load_c<NARROW>(f.ik, f.it, f.iw, nx.r0, nx.r1 - nx.r0, r);
      loaded = true;
    }
    cur = nx;
    par ^= 1u;  // wave 0 next writes the other slot; this one is read before the next barrier
  }
}

// The listed sub-buckets larger than one load: counted by D3, then sorted in
// pieces of one load, each piece's records of a D3 value following those of
// the pieces before.
template <int RB, bool NARROW>
__global__ __launch_bounds__(kCThreads) void k_msd_big_c(MsdPlan p) {
  M_C_LDS
  __shared__ uint32_t s_cur[kMNB];
  __shared__ uint32_t s_dx[kMNB];
  const CFields f = c_fields<NARROW>(p);
  char* const* s_blk = c_setup(p, s_blk_tab, s_wh);
  const uint32_t b3 = p.b3, nd = 1u << b3, d = TidOpaque::get();
  lds_barrier();
  for (uint32_t i = blockIdx.x; i < G(p.big_count)[0]; i += gridDim.x) {
    const uint32_t sb = G(p.big_list)[i];
    const uint32_t r0 = G(p.sbstart)[sb], n = G(p.sbstart)[sb + 1] - r0;
    const uint32_t base = (sb << b3) & f.km;
    for (uint32_t e = d; e < (uint32_t)kMNB; e += kCThreads) s_cur[e] = 0;
    lds_barrier();
    for (uint32_t j = d; j < n; j += kCThreads) atomicAdd(&s_cur[((G(f.ik)[r0 + j] >> f.ks) - base) & f.km], 1u);
    lds_barrier();
    {
      // a large sub-bucket may hold any number of records per digit: two scans
      const uint32_t h = d < nd ? s_cur[d] : 0u;
      uint32_t all_rec, all_present;
      const uint32_t hst = m_block_scan<kCWaves, TidOpaque>(h, s_tmp, &all_rec);
      const uint32_t ex = m_block_scan<kCWaves, TidOpaque>(h ? 1u : 0u, s_tmp, &all_present);
      tile_groups(p, sb, 1u, r0, h, hst, ex, all_present, s_ex, s_st, s_bal);
      lds_barrier();
      if (d < nd) s_cur[d] = r0 + hst;
    }
    for (uint32_t c0 = 0; c0 < n; c0 += CSize<NARROW>::TILE) {
      const uint32_t cnt = n - c0 < CSize<NARROW>::TILE ? n - c0 : CSize<NARROW>::TILE;
      Recs<CSize<NARROW>::ITEMS> r;
      load_c<NARROW>(f.ik, f.it, f.iw, r0 + c0, cnt, r);
      uint32_t pos[CSize<NARROW>::ITEMS];
      rank_digits<RB, CSize<NARROW>::ITEMS, false, TidOpaque>(r.k, f.ks, f.km, cnt, s_wh, s_sink, pos, base);
      lds_barrier();
      uint32_t st;
      const uint32_t tot = digit_starts<kCWaves, TidOpaque>(nd, s_wh, s_tmp, &st);
      if (d < nd) {
        const uint32_t cp = s_cur[d];
        s_dx[d] = cp - st;  // output position minus piece position
        s_cur[d] = cp + tot;
      }
      lds_barrier();  // every digit's wave starts are in s_wh
      c_stage<NARROW>(f, r, pos, cnt, base, s_wh, s_k, s_t, s_w);
      lds_barrier();
      clear_wh(s_wh);
      c_store<NARROW>(p, f, s_blk, s_k, s_t, s_w, cnt, base, sb << b3, s_dx, 0u);
      lds_barrier();
    }
  }
}

// group_start from the scanned group counts and the local group starts: one
// wave per sub-bucket copies its groups (up to 2^b3 of them), four
// sub-buckets per workgroup.  Workgroups past the sub-buckets' build
// group_ptr (Eq. (14)): the groups of all sources below i are the distinct
// keys below i << dbits, i.e. the groups of the sub-buckets before the one
// holding that key plus its present D3 values below the key's.
__global__ __launch_bounds__(256) void k_msd_groups(MsdPlan p) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t copy_blocks = (nsb + 3) / 4;
  if (blockIdx.x < copy_blocks) {
    const uint32_t sb = blockIdx.x * 4u + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
    if (sb < nsb) {
      const uint32_t g0 = p.gcount[sb], ng = p.gcount[sb + 1] - g0, start = p.sbstart[sb];
      for (uint32_t k = lane; k < ng; k += 64) p.group_start[g0 + k] = p.gslot[start + k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      p.group_start[p.gcount[nsb]] = p.n;
      *p.n_groups = p.gcount[nsb];
    }
    return;
  }
  const uint32_t i = (blockIdx.x - copy_blocks) * 256u + threadIdx.x;
  if (i <= p.n_nodes) {
    uint32_t v = p.gcount[nsb];
    if (i < p.n_nodes) {
      const uint32_t key = i << p.dbits;
      const uint32_t sb = key >> p.b3, local = key & ((1u << p.b3) - 1u);
      const uint32_t* gm = p.gmask + (uint64_t)sb * p.mask_words;
      v = p.gcount[sb];
      for (uint32_t w = 0; w < (local >> 5); ++w) v += (uint32_t)__popc(gm[w]);
      if (local & 31u) v += (uint32_t)__popc(gm[local >> 5] & ((1u << (local & 31u)) - 1u));
    }
    p.group_ptr[i] = v;
  }
}

// Digit widths have template instances 6, 8 and 9 (a digit uses the
// smallest one that holds it).
inline int rb_class(uint32_t bits) { return bits <= 6 ? 6 : (bits <= 8 ? 8 : 9); }

}  // namespace

uint32_t msd_cap(bool) { return kMsdTile; }

#define M_RB_SWITCH(bits, F) \
  switch (rb_class(bits)) {  \
    case 6: F(6); break;     \
    case 8: F(8); break;     \
    default: F(9); break;    \
  }

hipError_t launch_msd_count_a(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.ranges_a + 7) / 8));
  if (p.b2 + p.b3 < p.dbits) hipLaunchKernelGGL(k_msd_count_a<true>, grid, dim3(kCntThreads), 0, s, p);
  else hipLaunchKernelGGL(k_msd_count_a<false>, grid, dim3(kCntThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_msd_scatter_a(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.ranges_a + 7) / 8));
#define F(RB)                                                                                  \
  if (p.narrow_a) hipLaunchKernelGGL((k_msd_scatter_a<RB, true>), grid, dim3(kMThreads), 0, s, p); \
  else hipLaunchKernelGGL((k_msd_scatter_a<RB, false>), grid, dim3(kMThreads), 0, s, p);
  M_RB_SWITCH(p.b1, F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_plan_b(const MsdPlan& p, hipStream_t s) {
  hipLaunchKernelGGL(k_msd_plan_b, dim3(1), dim3(kMThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_msd_count_b(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.max_ranges_b + 7) / 8));
  if (p.narrow_a) hipLaunchKernelGGL(k_msd_count_b<IN_NARROW>, grid, dim3(kCntThreads), 0, s, p);
  else hipLaunchKernelGGL(k_msd_count_b<IN_WIDE>, grid, dim3(kCntThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_msd_scatter_b(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.max_ranges_b + 7) / 8));
  if (!(p.tile_b == kMsdTile || (p.narrow_a && p.tile_b == kMsdTileN))) return hipErrorInvalidValue;
#define F(RB)                                                                                                       \
  if (p.narrow_a && p.tile_b == kMsdTileN)                                                                           \
    hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_NARROW, true, kMItemsN>), grid, dim3(kMThreads), 0, s, p);            \
  else if (p.narrow_a) hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_NARROW, true, kMItems>), grid, dim3(kMThreads), 0, s, p); \
  else if (p.narrow_b) hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_WIDE, true, kMItems>), grid, dim3(kMThreads), 0, s, p);   \
  else hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_WIDE, false, kMItems>), grid, dim3(kMThreads), 0, s, p);
  M_RB_SWITCH(p.b2, F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_plan_c(const MsdPlan& p, hipStream_t s) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  if (p.b2) hipLaunchKernelGGL(k_msd_plan_c, dim3((nsb + 255) / 256), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_msd_zero, dim3(std::min<uint32_t>((nsb * p.mask_words + 255) / 256, 1024u)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_msd_split, dim3((p.wgs_c + 1 + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Combined-digit width of pass C's tiles: sub-bucket offset above D3.
static uint32_t c_digit_bits(const MsdPlan& p, bool narrow) {
  const uint32_t nd = msd_max_sub(p, narrow) << p.b3;
  uint32_t bits = 0;
  while ((1u << bits) < nd) ++bits;
  return bits;
}

hipError_t launch_msd_tiles_c(const MsdPlan& p, hipStream_t s) {
  const bool narrow = p.b2 ? p.narrow_b : p.narrow_a;
#define F(RB)                                                                                           \
  if (narrow) hipLaunchKernelGGL((k_msd_tiles_c<RB, true>), dim3(p.wgs_c), dim3(kCThreads), 0, s, p);   \
  else hipLaunchKernelGGL((k_msd_tiles_c<RB, false>), dim3(p.wgs_c), dim3(kCThreads), 0, s, p);
  M_RB_SWITCH(c_digit_bits(p, narrow), F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_big_c(const MsdPlan& p, hipStream_t s) {
  const bool narrow = p.b2 ? p.narrow_b : p.narrow_a;
  const dim3 grid(p.max_big < 256u ? p.max_big : 256u);
#define F(RB)                                                                                      \
  if (narrow) hipLaunchKernelGGL((k_msd_big_c<RB, true>), grid, dim3(kCThreads), 0, s, p);          \
  else hipLaunchKernelGGL((k_msd_big_c<RB, false>), grid, dim3(kCThreads), 0, s, p);
  M_RB_SWITCH(p.b3, F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_groups(const MsdPlan& p, hipStream_t s) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t blocks = (nsb + 3) / 4 + (p.n_nodes + 1 + 255) / 256;
  hipLaunchKernelGGL(k_msd_groups, dim3(blocks), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace ng
