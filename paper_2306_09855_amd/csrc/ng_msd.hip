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
constexpr int kMWaves = kMThreads / 64;
constexpr int kMItems = 20;
static_assert(kMThreads * kMItems == (int)kMsdTile, "tile of passes A and B");
constexpr int kMNB = 1 << kMsdMaxDigit;  // 512 digit values at most
static_assert(kMNB == kMThreads, "one thread per digit value");
constexpr int kCItemsN = 24;  // pass C, narrow records: 12288 per piece
constexpr int kCItemsW = 20;  // pass C, wide records: 10,240 per piece
constexpr int kMLdsBlocks = 512;

enum { IN_BLOCKS = 0, IN_NARROW = 1, IN_WIDE = 2 };

// Exclusive scan across the 512-thread workgroup; *total = the sum.
__device__ __forceinline__ uint32_t m_block_scan(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_tmp[wave] = inc;
  lds_barrier();
  uint32_t off = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < kMWaves; ++w) {
    const uint32_t t = s_tmp[w];
    if (w < wave) off += t;
    sum += t;
  }
  lds_barrier();
  *total = sum;
  return off + inc - v;
}

// XCD-aware range number: workgroup w runs on XCD w % 8, and each XCD takes
// a contiguous span of ranges, so neighbouring runs meet in one L2.
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

__device__ __forceinline__ uint32_t item_index(int ITEMS, int k) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t lj = item_index(ITEMS, k);
    if (FULL || lj < cnt) {
      const uint32_t j = base + lj;
      const char* blk = (j >> log2B) != b0 ? blk1 : blk0;
      const uint64_t o = j & (B - 1);
      const uint32_t s = G(reinterpret_cast<const uint32_t*>(blk))[o];
      r.t[k] = G(reinterpret_cast<const uint32_t*>(blk + 4 * B))[o];
      r.w[k] = G(reinterpret_cast<const uint32_t*>(blk + 8 * B))[o];
      r.k[k] = (s << dbits) | (uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o];
    } else {
      r.k[k] = r.t[k] = r.w[k] = 0;
    }
  }
}

template <int ITEMS, int IN, bool FULL>
__device__ __forceinline__ void load_arrays(const uint32_t* ik, const uint32_t* it, const uint32_t* iw,
                                            uint32_t base, uint32_t cnt, Recs<ITEMS>& r) {
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t lj = item_index(ITEMS, k);
    if (FULL || lj < cnt) {
      r.k[k] = G(ik)[base + lj];
      if constexpr (IN == IN_WIDE) r.t[k] = G(it)[base + lj];
      r.w[k] = G(iw)[base + lj];
    } else {
      r.k[k] = r.w[k] = 0;
      if constexpr (IN == IN_WIDE) r.t[k] = 0;
    }
  }
}

// Stable ranks of the tile's digits.  For each item slot the lanes holding
// the same digit (peers) come from one ballot per digit bit; a record's rank
// is the number of records of its digit in the wave's earlier slots plus its
// peers in lower lanes.  The lowest peer adds the slot's count to the wave's
// counter of that digit with one LDS atomic (other lanes add to a private
// word), and the old value reaches its peers through a lane permute a few
// slots later, so no slot waits on the one before it.  On return pos[k] is
// the rank within the wave's records of the digit, and wh[wave][d] holds the
// wave's count of digit d.
template <int RB, int ITEMS, bool FULL>
__device__ __forceinline__ void rank_digits(const uint32_t (&key)[ITEMS], uint32_t shift, uint32_t mask, uint32_t cnt,
                                            uint32_t* wh, uint32_t* sink, uint32_t (&pos)[ITEMS]) {
  constexpr int kLag = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t prv[ITEMS];
  // slots past the tile's end hold no record of this wave (a uniform test)
  auto slot_used = [&](int k) { return FULL || (uint32_t)(wave * ITEMS * 64 + k * 64) < cnt; };
#pragma unroll
  for (int k = 0; k < ITEMS + kLag; ++k) {
    if (k < ITEMS && slot_used(k)) {
      const uint32_t lj = (uint32_t)(wave * ITEMS * 64 + k * 64 + lane);
      const bool valid = FULL || lj < cnt;
      const uint32_t d = (key[k] >> shift) & mask;
      uint32_t plo = ~0u, phi = ~0u;
      if (!FULL) {
        const uint64_t v = __ballot(valid);
        plo = (uint32_t)v;
        phi = (uint32_t)(v >> 32);
      }
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const uint32_t sb = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // bit b, all ones or zero
        const uint64_t m = __ballot(sb != 0u);
        plo &= ~((uint32_t)m ^ sb);
        phi &= ~((uint32_t)(m >> 32) ^ sb);
      }
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
      const uint32_t tot = (uint32_t)__popc(plo) + (uint32_t)__popc(phi);
      const uint32_t lead = (uint32_t)__builtin_ctzll(((uint64_t)phi << 32) | plo | (1ull << 63));
      uint32_t* ctr = (valid && below == 0) ? &wh[wave * kMNB + d] : &sink[threadIdx.x];
      prv[k] = atomicAdd(ctr, tot);
      pos[k] = below | (lead << 8);
    }
    if (k >= kLag && slot_used(k - kLag)) {
      const int q = k - kLag;
      const uint32_t prev = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((pos[q] >> 8) << 2), (int)prv[q]);
      pos[q] = prev + (pos[q] & 0xFFu);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the lag: no permute moves up to its add
  }
}

// Thread d: digit d's counts over the waves become each wave's first tile
// position of that digit; returns the digit's count in the tile and sets
// *start to its first tile position.  Leaves wh[wave][d] = tile position.
__device__ __forceinline__ uint32_t digit_starts(uint32_t nd, uint32_t* wh, uint32_t* s_tmp, uint32_t* start) {
  const uint32_t d = threadIdx.x;
  uint32_t c[kMWaves];
  uint32_t tot = 0;
#pragma unroll
  for (int v = 0; v < kMWaves; ++v) {
    const uint32_t x = d < nd ? wh[v * kMNB + d] : 0u;
    c[v] = tot;
    tot += x;
  }
  uint32_t all;
  const uint32_t st = m_block_scan(tot, s_tmp, &all);
  if (d < nd) {
#pragma unroll
    for (int v = 0; v < kMWaves; ++v) wh[v * kMNB + d] = st + c[v];
  }
  *start = st;
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
  uint32_t* wh;          // [kMWaves][kMNB]
  uint4* dig;            // [kMNB]: x = global position of the digit's first record minus its
                         // tile position (mod 2^32); [y, y + z): positions whose 128-byte line
                         // the tile's run fills completely
  uint32_t* run;         // [kMNB] next global position per digit
  uint32_t* tmp;         // [kMWaves]
  uint32_t* sink;        // [kMThreads]
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
template <int RB, int IN, bool OUT_NARROW, bool FULL>
__device__ __forceinline__ void scatter_tile(const PassIO& io, uint32_t cnt, const ScatterLds& L, Recs<kMItems>& r,
                                             uint32_t next_base, uint32_t next_cnt) {
  constexpr bool HAS_T = IN != IN_NARROW;
  const int wave = threadIdx.x >> 6;
  uint32_t pos[kMItems];
  rank_digits<RB, kMItems, FULL>(r.k, io.shift, io.mask, cnt, L.wh, L.sink, pos);
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
  for (int k = 0; k < kMItems; ++k) {
    if (FULL || item_index(kMItems, k) < cnt) {
      const uint32_t p = pos[k] + L.wh[wave * kMNB + ((r.k[k] >> io.shift) & io.mask)];
      L.k[p] = r.k[k];
      if constexpr (HAS_T) L.t[p] = r.t[k];
      L.w[p] = r.w[k];
    }
  }
  lds_barrier();
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
#pragma unroll
    for (int v = 0; v < kMWaves; ++v) L.wh[v * kMNB + d] = 0;
  }
  if (next_cnt) load_tile_any<kMItems, IN>(io, next_base, next_cnt, r);
  // Runs of equal digits go to consecutive positions.  Stores of records
  // whose 128-byte lines the run fills are marked streaming; the partial
  // lines at a run's ends stay cached, so that the neighbouring tile's run
  // can complete them in L2 before they reach HBM.
#pragma unroll
  for (int k = 0; k < kMItems; ++k) {
    const uint32_t lp = (uint32_t)(k * kMThreads + threadIdx.x);
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
template <int RB, int IN, bool OUT_NARROW>
__device__ __forceinline__ void scatter_range(const PassIO& io, const ScatterLds& L, uint32_t span0, uint32_t span1,
                                              uint32_t t0, uint32_t t1) {
  if (t0 >= t1) return;
  Recs<kMItems> r;
  auto tile_cnt = [&](uint32_t t) {
    const uint32_t b = span0 + t * kMsdTile;
    return span1 - b < kMsdTile ? span1 - b : kMsdTile;
  };
  load_tile_any<kMItems, IN>(io, span0 + t0 * kMsdTile, tile_cnt(t0), r);
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t cnt = tile_cnt(t);
    const uint32_t nb = t + 1 < t1 ? span0 + (t + 1) * kMsdTile : 0u;
    const uint32_t nc = t + 1 < t1 ? tile_cnt(t + 1) : 0u;
    if (cnt == kMsdTile) scatter_tile<RB, IN, OUT_NARROW, true>(io, cnt, L, r, nb, nc);
    else scatter_tile<RB, IN, OUT_NARROW, false>(io, cnt, L, r, nb, nc);
  }
}

#define M_SCATTER_LDS                                   \
  __shared__ uint32_t s_k[kMsdTile];                    \
  __shared__ uint32_t s_t[IN == IN_NARROW ? 1 : kMsdTile]; \
  __shared__ uint32_t s_w[kMsdTile];                    \
  __shared__ uint32_t s_wh[kMWaves * kMNB];             \
  __shared__ uint4 s_dig[kMNB];                         \
  __shared__ uint32_t s_run[kMNB];                      \
  __shared__ uint32_t s_tmp[kMWaves];                   \
  __shared__ uint32_t s_sink[kMThreads];                \
  const ScatterLds L{s_k, s_t, s_w, s_wh, s_dig, s_run, s_tmp, s_sink};

// Pass A: range r of the creation-order records by D1.
template <int RB, bool OUT_NARROW>
__global__ __launch_bounds__(kMThreads) void k_msd_scatter_a(MsdPlan p) {
  constexpr int IN = IN_BLOCKS;
  M_SCATTER_LDS
  const uint32_t r = m_range((p.ranges_a + 7) / 8);
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
    for (int v = 0; v < kMWaves; ++v) s_wh[v * kMNB + d] = 0;
  }
  lds_barrier();
  const uint32_t ntiles = (p.n + kMsdTile - 1) / kMsdTile;
  const uint32_t t0 = r * p.tpr, t1 = min(t0 + p.tpr, ntiles);
  scatter_range<RB, IN, OUT_NARROW>(io, L, 0u, p.n, t0, t1);
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
template <int RB, int IN, bool OUT_NARROW>
__global__ __launch_bounds__(kMThreads) void k_msd_scatter_b(MsdPlan p) {
  M_SCATTER_LDS
  __shared__ uint32_t s_rb0[kMNB + 1];
  const uint32_t nb = 1u << p.b1, nd = 1u << p.b2;
  for (uint32_t b = threadIdx.x; b <= nb; b += kMThreads) s_rb0[b] = p.rangeb0[b];
  lds_barrier();
  const uint32_t r = m_range((p.max_ranges_b + 7) / 8);
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
  io.remmask = (1u << p.b3) - 1u;
  const uint64_t cb = ((uint64_t)s_rb0[b] << p.b2) + rl;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
    s_run[d] = d < nd ? p.cnt_b[cb + (uint64_t)d * nr] : 0u;
#pragma unroll
    for (int v = 0; v < kMWaves; ++v) s_wh[v * kMNB + d] = 0;
  }
  lds_barrier();
  const uint32_t ntiles = (be - bs + kMsdTile - 1) / kMsdTile;
  const uint32_t t0 = rl * p.tpr, t1 = min(t0 + p.tpr, ntiles);
  scatter_range<RB, IN, OUT_NARROW>(io, L, bs, be, t0, t1);
}

// ---------------------------------------------------------------------------
// Digit counts of the ranges of passes A and B.
// ---------------------------------------------------------------------------
// Pass A: D1 of every creation-order record (the delays are read only when
// D1 reaches into the delay bits).
template <bool NEED_DELAY>
__global__ __launch_bounds__(kMThreads) void k_msd_count_a(MsdPlan p) {
  __shared__ uint32_t hist[kMNB];
  const uint32_t r = m_range((p.ranges_a + 7) / 8);
  if (r >= p.ranges_a) return;
  const uint32_t nd = 1u << p.b1, shift = p.b2 + p.b3;
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) hist[d] = 0;
  __syncthreads();
  const uint32_t ntiles = (p.n + kMsdTile - 1) / kMsdTile;
  const uint32_t t0 = r * p.tpr, t1 = min(t0 + p.tpr, ntiles);
  const uint64_t B = 1ull << p.log2B;
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t base = t * kMsdTile;
    const uint32_t cnt = min(kMsdTile, p.n - base);
    // groups of 4 records never straddle a block: base and B are multiples of 4
    for (uint32_t q = threadIdx.x; 4 * q < cnt; q += kMThreads) {
      const uint32_t j = base + 4 * q;
      const char* blk = C(p.in_blocks, j >> p.log2B);
      const uint64_t o = j & (B - 1);
      uint32_t key[4];
      if (4 * q + 4 <= cnt) {
        const u32x4 s4 = *(const NG_GLOBAL u32x4*)(blk + 4 * o);
        uint32_t dl[4] = {0, 0, 0, 0};
        if constexpr (NEED_DELAY) {
          const u32x2 d4 = *(const NG_GLOBAL u32x2*)(blk + 12 * B + 2 * o);
          dl[0] = d4.x & 0xFFFFu;
          dl[1] = d4.x >> 16;
          dl[2] = d4.y & 0xFFFFu;
          dl[3] = d4.y >> 16;
        }
        key[0] = (s4.x << p.dbits) | dl[0];
        key[1] = (s4.y << p.dbits) | dl[1];
        key[2] = (s4.z << p.dbits) | dl[2];
        key[3] = (s4.w << p.dbits) | dl[3];
#pragma unroll
        for (int e = 0; e < 4; ++e) atomicAdd(&hist[(key[e] >> shift) & (nd - 1)], 1u);
      } else {
        for (uint32_t e = 0; 4 * q + e < cnt; ++e) {
          const uint32_t s = G(reinterpret_cast<const uint32_t*>(blk))[o + e];
          const uint32_t dl = NEED_DELAY ? (uint16_t)G(reinterpret_cast<const int16_t*>(blk + 12 * B))[o + e] : 0u;
          atomicAdd(&hist[(((s << p.dbits) | dl) >> shift) & (nd - 1)], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nd; d += kMThreads) p.cnt_a[(uint64_t)d * p.ranges_a + r] = hist[d];
}

// Pass B: D2 of the records of each range of each bucket.
template <int IN>
__global__ __launch_bounds__(kMThreads) void k_msd_count_b(MsdPlan p) {
  __shared__ uint32_t hist[kMNB];
  __shared__ uint32_t s_rb0[kMNB + 1];
  const uint32_t nb = 1u << p.b1, nd = 1u << p.b2;
  for (uint32_t b = threadIdx.x; b <= nb; b += kMThreads) s_rb0[b] = p.rangeb0[b];
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) hist[d] = 0;
  __syncthreads();
  const uint32_t r = m_range((p.max_ranges_b + 7) / 8);
  if (r >= s_rb0[nb]) return;
  const uint32_t b = bucket_of_range(s_rb0, nb, r);
  const uint32_t rl = r - s_rb0[b], nr = s_rb0[b + 1] - s_rb0[b];
  const uint32_t bs = p.bstart[b], be = p.bstart[b + 1];
  const uint32_t shift = (IN == IN_NARROW ? p.tbits : 0u) + p.b3;
  const uint32_t lo = bs + rl * p.tpr * kMsdTile;
  const uint32_t hi = (be - lo) / kMsdTile < p.tpr ? be : lo + p.tpr * kMsdTile;
  for (uint32_t j = lo + threadIdx.x; j < hi; j += kMThreads)
    atomicAdd(&hist[(G(p.a_key)[j] >> shift) & (nd - 1)], 1u);
  __syncthreads();
  const uint64_t cb = ((uint64_t)s_rb0[b] << p.b2) + rl;
  for (uint32_t d = threadIdx.x; d < nd; d += kMThreads) p.cnt_b[cb + (uint64_t)d * nr] = hist[d];
}

// ---------------------------------------------------------------------------
// Start tables.
// ---------------------------------------------------------------------------
// Bucket starts from the scanned counts of pass A, and the ranges of pass B
// (tiles of kMsdTile records from each bucket's start, tpr tiles per range).
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
  const uint32_t ntiles = (be - bs + kMsdTile - 1) / kMsdTile;
  const uint32_t nr = (ntiles + p.tpr - 1) / p.tpr;
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

// Workgroup w of pass C takes the sub-buckets whose first record lies in
// [w * n / wgs, (w + 1) * n / wgs): a split by records.
__global__ __launch_bounds__(256) void k_msd_split(MsdPlan p) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t w = blockIdx.x * 256u + threadIdx.x;
  if (w > p.wgs_c) return;
  if (w == p.wgs_c) {
    p.wg_sb0[w] = nsb;
    return;
  }
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
// Pass C: each sub-bucket sorted by D3 in LDS, written as calibrated blocks.
// ---------------------------------------------------------------------------
// Output block of a sorted position: from the LDS copy of the block table
// when it holds all of them.
__device__ __forceinline__ char* m_out_block(const MsdPlan& p, char* const* s_blk, uint32_t dest) {
  return s_blk ? s_blk[dest >> p.log2B] : C(p.out_blocks, dest >> p.log2B);
}

template <int RB, bool NARROW>
__global__ __launch_bounds__(kMThreads) void k_msd_local_c(MsdPlan p) {
  constexpr int ITEMS = NARROW ? kCItemsN : kCItemsW;
  constexpr uint32_t CAP = (uint32_t)(ITEMS * kMThreads);
  __shared__ uint32_t s_k[CAP];
  __shared__ uint32_t s_t[NARROW ? 1 : CAP];
  __shared__ uint32_t s_w[CAP];
  __shared__ uint32_t s_wh[kMWaves * kMNB];
  __shared__ uint32_t s_hist[kMNB];  // counts of the sub-bucket per D3 value
  __shared__ uint32_t s_cur[kMNB];   // next output position per D3 value
  __shared__ uint32_t s_dx[kMNB];    // output position minus piece position, per D3 value
  __shared__ uint32_t s_tmp[kMWaves];
  __shared__ uint32_t s_sink[kMThreads];
  __shared__ char* s_blk_tab[kMLdsBlocks];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nd = 1u << p.b3, m3 = nd - 1;
  const uint32_t kshift = NARROW ? p.tbits : 0u;
  const uint32_t tmask = NARROW ? ((1u << p.tbits) - 1u) : ~0u;
  const uint32_t dmask = (1u << p.dbits) - 1u;
  const uint32_t n_out_blocks = (uint32_t)(((uint64_t)p.n + (1ull << p.log2B) - 1) >> p.log2B);
  char* const* s_blk = n_out_blocks <= (uint32_t)kMLdsBlocks ? s_blk_tab : nullptr;
  if (s_blk)
    for (uint32_t b = threadIdx.x; b < n_out_blocks; b += kMThreads) s_blk_tab[b] = C(p.out_blocks, b);
  for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) {
#pragma unroll
    for (int v = 0; v < kMWaves; ++v) s_wh[v * kMNB + d] = 0;
  }
  const uint32_t* ik = p.b2 ? p.b_key : p.a_key;
  const uint32_t* it = p.b2 ? p.b_tgt : p.a_tgt;
  const uint32_t* iw = p.b2 ? p.b_w : p.a_w;
  const uint64_t B = 1ull << p.log2B;
  const uint32_t sb0 = p.wg_sb0[blockIdx.x], sb1 = p.wg_sb0[blockIdx.x + 1];
  lds_barrier();
  for (uint32_t sb = sb0; sb < sb1; ++sb) {
    const uint32_t start = p.sbstart[sb], n = p.sbstart[sb + 1] - start;
    if (n == 0) {  // no records, no groups
      uint32_t* gm = p.gmask + (uint64_t)sb * p.mask_words;
      for (uint32_t w = threadIdx.x; w < p.mask_words; w += kMThreads) G(gm)[w] = 0;
      if (threadIdx.x == 0) G(p.gcount)[sb] = 0;
      continue;
    }
    if (n > CAP) {  // counting pre-pass over the whole sub-bucket
      for (uint32_t d = threadIdx.x; d < (uint32_t)kMNB; d += kMThreads) s_hist[d] = 0;
      lds_barrier();
      for (uint32_t j = threadIdx.x; j < n; j += kMThreads)
        atomicAdd(&s_hist[(G(ik)[start + j] >> kshift) & m3], 1u);
      lds_barrier();
    }
    for (uint32_t c0 = 0; c0 < n; c0 += CAP) {
      const uint32_t cnt = n - c0 < CAP ? n - c0 : CAP;
      Recs<ITEMS> r;
      uint32_t pos[ITEMS];
      load_arrays<ITEMS, NARROW ? IN_NARROW : IN_WIDE, false>(ik, it, iw, start + c0, cnt, r);
      rank_digits<RB, ITEMS, false>(r.k, kshift, m3, cnt, s_wh, s_sink, pos);
      lds_barrier();
      const uint32_t d = threadIdx.x;
      uint32_t st;
      const uint32_t tot = digit_starts(nd, s_wh, s_tmp, &st);
      if (n <= CAP && d < nd) s_hist[d] = tot;
      if (c0 == 0) {
        // the sub-bucket's groups: its present D3 values (Sec. 2.2)
        lds_barrier();
        const uint32_t h = d < nd ? s_hist[d] : 0u;
        uint32_t all;
        const uint32_t ex = m_block_scan(h, s_tmp, &all);
        const bool present = h != 0;
        uint32_t ng;
        const uint32_t gi = m_block_scan(present ? 1u : 0u, s_tmp, &ng);
        if (d < nd) s_cur[d] = start + ex;
        if (present) G(p.gslot)[start + gi] = start + ex;
        const uint64_t bits = __ballot(present);
        const uint32_t mw = p.mask_words;
        uint32_t* gm = p.gmask + (uint64_t)sb * mw;
        if (lane == 0) {
          if (2u * (uint32_t)wave < mw) G(gm)[2 * wave] = (uint32_t)bits;
          if (2u * (uint32_t)wave + 1 < mw) G(gm)[2 * wave + 1] = (uint32_t)(bits >> 32);
        }
        if (threadIdx.x == 0) G(p.gcount)[sb] = ng;
      }
      lds_barrier();
      if (d < nd) {
        const uint32_t cur = s_cur[d];
        s_dx[d] = cur - st;
        s_cur[d] = cur + tot;
      }
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (item_index(ITEMS, k) < cnt) {
          const uint32_t q = pos[k] + s_wh[wave * kMNB + ((r.k[k] >> kshift) & m3)];
          s_k[q] = r.k[k];
          if constexpr (!NARROW) s_t[q] = r.t[k];
          s_w[q] = r.w[k];
        }
      }
      lds_barrier();
      for (uint32_t e = threadIdx.x; e < (uint32_t)kMNB; e += kMThreads) {
#pragma unroll
        for (int v = 0; v < kMWaves; ++v) s_wh[v * kMNB + e] = 0;
      }
      // Sorted records out: one piece is contiguous per D3 value, and a
      // sub-bucket that fits in one piece is one contiguous run.
      const uint32_t sbk = sb << p.b3;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const uint32_t lp = (uint32_t)(k * kMThreads + threadIdx.x);
        if (lp < cnt) {
          const uint32_t kk = s_k[lp];
          const uint32_t d3 = (kk >> kshift) & m3;
          const uint32_t dest = s_dx[d3] + lp;
          const uint32_t key = sbk | d3;
          char* blk = m_out_block(p, s_blk, dest);
          const uint64_t o = dest & (B - 1);
          G(reinterpret_cast<uint32_t*>(blk))[o] = key >> p.dbits;
          G(reinterpret_cast<uint32_t*>(blk + 4 * B))[o] = NARROW ? (kk & tmask) : s_t[lp];
          G(reinterpret_cast<uint32_t*>(blk + 8 * B))[o] = s_w[lp];
          G(reinterpret_cast<int16_t*>(blk + 12 * B))[o] = (int16_t)(key & dmask);
        }
      }
      lds_barrier();
    }
  }
}

// group_start from the scanned group counts and the local group starts;
// group_ptr (Eq. (14)): the groups of all sources below i are the distinct
// keys below i << dbits, i.e. the groups of the sub-buckets before the one
// holding that key plus its present D3 values below the key's.
__global__ __launch_bounds__(256) void k_msd_groups(MsdPlan p) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < nsb) {
    const uint32_t g0 = p.gcount[i], ng = p.gcount[i + 1] - g0, start = p.sbstart[i];
    for (uint32_t k = 0; k < ng; ++k) p.group_start[g0 + k] = p.gslot[start + k];
  }
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
  if (i == 0) {
    p.group_start[p.gcount[nsb]] = p.n;
    *p.n_groups = p.gcount[nsb];
  }
}

// Digit widths have template instances 6, 8 and 9 (a digit uses the
// smallest one that holds it).
inline int rb_class(uint32_t bits) { return bits <= 6 ? 6 : (bits <= 8 ? 8 : 9); }

}  // namespace

uint32_t msd_cap(bool narrow) { return (uint32_t)((narrow ? kCItemsN : kCItemsW) * kMThreads); }

#define M_RB_SWITCH(bits, F) \
  switch (rb_class(bits)) {  \
    case 6: F(6); break;     \
    case 8: F(8); break;     \
    default: F(9); break;    \
  }

hipError_t launch_msd_count_a(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.ranges_a + 7) / 8));
  if (p.b2 + p.b3 < p.dbits) hipLaunchKernelGGL(k_msd_count_a<true>, grid, dim3(kMThreads), 0, s, p);
  else hipLaunchKernelGGL(k_msd_count_a<false>, grid, dim3(kMThreads), 0, s, p);
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
  if (p.narrow_a) hipLaunchKernelGGL(k_msd_count_b<IN_NARROW>, grid, dim3(kMThreads), 0, s, p);
  else hipLaunchKernelGGL(k_msd_count_b<IN_WIDE>, grid, dim3(kMThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_msd_scatter_b(const MsdPlan& p, hipStream_t s) {
  const dim3 grid(8 * ((p.max_ranges_b + 7) / 8));
#define F(RB)                                                                                                \
  if (p.narrow_a) hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_NARROW, true>), grid, dim3(kMThreads), 0, s, p); \
  else if (p.narrow_b) hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_WIDE, true>), grid, dim3(kMThreads), 0, s, p); \
  else hipLaunchKernelGGL((k_msd_scatter_b<RB, IN_WIDE, false>), grid, dim3(kMThreads), 0, s, p);
  M_RB_SWITCH(p.b2, F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_plan_c(const MsdPlan& p, hipStream_t s) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  if (p.b2) hipLaunchKernelGGL(k_msd_plan_c, dim3((nsb + 255) / 256), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_msd_split, dim3((p.wgs_c + 1 + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_msd_local_c(const MsdPlan& p, hipStream_t s) {
  const bool narrow = p.b2 ? p.narrow_b : p.narrow_a;
#define F(RB)                                                                                  \
  if (narrow) hipLaunchKernelGGL((k_msd_local_c<RB, true>), dim3(p.wgs_c), dim3(kMThreads), 0, s, p); \
  else hipLaunchKernelGGL((k_msd_local_c<RB, false>), dim3(p.wgs_c), dim3(kMThreads), 0, s, p);
  M_RB_SWITCH(p.b3, F)
#undef F
  return hipGetLastError();
}

hipError_t launch_msd_groups(const MsdPlan& p, hipStream_t s) {
  const uint32_t nsb = 1u << (p.b1 + p.b2);
  const uint32_t m = std::max(nsb, p.n_nodes + 1);
  hipLaunchKernelGGL(k_msd_groups, dim3((m + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace ng
