// Device helpers shared by the kernel files (not part of the C ABI):
// the Philox4x32-10 streams, the per-synapse generation of a Connect call
// (Sec. 2.1 of Golosio et al.), the block-structured stores of generated
// records, workgroup scans and the LDS-only barrier.
#pragma once

#include "ng_internal.h"

namespace ng {
namespace {


// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
constexpr uint32_t kPhiloxMul0 = 0xD2511F53u;
constexpr uint32_t kPhiloxMul1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 three-input bit operation (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t* out) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = (uint64_t)c0 * kPhiloxMul0;
    const uint64_t b = (uint64_t)c2 * kPhiloxMul1;
    const uint32_t n0 = xor3((uint32_t)(b >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(a >> 32), c3, k1);
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = n0;
    c2 = n2;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// word block j of stream s of call cid
__device__ __forceinline__ void philox_block(uint64_t j, uint32_t cid, uint32_t s, uint32_t key0,
                                             uint32_t key1, uint32_t* out) {
  philox10((uint32_t)j, (uint32_t)(j >> 32), cid, s, key0, key1, out);
}

// rand(N): floor(x * N / 2^32)
__device__ __forceinline__ uint32_t rand_below(uint32_t x, uint32_t n) { return __umulhi(x, n); }

constexpr float kInv2p24 = 5.9604644775390625e-08f;  // 2^-24

enum { R_ONE_TO_ONE = 0, R_ALL_TO_ALL = 1, R_INDEG = 2, R_OUTDEG = 3, R_TOTAL = 4,
       R_INDEG_D = kRuleIndegDistinct, R_OUTDEG_D = kRuleOutdegDistinct, R_TOTAL_D = kRuleTotalDistinct };

// Distinct draws (no multapses): x -> pi(x), a permutation of [0, m) keyed by
// (call, node u).  A 4-round Feistel network on n bits, the smallest n >= 2
// with 2^n >= m, applied again until the value falls below m (the cycle
// through x returns below m; at most 2m values are visited per cycle step,
// so about 2 steps on average).  x = L * 2^nb + R, R the low nb = n -
// floor(n/2) bits, L the high na = floor(n/2) bits; rounds 0 and 2 set
// L ^= F_r(R) mod 2^na, rounds 1 and 3 R ^= F_r(L) mod 2^nb, with
// F_r(v) = lowbias32(v ^ k_r), lowbias32 the integer hash of C. Wellons
// (2018) and k_0..k_3 the words of Philox(u, 0, call, 131072).  Both halves
// fit 32 bits, so the rounds are 32-bit arithmetic.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

struct PermKeys {
  uint32_t k[4];
};

__device__ __forceinline__ void perm_keys(PermKeys& p, uint32_t u, uint32_t cid, uint32_t key0, uint32_t key1) {
  philox10(u, 0u, cid, 131072u, key0, key1, p.k);
}

// The walk from x returns below m only for x below m; it then takes at most
// 2^n - m + 1 steps, and more than kWalkCap steps only after kWalkCap
// consecutive cycle values at or above m, each of which has probability
// below one half.  Both conditions are checked: x >= m (a caller's bug) sets
// bit 0 and a walk that reaches the cap sets bit 1 of the call's error word,
// which the host reports as a sticky device error; the value is then 0, and
// every walk ends.
constexpr uint32_t kWalkCap = 4096;
__device__ __forceinline__ uint64_t permute_below(uint64_t x, uint64_t m, const PermKeys& p, uint32_t* err) {
  if (x >= m) {
    atomicOr(err, 1u);
    return 0;
  }
  const int n = m <= 4 ? 2 : 64 - __clzll((long long)(m - 1));
  const int na = n >> 1, nb = n - na;
  const uint32_t mask_a = (uint32_t)((1ull << na) - 1), mask_b = (uint32_t)((1ull << nb) - 1);
  uint64_t y = x;
  uint32_t steps = 0;
  do {
    uint32_t l = (uint32_t)(y >> nb), r = (uint32_t)y & mask_b;
    l ^= lowbias32(r ^ p.k[0]) & mask_a;
    r ^= lowbias32(l ^ p.k[1]) & mask_b;
    l ^= lowbias32(r ^ p.k[2]) & mask_a;
    r ^= lowbias32(l ^ p.k[3]) & mask_b;
    y = ((uint64_t)l << nb) | r;
  } while (y >= m && ++steps < kWalkCap);
  if (y >= m) {
    atomicOr(err, 2u);
    return 0;
  }
  return y;
}

// Word streams of a call: synapse i takes word i of its own stream for each
// random quantity (source draw, target draw, delay), so one Philox block of a
// stream serves a lane's four synapses; weights come from stream 1.
constexpr uint32_t kStreamSrc = 0u, kStreamW = 1u, kStreamTgt = 2u, kStreamDelay = 3u;

template <int RULE>
struct RuleDraws {  // which index draws a rule takes (the distinct draws take none)
  static constexpr bool src = RULE == R_TOTAL || RULE == R_INDEG;
  static constexpr bool tgt = RULE == R_TOTAL || RULE == R_OUTDEG;
};

struct Quad {
  uint32_t s[4], t[4];
  float w[4];
  int32_t d[4];
};

// Random delay from one word (Sec. 2.1): integer steps, or ms -> steps with a
// one-step minimum.
__device__ __forceinline__ int32_t delay_from_word(const GenDesc& d, uint32_t xd) {
  if (d.d_kind == D_UNIFORM_INT) return (int32_t)(d.d_lo + rand_below(xd, d.d_range));
  const float u = (float)(xd >> 8) * kInv2p24;
  const float ms = __fmaf_rn(d.d_ms_width, u, d.d_ms_lo);
  const float steps = rintf(__fdiv_rn(ms, d.h));
  return steps < 1.0f ? 1 : (int32_t)steps;
}

// A delay given in ms as integer steps (Sec. 2.1), at least one step.
__device__ __forceinline__ float ms_to_steps(float ms, float h) {
  const float steps = rintf(__fdiv_rn(ms, h));  // as the generation kernel's ms path
  return steps < 1.0f ? 1.0f : steps;
}

// Random weights from stream 1.  Normal: synapses 2j and 2j+1 take the cosine
// and sine outputs of Box-Muller on words 2j, 2j+1; uniform: synapse i takes
// word i.
__device__ __forceinline__ void normal_pair(const GenDesc& d, uint32_t y0, uint32_t y1, float& w_cos,
                                            float& w_sin) {
  const float u1 = (float)((y0 >> 8) + 1u) * kInv2p24;  // (0, 1]
  const float u2 = (float)(y1 >> 8) * kInv2p24;         // [0, 1)
  const float rad = __fsqrt_rn(-2.0f * logf(u1));
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  w_cos = __fmaf_rn(d.w_b, rad * cs, d.w_a);
  w_sin = __fmaf_rn(d.w_b, rad * sn, d.w_a);
}

__device__ __forceinline__ float uniform_weight(const GenDesc& d, uint32_t y) {
  return __fmaf_rn(d.w_b, (float)(y >> 8) * kInv2p24, d.w_a);
}

// Synapses i0..i0+3 of one call (i0 = 4g): block g of the source, target and
// delay streams the rule draws from.
template <int RULE, bool DRAND>
__device__ __forceinline__ void gen_quad(const GenDesc& d, uint32_t g, uint32_t key0, uint32_t key1,
                                         Quad& q) {
  const uint32_t i0 = g << 2;
  uint32_t xs[4], xt[4], xd[4];
  if constexpr (RuleDraws<RULE>::src) philox_block(g, d.cid, kStreamSrc, key0, key1, xs);
  if constexpr (RuleDraws<RULE>::tgt) philox_block(g, d.cid, kStreamTgt, key0, key1, xt);
  if constexpr (DRAND) philox_block(g, d.cid, kStreamDelay, key0, key1, xd);

  // source / target indices, Eqs. (4)-(13)
  if constexpr (RULE == R_INDEG_D || RULE == R_OUTDEG_D || RULE == R_TOTAL_D) {
    // no multapses: positions from a permutation keyed by the fixed node;
    // the node's keys are drawn once per quad unless the quad crosses nodes
    PermKeys pk;
    uint32_t node = 0, pos = 0;
    if constexpr (RULE == R_TOTAL_D) {
      perm_keys(pk, 0u, d.cid, key0, key1);
    } else {
      node = i0 / d.k;
      pos = i0 - node * d.k;
      perm_keys(pk, (RULE == R_INDEG_D ? d.t0 : d.s0) + node, d.cid, key0, key1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = i0 + r;
      if constexpr (RULE != R_TOTAL_D) {
        if (r > 0 && ++pos == d.k) {
          pos = 0;
          ++node;
          perm_keys(pk, (RULE == R_INDEG_D ? d.t0 : d.s0) + node, d.cid, key0, key1);
        }
      }
      if constexpr (RULE == R_INDEG_D) {
        const uint32_t t = d.t0 + node;
        const bool in_s = d.no_self && t - d.s0 < d.ns;
        uint32_t a = (uint32_t)permute_below(pos, d.ns - (in_s ? 1u : 0u), pk, d.err);
        if (in_s && a >= t - d.s0) ++a;
        q.s[r] = d.s0 + a;
        q.t[r] = t;
      } else if constexpr (RULE == R_OUTDEG_D) {
        const uint32_t s = d.s0 + node;
        const bool in_t = d.no_self && s - d.t0 < d.nt;
        uint32_t b = (uint32_t)permute_below(pos, d.nt - (in_t ? 1u : 0u), pk, d.err);
        if (in_t && b >= s - d.t0) ++b;
        q.s[r] = s;
        q.t[r] = d.t0 + b;
      } else {
        // pair index in all_to_all order (without the self-pairs when prohibited)
        // a lane past the call's end (its result is not stored) walks from 0:
        // the walk from x ends only for x below n_pairs, and i may not be
        // when the call takes nearly every pair
        const uint64_t k = permute_below(i < d.n_new ? i : 0u, d.n_pairs, pk, d.err);
        uint64_t a, b;
        if (!d.no_self) {
          a = k / d.nt;
          b = k - a * d.nt;
        } else {
          const uint64_t p1 = (uint64_t)d.a_lo * d.nt;
          const uint64_t p2 = p1 + (uint64_t)(d.a_hi - d.a_lo) * (d.nt - 1);
          if (k < p1) {
            a = k / d.nt;
            b = k - a * d.nt;
          } else if (k < p2) {
            const uint64_t l2 = d.nt > 1 ? d.nt - 1 : 1;
            a = d.a_lo + (k - p1) / l2;
            b = (k - p1) - (a - d.a_lo) * l2;
            if (d.t0 + b >= d.s0 + a) ++b;
          } else {
            a = d.a_hi + (k - p2) / d.nt;
            b = (k - p2) - (a - d.a_hi) * d.nt;
          }
        }
        q.s[r] = d.s0 + (uint32_t)a;
        q.t[r] = d.t0 + (uint32_t)b;
      }
    }
  } else if (d.no_self && RULE != R_ONE_TO_ONE) {
    // no connection from a node to itself (the ranges overlap)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = i0 + r;
      if constexpr (RULE == R_ALL_TO_ALL) {
        // rows before the overlap have N_t targets, rows of sources that are
        // targets N_t - 1 (their own node skipped), rows after it N_t
        const uint64_t p1 = (uint64_t)d.a_lo * d.nt;
        const uint32_t l2 = d.nt > 1 ? d.nt - 1 : 1;
        const uint64_t p2 = p1 + (uint64_t)(d.a_hi - d.a_lo) * (d.nt - 1);
        uint32_t a, b;
        if (i < p1) {
          a = i / d.nt;
          b = i - a * d.nt;
        } else if (i < p2) {
          const uint32_t j = (uint32_t)(i - p1);
          a = d.a_lo + j / l2;
          b = j - (a - d.a_lo) * l2;
          if (d.t0 + b >= d.s0 + a) ++b;  // skip t == s
        } else {
          const uint32_t j = (uint32_t)(i - p2);
          a = d.a_hi + j / d.nt;
          b = j - (a - d.a_hi) * d.nt;
        }
        q.s[r] = d.s0 + a;
        q.t[r] = d.t0 + b;
      } else if constexpr (RULE == R_OUTDEG) {
        const uint32_t s = d.s0 + i / d.k;
        const bool in_t = s - d.t0 < d.nt;  // s in [t0, t0 + nt)
        uint32_t b = rand_below(xt[r], d.nt - (in_t ? 1u : 0u));
        if (in_t && b >= s - d.t0) ++b;
        q.s[r] = s;
        q.t[r] = d.t0 + b;
      } else if constexpr (RULE == R_INDEG) {
        const uint32_t t = d.t0 + i / d.k;
        const bool in_s = t - d.s0 < d.ns;
        uint32_t a = rand_below(xs[r], d.ns - (in_s ? 1u : 0u));
        if (in_s && a >= t - d.s0) ++a;
        q.s[r] = d.s0 + a;
        q.t[r] = t;
      } else {  // R_TOTAL: redraw autapses from attempt streams 65536 + a, words 2i and 2i+1
        uint32_t a = rand_below(xs[r], d.ns), b = rand_below(xt[r], d.nt);
        for (uint32_t att = 1; d.s0 + a == d.t0 + b; ++att) {
          uint32_t y[4];
          philox_block(i >> 1, d.cid, 65536u + att, key0, key1, y);
          const uint32_t ys = y[(i & 1u) * 2], yt = y[(i & 1u) * 2 + 1];
          a = rand_below(ys, d.ns);
          if (att < 64) {
            b = rand_below(yt, d.nt);
          } else {  // the last attempt draws a target other than the source
            const uint32_t s = d.s0 + a;
            const bool in_t = s - d.t0 < d.nt;
            b = rand_below(yt, d.nt - (in_t ? 1u : 0u));
            if (in_t && b >= s - d.t0) ++b;
            break;
          }
        }
        q.s[r] = d.s0 + a;
        q.t[r] = d.t0 + b;
      }
    }
  } else if constexpr (RULE == R_ONE_TO_ONE) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q.s[r] = d.s0 + i0 + r;
      q.t[r] = d.t0 + i0 + r;
    }
  } else if constexpr (RULE == R_ALL_TO_ALL) {
    uint32_t a = i0 / d.nt, b = i0 - a * d.nt;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q.s[r] = d.s0 + a;
      q.t[r] = d.t0 + b;
      if (++b == d.nt) { b = 0; ++a; }
    }
  } else if constexpr (RULE == R_OUTDEG) {
    uint32_t a = i0 / d.k, b = i0 - a * d.k;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q.s[r] = d.s0 + a;
      q.t[r] = d.t0 + rand_below(xt[r], d.nt);
      if (++b == d.k) { b = 0; ++a; }
    }
  } else if constexpr (RULE == R_INDEG) {
    uint32_t a = i0 / d.k, b = i0 - a * d.k;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q.s[r] = d.s0 + rand_below(xs[r], d.ns);
      q.t[r] = d.t0 + a;
      if (++b == d.k) { b = 0; ++a; }
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      q.s[r] = d.s0 + rand_below(xs[r], d.ns);
      q.t[r] = d.t0 + rand_below(xt[r], d.nt);
    }
  }

  // delays (Sec. 2.1): integer steps, or ms -> steps with a one-step minimum
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if constexpr (DRAND) {
      q.d[r] = delay_from_word(d, xd[r]);
    } else {
      q.d[r] = d.d_const;
    }
  }

  // weights from stream 1, block g (words 4g..4g+3)
  if (d.w_kind == W_CONST) {
#pragma unroll
    for (int r = 0; r < 4; ++r) q.w[r] = d.w_a;
  } else {
    uint32_t y[4];
    philox_block(g, d.cid, kStreamW, key0, key1, y);
    if (d.w_kind == W_NORMAL) {
      normal_pair(d, y[0], y[1], q.w[0], q.w[1]);
      normal_pair(d, y[2], y[3], q.w[2], q.w[3]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) q.w[r] = uniform_weight(d, y[r]);
    }
  }
}

// Address spaces.  Pointers read from descriptors and block tables are
// generic to the compiler, but every one of them addresses device memory:
// saying so makes loads and stores take the global path instead of the flat
// one (a flat access also counts against the LDS counter, so every LDS wait
// would wait for it).  Descriptor tables are read through the constant path,
// with uniform indices, so they land in scalar registers.
#define NG_GLOBAL __attribute__((address_space(1)))
#define NG_CONST __attribute__((address_space(4)))
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ NG_GLOBAL T* G(T* p) { return (NG_GLOBAL T*)p; }
// element i of a read-only table (scalar loads when i is uniform)
template <class T>
__device__ __forceinline__ T C(const T* p, uint64_t i) { return ((const NG_CONST T*)p)[i]; }
// a descriptor struct from a read-only table, word by word through the
// constant path (i uniform)
template <class T>
__device__ __forceinline__ T C_struct(const T* p, uint32_t i) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size");
  T out;
  const NG_CONST uint32_t* w = (const NG_CONST uint32_t*)(p + i);
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (unsigned k = 0; k < sizeof(T) / 4; ++k) o[k] = w[k];
  return out;
}
__device__ __forceinline__ void st_u32x4(void* p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  *(NG_GLOBAL u32x4*)p = u32x4{a, b, c, d};
}
__device__ __forceinline__ void st_u32x2(void* p, uint32_t a, uint32_t b) { *(NG_GLOBAL u32x2*)p = u32x2{a, b}; }
// Stores marked streaming (non-temporal): for lines a store fills completely.
__device__ __forceinline__ void st_u32_nt(void* p, uint32_t a) { __builtin_nontemporal_store(a, (NG_GLOBAL uint32_t*)p); }
__device__ __forceinline__ void st_u32x2_nt(void* p, uint32_t a, uint32_t b) {
  __builtin_nontemporal_store(u32x2{a, b}, (NG_GLOBAL u32x2*)p);
}
__device__ __forceinline__ uint2 ld_u32x2(const void* p) {
  const u32x2 v = *(const NG_GLOBAL u32x2*)p;
  return make_uint2(v.x, v.y);
}

// Block layout: src u32[B] | tgt u32[B] | w f32[B] | delay i16[B]
__device__ __forceinline__ void store_one(char* const* __restrict__ blocks, int log2B, uint64_t p,
                                          uint32_t s, uint32_t t, float w, int32_t dl) {
  const uint64_t B = 1ull << log2B;
  char* base = G(blocks)[p >> log2B];
  const uint64_t o = p & (B - 1);
  G(reinterpret_cast<uint32_t*>(base))[o] = s;
  G(reinterpret_cast<uint32_t*>(base + 4 * B))[o] = t;
  G(reinterpret_cast<float*>(base + 8 * B))[o] = w;
  G(reinterpret_cast<int16_t*>(base + 12 * B))[o] = (int16_t)dl;
}

// The aligned 4-record chunk that starts s records into this lane's quad:
// [a[4-s..3], b[0..3-s]] (1 <= s <= 3), selected by value (a select between
// array elements would put the arrays in scratch memory).
struct Chunk4 {
  uint32_t v[4];
};
__device__ __forceinline__ Chunk4 chunk_of(const uint32_t (&a)[4], const uint32_t (&b)[4], uint32_t s) {
  const uint32_t a1 = a[1], a2 = a[2], a3 = a[3], b0 = b[0], b1 = b[1], b2 = b[2];
  Chunk4 c;
  c.v[0] = s == 1 ? a3 : (s == 2 ? a2 : a1);
  c.v[1] = s == 1 ? b0 : (s == 2 ? a3 : a2);
  c.v[2] = s == 1 ? b1 : (s == 2 ? b0 : a3);
  c.v[3] = s == 1 ? b2 : (s == 2 ? b1 : b0);
  return c;
}

// Store the quad of records p0..p0+nvalid-1.  A quad whose first position is
// a multiple of 4 goes out as 16-byte (8-byte for delays) stores.  A call
// whose first position is not leaves every quad misaligned by s = p0 mod 4;
// then each lane stores the aligned chunk that starts inside its quad,
// completed with the first 4-s records of the lane above (a shuffle), when
// that lane holds the next records of the same block table.  Records no
// aligned chunk covers (a wave's or a call's edges) go out one by one.  Every
// active lane of the wave must call this together.
__device__ __forceinline__ void store_quad(char* const* __restrict__ blocks, int log2B, uint64_t p0,
                                           uint32_t nvalid, const Quad& q) {
  const uint64_t B = 1ull << log2B;
  const int lane = threadIdx.x & 63;
  const uint64_t active = __ballot(1);
  const uint32_t s = (uint32_t)p0 & 3u;
  uint32_t w[4], dl[4], sn[4], tn[4], wn[4], dn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    w[r] = __float_as_uint(q.w[r]);
    dl[r] = (uint32_t)q.d[r] & 0xFFFFu;
    sn[r] = __shfl_down(q.s[r], 1);
    tn[r] = __shfl_down(q.t[r], 1);
    wn[r] = __shfl_down(w[r], 1);
    dn[r] = __shfl_down(dl[r], 1);
  }
  const uint64_t p0n = ((uint64_t)__shfl_down((uint32_t)(p0 >> 32), 1) << 32) | __shfl_down((uint32_t)p0, 1);
  const uint32_t nvn = __shfl_down(nvalid, 1);
  const uint64_t tab = (uint64_t)blocks;
  const uint64_t tabn = ((uint64_t)__shfl_down((uint32_t)(tab >> 32), 1) << 32) | __shfl_down((uint32_t)tab, 1);
  const bool next_active = lane < 63 && ((active >> ((lane + 1) & 63)) & 1ull);
  const bool chunk = s != 0 && next_active && p0n == p0 + 4 && tabn == tab && nvalid == 4 && nvn >= 4 - s;
  const bool head_done = __shfl_up(chunk ? 1u : 0u, 1) != 0u && lane > 0 && ((active >> ((lane - 1) & 63)) & 1ull);

  if (s == 0 && nvalid == 4) {
    char* base = G(blocks)[p0 >> log2B];
    const uint64_t o = p0 & (B - 1);
    st_u32x4(base + 4 * o, q.s[0], q.s[1], q.s[2], q.s[3]);
    st_u32x4(base + 4 * B + 4 * o, q.t[0], q.t[1], q.t[2], q.t[3]);
    st_u32x4(base + 8 * B + 4 * o, w[0], w[1], w[2], w[3]);
    st_u32x2(base + 12 * B + 2 * o, dl[0] | (dl[1] << 16), dl[2] | (dl[3] << 16));
    return;
  }
  const uint32_t head = s == 0 ? 4u : 4u - s;  // records before the first aligned chunk boundary
  auto single = [&](uint32_t r, uint32_t sv, uint32_t tv, float wv, int32_t dv) {
    const bool covered = r < head ? head_done : chunk;
    if (r < nvalid && !covered) store_one(blocks, log2B, p0 + r, sv, tv, wv, dv);
  };
  single(0, q.s[0], q.t[0], q.w[0], q.d[0]);
  single(1, q.s[1], q.t[1], q.w[1], q.d[1]);
  single(2, q.s[2], q.t[2], q.w[2], q.d[2]);
  single(3, q.s[3], q.t[3], q.w[3], q.d[3]);
  if (chunk) {
    const uint64_t pc = p0 + 4 - s;  // a multiple of 4: one block holds the chunk
    char* base = G(blocks)[pc >> log2B];
    const uint64_t o = pc & (B - 1);
    const Chunk4 cs = chunk_of(q.s, sn, s), ct = chunk_of(q.t, tn, s), cw = chunk_of(w, wn, s),
                 cd = chunk_of(dl, dn, s);
    st_u32x4(base + 4 * o, cs.v[0], cs.v[1], cs.v[2], cs.v[3]);
    st_u32x4(base + 4 * B + 4 * o, ct.v[0], ct.v[1], ct.v[2], ct.v[3]);
    st_u32x4(base + 8 * B + 4 * o, cw.v[0], cw.v[1], cw.v[2], cw.v[3]);
    st_u32x2(base + 12 * B + 2 * o, cd.v[0] | (cd.v[1] << 16), cd.v[2] | (cd.v[3] << 16));
  }
}

// Index arrays and per-connection values of synapses i0..i0+3 (those below
// n_new): generated positions become the nodes the arrays name.
__device__ __forceinline__ void apply_arrays(const GenDesc& d, uint32_t i0, Quad& q) {
  if (i0 + 3 < d.n_new && (((uintptr_t)d.w_arr | (uintptr_t)d.d_ms_arr) & 15) == 0) {
    // a whole quad and 16-byte aligned values: one vector load per array
    if (d.w_arr) {
      const u32x4 w4 = *(const NG_GLOBAL u32x4*)(const void*)(d.w_arr + i0);
      q.w[0] = __uint_as_float(w4.x);
      q.w[1] = __uint_as_float(w4.y);
      q.w[2] = __uint_as_float(w4.z);
      q.w[3] = __uint_as_float(w4.w);
    }
    if (d.d_ms_arr) {
      const u32x4 d4 = *(const NG_GLOBAL u32x4*)(const void*)(d.d_ms_arr + i0);
      q.d[0] = (int32_t)ms_to_steps(__uint_as_float(d4.x), d.h);
      q.d[1] = (int32_t)ms_to_steps(__uint_as_float(d4.y), d.h);
      q.d[2] = (int32_t)ms_to_steps(__uint_as_float(d4.z), d.h);
      q.d[3] = (int32_t)ms_to_steps(__uint_as_float(d4.w), d.h);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (d.src_idx) q.s[r] = G(d.src_idx)[q.s[r]];  // the generated value is a position < ns
      if (d.tgt_idx) q.t[r] = G(d.tgt_idx)[q.t[r]];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (i0 + r >= d.n_new) break;
    if (d.src_idx) q.s[r] = G(d.src_idx)[q.s[r]];
    if (d.tgt_idx) q.t[r] = G(d.tgt_idx)[q.t[r]];
    if (d.w_arr) q.w[r] = G(d.w_arr)[i0 + r];
    if (d.d_ms_arr) q.d[r] = (int32_t)ms_to_steps(G(d.d_ms_arr)[i0 + r], d.h);
  }
}


// ---------------------------------------------------------------------------
// Workgroup scan helpers (256 threads = 4 waves of 64)
// ---------------------------------------------------------------------------
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t n = __shfl_up(v, o, 64);
    if (lane >= o) v += n;
  }
  return v;
}

// Exclusive scan of one value per thread across the workgroup; returns the
// thread's exclusive prefix and sets *total.  s_tmp holds kWaves words.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_tmp[wave] = inc;
  __syncthreads();
  uint32_t wave_off = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t t = s_tmp[w];
    if (w < wave) wave_off += t;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return wave_off + inc - v;
}

// Barrier for LDS hand-offs only: global loads and stores stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace
}  // namespace ng
