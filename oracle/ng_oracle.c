/*
 * CPU oracle: plain, slow reference of connection generation and calibration.
 *
 * TEST INFRASTRUCTURE ONLY -- see ng_oracle.h.  Every function here follows a
 * passage of Golosio et al. (arXiv 2306.09855) or the frozen random-number
 * contract stated in ng_oracle.h; nothing is blocked, fused or reordered
 * beyond what those definitions state.  Build with -ffp-contract=off.
 */
#include "ng_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the timed mode (1 = the single-thread reference mode).  Each
 * synapse is a function of (seed, call, index) alone and the calibration
 * order is total, so every thread count gives the same bytes. */
static int g_threads = 1;

void ora_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int ora_get_threads(void) { return g_threads; }

/* ---------------------------------------------------------------------- */
/* Philox4x32-10, Salmon et al. SC'11: 10 rounds of the S-box built from    */
/* two 32x32->64 multiplications, with a Weyl sequence for the round keys. */
/* ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u /* golden ratio */
#define PHILOX_W1 0xBB67AE85u /* sqrt(3) - 1 */

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) { /* key schedule: bump before every round but the first */
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint32_t ora_word(uint64_t seed, uint32_t c, uint32_t s, uint64_t q) {
  uint64_t j = q >> 2;
  uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(j >> 32), c, s};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  ora_philox4x32_10(ctr, key, out);
  return out[q & 3];
}

/* The word streams of a call (stream numbers): every random quantity of
 * synapse i is word i of its own stream (pairwise_bernoulli: the decision
 * of pair q is word q of stream 0, and connection j takes the delay and
 * weight words of synapse j). */
#define ST_SRC 0u    /* source draws (fixed_indegree, fixed_total_number) */
#define ST_PAIR 0u   /* pairwise_bernoulli decisions */
#define ST_W 1u      /* weights */
#define ST_TGT 2u    /* target draws (fixed_outdegree, fixed_total_number) */
#define ST_DELAY 3u  /* delays */

/* rand(N) of Sec. 2.1: a uniform integer in [0, N); fixed-point product. */
uint32_t ora_rand_below(uint32_t x, uint32_t n) {
  return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

void ora_rand_below_batch(const uint32_t* x, uint64_t count, uint32_t n, uint32_t* out) {
  for (uint64_t k = 0; k < count; k++) out[k] = ora_rand_below(x[k], n);
}

/* 24-bit uniforms: u1 in (0,1], u2 in [0,1), both exact in fp32 and fp64 */
static double unit_open0(uint32_t y) { return ((double)(y >> 8) + 1.0) * (1.0 / 16777216.0); }
static double unit_open1(uint32_t y) { return (double)(y >> 8) * (1.0 / 16777216.0); }

/* Normal weights: Box-Muller on one pair of words, evaluated in fp64;
 * branch 0 is the cosine, branch 1 the sine (the two outputs are independent
 * standard normals). */
double ora_normal_weight2(uint32_t y0, uint32_t y1, int branch, double mean, double sd) {
  const double two_pi = 6.283185307179586476925286766559;
  double u1 = unit_open0(y0);
  double u2 = unit_open1(y1);
  double r = sqrt(-2.0 * log(u1));
  double z = branch ? r * sin(two_pi * u2) : r * cos(two_pi * u2);
  return mean + sd * z;
}

double ora_normal_weight(uint32_t y0, uint32_t y1, double mean, double sd) {
  return ora_normal_weight2(y0, y1, 0, mean, sd);
}

double ora_uniform_weight(uint32_t y0, double lo, double hi) {
  return lo + (hi - lo) * unit_open1(y0);
}

/* Sec. 2.1: a delay in ms becomes an integer number of steps by dividing by
 * the resolution and rounding; anything below one step becomes one step.
 * Rounding is to nearest, ties to even.  fp32 throughout. */
int32_t ora_delay_steps(float d_ms, float h) {
  float q = d_ms / h;
  float r = rintf(q);
  if (r < 1.0f) return 1;
  return (int32_t)r;
}

int32_t ora_uniform_ms_delay(uint32_t x, double lo, double hi, float h) {
  float u = (float)(x >> 8) * (1.0f / 16777216.0f);
  float d_ms = fmaf((float)(hi - lo), u, (float)lo);
  return ora_delay_steps(d_ms, h);
}

/* ---------------------------------------------------------------------- */
/* Connection rules, Sec. 2.1 Eqs. (4)-(13)                                */
/* ---------------------------------------------------------------------- */
/* number of nodes in both ranges */
static uint64_t overlap(const ora_call* c) {
  const uint64_t a = c->s0 > c->t0 ? c->s0 : c->t0;
  const uint64_t b0 = (uint64_t)c->s0 + c->ns, b1 = (uint64_t)c->t0 + c->nt;
  const uint64_t b = b0 < b1 ? b0 : b1;
  return b > a ? b - a : 0;
}

static int no_self(const ora_call* c) { return !c->allow_autapses && !c->src_idx && !c->tgt_idx; }

/* permutation of [0, m) for multapse-free draws: a 4-round Feistel network on
 * n bits (the smallest n >= 2 with 2^n >= m), walked until the value falls
 * below m.  x = L * 2^nb + R with R the low nb = n - floor(n/2) bits and L
 * the high na = floor(n/2) bits; rounds 0 and 2 set L ^= F_r(R) mod 2^na,
 * rounds 1 and 3 set R ^= F_r(L) mod 2^nb, F_r(v) = lowbias32(v ^ k_r) with
 * lowbias32 the integer hash of C. Wellons ("Prospecting for Hash
 * Functions", 2018) and k_0..k_3 the words of Philox(ctr = (u, 0, cid,
 * 131072)). */
uint32_t ora_lowbias32(uint32_t x);
static uint32_t lowbias32(uint32_t x) { return ora_lowbias32(x); }
uint32_t ora_lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

static uint64_t feistel(const uint32_t k[4], int na, int nb, uint64_t x) {
  const uint64_t mask_a = (1ull << na) - 1, mask_b = (1ull << nb) - 1;
  uint64_t left = x >> nb, right = x & mask_b;
  left ^= (uint64_t)lowbias32((uint32_t)right ^ k[0]) & mask_a;
  right ^= (uint64_t)lowbias32((uint32_t)left ^ k[1]) & mask_b;
  left ^= (uint64_t)lowbias32((uint32_t)right ^ k[2]) & mask_a;
  right ^= (uint64_t)lowbias32((uint32_t)left ^ k[3]) & mask_b;
  return (left << nb) | right;
}

/* The walk from x ends only for x < m (x's cycle then returns below m):
 * x >= m is a caller's error and gives -1. */
static int permute(uint64_t seed, uint32_t cid, uint32_t u, uint64_t m, uint64_t x, uint64_t* out) {
  if (x >= m) return -1;
  int n = 2;
  while (n < 64 && (1ull << n) < m) n++;
  const int na = n / 2, nb = n - na;
  uint32_t ctr[4] = {u, 0, cid, 131072u}, key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, k[4];
  ora_philox4x32_10(ctr, key, k);
  uint64_t y = feistel(k, na, nb, x);
  while (y >= m) y = feistel(k, na, nb, y);
  *out = y;
  return 0;
}

static int no_multi(const ora_call* c) { return !c->allow_multapses; }

/* pair index k in all_to_all order (without self-pairs when prohibited) */
static void a2a_pair(const ora_call* c, uint64_t k, uint64_t* s_off, uint64_t* t_off) {
  if (!no_self(c)) {
    *s_off = k / c->nt;
    *t_off = k % c->nt;
    return;
  }
  uint64_t rem = k, a = 0;
  for (;; a++) {
    const uint64_t s = c->s0 + a;
    const int in_t = s >= c->t0 && s < (uint64_t)c->t0 + c->nt;
    const uint64_t len = c->nt - (in_t ? 1 : 0);
    if (rem < len) {
      uint64_t t = rem;
      if (in_t && c->t0 + t >= s) t++;
      *s_off = a;
      *t_off = t;
      return;
    }
    rem -= len;
  }
}

/* pairwise_bernoulli: is pair (a, b) a connection */
static uint64_t pb_threshold(const ora_call* c) { return (uint64_t)floor(c->p * 4294967296.0); }
static int pb_pair(uint64_t seed, uint32_t cid, const ora_call* c, uint64_t a, uint64_t b) {
  if (no_self(c) && c->s0 + a == c->t0 + b) return 0;
  return (uint64_t)ora_word(seed, cid, ST_PAIR, a * c->nt + b) < pb_threshold(c);
}

int64_t ora_count(const ora_call* c) {
  if ((uint64_t)c->s0 + c->ns > 0xFFFFFFFFull || (uint64_t)c->t0 + c->nt > 0xFFFFFFFFull)
    return -1;
  if ((!c->allow_autapses || !c->allow_multapses) && (c->src_idx || c->tgt_idx)) return -1;
  const int ns_ = no_self(c);
  switch (c->rule) {
    case ORA_ONE_TO_ONE: /* N_new = N_sources = N_targets */
      if (c->ns != c->nt) return -1;
      if (ns_ && c->s0 == c->t0) return 0;  /* every pair would be an autapse */
      return (int64_t)c->ns;
    case ORA_ALL_TO_ALL: /* N_new = N_sources * N_targets (minus the pairs s == t) */
      return (int64_t)c->ns * (int64_t)c->nt - (ns_ ? (int64_t)overlap(c) : 0);
    case ORA_FIXED_OUTDEGREE: /* N_new = N_sources * K, random targets need N_t > 0 */
      if (c->nt == 0 && c->ns > 0 && c->k_or_n > 0) return -1;
      if (no_multi(c) && c->ns && c->k_or_n > (uint64_t)c->nt - (ns_ && overlap(c) ? 1 : 0)) return -1;
      if (ns_ && c->nt == 1 && overlap(c) && c->k_or_n > 0) return -1;  /* a source with no other target */
      return (int64_t)c->ns * (int64_t)c->k_or_n;
    case ORA_FIXED_INDEGREE: /* N_new = N_targets * K, random sources need N_s > 0 */
      if (c->ns == 0 && c->nt > 0 && c->k_or_n > 0) return -1;
      if (no_multi(c) && c->nt && c->k_or_n > (uint64_t)c->ns - (ns_ && overlap(c) ? 1 : 0)) return -1;
      if (ns_ && c->ns == 1 && overlap(c) && c->k_or_n > 0) return -1;  /* a target with no other source */
      return (int64_t)c->nt * (int64_t)c->k_or_n;
    case ORA_FIXED_TOTAL_NUMBER: /* N_new given */
      if ((c->ns == 0 || c->nt == 0) && c->k_or_n > 0) return -1;
      if (ns_ && (uint64_t)c->ns * c->nt == overlap(c) && c->k_or_n > 0) return -1;  /* only autapses */
      if (no_multi(c) && c->k_or_n > (uint64_t)c->ns * c->nt - (ns_ ? overlap(c) : 0)) return -1;
      return (int64_t)c->k_or_n;
    default:
      return -1;
  }
}

/* pairwise_bernoulli needs the seed and call id to count */
int64_t ora_count_pairwise(uint64_t seed, uint32_t cid, const ora_call* c) {
  if (c->rule != ORA_PAIRWISE_BERNOULLI) return ora_count(c);
  if (!(c->p >= 0.0 && c->p <= 1.0) || c->src_idx || c->tgt_idx) return -1;
  int64_t n = 0;
  for (uint64_t a = 0; a < c->ns; a++)
    for (uint64_t b = 0; b < c->nt; b++) n += pb_pair(seed, cid, c, a, b);
  return n;
}

/* pairwise_bernoulli, one row: the target offsets b of source offset a that
 * connect, ascending (out holds nt entries); returns their number or -1 */
int64_t ora_pairwise_row(uint64_t seed, uint32_t cid, const ora_call* c, uint32_t a, uint32_t* out) {
  if (c->rule != ORA_PAIRWISE_BERNOULLI || !(c->p >= 0.0 && c->p <= 1.0) || a >= c->ns) return -1;
  int64_t n = 0;
  for (uint64_t b = 0; b < c->nt; b++)
    if (pb_pair(seed, cid, c, a, b)) out[n++] = (uint32_t)b;
  return n;
}

static int delay_is_random(const ora_call* c) { return c->d_arr == NULL && c->d_kind != ORA_CONST; }

int ora_words_per_synapse(const ora_call* c) {
  int draws = 0;
  if (no_multi(c) && (c->rule == ORA_FIXED_INDEGREE || c->rule == ORA_FIXED_OUTDEGREE ||
                      c->rule == ORA_FIXED_TOTAL_NUMBER))
    return delay_is_random(c) ? 1 : 0; /* the permutation draws no source or target word */
  if (c->rule == ORA_FIXED_INDEGREE || c->rule == ORA_FIXED_TOTAL_NUMBER) draws++; /* source */
  if (c->rule == ORA_FIXED_OUTDEGREE || c->rule == ORA_FIXED_TOTAL_NUMBER) draws++; /* target */
  if (delay_is_random(c)) draws++;
  return draws;
}

static int weight_and_delay(uint64_t seed, float h, uint32_t cid, const ora_call* c, uint64_t i, double* w,
                            int32_t* delay);

int ora_synapse(uint64_t seed, float h, uint32_t cid, const ora_call* c, uint64_t i,
                uint32_t* src, uint32_t* tgt, double* w, int32_t* delay) {
  if (c->rule == ORA_PAIRWISE_BERNOULLI) {
    /* connection i is the i-th pair, in row order, that is a connection */
    uint64_t seen = 0;
    for (uint64_t a = 0; a < c->ns; a++)
      for (uint64_t b = 0; b < c->nt; b++)
        if (pb_pair(seed, cid, c, a, b) && seen++ == i) {
          *src = c->s0 + (uint32_t)a;
          *tgt = c->t0 + (uint32_t)b;
          return weight_and_delay(seed, h, cid, c, i, w, delay);
        }
    return -1;
  }
  uint64_t k = c->k_or_n;
  uint64_t s_off = 0, t_off = 0;
  if (no_multi(c) && c->rule == ORA_FIXED_INDEGREE) {
    t_off = i / k;
    const uint64_t t = c->t0 + t_off;
    const int in_s = no_self(c) && t >= c->s0 && t < (uint64_t)c->s0 + c->ns;
    if (permute(seed, cid, (uint32_t)t, c->ns - (in_s ? 1 : 0), i % k, &s_off)) return -1;
    if (in_s && s_off >= t - c->s0) s_off++;
    *src = c->s0 + (uint32_t)s_off;
    *tgt = (uint32_t)t;
    return weight_and_delay(seed, h, cid, c, i, w, delay);
  }
  if (no_multi(c) && c->rule == ORA_FIXED_OUTDEGREE) {
    s_off = i / k;
    const uint64_t s = c->s0 + s_off;
    const int in_t = no_self(c) && s >= c->t0 && s < (uint64_t)c->t0 + c->nt;
    if (permute(seed, cid, (uint32_t)s, c->nt - (in_t ? 1 : 0), i % k, &t_off)) return -1;
    if (in_t && t_off >= s - c->t0) t_off++;
    *src = (uint32_t)s;
    *tgt = c->t0 + (uint32_t)t_off;
    return weight_and_delay(seed, h, cid, c, i, w, delay);
  }
  if (no_multi(c) && c->rule == ORA_FIXED_TOTAL_NUMBER) {
    const uint64_t pairs = (uint64_t)c->ns * c->nt - (no_self(c) ? overlap(c) : 0);
    uint64_t pair;
    if (permute(seed, cid, 0, pairs, i, &pair)) return -1;
    a2a_pair(c, pair, &s_off, &t_off);
    *src = c->s0 + (uint32_t)s_off;
    *tgt = c->t0 + (uint32_t)t_off;
    return weight_and_delay(seed, h, cid, c, i, w, delay);
  }
  switch (c->rule) {
    case ORA_ONE_TO_ONE: /* Eqs. (4)-(5) */
      s_off = i;
      t_off = i;
      break;
    case ORA_ALL_TO_ALL: /* Eqs. (6)-(7) */
      if (!no_self(c)) {
        s_off = i / c->nt;
        t_off = i % c->nt;
      } else {
        /* walk the rows: row a has N_t targets, minus one if its source is a target */
        uint64_t rem = i, a = 0;
        for (;; a++) {
          const uint64_t s = c->s0 + a;
          const int in_t = s >= c->t0 && s < (uint64_t)c->t0 + c->nt;
          const uint64_t len = c->nt - (in_t ? 1 : 0);
          if (rem < len) {
            t_off = rem;
            if (in_t && c->t0 + t_off >= s) t_off++;  /* skip t == s */
            break;
          }
          rem -= len;
        }
        s_off = a;
      }
      break;
    case ORA_FIXED_OUTDEGREE: /* Eqs. (8)-(9) */
      s_off = i / k;
      {
        const uint64_t s = c->s0 + s_off;
        const int in_t = no_self(c) && s >= c->t0 && s < (uint64_t)c->t0 + c->nt;
        t_off = ora_rand_below(ora_word(seed, cid, ST_TGT, i), c->nt - (in_t ? 1 : 0));
        if (in_t && t_off >= s - c->t0) t_off++;
      }
      break;
    case ORA_FIXED_INDEGREE: /* Eqs. (10)-(11) */
      t_off = i / k;
      {
        const uint64_t t = c->t0 + t_off;
        const int in_s = no_self(c) && t >= c->s0 && t < (uint64_t)c->s0 + c->ns;
        s_off = ora_rand_below(ora_word(seed, cid, ST_SRC, i), c->ns - (in_s ? 1 : 0));
        if (in_s && s_off >= t - c->s0) s_off++;
      }
      break;
    case ORA_FIXED_TOTAL_NUMBER: /* Eqs. (12)-(13): a source draw and a target draw */
      s_off = ora_rand_below(ora_word(seed, cid, ST_SRC, i), c->ns);
      t_off = ora_rand_below(ora_word(seed, cid, ST_TGT, i), c->nt);
      if (no_self(c)) {
        for (uint32_t a = 1; c->s0 + s_off == c->t0 + t_off; a++) {
          const uint32_t st = 65536u + (a <= 64 ? a : 64);
          s_off = ora_rand_below(ora_word(seed, cid, st, 2 * i), c->ns);
          if (a < 64) {
            t_off = ora_rand_below(ora_word(seed, cid, st, 2 * i + 1), c->nt);
          } else {  /* last attempt: a target other than the source */
            const uint64_t s = c->s0 + s_off;
            const int in_t = s >= c->t0 && s < (uint64_t)c->t0 + c->nt;
            t_off = ora_rand_below(ora_word(seed, cid, st, 2 * i + 1), c->nt - (in_t ? 1 : 0));
            if (in_t && t_off >= s - c->t0) t_off++;
            break;
          }
        }
      }
      break;
    default:
      return -1;
  }
  /* explicit node arrays: the formulas give the array position */
  *src = c->src_idx ? c->src_idx[s_off] : c->s0 + (uint32_t)s_off;
  *tgt = c->tgt_idx ? c->tgt_idx[t_off] : c->t0 + (uint32_t)t_off;
  return weight_and_delay(seed, h, cid, c, i, w, delay);
}

/* delay of synapse i from word i of the delay stream (if random); a random
 * weight from the weight stream: normal weights of synapses 2j and 2j+1 are
 * the cosine and sine outputs of the Box-Muller pair on words 2j, 2j+1; a
 * uniform weight takes word i */
static int weight_and_delay(uint64_t seed, float h, uint32_t cid, const ora_call* c, uint64_t i, double* w,
                            int32_t* delay) {
  if (c->d_arr) {
    *delay = ora_delay_steps(c->d_arr[i], h);
  } else switch (c->d_kind) {
    case ORA_CONST:
      *delay = ora_delay_steps((float)c->d_a, h);
      break;
    case ORA_UNIFORM_INT: { /* integer steps lo..hi */
      uint32_t lo = (uint32_t)c->d_a, hi = (uint32_t)c->d_b;
      *delay = (int32_t)(lo + ora_rand_below(ora_word(seed, cid, ST_DELAY, i), hi - lo + 1));
      break;
    }
    case ORA_UNIFORM:
      *delay = ora_uniform_ms_delay(ora_word(seed, cid, ST_DELAY, i), c->d_a, c->d_b, h);
      break;
    default:
      return -1;
  }

  if (c->w_arr) {
    *w = (double)c->w_arr[i];
    return 0;
  }
  switch (c->w_kind) {
    case ORA_CONST:
      *w = c->w_a;
      break;
    case ORA_NORMAL: {
      const uint64_t j = i >> 1;
      *w = ora_normal_weight2(ora_word(seed, cid, ST_W, 2 * j), ora_word(seed, cid, ST_W, 2 * j + 1), (int)(i & 1),
                              c->w_a, c->w_b);
      break;
    }
    case ORA_UNIFORM:
      *w = ora_uniform_weight(ora_word(seed, cid, ST_W, i), c->w_a, c->w_b);
      break;
    default:
      return -1;
  }
  return 0;
}

/* pairwise_bernoulli: weight and delay of connection j (they depend on j
 * only: as synapse j of any call, delay word j of the delay stream, weight
 * from the weight stream) */
int ora_pairwise_values(uint64_t seed, float h, uint32_t cid, const ora_call* c, uint64_t j, double* w,
                        int32_t* delay) {
  if (c->rule != ORA_PAIRWISE_BERNOULLI) return -1;
  return weight_and_delay(seed, h, cid, c, j, w, delay);
}

int ora_connect(uint64_t seed, float h, uint32_t cid, const ora_call* c, uint32_t* src,
                uint32_t* tgt, double* w, int32_t* delay) {
  if (c->rule == ORA_PAIRWISE_BERNOULLI) {  /* one walk over the pairs */
    if (!(c->p >= 0.0 && c->p <= 1.0) || c->src_idx || c->tgt_idx) return -1;
    uint64_t j = 0;
    for (uint64_t a = 0; a < c->ns; a++)
      for (uint64_t b = 0; b < c->nt; b++)
        if (pb_pair(seed, cid, c, a, b)) {
          src[j] = c->s0 + (uint32_t)a;
          tgt[j] = c->t0 + (uint32_t)b;
          if (weight_and_delay(seed, h, cid, c, j, &w[j], &delay[j])) return -1;
          j++;
        }
    return 0;
  }
  int64_t n = ora_count(c);
  if (n < 0) return -1;
  int bad = 0;
#pragma omp parallel for num_threads(g_threads) schedule(static) reduction(| : bad) if (g_threads > 1)
  for (int64_t i = 0; i < n; i++)
    if (ora_synapse(seed, h, cid, c, (uint64_t)i, &src[i], &tgt[i], &w[i], &delay[i]) != 0) bad = 1;
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Calibration, Sec. 2.2                                                    */
/* ---------------------------------------------------------------------- */
typedef struct {
  uint32_t src;
  int32_t delay;
  uint64_t idx;
} sort_item;

/* Source is the first key and delay the second; the creation index breaks
 * ties, so the order is total and equals a stable sort by (source, delay). */
static int cmp_item(const void* a, const void* b) {
  const sort_item* x = (const sort_item*)a;
  const sort_item* y = (const sort_item*)b;
  if (x->src != y->src) return x->src < y->src ? -1 : 1;
  if (x->delay != y->delay) return x->delay < y->delay ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

/* bucket of x among the sorted splitters: how many of them precede x */
static uint32_t bucket_of(const sort_item* spl, uint32_t nspl, const sort_item* x) {
  uint32_t lo = 0, hi = nspl;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (cmp_item(&spl[mid], x) < 0) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* Sorts *items by the total order of cmp_item.  One thread: qsort.  Timed
 * mode: a sample sort -- splitters from a regular sample, every thread counts
 * and then moves its share of the items into the buckets, each bucket is
 * sorted with qsort.  Both give the one sorted sequence (the order is
 * total).  *items may be replaced by a new array.  Returns 0 or -1. */
static int sort_items(sort_item** pitems, uint64_t n) {
  sort_item* items = *pitems;
  const int T = g_threads;
  if (T <= 1 || n < (1u << 16)) {
    qsort(items, n, sizeof(sort_item), cmp_item);
    return 0;
  }
  const uint32_t nb = 8u * (uint32_t)T, nspl = nb - 1, ns = 64u * nb;
  sort_item* sample = (sort_item*)malloc(ns * sizeof(sort_item));
  sort_item* out = (sort_item*)malloc(n * sizeof(sort_item));
  uint64_t* counts = (uint64_t*)calloc((size_t)T * nb, sizeof(uint64_t));
  uint64_t* bstart = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
  if (!sample || !out || !counts || !bstart) {
    free(sample);
    free(out);
    free(counts);
    free(bstart);
    return -1;
  }
  for (uint32_t k = 0; k < ns; k++) sample[k] = items[(uint64_t)k * n / ns];
  qsort(sample, ns, sizeof(sort_item), cmp_item);
  sort_item* spl = (sort_item*)malloc(nspl * sizeof(sort_item));
  if (!spl) {
    free(sample);
    free(out);
    free(counts);
    free(bstart);
    return -1;
  }
  for (uint32_t b = 0; b < nspl; b++) spl[b] = sample[(uint64_t)(b + 1) * ns / nb];
  free(sample);
#pragma omp parallel num_threads(T)
  {
#ifdef _OPENMP
    const int t = omp_get_thread_num();
#else
    const int t = 0;
#endif
    const uint64_t lo = (uint64_t)t * n / T, hi = (uint64_t)(t + 1) * n / T;
    uint64_t* cnt = counts + (size_t)t * nb;
    for (uint64_t j = lo; j < hi; j++) cnt[bucket_of(spl, nspl, &items[j])]++;
#pragma omp barrier
#pragma omp single
    {
      uint64_t acc = 0;
      for (uint32_t b = 0; b < nb; b++) {
        bstart[b] = acc;
        for (int u = 0; u < T; u++) {
          const uint64_t c = counts[(size_t)u * nb + b];
          counts[(size_t)u * nb + b] = acc;
          acc += c;
        }
      }
      bstart[nb] = acc;
    }
    for (uint64_t j = lo; j < hi; j++) out[cnt[bucket_of(spl, nspl, &items[j])]++] = items[j];
#pragma omp barrier
#pragma omp for schedule(dynamic, 1)
    for (uint32_t b = 0; b < nb; b++)
      qsort(out + bstart[b], bstart[b + 1] - bstart[b], sizeof(sort_item), cmp_item);
  }
  free(spl);
  free(counts);
  free(bstart);
  free(items);
  *pitems = out;
  return 0;
}

int ora_calibrate(uint64_t n, uint32_t n_nodes, const uint32_t* src, const int32_t* delay,
                  uint64_t* perm, uint32_t* group_ptr, uint32_t* group_start,
                  uint64_t* n_groups) {
  for (uint64_t j = 0; j < n; j++)
    if (src[j] >= n_nodes) return -1;

  sort_item* items = (sort_item*)malloc((n ? n : 1) * sizeof(sort_item));
  if (!items) return -1;
  for (uint64_t j = 0; j < n; j++) {
    items[j].src = src[j];
    items[j].delay = delay[j];
    items[j].idx = j;
  }
  if (sort_items(&items, n) != 0) {
    free(items);
    return -1;
  }
  for (uint64_t j = 0; j < n; j++) perm[j] = items[j].idx;

  /* A connection starts a group when its source or its delay differs from
   * those of the previous connection.  Count groups per source (G_i) and
   * record the position of each group's first connection. */
  uint64_t* g_count = (uint64_t*)calloc((size_t)n_nodes + 1, sizeof(uint64_t));
  if (!g_count) {
    free(items);
    return -1;
  }
  uint64_t g = 0;
  for (uint64_t j = 0; j < n; j++) {
    int first = (j == 0) || items[j].src != items[j - 1].src ||
                items[j].delay != items[j - 1].delay;
    if (first) {
      group_start[g] = (uint32_t)j;
      g_count[items[j].src]++;
      g++;
    }
  }
  group_start[g] = (uint32_t)n;
  *n_groups = g;

  /* Eq. (14): p_i = sum_{j<i} G_j, p_0 = 0, for i = 0..n_nodes */
  uint64_t acc = 0;
  for (uint32_t i = 0; i <= n_nodes; i++) {
    group_ptr[i] = (uint32_t)acc;
    if (i < n_nodes) acc += g_count[i];
  }
  free(g_count);
  free(items);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* COPASS (Appendix A).                                                     */

/* number of elements of the sorted range a[lo..hi) that are <= t (le = 1) or
 * < t (le = 0), plus lo: the counts of the paper restricted to a bracket
 * that already holds the answer */
static uint64_t count_upto(const uint64_t* a, uint64_t lo, uint64_t hi, uint64_t t, int le) {
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (le ? a[mid] <= t : a[mid] < t) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

typedef struct {
  uint64_t v;
  uint32_t i;
} copass_cand;

static int cmp_cand(const void* a, const void* b) {
  const copass_cand* x = (const copass_cand*)a;
  const copass_cand* y = (const copass_cand*)b;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  if (x->i != y->i) return x->i < y->i ? -1 : 1;
  return 0;
}

int ora_copass_partition(uint32_t k, const uint64_t* vals, const uint64_t* off, uint64_t m,
                         uint64_t* m_out, uint64_t* iterations) {
  if (iterations) *iterations = 0;
  uint64_t total = 0;
  for (uint32_t i = 0; i < k; i++) {
    if (off[i + 1] < off[i]) return -1;
    total += off[i + 1] - off[i];
  }
  if (m > total) return -1;
  if (m == 0 || m == total) {
    for (uint32_t i = 0; i < k; i++) m_out[i] = m == 0 ? 0 : off[i + 1] - off[i];
    return 0;
  }
  /* bracket [ubar_m_i, bar_m_i] per subarray: ubar_m counts elements <= the
   * lower threshold, bar_m those < the upper one; initially the thresholds
   * lie below the minimum and above the maximum, so the brackets are [0, N_i] */
  uint64_t* lo = (uint64_t*)malloc((k ? k : 1) * sizeof(uint64_t));
  uint64_t* hi = (uint64_t*)malloc((k ? k : 1) * sizeof(uint64_t));
  uint64_t* mu_lo = (uint64_t*)malloc((k ? k : 1) * sizeof(uint64_t));
  uint64_t* mu_hi = (uint64_t*)malloc((k ? k : 1) * sizeof(uint64_t));
  if (!lo || !hi || !mu_lo || !mu_hi) {
    free(lo); free(hi); free(mu_lo); free(mu_hi);
    return -1;
  }
  for (uint32_t i = 0; i < k; i++) {
    lo[i] = 0;
    hi[i] = off[i + 1] - off[i];
  }
  int result = -1;
  uint64_t iter = 0;
  for (;;) {
    /* the widest bracket; stop when every bracket has width <= 1 */
    uint32_t l = 0;
    for (uint32_t i = 1; i < k; i++)
      if (hi[i] - lo[i] > hi[l] - lo[l]) l = i;
    if (hi[l] - lo[l] <= 1) break;
    iter++;
    /* trial threshold: the middle element of that bracket */
    const uint64_t mt = (lo[l] + hi[l]) / 2;
    const uint64_t t = vals[off[l] + mt];
    uint64_t s_lo = 0, s_hi = 0;
    for (uint32_t i = 0; i < k; i++) {
      const uint64_t* a = vals + off[i];
      mu_hi[i] = count_upto(a, lo[i], hi[i], t, 1);  /* #{S_ij <= t} */
      mu_lo[i] = count_upto(a, lo[i], mu_hi[i], t, 0);  /* #{S_ij < t} */
      s_lo += mu_lo[i];
      s_hi += mu_hi[i];
    }
    if (s_lo <= m && m <= s_hi) {
      /* t is the threshold: the elements equal to t, [mu_lo_i, mu_hi_i) in
       * each subarray, fill the remaining d = m - sum mu_lo, subarray by
       * subarray in ascending i */
      uint64_t d = m - s_lo;
      for (uint32_t i = 0; i < k; i++) {
        const uint64_t take = d < mu_hi[i] - mu_lo[i] ? d : mu_hi[i] - mu_lo[i];
        m_out[i] = mu_lo[i] + take;
        d -= take;
      }
      result = 1;
      break;
    }
    if (m < s_lo) {
      for (uint32_t i = 0; i < k; i++) hi[i] = mu_lo[i];  /* upper threshold := t */
    } else {
      for (uint32_t i = 0; i < k; i++) lo[i] = mu_hi[i];  /* lower threshold := t */
    }
  }
  if (result < 0) {
    /* every bracket has width <= 1: the subarrays with width one offer their
     * element ubar_m_i; the d = m - sum ubar_m smallest offers, ordered by
     * (value, i), go to the left partitions */
    copass_cand* c = (copass_cand*)malloc((k ? k : 1) * sizeof(copass_cand));
    if (c) {
      uint32_t nc = 0;
      uint64_t s = 0;
      for (uint32_t i = 0; i < k; i++) {
        s += lo[i];
        m_out[i] = lo[i];
        if (hi[i] == lo[i] + 1) {
          c[nc].v = vals[off[i] + lo[i]];
          c[nc].i = i;
          nc++;
        }
      }
      qsort(c, nc, sizeof(copass_cand), cmp_cand);
      const uint64_t d = m - s;
      for (uint64_t j = 0; j < d && j < nc; j++) m_out[c[j].i] += 1;
      free(c);
      result = 2;
    }
  }
  if (iterations) *iterations = iter;
  free(lo); free(hi); free(mu_lo); free(mu_hi);
  return result;
}

typedef struct {
  uint64_t v, p;
  uint64_t pos;
} copass_item;

static int cmp_copass_item(const void* a, const void* b) {
  const copass_item* x = (const copass_item*)a;
  const copass_item* y = (const copass_item*)b;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
  return 0;
}

/* the underlying sort: stable, by value, of vals/pay[a..a+len) */
static int stable_sort_range(uint64_t* vals, uint64_t* pay, uint64_t a, uint64_t len) {
  copass_item* it = (copass_item*)malloc((len ? len : 1) * sizeof(copass_item));
  if (!it) return -1;
  for (uint64_t j = 0; j < len; j++) {
    it[j].v = vals[a + j];
    it[j].p = pay[a + j];
    it[j].pos = j;
  }
  qsort(it, len, sizeof(copass_item), cmp_copass_item);
  for (uint64_t j = 0; j < len; j++) {
    vals[a + j] = it[j].v;
    pay[a + j] = it[j].p;
  }
  free(it);
  return 0;
}

int ora_copass_block_sort(uint64_t n, uint64_t B, uint64_t* vals, uint64_t* pay) {
  if (B == 0) return -1;
  const uint64_t nb = (n + B - 1) / B;
  if (nb > 0xFFFFFFFFull) return -1;
  const uint32_t k = (uint32_t)nb;
  if (k == 0) return 0;
  /* (B) every block sorted */
  for (uint32_t i = 0; i < k; i++) {
    const uint64_t a = (uint64_t)i * B, len = a + B <= n ? B : n - a;
    if (stable_sort_range(vals, pay, a, len)) return -1;
  }
  /* subarray i occupies [start_i, start_i + len_i) of the remaining region */
  uint64_t* start = (uint64_t*)malloc(k * sizeof(uint64_t));
  uint64_t* len = (uint64_t*)malloc(k * sizeof(uint64_t));
  uint64_t* off = (uint64_t*)malloc((k + 1) * sizeof(uint64_t));
  uint64_t* mi = (uint64_t*)malloc(k * sizeof(uint64_t));
  uint64_t* aux_v = (uint64_t*)malloc(B * sizeof(uint64_t));
  uint64_t* aux_p = (uint64_t*)malloc(B * sizeof(uint64_t));
  uint64_t* sub = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  int rc = (start && len && off && mi && aux_v && aux_p && sub) ? 0 : -1;
  for (uint32_t i = 0; i < k && rc == 0; i++) {
    start[i] = (uint64_t)i * B;
    len[i] = start[i] + B <= n ? B : n - start[i];
  }
  for (uint32_t b = 0; b < k && rc == 0; b++) {
    const uint64_t first = (uint64_t)b * B, m = first + B <= n ? B : n - first;
    /* the partition reads the subarrays as one concatenated sorted list each */
    off[0] = 0;
    for (uint32_t i = 0; i < k; i++) {
      memcpy(sub + off[i], vals + start[i], len[i] * sizeof(uint64_t));
      off[i + 1] = off[i] + len[i];
    }
    if (ora_copass_partition(k, sub, off, m, mi, NULL) < 0) {
      rc = -1;
      break;
    }
    /* (D) left partitions, in subarray order, to the auxiliary array */
    uint64_t q = 0;
    for (uint32_t i = 0; i < k; i++) {
      memcpy(aux_v + q, vals + start[i], mi[i] * sizeof(uint64_t));
      memcpy(aux_p + q, pay + start[i], mi[i] * sizeof(uint64_t));
      q += mi[i];
    }
    /* (E) right partitions shifted to the end of the array, last first, so
     * that block b is free; then the auxiliary array goes to block b */
    uint64_t end = n;
    for (uint32_t i = k; i-- > 0;) {
      const uint64_t r = len[i] - mi[i];
      memmove(vals + end - r, vals + start[i] + mi[i], r * sizeof(uint64_t));
      memmove(pay + end - r, pay + start[i] + mi[i], r * sizeof(uint64_t));
      end -= r;
      start[i] = end;
      len[i] = r;
    }
    memcpy(vals + first, aux_v, m * sizeof(uint64_t));
    memcpy(pay + first, aux_p, m * sizeof(uint64_t));
    /* (F) block b sorted */
    if (stable_sort_range(vals, pay, first, m)) rc = -1;
  }
  free(start); free(len); free(off); free(mi); free(aux_v); free(aux_p); free(sub);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Spike buffer and delivery (Sec. 2.3).                                    */

typedef struct {
  uint32_t time, group, mult;
} ora_spike;

int ora_deliver(uint32_t n_nodes, const uint32_t* group_ptr, const uint32_t* group_start,
                const uint32_t* tgt, const double* w, const int32_t* delay, uint32_t n_steps,
                const uint64_t* spk_off, const uint32_t* spk_node, const uint32_t* spk_mult, double* input) {
  /* a queue per node; a spike stays at most (largest delay) steps, plus the
   * step it was emitted in */
  int32_t dmax = 1;
  const uint64_t n_groups = group_ptr[n_nodes];
  for (uint64_t g = 0; g < n_groups; g++)
    if (delay[group_start[g]] > dmax) dmax = delay[group_start[g]];
  const uint64_t cap = (uint64_t)dmax + 1;
  ora_spike* q = (ora_spike*)malloc((n_nodes ? n_nodes : 1) * cap * sizeof(ora_spike));
  uint64_t* head = (uint64_t*)calloc(n_nodes ? n_nodes : 1, sizeof(uint64_t));
  uint64_t* cnt = (uint64_t*)calloc(n_nodes ? n_nodes : 1, sizeof(uint64_t));
  if (!q || !head || !cnt) {
    free(q); free(head); free(cnt);
    return -1;
  }
  int rc = 0;
  for (uint32_t s = 0; s < n_steps && rc == 0; s++) {
    double* in = input + (uint64_t)s * n_nodes;
    for (uint32_t t = 0; t < n_nodes; t++) in[t] = 0.0;
    /* the spike array of this step, delivered as it is filled */
    for (uint32_t i = 0; i < n_nodes; i++) {
      for (uint64_t e = 0; e < cnt[i]; e++) {
        ora_spike* sp = &q[(uint64_t)i * cap + (head[i] + e) % cap];
        sp->time += 1;
        const uint64_t g = group_ptr[i] + sp->group;
        if ((int32_t)sp->time == delay[group_start[g]]) {
          for (uint64_t j = group_start[g]; j < group_start[g + 1]; j++) in[tgt[j]] += w[j] * sp->mult;
          sp->group += 1;
        }
      }
      /* spikes past the node's last group leave from the front (they are the oldest) */
      while (cnt[i] > 0 && q[(uint64_t)i * cap + head[i]].group == group_ptr[i + 1] - group_ptr[i]) {
        head[i] = (head[i] + 1) % cap;
        cnt[i]--;
      }
    }
    /* spikes emitted this step */
    for (uint64_t e = spk_off[s]; e < spk_off[s + 1]; e++) {
      const uint32_t i = spk_node[e];
      if (i >= n_nodes || cnt[i] >= cap) {
        rc = -1;
        break;
      }
      if (group_ptr[i + 1] == group_ptr[i]) continue;  /* no outgoing connections */
      ora_spike* sp = &q[(uint64_t)i * cap + (head[i] + cnt[i]) % cap];
      sp->time = 0;
      sp->group = 0;
      sp->mult = spk_mult[e];
      cnt[i]++;
    }
  }
  free(q); free(head); free(cnt);
  return rc;
}
