/*
 * CPU oracle for rule-based connection generation and calibration.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent, plain and slow
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or constant with the GPU library, and the GPU library
 * never loads it.
 *
 * What it computes (Golosio et al., "Runtime Construction of Large-Scale
 * Spiking Neuronal Network Models on GPU Devices"):
 *   - node groups as consecutive index ranges (Sec. 2.1),
 *   - the five connection rules, Eqs. (4)-(13) of Sec. 2.1,
 *   - weights and delays: constant or drawn from a distribution, delays
 *     converted from ms to integer time steps with a minimum of one step
 *     (Sec. 2.1, last paragraph),
 *   - calibration: ordering by source (first key) and delay (second key),
 *     connection-group boundaries, group counts G_i and their cumulative sum
 *     p_i of Eq. (14) (Sec. 2.2),
 *   - the COPASS block sort and its partition of sorted subarrays
 *     (Appendix A), which sorts the block array in place.
 *
 * The random draws follow one frozen contract (the paper uses an unspecified
 * cuRAND generator and states that a change of generator preserves the
 * connectivity only statistically, Sec. 2.7):
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = seed split in two
 *   32-bit halves, word stream W_{c,s}[q] = Philox(ctr = (q/4 low, q/4 high,
 *   c, s))[q mod 4] for connect call c and stream s.  Synapse i takes word i
 *   of stream 0 for a source draw, of stream 2 for a target draw, of stream 3
 *   for its delay; its weight comes from stream 1 (two normal weights per
 *   pair of words, or word i for a uniform weight).  So the draws of any one
 *   kind can be evaluated without the others.
 *
 * Floating point: weights are evaluated in double precision (fp64).  The
 * ms-to-step delay conversion decides an integer, so it is evaluated in fp32,
 * the precision the GPU path uses for the same decision.
 */
#ifndef NG_ORACLE_H
#define NG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_ONE_TO_ONE = 0, ORA_ALL_TO_ALL = 1, ORA_FIXED_INDEGREE = 2,
       ORA_FIXED_OUTDEGREE = 3, ORA_FIXED_TOTAL_NUMBER = 4, ORA_PAIRWISE_BERNOULLI = 5 };

/* distribution kinds of a weight or delay specification */
enum { ORA_CONST = 0, ORA_NORMAL = 1, ORA_UNIFORM_INT = 2, ORA_UNIFORM = 3 };

typedef struct {
  int32_t rule;
  uint32_t s0, ns;      /* source range [s0, s0+ns) */
  uint32_t t0, nt;      /* target range [t0, t0+nt) */
  uint64_t k_or_n;      /* K for in/out-degree, total for fixed_total_number */
  int32_t w_kind;  double w_a, w_b;   /* CONST a | NORMAL(mean a, sd b) | UNIFORM [a,b) */
  int32_t d_kind;  double d_a, d_b;   /* CONST a ms | UNIFORM_INT {a..b} steps | UNIFORM [a,b) ms */
  /* Sec. 2.1, last paragraphs: node groups given as arrays, and weights or
   * delays given per connection.  NULL = not used.  With src_idx the rule's
   * source formula (taken with s0 = 0) gives the position in src_idx of the
   * source node (ns = array length); likewise tgt_idx.  w_arr[i] is the
   * weight of synapse i of the call; d_arr[i] its delay in ms, converted to
   * steps like a constant delay.  A delay given by an array is not random. */
  const uint32_t* src_idx;
  const uint32_t* tgt_idx;
  const float* w_arr;
  const float* d_arr;
  /* 0: no connection from a node to itself (Discussion: a flag the paper
   * names as future work).  Ranges only.  Definitions:
   *   one_to_one       the pairs with s != t (none if s0 == t0);
   *   all_to_all       the pairs with s != t, row by row (row s has N_t or
   *                    N_t - 1 targets), targets ascending;
   *   fixed_indegree   a target inside the source range draws from the other
   *                    N_s - 1 sources: r = rand(N_s - 1) from its usual word,
   *                    then r + 1 if r >= the target's position in the range;
   *   fixed_outdegree  the same with sources and targets exchanged;
   *   fixed_total_number  attempt 0 draws (s, t) from the usual words; while
   *                    s == t, attempt a >= 1 draws both from words 2i, 2i+1
   *                    of stream 65536 + a; after 64 attempts the target is
   *                    drawn from the other N_t - 1 targets as for
   *                    fixed_outdegree, from attempt 64's target word. */
  int32_t allow_autapses;
  /* pairwise_bernoulli (named as missing in the Discussion): every pair
   * (s, t), rows of sources in order, targets ascending, is a connection
   * when word (a * N_t + b) of stream 0 is below floor(p * 2^32) (a, b: the
   * positions of s and t; self-pairs never with allow_autapses = 0); the
   * connections are numbered in that order; connection j draws its delay
   * and weight as synapse j of any call would (word j of stream 3, stream 1). */
  double p;
  /* 0: no two connections join the same pair (sampling without
   * replacement; Discussion: future work).  Defined with a pseudorandom
   * permutation pi_u of [0, M): a 4-round Feistel network on n bits, the
   * smallest n >= 2 with 2^n >= M, walked until the value falls below M; the
   * value is L * 2^nb + R (R the low nb = n - floor(n/2) bits), rounds 0 and
   * 2 set L ^= lowbias32(R ^ k_r) mod 2^(n - nb), rounds 1 and 3 set
   * R ^= lowbias32(L ^ k_r) mod 2^nb, with k_0..k_3 the words of
   * Philox(ctr = (u, 0, c, 131072)) and lowbias32 the integer hash of
   * C. Wellons (2018).
   * fixed_indegree: target t gets the sources
   * at positions pi_t(0..K-1) of its candidates (the source range, or the
   * range without t, skip-self as above); fixed_outdegree likewise;
   * fixed_total_number: synapse i is the pair of index pi_0(i) in the
   * all_to_all order (without the self-pairs when those are prohibited).
   * The permutation draws no source or target word; synapse i's delay is
   * word i of the delay stream as for any rule. */
  int32_t allow_multapses;
} ora_call;

/* Threads of the generation and calibration loops.  1 (the default) is the
 * single-thread reference mode; n > 1 is the timed mode (OpenMP over
 * synapse indices, a sample sort for calibration), which gives the same
 * bytes. */
void ora_set_threads(int n);
int ora_get_threads(void);

/* the 32-bit integer hash "lowbias32" of C. Wellons (2018), used by the
 * permutation of the multapse-free draws */
uint32_t ora_lowbias32(uint32_t x);

/* Philox4x32-10 block function */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* word q of stream s of connect call c */
uint32_t ora_word(uint64_t seed, uint32_t c, uint32_t s, uint64_t q);
/* rand(n): uniform integer in [0, n) from one 32-bit word, floor(x*n / 2^32) */
uint32_t ora_rand_below(uint32_t x, uint32_t n);
void ora_rand_below_batch(const uint32_t* x, uint64_t count, uint32_t n, uint32_t* out);
/* weight transforms from stream-1 words */
double ora_normal_weight(uint32_t y0, uint32_t y1, double mean, double sd);
/* branch 0: cosine output (ora_normal_weight), 1: sine output */
double ora_normal_weight2(uint32_t y0, uint32_t y1, int branch, double mean, double sd);
double ora_uniform_weight(uint32_t y0, double lo, double hi);
/* delay in ms -> integer steps (fp32), minimum one step */
int32_t ora_delay_steps(float d_ms, float h);
/* uniform ms delay from one delay word, then to steps */
int32_t ora_uniform_ms_delay(uint32_t x, double lo, double hi, float h);

/* number of connections a call creates, or -1 if the call is invalid */
int64_t ora_count(const ora_call* call);
/* count of any rule; pairwise_bernoulli's depends on the seed and call id */
int64_t ora_count_pairwise(uint64_t seed, uint32_t connect_id, const ora_call* call);
/* pairwise_bernoulli, sampled checks of large calls: the connecting target
 * offsets of source offset a, ascending, into out (nt entries; returns their
 * number, -1 on a bad call), and the weight and delay of connection j */
int64_t ora_pairwise_row(uint64_t seed, uint32_t connect_id, const ora_call* call, uint32_t a, uint32_t* out);
int ora_pairwise_values(uint64_t seed, float h, uint32_t connect_id, const ora_call* call, uint64_t j,
                        double* w, int32_t* delay);
/* random source, target and delay draws of one synapse (one word each, of
 * their own streams) */
int ora_words_per_synapse(const ora_call* call);

/* synapse i of connect call `connect_id` */
int ora_synapse(uint64_t seed, float h, uint32_t connect_id, const ora_call* call,
                uint64_t i, uint32_t* src, uint32_t* tgt, double* w, int32_t* delay);
/* all synapses of one call, in creation order; returns 0 or -1 */
int ora_connect(uint64_t seed, float h, uint32_t connect_id, const ora_call* call,
                uint32_t* src, uint32_t* tgt, double* w, int32_t* delay);

/* Calibration of n connections held in creation order.
 * perm[j]        = creation index of the connection at sorted position j
 * group_ptr[i]   = p_i of Eq. (14), i = 0..n_nodes (n_nodes+1 entries)
 * group_start[g] = sorted position of the first connection of group g,
 *                  g = 0..G, with group_start[G] = n (capacity n+1)
 * *n_groups      = G
 * Returns 0, or -1 if a source index is >= n_nodes. */
int ora_calibrate(uint64_t n, uint32_t n_nodes, const uint32_t* src, const int32_t* delay,
                  uint64_t* perm, uint32_t* group_ptr, uint32_t* group_start,
                  uint64_t* n_groups);

/* Spike buffer and delivery (Sec. 2.3): the consumer of the calibrated
 * arrays.  Each node keeps a queue of spikes (time index, connection-group
 * index, multiplicity).  At each step every queued spike's time index grows
 * by one; a spike whose time index equals the delay of its current group is
 * put in the spike array and moves on to the node's next group (groups of a
 * node are in ascending delay), and leaves the queue after the last group;
 * then the spikes the nodes emit this step join their queues with time and
 * group index zero.  Every connection of every group in the spike array
 * adds weight x multiplicity to its target's input of this step.
 * Inputs: the calibrated arrays (tgt, w, delay in sorted order), group_ptr
 * (n_nodes + 1) and group_start (G + 1) as ora_calibrate gives them; steps
 * of spikes: spikes of step s are spk_node[spk_off[s] .. spk_off[s+1]) with
 * multiplicities spk_mult[...] (a node at most once per step).  Output:
 * input[s * n_nodes + t] (fp64) for s < n_steps.  Returns 0 or -1. */
int ora_deliver(uint32_t n_nodes, const uint32_t* group_ptr, const uint32_t* group_start,
                const uint32_t* tgt, const double* w, const int32_t* delay, uint32_t n_steps,
                const uint64_t* spk_off, const uint32_t* spk_node, const uint32_t* spk_mult, double* input);

/* COPASS partition (Appendix A, "The COPASS partition algorithm" and its two
 * last steps).  k subarrays, each sorted ascending, are given concatenated:
 * subarray i is vals[off[i] .. off[i+1]).  For 0 < m < total size it finds
 * left-partition sizes m_i with sum m_i = m such that every left element is
 * <= every right element.  Readings (the paper is silent or garbled here):
 * the candidate of the brackets-of-width-one step is element ubar_m_i
 * (0-based); its candidates are ordered by (value, i); the equal-to-t
 * elements of the other last step go to the subarrays in ascending i.
 * Returns 1 if the search ended with t found (last step "case 2"), 2 if it
 * ended with all brackets of width <= 1 (last step "case 1"), 0 if m is 0
 * or the total size (trivial), -1 on bad input.  *iterations (may be null)
 * receives the number of threshold iterations. */
int ora_copass_partition(uint32_t k, const uint64_t* vals, const uint64_t* off, uint64_t m,
                         uint64_t* m_out, uint64_t* iterations);

/* COPASS block sort (Appendix A, "The COPASS block-sort algorithm"): sorts n
 * values in place, keeping blocks of size B (the last one may be shorter),
 * with auxiliary storage of one block.  Each block is first sorted with a
 * stable sort; then block b = 0, 1, ... is extracted: the COPASS partition of
 * the remaining sorted subarrays with m = size of block b, left partitions
 * copied to the auxiliary array, right partitions shifted to the end, the
 * auxiliary array copied to block b and sorted.  pay[] is permuted alongside
 * vals[] (e.g. the creation index).  Returns 0, or -1 on bad input. */
int ora_copass_block_sort(uint64_t n, uint64_t B, uint64_t* vals, uint64_t* pay);

#ifdef __cplusplus
}
#endif
#endif
