/*
 * CPU oracle for the ShockHash leaf seed search -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, slow and deliberately unoptimised C.  It exists to
 * check the GPU library, never to serve it: only the tests, the smoke check
 * and the benchmark's CPU-baseline leg load it.  It shares no code, header or
 * table with the HIP path.
 *
 * What it computes (ShockHash, Section 4, the equation defining the seed):
 * for a leaf S of n keys, the smallest seed s in N such that some choice
 * f : S -> {0,1} makes x -> h_{f(x)}(x, s) a bijection onto [0, n), plus one
 * such f.  By the equivalence of Section 5 (equation "pseudoforests-orientable")
 * and the pseudoforest remark of Section 2, a seed qualifies exactly when the
 * graph G_s = ([n], {{h0(x,s), h1(x,s)} : x in S}) is a pseudoforest, i.e. no
 * connected component has more edges than nodes.  The oracle decides this by
 * counting nodes and edges per component (a depth-first search), which is a
 * different algorithm from the union-find test of Appendix A.1 used on the GPU.
 *
 * Hash functions (the paper assumes fully random h0, h1 evaluated on a 64-bit
 * master hash code, Section 8 and the footnote on uniform hashing in Section 5;
 * the concrete family below is this library's frozen choice):
 *   fmix64(k)   : MurmurHash3's 64-bit finaliser (Appleby), a bijection on u64
 *                 k ^= k>>33; k *= 0xff51afd7ed558ccd; k ^= k>>33;
 *                 k *= 0xc4ceb9fe1a85ec53; k ^= k>>33
 *   a(x)        = fmix64(x)                              (per key)
 *   t(s)        = fmix64((s + 1) * 0x9E3779B97F4A7C15)   (per seed, mod 2^64)
 *   P           = (lo32(a) XOR lo32(t)) * hi32(a) + t    (mod 2^64; one
 *                 32x32+64 multiply-add)
 *   z           = lo32(P) XOR hi32(P)
 *   Q           = z * n                                  (exact 64-bit product)
 *   h0          = Q >> 32                                (h0 in [0, n-1])
 *   r           = ((Q mod 2^32) * (n - 1)) >> 32         (r in [0, n-2])
 *   h1          = r + (r >= h0 ? 1 : 0)  for n >= 2;  h1 = 0 for n = 1
 * so h1 != h0 whenever n >= 2: the graph has no self-loops, which is the
 * variant the paper's implementation uses (footnote in Section 5).
 *
 * Orientation returned with a seed: the numerically smallest n-bit mask f
 * (bit i <-> i-th key of the leaf) for which i -> h_{f_i} is a bijection.
 * Section 5 (equation "orientations-cycles") shows a pseudoforest with c
 * components has exactly 2^c such f, differing only in the direction of each
 * component's cycle; the smallest mask directs every cycle so that its
 * highest-index key takes its h0 slot.
 */
#ifndef SHOCK_ORACLE_H
#define SHOCK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHOCK_ORACLE_OK 0
#define SHOCK_ORACLE_EINVAL (-1)
#define SHOCK_ORACLE_ENOTFOUND (-2)

/* MurmurHash3 fmix64. */
uint64_t shock_oracle_fmix64(uint64_t k);

/* The two candidate slots of key x under seed s in a leaf of n keys (1 <= n <= 64). */
void shock_oracle_slots(uint64_t x, uint64_t s, uint32_t n, uint32_t *h0, uint32_t *h1);

/* 1 if the multigraph on [n] with edges {h0[i], h1[i]} (i < n_edges) has no
 * component with more edges than nodes, else 0.  Self-loops and parallel
 * edges are allowed.  n <= 64, n_edges <= 64. */
int shock_oracle_is_pseudoforest(uint32_t n, uint32_t n_edges, const uint32_t *h0, const uint32_t *h1);

/* Canonical orientation (smallest valid mask) of n edges on n nodes.  Returns
 * SHOCK_ORACLE_OK and writes *f, or SHOCK_ORACLE_EINVAL if no bijective
 * choice exists (the graph is not a pseudoforest). */
int shock_oracle_orientation(uint32_t n, const uint32_t *h0, const uint32_t *h1, uint64_t *f);

/* Leaf seed search over a CSR batch (HOST pointers).
 *   keys[offsets[j] .. offsets[j+1]) are leaf j's keys, offsets has n_leaves+1
 *   nondecreasing entries, every leaf has at most 64 keys.
 *   Seeds start_seed, start_seed+1, ..., max_seed-1 are tried in order.
 *   use_filter = 1 first rejects seeds whose slots do not cover all n cells
 *   (Section 4, the bit-mask filter; a necessary condition, so results are
 *   identical with use_filter = 0).
 * Outputs: out_seeds[j] = smallest qualifying seed, out_orient[j] = its
 * canonical orientation; a leaf with no qualifying seed below max_seed gets
 * UINT64_MAX and 0.  Returns SHOCK_ORACLE_EINVAL (outputs untouched) on a
 * malformed batch, SHOCK_ORACLE_ENOTFOUND if any leaf hit the cap, else OK. */
int shock_oracle_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                             uint64_t *out_seeds, uint64_t *out_orient,
                             uint64_t start_seed, uint64_t max_seed, int use_filter);

/* Check claimed results leaf by leaf (HOST pointers).  For leaf j with
 * claimed seed s = seeds[j] (UINT64_MAX = none), flags[j] gets
 *   bit 0  s does not qualify (its graph is not a pseudoforest),
 *   bit 1  orient[j] differs from the canonical orientation at s,
 *   bit 2  some seed in [max(start_seed, s - window), s) qualifies,
 *   bit 3  no seed was claimed (s = UINT64_MAX; nothing else checked).
 * Returns SHOCK_ORACLE_EINVAL on a malformed batch, else OK. */
int shock_oracle_verify(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                        const uint64_t *seeds, const uint64_t *orient, uint64_t start_seed,
                        uint64_t window, uint8_t *flags);

/* ---- Rotation fitting (Section 4, "Rotation Fitting"; Appendix A.2) ----
 *
 * Keys are split into two fixed sets by a 1-bit hash of the key alone:
 *   side(x) = fmix64(x ^ 0xD1B54A32D192ED03) >> 63   (0 = first set, 1 = second).
 * A candidate is a pair (s, r), s a seed and r in [0, n) a rotation.  Under it
 *   a key x of the first set takes the slots  slots(x, s - (s mod k)),
 *   a key x of the second set takes           (slots(x, s) + r) mod n (both slots),
 * where k >= 1 is the partial-hash period of Appendix A.2 (k = 1: the first
 * set is hashed with s itself).  Rotating the second set's slots is the
 * cyclic rotation of its bit mask that the paper describes.  Candidates are
 * tried in the order s = start, start+1, ... and, for each s, r = 0 .. n-1;
 * the result is the first pair whose graph is a pseudoforest and the
 * canonical orientation of that graph. */

/* 1 if key x belongs to the second set. */
int shock_oracle_side(uint64_t x);

/* Slots of key x (leaf of n keys, index in the first or second set decided by
 * side(x)) under candidate (s, r) with partial-hash period k. */
void shock_oracle_rf_slots(uint64_t x, uint64_t s, uint32_t r, uint32_t k, uint32_t n, uint32_t *h0, uint32_t *h1);

/* Rotation-fitting leaf search over a CSR batch (HOST pointers); as
 * shock_oracle_leaf_search, plus the rotation of each result in out_rot
 * (0 for leaves without a result).  partial_k = 0 selects the paper's rule:
 * k = 8 for leaves of more than 32 keys, else 1. */
int shock_oracle_rf_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                                uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient,
                                uint64_t start_seed, uint64_t max_seed, uint32_t partial_k, int use_filter);

/* ---- Query (Section 4: a key x is answered by h_{s, f(x)}(x)) ------------
 * Key i of leaf j (global index offsets[j] + i) maps to
 *   offsets[j] + (bit i of orient[j] ? h1 : h0)(x_i, seeds[j]),
 * a global position in [0, offsets[n_leaves]).  Leaves whose seed is
 * UINT64_MAX (none found) map their keys to UINT64_MAX.  The rotation-fitting
 * form takes the slots of shock_oracle_rf_slots under (seeds[j], rot[j]) with
 * period partial_k (0: 8 above 32 keys, else 1).  HOST pointers; out_pos has
 * offsets[n_leaves] entries (indexed by the global key index). */
int shock_oracle_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            const uint64_t *seeds, const uint64_t *orient, uint64_t *out_pos);
int shock_oracle_rf_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                               const uint64_t *seeds, const uint32_t *rot, const uint64_t *orient,
                               uint32_t partial_k, uint64_t *out_pos);

/* ---- Golomb-Rice codes of per-leaf values (the seed encoding of Section 4;
 * Golomb 1966, Rice 1979) ----------------------------------------------------
 * Leaf j (n_j = offsets[j+1] - offsets[j] keys) codes value v_j with the Rice
 * parameter k = k_by_n[n_j] (k_by_n has 65 entries, each at most 56):
 *   - its k low bits go to the FIXED stream, least significant first;
 *   - its quotient q = v_j >> k goes to the UNARY stream as q zero bits
 *     followed by one 1 bit.
 * Each stream is the concatenation of the leaves' parts in leaf order.  Bit p
 * of a stream is bit (p mod 64) of 64-bit word p / 64 (least significant bit
 * first); unused bits are zero.
 * The sampled index has 2 * (ceil(n_leaves / 64) + 1) words: for m = 0, 1,
 * ..., entry (2m, 2m+1) is the (fixed, unary) bit position where leaf 64m's
 * codes start (the last pair: the total lengths).
 * encode: fixed / unary have fixed_words / unary_words words; bits[0], bits[1]
 * receive the two stream lengths in bits.  Returns EINVAL if a quotient is
 * 2^32 or more, or if a stream does not fit (bits[] still receive the lengths
 * needed).  decode: the inverse, from the streams alone (no index). */
int shock_oracle_rice_encode(const uint64_t *values, const uint64_t *offsets, uint64_t n_leaves,
                             const uint8_t *k_by_n, uint64_t *fixed, uint64_t fixed_words, uint64_t *unary,
                             uint64_t unary_words, uint64_t *index, uint64_t *bits);
int shock_oracle_rice_decode(const uint64_t *fixed, const uint64_t *unary, const uint64_t *offsets,
                             uint64_t n_leaves, const uint8_t *k_by_n, uint64_t *values);

/* ---- Bipartite ShockHash (the outlook of Section 9) -------------------------
 * The table's n cells are split into a left part [0, nl), nl = floor(n / 2),
 * and a right part [nl, n).  Under seed s, with z the 32-bit hash value of
 * key x of the frozen family (shock_oracle_slots' z):
 *   Q           = z * nl                               (exact 64-bit product)
 *   left(x, s)  = Q >> 32                              (0 when nl = 0)
 *   right(x, s) = nl + (((Q mod 2^32) * (n - nl)) >> 32)
 * A pair (a, b) of seeds gives key x the candidate cells left(x, a) and
 * right(x, b); the leaf's result is the pair whose graph is a pseudoforest
 * that comes first in the order max(a, b), then a, then b -- the order in
 * which a search that draws seeds 0, 1, 2, ... and pairs each new seed with
 * all earlier ones meets them.  Seed a is a left candidate if its left cells
 * cover [0, nl), b a right candidate if its right cells cover [nl, n); only
 * such pairs can qualify, and use_filter skips the others (same result).
 * Orientation: as shock_oracle_orientation on the edges (left, right).
 * Seeds are limited to max_seed (pairs with max(a, b) < max_seed). */
void shock_oracle_bip_slots(uint64_t x, uint64_t s, uint32_t n, uint32_t *left, uint32_t *right);
/* Rank of the pair (a, b) in that order: with m = max(a, b), the m^2 pairs
 * of smaller maximum come first, then (0, m) .. (m-1, m), then (m, 0) ..
 * (m, m); so the rank is m^2 + a if a < m, else m^2 + m + b.  A stored
 * bipartite leaf value in the flat MPHF. */
uint64_t shock_oracle_bip_pair_rank(uint64_t a, uint64_t b);
int shock_oracle_bip_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                                 uint64_t *out_a, uint64_t *out_b, uint64_t *out_orient, uint64_t max_seed,
                                 int use_filter);

/* ---- A flat ShockHash MPHF (Section 8's flat decomposition; the two-level
 * scheme of Appendix A.4 with per-bucket splitting seeds) ------------------
 * Definitions (this library's choices; the paper leaves the scheme open):
 *   B = max(1, ceil(N / bucket_size)) buckets;
 *   bucket(x) = hi64(fmix64(x ^ 0x5851F42D4C957F2D) * B);
 *   bucket i of m_i keys gets L_i = ceil(m_i / leaf_target) leaves;
 *   leaf(x, sigma, L) = (lo32(fmix64(x ^ fmix64((sigma + 1) * 0xD6E8FEB86659FD93))) * L) >> 32;
 *   sigma_i = the smallest sigma whose leaf sizes all lie in [base_i, base_i + 31]
 *   (shock_oracle_leaf_size_base) and are at most leaf_max;
 *   leaves are numbered globally bucket by bucket, and a leaf's keys are
 *   sorted ascending (so the leaf search and its canonical orientation are
 *   defined by the key set alone).
 * split: HOST arrays.  keys u64[N] (distinct); out: bucket_offset u64[B+1]
 * (key offsets), leaf_base u64[B+1] (leaf offsets), sigma u32[B],
 * leaf_sizes u8[leaf_cap], leaf_keys u64[N] (the keys in leaf order),
 * key_index u64[N] (original index of each of those keys), *n_leaves.
 * Returns EINVAL for bad parameters (leaf_max > 64, leaf_target 0 or above
 * leaf_max, bucket_size 0), leaf_cap too small or a bucket of more than 1024
 * leaves, and ENOTFOUND for a bucket with no splitting seed below 2^16. */
int shock_oracle_mphf_split(const uint64_t *keys, uint64_t n_keys, uint32_t bucket_size, uint32_t leaf_target,
                            uint32_t leaf_max, uint64_t n_buckets, uint64_t *bucket_offset, uint64_t *leaf_base,
                            uint32_t *sigma, uint8_t *leaf_sizes, uint64_t leaf_cap, uint64_t *leaf_keys,
                            uint64_t *key_index, uint64_t *n_leaves);

/* Leaf sizes of a bucket of m keys split into n_leaves leaves lie in
 * [base, base + 31] with base = max(0, floor(m / n_leaves) - 16), so each is
 * stored in 5 bits; the splitting seed is the smallest one whose sizes all
 * lie there and are at most leaf_max. */
uint32_t shock_oracle_leaf_size_base(uint64_t m, uint32_t n_leaves);

/* ---- Ribbon retrieval (Section 2's retrieval data structures; the paper
 * uses BuRR, a bumped ribbon).  One linear system over GF(2) per bucket.
 *
 * gf2_solve: rows u64[m][ceil(cols / 64)] (bit c of row r is column c),
 * right-hand sides b u8[m] (0/1).  Returns 1 and z u8[cols] if the system
 * has a solution, 0 if not (-1 on allocation failure).  z is the canonical
 * solution: every non-pivot column is 0, where the pivot columns are those
 * not in the span of the columns before them (the reduced row echelon form
 * with columns taken from 0 up; a solution with those zeros is unique).
 *
 * A bucket of m keys has cols(m) = max(64, m + ceil(m / 50)) columns (about
 * 2 % more than keys; 0 if m = 0).  Key x's row under ribbon seed r: with
 * h = fmix64(x ^ fmix64((r + 1) * 0x9E6C63D0676A9A99)), start
 * s = (hi32(h) * (cols - 63)) >> 32 and coefficient c = fmix64(h) | 1 (bit 0
 * set), the row holds c's bits at columns s .. s + 63.  The bucket's seed is
 * the smallest r < max_seeds whose system (values = the keys' choices) has a
 * solution; its bits are the canonical solution.  The value of x is the
 * parity of c AND z[s .. s + 63]. */
int shock_oracle_gf2_solve(const uint64_t *rows, const uint8_t *b, uint64_t m, uint64_t cols, uint8_t *z);
uint64_t shock_oracle_ribbon_cols(uint64_t m);
void shock_oracle_ribbon_row(uint64_t x, uint32_t rseed, uint64_t cols, uint64_t *start, uint64_t *coef);
int shock_oracle_ribbon_build(const uint64_t *keys, const uint8_t *values, uint64_t m, uint32_t max_seeds,
                              uint32_t *rseed, uint8_t *z);
uint8_t shock_oracle_ribbon_get(uint64_t x, uint32_t rseed, uint64_t cols, const uint8_t *z);
/* Every bucket's system: keys in leaf order (bucket b = leaf_keys[bucket_offset[b] ..
 * bucket_offset[b+1])), values u8[N]; out rseed u8[B], bit_offset u64[B+1]
 * (prefix sums of cols), z u8[bit_offset[B]]. */
int shock_oracle_mphf_ribbon(const uint64_t *leaf_keys, const uint8_t *values, uint64_t n_buckets,
                             const uint64_t *bucket_offset, uint32_t max_seeds, uint8_t *rseed,
                             uint64_t *bit_offset, uint8_t *z);

#define SHOCK_ORACLE_RETRIEVAL_RIBBON 0
#define SHOCK_ORACLE_RETRIEVAL_XOR 1

/* 1-bit retrieval by a 3-hypergraph XOR system (a simpler stand-in for the
 * ribbon retrieval of Section 2): M = 3 * seg cells, seg = ceil(1.23 N / 3) + 8,
 * each key x hashes under retrieval seed rho to one cell in each third:
 *   u = fmix64(x ^ fmix64((rho + 1) * 0xA0761D6478BD642F)), v = fmix64(u)
 *   c0 = (lo32(u) * seg) >> 32, c1 = seg + ((hi32(u) * seg) >> 32),
 *   c2 = 2 * seg + ((lo32(v) * seg) >> 32)
 * and the value of x is Z[c0] ^ Z[c1] ^ Z[c2].  Z is found by peeling in
 * synchronous rounds: in each round every remaining key with a cell of
 * exactly one remaining key is peeled at the first such cell (c0, c1, c2
 * order), all of them at once; then, rounds in reverse, each peeled key sets
 * its peel cell to its value XOR its other two cells.  rho is the smallest
 * seed from rho_start on (at most max_tries) for which every key peels.
 * build: HOST arrays; values u8[N] (0/1); Z u8[3 * seg] (one cell per byte).
 * Returns ENOTFOUND if no seed of the range peels. */
uint64_t shock_oracle_xor_segment(uint64_t n_keys);
int shock_oracle_xor_build(const uint64_t *keys, const uint8_t *values, uint64_t n_keys, uint64_t rho_start,
                           uint32_t max_tries, uint64_t *rho, uint8_t *z);
int shock_oracle_xor_get(const uint64_t *keys, uint64_t n_keys, uint64_t rho, const uint8_t *z, uint8_t *values);

/* The MPHF's value of each query key (which must be one of the built keys):
 * bucket, splitting seed, leaf and its key offset, then the leaf query
 * offset + h_{f(x)}(x, seed) with f(x) read from the retrieval structure.
 * leaf_values u64[n_leaves]: the leaf search's seeds, or with rf = 1 the
 * rotation-fitting candidates stored as s * n + r (slots of
 * shock_oracle_rf_slots with period partial_k; 0 = 8 above 32 keys, else 1),
 * or with rf = 2 the bipartite pair (a, b) stored as its rank
 * shock_oracle_bip_pair_rank(a, b): key x's two candidate cells are then the
 * left cell of x under a and the right cell of x under b.  f(x) comes from
 * the ribbon systems (retrieval = SHOCK_ORACLE_RETRIEVAL_RIBBON: rseed u8[B],
 * rbit_offset u64[B+1], z their bits) or from the XOR system (retrieval =
 * SHOCK_ORACLE_RETRIEVAL_XOR: rho and z its cells; rseed and rbit_offset
 * unused). */
int shock_oracle_mphf_query(const uint64_t *queries, uint64_t n_queries, uint64_t n_keys, uint32_t leaf_target,
                            uint64_t n_buckets, const uint64_t *bucket_offset, const uint64_t *leaf_base,
                            const uint32_t *sigma, const uint8_t *leaf_sizes, const uint64_t *leaf_values,
                            int rf, uint32_t partial_k, int retrieval, uint64_t rho, const uint8_t *rseed,
                            const uint64_t *rbit_offset, const uint8_t *z, uint64_t *out_pos);

/* Statistics helper: over seeds s0 .. s0+count-1 of one leaf of n keys, count
 * the seeds whose slots cover all n cells and, among them, the pseudoforests.
 * Also counts seeds where h0 alone is a bijection. */
void shock_oracle_seed_stats(const uint64_t *keys, uint32_t n, uint64_t s0, uint64_t count,
                             uint64_t *n_cover, uint64_t *n_pseudoforest, uint64_t *n_h0_bijective);

#ifdef __cplusplus
}
#endif
#endif
