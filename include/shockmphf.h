/*
 * shockmphf: a flat ShockHash minimal perfect hash function built and queried
 * on MI355X (gfx950).  Part of libshockleaf.so.
 *
 * The paper builds ShockHash-RS (ShockHash as the leaf search of RecSplit) and
 * outlines a flat alternative (Section 8; Appendix A.4: buckets split once into
 * leaves, prefix sums of bucket and leaf sizes).  This is that flat scheme,
 * with the open choices made as follows:
 *   - B = max(1, ceil(N / bucket_size)) buckets; bucket(x) =
 *     hi64(fmix64(x ^ 0x5851F42D4C957F2D) * B);
 *   - bucket i of m_i keys has L_i = ceil(m_i / leaf_target) leaves;
 *     leaf(x, sigma, L) = (lo32(fmix64(x ^ fmix64((sigma + 1) *
 *     0xD6E8FEB86659FD93))) * L) >> 32 with the bucket's splitting seed sigma_i
 *     (< 2^16; a per-bucket seed bounding leaf sizes, one of the measures
 *     Appendix A.4 lists; its rule is below);
 *   - a leaf's keys, sorted ascending, get the smallest ShockHash seed and the
 *     canonical orientation of shock_leaf_search (include/shockleaf.h), or
 *     with rotation_fitting the smallest candidate (s, r) of
 *     shock_rf_leaf_search_ex, stored as the value v = s * n + r, or with
 *     bipartite the first seed pair (a, b) of shock_bip_leaf_search_ex,
 *     stored as its rank in that search's order: with m = max(a, b),
 *     v = m^2 + a if a < m, else m^2 + m + b;
 *   - the leaf values are Golomb-Rice coded (include/shockcode.h) with the
 *     caller's table of Rice parameters by leaf size;
 *   - leaf sizes of bucket i lie in [base_i, base_i + 31] with base_i =
 *     max(0, floor(m_i / L_i) - 16) (the splitting seed sigma_i is the
 *     smallest whose sizes all lie there and are at most leaf_max), so each
 *     is stored as a 5-bit code;
 *   - each key's choice f(x) is stored in a 1-bit retrieval structure
 *     (Section 2; the paper uses BuRR, a bumped ribbon):
 *     retrieval = SHOCK_RETRIEVAL_RIBBON (default): one linear system over
 *     GF(2) per bucket with cols(m) = max(64, m + ceil(m / 50)) columns;
 *     key x's row under the bucket's ribbon seed r: h = fmix64(x ^
 *     fmix64((r + 1) * 0x9E6C63D0676A9A99)), start s = (hi32(h) * (cols -
 *     63)) >> 32, coefficient c = fmix64(h) | 1 at columns s .. s + 63; r is
 *     the smallest seed below 256 whose system is solvable, and the stored
 *     bits are the solution whose non-pivot columns (those in the span of
 *     the columns before them) are 0; f(x) = parity(c AND z[s .. s + 63]).
 *     About 1.02 bits per key.
 *     retrieval = SHOCK_RETRIEVAL_XOR: a 3-hypergraph XOR system over 3 * seg
 *     cells, seg = ceil(1.23 N / 3) + 8, solved by peeling in synchronous
 *     rounds; about 1.23 bits per key;
 *   - stored: per block of 16 buckets the absolute key, leaf, ribbon-bit
 *     and Rice-code offsets of its first bucket; per bucket its key and
 *     Rice-code offsets relative to its block (32 bits each), its splitting
 *     seed (16 bits) and ribbon seed (8 bits); a query reads one block, up to
 *     16 relative key offsets, and decodes the codes of the leaves before
 *     its own in its bucket;
 *   - the value of key x: (key offset of its leaf) + h_{f(x)}(x, seed); for a
 *     bipartite leaf h_0 is x's left cell under a and h_1 its right cell
 *     under b.
 * For the N distinct keys it was built from, the function is a bijection onto
 * [0, N).  For other keys it returns some value in [0, N) (or UINT64_MAX if
 * the key falls in an empty bucket).
 *
 * Keys and positions are DEVICE arrays unless marked host.  The structure
 * owns its device memory until shock_mphf_destroy.
 */
#ifndef SHOCKMPHF_H
#define SHOCKMPHF_H

#include <stdint.h>

#include "shockleaf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  uint32_t bucket_size; /* expected keys per bucket; default 3000 */
  uint32_t leaf_target; /* keys per leaf on average (L_i = ceil(m_i / leaf_target)); default 40 */
  uint32_t leaf_max;    /* largest leaf, at most 64; default 56 */
  uint32_t max_rho_tries; /* XOR retrieval: seeds tried; default 64 */
  const uint8_t *rice_k_by_n; /* HOST u8[65]: Rice parameter by leaf size (each at most 56); copied at build */
  uint32_t rotation_fitting; /* 1: leaves use rotation fitting (Section 4); default 0 */
  int32_t partial_k;         /* rotation fitting's partial-hash period: 0 (8 above 32 keys, else 1), 1 or 8 */
  uint32_t bipartite;        /* 1: leaves use bipartite ShockHash (Section 9); not with rotation_fitting;
                                repeated keys are then reported as SHOCK_ENOTFOUND (no retrieval seed
                                solves them) rather than SHOCK_EDUPKEY; default 0 */
  uint32_t retrieval;        /* SHOCK_RETRIEVAL_RIBBON (default) or SHOCK_RETRIEVAL_XOR */
  uint32_t ribbon_rows;      /* ribbon solver: rows one wave holds per 64-column block, at most 256;
                                0 = 256.  A bucket that needs more is solved by the sequential walk
                                instead, with the same result; smaller values only move buckets there */
  uint32_t reserved0;
  uint64_t reserved1;
} shock_mphf_params;

#define SHOCK_RETRIEVAL_RIBBON 0
#define SHOCK_RETRIEVAL_XOR 1

typedef struct shock_mphf shock_mphf;

typedef struct {
  uint64_t n_keys, n_buckets, n_leaves;
  uint64_t rho;          /* XOR retrieval: its seed */
  uint64_t seg;          /* XOR retrieval: cells per third of its table */
  uint32_t max_sigma;    /* largest splitting seed */
  uint32_t peel_rounds;  /* rounds of the successful retrieval peeling */
  uint64_t seed_fixed_bits, seed_unary_bits;
  /* stored bits by part: bucket offsets and splitting seeds; leaf sizes;
   * coded seeds with their offsets; the retrieval (with its seeds) */
  uint64_t bits_buckets, bits_leaf_sizes, bits_seeds, bits_retrieval, bits_total;
  double build_ms;       /* wall time of the build call */
  double search_ms;      /* of which the leaf search (kernel time) */
  /* wall time of the build's phases: bucket and leaf layout (with the leaf
   * sorts), the leaf search call, the seed codes, the retrieval */
  double layout_ms, search_call_ms, codes_ms, retrieval_ms;
  uint32_t rho_tries;    /* XOR retrieval seeds tried */
  uint32_t retrieval;    /* SHOCK_RETRIEVAL_* */
  uint32_t max_rseed;    /* ribbon retrieval: the largest bucket seed */
  uint32_t ribbon_walked; /* ribbon retrieval: buckets solved by the sequential walk */
} shock_mphf_stats;

/* Defaults as documented above (bucket_size 3000, leaf_target 40, leaf_max
 * 56, ribbon retrieval); rice_k_by_n = NULL. */
void shock_mphf_params_init(shock_mphf_params *p);

/* Build the function of n_keys distinct keys (device u64[n_keys]).  The Rice
 * table is required.  Synchronous on hip_stream.  Returns SHOCK_EINVAL for
 * bad parameters (leaf_max > 64, leaf_target 0 or above leaf_max, a bucket
 * needing more than 1024 leaves), SHOCK_EDUPKEY if keys repeat within a leaf,
 * SHOCK_ENOTFOUND if a leaf or the retrieval found no seed, SHOCK_ENOMEM /
 * SHOCK_EHIP on allocation or HIP failures.  On success *out owns the
 * structure.  The build's scratch comes from an arena cached per host thread
 * and device (grown as needed, freed by shock_release_scratch), so builds on
 * other threads and streams are not stalled by frees. */
int shock_mphf_build(const uint64_t *keys, uint64_t n_keys, const shock_mphf_params *params, shock_mphf **out,
                     void *hip_stream);

/* positions[i] = the function's value of queries[i] (device arrays).
 * Asynchronous on hip_stream. */
int shock_mphf_query(const shock_mphf *m, const uint64_t *queries, uint64_t n_queries, uint64_t *positions,
                     void *hip_stream);

/* Sizes and build figures. */
int shock_mphf_info(const shock_mphf *m, shock_mphf_stats *info);

/* Copy the stored parts to HOST arrays, decoded (any pointer may be NULL):
 * bucket offsets u64[B+1], leaf bases u64[B+1], splitting seeds u32[B], leaf
 * sizes u8[n_leaves], leaf values u64[n_leaves] (seeds, or s * n + r under
 * rotation fitting, or the pair rank with bipartite leaves), and with XOR
 * retrieval its cells u8[3 * seg] (one per byte). */
int shock_mphf_export(const shock_mphf *m, uint64_t *bucket_offset, uint64_t *leaf_base, uint32_t *sigma,
                      uint8_t *leaf_sizes, uint64_t *leaf_seeds, uint8_t *cells);

/* Ribbon retrieval's parts to HOST arrays (any pointer may be NULL): each
 * bucket's ribbon seed u8[B], its first bit u64[B+1], and the bits u8[total]
 * (one per byte; total = bit_offset[B]).  SHOCK_EINVAL with XOR retrieval. */
int shock_mphf_export_ribbon(const shock_mphf *m, uint8_t *rseed, uint64_t *bit_offset, uint8_t *bits);

/* Free the structure (NULL is allowed). */
int shock_mphf_destroy(shock_mphf *m);

#ifdef __cplusplus
}
#endif

#endif /* SHOCKMPHF_H */
