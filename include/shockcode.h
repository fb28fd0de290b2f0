/*
 * shockcode: leaf queries and Golomb-Rice seed codes for the ShockHash leaf
 * seed search (include/shockleaf.h), on MI355X (gfx950).  Part of
 * libshockleaf.so.
 *
 * All array arguments are DEVICE pointers unless marked host; the caller owns
 * every buffer.  Leaves are given as in shockleaf.h: a CSR batch, leaf j being
 * keys[offsets[j] .. offsets[j+1]), at most 64 keys.  Status codes are
 * shockleaf.h's SHOCK_*; HIP failures return SHOCK_EHIP with the message in
 * shock_last_error().
 */
#ifndef SHOCKCODE_H
#define SHOCKCODE_H

#include <stdint.h>

#include "shockleaf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Leaf query (Section 4: the MPHF answers key x with h_{s, f(x)}(x)).  For
 * key i of leaf j (global index g = offsets[j] + i):
 *   out_pos[g] = offsets[j] + (bit i of orient[j] ? h1 : h0)(x_g, seeds[j])
 * with the hash of shockleaf.h, i.e. the key's slot in its leaf, shifted to a
 * position in [0, offsets[n_leaves]).  A leaf whose seed is UINT64_MAX maps
 * its keys to UINT64_MAX.  With seeds and orientations from a search, the
 * positions of the batch are a permutation of [0, offsets[n_leaves]).
 * keys u64[offsets[n_leaves]], offsets u64[n_leaves+1], seeds u64[n_leaves],
 * orient u64[n_leaves], out_pos u64[offsets[n_leaves]].  Asynchronous on
 * hip_stream (NULL: the null stream).  offsets must be a valid CSR (as the
 * search checks); leaves are taken in groups of 64, and a group holding a leaf
 * of more than 64 keys or decreasing offsets is skipped (its keys' entries
 * left untouched).  Returns SHOCK_EINVAL for NULL pointers. */
int shock_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, const uint64_t *seeds,
                     const uint64_t *orient, uint64_t *out_pos, void *hip_stream);

/* The same under rotation fitting (shock_rf_leaf_search_ex): keys of the
 * first set take their slots under seed s - (s mod k), keys of the second set
 * under seed s shifted by rot[j] (mod n); k = partial_k (1 or 8; 0 = 8 above
 * 32 keys, else 1).  rot u32[n_leaves]. */
int shock_rf_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, const uint64_t *seeds,
                        const uint32_t *rot, const uint64_t *orient, int32_t partial_k, uint64_t *out_pos,
                        void *hip_stream);

/* Golomb-Rice codes of one value per leaf (Section 4 stores a leaf's seed in
 * 0.44n + o(n) bits in expectation with Golomb-Rice codes).  Leaf j of
 * n_j keys codes values[j] with the Rice parameter k = k_by_n[n_j]:
 *   - the k low bits go to the FIXED stream, least significant first;
 *   - the quotient q = values[j] >> k goes to the UNARY stream as q zero
 *     bits followed by one 1 bit.
 * Both streams concatenate the leaves' parts in leaf order; bit p of a stream
 * is bit (p mod 64) of 64-bit word p / 64, unused bits are zero.  index
 * (u64[2 * (ceil(n_leaves / 64) + 1)]) receives for every block of 64 leaves
 * the (fixed, unary) bit positions where its first leaf's codes start, and
 * finally the two total lengths; the decoder needs it.
 * k_by_n: HOST u8[65], every entry at most 56 (the best k for a geometric
 * seed with success probability p minimises k + 1 + t / (1 - t),
 * t = (1 - p)^(2^k)).
 * fixed / unary: fixed_words / unary_words words (may be NULL when 0).
 * bits: HOST u64[2], receives the stream lengths in bits.
 * Synchronous: returns when the streams are written.  SHOCK_EINVAL for a bad
 * argument or table, a leaf of more than 64 keys, a quotient of 2^32 or more,
 * or streams too short for the codes; in the last case bits[] still holds the
 * lengths needed (so a first call with zero capacities sizes the streams). */
int shock_rice_encode(const uint64_t *values, const uint64_t *offsets, uint64_t n_leaves, const uint8_t *k_by_n,
                      uint64_t *fixed, uint64_t fixed_words, uint64_t *unary, uint64_t unary_words, uint64_t *index,
                      uint64_t *bits, void *hip_stream);

/* Decode every leaf's value from the streams and index written by
 * shock_rice_encode for the same offsets and k_by_n (HOST u8[65]).  One wave
 * decodes a block of 64 leaves from its index entry alone.  values
 * u64[n_leaves]; a leaf of more than 64 keys decodes to UINT64_MAX.
 * Asynchronous on hip_stream.  Reads stay inside the given stream sizes. */
int shock_rice_decode(const uint64_t *fixed, uint64_t fixed_words, const uint64_t *unary, uint64_t unary_words,
                      const uint64_t *index, const uint64_t *offsets, uint64_t n_leaves, const uint8_t *k_by_n,
                      uint64_t *values, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SHOCKCODE_H */
