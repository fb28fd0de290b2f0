/*
 * CPU oracle for the ShockHash leaf seed search -- TEST INFRASTRUCTURE ONLY.
 * Definitions, notation and citations are in shock_oracle.h.  Plain C, one
 * thread, no blocking or fusion: every seed is hashed, optionally filtered,
 * tested for the pseudoforest property by counting the nodes and edges of
 * each connected component, and the first qualifying seed is returned.
 */
#include "shock_oracle.h"

#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

uint64_t shock_oracle_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

void shock_oracle_slots(uint64_t x, uint64_t s, uint32_t n, uint32_t *h0, uint32_t *h1) {
  uint64_t a = shock_oracle_fmix64(x);
  uint64_t t = shock_oracle_fmix64((s + 1) * GOLDEN);
  uint64_t p = (uint64_t)((uint32_t)a ^ (uint32_t)t) * (a >> 32) + t; /* mod 2^64 */
  uint32_t z = (uint32_t)p ^ (uint32_t)(p >> 32);
  uint64_t q = (uint64_t)z * n; /* z / 2^32 scaled to [0, n): integer part h0, fraction lo32(q) */
  uint32_t first = (uint32_t)(q >> 32);
  *h0 = first;
  if (n < 2) {
    *h1 = 0; /* a single cell: the only slot there is */
    return;
  }
  uint32_t r = (uint32_t)(((q & 0xFFFFFFFFu) * (n - 1)) >> 32);
  *h1 = r + (r >= first ? 1u : 0u);
}

/* Section 2 (pseudoforests) and Section 4: a graph is a pseudoforest iff no
 * connected component holds more edges than nodes.  Components are found by
 * an explicit-stack depth-first search over an edge scan. */
int shock_oracle_is_pseudoforest(uint32_t n, uint32_t n_edges, const uint32_t *h0, const uint32_t *h1) {
  int comp[64];
  uint32_t nodes_in[64], edges_in[64];
  uint32_t stack[64];
  uint32_t n_comp = 0;
  for (uint32_t v = 0; v < n; ++v) comp[v] = -1;
  for (uint32_t v = 0; v < n; ++v) {
    if (comp[v] >= 0) continue;
    uint32_t top = 0, count = 0;
    comp[v] = (int)n_comp;
    stack[top++] = v;
    while (top > 0) {
      uint32_t u = stack[--top];
      ++count;
      for (uint32_t e = 0; e < n_edges; ++e) {
        uint32_t w;
        if (h0[e] == u) w = h1[e];
        else if (h1[e] == u) w = h0[e];
        else continue;
        if (comp[w] < 0) {
          comp[w] = (int)n_comp;
          stack[top++] = w;
        }
      }
    }
    nodes_in[n_comp] = count;
    edges_in[n_comp] = 0;
    ++n_comp;
  }
  for (uint32_t e = 0; e < n_edges; ++e) edges_in[comp[h0[e]]] += 1;
  for (uint32_t c = 0; c < n_comp; ++c)
    if (edges_in[c] > nodes_in[c]) return 0;
  return 1;
}

/* Canonical (smallest-mask) orientation.  Keys forced by the structure come
 * first: a free cell with exactly one unplaced incident key must take that key
 * (the peeling of Section 5's proof).  What is left is a set of disjoint
 * cycles, each with two valid directions; the highest-index unplaced key takes
 * its h0 slot, which fixes its cycle's direction, and peeling resumes. */
int shock_oracle_orientation(uint32_t n, const uint32_t *h0, const uint32_t *h1, uint64_t *f_out) {
  int deg[64], used[64], placed[64];
  uint32_t queue[64 * 4];
  uint32_t head = 0, tail = 0, n_placed = 0;
  uint64_t f = 0;
  if (n > 64) return SHOCK_ORACLE_EINVAL;
  for (uint32_t c = 0; c < n; ++c) {
    deg[c] = 0;
    used[c] = 0;
  }
  for (uint32_t k = 0; k < n; ++k) {
    placed[k] = 0;
    deg[h0[k]] += 1;
    if (h1[k] != h0[k]) deg[h1[k]] += 1;
  }
  for (uint32_t c = 0; c < n; ++c)
    if (deg[c] == 1) queue[tail++] = c;

  for (;;) {
    while (head < tail) {
      uint32_t c = queue[head++];
      if (used[c] || deg[c] != 1) continue;
      uint32_t k = n;
      for (uint32_t e = 0; e < n; ++e)
        if (!placed[e] && (h0[e] == c || h1[e] == c)) {
          k = e;
          break;
        }
      if (k == n) return SHOCK_ORACLE_EINVAL;
      if (h0[k] != c) f |= 1ULL << k;
      used[c] = 1;
      placed[k] = 1;
      ++n_placed;
      deg[h0[k]] -= 1;
      if (h1[k] != h0[k]) deg[h1[k]] -= 1;
      uint32_t other = (h0[k] == c) ? h1[k] : h0[k];
      if (!used[other] && deg[other] == 1) {
        if (tail >= sizeof(queue) / sizeof(queue[0])) return SHOCK_ORACLE_EINVAL;
        queue[tail++] = other;
      }
    }
    if (n_placed == n) break;
    /* Only cycles remain: the highest-index unplaced key takes h0. */
    uint32_t m = n;
    for (uint32_t e = n; e-- > 0;)
      if (!placed[e]) {
        m = e;
        break;
      }
    uint32_t c = h0[m];
    if (used[c]) return SHOCK_ORACLE_EINVAL;
    used[c] = 1;
    placed[m] = 1;
    ++n_placed;
    deg[h0[m]] -= 1;
    if (h1[m] != h0[m]) deg[h1[m]] -= 1;
    if (!used[h1[m]] && deg[h1[m]] == 1) {
      if (tail >= sizeof(queue) / sizeof(queue[0])) return SHOCK_ORACLE_EINVAL;
      queue[tail++] = h1[m];
    }
  }
  /* The choice must be a bijection onto [0, n). */
  {
    uint64_t hit = 0;
    for (uint32_t k = 0; k < n; ++k) {
      uint32_t slot = ((f >> k) & 1) ? h1[k] : h0[k];
      if ((hit >> slot) & 1) return SHOCK_ORACLE_EINVAL;
      hit |= 1ULL << slot;
    }
  }
  *f_out = f;
  return SHOCK_ORACLE_OK;
}

static uint64_t full_mask(uint32_t n) { return n >= 64 ? ~0ULL : ((1ULL << n) - 1); }

int shock_oracle_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                             uint64_t *out_seeds, uint64_t *out_orient,
                             uint64_t start_seed, uint64_t max_seed, int use_filter) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (offsets == NULL || out_seeds == NULL || out_orient == NULL) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    if (offsets[j + 1] < offsets[j]) return SHOCK_ORACLE_EINVAL;
    if (offsets[j + 1] - offsets[j] > 64) return SHOCK_ORACLE_EINVAL;
  }
  if (keys == NULL && offsets[n_leaves] != offsets[0]) return SHOCK_ORACLE_EINVAL;

  int status = SHOCK_ORACLE_OK;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    const uint64_t *x = keys + offsets[j];
    uint32_t h0[64], h1[64];
    int found = 0;
    for (uint64_t s = start_seed; s < max_seed; ++s) {
      for (uint32_t i = 0; i < n; ++i) shock_oracle_slots(x[i], s, n, &h0[i], &h1[i]);
      if (use_filter) {
        uint64_t cover = 0;
        for (uint32_t i = 0; i < n; ++i) cover |= (1ULL << h0[i]) | (1ULL << h1[i]);
        if (cover != full_mask(n)) continue;
      }
      if (shock_oracle_is_pseudoforest(n, n, h0, h1)) {
        uint64_t f = 0;
        if (shock_oracle_orientation(n, h0, h1, &f) != SHOCK_ORACLE_OK) return SHOCK_ORACLE_EINVAL;
        out_seeds[j] = s;
        out_orient[j] = f;
        found = 1;
        break;
      }
    }
    if (!found) {
      out_seeds[j] = UINT64_MAX;
      out_orient[j] = 0;
      status = SHOCK_ORACLE_ENOTFOUND;
    }
  }
  return status;
}

static int seed_qualifies(const uint64_t *x, uint32_t n, uint64_t s, uint32_t *h0, uint32_t *h1) {
  for (uint32_t i = 0; i < n; ++i) shock_oracle_slots(x[i], s, n, &h0[i], &h1[i]);
  return shock_oracle_is_pseudoforest(n, n, h0, h1);
}

int shock_oracle_verify(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                        const uint64_t *seeds, const uint64_t *orient, uint64_t start_seed,
                        uint64_t window, uint8_t *flags) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (offsets == NULL || seeds == NULL || orient == NULL || flags == NULL) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j)
    if (offsets[j + 1] < offsets[j] || offsets[j + 1] - offsets[j] > 64) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    const uint64_t *x = keys + offsets[j];
    uint32_t h0[64], h1[64];
    uint8_t fl = 0;
    uint64_t s = seeds[j];
    if (s == UINT64_MAX) {
      flags[j] = 8;
      continue;
    }
    if (!seed_qualifies(x, n, s, h0, h1)) {
      fl |= 1;
    } else {
      uint64_t f = 0;
      if (shock_oracle_orientation(n, h0, h1, &f) != SHOCK_ORACLE_OK || f != orient[j]) fl |= 2;
    }
    uint64_t lo = s - start_seed > window ? s - window : start_seed;
    for (uint64_t t = lo; t < s; ++t)
      if (seed_qualifies(x, n, t, h0, h1)) {
        fl |= 4;
        break;
      }
    flags[j] = fl;
  }
  return SHOCK_ORACLE_OK;
}

void shock_oracle_seed_stats(const uint64_t *keys, uint32_t n, uint64_t s0, uint64_t count,
                             uint64_t *n_cover, uint64_t *n_pseudoforest, uint64_t *n_h0_bijective) {
  uint64_t cover_count = 0, pf_count = 0, bij_count = 0;
  uint32_t h0[64], h1[64];
  for (uint64_t s = s0; s < s0 + count; ++s) {
    uint64_t cover = 0, first = 0;
    for (uint32_t i = 0; i < n; ++i) {
      shock_oracle_slots(keys[i], s, n, &h0[i], &h1[i]);
      cover |= (1ULL << h0[i]) | (1ULL << h1[i]);
      first |= 1ULL << h0[i];
    }
    if (first == full_mask(n)) ++bij_count;
    if (cover != full_mask(n)) continue;
    ++cover_count;
    if (shock_oracle_is_pseudoforest(n, n, h0, h1)) ++pf_count;
  }
  *n_cover = cover_count;
  *n_pseudoforest = pf_count;
  *n_h0_bijective = bij_count;
}

/* ---- Rotation fitting (definitions in shock_oracle.h) ---- */

int shock_oracle_side(uint64_t x) { return (int)(shock_oracle_fmix64(x ^ 0xD1B54A32D192ED03ULL) >> 63); }

void shock_oracle_rf_slots(uint64_t x, uint64_t s, uint32_t r, uint32_t k, uint32_t n, uint32_t *h0, uint32_t *h1) {
  if (shock_oracle_side(x) == 0) {
    shock_oracle_slots(x, s - (s % k), n, h0, h1);
    return;
  }
  uint32_t g0, g1;
  shock_oracle_slots(x, s, n, &g0, &g1);
  *h0 = (g0 + r) % n;
  *h1 = (g1 + r) % n;
}

int shock_oracle_rf_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                                uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient,
                                uint64_t start_seed, uint64_t max_seed, uint32_t partial_k, int use_filter) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (offsets == NULL || out_seeds == NULL || out_rot == NULL || out_orient == NULL) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    if (offsets[j + 1] < offsets[j]) return SHOCK_ORACLE_EINVAL;
    if (offsets[j + 1] - offsets[j] > 64) return SHOCK_ORACLE_EINVAL;
  }
  if (keys == NULL && offsets[n_leaves] != offsets[0]) return SHOCK_ORACLE_EINVAL;

  int status = SHOCK_ORACLE_OK;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    const uint64_t *x = keys + offsets[j];
    uint32_t k = partial_k ? partial_k : (n > 32 ? 8u : 1u);
    uint32_t h0[64], h1[64];
    int found = 0;
    uint32_t rots = n > 0 ? n : 1;
    for (uint64_t s = start_seed; s < max_seed && !found; ++s) {
      for (uint32_t r = 0; r < rots; ++r) {
        for (uint32_t i = 0; i < n; ++i) shock_oracle_rf_slots(x[i], s, r, k, n, &h0[i], &h1[i]);
        if (use_filter) {
          uint64_t cover = 0;
          for (uint32_t i = 0; i < n; ++i) cover |= (1ULL << h0[i]) | (1ULL << h1[i]);
          if (cover != full_mask(n)) continue;
        }
        if (shock_oracle_is_pseudoforest(n, n, h0, h1)) {
          uint64_t f = 0;
          if (shock_oracle_orientation(n, h0, h1, &f) != SHOCK_ORACLE_OK) return SHOCK_ORACLE_EINVAL;
          out_seeds[j] = s;
          out_rot[j] = r;
          out_orient[j] = f;
          found = 1;
          break;
        }
      }
    }
    if (!found) {
      out_seeds[j] = UINT64_MAX;
      out_rot[j] = 0;
      out_orient[j] = 0;
      status = SHOCK_ORACLE_ENOTFOUND;
    }
  }
  return status;
}

/* ---- Query ---------------------------------------------------------------- */

static int check_csr(const uint64_t *offsets, uint64_t n_leaves) {
  if (offsets == NULL) return 0;
  for (uint64_t j = 0; j < n_leaves; ++j)
    if (offsets[j + 1] < offsets[j] || offsets[j + 1] - offsets[j] > 64) return 0;
  return 1;
}

int shock_oracle_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            const uint64_t *seeds, const uint64_t *orient, uint64_t *out_pos) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (!check_csr(offsets, n_leaves) || seeds == NULL || orient == NULL || out_pos == NULL) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    for (uint32_t i = 0; i < n; ++i) {
      uint64_t g = offsets[j] + i;
      if (seeds[j] == UINT64_MAX) {
        out_pos[g] = UINT64_MAX;
        continue;
      }
      uint32_t h0, h1;
      shock_oracle_slots(keys[g], seeds[j], n, &h0, &h1);
      out_pos[g] = offsets[j] + (((orient[j] >> i) & 1) ? h1 : h0);
    }
  }
  return SHOCK_ORACLE_OK;
}

int shock_oracle_rf_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                               const uint64_t *seeds, const uint32_t *rot, const uint64_t *orient,
                               uint32_t partial_k, uint64_t *out_pos) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (!check_csr(offsets, n_leaves) || seeds == NULL || rot == NULL || orient == NULL || out_pos == NULL)
    return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    uint32_t k = partial_k ? partial_k : (n > 32 ? 8u : 1u);
    for (uint32_t i = 0; i < n; ++i) {
      uint64_t g = offsets[j] + i;
      if (seeds[j] == UINT64_MAX) {
        out_pos[g] = UINT64_MAX;
        continue;
      }
      uint32_t h0, h1;
      shock_oracle_rf_slots(keys[g], seeds[j], rot[j], k, n, &h0, &h1);
      out_pos[g] = offsets[j] + (((orient[j] >> i) & 1) ? h1 : h0);
    }
  }
  return SHOCK_ORACLE_OK;
}

/* ---- Golomb-Rice codes ----------------------------------------------------- */

static void put_bit(uint64_t *stream, uint64_t p) { stream[p / 64] |= 1ULL << (p % 64); }
static int get_bit(const uint64_t *stream, uint64_t p) { return (int)((stream[p / 64] >> (p % 64)) & 1); }

int shock_oracle_rice_encode(const uint64_t *values, const uint64_t *offsets, uint64_t n_leaves,
                             const uint8_t *k_by_n, uint64_t *fixed, uint64_t fixed_words, uint64_t *unary,
                             uint64_t unary_words, uint64_t *index, uint64_t *bits) {
  if (bits == NULL || k_by_n == NULL) return SHOCK_ORACLE_EINVAL;
  if (n_leaves > 0 && (!check_csr(offsets, n_leaves) || values == NULL)) return SHOCK_ORACLE_EINVAL;
  for (int n = 0; n <= 64; ++n)
    if (k_by_n[n] > 56) return SHOCK_ORACLE_EINVAL;
  /* first pass: lengths, and the quotient limit */
  uint64_t fbits = 0, ubits = 0;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t k = k_by_n[offsets[j + 1] - offsets[j]];
    uint64_t q = values[j] >> k;
    if (q >= (1ULL << 32)) return SHOCK_ORACLE_EINVAL;
    fbits += k;
    ubits += q + 1;
  }
  bits[0] = fbits;
  bits[1] = ubits;
  if ((fbits + 63) / 64 > fixed_words || (ubits + 63) / 64 > unary_words) return SHOCK_ORACLE_EINVAL;
  if ((fixed_words > 0 && fixed == NULL) || (unary_words > 0 && unary == NULL) || index == NULL)
    return SHOCK_ORACLE_EINVAL;
  for (uint64_t w = 0; w < fixed_words; ++w) fixed[w] = 0;
  for (uint64_t w = 0; w < unary_words; ++w) unary[w] = 0;
  /* second pass: the codes, leaf by leaf */
  uint64_t fp = 0, up = 0;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    if (j % 64 == 0) {
      index[2 * (j / 64)] = fp;
      index[2 * (j / 64) + 1] = up;
    }
    uint32_t k = k_by_n[offsets[j + 1] - offsets[j]];
    for (uint32_t b = 0; b < k; ++b)
      if ((values[j] >> b) & 1) put_bit(fixed, fp + b);
    fp += k;
    up += values[j] >> k; /* q zero bits */
    put_bit(unary, up);   /* then the terminating one */
    up += 1;
  }
  uint64_t m = (n_leaves + 63) / 64;
  index[2 * m] = fp;
  index[2 * m + 1] = up;
  return SHOCK_ORACLE_OK;
}

int shock_oracle_rice_decode(const uint64_t *fixed, const uint64_t *unary, const uint64_t *offsets,
                             uint64_t n_leaves, const uint8_t *k_by_n, uint64_t *values) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (!check_csr(offsets, n_leaves) || k_by_n == NULL || values == NULL || unary == NULL) return SHOCK_ORACLE_EINVAL;
  uint64_t fp = 0, up = 0;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t k = k_by_n[offsets[j + 1] - offsets[j]];
    uint64_t low = 0;
    for (uint32_t b = 0; b < k; ++b) low |= (uint64_t)get_bit(fixed, fp + b) << b;
    fp += k;
    uint64_t q = 0;
    while (!get_bit(unary, up)) {
      ++q;
      ++up;
    }
    ++up;
    values[j] = (q << k) | low;
  }
  return SHOCK_ORACLE_OK;
}

/* ---- Bipartite ShockHash ---------------------------------------------------- */

void shock_oracle_bip_slots(uint64_t x, uint64_t s, uint32_t n, uint32_t *left, uint32_t *right) {
  uint64_t a = shock_oracle_fmix64(x);
  uint64_t t = shock_oracle_fmix64((s + 1) * GOLDEN);
  uint64_t p = (uint64_t)((uint32_t)a ^ (uint32_t)t) * (a >> 32) + t; /* mod 2^64 */
  uint32_t z = (uint32_t)p ^ (uint32_t)(p >> 32);
  uint32_t nl = n / 2, nr = n - nl;
  uint64_t q = (uint64_t)z * nl;
  *left = (uint32_t)(q >> 32);
  *right = nl + (uint32_t)(((q & 0xFFFFFFFFu) * nr) >> 32);
}

/* Candidate flags of seed s: bit 0 left part covered, bit 1 right part covered. */
static int bip_candidate(const uint64_t *x, uint32_t n, uint64_t s) {
  uint32_t nl = n / 2;
  uint64_t cover_l = 0, cover_r = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t l, r;
    shock_oracle_bip_slots(x[i], s, n, &l, &r);
    cover_l |= 1ULL << l;
    cover_r |= 1ULL << r;
  }
  uint64_t want_l = nl ? full_mask(nl) : 0;
  uint64_t want_r = full_mask(n) & ~want_l;
  int f = 0;
  if (nl == 0 || (cover_l & want_l) == want_l) f |= 1;
  if ((cover_r & want_r) == want_r) f |= 2;
  return f;
}

static int bip_pair_qualifies(const uint64_t *x, uint32_t n, uint64_t a, uint64_t b, uint64_t *f) {
  uint32_t h0[64], h1[64];
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t l, r, l2, r2;
    shock_oracle_bip_slots(x[i], a, n, &l, &r);
    shock_oracle_bip_slots(x[i], b, n, &l2, &r2);
    h0[i] = n / 2 ? l : r2; /* one cell only when n = 1 */
    h1[i] = r2;
  }
  if (!shock_oracle_is_pseudoforest(n, n, h0, h1)) return 0;
  return shock_oracle_orientation(n, h0, h1, f) == SHOCK_ORACLE_OK;
}

int shock_oracle_bip_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                                 uint64_t *out_a, uint64_t *out_b, uint64_t *out_orient, uint64_t max_seed,
                                 int use_filter) {
  if (n_leaves == 0) return SHOCK_ORACLE_OK;
  if (offsets == NULL || out_a == NULL || out_b == NULL || out_orient == NULL) return SHOCK_ORACLE_EINVAL;
  for (uint64_t j = 0; j < n_leaves; ++j)
    if (offsets[j + 1] < offsets[j] || offsets[j + 1] - offsets[j] > 64) return SHOCK_ORACLE_EINVAL;
  int status = SHOCK_ORACLE_OK;
  uint8_t *cand = (uint8_t *)malloc(max_seed < (1u << 26) ? max_seed + 1 : (1u << 26));
  if (!cand) return SHOCK_ORACLE_EINVAL;
  uint64_t cap = max_seed < (1u << 26) ? max_seed : (1u << 26);
  for (uint64_t j = 0; j < n_leaves; ++j) {
    uint32_t n = (uint32_t)(offsets[j + 1] - offsets[j]);
    const uint64_t *x = keys + offsets[j];
    int found = 0;
    if (n <= 1) {
      out_a[j] = 0;
      out_b[j] = 0;
      out_orient[j] = 0;
      continue;
    }
    for (uint64_t m = 0; m < cap && !found; ++m) {
      cand[m] = use_filter ? (uint8_t)bip_candidate(x, n, m) : 3;
      /* pairs with max(a, b) = m in the order (0, m), ..., (m-1, m), (m, 0), ..., (m, m) */
      for (uint64_t a = 0; a < m && !found; ++a) {
        if (!(cand[a] & 1) || !(cand[m] & 2)) continue;
        uint64_t f;
        if (bip_pair_qualifies(x, n, a, m, &f)) {
          out_a[j] = a;
          out_b[j] = m;
          out_orient[j] = f;
          found = 1;
        }
      }
      for (uint64_t b = 0; b <= m && !found; ++b) {
        if (!(cand[m] & 1) || !(cand[b] & 2)) continue;
        uint64_t f;
        if (bip_pair_qualifies(x, n, m, b, &f)) {
          out_a[j] = m;
          out_b[j] = b;
          out_orient[j] = f;
          found = 1;
        }
      }
    }
    if (!found) {
      out_a[j] = UINT64_MAX;
      out_b[j] = UINT64_MAX;
      out_orient[j] = 0;
      status = SHOCK_ORACLE_ENOTFOUND;
    }
  }
  free(cand);
  return status;
}

