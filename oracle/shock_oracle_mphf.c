/*
 * CPU oracle, flat ShockHash MPHF part -- TEST INFRASTRUCTURE ONLY.
 * Plain single-threaded C; definitions in shock_oracle.h.
 */
#include "shock_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static uint64_t bucket_of(uint64_t x, uint64_t n_buckets) {
  uint64_t h = shock_oracle_fmix64(x ^ 0x5851F42D4C957F2DULL);
  return (uint64_t)(((unsigned __int128)h * n_buckets) >> 64);
}

static uint32_t leaf_of(uint64_t x, uint32_t sigma, uint32_t n_leaves) {
  uint64_t t = shock_oracle_fmix64(((uint64_t)sigma + 1) * 0xD6E8FEB86659FD93ULL);
  uint64_t h = shock_oracle_fmix64(x ^ t);
  return (uint32_t)(((uint64_t)(uint32_t)h * n_leaves) >> 32);
}

uint32_t shock_oracle_leaf_size_base(uint64_t m, uint32_t n_leaves) {
  if (n_leaves == 0) return 0;
  uint64_t mean = m / n_leaves;
  return mean > 16 ? (uint32_t)(mean - 16) : 0;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : x > y ? 1 : 0;
}

int shock_oracle_mphf_split(const uint64_t *keys, uint64_t n_keys, uint32_t bucket_size, uint32_t leaf_target,
                            uint32_t leaf_max, uint64_t n_buckets, uint64_t *bucket_offset, uint64_t *leaf_base,
                            uint32_t *sigma, uint8_t *leaf_sizes, uint64_t leaf_cap, uint64_t *leaf_keys,
                            uint64_t *key_index, uint64_t *n_leaves) {
  if (bucket_size == 0 || leaf_target == 0 || leaf_max > 64 || leaf_target > leaf_max) return SHOCK_ORACLE_EINVAL;
  uint64_t want_b = n_keys == 0 ? 1 : (n_keys + bucket_size - 1) / bucket_size;
  if (n_buckets != want_b) return SHOCK_ORACLE_EINVAL;
  /* buckets: sizes, offsets, keys grouped by bucket (input order within) */
  for (uint64_t b = 0; b <= n_buckets; ++b) bucket_offset[b] = 0;
  for (uint64_t i = 0; i < n_keys; ++i) bucket_offset[bucket_of(keys[i], n_buckets) + 1] += 1;
  for (uint64_t b = 0; b < n_buckets; ++b) bucket_offset[b + 1] += bucket_offset[b];
  uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * (n_buckets + 1));
  uint64_t *grouped = (uint64_t *)malloc(sizeof(uint64_t) * (n_keys + 1));
  uint64_t *grouped_idx = (uint64_t *)malloc(sizeof(uint64_t) * (n_keys + 1));
  if (!fill || !grouped || !grouped_idx) return SHOCK_ORACLE_EINVAL;
  memcpy(fill, bucket_offset, sizeof(uint64_t) * (n_buckets + 1));
  for (uint64_t i = 0; i < n_keys; ++i) {
    uint64_t b = bucket_of(keys[i], n_buckets);
    grouped[fill[b]] = keys[i];
    grouped_idx[fill[b]] = i;
    fill[b] += 1;
  }
  /* leaves per bucket and their global numbering */
  leaf_base[0] = 0;
  for (uint64_t b = 0; b < n_buckets; ++b) {
    uint64_t m = bucket_offset[b + 1] - bucket_offset[b];
    leaf_base[b + 1] = leaf_base[b] + (m + leaf_target - 1) / leaf_target;
  }
  int rc = SHOCK_ORACLE_OK;
  if (leaf_base[n_buckets] > leaf_cap) rc = SHOCK_ORACLE_EINVAL;
  *n_leaves = leaf_base[n_buckets];
  uint64_t count[1 << 12];
  for (uint64_t b = 0; b < n_buckets && rc == SHOCK_ORACLE_OK; ++b) {
    uint64_t o = bucket_offset[b], m = bucket_offset[b + 1] - o;
    uint32_t L = (uint32_t)(leaf_base[b + 1] - leaf_base[b]);
    if (L > 1024) {  /* the library's bound on leaves per bucket */
      rc = SHOCK_ORACLE_EINVAL;
      break;
    }
    /* smallest splitting seed whose leaf sizes all lie in [lo, lo + 31] and
     * at most leaf_max */
    uint32_t lo = shock_oracle_leaf_size_base(m, L);
    uint32_t s = 0;
    for (;; ++s) {
      if (s >= (1u << 16)) {  /* no splitting seed: like a leaf without a seed */
        rc = SHOCK_ORACLE_ENOTFOUND;
        break;
      }
      for (uint32_t j = 0; j < L; ++j) count[j] = 0;
      for (uint64_t i = 0; i < m; ++i) count[leaf_of(grouped[o + i], s, L)] += 1;
      int fits = 1;
      for (uint32_t j = 0; j < L; ++j)
        if (count[j] > leaf_max || count[j] < lo || count[j] > lo + 31) fits = 0;
      if (fits) break;
    }
    if (rc != SHOCK_ORACLE_OK) break;
    sigma[b] = s;
    /* leaves: sizes, then keys leaf by leaf in ascending order */
    uint64_t start = o;
    for (uint32_t j = 0; j < L; ++j) {
      uint64_t k = 0;
      for (uint64_t i = 0; i < m; ++i)
        if (leaf_of(grouped[o + i], s, L) == j) {
          leaf_keys[start + k] = grouped[o + i];
          ++k;
        }
      leaf_sizes[leaf_base[b] + j] = (uint8_t)k;
      qsort(leaf_keys + start, k, sizeof(uint64_t), cmp_u64);
      start += k;
    }
  }
  /* original index of every key in leaf order (keys are distinct) */
  if (rc == SHOCK_ORACLE_OK) {
    for (uint64_t b = 0; b < n_buckets; ++b) {
      for (uint64_t i = bucket_offset[b]; i < bucket_offset[b + 1]; ++i) {
        for (uint64_t g = bucket_offset[b]; g < bucket_offset[b + 1]; ++g)
          if (grouped[g] == leaf_keys[i]) {
            key_index[i] = grouped_idx[g];
            break;
          }
      }
    }
  }
  free(fill);
  free(grouped);
  free(grouped_idx);
  return rc;
}

/* ---- XOR retrieval ---------------------------------------------------------- */

uint64_t shock_oracle_xor_segment(uint64_t n_keys) { return (123 * n_keys + 299) / 300 + 8; }

static void xor_cells(uint64_t x, uint64_t rho, uint64_t seg, uint64_t c[3]) {
  uint64_t u = shock_oracle_fmix64(x ^ shock_oracle_fmix64((rho + 1) * 0xA0761D6478BD642FULL));
  uint64_t v = shock_oracle_fmix64(u);
  c[0] = ((uint64_t)(uint32_t)u * seg) >> 32;
  c[1] = seg + (((u >> 32) * seg) >> 32);
  c[2] = 2 * seg + (((uint64_t)(uint32_t)v * seg) >> 32);
}

int shock_oracle_xor_build(const uint64_t *keys, const uint8_t *values, uint64_t n_keys, uint64_t rho_start,
                           uint32_t max_tries, uint64_t *rho, uint8_t *z) {
  uint64_t seg = shock_oracle_xor_segment(n_keys), m = 3 * seg;
  uint32_t *cnt = (uint32_t *)malloc(sizeof(uint32_t) * m);
  uint32_t *round = (uint32_t *)malloc(sizeof(uint32_t) * (n_keys + 1));
  uint8_t *peel = (uint8_t *)malloc(n_keys + 1);
  if (!cnt || !round || !peel) return SHOCK_ORACLE_EINVAL;
  int rc = SHOCK_ORACLE_ENOTFOUND;
  for (uint32_t t = 0; t < max_tries; ++t) {
    uint64_t r0 = rho_start + t;
    memset(cnt, 0, sizeof(uint32_t) * m);
    for (uint64_t i = 0; i < n_keys; ++i) {
      uint64_t c[3];
      xor_cells(keys[i], r0, seg, c);
      for (int q = 0; q < 3; ++q) cnt[c[q]] += 1;
      round[i] = 0; /* 0: not peeled; r >= 1: peeled in round r */
    }
    uint64_t left = n_keys;
    uint32_t r = 0;
    while (left > 0) {
      ++r;
      uint64_t peeled = 0;
      /* detect on the counts at the start of the round */
      for (uint64_t i = 0; i < n_keys; ++i) {
        if (round[i]) continue;
        uint64_t c[3];
        xor_cells(keys[i], r0, seg, c);
        for (int q = 0; q < 3; ++q)
          if (cnt[c[q]] == 1) {
            round[i] = r;
            peel[i] = (uint8_t)q;
            ++peeled;
            break;
          }
      }
      if (peeled == 0) break;
      /* then remove them */
      for (uint64_t i = 0; i < n_keys; ++i) {
        if (round[i] != r) continue;
        uint64_t c[3];
        xor_cells(keys[i], r0, seg, c);
        for (int q = 0; q < 3; ++q) cnt[c[q]] -= 1;
      }
      left -= peeled;
    }
    if (left > 0) continue;
    /* assignment, rounds in reverse */
    memset(z, 0, m);
    for (uint32_t rr = r; rr >= 1; --rr) {
      for (uint64_t i = 0; i < n_keys; ++i) {
        if (round[i] != rr) continue;
        uint64_t c[3];
        xor_cells(keys[i], r0, seg, c);
        uint8_t acc = values[i] & 1;
        for (int q = 0; q < 3; ++q)
          if (q != peel[i]) acc ^= z[c[q]];
        z[c[peel[i]]] = acc;
      }
    }
    *rho = r0;
    rc = SHOCK_ORACLE_OK;
    break;
  }
  free(cnt);
  free(round);
  free(peel);
  return rc;
}

int shock_oracle_xor_get(const uint64_t *keys, uint64_t n_keys, uint64_t rho, const uint8_t *z, uint8_t *values) {
  uint64_t seg = shock_oracle_xor_segment(n_keys);
  for (uint64_t i = 0; i < n_keys; ++i) {
    uint64_t c[3];
    xor_cells(keys[i], rho, seg, c);
    values[i] = z[c[0]] ^ z[c[1]] ^ z[c[2]];
  }
  return SHOCK_ORACLE_OK;
}

/* ---- ribbon retrieval -------------------------------------------------------- */

int shock_oracle_gf2_solve(const uint64_t *rows_in, const uint8_t *b_in, uint64_t m, uint64_t cols, uint8_t *z) {
  uint64_t W = (cols + 63) / 64;
  uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (m * W + 1));
  uint8_t *b = (uint8_t *)malloc(m + 1);
  uint64_t *pivot_col = (uint64_t *)malloc(sizeof(uint64_t) * (m + 1));
  if (!a || !b || !pivot_col) return -1;
  if (m) {
    memcpy(a, rows_in, sizeof(uint64_t) * m * W);
    memcpy(b, b_in, m);
  }
  /* Gauss-Jordan elimination, columns from 0 up: a column with no remaining
   * row holding it is free; otherwise that row becomes the column's pivot
   * row and the column is cleared from every other row. */
  uint64_t rank = 0;
  for (uint64_t c = 0; c < cols && rank < m; ++c) {
    uint64_t w = c >> 6, bit = 1ULL << (c & 63);
    uint64_t p = rank;
    while (p < m && !(a[p * W + w] & bit)) ++p;
    if (p == m) continue;
    if (p != rank) {
      for (uint64_t q = 0; q < W; ++q) {
        uint64_t t = a[p * W + q];
        a[p * W + q] = a[rank * W + q];
        a[rank * W + q] = t;
      }
      uint8_t t = b[p];
      b[p] = b[rank];
      b[rank] = t;
    }
    for (uint64_t r = 0; r < m; ++r) {
      if (r == rank || !(a[r * W + w] & bit)) continue;
      for (uint64_t q = 0; q < W; ++q) a[r * W + q] ^= a[rank * W + q];
      b[r] ^= b[rank];
    }
    pivot_col[rank] = c;
    ++rank;
  }
  /* rows beyond the rank are zero: the system is consistent iff their
   * right-hand sides are 0 */
  int ok = 1;
  for (uint64_t r = rank; r < m; ++r)
    if (b[r] & 1) ok = 0;
  if (ok) {
    memset(z, 0, cols);
    for (uint64_t r = 0; r < rank; ++r) z[pivot_col[r]] = b[r] & 1;
  }
  free(a);
  free(b);
  free(pivot_col);
  return ok;
}

uint64_t shock_oracle_ribbon_cols(uint64_t m) {
  if (m == 0) return 0;
  uint64_t c = m + (m + 49) / 50;
  return c < 64 ? 64 : c;
}

void shock_oracle_ribbon_row(uint64_t x, uint32_t rseed, uint64_t cols, uint64_t *start, uint64_t *coef) {
  uint64_t h = shock_oracle_fmix64(x ^ shock_oracle_fmix64(((uint64_t)rseed + 1) * 0x9E6C63D0676A9A99ULL));
  *start = ((h >> 32) * (cols - 63)) >> 32;
  *coef = shock_oracle_fmix64(h) | 1;
}

int shock_oracle_ribbon_build(const uint64_t *keys, const uint8_t *values, uint64_t m, uint32_t max_seeds,
                              uint32_t *rseed, uint8_t *z) {
  if (m == 0) {
    *rseed = 0;
    return SHOCK_ORACLE_OK;
  }
  uint64_t cols = shock_oracle_ribbon_cols(m), W = (cols + 63) / 64;
  uint64_t *rows = (uint64_t *)malloc(sizeof(uint64_t) * m * W);
  if (!rows) return SHOCK_ORACLE_EINVAL;
  int rc = SHOCK_ORACLE_ENOTFOUND;
  for (uint32_t r = 0; r < max_seeds; ++r) {
    memset(rows, 0, sizeof(uint64_t) * m * W);
    for (uint64_t i = 0; i < m; ++i) {
      uint64_t s, c;
      shock_oracle_ribbon_row(keys[i], r, cols, &s, &c);
      for (uint32_t k = 0; k < 64; ++k)
        if ((c >> k) & 1) rows[i * W + ((s + k) >> 6)] |= 1ULL << ((s + k) & 63);
    }
    int ok = shock_oracle_gf2_solve(rows, values, m, cols, z);
    if (ok < 0) {
      rc = SHOCK_ORACLE_EINVAL;
      break;
    }
    if (ok) {
      *rseed = r;
      rc = SHOCK_ORACLE_OK;
      break;
    }
  }
  free(rows);
  return rc;
}

uint8_t shock_oracle_ribbon_get(uint64_t x, uint32_t rseed, uint64_t cols, const uint8_t *z) {
  uint64_t s, c;
  shock_oracle_ribbon_row(x, rseed, cols, &s, &c);
  uint8_t v = 0;
  for (uint32_t k = 0; k < 64; ++k)
    if ((c >> k) & 1) v ^= z[s + k];
  return v;
}

int shock_oracle_mphf_ribbon(const uint64_t *leaf_keys, const uint8_t *values, uint64_t n_buckets,
                             const uint64_t *bucket_offset, uint32_t max_seeds, uint8_t *rseed,
                             uint64_t *bit_offset, uint8_t *z) {
  bit_offset[0] = 0;
  for (uint64_t b = 0; b < n_buckets; ++b)
    bit_offset[b + 1] = bit_offset[b] + shock_oracle_ribbon_cols(bucket_offset[b + 1] - bucket_offset[b]);
  for (uint64_t b = 0; b < n_buckets; ++b) {
    uint64_t o = bucket_offset[b], m = bucket_offset[b + 1] - o;
    uint32_t r = 0;
    int rc = shock_oracle_ribbon_build(leaf_keys + o, values + o, m, max_seeds, &r, z + bit_offset[b]);
    if (rc != SHOCK_ORACLE_OK) return rc;
    rseed[b] = (uint8_t)r;
  }
  return SHOCK_ORACLE_OK;
}

/* The pairs of bipartite seeds in the search order (by max(a, b) = m, then a,
 * then b): for each m, first (a, m) for a = 0 .. m-1, then (m, b) for
 * b = 0 .. m.  The m^2 pairs with a smaller maximum come before them, so the
 * rank of (a, b) is m^2 + a if a < m, else m^2 + m + b. */
uint64_t shock_oracle_bip_pair_rank(uint64_t a, uint64_t b) {
  uint64_t m = a > b ? a : b;
  return m * m + (a < m ? a : m + b);
}

static void bip_pair_of_rank(uint64_t v, uint64_t *a, uint64_t *b) {
  /* m = floor(sqrt(v)): a floating-point estimate, then corrected exactly;
   * m < 2^32 keeps every square below 2^64 */
  uint64_t m = (uint64_t)sqrt((double)v);
  if (m > 0xFFFFFFFFULL) m = 0xFFFFFFFFULL;
  while (m > 0 && m * m > v) --m;
  while (m < 0xFFFFFFFFULL && (m + 1) * (m + 1) <= v) ++m;
  uint64_t r = v - m * m;
  if (r < m) {
    *a = r;
    *b = m;
  } else {
    *a = m;
    *b = r - m;
  }
}

int shock_oracle_mphf_query(const uint64_t *queries, uint64_t n_queries, uint64_t n_keys, uint32_t leaf_target,
                            uint64_t n_buckets, const uint64_t *bucket_offset, const uint64_t *leaf_base,
                            const uint32_t *sigma, const uint8_t *leaf_sizes, const uint64_t *leaf_values,
                            int rf, uint32_t partial_k, int retrieval, uint64_t rho, const uint8_t *rseed,
                            const uint64_t *rbit_offset, const uint8_t *z, uint64_t *out_pos) {
  uint64_t seg = shock_oracle_xor_segment(n_keys);
  for (uint64_t q = 0; q < n_queries; ++q) {
    uint64_t x = queries[q];
    uint64_t b = bucket_of(x, n_buckets);
    uint64_t m = bucket_offset[b + 1] - bucket_offset[b];
    uint32_t L = (uint32_t)((m + leaf_target - 1) / leaf_target);
    if (L == 0) {
      out_pos[q] = UINT64_MAX;
      continue;
    }
    uint32_t j = leaf_of(x, sigma[b], L);
    uint64_t start = bucket_offset[b];
    for (uint32_t jj = 0; jj < j; ++jj) start += leaf_sizes[leaf_base[b] + jj];
    uint32_t n = leaf_sizes[leaf_base[b] + j];
    int f;
    if (retrieval == SHOCK_ORACLE_RETRIEVAL_RIBBON) {
      f = shock_oracle_ribbon_get(x, rseed[b], shock_oracle_ribbon_cols(m), z + rbit_offset[b]);
    } else {
      uint64_t c[3];
      xor_cells(x, rho, seg, c);
      f = z[c[0]] ^ z[c[1]] ^ z[c[2]];
    }
    uint32_t h0 = 0, h1 = 0;
    uint64_t v = leaf_values[leaf_base[b] + j];
    if (rf == 2 && n >= 1) {
      /* bipartite: v is the rank of the pair (a, b) in the search order */
      uint64_t a, bs, l, r;
      bip_pair_of_rank(v, &a, &bs);
      uint32_t cl, cr;
      shock_oracle_bip_slots(x, a, n, &cl, &cr);
      l = cl;
      shock_oracle_bip_slots(x, bs, n, &cl, &cr);
      r = cr;
      h0 = (uint32_t)l;
      h1 = (uint32_t)r;
    } else if (rf == 1 && n >= 2) {
      uint32_t k = partial_k ? partial_k : (n > 32 ? 8u : 1u);
      shock_oracle_rf_slots(x, v / n, (uint32_t)(v % n), k, n, &h0, &h1);
    } else if (n >= 1) {
      shock_oracle_slots(x, v, n, &h0, &h1);
    }
    out_pos[q] = start + (f ? h1 : h0);
  }
  return SHOCK_ORACLE_OK;
}
