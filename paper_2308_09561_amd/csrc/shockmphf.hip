// Flat ShockHash MPHF on MI355X (gfx950): build and query.  Definitions in
// include/shockmphf.h.
//
// Build, all on the device (the host only sizes buffers and reads back a few
// counters):
//   bucket counts (LDS histograms)  ->  one-workgroup scan of bucket sizes,
//   leaf counts and ribbon widths  ->  scatter keys by bucket  ->  per bucket
//   (a wave): the smallest splitting seed whose leaf sizes fit the bucket's
//   5-bit window (leaf histogram in LDS), then leaf sizes, offsets and a
//   scatter into leaf order  ->  per leaf (a wave): bitonic sort of its keys
//   in registers  ->  the leaf search (plain, rotation fitting or bipartite)
//   ->  Golomb-Rice codes of the leaf values, the packed size codes and the
//   16-bucket offset table  ->  the retrieval of each key's choice: by
//   default one ribbon system per bucket, solved by 64-column blocks (two
//   waves per bucket try consecutive seeds; the sequential walk takes any
//   bucket with more rows in a block than a wave holds); optionally a
//   3-hypergraph XOR system peeled in synchronous rounds over frontiers of
//   cells, then assigned rounds in reverse.
// Query: a thread per key: bucket, its block of 16 in the offset table,
// splitting seed, leaf, the leaf's key offset from the 5-bit size codes, its
// value decoded from the Rice streams (the fixed widths of the leaves before
// it in its bucket and a select in the unary stream), the retrieval bit (one
// ribbon row's parity, or three XOR cells), then the leaf's slot.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "shockcode.h"
#include "shockmphf.h"
#include "shock_hash.h"
#include "shock_internal.h"

namespace {

using shockhash::fmix64;
using shockhash::seed_mix;
using shockhash::slot_pair;

constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kBucketKey = 0x5851F42D4C957F2Dull;
constexpr uint64_t kSplitMul = 0xD6E8FEB86659FD93ull;
constexpr uint64_t kRetrievalMul = 0xA0761D6478BD642Full;
constexpr uint32_t kMaxLeavesPerBucket = 1024;
constexpr uint32_t kMaxSigma = 1u << 16;

constexpr uint64_t kErrTooManyLeaves = 1;
constexpr uint64_t kErrSigma = 2;
constexpr uint64_t kErrRibbon = 4;    // a bucket's ribbon system has no seed below kRibbonSeeds
constexpr uint64_t kErrCodeSpan = 8;  // a block of buckets spans 2^32 code bits or more
constexpr uint64_t kErrRibbonInternal = 16;  // internal: a bucket larger than the ribbon launch's LDS, or a walk past its band

// Ribbon retrieval: one GF(2) system per bucket (about 2 % more columns than
// keys, 64-bit coefficient rows), the smallest seed below kRibbonSeeds whose
// system is solvable, and its canonical solution (non-pivot columns 0).
constexpr uint64_t kRibbonMul = 0x9E6C63D0676A9A99ull;
constexpr uint32_t kRibbonSeeds = 256;
constexpr uint32_t kRetrievalRibbon = 0, kRetrievalXor = 1;

// The bucket table: blocks of 16 buckets hold absolute offsets, buckets hold
// 32-bit offsets relative to their block.
constexpr uint32_t kBlockShift = 4;
enum : uint32_t { kBkKey = 0, kBkLeaf, kBkRib, kBkFixed, kBkUnary, kBkWords };

// Leaf sizes are 5-bit codes: a bucket of m keys in L leaves has every leaf
// size in [base, base + 31], base = max(0, floor(m / L) - 16).
__host__ __device__ __forceinline__ uint32_t size_base(uint64_t m, uint32_t L) {
  if (L == 0) return 0;
  const uint64_t mean = m / L;
  return mean > 16 ? (uint32_t)(mean - 16) : 0u;
}
__host__ __device__ __forceinline__ uint64_t ribbon_cols(uint64_t m) {
  if (m == 0) return 0;
  const uint64_t c = m + (m + 49) / 50;
  return c < 64 ? 64 : c;
}
__device__ __forceinline__ uint64_t ribbon_mix(uint32_t rseed) { return fmix64(((uint64_t)rseed + 1) * kRibbonMul); }
// Key x's row: coefficient c (bit 0 set) at columns s .. s + 63 of its bucket's system.
__device__ __forceinline__ void ribbon_row(uint64_t x, uint64_t rmix, uint64_t cols, uint64_t &s, uint64_t &c) {
  const uint64_t h = fmix64(x ^ rmix);
  s = ((h >> 32) * (cols - 63)) >> 32;
  c = fmix64(h) | 1;
}
// 64 bits of a bit array from bit p on (bits past `words` words read as 0).
__device__ __forceinline__ uint64_t bits_at(const uint64_t *v, uint64_t words, uint64_t p) {
  const uint64_t w = p >> 6;
  const uint32_t sh = (uint32_t)(p & 63);
  uint64_t x = w < words ? v[w] >> sh : 0;
  if (sh && w + 1 < words) x |= v[w + 1] << (64 - sh);
  return x;
}
// The 5-bit code of leaf g.
__device__ __forceinline__ uint32_t size_code(const uint64_t *codes, uint64_t g) {
  const uint64_t p = 5 * g, w = p >> 6;
  const uint32_t sh = (uint32_t)(p & 63);
  uint64_t x = codes[w] >> sh;
  if (sh > 59) x |= codes[w + 1] << (64 - sh);
  return (uint32_t)(x & 31);
}
// Sum of the codes of leaves [a, b): per word, bit t is bit (t + 64 w) mod 5
// of its field, so the sum is that of the masked popcounts times their weights.
constexpr uint64_t kField0 = 0x1084210842108421ull;  // bits 0, 5, .., 60
__device__ __forceinline__ uint32_t code_sum(const uint64_t *codes, uint64_t a, uint64_t b) {
  uint32_t sum = 0;
  const uint64_t p0 = 5 * a, p1 = 5 * b;
  for (uint64_t w = p0 >> 6; (w << 6) < p1; ++w) {
    const uint64_t wb = w << 6;
    uint64_t x = codes[w];
    if (wb < p0) x &= ~0ull << (p0 - wb);
    if (p1 - wb < 64) x &= (1ull << (p1 - wb)) - 1;
    const uint32_t ph = (uint32_t)(wb % 5);
#pragma unroll
    for (uint32_t r = 0; r < 5; ++r) sum += (uint32_t)__popcll(x & (kField0 << ((r + 5 - ph) % 5))) << r;
  }
  return sum;
}

struct KTable {
  uint8_t k[65];
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ uint64_t bucket_of(uint64_t x, uint64_t n_buckets) {
  return __umul64hi(fmix64(x ^ kBucketKey), n_buckets);
}
__device__ __forceinline__ uint64_t split_mix(uint32_t sigma) { return fmix64(((uint64_t)sigma + 1) * kSplitMul); }
__device__ __forceinline__ uint32_t leaf_of(uint64_t x, uint64_t tmix, uint32_t n_leaves) {
  return (uint32_t)(((uint64_t)(uint32_t)fmix64(x ^ tmix) * n_leaves) >> 32);
}
__device__ __forceinline__ void xor_cells(uint64_t x, uint64_t rmix, uint64_t seg, uint64_t c[3]) {
  const uint64_t u = fmix64(x ^ rmix);
  const uint64_t v = fmix64(u);
  c[0] = ((u & 0xFFFFFFFFull) * seg) >> 32;
  c[1] = seg + (((u >> 32) * seg) >> 32);
  c[2] = 2 * seg + (((v & 0xFFFFFFFFull) * seg) >> 32);
}

__device__ __forceinline__ uint64_t wave_excl_scan(uint64_t v) {
  const uint32_t lane = lane_id();
  uint64_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  return x - v;
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
__global__ void fill_u64_kernel(unsigned long long *p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}
__global__ void fill_u8_kernel(uint8_t *p, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

// ---- layout -------------------------------------------------------------------

__global__ void bucket_count_kernel(const uint64_t *__restrict__ keys, uint64_t n_keys, uint64_t n_buckets,
                                    uint32_t *counts) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += stride)
    atomicAdd(&counts[bucket_of(keys[i], n_buckets)], 1u);
}

// Exclusive scans of bucket sizes (-> bucket_offset) and leaf counts
// ceil(m / leaf_target) (-> leaf_base), each with the total appended.  One
// workgroup of 1024 threads, 16 buckets per thread and chunk.
__global__ __launch_bounds__(1024) void layout_scan_kernel(const uint32_t *counts, uint64_t n_buckets,
                                                           uint32_t leaf_target, uint64_t *bucket_offset,
                                                           uint64_t *leaf_base, uint64_t *rib_base,
                                                           unsigned long long *err) {
  constexpr uint32_t kPer = 16;
  __shared__ uint64_t wm[16], wl[16], wr[16];
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint64_t carry_m = 0, carry_l = 0, carry_r = 0, most = 0;
  for (uint64_t c = 0; c < n_buckets; c += 1024ull * kPer) {
    const uint64_t b0 = c + (uint64_t)t * kPer;
    uint64_t sm = 0, sl = 0, sr = 0;
    for (uint32_t e = 0; e < kPer; ++e) {
      const uint64_t b = b0 + e;
      if (b < n_buckets) {
        const uint64_t m = counts[b], l = (m + leaf_target - 1) / leaf_target;
        if (l > kMaxLeavesPerBucket) atomicOr(err, kErrTooManyLeaves);
        sm += m;
        sl += l;
        sr += ribbon_cols(m);
        most = m > most ? m : most;
      }
    }
    const uint64_t xm = wave_excl_scan(sm), xl = wave_excl_scan(sl), xr = wave_excl_scan(sr);
    if (lane == 63) {
      wm[wave] = xm + sm;
      wl[wave] = xl + sl;
      wr[wave] = xr + sr;
    }
    __syncthreads();
    uint64_t pm = 0, pl = 0, pr = 0, tm = 0, tl = 0, tr = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      if (w < wave) {
        pm += wm[w];
        pl += wl[w];
        pr += wr[w];
      }
      tm += wm[w];
      tl += wl[w];
      tr += wr[w];
    }
    uint64_t rm = carry_m + pm + xm, rl = carry_l + pl + xl, rr = carry_r + pr + xr;
    for (uint32_t e = 0; e < kPer; ++e) {
      const uint64_t b = b0 + e;
      if (b < n_buckets) {
        const uint64_t m = counts[b];
        bucket_offset[b] = rm;
        leaf_base[b] = rl;
        rib_base[b] = rr;
        rm += m;
        rl += (m + leaf_target - 1) / leaf_target;
        rr += ribbon_cols(m);
      }
    }
    carry_m += tm;
    carry_l += tl;
    carry_r += tr;
    __syncthreads();
  }
  if (most) atomicMax(err + 1, (unsigned long long)most);  // the largest bucket, for the ribbon's LDS
  if (t == 0) {
    bucket_offset[n_buckets] = carry_m;
    leaf_base[n_buckets] = carry_l;
    rib_base[n_buckets] = carry_r;
  }
}

__global__ void bucket_scatter_kernel(const uint64_t *__restrict__ keys, uint64_t n_keys, uint64_t n_buckets,
                                      const uint64_t *__restrict__ bucket_offset, uint32_t *cursor,
                                      uint64_t *__restrict__ grouped) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += stride) {
    const uint64_t x = keys[i];
    const uint64_t b = bucket_of(x, n_buckets);
    grouped[bucket_offset[b] + atomicAdd(&cursor[b], 1u)] = x;
  }
}

// The same two passes with per-workgroup histograms in LDS, for tables of up
// to kLdsBuckets buckets: a workgroup takes kLayoutChunk consecutive keys,
// counts them per bucket in LDS, and makes one global atomic per bucket it
// saw (a bucket's counter otherwise takes one atomic per key, serialised
// across the whole launch).  Within a bucket the keys' order is arbitrary in
// both forms (each leaf is sorted later).
constexpr uint32_t kLdsBuckets = 8192;
constexpr uint32_t kLayoutChunk = 256 * 32;

__global__ __launch_bounds__(256) void bucket_count_lds_kernel(const uint64_t *__restrict__ keys, uint64_t n_keys,
                                                               uint64_t n_buckets, uint32_t *counts) {
  __shared__ uint32_t h[kLdsBuckets];
  for (uint32_t i = threadIdx.x; i < n_buckets; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kLayoutChunk;
  const uint64_t c1 = c0 + kLayoutChunk < n_keys ? c0 + kLayoutChunk : n_keys;
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) atomicAdd(&h[bucket_of(keys[i], n_buckets)], 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n_buckets; i += blockDim.x)
    if (h[i]) atomicAdd(&counts[i], h[i]);
}

__global__ __launch_bounds__(256) void bucket_scatter_lds_kernel(const uint64_t *__restrict__ keys, uint64_t n_keys,
                                                                 uint64_t n_buckets,
                                                                 const uint64_t *__restrict__ bucket_offset,
                                                                 uint32_t *cursor, uint64_t *__restrict__ grouped) {
  __shared__ uint32_t h[kLdsBuckets];
  for (uint32_t i = threadIdx.x; i < n_buckets; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kLayoutChunk;
  const uint64_t c1 = c0 + kLayoutChunk < n_keys ? c0 + kLayoutChunk : n_keys;
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) atomicAdd(&h[bucket_of(keys[i], n_buckets)], 1u);
  __syncthreads();
  // reserve each bucket's range: h[b] becomes the first slot of this chunk's keys
  for (uint32_t i = threadIdx.x; i < n_buckets; i += blockDim.x)
    if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
  __syncthreads();
  for (uint64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
    const uint64_t x = keys[i];
    const uint64_t b = bucket_of(x, n_buckets);
    grouped[bucket_offset[b] + atomicAdd(&h[b], 1u)] = x;
  }
}

// One wave per bucket: the smallest splitting seed whose leaves all fit, then
// leaf sizes, global leaf key offsets, and the keys scattered into leaf order
// (unsorted within a leaf).
__global__ __launch_bounds__(256) void split_kernel(const uint64_t *__restrict__ grouped,
                                                    const uint64_t *__restrict__ bucket_offset,
                                                    const uint64_t *__restrict__ leaf_base, uint64_t n_buckets,
                                                    uint32_t leaf_max, uint16_t *sigma, uint8_t *leaf_sizes,
                                                    uint8_t *leaf_codes, uint64_t *leaf_off,
                                                    uint64_t *__restrict__ leaf_keys, unsigned long long *err) {
  __shared__ uint32_t bins_all[4][kMaxLeavesPerBucket];
  const uint32_t lane = lane_id();
  uint32_t *bins = bins_all[threadIdx.x >> 6];
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < n_buckets; b += waves) {
    const uint64_t o = bucket_offset[b], m = bucket_offset[b + 1] - o;
    const uint64_t lb = leaf_base[b];
    const uint32_t L = (uint32_t)(leaf_base[b + 1] - lb);
    if (L == 0) {
      if (lane == 0) sigma[b] = 0;
      continue;
    }
    if (L > kMaxLeavesPerBucket) continue;  // flagged by the scan
    // the smallest seed whose leaf sizes all lie in [lo, lo + 31] and at most leaf_max
    const uint32_t lo = size_base(m, L), hi = lo + 31 < leaf_max ? lo + 31 : leaf_max;
    uint32_t s = 0;
    bool found = false;
    for (; s < kMaxSigma; ++s) {
      const uint64_t tm = split_mix(s);
      for (uint32_t j = lane; j < L; j += 64) bins[j] = 0;
      wave_sync();
      bool over = false;
      for (uint64_t i = lane; i < m; i += 64) {
        const uint32_t c = atomicAdd(&bins[leaf_of(grouped[o + i], tm, L)], 1u) + 1;
        over |= c > hi;
      }
      wave_sync();
      for (uint32_t j = lane; j < L; j += 64) over |= bins[j] < lo;
      if (__ballot(over) == 0) {
        found = true;
        break;
      }
    }
    if (!found) {
      // the build fails; its leaves are still written (empty, at the bucket's
      // start), so the sort queued behind this kernel reads no stale offsets
      for (uint32_t j = lane; j < L; j += 64) {
        leaf_sizes[lb + j] = 0;
        leaf_codes[lb + j] = 0;
        leaf_off[lb + j] = o;
      }
      if (lane == 0) {
        sigma[b] = 0;
        atomicOr(err, kErrSigma);
      }
      continue;
    }
    if (lane == 0) sigma[b] = (uint16_t)s;
    // sizes -> exclusive starts (in place), chunk by chunk of 64 leaves
    uint64_t carry = 0;
    for (uint32_t j0 = 0; j0 < L; j0 += 64) {
      const uint32_t j = j0 + lane;
      const uint32_t sz = j < L ? bins[j] : 0;
      const uint64_t start = carry + wave_excl_scan(sz);
      if (j < L) {
        leaf_sizes[lb + j] = (uint8_t)sz;
        leaf_codes[lb + j] = (uint8_t)(sz - lo);
        leaf_off[lb + j] = o + start;
        bins[j] = (uint32_t)start;
      }
      carry = __shfl(start + sz, 63);  // start already includes the carry
    }
    wave_sync();
    const uint64_t tm = split_mix(s);
    for (uint64_t i = lane; i < m; i += 64) {
      const uint64_t x = grouped[o + i];
      leaf_keys[o + atomicAdd(&bins[leaf_of(x, tm, L)], 1u)] = x;
    }
    wave_sync();
  }
}

// One wave per leaf: sort its keys ascending (bitonic network over the 64
// lanes; lanes beyond the leaf hold the largest value and stay at the end).
__global__ __launch_bounds__(256) void leaf_sort_kernel(uint64_t *keys, const uint64_t *__restrict__ leaf_off,
                                                        const uint8_t *__restrict__ leaf_sizes, uint64_t n_leaves) {
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t g = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g < n_leaves; g += waves) {
    const uint64_t o = leaf_off[g];
    const uint32_t n = leaf_sizes[g];
    uint64_t v = lane < n ? keys[o + lane] : kNone;
    for (uint32_t k = 2; k <= 64; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        const uint64_t w = __shfl_xor(v, j);
        const bool up = (lane & k) == 0;
        const bool lower = (lane & j) == 0;
        const uint64_t lo = v < w ? v : w, hi = v < w ? w : v;
        v = (lower == up) ? lo : hi;
      }
    }
    if (lane < n) keys[o + lane] = v;
  }
}

// Rotation fitting: a leaf's stored value is its candidate index s * n + r.
// Leaf kinds (shock_mphf::rf).
constexpr uint32_t kLeafPlain = 0, kLeafRf = 1, kLeafBip = 2;

// Bipartite leaves: the rank of the seed pair (a, b) in the search's order
// (by m = max(a, b), then a, then b): m^2 pairs precede maximum m, then
// (0, m) .. (m - 1, m), then (m, 0) .. (m, m).
__global__ void bip_values_kernel(const uint64_t *__restrict__ pa, const uint64_t *__restrict__ pb, uint64_t *values,
                                  uint64_t n_leaves) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_leaves; g += stride) {
    const uint64_t a = pa[g], b = pb[g];
    if (a == kNone || b == kNone) {
      values[g] = kNone;
      continue;
    }
    const uint64_t m = a > b ? a : b;
    values[g] = m * m + (a < m ? a : m + b);
  }
}

// The pair (a, b) of rank v: m = floor(sqrt(v)) (a double estimate, within
// one of the root, corrected to the exact integer root; m stays below 2^32,
// so no square overflows), r = v - m^2.
__device__ __forceinline__ void bip_pair_of(uint64_t v, uint64_t &a, uint64_t &b) {
  constexpr uint64_t kMaxRoot = 0xFFFFFFFFull;
  uint64_t m = (uint64_t)sqrt((double)v);
  if (m > kMaxRoot) m = kMaxRoot;
  while (m > 0 && m * m > v) --m;
  while (m < kMaxRoot && (m + 1) * (m + 1) <= v) ++m;
  const uint64_t r = v - m * m;
  a = r < m ? r : m;
  b = r < m ? m : r - m;
}

__global__ void rf_values_kernel(uint64_t *seeds, const uint32_t *__restrict__ rot,
                                 const uint8_t *__restrict__ leaf_sizes, uint64_t n_leaves) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_leaves; g += stride) {
    const uint32_t n = leaf_sizes[g];
    if (n >= 2 && seeds[g] != kNone) seeds[g] = seeds[g] * n + rot[g];
  }
}

// ---- retrieval ------------------------------------------------------------------

__global__ void choice_kernel(const uint64_t *__restrict__ leaf_off, const uint8_t *__restrict__ leaf_sizes,
                              const uint64_t *__restrict__ orient, uint64_t n_leaves, uint8_t *choice) {
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t g = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g < n_leaves; g += waves)
    if (lane < leaf_sizes[g]) choice[leaf_off[g] + lane] = (uint8_t)((orient[g] >> lane) & 1);
}

// ---- the stored tables ------------------------------------------------------------

// 5-bit size codes packed 64 bits a word: leaf g at bits 5g .. 5g + 4.
__global__ void pack_codes_kernel(const uint8_t *__restrict__ codes8, uint64_t n_leaves, uint64_t words,
                                  uint64_t *codes) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    uint64_t v = 0;
    const uint64_t p0 = w * 64;
    for (uint64_t g = p0 / 5; g < n_leaves && 5 * g < p0 + 64; ++g) {
      const uint64_t c = codes8[g] & 31, p = 5 * g;
      v |= p >= p0 ? c << (p - p0) : c >> (p0 - p);
    }
    codes[w] = v;
  }
}

// Code offsets of every bucket's first leaf (b in [0, B], entry B = the end):
// from the Rice encoder's index of blocks of 64 leaves, plus the fixed widths
// and unary lengths of the leaves before it in its block.
__global__ void rice_bucket_kernel(const uint64_t *__restrict__ leaf_base, uint64_t n_buckets,
                                   const uint64_t *__restrict__ index, const uint8_t *__restrict__ leaf_sizes,
                                   const uint64_t *__restrict__ values, KTable K, uint64_t *fixed_at,
                                   uint64_t *unary_at) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= n_buckets; b += stride) {
    const uint64_t g0 = leaf_base[b], blk = g0 >> 6;
    uint64_t F = index[2 * blk], U = index[2 * blk + 1];
    for (uint64_t g = blk * 64; g < g0; ++g) {
      const uint32_t k = K.k[leaf_sizes[g]];
      F += k;
      U += (values[g] >> k) + 1;
    }
    fixed_at[b] = F;
    unary_at[b] = U;
  }
}

// The bucket table: per block of 16 buckets the absolute key, leaf, ribbon,
// fixed-code and unary-code offsets of its first bucket; per bucket its key,
// fixed and unary offsets relative to its block (b in [0, B]; the key offset
// of entry B closes the last bucket).
__global__ void bucket_table_kernel(const uint64_t *__restrict__ bucket_offset, const uint64_t *__restrict__ leaf_base,
                                    const uint64_t *__restrict__ rib_base, const uint64_t *__restrict__ fixed_at,
                                    const uint64_t *__restrict__ unary_at, uint64_t n_buckets, uint64_t *block,
                                    uint32_t *key_rel, uint32_t *fixed_rel, uint32_t *unary_rel,
                                    unsigned long long *err) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= n_buckets; b += stride) {
    const uint64_t b0 = b & ~((1ull << kBlockShift) - 1);
    if (b == b0) {
      uint64_t *e = block + (b >> kBlockShift) * kBkWords;
      e[kBkKey] = bucket_offset[b];
      e[kBkLeaf] = leaf_base[b];
      e[kBkRib] = rib_base[b];
      e[kBkFixed] = fixed_at[b];
      e[kBkUnary] = unary_at[b];
    }
    key_rel[b] = (uint32_t)(bucket_offset[b] - bucket_offset[b0]);
    const uint64_t df = fixed_at[b] - fixed_at[b0], du = unary_at[b] - unary_at[b0];
    if (bucket_offset[b] - bucket_offset[b0] > 0xFFFFFFFFull || df > 0xFFFFFFFFull || du > 0xFFFFFFFFull)
      atomicOr(err, kErrCodeSpan);
    if (b < n_buckets) {
      fixed_rel[b] = (uint32_t)df;
      unary_rel[b] = (uint32_t)du;
    }
  }
}

// ---- ribbon retrieval ----------------------------------------------------------------

// One wave per bucket.  The wave hashes 64 keys at a time; then every lane
// runs the same insertion walk on wave-uniform values (scalar registers,
// broadcast LDS reads), so the walk has no divergent control flow.  A row is
// stored at its lowest column; a row meeting a stored row there takes their
// sum and moves on to its next set column; a row that vanishes contradicts
// the system unless its value vanished too.  Seeds are tried from 0 until
// none contradicts.  The stored rows are an echelon basis of the row space,
// so their leading columns are the pivot columns of the reduced row echelon
// form; back substitution from the last column sets each pivot column and
// leaves the others 0: the canonical solution.  The wave then writes the
// bits at the bucket's offset (words shared with the neighbours by atomic OR
// into the zeroed array).  Slots, values and the solution live in LDS (kLds)
// or in a global region per bucket.  With `only`, just the buckets it marks.
// The readlane builtins return int: each half is taken as uint32_t before it
// is widened, so the low half is never sign-extended into the high one.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t lane64(uint64_t x, uint32_t q) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(x >> 32), q);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)x, q);
  return ((uint64_t)hi << 32) | lo;
}

template <bool kLds>
__global__ __launch_bounds__(64) void ribbon_kernel(const uint64_t *__restrict__ keys,
                                                    const uint8_t *__restrict__ choice,
                                                    const uint64_t *__restrict__ bucket_offset,
                                                    const uint64_t *__restrict__ rib_base, uint64_t n_buckets,
                                                    uint64_t *slots_global, uint64_t lds_cap_words,
                                                    uint64_t *zbits, uint64_t zwords, uint8_t *rseed,
                                                    const uint8_t *__restrict__ only, unsigned long long *err) {
  extern __shared__ uint64_t lds_words[];
  const uint32_t lane = lane_id();
  for (uint64_t b = blockIdx.x; b < n_buckets; b += gridDim.x) {
    if (only && !only[b]) continue;
    const uint64_t o = bucket_offset[b], m = bucket_offset[b + 1] - o;
    if (m == 0) {
      if (lane == 0) rseed[b] = 0;
      continue;
    }
    const uint64_t cols = ribbon_cols(m), W = (cols + 63) / 64, rb = rib_base[b];
    // slots (cols words), their values (cols bytes, as cols / 8 + 1 words) and the solution (W + 1 words)
    const uint64_t need = cols + cols / 8 + 1 + W + 1;
    if (kLds && need > lds_cap_words) {  // the launch was sized for a smaller bucket
      if (lane == 0) atomicOr(err, kErrRibbonInternal);
      continue;
    }
    // a global region per bucket of at most 1.16 cols + 3 words: rb + (rb >> 3) + 3 b + 2 floor(rb / 64)
    uint64_t *coef = kLds ? lds_words : slots_global + rb + (rb >> 3) + 3 * b + 2 * (rb >> 6);
    uint8_t *val = reinterpret_cast<uint8_t *>(coef + cols);
    uint64_t *sol = coef + cols + cols / 8 + 1;
    uint32_t found = kRibbonSeeds;
    for (uint32_t r = 0; r < kRibbonSeeds; ++r) {
      for (uint64_t i = lane; i < cols; i += 64) coef[i] = 0;
      for (uint64_t i = lane; i < W + 1; i += 64) sol[i] = 0;
      __builtin_amdgcn_s_waitcnt(0);
      wave_sync();
      bool ok = true;
      const uint64_t rmix = ribbon_mix(r);
      for (uint64_t i0 = 0; i0 < m && ok; i0 += 64) {
        const uint64_t il = i0 + lane;
        uint64_t sl = 0, cl = 0;
        if (il < m) ribbon_row(keys[o + il], rmix, cols, sl, cl);
        const uint32_t vl = il < m ? (choice[o + il] & 1u) : 0u;
        const uint32_t cnt = m - i0 < 64 ? (uint32_t)(m - i0) : 64u;
        for (uint32_t q = 0; q < cnt && ok; ++q) {
          uint64_t s = (uint32_t)__builtin_amdgcn_readlane((uint32_t)sl, q);  // s <= cols - 64
          uint64_t c = lane64(cl, q);
          uint32_t v = (uint32_t)__builtin_amdgcn_readlane(vl, q) & 1u;
          for (;;) {
            // The row's bits stay within its start's 64 columns, so s < cols
            // always; the bound makes the walk end whatever the slots hold.
            if (s >= cols) {
              if (lane == 0) atomicOr(err, kErrRibbonInternal);
              ok = false;
              break;
            }
            const uint64_t e = uniform64(coef[s]);
            const uint32_t ev = (uint32_t)__builtin_amdgcn_readfirstlane(val[s]) & 1u;
            if (e == 0) {
              if (lane == 0) {
                coef[s] = c;
                val[s] = (uint8_t)v;
              }
              break;
            }
            c ^= e;
            v ^= ev;
            if (c == 0) {
              ok = v == 0;
              break;
            }
            if (c & 1) {  // a stored row always holds its lowest column: s then rises every step
              if (lane == 0) atomicOr(err, kErrRibbonInternal);
              ok = false;
              break;
            }
            const uint32_t tz = (uint32_t)__builtin_ctzll(c);
            c >>= tz;
            s += tz;
          }
        }
      }
      if (ok) {
        // back substitution: win holds z[s + 1 ..] while column s is solved;
        // the bits of one solution word are gathered before it is stored
        uint64_t win = 0, word = 0;
        for (uint64_t s = cols; s-- > 0;) {
          const uint64_t e = uniform64(coef[s]);
          uint64_t z = 0;
          if (e) z = ((uint32_t)__builtin_amdgcn_readfirstlane(val[s]) ^ (uint64_t)__popcll((e >> 1) & win)) & 1;
          win = (win << 1) | z;
          word |= z << (s & 63);
          if ((s & 63) == 0) {
            if (lane == 0) sol[s >> 6] = word;
            word = 0;
          }
        }
        found = r;
      }
      __builtin_amdgcn_s_waitcnt(0);
      wave_sync();
      if (ok) break;
    }
    if (found == kRibbonSeeds) {
      if (lane == 0) atomicOr(err, kErrRibbon);
      continue;
    }
    if (lane == 0) rseed[b] = (uint8_t)found;
    // write bits [rb, rb + cols) of the global array
    const uint64_t w0 = rb >> 6, w1 = (rb + cols - 1) >> 6;
    for (uint64_t w = w0 + lane; w <= w1 && w < zwords; w += 64) {
      const uint64_t gb = w << 6;
      uint64_t x;
      if (gb >= rb) {
        x = bits_at(sol, W, gb - rb);
      } else {
        x = sol[0] << (rb - gb);
      }
      if (gb + 64 <= rb + cols) {  // the word's bits past the bucket's end are 0 here
        if (gb >= rb) {
          zbits[w] = x;
        } else {
          atomicOr((unsigned long long *)&zbits[w], (unsigned long long)x);
        }
      } else {
        x &= (1ull << (rb + cols - gb)) - 1;
        atomicOr((unsigned long long *)&zbits[w], (unsigned long long)x);
      }
    }
  }
}

// Ribbon retrieval by column blocks: the systems, seeds and solutions of
// ribbon_kernel with few dependent memory round trips.  Each seed's rows are
// sorted by the 64-column block of their start (a counting sort of key
// indices in LDS).  A wave holds the rows that can have a set bit in the
// current block, each as a 128-bit window over that block and the next, up to
// kRowSlots rows per lane.  A row starting in the block reaches at most
// column 126 of the window and a row left from the block before at most 62,
// so bit 127 is free and carries the row's value, which every row sum then
// adds along.  For each column j of the block, in order, a ballot finds the
// rows whose lowest set bit is j (earlier columns are already clear in every
// row); the first of them is the column's pivot and is added to all of them,
// itself included, which clears column j everywhere.  A row that vanishes with
// value 1 contradicts the system.  After the block the surviving rows move 64
// columns on and are compacted in LDS with the rows that start in the next
// block.  The pivots' columns are the leading columns of an echelon form,
// hence the pivot columns of the system, so back substitution over the stored
// pivot rows with the other columns 0 gives the canonical solution; a seed is
// solvable here exactly when it is for the walk.  The kS waves of a workgroup
// try kS consecutive seeds of one bucket at once and the smallest that solves
// wins.  A bucket with more rows in a block than a wave holds (row_cap) is
// marked in `spill` for the walk.
//
// Two launches.  The first tries seeds 0 and 1 of every bucket (about three
// buckets in four end there) and lists the others; the second takes the
// listed buckets from seed 2 on, with as many waves per bucket as the LDS
// holds.  One launch of two waves per bucket took as long as its slowest
// bucket's rounds of two seeds (seeds up to 11 on 1399 buckets), with most
// SIMDs idle after the first round.
constexpr uint32_t kRowSlots = 4;
constexpr uint32_t kRowCapMax = 64 * kRowSlots;
constexpr uint64_t kBlockMaxM = 16384;        // larger buckets: the walk
constexpr uint64_t kErrRibbonSpill = 32;      // buckets marked for the walk
constexpr uint32_t kRibWaves = 2;             // seeds tried at once per bucket, first launch
constexpr uint64_t kValueBit = 1ull << 63;    // of a row's high word
enum : uint32_t { kTryContradiction = 0, kTrySolved = 1, kTrySpill = 2 };

__host__ __device__ __forceinline__ uint64_t rib_blocks(uint64_t m) { return (ribbon_cols(m) + 63) / 64; }
// LDS per wave for buckets of up to max_m keys: the row stage (low and high
// words), block starts and cursors (u32, W + 1 each), the sorted key indices
// (u16).
__host__ __device__ __forceinline__ uint32_t rib_lds_wave_bytes(uint64_t max_m) {
  const uint64_t b = (uint64_t)kRowCapMax * 16 + 8 * (rib_blocks(max_m) + 2) + 2 * max_m;
  return (uint32_t)((b + 15) & ~15ull);
}
// Global scratch per wave: every column's pivot row (low and high words).
__host__ __device__ __forceinline__ uint64_t rib_piv_wave_bytes(uint64_t max_m) {
  return ((16 * 64 * rib_blocks(max_m) + 255) / 256) * 256;
}
__device__ __forceinline__ uint32_t ribbon_start(uint64_t x, uint64_t rmix, uint64_t cols) {
  return (uint32_t)(((fmix64(x ^ rmix) >> 32) * (cols - 63)) >> 32);
}
// Columns 32 h .. 32 h + 31 of one block on NS row slots; lane j keeps column
// j's pivot row.
template <uint32_t NS, uint32_t h>
__device__ __forceinline__ void rib_half(uint64_t (&lo)[kRowSlots], uint64_t (&hi)[kRowSlots], uint64_t &plo,
                                         uint64_t &phi) {
  const uint32_t lane = lane_id();
  for (uint32_t jj = 0; jj < 32; ++jj) {
    bool bit[NS];
    uint64_t bm[NS], any = 0;
#pragma unroll
    for (uint32_t k = 0; k < NS; ++k) {
      bit[k] = (int32_t)((uint32_t)(lo[k] >> (32 * h)) << (31 - jj)) < 0;
      bm[k] = __ballot(bit[k]);
      any |= bm[k];
    }
    if (!any) continue;  // no row has this column: not a pivot column
    uint64_t Plo, Phi;
    if (bm[0]) {
      const uint32_t ls = (uint32_t)__builtin_ctzll(bm[0]);
      Plo = lane64(lo[0], ls);
      Phi = lane64(hi[0], ls);
    } else if (NS > 1 && bm[NS > 1 ? 1 : 0]) {
      const uint32_t ls = (uint32_t)__builtin_ctzll(bm[NS > 1 ? 1 : 0]);
      Plo = lane64(lo[NS > 1 ? 1 : 0], ls);
      Phi = lane64(hi[NS > 1 ? 1 : 0], ls);
    } else if (NS > 2 && bm[NS > 2 ? 2 : 0]) {
      const uint32_t ls = (uint32_t)__builtin_ctzll(bm[NS > 2 ? 2 : 0]);
      Plo = lane64(lo[NS > 2 ? 2 : 0], ls);
      Phi = lane64(hi[NS > 2 ? 2 : 0], ls);
    } else {
      const uint32_t ls = (uint32_t)__builtin_ctzll(bm[NS - 1]);
      Plo = lane64(lo[NS - 1], ls);
      Phi = lane64(hi[NS - 1], ls);
    }
    // lane j takes the pivot row; the rows with column j set take the sum.
    // The empty asm keeps these as lane-masked moves and sums instead of
    // selects, which cost a second instruction per word.
    if (lane == 32 * h + jj) {
      asm volatile("");
      plo = Plo;
      phi = Phi;
    }
#pragma unroll
    for (uint32_t k = 0; k < NS; ++k)
      if (bit[k]) {
        asm volatile("");
        lo[k] ^= Plo;
        hi[k] ^= Phi;
      }
  }
}

template <uint32_t NS>
__device__ __forceinline__ void rib_columns(uint64_t (&lo)[kRowSlots], uint64_t (&hi)[kRowSlots], uint64_t &plo,
                                            uint64_t &phi) {
  rib_half<NS, 0>(lo, hi, plo, phi);
  rib_half<NS, 1>(lo, hi, plo, phi);
}

// One seed's elimination; the pivot rows go to plo_g / phi_g.
__device__ uint32_t rib_try(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ choice, uint64_t o,
                           uint32_t m, uint64_t cols, uint32_t W, uint64_t rmix, uint32_t row_cap, uint64_t *st_lo,
                           uint64_t *st_hi, uint32_t *cnt, uint32_t *cur, uint16_t *idx, uint64_t *plo_g,
                           uint64_t *phi_g, unsigned long long *err) {
  const uint32_t lane = lane_id();
  // counting sort of the key indices by start block: cnt[k] = rows starting before block k
  for (uint32_t k = lane; k <= W; k += 64) cnt[k] = 0;
  wave_sync();
  for (uint32_t i = lane; i < m; i += 64) atomicAdd(&cnt[(ribbon_start(keys[o + i], rmix, cols) >> 6) + 1], 1u);
  wave_sync();
  uint32_t carry = 0;
  for (uint32_t k0 = 0; k0 <= W; k0 += 64) {
    const uint32_t k = k0 + lane;
    uint32_t x = k <= W ? cnt[k] : 0u;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= (uint32_t)d) x += y;
    }
    x += carry;
    if (k <= W) {
      cnt[k] = x;
      cur[k] = x;
    }
    carry = __shfl(x, 63);
  }
  wave_sync();
  for (uint32_t i = lane; i < m; i += 64) {
    const uint32_t p = atomicAdd(&cur[ribbon_start(keys[o + i], rmix, cols) >> 6], 1u);
    idx[p] = (uint16_t)i;
  }
  wave_sync();
  uint64_t lo[kRowSlots], hi[kRowSlots];
  uint32_t nslot = 0;
#pragma unroll
  for (uint32_t k = 0; k < kRowSlots; ++k) lo[k] = hi[k] = 0;
  for (uint32_t blk = 0; blk <= W; ++blk) {
    // the rows left from the previous block move on 64 columns; one that
    // vanished with value 1 contradicts the system
    uint32_t live = 0;
    bool bad = false, stray = false;
#pragma unroll
    for (uint32_t k = 0; k < kRowSlots; ++k) {
      if (k < nslot) {
        stray |= lo[k] != 0;
        const bool alive = (hi[k] & ~kValueBit) != 0;
        bad |= !alive && (hi[k] & kValueBit);
        const uint64_t am = __ballot(alive);
        if (alive) {
          const uint32_t p = live + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(am >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)am, 0u));
          st_lo[p] = hi[k] & ~kValueBit;
          st_hi[p] = hi[k] & kValueBit;
        }
        live += (uint32_t)__popcll(am);
      }
    }
    if (__ballot(stray)) {  // every column of the block was cleared: cannot happen
      if (lane == 0) atomicOr(err, kErrRibbonInternal);
      return kTryContradiction;
    }
    if (__ballot(bad)) return kTryContradiction;
    if (blk == W) {
      if (live) {  // rows past the last column: cannot happen
        if (lane == 0) atomicOr(err, kErrRibbonInternal);
        return kTryContradiction;
      }
      return kTrySolved;
    }
    // with the rows that start in this block
    const uint32_t a0 = cnt[blk], a1 = cnt[blk + 1];
    const uint32_t total = live + (a1 - a0);
    if (total > row_cap) return kTrySpill;
    for (uint32_t t = lane; t < a1 - a0; t += 64) {
      const uint32_t i = idx[a0 + t];
      uint64_t s, c;
      ribbon_row(keys[o + i], rmix, cols, s, c);
      const uint32_t off = (uint32_t)(s & 63);
      st_lo[live + t] = c << off;
      st_hi[live + t] = (off ? c >> (64 - off) : 0) | ((uint64_t)(choice[o + i] & 1) << 63);
    }
    wave_sync();
    nslot = (total + 63) >> 6;
#pragma unroll
    for (uint32_t k = 0; k < kRowSlots; ++k) {
      const uint32_t p = 64 * k + lane;
      const bool in = p < total;
      lo[k] = in ? st_lo[p] : 0;
      hi[k] = in ? st_hi[p] : 0;
    }
    wave_sync();
    uint64_t plo = 0, phi = 0;
    switch (nslot) {
      case 1: rib_columns<1>(lo, hi, plo, phi); break;
      case 2: rib_columns<2>(lo, hi, plo, phi); break;
      case 3: rib_columns<3>(lo, hi, plo, phi); break;
      case 4: rib_columns<4>(lo, hi, plo, phi); break;
      default: break;  // no rows
    }
    plo_g[64 * blk + lane] = plo;
    phi_g[64 * blk + lane] = phi;
  }
  return kTrySolved;  // not reached
}

// Back substitution over one wave's pivot rows, last block first: lane j holds
// column j's row; z of the next block enters through the rows' high words, and
// within the block column j takes its value plus the parity of its row with
// the columns after it.  sol: W words.
__device__ void rib_back(uint32_t W, const uint64_t *plo_g, const uint64_t *phi_g, uint64_t *sol) {
  const uint32_t lane = lane_id();
  uint64_t zn = 0;
  uint64_t nlo = plo_g[64 * (W - 1) + lane], nhi = phi_g[64 * (W - 1) + lane];
  for (int blk = (int)W - 1; blk >= 0; --blk) {
    const uint64_t plo = nlo, phi = nhi;
    if (blk > 0) {
      nlo = plo_g[64 * (blk - 1) + lane];
      nhi = phi_g[64 * (blk - 1) + lane];
    }
    const uint64_t pm = __ballot((plo >> lane) & 1);
    const uint64_t tm = __ballot((((phi >> 63) ^ (uint64_t)__popcll(phi & ~kValueBit & zn)) & 1) != 0);
    uint64_t zc = 0;
    for (uint64_t todo = pm; todo;) {
      const uint32_t j = 63 - (uint32_t)__builtin_clzll(todo);
      todo &= ~(1ull << j);
      const uint64_t row = lane64(plo, j);
      zc |= (((tm >> j) ^ (uint64_t)__popcll(row & zc)) & 1) << j;
    }
    if (lane == 0) sol[blk] = zc;
    zn = zc;
  }
}

template <uint32_t kS>
__global__ __launch_bounds__(64 * kS) void ribbon_block_kernel(
    const uint64_t *__restrict__ keys, const uint8_t *__restrict__ choice, const uint64_t *__restrict__ bucket_offset,
    const uint64_t *__restrict__ rib_base, uint64_t n_items, const uint32_t *__restrict__ list, uint32_t seed0,
    uint32_t *defer, unsigned long long *defer_n, uint8_t *piv, uint64_t piv_wave_bytes, uint32_t lds_wave_bytes,
    uint32_t row_cap, uint64_t *zbits, uint64_t zwords, uint8_t *rseed, uint8_t *spill, unsigned long long *err) {
  // items: buckets 0 .. n_items - 1, or those of `list`; seeds from seed0 on.
  // With `defer`, one round of kS seeds, and a bucket none of them settles is
  // appended to `defer` instead of failing.
  extern __shared__ __align__(16) unsigned char rib_lds[];
  __shared__ uint32_t outcome[kS];
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  unsigned char *lw = rib_lds + (size_t)wave * lds_wave_bytes;
  uint64_t *st_lo = reinterpret_cast<uint64_t *>(lw);
  uint64_t *st_hi = st_lo + kRowCapMax;
  uint32_t *cnt = reinterpret_cast<uint32_t *>(st_hi + kRowCapMax);
  uint8_t *pw = piv + ((uint64_t)blockIdx.x * kS + wave) * piv_wave_bytes;
  const uint32_t seed_end = defer ? seed0 + kS : kRibbonSeeds;
  for (uint64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const uint64_t b = list ? list[it] : it;
    const uint64_t o = bucket_offset[b], m = bucket_offset[b + 1] - o;
    if (m == 0) {
      if (threadIdx.x == 0) rseed[b] = 0;
      continue;
    }
    const uint64_t cols = ribbon_cols(m), rb = rib_base[b];
    const uint32_t W = (uint32_t)rib_blocks(m);
    uint32_t *cur = cnt + W + 1;
    uint16_t *idx = reinterpret_cast<uint16_t *>(cur + W + 1);
    uint64_t *plo_g = reinterpret_cast<uint64_t *>(pw), *phi_g = plo_g + 64 * (uint64_t)W;
    uint32_t win = kRibbonSeeds;
    bool spilled = false;
    for (uint32_t r0 = seed0; r0 < seed_end; r0 += kS) {
      const uint32_t seed = r0 + wave;  // seeds past the last are not tried
      const uint32_t res = seed < kRibbonSeeds ? rib_try(keys, choice, o, (uint32_t)m, cols, W, ribbon_mix(seed),
                                                         row_cap, st_lo, st_hi, cnt, cur, idx, plo_g, phi_g, err)
                                               : kTryContradiction;
      if (lane == 0) outcome[wave] = res;
      __syncthreads();
      uint32_t first = kS;
      bool sp = false;
      for (uint32_t w = 0; w < kS; ++w) {
        const uint32_t x = outcome[w];
        if (x == kTrySolved) {
          first = w;
          break;
        }
        if (x == kTrySpill) {  // a smaller seed's outcome is unknown here
          sp = true;
          break;
        }
      }
      __syncthreads();
      if (first < kS) {
        win = r0 + first;
        break;
      }
      if (sp) {
        spilled = true;
        break;
      }
    }
    if (spilled) {
      if (threadIdx.x == 0) {
        spill[b] = 1;
        atomicOr(err, kErrRibbonSpill);
      }
      continue;
    }
    if (win == kRibbonSeeds) {
      if (threadIdx.x == 0) {
        if (defer) defer[atomicAdd(defer_n, 1ull)] = (uint32_t)b;
        else atomicOr(err, kErrRibbon);
      }
      continue;
    }
    if (wave != (win - seed0) % kS) continue;  // the wave that solved seed win
    uint64_t *sol = st_lo;  // W <= 2 kRowCapMax words of the stage
    rib_back(W, plo_g, phi_g, sol);
    wave_sync();
    if (lane == 0) rseed[b] = (uint8_t)win;
    // bits [rb, rb + cols) of the global array
    const uint64_t w0 = rb >> 6, w1 = (rb + cols - 1) >> 6;
    for (uint64_t w = w0 + lane; w <= w1 && w < zwords; w += 64) {
      const uint64_t gb = w << 6;
      uint64_t x = gb >= rb ? bits_at(sol, W, gb - rb) : sol[0] << (rb - gb);
      if (gb + 64 <= rb + cols) {
        if (gb >= rb) {
          zbits[w] = x;
        } else {
          atomicOr((unsigned long long *)&zbits[w], (unsigned long long)x);
        }
      } else {
        x &= (1ull << (rb + cols - gb)) - 1;
        atomicOr((unsigned long long *)&zbits[w], (unsigned long long)x);
      }
    }
    wave_sync();  // the stage is the next bucket's
  }
}

// Retrieval peeling.  Each cell holds one 64-bit word: the number of keys not
// yet peeled that hash to it (bits 48..63) plus the sum of their indices (bits
// 0..47; a sum of fewer than 2^16 indices below 2^32 never carries into the
// count).  A cell of count one therefore names its key.  Rounds are
// synchronous: every key with a cell of count one at the start of a round is
// peeled in that round, at its first such cell.  The cells that can have count
// one at the start of a round are exactly those whose count fell to one in the
// previous round (the frontier), so a round touches only its frontier and the
// keys it peels.
constexpr uint64_t kCountOne = 1ull << 48;
constexpr uint32_t kMaxPeelRounds = 1u << 14;
enum : int { kPkFrBegin = 0, kPkFrEnd, kPkFrTail, kPkStBegin, kPkStTail, kPkRound, kPkWords };

// Block-wide append: each thread offers cnt slots; returns the index of its
// first one.  One global atomic per call and block (a counter shared by the
// whole grid serialises its atomics, about 12 ns each), so callers batch
// several items per thread.  Every thread of the block must call it.
constexpr uint32_t kAppendThreads = 256;
__device__ __forceinline__ uint64_t block_append(unsigned long long *tail, uint32_t cnt) {
  __shared__ uint32_t wave_sum[kAppendThreads / 64];
  __shared__ unsigned long long base_s;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t x = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wave_sum[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
      const uint32_t t = wave_sum[w];
      wave_sum[w] = tot;
      tot += t;
    }
    base_s = tot ? atomicAdd(tail, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  const uint64_t at = base_s + wave_sum[wave] + x - cnt;
  __syncthreads();  // the shared slots are reused by the next call
  return at;
}

__global__ void xor_count_kernel(const uint64_t *__restrict__ keys, uint64_t n_keys, uint64_t rmix, uint64_t seg,
                                 unsigned long long *cw) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_keys; i += stride) {
    uint64_t c[3];
    xor_cells(keys[i], rmix, seg, c);
    for (int q = 0; q < 3; ++q) atomicAdd(&cw[c[q]], kCountOne + i);
  }
}

// The first frontier: every cell of count one.  A block takes 8 cells per
// thread at a time.
constexpr uint32_t kFrontierPer = 8;
__global__ __launch_bounds__(kAppendThreads) void xor_frontier_kernel(const unsigned long long *__restrict__ cw,
                                                                      uint64_t cells, uint64_t *frontier,
                                                                      unsigned long long *pk) {
  const uint64_t chunk = (uint64_t)blockDim.x * kFrontierPer;
  for (uint64_t c0 = (uint64_t)blockIdx.x * chunk; c0 < cells; c0 += (uint64_t)gridDim.x * chunk) {
    uint32_t ones = 0;
#pragma unroll
    for (uint32_t j = 0; j < kFrontierPer; ++j) {
      const uint64_t c = c0 + (uint64_t)j * blockDim.x + threadIdx.x;
      if (c < cells && (cw[c] >> 48) == 1) ones |= 1u << j;
    }
    uint64_t at = block_append(&pk[kPkFrTail], __popc(ones));
#pragma unroll
    for (uint32_t j = 0; j < kFrontierPer; ++j)
      if ((ones >> j) & 1) {
        if (at < cells) frontier[at] = c0 + (uint64_t)j * blockDim.x + threadIdx.x;
        ++at;
      }
  }
}

// Opens the next round on the frontier appended by the previous one (none if
// it is empty: then the round's passes find nothing to do) and records where
// the previous round's peeled keys end.
__global__ void xor_advance_kernel(unsigned long long *pk, uint64_t *round_off) {
  if (threadIdx.x != 0) return;
  const uint64_t r = pk[kPkRound];
  const uint64_t st = pk[kPkStTail];
  round_off[r] = st;
  pk[kPkStBegin] = st;
  const uint64_t b = pk[kPkFrEnd], e = pk[kPkFrTail];
  pk[kPkFrEnd] = e;
  if (e > b && r < kMaxPeelRounds) {
    pk[kPkFrBegin] = b;
    pk[kPkRound] = r + 1;
  } else {
    pk[kPkFrBegin] = e;
  }
}

// Detect: the key of each frontier cell that still has count one is peeled at
// its first cell of count one (counts are not changed during this pass); a
// bitmap keeps a key that owns two frontier cells from being taken twice.  A
// thread takes up to 4 frontier cells at a time.
constexpr uint32_t kDetectPer = 4;
__global__ __launch_bounds__(kAppendThreads) void xor_detect_kernel(
    const uint64_t *__restrict__ keys, uint64_t n_keys, uint64_t rmix, uint64_t seg,
    const unsigned long long *__restrict__ cw, const uint64_t *__restrict__ frontier, uint64_t cells,
    uint32_t *taken, uint8_t *peel, uint32_t *stack, unsigned long long *pk) {
  // Ranges are clamped to the arrays (they always fit: a cell joins a frontier
  // at most once and a key is peeled at most once).
  const uint64_t e = pk[kPkFrEnd] < cells ? pk[kPkFrEnd] : cells;
  const uint64_t b = pk[kPkFrBegin] < e ? pk[kPkFrBegin] : e;
  const uint64_t chunk = (uint64_t)blockDim.x * kDetectPer;
  for (uint64_t k0 = b + (uint64_t)blockIdx.x * chunk; k0 < e; k0 += (uint64_t)gridDim.x * chunk) {
    uint32_t mine[kDetectPer];
    uint32_t got = 0;
#pragma unroll
    for (uint32_t j = 0; j < kDetectPer; ++j) {
      mine[j] = 0;
      const uint64_t k = k0 + (uint64_t)j * blockDim.x + threadIdx.x;
      if (k >= e) continue;
      const uint64_t w = cw[frontier[k]];
      const uint64_t i = w & (kCountOne - 1);
      if ((w >> 48) != 1 || i >= n_keys) continue;
      const uint32_t bit = 1u << (i & 31);
      if (atomicOr(&taken[i >> 5], bit) & bit) continue;
      uint64_t c[3];
      xor_cells(keys[i], rmix, seg, c);
      uint32_t q = 0;
      while (q < 2 && (cw[c[q]] >> 48) != 1) ++q;
      peel[i] = (uint8_t)q;
      mine[j] = (uint32_t)i;
      got |= 1u << j;
    }
    uint64_t at = block_append(&pk[kPkStTail], __popc(got));
#pragma unroll
    for (uint32_t j = 0; j < kDetectPer; ++j)
      if ((got >> j) & 1) {
        if (at < n_keys) stack[at] = mine[j];
        ++at;
      }
  }
}

// Remove the round's keys; a cell whose count falls from two to one joins the
// next frontier.  A thread takes up to 2 keys at a time.
constexpr uint32_t kRemovePer = 2;
__global__ __launch_bounds__(kAppendThreads) void xor_remove_kernel(
    const uint64_t *__restrict__ keys, uint64_t n_keys, uint64_t rmix, uint64_t seg, unsigned long long *cw,
    const uint32_t *__restrict__ stack, uint64_t *frontier, uint64_t cells, unsigned long long *pk) {
  const uint64_t e = pk[kPkStTail] < n_keys ? pk[kPkStTail] : n_keys;
  const uint64_t b = pk[kPkStBegin] < e ? pk[kPkStBegin] : e;
  const uint64_t chunk = (uint64_t)blockDim.x * kRemovePer;
  for (uint64_t k0 = b + (uint64_t)blockIdx.x * chunk; k0 < e; k0 += (uint64_t)gridDim.x * chunk) {
    uint64_t cell[3 * kRemovePer];
    uint32_t fell = 0;
#pragma unroll
    for (uint32_t j = 0; j < kRemovePer; ++j) {
      const uint64_t k = k0 + (uint64_t)j * blockDim.x + threadIdx.x;
      cell[3 * j] = cell[3 * j + 1] = cell[3 * j + 2] = 0;
      if (k >= e) continue;
      const uint32_t i = stack[k];
      xor_cells(keys[i], rmix, seg, &cell[3 * j]);
#pragma unroll
      for (uint32_t q = 0; q < 3; ++q)
        if ((atomicSub(&cw[cell[3 * j + q]], kCountOne + i) >> 48) == 2) fell |= 1u << (3 * j + q);
    }
    uint64_t at = block_append(&pk[kPkFrTail], __popc(fell));
#pragma unroll
    for (uint32_t j = 0; j < 3 * kRemovePer; ++j)
      if ((fell >> j) & 1) {
        if (at < cells) frontier[at] = cell[j];
        ++at;
      }
  }
}

// Assignment of one round's keys (keys of a round write distinct cells and read
// none written in that round).
__global__ void xor_assign_kernel(const uint64_t *__restrict__ keys, uint64_t rmix, uint64_t seg,
                                  const uint32_t *__restrict__ stack, uint64_t begin, uint64_t end,
                                  const uint8_t *__restrict__ peel, const uint8_t *__restrict__ choice, uint8_t *z) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = begin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < end; k += stride) {
    const uint32_t i = stack[k];
    uint64_t c[3];
    xor_cells(keys[i], rmix, seg, c);
    const uint32_t p = peel[i];
    uint8_t acc = choice[i] & 1;
    for (uint32_t q = 0; q < 3; ++q)
      if (q != p) acc ^= z[c[q]];
    z[c[p]] = acc;
  }
}

// Small systems: the first frontier, every peeling round and the assignment
// in one workgroup, the rounds separated by barriers instead of launches and
// the round state in LDS.  The rounds, the peel cell of every key and so the
// cells are those of the multi-launch passes above.  Data written earlier in
// the kernel by other threads is read with agent-scope atomic loads, which
// bypass the L1, after every thread's stores have completed (s_waitcnt 0)
// and a barrier.  A stack entry holds the key index and, in its top two
// bits, the key's peel cell.
constexpr uint32_t kSmallThreads = 1024;
constexpr uint64_t kSmallRetrievalKeys = 1u << 16;

__device__ __forceinline__ uint64_t ld_agent64(const void *p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const void *p) {
  return __hip_atomic_load(reinterpret_cast<const uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void phase_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// Workgroup-wide append onto an LDS counter: each thread offers cnt slots and
// gets the index of its first one.  Every thread of the workgroup must call it.
__device__ __forceinline__ uint32_t small_append(uint32_t *tail, uint32_t cnt, uint32_t *wave_sum, uint32_t *base) {
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t x = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wave_sum[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) {
      const uint32_t t = wave_sum[w];
      wave_sum[w] = tot;
      tot += t;
    }
    *base = *tail;
    *tail += tot;
  }
  __syncthreads();
  const uint32_t at = *base + wave_sum[wave] + x - cnt;
  __syncthreads();
  return at;
}

__global__ __launch_bounds__(kSmallThreads) void xor_solve_small_kernel(
    const uint64_t *__restrict__ keys, uint32_t n_keys, uint64_t rmix, uint64_t seg, unsigned long long *cw,
    uint32_t cells, uint64_t *frontier, uint32_t *taken, uint32_t *stack, uint64_t *round_off,
    const uint8_t *__restrict__ choice, uint8_t *z, unsigned long long *pk) {
  __shared__ uint32_t wave_sum[kSmallThreads / 64];
  __shared__ uint32_t base_s, fr_begin, fr_end, fr_tail, st_begin, st_tail, round_s;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) fr_begin = fr_end = fr_tail = st_begin = st_tail = round_s = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < cells; c0 += kSmallThreads) {
    const uint32_t c = c0 + tid;
    const bool one = c < cells && (ld_agent64(&cw[c]) >> 48) == 1;
    const uint32_t at = small_append(&fr_tail, one ? 1u : 0u, wave_sum, &base_s);
    if (one && at < cells) frontier[at] = c;
  }
  phase_sync();
  for (;;) {
    if (tid == 0) {
      // open the next round on the frontier the previous one appended
      round_off[round_s] = st_tail;
      st_begin = st_tail;
      const uint32_t b = fr_end, e = fr_tail;
      fr_end = e;
      if (e > b && round_s < kMaxPeelRounds) {
        fr_begin = b;
        ++round_s;
      } else {
        fr_begin = e;
      }
    }
    __syncthreads();
    const uint32_t fb = fr_begin, fe = fr_end < cells ? fr_end : cells;
    if (fb >= fe) break;
    // detect: each frontier cell still at count one peels its key at the key's
    // first cell of count one
    for (uint32_t k0 = fb; k0 < fe; k0 += kSmallThreads) {
      const uint32_t k = k0 + tid;
      uint32_t item = 0, got = 0;
      if (k < fe) {
        const uint64_t w = ld_agent64(&cw[ld_agent64(&frontier[k])]);
        const uint64_t i = w & (kCountOne - 1);
        if ((w >> 48) == 1 && i < n_keys) {
          const uint32_t bit = 1u << (i & 31);
          if (!(atomicOr(&taken[i >> 5], bit) & bit)) {
            uint64_t c[3];
            xor_cells(keys[i], rmix, seg, c);
            const uint64_t w0 = ld_agent64(&cw[c[0]]), w1 = ld_agent64(&cw[c[1]]);  // both in flight
            const uint32_t q = (w0 >> 48) == 1 ? 0u : ((w1 >> 48) == 1 ? 1u : 2u);
            item = (uint32_t)i | (q << 30);
            got = 1;
          }
        }
      }
      const uint32_t at = small_append(&st_tail, got, wave_sum, &base_s);
      if (got && at < n_keys) stack[at] = item;
    }
    phase_sync();
    // remove the round's keys; cells falling from two to one form the next frontier
    const uint32_t sb = st_begin, se = st_tail < n_keys ? st_tail : n_keys;
    for (uint32_t k0 = sb; k0 < se; k0 += kSmallThreads) {
      const uint32_t k = k0 + tid;
      uint64_t c[3] = {0, 0, 0};
      uint32_t fell = 0;
      if (k < se) {
        const uint32_t i = ld_agent32(&stack[k]) & ((1u << 30) - 1);
        xor_cells(keys[i], rmix, seg, c);
#pragma unroll
        for (uint32_t q = 0; q < 3; ++q)
          if ((atomicSub(&cw[c[q]], kCountOne + i) >> 48) == 2) fell |= 1u << q;
      }
      uint32_t at = small_append(&fr_tail, __popc(fell), wave_sum, &base_s);
#pragma unroll
      for (uint32_t q = 0; q < 3; ++q)
        if ((fell >> q) & 1) {
          if (at < cells) frontier[at] = c[q];
          ++at;
        }
    }
    phase_sync();
  }
  const uint32_t R = round_s, peeled = st_tail;
  if (tid == 0) {
    pk[kPkRound] = R;
    pk[kPkStTail] = peeled;
    pk[kPkFrTail] = fr_tail;
    pk[kPkFrEnd] = fr_end;
  }
  phase_sync();
  if (peeled != n_keys) return;  // a 2-core is left: the host tries the next retrieval seed
  // assignment, rounds in reverse (keys of one round write distinct cells and
  // read none written in that round); only the last round can be empty (a
  // frontier whose cells all fell to zero), and it is not counted
  uint32_t nonempty = 0;
  for (uint32_t r = R; r >= 1; --r) {
    const uint32_t b = (uint32_t)ld_agent64(&round_off[r - 1]);
    const uint32_t e = r == R ? peeled : (uint32_t)ld_agent64(&round_off[r]);
    nonempty += e > b ? 1u : 0u;
    for (uint32_t k = b + tid; k < e; k += kSmallThreads) {
      const uint32_t item = ld_agent32(&stack[k]);
      const uint32_t i = item & ((1u << 30) - 1), p = item >> 30;
      uint64_t c[3];
      xor_cells(keys[i], rmix, seg, c);
      uint32_t acc = choice[i] & 1;
#pragma unroll
      for (uint32_t q = 0; q < 3; ++q)
        if (q != p) acc ^= (ld_agent32(z + (c[q] & ~3ull)) >> (8 * (c[q] & 3))) & 0xFF;
      z[c[p]] = (uint8_t)acc;
    }
    phase_sync();
  }
  if (tid == 0) pk[kPkRound] = nonempty;
}

__global__ void pack_bits_kernel(const uint8_t *__restrict__ z, uint64_t cells, uint64_t *bits) {
  const uint64_t words = (cells + 63) / 64;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride) {
    uint64_t v = 0;
    for (uint32_t b = 0; b < 64; ++b) {
      const uint64_t c = w * 64 + b;
      if (c < cells && z[c]) v |= 1ull << b;
    }
    bits[w] = v;
  }
}

// ---- query ------------------------------------------------------------------

struct QueryArgs {
  const uint64_t *block;  // kBkWords per block of 16 buckets
  const uint32_t *key_rel, *fixed_rel, *unary_rel;
  const uint16_t *sigma;
  const uint8_t *rseed;
  const uint64_t *codes;  // 5-bit leaf size codes
  const uint64_t *fixed, *unary, *zbits;
  uint64_t fixed_words, unary_words, zwords;
  uint64_t n_buckets, seg, rmix;
  uint32_t leaf_target;
  uint32_t rf, partial_k, retrieval;
  KTable K;
};

// Where bucket b's keys, leaves, ribbon bits and codes start, and its size.
struct BucketAt {
  uint64_t o, m, lb, rb, F, U;
  uint32_t L;
};
__device__ __forceinline__ void bucket_at(const QueryArgs &A, uint64_t b, BucketAt &r) {
  const uint64_t k = b >> kBlockShift, b0 = k << kBlockShift;
  const uint64_t *e = A.block + k * kBkWords;
  uint64_t lb = e[kBkLeaf], rb = e[kBkRib];
  uint32_t prev = 0;  // key_rel of the block's first bucket is 0
  const uint32_t lt = A.leaf_target;
  for (uint64_t j = b0; j < b; ++j) {
    const uint32_t next = A.key_rel[j + 1];
    const uint32_t mj = next - prev;  // a bucket holds fewer than 2^32 keys
    lb += (mj + lt - 1) / lt;         // 32-bit division: a fraction of the 64-bit one's instructions
    rb += ribbon_cols(mj);
    prev = next;
  }
  r.o = e[kBkKey] + prev;
  r.m = A.block[((b + 1) >> kBlockShift) * kBkWords + kBkKey] + A.key_rel[b + 1] - r.o;
  r.L = ((uint32_t)r.m + lt - 1) / lt;
  r.lb = lb;
  r.rb = rb;
  r.F = e[kBkFixed] + A.fixed_rel[b];
  r.U = e[kBkUnary] + A.unary_rel[b];
}

// Position of the r-th one bit (0-based) at or after bit p of the stream.
// Position of the r-th set bit (from 0) of a word with more than r set bits.
__device__ __forceinline__ uint32_t select_in_word(uint64_t w, uint32_t r) {
  uint32_t pos = 0;
  for (uint32_t half = 32; half != 0; half >>= 1) {
    const uint32_t c = (uint32_t)__popcll((w >> pos) & ((1ull << half) - 1));
    if (r >= c) {
      r -= c;
      pos += half;
    }
  }
  return pos;
}

// Positions of the (r-1)-th and r-th ones of the bit stream s at or after
// bit p (r >= 1), or kNone: one scan of the words.
__device__ __forceinline__ void select_two(const uint64_t *s, uint64_t words, uint64_t p, uint32_t r, uint64_t &prev,
                                           uint64_t &cur) {
  prev = cur = kNone;
  uint64_t w = p >> 6;
  uint64_t word = w < words ? s[w] & (~0ull << (p & 63)) : 0;
  uint32_t want = r - 1;  // looking for the (r-1)-th one first
  for (;;) {
    const uint32_t c = (uint32_t)__popcll(word);
    if (c > want) {
      const uint32_t b = select_in_word(word, want);
      if (prev == kNone) {
        prev = w * 64 + b;
        // the next one: in the rest of this word, or further on
        const uint64_t rest = b == 63 ? 0 : word & (~0ull << (b + 1));
        if (rest) {
          cur = w * 64 + (uint64_t)__builtin_ctzll(rest);
          return;
        }
        want = 0;
        word = 0;  // continue with the next word
        if (w + 1 >= words) return;
        ++w;
        word = s[w];
        continue;
      }
      cur = w * 64 + b;
      return;
    }
    want -= c;
    if (w + 1 >= words) return;
    ++w;
    word = s[w];
  }
}

// The value stored for leaf j of a bucket: its fixed bits come after the
// fixed widths of the leaves before it in the bucket, its unary code is the
// j-th in the bucket's unary stream.
__device__ __forceinline__ uint64_t leaf_value(const QueryArgs &A, const uint8_t *K, const BucketAt &bk, uint32_t lo,
                                               uint32_t j, uint32_t n) {
  // the fixed widths of leaves lb .. lb + j - 1: twelve 5-bit codes per
  // 64-bit window of the code stream
  uint64_t F = bk.F;
  for (uint64_t g = bk.lb, ge = bk.lb + j; g < ge;) {
    const uint64_t p = 5 * g, w = p >> 6;
    const uint32_t sh = (uint32_t)(p & 63);
    uint64_t x = A.codes[w] >> sh;
    if (sh > 4) x |= A.codes[w + 1] << (64 - sh);
    const uint64_t take = ge - g < 12 ? ge - g : 12;
    for (uint64_t t = 0; t < take; ++t, x >>= 5) F += K[lo + (uint32_t)(x & 31)];
    g += take;
  }
  const uint32_t k = K[n];
  uint64_t low = 0;
  if (k) low = bits_at(A.fixed, A.fixed_words, F) & (~0ull >> (64 - k));
  uint64_t prev, end;
  if (j == 0) {
    select_two(A.unary, A.unary_words, bk.U, 1, end, prev);  // the 0-th one
    prev = bk.U - 1;
  } else {
    select_two(A.unary, A.unary_words, bk.U, j, prev, end);
  }
  return end == kNone ? kNone : (((end - (prev + 1)) << k) | low);
}

__global__ __launch_bounds__(256) void mphf_query_kernel(QueryArgs A, const uint64_t *__restrict__ queries,
                                                         uint64_t n_queries, uint64_t *__restrict__ out) {
  __shared__ uint8_t K[65];
  if (threadIdx.x < 65) K[threadIdx.x] = A.K.k[threadIdx.x];
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_queries; t += stride) {
    const uint64_t x = queries[t];
    const uint64_t b = bucket_of(x, A.n_buckets);
    BucketAt bk;
    bucket_at(A, b, bk);
    if (bk.m == 0) {
      out[t] = kNone;
      continue;
    }
    const uint32_t lo = size_base(bk.m, bk.L);
    const uint32_t j = leaf_of(x, split_mix(A.sigma[b]), bk.L);
    const uint64_t start = (uint64_t)j * lo + code_sum(A.codes, bk.lb, bk.lb + j);
    const uint32_t n = lo + size_code(A.codes, bk.lb + j);
    const uint64_t value = leaf_value(A, K, bk, lo, j, n);
    // the choice from the retrieval
    uint32_t f;
    if (A.retrieval == kRetrievalRibbon) {
      uint64_t s, c;
      ribbon_row(x, ribbon_mix(A.rseed[b]), ribbon_cols(bk.m), s, c);
      f = (uint32_t)__popcll(c & bits_at(A.zbits, A.zwords, bk.rb + s)) & 1;
    } else {
      uint64_t c[3];
      xor_cells(x, A.rmix, A.seg, c);
      f = (uint32_t)(((A.zbits[c[0] >> 6] >> (c[0] & 63)) ^ (A.zbits[c[1] >> 6] >> (c[1] & 63)) ^
                      (A.zbits[c[2] >> 6] >> (c[2] & 63))) & 1);
    }
    uint32_t h0 = 0, h1 = 0;
    if (A.rf == kLeafBip && n >= 2) {
      // left cell under a, right cell under b
      uint64_t pa = 0, pb = 0;
      bip_pair_of(value, pa, pb);
      const uint64_t ax = fmix64(x);
      const uint32_t nl = n / 2, nr = n - n / 2;
      uint32_t l, r;
      shockhash::bip_cells(ax, seed_mix(pa), nl, nr, h0, r);
      shockhash::bip_cells(ax, seed_mix(pb), nl, nr, l, h1);
    } else if (n >= 2) {
      uint64_t seed = value;
      uint32_t r = 0;
      if (A.rf == kLeafRf) {  // value = s * n + r; the first set hashes with s - s mod k
        seed = value / n;
        const uint32_t pk = A.partial_k ? A.partial_k : (n > 32 ? 8u : 1u);
        if (shockhash::key_side(x)) r = (uint32_t)(value - seed * n);
        else seed -= seed % pk;
      }
      const uint64_t a = fmix64(x), ts = seed_mix(seed);
      slot_pair((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)ts, (uint32_t)(ts >> 32), n, n - 1, h0, h1);
      h0 = h0 + r >= n ? h0 + r - n : h0 + r;
      h1 = h1 + r >= n ? h1 + r - n : h1 + r;
    }
    out[t] = bk.o + start + (f ? h1 : h0);
  }
}

// Export: every leaf's size and stored value, one thread per bucket.
__global__ void decode_leaves_kernel(QueryArgs A, uint8_t *sizes, uint64_t *values) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < A.n_buckets; b += stride) {
    BucketAt bk;
    bucket_at(A, b, bk);
    const uint32_t lo = size_base(bk.m, bk.L);
    uint64_t F = bk.F, U = bk.U;
    for (uint32_t j = 0; j < bk.L; ++j) {
      const uint32_t n = lo + size_code(A.codes, bk.lb + j), k = A.K.k[n];
      const uint64_t low = k ? bits_at(A.fixed, A.fixed_words, F) & (~0ull >> (64 - k)) : 0;
      F += k;
      uint64_t p = U;  // the next one at or after U
      while (p < A.unary_words * 64 && !((A.unary[p >> 6] >> (p & 63)) & 1)) ++p;
      sizes[bk.lb + j] = (uint8_t)n;
      values[bk.lb + j] = (p < A.unary_words * 64) ? (((p - U) << k) | low) : kNone;
      U = p + 1;
    }
  }
}

int grid_for(uint64_t items, uint32_t per_block) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g > 65536) g = 65536;
  return g == 0 ? 1 : (int)g;
}

}  // namespace

struct shock_mphf {
  uint64_t n_keys = 0, n_buckets = 0, n_leaves = 0;
  uint32_t leaf_target = 0, leaf_max = 0, bucket_size = 0;
  uint32_t rf = 0, partial_k = 0, retrieval = 0;
  uint64_t rho = 0, seg = 0;  // XOR retrieval
  uint32_t max_sigma = 0, peel_rounds = 0;
  KTable K{};
  // bucket table: kBkWords per block of 16 buckets, then per bucket
  uint64_t *block = nullptr;
  uint32_t *key_rel = nullptr, *fixed_rel = nullptr, *unary_rel = nullptr;
  uint16_t *sigma = nullptr;
  uint8_t *rseed = nullptr;  // ribbon seed per bucket
  uint64_t *codes = nullptr;  // 5-bit leaf size codes
  uint64_t *fixed = nullptr, *unary = nullptr, *zbits = nullptr;
  uint64_t n_blocks = 0, code_words = 0, fixed_words = 0, unary_words = 0, zwords = 0;
  uint64_t fixed_bits = 0, unary_bits = 0, rib_bits = 0;
  double build_ms = 0, search_ms = 0;
  double layout_ms = 0, search_call_ms = 0, codes_ms = 0, retrieval_ms = 0;
  uint32_t rho_tries = 0, max_rseed = 0;
  uint64_t rib_walked = 0;  // ribbon buckets solved by the walk
};

namespace {

// Scratch of one build: bump allocations from the calling thread's arena on
// the current device.  The arena is sized for the whole build before its
// first kernel and kept for the thread's next build, so a build makes no
// hipMalloc/hipFree for scratch (hipFree waits for the whole device, which
// would stall builds running on other streams) once the arena is large
// enough.  Also holds a few words of pinned host memory for read-backs.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  uint64_t *pinned = nullptr;  // kPinnedWords words
  // a second stream (default priority) on which the retrieval peels while
  // the leaf search runs on the caller's stream, and two events joining them
  hipStream_t aux = nullptr;
  hipEvent_t ev_choice = nullptr, ev_done = nullptr;
  int cus = 0;  // compute units of the device
};
constexpr size_t kPinnedWords = 16;
thread_local std::vector<Arena> t_arena;

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Scratch {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  uint64_t *pinned = nullptr;
  Arena *arena = nullptr;
  template <typename T>
  hipError_t alloc(T **p, size_t count) {
    const size_t bytes = align256((count ? count : 1) * sizeof(T));
    if (used + bytes > cap) return hipErrorOutOfMemory;  // the reservation covers every allocation
    *p = reinterpret_cast<T *>(base + used);
    used += bytes;
    return hipSuccess;
  }
};

// Reserve `bytes` of scratch for a build on the current device.
hipError_t reserve_scratch(size_t bytes, Scratch &S) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((int)t_arena.size() <= dev) t_arena.resize(dev + 1);
  Arena &A = t_arena[dev];
  if (A.pinned == nullptr) {
    e = hipHostMalloc((void **)&A.pinned, kPinnedWords * sizeof(uint64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
      A.pinned = nullptr;
      return e;
    }
  }
  if (A.cap < bytes) {
    if (A.base) {
      e = hipFree(A.base);  // the previous build on this thread has finished (builds are synchronous)
      A.base = nullptr;
      A.cap = 0;
      if (e != hipSuccess) return e;
    }
    const size_t grown = bytes + bytes / 8;
    e = hipMalloc((void **)&A.base, grown);
    if (e != hipSuccess) {
      A.base = nullptr;
      return e;
    }
    A.cap = grown;
  }
  if (!A.cus) {
    hipDeviceProp_t prop;
    A.cus = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 256;
  }
  S.base = A.base;
  S.cap = A.cap;
  S.used = 0;
  S.pinned = A.pinned;
  S.arena = &A;
  return hipSuccess;
}

// The arena's second stream and events, created on first use.
hipError_t aux_of(Arena &A) {
  hipError_t e = hipSuccess;
  if (!A.aux) e = hipStreamCreateWithFlags(&A.aux, hipStreamNonBlocking);
  if (e == hipSuccess && !A.ev_choice) e = hipEventCreateWithFlags(&A.ev_choice, hipEventDisableTiming);
  if (e == hipSuccess && !A.ev_done) e = hipEventCreateWithFlags(&A.ev_done, hipEventDisableTiming);
  return e;
}

void free_mphf(shock_mphf *m) {
  if (!m) return;
  void *ps[] = {m->block, m->key_rel, m->fixed_rel, m->unary_rel, m->sigma, m->rseed,
                m->codes, m->fixed, m->unary, m->zbits};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

}  // namespace

#define HIP_TRY(call)                       \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) {                 \
      shock_internal_set_error(#call, e_);  \
      return e_ == hipErrorOutOfMemory ? SHOCK_ENOMEM : SHOCK_EHIP; \
    }                                       \
  } while (0)

// Workgroups of kS waves of the ribbon block kernel that the LDS of one CU
// holds (160 KiB, at most 32 waves), for buckets of up to max_m keys; 0 if one
// workgroup's LDS would pass 64 KiB.
static uint64_t rib_groups_per_cu(uint64_t max_m, uint32_t kS = kRibWaves) {
  const uint64_t wg = (uint64_t)kS * rib_lds_wave_bytes(max_m);
  if (max_m > kBlockMaxM || wg > 65536) return 0;
  const uint64_t by_lds = (160ull << 10) / wg, by_waves = 32 / kS;
  return by_lds < by_waves ? by_lds : by_waves;
}

static double ms_since(std::chrono::steady_clock::time_point t) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

static int build_impl(const uint64_t *keys, uint64_t N, const shock_mphf_params &P, shock_mphf *M,
                      hipStream_t stream) {
  auto tp = std::chrono::steady_clock::now();
  const uint64_t B = N == 0 ? 1 : (N + P.bucket_size - 1) / P.bucket_size;
  M->n_keys = N;
  M->n_buckets = B;
  // Scratch for the whole build, with the leaf count bounded by its maximum
  // (each bucket of m keys gets ceil(m / leaf_target) leaves).
  const uint64_t Lmax = B + (N + P.leaf_target - 1) / P.leaf_target;
  const uint64_t seg_r = (123 * N + 299) / 300 + 8, cells_r = 3 * seg_r;
  const bool xor_ret = M->retrieval == kRetrievalXor;
  // ribbon slots in global memory, for buckets too large for the LDS variant
  // of the walk; the same region holds the block kernel's pivot rows, sized
  // here for buckets of up to 9/8 of the expected size plus 256 (the grid
  // shrinks to fit if the largest bucket is larger)
  const uint64_t rib_max = N + N / 50 + 65 * B;
  const uint64_t slot_words = rib_max + rib_max / 8 + 2 * (rib_max / 64) + 3 * B + 64;
  uint64_t m_est = (uint64_t)P.bucket_size + P.bucket_size / 8 + 256;
  if (m_est > kBlockMaxM) m_est = kBlockMaxM;
  int dev_now = 0;
  (void)hipGetDevice(&dev_now);
  const uint64_t cus_now = ((int)t_arena.size() > dev_now && t_arena[dev_now].cus) ? t_arena[dev_now].cus : 256;
  uint64_t groups_est = cus_now * rib_groups_per_cu(m_est);
  if (groups_est > B) groups_est = B;
  const uint64_t piv_bytes_est = groups_est * kRibWaves * rib_piv_wave_bytes(m_est);
  const uint64_t rib_area = xor_ret ? 0 : (slot_words * 8 > piv_bytes_est ? slot_words * 8 : piv_bytes_est);
  const size_t scratch_bytes = align256(2 * 8) + align256(B * 4) + 2 * align256(N * 8) + align256((Lmax + 1) * 8) +
                               2 * align256(Lmax * 8) + align256(Lmax * 4) + 2 * align256(N ? N : 1) +
                               3 * align256((B + 1) * 8) + 2 * align256(Lmax + 8) + align256((Lmax / 64 + 3) * 16) +
                               2 * align256((B + 1) * 8) + align256(rib_area) + align256(B) + align256(B * 4) +
                               align256(8) +
                               (xor_ret ? align256(((N + 31) / 32) * 4) + align256(N * 4) + 2 * align256(cells_r * 8) +
                                              align256((kMaxPeelRounds + 1) * 8) + align256(kPkWords * 8) +
                                              align256(cells_r)
                                        : 0) +
                               32 * 256 + (M->rf == kLeafBip ? 2 * align256(Lmax * 8) : 0);  // bipartite seed pairs
  Scratch S;
  HIP_TRY(reserve_scratch(scratch_bytes, S));
  unsigned long long *err = nullptr;
  // pinned: [0] error bits, [1] n_leaves, [2] largest bucket, [3] ribbon bits;
  // [4, 4 + kPkWords) the XOR retrieval's counters
  uint64_t *host = S.pinned;
  HIP_TRY(S.alloc(&err, 3));
  uint32_t *counts = nullptr;
  HIP_TRY(S.alloc(&counts, B));
  uint64_t *bucket_offset = nullptr, *leaf_base = nullptr, *rib_base = nullptr;
  HIP_TRY(S.alloc(&bucket_offset, B + 1));
  HIP_TRY(S.alloc(&leaf_base, B + 1));
  HIP_TRY(S.alloc(&rib_base, B + 1));
  HIP_TRY(hipMalloc((void **)&M->sigma, B * sizeof(uint16_t)));
  HIP_TRY(hipMemsetAsync(err, 0, 3 * sizeof(unsigned long long), stream));
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(B, 256)), dim3(256), 0, stream, counts, B, 0u);
  const bool lds_layout = B <= kLdsBuckets;
  const int layout_grid = (int)((N + kLayoutChunk - 1) / kLayoutChunk);
  if (N && lds_layout)
    hipLaunchKernelGGL(bucket_count_lds_kernel, dim3(layout_grid), dim3(256), 0, stream, keys, N, B, counts);
  else if (N)
    hipLaunchKernelGGL(bucket_count_kernel, dim3(grid_for(N, 256)), dim3(256), 0, stream, keys, N, B, counts);
  hipLaunchKernelGGL(layout_scan_kernel, dim3(1), dim3(1024), 0, stream, counts, B, P.leaf_target, bucket_offset,
                     leaf_base, rib_base, err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&host[2], err + 1, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&host[1], leaf_base + B, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&host[3], rib_base + B, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (host[0] & kErrTooManyLeaves) return SHOCK_EINVAL;
  const uint64_t L = host[1], max_m = host[2], rib_total = host[3];
  M->n_leaves = L;
  uint8_t *leaf_sizes = nullptr, *codes8 = nullptr;  // one byte per leaf, padded
  HIP_TRY(S.alloc(&leaf_sizes, L + 8));
  HIP_TRY(S.alloc(&codes8, L + 8));
  uint64_t *grouped = nullptr, *leaf_keys = nullptr, *leaf_off = nullptr;
  HIP_TRY(S.alloc(&grouped, N));
  HIP_TRY(S.alloc(&leaf_keys, N));
  HIP_TRY(S.alloc(&leaf_off, L + 1));
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(B, 256)), dim3(256), 0, stream, counts, B, 0u);
  if (N && !lds_layout)
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(grid_for(N, 256)), dim3(256), 0, stream, keys, N, B,
                       (const uint64_t *)bucket_offset, counts, grouped);
  if (N && lds_layout)
    hipLaunchKernelGGL(bucket_scatter_lds_kernel, dim3(layout_grid), dim3(256), 0, stream, keys, N, B,
                       (const uint64_t *)bucket_offset, counts, grouped);
  hipLaunchKernelGGL(split_kernel, dim3(grid_for(B, 4)), dim3(256), 0, stream, (const uint64_t *)grouped,
                     (const uint64_t *)bucket_offset, (const uint64_t *)leaf_base, B, P.leaf_max, M->sigma,
                     leaf_sizes, codes8, leaf_off, leaf_keys, err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(leaf_off + L, &N, 8, hipMemcpyHostToDevice, stream));
  if (L)
    hipLaunchKernelGGL(leaf_sort_kernel, dim3(grid_for(L, 4)), dim3(256), 0, stream, leaf_keys,
                       (const uint64_t *)leaf_off, (const uint8_t *)leaf_sizes, L);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (host[0] & kErrSigma) return SHOCK_ENOTFOUND;
  M->layout_ms = ms_since(tp);
  tp = std::chrono::steady_clock::now();

  // Retrieval buffers.  The peeling depends on the keys alone, so for
  // systems too large for one workgroup it starts here on the arena's second
  // stream and runs while the leaf search runs on the caller's stream; only
  // the assignment waits for the leaf orientations.
  uint8_t *choice = nullptr, *peel = nullptr, *z = nullptr;
  uint32_t *taken = nullptr, *stack = nullptr;
  unsigned long long *cw = nullptr, *pk = nullptr;
  uint64_t *frontier = nullptr, *round_off = nullptr, *pk_host = nullptr;
  const uint64_t seg = seg_r, cells = cells_r;
  const uint64_t taken_words = (N + 31) / 32;
  HIP_TRY(S.alloc(&choice, N));
  if (xor_ret) {
    M->seg = seg;
    HIP_TRY(S.alloc(&peel, N));
    HIP_TRY(S.alloc(&taken, taken_words));
    HIP_TRY(S.alloc(&stack, N));
    HIP_TRY(S.alloc(&cw, cells));
    HIP_TRY(S.alloc(&frontier, cells));
    HIP_TRY(S.alloc(&round_off, kMaxPeelRounds + 1));
    HIP_TRY(S.alloc(&pk, kPkWords));
    HIP_TRY(S.alloc(&z, cells));
  }
  static_assert(4 + kPkWords <= kPinnedWords, "pinned words");
  pk_host = S.pinned + 4;
  // Round passes run a fixed grid over device-held ranges; the host checks
  // for the end of the peeling after each chunk of rounds.
  const int round_grid = grid_for((cells + 3) / 4, 256 * kDetectPer) < 1024 ? grid_for((cells + 3) / 4, 256 * kDetectPer) : 1024;
  constexpr uint32_t kChunk = 16;
  const bool big = xor_ret && N > kSmallRetrievalKeys;
  hipStream_t ps = stream;  // the stream the multi-launch peeling runs on
  struct AuxGuard {         // no early return leaves work running on the second stream
    hipStream_t s = nullptr;
    ~AuxGuard() {
      if (s) (void)hipStreamSynchronize(s);
    }
  } guard;
  auto rmix_of = [](uint64_t rho) { return shockhash::fmix64((rho + 1) * kRetrievalMul); };
  auto start_peel = [&](uint64_t rmix) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(cells, 256)), dim3(256), 0, ps, cw, cells);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(taken_words, 256)), dim3(256), 0, ps, taken, taken_words, 0u);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, ps, pk, (uint64_t)kPkWords);
    if (N) hipLaunchKernelGGL(xor_count_kernel, dim3(grid_for(N, 256)), dim3(256), 0, ps, leaf_keys, N, rmix, seg, cw);
    hipLaunchKernelGGL(xor_frontier_kernel, dim3(grid_for(cells, 256 * kFrontierPer)), dim3(kAppendThreads), 0, ps,
                       (const unsigned long long *)cw, cells, frontier, pk);
  };
  auto peel_chunk = [&](uint64_t rmix) {
    for (uint32_t c = 0; c < kChunk; ++c) {
      hipLaunchKernelGGL(xor_advance_kernel, dim3(1), dim3(64), 0, ps, pk, round_off);
      hipLaunchKernelGGL(xor_detect_kernel, dim3(round_grid), dim3(256), 0, ps, leaf_keys, N, rmix, seg,
                         (const unsigned long long *)cw, (const uint64_t *)frontier, cells, taken, peel, stack, pk);
      hipLaunchKernelGGL(xor_remove_kernel, dim3(round_grid), dim3(256), 0, ps, leaf_keys, N, rmix, seg, cw,
                         (const uint32_t *)stack, frontier, cells, pk);
    }
  };
  if (big) {
    HIP_TRY(aux_of(*S.arena));
    ps = S.arena->aux;
    guard.s = ps;
    start_peel(rmix_of(0));
    peel_chunk(rmix_of(0));
    peel_chunk(rmix_of(0));
    HIP_TRY(hipGetLastError());
  }

  // leaf seeds and orientations
  uint64_t *seeds = nullptr, *orient = nullptr;
  HIP_TRY(S.alloc(&seeds, L));
  HIP_TRY(S.alloc(&orient, L));
  if (L) {
    shock_opts o;
    shock_opts_init(&o);
    o.check_dups = 1;
    int rc;
    if (M->rf == kLeafBip) {
      uint64_t *pa = nullptr, *pb = nullptr;
      HIP_TRY(S.alloc(&pa, L));
      HIP_TRY(S.alloc(&pb, L));
      shock_bip_stats bst;
      rc = shock_bip_leaf_search_ex(leaf_keys, leaf_off, L, pa, pb, orient, &o, stream, &bst);
      if (rc == SHOCK_OK) {
        M->search_ms = bst.kernel_ms;
        hipLaunchKernelGGL(bip_values_kernel, dim3(grid_for(L, 256)), dim3(256), 0, stream, (const uint64_t *)pa,
                           (const uint64_t *)pb, seeds, L);
        HIP_TRY(hipGetLastError());
      }
    } else if (M->rf == kLeafRf) {
      uint32_t *rot = nullptr;
      HIP_TRY(S.alloc(&rot, L));
      o.partial_k = (int32_t)M->partial_k;
      rc = shock_rf_leaf_search_ex(leaf_keys, leaf_off, L, seeds, rot, orient, &o, stream);
      if (rc == SHOCK_OK) {
        hipLaunchKernelGGL(rf_values_kernel, dim3(grid_for(L, 256)), dim3(256), 0, stream, seeds,
                           (const uint32_t *)rot, (const uint8_t *)leaf_sizes, L);
        HIP_TRY(hipGetLastError());
      }
    } else {
      rc = shock_leaf_search_ex(leaf_keys, leaf_off, L, seeds, orient, &o, stream);
    }
    if (rc != SHOCK_OK) return rc;
    shock_stats st;
    if (M->rf != kLeafBip && shock_last_stats(&st) == SHOCK_OK) M->search_ms = st.kernel_ms;
  }
  M->search_call_ms = ms_since(tp);
  tp = std::chrono::steady_clock::now();
  // Golomb-Rice codes of the seeds; the encoder's index of blocks of 64
  // leaves is scratch: the structure keeps each bucket's code offsets.
  uint64_t bits[2] = {0, 0};
  const uint64_t n_blocks64 = (L + 63) / 64;
  uint64_t *index = nullptr;
  HIP_TRY(S.alloc(&index, 2 * (n_blocks64 + 1)));
  int rc = shock_rice_encode(seeds, leaf_off, L, M->K.k, nullptr, 0, nullptr, 0, index, bits, stream);
  if (rc != SHOCK_OK && rc != SHOCK_EINVAL) return rc;
  M->fixed_bits = bits[0];
  M->unary_bits = bits[1];
  M->fixed_words = (bits[0] + 63) / 64;
  M->unary_words = (bits[1] + 63) / 64;
  HIP_TRY(hipMalloc((void **)&M->fixed, (M->fixed_words ? M->fixed_words : 1) * 8));
  HIP_TRY(hipMalloc((void **)&M->unary, (M->unary_words ? M->unary_words : 1) * 8));
  rc = shock_rice_encode(seeds, leaf_off, L, M->K.k, M->fixed, M->fixed_words, M->unary, M->unary_words, index,
                         bits, stream);
  if (rc != SHOCK_OK) return rc;
  // the bucket table and the 5-bit size codes
  uint64_t *fixed_at = nullptr, *unary_at = nullptr;
  HIP_TRY(S.alloc(&fixed_at, B + 1));
  HIP_TRY(S.alloc(&unary_at, B + 1));
  M->n_blocks = (B >> kBlockShift) + 1;
  M->code_words = (5 * L + 63) / 64 + 1;
  HIP_TRY(hipMalloc((void **)&M->block, M->n_blocks * kBkWords * 8));
  HIP_TRY(hipMalloc((void **)&M->key_rel, (B + 1) * 4));
  HIP_TRY(hipMalloc((void **)&M->fixed_rel, B * 4));
  HIP_TRY(hipMalloc((void **)&M->unary_rel, B * 4));
  HIP_TRY(hipMalloc((void **)&M->codes, M->code_words * 8));
  hipLaunchKernelGGL(rice_bucket_kernel, dim3(grid_for(B + 1, 256)), dim3(256), 0, stream,
                     (const uint64_t *)leaf_base, B, (const uint64_t *)index, (const uint8_t *)leaf_sizes,
                     (const uint64_t *)seeds, M->K, fixed_at, unary_at);
  hipLaunchKernelGGL(bucket_table_kernel, dim3(grid_for(B + 1, 256)), dim3(256), 0, stream,
                     (const uint64_t *)bucket_offset, (const uint64_t *)leaf_base, (const uint64_t *)rib_base,
                     (const uint64_t *)fixed_at, (const uint64_t *)unary_at, B, M->block, M->key_rel, M->fixed_rel,
                     M->unary_rel, err);
  hipLaunchKernelGGL(pack_codes_kernel, dim3(grid_for(M->code_words, 256)), dim3(256), 0, stream,
                     (const uint8_t *)codes8, L, M->code_words, M->codes);
  HIP_TRY(hipGetLastError());

  M->codes_ms = ms_since(tp);
  tp = std::chrono::steady_clock::now();
  // retrieval of each key's choice
  if (L)
    hipLaunchKernelGGL(choice_kernel, dim3(grid_for(L, 4)), dim3(256), 0, stream, (const uint64_t *)leaf_off,
                       (const uint8_t *)leaf_sizes, (const uint64_t *)orient, L, choice);
  HIP_TRY(hipGetLastError());
  if (!xor_ret) {
    // one ribbon system per bucket, one wave each; the LDS holds a bucket's
    // slots, values and solution unless its largest bucket is too large
    M->rib_bits = rib_total;
    M->zwords = (rib_total + 63) / 64;
    HIP_TRY(hipMalloc((void **)&M->zbits, (M->zwords ? M->zwords : 1) * 8));
    HIP_TRY(hipMalloc((void **)&M->rseed, B));
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(M->zwords, 256)), dim3(256), 0, stream,
                       (unsigned long long *)M->zbits, M->zwords);
    // the block kernel when a bucket's stage, counts and indices fit its
    // LDS; buckets it marks, or all if none fit, go to the walk, whose slots,
    // values and solution sit in LDS unless the largest bucket is too large
    uint8_t *rib_region = nullptr, *spill = nullptr;
    uint32_t *defer = nullptr;
    unsigned long long *defer_n = nullptr;
    HIP_TRY(S.alloc(&rib_region, rib_area));
    HIP_TRY(S.alloc(&spill, B));
    HIP_TRY(S.alloc(&defer, B));
    HIP_TRY(S.alloc(&defer_n, 1));
    const uint64_t max_cols = ribbon_cols(max_m);
    const size_t lds_bytes = (max_cols + max_cols / 8 + 1 + (max_cols + 63) / 64 + 1) * 8;
    const int grid = (int)(B < 65536 ? B : 65536);
    const uint32_t row_cap = P.ribbon_rows ? P.ribbon_rows : kRowCapMax;
    uint64_t groups = (uint64_t)S.arena->cus * rib_groups_per_cu(max_m);
    if (groups > B) groups = B;
    const uint64_t piv_wave = rib_piv_wave_bytes(max_m);
    if (groups * kRibWaves * piv_wave > rib_area) groups = rib_area / (kRibWaves * piv_wave);
    bool walk_all = groups == 0;
    if (!walk_all) {
      hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(B, 256)), dim3(256), 0, stream, spill, B);
      hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, stream, defer_n, (uint64_t)1);
      const uint32_t lw = rib_lds_wave_bytes(max_m);
      // seeds 0 and 1 of every bucket
      hipLaunchKernelGGL(ribbon_block_kernel<kRibWaves>, dim3((uint32_t)groups), dim3(64 * kRibWaves),
                         (size_t)kRibWaves * lw, stream, (const uint64_t *)leaf_keys, (const uint8_t *)choice,
                         (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, B, (const uint32_t *)nullptr,
                         0u, defer, defer_n, rib_region, piv_wave, lw, row_cap, M->zbits, M->zwords, M->rseed, spill,
                         err);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipMemcpyAsync(&host[4], defer_n, 8, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      const uint64_t nd = host[4];
      if (nd && !(host[0] & kErrRibbonInternal)) {
        // the listed buckets from seed 2 on, five (or four, or two) seeds at a
        // time: as many waves per workgroup as its LDS and the pivot region
        // hold (two always fit: the first launch ran with at least one group)
        auto fits = [&](uint32_t k) { return k * lw <= 65536 && k * piv_wave <= rib_area; };
        const uint32_t ks2 = fits(5) ? 5 : (fits(4) ? 4 : kRibWaves);
        uint64_t g2 = (uint64_t)S.arena->cus * rib_groups_per_cu(max_m, ks2);
        if (g2 > nd) g2 = nd;
        if (g2 * ks2 * piv_wave > rib_area) g2 = rib_area / (ks2 * piv_wave);
        const dim3 grid2((uint32_t)g2), block2(64 * ks2);
        const size_t lds2 = (size_t)ks2 * lw;
        if (ks2 == 5)
          hipLaunchKernelGGL(ribbon_block_kernel<5>, grid2, block2, lds2, stream, (const uint64_t *)leaf_keys,
                             (const uint8_t *)choice, (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, nd,
                             (const uint32_t *)defer, 2u, (uint32_t *)nullptr, (unsigned long long *)nullptr,
                             rib_region, piv_wave, lw, row_cap, M->zbits, M->zwords, M->rseed, spill, err);
        else if (ks2 == 4)
          hipLaunchKernelGGL(ribbon_block_kernel<4>, grid2, block2, lds2, stream, (const uint64_t *)leaf_keys,
                             (const uint8_t *)choice, (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, nd,
                             (const uint32_t *)defer, 2u, (uint32_t *)nullptr, (unsigned long long *)nullptr,
                             rib_region, piv_wave, lw, row_cap, M->zbits, M->zwords, M->rseed, spill, err);
        else
          hipLaunchKernelGGL(ribbon_block_kernel<kRibWaves>, grid2, block2, lds2, stream, (const uint64_t *)leaf_keys,
                             (const uint8_t *)choice, (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, nd,
                             (const uint32_t *)defer, 2u, (uint32_t *)nullptr, (unsigned long long *)nullptr,
                             rib_region, piv_wave, lw, row_cap, M->zbits, M->zwords, M->rseed, spill, err);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
      }
    }
    const bool walk_some = !walk_all && (host[0] & kErrRibbonSpill) && !(host[0] & (kErrRibbon | kErrRibbonInternal));
    if (walk_all || walk_some) {
      const uint8_t *only = walk_all ? nullptr : spill;
      if (lds_bytes <= 65536) {
        hipLaunchKernelGGL(ribbon_kernel<true>, dim3(grid), dim3(64), lds_bytes, stream, (const uint64_t *)leaf_keys,
                           (const uint8_t *)choice, (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, B,
                           (uint64_t *)nullptr, (uint64_t)(lds_bytes / 8), M->zbits, M->zwords, M->rseed, only, err);
      } else {
        hipLaunchKernelGGL(ribbon_kernel<false>, dim3(grid), dim3(64), 0, stream, (const uint64_t *)leaf_keys,
                           (const uint8_t *)choice, (const uint64_t *)bucket_offset, (const uint64_t *)rib_base, B,
                           reinterpret_cast<uint64_t *>(rib_region), (uint64_t)0, M->zbits, M->zwords, M->rseed,
                           only, err);
      }
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
    }
    if (walk_some) {
      std::vector<uint8_t> hsp(B);
      HIP_TRY(hipMemcpy(hsp.data(), spill, B, hipMemcpyDeviceToHost));
      for (uint64_t b = 0; b < B; ++b) M->rib_walked += hsp[b];
    } else if (walk_all) {
      M->rib_walked = B;
    }
    if (host[0] & kErrCodeSpan) return SHOCK_EINVAL;
    if (host[0] & kErrRibbonInternal) {
      shock_internal_set_error("ribbon retrieval: a bucket exceeded the launch's LDS or a row left its band",
                               hipErrorInvalidValue);
      return SHOCK_EHIP;
    }
    if (host[0] & kErrRibbon) return SHOCK_ENOTFOUND;
    if (B) {
      std::vector<uint8_t> hs(B);
      std::vector<uint16_t> hg(B);
      HIP_TRY(hipMemcpy(hs.data(), M->rseed, B, hipMemcpyDeviceToHost));
      HIP_TRY(hipMemcpy(hg.data(), M->sigma, B * 2, hipMemcpyDeviceToHost));
      for (uint64_t b = 0; b < B; ++b) {
        M->max_rseed = hs[b] > M->max_rseed ? hs[b] : M->max_rseed;
        M->max_sigma = hg[b] > M->max_sigma ? hg[b] : M->max_sigma;
      }
    }
    M->retrieval_ms = ms_since(tp);
    return SHOCK_OK;
  }
  if (big) HIP_TRY(hipEventRecord(S.arena->ev_choice, stream));
  bool solved = false;
  uint32_t rounds = 0;
  for (uint32_t t = 0; t < P.max_rho_tries && !solved; ++t) {
    const uint64_t rho = t;
    M->rho_tries = t + 1;
    const uint64_t rmix = rmix_of(rho);
    if (!big) {
      // one workgroup peels and assigns the whole system
      hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(cells, 256)), dim3(256), 0, stream, cw, cells);
      hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(taken_words, 256)), dim3(256), 0, stream, taken, taken_words,
                         0u);
      hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, stream, pk, (uint64_t)kPkWords);
      if (N)
        hipLaunchKernelGGL(xor_count_kernel, dim3(grid_for(N, 256)), dim3(256), 0, stream, leaf_keys, N, rmix, seg, cw);
      hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(cells, 256)), dim3(256), 0, stream, z, cells);
      hipLaunchKernelGGL(xor_solve_small_kernel, dim3(1), dim3(kSmallThreads), 0, stream, leaf_keys, (uint32_t)N, rmix,
                         seg, cw, (uint32_t)cells, frontier, taken, stack, round_off, (const uint8_t *)choice, z, pk);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(pk_host, pk, kPkWords * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (pk_host[kPkStTail] != N) continue;  // a 2-core is left: next retrieval seed
      rounds = (uint32_t)pk_host[kPkRound];
      M->rho = rho;
      solved = true;
      continue;
    }
    if (t > 0) {  // the first seed's peeling was started before the leaf search
      start_peel(rmix);
      peel_chunk(rmix);
    }
    HIP_TRY(hipGetLastError());
    for (;;) {
      HIP_TRY(hipMemcpyAsync(pk_host, pk, kPkWords * sizeof(uint64_t), hipMemcpyDeviceToHost, ps));
      HIP_TRY(hipStreamSynchronize(ps));
      // done when the last round appended no frontier cells
      if (pk_host[kPkFrTail] == pk_host[kPkFrEnd] || pk_host[kPkRound] >= kMaxPeelRounds) break;
      peel_chunk(rmix);
      HIP_TRY(hipGetLastError());
    }
    if (pk_host[kPkStTail] != N || pk_host[kPkFrTail] > cells) continue;  // a 2-core is left: next retrieval seed
    const uint32_t R = (uint32_t)pk_host[kPkRound];
    std::vector<uint64_t> off(R + 1);
    HIP_TRY(hipMemcpyAsync(off.data(), round_off, R * sizeof(uint64_t), hipMemcpyDeviceToHost, ps));
    HIP_TRY(hipStreamSynchronize(ps));
    off[R] = N;
    HIP_TRY(hipStreamWaitEvent(ps, S.arena->ev_choice, 0));  // the choices come from the leaf search
    hipLaunchKernelGGL(fill_u8_kernel, dim3(grid_for(cells, 256)), dim3(256), 0, ps, z, cells);
    rounds = 0;
    for (uint32_t rr = R; rr >= 1; --rr) {
      const uint64_t b = off[rr - 1], e = off[rr];
      if (e <= b) continue;
      ++rounds;
      hipLaunchKernelGGL(xor_assign_kernel, dim3(grid_for(e - b, 256)), dim3(256), 0, ps, leaf_keys, rmix, seg,
                         (const uint32_t *)stack, b, e, (const uint8_t *)peel, (const uint8_t *)choice, z);
    }
    HIP_TRY(hipGetLastError());
    M->rho = rho;
    solved = true;
  }
  if (big) {
    HIP_TRY(hipEventRecord(S.arena->ev_done, ps));
    HIP_TRY(hipStreamWaitEvent(stream, S.arena->ev_done, 0));
  }
  if (!solved) return SHOCK_ENOTFOUND;
  M->peel_rounds = rounds;
  M->zwords = (cells + 63) / 64;
  HIP_TRY(hipMalloc((void **)&M->zbits, M->zwords * 8));
  hipLaunchKernelGGL(pack_bits_kernel, dim3(grid_for(M->zwords, 256)), dim3(256), 0, stream, (const uint8_t *)z, cells,
                     M->zbits);
  HIP_TRY(hipGetLastError());
  // the largest splitting seed (for the record)
  if (B) {
    std::vector<uint16_t> hg(B);
    HIP_TRY(hipMemcpyAsync(hg.data(), M->sigma, B * 2, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&host[0], err, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (uint64_t b = 0; b < B; ++b) M->max_sigma = hg[b] > M->max_sigma ? hg[b] : M->max_sigma;
    if (host[0] & kErrCodeSpan) return SHOCK_EINVAL;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  M->retrieval_ms = ms_since(tp);
  return SHOCK_OK;
}

hipError_t shock_internal_release_mphf_scratch(int dev) {
  if ((int)t_arena.size() <= dev) return hipSuccess;
  Arena &A = t_arena[dev];
  hipError_t e = hipSuccess;
  if (A.base) e = hipFree(A.base);
  A.base = nullptr;
  A.cap = 0;
  if (A.pinned) {
    const hipError_t f = hipHostFree(A.pinned);
    if (e == hipSuccess) e = f;
  }
  A.pinned = nullptr;
  if (A.aux) {
    const hipError_t f = hipStreamDestroy(A.aux);
    if (e == hipSuccess) e = f;
  }
  A.aux = nullptr;
  for (hipEvent_t *ev : {&A.ev_choice, &A.ev_done}) {
    if (*ev) {
      const hipError_t f = hipEventDestroy(*ev);
      if (e == hipSuccess) e = f;
    }
    *ev = nullptr;
  }
  return e;
}

extern "C" {

void shock_mphf_params_init(shock_mphf_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->bucket_size = 3000;
  p->leaf_target = 40;
  p->leaf_max = 56;
  p->max_rho_tries = 64;
  p->rice_k_by_n = nullptr;
  p->retrieval = SHOCK_RETRIEVAL_RIBBON;
}

int shock_mphf_build(const uint64_t *keys, uint64_t n_keys, const shock_mphf_params *params, shock_mphf **out,
                     void *hip_stream) {
  if (!params || !out || (n_keys && !keys)) return SHOCK_EINVAL;
  const shock_mphf_params &P = *params;
  if (P.bucket_size == 0 || P.leaf_target == 0 || P.leaf_max > 64 || P.leaf_target > P.leaf_max) return SHOCK_EINVAL;
  if (P.max_rho_tries == 0 || !P.rice_k_by_n || n_keys >= (1ull << 32)) return SHOCK_EINVAL;
  if (P.rotation_fitting > 1 || (P.partial_k != 0 && P.partial_k != 1 && P.partial_k != 8)) return SHOCK_EINVAL;
  if (P.bipartite > 1 || (P.bipartite && P.rotation_fitting)) return SHOCK_EINVAL;
  if (P.retrieval != SHOCK_RETRIEVAL_RIBBON && P.retrieval != SHOCK_RETRIEVAL_XOR) return SHOCK_EINVAL;
  if (P.ribbon_rows > kRowCapMax) return SHOCK_EINVAL;
  *out = nullptr;
  shock_mphf *M = new shock_mphf;
  M->leaf_target = P.leaf_target;
  M->leaf_max = P.leaf_max;
  M->bucket_size = P.bucket_size;
  M->rf = P.bipartite ? kLeafBip : (P.rotation_fitting ? kLeafRf : kLeafPlain);
  M->partial_k = (uint32_t)P.partial_k;
  M->retrieval = P.retrieval == SHOCK_RETRIEVAL_XOR ? kRetrievalXor : kRetrievalRibbon;
  for (int n = 0; n <= 64; ++n) {
    if (P.rice_k_by_n[n] > 56) {
      delete M;
      return SHOCK_EINVAL;
    }
    M->K.k[n] = P.rice_k_by_n[n];
  }
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = build_impl(keys, n_keys, P, M, (hipStream_t)hip_stream);
  if (rc != SHOCK_OK) {
    // Kernels of a failed build may still be queued: let them finish before
    // the thread's scratch arena or the structure's arrays are reused.
    (void)hipStreamSynchronize((hipStream_t)hip_stream);
    free_mphf(M);
    return rc;
  }
  M->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = M;
  return SHOCK_OK;
}

static QueryArgs query_args(const shock_mphf *m) {
  QueryArgs A;
  A.block = m->block;
  A.key_rel = m->key_rel;
  A.fixed_rel = m->fixed_rel;
  A.unary_rel = m->unary_rel;
  A.sigma = m->sigma;
  A.rseed = m->rseed;
  A.codes = m->codes;
  A.fixed = m->fixed;
  A.unary = m->unary;
  A.zbits = m->zbits;
  A.fixed_words = m->fixed_words;
  A.unary_words = m->unary_words;
  A.zwords = m->zwords;
  A.n_buckets = m->n_buckets;
  A.seg = m->seg;
  A.rmix = shockhash::fmix64((m->rho + 1) * kRetrievalMul);
  A.leaf_target = m->leaf_target;
  A.rf = m->rf;
  A.partial_k = m->partial_k;
  A.retrieval = m->retrieval;
  A.K = m->K;
  return A;
}

int shock_mphf_query(const shock_mphf *m, const uint64_t *queries, uint64_t n_queries, uint64_t *positions,
                     void *hip_stream) {
  if (!m) return SHOCK_EINVAL;
  if (n_queries == 0) return SHOCK_OK;
  if (!queries || !positions) return SHOCK_EINVAL;
  hipLaunchKernelGGL(mphf_query_kernel, dim3(grid_for(n_queries, 256)), dim3(256), 0, (hipStream_t)hip_stream,
                     query_args(m), queries, n_queries, positions);
  HIP_TRY(hipGetLastError());
  return SHOCK_OK;
}

int shock_mphf_info(const shock_mphf *m, shock_mphf_stats *info) {
  if (!m || !info) return SHOCK_EINVAL;
  memset(info, 0, sizeof(*info));
  const uint64_t B = m->n_buckets;
  info->n_keys = m->n_keys;
  info->n_buckets = B;
  info->n_leaves = m->n_leaves;
  info->rho = m->rho;
  info->seg = m->seg;
  info->max_sigma = m->max_sigma;
  info->peel_rounds = m->peel_rounds;
  info->seed_fixed_bits = m->fixed_bits;
  info->seed_unary_bits = m->unary_bits;
  // buckets: per block the key and leaf offsets; per bucket its relative key
  // offset and splitting seed
  info->bits_buckets = m->n_blocks * 2 * 64 + (B + 1) * 32 + B * 16;
  info->bits_leaf_sizes = m->n_leaves * 5;
  // seeds: the Rice streams, per block their offsets, per bucket the relative
  // offsets, and the table of Rice parameters
  info->bits_seeds = m->fixed_bits + m->unary_bits + m->n_blocks * 2 * 64 + B * 64 + 65 * 8;
  info->bits_retrieval = m->retrieval == kRetrievalXor ? 3 * m->seg : m->rib_bits + B * 8 + m->n_blocks * 64;
  info->bits_total = info->bits_buckets + info->bits_leaf_sizes + info->bits_seeds + info->bits_retrieval;
  info->build_ms = m->build_ms;
  info->search_ms = m->search_ms;
  info->layout_ms = m->layout_ms;
  info->search_call_ms = m->search_call_ms;
  info->codes_ms = m->codes_ms;
  info->retrieval_ms = m->retrieval_ms;
  info->rho_tries = m->rho_tries;
  info->retrieval = m->retrieval == kRetrievalXor ? SHOCK_RETRIEVAL_XOR : SHOCK_RETRIEVAL_RIBBON;
  info->max_rseed = m->max_rseed;
  info->ribbon_walked = (uint32_t)m->rib_walked;
  return SHOCK_OK;
}

int shock_mphf_export(const shock_mphf *m, uint64_t *bucket_offset, uint64_t *leaf_base, uint32_t *sigma,
                      uint8_t *leaf_sizes, uint64_t *leaf_seeds, uint8_t *cells) {
  if (!m) return SHOCK_EINVAL;
  const uint64_t B = m->n_buckets, L = m->n_leaves;
  if (bucket_offset || leaf_base) {
    std::vector<uint64_t> blk(m->n_blocks * kBkWords);
    std::vector<uint32_t> rel(B + 1);
    HIP_TRY(hipMemcpy(blk.data(), m->block, blk.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(rel.data(), m->key_rel, (B + 1) * 4, hipMemcpyDeviceToHost));
    uint64_t lb = 0;
    for (uint64_t b = 0; b <= B; ++b) {
      const uint64_t o = blk[(b >> kBlockShift) * kBkWords + kBkKey] + rel[b];
      if (bucket_offset) bucket_offset[b] = o;
      if (leaf_base) leaf_base[b] = lb;
      if (b < B) {
        const uint64_t o1 = blk[((b + 1) >> kBlockShift) * kBkWords + kBkKey] + rel[b + 1];
        lb += (o1 - o + m->leaf_target - 1) / m->leaf_target;
      }
    }
  }
  if (sigma && B) {
    std::vector<uint16_t> hg(B);
    HIP_TRY(hipMemcpy(hg.data(), m->sigma, B * 2, hipMemcpyDeviceToHost));
    for (uint64_t b = 0; b < B; ++b) sigma[b] = hg[b];
  }
  if ((leaf_sizes || leaf_seeds) && L) {
    uint8_t *ds = nullptr;
    uint64_t *dv = nullptr;
    HIP_TRY(hipMalloc((void **)&ds, L));
    hipError_t e = hipMalloc((void **)&dv, L * 8);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(decode_leaves_kernel, dim3(grid_for(B, 256)), dim3(256), 0, 0, query_args(m), ds, dv);
      e = hipGetLastError();
    }
    if (e == hipSuccess && leaf_sizes) e = hipMemcpy(leaf_sizes, ds, L, hipMemcpyDeviceToHost);
    if (e == hipSuccess && leaf_seeds) e = hipMemcpy(leaf_seeds, dv, L * 8, hipMemcpyDeviceToHost);
    (void)hipFree(ds);
    if (dv) (void)hipFree(dv);
    HIP_TRY(e);
  }
  if (cells && m->retrieval == kRetrievalXor) {
    const uint64_t n = 3 * m->seg;
    std::vector<uint64_t> w(m->zwords);
    HIP_TRY(hipMemcpy(w.data(), m->zbits, m->zwords * 8, hipMemcpyDeviceToHost));
    for (uint64_t c = 0; c < n; ++c) cells[c] = (uint8_t)((w[c >> 6] >> (c & 63)) & 1);
  }
  return SHOCK_OK;
}

int shock_mphf_export_ribbon(const shock_mphf *m, uint8_t *rseed, uint64_t *bit_offset, uint8_t *bits) {
  if (!m || m->retrieval != kRetrievalRibbon) return SHOCK_EINVAL;
  const uint64_t B = m->n_buckets;
  if (rseed && B) HIP_TRY(hipMemcpy(rseed, m->rseed, B, hipMemcpyDeviceToHost));
  if (bit_offset) {
    std::vector<uint64_t> blk(m->n_blocks * kBkWords);
    std::vector<uint32_t> rel(B + 1);
    HIP_TRY(hipMemcpy(blk.data(), m->block, blk.size() * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(rel.data(), m->key_rel, (B + 1) * 4, hipMemcpyDeviceToHost));
    uint64_t rb = 0;
    for (uint64_t b = 0; b <= B; ++b) {
      bit_offset[b] = rb;
      if (b < B) {
        const uint64_t o = blk[(b >> kBlockShift) * kBkWords + kBkKey] + rel[b];
        const uint64_t o1 = blk[((b + 1) >> kBlockShift) * kBkWords + kBkKey] + rel[b + 1];
        rb += ribbon_cols(o1 - o);
      }
    }
  }
  if (bits && m->rib_bits) {
    std::vector<uint64_t> w(m->zwords);
    HIP_TRY(hipMemcpy(w.data(), m->zbits, m->zwords * 8, hipMemcpyDeviceToHost));
    for (uint64_t c = 0; c < m->rib_bits; ++c) bits[c] = (uint8_t)((w[c >> 6] >> (c & 63)) & 1);
  }
  return SHOCK_OK;
}

int shock_mphf_destroy(shock_mphf *m) {
  free_mphf(m);
  return SHOCK_OK;
}

}  // extern "C"
