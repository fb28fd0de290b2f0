// Leaf queries and Golomb-Rice seed codes on MI355X (gfx950).
//
// Query (Section 4: a key x is answered by h_{s, f(x)}(x)): every key is
// evaluated under its leaf's seed (and rotation) and takes slot h0 or h1 by
// its bit of the orientation.  The work is a few dozen integer operations per
// key against 16 bytes of traffic per key, so the kernel is bound by HBM; a
// workgroup stages 64 leaves' metadata in LDS and streams their keys.
//
// Golomb-Rice codes (the seed encoding of Section 4; Golomb 1966, Rice 1979):
// a wave takes a block of 64 leaves.  Encoding runs three kernels: per-block
// code lengths, an in-place exclusive scan of the block lengths into the
// sampled index, and the bit writes (a wave scan inside the block; 64-bit
// atomic ORs, since neighbouring codes share words).  Decoding needs only the
// block's index entry: a wave scan of the fixed-part widths locates the low
// bits; for the quotients the wave loads the block's unary segment a word per
// lane, counts ones, and scatters the position of every one into LDS, so lane
// i reads the end of its code and of the previous one.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "shockcode.h"
#include "shock_hash.h"
#include "shock_internal.h"

namespace {

using shockhash::fmix64;
using shockhash::key_side;
using shockhash::seed_mix;
using shockhash::slot_pair;

constexpr uint64_t kNone = ~0ull;
constexpr uint32_t kMaxRiceK = 56;
constexpr uint64_t kMaxQuotient = 1ull << 32;

constexpr uint64_t kCodeErrLeaf = 1;      // a leaf of more than 64 keys
constexpr uint64_t kCodeErrQuotient = 2;  // a quotient of 2^32 or more

struct RiceTable {
  uint8_t k[65];
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Exclusive prefix sum over the 64 lanes.
__device__ __forceinline__ uint64_t wave_excl_scan(uint64_t v) {
  const uint32_t lane = lane_id();
  uint64_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  return x - v;
}

// ---- query ------------------------------------------------------------------

// A workgroup takes a group of 64 consecutive leaves.  Their offsets, seed
// mixes and orientations are staged in LDS once, with a byte per key naming
// its leaf (at most 64 x 64 keys); then the 256 threads stride over the
// group's keys, which are contiguous in the CSR, so loads and stores are fully
// coalesced whatever the leaf sizes.
constexpr uint32_t kQueryGroup = 64;

template <bool RF>
__global__ __launch_bounds__(256) void query_kernel(const uint64_t *__restrict__ keys,
                                                    const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                    const uint64_t *__restrict__ seeds,
                                                    const uint32_t *__restrict__ rot,
                                                    const uint64_t *__restrict__ orient, uint32_t partial_k,
                                                    uint64_t *__restrict__ out_pos) {
  __shared__ uint64_t s_off[kQueryGroup + 1];
  __shared__ uint64_t s_t[kQueryGroup];   // seed mix of the leaf (second set under RF)
  __shared__ uint64_t s_ta[kQueryGroup];  // RF: seed mix of the first set
  __shared__ uint64_t s_f[kQueryGroup];   // orientation
  __shared__ uint32_t s_r[kQueryGroup];   // RF: rotation mod n
  __shared__ uint32_t s_miss[kQueryGroup];  // 1: the leaf has no seed
  __shared__ uint32_t s_ok;
  __shared__ uint8_t s_leaf[kQueryGroup * 64];  // key (relative to the group's first) -> leaf
  const uint32_t tid = threadIdx.x;
  const uint64_t n_groups = (n_leaves + kQueryGroup - 1) / kQueryGroup;
  for (uint64_t grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    const uint64_t j0 = grp * kQueryGroup;
    const uint32_t cnt = (uint32_t)(n_leaves - j0 < kQueryGroup ? n_leaves - j0 : kQueryGroup);
    if (tid == 0) s_ok = 1;
    if (tid <= cnt) s_off[tid] = offsets[j0 + tid];
    __syncthreads();
    if (tid < cnt) {
      const uint64_t n64 = s_off[tid + 1] - s_off[tid];
      if (s_off[tid + 1] < s_off[tid] || n64 > 64) s_ok = 0;
      const uint32_t n = (uint32_t)n64;
      const uint64_t sd = seeds[tid + j0];
      s_f[tid] = orient[tid + j0];
      s_miss[tid] = sd == kNone;
      s_t[tid] = seed_mix(sd);
      if (RF) {
        const uint32_t k = partial_k ? partial_k : (n > 32 ? 8u : 1u);
        s_ta[tid] = seed_mix(sd - sd % k);
        s_r[tid] = n ? rot[tid + j0] % n : 0;
      }
    }
    __syncthreads();
    // A group holding a leaf that is not one (more than 64 keys, decreasing
    // offsets) is skipped: its keys' entries are left untouched.
    if (s_ok) {
      const uint64_t k0 = s_off[0], k1 = s_off[cnt];
      // key -> leaf table: thread t fills leaf t / 4's quarter t % 4
      {
        const uint32_t lf = tid >> 2, part = tid & 3;
        if (lf < cnt) {
          const uint32_t a = (uint32_t)(s_off[lf] - k0), e = (uint32_t)(s_off[lf + 1] - k0);
          for (uint32_t i = a + part; i < e; i += 4) s_leaf[i] = (uint8_t)lf;
        }
      }
      __syncthreads();
      // four keys per thread and step, their loads issued together
      constexpr uint32_t kUnroll = 4;
      const uint64_t step = (uint64_t)blockDim.x * kUnroll;
      for (uint64_t g0 = k0 + tid; g0 < k1; g0 += step) {
        uint64_t x[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
          const uint64_t g = g0 + (uint64_t)u * blockDim.x;
          x[u] = g < k1 ? keys[g] : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
          const uint64_t g = g0 + (uint64_t)u * blockDim.x;
          if (g >= k1) break;
          const uint32_t lo = s_leaf[g - k0];
          const uint64_t base = s_off[lo];
          const uint32_t n = (uint32_t)(s_off[lo + 1] - base);
          const uint32_t i = (uint32_t)(g - base);
          uint64_t pos = kNone;
          if (!s_miss[lo]) {
            uint32_t h0 = 0, h1 = 0;
            if (n >= 2) {
              const uint64_t a = fmix64(x[u]);
              uint64_t t = s_t[lo];
              uint32_t r = 0;
              if (RF) {
                if (key_side(x[u])) r = s_r[lo];
                else t = s_ta[lo];
              }
              slot_pair((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)t, (uint32_t)(t >> 32), n, n - 1, h0, h1);
              if (RF) {
                h0 = h0 + r >= n ? h0 + r - n : h0 + r;
                h1 = h1 + r >= n ? h1 + r - n : h1 + r;
              }
            }
            pos = base + (((s_f[lo] >> i) & 1) ? h1 : h0);
          }
          out_pos[g] = pos;
        }
      }
    }
    __syncthreads();
  }
}

// ---- Golomb-Rice encode -----------------------------------------------------

// Code lengths of one leaf: fixed width k and unary length q + 1.
__device__ __forceinline__ void leaf_code(const uint64_t *offsets, const uint64_t *values, uint64_t j, const RiceTable &T,
                                          uint32_t &k, uint64_t &q, uint64_t &low, unsigned long long *err) {
  const uint64_t o0 = offsets[j], o1 = offsets[j + 1];
  k = 0;
  q = 0;
  low = 0;
  if (o1 < o0 || o1 - o0 > 64) {
    atomicOr(err, kCodeErrLeaf);
    return;
  }
  k = T.k[o1 - o0];
  const uint64_t v = values[j];
  q = v >> k;
  low = k ? (v & (~0ull >> (64 - k))) : 0;
  if (q >= kMaxQuotient) {
    atomicOr(err, kCodeErrQuotient);
    q = 0;
  }
}

// Phase 1: index[2b] = sum of fixed widths of block b, index[2b+1] = sum of
// unary lengths.
__global__ __launch_bounds__(256) void rice_len_kernel(const uint64_t *__restrict__ values,
                                                       const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                       RiceTable T, uint64_t *__restrict__ index,
                                                       unsigned long long *err) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < n_blocks; b += waves) {
    const uint64_t j = b * 64 + lane;
    uint32_t k = 0;
    uint64_t q = 0, low = 0;
    bool have = j < n_leaves;
    if (have) leaf_code(offsets, values, j, T, k, q, low, err);
    const uint64_t fs = wave_sum(have ? k : 0);
    const uint64_t us = wave_sum(have ? q + 1 : 0);
    if (lane == 0) {
      index[2 * b] = fs;
      index[2 * b + 1] = us;
    }
  }
}

// Phase 2: in-place exclusive scan of the block lengths (pairs), totals in the
// last pair and in totals[0..1].  One workgroup of 1024 threads; per chunk,
// thread t sums kScanPer consecutive pairs, the workgroup scans the 1024
// sums (wave shuffles, then the 16 wave totals), and each thread rewrites its
// pairs as running sums.
constexpr uint32_t kScanPer = 16;

__global__ __launch_bounds__(1024) void rice_scan_kernel(uint64_t *index, uint64_t n_blocks, uint64_t *totals) {
  __shared__ uint64_t wf[16], wu[16];
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint64_t carry_f = 0, carry_u = 0;
  for (uint64_t c = 0; c < n_blocks; c += 1024ull * kScanPer) {
    const uint64_t b0 = c + (uint64_t)t * kScanPer;
    uint64_t sf = 0, su = 0;
    for (uint32_t e = 0; e < kScanPer; ++e) {
      const uint64_t b = b0 + e;
      if (b < n_blocks) {
        sf += index[2 * b];
        su += index[2 * b + 1];
      }
    }
    const uint64_t xf = wave_excl_scan(sf), xu = wave_excl_scan(su);
    if (lane == 63) {
      wf[wave] = xf + sf;
      wu[wave] = xu + su;
    }
    __syncthreads();
    uint64_t pf = 0, pu = 0, tf = 0, tu = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      if (w < wave) {
        pf += wf[w];
        pu += wu[w];
      }
      tf += wf[w];
      tu += wu[w];
    }
    uint64_t rf = carry_f + pf + xf, ru = carry_u + pu + xu;
    for (uint32_t e = 0; e < kScanPer; ++e) {
      const uint64_t b = b0 + e;
      if (b < n_blocks) {
        const uint64_t f = index[2 * b], u = index[2 * b + 1];
        index[2 * b] = rf;
        index[2 * b + 1] = ru;
        rf += f;
        ru += u;
      }
    }
    carry_f += tf;
    carry_u += tu;
    __syncthreads();
  }
  if (t == 0) {
    index[2 * n_blocks] = carry_f;
    index[2 * n_blocks + 1] = carry_u;
    totals[0] = carry_f;
    totals[1] = carry_u;
  }
}

__global__ void fill_zero_kernel(uint64_t *p, uint64_t words) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

// OR the bits of one stream segment: words [w0, w0 + span) assembled in the
// wave's LDS buffer.  The first and last word may be shared with the
// neighbouring blocks and are ORed atomically; the others belong to this
// block alone and are stored.
__device__ __forceinline__ void flush_words(const unsigned long long *buf, uint64_t w0, uint32_t span,
                                            unsigned long long *stream) {
  const uint32_t lane = lane_id();
  if (lane < span) {
    const unsigned long long v = buf[lane];
    if (lane == 0 || lane == span - 1) {
      if (v) atomicOr(&stream[w0 + lane], v);
    } else {
      stream[w0 + lane] = v;
    }
  }
}

// Phase 3: write the codes.  The streams were zeroed and are large enough
// (checked on the host from the totals).  A block's fixed part spans at most
// 57 words; its unary part is assembled in LDS when it spans at most 64 words
// and ORed into the stream directly otherwise.
__global__ __launch_bounds__(256) void rice_write_kernel(const uint64_t *__restrict__ values,
                                                         const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                         RiceTable T, const uint64_t *__restrict__ index,
                                                         unsigned long long *fixed, unsigned long long *unary,
                                                         unsigned long long *err) {
  __shared__ unsigned long long bufs[4][2][64];
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long *fbuf = bufs[threadIdx.x >> 6][0];
  unsigned long long *ubuf = bufs[threadIdx.x >> 6][1];
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < n_blocks; b += waves) {
    const uint64_t j = b * 64 + lane;
    uint32_t k = 0;
    uint64_t q = 0, low = 0;
    const bool have = j < n_leaves;
    if (have) leaf_code(offsets, values, j, T, k, q, low, err);
    const uint64_t F = index[2 * b] + wave_excl_scan(have ? k : 0);
    const uint64_t U = index[2 * b + 1] + wave_excl_scan(have ? q + 1 : 0);
    const uint64_t f0 = index[2 * b], f1 = index[2 * b + 2];
    const uint64_t u0 = index[2 * b + 1], u1 = index[2 * b + 3];
    const uint64_t fw0 = f0 >> 6, uw0 = u0 >> 6;
    const uint32_t fspan = f1 > f0 ? (uint32_t)(((f1 - 1) >> 6) - fw0 + 1) : 0;
    const uint64_t uspan64 = u1 > u0 ? ((u1 - 1) >> 6) - uw0 + 1 : 0;
    const bool ulds = uspan64 <= 64;
    fbuf[lane] = 0;
    ubuf[lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (have) {
      if (k != 0 && low != 0) {
        const uint32_t w = (uint32_t)((F >> 6) - fw0);
        const uint32_t sh = (uint32_t)(F & 63);
        atomicOr(&fbuf[w], (unsigned long long)(low << sh));
        if (sh + k > 64) atomicOr(&fbuf[w + 1], (unsigned long long)(low >> (64 - sh)));
      }
      const uint64_t p = U + q;
      if (ulds) atomicOr(&ubuf[(p >> 6) - uw0], 1ull << (p & 63));
      else atomicOr(&unary[p >> 6], 1ull << (p & 63));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    flush_words(fbuf, fw0, fspan, fixed);
    if (ulds) flush_words(ubuf, uw0, (uint32_t)uspan64, unary);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

// ---- Golomb-Rice decode -----------------------------------------------------

// Position of the r-th set bit (from 0) of a word with more than r set bits.
__device__ __forceinline__ uint32_t select_bit(uint64_t w, uint32_t r) {
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

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
  const uint32_t lane = lane_id();
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(v, d);
    if (lane >= (uint32_t)d) v = y > v ? y : v;
  }
  return v;
}

// A wave decodes a block of 64 leaves.  The index gives the block's bit
// ranges; the loads that depend only on it (the block's unary words) are
// issued with the offsets.  The ones of the unary segment (one per leaf,
// ending its quotient) are found in parallel: each lane holds one word, a
// scan of popcounts gives every word's first one, and lane t finds the word
// holding the t-th one (a prefix maximum over the words' start slots) and
// the bit inside it (a binary search on popcounts).
__global__ __launch_bounds__(256) void rice_decode_kernel(const uint64_t *__restrict__ fixed, uint64_t fixed_words,
                                                          const uint64_t *__restrict__ unary, uint64_t unary_words,
                                                          const uint64_t *__restrict__ index,
                                                          const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                          RiceTable T, uint64_t *__restrict__ values) {
  __shared__ uint32_t start_slot[4][64];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;
  uint32_t *sel = start_slot[wave];
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; b < n_blocks; b += waves) {
    const uint64_t j = b * 64 + lane;
    const uint64_t F0 = index[2 * b], U0 = index[2 * b + 1], U1 = index[2 * b + 3];
    bool have = j < n_leaves;
    uint64_t o0 = 0, o1 = 0;
    if (have) {
      o0 = offsets[j];
      o1 = offsets[j + 1];
    }
    const uint64_t W0 = U0 >> 6, W1 = U1 > U0 ? (U1 - 1) >> 6 : W0;
    auto unary_word = [&](uint64_t w) -> uint64_t {
      if (U1 <= U0 || w > W1 || w >= unary_words) return 0;
      uint64_t x = unary[w];
      if (w == W0) x &= ~0ull << (U0 & 63);
      if (w == W1 && (U1 & 63) != 0) x &= ~0ull >> (64 - (U1 & 63));
      return x;
    };
    uint64_t word = unary_word(W0 + lane);
    uint32_t k = 0;
    if (have) {
      if (o1 < o0 || o1 - o0 > 64) have = false;
      else k = T.k[o1 - o0];
    }
    // low bits
    const uint64_t F = F0 + wave_excl_scan(k);
    uint64_t low = 0;
    if (have && k) {
      const uint64_t w = F >> 6;
      const uint32_t sh = (uint32_t)(F & 63);
      if (w < fixed_words) low = fixed[w] >> sh;
      if (sh + k > 64 && w + 1 < fixed_words) low |= fixed[w + 1] << (64 - sh);
      low &= ~0ull >> (64 - k);
    }
    // the position of the lane-th one of the segment: the end of leaf j's code
    uint64_t my_end = 0, found = 0;
    for (uint64_t base = W0; U1 > U0 && base <= W1; base += 64) {
      const uint32_t cnt = (uint32_t)__popcll(word);
      const uint64_t t0 = found + wave_excl_scan((uint64_t)cnt);
      const uint64_t total = __shfl(t0 + cnt, 63) - found;
      sel[lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (cnt != 0 && t0 < 64) sel[t0] = lane + 1;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      const uint32_t owner = wave_incl_max(sel[lane]);
      const uint64_t ow_word = __shfl(word, owner ? owner - 1 : 0);
      const uint64_t ow_t0 = __shfl(t0, owner ? owner - 1 : 0);
      if (owner != 0 && lane >= found && lane < found + total)
        my_end = (base + owner - 1) * 64 + select_bit(ow_word, (uint32_t)(lane - ow_t0));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      found += total;
      if (found >= 64 || base + 64 > W1) break;
      word = unary_word(base + 64 + lane);
    }
    const uint64_t prev_end = __shfl_up(my_end, 1);
    if (j < n_leaves) {
      uint64_t v = kNone;
      if (have && lane < found) {
        const uint64_t start = lane == 0 ? U0 : prev_end + 1;
        v = ((my_end - start) << k) | low;
      }
      values[j] = v;
    }
  }
}

int grid_for(uint64_t items, uint32_t per_block) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g > 16384) g = 16384;
  return g == 0 ? 1 : (int)g;
}

// One workgroup per group of 64 leaves, up to 2^20 workgroups (grid-stride beyond).
int query_grid(uint64_t n_leaves) {
  uint64_t g = (n_leaves + kQueryGroup - 1) / kQueryGroup;
  if (g > (1u << 20)) g = 1u << 20;
  return g == 0 ? 1 : (int)g;
}

bool load_table(const uint8_t *k_by_n, RiceTable &T) {
  if (!k_by_n) return false;
  for (int n = 0; n <= 64; ++n) {
    if (k_by_n[n] > kMaxRiceK) return false;
    T.k[n] = k_by_n[n];
  }
  return true;
}

}  // namespace

#define HIP_TRY(call)                       \
  do {                                      \
    hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) {                 \
      shock_internal_set_error(#call, e_);  \
      return SHOCK_EHIP;                    \
    }                                       \
  } while (0)

namespace {

// The encoder's three device words and their pinned host copy, cached per
// host thread and device (calls on one thread are synchronous), so an encode
// makes no allocation after the first.
struct EncodeScratch {
  uint64_t *dev = nullptr, *host = nullptr;
};
thread_local std::vector<EncodeScratch> t_encode;

hipError_t encode_scratch(uint64_t **dev_words, uint64_t **host_words) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return e;
  if ((int)t_encode.size() <= d) t_encode.resize(d + 1);
  EncodeScratch &S = t_encode[d];
  if (S.dev == nullptr) {
    e = hipMalloc((void **)&S.dev, 3 * sizeof(uint64_t));
    if (e != hipSuccess) {
      S.dev = nullptr;
      return e;
    }
  }
  if (S.host == nullptr) {
    e = hipHostMalloc((void **)&S.host, 3 * sizeof(uint64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
      S.host = nullptr;
      return e;
    }
  }
  *dev_words = S.dev;
  *host_words = S.host;
  return hipSuccess;
}

}  // namespace

hipError_t shock_internal_release_code_scratch(int dev) {
  if ((int)t_encode.size() <= dev) return hipSuccess;
  EncodeScratch &S = t_encode[dev];
  hipError_t e = hipSuccess;
  if (S.dev) e = hipFree(S.dev);
  if (S.host) {
    const hipError_t f = hipHostFree(S.host);
    if (e == hipSuccess) e = f;
  }
  S.dev = nullptr;
  S.host = nullptr;
  return e;
}

extern "C" {

int shock_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, const uint64_t *seeds,
                     const uint64_t *orient, uint64_t *out_pos, void *hip_stream) {
  if (n_leaves == 0) return SHOCK_OK;
  if (!keys || !offsets || !seeds || !orient || !out_pos || n_leaves > (1ull << 40)) return SHOCK_EINVAL;
  hipLaunchKernelGGL(query_kernel<false>, dim3(query_grid(n_leaves)), dim3(256), 0, (hipStream_t)hip_stream, keys,
                     offsets, n_leaves, seeds, (const uint32_t *)nullptr, orient, 0u, out_pos);
  HIP_TRY(hipGetLastError());
  return SHOCK_OK;
}

int shock_rf_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, const uint64_t *seeds,
                        const uint32_t *rot, const uint64_t *orient, int32_t partial_k, uint64_t *out_pos,
                        void *hip_stream) {
  if (n_leaves == 0) return SHOCK_OK;
  if (!keys || !offsets || !seeds || !rot || !orient || !out_pos || n_leaves > (1ull << 40)) return SHOCK_EINVAL;
  if (partial_k != 0 && partial_k != 1 && partial_k != 8) return SHOCK_EINVAL;
  hipLaunchKernelGGL(query_kernel<true>, dim3(query_grid(n_leaves)), dim3(256), 0, (hipStream_t)hip_stream, keys,
                     offsets, n_leaves, seeds, rot, orient, (uint32_t)partial_k, out_pos);
  HIP_TRY(hipGetLastError());
  return SHOCK_OK;
}

int shock_rice_encode(const uint64_t *values, const uint64_t *offsets, uint64_t n_leaves, const uint8_t *k_by_n,
                      uint64_t *fixed, uint64_t fixed_words, uint64_t *unary, uint64_t unary_words, uint64_t *index,
                      uint64_t *bits, void *hip_stream) {
  RiceTable T;
  if (!bits || !load_table(k_by_n, T) || !index) return SHOCK_EINVAL;
  if (n_leaves > 0 && (!values || !offsets)) return SHOCK_EINVAL;
  if (n_leaves > (1ull << 40)) return SHOCK_EINVAL;
  hipStream_t stream = (hipStream_t)hip_stream;
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  uint64_t *scratch = nullptr, *host = nullptr;  // [0] error bits, [1..2] totals
  HIP_TRY(encode_scratch(&scratch, &host));
  int rc = SHOCK_OK;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(64), 0, stream, scratch, (uint64_t)3);
  if (e == hipSuccess && n_blocks > 0) {
    hipLaunchKernelGGL(rice_len_kernel, dim3(grid_for(n_blocks, 4)), dim3(256), 0, stream, values, offsets, n_leaves,
                       T, index, (unsigned long long *)scratch);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(rice_scan_kernel, dim3(1), dim3(1024), 0, stream, index, n_blocks, scratch + 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host, scratch, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e == hipSuccess) {
    bits[0] = host[1];
    bits[1] = host[2];
    if (host[0] != 0) rc = SHOCK_EINVAL;
    else if ((host[1] + 63) / 64 > fixed_words || (host[2] + 63) / 64 > unary_words) rc = SHOCK_EINVAL;
    else if ((fixed_words && !fixed) || (unary_words && !unary)) rc = SHOCK_EINVAL;
  }
  if (e == hipSuccess && rc == SHOCK_OK) {
    if (fixed_words) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(fixed_words, 256)), dim3(256), 0, stream, fixed, fixed_words);
    if (unary_words) hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(unary_words, 256)), dim3(256), 0, stream, unary, unary_words);
    e = hipGetLastError();
    if (e == hipSuccess && n_blocks > 0) {
      hipLaunchKernelGGL(rice_write_kernel, dim3(grid_for(n_blocks, 4)), dim3(256), 0, stream, values, offsets,
                         n_leaves, T, index, (unsigned long long *)fixed, (unsigned long long *)unary,
                         (unsigned long long *)scratch);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  if (e != hipSuccess) {
    shock_internal_set_error("rice encode", e);
    return SHOCK_EHIP;
  }
  return rc;
}

int shock_rice_decode(const uint64_t *fixed, uint64_t fixed_words, const uint64_t *unary, uint64_t unary_words,
                      const uint64_t *index, const uint64_t *offsets, uint64_t n_leaves, const uint8_t *k_by_n,
                      uint64_t *values, void *hip_stream) {
  RiceTable T;
  if (!load_table(k_by_n, T)) return SHOCK_EINVAL;
  if (n_leaves == 0) return SHOCK_OK;
  if (!index || !offsets || !values || (fixed_words && !fixed) || (unary_words && !unary)) return SHOCK_EINVAL;
  if (n_leaves > (1ull << 40)) return SHOCK_EINVAL;
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  hipLaunchKernelGGL(rice_decode_kernel, dim3(grid_for(n_blocks, 4)), dim3(256), 0, (hipStream_t)hip_stream, fixed,
                     fixed_words, unary, unary_words, index, offsets, n_leaves, T, values);
  HIP_TRY(hipGetLastError());
  return SHOCK_OK;
}

}  // extern "C"
