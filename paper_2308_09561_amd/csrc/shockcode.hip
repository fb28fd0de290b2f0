// Leaf queries and Golomb-Rice seed codes on MI355X (gfx950).
//
// Query (Section 4: a key x is answered by h_{s, f(x)}(x)): one wave per
// leaf, lane i evaluates key i of the leaf under the leaf's seed (and
// rotation) and picks slot h0 or h1 by bit i of the orientation.  The work is
// a few dozen integer operations per key against 16 bytes of traffic per key,
// so the kernel is bound by HBM; loads and stores of a leaf are contiguous.
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

template <bool RF>
__global__ __launch_bounds__(256) void query_kernel(const uint64_t *__restrict__ keys,
                                                    const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                    const uint64_t *__restrict__ seeds,
                                                    const uint32_t *__restrict__ rot,
                                                    const uint64_t *__restrict__ orient, uint32_t partial_k,
                                                    uint64_t *__restrict__ out_pos) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t j = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); j < n_leaves; j += waves) {
    const uint64_t o0 = offsets[j], o1 = offsets[j + 1];
    if (o1 < o0 || o1 - o0 > 64) continue;  // not a leaf: its keys are left untouched
    const uint32_t n = (uint32_t)(o1 - o0);
    if (lane >= n) continue;
    const uint64_t s = seeds[j];
    const uint64_t x = keys[o0 + lane];
    uint64_t pos = kNone;
    if (s != kNone) {
      uint32_t h0 = 0, h1 = 0;
      if (n >= 2) {
        const uint64_t a = fmix64(x);
        uint64_t sk = s;
        uint32_t r = 0;
        if (RF) {
          const uint32_t k = partial_k ? partial_k : (n > 32 ? 8u : 1u);
          if (key_side(x)) r = rot[j] % n;
          else sk = s - s % k;
        }
        const uint64_t t = seed_mix(sk);
        slot_pair((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)t, (uint32_t)(t >> 32), n, n - 1, h0, h1);
        if (RF) {
          h0 = h0 + r >= n ? h0 + r - n : h0 + r;
          h1 = h1 + r >= n ? h1 + r - n : h1 + r;
        }
      }
      pos = o0 + (((orient[j] >> lane) & 1) ? h1 : h0);
    }
    out_pos[o0 + lane] = pos;
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
// last pair and in totals[0..1].  One workgroup of 1024 threads, chunk by chunk.
__global__ __launch_bounds__(1024) void rice_scan_kernel(uint64_t *index, uint64_t n_blocks, uint64_t *totals) {
  __shared__ uint64_t sf[1024], su[1024];
  const uint32_t t = threadIdx.x;
  uint64_t carry_f = 0, carry_u = 0;
  for (uint64_t c = 0; c < n_blocks; c += 1024) {
    const uint64_t b = c + t;
    const uint64_t f = b < n_blocks ? index[2 * b] : 0;
    const uint64_t u = b < n_blocks ? index[2 * b + 1] : 0;
    sf[t] = f;
    su[t] = u;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
      const uint64_t af = t >= d ? sf[t - d] : 0;
      const uint64_t au = t >= d ? su[t - d] : 0;
      __syncthreads();
      sf[t] += af;
      su[t] += au;
      __syncthreads();
    }
    if (b < n_blocks) {
      index[2 * b] = carry_f + sf[t] - f;
      index[2 * b + 1] = carry_u + su[t] - u;
    }
    carry_f += sf[1023];
    carry_u += su[1023];
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

// Phase 3: write the codes.  The streams were zeroed and are large enough
// (checked on the host from the totals).
__global__ __launch_bounds__(256) void rice_write_kernel(const uint64_t *__restrict__ values,
                                                         const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                         RiceTable T, const uint64_t *__restrict__ index,
                                                         unsigned long long *fixed, unsigned long long *unary,
                                                         unsigned long long *err) {
  const uint32_t lane = threadIdx.x & 63;
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
    if (!have) continue;
    if (k != 0 && low != 0) {
      const uint64_t w = F >> 6;
      const uint32_t sh = (uint32_t)(F & 63);
      atomicOr(&fixed[w], (unsigned long long)(low << sh));
      if (sh + k > 64) atomicOr(&fixed[w + 1], (unsigned long long)(low >> (64 - sh)));
    }
    const uint64_t p = U + q;
    atomicOr(&unary[p >> 6], 1ull << (p & 63));
  }
}

// ---- Golomb-Rice decode -----------------------------------------------------

__global__ __launch_bounds__(256) void rice_decode_kernel(const uint64_t *__restrict__ fixed, uint64_t fixed_words,
                                                          const uint64_t *__restrict__ unary, uint64_t unary_words,
                                                          const uint64_t *__restrict__ index,
                                                          const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                          RiceTable T, uint64_t *__restrict__ values) {
  __shared__ uint64_t ones[4][64];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = threadIdx.x >> 6;
  uint64_t *pos = ones[wave];
  const uint64_t n_blocks = (n_leaves + 63) / 64;
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  for (uint64_t b = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave; b < n_blocks; b += waves) {
    const uint64_t j = b * 64 + lane;
    bool have = j < n_leaves;
    uint32_t k = 0;
    if (have) {
      const uint64_t o0 = offsets[j], o1 = offsets[j + 1];
      if (o1 < o0 || o1 - o0 > 64) have = false;
      else k = T.k[o1 - o0];
    }
    // low bits
    const uint64_t F = index[2 * b] + wave_excl_scan(k);
    uint64_t low = 0;
    if (have && k) {
      const uint64_t w = F >> 6;
      const uint32_t sh = (uint32_t)(F & 63);
      if (w < fixed_words) low = fixed[w] >> sh;
      if (sh + k > 64 && w + 1 < fixed_words) low |= fixed[w + 1] << (64 - sh);
      low &= ~0ull >> (64 - k);
    }
    // quotients: positions of the ones in [U0, U1)
    const uint64_t U0 = index[2 * b + 1], U1 = index[2 * b + 3];
    uint64_t found = 0;
    if (U1 > U0) {
      const uint64_t W0 = U0 >> 6, W1 = (U1 - 1) >> 6;
      for (uint64_t base = W0; base <= W1; base += 64) {
        const uint64_t w = base + lane;
        uint64_t word = (w <= W1 && w < unary_words) ? unary[w] : 0;
        if (w == W0) word &= ~0ull << (U0 & 63);
        if (w == W1 && (U1 & 63) != 0) word &= ~0ull >> (64 - (U1 & 63));
        uint64_t t = found + wave_excl_scan((uint64_t)__popcll(word));
        while (word != 0) {
          const uint32_t bit = __builtin_ctzll(word);
          word &= word - 1;
          if (t < 64) pos[t] = w * 64 + bit;
          ++t;
        }
        found = __shfl(t, 63);  // lane 63's count includes every lane's ones
        if (found >= 64) break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (j < n_leaves) {
      uint64_t v = kNone;
      if (have && lane < found) {
        const uint64_t end = pos[lane];
        const uint64_t start = lane == 0 ? U0 : pos[lane - 1] + 1;
        v = ((end - start) << k) | low;
      }
      values[j] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

int grid_for(uint64_t items, uint32_t per_block) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g > 16384) g = 16384;
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

extern "C" {

int shock_leaf_query(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, const uint64_t *seeds,
                     const uint64_t *orient, uint64_t *out_pos, void *hip_stream) {
  if (n_leaves == 0) return SHOCK_OK;
  if (!keys || !offsets || !seeds || !orient || !out_pos || n_leaves > (1ull << 40)) return SHOCK_EINVAL;
  hipLaunchKernelGGL(query_kernel<false>, dim3(grid_for(n_leaves, 4)), dim3(256), 0, (hipStream_t)hip_stream, keys,
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
  hipLaunchKernelGGL(query_kernel<true>, dim3(grid_for(n_leaves, 4)), dim3(256), 0, (hipStream_t)hip_stream, keys,
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
  uint64_t *scratch = nullptr;  // [0] error bits, [1..2] totals
  HIP_TRY(hipMalloc(&scratch, 3 * sizeof(uint64_t)));
  uint64_t host[3] = {0, 0, 0};
  int rc = SHOCK_OK;
  hipError_t e = hipMemcpyAsync(scratch, host, sizeof(host), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && n_blocks > 0) {
    hipLaunchKernelGGL(rice_len_kernel, dim3(grid_for(n_blocks, 4)), dim3(256), 0, stream, values, offsets, n_leaves,
                       T, index, (unsigned long long *)scratch);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(rice_scan_kernel, dim3(1), dim3(1024), 0, stream, index, n_blocks, scratch + 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host, scratch, sizeof(host), hipMemcpyDeviceToHost, stream);
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
  hipError_t ef = hipFree(scratch);
  if (e != hipSuccess) {
    shock_internal_set_error("rice encode", e);
    return SHOCK_EHIP;
  }
  if (ef != hipSuccess) {
    shock_internal_set_error("hipFree", ef);
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
