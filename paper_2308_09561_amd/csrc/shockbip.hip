// Bipartite ShockHash (the outlook of Section 9) on MI355X (gfx950).
//
// The n cells of a leaf's table are split into a left part [0, nl) and a
// right part [nl, n), nl = floor(n / 2).  One evaluation of the frozen hash of
// key x under seed s gives both its left cell (the range reduction of z to
// [0, nl)) and its right cell (the leftover fraction reduced to [nl, n)).  A pair of seeds (a, b) gives key x the cells
// left(x, a) and right(x, b); the result is the first pair, in the order
// max(a, b), then a, then b, whose graph is a pseudoforest.
//
// One wave works on one leaf.  Per iteration lane l hashes seed base + l over
// the leaf's keys (premixed, LDS broadcasts) into a left and a right coverage
// mask; a seed whose left (right) cells cover the left (right) part joins the
// left (right) candidate pool, and only pairs of candidates can qualify
// (every cell needs a key).  Candidates are rare and pairs are formed as they
// arrive, so the seeds hashed grow like the square root of the pairs needed:
// the exponential gain over ShockHash the paper points to.  Each new
// candidate m is paired with the pool in the result order ((a, m) for left
// candidates a < m, then (m, b) for right candidates b <= m).  Each
// candidate, when it arrives, also records which keys are alone in their cell
// of its half.  A pair in which some key is alone in both of its cells has a
// one-edge tree, so with n keys on n cells it cannot be a pseudoforest: one
// AND of the two masks rejects it (most pairs, at full coverage of both
// halves).  The other pairs are checked by the wave-parallel peeling test.
// The pools (seed lists) and the first kFilter lone-key masks of each side
// stay in LDS, and so do the cells of the first kCache candidates of each
// side (one byte per key), so a pair test reads its partner's cells instead
// of hashing them again.  Workers take leaves from sixteen atomic counters,
// each over a slice of the batch; a leaf is short, so there is no work
// stealing within a leaf.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <vector>

#include "shockleaf.h"
#include "shock_hash.h"
#include "shock_internal.h"
#include "shock_wave.h"

namespace {

using shockhash::bip_cells;
using shockhash::fmix64;
using shockhash::seed_mix;
using shockwave::bcast64;
using shockwave::lane_id;
using shockwave::wave_lds_sync;

constexpr uint64_t kNone = ~0ull;
// Two passes.  The first keeps up to kPool candidates per side (four waves per
// workgroup, the pools with the rest of the wave's LDS); a leaf that gathers
// more is listed and searched again from its first seed by the second, one
// wave per workgroup with pools of up to kPoolBig (most of 64 KB of LDS).
// With a smaller limit L per side the first keeps L / 2 (at least 1) and the
// second L, so both passes run on small inputs too.  Uniform keys do not
// need the second: a leaf of 64 keys gathers about 35 candidates per side
// before its pair (1233 pairs formed per leaf), one of 48 keys about 13.
constexpr uint32_t kPool = 512;      // candidates per side and leaf, first pass
constexpr uint32_t kPoolBig = 7168;  // second pass
constexpr uint32_t kCache = 16;  // candidates per side whose cells are kept in LDS
constexpr uint32_t kFilter = 64;  // candidates per side whose lone-key masks are kept in LDS
constexpr uint32_t kWpw = 4;

// Device counters: three words for the batch, then one 256-byte line per
// slice of the batch: the slice's leaf counter and the statistics of the
// waves that started on it.
enum { kBipErr = 0, kBipNotFound = 1, kBipSpilled = 2 };
enum { kSliceNext = 0, kSliceSeeds = 1, kSlicePairs = 2, kSlicePeeled = 3 };
// Leaves are taken from kRanges counters, each over its own slice of the
// batch.  A workgroup starts on slice blockIdx % kRanges (two slices per
// XCD, which takes workgroups in turn); when that slice runs dry, its waves
// read all the counters at once and move to the next slice with leaves
// left.  A single counter for every wave is a queue: device-scope atomics on
// one address are serialised, and at twelve waves per CU the wait for a
// fresh leaf grew fivefold over one wave per SIMD (16384 leaves of 48 keys:
// 0.40 ms with one counter, 0.335 with 16).  The statistics are added on the
// slices' lines for the same reason.
constexpr uint32_t kBipRange = 8, kRangeStride = 32, kRanges = 16;
constexpr uint32_t kCtrWords = kBipRange + kRanges * kRangeStride;
constexpr uint64_t kErrInvalidLeaf = 1;
constexpr uint64_t kErrPool = 2;

template <uint32_t kP>
struct BipLds {
  uint64_t keys[64];
  unsigned long long inc0[64], inc1[64], hit;
  uint32_t pool_l[kP], pool_r[kP];
  uint8_t cell_l[kCache][64], cell_r[kCache][64];  // left (right) cell of key i under pool_l[q] (pool_r[q])
  uint64_t lone_l[kFilter], lone_r[kFilter];  // keys alone in their left (right) cell under pool_l[q] (pool_r[q])
};

struct BipParams {
  const uint64_t *keys, *offsets;
  uint64_t n_leaves, max_seed;  // n_leaves: of the batch, or of `list`
  uint64_t n_keys;  // keys in the keys buffer, 0 = unchecked
  uint32_t pool;    // candidates kept per side (at most the kernel's pool)
  const uint32_t *list;  // second pass: the leaves to search, or NULL (all)
  uint32_t *spill;       // first pass: where leaves past the pool are listed, or NULL (reported not found)
  uint64_t *out_a, *out_b, *out_orient;
  unsigned long long *ctr;
};

// Left cell l in [0, nl) and right cell index r in [0, nr) (the cell is
// nl + r) of a premixed key under a seed mix t.
__device__ __forceinline__ void bip_cell_idx(uint64_t a, uint64_t t, uint32_t nl, uint32_t nr, uint32_t &l,
                                             uint32_t &r) {
  const uint64_t p = (uint64_t)((uint32_t)a ^ (uint32_t)t) * (a >> 32) + t;
  const uint32_t z = (uint32_t)p ^ (uint32_t)(p >> 32);
  const uint64_t q = (uint64_t)z * nl;
  l = (uint32_t)(q >> 32);
  r = __umulhi((uint32_t)q, nr);
}



__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Cell of this lane's key under pool entry q of one side: from the LDS cache
// or hashed again.
template <class Lds>
__device__ __forceinline__ uint32_t pool_cell(uint64_t my_a, uint32_t q, bool left, uint32_t nl, uint32_t nr,
                                              const Lds &lds) {
  if (q < kCache) return left ? lds.cell_l[q][lane_id()] : lds.cell_r[q][lane_id()];
  uint32_t l, r;
  bip_cells(my_a, seed_mix(left ? lds.pool_l[q] : lds.pool_r[q]), nl, nr, l, r);
  return left ? l : r;
}

// Keys (lanes below n) alone in their left cell cl, and alone in their right
// cell cr, under one seed: a cell histogram as key masks in LDS.
template <class Lds>
__device__ __forceinline__ void lone_keys(uint32_t n, uint32_t cl, uint32_t cr, Lds &lds, uint64_t &lone_l,
                                          uint64_t &lone_r) {
  const uint32_t lane = lane_id();
  const bool act = lane < n;
  lds.inc0[lane] = 0;
  wave_lds_sync();
  if (act) {
    atomicOr(&lds.inc0[cl], 1ull << lane);
    atomicOr(&lds.inc0[cr], 1ull << lane);
  }
  wave_lds_sync();
  const uint64_t at_l = act ? lds.inc0[cl] : 0, at_r = act ? lds.inc0[cr] : 0;
  lone_l = __ballot(act && __popcll(at_l) == 1);
  lone_r = __ballot(act && __popcll(at_r) == 1);
  wave_lds_sync();
}

// Whether the pair with left cells cl and right cells cr (this lane's key)
// qualifies; lane i < n gets its edge in h0, h1.
template <class Lds>
__device__ bool bip_pair(uint32_t n, uint32_t cl, uint32_t cr, uint32_t &h0, uint32_t &h1, Lds &lds) {
  h0 = lane_id() < n ? cl : 0;
  h1 = lane_id() < n ? cr : 0;
  return shockwave::pf_peel_wave(n, h0, h1, lds.inc0);
}

template <uint32_t kP, uint32_t kW>
__global__ __launch_bounds__(64 * kW) void bip_kernel(BipParams P) {
  __shared__ BipLds<kP> lds_all[kW];
  BipLds<kP> &lds = lds_all[threadIdx.x >> 6];
  const uint32_t lane = lane_id();
  uint64_t seeds_hashed = 0, pairs = 0, peeled = 0;
  const uint32_t home = blockIdx.x % kRanges;
  uint32_t slice = home;  // the slice leaves are taken from
  for (;;) {
    uint64_t idx = kNone;
    for (;;) {
      const uint64_t lo = P.n_leaves * slice / kRanges, hi = P.n_leaves * (slice + 1) / kRanges;
      unsigned long long c = 0;
      if (lane == 0) c = atomicAdd(&P.ctr[kBipRange + slice * kRangeStride + kSliceNext], 1ull);
      c = bcast64(c);
      if (c < hi - lo) {
        idx = lo + c;
        break;
      }
      // the slice is dry (counters only grow): lane i reads slice i's counter.
      // Each pass finds one more slice dry, so at most kRanges passes run.
      bool open = false;
      if (lane < kRanges) {
        const unsigned long long v = __hip_atomic_load(&P.ctr[kBipRange + lane * kRangeStride + kSliceNext],
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        open = v < P.n_leaves * (lane + 1) / kRanges - P.n_leaves * lane / kRanges;
      }
      const uint64_t opened = __ballot(open);
      if (opened == 0) break;
      const uint64_t after = opened & ~((2ull << slice) - 1);  // open slices past this one
      slice = __builtin_ctzll(after ? after : opened);
    }
    if (idx == kNone) break;
    const uint64_t j = P.list ? P.list[idx] : idx;
    const uint64_t o0 = P.offsets[j], o1 = P.offsets[j + 1];
    if (o1 < o0 || o1 - o0 > 64 || (P.n_keys != 0 && o1 > P.n_keys)) {
      if (lane == 0) {
        atomicOr(&P.ctr[kBipErr], kErrInvalidLeaf);
        P.out_a[j] = kNone;
        P.out_b[j] = kNone;
        P.out_orient[j] = 0;
      }
      continue;
    }
    const uint32_t n = (uint32_t)(o1 - o0);
    if (n <= 1) {
      if (lane == 0) {
        P.out_a[j] = 0;
        P.out_b[j] = 0;
        P.out_orient[j] = 0;
      }
      continue;
    }
    const uint64_t my_a = lane < n ? fmix64(P.keys[o0 + lane]) : 0;
    lds.keys[lane] = my_a;
    wave_lds_sync();
    const uint32_t nl = n / 2, nr = n - nl;
    // each half has at most 32 cells: one 32-bit coverage word per half
    const uint32_t want_l = nl >= 32 ? ~0u : (1u << nl) - 1, want_r = nr >= 32 ? ~0u : (1u << nr) - 1;
    uint32_t n_l = 0, n_r = 0;
    bool found = false, overflow = false;
    uint64_t ra = kNone, rb = kNone;
    uint32_t fh0 = 0, fh1 = 0;
    for (uint64_t base = 0; base < P.max_seed && !found && !overflow; base += 64) {
      const uint64_t s = base + lane;
      const uint64_t t = seed_mix(s);
      uint32_t ml = 0, mr = 0;
      auto eval_key = [&](uint64_t a) {
        uint32_t l, r;
        bip_cell_idx(a, t, nl, nr, l, r);
        ml |= 1u << l;
        mr |= 1u << r;
      };
      // eight keys' LDS reads in flight at once
      uint32_t i = 0;
      for (; i + 8 <= n; i += 8) {
        uint64_t a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = lds.keys[i + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) eval_key(a[u]);
      }
      for (; i < n; ++i) eval_key(lds.keys[i]);
      const uint64_t span = P.max_seed - base;
      seeds_hashed += span < 64 ? span : 64;
      const bool in = s < P.max_seed;
      const uint64_t cl = __ballot(in && ml == want_l);
      const uint64_t cr = __ballot(in && mr == want_r);
      uint64_t any = cl | cr;
      while (any != 0 && !found && !overflow) {
        const uint32_t lm = __builtin_ctzll(any);
        any &= any - 1;
        const uint64_t m = base + lm;
        const bool is_l = (cl >> lm) & 1, is_r = (cr >> lm) & 1;
        // this lane's key's cells under the new candidate m, and the keys
        // alone in their left (right) cell under m
        uint32_t ml_cell, mr_cell;
        bip_cells(my_a, readlane64(t, lm), nl, nr, ml_cell, mr_cell);  // lane lm mixed seed m
        uint64_t m_lone_l, m_lone_r;
        lone_keys(n, ml_cell, mr_cell, lds, m_lone_l, m_lone_r);
        if (is_r) {
          for (uint32_t q0 = 0; q0 < n_l && !found; q0 += 64) {
            // pairs whose graph has an isolated edge (a key alone in both of its
            // cells: a one-edge tree) cannot qualify and are not peeled
            const uint32_t q = q0 + lane;
            const uint64_t lone = q < kFilter ? lds.lone_l[q] : 0;
            uint64_t todo = __ballot(q < n_l && (lone & m_lone_r) == 0);
            uint32_t formed = n_l - q0 < 64 ? n_l - q0 : 64;
            while (todo != 0 && !found) {
              const uint32_t qq = q0 + __builtin_ctzll(todo);
              todo &= todo - 1;
              ++peeled;
              if (bip_pair(n, pool_cell(my_a, qq, true, nl, nr, lds), mr_cell, fh0, fh1, lds)) {
                found = true;
                ra = lds.pool_l[qq];
                rb = m;
                formed = qq - q0 + 1;
              }
            }
            pairs += formed;
          }
          if (!found) {
            if (n_r == P.pool) overflow = true;
            else {
              if (lane == 0) lds.pool_r[n_r] = (uint32_t)m;
              if (lane == 0 && n_r < kFilter) lds.lone_r[n_r] = m_lone_r;
              if (n_r < kCache) lds.cell_r[n_r][lane] = (uint8_t)mr_cell;
              ++n_r;
              wave_lds_sync();
            }
          }
        }
        if (!found && !overflow && is_l) {
          for (uint32_t q0 = 0; q0 < n_r && !found; q0 += 64) {
            const uint32_t q = q0 + lane;
            const uint64_t lone = q < kFilter ? lds.lone_r[q] : 0;
            uint64_t todo = __ballot(q < n_r && (lone & m_lone_l) == 0);
            uint32_t formed = n_r - q0 < 64 ? n_r - q0 : 64;
            while (todo != 0 && !found) {
              const uint32_t qq = q0 + __builtin_ctzll(todo);
              todo &= todo - 1;
              ++peeled;
              if (bip_pair(n, ml_cell, pool_cell(my_a, qq, false, nl, nr, lds), fh0, fh1, lds)) {
                found = true;
                ra = m;
                rb = lds.pool_r[qq];
                formed = qq - q0 + 1;
              }
            }
            pairs += formed;
          }
          if (!found) {
            if (n_l == P.pool) overflow = true;
            else {
              if (lane == 0) lds.pool_l[n_l] = (uint32_t)m;
              if (lane == 0 && n_l < kFilter) lds.lone_l[n_l] = m_lone_l;
              if (n_l < kCache) lds.cell_l[n_l][lane] = (uint8_t)ml_cell;
              ++n_l;
              wave_lds_sync();
            }
          }
        }
      }
    }
    uint64_t f = 0;
    if (found && !shockwave::orient_wave(n, fh0, fh1, lds.inc0, lds.inc1, &lds.hit, f)) found = false;
    if (lane == 0) {
      if (overflow && P.spill) {  // searched again by the second pass
        P.spill[atomicAdd(&P.ctr[kBipSpilled], 1ull)] = (uint32_t)j;
      } else {
        if (overflow) atomicOr(&P.ctr[kBipErr], kErrPool);
        if (!found) atomicAdd(&P.ctr[kBipNotFound], 1ull);
      }
      P.out_a[j] = found ? ra : kNone;
      P.out_b[j] = found ? rb : kNone;
      P.out_orient[j] = found ? f : 0;
    }
    wave_lds_sync();
  }
  if (lane == 0) {
    unsigned long long *line = P.ctr + kBipRange + home * kRangeStride;
    if (seeds_hashed) atomicAdd(line + kSliceSeeds, (unsigned long long)seeds_hashed);
    if (pairs) atomicAdd(line + kSlicePairs, (unsigned long long)pairs);
    if (peeled) atomicAdd(line + kSlicePeeled, (unsigned long long)peeled);
  }
}

// Per host thread and device: the device counters and their pinned host
// copy, two timing events and the CU count, kept between calls (a hipFree
// per call would wait for the whole device, including other streams' work).
struct BipCache {
  unsigned long long *ctr = nullptr;
  unsigned long long *host = nullptr;  // pinned, kCtrWords words
  uint32_t *spill = nullptr;  // the first pass's list of leaves past its pool
  uint64_t spill_cap = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int cus = 0;
};
thread_local std::vector<BipCache> t_bip;

hipError_t bip_cache(int dev, BipCache *&c) {
  if ((int)t_bip.size() <= dev) t_bip.resize(dev + 1);
  c = &t_bip[dev];
  hipError_t e = hipSuccess;
  if (!c->ctr) e = hipMalloc((void **)&c->ctr, kCtrWords * sizeof(unsigned long long));
  if (e == hipSuccess && !c->host)
    e = hipHostMalloc((void **)&c->host, kCtrWords * sizeof(unsigned long long), hipHostMallocDefault);
  if (e == hipSuccess && !c->e0) e = hipEventCreate(&c->e0);
  if (e == hipSuccess && !c->e1) e = hipEventCreate(&c->e1);
  if (e == hipSuccess && !c->cus) {
    hipDeviceProp_t prop;
    c->cus = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 256;
  }
  return e;
}

}  // namespace

hipError_t shock_internal_release_bip_scratch(int dev) {
  if ((int)t_bip.size() <= dev) return hipSuccess;
  BipCache &c = t_bip[dev];
  hipError_t e = hipSuccess;
  if (c.ctr) e = hipFree(c.ctr);
  if (c.host) {
    const hipError_t f = hipHostFree(c.host);
    if (e == hipSuccess) e = f;
  }
  c.host = nullptr;
  if (c.spill) {
    const hipError_t f = hipFree(c.spill);
    if (e == hipSuccess) e = f;
  }
  c.spill = nullptr;
  c.spill_cap = 0;
  for (hipEvent_t *ev : {&c.e0, &c.e1}) {
    if (*ev) {
      const hipError_t f = hipEventDestroy(*ev);
      if (e == hipSuccess) e = f;
    }
    *ev = nullptr;
  }
  c.ctr = nullptr;
  c.cus = 0;
  return e;
}

extern "C" {

int shock_bip_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_a,
                             uint64_t *out_b, uint64_t *out_orient, const shock_opts *opts_in, void *hip_stream,
                             shock_bip_stats *stats) {
  shock_opts opts;
  shock_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n_leaves == 0) return SHOCK_OK;
  if (!keys || !offsets || !out_a || !out_b || !out_orient || n_leaves > (1ull << 31)) return SHOCK_EINVAL;
  if (opts.max_seed > (1ull << 32) || opts.workers < 0 || opts.workers > (1 << 20)) return SHOCK_EINVAL;
  if (opts.bip_pool < 0 || opts.bip_pool > (int32_t)kPoolBig) return SHOCK_EINVAL;
  hipStream_t stream = (hipStream_t)hip_stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  BipCache *cache = nullptr;
  hipError_t e = bip_cache(dev, cache);
  if (e != hipSuccess) {
    shock_internal_set_error("bipartite counters and events", e);
    return e == hipErrorOutOfMemory ? SHOCK_ENOMEM : SHOCK_EHIP;
  }
  unsigned long long *ctr = cache->ctr;
  unsigned long long *host = cache->host;  // the batch's counters, then the slices' lines
  uint64_t sums[4] = {0, 0, 0, 0};          // statistics over the slices and passes
  auto add_slices = [&]() {
    for (uint32_t r = 0; r < kRanges; ++r)
      for (uint32_t w = kSliceSeeds; w <= kSlicePeeled; ++w) sums[w] += host[kBipRange + r * kRangeStride + w];
  };
  // candidates kept per side in all; the first pass keeps half of them, at
  // most kPool, and lists the leaves past that for the second
  const uint32_t cap = opts.bip_pool ? (uint32_t)opts.bip_pool : kPoolBig;
  const uint32_t first = cap / 2 == 0 ? 1 : (cap / 2 < kPool ? cap / 2 : kPool);
  const bool second = cap > first;
  if (second && cache->spill_cap < n_leaves) {
    if (cache->spill) (void)hipFree(cache->spill);
    cache->spill = nullptr;
    cache->spill_cap = 0;
    e = hipMalloc((void **)&cache->spill, n_leaves * sizeof(uint32_t));
    if (e != hipSuccess) {
      cache->spill = nullptr;
      shock_internal_set_error("bipartite second-pass list", e);
      return e == hipErrorOutOfMemory ? SHOCK_ENOMEM : SHOCK_EHIP;
    }
    cache->spill_cap = n_leaves;
  }
  const int cus = cache->cus;
  // four waves per SIMD, as many as the LDS holds (16384 leaves of 48 keys:
  // 0.31 ms at four, 0.33 at three, 0.39 at two)
  uint64_t workers = opts.workers ? (uint64_t)opts.workers : (uint64_t)cus * 16;
  if (workers > n_leaves) workers = n_leaves;
  const uint32_t groups = (uint32_t)((workers + kWpw - 1) / kWpw);
  BipParams P;
  P.keys = keys;
  P.offsets = offsets;
  P.n_leaves = n_leaves;
  P.max_seed = opts.max_seed;
  P.n_keys = opts.n_keys;
  P.pool = first;
  P.list = nullptr;
  P.spill = second ? cache->spill : nullptr;
  P.out_a = out_a;
  P.out_b = out_b;
  P.out_orient = out_orient;
  P.ctr = ctr;
  hipEvent_t e0 = cache->e0, e1 = cache->e1;
  e = hipMemsetAsync(ctr, 0, kCtrWords * sizeof(host[0]), stream);
  if (e == hipSuccess) e = hipEventRecord(e0, stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((bip_kernel<kPool, kWpw>), dim3(groups), dim3(64 * kWpw), 0, stream, P);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(host, ctr, kCtrWords * sizeof(host[0]), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) add_slices();
  const uint64_t nsp = e == hipSuccess ? host[kBipSpilled] : 0;
  if (nsp > 0) {
    // the second pass over the listed leaves, one wave per workgroup
    P.list = cache->spill;
    P.n_leaves = nsp;
    P.pool = cap;
    P.spill = nullptr;
    e = hipMemsetAsync(ctr + kBipRange, 0, (kCtrWords - kBipRange) * sizeof(host[0]), stream);
    const uint64_t g2 = nsp < (uint64_t)cus * 2 ? nsp : (uint64_t)cus * 2;
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL((bip_kernel<kPoolBig, 1>), dim3((uint32_t)g2), dim3(64), 0, stream, P);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host, ctr, kCtrWords * sizeof(host[0]), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    float ms2 = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms2, e0, e1);
    if (e == hipSuccess) add_slices();
    ms += ms2;  // the two passes' kernel time
  }
  if (e != hipSuccess) {
    shock_internal_set_error("bipartite search", e);
    return SHOCK_EHIP;
  }
  if (stats) {
    stats->seeds_hashed = sums[kSliceSeeds];
    stats->pairs_tested = sums[kSlicePairs];
    stats->pairs_peeled = sums[kSlicePeeled];
    stats->kernel_ms = ms;
    stats->workers = (int32_t)(groups * kWpw);
    stats->second_pass_leaves = (int32_t)(nsp < 0x7fffffffull ? nsp : 0x7fffffffull);
  }
  if (host[kBipErr] & kErrInvalidLeaf) return SHOCK_EINVAL;
  if (host[kBipErr] & kErrPool) return SHOCK_ENOTFOUND;
  if (host[kBipNotFound]) return SHOCK_ENOTFOUND;
  return SHOCK_OK;
}

}  // extern "C"
