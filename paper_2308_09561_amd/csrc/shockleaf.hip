// ShockHash leaf seed search on MI355X (gfx950): kernels and the C ABI.
//
// The operation, hash family and output conventions are documented in
// include/shockleaf.h.  Design in brief:
//
//  * One wave (64 lanes) is one worker.  A worker holds one leaf at a time and
//    tests 64*SPL consecutive seeds per iteration, SPL seeds per lane.  The
//    leaf's premixed keys are wave-uniform and come from scalar loads, so the
//    per-(key, seed) work is pure VALU integer arithmetic: two xors, one
//    32x32->64 multiply, an xor fold, two fastrange multiplies, the h1
//    adjustment and the coverage bit-mask update (Section 4, filter by bit
//    mask; the mask lives in registers).
//  * A seed passes the filter when its mask covers all n cells; the wave
//    ballot of those lanes gives the survivors in seed order.  Each survivor
//    is confirmed by a wave-parallel union-find over the n cells in LDS
//    (Appendix A.1 uses union-find for this test; every component must hold no
//    more edges than nodes, the pseudoforest criterion of Section 2).
//  * Seeds of a leaf are handed out in blocks by an atomic counter, so several
//    workers can search one leaf.  Every block below the best accepted seed is
//    searched to its first acceptance; a block may be skipped only if its
//    first seed is not below the current best, so the minimum of the
//    definition in Section 4 is exact whatever the interleaving.
//  * Workers first take fresh leaves in order; once none are left they help
//    unfinished leaves (work stealing at seed-block granularity).  The last
//    worker to leave a closed leaf writes the seed and the canonical
//    orientation, computed wave-parallel by peeling (Section 5's peeling
//    process) and directing each cycle by its highest-index key.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "shockleaf.h"
#include "shock_hash.h"

#include "shock_internal.h"
#include "shock_wave.h"

namespace {

using shockhash::fmix64;
using shockhash::kGolden;
using shockhash::kSideKey;
using shockhash::slot_pair;

constexpr uint64_t kNone = ~0ull;
// Rotation fitting: candidates (s, r) are encoded as s * 64 + r, which orders
// them as the search does (seed first, then rotation).
constexpr uint32_t kRfPeriod = 8;        // the partial-hash period k: seeds s - s mod 8 share the first set's hash
constexpr uint32_t kRfSeedsPerLane = 2;  // consecutive seeds per lane and iteration: a quad covers one period

// Leaf claim word: bits 0..39 next unclaimed unit (a unit is one iteration:
// 64*SPL consecutive seeds, or 64*kRfSeedsPerLane under rotation fitting), bits
// 40..62 workers inside the leaf, bit 63 set once the leaf's result has been
// written.
constexpr uint64_t kBlockMask = (1ull << 40) - 1;
constexpr uint64_t kInflightOne = 1ull << 40;
constexpr uint64_t kInflightMask = ((1ull << 23) - 1) << 40;
constexpr uint64_t kFinalBit = 1ull << 63;

// Global counters of one call (uint64 each).  Atomics on one address
// serialise (about 12 ns each on MI355X), so the statistics are spread over
// kStatSlots slots that the host sums.
constexpr int kStatSlots = 64;
enum {
  kCtrErr = 0,        // error bits, see kErr*
  kCtrNotFound = 1,   // leaves that hit max_seed
  kCtrStats = 8,      // kStatSlots x {seeds hashed, filter passes, union-find tests, blocks}
  kCtrGlobalCount = 8 + kStatSlots * 4
};
enum { kStSeeds = 0, kStPasses = 1, kStPf = 2, kStBlocks = 3 };
// Per-launch counters (one set per kernel launch of a call).  Single-leaf
// launches count finished workgroups in kExitGroups group counters and one
// top counter, so no address sees more than ~64 increments.
constexpr int kExitGroups = 64;
enum { kLcNextLeaf = 0, kLcDone = 1, kLcExitTop = 2, kLcExitGroups = 4, kLcCount = 4 + kExitGroups };

constexpr uint64_t kErrInvalid = 1;
constexpr uint64_t kErrDup = 2;
constexpr uint64_t kErrOrient = 4;
constexpr uint64_t kErrCancel = 8;

constexpr int kMaxWavesPerWg = 16;

struct Params {
  const uint64_t *__restrict__ offsets;  // CSR offsets of the whole call
  const uint64_t *__restrict__ premix;   // [n_leaves][64] premixed keys fmix64(x), zero padded
  uint64_t leaf_begin;                   // first leaf of this launch
  uint64_t leaf_count;                   // leaves of this launch
  uint64_t start_seed, max_seed;
  uint64_t *__restrict__ out_seeds;
  uint64_t *__restrict__ out_orient;
  unsigned long long *state;  // [n_leaves] claim words
  unsigned long long *best;   // [n_leaves] smallest accepted seed so far
  unsigned int *wleaf;        // [workers] leaf each worker is on (scan table for helpers)
  unsigned long long *gctr;   // global counters of the call
  unsigned long long *lctr;   // counters of this launch
  const volatile int32_t *cancel;
  uint64_t block;        // seeds per claimed block = 64 * SPL * block_iters (split launches)
  uint64_t unit;         // seeds per claim unit = 64 * SPL
  uint32_t block_iters;  // units per block of a single-leaf (split) launch
  uint32_t workers;
  uint32_t split;  // 1: one leaf, static block striding over the workers (no claim atomics)
  uint32_t team;   // 1: the waves of a workgroup share each fresh leaf (persistent launches)
  uint32_t partial_k;  // rotation fitting (best holds candidates s * 64 + r): 0 = 8 above 32 keys else 1; or 1 / 8
  uint32_t *__restrict__ out_rot;              // rotation fitting: rotation per leaf
  const unsigned long long *__restrict__ sides;  // [n_leaves] bit i = set of key i
  uint16_t units_by_n[65];  // most units one claim takes, by leaf size (persistent launches)
};

using shockwave::bcast32;
using shockwave::bcast64;
using shockwave::lane_id;
using shockwave::wave_lds_sync;

// m |= a | b as one 3-input OR.  Written out because the compiler otherwise
// reassociates the mask updates of unrolled keys into two-input ORs.
__device__ __forceinline__ void or3_into(uint32_t &m, uint32_t a, uint32_t b) {
  asm("v_or3_b32 %0, %0, %1, %2" : "+v"(m) : "v"(a), "v"(b));
}


__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long *p) {
  return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether chunk index u (of `size` seeds each, counted from start) begins
// below lim.  u < 2^40 and size <= 2^24 by construction, so u * size cannot
// overflow; the host caps max_seed at 2^63.
__device__ __forceinline__ bool chunk_below(uint64_t u, uint64_t size, uint64_t start, uint64_t lim) {
  return start < lim && u * size < lim - start;
}

// Waves communicate only through device-scope atomics (claim words, best
// seeds, counters); every other buffer a kernel reads was written by an
// earlier kernel.  Ordering between a wave's atomics on different words comes
// from waiting for each returning atomic before issuing the next: the
// returned value is moved to scalar registers, which the hardware cannot do
// before the atomic has been performed.  No cache write-back or invalidate
// fences are needed.
__device__ __forceinline__ void depend_on(uint64_t v) { asm volatile("" ::"s"(v) : "memory"); }

// Lower *p to v if smaller; returns only after the update is performed.
__device__ __forceinline__ void wave_atomic_min_wait(unsigned long long *p, uint64_t v) {
  unsigned long long old = 0;
  if (lane_id() == 0) old = atomicMin(p, (unsigned long long)v);
  depend_on(bcast64(old));
}

// Wave-uniform atomic add done by lane 0.
__device__ __forceinline__ unsigned long long wave_atomic_add(unsigned long long *p, unsigned long long v) {
  unsigned long long old = 0;
  if (lane_id() == 0) old = atomicAdd(p, v);
  return bcast64(old);
}

// Per-wave LDS scratch: union-find arrays for the pseudoforest test, or
// incidence masks for the orientation (never live at the same time).
struct WaveLds {
  uint64_t keys[64];  // premixed keys of the leaf the wave is working on
  uint64_t keys_a[64];  // rotation fitting: premixed keys of the first set, compacted
  uint64_t keys_b[64];  // rotation fitting: premixed keys of the second set, compacted
  uint64_t rf_sides;    // rotation fitting: bit i set if key i is in the second set
  uint32_t rf_na, rf_nb;  // rotation fitting: sizes of the two sets
  uint64_t rf_masks[64][4];  // rotation fitting: lane l's coverage masks ma, mb of its two seeds (flagged lanes)
  union {
    struct {
      uint32_t parent[64];
      uint32_t ecount[64];
      uint32_t ncount[64];
    } uf;
    struct {
      unsigned long long inc0[64];
      unsigned long long inc1[64];
      unsigned long long hit;
    } ori;
  };
};

// Pseudoforest test of one seed, wave-parallel.  Lane i < n holds edge i
// (h0, h1); lane c < n also stands for cell c.  Components are found by
// union-find with min-index hooking and pointer jumping; the graph is a
// pseudoforest iff no component holds more edges than nodes.
__device__ bool pf_test_wave(uint32_t n, uint32_t h0, uint32_t h1, WaveLds &lds) {
  const uint32_t lane = lane_id();
  const bool act = lane < n;
  uint32_t *par = lds.uf.parent;
  par[lane] = lane;
  lds.uf.ecount[lane] = 0;
  lds.uf.ncount[lane] = 0;
  wave_lds_sync();
  for (int round = 0; round < 64; ++round) {
    for (int jump = 0; jump < 8; ++jump) {
      const uint32_t p = par[lane];
      const uint32_t pp = par[p];
      const bool changed = act && pp != p;
      wave_lds_sync();
      if (changed) par[lane] = pp;
      wave_lds_sync();
      if (__ballot(changed) == 0) break;
    }
    bool pending = false;
    if (act) {
      const uint32_t ru = par[h0];
      const uint32_t rv = par[h1];
      if (ru != rv) {
        atomicMin(&par[ru > rv ? ru : rv], ru < rv ? ru : rv);
        pending = true;
      }
    }
    wave_lds_sync();
    if (__ballot(pending) == 0) break;
  }
  if (act) {
    atomicAdd(&lds.uf.ecount[par[h0]], 1u);
    atomicAdd(&lds.uf.ncount[par[lane]], 1u);
  }
  wave_lds_sync();
  const bool bad = act && lds.uf.ecount[lane] > lds.uf.ncount[lane];
  return __ballot(bad) == 0;
}

// Canonical orientation (shockwave::orient_wave) on the wave's LDS.
__device__ __forceinline__ bool orient_wave(uint32_t n, uint32_t h0, uint32_t h1, WaveLds &lds, uint64_t &f_out) {
  return shockwave::orient_wave(n, h0, h1, lds.ori.inc0, lds.ori.inc1, &lds.ori.hit, f_out);
}

struct WaveStats {
  uint64_t seeds = 0, passes = 0, pf = 0, blocks = 0;
};

// Search seeds [base, end) of one leaf for the first seed whose graph is a
// pseudoforest.  `a` points at the leaf's premixed keys (wave-uniform).
// With `poll`, stops early once the leaf's best accepted seed is at or below
// the start of the next iteration; polling only matters when other workers
// hold lower parts of the leaf's seed range.  Returns kNone if no seed of the
// range qualifies.
template <int SPL, bool WIDE>
__device__ uint64_t search_block(const uint64_t *a, uint32_t n, uint64_t base, uint64_t end,
                                 const unsigned long long *best_j, bool poll, uint32_t my_alo, uint32_t my_ahi,
                                 WaveLds &lds, WaveStats &st) {
  const uint32_t lane = lane_id();
  const uint32_t nm1 = n - 1;
  const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1);
  for (uint64_t ib = base; ib < end; ib += 64 * SPL) {
    const unsigned long long cur_best = poll ? load_relaxed(best_j) : kNone;
    uint32_t tlo[SPL], thi[SPL], mlo[SPL], mhi[SPL];
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      const uint64_t s = ib + (uint64_t)(j * 64 + lane);
      const uint64_t t = fmix64((s + 1) * kGolden);
      tlo[j] = (uint32_t)t;
      thi[j] = (uint32_t)(t >> 32);
      mlo[j] = 0;
      mhi[j] = 0;
    }
    auto eval_key = [&](uint64_t ai) {
      const uint32_t alo = (uint32_t)ai, ahi = (uint32_t)(ai >> 32);
#pragma unroll
      for (int j = 0; j < SPL; ++j) {
        uint32_t h0, h1;
        slot_pair(alo, ahi, tlo[j], thi[j], n, nm1, h0, h1);
        if (WIDE) {
          const uint64_t b0 = 1ull << h0, b1 = 1ull << h1;
          or3_into(mlo[j], (uint32_t)b0, (uint32_t)b1);
          or3_into(mhi[j], (uint32_t)(b0 >> 32), (uint32_t)(b1 >> 32));
        } else {
          or3_into(mlo[j], 1u << h0, 1u << h1);
        }
      }
    };
    uint32_t i = 0;
    for (; i + 4 <= n; i += 4) {
      const uint64_t a0 = a[i], a1 = a[i + 1], a2 = a[i + 2], a3 = a[i + 3];
      eval_key(a0);
      eval_key(a1);
      eval_key(a2);
      eval_key(a3);
    }
    for (; i < n; ++i) eval_key(a[i]);
    const uint64_t span = end - ib;
    st.seeds += span < (uint64_t)(64 * SPL) ? span : (uint64_t)(64 * SPL);
#pragma unroll
    for (int j = 0; j < SPL; ++j) {
      const uint64_t m = WIDE ? (((uint64_t)mhi[j] << 32) | mlo[j]) : (uint64_t)mlo[j];
      const bool ok = m == full && (uint64_t)(j * 64 + lane) < span;
      uint64_t surv = __ballot(ok);
      while (surv != 0) {
        const uint32_t l = __builtin_ctzll(surv);
        surv &= surv - 1;
        const uint64_t s = ib + (uint64_t)(j * 64) + l;
        st.passes += 1;
        st.pf += 1;
        const uint64_t t = fmix64((s + 1) * kGolden);
        uint32_t h0 = 0, h1 = 0;
        slot_pair(my_alo, my_ahi, (uint32_t)t, (uint32_t)(t >> 32), n, nm1, h0, h1);
        if (pf_test_wave(n, h0, h1, lds)) return s;
      }
    }
    if (bcast64(cur_best) <= ib + 64 * SPL) break;
  }
  return kNone;
}


// ---- Rotation fitting (Section 4; partial hash calculation, Appendix A.2) --

// Coverage mask of `cnt` premixed keys (wave-uniform, LDS) under one seed.
template <bool WIDE>
__device__ __forceinline__ uint64_t cover_mask(const uint64_t *a, uint32_t cnt, uint32_t tlo, uint32_t thi, uint32_t n,
                                               uint32_t nm1) {
  uint32_t mlo = 0, mhi = 0;
  auto eval_key = [&](uint64_t ai) {
    uint32_t h0, h1;
    slot_pair((uint32_t)ai, (uint32_t)(ai >> 32), tlo, thi, n, nm1, h0, h1);
    if (WIDE) {
      const uint64_t b0 = 1ull << h0, b1 = 1ull << h1;
      or3_into(mlo, (uint32_t)b0, (uint32_t)b1);
      or3_into(mhi, (uint32_t)(b0 >> 32), (uint32_t)(b1 >> 32));
    } else {
      or3_into(mlo, 1u << h0, 1u << h1);
    }
  };
  uint32_t i = 0;
  for (; i + 4 <= cnt; i += 4) {
    const uint64_t a0 = a[i], a1 = a[i + 1], a2 = a[i + 2], a3 = a[i + 3];
    eval_key(a0);
    eval_key(a1);
    eval_key(a2);
    eval_key(a3);
  }
  for (; i < cnt; ++i) eval_key(a[i]);
  return WIDE ? (((uint64_t)mhi << 32) | mlo) : (uint64_t)mlo;
}

// Whether some rotation r in [0, n) makes rot_n(mb, r) | ma cover [0, n),
// rot_n moving bit i to (i + r) mod n.  With D = mb | mb << n (mb repeated),
// rot_n(mb, r) is bits [n - r, 2n - r) of D, so each rotation is one funnel
// shift (v_alignbit) per 32-bit word and an OR with ma (plus the bits at or
// above n).  A rotation covers iff that word (the AND of both words above 32
// keys) is all ones, the largest 32-bit value, so the test keeps a running
// maximum (v_max3, two rotations per instruction) in a vector register
// instead of a lane mask per rotation.  `pad` has every bit at or above n set.
__device__ __forceinline__ uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t m = a > b ? a : b;
  return m > c ? m : c;
}

template <bool WIDE>
__device__ __forceinline__ bool any_rotation_covers(uint64_t ma, uint64_t mb, uint32_t n, uint64_t pad) {
  const uint64_t z = ma | pad;
  const uint64_t m0 = mb | z;  // r = 0
  uint32_t acc = (uint32_t)m0 & (uint32_t)(m0 >> 32);
  if (!WIDE) {
    const uint32_t z32 = (uint32_t)z;
    const uint64_t d = mb | (mb << n);  // n <= 32: 2n bits
    const uint32_t d0 = (uint32_t)d, d1 = (uint32_t)(d >> 32);
    uint32_t sh = 1;
    for (; sh + 1 < n; sh += 2)
      acc = umax3(acc, __builtin_amdgcn_alignbit(d1, d0, sh) | z32, __builtin_amdgcn_alignbit(d1, d0, sh + 1) | z32);
    if (sh < n) acc = umax3(acc, acc, __builtin_amdgcn_alignbit(d1, d0, sh) | z32);
  } else {
    const uint32_t zlo = (uint32_t)z, zhi = (uint32_t)(z >> 32);
    const unsigned __int128 d = (unsigned __int128)mb | ((unsigned __int128)mb << n);  // 33 <= n <= 64
    const uint32_t w0 = (uint32_t)d, w1 = (uint32_t)(d >> 32), w2 = (uint32_t)(d >> 64), w3 = (uint32_t)(d >> 96);
    auto word = [&](uint32_t a1, uint32_t a0, uint32_t b1, uint32_t b0, uint32_t sh) {
      return (__builtin_amdgcn_alignbit(a1, a0, sh) | zlo) & (__builtin_amdgcn_alignbit(b1, b0, sh) | zhi);
    };
    for (uint32_t sh = 1; sh < 31; sh += 2)  // shifts 1..30, then 31 with the next range's first
      acc = umax3(acc, word(w1, w0, w2, w1, sh), word(w1, w0, w2, w1, sh + 1));
    uint32_t sh = 0;  // shifts 32 + sh
    acc = umax3(acc, word(w1, w0, w2, w1, 31), word(w2, w1, w3, w2, 0));
    for (sh = 1; sh + 33 < n; sh += 2)
      acc = umax3(acc, word(w2, w1, w3, w2, sh), word(w2, w1, w3, w2, sh + 1));
    if (sh + 32 < n) acc = umax3(acc, acc, word(w2, w1, w3, w2, sh));
  }
  return acc == ~0u;
}

// Slots of this lane's key (lane < n) under candidate (s, r).
__device__ __forceinline__ void rf_lane_slots(uint32_t my_alo, uint32_t my_ahi, uint32_t my_side, uint64_t s, uint32_t r,
                                              bool partial, uint32_t n, uint32_t &h0, uint32_t &h1) {
  const uint64_t sa = partial ? s - (s % kRfPeriod) : s;
  const uint64_t t = fmix64(((my_side ? s : sa) + 1) * kGolden);
  slot_pair(my_alo, my_ahi, (uint32_t)t, (uint32_t)(t >> 32), n, n - 1, h0, h1);
  if (my_side) {
    h0 += r;
    h0 = h0 >= n ? h0 - n : h0;
    h1 += r;
    h1 = h1 >= n ? h1 - n : h1;
  }
}

// Pseudoforest test by peeling (shockwave::pf_peel_wave) on the wave's LDS.
__device__ __forceinline__ bool pf_peel_wave(uint32_t n, uint32_t h0, uint32_t h1, WaveLds &lds) {
  return shockwave::pf_peel_wave(n, h0, h1, lds.ori.inc0);
}

// Rotations of seed s whose graphs pass the coverage filter, one bit per
// rotation: lane r tests rotation r on the seed's two coverage masks ma, mb
// (wave-uniform, as the lane that tested the seed left them in LDS).  h0, h1
// return this lane's slots under (s, 0) for the pseudoforest test.
__device__ uint64_t rf_rotations(uint32_t n, uint64_t s, bool partial, uint32_t my_alo, uint32_t my_ahi,
                                 uint32_t my_side, uint64_t ma, uint64_t mb, uint32_t &h0, uint32_t &h1) {
  const uint32_t lane = lane_id();
  h0 = 0;
  h1 = 0;
  if (lane < n) rf_lane_slots(my_alo, my_ahi, my_side, s, 0, partial, n, h0, h1);
  const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1);
  const uint64_t rot = lane == 0 ? mb : ((mb << lane) | (mb >> (n - lane))) & full;
  return __ballot(lane < n && (rot | ma) == full);
}

// DPP quad permutations (within each aligned group of 4 lanes).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  return ((uint64_t)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}
constexpr int kDppXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int kDppQuad0 = 0x00;  // quad_perm [0, 0, 0, 0]

__device__ __forceinline__ uint64_t quad_or(uint64_t x) {
  x |= dpp64<kDppXor1>(x);
  return x | dpp64<kDppXor2>(x);
}

// Search seeds [base, end) of one leaf for the first candidate (s, r), in the
// order s ascending then r ascending, whose graph is a pseudoforest.  An
// iteration covers 64 * kRfSeedsPerLane consecutive seeds from a start aligned
// to the partial-hash period (seeds outside [base, end) are masked); lane l
// takes seeds ib + 2l and ib + 2l + 1, so each quad of lanes holds one period.
// With partial hashing the quad shares the first set's seed s - s mod 8: each
// lane hashes every 4th key of that set and the quad ORs the masks.  Returns
// the encoded candidate s * 64 + r, or kNone.
template <bool WIDE>
__device__ uint64_t rf_search_block(uint32_t n, uint32_t na, uint32_t nb, bool partial, uint64_t base, uint64_t end,
                                    const unsigned long long *best_j, bool poll, uint32_t my_alo, uint32_t my_ahi,
                                    uint32_t my_side, WaveLds &lds, WaveStats &st) {
  static_assert(kRfSeedsPerLane == 2 && kRfPeriod == 8, "a quad of lanes covers one partial-hash period");
  const uint32_t lane = lane_id();
  const uint32_t nm1 = n - 1;
  const uint64_t full = n >= 64 ? ~0ull : ((1ull << n) - 1);
  const uint64_t pad = ~full;
  constexpr uint32_t kSeeds = 64 * kRfSeedsPerLane;
  const uint64_t ib0 = base - base % kRfPeriod;
  for (uint64_t ib = ib0; ib < end; ib += kSeeds) {
    const unsigned long long cur_best = poll ? load_relaxed(best_j) : kNone;
    const uint64_t s0 = ib + (uint64_t)lane * kRfSeedsPerLane;
    const uint64_t t0 = fmix64((s0 + 1) * kGolden);
    const uint64_t t1 = fmix64((s0 + 2) * kGolden);
    uint64_t ma0, ma1;
    if (partial) {
      // the quad's first lane holds seed s0 = ib + 8q, the period start
      const uint64_t ta = dpp64<kDppQuad0>(t0);
      uint32_t mlo = 0, mhi = 0;
      for (uint32_t k = lane & 3; k < na; k += 4) {
        const uint64_t ak = lds.keys_a[k];
        uint32_t h0, h1;
        slot_pair((uint32_t)ak, (uint32_t)(ak >> 32), (uint32_t)ta, (uint32_t)(ta >> 32), n, nm1, h0, h1);
        if (WIDE) {
          const uint64_t b0 = 1ull << h0, b1 = 1ull << h1;
          or3_into(mlo, (uint32_t)b0, (uint32_t)b1);
          or3_into(mhi, (uint32_t)(b0 >> 32), (uint32_t)(b1 >> 32));
        } else {
          or3_into(mlo, 1u << h0, 1u << h1);
        }
      }
      ma0 = ma1 = quad_or(((uint64_t)mhi << 32) | mlo);
    } else {
      ma0 = cover_mask<WIDE>(lds.keys_a, na, (uint32_t)t0, (uint32_t)(t0 >> 32), n, nm1);
      ma1 = cover_mask<WIDE>(lds.keys_a, na, (uint32_t)t1, (uint32_t)(t1 >> 32), n, nm1);
    }
    const uint64_t mb0 = cover_mask<WIDE>(lds.keys_b, nb, (uint32_t)t0, (uint32_t)(t0 >> 32), n, nm1);
    const uint64_t mb1 = cover_mask<WIDE>(lds.keys_b, nb, (uint32_t)t1, (uint32_t)(t1 >> 32), n, nm1);
    uint32_t flags = 0;
    if (any_rotation_covers<WIDE>(ma0, mb0, n, pad) && s0 >= base && s0 < end) flags |= 1u;
    if (any_rotation_covers<WIDE>(ma1, mb1, n, pad) && s0 + 1 >= base && s0 + 1 < end) flags |= 2u;
    if (flags != 0) {
      lds.rf_masks[lane][0] = ma0;
      lds.rf_masks[lane][1] = mb0;
      lds.rf_masks[lane][2] = ma1;
      lds.rf_masks[lane][3] = mb1;
    }
    wave_lds_sync();
    const uint64_t lo = ib > base ? ib : base;
    const uint64_t hi = ib + kSeeds < end ? ib + kSeeds : end;
    st.seeds += hi - lo;
    uint64_t surv = __ballot(flags != 0);
    while (surv != 0) {
      const uint32_t l = __builtin_ctzll(surv);
      surv &= surv - 1;
      uint32_t fl = __builtin_amdgcn_readlane(flags, l);
      while (fl != 0) {
        const uint32_t i = __builtin_ctz(fl);
        fl &= fl - 1;
        const uint64_t s = ib + (uint64_t)l * kRfSeedsPerLane + i;
        uint32_t g0, g1;
        uint64_t rots = rf_rotations(n, s, partial, my_alo, my_ahi, my_side, lds.rf_masks[l][2 * i],
                                     lds.rf_masks[l][2 * i + 1], g0, g1);
        while (rots != 0) {
          const uint32_t r = __builtin_ctzll(rots);
          rots &= rots - 1;
          st.passes += 1;
          st.pf += 1;
          // second-set slots move by r (mod n); both are below n
          const uint32_t add = my_side ? r : 0u;
          const uint32_t h0 = g0 + add >= n ? g0 + add - n : g0 + add;
          const uint32_t h1 = g1 + add >= n ? g1 + add - n : g1 + add;
          if (pf_peel_wave(n, h0, h1, lds)) return s * 64 + r;
        }
      }
    }
    if (bcast64(cur_best) <= (ib + kSeeds) * 64) break;
  }
  return kNone;
}

// Split the leaf's keys into the two sets in LDS (compacted, input order).
__device__ void rf_stage(const Params &P, uint64_t j, uint32_t n, uint64_t ai, uint32_t &na, uint32_t &nb,
                         uint32_t &my_side, WaveLds &lds) {
  const uint32_t lane = lane_id();
  const uint64_t valid = n >= 64 ? ~0ull : ((1ull << n) - 1);
  const uint64_t sides = P.sides[j] & valid;
  my_side = (uint32_t)((sides >> lane) & 1);
  const uint64_t below = lane == 0 ? 0 : (~0ull >> (64 - lane));
  const uint32_t rank_b = __popcll(sides & below);
  const uint32_t rank_a = __popcll(~sides & valid & below);
  if (lane < n) {
    if (my_side) lds.keys_b[rank_b] = ai;
    else lds.keys_a[rank_a] = ai;
  }
  nb = (uint32_t)__popcll(sides);
  na = n - nb;
  if (lane == 0) {
    lds.rf_sides = sides;
    lds.rf_na = na;
    lds.rf_nb = nb;
  }
  wave_lds_sync();
}

// Seed-space limit of a leaf from its best value (an encoded candidate under
// rotation fitting): seeds at or above it cannot improve the result.
template <bool RF>
__device__ __forceinline__ uint64_t seed_limit(uint64_t best) {
  if (best == kNone || !RF) return best;
  return (best >> 6) + ((best & 63) != 0 ? 1 : 0);
}

// Write the result of leaf j.  Called by exactly one worker per leaf.
template <bool RF>
__device__ void finalize_leaf(const Params &P, uint64_t j, uint32_t n, WaveLds &lds) {
  const uint32_t lane = lane_id();
  const uint64_t b = bcast64(load_relaxed(&P.best[j]));
  const uint64_t s = (b == kNone || !RF) ? b : (b >> 6);
  const uint32_t r = (b == kNone || !RF) ? 0u : (uint32_t)(b & 63);
  uint64_t seed_out = s, f = 0;
  if (s == kNone) {
    if (lane == 0) atomicAdd(&P.gctr[kCtrNotFound], 1ull);
    f = 0;
  } else if (n >= 2) {
    const uint64_t ai = P.premix[j * 64 + lane];
    uint32_t h0 = 0, h1 = 0;
    if (RF) {
      const uint32_t my_side = (uint32_t)((P.sides[j] >> lane) & 1);
      const bool partial = P.partial_k ? P.partial_k == kRfPeriod : n > 32;
      rf_lane_slots((uint32_t)ai, (uint32_t)(ai >> 32), my_side, s, r, partial, n, h0, h1);
    } else {
      const uint64_t t = fmix64((s + 1) * kGolden);
      slot_pair((uint32_t)ai, (uint32_t)(ai >> 32), (uint32_t)t, (uint32_t)(t >> 32), n, n - 1, h0, h1);
    }
    if (!orient_wave(n, h0, h1, lds, f)) {
      if (lane == 0) atomicOr(&P.gctr[kCtrErr], kErrOrient);
    }
  }
  if (lane == 0) {
    P.out_seeds[j] = seed_out;
    P.out_orient[j] = f;
    if (RF) P.out_rot[j] = r;
    atomicAdd(&P.lctr[kLcDone], 1ull);
  }
}

template <int SPL, bool RF>
__device__ uint64_t search_range(const Params &P, uint64_t j, uint32_t n, uint64_t base, uint64_t end, bool poll,
                                 uint32_t my_alo, uint32_t my_ahi, WaveLds &lds, WaveStats &st) {
  const uint64_t *a = lds.keys;
  if (n <= 1) return RF ? base * 64 : base;  // every seed qualifies
  if (RF) {
    // the leaf's split, staged in LDS by rf_stage
    const uint32_t na = bcast32(lds.rf_na), nb = bcast32(lds.rf_nb);
    const uint32_t my_side = (uint32_t)((lds.rf_sides >> lane_id()) & 1);
    const bool partial = P.partial_k ? P.partial_k == kRfPeriod : n > 32;
    if (n <= 32) return rf_search_block<false>(n, na, nb, partial, base, end, &P.best[j], poll, my_alo, my_ahi, my_side, lds, st);
    return rf_search_block<true>(n, na, nb, partial, base, end, &P.best[j], poll, my_alo, my_ahi, my_side, lds, st);
  }
  if (n <= 32) return search_block<SPL, false>(a, n, base, end, &P.best[j], poll, my_alo, my_ahi, lds, st);
  return search_block<SPL, true>(a, n, base, end, &P.best[j], poll, my_alo, my_ahi, lds, st);
}

// Work on leaf j until it is closed: claim runs of units in order, search
// each.  A worker alone on a leaf claims block_iters units at a time; with k
// workers inside it claims about block_iters/k, so speculative work beyond
// the answer stays small when many helpers share a leaf.
template <int SPL, bool RF>
__device__ void work_leaf(const Params &P, uint64_t j, bool helper, WaveLds &lds, WaveStats &st) {
  const uint32_t lane = lane_id();
  const uint64_t unit = P.unit;
  const uint64_t o0 = P.offsets[j], o1 = P.offsets[j + 1];
  const uint32_t n = (uint32_t)(o1 - o0);
  const uint64_t ai = P.premix[j * 64 + lane];
  const uint32_t my_alo = (uint32_t)ai, my_ahi = (uint32_t)(ai >> 32);
  lds.keys[lane] = ai;
  if (RF) {
    uint32_t na, nb, side;
    rf_stage(P, j, n, ai, na, nb, side, lds);
  }
  wave_lds_sync();
  const uint64_t most = P.units_by_n[n];
  uint64_t take = helper ? 1 : most;  // a helper does not know the crowd yet
  uint64_t claim = wave_atomic_add(&P.state[j], kInflightOne + take);
  if (claim & kFinalBit) {
    wave_atomic_add(&P.state[j], (unsigned long long)(0 - kInflightOne));
    return;
  }
  for (;;) {
    const uint64_t u = claim & kBlockMask;
    const uint64_t bst = seed_limit<RF>(bcast64(load_relaxed(&P.best[j])));
    const uint64_t lim = bst < P.max_seed ? bst : P.max_seed;
    if (!chunk_below(u, unit, P.start_seed, lim)) break;
    if (P.cancel != nullptr && *P.cancel != 0) {
      if (lane == 0) atomicOr(&P.gctr[kCtrErr], kErrCancel);
      break;
    }
    const uint64_t base = P.start_seed + u * unit;
    const uint64_t span = take * unit;
    const uint64_t end = (lim - base) < span ? lim : base + span;
    st.blocks += 1;
    const uint64_t inflight = (claim & kInflightMask) >> 40;
    // Claim the next run now and read the answer after this run's search, so
    // the atomic's round trip overlaps the hashing.  A claimed run is either
    // searched or skipped because it starts at or above the best seed, so
    // claiming ahead never loses a seed below the minimum.
    uint64_t next_take = most / (inflight ? inflight : 1);
    if (next_take == 0) next_take = 1;
    unsigned long long next_claim = 0;
    if (lane == 0) next_claim = atomicAdd(&P.state[j], (unsigned long long)next_take);
    // Alone on the leaf at claim time: later joiners claim higher seeds, so no
    // one can lower best below this range and polling is pointless.
    const uint64_t found = search_range<SPL, RF>(P, j, n, base, end, inflight > 1, my_alo, my_ahi, lds, st);
    if (found != kNone) wave_atomic_min_wait(&P.best[j], found);
    take = next_take;
    claim = bcast64(next_claim);
  }
  const uint64_t old = wave_atomic_add(&P.state[j], (unsigned long long)(0 - kInflightOne));
  if (((old & kInflightMask) >> 40) == 1) {
    bool cancelled = P.cancel != nullptr && *P.cancel != 0;
    if (!cancelled) {
      unsigned long long was = 0;
      if (lane == 0) was = atomicOr(&P.state[j], kFinalBit);
      was = bcast64(was);
      if (!(was & kFinalBit)) finalize_leaf<RF>(P, j, n, lds);
    }
  }
}

// One leaf searched by all workers of the launch with a static split: worker
// w takes blocks w, w + W, w + 2W, ...  A worker stops at its first block
// that starts at or above the best seed found so far, so every block below
// the final best is searched to its first acceptance.  The last worker to
// finish (counted per workgroup in LDS, then per launch) writes the result.
template <int SPL, bool RF>
__device__ void split_leaf(const Params &P, uint64_t j, uint32_t wid, WaveLds &lds, WaveStats &st,
                           uint32_t *wg_exits) {
  const uint32_t lane = lane_id();
  const uint64_t block = P.block;
  const uint32_t n = (uint32_t)(P.offsets[j + 1] - P.offsets[j]);
  const uint64_t ai = P.premix[j * 64 + lane];
  lds.keys[lane] = ai;
  if (RF) {
    uint32_t na, nb, side;
    rf_stage(P, j, n, ai, na, nb, side, lds);
  }
  wave_lds_sync();
  for (uint64_t b = wid;; b += P.workers) {
    const uint64_t bst = seed_limit<RF>(bcast64(load_relaxed(&P.best[j])));
    const uint64_t lim = bst < P.max_seed ? bst : P.max_seed;
    if (b >= (1ull << 40) || !chunk_below(b, block, P.start_seed, lim)) break;
    if (P.cancel != nullptr && *P.cancel != 0) {
      if (lane == 0) atomicOr(&P.gctr[kCtrErr], kErrCancel);
      break;
    }
    const uint64_t base = P.start_seed + b * block;
    const uint64_t end = (lim - base) < block ? lim : base + block;
    st.blocks += 1;
    const uint64_t found = search_range<SPL, RF>(P, j, n, base, end, true, (uint32_t)ai, (uint32_t)(ai >> 32), lds, st);
    if (found != kNone) wave_atomic_min_wait(&P.best[j], found);
  }
  uint32_t c = 0;
  if (lane == 0) c = atomicAdd(wg_exits, 1u);
  c = bcast32(c);
  const uint32_t wpw = blockDim.x >> 6;
  if (c != wpw - 1) return;
  // Workgroup done: count it in its group, then count finished groups.
  const uint32_t groups = gridDim.x < (uint32_t)kExitGroups ? gridDim.x : (uint32_t)kExitGroups;
  const uint32_t grp = blockIdx.x % groups;
  const uint32_t members = gridDim.x / groups + (grp < gridDim.x % groups ? 1u : 0u);
  const uint64_t gc = wave_atomic_add(&P.lctr[kLcExitGroups + grp], 1);
  if (gc != members - 1) return;
  const uint64_t g = wave_atomic_add(&P.lctr[kLcExitTop], 1);
  if (g != groups - 1) return;
  if (P.cancel != nullptr && *P.cancel != 0) return;
  unsigned long long was = 0;
  if (lane == 0) was = atomicOr(&P.state[j], kFinalBit);
  was = bcast64(was);
  if (!(was & kFinalBit)) finalize_leaf<RF>(P, j, n, lds);
}

// Pick a leaf to help: an unfinished leaf whose next block still lies below
// its best seed.  Helpers scan the table of leaves the workers are on (or the
// launch's leaves directly when there are at most 64) in chunks of 64 and pick
// a candidate by rotating the ballot with the worker id, which spreads helpers
// over the open leaves.  Returns kNone if no open leaf was seen.
template <bool RF>
__device__ uint64_t find_help_leaf(const Params &P, uint32_t wid) {
  const uint32_t lane = lane_id();
  const uint64_t end = P.leaf_begin + P.leaf_count;
  const bool direct = P.leaf_count <= 64;
  const uint32_t n_entries = direct ? (uint32_t)P.leaf_count : P.workers;
  const uint32_t chunks = (n_entries + 63) / 64;
  const uint32_t first = direct ? 0 : (wid * 2654435761u) % chunks;
  for (uint32_t c = 0; c < chunks; ++c) {
    const uint32_t chunk = (first + c) % chunks;
    const uint32_t idx = chunk * 64 + lane;
    uint64_t leaf = kNone;
    if (idx < n_entries) {
      if (direct) {
        leaf = P.leaf_begin + idx;
      } else {
        const uint32_t w = __hip_atomic_load(&P.wleaf[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (w != 0xFFFFFFFFu) leaf = w;
      }
    }
    bool open = false;
    if (leaf != kNone && leaf >= P.leaf_begin && leaf < end) {
      const uint64_t stw = load_relaxed(&P.state[leaf]);
      const uint64_t bst = seed_limit<RF>(load_relaxed(&P.best[leaf]));
      const uint64_t lim = bst < P.max_seed ? bst : P.max_seed;
      open = !(stw & kFinalBit) && chunk_below(stw & kBlockMask, P.unit, P.start_seed, lim);
    }
    const uint64_t cand = __ballot(open);
    if (cand != 0) {
      const uint32_t rot = wid & 63;
      const uint64_t rotated = rot ? ((cand >> rot) | (cand << (64 - rot))) : cand;
      const uint32_t pick = (__builtin_ctzll(rotated) + rot) & 63;
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)leaf, pick);
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(leaf >> 32), pick);
      return ((uint64_t)hi << 32) | lo;
    }
  }
  return kNone;
}

__device__ __forceinline__ void flush_stats(const Params &P, const WaveStats &st, uint32_t wid) {
  if (lane_id() == 0) {
    unsigned long long *slot = P.gctr + kCtrStats + (wid % kStatSlots) * 4;
    if (st.seeds) atomicAdd(slot + kStSeeds, (unsigned long long)st.seeds);
    if (st.passes) atomicAdd(slot + kStPasses, (unsigned long long)st.passes);
    if (st.pf) atomicAdd(slot + kStPf, (unsigned long long)st.pf);
    if (st.blocks) atomicAdd(slot + kStBlocks, (unsigned long long)st.blocks);
  }
}

// Plain search (RF false, SPL seeds per lane) or rotation fitting (RF true;
// SPL unused): separate instances, so each gets its own register budget.  The
// rotation-fitting instance is held to 96 registers, five waves per SIMD (the
// occupancy its launch is sized for).
template <int SPL, bool RF>
__global__ __launch_bounds__(64 * kMaxWavesPerWg) __attribute__((amdgpu_waves_per_eu(RF ? 5 : 1)))
void search_kernel(Params P) {
  extern __shared__ unsigned long long lds_raw[];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const uint32_t wpw = blockDim.x >> 6;
  WaveLds &lds = reinterpret_cast<WaveLds *>(lds_raw)[wave];
  uint32_t *wg_exits = reinterpret_cast<uint32_t *>(reinterpret_cast<WaveLds *>(lds_raw) + wpw);
  const uint32_t wid = blockIdx.x * wpw + wave;
  WaveStats st;
  // A batch that failed validation (checked by prepare_kernel) is not searched.
  if (__hip_atomic_load(&P.gctr[kCtrErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (kErrInvalid | kErrDup)) return;
  if (P.split) {
    if (threadIdx.x == 0) *wg_exits = 0;
    __syncthreads();
    split_leaf<SPL, RF>(P, P.leaf_begin, wid, lds, st, wg_exits);
    flush_stats(P, st, wid);
    return;
  }
  bool fresh = true;
  if (P.team) {
    // Fresh leaves for the whole workgroup: thread 0 draws one (or ends the
    // phase, also on cancel) and every wave of the group works on it, so all
    // waves pass the same barriers.  Then each wave helps on its own.
    unsigned long long *shared_leaf = reinterpret_cast<unsigned long long *>(wg_exits);
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) {
        unsigned long long next = kNone;
        if (P.cancel != nullptr && *P.cancel != 0) {
          atomicOr(&P.gctr[kCtrErr], kErrCancel);
        } else {
          const unsigned long long k = atomicAdd(&P.lctr[kLcNextLeaf], 1ull);
          if (k < P.leaf_count) next = P.leaf_begin + k;
        }
        *shared_leaf = next;
      }
      __syncthreads();
      const uint64_t j = *shared_leaf;
      if (j == kNone) break;
      if (P.leaf_count > 64 && lane == 0)
        __hip_atomic_store(&P.wleaf[wid], (uint32_t)j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      work_leaf<SPL, RF>(P, j, wave != 0, lds, st);
    }
    fresh = false;
  }
  uint32_t idle_rounds = 0;
  for (;;) {
    if (P.cancel != nullptr && *P.cancel != 0) {
      if (lane == 0) atomicOr(&P.gctr[kCtrErr], kErrCancel);
      break;
    }
    uint64_t j = kNone;
    bool helper = false;
    if (fresh) {
      const uint64_t k = wave_atomic_add(&P.lctr[kLcNextLeaf], 1);
      if (k < P.leaf_count) j = P.leaf_begin + k;
      else fresh = false;
    }
    if (j == kNone) {
      helper = true;
      j = find_help_leaf<RF>(P, wid);
      if (j == kNone) {
        // Nothing open to help: leave, so that a kernel queued behind this
        // one can use the slot.  A few retries cover owners that have not yet
        // published their leaf.
        if (load_relaxed(&P.lctr[kLcDone]) >= P.leaf_count || ++idle_rounds > 16) break;
        __builtin_amdgcn_s_sleep(32);
        continue;
      }
      idle_rounds = 0;
    }
    if (P.leaf_count > 64 && lane == 0) __hip_atomic_store(&P.wleaf[wid], (uint32_t)j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    work_leaf<SPL, RF>(P, j, helper, lds, st);
  }
  flush_stats(P, st, wid);
}

// Validate the batch, initialise per-leaf state and premix the keys.  One
// wave per leaf; lane i premixes key i.  Also checks repeated keys on request.
// A nonzero n_keys bounds the keys buffer: a leaf reaching past it is invalid
// and none of its keys is read.
__global__ __launch_bounds__(256) void prepare_kernel(const uint64_t *__restrict__ keys,
                                                      const uint64_t *__restrict__ offsets, uint64_t n_leaves,
                                                      uint64_t n_keys, uint64_t *__restrict__ premix,
                                                      unsigned long long *state, unsigned long long *best,
                                                      unsigned long long *gctr, unsigned long long *sides,
                                                      int check_dups) {
  const uint64_t j = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63;
  if (j >= n_leaves) return;
  const uint64_t o0 = offsets[j], o1 = offsets[j + 1];
  if (o1 < o0 || o1 - o0 > 64 || (n_keys != 0 && o1 > n_keys)) {
    if (lane == 0) atomicOr(&gctr[kCtrErr], kErrInvalid);
    return;
  }
  const uint32_t n = (uint32_t)(o1 - o0);
  uint64_t x = 0;
  if (lane < n) x = keys[o0 + lane];
  premix[j * 64 + lane] = lane < n ? fmix64(x) : 0;
  const uint64_t side_bits = __ballot(lane < n && (fmix64(x ^ kSideKey) >> 63) != 0);
  if (lane == 0) {
    state[j] = 0;
    best[j] = kNone;
    sides[j] = side_bits;
  }
  if (check_dups) {
    bool dup = false;
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, k);
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), k);
      const uint64_t y = ((uint64_t)hi << 32) | lo;
      dup |= (lane < n && k != lane && y == x);
    }
    if (__ballot(dup) != 0 && lane == 0) atomicOr(&gctr[kCtrErr], kErrDup);
  }
}

__global__ void init_counters_kernel(unsigned long long *gctr, unsigned long long *lctr, uint64_t n_lctr,
                                     unsigned int *wleaf, uint32_t workers) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kCtrGlobalCount) gctr[i] = 0;
  if (i < n_lctr) lctr[i] = 0;
  if (i < workers) wleaf[i] = 0xFFFFFFFFu;
}

// Leaves left unfinished by a cancelled call report "no seed".  Does nothing
// unless the call was cancelled.
__global__ void mark_unfinished_kernel(const unsigned long long *gctr, const unsigned long long *state,
                                       uint64_t n_leaves, uint64_t *out_seeds, uint64_t *out_orient,
                                       uint32_t *out_rot) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!(gctr[kCtrErr] & kErrCancel) || (gctr[kCtrErr] & (kErrInvalid | kErrDup))) return;
  if (j < n_leaves && !(state[j] & kFinalBit)) {
    out_seeds[j] = kNone;
    out_orient[j] = 0;
    if (out_rot) out_rot[j] = 0;
  }
}


// ------------------------------------------------------------------ host --

thread_local char g_err[512];
thread_local shock_stats g_stats;

void set_err(const char *what, hipError_t e) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                 \
  do {                                \
    hipError_t e_ = (call);           \
    if (e_ != hipSuccess) {           \
      set_err(#call, e_);             \
      return SHOCK_EHIP;              \
    }                                 \
  } while (0)

// Scratch of one call: premixed keys, claim words, best seeds, the worker
// table and counters.
struct Layout {
  size_t premix, state, best, sides, wleaf, gctr, lctr, total;
};

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr Layout layout(uint64_t n_leaves, uint32_t workers, uint64_t n_launches) {
  auto up = up256;
  Layout l{};
  size_t o = 0;
  l.premix = o; o = up(o + n_leaves * 64 * 8);
  l.state = o; o = up(o + n_leaves * 8);
  l.best = o; o = up(o + n_leaves * 8);
  l.sides = o; o = up(o + n_leaves * 8);
  l.wleaf = o; o = up(o + (size_t)workers * 4);
  l.gctr = o; o = up(o + kCtrGlobalCount * 8);
  l.lctr = o; o = up(o + n_launches * kLcCount * 8);
  l.total = o;
  return l;
}

// Rough expected number of seeds per leaf of n keys: the bound of the
// construction theorem, (e/2)^n * e / sqrt(pi) (Section 5), shrunk by
// 1.5 sqrt(n), which tracks the exact loop-free expectation within ~20% for
// 16 <= n <= 64.  Only used to size launches.
double expected_seeds(uint32_t n) {
  if (n < 2) return 1.0;
  const double e = 2.718281828459045;
  double v = 1.0;
  for (uint32_t i = 0; i < n; ++i) v *= e / 2.0;
  v *= e / 1.7724538509055159 / (1.5 * sqrt((double)n));
  return v < 1.0 ? 1.0 : v;
}

// Default most units (of 64*spl seeds) one claim takes, by leaf size, as the
// autotuner found on MI355X: claims shrink by themselves when several workers
// share a leaf, so large leaves prefer large claims (fewer atomics).
int default_units(uint32_t n) {
  if (n <= 28) return 32;
  if (n <= 36) return 1;
  if (n <= 44) return 16;
  if (n <= 60) return 64;
  return 32;
}

// Workers for a single-leaf (split) launch: enough blocks to cover about
// twice the expected seed count in one round, at least one workgroup.
int plain_workers(uint32_t n, uint64_t block, int wpw, int max_workers, int rf) {
  double w = 2.0 * expected_seeds(n) / (rf && n > 1 ? (double)n : 1.0) / (double)block;
  int wi = w > max_workers ? max_workers : (int)w;
  if (wi < wpw) wi = wpw;
  return (wi / wpw) * wpw;
}

template <int SPL, bool RF>
hipError_t launch_search(const Params &P, int wpw, hipStream_t stream) {
  const uint32_t wgs = P.workers / wpw;
  hipLaunchKernelGGL((search_kernel<SPL, RF>), dim3(wgs), dim3(64 * wpw), sizeof(WaveLds) * wpw + 16, stream, P);
  return hipGetLastError();
}

hipError_t launch_search_spl(int spl, int rf, const Params &P, int wpw, hipStream_t stream) {
  if (rf) return launch_search<1, true>(P, wpw, stream);
  switch (spl) {
    case 1: return launch_search<1, false>(P, wpw, stream);
    case 4: return launch_search<4, false>(P, wpw, stream);
    default: return launch_search<2, false>(P, wpw, stream);
  }
}

// Resident workers the device holds for a search kernel configuration
// (cached per device, kernel instance and waves per workgroup).
int resident_workers(int spl, int rf, int wpw) {
  static std::mutex mu;
  static int cache[16][5][kMaxWavesPerWg + 1];
  int dev = 0, cus = 256, per_cu = 0;
  (void)hipGetDevice(&dev);
  const int si = rf ? 0 : spl == 1 ? 1 : spl == 4 ? 4 : 2;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 16 && cache[dev][si][wpw] > 0) return cache[dev][si][wpw];
  }
  {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
  }
  const void *fn = si == 0   ? (const void *)search_kernel<1, true>
                   : si == 1 ? (const void *)search_kernel<1, false>
                   : si == 4 ? (const void *)search_kernel<4, false>
                             : (const void *)search_kernel<2, false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * wpw, sizeof(WaveLds) * wpw + 16) != hipSuccess ||
      per_cu <= 0)
    per_cu = 32 / wpw;
  const int w = per_cu * cus * wpw;
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 16) cache[dev][si][wpw] = w;
  return w;
}

// Everything needed to enqueue one call.
struct Plan {
  int mode;
  int rf;
  int spl, units, wpw, workers;
  uint64_t n_launches;
  uint16_t units_by_n[65];
};

// Rotation fitting: claim units are 64 lanes x 8 seeds and a leaf needs
// about n times fewer seeds, so claims are small.
int default_rf_units(uint32_t) { return 2; }

// Default workers of a persistent launch.  A full device of workers on a
// small batch crowds each leaf's claim word (thousands of atomics on one
// address) and searches past the answers, which costs far more than it
// gains: 16384 leaves want every resident wave, but ten 48-key leaves ran 4x
// faster with 512 waves than with 5120.  Measured on MI355X over 10 to 10000
// leaves, about one wave per leaf does best for light leaves, with at least
// 512 workers.  Heavy leaves (more than ~1000 claim units of expected work:
// plain search above 44 keys) get one wave per 128 units, up to 32: with
// only four waves per leaf, 256 leaves of 64 keys held one wave per SIMD and
// ran 20% below a full device.
int batch_workers(int resident, uint64_t n_leaves, uint32_t n, int rf, int spl) {
  const double unit = 64.0 * (rf ? kRfSeedsPerLane : spl);
  const double units = expected_seeds(n) / (rf && n > 1 ? (double)n : 1.0) / unit;
  const uint64_t per_leaf = units >= 1000.0 ? (units >= 4096.0 ? 32 : (uint64_t)(units / 128.0)) : 1;
  const uint64_t want = n_leaves * per_leaf < 512 ? 512 : n_leaves * per_leaf;
  return want < (uint64_t)resident ? (int)want : resident;
}

int make_plan(const shock_opts &opts, uint64_t n_leaves, uint32_t n_typical, int rf, Plan &pl) {
  pl.mode = opts.mode == SHOCK_MODE_AUTO ? SHOCK_MODE_PERSISTENT : opts.mode;
  if (pl.mode != SHOCK_MODE_PERSISTENT && pl.mode != SHOCK_MODE_PLAIN_PER_LEAF) return SHOCK_EINVAL;
  pl.rf = rf;
  pl.spl = opts.spl ? opts.spl : 2;
  pl.wpw = opts.waves_per_wg ? opts.waves_per_wg : 4;
  pl.units = opts.block_iters ? opts.block_iters
                              : (pl.mode == SHOCK_MODE_PLAIN_PER_LEAF ? 1
                                                                      : (rf ? default_rf_units(n_typical)
                                                                            : default_units(n_typical)));
  for (int n = 0; n <= 64; ++n) {
    int u = opts.block_iters ? opts.block_iters : (rf ? default_rf_units((uint32_t)n) : default_units((uint32_t)n));
    if (opts.block_iters_by_n && opts.block_iters_by_n[n] > 0) u = opts.block_iters_by_n[n];
    pl.units_by_n[n] = (uint16_t)(u > 65535 ? 65535 : u);
  }
  int w = opts.workers ? opts.workers : resident_workers(pl.spl, rf, pl.wpw);
  if (!opts.workers && pl.mode == SHOCK_MODE_PERSISTENT) w = batch_workers(w, n_leaves, n_typical, rf, pl.spl);
  w = ((w + pl.wpw - 1) / pl.wpw) * pl.wpw;
  if (w <= 0) return SHOCK_EINVAL;
  pl.workers = w;
  pl.n_launches = pl.mode == SHOCK_MODE_PLAIN_PER_LEAF ? n_leaves : 1;
  return SHOCK_OK;
}

int check_opts(const shock_opts &opts, uint64_t n_leaves, const void *offsets, const void *out_seeds,
               const void *out_orient) {
  if (!offsets || !out_seeds || !out_orient) return SHOCK_EINVAL;
  if (n_leaves > (1ull << 31)) return SHOCK_EINVAL;
  if (opts.max_seed > (1ull << 63)) return SHOCK_EINVAL;
  if (opts.spl != 0 && opts.spl != 1 && opts.spl != 2 && opts.spl != 4) return SHOCK_EINVAL;
  if (opts.block_iters < 0 || opts.block_iters > (1 << 16)) return SHOCK_EINVAL;
  if (opts.waves_per_wg < 0 || opts.waves_per_wg > kMaxWavesPerWg) return SHOCK_EINVAL;
  if (opts.workers < 0 || opts.workers > (1 << 20)) return SHOCK_EINVAL;
  if (opts.leaf_size_hint < 0 || opts.leaf_size_hint > 64) return SHOCK_EINVAL;
  if (opts.partial_k != 0 && opts.partial_k != 1 && opts.partial_k != 8) return SHOCK_EINVAL;
  if (opts.team < 0 || opts.team > 2) return SHOCK_EINVAL;
  return SHOCK_OK;
}

// Device buffers and host mirrors of one call.
struct CallBufs {
  uint64_t *premix;
  unsigned long long *state, *best, *sides, *gctr, *lctr;
  unsigned int *wleaf;
};

CallBufs carve(void *buf, const Layout &lay) {
  char *b = (char *)buf;
  CallBufs c;
  c.premix = (uint64_t *)(b + lay.premix);
  c.state = (unsigned long long *)(b + lay.state);
  c.best = (unsigned long long *)(b + lay.best);
  c.sides = (unsigned long long *)(b + lay.sides);
  c.wleaf = (unsigned int *)(b + lay.wleaf);
  c.gctr = (unsigned long long *)(b + lay.gctr);
  c.lctr = (unsigned long long *)(b + lay.lctr);
  return c;
}

hipError_t enqueue_prologue(const CallBufs &cb, const Plan &pl, const uint64_t *keys, const uint64_t *offsets,
                            uint64_t n_leaves, const shock_opts &opts, uint32_t workers_cap, hipStream_t stream) {
  const uint64_t n_l = pl.n_launches * kLcCount;
  uint64_t m = n_l > (uint64_t)workers_cap ? n_l : (uint64_t)workers_cap;
  if (m < (uint64_t)kCtrGlobalCount) m = kCtrGlobalCount;
  hipLaunchKernelGGL(init_counters_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, cb.gctr, cb.lctr,
                     n_l, cb.wleaf, workers_cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)((n_leaves + 3) / 4)), dim3(256), 0, stream, keys, offsets,
                     n_leaves, opts.n_keys, cb.premix, cb.state, cb.best, cb.gctr, cb.sides, opts.check_dups);
  return hipGetLastError();
}

Params base_params(const CallBufs &cb, const Plan &pl, const shock_opts &opts, const uint64_t *offsets,
                   uint64_t *out_seeds, uint64_t *out_orient, uint32_t *out_rot) {
  Params P;
  memset(&P, 0, sizeof(P));
  P.offsets = offsets;
  P.premix = cb.premix;
  P.start_seed = opts.start_seed;
  P.max_seed = opts.max_seed;
  P.out_seeds = out_seeds;
  P.out_orient = out_orient;
  P.out_rot = out_rot;
  P.state = cb.state;
  P.best = cb.best;
  P.wleaf = cb.wleaf;
  P.gctr = cb.gctr;
  P.cancel = opts.cancel;
  P.block_iters = (uint32_t)pl.units;
  P.unit = pl.rf ? 64ull * kRfSeedsPerLane : 64ull * (uint64_t)pl.spl;
  P.block = P.unit * (uint64_t)pl.units;
  P.partial_k = (uint32_t)opts.partial_k;
  P.team = opts.team == 1 ? 0u : 1u;
  P.sides = cb.sides;
  P.workers = (uint32_t)pl.workers;
  memcpy(P.units_by_n, pl.units_by_n, sizeof(P.units_by_n));
  return P;
}

// Enqueue the search kernel(s).  leaf_sizes (host, n_leaves + 1 offsets) sizes
// per-leaf launches when known; otherwise n_typical is used for every leaf.
hipError_t enqueue_search(Params P, const CallBufs &cb, const Plan &pl, uint64_t n_leaves, const uint64_t *h_off,
                          uint32_t n_typical, bool workers_fixed, hipStream_t stream) {
  if (pl.mode == SHOCK_MODE_PERSISTENT) {
    P.leaf_begin = 0;
    P.leaf_count = n_leaves;
    P.lctr = cb.lctr;
    P.split = 0;
    return launch_search_spl(pl.spl, pl.rf, P, pl.wpw, stream);
  }
  P.split = 1;
  for (uint64_t j = 0; j < n_leaves; ++j) {
    P.leaf_begin = j;
    P.leaf_count = 1;
    P.lctr = cb.lctr + j * kLcCount;
    const uint32_t nj = h_off ? (uint32_t)(h_off[j + 1] - h_off[j]) : n_typical;
    P.workers = workers_fixed ? (uint32_t)pl.workers
                              : (uint32_t)plain_workers(nj, P.block, pl.wpw, pl.workers, pl.rf);
    hipError_t e = launch_search_spl(pl.spl, pl.rf, P, pl.wpw, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int status_from(const unsigned long long *host_ctr, shock_stats *st) {
  if (st) {
    for (int i = 0; i < kStatSlots; ++i) {
      const unsigned long long *slot = host_ctr + kCtrStats + i * 4;
      st->seeds_tested += slot[kStSeeds];
      st->filter_passes += slot[kStPasses];
      st->pf_checks += slot[kStPf];
      st->blocks_claimed += slot[kStBlocks];
    }
  }
  const uint64_t err = host_ctr[kCtrErr];
  if (err & kErrInvalid) return SHOCK_EINVAL;
  if (err & kErrDup) return SHOCK_EDUPKEY;
  if (err & kErrOrient) {
    snprintf(g_err, sizeof(g_err), "internal error: orientation of an accepted seed is not a bijection");
    return SHOCK_EHIP;
  }
  if (err & kErrCancel) return SHOCK_ECANCELED;
  if (host_ctr[kCtrNotFound] != 0) return SHOCK_ENOTFOUND;
  return SHOCK_OK;
}

// Scratch cache of the synchronous entry points, per host thread and device:
// a synchronous call holds its scratch until it returns, so calls from
// different threads must not share it.
struct Scratch {
  void *buf = nullptr;
  size_t bytes = 0;
  void *host_ctr = nullptr;  // pinned copy of the global counters
};
thread_local std::vector<Scratch> t_scratch;

int get_scratch(size_t bytes, void **buf, unsigned long long **host_ctr) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if ((int)t_scratch.size() <= dev) t_scratch.resize(dev + 1);
  Scratch &s = t_scratch[dev];
  if (s.host_ctr == nullptr) {
    hipError_t e = hipHostMalloc(&s.host_ctr, kCtrGlobalCount * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
      set_err("hipHostMalloc", e);
      return SHOCK_ENOMEM;
    }
  }
  if (s.bytes < bytes) {
    if (s.buf) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(s.buf));
      s.buf = nullptr;
      s.bytes = 0;
    }
    hipError_t e = hipMalloc(&s.buf, bytes);
    if (e != hipSuccess) {
      set_err("hipMalloc(scratch)", e);
      return SHOCK_ENOMEM;
    }
    s.bytes = bytes;
  }
  *buf = s.buf;
  *host_ctr = (unsigned long long *)s.host_ctr;
  return SHOCK_OK;
}

// Scratch is laid out for the largest worker count any launch may use.
constexpr uint32_t kCallWorkersCap = 32 * 256 * 4 + kMaxWavesPerWg;

// Enqueue a whole search (init, validation and premix, search, unfinished
// marks, counters copied to host_ctr) on `stream` with no host
// synchronisation.  `buf` holds layout(n_leaves, kCallWorkersCap, launches)
// bytes; launch sizes come from n_typical.  opts are complete (max_seed set).
int enqueue_call(void *buf, uint64_t n_leaves, const uint64_t *keys, const uint64_t *offsets, uint64_t *out_seeds,
                 uint32_t *out_rot, uint64_t *out_orient, const shock_opts &opts, uint32_t n_typical,
                 hipStream_t stream, unsigned long long *host_ctr, hipEvent_t ev_begin, hipEvent_t ev_search,
                 Plan &pl) {
  int rc = make_plan(opts, n_leaves, n_typical, out_rot != nullptr, pl);
  if (rc != SHOCK_OK) return rc;
  if (pl.workers > (int)kCallWorkersCap) return SHOCK_EINVAL;
  const CallBufs cb = carve(buf, layout(n_leaves, kCallWorkersCap, pl.n_launches));
  HIP_TRY(enqueue_prologue(cb, pl, keys, offsets, n_leaves, opts, kCallWorkersCap, stream));
  Params P = base_params(cb, pl, opts, offsets, out_seeds, out_orient, out_rot);
  if (ev_begin) HIP_TRY(hipEventRecord(ev_begin, stream));
  HIP_TRY(enqueue_search(P, cb, pl, n_leaves, nullptr, n_typical, opts.workers != 0, stream));
  if (ev_search) HIP_TRY(hipEventRecord(ev_search, stream));
  hipLaunchKernelGGL(mark_unfinished_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, stream, cb.gctr,
                     cb.state, n_leaves, out_seeds, out_orient, out_rot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host_ctr, cb.gctr, kCtrGlobalCount * 8, hipMemcpyDeviceToHost, stream));
  return SHOCK_OK;
}

// Options with defaults filled in, checked as every entry point checks them.
int complete_opts(const shock_opts *in, uint64_t n_leaves, const void *keys, const void *offsets,
                  const void *out_seeds, const void *out_orient, int rf, shock_opts &opts) {
  shock_opts_init(&opts);
  if (in) opts = *in;
  if (opts.max_seed == 0) opts.max_seed = SHOCK_DEFAULT_MAX_SEED;
  const int rc = check_opts(opts, n_leaves, offsets, out_seeds, out_orient);
  if (rc != SHOCK_OK) return rc;
  if (!keys) return SHOCK_EINVAL;
  if (rf && opts.max_seed > (1ull << 57)) return SHOCK_EINVAL;
  return SHOCK_OK;
}

}  // namespace

void shock_internal_set_error(const char *what, hipError_t e) { set_err(what, e); }

size_t shock_internal_search_bytes(uint64_t n_leaves, int per_leaf) {
  return layout(n_leaves, kCallWorkersCap, per_leaf ? n_leaves : 1).total;
}

size_t shock_internal_counter_bytes(void) { return kCtrGlobalCount * 8; }

int shock_internal_complete_opts(const shock_opts *in, uint64_t n_leaves, const void *keys, const void *offsets,
                                 const void *out_seeds, const void *out_orient, int rf, shock_opts *out) {
  return complete_opts(in, n_leaves, keys, offsets, out_seeds, out_orient, rf, *out);
}

int shock_internal_enqueue(void *buf, uint64_t n_leaves, const uint64_t *keys, const uint64_t *offsets,
                           uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts,
                           uint32_t n_typical, hipStream_t stream, unsigned long long *host_ctr) {
  Plan pl;
  return enqueue_call(buf, n_leaves, keys, offsets, out_seeds, out_rot, out_orient, *opts, n_typical, stream,
                      host_ctr, nullptr, nullptr, pl);
}

int shock_internal_status(const unsigned long long *host_ctr) { return status_from(host_ctr, nullptr); }

// A search context: its own scratch for batches of up to max_leaves leaves,
// pinned counters, events and an optional captured graph.
struct shock_ctx {
  int device = 0;
  uint64_t max_leaves = 0;
  uint32_t workers_cap = 0;
  void *buf = nullptr;
  size_t bytes = 0;
  unsigned long long *host_ctr = nullptr;
  hipEvent_t ev_begin = nullptr, ev_search = nullptr, ev_done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  Plan last_plan{};
  bool pending = false;
};

extern "C" {

void shock_opts_init(shock_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->max_seed = SHOCK_DEFAULT_MAX_SEED;
  o->mode = SHOCK_MODE_AUTO;
}

const char *shock_last_error(void) { return g_err; }

const char *shock_strerror(int s) {
  switch (s) {
    case SHOCK_OK: return "ok";
    case SHOCK_EINVAL: return "invalid argument or malformed batch";
    case SHOCK_ENOTFOUND: return "no qualifying seed below max_seed for some leaf";
    case SHOCK_EDUPKEY: return "repeated key within a leaf";
    case SHOCK_ECANCELED: return "cancelled";
    case SHOCK_EHIP: return "HIP runtime error";
    case SHOCK_ENOMEM: return "out of device memory";
    case SHOCK_EPENDING: return "not complete yet";
    default: return "unknown status";
  }
}

int shock_spec_version(void) { return 3; }

int shock_last_stats(shock_stats *out) {
  if (!out) return SHOCK_EINVAL;
  *out = g_stats;
  return SHOCK_OK;
}

int shock_release_scratch(void) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceSynchronize());
  if ((int)t_scratch.size() > dev && t_scratch[dev].buf) {
    HIP_TRY(hipFree(t_scratch[dev].buf));
    t_scratch[dev].buf = nullptr;
    t_scratch[dev].bytes = 0;
  }
  HIP_TRY(shock_internal_release_code_scratch(dev));
  HIP_TRY(shock_internal_release_bip_scratch(dev));
  HIP_TRY(shock_internal_release_mphf_scratch(dev));
  HIP_TRY(shock_internal_release_stream_scratch(dev));
  return SHOCK_OK;
}

}  // extern "C"

static int search_sync(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                       uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts_in, void *hip_stream, int rf) {
  shock_opts opts;
  shock_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.max_seed == 0) opts.max_seed = SHOCK_DEFAULT_MAX_SEED;
  memset(&g_stats, 0, sizeof(g_stats));
  if (n_leaves == 0) return SHOCK_OK;
  int rc = check_opts(opts, n_leaves, offsets, out_seeds, out_orient);
  if (rc != SHOCK_OK) return rc;
  if (!keys) return SHOCK_EINVAL;
  if (rf && (!out_rot || opts.max_seed > (1ull << 57))) return SHOCK_EINVAL;
  hipStream_t stream = (hipStream_t)hip_stream;
  const int mode = opts.mode == SHOCK_MODE_AUTO ? SHOCK_MODE_PERSISTENT : opts.mode;
  if (mode != SHOCK_MODE_PERSISTENT && mode != SHOCK_MODE_PLAIN_PER_LEAF) return SHOCK_EINVAL;

  // Scratch is laid out for the largest worker count any launch may use.
  const int workers_cap = (opts.workers > 32 * 256 * 4 ? opts.workers : 32 * 256 * 4) + kMaxWavesPerWg;
  const uint64_t n_launches = mode == SHOCK_MODE_PLAIN_PER_LEAF ? n_leaves : 1;
  const Layout lay = layout(n_leaves, (uint32_t)workers_cap, n_launches);
  void *buf = nullptr;
  unsigned long long *host_ctr = nullptr;
  rc = get_scratch(lay.total, &buf, &host_ctr);
  if (rc != SHOCK_OK) return rc;
  const CallBufs cb = carve(buf, lay);

  Plan pl;
  rc = make_plan(opts, n_leaves, 48, rf, pl);
  if (rc != SHOCK_OK) return rc;
  HIP_TRY(enqueue_prologue(cb, pl, keys, offsets, n_leaves, opts, (uint32_t)workers_cap, stream));
  // Validation result and leaf sizes for launch sizing: all offsets for
  // per-leaf launches, the first and last otherwise (mean leaf size).
  std::vector<uint64_t> h_off(mode == SHOCK_MODE_PLAIN_PER_LEAF ? n_leaves + 1 : 2);
  HIP_TRY(hipMemcpyAsync(host_ctr, cb.gctr, kCtrGlobalCount * 8, hipMemcpyDeviceToHost, stream));
  if (mode == SHOCK_MODE_PLAIN_PER_LEAF) {
    HIP_TRY(hipMemcpyAsync(h_off.data(), offsets, (n_leaves + 1) * 8, hipMemcpyDeviceToHost, stream));
  } else {
    HIP_TRY(hipMemcpyAsync(&h_off[0], offsets, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&h_off[1], offsets + n_leaves, 8, hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  if (host_ctr[kCtrErr] & kErrInvalid) return SHOCK_EINVAL;
  if (host_ctr[kCtrErr] & kErrDup) return SHOCK_EDUPKEY;

  const uint32_t n_mean = (uint32_t)((h_off.back() - h_off.front() + n_leaves / 2) / n_leaves);
  rc = make_plan(opts, n_leaves, n_mean, rf, pl);
  if (rc != SHOCK_OK) return rc;
  if (pl.workers > workers_cap) return SHOCK_EINVAL;
  Params P = base_params(cb, pl, opts, offsets, out_seeds, out_orient, out_rot);

  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, stream));
  HIP_TRY(enqueue_search(P, cb, pl, n_leaves, mode == SHOCK_MODE_PLAIN_PER_LEAF ? h_off.data() : nullptr, n_mean,
                         opts.workers != 0, stream));
  HIP_TRY(hipEventRecord(e1, stream));
  hipLaunchKernelGGL(mark_unfinished_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, stream, cb.gctr,
                     cb.state, n_leaves, out_seeds, out_orient, out_rot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host_ctr, cb.gctr, kCtrGlobalCount * 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  HIP_TRY(hipEventDestroy(e0));
  HIP_TRY(hipEventDestroy(e1));
  rc = status_from(host_ctr, &g_stats);
  g_stats.kernel_ms = ms;
  g_stats.workers = (int32_t)P.workers;
  g_stats.spl = pl.spl;
  g_stats.block_iters = pl.units;
  g_stats.waves_per_wg = pl.wpw;
  return rc;
}

// ---- the search without allocations ---------------------------------------
//
// One fixed scratch array per GPU, part of the code object (so the runtime
// places it when the library's device code is loaded).  In host code `scratch`
// names only a host-side stand-in: its device address is looked up once per
// device with hipGetSymbolAddress and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SHOCK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocMaxDevices = 64;
constexpr uint32_t kNoAllocWorkersCap = SHOCK_NOALLOC_MAX_WORKERS + kMaxWavesPerWg;
static_assert(layout(SHOCK_NOALLOC_MAX_LEAVES, kNoAllocWorkersCap, 1).total <= SHOCK_NOALLOC_SCRATCH_BYTES,
              "the no-allocation scratch array must hold the largest batch it accepts");

std::mutex g_noalloc_init_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices];
std::mutex g_noalloc_call_mu[kNoAllocMaxDevices];

// Device address of this device's scratch array (looked up on first use).
int noalloc_scratch(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_noalloc_init_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_err("hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorInvalidSymbol);
      return SHOCK_EHIP;
    }
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return SHOCK_OK;
}

}  // namespace

extern "C" {

int shock_leaf_search_noalloc(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                              uint64_t *out_orient, const shock_opts *opts_in, void *hip_stream) {
  shock_opts opts;
  shock_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.max_seed == 0) opts.max_seed = SHOCK_DEFAULT_MAX_SEED;
  memset(&g_stats, 0, sizeof(g_stats));
  if (n_leaves == 0) return SHOCK_OK;
  int rc = check_opts(opts, n_leaves, offsets, out_seeds, out_orient);
  if (rc != SHOCK_OK) return rc;
  if (!keys) return SHOCK_EINVAL;
  if (opts.mode != SHOCK_MODE_AUTO && opts.mode != SHOCK_MODE_PERSISTENT) return SHOCK_EINVAL;
  if (n_leaves > SHOCK_NOALLOC_MAX_LEAVES || opts.workers > SHOCK_NOALLOC_MAX_WORKERS) {
    snprintf(g_err, sizeof(g_err), "shock_leaf_search_noalloc: at most %d leaves and %d workers",
             SHOCK_NOALLOC_MAX_LEAVES, SHOCK_NOALLOC_MAX_WORKERS);
    return SHOCK_EINVAL;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return SHOCK_EINVAL;
  void *buf = nullptr;
  rc = noalloc_scratch(dev, &buf);
  if (rc != SHOCK_OK) return rc;
  std::lock_guard<std::mutex> lk(g_noalloc_call_mu[dev]);
  hipStream_t stream = (hipStream_t)hip_stream;
  const Layout lay = layout(n_leaves, kNoAllocWorkersCap, 1);
  const CallBufs cb = carve(buf, lay);

  Plan pl;
  rc = make_plan(opts, n_leaves, 48, 0, pl);
  if (rc != SHOCK_OK) return rc;
  HIP_TRY(enqueue_prologue(cb, pl, keys, offsets, n_leaves, opts, kNoAllocWorkersCap, stream));
  unsigned long long host_ctr[kCtrGlobalCount];
  uint64_t h_off[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(host_ctr, cb.gctr, sizeof(host_ctr), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&h_off[0], offsets, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&h_off[1], offsets + n_leaves, 8, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (host_ctr[kCtrErr] & kErrInvalid) return SHOCK_EINVAL;
  if (host_ctr[kCtrErr] & kErrDup) return SHOCK_EDUPKEY;

  const uint32_t n_mean = (uint32_t)((h_off[1] - h_off[0] + n_leaves / 2) / n_leaves);
  rc = make_plan(opts, n_leaves, n_mean, 0, pl);
  if (rc != SHOCK_OK) return rc;
  if (pl.workers > (int)kNoAllocWorkersCap) return SHOCK_EINVAL;
  Params P = base_params(cb, pl, opts, offsets, out_seeds, out_orient, nullptr);
  HIP_TRY(enqueue_search(P, cb, pl, n_leaves, nullptr, n_mean, opts.workers != 0, stream));
  hipLaunchKernelGGL(mark_unfinished_kernel, dim3((unsigned)((n_leaves + 255) / 256)), dim3(256), 0, stream, cb.gctr,
                     cb.state, n_leaves, out_seeds, out_orient, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(host_ctr, cb.gctr, sizeof(host_ctr), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  rc = status_from(host_ctr, &g_stats);
  g_stats.workers = (int32_t)P.workers;
  g_stats.spl = pl.spl;
  g_stats.block_iters = pl.units;
  g_stats.waves_per_wg = pl.wpw;
  return rc;
}

int shock_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                         uint64_t *out_orient, const shock_opts *opts, void *hip_stream) {
  return search_sync(keys, offsets, n_leaves, out_seeds, nullptr, out_orient, opts, hip_stream, 0);
}

int shock_rf_leaf_search_ex(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                            uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts, void *hip_stream) {
  return search_sync(keys, offsets, n_leaves, out_seeds, out_rot, out_orient, opts, hip_stream, 1);
}

int shock_leaf_search(const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves, uint64_t *out_seeds,
                      uint64_t *out_orient) {
  return shock_leaf_search_ex(keys, offsets, n_leaves, out_seeds, out_orient, nullptr, nullptr);
}

int shock_ctx_create(uint64_t max_leaves, shock_ctx **out) {
  if (!out || max_leaves == 0 || max_leaves > (1ull << 31)) return SHOCK_EINVAL;
  *out = nullptr;
  shock_ctx *c = new shock_ctx();
  HIP_TRY(hipGetDevice(&c->device));
  c->max_leaves = max_leaves;
  c->workers_cap = kCallWorkersCap;
  const Layout lay = layout(max_leaves, c->workers_cap, max_leaves);
  c->bytes = lay.total;
  hipError_t e = hipMalloc(&c->buf, c->bytes);
  if (e != hipSuccess) {
    set_err("hipMalloc(context scratch)", e);
    delete c;
    return SHOCK_ENOMEM;
  }
  e = hipHostMalloc((void **)&c->host_ctr, kCtrGlobalCount * 8, hipHostMallocDefault);
  if (e != hipSuccess) {
    set_err("hipHostMalloc(context counters)", e);
    (void)hipFree(c->buf);
    delete c;
    return SHOCK_ENOMEM;
  }
  memset(c->host_ctr, 0, kCtrGlobalCount * 8);
  if (hipEventCreate(&c->ev_begin) != hipSuccess || hipEventCreate(&c->ev_search) != hipSuccess ||
      hipEventCreate(&c->ev_done) != hipSuccess) {
    set_err("hipEventCreate", hipErrorUnknown);
    return SHOCK_EHIP;
  }
  *out = c;
  return SHOCK_OK;
}

int shock_ctx_destroy(shock_ctx *c) {
  if (!c) return SHOCK_EINVAL;
  (void)hipSetDevice(c->device);
  if (c->pending) (void)hipEventSynchronize(c->ev_done);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  (void)hipEventDestroy(c->ev_begin);
  (void)hipEventDestroy(c->ev_search);
  (void)hipEventDestroy(c->ev_done);
  (void)hipHostFree(c->host_ctr);
  (void)hipFree(c->buf);
  delete c;
  return SHOCK_OK;
}

// Enqueue the whole call on `stream` without any host synchronisation.
static int ctx_enqueue(shock_ctx *c, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                       uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient, const shock_opts &opts,
                       hipStream_t stream, bool with_events) {
  Plan pl;
  const int rc = enqueue_call(c->buf, n_leaves, keys, offsets, out_seeds, out_rot, out_orient, opts,
                              opts.leaf_size_hint ? (uint32_t)opts.leaf_size_hint : 48, stream, c->host_ctr,
                              with_events ? c->ev_begin : nullptr, with_events ? c->ev_search : nullptr, pl);
  if (rc == SHOCK_OK) c->last_plan = pl;
  return rc;
}

static int ctx_async(shock_ctx *c, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                     uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts_in,
                     void *hip_stream) {
  if (!c) return SHOCK_EINVAL;
  shock_opts opts;
  shock_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.max_seed == 0) opts.max_seed = SHOCK_DEFAULT_MAX_SEED;
  if (n_leaves == 0 || n_leaves > c->max_leaves || !keys) return SHOCK_EINVAL;
  int rc = check_opts(opts, n_leaves, offsets, out_seeds, out_orient);
  if (rc != SHOCK_OK) return rc;
  if (c->pending) HIP_TRY(hipEventSynchronize(c->ev_done));  // the counters buffer is reused
  hipStream_t stream = (hipStream_t)hip_stream;
  if (out_rot && opts.max_seed > (1ull << 57)) return SHOCK_EINVAL;
  rc = ctx_enqueue(c, keys, offsets, n_leaves, out_seeds, out_rot, out_orient, opts, stream, true);
  if (rc != SHOCK_OK) return rc;
  HIP_TRY(hipEventRecord(c->ev_done, stream));
  c->pending = true;
  return SHOCK_OK;
}

int shock_ctx_search_async(shock_ctx *c, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                           uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts, void *hip_stream) {
  return ctx_async(c, keys, offsets, n_leaves, out_seeds, nullptr, out_orient, opts, hip_stream);
}

int shock_ctx_rf_search_async(shock_ctx *c, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                              uint64_t *out_seeds, uint32_t *out_rot, uint64_t *out_orient, const shock_opts *opts,
                              void *hip_stream) {
  if (!out_rot) return SHOCK_EINVAL;
  return ctx_async(c, keys, offsets, n_leaves, out_seeds, out_rot, out_orient, opts, hip_stream);
}

int shock_ctx_query(shock_ctx *c) {
  if (!c) return SHOCK_EINVAL;
  if (!c->pending) return 1;
  hipError_t e = hipEventQuery(c->ev_done);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  set_err("hipEventQuery", e);
  return SHOCK_EHIP;
}

int shock_ctx_wait(shock_ctx *c, shock_stats *stats) {
  if (!c) return SHOCK_EINVAL;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (!c->pending) return SHOCK_EINVAL;
  HIP_TRY(hipEventSynchronize(c->ev_done));
  c->pending = false;
  int rc = status_from(c->host_ctr, stats);
  if (stats) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev_begin, c->ev_search) == hipSuccess) stats->kernel_ms = ms;
    stats->workers = c->last_plan.workers;
    stats->spl = c->last_plan.spl;
    stats->block_iters = c->last_plan.units;
    stats->waves_per_wg = c->last_plan.wpw;
  }
  return rc;
}

int shock_ctx_graph_capture(shock_ctx *c, const uint64_t *keys, const uint64_t *offsets, uint64_t n_leaves,
                            uint64_t *out_seeds, uint64_t *out_orient, const shock_opts *opts_in, void *hip_stream) {
  if (!c) return SHOCK_EINVAL;
  shock_opts opts;
  shock_opts_init(&opts);
  if (opts_in) opts = *opts_in;
  if (opts.max_seed == 0) opts.max_seed = SHOCK_DEFAULT_MAX_SEED;
  if (n_leaves == 0 || n_leaves > c->max_leaves || !keys) return SHOCK_EINVAL;
  int rc = check_opts(opts, n_leaves, offsets, out_seeds, out_orient);
  if (rc != SHOCK_OK) return rc;
  if (opts.cancel) return SHOCK_EINVAL;  // a captured graph cannot watch a host flag reliably across replays
  if (c->pending) HIP_TRY(hipEventSynchronize(c->ev_done));
  c->pending = false;
  if (c->graph_exec) {
    HIP_TRY(hipGraphExecDestroy(c->graph_exec));
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    HIP_TRY(hipGraphDestroy(c->graph));
    c->graph = nullptr;
  }
  {
    Plan warm;  // resolves and caches occupancy queries before capture starts
    rc = make_plan(opts, n_leaves, opts.leaf_size_hint ? (uint32_t)opts.leaf_size_hint : 48, 0, warm);
    if (rc != SHOCK_OK) return rc;
  }
  hipStream_t cap;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  rc = ctx_enqueue(c, keys, offsets, n_leaves, out_seeds, nullptr, out_orient, opts, cap, false);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cap, &g);
  (void)hipStreamDestroy(cap);
  if (rc != SHOCK_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_err("hipStreamEndCapture", e);
    return SHOCK_EHIP;
  }
  c->graph = g;
  HIP_TRY(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
  (void)hip_stream;
  return SHOCK_OK;
}

int shock_ctx_graph_launch(shock_ctx *c, void *hip_stream) {
  if (!c || !c->graph_exec) return SHOCK_EINVAL;
  if (c->pending) HIP_TRY(hipEventSynchronize(c->ev_done));
  hipStream_t stream = (hipStream_t)hip_stream;
  HIP_TRY(hipEventRecord(c->ev_begin, stream));
  HIP_TRY(hipGraphLaunch(c->graph_exec, stream));
  HIP_TRY(hipEventRecord(c->ev_search, stream));
  HIP_TRY(hipEventRecord(c->ev_done, stream));
  c->pending = true;
  return SHOCK_OK;
}

}  // extern "C"
