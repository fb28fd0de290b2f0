// Wave-level building blocks shared by the search kernels: lane helpers, and
// the two wave-parallel graph routines on a leaf's n <= 64 keys (lane i holds
// key i's edge {h0, h1}, lane c stands for cell c).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shockwave {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t bcast64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t bcast32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Pseudoforest test by peeling, wave-parallel: lane i < n holds edge i
// (h0, h1), lane c stands for cell c.  Each round removes, all at once, every
// edge at a cell of degree one.
//
// The test counts instead of inspecting the 2-core.  With n edges on n cells,
// the sum over components of (edges - cells) is zero, and the graph is a
// pseudoforest iff every component has as many edges as cells.  Count only
// the cells that still have an edge.  In a component with a cycle, each
// removed edge takes exactly its leaf cell with it, so edges - cells stays the
// same; a tree stands at -1 until its last edge goes, then at 0.  So over the
// whole graph, (edges left) - (cells left) stays zero for a pseudoforest and
// turns positive in the round where the first tree (or, from the start, an
// empty cell) is gone.  The test rejects there, which for the candidates the
// searches send (every cell covered, nearly all with a small tree) is after
// one or two rounds, and accepts when no cell of degree one is left.  Apart
// from building the incidence masks in LDS, a round is a few register
// operations, two ballots and two scalar popcounts; the union-find needs LDS
// round trips per step.  Lanes at or above n and cells they name (a one-key
// leaf's second cell) take no part.  inc: 64 words of the wave's LDS.
__device__ inline bool pf_peel_wave(uint32_t n, uint32_t h0, uint32_t h1, unsigned long long *inc) {
  const uint32_t lane = lane_id();
  const bool act = lane < n;
  inc[lane] = 0;
  wave_lds_sync();
  if (act) {
    atomicOr(&inc[h0], 1ull << lane);
    atomicOr(&inc[h1], 1ull << lane);
  }
  wave_lds_sync();
  const uint64_t mine = act ? inc[lane] : 0;
  uint64_t rem = n >= 64 ? ~0ull : ((1ull << n) - 1);
  // A round that does not return removes at least one edge, so at most n + 1
  // rounds run.
  for (uint32_t round = 0; round <= 64; ++round) {
    const uint32_t deg = __popcll(mine & rem);
    if (__popcll(rem) != __popcll(__ballot(deg != 0))) return false;
    const uint64_t d1 = __ballot(deg == 1);
    if (d1 == 0) return true;
    rem &= ~__ballot(act && (((d1 >> h0) | (d1 >> h1)) & 1));
  }
  return false;
}

// Canonical orientation of an accepted seed, wave-parallel.  A free cell with
// exactly one unplaced incident key takes that key (forced); when no such
// cell remains, only disjoint cycles are left and the highest-index unplaced
// key takes its h0 slot.  Returns false if the choice is not a bijection
// (which cannot happen for a pseudoforest).
__device__ inline bool orient_wave(uint32_t n, uint32_t h0, uint32_t h1, unsigned long long *inc0,
                                   unsigned long long *inc1, unsigned long long *hit, uint64_t &f_out) {
  const uint32_t lane = lane_id();
  const bool act = lane < n;
  inc0[lane] = 0;
  inc1[lane] = 0;
  if (lane == 0) *hit = 0;
  wave_lds_sync();
  if (act) {
    atomicOr(&inc0[h0], 1ull << lane);
    atomicOr(&inc1[h1], 1ull << lane);
  }
  wave_lds_sync();
  const uint64_t inc = inc0[lane] | inc1[lane];
  const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
  uint64_t rem = all, avail = all, f = 0;
  for (int round = 0; round < 2 * 64 + 2 && rem != 0; ++round) {
    const bool cell_free = act && ((avail >> lane) & 1);
    const bool one = cell_free && __popcll(inc & rem) == 1;
    const uint64_t d1 = __ballot(one);
    if (d1 == 0) {
      const uint32_t m = 63 - __clzll(rem);
      const uint32_t c0 = __builtin_amdgcn_readlane(h0, m);
      rem &= ~(1ull << m);
      avail &= ~(1ull << c0);
      continue;
    }
    const bool mine = act && ((rem >> lane) & 1);
    const bool take0 = mine && ((d1 >> h0) & 1);
    const bool take1 = mine && !take0 && ((d1 >> h1) & 1);
    const uint64_t got = __ballot(take0 || take1);
    const uint64_t fb = __ballot(take1);
    rem &= ~got;
    avail &= ~d1;
    f |= fb;
  }
  if (act) {
    const uint32_t slot = ((f >> lane) & 1) ? h1 : h0;
    atomicOr(hit, 1ull << slot);
  }
  wave_lds_sync();
  f_out = f;
  return rem == 0 && *hit == all;
}

}  // namespace shockwave
