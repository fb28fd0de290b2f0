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
// (h0, h1), lane c stands for cell c.  Cells of degree one lose their edge,
// all at once, until none is left; the graph is a pseudoforest iff what
// remains (its 2-core) has no cell of degree above two, i.e. is a set of
// disjoint cycles: a component with two or more cycles keeps a cell of degree
// three or more in its 2-core.  Apart from building the incidence masks in
// LDS, every round is a few register operations and two ballots, where the
// union-find needs LDS round trips per step; rotation fitting tests many
// more candidates per leaf, so it uses this form.  Needs n >= 2 (no loops).
// inc: 64 words of the wave's LDS.
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
  const uint64_t mine = inc[lane];
  uint64_t rem = n >= 64 ? ~0ull : ((1ull << n) - 1);
  // Two rounds per iteration with one exit test: a round that finds no cell
  // of degree one changes nothing, so the pair ends the loop when its second
  // round finds none.  Every round that finds one removes an edge, so at most
  // n + 1 rounds (33 iterations) run.
  for (uint32_t it = 0; it < 33; ++it) {
    const uint64_t d1 = __ballot(__popcll(mine & rem) == 1);
    rem &= ~__ballot(act && (((d1 >> h0) | (d1 >> h1)) & 1));
    const uint64_t d2 = __ballot(__popcll(mine & rem) == 1);
    rem &= ~__ballot(act && (((d2 >> h0) | (d2 >> h1)) & 1));
    if (d2 == 0) break;
  }
  return __ballot(__popcll(mine & rem) > 2) == 0;
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
