// The library's frozen hash family (spec version 3), shared by the search and
// query kernels.  The paper assumes fully random h0, h1 evaluated on a 64-bit
// master hash code (Sections 5 and 8); this is the concrete choice:
//   a = fmix64(x)                              MurmurHash3's 64-bit finaliser
//   t = fmix64((s + 1) * 0x9E3779B97F4A7C15)   per seed, mod 2^64
//   P = (lo32(a) ^ lo32(t)) * hi32(a) + t  (mod 2^64: one 32x32+64 multiply-add);
//   z = lo32(P) ^ hi32(P);  Q = z * n   (exact 64-bit product)
//   h0 = hi32(Q);  r = (lo32(Q) * (n - 1)) >> 32   (r reuses the fraction
//   that the multiply-shift range reduction of h0 leaves behind)
//   h1 = r + (r >= h0)   (h1 != h0 for n >= 2; no self-loops)
// Rotation fitting's 1-bit set hash: the top bit of fmix64(x ^ kSideKey).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shockhash {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kMix1 = 0xff51afd7ed558ccdull;
constexpr uint64_t kMix2 = 0xc4ceb9fe1a85ec53ull;
constexpr uint64_t kSideKey = 0xD1B54A32D192ED03ull;

__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= kMix1;
  k ^= k >> 33;
  k *= kMix2;
  k ^= k >> 33;
  return k;
}

// Per-seed mix t(s).
__device__ __forceinline__ uint64_t seed_mix(uint64_t s) { return fmix64((s + 1) * kGolden); }

// Slots of one key under one seed from the premixed key halves (alo, ahi) and
// the per-seed halves (tlo, thi); nm1 = n - 1, n >= 2.
__device__ __forceinline__ void slot_pair(uint32_t alo, uint32_t ahi, uint32_t tlo, uint32_t thi, uint32_t n,
                                          uint32_t nm1, uint32_t &h0, uint32_t &h1) {
  const uint64_t t = ((uint64_t)thi << 32) | tlo;
  const uint64_t p = (uint64_t)(alo ^ tlo) * (uint64_t)ahi + t;
  const uint32_t z = (uint32_t)p ^ (uint32_t)(p >> 32);
  const uint64_t q = (uint64_t)z * n;             // one v_mad_u64_u32
  uint32_t f0 = (uint32_t)(q >> 32);
  uint32_t r = __umulhi((uint32_t)q, nm1);
  // h1 = r + (r >= h0).  The empty asm statements hide the operands' origin
  // so that the compare stays 32-bit (one v_cmp + one v_addc) instead of
  // being widened to 64 bits for the later 64-bit shift.
  asm("" : "+v"(f0));
  asm("" : "+v"(r));
  uint32_t f1 = r + (uint32_t)(r >= f0);
  asm("" : "+v"(f1));
  h0 = f0;
  h1 = f1;
}

// Bipartite ShockHash: the left cell l in [0, nl) and the right cell r in
// [nl, nl + nr) of a premixed key a under a seed mix t.
__device__ __forceinline__ void bip_cells(uint64_t a, uint64_t t, uint32_t nl, uint32_t nr, uint32_t &l,
                                          uint32_t &r) {
  const uint64_t p = (uint64_t)((uint32_t)a ^ (uint32_t)t) * (a >> 32) + t;
  const uint32_t z = (uint32_t)p ^ (uint32_t)(p >> 32);
  const uint64_t q = (uint64_t)z * nl;
  l = (uint32_t)(q >> 32);
  r = nl + __umulhi((uint32_t)q, nr);
}

// 1 if key x belongs to rotation fitting's second set.
__device__ __forceinline__ uint32_t key_side(uint64_t x) { return (uint32_t)(fmix64(x ^ kSideKey) >> 63); }

}  // namespace shockhash
