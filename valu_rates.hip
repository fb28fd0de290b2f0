// VALU issue-rate probe for gfx950: independent register-only chains of one
// instruction per kernel, no memory access in the asm, timed with HIP events.
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops valu_rates.hip -o valu_rates
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "paper_2308_09561_amd/csrc/shock_hash.h"
#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)
#define ITERS 2048
#define NCH 8

#define K32(NAME, ASM)                                                              \
__global__ __launch_bounds__(256) void NAME(uint32_t* out, uint32_t s1, uint32_t s2) { \
  uint32_t a[NCH]; uint32_t b = threadIdx.x * 0x9E3779B9u + s1, c = s2 ^ threadIdx.x;   \
  _Pragma("unroll") for (int i = 0; i < NCH; ++i) a[i] = threadIdx.x + i * 77u + s1;   \
  for (int it = 0; it < ITERS; ++it) {                                                  \
    _Pragma("unroll") for (int i = 0; i < NCH; ++i) asm volatile(ASM : "+v"(a[i]) : "v"(b), "v"(c)); \
  }                                                                                     \
  uint32_t r = 0; _Pragma("unroll") for (int i = 0; i < NCH; ++i) r ^= a[i];            \
  out[blockIdx.x * 256 + threadIdx.x] = r;                                              \
}

K32(k_xor, "v_xor_b32 %0, %0, %1")
K32(k_add, "v_add_u32 %0, %0, %1")
K32(k_mul_lo, "v_mul_lo_u32 %0, %0, %1")
K32(k_mul_hi, "v_mul_hi_u32 %0, %0, %1")
K32(k_mul_u24, "v_mul_u32_u24 %0, %0, %1")
K32(k_mul_hi_u24, "v_mul_hi_u32_u24 %0, %0, %1")
K32(k_perm, "v_perm_b32 %0, %0, %1, %2")
K32(k_alignbit, "v_alignbit_b32 %0, %0, %1, 7")
K32(k_add3, "v_add3_u32 %0, %0, %1, %2")
K32(k_or3, "v_or3_b32 %0, %0, %1, %2")
K32(k_lshl_or, "v_lshl_or_b32 %0, %1, %0, %2")
K32(k_bfe, "v_bfe_u32 %0, %0, %1, 8")
K32(k_xad, "v_xad_u32 %0, %0, %1, %2")
K32(k_lshr, "v_lshrrev_b32 %0, 8, %0")
K32(k_bcnt, "v_bcnt_u32_b32 %0, %0, %1")
K32(k_cmp_cnd, "v_cmp_ge_u32 vcc, %0, %1\n v_addc_co_u32 %0, vcc, %0, 0, vcc")

#define K64(NAME, ASM)                                                              \
__global__ __launch_bounds__(256) void NAME(uint32_t* out, uint32_t s1, uint32_t s2) { \
  uint64_t a[NCH]; uint32_t b = threadIdx.x * 0x9E3779B9u + s1, c = s2 ^ threadIdx.x;   \
  _Pragma("unroll") for (int i = 0; i < NCH; ++i) a[i] = ((uint64_t)(threadIdx.x + i) << 32) | (s1 + i); \
  for (int it = 0; it < ITERS; ++it) {                                                  \
    _Pragma("unroll") for (int i = 0; i < NCH; ++i) asm volatile(ASM : "+v"(a[i]) : "v"(b), "v"(c) : "vcc"); \
  }                                                                                     \
  uint64_t r = 0; _Pragma("unroll") for (int i = 0; i < NCH; ++i) r ^= a[i];            \
  out[blockIdx.x * 256 + threadIdx.x] = (uint32_t)(r ^ (r >> 32));                      \
}
K64(k_mad_u64, "v_mad_u64_u32 %0, vcc, %1, %2, %0")
K64(k_lshl_b64, "v_lshlrev_b64 %0, %1, %0")
K64(k_lshl_add_u64, "v_lshl_add_u64 %0, %0, 1, %0")

K32(k_lshl_one, "v_lshlrev_b32_e64 %0, %0, 1")

// The search kernel's hash-and-filter loop, register only: 12 keys x 2 seeds
// per iteration with the library's own slot_pair and mask updates (the same
// instructions as the compiled loop: 11 per key evaluation with a 64-bit
// mask, 10 with a 32-bit one), keys loop-invariant, the seed words moved by
// one add per seed and iteration.  Counts key evaluations.
#define HASH_KEYS 12
template <bool WIDE>
__global__ __launch_bounds__(256) void k_hash_loop(uint32_t* out, uint32_t s1, uint32_t s2) {
  uint32_t alo[HASH_KEYS], ahi[HASH_KEYS];
  _Pragma("unroll") for (int i = 0; i < HASH_KEYS; ++i) {
    const uint64_t a = shockhash::fmix64(((uint64_t)s1 << 32) + i * 977u + s2);
    alo[i] = (uint32_t)a;
    ahi[i] = (uint32_t)(a >> 32);
  }
  const uint32_t n = (WIDE ? 48 : 32) - (s1 >> 8), nm1 = n - 1;  // s1 = 1: 48 or 32, unknown to the compiler
  uint32_t tlo[2], thi[2], mlo[2] = {0, 0}, mhi[2] = {0, 0};
  _Pragma("unroll") for (int j = 0; j < 2; ++j) {
    const uint64_t t = shockhash::fmix64(threadIdx.x * 2 + j + s1);
    tlo[j] = (uint32_t)t;
    thi[j] = (uint32_t)(t >> 32);
  }
  for (int it = 0; it < ITERS; ++it) {
    _Pragma("unroll") for (int i = 0; i < HASH_KEYS; ++i) {
      _Pragma("unroll") for (int j = 0; j < 2; ++j) {
        uint32_t h0, h1;
        shockhash::slot_pair(alo[i], ahi[i], tlo[j], thi[j], n, nm1, h0, h1);
        if (WIDE) {
          const uint64_t b0 = 1ull << h0, b1 = 1ull << h1;
          asm("v_or3_b32 %0, %0, %1, %2" : "+v"(mlo[j]) : "v"((uint32_t)b0), "v"((uint32_t)b1));
          asm("v_or3_b32 %0, %0, %1, %2" : "+v"(mhi[j]) : "v"((uint32_t)(b0 >> 32)), "v"((uint32_t)(b1 >> 32)));
        } else {
          asm("v_or3_b32 %0, %0, %1, %2" : "+v"(mlo[j]) : "v"(1u << h0), "v"(1u << h1));
        }
      }
    }
    _Pragma("unroll") for (int j = 0; j < 2; ++j) tlo[j] += 0x9E3779B9u;
  }
  out[blockIdx.x * 256 + threadIdx.x] = mlo[0] ^ mlo[1] ^ mhi[0] ^ mhi[1];
}

// The per-seed mix t(s) = fmix64((s + 1) * gamma) of consecutive seeds,
// 4 chains per thread.  Counts seeds.
__global__ __launch_bounds__(256) void k_seed_mix(uint32_t* out, uint32_t s1, uint32_t s2) {
  uint64_t acc[4] = {0, 0, 0, 0};
  uint64_t s = ((uint64_t)s2 << 32) + threadIdx.x * 4 + s1;
  for (int it = 0; it < ITERS; ++it) {
    _Pragma("unroll") for (int c = 0; c < 4; ++c) acc[c] ^= shockhash::seed_mix(s + c);
    s += 256 * 4;
  }
  out[blockIdx.x * 256 + threadIdx.x] = (uint32_t)(acc[0] ^ acc[1] ^ acc[2] ^ acc[3]);
}

__global__ void k_empty(uint32_t* out) { if (threadIdx.x == 1000000) out[0] = 1; }

__global__ void k_clock(uint64_t* out) {
  uint64_t t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  uint32_t a = threadIdx.x;
  for (int it = 0; it < 2000000; ++it) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a) : "v"(it));
  uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0 && blockIdx.x == 0) { out[0] = t1 - t0; out[1] = r1 - r0; }
  if (a == 0xFFFFFFFFu) out[2] = a;
}

typedef void (*kfn)(uint32_t*, uint32_t, uint32_t);
struct T { const char* name; kfn f; int insts_per; };

int main() {
  hipDeviceProp_t p; CHECK(hipGetDeviceProperties(&p, 0));
  printf("device %s CUs %d clock %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
  const int blocks = p.multiProcessorCount * 16;  // 16 WGs x 4 waves per CU
  uint32_t* out; CHECK(hipMalloc(&out, (size_t)blocks * 256 * 4));
  T tests[] = {
    {"v_xor_b32", k_xor, 1}, {"v_add_u32", k_add, 1}, {"v_mul_lo_u32", k_mul_lo, 1},
    {"v_mul_hi_u32", k_mul_hi, 1}, {"v_mul_u32_u24", k_mul_u24, 1}, {"v_mul_hi_u32_u24", k_mul_hi_u24, 1},
    {"v_perm_b32", k_perm, 1}, {"v_alignbit_b32", k_alignbit, 1}, {"v_add3_u32", k_add3, 1},
    {"v_or3_b32", k_or3, 1}, {"v_lshl_or_b32", k_lshl_or, 1}, {"v_bfe_u32", k_bfe, 1},
    {"v_xad_u32", k_xad, 1}, {"v_lshrrev_b32", k_lshr, 1}, {"v_bcnt_u32_b32", k_bcnt, 1},
    {"v_cmp+v_addc (2 insts)", k_cmp_cnd, 2},
    {"v_mad_u64_u32", (kfn)k_mad_u64, 1}, {"v_lshlrev_b64", (kfn)k_lshl_b64, 1},
    {"v_lshl_add_u64", (kfn)k_lshl_add_u64, 1},
    {"v_lshlrev_b32_e64 (1 << v)", k_lshl_one, 1},
  };
  hipEvent_t e0, e1; CHECK(hipEventCreate(&e0)); CHECK(hipEventCreate(&e1));
  const double peak_lane_ops = (double)p.multiProcessorCount * 64.0 * 2.4e9;
  for (auto& t : tests) {
    hipLaunchKernelGGL(t.f, dim3(blocks), dim3(256), 0, 0, out, 1u, 2u);  // warm
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(t.f, dim3(blocks), dim3(256), 0, 0, out, 1u, 2u);
    CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
    float ms; CHECK(hipEventElapsedTime(&ms, e0, e1));
    double lane_insts = 5.0 * blocks * 256.0 * ITERS * NCH * t.insts_per;
    double rate = lane_insts / (ms * 1e-3);
    printf("%-26s %.3e lane-inst/s  = %.3f of 256CU*64*2.4GHz\n", t.name, rate, rate / peak_lane_ops);
    fflush(stdout);
  }
  // The search loop and the seed mix: throughput in the units the benchmark
  // counts (key evaluations, seeds), and as lane-ops/s at 11 (64-bit mask) or
  // 10 (32-bit mask) ops per evaluation.
  struct L { const char* name; kfn f; double units_per_thread_iter; double ops_per_unit; };
  L loops[] = {
    {"hash loop, 64-bit mask (key-evals)", k_hash_loop<true>, HASH_KEYS * 2, 11},
    {"hash loop, 32-bit mask (key-evals)", k_hash_loop<false>, HASH_KEYS * 2, 10},
    {"seed mix (seeds)", k_seed_mix, 4, 1},
  };
  for (auto& t : loops) {
    hipLaunchKernelGGL(t.f, dim3(blocks), dim3(256), 0, 0, out, 1u, 2u);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(t.f, dim3(blocks), dim3(256), 0, 0, out, 1u, 2u);
    CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
    float ms; CHECK(hipEventElapsedTime(&ms, e0, e1));
    double units = 5.0 * blocks * 256.0 * ITERS * t.units_per_thread_iter;
    double rate = units / (ms * 1e-3);
    printf("%-36s %.4e units/s  = %.4e lane-ops/s = %.4f of 256CU*64*2.4GHz\n", t.name, rate, rate * t.ops_per_unit,
           rate * t.ops_per_unit / peak_lane_ops);
    fflush(stdout);
  }
  // launch overhead: back-to-back empty kernels
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 2000; ++r) hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, 0, out);
  CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
  { float ms; CHECK(hipEventElapsedTime(&ms, e0, e1)); printf("empty kernel back-to-back: %.2f us/launch\n", ms * 1e3 / 2000); }
  CHECK(hipEventRecord(e0));
  for (int r = 0; r < 2000; ++r) hipLaunchKernelGGL(k_empty, dim3(4096), dim3(256), 0, 0, out);
  CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
  { float ms; CHECK(hipEventElapsedTime(&ms, e0, e1)); printf("empty 4096x256 kernel back-to-back: %.2f us/launch\n", ms * 1e3 / 2000); }
  uint64_t* clk; CHECK(hipMalloc(&clk, 64));
  hipLaunchKernelGGL(k_clock, dim3(blocks), dim3(256), 0, 0, clk);
  CHECK(hipDeviceSynchronize());
  uint64_t h[2]; CHECK(hipMemcpy(h, clk, 16, hipMemcpyDeviceToHost));
  printf("s_memtime delta %llu, s_memrealtime delta %llu -> shader clock ~ %.0f MHz (if realtime is 100 MHz)\n",
         (unsigned long long)h[0], (unsigned long long)h[1], 100.0 * (double)h[0] / (double)h[1]);
  return 0;
}
