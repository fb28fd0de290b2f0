// VALU issue-rate probe for gfx950: independent register-only chains of one
// instruction per kernel, no memory access in the asm, timed with HIP events.
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops valu_rates.hip -o valu_rates
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
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
