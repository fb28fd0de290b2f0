// Throughput of device-scope loads and atomics on one address versus spread
// addresses (all accesses in bounds by construction).
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops atomic_contention.hip -o atomic_contention
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e_), __LINE__); return 1; } } while (0)
// mode 0: relaxed agent atomic load same address; 1: spread (per wave); 2: atomicAdd same; 3: atomicAdd spread; 4: plain load same
__global__ void k(unsigned long long* buf, int mode, int iters, unsigned long long* sink) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63;
  unsigned long long acc = 0;
  unsigned long long* p = (mode & 1) ? buf + (uint64_t)(wave % 4096) * 16 : buf;
  for (int i = 0; i < iters; ++i) {
    unsigned long long v = 0;
    if (lane == 0) {
      if (mode < 2) v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else if (mode < 4) v = atomicAdd(p, 1ull);
      else v = *(volatile unsigned long long*)p;
    }
    acc += __builtin_amdgcn_readfirstlane((uint32_t)v);
  }
  if (acc == 0x123456789ull) sink[0] = acc;
}
int main() {
  unsigned long long *buf, *sink;
  CHECK(hipMalloc(&buf, 4096 * 16 * 8 + 64)); CHECK(hipMalloc(&sink, 64));
  CHECK(hipMemset(buf, 0, 4096 * 16 * 8 + 64));
  hipEvent_t e0, e1; CHECK(hipEventCreate(&e0)); CHECK(hipEventCreate(&e1));
  const char* names[] = {"atomic-load same addr", "atomic-load spread", "atomicAdd same addr", "atomicAdd spread", "volatile load same addr"};
  int wavesets[] = {256, 1024, 4096};
  for (int mode = 0; mode < 5; ++mode) for (int w : wavesets) {
    int iters = 64;
    hipLaunchKernelGGL(k, dim3(w / 4), dim3(256), 0, 0, buf, mode, iters, sink);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL(k, dim3(w / 4), dim3(256), 0, 0, buf, mode, iters, sink);
    CHECK(hipEventRecord(e1)); CHECK(hipEventSynchronize(e1));
    float ms; CHECK(hipEventElapsedTime(&ms, e0, e1));
    double ops = (double)w * iters;
    printf("%-26s waves %5d: %8.1f us, %.3e ops/s, %.1f ns/op\n", names[mode], w, ms * 1e3, ops / (ms * 1e-3), ms * 1e6 / ops);
    fflush(stdout);
  }
  return 0;
}
