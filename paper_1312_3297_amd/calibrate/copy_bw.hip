// Plain device-to-device copy kernels of known size, used to calibrate the
// rocprofv3 FETCH_SIZE / WRITE_SIZE counters against bytes actually moved and
// to measure the achievable HBM copy bandwidth on this GPU.
//   copy4:   16-byte loads/stores, grid-stride loop (optionally non-temporal)
//   copy1x:  16 independent 4-byte loads then 16 stores per thread, strided
//            by the block size like the populations of a lattice node
// Buffer size 1270 MiB each (the size of one D3Q19 256^3 FP32 population array).
#include <hip/hip_runtime.h>
#include <cstdio>
typedef float f4 __attribute__((ext_vector_type(4)));
template <int NT>
__global__ void copy4(const f4* __restrict__ a, f4* __restrict__ b, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    if (NT) { f4 v = __builtin_nontemporal_load(&a[i]); __builtin_nontemporal_store(v, &b[i]); }
    else b[i] = a[i];
  }
}
template <int NT>
__global__ void copy1x(const float* __restrict__ a, float* __restrict__ b, size_t n) {
  // 16 floats per thread, strided by blockDim (like 16 populations)
  size_t base = blockIdx.x * (size_t)blockDim.x * 16 + threadIdx.x;
  float v[16];
  #pragma unroll
  for (int k = 0; k < 16; ++k) { size_t i = base + (size_t)k * blockDim.x; v[k] = i < n ? (NT ? __builtin_nontemporal_load(&a[i]) : a[i]) : 0.f; }
  #pragma unroll
  for (int k = 0; k < 16; ++k) { size_t i = base + (size_t)k * blockDim.x; if (i < n) { if (NT) __builtin_nontemporal_store(v[k], &b[i]); else b[i] = v[k]; } }
}
int main() {
  size_t bytes = (size_t)1270 << 20;  // like one D3Q19 256^3 FP32 array
  size_t n4 = bytes / 16, n1 = bytes / 4;
  float *a, *b;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) { printf("alloc fail\n"); return 1; }
  hipMemset(a, 0, bytes); hipMemset(b, 0, bytes);
  hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
  auto run = [&](const char* name, auto launch) {
    for (int w = 0; w < 3; w++) launch();
    hipEventRecord(e0);
    for (int r = 0; r < 10; r++) launch();
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    printf("%s: %.1f GB/s\n", name, 2.0 * bytes * 10 / (ms * 1e-3) / 1e9); fflush(stdout);
  };
  for (int grid : {1024, 2048, 4096, 65536}) {
    char nm[64];
    snprintf(nm, 64, "copy4 grid %d", grid); run(nm, [&] { hipLaunchKernelGGL(copy4<0>, dim3(grid), dim3(256), 0, 0, (const f4*)a, (f4*)b, n4); });
    snprintf(nm, 64, "copy4 NT grid %d", grid); run(nm, [&] { hipLaunchKernelGGL(copy4<1>, dim3(grid), dim3(256), 0, 0, (const f4*)a, (f4*)b, n4); });
  }
  unsigned g16 = (unsigned)((n1 + 256 * 16 - 1) / (256 * 16));
  run("copy1x16", [&] { hipLaunchKernelGGL(copy1x<0>, dim3(g16), dim3(256), 0, 0, a, b, n1); });
  run("copy1x16 NT", [&] { hipLaunchKernelGGL(copy1x<1>, dim3(g16), dim3(256), 0, 0, a, b, n1); });
  printf("done\n");
  return 0;
}
