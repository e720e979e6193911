// Empirical bandwidth ceiling of the collide-and-stream kernels' memory
// pattern without their arithmetic: q structure-of-arrays population fields of
// N nodes are read at node n and written at node n (one element per lane,
// non-temporal, as the kernels' aligned accesses), for the element sizes of
// the storages.  One line per (lattice shape, element size):
//   <name> q=<q> N=<N> bytes=<b>: <GB/s> (<us per pass>)
// where GB/s counts 2 q b N bytes per pass.  Buffers: q N 8 bytes each.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

template <int Q, class E>
__global__ __launch_bounds__(256) void stream_q(const E* __restrict__ a, E* __restrict__ b, uint64_t N) {
  const uint64_t n = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  E v[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) v[j] = __builtin_nontemporal_load(&a[(uint64_t)j * N + n]);
#pragma unroll
  for (int j = 0; j < Q; ++j) __builtin_nontemporal_store(v[j], &b[(uint64_t)j * N + n]);
}

static hipEvent_t e0, e1;

template <int Q, class E>
static int run(const char* name, uint64_t N) {
  const size_t bytes = (size_t)Q * N * sizeof(E);
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    printf("%s: allocation failed\n", name);
    return 1;
  }
  if (hipMemset(a, 0, bytes) != hipSuccess || hipMemset(b, 0, bytes) != hipSuccess) return 1;
  auto launch = [&] {
    hipLaunchKernelGGL((stream_q<Q, E>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, 0, (const E*)a, (E*)b, N);
  };
  for (int w = 0; w < 3; w++) launch();
  const int reps = 20;
  if (hipEventRecord(e0) != hipSuccess) return 1;
  for (int r = 0; r < reps; r++) launch();
  if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1;
  float ms = 0;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
  printf("%s q=%d N=%llu bytes=%zu: %.1f GB/s (%.1f us)\n", name, Q, (unsigned long long)N, sizeof(E),
         2.0 * bytes * reps / (ms * 1e-3) / 1e9, ms * 1e3 / reps);
  fflush(stdout);
  return (hipFree(a) != hipSuccess || hipFree(b) != hipSuccess) ? 1 : 0;
}

int main() {
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const uint64_t n256 = 256ull * 256 * 256, n192 = 192ull * 192 * 192, n4096 = 4096ull * 4096,
                 n2048 = 2048ull * 2048;
  int rc = 0;
  rc |= run<19, float>("d3q19_256^3", n256);
  rc |= run<19, uint16_t>("d3q19_256^3", n256);
  rc |= run<19, double>("d3q19_256^3", n256);
  rc |= run<27, float>("d3q27_192^3", n192);
  rc |= run<27, uint16_t>("d3q27_192^3", n192);
  rc |= run<9, float>("d2q9_4096^2", n4096);
  rc |= run<9, float>("d2q9_2048^2", n2048);
  printf(rc ? "failed\n" : "done\n");
  return rc;
}
