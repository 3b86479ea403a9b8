// copy_probe.hip -- device-copy bandwidth by access width: the practical HBM
// ceilings the step kernels are compared with.  Copies 1 GiB with 2-, 4- and
// 16-byte accesses per lane, 1 to 16 loads in flight per lane, non-temporal
// stores, several grid sizes, and prints read + write bytes per second.
// Standalone; not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef float f4 __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over n elements, U loads in flight per lane, grid-stride;
// every index is checked against n
template <class E, int U>
__global__ __launch_bounds__(256) void k_copy(const E* __restrict__ src, E* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * 256 * U;
  for (long long base = (long long)blockIdx.x * 256 * U + threadIdx.x; base < n; base += stride) {
    E v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * 256;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * 256;
      if (i < n) __builtin_nontemporal_store(v[u], &dst[i]);
    }
  }
}

template <class E, int U>
static double gbs(const void* s, void* d, long long bytes, int grid) {
  const long long n = bytes / (long long)sizeof(E);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  k_copy<E, U><<<grid, 256>>>((const E*)s, (E*)d, n);
  (void)hipEventRecord(a);
  for (int r = 0; r < 10; r++) k_copy<E, U><<<grid, 256>>>((const E*)s, (E*)d, n);
  (void)hipEventRecord(b);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return 2.0 * (double)bytes / ((double)ms / 10.0 * 1e6);
}

int main() {
  const long long bytes = 1ll << 30;
  void *s = nullptr, *d = nullptr;
  if (hipMalloc(&s, bytes) != hipSuccess || hipMalloc(&d, bytes) != hipSuccess) {
    printf("device allocation failed\n");
    return 1;
  }
  (void)hipMemset(s, 0, bytes);
  (void)hipMemset(d, 0, bytes);
  printf("GB/s (read + write) by access width per lane x loads in flight per lane\n");
  for (int grid : {2048, 8192, 32768}) {
    printf("grid %5d  2B x1 %5.0f  2B x4 %5.0f  2B x16 %5.0f  4B x1 %5.0f  4B x16 %5.0f  16B x1 %5.0f  16B x4 %5.0f\n",
           grid, gbs<unsigned short, 1>(s, d, bytes, grid), gbs<unsigned short, 4>(s, d, bytes, grid),
           gbs<unsigned short, 16>(s, d, bytes, grid), gbs<unsigned, 1>(s, d, bytes, grid),
           gbs<unsigned, 16>(s, d, bytes, grid), gbs<f4, 1>(s, d, bytes, grid), gbs<f4, 4>(s, d, bytes, grid));
  }
  const hipError_t e = hipDeviceSynchronize();
  printf("status %s\n", hipGetErrorString(e));
  (void)hipFree(s);
  (void)hipFree(d);
  return e == hipSuccess ? 0 : 1;
}
