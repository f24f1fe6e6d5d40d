// Copy yardstick for the HBM roofline: device-to-device copies of a known
// size with the access patterns the PPF kernels use, timed with HIP events
// after a long warm-up (clock and power state settle over tens of
// milliseconds). Prints one JSON line per pattern:
//   grid-stride 16-byte non-temporal copy (the fastest plain copy),
//   tile copy: a workgroup per contiguous tile of 8 KiB blocks, 256 threads
//   moving 8 bytes each per block (the fused kernel's block traffic),
//   write only and read only (grid-stride, 16 bytes per lane), and
//   expand: 2 bytes read per 8 bytes written, the traffic of complex int8
//   input to complex FP32 spectra.
// The byte counters of a profiled run of this program scale FETCH_SIZE and
// WRITE_SIZE to bytes.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace {

#define CK(x)                                                                               \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) {                                                                 \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      exit(2);                                                                              \
    }                                                                                       \
  } while (0)

typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) copy_stride16(const v4f* __restrict__ s, v4f* __restrict__ d, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}

// tile t covers blocks [t*S, t*S + S) of 1024 eight-byte elements; 4 blocks
// of loads in flight per thread (S is a multiple of 4)
__global__ void __launch_bounds__(256) copy_tile8(const v2f* __restrict__ s, v2f* __restrict__ d, int S, int M) {
  const int m0 = blockIdx.x * S;
  for (int m = m0; m + 3 < m0 + S && m + 3 < M; m += 4) {
    v2f a[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        a[b][e] = __builtin_nontemporal_load(s + (long long)(m + b) * 1024 + threadIdx.x + e * 256);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        __builtin_nontemporal_store(a[b][e], d + (long long)(m + b) * 1024 + threadIdx.x + e * 256);
  }
}

__global__ void __launch_bounds__(256) write16(v4f* __restrict__ d, long long n) {
  const v4f v = {1.f, 2.f, 3.f, 4.f};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    __builtin_nontemporal_store(v, d + i);
}

// the sum keeps the loads live; one value per thread is written
__global__ void __launch_bounds__(256) read16(const v4f* __restrict__ s, v4f* __restrict__ out, long long n) {
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc += __builtin_nontemporal_load(s + i);
  out[blockIdx.x * 256 + threadIdx.x] = acc;
}

// element i: read 4 bytes (two int8 pairs), write 16 bytes (two FP32 pairs)
__global__ void __launch_bounds__(256) expand4(const unsigned* __restrict__ s, v4f* __restrict__ d, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const unsigned w = __builtin_nontemporal_load(s + i);
    const v4f v = {(float)(signed char)(w & 0xFF), (float)(signed char)((w >> 8) & 0xFF),
                   (float)(signed char)((w >> 16) & 0xFF), (float)(signed char)(w >> 24)};
    __builtin_nontemporal_store(v, d + i);
  }
}

double arg_d(int argc, char** argv, const char* name, double def) {
  for (int i = 1; i + 1 < argc; ++i)
    if (!strcmp(argv[i], name)) return atof(argv[i + 1]);
  return def;
}

}  // namespace

int main(int argc, char** argv) {
  const size_t mib = (size_t)arg_d(argc, argv, "--mib", 1024);
  const int reps = (int)arg_d(argc, argv, "--reps", 100);
  const int warm = (int)arg_d(argc, argv, "--warmup", 300);
  const size_t bytes = mib << 20;
  if (bytes % (8192ull * 4 * 4096) != 0) {
    fprintf(stderr, "--mib must be a multiple of 128\n");
    return 1;
  }
  void *s = nullptr, *d = nullptr;
  CK(hipMalloc(&s, bytes));
  CK(hipMalloc(&d, bytes));
  CK(hipMemset(s, 0, bytes));
  CK(hipMemset(d, 0, bytes));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const long long n16 = (long long)(bytes / 16);
  const int M = (int)(bytes / 8192);
  auto timed = [&](const char* name, auto launch, int warmup, size_t rd, size_t wr) {
    for (int i = 0; i < warmup; ++i) launch();
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(e0));
    for (int i = 0; i < reps; ++i) launch();
    CK(hipEventRecord(e1));
    CK(hipEventSynchronize(e1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    ms /= reps;
    printf("{\"pattern\": \"%s\", \"bytes_read\": %zu, \"bytes_written\": %zu, \"ms_per_copy\": %.5f, "
           "\"GBps_moved\": %.1f, \"frac_of_8TBps\": %.4f}\n",
           name, rd, wr, ms, (double)(rd + wr) / ms / 1e6, (double)(rd + wr) / ms / 1e6 / 8000.0);
    fflush(stdout);
  };
  timed("stride16_grid1024", [&] {
    hipLaunchKernelGGL(copy_stride16, dim3(1024), dim3(256), 0, 0, (const v4f*)s, (v4f*)d, n16);
  }, warm, bytes, bytes);
  for (int nb : {512, 4096}) {
    const int S = M / nb;
    char name[64];
    snprintf(name, sizeof name, "tile8_%dblocks", nb);
    timed(name, [&] {
      hipLaunchKernelGGL(copy_tile8, dim3(nb), dim3(256), 0, 0, (const v2f*)s, (v2f*)d, S, M);
    }, 20, bytes, bytes);
  }
  timed("write16_grid1024", [&] {
    hipLaunchKernelGGL(write16, dim3(1024), dim3(256), 0, 0, (v4f*)d, n16);
  }, 20, 0, bytes);
  timed("read16_grid1024", [&] {
    hipLaunchKernelGGL(read16, dim3(1024), dim3(256), 0, 0, (const v4f*)s, (v4f*)d, n16);
  }, 20, bytes, (size_t)1024 * 256 * 16);
  timed("expand_int8_to_f32_grid1024", [&] {
    hipLaunchKernelGGL(expand4, dim3(1024), dim3(256), 0, 0, (const unsigned*)s, (v4f*)d, n16);
  }, 20, bytes / 4, bytes);
  CK(hipFree(s));
  CK(hipFree(d));
  return 0;
}
