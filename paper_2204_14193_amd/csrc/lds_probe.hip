// LDS read bandwidth of the device, measured for roofline accounting: every
// workgroup streams conflict-free 16-byte reads (64 consecutive lanes read
// 1 KiB of consecutive entries) from a 32 KiB LDS array, one xor per read
// into a value each thread stores, so that no read can be dropped and the
// vector unit is not the limit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fse.h"

namespace {

constexpr int kProbeThreads = 256, kProbeEntries = 2048, kProbeUnroll = 8;

__global__ __launch_bounds__(kProbeThreads) void k_lds_read(int iters, uint32_t* sink) {
  __shared__ uint4 buf[kProbeEntries];
  const int t = threadIdx.x;
  for (int i = t; i < kProbeEntries; i += kProbeThreads)
    buf[i] = make_uint4((uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u);
  __syncthreads();
  uint32_t a0 = 0;
  const uint4* p = buf + t;  // entries t + u * 256, u < 8: the whole array, immediate offsets
  static_assert(kProbeUnroll * kProbeThreads == kProbeEntries, "one pass reads the array once");
  for (int it = 0; it < iters; ++it) {
    asm volatile("" ::: "memory");  // every pass reads LDS again
    uint4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = p[u * kProbeThreads];  // eight reads in flight
#pragma unroll
    for (int u = 0; u < kProbeUnroll; u += 2)  // all 16 bytes of every read are used
      asm volatile("" ::"v"(v[u].x), "v"(v[u].y), "v"(v[u].z), "v"(v[u].w), "v"(v[u + 1].x), "v"(v[u + 1].y),
                   "v"(v[u + 1].z), "v"(v[u + 1].w));
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) a0 ^= v[u].x;
  }
  sink[(size_t)blockIdx.x * kProbeThreads + t] = a0;
}

}  // namespace

extern "C" fse_status_t fse_measure_lds_bandwidth(int32_t iters, void* stream, double* bytes_per_s) {
  if (!bytes_per_s || iters < 1 || iters > (1 << 20)) return FSE_ERR_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return FSE_ERR_HIP;
  const int grid = prop.multiProcessorCount * 5;
  uint32_t* sink = nullptr;
  if (hipMalloc(&sink, (size_t)grid * kProbeThreads * sizeof(uint32_t)) != hipSuccess) return FSE_ERR_OOM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fse_status_t st = FSE_OK;
  float ms = 0.f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = FSE_ERR_HIP;
  } else {
    for (int w = 0; w < 3; ++w)  // warm-up (clocks)
      hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(kProbeThreads), 0, s, iters, sink);
    // the median of five timed launches
    float t[5];
    for (int r = 0; r < 5 && st == FSE_OK; ++r) {
      const hipError_t r0 = hipEventRecord(e0, s);
      hipLaunchKernelGGL(k_lds_read, dim3(grid), dim3(kProbeThreads), 0, s, iters, sink);
      const hipError_t r1 = hipEventRecord(e1, s);
      if (r0 != hipSuccess || r1 != hipSuccess || hipGetLastError() != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t[r], e0, e1) != hipSuccess || !(t[r] > 0.f))
        st = FSE_ERR_HIP;
    }
    if (st == FSE_OK) {
      std::sort(t, t + 5);
      ms = t[2];
    }
  }
  if (st == FSE_OK)
    *bytes_per_s = (double)grid * kProbeThreads * iters * kProbeUnroll * 16.0 / (ms * 1e-3);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(sink);
  return st;
}
