// Sustainable peaks of the machine resources the hot path is bound by,
// measured on the device in use (the figures a roofline fraction divides
// by; datasheet numbers assume issue patterns no real kernel reaches).
//
//   valu_i32 : independent 32-bit integer adds and xors, eight chains per
//              lane, every lane busy: int32 lane-operations per second.
//   l2/mall  : 4-byte gathers at pseudo-random offsets of a table that
//              fits one XCD's L2 (2 MiB) or only the last-level MALL
//              (128 MiB), eight loads in flight per lane: lane loads per
//              second (each touches its own cache line).
//   hbm_read : a streaming read of a buffer far larger than every cache,
//              16 bytes per lane per load: bytes per second.
//   hbm_copy : the same buffer copied: bytes read plus bytes written per
//              second.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "reloc.h"
#include "runtime_internal.h"

namespace reloc {
namespace {

constexpr int kPeakThreads = 256;

__global__ __launch_bounds__(kPeakThreads) void valu_i32_kernel(uint32_t* out, uint32_t seed,
                                                                int iters) {
  const uint32_t t = blockIdx.x * kPeakThreads + threadIdx.x;
  uint32_t a0 = seed ^ t, a1 = a0 * 3u + 1u, a2 = a0 * 5u + 2u, a3 = a0 * 7u + 3u;
  uint32_t a4 = a0 * 11u + 4u, a5 = a0 * 13u + 5u, a6 = a0 * 17u + 6u, a7 = a0 * 19u + 7u;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      a0 += a1;
      a1 ^= a2;
      a2 += a3;
      a3 ^= a4;
      a4 += a5;
      a5 ^= a6;
      a6 += a7;
      a7 ^= a0;
    }
  }
  const uint32_t r = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
  if (r == 0x12345678u) out[t] = r;   // practically never: keeps the work live
}

// Eight independent gathers per lane per iteration from tab[0, mask]; the
// offsets come from a per-lane linear congruential sequence that does not
// depend on the loaded values, so the loads can all be in flight.
__global__ __launch_bounds__(kPeakThreads) void gather_kernel(const uint32_t* __restrict__ tab,
                                                              uint32_t mask, uint32_t* out,
                                                              int iters) {
  const uint32_t t = blockIdx.x * kPeakThreads + threadIdx.x;
  uint32_t h = t * 2654435761u + 12345u;
  uint32_t acc = 0;
  for (int i = 0; i < iters; ++i) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      h = h * 1664525u + 1013904223u;
      v[u] = tab[(h >> 4) & mask];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  if (acc == 0x12345678u) out[t] = acc;
}

__global__ __launch_bounds__(kPeakThreads) void read_kernel(const uint4* __restrict__ src,
                                                            size_t n, uint32_t* out) {
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  uint32_t acc = 0;
  for (size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x; i < n; i += stride) {
    const uint4 v = src[i];
    acc += v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x12345678u) out[blockIdx.x * kPeakThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kPeakThreads) void copy_kernel(const uint4* __restrict__ src,
                                                            uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  for (size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

__global__ void fill_kernel(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)(i * 2654435761u);
}

// Best of `reps` timed launches (after one warm-up) in milliseconds.
template <typename F>
hipError_t time_best(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, F launch,
                     float* best) {
  launch();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  *best = -1.f;
  for (int r = 0; r < reps; ++r) {
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
    launch();
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
    if (*best < 0.f || ms < *best) *best = ms;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace reloc

using namespace reloc;

extern "C" int32_t reloc_measure_peaks(int32_t device, reloc_peaks* out) {
  if (!out) return fail(RELOC_E_INVALID, "null out");
  std::memset(out, 0, sizeof *out);
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(RELOC_E_DEVICE, "device %d not available", device);
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  const int cus = prop.multiProcessorCount;
  // buffers: a 1 GiB stream source and destination, a 128 MiB gather table
  const size_t big = (size_t)1 << 30, tab_bytes = (size_t)128 << 20;
  void *src = nullptr, *dst = nullptr, *tab = nullptr, *sink = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&src, big);
  if (e == hipSuccess) e = hipMalloc(&dst, big);
  if (e == hipSuccess) e = hipMalloc(&tab, tab_bytes);
  const size_t sink_n = (size_t)cus * 64 * kPeakThreads;
  if (e == hipSuccess) e = hipMalloc(&sink, sink_n * sizeof(uint32_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    const size_t nw = big / 4;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                       (uint32_t*)src, nw);
    const size_t nt = tab_bytes / 4;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s,
                       (uint32_t*)tab, nt);
    e = hipGetLastError();
  }
  float ms = 0.f;
  const int reps = 5;
  if (e == hipSuccess) {
    // 32 waves per CU (eight per SIMD), 128 iterations x 128 ops per lane
    const int blocks = cus * 8, iters = 2048;
    e = time_best(s, e0, e1, reps, [&] {
      hipLaunchKernelGGL(valu_i32_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                         (uint32_t*)sink, 17u, iters);
    }, &ms);
    if (e == hipSuccess)
      out->valu_i32_ops = (double)blocks * kPeakThreads * iters * 16.0 * 8.0 / (ms * 1e-3);
  }
  auto gather_rate = [&](size_t bytes, double* rate) -> hipError_t {
    const uint32_t mask = (uint32_t)(bytes / 4 - 1);
    const int blocks = cus * 8, iters = 256;
    hipError_t ee = time_best(s, e0, e1, reps, [&] {
      hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                         (const uint32_t*)tab, mask, (uint32_t*)sink, iters);
    }, &ms);
    if (ee == hipSuccess) *rate = (double)blocks * kPeakThreads * iters * 8.0 / (ms * 1e-3);
    return ee;
  };
  if (e == hipSuccess) e = gather_rate((size_t)2 << 20, &out->l2_gathers);
  if (e == hipSuccess) e = gather_rate(tab_bytes, &out->mall_gathers);
  if (e == hipSuccess) {
    const size_t n16 = big / 16;
    const int blocks = cus * 16;
    e = time_best(s, e0, e1, reps, [&] {
      hipLaunchKernelGGL(read_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                         (const uint4*)src, n16, (uint32_t*)sink);
    }, &ms);
    if (e == hipSuccess) out->hbm_read = (double)big / (ms * 1e-3);
  }
  if (e == hipSuccess) {
    const size_t n16 = big / 16;
    const int blocks = cus * 16;
    e = time_best(s, e0, e1, reps, [&] {
      hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                         (const uint4*)src, (uint4*)dst, n16);
    }, &ms);
    if (e == hipSuccess) out->hbm_copy = 2.0 * (double)big / (ms * 1e-3);
  }
  out->compute_units = cus;
  out->clock_khz = prop.clockRate;
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  (void)hipFree(src);
  (void)hipFree(dst);
  (void)hipFree(tab);
  (void)hipFree(sink);
  if (e != hipSuccess) {
    std::memset(out, 0, sizeof *out);
    return fail(RELOC_E_DEVICE, "peak measurement failed: %s", hipGetErrorString(e));
  }
  return RELOC_OK;
}
