// Map residency kernels: 8x8-tile bit packing of the occupancy grid and the
// exact Euclidean distance transform (the lookup table behind
// MinDistToObstacle, Sec. III-A, and TAM's d_obs, eq. 23).
#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int32_t kFar = 1 << 20;   // "no obstacle in this column" marker

__global__ void bitpack_kernel(const int8_t* __restrict__ occ, int W, int H, int thr,
                               uint64_t* __restrict__ bits, int tpr, int tph) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tpr * tph) return;
  const int tx = t % tpr, ty = t / tpr;
  uint64_t w = 0;
  for (int r = 0; r < 8; ++r) {
    const int y = ty * 8 + r;
    if (y >= H) break;
    for (int c = 0; c < 8; ++c) {
      const int x = tx * 8 + c;
      if (x >= W) break;
      if ((int)occ[(size_t)y * W + x] >= thr) w |= 1ull << (r * 8 + c);
    }
  }
  bits[t] = w;
}

// Pass 1: per column, the distance (in cells) to the nearest occupied cell of
// the same column, by a forward and a backward sweep. Adjacent threads take
// adjacent columns, so every row access is coalesced.
__global__ void edt_cols_kernel(const int8_t* __restrict__ occ, int W, int H, int thr,
                                int32_t* __restrict__ g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  int last = -1;
  for (int y = 0; y < H; ++y) {
    if ((int)occ[(size_t)y * W + x] >= thr) last = y;
    g[(size_t)y * W + x] = last < 0 ? kFar : y - last;
  }
  last = -1;
  for (int y = H - 1; y >= 0; --y) {
    if ((int)occ[(size_t)y * W + x] >= thr) last = y;
    if (last >= 0) {
      const int d = last - y;
      int32_t* p = g + (size_t)y * W + x;
      if (d < *p) *p = d;
    }
  }
}

// Pass 2: k(x, y) = min over x' of (x - x')^2 + g(x', y)^2, scanning x' outward
// from x and stopping once (x - x')^2 alone reaches the best value found.
// Exact in 64-bit integers; the work per cell is proportional to its
// distance to the nearest obstacle.
__global__ void edt_rows_kernel(const int32_t* __restrict__ g, int W, int H,
                                uint32_t* __restrict__ k) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  const int32_t* row = g + (size_t)y * W;
  int64_t g0 = row[x];
  int64_t best = g0 >= kFar ? INT64_MAX : g0 * g0;
  for (int d = 1; d < W; ++d) {
    const int64_t d2 = (int64_t)d * d;
    if (d2 >= best) break;
    if (x - d >= 0) {
      const int64_t gl = row[x - d];
      if (gl < kFar) {
        const int64_t v = d2 + gl * gl;
        if (v < best) best = v;
      }
    }
    if (x + d < W) {
      const int64_t gr = row[x + d];
      if (gr < kFar) {
        const int64_t v = d2 + gr * gr;
        if (v < best) best = v;
      }
    }
  }
  k[(size_t)y * W + x] = best == INT64_MAX ? 0xFFFFFFFFu : (uint32_t)best;
}

// TAM planes: 2 k per cell in strips of 8 columns, 32-bit and 16-bit (2 k
// below 2^15, else the escape 0xFFFE), the sentinel in column W and row H
// (and the padding of the last strip and rows); one entry of each per
// thread, written in plane order.
__global__ void tam_plane_kernel(const uint32_t* __restrict__ k, int W, int H,
                                 uint32_t* __restrict__ plane, uint16_t* __restrict__ plane16) {
  const size_t per_strip = (size_t)8 * tam_plane_rows(H);
  const size_t n = tam_plane_entries(W, H);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const size_t st = i / per_strip, r = i - st * per_strip;
  const uint32_t y = (uint32_t)(r >> 3), x = (uint32_t)(st * 8 + (r & 7));
  uint32_t v = 0xFFFFFFFFu;
  uint16_t h = 0xFFFFu;
  if (x < (uint32_t)W && y < (uint32_t)H) {
    const uint32_t kk = k[(size_t)y * W + x];
    v = 2u * kk;
    h = kk < (1u << 14) ? (uint16_t)v : (uint16_t)0xFFFEu;
  }
  plane[i] = v;
  plane16[i] = h;
}

}  // namespace

hipError_t launch_tam_plane(const uint32_t* k, int W, int H, uint32_t* plane, hipStream_t s) {
  const size_t n = tam_plane_entries(W, H);
  hipLaunchKernelGGL(tam_plane_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, W, H,
                     plane, reinterpret_cast<uint16_t*>(plane + n));
  return hipGetLastError();
}

hipError_t launch_bitpack(const int8_t* occ, int W, int H, int thr, uint64_t* bits, int tpr,
                          int tph, hipStream_t s) {
  const int n = tpr * tph;
  hipLaunchKernelGGL(bitpack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, occ, W, H, thr,
                     bits, tpr, tph);
  return hipGetLastError();
}

hipError_t launch_edt(const int8_t* occ, int W, int H, int thr, int32_t* g, uint32_t* k,
                      hipStream_t s) {
  hipLaunchKernelGGL(edt_cols_kernel, dim3((W + 255) / 256), dim3(256), 0, s, occ, W, H, thr,
                     g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(edt_rows_kernel, dim3((W + 255) / 256, H), dim3(256), 0, s, g, W, H, k);
  return hipGetLastError();
}

}  // namespace reloc
