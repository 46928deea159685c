// Stable sorts for the SMAD order (ascending (SMAD, index)) and for the
// final ranking of evaluated poses: hipCUB / rocPRIM device radix sorts, and
// for up to kSmallSortMax keys a two-kernel sort: every 1024-key tile is
// sorted in LDS by a stable block radix sort, then every key finds its final
// position as its position in its tile plus, for every other tile, the
// number of keys there that precede it (binary searches, one thread per
// key and tile; keys of earlier tiles that are equal precede it, since
// indices grow with the tile).
#include <hipcub/hipcub.hpp>

#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int kTileThreads = 256, kTileItems = 4, kTile = kTileThreads * kTileItems;

// Stable sort of each tile of (key, index) pairs; indices are positions in
// the input. Padding keys (~0) sort last and are not stored.
__global__ __launch_bounds__(kTileThreads) void tile_sort_kernel(const uint64_t* __restrict__ kin,
                                                                 int n, uint64_t* __restrict__ kout,
                                                                 int32_t* __restrict__ vout) {
  using BRS = hipcub::BlockRadixSort<uint64_t, kTileThreads, kTileItems, int32_t>;
  __shared__ typename BRS::TempStorage tmp;
  const int base = blockIdx.x * kTile;
  uint64_t k[kTileItems];
  int32_t v[kTileItems];
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) {
    const int idx = base + threadIdx.x * kTileItems + i;
    k[i] = idx < n ? kin[idx] : ~0ull;
    v[i] = idx;
  }
  BRS(tmp).Sort(k, v);
#pragma unroll
  for (int i = 0; i < kTileItems; ++i) {
    const int idx = base + threadIdx.x * kTileItems + i;
    if (idx < n) {
      kout[idx] = k[i];
      vout[idx] = v[i];
    }
  }
}

// number of keys in a[0, len) that are < x (strict) or <= x
__device__ __forceinline__ int count_before(const uint64_t* a, int len, uint64_t x, bool le) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const uint64_t v = a[mid];
    if (v < x || (le && v == x)) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Every key's final position: its position in its tile plus, for every
// other tile, the number of keys there that precede it. One thread per
// (key, tile) pair, so a key's binary searches run side by side rather than
// one after another; the counts meet in LDS. nt <= 64 tiles (n <= 65 536),
// 256 / nt keys per workgroup.
__global__ __launch_bounds__(256) void merge_rank_kernel(const uint64_t* __restrict__ kt,
                                                         const int32_t* __restrict__ vt, int n,
                                                         int nt, uint64_t* __restrict__ kout,
                                                         int32_t* __restrict__ vout) {
  __shared__ int acc[256];
  const int tid = threadIdx.x;
  const int E = 256 / nt;                      // keys of this workgroup
  const int e = tid / nt, u = tid - e * nt;    // key e, tile u
  const int g = blockIdx.x * E + e;
  if (tid < E) acc[tid] = 0;
  __syncthreads();
  if (e < E && g < n) {
    const int t = g / kTile;
    const int cnt = u == t ? g - t * kTile
                           : count_before(kt + (size_t)u * kTile, min(kTile, n - u * kTile),
                                          kt[g], u < t);
    atomicAdd(&acc[e], cnt);
  }
  __syncthreads();
  const int gg = blockIdx.x * E + tid;
  if (tid < E && gg < n) {
    const int rank = acc[tid];
    if (kout) kout[rank] = kt[gg];
    vout[rank] = vt[gg];
  }
}

// Ranking of n <= 2048 evaluated ranks in one workgroup: the keys
// ((~T bits) << 32 | rank) are distinct, so a key's position in the
// ascending order (T desc, rank asc) is the number of keys below it, counted
// against a copy of all keys in LDS; rows for the first nrow positions.
__global__ __launch_bounds__(1024) void rank_small_kernel(const uint64_t* __restrict__ best, int n,
                                                          const int32_t* __restrict__ order,
                                                          const double* __restrict__ smad,
                                                          int nrow, PoseRow* __restrict__ rows) {
  __shared__ uint64_t sk[2048];
  for (int r = threadIdx.x; r < n; r += blockDim.x)
    sk[r] = ((uint64_t)(0xFFFFFFFFu - (uint32_t)(best[r] >> 32)) << 32) | (uint32_t)r;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const uint64_t x = sk[r];
    int p = 0;
    for (int j = 0; j < n; ++j) p += sk[j] < x ? 1 : 0;
    if (p < nrow) {
      const uint64_t b = best[r];
      PoseRow row;
      row.rank = r;
      row.k = (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFu));
      row.hyp = order[r];
      row.tbits = (uint32_t)(b >> 32);
      row.smad = smad[row.hyp];
      rows[p] = row;
    }
  }
}

}  // namespace

hipError_t launch_rank_small(const uint64_t* best, int n, const int32_t* order,
                             const double* smad, int nrow, PoseRow* rows, hipStream_t s) {
  if (n <= 0 || n > 2048) return hipErrorInvalidValue;
  const int threads = n <= 64 ? 64 : (n <= 256 ? 256 : 1024);
  hipLaunchKernelGGL(rank_small_kernel, dim3(1), dim3(threads), 0, s, best, n, order, smad, nrow,
                     rows);
  return hipGetLastError();
}

hipError_t small_sort_pairs_u64(const uint64_t* kin, uint64_t* ktmp, int32_t* vtmp,
                                uint64_t* kout, int32_t* vout, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > kSmallSortMax) return hipErrorInvalidValue;
  const int nt = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL(tile_sort_kernel, dim3(nt), dim3(kTileThreads), 0, s, kin, n, ktmp, vtmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int per = 256 / nt;                    // nt <= 64 for n <= kSmallSortMax
  hipLaunchKernelGGL(merge_rank_kernel, dim3((n + per - 1) / per), dim3(256), 0, s, ktmp, vtmp,
                     n, nt, kout, vout);
  return hipGetLastError();
}

hipError_t sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                              uint64_t* kout, const int32_t* vin, int32_t* vout, int n,
                              hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin, vout, n, 0, 64,
                                            s);
}

hipError_t sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                         int n, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortKeys(tmp, *tmp_bytes, kin, kout, n, 0, 64, s);
}

hipError_t seg_sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                                  uint64_t* kout, const int32_t* vin, int32_t* vout, int64_t n,
                                  int nseg, const int64_t* offsets, hipStream_t s) {
  return hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin, vout,
                                                     (int)n, nseg, offsets, offsets + 1, 0, 64,
                                                     s);
}

hipError_t seg_sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                             int64_t n, int nseg, const int64_t* offsets, hipStream_t s) {
  return hipcub::DeviceSegmentedRadixSort::SortKeys(tmp, *tmp_bytes, kin, kout, (int)n, nseg,
                                                    offsets, offsets + 1, 0, 64, s);
}

}  // namespace reloc
