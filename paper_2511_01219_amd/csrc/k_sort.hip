// Stable orders of 64-bit keys: the SMAD order (ascending (SMAD, index),
// Sec. III pipeline) and the final ranking of evaluated poses (ascending
// ((~T bits) << 32 | rank), eq. 8-9), for one request or for the segments
// of several requests at once.
//
// The order of a segment is an argsort of (key, position) pairs, which are
// all distinct, so any correct sort of the pairs is the stable order of the
// keys:
//  1. every 1024-key tile of a segment is sorted in LDS by a bitonic network
//     over (key, position) (one workgroup per tile, in place);
//  2. merge levels: sorted runs of length L are merged G at a time into runs
//     of length G L (G <= 8). A key's place in the merged run is its place
//     in its own run plus, for every other run of its group, the number of
//     keys there that precede it: keys of an earlier run that are equal
//     precede it (smaller positions), those of a later run do not. The
//     counts come from binary searches, one thread per (key, run) pair, and
//     meet in LDS.
// A 200 000-key segment takes the tile sort and three merge levels (runs of
// 1024, 8192 and 65 536 keys merged 8, 8 and 4 at a time). No kernel waits
// on another workgroup.
#include <climits>
#include <vector>

#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int kTileThreads = 256, kTile = 1024;
constexpr int kRankMax = 2 * kTileThreads;   // tiles of at most this many keys are ranked

// Index of the segment holding item t: prefix[s] <= t < prefix[s + 1].
__device__ __forceinline__ int find_seg(const int64_t* prefix, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Segment bounds of a launch: one segment [0, n) when off is null.
struct Segs {
  const int64_t* off;    // [nseg + 1] key offsets, or null
  const int64_t* tpre;   // [nseg + 1] tile prefix (tiles of 1024 keys per segment), or null
  int nseg;
  int64_t n;             // total keys
};

__device__ __forceinline__ bool pair_less(uint64_t ka, int32_t pa, uint64_t kb, int32_t pb) {
  return ka < kb || (ka == kb && pa < pb);
}

// Sort of one tile of (key, position) pairs: kin[base + t0 + i] for
// i < cnt, sorted into kout / pos at the same places (kout may be kin: the
// tile is read whole before it is written); positions are positions in the
// segment. A bitonic network in LDS, or for a tile of at most 512 keys a
// rank count; padding pairs (~0, INT_MAX) of the network sort last and are
// not stored.
__global__ __launch_bounds__(kTileThreads) void tile_sort_kernel(const uint64_t* kin, Segs sg,
                                                                 uint64_t* kout,
                                                                 int32_t* __restrict__ pos) {
  __shared__ uint64_t sk[kTile];
  __shared__ int32_t sp[kTile];
  int64_t base = 0, n_s = sg.n, t = blockIdx.x;
  if (sg.off) {
    const int s = find_seg(sg.tpre, sg.nseg, t);
    t -= sg.tpre[s];
    base = sg.off[s];
    n_s = sg.off[s + 1] - base;
  }
  const int64_t t0 = t * kTile;
  const int cnt = (int)min((int64_t)kTile, n_s - t0);
  if (cnt <= kRankMax) {                 // workgroup-uniform
    // a small tile: every pair's place is the number of pairs that precede
    // it (keys of smaller position that are equal or smaller, keys of larger
    // position that are smaller; the pairs are distinct, so the places are
    // a permutation), two pairs per thread against the tile in LDS, all lanes
    // of a wavefront reading the same word at a time: no barrier between
    // steps (the network below takes 55 barrier-separated steps, 28 us,
    // whatever the count)
    constexpr int PER = kRankMax / kTileThreads;
    uint64_t mine[PER];
    int rank[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = threadIdx.x + r * kTileThreads;
      mine[r] = 0;
      rank[r] = 0;
      if (i < cnt) sk[i] = mine[r] = kin[base + t0 + i];
    }
    __syncthreads();
    for (int j = 0; j < cnt; ++j) {
      const uint64_t kj = sk[j];
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * kTileThreads;
        rank[r] += (kj < mine[r] || (kj == mine[r] && j < i)) ? 1 : 0;
      }
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int i = threadIdx.x + r * kTileThreads;
      if (i < cnt) {
        kout[base + t0 + rank[r]] = mine[r];
        pos[base + t0 + rank[r]] = (int32_t)(t0 + i);
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < kTile; i += kTileThreads) {
    const bool in = i < cnt;
    sk[i] = in ? kin[base + t0 + i] : ~0ull;
    sp[i] = in ? (int32_t)(t0 + i) : INT_MAX;
  }
  __syncthreads();
  for (int k = 2; k <= kTile; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int r = 0; r < kTile / 2 / kTileThreads; ++r) {
        const int q = threadIdx.x + r * kTileThreads;   // pair index
        const int i = 2 * j * (q / j) + (q % j), l = i + j;
        const bool asc = (i & k) == 0;
        const uint64_t ki = sk[i], kl = sk[l];
        const int32_t pi = sp[i], pl = sp[l];
        const bool swap = asc ? pair_less(kl, pl, ki, pi) : pair_less(ki, pi, kl, pl);
        if (swap) {
          sk[i] = kl;
          sk[l] = ki;
          sp[i] = pl;
          sp[l] = pi;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < cnt; i += kTileThreads) {
    kout[base + t0 + i] = sk[i];
    pos[base + t0 + i] = sp[i];
  }
}

// number of keys in a[0, len) that are < x (strict) or <= x
__device__ __forceinline__ int64_t count_before(const uint64_t* a, int64_t len, uint64_t x,
                                                bool le) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const uint64_t v = a[mid];
    if (v < x || (le && v == x)) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One merge level: runs of L keys of every segment merged G at a time.
// Workgroup: 256 / G keys, one thread per (key, run of its group).
__global__ __launch_bounds__(256) void merge_level_kernel(const uint64_t* __restrict__ kin,
                                                          const int32_t* __restrict__ pin,
                                                          Segs sg, int64_t L, int G,
                                                          uint64_t* __restrict__ kout,
                                                          int32_t* __restrict__ pout) {
  __shared__ int64_t acc[256];
  const int tid = threadIdx.x;
  const int E = 256 / G;
  const int e = tid / G, u = tid - e * G;
  const int64_t g = (int64_t)blockIdx.x * E + e;
  if (tid < E) acc[tid] = 0;
  __syncthreads();
  if (e < E && g < sg.n) {
    int64_t base = 0, n_s = sg.n;
    if (sg.off) {
      const int s = find_seg(sg.off, sg.nseg, g);
      base = sg.off[s];
      n_s = sg.off[s + 1] - base;
    }
    const int64_t i = g - base, r = i / L, r0 = r / G * G, ru = r0 + u;
    if (ru * L < n_s) {
      const int64_t c = ru == r ? i - r * L
                                : count_before(kin + base + ru * L, min(L, n_s - ru * L), kin[g],
                                               ru < r);
      atomicAdd((unsigned long long*)&acc[e], (unsigned long long)c);
    }
  }
  __syncthreads();
  const int64_t gg = (int64_t)blockIdx.x * E + tid;
  if (tid < E && gg < sg.n) {
    int64_t base = 0;
    if (sg.off) base = sg.off[find_seg(sg.off, sg.nseg, gg)];
    const int64_t r0 = (gg - base) / L / G * G;
    const int64_t d = base + r0 * L + acc[tid];
    kout[d] = kin[gg];
    pout[d] = pin[gg];
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

// Group size of a level: runs of L keys of the largest segment, merged at
// most 8 at a time (a power of two, so 256 / G keys fill a workgroup). A
// level costs each key G binary searches of log2(L) steps: merging 64 runs
// of 1024 at once (two levels for 200 000 keys) made 2.8x the searches of
// three levels of at most 8 (200 000 keys: 0.25 ms of merging before, the
// whole stress relocalization 0.18 ms shorter after).
int level_group(int64_t max_n, int64_t L) {
  const int64_t runs = (max_n + L - 1) / L;
  int G = 2;
  while (G < 8 && G < runs) G <<= 1;
  return G;
}

}  // namespace

int argsort_levels(int64_t max_n) {
  int m = 0;
  for (int64_t L = kTile; L < max_n; L *= level_group(max_n, L)) ++m;
  return m;
}

hipError_t argsort_u64(uint64_t* keys, uint64_t* tmp_k, int32_t* tmp_p, int32_t* pos,
                       int64_t n, int nseg, const int64_t* off, const int64_t* tpre,
                       int64_t tiles, int64_t max_n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (nseg < 1 || (nseg > 1 && (!off || !tpre))) return hipErrorInvalidValue;
  Segs sg{nseg > 1 ? off : nullptr, nseg > 1 ? tpre : nullptr, nseg, n};
  if (nseg == 1) {
    tiles = (n + kTile - 1) / kTile;
    max_n = n;
  }
  const int m = argsort_levels(max_n);
  // the levels alternate between (tmp_k, tmp_p) and (keys, pos) and must
  // end in (keys, pos): the tile sort (in place) writes the buffer pair the
  // parity of the level count calls for
  uint64_t* ka = (m % 2 == 0) ? keys : tmp_k;
  int32_t* pa = (m % 2 == 0) ? pos : tmp_p;
  hipLaunchKernelGGL(tile_sort_kernel, dim3((unsigned)tiles), dim3(kTileThreads), 0, s, keys, sg,
                     ka, pa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t* kb = ka == keys ? tmp_k : keys;
  int32_t* pb = pa == pos ? tmp_p : pos;
  for (int64_t L = kTile; L < max_n;) {
    const int G = level_group(max_n, L);
    const int E = 256 / G;
    hipLaunchKernelGGL(merge_level_kernel, dim3((unsigned)((n + E - 1) / E)), dim3(256), 0, s,
                       ka, pa, sg, L, G, kb, pb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(ka, kb);
    std::swap(pa, pb);
    L *= G;
  }
  return hipSuccess;
}

int64_t argsort_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

hipError_t launch_rank_small(const uint64_t* best, int n, const int32_t* order,
                             const double* smad, int nrow, PoseRow* rows, hipStream_t s) {
  if (n <= 0 || n > 2048) return hipErrorInvalidValue;
  const int threads = n <= 64 ? 64 : (n <= 256 ? 256 : 1024);
  hipLaunchKernelGGL(rank_small_kernel, dim3(1), dim3(threads), 0, s, best, n, order, smad, nrow,
                     rows);
  return hipGetLastError();
}

}  // namespace reloc
