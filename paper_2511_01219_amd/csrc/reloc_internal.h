// Internal declarations shared by the host runtime and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "raycast.h"

namespace reloc {

// ---- sorting --------------------------------------------------------------
// Stable argsort of uint64 keys, per segment: pos[off[s] + j] = position in
// segment s of its j-th smallest key (ties: smaller position first), and
// keys[off[s] + j] = that key (the sorted keys end in `keys`). tmp_k /
// tmp_p: scratch of n entries. One segment [0, n) when nseg == 1 (off, tpre,
// tiles, max_n unused); else off / tpre: device int64[nseg + 1] key
// offsets and tile prefix (argsort_tiles(n_s) tiles per segment), tiles their
// total, max_n the largest segment. Every launch is a kernel (no memset or
// copy nodes, no library scratch), so the whole sort can be captured.
hipError_t argsort_u64(uint64_t* keys, uint64_t* tmp_k, int32_t* tmp_p, int32_t* pos,
                       int64_t n, int nseg, const int64_t* off, const int64_t* tpre,
                       int64_t tiles, int64_t max_n, hipStream_t s);
int64_t argsort_tiles(int64_t n);
// Merge levels after the tile sort for a largest segment of max_n keys.
int argsort_levels(int64_t max_n);

// ---- TAM -----------------------------------------------------------------
// TAM planes of a W x H map from its squared EDT k, one allocation of
// tam_plane_bytes: first the 32-bit plane, cell (x, y) holding 2 k (below
// 2^32 for maps up to 32767 cells a side), then the 16-bit plane the TAM
// gathers read, holding 2 k for k < 2^14 (below 2^15) and the escape
// 0xFFFE for farther cells (whose 2 k the 32-bit plane gives). Column W and
// row H hold the sentinel, 2^32 - 1 and 0xFFFF (odd, so never 2 k). Both
// in one layout: strips of 8 columns side by side, each tam_plane_rows(H)
// rows of 8 entries, so a 128-byte line of the 16-bit plane is 8 x 8 cells
// (4 rows of a strip: 8 x 4 cells in the 32-bit plane); at most 2^30
// entries, so a byte offset fits in 32 bits.
__host__ __device__ inline uint32_t tam_plane_rows(int H) { return (((uint32_t)H + 4u) >> 2) << 2; }
__host__ __device__ inline size_t tam_plane_entries(int W, int H) {
  return (size_t)(((uint32_t)W + 8u) >> 3) * 8 * tam_plane_rows(H);
}
__host__ __device__ inline size_t tam_plane_bytes(int W, int H) { return tam_plane_entries(W, H) * 6; }
// entry (x >> 3) 8 rows + 8 y + (x & 7), written as (x & ~7)(rows - 1) + 8 y + x
// (one 24-bit multiply-add); rows1 = tam_plane_rows(H) - 1
__device__ __forceinline__ uint32_t tam_plane_index(uint32_t x, uint32_t y, uint32_t rows1) {
  return __umul24(x & ~7u, rows1) + ((y << 3) + x);
}
hipError_t launch_tam_plane(const uint32_t* k, int W, int H, uint32_t* plane, hipStream_t s);

struct TamArgs {
  const uint32_t* kmap;      // [W H] squared EDT
  const uint32_t* plane;     // 32-bit TAM plane (launch_tam_plane)
  const uint16_t* plane16;   // 16-bit TAM plane, after the 32-bit one
  const uint32_t* off;       // [Ng][off_stride] endpoint offsets (launch_tam_offsets)
  int off_stride;            // 64 x keys per lane of the request's kernel class
  int W, H;
  const int32_t* hyp_xy;
  const int32_t* order;      // hypothesis index per SMAD rank
  int r0, nb;                // ranks [r0, r0 + nb)
  const int2* beams;         // [nvp] ((b * j_v) mod Ng, range in Q8 cells), padded
                             // with (0, 0) to nvp = tam_beams_padded(nv)
  int nv;
  const int2* dirs;          // [2 Ng] direction table, stored twice
  int Ng, o, Nt;             // o = Ng / Nt
  const int32_t* lut;        // [2^keybits + 1] l - lmin per selection key (Q26), 0 last
  int lmin;                  // the smallest l of the table (Q26)
  int kcap, key_off, keybits;
  int kmid;
  double res, d_max;
  int fine;                  // score: 0 T (eq. 31), 1 T_mean (eq. 34), 2 baseline (eq. 33),
                             // 3 LF (eq. 32)
  float* T_out;              // optional [nb][Nt]
  uint64_t* best;            // [>= r0 + nb] packed (score_key(T), ~k) per rank
};
hipError_t launch_tam(const TamArgs& a, hipStream_t s);
// Workgroups per rank of the TAM kernels: 16 orientations each.
__host__ __device__ inline int tam_tiles_per_rank(const TamArgs& a) { return (a.Nt + 15) / 16; }
// Beam-table length: nv rounded up to 512 entries (padded with (0, 0)).
constexpr int kTamBeamPad = 512;
__host__ __device__ inline int tam_beams_padded(int nv) {
  return (nv + kTamBeamPad - 1) / kTamBeamPad * kTamBeamPad;
}
// Valid beams per lane of a TAM kernel class: nv beams spread over 64
// lanes, rounded up to 4, 8, 12, 16, 24, 32, 48 or 64 (0: more than 4096).
__host__ __device__ inline int tam_keys_per_lane(int nv) {
  const int r = (nv + 63) / 64;
  return r <= 4 ? 4 : r <= 8 ? 8 : r <= 12 ? 12 : r <= 16 ? 16 : r <= 24 ? 24
       : r <= 32 ? 32 : r <= 48 ? 48 : r <= 64 ? 64 : 0;
}
// Endpoint-offset table of a request: for every heading g < Ng and beam slot
// v < stride = 64 tam_keys_per_lane(nv), the endpoint cell of beam v at
// heading g relative to the hypothesis cell,
//   dx = floor((2^27 + zq U_x) / 2^28), dy likewise (exact in 64 bits; the
//   hypothesis sits at its cell centre, X = 256 ix + 128 in Q8),
// clamped to [-32767, 32767] and packed as (uint16)dx | (uint16)dy << 16;
// slots of beams v >= nv hold dy = -32768 (never inside a map). Row g is
// read in 16-byte groups, slot 4 (64 b + l) + q holding beam 256 b + 64 q
// + l: lane l's q-th gather of batch b, so each gather instruction covers
// 64 consecutive beams.
// beams: [nv] (b j_v, zq_v); dirs: [2 Ng]; off: [Ng][stride], 16-byte aligned.
hipError_t launch_tam_offsets(const int2* beams, int nv, const int2* dirs, int Ng, int stride,
                              uint32_t* off, hipStream_t s);


// Scores (the request's fine metric) of n explicit poses: cell xy[2q],
// xy[2q + 1] (in the map) and heading index g[q] on the Ng grid (< Ng).
struct PoseArgs {
  TamArgs t;
  const int32_t* xy;         // [n][2]
  const int32_t* g;          // [n]
  int n;
  float* out;                // [n]
};
hipError_t launch_score_poses(const PoseArgs& a, hipStream_t s);

// Local refinement of each stage's best poses: an exhaustive TAM search over
// the lattice of poses next to each (cells within +-h, headings within +-s
// steps of the Ng direction grid; off-map and occupied cells other than the
// pose's own are skipped; ties to the pose itself, then the smaller raster
// index q = ((dg + s)(2h + 1) + dy + h)(2h + 1) + dx + h).
struct RefineArgs {
  TamArgs t;                 // TAM tables of the request; t.best per rank
  const int32_t* sel;        // [n_slots] rank refined in each slot, -1 none
  uint64_t* rbest;           // [n_slots] lattice best (score_key(T), ~tie key)
  int n_slots;
  int h, s, L;               // half-widths (cells, headings), lattice size
};
// Slots [b kr, (b + 1) kr) of stage b < ns (ranks [r0 + b K, ...) up to n):
// its kr best ranks by (T desc, rank asc), or -1; clears their rbest.
hipError_t launch_refine_select(const uint64_t* best, int r0, int K, int n, int ns, int kr,
                                int32_t* sel, uint64_t* rbest, hipStream_t s);
// Lattice TAM of every slot into rbest (atomic max of (score key, ~tie key)).
hipError_t launch_refine(const RefineArgs& a, hipStream_t s);
// best[sel[j]] = (refined score key, g << 10 | (dy + 15) << 5 | (dx + 15)).
hipError_t launch_refine_commit(const RefineArgs& a, hipStream_t s);

// The packed per-rank words hold an order-preserving 32-bit key of the
// score in their high half (larger score, larger key; negative scores too).
__host__ __device__ inline uint32_t score_key(float v) {
  const uint32_t b = __builtin_bit_cast(uint32_t, v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float score_of_key(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __builtin_bit_cast(float, b);
}

struct StageArgs {
  const uint64_t* best;      // per rank
  int r0, nb;
  double tau;                // NaN: never stop
  uint64_t* stage_out;       // [1] packed (score_key(T), ~rank)
  int32_t* flag_out;         // [1] 1 = stop
};
hipError_t launch_stage_reduce(const StageArgs& a, hipStream_t s);
// ns consecutive stages of K ranks from a.r0 (the last ends at n); stage j
// writes a.stage_out[j], a.flag_out[j]
hipError_t launch_stage_reduce_multi(const StageArgs& a, int K, int ns, int n, hipStream_t s);



hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);

// rank keys: ((~T bits) << 32 | rank) for ranks [0, n)
hipError_t launch_rank_keys(const uint64_t* best, int n, uint64_t* keys, hipStream_t s);

struct PoseRow {
  int32_t rank, k, hyp;
  uint32_t tbits;
  double smad;
};
// rows[i] for i < n from the sorted rank keys
hipError_t launch_rank_gather(const uint64_t* sorted, const uint64_t* best,
                              const int32_t* order, const double* smad, int n, PoseRow* rows,
                              hipStream_t s);

// Ambiguity: the best evaluated pose distinct from the top-1 (row 0) by the
// paper's success criterion (Sec. IV-C): position at least 0.5 m away,
// (dx^2 + dy^2) res^2 >= 0.25 in FP64 over cells, or heading at least 30 deg
// away, 12 * (circular distance in Ng steps) >= Ng. out[0] = its packed
// (score key, ~rank), 0 when there is none; out[1] = 1 when a stage's stop
// decision was within 1e-4 of tau (stage bests of the n_stages stages run;
// stage may be null); out[2] = the top-1 rank's packed word (0 when the top
// row names no evaluated rank). One workgroup.
struct MarginArgs {
  const uint64_t* best;      // [n_eval] packed per-rank words
  const int32_t* order;      // hypothesis per rank
  const int32_t* hyp_xy;     // cells of the set
  const PoseRow* top;        // row 0 of the ranking
  int n_eval, Ng, o;
  double res;
  const uint64_t* stage;     // [n_stages] packed stage bests
  int n_stages, stopped;
  double tau;                // NaN: no stop decisions
  uint64_t* out;             // [3]: best distinct, stop fragility, top-1 word
};
hipError_t launch_margin(const MarginArgs& a, hipStream_t s);

// Ranking of n <= 2048 ranks in one launch (T desc, rank asc), first nrow rows.
constexpr int kRankSmallMax = 2048;
hipError_t launch_rank_small(const uint64_t* best, int n, const int32_t* order,
                             const double* smad, int nrow, PoseRow* rows, hipStream_t s);

// ---- batched TAM / stage control / ranking -------------------------------
// Kernel class of a TAM argument set (keys per lane x key bits x whether
// the score needs the full l sum), -1 if unsupported; items of one launch
// share a class.
constexpr int kTamClasses = 32;
int tam_class(const TamArgs& a);
size_t tam_lds_bytes(const TamArgs& a);
// items: device TamArgs[n] (each a rank range of one request); prefix:
// device int64[n + 1] block offsets, nb x ceil(Nt / 16) blocks per item.
hipError_t launch_tam_batch(int cls, const TamArgs* items, const int64_t* prefix, int n,
                            int64_t blocks, size_t lds, hipStream_t s);
// items: device StageArgs[n], one workgroup each
hipError_t launch_stage_reduce_batch(const StageArgs* items, int n, hipStream_t s);

struct RankArgs {
  const uint64_t* best;      // per rank
  const int32_t* order;      // hypothesis per rank
  const double* smad;        // per hypothesis
};
// keys[prefix[r] + i] for ranks i < prefix[r + 1] - prefix[r] of request r
hipError_t launch_rank_keys_batch(const RankArgs* reqs, const int64_t* prefix, int n,
                                  int64_t total, uint64_t* keys, hipStream_t s);
// rows[row_prefix[r] + i] from sorted[key_prefix[r] + i]
hipError_t launch_rank_gather_batch(const RankArgs* reqs, const int64_t* row_prefix,
                                    const int64_t* key_prefix, int n, int64_t total,
                                    const uint64_t* sorted, PoseRow* rows, hipStream_t s);

}  // namespace reloc
