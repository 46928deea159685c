// Internal declarations shared by the host runtime and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace reloc {

// ---- map residency -------------------------------------------------------
// Bit-packed occupancy: one uint64 per 8x8-cell tile, tiles row-major
// (tpr tiles per row); bit ((y & 7) << 3) | (x & 7) of tile (x >> 3, y >> 3).
hipError_t launch_bitpack(const int8_t* occ, int W, int H, int thr, uint64_t* bits,
                          int tpr, int tph, hipStream_t s);
// Exact squared EDT in cells; g is int32 scratch of W*H.
hipError_t launch_edt(const int8_t* occ, int W, int H, int thr, int32_t* g, uint32_t* k,
                      hipStream_t s);

// ---- ray cast + SMAD (fused) --------------------------------------------
struct RayArgs {
  const uint64_t* bits;
  const uint16_t* walk;      // [4][H][W] walk words (see launch_walkmap), or null
  uint32_t walk_bytes;
  const int4* dir_i;         // [Ns] (|U_major|, |U_minor|, code, bits of 1/(256 |U_minor|));
                             // code bit 0 x major, bit 1 U_major < 0, bit 2 U_minor < 0
  const float4* dir_f;       // [Ns] (f, r, kappa_major, kappa_minor) per direction
  int variant;               // 0: bit tiles; 1-4: distance skipping with wavefront
                             // ray refill once 1 / 8 / 16 / 32 lanes are idle
  int W, H, tpr;
  const int32_t* hyp_xy;     // [n_hyp][2]
  int n_hyp;
  const int2* dirs;          // [Ns] ray directions (Q20 integer vectors)
  const float2* kap;         // [Ns] metres per Q8 unit along x / y
  int Ns;
  float rmax;                // fl32(range_max)
  int rcells;                // Chebyshev cut-off (result neutral)
  const int2* runs;          // [n_runs] (start index u, length L) of FoV runs
  int n_runs;
  int nfov;                  // N_FoV
  double zbar;               // measured mean (eq. 16)
  int n_shifts, n_enum;
  double* smad;              // [n_hyp]
  int32_t* argm;             // [n_hyp]
  uint64_t* keys;            // [n_hyp] sort key = bits of SMAD
  int32_t* vals;             // [n_hyp] hypothesis index
  float* zbuf;                // [n_hyp][Ns] synthetic ranges (ray cast -> SMAD)
  const int32_t* perm;       // [n_hyp] casting order (Morton order of the cells), or null
  uint64_t* best0;           // SMAD kernel: per-rank best to clear ([n_hyp]), or null
  int chunk;                 // skip variant: rays owned by one wavefront
  int32_t* dbg_hit;          // optional [n_hyp][Ns]
  int32_t* dbg_steps;        // optional [n_hyp][Ns] traversal iterations per ray
  // coarse metric that orders the hypotheses: 0 SMAD by prefix sums
  // (eq. 17-20, smad_kernel); 1 SMAD by direct sums and 2 CAER (eq. 21),
  // both by coarse_direct_kernel; 3 none (zero keys: the set's own order)
  int coarse;
  const double* fov_z;       // [nfov] measured z' of each FoV beam in beam order (0 invalid)
  const int32_t* fov_j;      // [nfov] panoramic index of each FoV beam
};
hipError_t launch_raycast(const RayArgs& a, hipStream_t s);   // ranges into zbuf
hipError_t launch_smad(const RayArgs& a, hipStream_t s);      // zbuf -> smad, argm, keys
// The coarse metric a.coarse (prefix-sum SMAD, direct-sum SMAD, CAER or
// none) into smad, argm, keys, vals (and best0 cleared); none needs no ranges.
hipError_t launch_coarse(const RayArgs& a, hipStream_t s);
// Fused ray cast + SMAD (coarse metric 0, maps with walk words): one
// workgroup of nw wavefronts (1, 2 or 4) per hypothesis casts its Ns rays
// (lanes refilled once `refill` of a wavefront's lanes, 8, 16 or 32, are
// idle) and forms its SMAD on chip: smad, argm, keys, vals (and best0
// cleared); zbuf / dbg_hit / dbg_steps are written only when non-null.
// Dynamic LDS of a non-panoramic scan: Z[Ns] FP32 (padded to 8 bytes) and
// nw * 64 FP64 block prefixes; a panoramic scan needs none.
__host__ __device__ inline size_t fused_lds_bytes(int Ns, int nw) {
  return (((size_t)Ns * 4 + 7) & ~(size_t)7) + (size_t)nw * 64 * 8;
}
hipError_t launch_raycast_smad_fused(const RayArgs& a, int nw, int refill, hipStream_t s);
// Several requests: request r owns workgroups [prefix[r], prefix[r + 1]),
// one per hypothesis, refill 16; lds = fused_lds_bytes of the largest Ns
// among the non-panoramic requests (0 when all are panoramic).
hipError_t launch_raycast_smad_fused_batch(const RayArgs* reqs, const int64_t* prefix, int n,
                                           int64_t blocks, int nw, size_t lds, hipStream_t s);
// Walk words from the squared EDT: four row-major planes, one per major
// direction of travel (+x, -x, +y, -y). A word is 0 for an occupied cell,
// else s | run << 8 with s = 1 + free-space radius byte and run = free
// cells that follow in the plane's direction inside the map (at most 255).
constexpr size_t kWalkMaxCells = (size_t)1 << 28;
hipError_t launch_walkmap(const uint32_t* k, int W, int H, uint16_t* out, hipStream_t s);

// ---- sorting (hipCUB radix sort) -----------------------------------------
hipError_t sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                              uint64_t* kout, const int32_t* vin, int32_t* vout, int n,
                              hipStream_t s);
hipError_t sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                         int n, hipStream_t s);
// Stable sort of (key, input position) for n <= kSmallSortMax in two
// launches; ktmp / vtmp are scratch of n entries. vout receives input
// positions (the value of key i is i); kout (sorted keys) may be null.
constexpr int kSmallSortMax = 65536;
hipError_t small_sort_pairs_u64(const uint64_t* kin, uint64_t* ktmp, int32_t* vtmp,
                                uint64_t* kout, int32_t* vout, int n, hipStream_t s);
// stable segmented sorts; offsets: device int64[nseg + 1]
hipError_t seg_sort_pairs_u64_i32(void* tmp, size_t* tmp_bytes, const uint64_t* kin,
                                  uint64_t* kout, const int32_t* vin, int32_t* vout, int64_t n,
                                  int nseg, const int64_t* offsets, hipStream_t s);
hipError_t seg_sort_keys_u64(void* tmp, size_t* tmp_bytes, const uint64_t* kin, uint64_t* kout,
                             int64_t n, int nseg, const int64_t* offsets, hipStream_t s);

// ---- TAM -----------------------------------------------------------------
struct TamArgs {
  const uint32_t* kmap;
  int W, H;
  const int32_t* hyp_xy;
  const int32_t* order;      // hypothesis index per SMAD rank
  int r0, nb;                // ranks [r0, r0 + nb)
  const int2* beams;         // [nvp] ((b * j_v) mod Ng, range in Q8 cells), padded
                             // with (0, 0) to nvp = tam_beams_padded(nv)
  int nv;
  const int2* dirs;          // [2 Ng] direction table, stored twice
  int Ng, o, Nt;             // o = Ng / Nt
  const int32_t* lut;        // [n_keys] likelihood per selection key, Q26
  int kcap, key_off, keybits;
  int kmid;
  double res, d_max;
  int fine;                  // score: 0 T (eq. 31), 1 T_mean (eq. 34), 2 baseline (eq. 33),
                             // 3 LF (eq. 32)
  float* T_out;              // optional [nb][Nt]
  uint64_t* best;            // [>= r0 + nb] packed (score_key(T), ~k) per rank
};
hipError_t launch_tam(const TamArgs& a, hipStream_t s);
// Beam-table length the TAM kernels read: nv rounded up to 512, a whole
// gather batch of every kernel class (64 lanes x up to 8 keys).
constexpr int kTamBeamPad = 512;
__host__ __device__ inline int tam_beams_padded(int nv) {
  return (nv + kTamBeamPad - 1) / kTamBeamPad * kTamBeamPad;
}

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
constexpr int kTamClasses = 20;
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
