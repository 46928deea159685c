// Declarations of the map-residency and ray-cast kernels (k_map.hip,
// k_raycast.hip) shared with the host runtime.
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

}  // namespace reloc
