// TAM over enumerated orientations (eq. 22-31), per-hypothesis argmax,
// batch reduction with the early-termination test, and final ranking.
//
// Work layout: one workgroup (4 wavefronts) per (hypothesis, tile of 16
// orientations); each wavefront evaluates one (p, theta_k) at a time with the
// valid beams spread over its 64 lanes, R per lane.
//
// A hypothesis sits at its cell centre, so the endpoint cell of beam v at
// heading g is the hypothesis cell plus an offset that depends on (g, v)
// only: e = (ix, iy) + (dx, dy), dx = floor((2^27 + zq U_x) / 2^28) (eq. 22's
// projection in exact fixed point). The request's offset table holds every
// (g, v) offset, so a lookup is one coalesced offset load (four beams per
// lane at a time), two clamps and one 2-byte gather from the map's 16-bit
// TAM plane: 2 k per cell in strips of 8 columns, so a 128-byte line holds
// 8 x 8 cells (an endpoint run along a wall in any direction stays within
// few lines) and the index is one multiply-add, with a sentinel column and
// row that endpoints off the map (and padded beam slots) are clamped onto,
// so no lookup needs a mask; sqrt(k) in Q16 is computed. Cells 128 or more
// cells from any obstacle hold an escape instead (2 k does not fit); a
// wavefront that meets one reads those slots again from the 32-bit plane.
// The likelihood l(k) of eq. 23 is monotone non-increasing in k, so the
// top-k_mid selection of eq. 24-27 is a selection of the k_mid smallest
// integer keys: key = 2 * min(k, kcap) for in-map endpoints and a
// host-chosen odd key for off-map ones (d = d_max). kcap is where l(k) has
// converged to within 1e-10 of its limit. A slot holds its raw plane value
// (times 4, a table byte offset) as its key: every candidate threshold is at
// most 2 kcap, so the cap needs no instruction, and the sentinel (2^32 - 1
// sign-extended) lies above every candidate; the wavefront's sentinel count
// then moves the off-map slots to key_off and drops the padded ones, in
// closed form, in every count and sum. The threshold key comes from a
// search whose counts are wavefront ballots; the likelihood sums are exact
// integers (l - lmin in Q26 fixed point from a host table, lmin added back
// per selected beam), k is summed exactly and sqrt(k) in FP32 within a lane
// then exactly across lanes, so the result does not depend on lane order or
// co-scheduling.
// The median of eq. 27 is always the top-k_mid mean (top-k means are
// non-increasing in k and k_low <= k_mid <= k_full).
//
// The score may also be one of the ablation metrics of Sec. IV (Case 3):
// T_mean (eq. 34) from the same sums, or baseline (eq. 33) and LF (eq. 32)
// from the sum of l over every valid beam (no selection). Scores are packed
// with score_key, which orders negative LF values correctly.
#include <cmath>

#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int TB = 256;
constexpr int NW = TB / 64;
constexpr int THETA_PER_BLOCK = 16;

// The likelihood table (2^keybits entries) through a buffer resource, for
// the 16-bit key class that does not keep it in LDS.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lut_rsrc(const TamArgs& a) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)a.lut, (short)0, 4 * (1 << a.keybits),
                                           0x00020000);
}

// Sum over the 64 lanes of a wavefront (every lane active), returned to
// every lane. Quad permutes and row rotations leave each lane of a 16-lane
// row with the row's sum; two row broadcasts then carry rows 0-2 into lane
// 63, which is read back. The moves are DPP operands of VALU instructions:
// no LDS round trips. Integer sums, so the order of the additions does not
// change the result. The 64-bit sum moves each half on its own and leaves
// lanes with no source lane (rows 0-1 under the broadcasts) unspecified,
// which lane 63 never reads from.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xf, 0xf, false);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
  v += dpp64<0xb1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp64<0x4e>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp64<0x124>(v);   // row_ror:4
  v += dpp64<0x128>(v);   // row_ror:8
  v += dpp64<0x142>(v);   // row_bcast:15
  v += dpp64<0x143>(v);   // row_bcast:31
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// The same over 32-bit values: each move is the DPP operand of the add.
// Integer sums do not depend on the order of the additions; the FP32 sum
// takes its additions in one fixed order, so it is the same on every run.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
  v += dpp32<0xb1>(v);
  v += dpp32<0x4e>(v);
  v += dpp32<0x124>(v);
  v += dpp32<0x128>(v);
  v += dpp32<0x142>(v);
  v += dpp32<0x143>(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ float wave_sumf(float v) {
  v += __uint_as_float(dpp32<0xb1>(__float_as_uint(v)));
  v += __uint_as_float(dpp32<0x4e>(__float_as_uint(v)));
  v += __uint_as_float(dpp32<0x124>(__float_as_uint(v)));
  v += __uint_as_float(dpp32<0x128>(__float_as_uint(v)));
  v += __uint_as_float(dpp32<0x142>(__float_as_uint(v)));
  v += __uint_as_float(dpp32<0x143>(__float_as_uint(v)));
  return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(v), 63));
}

// A 64-bit running sum of 32-bit values kept as two words: an add with carry
// out and an add of the carry, so no zeroed upper word is held beside each
// value.
struct Sum64 {
  uint32_t lo = 0, hi = 0;
  __device__ __forceinline__ void add(uint32_t v) {
    uint32_t c;
    lo = __builtin_addc(lo, v, 0u, &c);
    hi += c;
  }
  __device__ __forceinline__ uint64_t get() const { return ((uint64_t)hi << 32) | lo; }
};

// sqrt(|v|) in FP32 for a plane entry read sign-extended: sqrt(2 k) for an
// in-map cell, 1 for the sentinel (-1), sqrt 2 for the escape (-2). The
// absolute value is a source modifier of the square root: one conversion
// and one square root per slot.
__device__ __forceinline__ float sqrt_abs(uint32_t v) {
  return __fsqrt_rn(fabsf((float)(int32_t)v));
}

// The 16 poses of one workgroup come from a pose source: has(j) tells
// whether pose j of the tile is evaluated, pose(j) gives its cell and
// heading index g on the Ng grid (false when it is not evaluated), tie(j)
// the low word that orders equal T in the atomic max (larger wins),
// record(j, T) an optional per-pose output, and dst the packed (T bits,
// tie) word the tile's best is folded into.
//
// Orientation tile: hypothesis cell (ix, iy), orientations [k0, k0 + 16) of
// eq. 22, heading index o k on the Ng grid; ties go to the smaller k.
struct ThetaSrc {
  static constexpr bool kPrefix = true;   // the evaluated poses are a prefix
  static constexpr bool kPublish = true;  // fold the tile's best into *dst
  int ix, iy;
  int k0, Nt, o, Ng;
  float* T_row;           // optional [Nt]
  uint64_t* dst;
  __device__ __forceinline__ bool pose(int j, int& x, int& y, int& g) const {
    const int k = k0 + j;
    if (k >= Nt) return false;
    x = ix;
    y = iy;
    g = o * k;            // o = floor(Ng / Nt) and k < Nt: below Ng, no reduction
    return true;
  }
  __device__ __forceinline__ bool has(int j) const { return k0 + j < Nt; }
  __device__ __forceinline__ uint32_t tie(int j) const { return 0xFFFFFFFFu - (uint32_t)(k0 + j); }
  __device__ __forceinline__ void record(int j, float T) const {
    if (T_row) T_row[k0 + j] = T;
  }
};

// Refinement lattice tile: points [q0, q0 + 16) of the lattice around the
// pose (cell (ix, iy), heading index g0): q = ((dg + s) w + dy + h) w + dx + h,
// w = 2h + 1. Cells other than the pose's own that lie off the map or are
// occupied (k == 0) are not evaluated. Ties go to the pose itself (q = qc),
// then to the smaller q.
struct LatticeSrc {
  static constexpr bool kPrefix = false;
  static constexpr bool kPublish = true;
  int ix, iy, g0, h, s, w, L, q0, W, H, Ng;
  const uint32_t* kmap;
  uint64_t* dst;
  __device__ __forceinline__ bool has(int j) const {
    const int q = q0 + j;
    if (q >= L) return false;
    const int t = q / w;
    const int dx = q - t * w - h, dy = t % w - h;
    if (dx == 0 && dy == 0) return true;
    const int cx = ix + dx, cy = iy + dy;
    if ((uint32_t)cx >= (uint32_t)W || (uint32_t)cy >= (uint32_t)H) return false;
    return kmap[(size_t)cy * (size_t)W + (size_t)cx] != 0u;
  }
  __device__ __forceinline__ bool pose(int j, int& x, int& y, int& g) const {
    if (!has(j)) return false;
    const int q = q0 + j, t = q / w;
    const int dx = q - t * w - h, dy = t % w - h, dg = t / w - s;
    x = ix + dx;
    y = iy + dy;
    const int gg = (g0 + dg) % Ng;
    g = gg < 0 ? gg + Ng : gg;
    return true;
  }
  __device__ __forceinline__ uint32_t tie(int j) const {
    const int q = q0 + j, qc = (s * w + h) * w + h;
    return 0xFFFFFFFFu - (uint32_t)(q == qc ? 0 : q + 1);
  }
  __device__ __forceinline__ void record(int, float) const {}
};

// Explicit poses: poses [q0, q0 + 16) of a list of n (cell, heading index
// on the Ng grid); each score is written out, nothing is reduced.
struct PoseListSrc {
  static constexpr bool kPrefix = true;
  static constexpr bool kPublish = false;
  const int32_t* xy;
  const int32_t* g;
  int q0, n;
  float* out;
  uint64_t* dst;
  __device__ __forceinline__ bool has(int j) const { return q0 + j < n; }
  __device__ __forceinline__ bool pose(int j, int& x, int& y, int& gg) const {
    const int q = q0 + j;
    if (q >= n) return false;
    x = xy[2 * q];
    y = xy[2 * q + 1];
    gg = g[q];
    return true;
  }
  __device__ __forceinline__ uint32_t tie(int) const { return 0u; }
  __device__ __forceinline__ void record(int j, float T) const { out[q0 + j] = T; }
};

// LDS of a tile: the likelihood table (2^12 keys) for the 12-bit key class;
// the 16-bit class reads it from memory.
__host__ __device__ constexpr size_t tam_lut_lds(int kb) {
  return kb <= 12 ? (size_t)(1 << 12) * 4 : 0;
}

// One workgroup's work: the 16 poses of a tile; wavefront w takes poses
// w + 4 g, g = 0..3.
//
// Per pose the R beam slots of a lane come SB at a time: one 16-byte load
// of four offsets per four slots, then SB plane gathers, all in flight
// before any is used. The per-pose sums (wavefront-uniform) go to LDS as
// each pose ends; the FP64 tail (eq. 27-31) runs once per workgroup, for the
// 16 poses in lanes 0..15 of wavefront 0, and one atomic max per workgroup
// publishes the best (T, tie). The other wavefronts end there: every
// caller ends with the tile.
template <int R, int KB, bool FULL, class Src>
__device__ __forceinline__ void tam_tile(const TamArgs& a, const Src& src, int32_t* smem) {
  // beam slots per lane in flight together: every slot up to 12 keys per
  // lane, then batches of 12 or 8 (register pressure; at 24 keys, batches
  // of 12 take 71 VGPRs against 78 for batches of 8, and TAM at stress
  // 1.77 -> 1.67 ms)
  constexpr int SB = R <= 12 ? R : (R % 12 == 0 ? 12 : 8);
  constexpr int G = THETA_PER_BLOCK / NW;
  constexpr bool kLdsLut = KB <= 12;
  static_assert(R % SB == 0, "whole gather batches");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nv = a.nv;
  const __amdgpu_buffer_rsrc_t lut = lut_rsrc(a);
  const uint32_t kcap2 = 2u * (uint32_t)a.kcap, key_off = (uint32_t)a.key_off;
  if constexpr (kLdsLut) {
    // the entries keys can reach, 0 .. 2 kcap (below 4096 here), four per
    // 16-byte load: at most four loads per lane, all in flight before the
    // first store
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const int n4 = (int)(kcap2 >> 2) + 1;
    u32x4 q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (tid + j * TB < n4) q[j] = __builtin_amdgcn_raw_buffer_load_b128(lut, (tid + j * TB) << 4, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (tid + j * TB < n4) reinterpret_cast<u32x4*>(smem)[tid + j * TB] = q[j];
    __syncthreads();
  }
  // the table entry at byte offset k4 = 4 key (keys are held as 4 key, so a
  // lookup needs no shift)
  auto ell4 = [&](uint32_t k4) -> int32_t {
    if constexpr (kLdsLut) return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(smem) + k4);
    else return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(lut, (int)k4, 0, 0);
  };
  auto ell = [&](uint32_t key) -> int32_t { return ell4(key << 2); };
  const char* __restrict__ plane = reinterpret_cast<const char*>(a.plane);
  const char* __restrict__ plane16 = reinterpret_cast<const char*>(a.plane16);
  const uint32_t Wc = (uint32_t)a.W, Hc = (uint32_t)a.H, rows1 = tam_plane_rows(a.H) - 1u;
  // plane entry of the endpoint at offset word o (dx low, dy high) from the
  // pose's cell; off the map (either side) clamps onto the sentinel column
  // or row
  auto entry_index = [&](uint32_t o, int px, int py) -> uint32_t {
    const uint32_t ex = (uint32_t)px + (uint32_t)(int32_t)(int16_t)(o & 0xFFFFu);
    const uint32_t ey = (uint32_t)py + (uint32_t)((int32_t)o >> 16);
    return tam_plane_index(min(ex, Wc), min(ey, Hc), rows1);
  };
  // the escape's share of a square-root sum (the sentinel's is 1), by the
  // same instructions as a slot's (the empty asm keeps the compiler from
  // folding it)
  uint32_t e_raw = 0xFFFFFFFEu;
  asm volatile("" : "+v"(e_raw));
  const float sq_esc = sqrt_abs(e_raw);

  // per-pose results (wavefront-uniform) go to LDS as each pose ends, for
  // the FP64 tail
  __shared__ int64_t t_sl[THETA_PER_BLOCK];
  __shared__ uint64_t t_sumk[THETA_PER_BLOCK];
  __shared__ double t_sq[THETA_PER_BLOCK];
  __shared__ int t_noff[THETA_PER_BLOCK];

  uint32_t t_prev = kcap2;              // the selection's first guess
  for (int g = 0; g < G; ++g) {
    int px, py, pg;
    if (!src.pose(wv + NW * g, px, py, pg)) {           // wavefront-uniform
      if (Src::kPrefix) break;
      continue;
    }
    const uint4* __restrict__ orow =
        reinterpret_cast<const uint4*>(a.off + (size_t)pg * (size_t)a.off_stride) + lane;
    // raw keys: 4 x the 16-bit plane value read sign-extended, so the
    // sentinel (2^32 - 1) and the escape (2^32 - 2) wrap to near 2^32,
    // above every candidate (the counts and sums below move the off-map
    // slots to key_off and drop the padded ones; the rare far ones are fixed
    // from the 32-bit plane)
    uint32_t keys[R];
    // per lane: the sum of the raw values (in-map 2 k below 2^15, -1 per
    // sentinel, -2 per escape: exact in 32 bits), the counts of sentinels
    // (low half) and of sentinels and escapes (high half), and the FP32 sum
    // of sqrt(|raw|)
    uint32_t sk = 0, cnt = 0;
    float sq = 0.0f;
#pragma unroll
    for (int b = 0; b < R / SB; ++b) {
      uint32_t o[SB];
#pragma unroll
      for (int q = 0; q < SB / 4; ++q) {
        const uint4 o4 = orow[64 * (b * (SB / 4) + q)];
        o[4 * q] = o4.x;
        o[4 * q + 1] = o4.y;
        o[4 * q + 2] = o4.z;
        o[4 * q + 3] = o4.w;
      }
      uint32_t idx[SB];
#pragma unroll
      for (int s2 = 0; s2 < SB; ++s2) idx[s2] = entry_index(o[s2], px, py);
      // 32-bit byte offsets from the plane base (below 2^31)
      uint32_t v[SB];
#pragma unroll
      for (int s2 = 0; s2 < SB; ++s2)
        v[s2] = (uint32_t)(int32_t)*reinterpret_cast<const int16_t*>(plane16 + (idx[s2] << 1));
#pragma unroll
      for (int s2 = 0; s2 < SB; ++s2) {
        const uint32_t k2 = v[s2];
        keys[SB * b + s2] = k2 << 2;    // the sentinel and the escape wrap far above 8 kcap
        sk += k2;
        cnt += k2 & 0x10001u;          // -1: both bits; -2: bit 16; 2 k < 2^15: neither
        sq += sqrt_abs(k2);            // no branch: the shares of -1 and -2 come out below
      }
      // one gather batch at a time: without this the scheduler issues every
      // batch's loads together and holds them all
      __builtin_amdgcn_sched_barrier(0);
    }
    // wavefront totals first: the selection needs the off-map count
    cnt = wave_sum32(cnt);
    const int nsent = (int)(cnt & 0xFFFFu);        // sentinel slots: off-map beams and padding
    const int nesc = (int)(cnt >> 16) - nsent;     // escape slots
    // sum of 2 k over the in-map slots that are not escapes
    uint64_t sumk = (uint64_t)((int64_t)(int32_t)wave_sum32(sk) + nsent + 2 * nesc);
    // each lane's FP32 sum of sqrt(|raw|) (at most 64 x 182) in Q12, then
    // an exact wavefront sum (below 2^32)
    const uint32_t sq12 = wave_sum32((uint32_t)(sq * 4096.0f));
    float sq_far = 0.0f;                   // sqrt(2 k) of the escape slots
    if (nesc > 0) {                        // wavefront-uniform; rare
      // cells 128 or more cells from any obstacle: their 2 k from the 32-bit
      // plane (in-map entries of 2^15 or more; its sentinel is odd) gives
      // their keys and their shares of the sums
      Sum64 ek;
      float es = 0.0f;
#pragma unroll
      for (int m = 0; m < R / 4; ++m) {
        const uint4 o4 = orow[64 * m];
        const uint32_t o[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t w =
              *reinterpret_cast<const uint32_t*>(plane + (entry_index(o[q], px, py) << 2));
          const bool far = w >= (1u << 15) && !(w & 1u);
          ek.add(far ? w : 0u);
          es += far ? __fsqrt_rn((float)w) : 0.0f;
          if (far) keys[4 * m + q] = min(w, kcap2) << 2;
        }
        __builtin_amdgcn_sched_barrier(0);   // four gathers in flight at a time
      }
      sumk += wave_sum64(ek.get());
      sq_far = wave_sumf(es);
    }
    const int nin = 64 * R - nsent;
    const int noff = nv - nin;
    // the selection over the true keys (in-map keys, noff copies of key_off):
    // a count or sum over raw keys below c, plus the off-map beams when
    // key_off < c
    int64_t sl = 0;
    if constexpr (!FULL) {
      // TAM and T_mean: the top-k_mid sum of eq. 24-27. The threshold t,
      // the k_mid-th smallest key, is the largest t with fewer than k_mid
      // keys below it; counts come from wavefront ballots over the raw keys,
      // corrected as above. Candidates are multiples of 2^sh (when key_off
      // is even every key is). The previous pose's t (2 kcap for the first)
      // is tried first: nearby orientations and lattice poses often share
      // t, and 2 kcap is where every far miss sits. One or two rounds settle
      // it; otherwise a binary search runs on the side where t lies. The
      // count below t is that of the last candidate taken (0 if none).
      // Every candidate is at most 2 kcap, so raw keys (4 x the plane value,
      // no cap) count as capped ones would and the sentinel slots (2^34 - 4
      // wrapped) never count.
      auto cnt = [&](uint32_t c) -> int {
        int n = key_off < c ? noff : 0;
        const uint32_t c4 = c << 2;
#pragma unroll
        for (int i = 0; i < R; ++i) n += __popcll(__ballot(keys[i] < c4));
        return n;
      };
      const int sh = (int)(key_off & 1u) ^ 1;
      const uint32_t umax = kcap2 >> sh;
      const uint32_t ug = t_prev >> sh;
      uint32_t lo = 0, hi = umax;
      int below = 0;
      const int cg = cnt(ug << sh);
      if (cg >= a.kmid) {
        hi = ug - 1;                         // count(< 0) = 0 < k_mid: ug >= 1
      } else {
        lo = ug;
        below = cg;
        if (ug < umax) {
          const int c2 = cnt((ug + 1) << sh);
          if (c2 >= a.kmid) {
            hi = ug;
          } else {
            lo = ug + 1;
            below = c2;
          }
        }
      }
      while (lo < hi) {                      // wavefront-uniform
        const uint32_t mid = (lo + hi + 1) >> 1;
        const int c = cnt(mid << sh);
        if (c < a.kmid) {
          lo = mid;
          below = c;
        } else {
          hi = mid - 1;
        }
      }
      const uint32_t tkey = lo << sh;
      t_prev = tkey;
      // the sum of l over the raw keys below t, as the sum of l(min(key, t))
      // over every raw key less l(t) once per raw key at or above t (one
      // min per key, no compare and select); table entries are l - lmin >= 0,
      // below 2^31: pairs add in 32 bits
#pragma unroll
      for (int i = 0; i < R; i += 2) {
        const uint32_t l0 = (uint32_t)ell4(min(keys[i], tkey << 2));
        const uint32_t l1 = (uint32_t)ell4(min(keys[i + 1], tkey << 2));
        sl += (int64_t)(uint64_t)(l0 + l1);
      }
      const int64_t lt = ell(tkey);
      const int below_raw = below - (key_off < tkey ? noff : 0);
      sl = (int64_t)wave_sum64((uint64_t)sl) - (int64_t)(64 * R - below_raw) * lt;
      if (key_off < tkey) sl += (int64_t)noff * (int64_t)ell(key_off);
      sl += (int64_t)(a.kmid - below) * lt;
      sl += (int64_t)a.kmid * (int64_t)a.lmin;
    } else {
      // baseline and LF: the sum of l over every valid beam (eq. 32)
#pragma unroll
      for (int i = 0; i < R; i += 2)
        sl += (int64_t)(uint64_t)((uint32_t)ell4(min(keys[i], kcap2 << 2)) +
                                  (uint32_t)ell4(min(keys[i + 1], kcap2 << 2)));
      sl = (int64_t)wave_sum64((uint64_t)sl);
      sl += (int64_t)noff * (int64_t)ell(key_off) - (int64_t)nsent * (int64_t)ell(kcap2);
      sl += (int64_t)nv * (int64_t)a.lmin;
    }
    if (lane == 0) {
      const int jj = wv + NW * g;
      t_sl[jj] = sl;
      t_sumk[jj] = sumk >> 1;           // the plane holds 2 k
      // sum of sqrt(2 k) over the in-map slots: less 1 per sentinel and
      // sqrt 2 per escape, plus the escapes' own
      t_sq[jj] = (double)sq12 * (1.0 / 4096.0) - (double)nsent - (double)nesc * (double)sq_esc +
                 (double)sq_far;
      t_noff[jj] = noff;
    }
  }
  // wavefront 0 then runs the FP64 tail once, one pose per lane
  __syncthreads();
  if (wv != 0) return;                  // the caller's work ends with the tile
  const int j = lane;
  const bool mine = lane < THETA_PER_BLOCK && src.has(j);
  uint64_t packed = 0;
  if (mine) {
    const int64_t q_sl = t_sl[j];
    const uint64_t q_sumk = t_sumk[j];
    const double q_sq = t_sq[j] * 0.70710678118654752;   // sum of sqrt(k)
    const int q_noff = t_noff[j];
    const double nvd = (double)nv;
    const double sum_d = a.res * q_sq + (double)q_noff * a.d_max;
    const double sum_d2 = a.res * a.res * (double)q_sumk + (double)q_noff * a.d_max * a.d_max;
    const double dbar = sum_d / nvd;
    double var = sum_d2 / nvd - dbar * dbar;
    if (var < 0.0) var = 0.0;
    const double dmin = 0.5 * a.res;
    const double dt = fmin(fmax(dbar, dmin), a.d_max);
    const double sd = 1.0 - (dt - dmin) / (a.d_max - dmin);
    double v;
    if constexpr (!FULL) {
      const double Lbar = (double)q_sl / (67108864.0 * (double)a.kmid);
      const double Pl = exp(Lbar);
      const double c = exp(-0.5 * var);
      v = a.fine == 0 ? cbrt(Pl * sd * c) : (Pl + sd + c) / 3.0;   // eq. 31 / eq. 34
    } else {
      const double lf = (double)q_sl / 67108864.0;                 // eq. 32
      v = a.fine == 3 ? lf : sqrt(exp(lf / nvd) * sd);               // eq. 33
    }
    const float T = (float)v;
    src.record(j, T);
    packed = ((uint64_t)score_key(T) << 32) | (uint64_t)src.tie(j);
  }
  if constexpr (Src::kPublish) {
    for (int off = THETA_PER_BLOCK / 2; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(packed, off, 64);
      packed = o > packed ? o : packed;
    }
    if (lane == 0 && packed) atomicMax((unsigned long long*)src.dst, (unsigned long long)packed);
  }
}

// Orientation tile kb of rank a.r0 + i.
template <int R, int KB, bool FULL>
__device__ __forceinline__ void tam_block(const TamArgs& a, int i, int kb, int32_t* smem) {
  const int r = a.r0 + i;
  const int hyp = a.order[r];
  ThetaSrc src;
  src.ix = a.hyp_xy[2 * hyp];
  src.iy = a.hyp_xy[2 * hyp + 1];
  src.k0 = kb * THETA_PER_BLOCK;
  src.Nt = a.Nt;
  src.o = a.o;
  src.Ng = a.Ng;
  src.T_row = a.T_out ? a.T_out + (size_t)i * a.Nt : nullptr;
  src.dst = &a.best[r];
  tam_tile<R, KB, FULL>(a, src, smem);
}

// Wavefronts per SIMD the register allocation of a TAM launch aims for:
// 8 (at most 64 VGPRs) up to 24 keys per lane, which fit it without spills
// (and schedule better for it: TAM at the stress workload 1.55 -> 1.49 ms);
// no target above.
constexpr int tam_waves(int R) { return R <= 24 ? 8 : 1; }

// Workgroup b of an n-workgroup grid runs on XCD b % 8 (round-robin
// dispatch); the returned index gives every XCD one contiguous slice of
// [0, n), so the orientation tiles of one hypothesis (whose endpoints touch
// nearly the same EDT cells) share one XCD's L2.
__device__ __forceinline__ int xcd_slice(int b, int n) {
  const int x = b & 7, i = b >> 3;
  const int q = n >> 3, rem = n & 7;
  return x * q + min(x, rem) + i;
}

template <int R, int KB, bool FULL>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(tam_waves(R))))
void tam_kernel(TamArgs a) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  const int ntb = tam_tiles_per_rank(a);
  const int L = xcd_slice(blockIdx.x, gridDim.x);
  tam_block<R, KB, FULL>(a, L / ntb, L % ntb, smem);
}

// Local refinement, lattice tiles: workgroup b covers slot b / tiles and
// lattice points [16 (b % tiles), + 16) around that slot's rank (its cell
// and heading o k*, k* read from the rank's packed TAM best).
template <int R, int KB, bool FULL>
__global__ __launch_bounds__(TB) void refine_kernel(RefineArgs a) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  const int tiles = (a.L + THETA_PER_BLOCK - 1) / THETA_PER_BLOCK;
  const int b = xcd_slice(blockIdx.x, gridDim.x);
  const int slot = b / tiles, tile = b - slot * tiles;
  const int r = a.sel[slot];
  if (r < 0) return;                           // workgroup-uniform
  const TamArgs& t = a.t;
  const int hyp = t.order[r];
  const int kstar = (int)(0xFFFFFFFFu - (uint32_t)(t.best[r] & 0xFFFFFFFFu));
  LatticeSrc src;
  src.ix = t.hyp_xy[2 * hyp];
  src.iy = t.hyp_xy[2 * hyp + 1];
  src.g0 = (int)(((int64_t)t.o * kstar) % t.Ng);
  src.h = a.h;
  src.s = a.s;
  src.w = 2 * a.h + 1;
  src.L = a.L;
  src.q0 = tile * THETA_PER_BLOCK;
  src.W = t.W;
  src.H = t.H;
  src.Ng = t.Ng;
  src.kmap = t.kmap;
  src.dst = &a.rbest[slot];
  tam_tile<R, KB, FULL>(t, src, smem);
}

// Refinement selection, one workgroup per stage b: the kr best ranks of
// [r0 + b K, min(r0 + (b + 1) K, n)) by (T desc, rank asc), found as kr
// successive maxima of the unique key (T bits, ~rank) below the previous
// one; slot b kr + j gets the j-th (or -1) and its lattice best is cleared.
__global__ __launch_bounds__(TB) void refine_select_kernel(const uint64_t* __restrict__ best,
                                                           int r0, int K, int n, int kr,
                                                           int32_t* __restrict__ sel,
                                                           uint64_t* __restrict__ rbest) {
  __shared__ unsigned long long red[NW];
  __shared__ unsigned long long prev_s;
  const int lo = r0 + (int)blockIdx.x * K, hi = min(lo + K, n);
  unsigned long long prev = ~0ull;
  for (int j = 0; j < kr; ++j) {
    unsigned long long m = 0;
    for (int r = lo + (int)threadIdx.x; r < hi; r += TB) {
      const unsigned long long key =
          ((best[r] >> 32) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)r);
      if (key < prev && key > m) m = key;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(m, off, 64);
      if (o > m) m = o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < NW; ++q)
        if (red[q] > m) m = red[q];
      const int slot = (int)blockIdx.x * kr + j;
      sel[slot] = m ? (int)(0xFFFFFFFFu - (uint32_t)(m & 0xFFFFFFFFu)) : -1;
      rbest[slot] = 0;
      prev_s = m;
    }
    __syncthreads();
    prev = prev_s;
  }
}

// Folds each slot's lattice best into its rank's packed word: (T bits,
// code), code = g << 10 | (dy + 15) << 5 | (dx + 15) with bit 31 clear, so
// the ranking kernels (which report ~low) give refined poses a negative k.
__global__ void refine_commit_kernel(RefineArgs a) {
  const int slot = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (slot >= a.n_slots) return;
  const int r = a.sel[slot];
  if (r < 0) return;
  const uint64_t v = a.rbest[slot];
  if (v == 0) return;
  const uint32_t tie = 0xFFFFFFFFu - (uint32_t)(v & 0xFFFFFFFFu);
  const int w = 2 * a.h + 1, qc = (a.s * w + a.h) * w + a.h;
  const int q = tie == 0u ? qc : (int)tie - 1;
  const int t = q / w;
  const int dx = q - t * w - a.h, dy = t % w - a.h, dg = t / w - a.s;
  const int kstar = (int)(0xFFFFFFFFu - (uint32_t)(a.t.best[r] & 0xFFFFFFFFu));
  int g = (int)(((int64_t)a.t.o * kstar + dg) % a.t.Ng);
  if (g < 0) g += a.t.Ng;
  const uint32_t code = ((uint32_t)g << 10) | ((uint32_t)(dy + 15) << 5) | (uint32_t)(dx + 15);
  a.t.best[r] = (v & 0xFFFFFFFF00000000ull) | (uint64_t)code;
}

template <int R, int KB, bool FULL>
hipError_t launch_refine_t(const RefineArgs& a, hipStream_t s) {
  const int tiles = (a.L + THETA_PER_BLOCK - 1) / THETA_PER_BLOCK;
  hipLaunchKernelGGL((refine_kernel<R, KB, FULL>), dim3(tiles * a.n_slots), dim3(TB),
                     tam_lut_lds(KB), s, a);
  return hipGetLastError();
}

// Kernel class dispatch on the keys per lane of the request's beams.
#define RELOC_TAM_CLASSES(F, KB, FULL, ...)                                   \
  switch (tam_keys_per_lane(nv)) {                                           \
    case 4: return F<4, KB, FULL>(__VA_ARGS__);                              \
    case 8: return F<8, KB, FULL>(__VA_ARGS__);                              \
    case 12: return F<12, KB, FULL>(__VA_ARGS__);                            \
    case 16: return F<16, KB, FULL>(__VA_ARGS__);                            \
    case 24: return F<24, KB, FULL>(__VA_ARGS__);                            \
    case 32: return F<32, KB, FULL>(__VA_ARGS__);                            \
    case 48: return F<48, KB, FULL>(__VA_ARGS__);                            \
    case 64: return F<64, KB, FULL>(__VA_ARGS__);                            \
    default: return hipErrorInvalidValue;                                    \
  }

template <int KB, bool FULL>
hipError_t launch_refine_kb(const RefineArgs& a, hipStream_t s) {
  const int nv = a.t.nv;
  RELOC_TAM_CLASSES(launch_refine_t, KB, FULL, a, s)
}

// Scores of an explicit pose list, 16 poses per workgroup.
template <int R, int KB, bool FULL>
__global__ __launch_bounds__(TB) void pose_kernel(PoseArgs a) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  PoseListSrc src;
  src.xy = a.xy;
  src.g = a.g;
  src.q0 = (int)blockIdx.x * THETA_PER_BLOCK;
  src.n = a.n;
  src.out = a.out;
  src.dst = nullptr;
  tam_tile<R, KB, FULL>(a.t, src, smem);
}

template <int R, int KB, bool FULL>
hipError_t launch_poses_t(const PoseArgs& a, hipStream_t s) {
  const int blocks = (a.n + THETA_PER_BLOCK - 1) / THETA_PER_BLOCK;
  hipLaunchKernelGGL((pose_kernel<R, KB, FULL>), dim3(blocks), dim3(TB), tam_lut_lds(KB), s, a);
  return hipGetLastError();
}

template <int KB, bool FULL>
hipError_t launch_poses_kb(const PoseArgs& a, hipStream_t s) {
  const int nv = a.t.nv;
  RELOC_TAM_CLASSES(launch_poses_t, KB, FULL, a, s)
}

// Index of the segment holding item t: prefix[e] <= t < prefix[e + 1].
__device__ __forceinline__ int find_segment(const int64_t* prefix, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// TAM over several rank ranges (of one or several requests) in one launch:
// item e owns blocks [prefix[e], prefix[e + 1]) = nb x ceil(Nt / 16).
template <int R, int KB, bool FULL>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(tam_waves(R))))
void tam_batch_kernel(const TamArgs* __restrict__ items, const int64_t* __restrict__ prefix, int n) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  const int t = xcd_slice(blockIdx.x, gridDim.x);
  const int e = find_segment(prefix, n, t);
  const TamArgs& a = items[e];
  const int ntb = tam_tiles_per_rank(a);
  const int local = (int)(t - prefix[e]);
  tam_block<R, KB, FULL>(a, local / ntb, local % ntb, smem);
}

template <int R, int KB, bool FULL>
hipError_t launch_tam_t(const TamArgs& a, hipStream_t s) {
  const int ntb = tam_tiles_per_rank(a);
  hipLaunchKernelGGL((tam_kernel<R, KB, FULL>), dim3(ntb * a.nb), dim3(TB), tam_lut_lds(KB), s,
                     a);
  return hipGetLastError();
}

template <int KB, bool FULL>
hipError_t launch_tam_kb(const TamArgs& a, hipStream_t s) {
  const int nv = a.nv;
  RELOC_TAM_CLASSES(launch_tam_t, KB, FULL, a, s)
}


// Endpoint-offset table: one thread per (heading g, beam slot v).
__global__ void tam_offsets_kernel(const int2* __restrict__ beams, int nv,
                                   const int2* __restrict__ dirs, int Ng, int stride,
                                   uint32_t* __restrict__ off) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Ng * stride) return;
  const int g = (int)(t / stride);
  // slot p = 4 (64 b + l) + q holds beam 256 b + 64 q + l
  const int p = (int)(t - (int64_t)g * stride);
  const int v = (p & ~255) + 64 * (p & 3) + ((p & 255) >> 2);
  if (v >= nv) {
    off[t] = 0x80000000u;                      // dy = -32768: never inside a map
    return;
  }
  const int2 bz = beams[v];
  const int2 U = dirs[bz.x + g];               // the table is stored twice: no wrap
  const int64_t half = (int64_t)1 << 27;
  // ranges stay below 64 m at cells of at least 1/32 m, so an offset is at
  // most 2048 cells and 16 bits hold it; the clamp only guards the packing
  // (maps are at most 32767 cells a side, so 32767 leaves the map anyway)
  const int64_t dx = (half + (int64_t)bz.y * U.x) >> 28;
  const int64_t dy = (half + (int64_t)bz.y * U.y) >> 28;
  const int cx = (int)(dx < -32767 ? -32767 : (dx > 32767 ? 32767 : dx));
  const int cy = (int)(dy < -32767 ? -32767 : (dy > 32767 ? 32767 : dy));
  off[t] = (uint32_t)(uint16_t)(int16_t)cx | ((uint32_t)(uint16_t)(int16_t)cy << 16);
}

__device__ __forceinline__ void stage_reduce_run(const StageArgs& a) {
  __shared__ unsigned long long red[TB / 64];
  unsigned long long best = 0;
  for (int i = threadIdx.x; i < a.nb; i += TB) {
    const int r = a.r0 + i;
    const uint64_t tb = a.best[r] >> 32;
    const unsigned long long key = (tb << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)r);
    if (key > best) best = key;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(best, off, 64);
    if (o > best) best = o;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < TB / 64; ++q)
      if (red[q] > best) best = red[q];
    a.stage_out[0] = best;
    const float T = score_of_key((uint32_t)(best >> 32));
    a.flag_out[0] = ((double)T > a.tau) ? 1 : 0;
  }
}

__global__ void stage_reduce_kernel(StageArgs a) { stage_reduce_run(a); }

// stages [0, gridDim.x) of K ranks each starting at a.r0 (the last one
// ends at n), one workgroup each
__global__ void stage_reduce_multi_kernel(StageArgs a, int K, int n) {
  StageArgs b = a;
  b.r0 = a.r0 + (int)blockIdx.x * K;
  b.nb = min(K, n - b.r0);
  b.stage_out = a.stage_out + blockIdx.x;
  b.flag_out = a.flag_out + blockIdx.x;
  stage_reduce_run(b);
}

// one workgroup per stage entry
__global__ void stage_reduce_batch_kernel(const StageArgs* __restrict__ items) {
  stage_reduce_run(items[blockIdx.x]);
}

__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void rank_keys_kernel(const uint64_t* best, int n, uint64_t* keys) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t tb = (uint32_t)(best[r] >> 32);
  keys[r] = ((uint64_t)(0xFFFFFFFFu - tb) << 32) | (uint64_t)(uint32_t)r;
}

__global__ void rank_gather_kernel(const uint64_t* sorted, const uint64_t* best,
                                   const int32_t* order, const double* smad, int n,
                                   PoseRow* rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = (int)(uint32_t)(sorted[i] & 0xFFFFFFFFu);
  const uint64_t b = best[r];
  PoseRow row;
  row.rank = r;
  row.k = (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFu));
  row.hyp = order[r];
  row.tbits = (uint32_t)(b >> 32);
  row.smad = smad[row.hyp];
  rows[i] = row;
}

// rank keys of several requests: item t of request r = ranks [0, n_eval_r)
__global__ void rank_keys_batch_kernel(const RankArgs* __restrict__ reqs,
                                       const int64_t* __restrict__ prefix, int n,
                                       uint64_t* __restrict__ keys) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= prefix[n]) return;
  const int r = find_segment(prefix, n, t);
  const int i = (int)(t - prefix[r]);
  const uint32_t tb = (uint32_t)(reqs[r].best[i] >> 32);
  keys[t] = ((uint64_t)(0xFFFFFFFFu - tb) << 32) | (uint64_t)(uint32_t)i;
}

__global__ void rank_gather_batch_kernel(const RankArgs* __restrict__ reqs,
                                         const int64_t* __restrict__ row_prefix,
                                         const int64_t* __restrict__ key_prefix, int n,
                                         const uint64_t* __restrict__ sorted,
                                         PoseRow* __restrict__ rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= row_prefix[n]) return;
  const int q = find_segment(row_prefix, n, t);
  const int64_t i = t - row_prefix[q];
  const RankArgs& a = reqs[q];
  const int r = (int)(uint32_t)(sorted[key_prefix[q] + i] & 0xFFFFFFFFu);
  const uint64_t b = a.best[r];
  PoseRow row;
  row.rank = r;
  row.k = (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFu));
  row.hyp = a.order[r];
  row.tbits = (uint32_t)(b >> 32);
  row.smad = a.smad[row.hyp];
  rows[t] = row;
}

// Cell offset and heading index (Ng grid) of a rank's packed word: a
// refined code (bit 31 of the low word clear) or ~k.
__device__ __forceinline__ void decode_pose(uint64_t b, int o, int* dx, int* dy, int* g) {
  const uint32_t low = (uint32_t)(b & 0xFFFFFFFFu);
  if (low & 0x80000000u) {
    *dx = 0;
    *dy = 0;
    *g = o * (int)(0xFFFFFFFFu - low);
  } else {
    *dx = (int)(low & 31u) - 15;
    *dy = (int)((low >> 5) & 31u) - 15;
    *g = (int)(low >> 10);
  }
}

__global__ __launch_bounds__(TB) void margin_kernel(MarginArgs a) {
  __shared__ unsigned long long red[NW];
  const int r1 = a.top->rank;
  if (r1 < 0 || r1 >= a.n_eval) {               // workgroup-uniform
    if (threadIdx.x == 0) {
      a.out[0] = 0;
      a.out[1] = 0;
      a.out[2] = 0;
    }
    return;
  }
  int dx1, dy1, g1;
  decode_pose(a.best[r1], a.o, &dx1, &dy1, &g1);
  const int h1 = a.order[r1];
  const int x1 = a.hyp_xy[2 * h1] + dx1, y1 = a.hyp_xy[2 * h1 + 1] + dy1;
  unsigned long long m = 0;
  for (int r = threadIdx.x; r < a.n_eval; r += TB) {
    const uint64_t b = a.best[r];
    int dx, dy, g;
    decode_pose(b, a.o, &dx, &dy, &g);
    const int h = a.order[r];
    const int64_t ex = (int64_t)(a.hyp_xy[2 * h] + dx - x1), ey = (int64_t)(a.hyp_xy[2 * h + 1] + dy - y1);
    int dgc = g - g1;
    if (dgc < 0) dgc = -dgc;
    if (2 * dgc > a.Ng) dgc = a.Ng - dgc;
    const bool far = (double)(ex * ex + ey * ey) * a.res * a.res >= 0.25 || 12 * dgc >= a.Ng;
    if (!far) continue;
    const unsigned long long key =
        ((b >> 32) << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)r);
    if (key > m) m = key;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o2 = __shfl_xor(m, off, 64);
    if (o2 > m) m = o2;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NW; ++q)
      if (red[q] > m) m = red[q];
    a.out[0] = m;
    uint64_t frag = 0;
    if (a.stage && !isnan(a.tau)) {
      for (int b = 0; b < a.n_stages; ++b) {
        const double T = (double)score_of_key((uint32_t)(a.stage[b] >> 32));
        if (T >= a.tau - 1e-4 && T <= a.tau + 1e-4) frag = 1;
      }
    }
    a.out[1] = frag;
    a.out[2] = a.best[r1];
  }
}

template <int R, int KB, bool FULL>
hipError_t launch_tam_batch_t(const TamArgs* items, const int64_t* prefix, int n, int64_t blocks,
                              size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((tam_batch_kernel<R, KB, FULL>), dim3((unsigned)blocks), dim3(TB), lds, s,
                     items, prefix, n);
  return hipGetLastError();
}

constexpr int kTamR[8] = {4, 8, 12, 16, 24, 32, 48, 64};

template <int KB, bool FULL>
hipError_t launch_tam_batch_kb(int R, const TamArgs* items, const int64_t* prefix, int n,
                               int64_t blocks, size_t lds, hipStream_t s) {
  const int nv = 64 * R;
  RELOC_TAM_CLASSES(launch_tam_batch_t, KB, FULL, items, prefix, n, blocks, lds, s)
}

}  // namespace

hipError_t launch_tam(const TamArgs& a, hipStream_t s) {
  if (a.nb <= 0) return hipSuccess;
  if (a.fine < 0 || a.fine > 3) return hipErrorInvalidValue;
  const bool full = a.fine >= 2;
  if (a.keybits <= 12) return full ? launch_tam_kb<12, true>(a, s) : launch_tam_kb<12, false>(a, s);
  if (a.keybits <= 16) return full ? launch_tam_kb<16, true>(a, s) : launch_tam_kb<16, false>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_refine_select(const uint64_t* best, int r0, int K, int n, int ns, int kr,
                                int32_t* sel, uint64_t* rbest, hipStream_t s) {
  if (ns <= 0 || kr <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_select_kernel, dim3(ns), dim3(TB), 0, s, best, r0, K, n, kr, sel,
                     rbest);
  return hipGetLastError();
}

hipError_t launch_refine(const RefineArgs& a, hipStream_t s) {
  if (a.n_slots <= 0) return hipSuccess;
  const int w = 2 * a.h + 1;
  if (a.h < 0 || a.h > 15 || a.s < 0 || a.s >= a.t.Ng || a.L != (2 * a.s + 1) * w * w)
    return hipErrorInvalidValue;
  if (a.t.fine < 0 || a.t.fine > 3) return hipErrorInvalidValue;
  const bool full = a.t.fine >= 2;
  if (a.t.keybits <= 12)
    return full ? launch_refine_kb<12, true>(a, s) : launch_refine_kb<12, false>(a, s);
  if (a.t.keybits <= 16)
    return full ? launch_refine_kb<16, true>(a, s) : launch_refine_kb<16, false>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_score_poses(const PoseArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.t.fine < 0 || a.t.fine > 3) return hipErrorInvalidValue;
  const bool full = a.t.fine >= 2;
  if (a.t.keybits <= 12)
    return full ? launch_poses_kb<12, true>(a, s) : launch_poses_kb<12, false>(a, s);
  if (a.t.keybits <= 16)
    return full ? launch_poses_kb<16, true>(a, s) : launch_poses_kb<16, false>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_refine_commit(const RefineArgs& a, hipStream_t s) {
  if (a.n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_commit_kernel, dim3((a.n_slots + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

int tam_class(const TamArgs& a) {
  const int R = tam_keys_per_lane(a.nv);
  int rc = -1;
  for (int i = 0; i < 8; ++i)
    if (kTamR[i] == R) rc = i;
  const int kc = a.keybits <= 12 ? 0 : a.keybits <= 16 ? 1 : -1;
  if (rc < 0 || kc < 0 || a.fine < 0 || a.fine > 3) return -1;
  return (a.fine >= 2 ? 16 : 0) + kc * 8 + rc;
}

size_t tam_lds_bytes(const TamArgs& a) { return tam_lut_lds(a.keybits <= 12 ? 12 : 16); }

hipError_t launch_tam_offsets(const int2* beams, int nv, const int2* dirs, int Ng, int stride,
                              uint32_t* off, hipStream_t s) {
  const int64_t n = (int64_t)Ng * stride;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(tam_offsets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     beams, nv, dirs, Ng, stride, off);
  return hipGetLastError();
}

hipError_t launch_tam_batch(int cls, const TamArgs* items, const int64_t* prefix, int n,
                            int64_t blocks, size_t lds, hipStream_t s) {
  if (n <= 0 || blocks <= 0) return hipSuccess;
  if (cls < 0 || cls >= kTamClasses) return hipErrorInvalidValue;
  const int R = kTamR[cls % 8];
  switch (cls / 8) {
    case 0: return launch_tam_batch_kb<12, false>(R, items, prefix, n, blocks, lds, s);
    case 1: return launch_tam_batch_kb<16, false>(R, items, prefix, n, blocks, lds, s);
    case 2: return launch_tam_batch_kb<12, true>(R, items, prefix, n, blocks, lds, s);
    default: return launch_tam_batch_kb<16, true>(R, items, prefix, n, blocks, lds, s);
  }
}

hipError_t launch_stage_reduce_multi(const StageArgs& a, int K, int ns, int n, hipStream_t s) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_reduce_multi_kernel, dim3(ns), dim3(TB), 0, s, a, K, n);
  return hipGetLastError();
}

hipError_t launch_stage_reduce_batch(const StageArgs* items, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_reduce_batch_kernel, dim3(n), dim3(TB), 0, s, items);
  return hipGetLastError();
}

hipError_t launch_rank_keys_batch(const RankArgs* reqs, const int64_t* prefix, int n,
                                  int64_t total, uint64_t* keys, hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_keys_batch_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     s, reqs, prefix, n, keys);
  return hipGetLastError();
}

hipError_t launch_rank_gather_batch(const RankArgs* reqs, const int64_t* row_prefix,
                                    const int64_t* key_prefix, int n, int64_t total,
                                    const uint64_t* sorted, PoseRow* rows, hipStream_t s) {
  if (n <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_gather_batch_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256),
                     0, s, reqs, row_prefix, key_prefix, n, sorted, rows);
  return hipGetLastError();
}

hipError_t launch_margin(const MarginArgs& a, hipStream_t s) {
  if (a.n_eval <= 0) return hipSuccess;
  hipLaunchKernelGGL(margin_kernel, dim3(1), dim3(TB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_stage_reduce(const StageArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(stage_reduce_kernel, dim3(1), dim3(TB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v,
                     n);
  return hipGetLastError();
}

hipError_t launch_rank_keys(const uint64_t* best, int n, uint64_t* keys, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_keys_kernel, dim3((n + 255) / 256), dim3(256), 0, s, best, n, keys);
  return hipGetLastError();
}

hipError_t launch_rank_gather(const uint64_t* sorted, const uint64_t* best,
                              const int32_t* order, const double* smad, int n, PoseRow* rows,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(rank_gather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, sorted, best,
                     order, smad, n, rows);
  return hipGetLastError();
}

}  // namespace reloc
