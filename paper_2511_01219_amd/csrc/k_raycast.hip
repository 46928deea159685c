// Panoramic ray cast (eq. 13-14) and SMAD scoring (eq. 16-20).
//
// Default path: one fused kernel casts the Ns rays of a hypothesis with one
// workgroup, keeps the ranges on chip and forms the hypothesis' SMAD there;
// no range reaches memory. The split path (the bit-tile variant for maps
// without walk words, explicit variants, and the ablation coarse metrics
// that read every range) writes one range per (hypothesis, direction) to a
// range buffer, and a SMAD kernel loads a hypothesis' Ns ranges into LDS.
// Either way the cyclic prefix sums of eq. 17 are FP64 sums whose every
// partial value is an exact multiple of 2^-29 below 2^18 (ranges lie in
// [2^-6, 2^6) m), so the summation order cannot change a bit; every
// circular shift is scored with eq. 18-19 and reduced to the eq. 20
// minimum.
//
// Traversal. The ray leaves the centre of cell (ix0, iy0), X = 256 ix0 + 128
// in Q8 units, along the integer direction U. After nx x-crossings and ny
// y-crossings, D = (128 + 256 nx)|Uy| - (128 + 256 ny)|Ux| compares the next
// two crossing parameters: D < 0 x first, D > 0 y first, D = 0 an exact corner
// where the x-neighbour, the y-neighbour and the diagonal are entered at the
// same parameter. |D| < 2^28 for every reachable state. The range of a hit is
// fl32(fl32(entry offset along the entry axis) * kappa_axis), x axis at a
// corner; 0 when the ray leaves the map, passes the (result-neutral) Chebyshev
// cut-off, or the range exceeds range_max.
//
// Two interchangeable variants (identical results):
//  * bits: one 8x8-cell tile per uint64, one occupancy test per crossing,
//    one workgroup per hypothesis;
//  * skip: walk words (0 occupied; else a free-space radius byte 1 + s,
//    s = floor(sqrt(k) - 1.4145) cells with k the squared EDT value, and the
//    number of free cells that follow along the ray's major direction). No
//    occupied cell centre lies within sqrt(k) of the cell's centre, so a ray
//    segment of length s starting inside the cell only touches free cells (a
//    touched cell's centre is within 0.7072 of the segment, the segment starts
//    within 0.7072 of this centre). The traversal jumps over such free space
//    and recomputes the exact crossing state at the landing point, so hits,
//    ranges and tie rules are those of the step-by-step traversal. Lanes
//    are refilled with the next rays as rays end (the fused kernel: the
//    rays of one hypothesis per workgroup; the split kernel: the rays of
//    all hypotheses as one index space cut into single-wavefront chunks).
#include <climits>
#include <cmath>

#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int RT = 256;   // threads per workgroup

__device__ __forceinline__ uint32_t tile_off(int x, int y, int tpr) {
  return ((uint32_t)(y >> 3) * (uint32_t)tpr + (uint32_t)(x >> 3));
}

// ----------------------------------------------------------------- variant: bits
__device__ __forceinline__ bool occ_bit(const uint64_t* __restrict__ bits, int tpr, int x,
                                        int y) {
  const uint64_t w = bits[tile_off(x, y, tpr)];
  return (w >> (((y & 7) << 3) | (x & 7))) & 1ull;
}

__device__ float cast_ray_bits(const uint64_t* __restrict__ bits, int W, int H, int tpr, int ix0,
                               int iy0, int ux, int uy, float kx, float ky, float rmax,
                               int rcells, int* hit, int* steps) {
  const int ax = ux < 0 ? -ux : ux, ay = uy < 0 ? -uy : uy;
  const int sx = ux > 0 ? 1 : (ux < 0 ? -1 : 0);
  const int sy = uy > 0 ? 1 : (uy < 0 ? -1 : 0);
  const int dA = ay << 8, dB = ax << 8;
  int D = (ay - ax) << 7;
  int cx = ix0, cy = iy0, nx = 0, ny = 0, it = 0;
  int h = -1;
  float z = 0.f;
  for (;;) {
    ++it;
    if (D != 0) {
      const bool stx = D < 0;
      cx += stx ? sx : 0;
      cy += stx ? 0 : sy;
      nx += stx ? 1 : 0;
      ny += stx ? 0 : 1;
      D += stx ? dA : -dB;
      if ((unsigned)cx >= (unsigned)W || (unsigned)cy >= (unsigned)H) break;
      if (occ_bit(bits, tpr, cx, cy)) {
        const int n = stx ? nx : ny;
        z = __fmul_rn((float)(128 + 256 * (n - 1)), stx ? kx : ky);
        h = cy * W + cx;
        break;
      }
    } else {
      const int x1 = cx + sx, y1 = cy + sy;
      const bool inx = (unsigned)x1 < (unsigned)W, iny = (unsigned)y1 < (unsigned)H;
      int best = -1;
      if (inx && occ_bit(bits, tpr, x1, cy)) best = cy * W + x1;
      if (iny && occ_bit(bits, tpr, cx, y1)) {
        const int li = y1 * W + cx;
        if (best < 0 || li < best) best = li;
      }
      if (inx && iny && occ_bit(bits, tpr, x1, y1)) {
        const int li = y1 * W + x1;
        if (best < 0 || li < best) best = li;
      }
      cx = x1; cy = y1; ++nx; ++ny; D += dA - dB;
      if (best >= 0) {
        z = __fmul_rn((float)(128 + 256 * (nx - 1)), kx);
        h = best;
        break;
      }
      if (!inx || !iny) break;
    }
    if (max(nx, ny) > rcells) break;
  }
  if (z > rmax) {
    z = 0.f;
    h = -1;
  }
  *hit = h;
  *steps = it;
  return z;
}

// ----------------------------------------------------------------- variant: skip
// Walk words read through a buffer resource with 32-bit byte offsets; a
// ray reads the plane of its major direction of travel.
struct WalkMap {
  __amdgpu_buffer_rsrc_t rsrc;
  __device__ __forceinline__ uint32_t at(uint32_t pbase, int off) const {
    return __builtin_amdgcn_raw_buffer_load_b16(rsrc, pbase + 2u * (uint32_t)off, 0, 0);
  }
};

// Per-lane traversal state of one ray in its major/minor frame: the major
// axis is the one with the larger |U| component (a = |U_major|,
// b = |U_minor|). With na major and nb minor crossings done,
// Dm = (128 + 256 na) b - (128 + 256 nb) a is negative when the next major
// crossing comes first, positive when the minor one does, zero at an exact
// corner (Dm is D of the x/y form for x-major rays and -D for y-major ones).
struct SkipRay {
  int a, b;            // |U_major|, |U_minor|
  int om, on;          // cell-offset change of a major / minor crossing
  int Dm, na, nb, off;
  int it;              // skip_iter calls so far (counted only where reported)
  int la, lb;          // last in-range major / minor crossing count
  int b8, na8, dab8;   // Dm change of a major crossing (256 b), of a minor one
                       // (-256 a), of a corner (256 (b - a))
  uint32_t pbase;      // byte offset of the ray's walk plane
  float f, r;          // major crossings per cell of path (rounded down), b / a
  float c;             // (1 - r) / 2 - 2^-7: the landing estimate is na r + c
  float ninv;          // -1 / (256 b), -inf for b = 0
  float kmaj, kmin;    // metres per Q8 unit along the major / minor axis
  uint32_t v;          // walk word of the current cell
  bool xmaj;
};

// What a ray's crossings depend on besides its direction, for one start
// cell and one direction class (code bit 0: x is the major axis, bit 1: the
// major step is negative, bit 2: the minor step is negative): cell-offset
// change of a major / minor crossing, last in-range major / minor crossing
// count (the minor one for b > 0), byte offset of the walk plane.
struct RayClass {
  int om, on, la, lb;
  uint32_t pbase;
};

__device__ __forceinline__ RayClass ray_class(int code, int ix0, int iy0, int W, int H,
                                              int rcells, uint32_t plane_bytes) {
  const bool xmaj = (code & 1) != 0, mneg = (code & 2) != 0, nneg = (code & 4) != 0;
  const int sM = xmaj ? 1 : W, sN = xmaj ? W : 1;
  const int pM = xmaj ? ix0 : iy0, eM = xmaj ? W : H;
  const int pN = xmaj ? iy0 : ix0, eN = xmaj ? H : W;
  RayClass k;
  k.om = mneg ? -sM : sM;
  k.on = nneg ? -sN : sN;
  k.la = min(rcells, mneg ? pM : eM - 1 - pM);
  k.lb = min(rcells, nneg ? pN : eN - 1 - pN);
  k.pbase = (uint32_t)((xmaj ? 0 : 2) + (mneg ? 1 : 0)) * plane_bytes;
  return k;
}

// Starts the ray of direction (di, df) from the cell at offset off0, whose
// class entry is k.
__device__ __forceinline__ void skip_start(SkipRay& r, int4 di, float4 df, const RayClass& k,
                                           int off0, int rcells, const WalkMap& sm) {
  r.xmaj = (di.z & 1) != 0;
  r.a = di.x;
  r.b = di.y;
  r.om = k.om;
  r.on = k.on;
  r.la = k.la;
  r.lb = r.b == 0 ? rcells : k.lb;
  r.pbase = k.pbase;
  r.ninv = -__int_as_float(di.w);
  r.f = df.x;
  r.r = df.y;
  r.kmaj = df.z;
  r.kmin = df.w;
  r.Dm = (r.b - r.a) << 7;
  r.b8 = r.b << 8;
  r.na8 = -(r.a << 8);
  r.dab8 = (r.b - r.a) << 8;
  r.c = (0.5f - 0.5f * r.r) - 0x1p-7f;
  r.na = r.nb = r.it = 0;
  r.off = off0;
  r.v = sm.at(r.pbase, r.off);
}

__device__ __forceinline__ void skip_init(SkipRay& r, int4 di, float4 df, int ix0, int iy0,
                                          int W, int H, int rcells, uint32_t plane_bytes,
                                          const WalkMap& sm) {
  skip_start(r, di, df, ray_class(di.z, ix0, iy0, W, H, rcells, plane_bytes),
             (int)__umul24(iy0, W) + ix0, rcells, sm);
}

// One iteration: at most one exact free-space jump, then one exact crossing
// with an occupancy test of the entered cell(s). Returns 0 while the ray
// goes on, else 1-3: the ray has ended, and with r.v == 0 and code 2 / 3 in
// the occupied cell r.off, entered across a major / minor boundary
// (skip_hit, skip_range); otherwise without a hit. Counts beyond la / lb
// mean the ray left the map or passed the cut-off: a miss.
//
// Two jumps are possible from the current cell, both landing just after a
// major crossing on the exact crossing sequence; the one reaching further
// is taken.
//  * Run jump: while Dm < 0 the next ceil(-Dm / 256 b) crossings are all
//    major, i.e. cells of the current minor row; the walk word says how
//    many of those are free (run). A float estimate of the ceiling, biased
//    low, is it or one below it: a run jump no longer than allowed, as exact
//    as any other.
//  * Radius jump: J major crossings are safe when all cells within the
//    free-space radius are free. The state just after the (na + J)-th major
//    crossing has the unique minor count with 256 (b - a) <= Dm < 256 b. A
//    float estimate of that count, biased low, is the count or one below it;
//    Dm is evaluated in wrapping 32-bit arithmetic (exact, the true value is
//    within one step of the window) and at most one step up lands in the
//    window.
// Every product here has factors below 2^23 (counts below 2^12 for ranges
// under 64 m at >= 1/32 m cells, |U| <= 2^20, strides <= 32768) and only its
// low 32 bits are used, so the full-rate 24-bit multiplies are exact.
__device__ __forceinline__ int skip_iter(SkipRay& r, const WalkMap& sm, int off0) {
  // f < 1, so s <= 1 (s = -1 only for an occupied start cell) gives J = 0
  const int s = (int)(r.v & 255u) - 1;
  const int J = (int)((float)s * r.f);
  // t = -Dm / (256 b) less 2^-12, more than the float error of the product
  // (below 2^-14 for t <= 256), so ceil(est) is ceil(t) or one less: never
  // more major crossings than come before the next minor one. No test of
  // Dm < 0: for Dm >= 0 the minor step b is positive, est < 0 and kr <= 0
  // leaves the jump to J
  const float est = fminf(__builtin_fmaf((float)r.Dm, r.ninv, -0x1p-12f), 256.f);
  const int kr = min((int)(r.v >> 8), (int)ceilf(est));
  // one update for both jumps: a run jump ends in the same window as the
  // radius jump (only major crossings on the way, nb unchanged), so the
  // state after the farther one is computed the same way for either, and
  // lanes that take different jumps share one instruction stream
  const int Jt = max(kr, J);
  if (Jt > 0) {
    const int na = r.na + Jt;
    // nb = floor(x) with x = (na - 1/2) r + 1/2 >= 1/2. The float value of
    // x - 2^-7 is within 2^-10 of it (na < 2^13, r < 1), so it lies in
    // (x - 1, x) and is positive: truncated it is nb or nb - 1, and one
    // exact step up settles it
    int nb = (int)__builtin_fmaf((float)na, r.r, r.c);
    int Dm = (int)(__umul24(128 + 256 * na, r.b) - __umul24(128 + 256 * nb, r.a));
    if (Dm >= r.b8) { ++nb; Dm += r.na8; }
    r.na = na;
    r.nb = nb;
    r.Dm = Dm;
    r.off = off0 + __mul24(na, r.om) + __mul24(nb, r.on);
    if (na > r.la || nb > r.lb) return 1;
  }
  if (r.Dm != 0) {
    const bool maj = r.Dm < 0;
    r.na += maj ? 1 : 0;
    r.nb += maj ? 0 : 1;
    r.Dm += maj ? r.b8 : r.na8;
    r.off += maj ? r.om : r.on;
    const bool out = r.na > r.la || r.nb > r.lb;
    r.v = out ? 1u : sm.at(r.pbase, r.off);
    return out || r.v == 0 ? (maj ? 2 : 3) : 0;
  }
  // exact corner: both neighbours and the diagonal share the entry parameter
  const bool ina = r.na + 1 <= r.la, inb = r.nb + 1 <= r.lb;
  int best = -1;
  if (ina && sm.at(r.pbase, r.off + r.om) == 0) best = r.off + r.om;
  if (inb && sm.at(r.pbase, r.off + r.on) == 0)
    best = (best < 0 || r.off + r.on < best) ? r.off + r.on : best;
  const bool ind = ina && inb;
  const int dg = r.off + r.om + r.on;
  const uint32_t vd = ind ? sm.at(r.pbase, dg) : 1u;
  if (ind && vd == 0) best = (best < 0 || dg < best) ? dg : best;
  r.off = dg;
  ++r.na;
  ++r.nb;
  r.Dm += r.dab8;
  r.v = vd;
  if (best >= 0) {
    // the entry offset is measured along x at a corner
    r.off = best;
    r.v = 0;
    return r.xmaj ? 2 : 3;
  }
  return ind ? 0 : 1;
}

// Whether the ray that skip_iter ended with code e stopped in an occupied
// cell (r.off).
__device__ __forceinline__ bool skip_hit(const SkipRay& r, int e) { return e >= 2 && r.v == 0; }

// Range of a ray that skip_iter ended with code e: the entry offset along the
// crossing's axis (n crossings of that axis done) times that axis' metres per
// Q8 unit; 0 for a miss.
__device__ __forceinline__ float skip_range(const SkipRay& r, int e) {
  const bool mj = e == 2;
  const int n = mj ? r.na : r.nb;
  return skip_hit(r, e) ? __fmul_rn((float)(128 + 256 * (n - 1)), mj ? r.kmaj : r.kmin) : 0.f;
}

__device__ __forceinline__ WalkMap make_walkmap(const RayArgs& a) {
  WalkMap sm;
  sm.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)a.walk, (short)0, (int)a.walk_bytes,
                                              0x00020000);
  return sm;
}

// Skip-variant ray cast. The rays of all hypotheses form one index space
// (ray q = hypothesis q / Ns, direction q % Ns); each single-wavefront
// workgroup owns a contiguous chunk of it. A lane whose ray ends writes the
// range and goes idle; once at least REFILL lanes are idle they take the
// next consecutive rays of the chunk together (positions by mbcnt, the chunk
// counter is wavefront-uniform), so lanes stay busy and neighbouring lanes
// work on neighbouring directions. The hardware balances the many chunks.
template <int REFILL>
__device__ __forceinline__ void raycast_skip_run(const RayArgs& a, int block) {
  const int lane = threadIdx.x;
  const int Ns = a.Ns, W = a.W, H = a.H, rcells = a.rcells;
  const int64_t total = (int64_t)a.n_hyp * Ns;
  const int64_t q0 = (int64_t)block * a.chunk;
  const int pool = (int)min((int64_t)a.chunk, total - q0);
  // hypothesis and direction of the chunk's first ray (wavefront-uniform)
  const int h0 = (int)(q0 / Ns);
  const int j0 = (int)(q0 - (int64_t)h0 * Ns);
  const float inv_ns = 1.0f / (float)Ns;
  const WalkMap sm = make_walkmap(a);
  const uint32_t plane_bytes = a.walk_bytes >> 2;
  int next = 64;
  int q = lane, off0 = 0, oh = 0, oj = 0;   // oh, oj: hypothesis and direction of the ray
  bool busy = q < pool;
  bool dry = pool <= 64;
  SkipRay r;
  auto start = [&](int qq) {
    // t < Ns + chunk < 2^13: the float quotient is within one of t / Ns
    const int t = j0 + qq;
    int dh = (int)((float)t * inv_ns);
    int jj = t - __mul24(dh, Ns);
    if (jj < 0) {
      --dh;
      jj += Ns;
    } else if (jj >= Ns) {
      ++dh;
      jj -= Ns;
    }
    const int h = a.perm ? a.perm[h0 + dh] : h0 + dh;
    oh = h;
    oj = jj;
    const int ix0 = a.hyp_xy[2 * h], iy0 = a.hyp_xy[2 * h + 1];
    off0 = (int)__umul24(iy0, W) + ix0;
    skip_init(r, a.dir_i[jj], a.dir_f[jj], ix0, iy0, W, H, rcells, plane_bytes, sm);
  };
  if (busy) start(q);
  for (;;) {
    if (busy) {
      ++r.it;
      const int e = skip_iter(r, sm, off0);
      if (e != 0) {
        float z = skip_range(r, e);
        int hit = skip_hit(r, e) ? r.off : -1;
        if (z > a.rmax) {
          z = 0.f;
          hit = -1;
        }
        const size_t o = (size_t)oh * Ns + oj;
        a.zbuf[o] = z;
        if (a.dbg_hit) a.dbg_hit[o] = hit;
        if (a.dbg_steps) a.dbg_steps[o] = r.it;
        busy = false;
      }
    }
    // one back edge: the state is updated in place on every path
    const unsigned long long idle = __ballot(!busy);
    const int cnt = __popcll(idle);
    if (dry && cnt == 64) break;
    if (!dry && cnt >= REFILL) {
      const int base = next;
      next += cnt;
      dry = next >= pool;
      const int qn = base + (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(idle >> 32),
                                __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
      if (!busy && qn < pool) {
        q = qn;
        start(q);
        busy = true;
      }
    }
  }
}

// Workgroup b of an n-workgroup grid runs on XCD b % 8 (round-robin
// dispatch). The returned index gives every XCD one contiguous slice of
// [0, n), walked in dispatch order, so one XCD's L2 serves rays from one
// compact run of the casting order.
__device__ __forceinline__ int xcd_slice(int b, int n) {
  const int x = b & 7, i = b >> 3;
  const int q = n >> 3, rem = n & 7;
  return x * q + min(x, rem) + i;
}

template <int REFILL>
__global__ __launch_bounds__(64) void raycast_skip_kernel(RayArgs a) {
  raycast_skip_run<REFILL>(a, xcd_slice(blockIdx.x, gridDim.x));
}

// Index of the segment holding item t: prefix[r] <= t < prefix[r + 1]
// (prefix[0] = 0, n segments, t < prefix[n]); wavefront-uniform.
__device__ __forceinline__ int find_segment(const int64_t* prefix, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Bit-tile ray cast: one workgroup per hypothesis, rays from a shared counter.
__global__ __launch_bounds__(RT) void raycast_bits_kernel(RayArgs a) {
  __shared__ int next_ray;
  const int h = blockIdx.x;
  const int tid = threadIdx.x;
  const int Ns = a.Ns;
  const int ix0 = a.hyp_xy[2 * h], iy0 = a.hyp_xy[2 * h + 1];
  if (tid == 0) next_ray = RT;
  __syncthreads();
  for (int j = tid; j < Ns; j = atomicAdd(&next_ray, 1)) {
    const int2 U = a.dirs[j];
    const float2 kk = a.kap[j];
    int hit, steps;
    const float z = cast_ray_bits(a.bits, a.W, a.H, a.tpr, ix0, iy0, U.x, U.y, kk.x, kk.y,
                                  a.rmax, a.rcells, &hit, &steps);
    const size_t o = (size_t)h * Ns + j;
    a.zbuf[o] = z;
    if (a.dbg_hit) a.dbg_hit[o] = hit;
    if (a.dbg_steps) a.dbg_steps[o] = steps;
  }
}

// ------------------------------------------- fused ray cast + SMAD (default)
// One workgroup of NW wavefronts per hypothesis: its Ns rays come from a
// counter shared by the wavefronts (lanes are refilled once REFILL of a
// wavefront's lanes are idle), the ranges stay on chip, and the same
// workgroup then forms SMAD (eq. 16-20), so no range ever goes to memory.
//
//  * Panoramic scans (one shift, eq. 20): a lane adds each of its finished
//    rays that lies in the FoV to an FP64 accumulator; the workgroup sum of
//    the accumulators is the interval sum of m = 0.
//  * Otherwise the ranges go to LDS (Z[Ns], FP32). Each thread sums one
//    contiguous block of Z, an exclusive scan of the block sums gives
//    prefix values Pb, so S(x) = sum of Z[0, x) = Pb[x / cb] plus at most
//    cb - 1 terms. Each thread scores a contiguous range of shifts: the
//    first from S (eq. 17-18), each next one (shift stride 1) by adding the
//    range that enters each FoV run and subtracting the one that leaves.
// Every partial sum is a multiple of 2^-29 below 2^18 (see the file
// header), so every FP64 addition and subtraction here is exact and the
// result equals the prefix-sum form bit for bit, whatever the order.
__device__ __forceinline__ bool in_fov(const RayArgs& a, int j) {
  for (int r = 0; r < a.n_runs; ++r) {
    const int2 rr = a.runs[r];
    int d = j - rr.x;
    if (d < 0) d += a.Ns;
    if (d < rr.y) return true;
  }
  return false;
}

__device__ __forceinline__ void smad_store(const RayArgs& a, int h, double v, int m) {
  a.smad[h] = v;
  a.argm[h] = m;
  a.keys[h] = (uint64_t)__double_as_longlong(v);
  a.vals[h] = h;
  if (a.best0) a.best0[h] = 0;
}

// DBG: the launch carries a range, hit or step buffer (reloc_debug_raycast)
// and the kernel counts steps and writes them; the timed path does neither.
template <int NW, int REFILL, bool PANO, bool DBG>
__device__ __forceinline__ void raycast_smad_run(const RayArgs& a, int pos, uint8_t* dyn) {
  constexpr int NT = NW * 64;
  __shared__ int s_next;
  __shared__ double s_wsum[NW];
  __shared__ double s_bv[NW];
  __shared__ int s_bm[NW];
  __shared__ uint32_t s_fov[4096 / 32];   // panoramic: FoV membership bit per direction
  __shared__ int4 s_cls[8];                // the hypothesis' ray classes (om, on, la, lb)
  __shared__ uint32_t s_clp[8];            // and their walk planes
  float* Z = (float*)dyn;
  double* Pb = (double*)(dyn + (((size_t)a.Ns * 4 + 7) & ~(size_t)7));
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Ns = a.Ns, W = a.W, H = a.H;
  const int h = a.perm ? a.perm[pos] : pos;
  const int ix0 = a.hyp_xy[2 * h], iy0 = a.hyp_xy[2 * h + 1];
  const int off0 = (int)__umul24(iy0, W) + ix0;
  const WalkMap sm = make_walkmap(a);
  const uint32_t plane_bytes = a.walk_bytes >> 2;
  // the eight ray classes of the hypothesis, so that starting a ray takes
  // its class entry instead of deriving it
  if (tid < 8) {
    const RayClass k = ray_class(tid, ix0, iy0, W, H, a.rcells, plane_bytes);
    s_cls[tid] = make_int4(k.om, k.on, k.la, k.lb);
    s_clp[tid] = k.pbase;
  }
  // panoramic scans: whether each direction lies in the FoV, taken when a
  // ray starts (a full turn needs no test); the bits are built once per
  // workgroup so the loop never waits on the FoV table
  const bool all_in = a.nfov == Ns;
  if constexpr (PANO) {
    if (!all_in) {
      for (int wd = tid; wd < (Ns + 31) / 32; wd += NT) {
        uint32_t bits = 0;
        for (int b = 0; b < 32; ++b)
          if (wd * 32 + b < Ns && in_fov(a, wd * 32 + b)) bits |= 1u << b;
        s_fov[wd] = bits;
      }
    }
  }
  if constexpr (NW > 1) {
    if (tid == 0) s_next = NT;
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  int nxt = NT;            // NW == 1: the wavefront's own (uniform) counter
  int q = tid;             // direction of the lane's ray
  // lane state: 0 casting; 1-3 the ray ended with that skip_iter code and its
  // range is not taken yet; 4 nothing to take. A lane's ended ray is taken
  // when the lane is refilled or at the end (its state stays as it ended), so
  // the loop does not form a range on every trip
  int st = q < Ns ? 0 : 4;
  bool dry = NT >= Ns;
  double acc = 0.0;        // panoramic: FoV sum of the lane's finished rays
  float fov = 1.f;         // panoramic: 1 when the lane's ray lies in the FoV, else 0
  auto fov_of = [&](int j) { return all_in || ((s_fov[j >> 5] >> (j & 31)) & 1u) != 0; };
  SkipRay r;
  auto start = [&](int j) {
    const int4 di = a.dir_i[j];
    const int c = di.z & 7;
    const int4 e = s_cls[c];
    const RayClass k{e.x, e.y, e.z, e.w, s_clp[c]};
    skip_start(r, di, a.dir_f[j], k, off0, a.rcells, sm);
  };
  // the range of the lane's ended ray (state e in 1-3) into the FoV sum or
  // LDS, and into the debug buffers
  auto take = [&](int e) {
    float z = skip_range(r, e);
    const bool far = z > a.rmax;
    if (far) z = 0.f;
    if constexpr (PANO) {
      acc += (double)(z * fov);   // z is finite and >= 0: exact, in any order
    } else {
      Z[q] = z;
    }
    if constexpr (DBG) {
      const size_t o = (size_t)h * Ns + q;
      if (a.zbuf) a.zbuf[o] = z;
      if (a.dbg_hit) a.dbg_hit[o] = skip_hit(r, e) && !far ? r.off : -1;
      if (a.dbg_steps) a.dbg_steps[o] = r.it;
    }
  };
  if (st == 0) {
    start(q);
    if constexpr (PANO) fov = fov_of(q) ? 1.f : 0.f;
  }
  for (;;) {
    if (st == 0) {
      if constexpr (DBG) ++r.it;
      st = skip_iter(r, sm, off0);
    }
    const unsigned long long idle = __ballot(st != 0);
    const int cnt = __popcll(idle);
    if (dry && cnt == 64) break;
    if (!dry && cnt >= REFILL) {
      int base;
      if constexpr (NW == 1) {
        base = nxt;
        nxt += cnt;
      } else {
        int b = 0;
        if (lane == 0) b = atomicAdd(&s_next, cnt);
        base = __builtin_amdgcn_readfirstlane(b);
      }
      dry = base + cnt >= Ns;
      const int qn = base + (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
      if (st != 0) {
        if (st != 4) take(st);
        st = 4;
        if (qn < Ns) {
          q = qn;
          start(q);
          if constexpr (PANO) fov = fov_of(q) ? 1.f : 0.f;
          st = 0;
        }
      }
    }
  }
  if (st != 4) take(st);

  if constexpr (PANO) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if constexpr (NW > 1) {
      if (lane == 0) s_wsum[wv] = acc;
      __syncthreads();
      if (tid == 0) {
        acc = 0.0;
        for (int w = 0; w < NW; ++w) acc += s_wsum[w];
      }
    }
    if (tid == 0) smad_store(a, h, fabs(a.zbar - acc / (double)a.nfov), 0);
    return;
  }

  // every range of the hypothesis is in Z
  if constexpr (NW > 1) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  const int cb = (Ns + NT - 1) / NT;
  const int b0 = min(Ns, tid * cb), b1 = min(Ns, b0 + cb);
  double local = 0.0;
  for (int i = b0; i < b1; ++i) local += (double)Z[i];
  double incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  double excl = incl - local, total;
  if constexpr (NW > 1) {
    if (lane == 63) s_wsum[wv] = incl;
    __syncthreads();
    total = 0.0;
    for (int w = 0; w < NW; ++w) {
      if (w < wv) excl += s_wsum[w];
      total += s_wsum[w];
    }
  } else {
    total = __shfl(incl, 63, 64);
  }
  Pb[tid] = excl;
  if constexpr (NW > 1) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // S(x) = sum of Z[0, x) for 0 <= x < Ns; C(x) the cyclic form for x < 3 Ns
  auto S = [&](int x) -> double {
    const int b = x / cb;
    double s = Pb[b];
    for (int i = b * cb; i < x; ++i) s += (double)Z[i];
    return s;
  };
  auto C = [&](int x) -> double {
    const int qq = x >= 2 * Ns ? 2 : (x >= Ns ? 1 : 0);
    return (double)qq * total + S(x - qq * Ns);
  };
  auto wrap = [&](int x) { return x >= 2 * Ns ? x - 2 * Ns : (x >= Ns ? x - Ns : x); };
  const int nsh = a.n_shifts, ne = a.n_enum;
  const int cs = (nsh + NT - 1) / NT;
  const int s0 = tid * cs, s1 = min(nsh, s0 + cs);
  double bv = INFINITY;
  int bm = INT_MAX;
  double tot = 0.0;
  for (int sh = s0; sh < s1; ++sh) {
    const int m = sh * ne;
    if (sh == s0 || ne != 1) {
      tot = 0.0;
      for (int rr = 0; rr < a.n_runs; ++rr) {
        const int2 ru = a.runs[rr];
        tot += C(ru.x + m + ru.y) - C(ru.x + m);
      }
    } else {
      // shift m - 1 -> m: each run gains Z[u + m - 1 + L] and loses Z[u + m - 1]
      for (int rr = 0; rr < a.n_runs; ++rr) {
        const int2 ru = a.runs[rr];
        tot += (double)Z[wrap(ru.x + m - 1 + ru.y)] - (double)Z[wrap(ru.x + m - 1)];
      }
    }
    const double v = fabs(a.zbar - tot / (double)a.nfov);
    if (v < bv) {
      bv = v;
      bm = m;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int om = __shfl_xor(bm, off, 64);
    if (ov < bv || (ov == bv && om < bm)) {
      bv = ov;
      bm = om;
    }
  }
  if constexpr (NW > 1) {
    if (lane == 0) {
      s_bv[wv] = bv;
      s_bm[wv] = bm;
    }
    __syncthreads();
    if (tid == 0)
      for (int w = 1; w < NW; ++w)
        if (s_bv[w] < bv || (s_bv[w] == bv && s_bm[w] < bm)) {
          bv = s_bv[w];
          bm = s_bm[w];
        }
  }
  if (tid == 0) smad_store(a, h, bv, bm);
}

template <int NW, int REFILL, bool PANO, bool DBG>
__global__ __launch_bounds__(NW * 64) void raycast_smad_kernel(RayArgs a) {
  extern __shared__ __align__(8) uint8_t fused_dyn[];
  raycast_smad_run<NW, REFILL, PANO, DBG>(a, xcd_slice(blockIdx.x, gridDim.x), fused_dyn);
}

// Several requests, one workgroup per hypothesis: request r owns workgroups
// [prefix[r], prefix[r + 1]) (its hypotheses in casting order).
template <int NW, int REFILL>
__global__ __launch_bounds__(NW * 64) void raycast_smad_batch_kernel(
    const RayArgs* __restrict__ reqs, const int64_t* __restrict__ prefix, int n) {
  extern __shared__ __align__(8) uint8_t fused_dyn[];
  const int t = xcd_slice(blockIdx.x, gridDim.x);
  const int r = find_segment(prefix, n, t);
  const RayArgs& a = reqs[r];
  const int pos = (int)(t - prefix[r]);
  if (a.n_shifts == 1)                         // workgroup-uniform
    raycast_smad_run<NW, REFILL, true, false>(a, pos, fused_dyn);
  else
    raycast_smad_run<NW, REFILL, false, false>(a, pos, fused_dyn);
}

// ------------------------------------------------------------------- SMAD
// SMAD of hypothesis h (eq. 16-20) by one wavefront from its ranges in
// zbuf: cyclic prefix sums S[0..Ns] in LDS (private to the wavefront), then
// every shift m scored from K interval sums, and the minimum with the
// smallest m on ties. Every partial sum is exact (see the file header), so
// lane order does not matter.
__device__ __forceinline__ void smad_wave(const RayArgs& a, int h, double* S) {
  const int lane = threadIdx.x & 63;
  const int Ns = a.Ns;
  const float* z = a.zbuf + (size_t)h * Ns;
  for (int i = lane; i < Ns; i += 64) S[i + 1] = (double)z[i];
  if (lane == 0) S[0] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // lane l owns S[1 + l c .. 1 + (l + 1) c)
  const int c = (Ns + 63) >> 6;
  const int b0 = 1 + lane * c, b1 = min(Ns + 1, b0 + c);
  double local = 0.0;
  for (int i = b0; i < b1; ++i) local += S[i];
  double incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  double run = incl - local;
  for (int i = b0; i < b1; ++i) {
    run += S[i];
    S[i] = run;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double total = S[Ns];
  double bv = INFINITY;
  int bm = INT_MAX;
  for (int sh = lane; sh < a.n_shifts; sh += 64) {
    const int m = sh * a.n_enum;
    double tot = 0.0;
    for (int r = 0; r < a.n_runs; ++r) {
      const int2 rr = a.runs[r];
      const int t1 = rr.x + m + rr.y, t0 = rr.x + m;
      const int q1 = t1 >= 2 * Ns ? 2 : (t1 >= Ns ? 1 : 0);
      const int q0 = t0 >= 2 * Ns ? 2 : (t0 >= Ns ? 1 : 0);
      const double c1 = (double)q1 * total + S[t1 - q1 * Ns];
      const double c0 = (double)q0 * total + S[t0 - q0 * Ns];
      tot += c1 - c0;
    }
    const double v = fabs(a.zbar - tot / (double)a.nfov);
    if (v < bv) {
      bv = v;
      bm = m;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int om = __shfl_xor(bm, off, 64);
    if (ov < bv || (ov == bv && om < bm)) {
      bv = ov;
      bm = om;
    }
  }
  if (lane == 0) {
    a.smad[h] = bv;
    a.argm[h] = bm;
    a.keys[h] = (uint64_t)__double_as_longlong(bv);
    a.vals[h] = h;
    if (a.best0) a.best0[h] = 0;
  }
}

// Panoramic scans score the single shift m = 0: the interval sums are plain
// masked sums of the ranges (exact in any order), no prefix array needed.
__device__ __forceinline__ void smad_wave_pano(const RayArgs& a, int h) {
  const int lane = threadIdx.x & 63;
  const int Ns = a.Ns;
  const float* z = a.zbuf + (size_t)h * Ns;
  double tot = 0.0;
  for (int j = lane; j < Ns; j += 64) {
    const double zj = (double)z[j];
    for (int r = 0; r < a.n_runs; ++r) {
      const int2 rr = a.runs[r];
      int d = j - rr.x;
      if (d < 0) d += Ns;
      if (d < rr.y) tot += zj;
    }
  }
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
  if (lane == 0) {
    const double v = fabs(a.zbar - tot / (double)a.nfov);
    a.smad[h] = v;
    a.argm[h] = 0;
    a.keys[h] = (uint64_t)__double_as_longlong(v);
    a.vals[h] = h;
    if (a.best0) a.best0[h] = 0;
  }
}

// One workgroup per hypothesis (long non-panoramic scans): S[1..Ns] hold the
// ranges; prefix sums by all 256 threads, shifts spread over the workgroup.
__device__ void smad_block(const RayArgs& a, double* S, int h) {
  __shared__ double wsum[RT / 64];
  __shared__ double rv[RT / 64];
  __shared__ int rm[RT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Ns = a.Ns;
  const int c = (Ns + RT - 1) / RT;
  const int b0 = 1 + tid * c, b1 = min(Ns + 1, b0 + c);
  double local = 0.0;
  for (int i = b0; i < b1; ++i) local += S[i];
  double incl = local;
  for (int off = 1; off < 64; off <<= 1) {
    const double v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  double run = incl - local;
  for (int q = 0; q < wv; ++q) run += wsum[q];
  for (int i = b0; i < b1; ++i) {
    run += S[i];
    S[i] = run;
  }
  if (tid == 0) S[0] = 0.0;
  __syncthreads();

  const double total = S[Ns];
  double bv = INFINITY;
  int bm = INT_MAX;
  for (int s = tid; s < a.n_shifts; s += RT) {
    const int m = s * a.n_enum;
    double tot = 0.0;
    for (int r = 0; r < a.n_runs; ++r) {
      const int2 rr = a.runs[r];
      const int t1 = rr.x + m + rr.y, t0 = rr.x + m;
      const int q1 = t1 >= 2 * Ns ? 2 : (t1 >= Ns ? 1 : 0);
      const int q0 = t0 >= 2 * Ns ? 2 : (t0 >= Ns ? 1 : 0);
      const double c1 = (double)q1 * total + S[t1 - q1 * Ns];
      const double c0 = (double)q0 * total + S[t0 - q0 * Ns];
      tot += c1 - c0;
    }
    const double v = fabs(a.zbar - tot / (double)a.nfov);
    if (v < bv) {
      bv = v;
      bm = m;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int om = __shfl_xor(bm, off, 64);
    if (ov < bv || (ov == bv && om < bm)) {
      bv = ov;
      bm = om;
    }
  }
  if (lane == 0) {
    rv[wv] = bv;
    rm[wv] = bm;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < RT / 64; ++q)
      if (rv[q] < bv || (rv[q] == bv && rm[q] < bm)) {
        bv = rv[q];
        bm = rm[q];
      }
    a.smad[h] = bv;
    a.argm[h] = bm;
    a.keys[h] = (uint64_t)__double_as_longlong(bv);
    a.vals[h] = h;
    if (a.best0) a.best0[h] = 0;
  }
}

// SMAD of hypothesis h of request a by the layout smad_layout chose:
// wpb > 0: wpb hypotheses per workgroup, one wavefront each (prefix sums in
// LDS unless the scan is panoramic); wpb == 0: one workgroup.
__device__ __forceinline__ void smad_dispatch(const RayArgs& a, int blk, int wpb, double* S) {
  if (wpb == 0) {
    const int h = blk;
    for (int j = threadIdx.x; j < a.Ns; j += RT) S[j + 1] = (double)a.zbuf[(size_t)h * a.Ns + j];
    __syncthreads();
    smad_block(a, S, h);
    return;
  }
  const int w = threadIdx.x >> 6;
  const int h = blk * wpb + w;
  if (h >= a.n_hyp) return;
  if (a.n_shifts == 1)
    smad_wave_pano(a, h);
  else
    smad_wave(a, h, S + (size_t)w * (a.Ns + 1));
}

__global__ __launch_bounds__(RT) void smad_kernel(RayArgs a, int wpb) {
  extern __shared__ double S[];
  smad_dispatch(a, blockIdx.x, wpb, S);
}

// ------------------------------------------------- direct coarse metrics
// SMAD by direct sums (eq. 16-20 without the prefix sums of eq. 17-18) or
// CAER (eq. 21) of hypothesis blockIdx.x by one workgroup. The synthetic
// ranges are stored three times over in LDS as FP32 (converting them back
// to FP64 is exact), plus kZPad more, so an index run start (< Ns) + shift
// (< Ns) + run offset (<= Ns + 1) never wraps. Each shift sums its FoV
// beams one at a time in beam order (run by run), the order the definition
// is written in, so the sums equal a sequential evaluation bit for bit. SMAD
// scores the shifts of eq. 20 (m = 0 only for panoramic scans); CAER is not
// rotation invariant and scores every shift.
//
// With n_enum = 1 a thread scores the shift pair (m, m + 1): beam t of a run
// needs Z[j + t + m] and Z[j + t + m + 1], so 9 loads serve 8 beams of both
// shifts; the loads of a batch are issued before any is used.
constexpr int kZPad = 8;

template <bool CAER>
__device__ __forceinline__ double coarse_term(double acc, double zm, double zs) {
  return CAER ? acc + fabs(zm - zs) : acc + zs;
}

template <bool CAER>
__device__ __forceinline__ void coarse_pair(const RayArgs& a, const float* Z, int m,
                                            double& acc0, double& acc1) {
  int i = 0;                                   // FoV beam index (into fov_z)
  for (int r = 0; r < a.n_runs; ++r) {
    const int2 rr = a.runs[r];
    const float* zb = Z + rr.x + m;
    int t = 0;
    for (; t + 8 <= rr.y; t += 8, i += 8) {
      float f[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) f[q] = zb[t + q];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double zm = CAER ? a.fov_z[i + q] : 0.0;
        acc0 = coarse_term<CAER>(acc0, zm, (double)f[q]);
        acc1 = coarse_term<CAER>(acc1, zm, (double)f[q + 1]);
      }
    }
    for (; t < rr.y; ++t, ++i) {
      const double zm = CAER ? a.fov_z[i] : 0.0;
      acc0 = coarse_term<CAER>(acc0, zm, (double)zb[t]);
      acc1 = coarse_term<CAER>(acc1, zm, (double)zb[t + 1]);
    }
  }
}

template <bool CAER>
__global__ __launch_bounds__(RT) void coarse_direct_kernel(RayArgs a) {
  extern __shared__ float Z[];             // [3 Ns + kZPad]
  __shared__ double rv[RT / 64];
  __shared__ int rm[RT / 64];
  const int h = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Ns = a.Ns;
  const float* z = a.zbuf + (size_t)h * Ns;
  for (int i = tid; i < Ns; i += RT) {
    const float v = z[i];
    Z[i] = v;
    Z[i + Ns] = v;
    Z[i + 2 * Ns] = v;
  }
  for (int i = tid; i < kZPad; i += RT) Z[3 * Ns + i] = z[i % Ns];
  __syncthreads();
  const int nsh = CAER ? (Ns + a.n_enum - 1) / a.n_enum : a.n_shifts;
  const double nfov = (double)a.nfov;
  double bv = INFINITY;
  int bm = INT_MAX;
  auto take = [&](double acc, int m) {
    const double mean = acc / nfov;
    const double v = CAER ? mean : fabs(a.zbar - mean);
    if (v < bv) {
      bv = v;
      bm = m;
    }
  };
  if (a.n_enum == 1 && nsh >= 2) {
    for (int m = 2 * tid; m < nsh; m += 2 * RT) {
      double acc0 = 0.0, acc1 = 0.0;
      coarse_pair<CAER>(a, Z, m, acc0, acc1);
      take(acc0, m);
      if (m + 1 < nsh) take(acc1, m + 1);
    }
  } else {
    for (int sh = tid; sh < nsh; sh += RT) {
      const int m = sh * a.n_enum;
      double acc = 0.0;
      int i = 0;
      for (int r = 0; r < a.n_runs; ++r) {
        const int2 rr = a.runs[r];
        for (int t = 0; t < rr.y; ++t, ++i)
          acc = coarse_term<CAER>(acc, CAER ? a.fov_z[i] : 0.0, (double)Z[rr.x + t + m]);
      }
      take(acc, m);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int om = __shfl_xor(bm, off, 64);
    if (ov < bv || (ov == bv && om < bm)) {
      bv = ov;
      bm = om;
    }
  }
  if (lane == 0) {
    rv[wv] = bv;
    rm[wv] = bm;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < RT / 64; ++q)
      if (rv[q] < bv || (rv[q] == bv && rm[q] < bm)) {
        bv = rv[q];
        bm = rm[q];
      }
    a.smad[h] = bv;
    a.argm[h] = bm;
    a.keys[h] = (uint64_t)__double_as_longlong(bv);
    a.vals[h] = h;
    if (a.best0) a.best0[h] = 0;
  }
}

// No coarse ordering: every key 0, so the stable sort keeps the set's order.
__global__ __launch_bounds__(RT) void coarse_none_kernel(RayArgs a) {
  const int h = blockIdx.x * RT + threadIdx.x;
  if (h >= a.n_hyp) return;
  a.smad[h] = 0.0;
  a.argm[h] = 0;
  a.keys[h] = 0;
  a.vals[h] = h;
  if (a.best0) a.best0[h] = 0;
}

}  // namespace

hipError_t launch_raycast(const RayArgs& a, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  if (a.walk && a.variant >= 1) {
    const int64_t total = (int64_t)a.n_hyp * a.Ns;
    const dim3 g((unsigned)((total + a.chunk - 1) / a.chunk)), w(64);
    switch (a.variant) {
      case 1: hipLaunchKernelGGL(raycast_skip_kernel<1>, g, w, 0, s, a); break;
      case 2: hipLaunchKernelGGL(raycast_skip_kernel<8>, g, w, 0, s, a); break;
      case 3: hipLaunchKernelGGL(raycast_skip_kernel<16>, g, w, 0, s, a); break;
      default: hipLaunchKernelGGL(raycast_skip_kernel<32>, g, w, 0, s, a); break;
    }
  } else {
    hipLaunchKernelGGL(raycast_bits_kernel, dim3(a.n_hyp), dim3(RT), 0, s, a);
  }
  return hipGetLastError();
}

void smad_layout(int max_ns, bool all_pano, int* wpb, size_t* lds) {
  if (all_pano) {
    *wpb = RT / 64;
    *lds = 0;
  } else if (max_ns <= 1024) {
    *wpb = RT / 64;
    *lds = (size_t)(RT / 64) * (max_ns + 1) * sizeof(double);
  } else {
    *wpb = 0;
    *lds = (size_t)(max_ns + 1) * sizeof(double);
  }
}

hipError_t launch_smad(const RayArgs& a, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  int wpb;
  size_t lds;
  smad_layout(a.Ns, a.n_shifts == 1, &wpb, &lds);
  const int blocks = wpb ? (a.n_hyp + wpb - 1) / wpb : a.n_hyp;
  hipLaunchKernelGGL(smad_kernel, dim3(blocks), dim3(RT), lds, s, a, wpb);
  return hipGetLastError();
}

namespace {
template <int NW, bool PANO, bool DBG>
void launch_fused_refill(const RayArgs& a, int refill, size_t lds, hipStream_t s) {
  const dim3 g((unsigned)a.n_hyp), w(NW * 64);
  switch (refill) {
    case 8: hipLaunchKernelGGL((raycast_smad_kernel<NW, 8, PANO, DBG>), g, w, lds, s, a); break;
    case 32: hipLaunchKernelGGL((raycast_smad_kernel<NW, 32, PANO, DBG>), g, w, lds, s, a); break;
    default: hipLaunchKernelGGL((raycast_smad_kernel<NW, 16, PANO, DBG>), g, w, lds, s, a); break;
  }
}

template <int NW, bool PANO>
hipError_t launch_fused_nw(const RayArgs& a, int refill, size_t lds, hipStream_t s) {
  if (a.zbuf || a.dbg_hit || a.dbg_steps)
    launch_fused_refill<NW, PANO, true>(a, refill, lds, s);
  else
    launch_fused_refill<NW, PANO, false>(a, refill, lds, s);
  return hipGetLastError();
}

template <bool PANO>
hipError_t launch_fused_pano(const RayArgs& a, int nw, int refill, hipStream_t s) {
  const size_t lds = PANO ? 0 : fused_lds_bytes(a.Ns, nw);
  switch (nw) {
    case 1: return launch_fused_nw<1, PANO>(a, refill, lds, s);
    case 2: return launch_fused_nw<2, PANO>(a, refill, lds, s);
    default: return launch_fused_nw<4, PANO>(a, refill, lds, s);
  }
}
}  // namespace

hipError_t launch_raycast_smad_fused(const RayArgs& a, int nw, int refill, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  if (!a.walk || (nw != 1 && nw != 2 && nw != 4) || (refill != 8 && refill != 16 && refill != 32))
    return hipErrorInvalidValue;
  return a.n_shifts == 1 ? launch_fused_pano<true>(a, nw, refill, s)
                         : launch_fused_pano<false>(a, nw, refill, s);
}

hipError_t launch_raycast_smad_fused_batch(const RayArgs* reqs, const int64_t* prefix, int n,
                                           int64_t blocks, int nw, size_t lds, hipStream_t s) {
  if (n <= 0 || blocks <= 0) return hipSuccess;
  const dim3 g((unsigned)blocks);
  switch (nw) {
    case 1:
      hipLaunchKernelGGL((raycast_smad_batch_kernel<1, 16>), g, dim3(64), lds, s, reqs, prefix, n);
      break;
    case 2:
      hipLaunchKernelGGL((raycast_smad_batch_kernel<2, 16>), g, dim3(128), lds, s, reqs, prefix, n);
      break;
    case 4:
      hipLaunchKernelGGL((raycast_smad_batch_kernel<4, 16>), g, dim3(256), lds, s, reqs, prefix, n);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_coarse(const RayArgs& a, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  switch (a.coarse) {
    case 0:
      return launch_smad(a, s);
    case 1:
    case 2: {
      if (a.nfov <= 0 || !a.fov_z) return hipErrorInvalidValue;
      const size_t lds = ((size_t)3 * a.Ns + kZPad) * sizeof(float);
      if (a.coarse == 2)
        hipLaunchKernelGGL(coarse_direct_kernel<true>, dim3(a.n_hyp), dim3(RT), lds, s, a);
      else
        hipLaunchKernelGGL(coarse_direct_kernel<false>, dim3(a.n_hyp), dim3(RT), lds, s, a);
      return hipGetLastError();
    }
    case 3:
      hipLaunchKernelGGL(coarse_none_kernel, dim3((a.n_hyp + RT - 1) / RT), dim3(RT), 0, s, a);
      return hipGetLastError();
    default:
      return hipErrorInvalidValue;
  }
}

// Walk words from the squared EDT. The radius byte is 1 + s with
// s = floor(sqrt(k) - 1.4145) clamped to [0, 254]: every cell whose centre
// lies within s cells of a free cell's centre is free. Runs are counted by
// one thread per row (x planes) or per column (y planes), walking against
// the plane's direction.
namespace {
__device__ __forceinline__ uint32_t radius_byte(uint32_t kk) {
  if (kk == 0) return 0;
  const float s = floorf(__fsqrt_rn((float)kk) - 1.4145f);
  return 1u + (uint32_t)fminf(254.f, fmaxf(0.f, s));
}

__global__ void walk_rows_kernel(const uint32_t* __restrict__ k, int W, int H,
                                 uint16_t* __restrict__ out) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= H) return;
  const size_t N = (size_t)W * H;
  const size_t row = (size_t)y * W;
  uint32_t run = 0;   // free cells after x towards +x
  for (int x = W - 1; x >= 0; --x) {
    const uint32_t s = radius_byte(k[row + x]);
    out[row + x] = (uint16_t)(s ? (s | run << 8) : 0u);
    run = s ? min(run + 1u, 255u) : 0u;
  }
  run = 0;            // free cells after x towards -x
  for (int x = 0; x < W; ++x) {
    const uint32_t s = radius_byte(k[row + x]);
    out[N + row + x] = (uint16_t)(s ? (s | run << 8) : 0u);
    run = s ? min(run + 1u, 255u) : 0u;
  }
}

__global__ void walk_cols_kernel(const uint32_t* __restrict__ k, int W, int H,
                                 uint16_t* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const size_t N = (size_t)W * H;
  uint32_t run = 0;   // towards +y
  for (int y = H - 1; y >= 0; --y) {
    const size_t c = (size_t)y * W + x;
    const uint32_t s = radius_byte(k[c]);
    out[2 * N + c] = (uint16_t)(s ? (s | run << 8) : 0u);
    run = s ? min(run + 1u, 255u) : 0u;
  }
  run = 0;            // towards -y
  for (int y = 0; y < H; ++y) {
    const size_t c = (size_t)y * W + x;
    const uint32_t s = radius_byte(k[c]);
    out[3 * N + c] = (uint16_t)(s ? (s | run << 8) : 0u);
    run = s ? min(run + 1u, 255u) : 0u;
  }
}
}  // namespace

hipError_t launch_walkmap(const uint32_t* k, int W, int H, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(walk_rows_kernel, dim3((H + 63) / 64), dim3(64), 0, s, k, W, H, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(walk_cols_kernel, dim3((W + 63) / 64), dim3(64), 0, s, k, W, H, out);
  return hipGetLastError();
}

}  // namespace reloc
