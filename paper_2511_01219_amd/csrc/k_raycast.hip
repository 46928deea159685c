// Fused panoramic ray cast (eq. 13-14) and SMAD scoring (eq. 16-20).
//
// One workgroup per positional hypothesis. Its threads cast the Ns rays of
// the panoramic synthetic scan with an exact integer supercover traversal,
// leave the ranges in LDS, form the cyclic prefix sums of eq. 17 in FP64
// (every partial sum is an exact multiple of 2^-29 below 2^18 for ranges in
// [2^-6, 2^6) m, so the summation order cannot change a bit), score every
// circular shift with eq. 18-19 and reduce to the eq. 20 minimum.
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
//  * bits: one 8x8-cell tile per uint64, one occupancy test per crossing;
//  * skip: one byte per cell in 8x8 tiles holding 0 for occupied cells and
//    1 + s for free ones, s = floor(sqrt(k) - 1.4145) cells, k the squared
//    EDT value. No occupied cell centre lies within sqrt(k) of this cell's
//    centre, so any ray segment of length s starting inside the cell only
//    touches free cells (a touched cell's centre is within 0.7072 of the
//    segment, the segment starts within 0.7072 of this centre). The traversal
//    then jumps J = floor(s |U_major| / |U|) crossings along the major axis in
//    one step and recomputes the exact state: the count of minor-axis
//    crossings at or before the landing parameter (integer division, exact)
//    and D from the counts. Jumps never skip an occupied cell, so hits,
//    ranges and tie rules are those of the step-by-step traversal.
// Rays are handed to lanes dynamically (LDS counter), so a lane that finishes
// a short ray starts the next one at once instead of idling.
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
struct SkipMap {
  __amdgpu_buffer_rsrc_t rsrc;
  int tpr;
  __device__ __forceinline__ uint32_t at(int x, int y) const {
    const uint32_t off = (tile_off(x, y, tpr) << 6) | ((uint32_t)(y & 7) << 3) | (uint32_t)(x & 7);
    return __builtin_amdgcn_raw_buffer_load_b8(rsrc, off, 0, 0);
  }
};

__device__ float cast_ray_skip(const SkipMap& sm, int W, int H, int ix0, int iy0, int ux, int uy,
                               float kx, float ky, float rmax, int rcells, int* hit,
                               int* steps) {
  const int ax = ux < 0 ? -ux : ux, ay = uy < 0 ? -uy : uy;
  const int sx = ux > 0 ? 1 : (ux < 0 ? -1 : 0);
  const int sy = uy > 0 ? 1 : (uy < 0 ? -1 : 0);
  const int dA = ay << 8, dB = ax << 8;
  const bool xmaj = ax >= ay;
  const int amaj = xmaj ? ax : ay, bmin = xmaj ? ay : ax;
  const int64_t den = (int64_t)amaj << 8;
  const float rden = 1.0f / (float)den;
  // crossings of the major axis per cell of path length, rounded down a hair
  const float f = (float)amaj / sqrtf((float)ax * (float)ax + (float)ay * (float)ay) * 0.99999f;
  int D = (ay - ax) << 7;
  int cx = ix0, cy = iy0, nx = 0, ny = 0, it = 0;
  uint32_t v = sm.at(cx, cy);
  int h = -1;
  float z = 0.f;
  for (;;) {
    ++it;
    // free-space jump: J major crossings, all touched cells guaranteed free
    const int s = (int)v - 1;
    if (s >= 2) {
      const int J = (int)((float)s * f);
      if (J > 0) {
        const int na = (xmaj ? nx : ny) + J;
        const int64_t N = (int64_t)(128 + 256 * (na - 1)) * bmin - (int64_t)128 * amaj;
        int nb = 0;
        if (N >= 0) {
          int q = (int)((float)N * rden);
          const int64_t r = N - (int64_t)q * den;
          q += (r < 0) ? -1 : (r >= den ? 1 : 0);
          nb = q + 1;
        }
        nx = xmaj ? na : nb;
        ny = xmaj ? nb : na;
        cx = ix0 + sx * nx;
        cy = iy0 + sy * ny;
        D = (int)((int64_t)(128 + 256 * nx) * ay - (int64_t)(128 + 256 * ny) * ax);
        if ((unsigned)cx >= (unsigned)W || (unsigned)cy >= (unsigned)H) break;
        if (max(nx, ny) > rcells) break;
      }
    }
    // one exact crossing, then test the entered cell
    if (D != 0) {
      const bool stx = D < 0;
      cx += stx ? sx : 0;
      cy += stx ? 0 : sy;
      nx += stx ? 1 : 0;
      ny += stx ? 0 : 1;
      D += stx ? dA : -dB;
      if ((unsigned)cx >= (unsigned)W || (unsigned)cy >= (unsigned)H) break;
      v = sm.at(cx, cy);
      if (v == 0) {
        const int n = stx ? nx : ny;
        z = __fmul_rn((float)(128 + 256 * (n - 1)), stx ? kx : ky);
        h = cy * W + cx;
        break;
      }
    } else {
      const int x1 = cx + sx, y1 = cy + sy;
      const bool inx = (unsigned)x1 < (unsigned)W, iny = (unsigned)y1 < (unsigned)H;
      int best = -1;
      if (inx && sm.at(x1, cy) == 0) best = cy * W + x1;
      if (iny && sm.at(cx, y1) == 0) {
        const int li = y1 * W + cx;
        if (best < 0 || li < best) best = li;
      }
      const bool ind = inx && iny;
      const uint32_t vd = ind ? sm.at(x1, y1) : 1u;
      if (ind && vd == 0) {
        const int li = y1 * W + x1;
        if (best < 0 || li < best) best = li;
      }
      cx = x1; cy = y1; ++nx; ++ny; D += dA - dB;
      if (best >= 0) {
        z = __fmul_rn((float)(128 + 256 * (nx - 1)), kx);
        h = best;
        break;
      }
      if (!ind) break;
      v = vd;
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

// ------------------------------------------------------------ SMAD epilogue
// S[1..Ns] hold the ranges; turns them into prefix sums and scores every shift
__device__ void smad_epilogue(const RayArgs& a, double* S, int h) {
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
  }
}

template <int VARIANT>
__global__ __launch_bounds__(RT) void raycast_smad_kernel(RayArgs a) {
  extern __shared__ double S[];   // [Ns + 1]: S[j + 1] = range j, then prefix sums
  __shared__ int next_ray;
  const int h = blockIdx.x;
  const int tid = threadIdx.x;
  const int Ns = a.Ns;
  const int ix0 = a.hyp_xy[2 * h], iy0 = a.hyp_xy[2 * h + 1];
  if (tid == 0) next_ray = RT;
  __syncthreads();
  SkipMap sm;
  if (VARIANT == 1) {
    sm.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)a.skip, (short)0, (int)a.skip_bytes,
                                                0x00020000);
    sm.tpr = a.tpr;
  }
  for (int j = tid; j < Ns; j = atomicAdd(&next_ray, 1)) {
    const int2 U = a.dirs[j];
    const float2 kk = a.kap[j];
    int hit, steps;
    float z;
    if (VARIANT == 1)
      z = cast_ray_skip(sm, a.W, a.H, ix0, iy0, U.x, U.y, kk.x, kk.y, a.rmax, a.rcells, &hit,
                        &steps);
    else
      z = cast_ray_bits(a.bits, a.W, a.H, a.tpr, ix0, iy0, U.x, U.y, kk.x, kk.y, a.rmax,
                        a.rcells, &hit, &steps);
    S[j + 1] = (double)z;
    if (a.dbg_hit) a.dbg_hit[(size_t)h * Ns + j] = hit;
    if (a.dbg_rng) a.dbg_rng[(size_t)h * Ns + j] = z;
    if (a.dbg_steps) a.dbg_steps[(size_t)h * Ns + j] = steps;
  }
  __syncthreads();
  smad_epilogue(a, S, h);
}

}  // namespace

hipError_t launch_raycast_smad(const RayArgs& a, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  const size_t lds = (size_t)(a.Ns + 1) * sizeof(double);
  if (a.variant == 1 && a.skip)
    hipLaunchKernelGGL(raycast_smad_kernel<1>, dim3(a.n_hyp), dim3(RT), lds, s, a);
  else
    hipLaunchKernelGGL(raycast_smad_kernel<0>, dim3(a.n_hyp), dim3(RT), lds, s, a);
  return hipGetLastError();
}

// Skip byte per cell from the squared EDT: 0 occupied, else 1 + s with
// s = floor(sqrt(k) - 1.4145) clamped to [0, 254]. Tiles of 8x8 bytes.
namespace {
__global__ void skipmap_kernel(const uint32_t* __restrict__ k, int W, int H, int tpr, int tph,
                               uint8_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = (uint32_t)tpr * (uint32_t)tph * 64u;
  if (i >= n) return;
  const uint32_t tile = i >> 6;
  const int x = (int)(tile % (uint32_t)tpr) * 8 + (int)(i & 7);
  const int y = (int)(tile / (uint32_t)tpr) * 8 + (int)((i >> 3) & 7);
  uint8_t v = 0;
  if (x < W && y < H) {
    const uint32_t kk = k[(size_t)y * W + x];
    if (kk != 0) {
      const float s = floorf(__fsqrt_rn((float)kk) - 1.4145f);
      v = (uint8_t)(1 + (int)fminf(254.f, fmaxf(0.f, s)));
    }
  }
  out[i] = v;
}
}  // namespace

hipError_t launch_skipmap(const uint32_t* k, int W, int H, int tpr, int tph, uint8_t* out,
                          hipStream_t s) {
  const uint32_t n = (uint32_t)tpr * (uint32_t)tph * 64u;
  hipLaunchKernelGGL(skipmap_kernel, dim3((n + 255) / 256), dim3(256), 0, s, k, W, H, tpr, tph,
                     out);
  return hipGetLastError();
}

}  // namespace reloc
