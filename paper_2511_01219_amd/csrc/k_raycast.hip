// Fused panoramic ray cast (eq. 13-14) and SMAD scoring (eq. 16-20).
//
// One workgroup per positional hypothesis. Its threads cast the Ns rays of
// the panoramic synthetic scan with an integer supercover DDA on the
// bit-packed grid, leave the ranges in LDS, form the cyclic prefix sums of
// eq. 17 in FP64 (every partial sum is an exact multiple of 2^-29 below 2^18
// for ranges in [2^-6, 2^6) m, so the summation order cannot change a bit),
// score every circular shift with eq. 18-19 and reduce to the eq. 20 minimum.
#include <climits>
#include <cmath>

#include "reloc_internal.h"

namespace reloc {

namespace {

constexpr int RT = 256;   // threads per workgroup

__device__ __forceinline__ bool occ_at(const uint64_t* __restrict__ bits, int tpr, int x,
                                       int y) {
  const uint64_t w = bits[(size_t)(y >> 3) * tpr + (x >> 3)];
  return (w >> (((y & 7) << 3) | (x & 7))) & 1ull;
}

// One ray from the centre of cell (ix0, iy0) along the Q20 direction (ux, uy).
// The ray visits every cell whose closed box it meets. With A = |Bx - X| |Uy|
// and B = |By - Y| |Ux| (Bx, By the next grid lines in Q8 units), the sign of
// D = A - B decides the next crossing: x first, y first, or an exact corner
// where the x-neighbour, the y-neighbour and the diagonal cell are entered at
// the same parameter. D stays within +-2^28, so 32-bit integers suffice.
// Range = fl32(fl32(entry offset along the entry axis) * kappa_axis), the
// x axis at a corner; 0 when the ray leaves the map, reaches no occupied cell
// within the cut-off, or the range exceeds rmax.
__device__ float cast_ray(const uint64_t* __restrict__ bits, int W, int H, int tpr, int ix0,
                          int iy0, int ux, int uy, float kx, float ky, float rmax, int rcells,
                          int* hit, int* steps) {
  const int ax = ux < 0 ? -ux : ux, ay = uy < 0 ? -uy : uy;
  const int sx = ux > 0 ? 1 : (ux < 0 ? -1 : 0);
  const int sy = uy > 0 ? 1 : (uy < 0 ? -1 : 0);
  const int dA = ay << 8, dB = ax << 8;
  int D = (ay - ax) << 7;
  int cx = ix0, cy = iy0, nx = 0, ny = 0, nc = 0;
  int h = -1;
  float z = 0.f;
  for (;;) {
    if (D != 0) {
      const bool stx = D < 0;
      if (stx) {
        cx += sx; ++nx; D += dA;
      } else {
        cy += sy; ++ny; D -= dB;
      }
      if ((unsigned)cx >= (unsigned)W || (unsigned)cy >= (unsigned)H) break;
      if (occ_at(bits, tpr, cx, cy)) {
        const int n = stx ? nx : ny;
        z = __fmul_rn((float)(128 + 256 * (n - 1)), stx ? kx : ky);
        h = cy * W + cx;
        break;
      }
    } else {
      const int x1 = cx + sx, y1 = cy + sy;
      const bool inx = (unsigned)x1 < (unsigned)W, iny = (unsigned)y1 < (unsigned)H;
      int best = -1;
      if (inx && occ_at(bits, tpr, x1, cy)) best = cy * W + x1;
      if (iny && occ_at(bits, tpr, cx, y1)) {
        const int li = y1 * W + cx;
        if (best < 0 || li < best) best = li;
      }
      if (inx && iny && occ_at(bits, tpr, x1, y1)) {
        const int li = y1 * W + x1;
        if (best < 0 || li < best) best = li;
      }
      cx = x1; cy = y1; ++nx; ++ny; ++nc; D += dA - dB;
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
  *steps = nx + ny - nc;   // loop iterations (a corner enters three cells at once)
  return z;
}

__global__ __launch_bounds__(RT) void raycast_smad_kernel(RayArgs a) {
  extern __shared__ double S[];   // [Ns + 1]: S[j + 1] = range j, then prefix sums
  __shared__ double wsum[RT / 64];
  __shared__ double rv[RT / 64];
  __shared__ int rm[RT / 64];
  const int h = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int Ns = a.Ns;
  const int ix0 = a.hyp_xy[2 * h], iy0 = a.hyp_xy[2 * h + 1];

  for (int j = tid; j < Ns; j += RT) {
    const int2 U = a.dirs[j];
    const float2 kk = a.kap[j];
    int hit, steps;
    const float z = cast_ray(a.bits, a.W, a.H, a.tpr, ix0, iy0, U.x, U.y, kk.x, kk.y, a.rmax,
                             a.rcells, &hit, &steps);
    S[j + 1] = (double)z;
    if (a.dbg_hit) a.dbg_hit[(size_t)h * Ns + j] = hit;
    if (a.dbg_rng) a.dbg_rng[(size_t)h * Ns + j] = z;
    if (a.dbg_steps) a.dbg_steps[(size_t)h * Ns + j] = steps;
  }
  __syncthreads();

  // inclusive prefix sums over S[1 .. Ns], one contiguous chunk per thread
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

  // eq. 18-19 for every shift m; C(t) is the prefix sum of the cyclically
  // extended scan (eq. 17), t < 3 Ns
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
  // (value, smallest m) minimum over the workgroup
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

}  // namespace

hipError_t launch_raycast_smad(const RayArgs& a, hipStream_t s) {
  if (a.n_hyp <= 0) return hipSuccess;
  const size_t lds = (size_t)(a.Ns + 1) * sizeof(double);
  hipLaunchKernelGGL(raycast_smad_kernel, dim3(a.n_hyp), dim3(RT), lds, s, a);
  return hipGetLastError();
}

}  // namespace reloc
