// Plain, slow, FP64 CPU oracle of the relocalization hot path.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes
// or calls this file; only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load it (through oracle/__init__.py).
// It shares no code, header, table or constant generator with the HIP path.
//
// Every function follows the paper's definitions step by step; where the
// paper is silent the documented reading is implemented and named at the
// function. Section / equation references are to arXiv 2511.01219.
//
// Build: g++ -O2 -std=c++17 -fopenmp -shared -fPIC (see oracle/build.py).
// Deliberately no -ffast-math: the FP64 and FP32 arithmetic below is meant
// to be IEEE round-to-nearest, one operation at a time.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <queue>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef int64_t i64;
typedef uint64_t u64;

inline bool is_occ(int8_t v, int thr) { return (int)v >= thr; }
inline bool is_free(int8_t v, int thr) { return v >= 0 && (int)v < thr; }

i64 floor_div(i64 a, i64 b) {  // b > 0
  i64 q = a / b;
  if ((a % b) != 0 && (a < 0)) --q;
  return q;
}

// splitmix64 output function (Steele, Lea & Flood 2014): the published
// constants, applied to x + golden gamma.
u64 mix64(u64 x) {
  u64 z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

i64 gcd64(i64 a, i64 b) { while (b) { i64 t = a % b; a = b; b = t; } return a; }

}  // namespace

extern "C" {

// The sampler's priority function on its own (known-answer tests).
u64 orc_mix64(u64 x) { return mix64(x); }

// ---------------------------------------------------------------------------
// Euclidean distance transform (Sec. III-A, MinDistToObstacle: a
// precomputed EDT lookup table). Definition: k[c] = min over occupied cells o
// of (dx^2 + dy^2) between cell indices; -1 when the map has no occupied
// cell. Unknown cells (< 0) are not obstacles.
// ---------------------------------------------------------------------------

// Brute force over every occupied cell (tiny maps only).
int orc_edt_brute(int W, int H, const int8_t* occ, int thr, i64* k) {
  std::vector<int> ox, oy;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      if (is_occ(occ[(i64)y * W + x], thr)) { ox.push_back(x); oy.push_back(y); }
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      i64 best = -1;
      for (size_t i = 0; i < ox.size(); ++i) {
        i64 dx = x - ox[i], dy = y - oy[i];
        i64 d = dx * dx + dy * dy;
        if (best < 0 || d < best) best = d;
      }
      k[(i64)y * W + x] = best;
    }
  return 0;
}

// Separable exact EDT: per-column 1-D distance g, then per row the lower
// envelope of the parabolas (x - q)^2 + g(q)^2 (Felzenszwalb & Huttenlocher
// 2012), with every intersection compared in exact integer arithmetic.
int orc_edt(int W, int H, const int8_t* occ, int thr, i64* k) {
  const i64 INF = std::numeric_limits<i64>::max() / 4;
  std::vector<i64> g((size_t)W * H);
  bool any = false;
#pragma omp parallel for schedule(static) reduction(|| : any)
  for (int x = 0; x < W; ++x) {
    i64 last = -1;
    for (int y = 0; y < H; ++y) {
      if (is_occ(occ[(i64)y * W + x], thr)) { last = y; any = true; }
      g[(i64)y * W + x] = last < 0 ? INF : (y - last);
    }
    last = -1;
    for (int y = H - 1; y >= 0; --y) {
      if (is_occ(occ[(i64)y * W + x], thr)) last = y;
      if (last >= 0) {
        i64 d = last - y;
        if (d < g[(i64)y * W + x]) g[(i64)y * W + x] = d;
      }
    }
  }
  if (!any) {
    for (i64 i = 0; i < (i64)W * H; ++i) k[i] = -1;
    return 0;
  }
#pragma omp parallel
  {
    std::vector<int> v(W);
    std::vector<i64> f(W);
#pragma omp for schedule(static)
    for (int y = 0; y < H; ++y) {
      // f(q) = g(q)^2, only finite parabolas participate.
      int n = 0;  // number of parabolas in the envelope
      for (int q = 0; q < W; ++q) {
        i64 gq = g[(i64)y * W + q];
        f[q] = gq >= INF ? INF : gq * gq;
      }
      // z boundaries stored as rationals num/den (den > 0).
      std::vector<i64> zn(W + 1), zd(W + 1);
      for (int q = 0; q < W; ++q) {
        if (f[q] >= INF) continue;
        if (n == 0) { v[0] = q; n = 1; zn[0] = -INF; zd[0] = 1; continue; }
        while (true) {
          int p = v[n - 1];
          // intersection s of parabolas p and q: ((f[q]+q^2)-(f[p]+p^2)) / (2q-2p)
          i64 sn = (f[q] + (i64)q * q) - (f[p] + (i64)p * p);
          i64 sd = 2 * (i64)(q - p);
          // pop while s <= z[n-1]
          bool le;
          if (zn[n - 1] == -INF) le = false;
          else le = (__int128)sn * zd[n - 1] <= (__int128)zn[n - 1] * sd;
          if (le) { --n; if (n == 0) break; continue; }
          v[n] = q; zn[n] = sn; zd[n] = sd; ++n;
          break;
        }
        if (n == 0) { v[0] = q; n = 1; zn[0] = -INF; zd[0] = 1; }
      }
      int j = 0;
      for (int x = 0; x < W; ++x) {
        // advance while z[j+1] < x   (z[j+1] = zn/zd)
        while (j + 1 < n && (__int128)zn[j + 1] < (__int128)x * zd[j + 1]) ++j;
        i64 dx = x - v[j];
        k[(i64)y * W + x] = dx * dx + f[v[j]];
      }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Direction table shared as a definition (not as code) with the library:
// for the turn fraction t/Ng reduced to lowest terms p/q,
// U[t] = round-half-even(2^20 * (cos a, sin a)), a = (2*pi*p)/q in FP64 with
// the C library. Reducing the fraction makes a direction independent of the
// grid it is indexed in. Beam / heading directions of eq. 13-15 and eq. 22
// are indices into this table.
// ---------------------------------------------------------------------------
void orc_dirs(int Ng, int32_t* U) {
  for (int t = 0; t < Ng; ++t) {
    const i64 g = gcd64(t, Ng);
    const i64 p = t / g, q = Ng / g;
    double a = (2.0 * M_PI * (double)p) / (double)q;
    U[2 * t] = (int32_t)std::llrint(std::ldexp(std::cos(a), 20));
    U[2 * t + 1] = (int32_t)std::llrint(std::ldexp(std::sin(a), 20));
  }
}

// Range scale for a ray direction U along one axis: metres per Q8 unit of
// travel along that axis, rounded to FP32 after an FP64 evaluation in this
// exact operation order.
static float kappa(int32_t ua, int32_t ub, double res) {
  double a = std::fabs((double)ua);
  double n = std::sqrt((double)ua * (double)ua + (double)ub * (double)ub);
  return (float)(((res / 256.0) * n) / a);
}

// ---------------------------------------------------------------------------
// Ray casting of the panoramic synthetic scan (eq. 13-14). The paper only
// says "ray casting"; the reading used here: the ray leaves the hypothesis
// cell centre (Q8 fixed point X = 256*ix + 128) along the integer direction
// U and visits every cell whose CLOSED box it meets (supercover). The hit is
// the first occupied visited cell; among occupied cells entered at the same
// parameter the smallest linear index wins. The range is the distance to the
// entry boundary, fl32(fl32(delta) * kappa_axis), delta being the Q8 offset
// along the entry axis (x at a corner). No hit inside the map, or a range
// above fl32(range_max), gives the placeholder 0 and hit -1.
//
// This version merges the exact crossing parameters of the x and y grid
// lines, t_x(n) = (128 + 256 (n-1)) / |Ux|, t_y(m) = (128 + 256 (m-1)) / |Uy|,
// comparing them by cross-multiplication.
// ---------------------------------------------------------------------------
static void cast_one(int W, int H, const int8_t* occ, int thr, int ix0, int iy0,
                     int32_t ux, int32_t uy, double res, float rmax_f, i64 rcells,
                     int32_t* hit, float* rng) {
  const i64 ax = ux < 0 ? -(i64)ux : ux, ay = uy < 0 ? -(i64)uy : uy;
  const int sx = ux > 0 ? 1 : (ux < 0 ? -1 : 0);
  const int sy = uy > 0 ? 1 : (uy < 0 ? -1 : 0);
  const float kx = ax ? kappa(ux, uy, res) : 0.f;
  const float ky = ay ? kappa(uy, ux, res) : 0.f;
  i64 n = 1, m = 1;
  int cx = ix0, cy = iy0;
  *hit = -1;
  *rng = 0.f;
  while (true) {
    i64 px = 128 + 256 * (n - 1), py = 128 + 256 * (m - 1);
    int cmp;
    if (ax == 0) cmp = 1;
    else if (ay == 0) cmp = -1;
    else {
      i64 l = px * ay, r = py * ax;
      cmp = l < r ? -1 : (l > r ? 1 : 0);
    }
    int ex[3], ey[3], ne = 0;
    i64 delta;
    bool xaxis;
    if (cmp < 0) {
      ex[0] = cx + sx; ey[0] = cy; ne = 1; delta = px; xaxis = true; cx += sx; ++n;
    } else if (cmp > 0) {
      ex[0] = cx; ey[0] = cy + sy; ne = 1; delta = py; xaxis = false; cy += sy; ++m;
    } else {
      ex[0] = cx + sx; ey[0] = cy;
      ex[1] = cx;      ey[1] = cy + sy;
      ex[2] = cx + sx; ey[2] = cy + sy;
      ne = 3; delta = px; xaxis = true; cx += sx; cy += sy; ++n; ++m;
    }
    i64 best = -1;
    bool out = false;
    for (int e = 0; e < ne; ++e) {
      if (ex[e] < 0 || ex[e] >= W || ey[e] < 0 || ey[e] >= H) { out = true; continue; }
      i64 li = (i64)ey[e] * W + ex[e];
      if (is_occ(occ[li], thr) && (best < 0 || li < best)) best = li;
    }
    if (best >= 0) {
      float z = (float)delta * (xaxis ? kx : ky);
      if (z <= rmax_f) { *hit = (int32_t)best; *rng = z; }
      return;
    }
    if (out) return;
    i64 cheb = std::max<i64>(std::llabs(cx - ix0), std::llabs(cy - iy0));
    if (cheb > rcells) return;   // every later entry lies beyond range_max
  }
}

// Brute-force version for tiny maps: the entry parameter of the ray into the
// closed box of EVERY occupied cell by exact slab intersection, the minimum
// over cells (ties: smallest index), then the map-exit rule.
static void cast_brute(int W, int H, const int8_t* occ, int thr, int ix0, int iy0,
                       int32_t ux, int32_t uy, double res, float rmax_f,
                       int32_t* hit, float* rng) {
  const i64 X = 256 * (i64)ix0 + 128, Y = 256 * (i64)iy0 + 128;
  *hit = -1;
  *rng = 0.f;
  // rational t = num/den with den > 0
  struct R { i64 n, d; };
  auto lt = [](R a, R b) { return (__int128)a.n * b.d < (__int128)b.n * a.d; };
  auto eq = [](R a, R b) { return (__int128)a.n * b.d == (__int128)b.n * a.d; };
  auto slab = [&](i64 P, i64 u, i64 lo, i64 hi, R& tlo, R& thi, bool& inf) -> bool {
    // returns false if no intersection; inf=true means unbounded slab
    if (u == 0) { inf = true; return P >= lo && P <= hi; }
    inf = false;
    i64 au = u < 0 ? -u : u;
    i64 a = (lo - P) * (u < 0 ? -1 : 1), b = (hi - P) * (u < 0 ? -1 : 1);
    if (a > b) std::swap(a, b);
    tlo = R{a, au}; thi = R{b, au};
    return true;
  };
  // map exit parameter: first t > 0 at which the ray reaches the boundary of
  // [0, 256W] x [0, 256H]
  R texit{0, 0};
  bool have_exit = false;
  {
    R cand[2]; int nc = 0;
    if (ux > 0) cand[nc++] = R{256 * (i64)W - X, ux};
    if (ux < 0) cand[nc++] = R{X, -(i64)ux};
    if (uy > 0) cand[nc++] = R{256 * (i64)H - Y, uy};
    if (uy < 0) cand[nc++] = R{Y, -(i64)uy};
    for (int i = 0; i < nc; ++i)
      if (!have_exit || lt(cand[i], texit)) { texit = cand[i]; have_exit = true; }
  }
  R tbest{0, 1};
  i64 best = -1;
  bool best_x = true;
  i64 best_delta = 0;
  for (int oy = 0; oy < H; ++oy)
    for (int ox = 0; ox < W; ++ox) {
      i64 li = (i64)oy * W + ox;
      if (!is_occ(occ[li], thr) || (ox == ix0 && oy == iy0)) continue;
      R xl{0, 1}, xh{0, 1}, yl{0, 1}, yh{0, 1};
      bool xi, yi;
      if (!slab(X, ux, 256 * (i64)ox, 256 * (i64)(ox + 1), xl, xh, xi)) continue;
      if (!slab(Y, uy, 256 * (i64)oy, 256 * (i64)(oy + 1), yl, yh, yi)) continue;
      R tin, tout;
      bool xent;
      if (xi) { tin = yl; xent = false; }
      else if (yi) { tin = xl; xent = true; }
      else if (lt(yl, xl)) { tin = xl; xent = true; }
      else if (lt(xl, yl)) { tin = yl; xent = false; }
      else { tin = xl; xent = true; }  // corner: x formula
      if (xi) tout = yh; else if (yi) tout = xh; else tout = lt(xh, yh) ? xh : yh;
      if (lt(tout, tin)) continue;
      if (tin.n <= 0) continue;  // only the start cell contains t <= 0
      if (have_exit && lt(texit, tin)) continue;
      if (best < 0 || lt(tin, tbest) || (eq(tin, tbest) && li < best)) {
        best = li; tbest = tin; best_x = xent;
        best_delta = tin.n;  // numerator = |boundary - P| along the entry axis
      }
    }
  if (best < 0) return;
  float kx = kappa(ux, uy, res);
  float ky = kappa(uy, ux, res);
  if (!best_x) kx = ky;
  // the numerator of t is the Q8 offset only when den = |U_axis|
  float z = (float)best_delta * kx;
  if (z <= rmax_f) { *hit = (int32_t)best; *rng = z; }
}

// For every hypothesis cell and every panoramic direction j < Ns (direction
// index j * (Ng / Ns) of the table), the hit cell and range.
int orc_raycast(int W, int H, const int8_t* occ, int thr, int Ng, int Ns,
                double res, float range_max, int n_hyp, const int32_t* hyp_xy,
                int brute, int32_t* hit, float* rng, int threads) {
  if (Ng % Ns) return -1;
  std::vector<int32_t> U(2 * (size_t)Ng);
  orc_dirs(Ng, U.data());
  const int b = Ng / Ns;
  const i64 rcells = (i64)std::ceil((double)range_max / res) + 2;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int h = 0; h < n_hyp; ++h)
    for (int j = 0; j < Ns; ++j) {
      int32_t ux = U[2 * (size_t)j * b], uy = U[2 * (size_t)j * b + 1];
      size_t o = (size_t)h * Ns + j;
      if (brute)
        cast_brute(W, H, occ, thr, hyp_xy[2 * h], hyp_xy[2 * h + 1], ux, uy, res,
                   range_max, &hit[o], &rng[o]);
      else
        cast_one(W, H, occ, thr, hyp_xy[2 * h], hyp_xy[2 * h + 1], ux, uy, res,
                 range_max, rcells, &hit[o], &rng[o]);
    }
  return 0;
}

// ---------------------------------------------------------------------------
// Scan preprocessing (eq. 11, 12, 14, 16, 25, 26 and the invalid-beam
// placeholder of Sec. III-B).
//   * downsample by n_skip (eq. 11); beam i' has robot-frame angle
//     angle_min + (i' * n_skip) * angle_increment;
//   * Ns = 2*pi / (angle_increment * n_skip) must be an integer (eq. 14) and
//     angle_min a multiple of the step, both within 1e-6 * Ns;
//   * FoV beams: angle inside some [lo, hi] (all beams when no interval);
//     valid: FoV, finite, range_min <= z <= range_max;
//   * z' = z if valid else 0; N_FoV counts FoV beams (placeholders too);
//     zbar = sum of z' over FoV beams in index order / N_FoV (eq. 16);
//   * lambda = N_FoV / Ns; N'_Z = number of valid beams;
//     k_mid = floor(N'_Z * (A0*Ns + (A1-A0)*N_FoV) / (1000*Ns)) with
//     (A0, A1) the per-mille alpha_mid at lambda = 0 and 1 (eq. 25-26), same
//     for k_low;
//   * TAM range in Q8 cells: zq = rint(z * 256 / res).
// info: [0] status [1] Ns [2] Ntheta [3] Ng [4] N_FoV [5] N'_Z [6] k_full
//       [7] k_mid [8] k_low [9] panoramic (10*N_FoV >= 9*Ns) [10] n_runs
//       [11] j0 [12] N' (beams after downsampling) [13] number of SMAD shifts
// dinfo: [0] zbar [1] lambda
// beam_j[N'], beam_state[N'] (0 outside FoV, 1 FoV invalid, 2 valid),
// beam_z[N'] (z' as FP64), beam_zq[N'] (valid beams only, else 0)
// ---------------------------------------------------------------------------
int orc_prep(int n_beams, const float* ranges, double angle_min, double angle_inc,
             int n_fov, const double* fov_lo, const double* fov_hi,
             float range_min, float range_max, int n_skip_beam, int n_skip_enum,
             int n_theta, double res, const int32_t* alpha_mid_pm,
             const int32_t* alpha_low_pm, i64* info, double* dinfo,
             int32_t* beam_j, int32_t* beam_state, double* beam_z, int32_t* beam_zq) {
  for (int i = 0; i < 16; ++i) info[i] = 0;
  if (n_beams <= 0 || n_skip_beam <= 0 || n_skip_enum <= 0 || !(angle_inc > 0)) return info[0] = -1;
  const double step = angle_inc * (double)n_skip_beam;
  const double r = (2.0 * M_PI) / step;
  const i64 Ns = std::llround(r);
  if (Ns < 1 || std::fabs(r - (double)Ns) > 1e-6 * (double)Ns) return info[0] = -4;
  const double j0r = angle_min / step;
  const i64 j0 = std::llround(j0r);
  if (std::fabs(j0r - (double)j0) > 1e-6 * (double)Ns) return info[0] = -4;
  const int nd = (n_beams + n_skip_beam - 1) / n_skip_beam;
  if (nd > Ns) return info[0] = -4;
  const i64 Nt = n_theta > 0 ? n_theta : Ns;
  const i64 Ng = Ns / gcd64(Ns, Nt) * Nt;
  i64 nfov = 0, nvalid = 0, runs = 0;
  bool prev = false;
  double sum = 0.0;
  for (int i = 0; i < nd; ++i) {
    const int src = i * n_skip_beam;
    const double phi = angle_min + (double)src * angle_inc;
    bool in = (n_fov <= 0);
    for (int f = 0; f < n_fov && !in; ++f) in = (fov_lo[f] <= phi && phi <= fov_hi[f]);
    const float z = ranges[src];
    const bool valid = in && std::isfinite(z) && z >= range_min && z <= range_max;
    beam_j[i] = (int32_t)(((j0 + i) % Ns + Ns) % Ns);
    beam_state[i] = in ? (valid ? 2 : 1) : 0;
    beam_z[i] = valid ? (double)z : 0.0;
    beam_zq[i] = valid ? (int32_t)std::llrint(((double)z * 256.0) / res) : 0;
    if (in) { ++nfov; sum += beam_z[i]; if (!prev) ++runs; }
    if (valid) ++nvalid;
    prev = in;
  }
  if (nfov == 0 || nvalid == 0) return info[0] = -5;
  const i64 a0 = alpha_mid_pm[0], a1 = alpha_mid_pm[1];
  const i64 b0 = alpha_low_pm[0], b1 = alpha_low_pm[1];
  // eq. 25: alpha_low < alpha_mid (< alpha_full = 1) at every lambda
  if (b0 > a0 || b1 > a1) return info[0] = -1;
  const i64 kmid = (nvalid * (a0 * Ns + (a1 - a0) * nfov)) / (1000 * Ns);
  const i64 klow = (nvalid * (b0 * Ns + (b1 - b0) * nfov)) / (1000 * Ns);
  info[1] = Ns; info[2] = Nt; info[3] = Ng; info[4] = nfov; info[5] = nvalid;
  info[6] = nvalid; info[7] = kmid; info[8] = klow;
  info[9] = (10 * nfov >= 9 * Ns) ? 1 : 0;
  info[10] = runs; info[11] = ((j0 % Ns) + Ns) % Ns; info[12] = nd;
  info[13] = info[9] ? 1 : (Ns + n_skip_enum - 1) / n_skip_enum;
  dinfo[0] = sum / (double)nfov;
  dinfo[1] = (double)nfov / (double)Ns;
  if (kmid < 1 || klow < 1) return info[0] = -5;
  return 0;
}

// ---------------------------------------------------------------------------
// SMAD (eq. 16-20), "without prefix sums": every shift m is summed directly.
//   zsyn(m) = (sum over FoV beams i of zhat[(j_i + m) mod Ns]) / N_FoV
//   SMAD(m) = |zbar - zsyn(m)|,  m = 0, n_enum, 2 n_enum, ... < Ns (eq. 15)
//   SMAD(p) = SMAD(0) if 10 N_FoV >= 9 Ns (eq. 20, lambda >= 0.9), else the
//   minimum over m (ties: smallest m).
// zhat: [n_hyp][Ns] synthetic ranges; fov_j: panoramic index of each FoV beam.
// all_out (optional): [n_hyp][n_shifts] every SMAD(p, theta_m).
// ---------------------------------------------------------------------------
int orc_smad(int n_hyp, int Ns, const float* zhat, int n_fov_beams,
             const int32_t* fov_j, double zbar, int n_enum, int panoramic,
             double* smad, int32_t* argm, double* all_out, int threads) {
  const int nsh = panoramic ? 1 : (Ns + n_enum - 1) / n_enum;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(static)
  for (int h = 0; h < n_hyp; ++h) {
    const float* z = zhat + (size_t)h * Ns;
    double best = 0.0;
    int bm = -1;
    for (int s = 0; s < nsh; ++s) {
      const int m = s * n_enum;
      double acc = 0.0;
      for (int i = 0; i < n_fov_beams; ++i) acc += (double)z[(fov_j[i] + m) % Ns];
      const double zs = acc / (double)n_fov_beams;
      const double v = std::fabs(zbar - zs);
      if (all_out) all_out[(size_t)h * nsh + s] = v;
      if (bm < 0 || v < best) { best = v; bm = m; }
    }
    smad[h] = best;
    argm[h] = bm;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// CAER (eq. 21, Remark 5), the beam-level coarse metric of the ablation:
//   CAER(m) = (sum over FoV beams i, in FoV order, of
//              |z'_i - zhat[(j_i + m) mod Ns]|) / N_FoV,
// z'_i the measured range of FoV beam i (0 when invalid), m = 0, n_enum,
// 2 n_enum, ... < Ns. Unlike SMAD it is not rotation invariant, so every
// shift is scored even for panoramic scans; CAER(p) = min over m (ties:
// smallest m).
// ---------------------------------------------------------------------------
int orc_caer(int n_hyp, int Ns, const float* zhat, int n_fov_beams, const int32_t* fov_j,
             const double* fov_z, int n_enum, double* caer, int32_t* argm, double* all_out,
             int threads) {
  const int nsh = (Ns + n_enum - 1) / n_enum;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(static)
  for (int h = 0; h < n_hyp; ++h) {
    const float* z = zhat + (size_t)h * Ns;
    double best = 0.0;
    int bm = -1;
    for (int s = 0; s < nsh; ++s) {
      const int m = s * n_enum;
      double acc = 0.0;
      for (int i = 0; i < n_fov_beams; ++i)
        acc += std::fabs(fov_z[i] - (double)z[(fov_j[i] + m) % Ns]);
      const double v = acc / (double)n_fov_beams;
      if (all_out) all_out[(size_t)h * nsh + s] = v;
      if (bm < 0 || v < best) { best = v; bm = m; }
    }
    caer[h] = best;
    argm[h] = bm;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// TAM at pose (p, theta_k) (eq. 22-31), literal.
//   endpoint of valid beam v at heading k: direction t = (b*j_v + o*k) mod Ng
//   with b = Ng/Ns, o = Ng/Ntheta; e = floor((X*2^20 + zq*U_t) / 2^28) per
//   axis (exact integers); d = sqrt(k_EDT[e]) * res, or d_max off the map;
//   l = ln(z_hit * exp(-d^2 / (2 sigma^2)) + z_rand + 1e-6)          (23)
//   sorted descending (24); means of the top k_full, k_mid, k_low (26);
//   Lbar = their median (27); P = exp(Lbar) (28);
//   dbar, population variance of d (two passes); dt = clamp(dbar, res/2,
//   d_max); s_d = 1 - (dt - res/2)/(d_max - res/2) (29); c = exp(-var/2)
//   (30); T = cbrt(P * s_d * c) (31).
// out[11*i + 0..10] = T, P, s_d, c, Lbar, mean top-k_full, top-k_mid,
// top-k_low, and the ablation metrics of Sec. IV (Case 3):
//   LF = sum of l_i over the N'_Z valid beams (eq. 32, in beam order);
//   baseline = (exp(LF / N'_Z) s_d)^(1/2) (eq. 33);
//   T_mean = (P + s_d + c) / 3 (eq. 34);
// for query i = (cell, heading k).
// ---------------------------------------------------------------------------
struct TamCtx {
  int W, H; const i64* kmap; double res;
  int Ns, Nt, Ng; const int32_t* U;
  int nv; const int32_t* vj; const int32_t* vzq;
  i64 kfull, kmid, klow;
  double z_hit, sigma, z_rand, d_max;
  int fine;   // score that picks theta* and ranks poses: 0 T, 1 T_mean, 2 baseline, 3 LF
};

constexpr int TOUT = 11;   // values per TAM evaluation
// column of tam_eval's output holding the score of each fine metric
inline int fine_col(int fine) { return fine == 1 ? 10 : fine == 2 ? 9 : fine == 3 ? 8 : 0; }

// The heading is given as its index g on the Ng direction grid: heading
// theta_k of eq. 22 is g = o*k; the local refinement below also visits the
// headings between them.
static void tam_eval(const TamCtx& c, int ix, int iy, i64 g, double* out,
                     std::vector<double>& l, std::vector<double>& d) {
  const i64 X = 256 * (i64)ix + 128, Y = 256 * (i64)iy + 128;
  const int b = c.Ng / c.Ns;
  l.resize(c.nv); d.resize(c.nv);
  for (int v = 0; v < c.nv; ++v) {
    const i64 t = ((i64)b * c.vj[v] + g) % c.Ng;
    const i64 ex = floor_div(X * (1LL << 20) + (i64)c.vzq[v] * c.U[2 * t], 1LL << 28);
    const i64 ey = floor_div(Y * (1LL << 20) + (i64)c.vzq[v] * c.U[2 * t + 1], 1LL << 28);
    double dist;
    if (ex >= 0 && ex < c.W && ey >= 0 && ey < c.H)
      dist = std::sqrt((double)c.kmap[ey * c.W + ex]) * c.res;
    else
      dist = c.d_max;
    d[v] = dist;
    l[v] = std::log(c.z_hit * std::exp(-(dist * dist) / (2.0 * c.sigma * c.sigma)) +
                    c.z_rand + 1e-6);
  }
  std::vector<double> s(l);
  std::sort(s.begin(), s.end(), [](double a, double b2) { return a > b2; });
  auto topmean = [&](i64 kk) {
    double acc = 0.0;
    for (i64 i = 0; i < kk; ++i) acc += s[i];
    return acc / (double)kk;
  };
  const double mf = topmean(c.kfull), mm = topmean(c.kmid), ml = topmean(c.klow);
  double m3[3] = {mf, mm, ml};
  std::sort(m3, m3 + 3);
  const double Lbar = m3[1];
  const double P = std::exp(Lbar);
  double dbar = 0.0;
  for (int v = 0; v < c.nv; ++v) dbar += d[v];
  dbar /= (double)c.nv;
  double var = 0.0;
  for (int v = 0; v < c.nv; ++v) var += (d[v] - dbar) * (d[v] - dbar);
  var /= (double)c.nv;
  const double dmin = c.res / 2.0;
  const double dt = std::min(std::max(dbar, dmin), c.d_max);
  const double sd = 1.0 - (dt - dmin) / (c.d_max - dmin);
  const double cc = std::exp(-0.5 * var);
  out[0] = std::cbrt(P * sd * cc);
  out[1] = P; out[2] = sd; out[3] = cc; out[4] = Lbar;
  out[5] = mf; out[6] = mm; out[7] = ml;
  double lf = 0.0;
  for (int v = 0; v < c.nv; ++v) lf += l[v];
  out[8] = lf;
  out[9] = std::sqrt(std::exp(lf / (double)c.nv) * sd);
  out[10] = (P + sd + cc) / 3.0;
}

int orc_tam(int W, int H, const i64* kmap, double res, int Ns, int Nt,
            int nv, const int32_t* vj, const int32_t* vzq, i64 kfull, i64 kmid, i64 klow,
            double z_hit, double sigma, double z_rand, double d_max,
            int nq, const int32_t* q_xy, const int32_t* q_k, double* out, int threads) {
  const i64 Ng = (i64)Ns / gcd64(Ns, Nt) * Nt;
  std::vector<int32_t> U(2 * (size_t)Ng);
  orc_dirs((int)Ng, U.data());
  TamCtx c{W, H, kmap, res, Ns, Nt, (int)Ng, U.data(), nv, vj, vzq, kfull, kmid, klow,
           z_hit, sigma, z_rand, d_max, 0};
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
  {
    std::vector<double> l, d;
#pragma omp for schedule(dynamic, 16)
    for (int i = 0; i < nq; ++i)
      tam_eval(c, q_xy[2 * i], q_xy[2 * i + 1], (Ng / Nt) * (i64)q_k[i],
               out + TOUT * (size_t)i, l, d);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Local refinement of a pose (Sec. III pipeline text: the top-k poses of a
// batch are refined by a local operator G and re-evaluated with TAM; Remark
// 2 names ICP as one such G). The paper fixes neither the operator nor its
// parameters. Reading used here: G is an exhaustive TAM search over the
// lattice of poses next to the pose (cell (ix, iy), heading index g0 on the
// Ng direction grid):
//   cells (ix + dx, iy + dy), |dx|, |dy| <= h; headings g0 + dg (mod Ng),
//   |dg| <= s; raster index q = ((dg + s)(2h + 1) + dy + h)(2h + 1) + dx + h.
// Lattice cells other than the pose's own cell that lie off the map or are
// occupied (EDT k == 0) are not visited, at any heading. The refined pose
// maximises T; among equal T the pose itself wins, then the smaller raster
// index.
// Because the pose itself is a lattice point, the refined T is never below
// its unrefined T.
// all (optional): [L] the T of every lattice point in raster order, NaN for
// the cells not visited.
// ---------------------------------------------------------------------------
static void refine_one(const TamCtx& c, int ix, int iy, i64 g0, int h, int s, double* bestT,
                       int* bdx, int* bdy, i64* bg, double* all, std::vector<double>& l,
                       std::vector<double>& d) {
  const int w = 2 * h + 1;
  double out[TOUT];
  const int col = fine_col(c.fine);
  double best = 0.0;
  i64 bkey = -1;
  for (int dg = -s; dg <= s; ++dg)
    for (int dy = -h; dy <= h; ++dy)
      for (int dx = -h; dx <= h; ++dx) {
        const i64 q = ((i64)(dg + s) * w + (dy + h)) * w + (dx + h);
        const bool own = dx == 0 && dy == 0, centre = own && dg == 0;
        const int x = ix + dx, y = iy + dy;
        if (!own && (x < 0 || x >= c.W || y < 0 || y >= c.H || c.kmap[(i64)y * c.W + x] == 0)) {
          if (all) all[q] = std::numeric_limits<double>::quiet_NaN();
          continue;
        }
        const i64 g = ((g0 + dg) % c.Ng + c.Ng) % c.Ng;
        tam_eval(c, x, y, g, out, l, d);
        if (all) all[q] = out[col];
        const i64 key = centre ? 0 : q + 1;
        if (bkey < 0 || out[col] > best || (out[col] == best && key < bkey)) {
          best = out[col];
          bkey = key;
          *bdx = dx;
          *bdy = dy;
          *bg = g;
        }
      }
  *bestT = best;
}

// Refinement of nq poses (cell q_xy, heading index q_g on the Ng grid) by
// the score of fine metric `fine`.
int orc_refine(int W, int H, const i64* kmap, double res, int Ns, int Nt,
               int nv, const int32_t* vj, const int32_t* vzq, i64 kfull, i64 kmid, i64 klow,
               double z_hit, double sigma, double z_rand, double d_max, int fine, int h, int s,
               int nq, const int32_t* q_xy, const i64* q_g, double* T, int32_t* dxy, i64* g,
               double* all, int threads) {
  const i64 Ng = (i64)Ns / gcd64(Ns, Nt) * Nt;
  std::vector<int32_t> U(2 * (size_t)Ng);
  orc_dirs((int)Ng, U.data());
  TamCtx c{W, H, kmap, res, Ns, Nt, (int)Ng, U.data(), nv, vj, vzq, kfull, kmid, klow,
           z_hit, sigma, z_rand, d_max, fine};
  const size_t L = (size_t)(2 * s + 1) * (2 * h + 1) * (2 * h + 1);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
  {
    std::vector<double> l, d;
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < nq; ++i)
      refine_one(c, q_xy[2 * i], q_xy[2 * i + 1], q_g[i], h, s, T + i, dxy + 2 * i,
                 dxy + 2 * i + 1, g + i, all ? all + L * i : nullptr, l, d);
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Batched multi-stage inference (Sec. III, Fig. 1 pipeline text; eq. 8-9,
// 22; early termination). Given the coarse score of every hypothesis (SMAD,
// or an ablation's CAER; all equal for no ordering) and the fine metric
// `fine` that stands for T below (0 TAM, 1 T_mean, 2 baseline, 3 LF):
//   order pi = ascending (SMAD, index); batch b = pi[bK, (b+1)K);
//   per hypothesis theta* = argmax_k T (ties: smallest k) (eq. 22);
//   batch best T*_b = max over the batch (ties: earlier rank); stop when
//   T*_b > tau (tau NaN: never); otherwise continue until exhausted.
// Local refinement (kr > 0): after a batch's TAM, its kr best hypotheses by
// (T* desc, rank asc) are refined by refine_one around (cell, o*k*) and
// their T* replaced by the refined T before the batch best is taken, so the
// threshold is tested on the best re-evaluated T. With kr == 0 the threshold
// is tested on the unrefined batch best.
// Outputs per rank r < n_eval: hyp[r] = pi[r], tstar[r] (refined T where
// refined), kstar[r]; ref[4r..4r+3] = (refined 1/0, dx, dy, heading index g
// on the Ng grid) with (0, 0, 0, o*k*) for unrefined ranks;
// stage_info: [0] stages run, [1] stopped early (1/0), [2] n_eval.
// all_T (optional): [n_eval][Nt] every (unrefined) TAM value, rank-major.
// ---------------------------------------------------------------------------
int orc_stages(int W, int H, const i64* kmap, double res, int Ns, int Nt,
               int nv, const int32_t* vj, const int32_t* vzq, i64 kfull, i64 kmid, i64 klow,
               double z_hit, double sigma, double z_rand, double d_max,
               int n_hyp, const int32_t* hyp_xy, const double* smad, int K, double tau,
               int fine, int kr, int rh, int rs, int32_t* order, double* tstar, int32_t* kstar,
               i64* ref, i64* stage_info, double* all_T, int threads) {
  std::vector<int32_t> pi(n_hyp);
  std::iota(pi.begin(), pi.end(), 0);
  std::stable_sort(pi.begin(), pi.end(), [&](int32_t a, int32_t b) {
    return smad[a] < smad[b] || (smad[a] == smad[b] && a < b);
  });
  for (int i = 0; i < n_hyp; ++i) order[i] = pi[i];
  const i64 Ng = (i64)Ns / gcd64(Ns, Nt) * Nt;
  std::vector<int32_t> U(2 * (size_t)Ng);
  orc_dirs((int)Ng, U.data());
  TamCtx c{W, H, kmap, res, Ns, Nt, (int)Ng, U.data(), nv, vj, vzq, kfull, kmid, klow,
           z_hit, sigma, z_rand, d_max, fine};
  const int col = fine_col(fine);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  int stages = 0, stopped = 0, n_eval = 0;
  for (int b0 = 0; b0 < n_hyp; b0 += K) {
    const int b1 = std::min(n_hyp, b0 + K);
#pragma omp parallel
    {
      std::vector<double> l, d;
      double out[TOUT];
#pragma omp for schedule(dynamic, 1)
      for (int r = b0; r < b1; ++r) {
        const int h = pi[r];
        double best = 0.0;
        int bk = -1;
        for (int k = 0; k < Nt; ++k) {
          tam_eval(c, hyp_xy[2 * h], hyp_xy[2 * h + 1], (Ng / Nt) * (i64)k, out, l, d);
          if (all_T) all_T[(size_t)r * Nt + k] = out[col];
          if (bk < 0 || out[col] > best) { best = out[col]; bk = k; }
        }
        tstar[r] = best;
        kstar[r] = bk;
      }
    }
    const i64 o = Ng / Nt;
    for (int r = b0; r < b1; ++r) {
      ref[4 * r] = 0; ref[4 * r + 1] = 0; ref[4 * r + 2] = 0;
      ref[4 * r + 3] = o * kstar[r];
    }
    if (kr > 0) {
      std::vector<int> sel(b1 - b0);
      std::iota(sel.begin(), sel.end(), b0);
      std::stable_sort(sel.begin(), sel.end(), [&](int a, int b2) { return tstar[a] > tstar[b2]; });
      const int nsel = std::min(kr, b1 - b0);
#pragma omp parallel
      {
        std::vector<double> l, d;
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < nsel; ++j) {
          const int r = sel[j];
          const int hh = pi[r];
          double T;
          int dx = 0, dy = 0;
          i64 g = 0;
          refine_one(c, hyp_xy[2 * hh], hyp_xy[2 * hh + 1], o * kstar[r], rh, rs, &T, &dx, &dy,
                     &g, nullptr, l, d);
          tstar[r] = T;
          ref[4 * r] = 1; ref[4 * r + 1] = dx; ref[4 * r + 2] = dy; ref[4 * r + 3] = g;
        }
      }
    }
    ++stages;
    n_eval = b1;
    double bb = tstar[b0];
    for (int r = b0 + 1; r < b1; ++r) if (tstar[r] > bb) bb = tstar[r];
    if (!std::isnan(tau) && bb > tau) { stopped = 1; break; }
  }
  stage_info[0] = stages; stage_info[1] = stopped; stage_info[2] = n_eval;
  return 0;
}

// ---------------------------------------------------------------------------
// Hypothesis sampling (replaces the RRT of Algorithm 1 with a deterministic
// integer sampler that keeps its constraints):
//   feasible: known-free cells with EDT k >= ceil((r_robot/res)^2 - 1e-9)
//     (TraversabilityCheck, d_obs >= r_robot, at cell centres);
//   reachable: the 4-connected feasible component of the cell of p0 (the
//     traversable set R(p0)); without p0, the largest component (ties: the
//     one containing the smallest cell index);
//   visiting order: ascending (splitmix64(seed + c), c);
//   accept c when every accepted c' has dx^2 + dy^2 >= ceil((rho/res)^2 -
//     1e-9) (VoxelDownsample spacing rho); stop at n_target.
// Output: accepted cells (x, y) in acceptance order.
// ---------------------------------------------------------------------------
int orc_sample(int W, int H, const int8_t* occ, int thr, const i64* kmap, double res,
               double ox, double oy, double min_spacing, double robot_radius,
               int has_p0, double p0x, double p0y, u64 seed, int n_target,
               int32_t* out_xy, int32_t* n_out) {
  *n_out = 0;
  const double qr = robot_radius / res, qs = min_spacing / res;
  const i64 Kr = (i64)std::ceil(qr * qr - 1e-9);
  const i64 S = (i64)std::ceil(qs * qs - 1e-9);
  const i64 N = (i64)W * H;
  std::vector<uint8_t> F(N);
  for (i64 c = 0; c < N; ++c) F[c] = is_free(occ[c], thr) && kmap[c] >= Kr;
  std::vector<int32_t> comp(N, -1);
  auto bfs = [&](i64 s, int id, std::vector<i64>* cells) {
    std::queue<i64> q;
    q.push(s); comp[s] = id;
    i64 count = 0;
    while (!q.empty()) {
      i64 c = q.front(); q.pop(); ++count;
      if (cells) cells->push_back(c);
      const int x = (int)(c % W), y = (int)(c / W);
      const int nx[4] = {x - 1, x + 1, x, x}, ny[4] = {y, y, y - 1, y + 1};
      for (int e = 0; e < 4; ++e) {
        if (nx[e] < 0 || nx[e] >= W || ny[e] < 0 || ny[e] >= H) continue;
        i64 n = (i64)ny[e] * W + nx[e];
        if (F[n] && comp[n] < 0) { comp[n] = id; q.push(n); }
      }
    }
    return count;
  };
  std::vector<i64> R;
  if (has_p0) {
    const i64 cx = (i64)std::floor((p0x - ox) / res), cy = (i64)std::floor((p0y - oy) / res);
    if (cx < 0 || cx >= W || cy < 0 || cy >= H) return -5;
    const i64 s = cy * W + cx;
    if (!F[s]) return -5;
    bfs(s, 0, &R);
  } else {
    i64 best = 0, best_s = -1;
    int id = 0;
    for (i64 c = 0; c < N; ++c)
      if (F[c] && comp[c] < 0) {
        i64 n = bfs(c, id++, nullptr);
        if (n > best) { best = n; best_s = c; }
      }
    if (best_s < 0) return -5;
    const int bid = comp[best_s];
    for (i64 c = 0; c < N; ++c) if (comp[c] == bid) R.push_back(c);
  }
  std::vector<std::pair<u64, i64>> ord(R.size());
  for (size_t i = 0; i < R.size(); ++i) ord[i] = {mix64(seed + (u64)R[i]), R[i]};
  std::sort(ord.begin(), ord.end());
  std::vector<uint8_t> blocked(N, 0);
  const int rad = (int)std::ceil(std::sqrt((double)S)) + 1;
  int n = 0;
  for (auto& pr : ord) {
    if (n >= n_target) break;
    const i64 c = pr.second;
    if (blocked[c]) continue;
    const int x = (int)(c % W), y = (int)(c / W);
    out_xy[2 * n] = x; out_xy[2 * n + 1] = y; ++n;
    for (int dy = -rad; dy <= rad; ++dy)
      for (int dx = -rad; dx <= rad; ++dx) {
        if ((i64)dx * dx + (i64)dy * dy >= S) continue;
        const int xx = x + dx, yy = y + dy;
        if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
        blocked[(i64)yy * W + xx] = 1;
      }
  }
  *n_out = n;
  return 0;
}

// ---------------------------------------------------------------------------
// Traversability-constrained RRT sampling (Algorithm 1, Sec. III-A items
// 1-7, Remark 4), literal, with a brute-force NearestNode. Readings where
// the paper is silent:
//   * random point: attempt t (counted over all rounds from 0) draws
//     u = (mix64(seed + 2t) >> 11) 2^-53 and v from seed + 2t + 1;
//     p_rand = (ox + u (W res), oy + v (H res)) (B = the map rectangle);
//   * NearestNode: smallest FP64 (dx*dx + dy*dy), ties: smallest node index;
//   * MinDistToObstacle(p) = sqrt(k) res of the cell holding p (EDT lookup);
//     no occupied cell at all: infinite;
//   * AdaptiveExpandDist: eta_max if d >= 2 r_robot, r_robot if d <= r_robot,
//     else r_robot + (eta_max - r_robot)(d - r_robot) / r_robot;
//   * ExtendPoint: p_rand itself when |p_rand - p_nearest| <= eta, else the
//     point at distance eta towards it (s = eta / L; p = p_near + s v);
//     L == 0 adds nothing;
//   * TraversabilityCheck: the points p_near + (i/n)(p_new - p_near),
//     i = 0..n, n = max(1, ceil(L / (res/2))), each in a known-free in-map
//     cell with k >= ceil((r_robot/res)^2 - 1e-9) (d_obs >= r_robot);
//   * VoxelDownsample: voxels of side rho from the map origin, each
//     represented by its first node (smallest index); gain = new voxels;
//   * the root p0 must pass the same cell test; rounds stop when gain <=
//     eps_gain, after max_rounds, or when the tree holds max_nodes nodes.
// Output: the nodes (x, y, parent) in insertion order, the representatives'
// cells in node order without repeated cells, and info = (rounds, attempts,
// nodes, N_sampling).
// ---------------------------------------------------------------------------
int orc_rrt(int W, int H, const int8_t* occ, int thr, const i64* kmap, double res, double ox,
            double oy, double p0x, double p0y, double rho, double r_robot, double eta_max,
            int eps_gain, u64 seed, int max_rounds, int max_nodes, double* nodes_xy,
            int32_t* parent, int32_t* cells_xy, i64* info) {
  for (int i = 0; i < 4; ++i) info[i] = 0;
  const double q = r_robot / res;
  const i64 Kr = (i64)std::ceil(q * q - 1e-9);
  auto cell_of = [&](double x, double y, i64* cx, i64* cy) {
    *cx = (i64)std::floor((x - ox) / res);
    *cy = (i64)std::floor((y - oy) / res);
  };
  auto feasible = [&](double x, double y) {
    i64 cx, cy;
    cell_of(x, y, &cx, &cy);
    if (cx < 0 || cx >= W || cy < 0 || cy >= H) return false;
    const i64 c = cy * W + cx;
    return is_free(occ[c], thr) && kmap[c] >= Kr;
  };
  if (!feasible(p0x, p0y)) return -5;
  const i64 N = (i64)std::ceil((double)W * (double)H * res * res / (rho * rho));
  info[3] = N;
  std::vector<double> nx{p0x}, ny{p0y};
  std::vector<int32_t> par{-1};
  const double wx = (double)W * res, wy = (double)H * res;
  const i64 VW = (i64)std::ceil(wx / rho) + 1;
  std::vector<int32_t> reps;         // representative node per voxel, in node order
  std::vector<uint8_t> have;         // voxel key -> represented
  const i64 VH = (i64)std::ceil(wy / rho) + 1;
  have.assign((size_t)(VW * VH), 0);
  size_t scanned = 0;                // nodes already downsampled
  i64 t = 0;
  int rounds = 0;
  bool full = false;
  while (true) {
    for (i64 i = 0; i < N && !full; ++i, ++t) {
      const double u = (double)(mix64(seed + 2 * (u64)t) >> 11) * (1.0 / 9007199254740992.0);
      const double v = (double)(mix64(seed + 2 * (u64)t + 1) >> 11) * (1.0 / 9007199254740992.0);
      const double rx = ox + u * wx, ry = oy + v * wy;
      // NearestNode (brute force)
      size_t best = 0;
      double bd = 0.0;
      for (size_t j = 0; j < nx.size(); ++j) {
        const double dx = nx[j] - rx, dy = ny[j] - ry;
        const double d2 = dx * dx + dy * dy;
        if (j == 0 || d2 < bd) { bd = d2; best = j; }
      }
      const double px = nx[best], py = ny[best];
      // AdaptiveExpandDist
      i64 cx, cy;
      cell_of(px, py, &cx, &cy);
      const i64 kk = kmap[cy * W + cx];
      const double d = kk < 0 ? INFINITY : std::sqrt((double)kk) * res;
      double eta;
      if (d >= 2.0 * r_robot) eta = eta_max;
      else if (d <= r_robot) eta = r_robot;
      else eta = r_robot + (eta_max - r_robot) * (d - r_robot) / r_robot;
      // ExtendPoint
      const double vx = rx - px, vy = ry - py;
      const double L = std::sqrt(vx * vx + vy * vy);
      if (L == 0.0) continue;
      double ex, ey;
      if (L <= eta) { ex = rx; ey = ry; }
      else { const double sc = eta / L; ex = px + vx * sc; ey = py + vy * sc; }
      // InSamplingBoundary and TraversabilityCheck
      if (!(ex >= ox && ex < ox + wx && ey >= oy && ey < oy + wy)) continue;
      const double sx = ex - px, sy = ey - py;
      const double Ls = std::sqrt(sx * sx + sy * sy);
      const i64 n = std::max<i64>(1, (i64)std::ceil(Ls / (0.5 * res)));
      bool ok = true;
      for (i64 k2 = 0; k2 <= n && ok; ++k2) {
        const double tt = (double)k2 / (double)n;
        ok = feasible(px + sx * tt, py + sy * tt);
      }
      if (!ok) continue;
      nx.push_back(ex);
      ny.push_back(ey);
      par.push_back((int32_t)best);
      if ((int)nx.size() >= max_nodes) full = true;
    }
    ++rounds;
    // VoxelDownsample over the new nodes (earlier voxels keep their node)
    i64 gain = 0;
    for (; scanned < nx.size(); ++scanned) {
      const i64 vx = (i64)std::floor((nx[scanned] - ox) / rho);
      const i64 vy = (i64)std::floor((ny[scanned] - oy) / rho);
      const i64 key = vy * VW + vx;
      if (!have[key]) { have[key] = 1; reps.push_back((int32_t)scanned); ++gain; }
    }
    if (gain <= eps_gain || rounds >= max_rounds || full) break;
  }
  for (size_t j = 0; j < nx.size(); ++j) {
    nodes_xy[2 * j] = nx[j];
    nodes_xy[2 * j + 1] = ny[j];
    parent[j] = par[j];
  }
  std::vector<uint8_t> used((size_t)W * H, 0);
  i64 nc = 0;
  for (int32_t r : reps) {
    i64 cx, cy;
    cell_of(nx[r], ny[r], &cx, &cy);
    const i64 c = cy * W + cx;
    if (used[c]) continue;
    used[c] = 1;
    cells_xy[2 * nc] = (int32_t)cx;
    cells_xy[2 * nc + 1] = (int32_t)cy;
    ++nc;
  }
  info[0] = rounds; info[1] = t; info[2] = (i64)nx.size();
  return (int)nc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
