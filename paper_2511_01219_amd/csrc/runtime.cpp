// Host runtime of libreloc: context, device memory accounting, map registry,
// hypothesis sampler, scan preprocessing and the staged relocalization driver.
// Every arithmetic step of the hot path runs in the HIP kernels; this file
// prepares their tables and sequences them on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "reloc.h"
#include "reloc_internal.h"

#include "runtime_internal.h"

namespace reloc {

namespace {
thread_local std::string g_err = "no error";
}  // namespace

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}



constexpr int kMaxNs = 4096;
constexpr int64_t kPlainFillBlocks = 4096;   // TAM workgroups one plain-path launch aims at
constexpr int64_t kPlainFirstFillBlocks = 1024;  // ... and its first launch
constexpr int kPlainMaxStages = 64;          // stages of a later plain-path launch, at most
constexpr int kMaxDim = 32767;
constexpr int kMaxNg = 1 << 20;

// ---- direction table -------------------------------------------------------
// U[t] for the turn fraction t / Ng reduced to lowest terms p / q:
// round-half-even(2^20 * (cos a, sin a)), a = (2 pi p) / q in FP64 (libm).
int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

std::vector<int2> direction_table(int Ng) {
  std::vector<int2> U(Ng);
  for (int t = 0; t < Ng; ++t) {
    const int64_t g = gcd64(t, Ng);
    const double a = (2.0 * M_PI * (double)(t / g)) / (double)(Ng / g);
    U[t].x = (int)std::llrint(std::ldexp(std::cos(a), 20));
    U[t].y = (int)std::llrint(std::ldexp(std::sin(a), 20));
  }
  return U;
}

// Metres travelled per Q8 unit of progress along axis a for direction (ua, ub).
float axis_scale(int ua, int ub, double res) {
  const double n = std::sqrt((double)ua * (double)ua + (double)ub * (double)ub);
  return (float)(((res / 256.0) * n) / std::fabs((double)ua));
}

// splitmix64 output function (Steele, Lea & Flood 2014).
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// ---- scan preprocessing (eq. 11-16, 25-26) ---------------------------------

int32_t preprocess(const reloc_scan* sc, const reloc_search_params* p, double res, Prep* out) {
  if (!sc || !p) return fail(RELOC_E_INVALID, "null scan or params");
  if (sc->n_beams <= 0 || !sc->ranges) return fail(RELOC_E_INVALID, "scan has no beams");
  if (p->n_skip_beam <= 0 || p->n_skip_enum <= 0)
    return fail(RELOC_E_INVALID, "n_skip_beam and n_skip_enum must be >= 1");
  if (!(sc->angle_increment > 0) || !std::isfinite(sc->angle_min))
    return fail(RELOC_E_INVALID, "angle_increment must be > 0");
  if (!(sc->range_max > 0) || !(sc->range_max < 64.f) || !(sc->range_min >= 0))
    return fail(RELOC_E_INVALID, "need 0 < range_max < 64 m and range_min >= 0");
  if (sc->n_fov < 0 || (sc->n_fov > 0 && !sc->fov))
    return fail(RELOC_E_INVALID, "bad FoV interval list");
  const double step = sc->angle_increment * (double)p->n_skip_beam;
  const double turns = (2.0 * M_PI) / step;
  const int64_t Ns = std::llround(turns);
  if (Ns < 1 || std::fabs(turns - (double)Ns) > 1e-6 * (double)Ns)
    return fail(RELOC_E_BEAMGRID, "2*pi / beam step = %.9f is not an integer", turns);
  if (Ns > kMaxNs) return fail(RELOC_E_INVALID, "Ns = %lld exceeds %d", (long long)Ns, kMaxNs);
  const double j0r = sc->angle_min / step;
  const int64_t j0 = std::llround(j0r);
  if (std::fabs(j0r - (double)j0) > 1e-6 * (double)Ns)
    return fail(RELOC_E_BEAMGRID, "angle_min is not on the beam grid");
  const int nd = (sc->n_beams + p->n_skip_beam - 1) / p->n_skip_beam;
  if (nd > Ns) return fail(RELOC_E_BEAMGRID, "more beams than grid directions");
  const int64_t Nt = p->n_theta > 0 ? p->n_theta : Ns;
  const int64_t Ng = Ns / gcd64(Ns, Nt) * Nt;
  if (Ng > kMaxNg) return fail(RELOC_E_INVALID, "lcm(Ns, n_theta) = %lld too large", (long long)Ng);

  Prep P;
  int64_t nfov = 0, nvalid = 0;
  double sum = 0.0;
  bool prev_in = false;
  for (int i = 0; i < nd; ++i) {
    const int src = i * p->n_skip_beam;
    const double phi = sc->angle_min + (double)src * sc->angle_increment;
    bool in = sc->n_fov == 0;
    for (int f = 0; f < sc->n_fov && !in; ++f) in = sc->fov[f].lo <= phi && phi <= sc->fov[f].hi;
    const int jj = (int)(((j0 + i) % Ns + Ns) % Ns);
    if (in) {
      const float z = sc->ranges[src];
      const bool ok = std::isfinite(z) && z >= sc->range_min && z <= sc->range_max;
      ++nfov;
      P.fj.push_back(jj);
      P.fz.push_back(ok ? (double)z : 0.0);
      if (ok) {
        sum += (double)z;
        ++nvalid;
        P.vj.push_back(jj);
        P.vzq.push_back((int32_t)std::llrint(((double)z * 256.0) / res));
      } else {
        sum += 0.0;
      }
      if (!prev_in) P.runs.push_back(make_int2(jj, 0));
      P.runs.back().y += 1;
    }
    prev_in = in;
  }
  if (nfov == 0) return fail(RELOC_E_EMPTY, "no beam inside the FoV");
  if (nvalid == 0) return fail(RELOC_E_EMPTY, "no valid beam");
  const int64_t a0 = p->alpha_mid_pm[0], a1 = p->alpha_mid_pm[1];
  const int64_t c0 = p->alpha_low_pm[0], c1 = p->alpha_low_pm[1];
  if (a0 < 1 || a0 > 1000 || a1 < 1 || a1 > 1000 || c0 < 1 || c0 > 1000 || c1 < 1 || c1 > 1000)
    return fail(RELOC_E_INVALID, "alpha per-mille values must be in [1, 1000]");
  // eq. 25 orders the fractions alpha_low < alpha_mid at every lambda; with
  // alpha_low <= alpha_mid at both ends, k_low <= k_mid for every FoV, which
  // is what makes the median of eq. 27 the top-k_mid mean
  if (c0 > a0 || c1 > a1)
    return fail(RELOC_E_INVALID, "alpha_low (%lld, %lld) must not exceed alpha_mid (%lld, %lld)",
                (long long)c0, (long long)c1, (long long)a0, (long long)a1);
  const int64_t kmid = (nvalid * (a0 * Ns + (a1 - a0) * nfov)) / (1000 * Ns);
  const int64_t klow = (nvalid * (c0 * Ns + (c1 - c0) * nfov)) / (1000 * Ns);
  if (kmid < 1 || klow < 1) return fail(RELOC_E_EMPTY, "too few valid beams for TAM");
  reloc_scan_info& I = P.info;
  I.Ns = (int)Ns;
  I.Ntheta = (int)Nt;
  I.Ng = (int)Ng;
  I.n_down = nd;
  I.n_fov = (int)nfov;
  I.n_valid = (int)nvalid;
  I.k_full = (int)nvalid;
  I.k_mid = (int)kmid;
  I.k_low = (int)klow;
  I.panoramic = (10 * nfov >= 9 * Ns) ? 1 : 0;
  I.n_runs = (int)P.runs.size();
  I.n_shifts = I.panoramic ? 1 : (int)((Ns + p->n_skip_enum - 1) / p->n_skip_enum);
  I.j0 = (int)(((j0 % Ns) + Ns) % Ns);
  I.zbar = sum / (double)nfov;
  I.lambda = (double)nfov / (double)Ns;
  *out = std::move(P);
  return RELOC_OK;
}

// ---- likelihood table for TAM (eq. 23) --------------------------------------

int32_t build_lut(const reloc_search_params* p, double res, Lut* L) {
  const double zh = p->z_hit, sg = p->sigma_hit, zr = p->z_rand, dm = p->d_max;
  if (!(zh >= 0 && zh <= 1e6) || !(sg > 0) || !(zr >= 0 && zr <= 1e6) || !(dm > res / 2.0))
    return fail(RELOC_E_INVALID, "need z_hit, z_rand in [0, 1e6], sigma_hit > 0, d_max > res/2");
  auto ell = [&](double d) { return std::log(zh * std::exp(-(d * d) / (2.0 * sg * sg)) + zr + 1e-6); };
  // smallest k where l(k) is within 1e-10 of its limit ln(z_rand + 1e-6)
  double need = 1.0;
  if (zh > 0) need = std::ceil((2.0 * sg * sg) / (res * res) * std::log(zh / (1e-10 * (zr + 1e-6))));
  int kcap = (int)std::min(32767.0, std::max(1.0, need));
  L->kcap = kcap;
  L->keybits = (2 * kcap + 2 <= 4096) ? 12 : 16;
  const int nk = 1 << L->keybits;
  L->q.assign(nk, 0);
  for (int k = 0; k <= kcap; ++k) {
    const double v = ell(std::sqrt((double)k) * res);
    L->q[2 * k] = (int32_t)std::llrint(v * 67108864.0);
    if (2 * k + 1 < nk) L->q[2 * k + 1] = L->q[2 * k];
  }
  const double koff = (dm / res) * (dm / res);
  if (koff >= (double)kcap) {
    L->key_off = 2 * kcap;
  } else {
    const int fk = (int)std::floor(koff);
    L->key_off = 2 * fk + 1;
    L->q[L->key_off] = (int32_t)std::llrint(ell(dm) * 67108864.0);
  }
  // reachable keys are 0 .. 2 kcap (key_off among them); the TAM kernels
  // add l - qmin (at most ln(1e12) in Q26, below 2^31) in 32 bits pairwise
  int32_t qmin = L->q[0];
  for (int k = 0; k <= 2 * kcap; ++k) qmin = std::min(qmin, L->q[k]);
  for (int k = 0; k <= 2 * kcap; ++k) L->q[k] -= qmin;
  L->qmin = qmin;
  return RELOC_OK;
}


// ============================================================================


int32_t set_device(reloc_ctx* c) {
  HIP_TRY(hipSetDevice(c->device));
  return RELOC_OK;
}

void release_request(reloc_ctx* c, Request& r) {
  drop_head(r);
  for (void* p : r.owned) c->dfree(p);
  r.owned.clear();
}

void drop_head(Request& r) {
  if (r.head) (void)hipGraphExecDestroy(r.head);
  r.head = nullptr;
}



int32_t ensure_khost(reloc_ctx* c, DevMap& m) {
  if (!m.khost.empty()) return RELOC_OK;
  m.khost.resize((size_t)m.W * m.H);
  HIP_TRY(hipMemcpyAsync(m.khost.data(), m.kmap, m.khost.size() * sizeof(uint32_t),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return RELOC_OK;
}

// Deterministic integer sampler (documented in reloc.h). Component search by
// breadth-first flood fill; the visiting order is produced chunk by chunk
// with nth_element; spacing is checked in a bucket grid of side
// ceil(sqrt(S)) cells, so only the 3 x 3 neighbouring buckets can conflict.
int32_t sample_cells(const DevMap& m, const reloc_sample_params* p, std::vector<int32_t>* out) {
  const int W = m.W, H = m.H;
  const double qr = p->robot_radius / m.res, qs = p->min_spacing / m.res;
  const int64_t Kr = (int64_t)std::ceil(qr * qr - 1e-9);
  const int64_t S = (int64_t)std::ceil(qs * qs - 1e-9);
  const int64_t N = (int64_t)W * H;
  std::vector<uint8_t> feas(N);
  for (int64_t c = 0; c < N; ++c) {
    const int8_t v = m.occ[c];
    feas[c] = (v >= 0 && (int)v < m.thr && (int64_t)m.khost[c] >= Kr) ? 1 : 0;
  }
  std::vector<int32_t> label(N, -1);
  std::vector<int64_t> queue;
  auto flood = [&](int64_t s, int id, std::vector<int64_t>* cells) -> int64_t {
    queue.clear();
    queue.push_back(s);
    label[s] = id;
    for (size_t qi = 0; qi < queue.size(); ++qi) {
      const int64_t c = queue[qi];
      const int x = (int)(c % W), y = (int)(c / W);
      if (x > 0 && feas[c - 1] && label[c - 1] < 0) { label[c - 1] = id; queue.push_back(c - 1); }
      if (x + 1 < W && feas[c + 1] && label[c + 1] < 0) { label[c + 1] = id; queue.push_back(c + 1); }
      if (y > 0 && feas[c - W] && label[c - W] < 0) { label[c - W] = id; queue.push_back(c - W); }
      if (y + 1 < H && feas[c + W] && label[c + W] < 0) { label[c + W] = id; queue.push_back(c + W); }
    }
    if (cells) *cells = queue;
    return (int64_t)queue.size();
  };
  std::vector<int64_t> region;
  if (p->has_p0) {
    const double fx = std::floor((p->p0_x - m.ox) / m.res), fy = std::floor((p->p0_y - m.oy) / m.res);
    if (!(fx >= 0 && fx < W && fy >= 0 && fy < H))
      return fail(RELOC_E_EMPTY, "p0 lies outside the map");
    const int64_t s = (int64_t)fy * W + (int64_t)fx;
    if (!feas[s]) return fail(RELOC_E_EMPTY, "p0 is not a feasible cell");
    flood(s, 0, &region);
  } else {
    int64_t best_n = 0, best_seed = -1;
    int id = 0;
    for (int64_t c = 0; c < N; ++c)
      if (feas[c] && label[c] < 0) {
        const int64_t n = flood(c, id++, nullptr);
        if (n > best_n) { best_n = n; best_seed = c; }
      }
    if (best_seed < 0) return fail(RELOC_E_EMPTY, "map has no feasible cell");
    const int bid = label[best_seed];
    region.reserve(best_n);
    for (int64_t c = 0; c < N; ++c)
      if (label[c] == bid) region.push_back(c);
  }
  std::vector<std::pair<uint64_t, int64_t>> cand(region.size());
  for (size_t i = 0; i < region.size(); ++i)
    cand[i] = {splitmix64(p->seed + (uint64_t)region[i]), region[i]};
  const int side = std::max<int>(1, (int)std::ceil(std::sqrt((double)S)));
  const int bw = (W + side - 1) / side, bh = (H + side - 1) / side;
  std::vector<std::vector<int32_t>> bucket((size_t)bw * bh);
  out->clear();
  size_t lo = 0;
  const size_t chunk = std::max<size_t>(65536, 8 * (size_t)p->n_target);
  while (lo < cand.size() && (int)(out->size() / 2) < p->n_target) {
    const size_t hi = std::min(cand.size(), lo + chunk);
    if (hi < cand.size())
      std::nth_element(cand.begin() + lo, cand.begin() + hi, cand.end());
    std::sort(cand.begin() + lo, cand.begin() + hi);
    for (size_t i = lo; i < hi && (int)(out->size() / 2) < p->n_target; ++i) {
      const int64_t c = cand[i].second;
      const int x = (int)(c % W), y = (int)(c / W);
      const int bx = x / side, by = y / side;
      bool ok = true;
      for (int yy = std::max(0, by - 1); yy <= std::min(bh - 1, by + 1) && ok; ++yy)
        for (int xx = std::max(0, bx - 1); xx <= std::min(bw - 1, bx + 1) && ok; ++xx)
          for (int32_t q : bucket[(size_t)yy * bw + xx]) {
            const int64_t dx = x - (*out)[2 * q], dy = y - (*out)[2 * q + 1];
            if (dx * dx + dy * dy < S) { ok = false; break; }
          }
      if (!ok) continue;
      bucket[(size_t)by * bw + bx].push_back((int32_t)(out->size() / 2));
      out->push_back(x);
      out->push_back(y);
    }
    lo = hi;
  }
  return RELOC_OK;
}

// Morton (Z-order) casting order of the cells xy[0, n), ties by index: the
// rays in flight on one XCD then start in one compact region of the map.
std::vector<int32_t> morton_order(const std::vector<int32_t>& xy, int n) {
  auto spread = [](uint32_t v) {
    v &= 0xFFFF;
    v = (v | (v << 8)) & 0x00FF00FF;
    v = (v | (v << 4)) & 0x0F0F0F0F;
    v = (v | (v << 2)) & 0x33333333;
    v = (v | (v << 1)) & 0x55555555;
    return v;
  };
  std::vector<std::pair<uint32_t, int32_t>> mc(n);
  for (int h = 0; h < n; ++h)
    mc[h] = {spread((uint32_t)xy[2 * h]) | (spread((uint32_t)xy[2 * h + 1]) << 1), h};
  std::sort(mc.begin(), mc.end());
  std::vector<int32_t> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = mc[i].second;
  return perm;
}

int32_t new_set(reloc_ctx* c, int map_id, std::vector<int32_t>&& xy, int32_t* set_id) {
  HypSet hs;
  hs.map_id = map_id;
  hs.n = (int)(xy.size() / 2);
  hs.host = std::move(xy);
  hs.morton = morton_order(hs.host, hs.n);
  hs.dev = (int32_t*)c->dalloc(std::max<size_t>(1, hs.host.size()) * sizeof(int32_t));
  hs.morton_dev = (int32_t*)c->dalloc(std::max<size_t>(1, hs.morton.size()) * sizeof(int32_t));
  if (!hs.dev || !hs.morton_dev) {
    c->dfree(hs.dev);
    c->dfree(hs.morton_dev);
    return RELOC_E_NOMEM;
  }
  int32_t e = upload(c, hs.dev, hs.host.data(), hs.host.size());
  if (e == RELOC_OK) e = upload(c, hs.morton_dev, hs.morton.data(), hs.morton.size());
  if (e == RELOC_OK && hipStreamSynchronize(c->stream) != hipSuccess) e = RELOC_E_DEVICE;
  if (e != RELOC_OK) {
    c->dfree(hs.dev);
    c->dfree(hs.morton_dev);
    return e;
  }
  const int id = c->next_id++;
  c->maps[map_id].n_sets += 1;
  std::lock_guard<std::mutex> rg(c->reg_mu);
  c->sets[id] = std::move(hs);
  *set_id = id;
  return RELOC_OK;
}

// Host image of several tables, each at a 256-byte aligned offset.
struct TableBlob {
  std::vector<uint8_t> b;
  template <typename T>
  size_t add(const std::vector<T>& v) {
    const size_t off = (b.size() + 255) & ~(size_t)255;
    b.resize(off + std::max<size_t>(1, v.size()) * sizeof(T));
    if (!v.empty()) std::memcpy(b.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

// Builds the request's device tables and work buffers.
// The direction tables of a beam grid, from the context's recent ones or
// built (and kept).
std::shared_ptr<const DirTables> dir_tables(reloc_ctx* c, int Ng, int Ns, double res) {
  {
    std::lock_guard<std::mutex> lk(c->lut_mu);
    for (auto it = c->dirs.begin(); it != c->dirs.end(); ++it)
      if ((*it)->Ng == Ng && (*it)->Ns == Ns && std::memcmp(&(*it)->res, &res, sizeof res) == 0) {
        std::shared_ptr<const DirTables> d = *it;
        if (it + 1 != c->dirs.end()) std::rotate(it, it + 1, c->dirs.end());
        return d;
      }
  }
  auto D = std::make_shared<DirTables>();
  D->Ng = Ng;
  D->Ns = Ns;
  D->res = res;
  D->U = direction_table(Ng);
  const int b = Ng / Ns;
  D->rd.resize(Ns);
  D->kp.resize(Ns);
  D->di.resize(Ns);
  D->df.resize(Ns);
  for (int j = 0; j < Ns; ++j) {
    const int2 u = D->U[(size_t)j * b];
    D->rd[j] = u;
    D->kp[j].x = u.x ? axis_scale(u.x, u.y, res) : 0.f;
    D->kp[j].y = u.y ? axis_scale(u.y, u.x, res) : 0.f;
    // per-direction constants of the skip traversal
    const int ax = std::abs(u.x), ay = std::abs(u.y);
    const bool xmaj = ax >= ay;
    const int amaj = xmaj ? ax : ay, bmin = xmaj ? ay : ax;
    // (a, b, code, bits of 1/(256 b)) with a = |U_major|, b = |U_minor|;
    // code bit 0: x is the major axis, bit 1: U_major < 0, bit 2: U_minor < 0
    const int umaj = xmaj ? u.x : u.y, umin = xmaj ? u.y : u.x;
    int4& di = D->di[j];
    di.x = amaj;
    di.y = bmin;
    di.z = (xmaj ? 1 : 0) | (umaj < 0 ? 2 : 0) | (umin < 0 ? 4 : 0);
    const float inv = bmin > 0 ? (float)(1.0 / (256.0 * bmin)) : INFINITY;
    std::memcpy(&di.w, &inv, sizeof(float));
    const double nrm = std::sqrt((double)ax * ax + (double)ay * ay);
    // (f, r, kappa_major, kappa_minor)
    float4& df = D->df[j];
    df.x = (float)((double)amaj / nrm * 0.99999);   // rounds down a hair
    df.y = (float)((double)bmin / (double)amaj);
    df.z = xmaj ? D->kp[j].x : D->kp[j].y;
    df.w = xmaj ? D->kp[j].y : D->kp[j].x;
  }
  std::shared_ptr<const DirTables> d = D;
  std::lock_guard<std::mutex> lk(c->lut_mu);
  if (c->dirs.size() >= reloc_ctx::kLutCache) c->dirs.erase(c->dirs.begin());
  c->dirs.push_back(d);
  return d;
}

int32_t build_request(reloc_ctx* c, Request& R) {
  DevMap& m = c->maps[R.map_id];
  const reloc_scan_info& I = R.prep.info;
  const int Ns = I.Ns, Ng = I.Ng, b = Ng / Ns;
  const std::shared_ptr<const DirTables> D = dir_tables(c, Ng, Ns, m.res);
  const std::vector<int2>& U = D->U;
  const std::vector<int2>& rd = D->rd;
  const std::vector<float2>& kp = D->kp;
  const std::vector<int4>& di = D->di;
  const std::vector<float4>& df = D->df;
  std::vector<int32_t> base(R.prep.vj.size());
  for (size_t v = 0; v < base.size(); ++v) base[v] = b * R.prep.vj[v];
  const int n = R.n_hyp, nv = I.n_valid;
  const int nvp = tam_beams_padded(nv);
  const bool direct = R.prm.coarse_metric == 1 || R.prm.coarse_metric == 2;
  const HypSet& hs = c->sets[R.set_id];
  // the read-only tables of the request in one device block, one copy
  std::vector<int2> beams(nvp, int2{0, 0});
  for (int v = 0; v < nv; ++v) beams[v] = int2{base[v], R.prep.vzq[v]};
  std::vector<int2> U2(2 * (size_t)Ng);
  std::copy(U.begin(), U.end(), U2.begin());
  std::copy(U.begin(), U.end(), U2.begin() + Ng);
  // a request over a prefix of the set casts in the set's order restricted
  // to the prefix (the Morton order of the prefix)
  std::vector<int32_t> perm;
  if (n < hs.n) {
    perm.reserve(n);
    for (int32_t h : hs.morton)
      if (h < n) perm.push_back(h);
  }
  TableBlob tb;
  const size_t o_rd = tb.add(rd), o_kp = tb.add(kp), o_di = tb.add(di), o_df = tb.add(df);
  const size_t o_runs = tb.add(R.prep.runs), o_beams = tb.add(beams), o_dirs = tb.add(U2);
  const size_t o_lut = tb.add(R.lut.q);
  const size_t o_fz = direct ? tb.add(R.prep.fz) : 0, o_fj = direct ? tb.add(R.prep.fj) : 0;
  const size_t o_perm = perm.empty() ? 0 : tb.add(perm);
  uint8_t* tables = req_alloc<uint8_t>(c, R, tb.b.size());
  if (!tables) return RELOC_E_NOMEM;
  R.raydirs = (int2*)(tables + o_rd);
  R.kap = (float2*)(tables + o_kp);
  R.dir_i = (int4*)(tables + o_di);
  R.dir_f = (float4*)(tables + o_df);
  R.runs = (int2*)(tables + o_runs);
  R.beams = (int2*)(tables + o_beams);
  R.dirs = (int2*)(tables + o_dirs);
  R.dlut = (int32_t*)(tables + o_lut);
  if (direct) {
    R.fov_z = (double*)(tables + o_fz);
    R.fov_j = (int32_t*)(tables + o_fj);
  }
  R.perm = perm.empty() ? hs.morton_dev : (int32_t*)(tables + o_perm);
  // the range buffer only for the split ray cast (the fused kernel keeps
  // every range on chip)
  const bool split = !fused_path(c, R);
  if (split && !(R.zbuf = req_alloc<float>(c, R, (size_t)n * Ns))) return RELOC_E_NOMEM;
  R.smad = req_alloc<double>(c, R, n);
  R.argm = req_alloc<int32_t>(c, R, n);
  R.keys = req_alloc<uint64_t>(c, R, n);
  R.keys2 = req_alloc<uint64_t>(c, R, n);
  R.vals = req_alloc<int32_t>(c, R, n);
  R.order = req_alloc<int32_t>(c, R, n);
  R.best = req_alloc<uint64_t>(c, R, n);
  if (!R.smad || !R.argm || !R.keys || !R.keys2 || !R.vals || !R.order || !R.best)
    return RELOC_E_NOMEM;
  const int max_stages = (n + R.prm.batch_k - 1) / R.prm.batch_k;
  if (R.prm.refine_k > 0) {
    // slots for one launch of the plain path or one tick of the batched one
    R.ref_slots = std::max(plain_max_stages_per_launch(R), kMaxTickStages) * R.prm.refine_k;
    R.rsel = req_alloc<int32_t>(c, R, R.ref_slots);
    R.rbest = req_alloc<uint64_t>(c, R, R.ref_slots);
    if (!R.rsel || !R.rbest) return RELOC_E_NOMEM;
  }
  R.stage = req_alloc<uint64_t>(c, R, max_stages);
  R.rows_cap = std::max(1, std::min(n, R.prm.k_out));
  R.rows = req_alloc<PoseRow>(c, R, R.rows_cap);
  if (!R.stage || !R.rows) return RELOC_E_NOMEM;
  // second position buffer of the ranking sort (the SMAD order in R.order
  // must survive it)
  R.pos2 = req_alloc<int32_t>(c, R, n);
  if (!R.pos2) return RELOC_E_NOMEM;
  // TAM endpoint offsets, every heading x the beam slots of the kernel class
  R.off_stride = 64 * tam_keys_per_lane(nv);
  R.off = req_alloc<uint32_t>(c, R, (size_t)Ng * (size_t)R.off_stride);
  if (!R.off) return RELOC_E_NOMEM;
  if (R.carve_base) {
    // no allocation of any kind: a copy from the host vectors, drained
    // before they go out of scope
    if (int32_t e = upload(c, tables, tb.b.data(), tb.b.size())) return e;
    HIP_TRY(launch_tam_offsets(R.beams, nv, R.dirs, Ng, R.off_stride, R.off, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return RELOC_OK;
  }
  // through pinned staging: the request's kernels queue behind the copy and
  // the host does not wait for it
  if (int32_t e = upload_staged(c, tables, tb.b.data(), tb.b.size())) return e;
  HIP_TRY(launch_tam_offsets(R.beams, nv, R.dirs, Ng, R.off_stride, R.off, c->stream));
  return RELOC_OK;
}

int32_t upload_staged(reloc_ctx* c, void* dst, const void* src, size_t n) {
  if (n == 0) return RELOC_OK;
  const int i = c->tstage_next;
  c->tstage_next ^= 1;
  if (c->tstage_armed[i]) {
    HIP_TRY(hipEventSynchronize(c->tstage_ev[i]));
    c->tstage_armed[i] = false;
  }
  if (n > c->tstage_cap[i]) {
    if (c->tstage[i]) (void)hipHostFree(c->tstage[i]);
    c->tstage[i] = nullptr;
    c->tstage_cap[i] = 0;
    const size_t cap = std::max(n, (size_t)1 << 16);
    HIP_TRY(hipHostMalloc(&c->tstage[i], cap, hipHostMallocDefault));
    c->tstage_cap[i] = cap;
  }
  if (!c->tstage_ev[i]) HIP_TRY(hipEventCreateWithFlags(&c->tstage_ev[i], hipEventDisableTiming));
  std::memcpy(c->tstage[i], src, n);
  HIP_TRY(hipMemcpyAsync(dst, c->tstage[i], n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->tstage_ev[i], c->stream));
  c->tstage_armed[i] = true;
  return RELOC_OK;
}

bool fused_path(const reloc_ctx*, const Request& R) { return R.fused; }

// Wavefronts per hypothesis workgroup of the fused kernel. Few hypotheses
// cannot fill the device with one wavefront each, so a hypothesis' rays are
// spread over four (256 lanes); many hypotheses are best served by one
// wavefront each (no workgroup barrier, the tail of one hypothesis' rays
// overlaps other wavefronts' work). Measured on MI355X: 300 hypotheses
// 0.038 / 0.050 / 0.075 ms for 4 / 2 / 1; 20 000: 0.68 / 0.63 / 0.63 ms;
// 200 000: 8.5 / 7.9 / 7.6 ms.
int fused_default_nw(int64_t n_hyp) { return n_hyp < 4096 ? 4 : (n_hyp < 32768 ? 2 : 1); }

void fused_shape(const Request& R, int* nw, int* refill) {
  *nw = R.fuse_nw > 0 ? R.fuse_nw : fused_default_nw(R.n_hyp);
  *refill = R.fuse_refill > 0 ? R.fuse_refill : 16;
}

int32_t enqueue_front(reloc_ctx* c, Request& R, const RayArgs& ra, hipEvent_t mid) {
  hipStream_t s = c->stream;
  if (fused_path(c, R)) {
    int nw, rf;
    fused_shape(R, &nw, &rf);
    HIP_TRY(launch_raycast_smad_fused(ra, nw, rf, s));
    if (mid) HIP_TRY(hipEventRecord(mid, s));
    return RELOC_OK;
  }
  if (R.prm.coarse_metric != 3) HIP_TRY(launch_raycast(ra, s));   // none needs no ranges
  if (mid) HIP_TRY(hipEventRecord(mid, s));
  HIP_TRY(launch_coarse(ra, s));
  return RELOC_OK;
}

RayArgs ray_args(reloc_ctx* c, Request& R, int32_t* dbg_hit, int32_t* dbg_steps) {
  DevMap& m = c->maps[R.map_id];
  const reloc_scan_info& I = R.prep.info;
  RayArgs a;
  a.bits = m.bits;
  a.walk = m.walk;
  a.walk_bytes = (uint32_t)(4 * sizeof(uint16_t) * (size_t)m.W * m.H);
  a.dir_i = R.dir_i;
  a.dir_f = R.dir_f;
  // public variant: 1 bit tiles; 2, 3, 4, 5 skipping with wavefront refill
  // at 1, 8, 16, 32 idle lanes; 0 the default
  static const int kv[6] = {3, 0, 1, 2, 3, 4};
  a.variant = kv[R.prm.variant];
  {
    const int64_t rays = (int64_t)R.n_hyp * I.Ns;
    // many short chunks balance the waves across the CUs (a wave's cost
    // varies with its rays' lengths); measured flat between 256 and 512
    a.chunk = R.tuned_chunk > 0
                  ? R.tuned_chunk
                  : (int)std::max<int64_t>(256, std::min<int64_t>(1024, rays / 49152));
  }
  a.zbuf = R.zbuf;
  a.perm = R.perm;
  a.best0 = nullptr;
  a.W = m.W;
  a.H = m.H;
  a.tpr = m.tpr;
  a.hyp_xy = c->sets[R.set_id].dev;
  a.n_hyp = R.n_hyp;
  a.dirs = R.raydirs;
  a.kap = R.kap;
  a.Ns = I.Ns;
  a.rmax = R.rmax;
  a.rcells = R.rcells;
  a.runs = R.runs;
  a.n_runs = I.n_runs;
  a.nfov = I.n_fov;
  a.zbar = I.zbar;
  a.n_shifts = I.n_shifts;
  a.n_enum = R.prm.n_skip_enum;
  a.smad = R.smad;
  a.argm = R.argm;
  a.keys = R.keys;
  a.vals = R.vals;
  a.dbg_hit = dbg_hit;
  a.dbg_steps = dbg_steps;
  a.coarse = R.prm.coarse_metric;
  a.fov_z = R.fov_z;
  a.fov_j = R.fov_j;
  return a;
}

TamArgs tam_args(reloc_ctx* c, Request& R, int r0, int nb, float* T_out) {
  DevMap& m = c->maps[R.map_id];
  const reloc_scan_info& I = R.prep.info;
  TamArgs a;
  a.kmap = m.kmap;
  a.plane = m.plane;
  a.plane16 = reinterpret_cast<const uint16_t*>(m.plane + tam_plane_entries(m.W, m.H));
  a.off = R.off;
  a.off_stride = R.off_stride;
  a.W = m.W;
  a.H = m.H;
  a.hyp_xy = c->sets[R.set_id].dev;
  a.order = R.order;
  a.r0 = r0;
  a.nb = nb;
  a.beams = R.beams;
  a.nv = I.n_valid;
  a.dirs = R.dirs;
  a.Ng = I.Ng;
  a.o = I.Ng / I.Ntheta;
  a.Nt = I.Ntheta;
  a.lut = R.dlut;
  a.lmin = R.lut.qmin;
  a.kcap = R.lut.kcap;
  a.key_off = R.lut.key_off;
  a.keybits = R.lut.keybits;
  a.kmid = I.k_mid;
  a.res = m.res;
  a.d_max = R.prm.d_max;
  a.fine = R.prm.fine_metric;
  a.T_out = T_out;
  a.best = R.best;
  return a;
}

RefineArgs refine_args(reloc_ctx* c, Request& R, int n_slots) {
  RefineArgs a;
  a.t = tam_args(c, R, 0, 0, nullptr);
  a.sel = R.rsel;
  a.rbest = R.rbest;
  a.n_slots = n_slots;
  a.h = R.ref_h;
  a.s = R.ref_s;
  a.L = R.ref_L;
  return a;
}

int plain_max_stages_per_launch(const Request& R) {
  return std::max(plain_stages_per_launch(R), kPlainMaxStages);
}

// stages of a launch that aims at `fill` TAM workgroups (at least one)
static int stages_for_fill(const Request& R, int64_t fill) {
  const int64_t K = R.prm.batch_k;
  const int64_t bps = K * ((R.prep.info.Ntheta + 15) / 16);
  const int64_t stages = (R.n_hyp + K - 1) / K;
  return (int)std::max<int64_t>(1, std::min<int64_t>(stages, std::min<int64_t>(512, fill / bps)));
}

int plain_stages_per_launch(const Request& R) { return stages_for_fill(R, kPlainFillBlocks); }

// The first launch aims lower: a search that stops in it discards fewer
// speculative stages (when one stage alone fills the device both are one).
static int plain_first_stages_per_launch(const Request& R) {
  return stages_for_fill(R, kPlainFirstFillBlocks);
}

// stable SMAD order of the request (after the SMAD kernel)
int32_t smad_order(reloc_ctx* c, Request& R) {
  HIP_TRY(argsort_u64(R.keys, R.keys2, R.vals, R.order, R.n_hyp, 1, nullptr, nullptr, 0, 0,
                      c->stream));
  return RELOC_OK;
}

// ray cast + SMAD for all hypotheses, then the stable SMAD order
int32_t run_smad_order(reloc_ctx* c, Request& R) {
  if (int32_t e = enqueue_front(c, R, ray_args(c, R, nullptr, nullptr), nullptr)) return e;
  return smad_order(c, R);
}

// ranking of ranks [0, n_eval) (T desc, rank asc); the first nrow rows are
// copied to host_rows (pinned) on the stream
// Ranking of the first n_eval ranks, nrow rows to the pinned host_rows;
// *top receives where the kernels find row 0 (the ambiguity statistics read
// it): host_rows itself when the single-launch ranking writes the rows there
// directly, else the request's device rows.
int32_t enqueue_rank(reloc_ctx* c, Request& R, int n_eval, int nrow, PoseRow* host_rows,
                     const PoseRow** top) {
  hipStream_t s = c->stream;
  const int ndev = std::min(n_eval, std::max(1, nrow));
  if (n_eval <= kRankSmallMax) {
    // host_rows holds at least one row (pinned_rows allocates max(1, n))
    HIP_TRY(launch_rank_small(R.best, n_eval, R.order, R.smad, ndev, host_rows, s));
    *top = host_rows;
    return RELOC_OK;
  } else {
    // the SMAD keys are no longer needed: the rank keys take their buffer
    HIP_TRY(launch_rank_keys(R.best, n_eval, R.keys, s));
    HIP_TRY(argsort_u64(R.keys, R.keys2, R.vals, R.pos2, n_eval, 1, nullptr, nullptr, 0, 0, s));
    HIP_TRY(launch_rank_gather(R.keys, R.best, R.order, R.smad, ndev, R.rows, s));
  }
  if (nrow > 0)   // pinned host rows, or device rows on the no-allocation path
    HIP_TRY(hipMemcpyAsync(host_rows, R.rows, nrow * sizeof(PoseRow), hipMemcpyDefault, s));
  *top = R.rows;
  return RELOC_OK;
}

int32_t enqueue_margin(reloc_ctx* c, Request& R, const uint64_t* best, const int32_t* order,
                       const PoseRow* rows, int n_eval, const uint64_t* stage, int n_stages,
                       uint64_t* out) {
  const reloc_scan_info& I = R.prep.info;
  MarginArgs a;
  a.best = best;
  a.order = order;
  a.hyp_xy = c->sets[R.set_id].dev;
  a.top = rows;
  a.n_eval = n_eval;
  a.Ng = I.Ng;
  a.o = I.Ng / I.Ntheta;
  a.res = c->maps[R.map_id].res;
  a.stage = stage;
  a.n_stages = n_stages;
  a.stopped = 0;
  a.tau = R.prm.tau;
  a.out = out;
  HIP_TRY(launch_margin(a, c->stream));
  return RELOC_OK;
}

void fill_ambiguity(const uint64_t* marg, bool fragile, reloc_stats* st) {
  st->best_margin = -1.f;
  st->ambiguous = (marg[1] || fragile) ? 1 : 0;
  if (marg[2] == 0 || marg[0] == 0) return;
  const float t1 = score_of_key((uint32_t)(marg[2] >> 32));
  const float t2 = score_of_key((uint32_t)(marg[0] >> 32));
  st->best_margin = t1 - t2;
  if ((double)st->best_margin <= 1e-4 * std::fabs((double)t1) + 1e-7) st->ambiguous |= 2;
}

// TAM stages [r0, r0 + nb) (ns of them, the first being stage number
// `stage`) with refinement and stage control, then their stop flags to the
// pinned hflag.
int32_t enqueue_stages(reloc_ctx* c, Request& R, int r0, int ns, int nb, int stage,
                       int32_t* hflag) {
  hipStream_t s = c->stream;
  const int K = R.prm.batch_k, kr = R.prm.refine_k;
  HIP_TRY(launch_tam(tam_args(c, R, r0, nb, nullptr), s));
  if (kr > 0) {
    // each stage's kr best poses: lattice search, then their refined T
    // replaces T* before the stage's best is taken
    HIP_TRY(launch_refine_select(R.best, r0, K, R.n_hyp, ns, kr, R.rsel, R.rbest, s));
    const RefineArgs fa = refine_args(c, R, ns * kr);
    HIP_TRY(launch_refine(fa, s));
    HIP_TRY(launch_refine_commit(fa, s));
  }
  // the stop flags go straight to the pinned words the host reads
  StageArgs sa{R.best, r0, nb, R.prm.tau, R.stage + stage, hflag};
  HIP_TRY(launch_stage_reduce_multi(sa, K, ns, R.n_hyp, s));
  return RELOC_OK;
}

// Pinned words the margin kernel writes (best distinct, stop fragility,
// top-1 word).
static uint64_t* head_margin_words(reloc_ctx* c) { return (uint64_t*)((char*)c->pinned + 2048); }

// The device work of a run up to its first stop-flag read, the same on
// every run of the request: ray cast, coarse metric, order, the first ns0
// stages (nb0 ranks) and, when that is one stage, its ranking with the rows
// copied to the pinned hrows (the result is ready at the first
// synchronisation when the search stops there), followed by the ambiguity
// statistics of that result. When timed, events 0, 5,
// 1, 2 (and 3, 4 around the ranking) time the phases; a captured head is
// not timed (event records inside a graph give no usable timestamps here).
int32_t enqueue_head(reloc_ctx* c, Request& R, int ns0, int nb0, int32_t* hflag,
                     PoseRow* hrows, bool timed) {
  hipStream_t s = c->stream;
  auto mark = [&](int i) { return timed ? hipEventRecord(c->ev[i], s) : hipSuccess; };
  RayArgs ra = ray_args(c, R, nullptr, nullptr);
  ra.best0 = R.best;                 // the coarse kernel clears the per-rank best
  HIP_TRY(mark(0));
  if (int32_t e = enqueue_front(c, R, ra, timed ? c->ev[5] : nullptr)) return e;
  HIP_TRY(mark(1));
  if (int32_t e = smad_order(c, R)) return e;
  HIP_TRY(mark(2));
  if (int32_t e = enqueue_stages(c, R, 0, ns0, nb0, 0, hflag)) return e;
  if (ns0 == 1) {
    HIP_TRY(mark(3));
    const PoseRow* top = nullptr;
    if (int32_t e = enqueue_rank(c, R, nb0, std::min(R.rows_cap, nb0), hrows, &top)) return e;
    HIP_TRY(mark(4));
    // the ambiguity statistics of that one-stage result, after the timed region
    if (int32_t e = enqueue_margin(c, R, R.best, R.order, top, nb0, R.stage, 1,
                                   head_margin_words(c)))
      return e;
  }
  return RELOC_OK;
}

// pinned host buffer for result rows, grown on demand; growing it drops
// every captured head graph (they copy rows into the old buffer)
int32_t pinned_rows(reloc_ctx* c, size_t n, PoseRow** out) {
  const size_t need = std::max<size_t>(1, n) * sizeof(PoseRow);
  if (need > c->prows_cap) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& kv : c->reqs) drop_head(kv.second);
    if (c->prows) (void)hipHostFree(c->prows);
    c->prows = nullptr;
    c->prows_cap = 0;
    HIP_TRY(hipHostMalloc(&c->prows, need, hipHostMallocDefault));
    c->prows_cap = need;
  }
  *out = (PoseRow*)c->prows;
  return RELOC_OK;
}

int32_t validate_search(const reloc_search_params* p) {
  if (!p) return fail(RELOC_E_INVALID, "null search params");
  if (p->batch_k <= 0) return fail(RELOC_E_INVALID, "batch_k must be >= 1");
  if (p->k_out <= 0) return fail(RELOC_E_INVALID, "k_out must be >= 1");
  if (p->n_theta < 0 || p->n_hyp < 0) return fail(RELOC_E_INVALID, "negative n_theta / n_hyp");
  if (p->variant < 0 || p->variant > 5) return fail(RELOC_E_INVALID, "variant must be in 0..5");
  if (p->refine_k < 0 || p->refine_k > 64) return fail(RELOC_E_INVALID, "refine_k must be in 0..64");
  if (p->refine_cells < 0 || p->refine_cells > 15)
    return fail(RELOC_E_INVALID, "refine_cells must be in 0..15");
  if (p->refine_dirs < -1) return fail(RELOC_E_INVALID, "refine_dirs must be >= -1");
  if (p->coarse_metric < 0 || p->coarse_metric > 3)
    return fail(RELOC_E_INVALID, "coarse_metric must be in 0..3");
  if (p->fine_metric < 0 || p->fine_metric > 3)
    return fail(RELOC_E_INVALID, "fine_metric must be in 0..3");
  if (p->ray_waves != 0 && p->ray_waves != 1 && p->ray_waves != 2 && p->ray_waves != 4)
    return fail(RELOC_E_INVALID, "ray_waves must be 0, 1, 2 or 4");
  if (p->ray_refill != 0 && p->ray_refill != 8 && p->ray_refill != 16 && p->ray_refill != 32)
    return fail(RELOC_E_INVALID, "ray_refill must be 0, 8, 16 or 32");
  return RELOC_OK;
}

int64_t coarse_evals(const Request& R) {
  const reloc_scan_info& I = R.prep.info;
  switch (R.prm.coarse_metric) {
    case 2: return (int64_t)R.n_hyp * ((I.Ns + R.prm.n_skip_enum - 1) / R.prm.n_skip_enum);
    case 3: return 0;
    default: return (int64_t)R.n_hyp * I.n_shifts;
  }
}

int32_t refine_lattice(const reloc_search_params* p, const reloc_scan_info& I, int* h, int* s,
                       int* L) {
  const int64_t hh = p->refine_cells;
  const int64_t ss = p->refine_dirs < 0 ? I.Ng / I.Ntheta : p->refine_dirs;
  const int64_t LL = (2 * ss + 1) * (2 * hh + 1) * (2 * hh + 1);
  if (ss >= I.Ng) return fail(RELOC_E_INVALID, "refine_dirs %lld >= Ng = %d", (long long)ss, I.Ng);
  if (LL > 65536)
    return fail(RELOC_E_INVALID, "refinement lattice of %lld points exceeds 65536", (long long)LL);
  *h = (int)hh;
  *s = (int)ss;
  *L = (int)LL;
  return RELOC_OK;
}

// The likelihood table of a parameter set: from the context's recent ones
// when the parameters match exactly, else built (and kept).
int32_t cached_lut(reloc_ctx* c, const reloc_search_params* p, double res, Lut* L) {
  const double key[5] = {p->z_hit, p->sigma_hit, p->z_rand, p->d_max, res};
  {
    std::lock_guard<std::mutex> lk(c->lut_mu);
    for (auto it = c->luts.begin(); it != c->luts.end(); ++it)
      if (std::memcmp(it->key, key, sizeof key) == 0) {
        *L = it->lut;
        if (it + 1 != c->luts.end()) std::rotate(it, it + 1, c->luts.end());
        return RELOC_OK;
      }
  }
  if (int32_t e = build_lut(p, res, L)) return e;
  std::lock_guard<std::mutex> lk(c->lut_mu);
  if (c->luts.size() >= reloc_ctx::kLutCache) c->luts.erase(c->luts.begin());
  c->luts.push_back(reloc_ctx::LutEntry{{key[0], key[1], key[2], key[3], key[4]}, *L});
  return RELOC_OK;
}

int32_t init_request(reloc_ctx* c, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                     const reloc_search_params* params, Request* R) {
  if (int32_t e = validate_search(params)) return e;
  auto mi = c->maps.find(map_id);
  if (mi == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  auto si = c->sets.find(set_id);
  if (si == c->sets.end()) return fail(RELOC_E_NOTFOUND, "unknown hypothesis set %d", set_id);
  if (si->second.map_id != map_id)
    return fail(RELOC_E_INVALID, "set %d belongs to another map", set_id);
  R->map_id = map_id;
  R->set_id = set_id;
  R->prm = *params;
  R->n_hyp = params->n_hyp > 0 ? std::min(params->n_hyp, si->second.n) : si->second.n;
  if (int32_t e = preprocess(scan, params, mi->second.res, &R->prep)) return e;
  if (int32_t e = cached_lut(c, params, mi->second.res, &R->lut)) return e;
  R->rmax = scan->range_max;
  R->rcells = (int)std::ceil((double)scan->range_max / mi->second.res) + 2;
  R->fused = params->coarse_metric == 0 && params->variant == 0 && mi->second.walk != nullptr;
  // a map's tuned fused shape carries over to its later requests of the
  // same beam grid (a tuning done once per map)
  if (R->fused && mi->second.fuse_ns == R->prep.info.Ns) {
    R->fuse_nw = mi->second.fuse_nw;
    R->fuse_refill = mi->second.fuse_refill;
  }
  if (params->ray_waves > 0) R->fuse_nw = params->ray_waves;
  if (params->ray_refill > 0) R->fuse_refill = params->ray_refill;
  if (params->refine_k > 0)
    if (int32_t e = refine_lattice(params, R->prep.info, &R->ref_h, &R->ref_s, &R->ref_L))
      return e;
  return RELOC_OK;
}

size_t request_bytes(const Request& R) {
  const reloc_scan_info& I = R.prep.info;
  const size_t n = (size_t)std::max(1, R.n_hyp), Ns = (size_t)I.Ns;
  const size_t stages = (n + (size_t)R.prm.batch_k - 1) / (size_t)R.prm.batch_k;
  size_t b = n * (8 + 4 + 8 + 8 + 4 + 4 + 8);                  // work buffers
  if (!R.fused) b += n * 4 * Ns;                                // range buffer
  b += Ns * (8 + 8 + 16 + 16) + (size_t)I.Ng * 8 + R.prep.runs.size() * 8;
  b += R.prep.vj.size() * 8 + R.lut.q.size() * 4 + stages * 12;
  b += (size_t)std::min<size_t>(n, (size_t)R.prm.k_out) * sizeof(PoseRow);
  if (R.prm.refine_k > 0)
    b += (size_t)std::max(plain_max_stages_per_launch(R), kMaxTickStages) * R.prm.refine_k * 12;
  if (R.prm.coarse_metric == 1 || R.prm.coarse_metric == 2) b += (size_t)I.n_fov * 12;
  b += n * 4;                                                   // ranking sort positions
  b += (size_t)I.Ng * 64 * (size_t)tam_keys_per_lane(I.n_valid) * 4;   // TAM offsets
  b += 32 * 256;                                                // allocation rounding
  return b;
}

void rows_to_poses(const reloc_ctx* c, const Request& R, const PoseRow* rows, int n,
                   reloc_pose* out) {
  const DevMap& m = c->maps.at(R.map_id);
  const HypSet& hs = c->sets.at(R.set_id);
  const reloc_scan_info& I = R.prep.info;
  for (int i = 0; i < n; ++i) {
    const PoseRow& w = rows[i];
    reloc_pose& p = out[i];
    int ix = hs.host[2 * w.hyp], iy = hs.host[2 * w.hyp + 1];
    double th;
    if (w.k < 0) {
      // refined: code = g << 10 | (dy + 15) << 5 | (dx + 15)
      const uint32_t code = 0xFFFFFFFFu - (uint32_t)w.k;
      ix += (int)(code & 31u) - 15;
      iy += (int)((code >> 5) & 31u) - 15;
      p.g = (int32_t)(code >> 10);
      p.k = -1;
      p.refined = 1;
      th = (2.0 * M_PI * (double)p.g) / (double)I.Ng;
    } else {
      p.g = (int32_t)((int64_t)w.k * (I.Ng / I.Ntheta));
      p.k = w.k;
      p.refined = 0;
      th = (2.0 * M_PI * (double)w.k) / (double)I.Ntheta;
    }
    p.cx = ix;
    p.cy = iy;
    p.x = m.ox + ((double)ix + 0.5) * m.res;
    p.y = m.oy + ((double)iy + 0.5) * m.res;
    if (th >= M_PI) th -= 2.0 * M_PI;
    p.theta = th;
    p.tam = score_of_key(w.tbits);
    p.smad = (float)w.smad;
    p.hyp = w.hyp;
    p.rank = w.rank;
    p.stage = w.rank / R.prm.batch_k;
  }
}

}  // namespace reloc

using namespace reloc;

// ============================================================================
extern "C" {

int32_t reloc_version(void) { return RELOC_VERSION; }

const char* reloc_last_error(void) { return g_err.c_str(); }

void reloc_search_defaults(reloc_search_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->n_theta = 0;
  p->n_skip_beam = 1;
  p->n_skip_enum = 1;
  p->batch_k = 64;
  p->k_out = 10;
  p->tau = 0.95;
  p->n_hyp = 0;
  p->z_hit = 1.0;
  p->sigma_hit = 0.2;
  p->z_rand = 0.0;
  p->d_max = 2.0;
  p->alpha_mid_pm[0] = 900;
  p->alpha_mid_pm[1] = 700;
  p->alpha_low_pm[0] = 700;
  p->alpha_low_pm[1] = 500;
  p->deadline_s = 0.0;
  p->variant = 0;
  p->refine_k = 0;
  p->refine_cells = 3;
  p->refine_dirs = -1;
  p->coarse_metric = 0;
  p->fine_metric = 0;
  p->use_graph = 0;
  p->ray_waves = 0;
  p->ray_refill = 0;
}

int32_t reloc_ctx_create(int32_t device, const reloc_allocator* alloc, void* stream,
                         size_t hbm_budget, reloc_ctx** out) {
  if (!out) return fail(RELOC_E_INVALID, "null out");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(RELOC_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= n) return fail(RELOC_E_DEVICE, "device %d out of range", device);
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(RELOC_E_INVALID, "allocator needs both alloc and free");
  std::unique_ptr<reloc_ctx> c(new reloc_ctx());
  c->device = device;
  HIP_TRY(hipSetDevice(device));
  if (alloc) {
    c->alloc = *alloc;
    c->has_alloc = true;
  }
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  size_t fr = 0, tot = 0;
  HIP_TRY(hipMemGetInfo(&fr, &tot));
  c->budget = hbm_budget ? hbm_budget : fr;
  for (auto& e : c->ev) HIP_TRY(hipEventCreate(&e));
  c->serve = serve_create();
  HIP_TRY(hipHostMalloc(&c->pinned, 4096, hipHostMallocDefault));
  if (int32_t e = noalloc_setup(device)) return e;
  *out = c.release();
  return RELOC_OK;
}

void reloc_ctx_destroy(reloc_ctx* c) {
  if (!c) return;
  ctx_stop_serving(c);
  {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->reqs) release_request(c, kv.second);
    for (auto& kv : c->sets) {
      c->dfree(kv.second.dev);
      c->dfree(kv.second.morton_dev);
    }
    for (auto& kv : c->maps) {
      c->dfree(kv.second.bits);
      c->dfree(kv.second.walk);
      c->dfree(kv.second.kmap);
      c->dfree(kv.second.plane);
    }
    c->reqs.clear();
    c->sets.clear();
    c->maps.clear();
    c->flush_cache();
    for (auto& e : c->ev)
      if (e) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->prows) (void)hipHostFree(c->prows);
    for (int i = 0; i < 2; ++i) {
      if (c->tstage[i]) (void)hipHostFree(c->tstage[i]);
      if (c->tstage_ev[i]) (void)hipEventDestroy(c->tstage_ev[i]);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

size_t reloc_ctx_bytes(const reloc_ctx* c) { return c ? c->used : 0; }

int32_t reloc_load_map(reloc_ctx* c, const reloc_map_desc* d, const int8_t* occ,
                       int32_t* map_id) {
  if (map_id) *map_id = -1;
  if (!c || !d || !occ || !map_id) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  if (d->width < 1 || d->height < 1 || d->width > kMaxDim || d->height > kMaxDim)
    return fail(RELOC_E_INVALID, "map size %dx%d outside 1..%d", d->width, d->height, kMaxDim);
  if (!(d->resolution >= 1.0 / 32.0) || !(d->resolution <= 100.0))
    return fail(RELOC_E_INVALID, "resolution must be in [1/32, 100] m");
  if (!std::isfinite(d->origin_x) || !std::isfinite(d->origin_y))
    return fail(RELOC_E_INVALID, "origin must be finite");
  const size_t N = (size_t)d->width * d->height;
  bool any = false;
  for (size_t i = 0; i < N && !any; ++i) any = (int)occ[i] >= d->occ_threshold;
  if (!any) return fail(RELOC_E_EMPTY, "map has no occupied cell");
  if (int32_t e = set_device(c)) return e;
  DevMap m;
  m.W = d->width;
  m.H = d->height;
  m.thr = d->occ_threshold;
  m.res = d->resolution;
  m.ox = d->origin_x;
  m.oy = d->origin_y;
  m.tpr = (m.W + 7) / 8;
  m.tph = (m.H + 7) / 8;
  m.occ.assign(occ, occ + N);
  int8_t* docc = (int8_t*)c->dalloc(N);
  int32_t* g = (int32_t*)c->dalloc(N * sizeof(int32_t));
  m.bits = (uint64_t*)c->dalloc((size_t)m.tpr * m.tph * sizeof(uint64_t));
  if (N <= kWalkMaxCells) m.walk = (uint16_t*)c->dalloc(4 * N * sizeof(uint16_t));
  m.kmap = (uint32_t*)c->dalloc(N * sizeof(uint32_t));
  m.plane = (uint32_t*)c->dalloc(tam_plane_bytes(m.W, m.H));
  auto cleanup = [&]() {
    c->dfree(docc);
    c->dfree(g);
  };
  if (!docc || !g || !m.bits || (N <= kWalkMaxCells && !m.walk) || !m.kmap || !m.plane) {
    cleanup();
    c->dfree(m.bits);
    c->dfree(m.walk);
    c->dfree(m.kmap);
    c->dfree(m.plane);
    return RELOC_E_NOMEM;
  }
  hipError_t e = hipMemcpyAsync(docc, occ, N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_bitpack(docc, m.W, m.H, m.thr, m.bits, m.tpr, m.tph, c->stream);
  if (e == hipSuccess) e = launch_edt(docc, m.W, m.H, m.thr, g, m.kmap, c->stream);
  if (e == hipSuccess && m.walk) e = launch_walkmap(m.kmap, m.W, m.H, m.walk, c->stream);
  if (e == hipSuccess) e = launch_tam_plane(m.kmap, m.W, m.H, m.plane, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) {
    c->dfree(m.bits);
    c->dfree(m.walk);
    c->dfree(m.kmap);
    c->dfree(m.plane);
    return fail(RELOC_E_DEVICE, "map upload failed: %s", hipGetErrorString(e));
  }
  const int id = c->next_id++;
  {
    std::lock_guard<std::mutex> rg(c->reg_mu);
    c->maps[id] = std::move(m);
  }
  *map_id = id;
  return RELOC_OK;
}

int32_t reloc_unload_map(reloc_ctx* c, int32_t map_id) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->maps.find(map_id);
  if (it == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  if (it->second.n_sets > 0) return fail(RELOC_E_BUSY, "map %d has live hypothesis sets", map_id);
  (void)hipStreamSynchronize(c->stream);
  c->dfree(it->second.bits);
  c->dfree(it->second.walk);
  c->dfree(it->second.kmap);
  c->dfree(it->second.plane);
  std::lock_guard<std::mutex> rg(c->reg_mu);
  c->maps.erase(it);
  return RELOC_OK;
}

int32_t reloc_read_edt(reloc_ctx* c, int32_t map_id, uint32_t* k_out) {
  if (!c || !k_out) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->maps.find(map_id);
  if (it == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  if (int32_t e = set_device(c)) return e;
  DevMap& m = it->second;
  HIP_TRY(hipMemcpyAsync(k_out, m.kmap, (size_t)m.W * m.H * sizeof(uint32_t),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return RELOC_OK;
}

int32_t reloc_sample_hypotheses(reloc_ctx* c, int32_t map_id, const reloc_sample_params* p,
                                int32_t* set_id, int32_t* n_out) {
  if (n_out) *n_out = 0;
  if (set_id) *set_id = -1;
  if (!c || !p || !set_id || !n_out) return fail(RELOC_E_INVALID, "null argument");
  *set_id = -1;
  if (p->n_target < 1) return fail(RELOC_E_INVALID, "n_target must be >= 1");
  if (!(p->min_spacing >= 0) || !(p->robot_radius >= 0))
    return fail(RELOC_E_INVALID, "min_spacing and robot_radius must be >= 0");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->maps.find(map_id);
  if (it == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  if (int32_t e = set_device(c)) return e;
  DevMap& m = it->second;
  if (int32_t e = ensure_khost(c, m)) return e;
  std::vector<int32_t> xy;
  if (int32_t e = sample_cells(m, p, &xy)) return e;
  if (xy.empty()) return fail(RELOC_E_EMPTY, "no feasible hypothesis");
  const int n = (int)(xy.size() / 2);
  if (int32_t e = new_set(c, map_id, std::move(xy), set_id)) return e;
  *n_out = n;
  return RELOC_OK;
}

int32_t reloc_set_hypotheses(reloc_ctx* c, int32_t map_id, const int32_t* cell_xy, int32_t n,
                             int32_t* set_id) {
  if (set_id) *set_id = -1;
  if (!c || !cell_xy || !set_id) return fail(RELOC_E_INVALID, "null argument");
  if (n < 1) return fail(RELOC_E_INVALID, "empty hypothesis set");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->maps.find(map_id);
  if (it == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  const DevMap& m = it->second;
  for (int i = 0; i < n; ++i) {
    const int x = cell_xy[2 * i], y = cell_xy[2 * i + 1];
    if (x < 0 || x >= m.W || y < 0 || y >= m.H)
      return fail(RELOC_E_INVALID, "hypothesis %d (%d, %d) outside the map", i, x, y);
    const int8_t v = m.occ[(size_t)y * m.W + x];
    if (v < 0 || (int)v >= m.thr)
      return fail(RELOC_E_INVALID, "hypothesis %d (%d, %d) is not a free cell", i, x, y);
  }
  if (int32_t e = set_device(c)) return e;
  return new_set(c, map_id, std::vector<int32_t>(cell_xy, cell_xy + 2 * (size_t)n), set_id);
}

int32_t reloc_read_hypotheses(reloc_ctx* c, int32_t set_id, int32_t* cell_xy, int32_t cap,
                              int32_t* n_out) {
  if (!c || !n_out) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->sets.find(set_id);
  if (it == c->sets.end()) {
    *n_out = 0;
    return fail(RELOC_E_NOTFOUND, "unknown hypothesis set %d", set_id);
  }
  const HypSet& s = it->second;
  if (cell_xy && cap > 0)
    std::memcpy(cell_xy, s.host.data(), (size_t)std::min(cap, s.n) * 2 * sizeof(int32_t));
  *n_out = s.n;
  return RELOC_OK;
}

int32_t reloc_free_hypotheses(reloc_ctx* c, int32_t set_id) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->sets.find(set_id);
  if (it == c->sets.end()) return fail(RELOC_E_NOTFOUND, "unknown hypothesis set %d", set_id);
  for (auto& kv : c->reqs)
    if (kv.second.set_id == set_id) return fail(RELOC_E_BUSY, "set %d used by a request", set_id);
  // registry lock first: a concurrent submit either sees the set gone or
  // has registered its ticket before this check
  std::lock_guard<std::mutex> rg(c->reg_mu);
  if (serve_holds_set(c, set_id)) return fail(RELOC_E_BUSY, "set %d used by a queued request", set_id);
  (void)hipStreamSynchronize(c->stream);
  c->dfree(it->second.dev);
  c->dfree(it->second.morton_dev);
  c->maps[it->second.map_id].n_sets -= 1;
  c->sets.erase(it);
  return RELOC_OK;
}

int32_t reloc_scan_info_get(const reloc_scan* scan, const reloc_search_params* params,
                            double resolution, reloc_scan_info* out) {
  if (!out) return fail(RELOC_E_INVALID, "null out");
  std::memset(out, 0, sizeof *out);
  if (!(resolution >= 1.0 / 32.0)) return fail(RELOC_E_INVALID, "resolution must be >= 1/32 m");
  if (int32_t e = validate_search(params)) return e;
  Prep P;
  if (int32_t e = preprocess(scan, params, resolution, &P)) return e;
  if (params->refine_k > 0) {
    int h, s, L;
    if (int32_t e = refine_lattice(params, P.info, &h, &s, &L)) return e;
  }
  *out = P.info;
  return RELOC_OK;
}

int32_t reloc_prepare(reloc_ctx* c, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                      const reloc_search_params* params, int32_t* request_id) {
  if (request_id) *request_id = -1;
  if (!c || !request_id) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  Request R;
  if (int32_t e = init_request(c, map_id, set_id, scan, params, &R)) return e;
  if (int32_t e = set_device(c)) return e;
  if (int32_t e = build_request(c, R)) {
    release_request(c, R);
    return e;
  }
  const int id = c->next_id++;
  c->reqs[id] = std::move(R);
  *request_id = id;
  return RELOC_OK;
}

int32_t reloc_release(reloc_ctx* c, int32_t request_id) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  (void)hipStreamSynchronize(c->stream);
  release_request(c, it->second);
  c->reqs.erase(it);
  return RELOC_OK;
}

int32_t reloc_run(reloc_ctx* c, int32_t request_id, reloc_pose* out, int32_t cap,
                  int32_t* n_out, reloc_stats* st) {
  if (n_out) *n_out = 0;
  if (!c || !n_out || (!out && cap > 0)) return fail(RELOC_E_INVALID, "null argument");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  if (int32_t e = set_device(c)) return e;
  return run_request(c, it->second, out, cap, n_out, st, nullptr);
}

}  // extern "C"

namespace reloc {

int32_t run_request(reloc_ctx* c, Request& R, reloc_pose* out, int32_t cap, int32_t* n_out,
                    reloc_stats* st, PoseRow* dev_rows) {
  const reloc_scan_info& I = R.prep.info;
  const DevMap& m = c->maps[R.map_id];
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = c->stream;
  const int K = R.prm.batch_k;
  int stages = 0, stopped = 0, n_eval = 0;
  int32_t status = RELOC_OK;
  int32_t* hflag = (int32_t*)c->pinned;
  const int ncap = std::min(R.rows_cap, std::max(0, cap));
  PoseRow* hrows = dev_rows;
  if (!hrows)
    if (int32_t e = pinned_rows(c, (size_t)R.rows_cap, &hrows)) return e;
  bool ranked = false;   // rows of the final n_eval already on the host
  int nrow = 0;
  // the first launch holds enough stages for a quarter of the device, the
  // second enough to fill it; when the search goes on, each later launch
  // holds twice as many as the one before, up to plain_max_stages_per_launch
  // (few speculative stages when the search stops early, few stop-flag round
  // trips on long searches, and when one stage fills the device no wasted
  // stage when the search stops in its second launch). Stages after the
  // first one that stops are discarded, so the result is that of one stage
  // at a time.
  int per = plain_first_stages_per_launch(R);
  const int per_max = plain_max_stages_per_launch(R);
  int launches = 0;
  const int kr = R.prm.refine_k;
  bool replayed = false;
  // the head: everything up to the first stop-flag read, replayed as a
  // captured graph when possible
  {
    const int ns0 = std::min(per, (R.n_hyp + K - 1) / K);
    const int nb0 = std::min(ns0 * K, R.n_hyp);
    // captured on the request's second run (a one-shot relocalization would
    // pay the capture and gain nothing)
    const bool graph = R.prm.use_graph && !dev_rows && s != nullptr &&
                       (ns0 != 1 || nb0 <= kRankSmallMax) && (R.head || R.runs_done >= 1);
    if (graph && !R.head) {
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const int32_t e = enqueue_head(c, R, ns0, nb0, hflag, hrows, false);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(s, &g);
      if (e != RELOC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
      }
      if (ec != hipSuccess) return fail(RELOC_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&R.head, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        R.head = nullptr;
        return fail(RELOC_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
      }
    }
    replayed = graph;
    if (graph) {
      HIP_TRY(hipEventRecord(c->ev[0], s));
      HIP_TRY(hipGraphLaunch(R.head, s));
      if (ns0 == 1) HIP_TRY(hipEventRecord(c->ev[4], s));
    } else if (int32_t e = enqueue_head(c, R, ns0, nb0, hflag, hrows, true)) {
      return e;
    }
  }
  for (int r0 = 0; r0 < R.n_hyp;) {
    const int left = (R.n_hyp - r0 + K - 1) / K;
    const int ns = std::min(per, left);
    const int nb = std::min(ns * K, R.n_hyp - r0);
    const bool spec = r0 == 0 && ns == 1;
    if (r0 > 0) {
      if (int32_t e = enqueue_stages(c, R, r0, ns, nb, stages, hflag)) return e;
    }
    HIP_TRY(hipStreamSynchronize(s));
    int hit = -1;
    for (int j = 0; j < ns; ++j)
      if (hflag[j]) {
        hit = j;
        break;
      }
    if (hit >= 0) {
      stages += hit + 1;
      n_eval = std::min(R.n_hyp, r0 + (hit + 1) * K);
      stopped = 1;
      ranked = spec;
      break;
    }
    stages += ns;
    r0 += nb;
    n_eval = r0;
    if (n_eval >= R.n_hyp) {
      ranked = spec;
      break;
    }
    if (++launches >= 2)
      per = std::min(per_max, 2 * per);
    else
      per = plain_stages_per_launch(R);
    if (R.prm.deadline_s > 0) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      if (el > R.prm.deadline_s && n_eval < R.n_hyp) {
        status = fail(RELOC_E_TIMEOUT, "deadline of %.3f s passed after %d stages", R.prm.deadline_s, stages);
        break;
      }
    }
  }
  nrow = std::min(ncap, n_eval);
  const PoseRow* top = nullptr;   // where row 0 is for the ambiguity kernel
  if (!ranked) {
    HIP_TRY(hipEventRecord(c->ev[3], s));
    if (int32_t e = enqueue_rank(c, R, n_eval, nrow, hrows, &top)) return e;
    HIP_TRY(hipEventRecord(c->ev[4], s));
  }
  // ambiguity statistics, after the timed region (row 0 at `top`); the
  // kernel writes its three words straight into pinned host memory (a
  // result ranked in the head has its statistics from the head too)
  uint64_t* hmarg = head_margin_words(c);
  if (st && n_eval > 0 && !ranked)
    if (int32_t e = enqueue_margin(c, R, R.best, R.order, top, n_eval, R.stage, stages,
                                   hmarg))
      return e;
  std::vector<PoseRow> copied;
  if (dev_rows && nrow > 0) {
    copied.resize(nrow);
    HIP_TRY(hipMemcpyAsync(copied.data(), dev_rows, nrow * sizeof(PoseRow), hipMemcpyDeviceToHost,
                           s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  ++R.runs_done;
  rows_to_poses(c, R, dev_rows ? copied.data() : hrows, nrow, out);
  *n_out = nrow;
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->n_hyp = R.n_hyp;
    st->smad_evals = coarse_evals(R);
    st->tam_evals = (int64_t)n_eval * I.Ntheta;
    st->rays = R.prm.coarse_metric == 3 ? 0 : (int64_t)R.n_hyp * I.Ns;
    st->tam_lookups = st->tam_evals * I.n_valid;
    st->stages = stages;
    st->early_stopped = stopped;
    st->n_eval = n_eval;
    if (n_eval > 0) fill_ambiguity(hmarg, false, st);
    else st->best_margin = -1.f;
    if (kr > 0) {
      for (int b = 0; b < stages; ++b)
        st->refined += std::min(kr, std::min(K, R.n_hyp - b * K));
      st->refine_points = st->refined * R.ref_L;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[4]);
    st->ms_total = ms;
    if (!replayed) {
      (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[5]);
      st->ms_raycast = ms;
      (void)hipEventElapsedTime(&ms, c->ev[5], c->ev[1]);
      st->ms_smad = ms;
      (void)hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
      st->ms_sort = ms;
      (void)hipEventElapsedTime(&ms, c->ev[2], c->ev[3]);
      st->ms_tam = ms;
      (void)hipEventElapsedTime(&ms, c->ev[3], c->ev[4]);
      st->ms_rank = ms;
    }
  }
  return status;
}

}  // namespace reloc

extern "C" {

int32_t reloc_relocalize(reloc_ctx* c, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                         const reloc_search_params* params, reloc_pose* out, int32_t cap,
                         int32_t* n_out, reloc_stats* st) {
  if (n_out) *n_out = 0;
  int32_t rid = -1;
  if (int32_t e = reloc_prepare(c, map_id, set_id, scan, params, &rid)) return e;
  const int32_t e = reloc_run(c, rid, out, cap, n_out, st);
  const std::string msg = g_err;
  reloc_release(c, rid);
  g_err = msg;
  return e;
}

int32_t reloc_autotune(reloc_ctx* c, int32_t request_id, int32_t reps, int32_t* variant_out,
                       int32_t* chunk_out, float* ms_out) {
  if (variant_out) *variant_out = 0;
  if (chunk_out) *chunk_out = 0;
  if (ms_out) *ms_out = 0.f;
  if (!c || reps < 1) return fail(RELOC_E_INVALID, "null ctx or reps < 1");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  if (int32_t e = set_device(c)) return e;
  Request& R = it->second;
  hipStream_t s = c->stream;
  float best_ms = -1.f;
  int best_v = R.prm.variant, best_c = R.tuned_chunk;
  auto time_launch = [&](auto launch, float* ms) -> int32_t {
    HIP_TRY(launch());   // warm-up
    HIP_TRY(hipEventRecord(c->ev[0], s));
    for (int r = 0; r < reps; ++r) HIP_TRY(launch());
    HIP_TRY(hipEventRecord(c->ev[5], s));
    HIP_TRY(hipEventSynchronize(c->ev[5]));
    HIP_TRY(hipEventElapsedTime(ms, c->ev[0], c->ev[5]));
    *ms /= (float)reps;
    return RELOC_OK;
  };
  if (R.fused) {
    // fused kernel: wavefronts per hypothesis workgroup x lane-refill
    // threshold; every shape gives bit-identical SMAD values
    static const int nws[3] = {1, 2, 4};
    static const int refills[3] = {8, 16, 32};
    const RayArgs a = ray_args(c, R, nullptr, nullptr);
    int bnw = 0, brf = 0;
    for (int nw : nws)
      for (int rf : refills) {
        float ms = 0.f;
        if (int32_t e = time_launch([&] { return launch_raycast_smad_fused(a, nw, rf, s); }, &ms))
          return e;
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          bnw = nw;
          brf = rf;
        }
      }
    R.fuse_nw = bnw;
    R.fuse_refill = brf;
    DevMap& m = c->maps.at(R.map_id);
    m.fuse_ns = R.prep.info.Ns;
    m.fuse_nw = bnw;
    m.fuse_refill = brf;
    drop_head(R);
    if (variant_out) *variant_out = brf == 8 ? 3 : (brf == 16 ? 4 : 5);
    if (chunk_out) *chunk_out = bnw;
    if (ms_out) *ms_out = best_ms;
    return RELOC_OK;
  }
  if (c->maps.at(R.map_id).walk) {
    // lane-refill threshold (public variants 3, 4, 5: 8, 16, 32 idle lanes)
    // x rays per chunk; every shape gives bit-identical ranges
    static const int variants[3] = {3, 4, 5};
    static const int chunks[5] = {256, 384, 512, 768, 1024};
    for (int v : variants)
      for (int ch : chunks) {
        R.prm.variant = v;
        R.tuned_chunk = ch;
        const RayArgs a = ray_args(c, R, nullptr, nullptr);
        float ms = 0.f;
        if (int32_t e = time_launch([&] { return launch_raycast(a, s); }, &ms)) return e;
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          best_v = v;
          best_c = ch;
        }
      }
    R.prm.variant = best_v;
    R.tuned_chunk = best_c;
    drop_head(R);                    // the captured head holds the old launch shape
  }
  if (variant_out) *variant_out = R.prm.variant;
  if (chunk_out) *chunk_out = R.tuned_chunk;
  if (ms_out) *ms_out = best_ms < 0.f ? 0.f : best_ms;
  return RELOC_OK;
}

int32_t reloc_debug_raycast(reloc_ctx* c, int32_t request_id, int32_t* hit_cell, float* range,
                            int32_t* steps) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  if (int32_t e = set_device(c)) return e;
  Request& R = it->second;
  const size_t n = (size_t)R.n_hyp * R.prep.info.Ns;
  // the fused kernel writes ranges only into a buffer it is given
  const bool fz = R.fused;
  int32_t* dh = hit_cell ? (int32_t*)c->dalloc(n * sizeof(int32_t)) : nullptr;
  int32_t* ds = steps ? (int32_t*)c->dalloc(n * sizeof(int32_t)) : nullptr;
  float* dz = fz && range ? (float*)c->dalloc(n * sizeof(float)) : nullptr;
  if ((hit_cell && !dh) || (steps && !ds) || (fz && range && !dz)) {
    c->dfree(dh);
    c->dfree(ds);
    c->dfree(dz);
    return RELOC_E_NOMEM;
  }
  RayArgs ra = ray_args(c, R, dh, ds);
  if (fz) ra.zbuf = dz;
  const int32_t ef = enqueue_front(c, R, ra, nullptr);
  hipError_t e = ef == RELOC_OK ? hipSuccess : hipErrorLaunchFailure;
  if (e == hipSuccess && hit_cell)
    e = hipMemcpyAsync(hit_cell, dh, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && range)
    e = hipMemcpyAsync(range, fz ? dz : R.zbuf, n * sizeof(float), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess && steps)
    e = hipMemcpyAsync(steps, ds, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  const hipError_t es = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = es;
  c->dfree(dh);
  c->dfree(ds);
  c->dfree(dz);
  if (ef != RELOC_OK) return ef;
  if (e != hipSuccess) return fail(RELOC_E_DEVICE, "debug ray cast failed: %s", hipGetErrorString(e));
  return RELOC_OK;
}

int32_t reloc_coarse_scores(reloc_ctx* c, int32_t request_id, int32_t cap, double* score,
                            int32_t* shift, int32_t* order, reloc_stats* st) {
  if (st) std::memset(st, 0, sizeof *st);
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  Request& R = it->second;
  if ((score || shift || order) && cap < R.n_hyp)
    return fail(RELOC_E_INVALID, "buffers of %d entries, the request has %d hypotheses", cap,
                R.n_hyp);
  if (int32_t e = set_device(c)) return e;
  hipStream_t s = c->stream;
  const RayArgs ra = ray_args(c, R, nullptr, nullptr);
  HIP_TRY(hipEventRecord(c->ev[0], s));
  if (int32_t e = enqueue_front(c, R, ra, c->ev[1])) return e;
  HIP_TRY(hipEventRecord(c->ev[2], s));
  if (int32_t e = smad_order(c, R)) return e;
  HIP_TRY(hipEventRecord(c->ev[3], s));
  const size_t n = (size_t)R.n_hyp;
  if (score) HIP_TRY(hipMemcpyAsync(score, R.smad, n * sizeof(double), hipMemcpyDeviceToHost, s));
  if (shift) HIP_TRY(hipMemcpyAsync(shift, R.argm, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (order) HIP_TRY(hipMemcpyAsync(order, R.order, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (st) {
    const reloc_scan_info& I = R.prep.info;
    st->n_hyp = R.n_hyp;
    st->smad_evals = coarse_evals(R);
    st->rays = R.prm.coarse_metric == 3 ? 0 : (int64_t)R.n_hyp * I.Ns;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[3]);
    st->ms_total = ms;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    st->ms_raycast = ms;
    (void)hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
    st->ms_smad = ms;
    (void)hipEventElapsedTime(&ms, c->ev[2], c->ev[3]);
    st->ms_sort = ms;
  }
  return RELOC_OK;
}

int32_t reloc_score_poses(reloc_ctx* c, int32_t request_id, const int32_t* cell_xy,
                          const int32_t* heading, int32_t n, float* score, float* ms_out) {
  if (ms_out) *ms_out = 0.f;
  if (!c || n < 0 || (n > 0 && (!cell_xy || !heading || !score)))
    return fail(RELOC_E_INVALID, "null argument or negative n");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  Request& R = it->second;
  const DevMap& m = c->maps[R.map_id];
  const int Ng = R.prep.info.Ng;
  for (int32_t i = 0; i < n; ++i) {
    if (cell_xy[2 * i] < 0 || cell_xy[2 * i] >= m.W || cell_xy[2 * i + 1] < 0 ||
        cell_xy[2 * i + 1] >= m.H)
      return fail(RELOC_E_INVALID, "pose %d: cell (%d, %d) outside the map", i, cell_xy[2 * i],
                  cell_xy[2 * i + 1]);
    if (heading[i] < 0 || heading[i] >= Ng)
      return fail(RELOC_E_INVALID, "pose %d: heading index %d outside [0, %d)", i, heading[i], Ng);
  }
  if (n == 0) return RELOC_OK;
  if (int32_t e = set_device(c)) return e;
  int32_t* dxy = (int32_t*)c->dalloc((size_t)n * 2 * sizeof(int32_t));
  int32_t* dg = (int32_t*)c->dalloc((size_t)n * sizeof(int32_t));
  float* dout = (float*)c->dalloc((size_t)n * sizeof(float));
  auto release = [&]() {
    c->dfree(dxy);
    c->dfree(dg);
    c->dfree(dout);
  };
  if (!dxy || !dg || !dout) {
    release();
    return RELOC_E_NOMEM;
  }
  hipStream_t s = c->stream;
  PoseArgs a;
  a.t = tam_args(c, R, 0, 0, nullptr);
  a.xy = dxy;
  a.g = dg;
  a.n = n;
  a.out = dout;
  hipError_t e = hipMemcpyAsync(dxy, cell_xy, (size_t)n * 2 * sizeof(int32_t),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dg, heading, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(c->ev[0], s);
  if (e == hipSuccess) e = launch_score_poses(a, s);
  if (e == hipSuccess) e = hipEventRecord(c->ev[1], s);
  if (e == hipSuccess) e = hipMemcpyAsync(score, dout, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && ms_out) (void)hipEventElapsedTime(ms_out, c->ev[0], c->ev[1]);
  release();
  if (e != hipSuccess) return fail(RELOC_E_DEVICE, "pose scoring failed: %s", hipGetErrorString(e));
  return RELOC_OK;
}

int32_t reloc_debug_smad(reloc_ctx* c, int32_t request_id, double* smad, int32_t* argmin,
                         int32_t* order) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  return reloc_coarse_scores(c, request_id, it->second.n_hyp, smad, argmin, order, nullptr);
}

int32_t reloc_debug_tam(reloc_ctx* c, int32_t request_id, int32_t r0, int32_t n, float* T,
                        float* tstar, int32_t* kstar) {
  if (!c) return fail(RELOC_E_INVALID, "null ctx");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->reqs.find(request_id);
  if (it == c->reqs.end()) return fail(RELOC_E_NOTFOUND, "unknown request %d", request_id);
  Request& R = it->second;
  // n > n_hyp - r0 rather than r0 + n > n_hyp: the sum can wrap in 32 bits
  if (r0 < 0 || r0 >= R.n_hyp || n < 1 || n > R.n_hyp - r0)
    return fail(RELOC_E_INVALID, "rank range [%d, %d + %d) outside [0, %d)", r0, r0, n, R.n_hyp);
  if (int32_t e = set_device(c)) return e;
  if (int32_t e = run_smad_order(c, R)) return e;
  const int Nt = R.prep.info.Ntheta;
  float* dT = nullptr;
  if (T) {
    dT = (float*)c->dalloc((size_t)n * Nt * sizeof(float));
    if (!dT) return RELOC_E_NOMEM;
  }
  std::vector<uint64_t> best(n);
  hipError_t e = launch_fill_u64(R.best + r0, 0, (size_t)n, c->stream);
  // TAM launches cover at most batch_k ranks each, like the staged path
  for (int q = 0; q < n && e == hipSuccess; q += R.prm.batch_k) {
    const int nb = std::min(R.prm.batch_k, n - q);
    e = launch_tam(tam_args(c, R, r0 + q, nb, dT ? dT + (size_t)q * Nt : nullptr), c->stream);
  }
  if (e == hipSuccess && T)
    e = hipMemcpyAsync(T, dT, (size_t)n * Nt * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(best.data(), R.best + r0, n * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->dfree(dT);
  if (e != hipSuccess) return fail(RELOC_E_DEVICE, "debug TAM failed: %s", hipGetErrorString(e));
  for (int i = 0; i < n; ++i) {
    if (tstar) tstar[i] = score_of_key((uint32_t)(best[i] >> 32));
    if (kstar) kstar[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)(best[i] & 0xFFFFFFFFu));
  }
  return RELOC_OK;
}

}  // extern "C"
