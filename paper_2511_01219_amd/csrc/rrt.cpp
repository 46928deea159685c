// Traversability-constrained RRT sampling (Algorithm 1; Sec. III-A items
// 1-7; Remark 4) on the host copy of a resident map: tree growth is
// sequential (each NearestNode query sees every node added before it), so
// it runs on the CPU beside the device work, with a k-d tree for
// NearestNode.
//
// The arithmetic of every step is fixed (see reloc.h), so the tree, and the
// hypothesis set drawn from it, are a deterministic function of the map,
// the parameters and the seed.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "runtime_internal.h"

namespace reloc {

namespace {

// splitmix64 output function (Steele, Lea & Flood 2014): the published
// constants, applied to x + golden gamma.
uint64_t mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Uniform double in [0, 1) from the top 53 bits.
double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// 2-d tree over the RRT nodes, built by insertion (the split axis alternates
// with depth; points with an equal coordinate go right). The nearest-node
// search prunes a subtree only when the squared distance to its splitting
// line exceeds the best squared distance found. Both squared distances are
// rounded the same way and rounding is monotone, so no node that could
// equal or beat the best is ever skipped: the result is the node with the
// smallest rounded (dx*dx + dy*dy), ties to the smallest index, exactly as
// a scan over all nodes gives.
struct KdTree {
  const std::vector<double>& x;
  const std::vector<double>& y;
  std::vector<int32_t> left, right;
  std::vector<uint8_t> axis;
  int32_t root = -1;
  std::vector<std::pair<int32_t, double>> stack;

  KdTree(const std::vector<double>& xs, const std::vector<double>& ys) : x(xs), y(ys) {}

  void insert(int32_t i) {
    left.push_back(-1);
    right.push_back(-1);
    axis.push_back(0);
    if (root < 0) {
      root = i;
      return;
    }
    int32_t n = root;
    while (true) {
      const bool go_left = axis[n] ? y[i] < y[n] : x[i] < x[n];
      int32_t& child = go_left ? left[n] : right[n];
      if (child < 0) {
        child = i;
        axis[i] = (uint8_t)(1 - axis[n]);
        return;
      }
      n = child;
    }
  }

  int32_t nearest(double qx, double qy) {
    int32_t best = -1;
    double bd = INFINITY;
    stack.clear();
    stack.emplace_back(root, 0.0);
    while (!stack.empty()) {
      const auto e = stack.back();
      stack.pop_back();
      const int32_t n = e.first;
      if (n < 0 || e.second > bd) continue;
      const double dx = x[n] - qx, dy = y[n] - qy;
      const double d2 = dx * dx + dy * dy;
      if (d2 < bd || (d2 == bd && n < best)) {
        bd = d2;
        best = n;
      }
      const double diff = axis[n] ? qy - y[n] : qx - x[n];
      const int32_t near_c = diff < 0 ? left[n] : right[n];
      const int32_t far_c = diff < 0 ? right[n] : left[n];
      stack.emplace_back(far_c, diff * diff);
      stack.emplace_back(near_c, 0.0);
    }
    return best;
  }
};

}  // namespace

int32_t rrt_sample(const DevMap& m, const reloc_rrt_params* p, std::vector<int32_t>* cells,
                   std::vector<double>* nodes, std::vector<int32_t>* parents,
                   reloc_rrt_info* info) {
  const int W = m.W, H = m.H;
  const double res = m.res, ox = m.ox, oy = m.oy;
  const double q = p->robot_radius / res;
  const int64_t Kr = (int64_t)std::ceil(q * q - 1e-9);
  const std::vector<int8_t>& occ = m.occ;
  const std::vector<uint32_t>& k = m.khost;
  auto feasible = [&](double px, double py) {
    const int64_t cx = (int64_t)std::floor((px - ox) / res);
    const int64_t cy = (int64_t)std::floor((py - oy) / res);
    if (cx < 0 || cx >= W || cy < 0 || cy >= H) return false;
    const int64_t c = cy * W + cx;
    return occ[c] >= 0 && (int)occ[c] < m.thr && (int64_t)k[c] >= Kr;
  };
  if (!feasible(p->p0_x, p->p0_y))
    return fail(RELOC_E_EMPTY, "p0 (%.3f, %.3f) is not traversable", p->p0_x, p->p0_y);
  const double wx = (double)W * res, wy = (double)H * res;
  // Remark 4: expansion attempts per round
  const int64_t N = (int64_t)std::ceil((double)W * (double)H * res * res / (p->rho * p->rho));
  std::vector<double> nx{p->p0_x}, ny{p->p0_y};
  std::vector<int32_t> par{-1};
  KdTree kd(nx, ny);
  kd.insert(0);
  const int64_t VW = (int64_t)std::ceil(wx / p->rho) + 1, VH = (int64_t)std::ceil(wy / p->rho) + 1;
  std::vector<uint8_t> have((size_t)(VW * VH), 0);
  std::vector<int32_t> reps;
  size_t scanned = 0;
  int64_t t = 0;
  int rounds = 0;
  bool full = false;
  const double r = p->robot_radius, emax = p->eta_max;
  while (true) {
    for (int64_t i = 0; i < N && !full; ++i, ++t) {
      const double rx = ox + unit(mix(p->seed + 2 * (uint64_t)t)) * wx;
      const double ry = oy + unit(mix(p->seed + 2 * (uint64_t)t + 1)) * wy;
      const int32_t nb = kd.nearest(rx, ry);
      const double px = nx[nb], py = ny[nb];
      // AdaptiveExpandDist from the EDT of p_nearest's cell
      const int64_t cx = (int64_t)std::floor((px - ox) / res);
      const int64_t cy = (int64_t)std::floor((py - oy) / res);
      const double d = std::sqrt((double)k[cy * W + cx]) * res;
      double eta;
      if (d >= 2.0 * r) eta = emax;
      else if (d <= r) eta = r;
      else eta = r + (emax - r) * (d - r) / r;
      // ExtendPoint
      const double vx = rx - px, vy = ry - py;
      const double L = std::sqrt(vx * vx + vy * vy);
      if (L == 0.0) continue;
      double ex, ey;
      if (L <= eta) {
        ex = rx;
        ey = ry;
      } else {
        const double sc = eta / L;
        ex = px + vx * sc;
        ey = py + vy * sc;
      }
      // InSamplingBoundary, TraversabilityCheck at spacing <= res / 2
      if (!(ex >= ox && ex < ox + wx && ey >= oy && ey < oy + wy)) continue;
      const double sx = ex - px, sy = ey - py;
      const double Ls = std::sqrt(sx * sx + sy * sy);
      const int64_t n = std::max<int64_t>(1, (int64_t)std::ceil(Ls / (0.5 * res)));
      bool ok = true;
      for (int64_t j = 0; j <= n && ok; ++j) {
        const double tt = (double)j / (double)n;
        ok = feasible(px + sx * tt, py + sy * tt);
      }
      if (!ok) continue;
      nx.push_back(ex);
      ny.push_back(ey);
      par.push_back(nb);
      kd.insert((int32_t)nx.size() - 1);
      if ((int64_t)nx.size() >= p->max_nodes) full = true;
    }
    ++rounds;
    // VoxelDownsample: the first node of each new voxel represents it
    int64_t gain = 0;
    for (; scanned < nx.size(); ++scanned) {
      const int64_t vx = (int64_t)std::floor((nx[scanned] - ox) / p->rho);
      const int64_t vy = (int64_t)std::floor((ny[scanned] - oy) / p->rho);
      const int64_t key = vy * VW + vx;
      if (!have[key]) {
        have[key] = 1;
        reps.push_back((int32_t)scanned);
        ++gain;
      }
    }
    if (gain <= p->eps_gain || rounds >= p->max_rounds || full) break;
  }
  cells->clear();
  std::vector<uint8_t> used((size_t)W * H, 0);
  for (int32_t rp : reps) {
    const int64_t cx = (int64_t)std::floor((nx[rp] - ox) / res);
    const int64_t cy = (int64_t)std::floor((ny[rp] - oy) / res);
    const int64_t c = cy * W + cx;
    if (used[c]) continue;
    used[c] = 1;
    cells->push_back((int32_t)cx);
    cells->push_back((int32_t)cy);
  }
  if (nodes) {
    nodes->resize(2 * nx.size());
    for (size_t j = 0; j < nx.size(); ++j) {
      (*nodes)[2 * j] = nx[j];
      (*nodes)[2 * j + 1] = ny[j];
    }
  }
  if (parents) *parents = par;
  if (info) {
    info->rounds = rounds;
    info->attempts = t;
    info->nodes = (int64_t)nx.size();
    info->n_sampling = N;
  }
  return RELOC_OK;
}

}  // namespace reloc

using namespace reloc;

extern "C" {

void reloc_rrt_defaults(reloc_rrt_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->rho = 0.3;
  p->robot_radius = 0.21;
  p->eta_max = 0.6;
  p->eps_gain = 2;
  p->max_rounds = 64;
  p->max_nodes = 16 << 20;
  p->seed = 0;
}

int32_t reloc_sample_rrt(reloc_ctx* c, int32_t map_id, const reloc_rrt_params* p,
                         int32_t* set_id, int32_t* n_out, reloc_rrt_info* info, double* nodes_xy,
                         int32_t* parent, int32_t nodes_cap) {
  if (n_out) *n_out = 0;
  if (info) std::memset(info, 0, sizeof *info);
  if (!c || !p || !set_id || !n_out) return fail(RELOC_E_INVALID, "null argument");
  if ((nodes_xy || parent) && nodes_cap < 0) return fail(RELOC_E_INVALID, "negative nodes_cap");
  if (!std::isfinite(p->p0_x) || !std::isfinite(p->p0_y) || !std::isfinite(p->rho) ||
      !std::isfinite(p->eta_max))
    return fail(RELOC_E_INVALID, "p0, rho and eta_max must be finite");
  if (!(p->rho > 0) || !(p->robot_radius > 0) || !(p->eta_max >= p->robot_radius))
    return fail(RELOC_E_INVALID, "need rho > 0, robot_radius > 0, eta_max >= robot_radius");
  if (p->eps_gain < 0 || p->max_rounds < 1 || p->max_nodes < 1)
    return fail(RELOC_E_INVALID, "need eps_gain >= 0, max_rounds >= 1, max_nodes >= 1");
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  auto it = c->maps.find(map_id);
  if (it == c->maps.end()) return fail(RELOC_E_NOTFOUND, "unknown map %d", map_id);
  DevMap& m = it->second;
  // representatives end up de-duplicated per cell, so a voxel finer than a
  // cell adds nothing but attempts (Remark 4: N grows as 1 / rho^2) and
  // voxel flags (one byte per rho^2)
  if (!(p->rho >= m.res))
    return fail(RELOC_E_INVALID, "rho = %g m is below the map resolution %g m", p->rho, m.res);
  RELOC_GUARD_BEGIN
  if (int32_t e = ensure_khost(c, m)) return e;
  std::vector<int32_t> cells;
  std::vector<double> nodes;
  std::vector<int32_t> par;
  const bool want_tree = nodes_xy || parent;
  reloc_rrt_info inf{};
  if (int32_t e = rrt_sample(m, p, &cells, want_tree ? &nodes : nullptr,
                             want_tree ? &par : nullptr, &inf))
    return e;
  if (info) *info = inf;
  if (want_tree) {
    const size_t nn = std::min<size_t>(par.size(), (size_t)nodes_cap);
    if (nodes_xy) std::memcpy(nodes_xy, nodes.data(), 2 * nn * sizeof(double));
    if (parent) std::memcpy(parent, par.data(), nn * sizeof(int32_t));
  }
  const int32_t n = (int32_t)(cells.size() / 2);
  if (int32_t e = new_set(c, map_id, std::move(cells), set_id)) return e;
  *n_out = n;
  return RELOC_OK;
  RELOC_GUARD_END
}

}  // extern "C"
