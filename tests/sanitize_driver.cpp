// Drives every function of the oracle on small seeded inputs. The sanitizer
// test compiles this file together with oracle/reloc_oracle.cpp under
// AddressSanitizer and UndefinedBehaviorSanitizer (no OpenMP) and runs it;
// any out-of-bounds access, leak or undefined operation aborts the run.
// Cross-checks on the way: the fast EDT equals the brute-force one, and the
// crossing-merge ray cast equals the slab-intersection one.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

typedef int64_t i64;
typedef uint64_t u64;

extern "C" {
int orc_edt_brute(int W, int H, const int8_t* occ, int thr, i64* k);
int orc_edt(int W, int H, const int8_t* occ, int thr, i64* k);
void orc_dirs(int Ng, int32_t* U);
int orc_raycast(int W, int H, const int8_t* occ, int thr, int Ng, int Ns, double res,
                float range_max, int n_hyp, const int32_t* hyp_xy, int brute, int32_t* hit,
                float* rng, int threads);
int orc_prep(int n_beams, const float* ranges, double angle_min, double angle_inc, int n_fov,
             const double* fov_lo, const double* fov_hi, float range_min, float range_max,
             int n_skip_beam, int n_skip_enum, int n_theta, double res,
             const int32_t* alpha_mid_pm, const int32_t* alpha_low_pm, i64* info, double* dinfo,
             int32_t* beam_j, int32_t* beam_state, double* beam_z, int32_t* beam_zq);
int orc_smad(int n_hyp, int Ns, const float* zhat, int n_fov_beams, const int32_t* fov_j,
             double zbar, int n_enum, int panoramic, double* smad, int32_t* argm,
             double* all_out, int threads);
int orc_caer(int n_hyp, int Ns, const float* zhat, int n_fov_beams, const int32_t* fov_j,
             const double* fov_z, int n_enum, double* caer, int32_t* argm, double* all_out,
             int threads);
int orc_tam(int W, int H, const i64* kmap, double res, int Ns, int Nt, int nv, const int32_t* vj,
            const int32_t* vzq, i64 kfull, i64 kmid, i64 klow, double z_hit, double sigma,
            double z_rand, double d_max, int nq, const int32_t* q_xy, const int32_t* q_k,
            double* out, int threads);
int orc_refine(int W, int H, const i64* kmap, double res, int Ns, int Nt, int nv,
               const int32_t* vj, const int32_t* vzq, i64 kfull, i64 kmid, i64 klow,
               double z_hit, double sigma, double z_rand, double d_max, int fine, int h, int s,
               int nq, const int32_t* q_xy, const i64* q_g, double* T, int32_t* dxy, i64* g,
               double* all, int threads);
int orc_stages(int W, int H, const i64* kmap, double res, int Ns, int Nt, int nv,
               const int32_t* vj, const int32_t* vzq, i64 kfull, i64 kmid, i64 klow,
               double z_hit, double sigma, double z_rand, double d_max, int n_hyp,
               const int32_t* hyp_xy, const double* smad, int K, double tau, int fine, int kr,
               int rh, int rs, int32_t* order, double* tstar, int32_t* kstar, i64* ref,
               i64* stage_info, double* all_T, int threads);
int orc_sample(int W, int H, const int8_t* occ, int thr, const i64* kmap, double res, double ox,
               double oy, double min_spacing, double robot_radius, int has_p0, double p0x,
               double p0y, u64 seed, int n_target, int32_t* out_xy, int32_t* n_out);
int orc_rrt(int W, int H, const int8_t* occ, int thr, const i64* kmap, double res, double ox,
            double oy, double p0x, double p0y, double rho, double r_robot, double eta_max,
            int eps_gain, u64 seed, int max_rounds, int max_nodes, double* nodes_xy,
            int32_t* parent, int32_t* cells_xy, i64* info);
}

static u64 state = 88172645463325252ULL;
static u64 next_u64() {   // xorshift64: input generation only
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return state;
}
static double uni() { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                               \
    }                                                         \
  } while (0)

static int one_map(int W, int H, int n_boxes) {
  std::vector<int8_t> occ((size_t)W * H, 0);
  for (int x = 0; x < W; ++x) occ[x] = occ[(size_t)(H - 1) * W + x] = 100;
  for (int y = 0; y < H; ++y) occ[(size_t)y * W] = occ[(size_t)y * W + W - 1] = 100;
  for (int b = 0; b < n_boxes; ++b) {
    const int x0 = 2 + (int)(uni() * (W - 8)), y0 = 2 + (int)(uni() * (H - 8));
    for (int y = y0; y < y0 + 3; ++y)
      for (int x = x0; x < x0 + 3; ++x) occ[(size_t)y * W + x] = 100;
  }
  for (size_t c = 0; c < occ.size(); ++c)
    if (occ[c] == 0 && uni() < 0.02) occ[c] = -1;   // a few unknown cells
  const double res = 0.05;
  std::vector<i64> k((size_t)W * H), kb((size_t)W * H);
  CHECK(orc_edt(W, H, occ.data(), 65, k.data()) == 0);
  CHECK(orc_edt_brute(W, H, occ.data(), 65, kb.data()) == 0);
  for (size_t c = 0; c < k.size(); ++c) CHECK(k[c] == kb[c]);
  // hypotheses
  std::vector<int32_t> hyp(2 * 40);
  int32_t nh = 0;
  CHECK(orc_sample(W, H, occ.data(), 65, k.data(), res, 0.0, 0.0, 0.15, 0.1, 0, 0, 0, 7, 40,
                   hyp.data(), &nh) == 0);
  CHECK(nh > 0);
  // scan (270 deg of a 240-direction grid) and preprocessing
  const int Ns = 240, nb = 180;
  std::vector<float> z(nb);
  for (int i = 0; i < nb; ++i) z[i] = uni() < 0.05 ? NAN : (float)(0.1 + 2.0 * uni());
  std::vector<i64> info(16);
  std::vector<double> dinfo(4);
  std::vector<int32_t> bj(nb), bs(nb), bq(nb);
  std::vector<double> bz(nb);
  const int32_t am[2] = {900, 700}, al[2] = {700, 500};
  const double inc = 2 * M_PI / Ns;
  CHECK(orc_prep(nb, z.data(), -(nb / 2) * inc, inc, 0, nullptr, nullptr, 0.02f, 10.f, 1, 1, 60,
                 res, am, al, info.data(), dinfo.data(), bj.data(), bs.data(), bz.data(),
                 bq.data()) == 0);
  const int Ng = (int)info[3], Nt = (int)info[2];
  std::vector<int32_t> fj, vj, vzq;
  std::vector<double> fz;
  for (int i = 0; i < nb; ++i) {
    if (bs[i] >= 1) {
      fj.push_back(bj[i]);
      fz.push_back(bz[i]);
    }
    if (bs[i] == 2) {
      vj.push_back(bj[i]);
      vzq.push_back(bq[i]);
    }
  }
  // ray casts (fast and brute force agree)
  std::vector<int32_t> hit((size_t)nh * Ns), hit2((size_t)nh * Ns);
  std::vector<float> zh((size_t)nh * Ns), zh2((size_t)nh * Ns);
  CHECK(orc_raycast(W, H, occ.data(), 65, Ng, Ns, res, 10.f, nh, hyp.data(), 0, hit.data(),
                    zh.data(), 0) == 0);
  CHECK(orc_raycast(W, H, occ.data(), 65, Ng, Ns, res, 10.f, nh, hyp.data(), 1, hit2.data(),
                    zh2.data(), 0) == 0);
  for (size_t i = 0; i < hit.size(); ++i) CHECK(hit[i] == hit2[i] && zh[i] == zh2[i]);
  // coarse metrics
  std::vector<double> sm(nh), ca(nh), all((size_t)nh * Ns);
  std::vector<int32_t> sa(nh), ca_m(nh);
  CHECK(orc_smad(nh, Ns, zh.data(), (int)fj.size(), fj.data(), dinfo[0], 1, (int)info[9],
                 sm.data(), sa.data(), all.data(), 0) == 0);
  CHECK(orc_caer(nh, Ns, zh.data(), (int)fj.size(), fj.data(), fz.data(), 1, ca.data(),
                 ca_m.data(), all.data(), 0) == 0);
  // TAM, refinement and the stage loop, every fine metric
  const int nv = (int)vj.size();
  std::vector<int32_t> qk(nh);
  for (int i = 0; i < nh; ++i) qk[i] = i % Nt;
  std::vector<double> out((size_t)nh * 11);
  CHECK(orc_tam(W, H, k.data(), res, Ns, Nt, nv, vj.data(), vzq.data(), info[6], info[7],
                info[8], 1.0, 0.2, 0.0, 2.0, nh, hyp.data(), qk.data(), out.data(), 0) == 0);
  for (int fine = 0; fine < 4; ++fine) {
    std::vector<i64> qg(nh);
    for (int i = 0; i < nh; ++i) qg[i] = (i * 7) % Ng;
    std::vector<double> T(nh), lat((size_t)nh * 3 * 9);
    std::vector<int32_t> dxy(2 * nh);
    std::vector<i64> g(nh);
    CHECK(orc_refine(W, H, k.data(), res, Ns, Nt, nv, vj.data(), vzq.data(), info[6], info[7],
                     info[8], 1.0, 0.2, 0.0, 2.0, fine, 1, 1, nh, hyp.data(), qg.data(),
                     T.data(), dxy.data(), g.data(), lat.data(), 0) == 0);
    std::vector<int32_t> order(nh), kstar(nh);
    std::vector<double> tstar(nh), allT((size_t)nh * Nt);
    std::vector<i64> ref(4 * (size_t)nh), si(4);
    CHECK(orc_stages(W, H, k.data(), res, Ns, Nt, nv, vj.data(), vzq.data(), info[6], info[7],
                     info[8], 1.0, 0.2, 0.0, 2.0, nh, hyp.data(), sm.data(), 7, 0.5, fine, 2, 2,
                     1, order.data(), tstar.data(), kstar.data(), ref.data(), si.data(),
                     allT.data(), 0) == 0);
  }
  // RRT from the first hypothesis
  const int cap = 200000;
  std::vector<double> nodes(2 * (size_t)cap);
  std::vector<int32_t> par(cap), cells(2 * (size_t)cap);
  std::vector<i64> rinfo(4);
  const int nc = orc_rrt(W, H, occ.data(), 65, k.data(), res, 0.0, 0.0, (hyp[0] + 0.5) * res,
                         (hyp[1] + 0.5) * res, 0.2, 0.1, 0.4, 2, 3, 64, cap, nodes.data(),
                         par.data(), cells.data(), rinfo.data());
  CHECK(nc > 0 && rinfo[2] > 1);
  return 0;
}

int main() {
  std::vector<int> dims = {31, 23, 64, 48, 90, 70};
  for (size_t i = 0; i < dims.size(); i += 2)
    if (one_map(dims[i], dims[i + 1], 4 + (int)i)) return 1;
  std::printf("sanitized oracle run ok\n");
  return 0;
}
