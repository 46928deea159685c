// Host-side state of libreloc shared by the single-request driver
// (runtime.cpp) and the batched / serving driver (batch.cpp).
#ifndef RELOC_RUNTIME_INTERNAL_H
#define RELOC_RUNTIME_INTERNAL_H

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "reloc.h"
#include "reloc_internal.h"

namespace reloc {

// Sets the thread-local error message; returns code.
int32_t fail(int32_t code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RELOC_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

// Body guard of an extern "C" entry point: a host allocation that fails
// (std::bad_alloc) becomes RELOC_E_NOMEM and any other exception
// RELOC_E_DEVICE, so nothing propagates across the ABI.
#define RELOC_GUARD_BEGIN try {
#define RELOC_GUARD_END                                                                \
  }                                                                                    \
  catch (const std::bad_alloc&) {                                                      \
    return fail(RELOC_E_NOMEM, "host allocation failed");                              \
  }                                                                                    \
  catch (...) {                                                                        \
    return fail(RELOC_E_DEVICE, "unexpected host exception");                          \
  }

// ---- scan preprocessing (eq. 11-16, 25-26) ---------------------------------
struct Prep {
  reloc_scan_info info{};
  std::vector<int2> runs;         // (panoramic start, length) per FoV run
  std::vector<int32_t> vj, vzq;   // valid beams: panoramic index, range in Q8 cells
  std::vector<int32_t> fj;        // FoV beams in beam order: panoramic index
  std::vector<double> fz;         //   and measured range z' (0 when invalid)
};
int32_t preprocess(const reloc_scan* sc, const reloc_search_params* p, double res, Prep* out);

// ---- likelihood table for TAM (eq. 23) --------------------------------------
struct Lut {
  // Q26 likelihood per selection key less qmin (>= 0); 2^keybits entries
  std::vector<int32_t> q;
  int32_t qmin = 0;         // the smallest likelihood of a reachable key
  int kcap = 1, key_off = 2, keybits = 12;
};
int32_t build_lut(const reloc_search_params* p, double res, Lut* L);

// Direction-derived tables of one beam grid: the N_g direction table, and
// per panoramic beam its direction, metres per Q8 unit along each axis and
// the skip traversal's per-direction constants.
struct DirTables {
  int Ng = 0, Ns = 0;
  double res = 0.0;
  std::vector<int2> U, rd;
  std::vector<float2> kp;
  std::vector<int4> di;
  std::vector<float4> df;
};

struct ServeState;   // batch.cpp

// Stages of one request in one batched tick, at most.
constexpr int kMaxTickStages = 32;

}  // namespace reloc

using reloc::fail;
using reloc::Lut;
using reloc::PoseRow;
using reloc::Prep;

struct DevMap {
  // fused ray-cast shape last chosen by reloc_autotune for requests of this
  // map with fuse_ns directions (0: none); later requests start from it
  int fuse_ns = 0, fuse_nw = 0, fuse_refill = 0;
  int W = 0, H = 0, thr = 65, tpr = 0, tph = 0;
  double res = 0.05, ox = 0, oy = 0;
  uint64_t* bits = nullptr;
  uint16_t* walk = nullptr;       // null when the map exceeds kWalkMaxCells
  uint32_t* kmap = nullptr;
  uint32_t* plane = nullptr;      // TAM planes (tam_plane_bytes)
  std::vector<int8_t> occ;        // host copy for the sampler
  std::vector<uint32_t> khost;    // host copy of the EDT (filled on demand)
  int n_sets = 0;
};

struct HypSet {
  int map_id = -1;
  int n = 0;
  int32_t* dev = nullptr;         // [n][2]
  std::vector<int32_t> host;
  // casting order: the hypotheses sorted by the Morton (Z-order) code of
  // their cells, ties by index; on the host and on the device
  std::vector<int32_t> morton;
  int32_t* morton_dev = nullptr;  // [n]
};

struct Request {
  int map_id = -1, set_id = -1, n_hyp = 0;
  Prep prep;
  reloc_search_params prm{};
  float rmax = 0.f;
  int rcells = 0;
  int tuned_chunk = 0;            // rays per ray-cast chunk chosen by reloc_autotune (0: rule)
  // fused ray cast + SMAD: wavefronts per hypothesis workgroup and lane
  // refill threshold chosen by reloc_autotune (0: the default rule)
  int fuse_nw = 0, fuse_refill = 0;
  bool fused = false;             // set by init_request: see fused_path
  Lut lut;
  // device tables
  int2* raydirs = nullptr;
  float2* kap = nullptr;
  int4* dir_i = nullptr;
  float4* dir_f = nullptr;
  float* zbuf = nullptr;
  int32_t* perm = nullptr;        // hypotheses in Morton order of their cells
  int2* runs = nullptr;
  int2* beams = nullptr;          // valid beams (direction base, Q8 range), padded
  double* fov_z = nullptr;        // FoV beams' z' and panoramic index (direct coarse
  int32_t* fov_j = nullptr;       // metrics only)
  int2* dirs = nullptr;
  int32_t* dlut = nullptr;
  uint32_t* off = nullptr;        // TAM endpoint offsets [Ng][off_stride]
  int off_stride = 0;
  // device work
  double* smad = nullptr;
  int32_t* argm = nullptr;
  uint64_t* keys = nullptr;
  uint64_t* keys2 = nullptr;
  int32_t* vals = nullptr;
  int32_t* order = nullptr;
  int32_t* pos2 = nullptr;        // [n] scratch of the ranking sort
  uint64_t* best = nullptr;
  // local refinement: lattice half-widths and size, slots per launch
  int ref_h = 0, ref_s = 0, ref_L = 0, ref_slots = 0;
  int32_t* rsel = nullptr;        // [ref_slots] refined rank per slot
  uint64_t* rbest = nullptr;      // [ref_slots] lattice best per slot
  uint64_t* stage = nullptr;
  int32_t* flag = nullptr;
  PoseRow* rows = nullptr;
  int rows_cap = 0;
  hipGraphExec_t head = nullptr;  // captured head of reloc_run, or null
  int runs_done = 0;              // completed runs (the head is captured on the second)
  std::vector<void*> owned;
  // when set, req_alloc carves the request's device buffers out of this
  // region (256-byte aligned) instead of allocating them; nothing is owned
  uint8_t* carve_base = nullptr;
  size_t carve_cap = 0, carve_used = 0;
};

struct reloc_ctx {
  reloc::ServeState* serve = nullptr;   // batch staging and the submit / poll scheduler
  std::mutex reg_mu;                    // guards the maps / sets registries for submit

  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  reloc_allocator alloc{};
  bool has_alloc = false;
  size_t budget = 0, used = 0;
  std::map<void*, size_t> sizes;
  std::recursive_mutex mu;
  std::map<int, DevMap> maps;
  std::map<int, HypSet> sets;
  std::map<int, Request> reqs;
  int next_id = 1;
  hipEvent_t ev[6] = {};
  void* pinned = nullptr;         // small pinned staging buffer
  void* prows = nullptr;          // pinned result rows
  size_t prows_cap = 0;
  // two pinned staging buffers for request tables: a copy out of one is
  // asynchronous, and the buffer is rewritten only after its event
  void* tstage[2] = {};
  size_t tstage_cap[2] = {};
  hipEvent_t tstage_ev[2] = {};
  bool tstage_armed[2] = {};
  int tstage_next = 0;

  // Device blocks are handed out in size classes (powers of two up to
  // 1 MiB, then multiples of 2 MiB). A freed block of at most
  // kCacheBlockMax bytes is kept for a later allocation of its class
  // instead of going back to the allocator: every use of device memory is
  // queued on `stream`, so work that reuses a block runs after the last use
  // of its previous owner. Live blocks (`used`) plus kept ones never exceed
  // the budget: kept blocks go back to the allocator before an allocation
  // would pass it, when the allocator fails, and at destruction.
  // likelihood tables of recent parameter sets (z_hit, sigma_hit, z_rand,
  // d_max, resolution), so that requests with the same ones skip the host
  // build (about 40 us at sigma_hit = 0.2 m, r = 0.05 m); own lock, since
  // submit prepares requests on the caller's thread
  struct LutEntry {
    double key[5];
    Lut lut;
  };
  std::mutex lut_mu;
  std::vector<LutEntry> luts;     // most recent last, at most kLutCache
  static constexpr size_t kLutCache = 8;
  // direction tables of recent beam grids (N_g, N_s, resolution): the same
  // for every request of a grid (68 us at N_g = 720, 158 us at 1440 to
  // build); guarded by lut_mu too, most recent last
  std::vector<std::shared_ptr<const reloc::DirTables>> dirs;

  std::multimap<size_t, void*> cache;
  size_t cached = 0;
  static constexpr size_t kCacheBlockMax = (size_t)256 << 20;
  static constexpr size_t kCacheMax = (size_t)2 << 30;

  static size_t size_class(size_t bytes) {
    if (bytes <= ((size_t)1 << 20)) {
      size_t c = 256;
      while (c < bytes) c <<= 1;
      return c;
    }
    const size_t m = (size_t)2 << 20;
    return (bytes + m - 1) / m * m;
  }
  void* raw_alloc(size_t bytes) {
    void* p = nullptr;
    if (has_alloc) return alloc.alloc(bytes, alloc.user);
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void raw_free(void* p) {
    if (has_alloc)
      alloc.free(p, alloc.user);
    else
      (void)hipFree(p);
  }
  void flush_cache() {
    for (auto& kv : cache) raw_free(kv.second);
    cache.clear();
    cached = 0;
  }
  void* dalloc(size_t bytes) {
    const size_t cls = size_class(bytes == 0 ? 1 : bytes);
    if (used + cls > budget) {
      fail(RELOC_E_NOMEM, "HBM budget exceeded: %zu in use + %zu requested > %zu", used, cls,
           budget);
      return nullptr;
    }
    void* p = nullptr;
    auto it = cache.find(cls);
    if (it != cache.end()) {
      p = it->second;
      cache.erase(it);
      cached -= cls;
    } else {
      if (used + cached + cls > budget) flush_cache();
      p = raw_alloc(cls);
      if (!p && !cache.empty()) {
        flush_cache();
        p = raw_alloc(cls);
      }
    }
    if (!p) {
      fail(RELOC_E_NOMEM, "device allocation of %zu bytes failed", cls);
      return nullptr;
    }
    sizes[p] = cls;
    used += cls;
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    auto it = sizes.find(p);
    if (it == sizes.end()) return;
    const size_t sz = it->second;
    used -= sz;
    sizes.erase(it);
    if (sz <= kCacheBlockMax && cached + sz <= kCacheMax) {
      cache.emplace(sz, p);
      cached += sz;
    } else {
      raw_free(p);
    }
  }
};

namespace reloc {

int32_t set_device(reloc_ctx* c);
void release_request(reloc_ctx* c, Request& r);
// Destroys the request's captured head graph, if any.
void drop_head(Request& r);
int32_t validate_search(const reloc_search_params* p);
// Coarse-metric evaluations of a request (hypotheses x shifts scored).
int64_t coarse_evals(const Request& R);
// Refinement lattice of a request: half-widths h (cells), s (Ng headings;
// refine_dirs < 0 means Ng / N_theta) and size L = (2s + 1)(2h + 1)^2;
// RELOC_E_INVALID when s >= Ng or L > 65536.
int32_t refine_lattice(const reloc_search_params* p, const reloc_scan_info& I, int* h, int* s,
                       int* L);
// Host preprocessing of a request (no device work): fills R's map, set,
// parameters, Prep and limits. build_request then allocates and uploads.
int32_t init_request(reloc_ctx* c, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                     const reloc_search_params* params, Request* R);
int32_t build_request(reloc_ctx* c, Request& R);
// The whole device path of a built request (reloc_run's body). dev_rows:
// null to stage result rows in the context's pinned buffer, else device
// memory of at least R.rows_cap rows that receives them (copied to the host
// before returning); no head graph then.
int32_t run_request(reloc_ctx* c, Request& R, reloc_pose* out, int32_t cap, int32_t* n_out,
                    reloc_stats* st, PoseRow* dev_rows);
// Per-device scratch of the no-allocation entry point (noalloc.hip): looks
// up the address of the device's copy once, with the device current.
int32_t noalloc_setup(int device);
RayArgs ray_args(reloc_ctx* c, Request& R, int32_t* dbg_hit, int32_t* dbg_steps);
// Whether the request's ray cast and SMAD run as the fused kernel (coarse
// metric 0, default variant, a map with walk words): no range buffer then.
bool fused_path(const reloc_ctx* c, const Request& R);
// Workgroup shape of the fused kernel for R: tuned, else the default rule.
void fused_shape(const Request& R, int* nw, int* refill);
int fused_default_nw(int64_t n_hyp);
// Ray cast and coarse metric of every hypothesis of R (smad, argm, keys,
// vals; ra.best0 cleared when set): the fused kernel, or the ray cast into
// the range buffer and the coarse kernel. `mid`, when not null, is recorded
// between the two launches (after the fused kernel).
int32_t enqueue_front(reloc_ctx* c, Request& R, const RayArgs& ra, hipEvent_t mid);
TamArgs tam_args(reloc_ctx* c, Request& R, int r0, int nb, float* T_out);
RefineArgs refine_args(reloc_ctx* c, Request& R, int n_slots);
// Stages per TAM launch of the plain path (several when a stage alone
// cannot fill the device).
int plain_stages_per_launch(const Request& R);
// Stages of the later plain-path launches, at most (each launch after the
// first doubles the previous one up to this).
int plain_max_stages_per_launch(const Request& R);
// Device bytes build_request will allocate for R (admission control).
size_t request_bytes(const Request& R);
// Ambiguity statistics from the margin kernel's three words (fragile: the
// stop-decision bit when the caller tracked it itself).
void fill_ambiguity(const uint64_t* marg, bool fragile, reloc_stats* st);
// Launches the ambiguity kernel of a finished request: per-rank words best,
// SMAD order, device rows (row 0 = top-1), stage bests (or null); writes
// out[0..2] (device memory, or pinned host memory the device can address).
int32_t enqueue_margin(reloc_ctx* c, Request& R, const uint64_t* best, const int32_t* order,
                       const PoseRow* rows, int n_eval, const uint64_t* stage, int n_stages,
                       uint64_t* out);
// Converts device result rows to poses in world coordinates.
void rows_to_poses(const reloc_ctx* c, const Request& R, const PoseRow* rows, int n,
                   reloc_pose* out);
// Host copy of the map's EDT (copied from the device on first use).
int32_t ensure_khost(reloc_ctx* c, DevMap& m);
// Registers a hypothesis set of (ix, iy) cells on the map.
int32_t new_set(reloc_ctx* c, int map_id, std::vector<int32_t>&& xy, int32_t* set_id);
// Traversability-constrained RRT on the host copy of a map (rrt.cpp):
// hypothesis cells (x, y pairs), optionally the tree (x, y pairs and
// parents), and the run's counts.
int32_t rrt_sample(const DevMap& m, const reloc_rrt_params* p, std::vector<int32_t>* cells,
                   std::vector<double>* nodes, std::vector<int32_t>* parents,
                   reloc_rrt_info* info);
ServeState* serve_create();
void ctx_stop_serving(reloc_ctx* c);
// true while a queued or running served request uses the set
bool serve_holds_set(reloc_ctx* c, int32_t set_id);

template <typename T>
T* req_alloc(reloc_ctx* c, Request& r, size_t count) {
  if (r.carve_base) {
    const size_t off = (r.carve_used + 255) & ~(size_t)255;
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    if (off > r.carve_cap || bytes > r.carve_cap - off) {
      fail(RELOC_E_NOMEM, "the request needs more than the %zu-byte no-allocation scratch "
                          "(about %zu bytes by the admission estimate)",
           r.carve_cap, request_bytes(r));
      return nullptr;
    }
    r.carve_used = off + bytes;
    return (T*)(r.carve_base + off);
  }
  void* p = c->dalloc(count * sizeof(T));
  if (p) r.owned.push_back(p);
  return (T*)p;
}

template <typename T>
int32_t upload(reloc_ctx* c, T* dst, const T* src, size_t count) {
  if (count == 0) return RELOC_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return RELOC_OK;
}

// Copies n bytes to the device through the context's next pinned staging
// buffer, on c->stream; returns without waiting for the copy (the source
// may go out of scope at once).
int32_t upload_staged(reloc_ctx* c, void* dst, const void* src, size_t n);

}  // namespace reloc

#endif  // RELOC_RUNTIME_INTERNAL_H
