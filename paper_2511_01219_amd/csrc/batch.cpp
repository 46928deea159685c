// Batched execution of many prepared requests (possibly on different maps
// and scans) and the serving scheduler behind reloc_submit / reloc_poll.
//
// A batch runs in three phases on the context's stream:
//   front : one ray-cast launch and one SMAD launch over the hypotheses of
//           every request (per-request descriptors in device memory), then
//           one segmented stable sort for all SMAD orders (for small groups
//           one small sort per request);
//   ticks : each tick is one TAM launch per kernel class over a rank range
//           of every unfinished request plus one stage-control launch that
//           reduces every stage of the tick on the device; the host reads
//           one flag per stage. A request's range covers `spec` consecutive
//           stages (in its first two ticks as many as the plain path's first
//           launch, then twice as many each tick up to kMaxSpec), granted
//           oldest request first out of a per-tick budget
//           of TAM workgroups, at least one stage each; stages after the
//           first one whose best T exceeds tau are discarded, so the
//           evaluated set and every result equal those of the
//           one-stage-at-a-time path;
//   rank  : one segmented sort and one gather for every finished request.
// The serving scheduler repeats: admission -> front of the admitted requests
// on a second stream (same priority) -> one more tick of every request whose
// front has finished, on the context's stream -> the stop flags of the tick
// before it -> rank of the finished ones. Requests that arrive while others
// run start at once on the front stream and join the ticks at the next
// stage boundary after their front; two ticks are in flight, so the device
// works on tick t + 1 while the host reads the flags of tick t (a request
// that stopped in tick t has its share of tick t + 1 discarded). A small
// request that finds the device idle and nobody else waiting runs the plain
// path instead.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>

#include "runtime_internal.h"

namespace reloc {

namespace {

constexpr int kMaxSpec = kMaxTickStages;
constexpr int kSmallSortGroup = 8;      // front groups up to this size sort per request
constexpr int64_t kTickBlocks = 65536;  // TAM workgroups one tick may grant beyond one stage each
constexpr int kSoloMaxHyp = 8000;       // largest request served alone on the plain path

// Contiguous buffers of one front-phase group: SMAD sort keys / values, the
// SMAD order and the per-rank best of every request of the group.
struct Arena {
  reloc_ctx* c = nullptr;
  std::vector<void*> owned;
  uint64_t *keys = nullptr, *keys2 = nullptr, *best = nullptr;
  int32_t *vals = nullptr, *order = nullptr;
  ~Arena() {
    for (void* p : owned) c->dfree(p);
  }
  template <typename T>
  T* get(size_t n) {
    void* p = c->dalloc(std::max<size_t>(1, n) * sizeof(T));
    if (p) owned.push_back(p);
    return (T*)p;
  }
};

// The requests admitted together: their front phase's timing marks (the
// last one ends the phase) and, once it has ended, its phase times.
struct FrontGroup {
  hipEvent_t ev[4] = {};
  bool ready = false;
  float raycast = 0, smad = 0, sort = 0;
  ~FrontGroup() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// One request in batched execution.
struct Flight {
  int rid = -1;                     // key in c->reqs
  std::shared_ptr<Arena> arena;
  int64_t off = 0;                  // first hypothesis of the request in the arena
  int next_rank = 0, spec = 1, stages = 0, n_eval = 0, ticks = 0;
  int plan_rank = 0;                // first rank not yet in an enqueued tick
  int pending = 0;                  // enqueued ticks not yet completed
  float tam_ms = 0;                 // device time of the ticks it took part in
  std::shared_ptr<FrontGroup> fg;   // its front phase
  bool done = false, stopped = false;
  int32_t status = RELOC_OK;
  std::chrono::steady_clock::time_point t_start;
  int tentry = 0, tstages = 0, tnb = 0;   // the current tick
  uint64_t ticket = 0;                    // serving only
  bool fragile = false;                   // a stop decision within 1e-4 of tau
  uint64_t marg[3] = {0, 0, 0};           // ambiguity kernel output
};

struct Ticket {
  uint64_t id = 0;
  Request R;                        // host part prepared at submit
  bool done = false;
  int32_t status = RELOC_E_PENDING;
  std::string msg;                  // error text when status is an error
  std::vector<reloc_pose> poses;
  reloc_stats st{};
  std::chrono::steady_clock::time_point t_submit;
};

// Byte blob of descriptor tables, copied to the device in one transfer.
struct Blob {
  std::vector<uint8_t> b;
  template <typename T>
  size_t add(const T* p, size_t n) {
    const size_t off = (b.size() + 255) & ~(size_t)255;
    b.resize(off + n * sizeof(T));
    if (n) std::memcpy(b.data() + off, p, n * sizeof(T));
    return off;
  }
};

}  // namespace

// One staging slot for descriptor tables: a pinned host buffer, its device
// copy, and an event recorded after the copy out of the host buffer.
struct Staging {
  void* h = nullptr;
  size_t hcap = 0;
  uint8_t* d = nullptr;
  size_t dcap = 0;
  hipEvent_t ev = nullptr;
  bool armed = false;   // ev marks a copy that may still be reading h
};
constexpr int kStagingRing = 4;

// A ring of staging slots used by one stream: a slot's device buffer is
// rewritten by a copy queued on that stream behind every kernel that read it.
struct StagingRing {
  Staging slot[kStagingRing];
  int next = 0;
};

// One tick's share of a request: ranks [r0, r0 + nb), ns stages, whose
// stop flags start at entry.
struct TickItem {
  Flight* f;
  int r0, ns, nb, entry;
};

// One tick: its events (start, end), the pinned stop flags and stage words
// its stage kernel writes, and the requests it covers.
struct TickSlot {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t* hflag = nullptr;
  uint64_t* hstage = nullptr;
  size_t cap = 0;
  std::vector<TickItem> items;
};

// Ticks of one driver (a batch call or the serving worker), at most two in
// flight, completed in order.
struct TickPipe {
  TickSlot slot[2];
  std::deque<int> inflight;
  int next = 0;
};

struct ServeState {
  // staging of descriptor tables: a ring of slots per stream, so a commit
  // waits only for the copy made kStagingRing commits earlier, not for the
  // stream
  StagingRing ring;                 // the context's stream
  StagingRing fring;                // the serving front stream
  StagingRing rring;                // the serving rank stream
  hipStream_t sfront = nullptr;     // serving front phases (default priority)
  hipStream_t srank = nullptr;      // serving rankings (default priority)
  TickPipe pipe_batch, pipe_serve;
  // ranking scratch, grown on demand and kept between calls
  uint64_t* rk1 = nullptr;
  uint64_t* rk2 = nullptr;
  int32_t* rp1 = nullptr;          // positions of the ranking sort
  int32_t* rp2 = nullptr;
  size_t rk_cap = 0;
  PoseRow* rrows = nullptr;
  size_t rrows_cap = 0;
  uint64_t* rmarg = nullptr;
  size_t rmarg_cap = 0;
  // serving
  std::thread worker;
  bool running = false;
  std::mutex qmu;
  std::condition_variable qcv, dcv;
  bool stop = false;
  int pollers = 0;                  // reloc_poll calls inside (under qmu)
  std::deque<Ticket*> pending;
  std::map<uint64_t, std::unique_ptr<Ticket>> tickets;
  uint64_t next_ticket = 1;
  std::list<Flight> active;         // touched by the worker only (stable addresses)
  reloc_serve_config cfg{64, 0, 16};
  reloc_serve_stats stats{};
  int32_t worker_error = RELOC_OK;
};

namespace {

ServeState* state(reloc_ctx* c) { return c->serve; }

// Copies the blob to device memory through the next staging slot of the ring
// of c->stream; *dev receives the device address of offset 0. The slot's
// host buffer is rewritten only after the copy that last read it has
// completed; its device buffer is rewritten by a copy queued behind every
// kernel that read it.
int32_t commit(reloc_ctx* c, StagingRing& ring, const Blob& bl, uint8_t** dev) {
  Staging& g = ring.slot[ring.next];
  ring.next = (ring.next + 1) % kStagingRing;
  if (g.armed) {
    HIP_TRY(hipEventSynchronize(g.ev));
    g.armed = false;
  }
  const size_t need = std::max<size_t>(bl.b.size(), 256);
  if (need > g.hcap) {
    if (g.h) (void)hipHostFree(g.h);
    g.h = nullptr;
    const size_t cap = std::max(need, g.hcap * 2);
    g.hcap = 0;
    HIP_TRY(hipHostMalloc(&g.h, cap, hipHostMallocDefault));
    g.hcap = cap;
  }
  if (need > g.dcap) {
    // kernels queued earlier may still read the old device buffer
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->dfree(g.d);
    g.d = nullptr;
    g.dcap = 0;
    const size_t cap = std::max(need, (size_t)1 << 16);
    g.d = (uint8_t*)c->dalloc(cap);
    if (!g.d) return RELOC_E_NOMEM;
    g.dcap = cap;
  }
  if (!g.ev) HIP_TRY(hipEventCreateWithFlags(&g.ev, hipEventDisableTiming));
  std::memcpy(g.h, bl.b.data(), bl.b.size());
  HIP_TRY(hipMemcpyAsync(g.d, g.h, bl.b.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(g.ev, c->stream));
  g.armed = true;
  *dev = g.d;
  return RELOC_OK;
}

// Grow-only device scratch of n elements (at least); the stream is drained
// before a buffer that earlier work may still use is replaced.
template <typename T>
int32_t grow_scratch(reloc_ctx* c, T*& p, size_t& cap, size_t n) {
  n = std::max<size_t>(n, 1);
  if (p && n <= cap) return RELOC_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t nc = std::max(n, cap * 2);
  c->dfree(p);
  p = nullptr;
  cap = 0;
  p = (T*)c->dalloc(nc * sizeof(T));
  if (!p) return RELOC_E_NOMEM;
  cap = nc;
  return RELOC_OK;
}

// Stage outputs of a slot that no tick in flight uses.
int32_t ensure_stage_cap(TickSlot& t, size_t n) {
  if (!t.e0) HIP_TRY(hipEventCreate(&t.e0));
  if (!t.e1) HIP_TRY(hipEventCreate(&t.e1));
  if (n <= t.cap) return RELOC_OK;
  if (t.hflag) (void)hipHostFree(t.hflag);
  if (t.hstage) (void)hipHostFree(t.hstage);
  t.hflag = nullptr;
  t.hstage = nullptr;
  t.cap = 0;
  const size_t cap = std::max<size_t>(n, 1024);
  HIP_TRY(hipHostMalloc((void**)&t.hflag, cap * sizeof(int32_t), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&t.hstage, cap * sizeof(uint64_t), hipHostMallocDefault));
  t.cap = cap;
  return RELOC_OK;
}

void free_pipe(TickPipe& P) {
  for (TickSlot& t : P.slot) {
    if (t.hflag) (void)hipHostFree(t.hflag);
    if (t.hstage) (void)hipHostFree(t.hstage);
    if (t.e0) (void)hipEventDestroy(t.e0);
    if (t.e1) (void)hipEventDestroy(t.e1);
    t = TickSlot{};
  }
  P.inflight.clear();
}

void free_ring(reloc_ctx* c, StagingRing& r) {
  for (Staging& g : r.slot) {
    c->dfree(g.d);
    if (g.h) (void)hipHostFree(g.h);
    if (g.ev) (void)hipEventDestroy(g.ev);
    g = Staging{};
  }
}

struct PhaseTimes {
  float raycast = 0, smad = 0, sort = 0, tam = 0, rank = 0;
};

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventSynchronize(b);
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

// Ray cast, SMAD and SMAD order of the requests of F on c->stream, its
// descriptors through `ring` (the ring of that stream); F's flights get a
// shared arena, the group's events, and start at stage 0. Nothing waits
// for the device.
int32_t front(reloc_ctx* c, StagingRing& ring, std::vector<Flight*>& F) {
  const int n = (int)F.size();
  if (n == 0) return RELOC_OK;
  auto G = std::make_shared<FrontGroup>();
  for (hipEvent_t& e : G->ev) HIP_TRY(hipEventCreate(&e));
  auto A = std::make_shared<Arena>();
  A->c = c;
  std::vector<int64_t> hpre(n + 1, 0);
  for (int i = 0; i < n; ++i) hpre[i + 1] = hpre[i] + c->reqs.at(F[i]->rid).n_hyp;
  const int64_t N = hpre[n];
  if (N > INT32_MAX) return fail(RELOC_E_INVALID, "batch holds more than 2^31 hypotheses");
  A->keys = A->get<uint64_t>(N);
  A->keys2 = A->get<uint64_t>(N);
  A->best = A->get<uint64_t>(N);
  A->vals = A->get<int32_t>(N);
  A->order = A->get<int32_t>(N);
  if (!A->keys || !A->keys2 || !A->best || !A->vals || !A->order) return RELOC_E_NOMEM;
  // every request's SMAD order in one segmented sort (tiles of 1024 keys
  // per request, then the merge levels of the largest request)
  std::vector<int64_t> tpre(n + 1, 0);
  int64_t max_n = 0;
  for (int i = 0; i < n; ++i) {
    tpre[i + 1] = tpre[i] + argsort_tiles(hpre[i + 1] - hpre[i]);
    max_n = std::max(max_n, hpre[i + 1] - hpre[i]);
  }
  // requests on the fused path share one launch (one workgroup per
  // hypothesis); the others (ablation metrics, maps without walk words)
  // cast into their range buffers and run their coarse kernel one by one
  std::vector<RayArgs> ra(n), fra;
  std::vector<int64_t> fpre(1, 0);
  int max_ns = 0;                     // largest Ns of a non-panoramic fused request
  for (int i = 0; i < n; ++i) {
    Request& R = c->reqs.at(F[i]->rid);
    RayArgs a = ray_args(c, R, nullptr, nullptr);
    a.keys = A->keys + hpre[i];
    a.vals = A->vals + hpre[i];
    a.best0 = A->best + hpre[i];      // the coarse kernel clears the per-rank best
    ra[i] = a;
    if (R.fused) {
      fra.push_back(a);
      fpre.push_back(fpre.back() + R.n_hyp);
      if (a.n_shifts != 1) max_ns = std::max(max_ns, a.Ns);
    }
  }
  const int nf = (int)fra.size();
  const int nw = fused_default_nw(fpre.back());
  const size_t lds = max_ns ? fused_lds_bytes(max_ns, nw) : 0;
  Blob bl;
  const size_t o_ra = bl.add(fra.data(), std::max(nf, 1));
  const size_t o_fp = bl.add(fpre.data(), nf + 1);
  const size_t o_hp = bl.add(hpre.data(), n + 1);
  const size_t o_tp = bl.add(tpre.data(), n + 1);
  uint8_t* d = nullptr;
  if (int32_t e = commit(c, ring, bl, &d)) return e;
  const RayArgs* d_ra = (const RayArgs*)(d + o_ra);
  const int64_t* d_fp = (const int64_t*)(d + o_fp);
  const int64_t* d_hp = (const int64_t*)(d + o_hp);
  const int64_t* d_tp = (const int64_t*)(d + o_tp);
  hipStream_t s = c->stream;
  HIP_TRY(hipEventRecord(G->ev[0], s));
  if (nf > 0) HIP_TRY(launch_raycast_smad_fused_batch(d_ra, d_fp, nf, fpre.back(), nw, lds, s));
  for (int i = 0; i < n; ++i)
    if (!c->reqs.at(F[i]->rid).fused && ra[i].coarse != 3) HIP_TRY(launch_raycast(ra[i], s));
  HIP_TRY(hipEventRecord(G->ev[1], s));
  for (int i = 0; i < n; ++i)
    if (!c->reqs.at(F[i]->rid).fused) HIP_TRY(launch_coarse(ra[i], s));
  HIP_TRY(hipEventRecord(G->ev[2], s));
  // keys2 and vals serve as the sort's scratch
  HIP_TRY(argsort_u64(A->keys, A->keys2, A->vals, A->order, N, n, d_hp, d_tp, tpre[n], max_n, s));
  HIP_TRY(hipEventRecord(G->ev[3], s));
  for (int i = 0; i < n; ++i) {
    Flight& f = *F[i];
    f.fg = G;
    f.arena = A;
    f.off = hpre[i];
    f.next_rank = 0;
    f.plan_rank = 0;
    f.pending = 0;
    // first ticks as large as the plain path's first launches
    f.spec = std::min(kMaxSpec, plain_stages_per_launch(c->reqs.at(f.rid)));
    f.ticks = 0;
    f.stages = 0;
    f.n_eval = 0;
    f.done = false;
  }
  return RELOC_OK;
}

// Whether the group's front phase has ended (its phase times taken then);
// with wait, blocks until it has.
bool front_done(FrontGroup& G, bool wait) {
  if (G.ready) return true;
  if (wait) {
    if (hipEventSynchronize(G.ev[3]) != hipSuccess) return false;
  } else if (hipEventQuery(G.ev[3]) != hipSuccess) {
    return false;
  }
  G.raycast = elapsed(G.ev[0], G.ev[1]);
  G.smad = elapsed(G.ev[1], G.ev[2]);
  G.sort = elapsed(G.ev[2], G.ev[3]);
  G.ready = true;
  return true;
}

// Enqueues one tick over the flights of F that are not done and have
// stages left (from their planned rank on), into the pipe's next slot, on
// c->stream; *enq tells whether there was any. Nothing waits for the device.
int32_t enqueue_tick(reloc_ctx* c, TickPipe& P, StagingRing& ring, std::vector<Flight*>& F,
                     bool* enq) {
  *enq = false;
  std::vector<TamArgs> items[kTamClasses];
  std::vector<StageArgs> st;
  std::vector<Flight*> live;
  for (Flight* f : F)
    if (!f->done && f->plan_rank < c->reqs.at(f->rid).n_hyp) live.push_back(f);
  if (live.empty()) return RELOC_OK;
  if (P.inflight.size() >= 2) return fail(RELOC_E_INVALID, "two ticks already in flight");
  const int si = P.next;
  TickSlot& T = P.slot[si];
  // stages per request this tick: the speculation schedule, granted oldest
  // request first out of a budget of TAM workgroups, at least one stage each
  std::vector<size_t> by_age(live.size());
  for (size_t j = 0; j < live.size(); ++j) by_age[j] = j;
  std::stable_sort(by_age.begin(), by_age.end(), [&](size_t x, size_t y) {
    return live[x]->t_start < live[y]->t_start;
  });
  std::vector<int> nst(live.size());
  size_t n_entries = 0;
  int64_t budget = kTickBlocks;
  for (size_t j : by_age) {
    const Flight* f = live[j];
    const Request& R = c->reqs.at(f->rid);
    const int K = R.prm.batch_k;
    const int left = (R.n_hyp - f->plan_rank + K - 1) / K;
    const int64_t bps = (int64_t)K * ((R.prep.info.Ntheta + 15) / 16);
    const int64_t cap = std::max<int64_t>(1, budget / bps);
    nst[j] = (int)std::min<int64_t>(std::min(f->spec, left), cap);
    budget -= nst[j] * bps;
    n_entries += (size_t)nst[j];
  }
  if (int32_t e = ensure_stage_cap(T, n_entries)) return e;
  T.items.clear();
  for (size_t j = 0; j < live.size(); ++j) {
    Flight* f = live[j];
    Request& R = c->reqs.at(f->rid);
    const int K = R.prm.batch_k;
    const int ns = nst[j];
    const int nb = std::min(ns * K, R.n_hyp - f->plan_rank);
    TamArgs a = tam_args(c, R, f->plan_rank, nb, nullptr);
    a.order = f->arena->order + f->off;
    a.best = f->arena->best + f->off;
    const int cls = tam_class(a);
    if (cls < 0) return fail(RELOC_E_INVALID, "TAM configuration outside the kernel classes");
    items[cls].push_back(a);
    T.items.push_back(TickItem{f, f->plan_rank, ns, nb, (int)st.size()});
    for (int b = 0; b < ns; ++b) {
      const int r0 = f->plan_rank + b * K;
      const size_t e = st.size();
      st.push_back(StageArgs{a.best, r0, std::min(K, R.n_hyp - r0), R.prm.tau, T.hstage + e,
                             T.hflag + e});
    }
  }
  Blob bl;
  size_t o_items[kTamClasses], o_pre[kTamClasses];
  int64_t blocks[kTamClasses];
  size_t lds[kTamClasses];
  for (int k = 0; k < kTamClasses; ++k) {
    const int m = (int)items[k].size();
    blocks[k] = 0;
    lds[k] = 0;
    if (!m) continue;
    std::vector<int64_t> pre(m + 1, 0);
    for (int i = 0; i < m; ++i) {
      const TamArgs& a = items[k][i];
      pre[i + 1] = pre[i] + (int64_t)a.nb * tam_tiles_per_rank(a);
      lds[k] = std::max(lds[k], tam_lds_bytes(a));
    }
    blocks[k] = pre[m];
    o_items[k] = bl.add(items[k].data(), m);
    o_pre[k] = bl.add(pre.data(), m + 1);
  }
  const size_t o_st = bl.add(st.data(), st.size());
  uint8_t* d = nullptr;
  if (int32_t e = commit(c, ring, bl, &d)) return e;
  hipStream_t s = c->stream;
  HIP_TRY(hipEventRecord(T.e0, s));
  for (int k = 0; k < kTamClasses; ++k) {
    if (!blocks[k]) continue;
    HIP_TRY(launch_tam_batch(k, (const TamArgs*)(d + o_items[k]), (const int64_t*)(d + o_pre[k]),
                             (int)items[k].size(), blocks[k], lds[k], s));
  }
  // local refinement of each stage's best poses, per refining request
  for (const TickItem& it : T.items) {
    Flight* f = it.f;
    Request& R = c->reqs.at(f->rid);
    const int kr = R.prm.refine_k;
    if (kr <= 0) continue;
    RefineArgs fa = refine_args(c, R, it.ns * kr);
    fa.t.order = f->arena->order + f->off;
    fa.t.best = f->arena->best + f->off;
    HIP_TRY(launch_refine_select(fa.t.best, it.r0, R.prm.batch_k, R.n_hyp, it.ns, kr, R.rsel,
                                 R.rbest, s));
    HIP_TRY(launch_refine(fa, s));
    HIP_TRY(launch_refine_commit(fa, s));
  }
  HIP_TRY(launch_stage_reduce_batch((const StageArgs*)(d + o_st), (int)st.size(), s));
  HIP_TRY(hipEventRecord(T.e1, s));
  for (const TickItem& it : T.items) {
    Flight* f = it.f;
    f->plan_rank += it.nb;
    ++f->pending;
    // the first two ticks as planned, then twice as many stages each tick
    if (++f->ticks >= 2) f->spec = std::min(kMaxSpec, f->spec * 2);
  }
  P.inflight.push_back(si);
  P.next ^= 1;
  *enq = true;
  return RELOC_OK;
}

// Waits for the oldest tick in flight and applies its stop flags: a request
// stops at the first of its stages whose best T exceeds tau (its share of
// later ticks is discarded), or advances by the tick's ranks.
int32_t complete_tick(reloc_ctx* c, TickPipe& P, PhaseTimes* pt) {
  if (P.inflight.empty()) return RELOC_OK;
  TickSlot& T = P.slot[P.inflight.front()];
  P.inflight.pop_front();
  HIP_TRY(hipEventSynchronize(T.e1));
  const float ms = elapsed(T.e0, T.e1);
  if (pt) pt->tam += ms;
  const auto now = std::chrono::steady_clock::now();
  for (const TickItem& it : T.items) {
    Flight* f = it.f;
    --f->pending;
    f->tam_ms += ms;
    if (f->done) continue;                  // stopped in an earlier tick
    const Request& R = c->reqs.at(f->rid);
    const int K = R.prm.batch_k;
    int hit = -1;
    for (int b = 0; b < it.ns; ++b)
      if (T.hflag[it.entry + b]) {
        hit = b;
        break;
      }
    if (!std::isnan(R.prm.tau)) {
      const int used = hit >= 0 ? hit + 1 : it.ns;
      for (int b = 0; b < used; ++b) {
        const double Tb = (double)score_of_key((uint32_t)(T.hstage[it.entry + b] >> 32));
        if (Tb >= R.prm.tau - 1e-4 && Tb <= R.prm.tau + 1e-4) f->fragile = true;
      }
    }
    if (hit >= 0) {
      f->stages += hit + 1;
      f->n_eval = std::min(R.n_hyp, it.r0 + (hit + 1) * K);
      f->done = true;
      f->stopped = true;
      continue;
    }
    f->stages += it.ns;
    f->next_rank = it.r0 + it.nb;
    f->n_eval = f->next_rank;
    if (f->next_rank >= R.n_hyp) {
      f->done = true;
      continue;
    }
    if (R.prm.deadline_s > 0 &&
        std::chrono::duration<double>(now - f->t_start).count() > R.prm.deadline_s) {
      f->done = true;
      f->status = RELOC_E_TIMEOUT;
    }
  }
  T.items.clear();
  return RELOC_OK;
}

// Ranked poses of finished flights: rows[i] receives min(cap[i], k_out,
// n_eval) rows of flight F[i].
int32_t rank(reloc_ctx* c, ServeState& S, StagingRing& ring, std::vector<Flight*>& F,
             const std::vector<int>& cap, std::vector<std::vector<PoseRow>>* rows,
             PhaseTimes* pt) {
  const int n = (int)F.size();
  rows->assign(n, {});
  if (n == 0) return RELOC_OK;
  std::vector<int64_t> kpre(n + 1, 0), rpre(n + 1, 0);
  std::vector<int> nrow(n, 0);
  std::vector<RankArgs> ra(n);
  for (int i = 0; i < n; ++i) {
    const Request& R = c->reqs.at(F[i]->rid);
    const int nr = std::max(0, std::min(std::min(R.rows_cap, F[i]->n_eval), cap[i]));
    nrow[i] = nr;
    kpre[i + 1] = kpre[i] + F[i]->n_eval;
    // the device holds row 0 of every evaluated request (the ambiguity
    // statistics read it)
    rpre[i + 1] = rpre[i] + (F[i]->n_eval > 0 ? std::max(1, nr) : 0);
    ra[i] = RankArgs{F[i]->arena->best + F[i]->off, F[i]->arena->order + F[i]->off, R.smad};
  }
  const int64_t NK = kpre[n], NR = rpre[n];
  // a small group of short rankings: one single-launch ranking per request
  // (the plain path's); otherwise one segmented sort for all. Both order by
  // (T desc, rank asc) over distinct keys, so the rows agree.
  bool per_request = n <= kSmallSortGroup;
  for (int i = 0; i < n && per_request; ++i) per_request = F[i]->n_eval <= kRankSmallMax;
  if (int32_t e = grow_scratch(c, S.rrows, S.rrows_cap, (size_t)NR)) return e;
  if (int32_t e = grow_scratch(c, S.rmarg, S.rmarg_cap, 3 * (size_t)n)) return e;
  PoseRow* dr = S.rrows;
  uint64_t* dmarg = S.rmarg;
  uint64_t* k1 = nullptr;
  uint64_t* k2 = nullptr;
  std::vector<int64_t> tpre(n + 1, 0);
  int64_t max_n = 0;
  if (!per_request) {
    // both key buffers and both position buffers share one capacity
    if (!S.rk1 || !S.rk2 || !S.rp1 || !S.rp2 || (size_t)NK > S.rk_cap) {
      size_t c1 = S.rk_cap, c2 = S.rk_cap, c3 = S.rk_cap, c4 = S.rk_cap;
      if (int32_t e = grow_scratch(c, S.rk1, c1, (size_t)NK)) return e;
      if (int32_t e = grow_scratch(c, S.rk2, c2, c1)) return e;
      if (int32_t e = grow_scratch(c, S.rp1, c3, c1)) return e;
      if (int32_t e = grow_scratch(c, S.rp2, c4, c1)) return e;
      S.rk_cap = std::min(std::min(c1, c2), std::min(c3, c4));
    }
    k1 = S.rk1;
    k2 = S.rk2;
    for (int i = 0; i < n; ++i) {
      tpre[i + 1] = tpre[i] + argsort_tiles(F[i]->n_eval);
      max_n = std::max<int64_t>(max_n, F[i]->n_eval);
    }
  }
  Blob bl;
  const size_t o_ra = bl.add(ra.data(), n);
  const size_t o_kp = bl.add(kpre.data(), n + 1);
  const size_t o_rp = bl.add(rpre.data(), n + 1);
  const size_t o_tp = bl.add(tpre.data(), n + 1);
  uint8_t* d = nullptr;
  if (int32_t e = commit(c, ring, bl, &d)) return e;
  const RankArgs* d_ra = (const RankArgs*)(d + o_ra);
  const int64_t* d_kp = (const int64_t*)(d + o_kp);
  const int64_t* d_rp = (const int64_t*)(d + o_rp);
  const int64_t* d_tp = (const int64_t*)(d + o_tp);
  hipStream_t s = c->stream;
  std::vector<PoseRow> host(NR);
  HIP_TRY(hipEventRecord(c->ev[4], s));
  if (per_request) {
    for (int i = 0; i < n; ++i) {
      if (F[i]->n_eval <= 0) continue;
      // at least row 0: the ambiguity statistics read it
      HIP_TRY(launch_rank_small(ra[i].best, F[i]->n_eval, ra[i].order, ra[i].smad,
                                std::max(1, nrow[i]), dr + rpre[i], s));
    }
  } else {
    HIP_TRY(launch_rank_keys_batch(d_ra, d_kp, n, NK, k1, s));
    // the sorted keys end in k1
    HIP_TRY(argsort_u64(k1, k2, S.rp2, S.rp1, NK, n, d_kp, d_tp, tpre[n], max_n, s));
    HIP_TRY(launch_rank_gather_batch(d_ra, d_rp, d_kp, n, NR, k1, dr, s));
  }
  if (NR > 0)
    HIP_TRY(hipMemcpyAsync(host.data(), dr, NR * sizeof(PoseRow), hipMemcpyDeviceToHost, s));
  std::vector<uint64_t> hm(3 * (size_t)n, 0);
  bool any_margin = false;
  for (int i = 0; i < n; ++i) {
    if (F[i]->n_eval <= 0) continue;
    Request& R = c->reqs.at(F[i]->rid);
    if (int32_t e = enqueue_margin(c, R, F[i]->arena->best + F[i]->off,
                                   F[i]->arena->order + F[i]->off, dr + rpre[i], F[i]->n_eval,
                                   nullptr, 0, dmarg + 3 * (size_t)i))
      return e;
    any_margin = true;
  }
  if (any_margin)
    HIP_TRY(hipMemcpyAsync(hm.data(), dmarg, hm.size() * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           s));
  HIP_TRY(hipEventRecord(c->ev[5], s));
  HIP_TRY(hipStreamSynchronize(s));
  if (pt) pt->rank += elapsed(c->ev[4], c->ev[5]);
  for (int i = 0; i < n; ++i) {
    (*rows)[i].assign(host.begin() + rpre[i], host.begin() + rpre[i] + nrow[i]);
    for (int q = 0; q < 3; ++q) F[i]->marg[q] = hm[3 * (size_t)i + q];
  }
  return RELOC_OK;
}

void fill_stats(const Request& R, const Flight& f, const PhaseTimes& pt, float total,
                reloc_stats* st) {
  const reloc_scan_info& I = R.prep.info;
  std::memset(st, 0, sizeof *st);
  st->n_hyp = R.n_hyp;
  st->smad_evals = coarse_evals(R);
  st->tam_evals = (int64_t)f.n_eval * I.Ntheta;
  st->rays = (int64_t)R.n_hyp * I.Ns;   // the batched front casts every request
  st->tam_lookups = st->tam_evals * I.n_valid;
  st->stages = f.stages;
  st->early_stopped = f.stopped ? 1 : 0;
  st->n_eval = f.n_eval;
  st->ms_total = total;
  st->ms_raycast = pt.raycast;
  st->ms_smad = pt.smad;
  st->ms_sort = pt.sort;
  st->ms_tam = pt.tam;
  st->ms_rank = pt.rank;
  if (f.n_eval > 0)
    fill_ambiguity(f.marg, f.fragile, st);
  else
    st->best_margin = -1.f;
  const int kr = R.prm.refine_k, K = R.prm.batch_k;
  if (kr > 0) {
    for (int b = 0; b < f.stages; ++b) st->refined += std::min(kr, std::min(K, R.n_hyp - b * K));
    st->refine_points = st->refined * R.ref_L;
  }
}

// ---- serving worker --------------------------------------------------------

void finish_ticket(ServeState& S, Ticket* t, int32_t status) {
  // the scheduler thread's own error text (thread-local) travels with the ticket
  const std::string msg = status != RELOC_OK ? reloc_last_error() : "";
  std::lock_guard<std::mutex> lk(S.qmu);
  t->status = status;
  t->msg = msg;
  t->done = true;
  if (status == RELOC_OK || status == RELOC_E_TIMEOUT)
    ++S.stats.completed;
  else
    ++S.stats.failed;
}

Ticket* ticket_of(ServeState& S, uint64_t id) {
  std::lock_guard<std::mutex> lk(S.qmu);
  auto it = S.tickets.find(id);
  return it == S.tickets.end() ? nullptr : it->second.get();
}

// One scheduler round; returns false when there was nothing to do.
bool serve_round(reloc_ctx* c, ServeState& S) {
  std::vector<Ticket*> adm;
  {
    std::unique_lock<std::mutex> lk(S.qmu);
    S.stats.queued = (int32_t)S.pending.size();
    if (S.pending.empty() && S.active.empty()) return false;
  }
  std::lock_guard<std::recursive_mutex> cl(c->mu);
  if (set_device(c) != RELOC_OK) return true;
  const auto t0 = std::chrono::steady_clock::now();
  // admission: slots and free HBM
  {
    std::unique_lock<std::mutex> lk(S.qmu);
    size_t planned = 0;
    while (!S.pending.empty() && (int)(S.active.size() + adm.size()) < S.cfg.max_inflight &&
           (int)adm.size() < S.cfg.max_admit) {
      Ticket* t = S.pending.front();
      const size_t need = request_bytes(t->R) + (size_t)t->R.n_hyp * 40 + (1 << 20);
      const size_t budget = c->budget > S.cfg.hbm_reserve ? c->budget - S.cfg.hbm_reserve : 0;
      if (c->used + planned + need > budget) {
        if (S.active.empty() && adm.empty()) {   // can never fit
          S.pending.pop_front();
          lk.unlock();
          fail(RELOC_E_NOMEM, "request needs %zu bytes, budget %zu", need, budget);
          finish_ticket(S, t, RELOC_E_NOMEM);
          lk.lock();
          continue;
        }
        break;
      }
      planned += need;
      S.pending.pop_front();
      adm.push_back(t);
    }
    S.stats.queued = (int32_t)S.pending.size();
  }
  int32_t err = RELOC_OK;
  // a small request on an idle device with nothing else waiting runs the
  // plain path at once: nothing to batch with, no stream hand-offs, and
  // (small) it cannot hold later arrivals back for long; a large one is
  // run in ticks, which later arrivals join
  bool alone = false;
  if (adm.size() == 1 && S.active.empty() && S.pipe_serve.inflight.empty() &&
      adm[0]->R.n_hyp <= kSoloMaxHyp) {
    std::lock_guard<std::mutex> lk(S.qmu);
    alone = S.pending.empty();
  }
  if (alone) {
    Ticket* t = adm[0];
    Request R = t->R;
    int32_t e = build_request(c, R);
    if (e == RELOC_OK) {
      std::vector<reloc_pose> out((size_t)std::max(1, R.rows_cap));
      int32_t n = 0;
      reloc_stats st{};
      e = run_request(c, R, out.data(), R.rows_cap, &n, &st, nullptr);
      if (e == RELOC_OK || e == RELOC_E_TIMEOUT) {
        out.resize((size_t)n);
        t->poses = std::move(out);
        st.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                               t->t_submit).count();
        t->st = st;
      }
    }
    (void)hipStreamSynchronize(c->stream);
    release_request(c, R);
    finish_ticket(S, t, e);
    {
      std::lock_guard<std::mutex> lk(S.qmu);
      ++S.stats.ticks;
      S.stats.busy_s +=
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    S.dcv.notify_all();
    return true;
  }
  // the admitted requests' tables and front phase go to the front stream,
  // beside the ticks in flight on the context's stream
  if (!adm.empty()) {
    if (!S.sfront && hipStreamCreateWithFlags(&S.sfront, hipStreamNonBlocking) != hipSuccess)
      S.sfront = nullptr;               // then everything runs on the context's stream
    const hipStream_t main = c->stream;
    c->stream = S.sfront ? S.sfront : main;
    StagingRing& fr = S.sfront ? S.fring : S.ring;
    std::vector<Flight*> fresh;
    for (Ticket* t : adm) {
      Request R = t->R;   // host part; the ticket keeps its copy
      int32_t e = build_request(c, R);
      if (e != RELOC_OK) {
        release_request(c, R);
        finish_ticket(S, t, e);
        continue;
      }
      const int id = c->next_id++;
      c->reqs[id] = std::move(R);
      S.active.emplace_back();
      Flight& f = S.active.back();
      f.rid = id;
      f.ticket = t->id;
      f.t_start = t->t_submit;
      fresh.push_back(&f);
    }
    const int32_t e = front(c, fr, fresh);
    if (e != RELOC_OK) {
      (void)hipStreamSynchronize(c->stream);   // what the front queued ends first
      for (Flight* f : fresh) {
        f->done = true;
        f->status = e;
      }
    }
    c->stream = main;
  }
  // every request with its front queued joins the ticks: the context's
  // stream waits (on the device) for the fronts still running, which run
  // beside the tick in flight
  std::vector<Flight*> ready;
  std::vector<FrontGroup*> waits;
  for (Flight& f : S.active) {
    if (f.done || !f.fg) continue;
    if (!front_done(*f.fg, false) &&
        std::find(waits.begin(), waits.end(), f.fg.get()) == waits.end())
      waits.push_back(f.fg.get());
    ready.push_back(&f);
  }
  for (FrontGroup* g : waits)
    if (err == RELOC_OK && hipStreamWaitEvent(c->stream, g->ev[3], 0) != hipSuccess)
      err = fail(RELOC_E_DEVICE, "stream wait on a front phase failed");
  TickPipe& P = S.pipe_serve;
  bool enq = false;
  if (err == RELOC_OK && P.inflight.size() < 2) err = enqueue_tick(c, P, S.ring, ready, &enq);
  // the stop flags of the oldest tick, read once a newer one is queued
  // behind it, when several requests are in flight (one alone reads its
  // flags at once: nothing to overlap, and no speculative tick to wait for)
  const size_t depth = ready.size() >= 2 ? 2 : 1;
  if (err == RELOC_OK && !P.inflight.empty() && (P.inflight.size() >= depth || !enq))
    err = complete_tick(c, P, nullptr);
  else if (err == RELOC_OK && !enq && P.inflight.empty())
    for (Flight& f : S.active)       // only front phases running: wait for one
      if (!f.done && f.fg && !f.fg->ready) {
        (void)front_done(*f.fg, true);
        break;
      }
  if (err != RELOC_OK) {
    // the device work queued so far ends before anything is released
    (void)hipStreamSynchronize(c->stream);
    if (S.sfront) (void)hipStreamSynchronize(S.sfront);
    if (S.srank) (void)hipStreamSynchronize(S.srank);
    P.inflight.clear();
    for (Flight& f : S.active) {
      f.done = true;
      f.pending = 0;
      if (f.status == RELOC_OK) f.status = err;
    }
  }
  // finished requests that no tick in flight covers: rank, answer, release
  std::vector<Flight*> fin;
  std::vector<int> caps;
  for (Flight& f : S.active)
    if (f.done && f.pending == 0) {
      if (f.fg) (void)front_done(*f.fg, true);   // its front work has ended too
      fin.push_back(&f);
      caps.push_back(INT32_MAX);
    }
  std::vector<std::vector<PoseRow>> rows;
  PhaseTimes rpt;
  if (!fin.empty() && err == RELOC_OK) {
    // on a stream of its own: the answer does not wait for the tick in
    // flight (which no finished request takes part in)
    if (!S.srank && hipStreamCreateWithFlags(&S.srank, hipStreamNonBlocking) != hipSuccess)
      S.srank = nullptr;
    const hipStream_t main = c->stream;
    c->stream = S.srank ? S.srank : main;
    err = rank(c, S, S.srank ? S.rring : S.ring, fin, caps, &rows, &rpt);
    c->stream = main;
  }
  for (size_t i = 0; i < fin.size(); ++i) {
    Flight& f = *fin[i];
    Ticket* t = ticket_of(S, f.ticket);
    Request& R = c->reqs.at(f.rid);
    if (t) {
      int32_t status = err != RELOC_OK ? err : f.status;
      if (err == RELOC_OK) {
        t->poses.resize(rows[i].size());
        rows_to_poses(c, R, rows[i].data(), (int)rows[i].size(), t->poses.data());
        const float total =
            std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                     t->t_submit).count();
        PhaseTimes pt = rpt;
        if (f.fg) {
          pt.raycast = f.fg->raycast;
          pt.smad = f.fg->smad;
          pt.sort = f.fg->sort;
        }
        pt.tam = f.tam_ms;
        fill_stats(R, f, pt, total, &t->st);
      }
      finish_ticket(S, t, status);
    }
    release_request(c, R);
    c->reqs.erase(f.rid);
    f.arena.reset();
    f.fg.reset();
  }
  S.active.remove_if([](const Flight& f) { return f.done && f.pending == 0; });
  {
    std::lock_guard<std::mutex> lk(S.qmu);
    ++S.stats.ticks;
    S.stats.inflight = (int32_t)S.active.size();
    S.stats.busy_s +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  S.dcv.notify_all();
  return true;
}

void serve_loop(reloc_ctx* c) {
  ServeState& S = *c->serve;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S.qmu);
      S.qcv.wait(lk, [&] { return S.stop || !S.pending.empty() || !S.active.empty(); });
      if (S.stop) break;
    }
    serve_round(c, S);
  }
}

}  // namespace

ServeState* serve_create() { return new ServeState(); }

bool serve_holds_set(reloc_ctx* c, int32_t set_id) {
  if (!c->serve) return false;
  std::lock_guard<std::mutex> lk(c->serve->qmu);
  for (auto& kv : c->serve->tickets)
    if (!kv.second->done && kv.second->R.set_id == set_id) return true;
  return false;
}

void ctx_stop_serving(reloc_ctx* c) {
  ServeState* S = c->serve;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->qmu);
    S->stop = true;
  }
  S->qcv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  std::lock_guard<std::recursive_mutex> cl(c->mu);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (hipStream_t* q : {&S->sfront, &S->srank})
    if (*q) {
      (void)hipStreamSynchronize(*q);
      (void)hipStreamDestroy(*q);
      *q = nullptr;
    }
  for (Flight& f : S->active) {
    auto it = c->reqs.find(f.rid);
    if (it != c->reqs.end()) {
      release_request(c, it->second);
      c->reqs.erase(it);
    }
    f.arena.reset();
  }
  S->active.clear();
  free_ring(c, S->ring);
  free_ring(c, S->fring);
  free_ring(c, S->rring);
  free_pipe(S->pipe_batch);
  free_pipe(S->pipe_serve);
  c->dfree(S->rk1);
  c->dfree(S->rk2);
  c->dfree(S->rrows);
  c->dfree(S->rmarg);
  c->dfree(S->rp1);
  c->dfree(S->rp2);
  {
    // polls still waiting see stop and return; the state outlives them
    std::unique_lock<std::mutex> lk(S->qmu);
    S->dcv.notify_all();
    S->dcv.wait(lk, [&] { return S->pollers == 0; });
  }
  delete S;
  c->serve = nullptr;
}

}  // namespace reloc

using namespace reloc;

extern "C" {

int32_t reloc_run_batch(reloc_ctx* c, int32_t n, const int32_t* request_ids, reloc_pose* out,
                        int32_t cap, int32_t* n_out, int32_t* status, reloc_stats* stats) {
  for (int i = 0; n_out && i < n; ++i) n_out[i] = 0;
  for (int i = 0; status && i < n; ++i) status[i] = RELOC_E_PENDING;
  if (!c || n < 0 || (n > 0 && (!request_ids || !n_out || !status)) || (!out && cap > 0))
    return fail(RELOC_E_INVALID, "null argument");
  if (n == 0) return RELOC_OK;
  std::lock_guard<std::recursive_mutex> lk(c->mu);
  for (int i = 0; i < n; ++i) {
    if (!c->reqs.count(request_ids[i]))
      return fail(RELOC_E_NOTFOUND, "unknown request %d", request_ids[i]);
    for (int j = 0; j < i; ++j)
      if (request_ids[j] == request_ids[i])
        return fail(RELOC_E_INVALID, "request %d listed twice", request_ids[i]);
  }
  if (int32_t e = set_device(c)) return e;
  ServeState& S = *state(c);
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<Flight> fl(n);
  std::vector<Flight*> F(n);
  for (int i = 0; i < n; ++i) {
    fl[i].rid = request_ids[i];
    fl[i].t_start = t0;
    F[i] = &fl[i];
  }
  PhaseTimes pt;
  // on an error, the device work queued so far ends before the flights'
  // buffers go
  auto bail = [&](int32_t e) {
    (void)hipStreamSynchronize(c->stream);
    S.pipe_batch.inflight.clear();
    return e;
  };
  if (int32_t e = front(c, S.ring, F)) return bail(e);
  if (!front_done(*F[0]->fg, true)) return bail(fail(RELOC_E_DEVICE, "front phase failed"));
  pt.raycast = F[0]->fg->raycast;
  pt.smad = F[0]->fg->smad;
  pt.sort = F[0]->fg->sort;
  // one tick at a time: a batch has no later arrivals to overlap with
  TickPipe& P = S.pipe_batch;
  for (;;) {
    bool enq = false;
    if (int32_t e = enqueue_tick(c, P, S.ring, F, &enq)) return bail(e);
    if (!enq) break;
    if (int32_t e = complete_tick(c, P, &pt)) return bail(e);
  }
  std::vector<int> caps(n, std::max(0, cap));
  std::vector<std::vector<PoseRow>> rows;
  if (int32_t e = rank(c, S, S.ring, F, caps, &rows, &pt)) return bail(e);
  const float total =
      std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < n; ++i) {
    const Request& R = c->reqs.at(request_ids[i]);
    // rows exist only when cap > 0, and then out is a buffer of n * cap poses
    if (!rows[i].empty())
      rows_to_poses(c, R, rows[i].data(), (int)rows[i].size(), out + (size_t)i * (size_t)cap);
    n_out[i] = (int32_t)rows[i].size();
    status[i] = fl[i].status;
    if (stats) fill_stats(R, fl[i], pt, total, &stats[i]);
  }
  return RELOC_OK;
}

int32_t reloc_serve_configure(reloc_ctx* c, const reloc_serve_config* cfg) {
  if (!c || !cfg) return fail(RELOC_E_INVALID, "null argument");
  if (cfg->max_inflight < 1 || cfg->max_admit < 1)
    return fail(RELOC_E_INVALID, "max_inflight and max_admit must be >= 1");
  ServeState& S = *state(c);
  std::lock_guard<std::mutex> lk(S.qmu);
  S.cfg = *cfg;
  return RELOC_OK;
}

int32_t reloc_submit(reloc_ctx* c, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                     const reloc_search_params* params, uint64_t* ticket) {
  if (ticket) *ticket = 0;
  if (!c || !ticket) return fail(RELOC_E_INVALID, "null argument");
  auto t = std::make_unique<Ticket>();
  t->t_submit = std::chrono::steady_clock::now();
  {
    // host preprocessing only: the registry lock, not the context lock, so
    // that submit does not wait for the scheduler's device work; held until
    // the ticket is registered so the set cannot be freed in between
    std::lock_guard<std::mutex> rg(c->reg_mu);
    if (int32_t e = init_request(c, map_id, set_id, scan, params, &t->R)) return e;
    ServeState& S = *state(c);
    std::lock_guard<std::mutex> lk(S.qmu);
    if (S.stop) return fail(RELOC_E_INVALID, "context is shutting down");
    if (!S.running) {
      S.worker = std::thread(serve_loop, c);
      S.running = true;
    }
    t->id = S.next_ticket++;
    *ticket = t->id;
    S.pending.push_back(t.get());
    S.tickets[t->id] = std::move(t);
    ++S.stats.submitted;
    S.stats.queued = (int32_t)S.pending.size();
  }
  c->serve->qcv.notify_all();
  return RELOC_OK;
}

int32_t reloc_poll(reloc_ctx* c, uint64_t ticket, int32_t wait_ms, reloc_pose* out, int32_t cap,
                   int32_t* n_out, reloc_stats* st) {
  if (n_out) *n_out = 0;
  if (!c || !n_out || (!out && cap > 0)) return fail(RELOC_E_INVALID, "null argument");
  ServeState* S = c->serve;
  std::unique_lock<std::mutex> lk(S->qmu);
  // counted while inside, so that destroying the context waits for a
  // blocked poll to leave before the state goes (released under qmu)
  ++S->pollers;
  struct Leave {
    ServeState* S;
    ~Leave() {
      --S->pollers;
      S->dcv.notify_all();
    }
  } leave{S};
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end())
    return fail(RELOC_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket* t = it->second.get();
  if (!t->done && wait_ms != 0) {
    auto pred = [&] { return t->done || S->stop; };
    if (wait_ms < 0)
      S->dcv.wait(lk, pred);
    else
      S->dcv.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
  }
  if (!t->done) return fail(RELOC_E_PENDING, "ticket %llu not finished", (unsigned long long)ticket);
  const int32_t status = t->status;
  const int n = std::min<int>((int)t->poses.size(), std::max(0, cap));
  for (int i = 0; i < n; ++i) out[i] = t->poses[i];
  *n_out = n;
  if (st) *st = t->st;
  const std::string msg = t->msg;
  S->tickets.erase(it);
  if (status != RELOC_OK && status != RELOC_E_TIMEOUT)
    return fail(status, "request failed: %s", msg.c_str());
  return status;
}

int32_t reloc_serve_stats_get(reloc_ctx* c, reloc_serve_stats* out) {
  if (!c || !out) return fail(RELOC_E_INVALID, "null argument");
  std::memset(out, 0, sizeof *out);
  ServeState* S = c->serve;
  std::lock_guard<std::mutex> lk(S->qmu);
  *out = S->stats;
  out->pollers = S->pollers;
  return RELOC_OK;
}

}  // extern "C"
