/*
 * reloc.h - C ABI of the MI355X relocalization library (libreloc.so).
 *
 * Passive 2-D global relocalization by batched multi-stage hypothesis
 * inference (arXiv 2511.01219, Sec. III): for every feasible positional
 * hypothesis ray-cast a panoramic synthetic scan (eq. 13-14), score every
 * circular beam shift with SMAD (eq. 16-20), order the hypotheses by SMAD,
 * re-score them batch by batch over all orientations with TAM against a
 * distance field (eq. 22-31) and stop as soon as a batch's best TAM exceeds
 * the threshold tau (Sec. III, pipeline description).
 *
 * Conventions
 *   - SI units (metres, radians). World frame: x right, y up, theta counter-
 *     clockwise from +x, reported in [-pi, pi) (eq. 1).
 *   - A map is a row-major int8 grid, row 0 at the minimum y; cell (ix, iy)
 *     covers [ox + ix*res, ox + (ix+1)*res) x [oy + iy*res, ...). A cell is
 *     occupied iff value >= occ_threshold, unknown iff value < 0, otherwise
 *     free. Unknown cells are free for ray casting, not obstacles for the
 *     distance transform, and infeasible for hypotheses.
 *   - Every call returns an int32 status: RELOC_OK (0) or a negative
 *     RELOC_E_* code. On error no output is written (counts are set to 0)
 *     and reloc_last_error() describes the failure. Nothing throws across
 *     the ABI.
 *   - Ownership: the caller owns every buffer it passes; inputs are copied
 *     before the call returns. Maps, hypothesis sets and requests live in the
 *     context and are named by integer ids. Pointers documented as "host"
 *     are host memory.
 *   - Device memory comes from the allocator given to reloc_ctx_create
 *     (hipMalloc when NULL). The context keeps blocks it no longer needs
 *     (up to 256 MiB each, 2 GiB in all) for later allocations of the same
 *     size class, and returns them to the allocator when an allocation
 *     would pass the HBM budget, when the allocator fails, and at
 *     destruction; live plus kept blocks never exceed the budget. Work is
 *     issued on the stream given there (a
 *     hipStream_t passed as void*; a private default-priority stream when
 *     NULL). Calls on one context are serialized internally.
 *   - Results are deterministic: the same inputs give bit-identical outputs,
 *     whatever else runs on the device.
 */
#ifndef RELOC_H
#define RELOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RELOC_VERSION 1

enum {
  RELOC_OK = 0,
  RELOC_E_INVALID = -1,   /* bad argument */
  RELOC_E_NOMEM = -2,     /* allocation failed or the HBM budget is exceeded */
  RELOC_E_NOTFOUND = -3,  /* unknown map, hypothesis set or request id */
  RELOC_E_BEAMGRID = -4,  /* beams not on an equiangular grid dividing 2*pi */
  RELOC_E_EMPTY = -5,     /* no feasible hypothesis, no valid beam, empty map */
  RELOC_E_BUSY = -6,      /* object in use (e.g. map with live hypothesis sets) */
  RELOC_E_PENDING = -7,   /* result not ready yet */
  RELOC_E_TIMEOUT = -8,   /* deadline passed */
  RELOC_E_DEVICE = -9     /* HIP runtime / device error */
};

/* What every call returns: RELOC_OK or one of the RELOC_E_* codes above
 * (the functions are declared with its underlying type, int32_t). */
typedef int32_t reloc_status;

typedef struct reloc_ctx reloc_ctx;

/* Device allocator hook. alloc returns device memory of at least `bytes`
 * bytes (NULL on failure); free releases it. Both are called with `user`. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} reloc_allocator;

/* Library version (RELOC_VERSION of the build). */
int32_t reloc_version(void);

/* Thread-local description of the last error on this thread; valid until
 * the next call on the same thread. Never NULL. */
const char* reloc_last_error(void);

/* Create a context on HIP device `device`.
 *   alloc      : allocator hook, or NULL for hipMalloc/hipFree.
 *   stream     : hipStream_t (as void*) all work is issued on, or NULL for a
 *                private stream owned by the context.
 *   hbm_budget : bytes of device memory the context may hold; 0 means the
 *                free device memory at creation. Allocations beyond it fail
 *                with RELOC_E_NOMEM.
 * Errors: RELOC_E_INVALID (null out), RELOC_E_DEVICE (no such device). */
int32_t reloc_ctx_create(int32_t device, const reloc_allocator* alloc, void* stream,
                         size_t hbm_budget, reloc_ctx** out);

/* Waits for outstanding work and frees everything the context holds. A
 * reloc_poll blocked on the context returns first (RELOC_E_PENDING for an
 * unfinished ticket); no call may start on the context once destroy has
 * begun. */
void reloc_ctx_destroy(reloc_ctx* ctx);

/* Bytes of device memory in live use by the context's maps, sets,
 * requests and scratch (size classes: powers of two up to 1 MiB, then
 * multiples of 2 MiB); blocks kept for reuse are not counted. */
size_t reloc_ctx_bytes(const reloc_ctx* ctx);

/* ------------------------------------------------------------------------
 * Map residency. The occupancy grid M (Sec. II-A) is bit-packed on the
 * device in 8x8-cell tiles (one uint64 per tile), and the exact Euclidean
 * distance transform used by MinDistToObstacle (Sec. III-A) and by TAM's
 * d_obs (eq. 23) is computed on the device as k[c] = min over occupied o of
 * (dx^2 + dy^2) in cells (uint32). Both stay resident until unload.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t width, height;    /* cells, 1 .. 32767 each */
  double resolution;        /* metres per cell, >= 1/32 */
  double origin_x, origin_y;/* world position of the lower-left map corner */
  int32_t occ_threshold;    /* occupied iff value >= threshold (65) */
} reloc_map_desc;

/* occ: host int8[height*width]. Errors: RELOC_E_INVALID (bad sizes),
 * RELOC_E_EMPTY (no occupied cell), RELOC_E_NOMEM, RELOC_E_DEVICE. */
int32_t reloc_load_map(reloc_ctx* ctx, const reloc_map_desc* desc, const int8_t* occ,
                       int32_t* map_id);

/* RELOC_E_BUSY while hypothesis sets of the map exist. */
int32_t reloc_unload_map(reloc_ctx* ctx, int32_t map_id);

/* Copies the squared-distance transform k (uint32[height*width], row-major,
 * host) of a resident map. */
int32_t reloc_read_edt(reloc_ctx* ctx, int32_t map_id, uint32_t* k_out);

/* ------------------------------------------------------------------------
 * Hypothesis sets (the positions P of eq. 6). The sampler keeps the
 * constraints of Algorithm 1 with a deterministic integer procedure:
 *   feasible  : known-free cells with k >= ceil((robot_radius/res)^2 - 1e-9)
 *               (TraversabilityCheck at cell centres);
 *   reachable : the 4-connected feasible component of p0's cell (R(p0)),
 *               or the largest component (ties: smallest cell index) when
 *               has_p0 == 0;
 *   order     : ascending (splitmix64(seed + c), c) over reachable cells c
 *               (linear index), splitmix64 being the published output
 *               function applied to x + 0x9E3779B97F4A7C15;
 *   spacing   : accept c iff every accepted c' has dx^2 + dy^2 >=
 *               ceil((min_spacing/res)^2 - 1e-9) (VoxelDownsample spacing);
 *               stop after n_target acceptances.
 * Positions are cell centres, kept in acceptance order, so any prefix of a
 * set is itself a valid set. Returning fewer than n_target is not an error.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_target;
  double min_spacing;       /* rho, metres (0.3) */
  double robot_radius;      /* r_robot, metres (0.21) */
  int32_t has_p0;
  double p0_x, p0_y;        /* world position of the reachability seed */
  uint64_t seed;
} reloc_sample_params;

int32_t reloc_sample_hypotheses(reloc_ctx* ctx, int32_t map_id,
                                const reloc_sample_params* params, int32_t* set_id,
                                int32_t* n_out);

/* Traversability-constrained RRT sampling (Algorithm 1; Sec. III-A items
 * 1-7; Remark 4), run on the host copy of the map (tree growth is
 * sequential), producing a hypothesis set. Rounds of N_sampling =
 * ceil(W H res^2 / rho^2) expansion attempts; attempt t (counted over all
 * rounds from 0) draws p_rand = (ox + u W res, oy + v H res) with
 * u = (splitmix64(seed + 2t) >> 11) 2^-53, v likewise from seed + 2t + 1;
 *   NearestNode : smallest FP64 dx*dx + dy*dy, ties: smallest node index;
 *   eta         : AdaptiveExpandDist of p_nearest from d = sqrt(k) res of its
 *                 cell: eta_max if d >= 2 r_robot, r_robot if d <= r_robot,
 *                 r_robot + (eta_max - r_robot)(d - r_robot)/r_robot between;
 *   p_new       : p_rand when |p_rand - p_nearest| <= eta, else p_nearest +
 *                 (eta / L)(p_rand - p_nearest); L == 0 adds nothing;
 *   accepted    : p_new inside the map rectangle (InSamplingBoundary) and
 *                 every point p_nearest + (i/n)(p_new - p_nearest), i = 0..n,
 *                 n = max(1, ceil(L / (res/2))), in a known-free cell with
 *                 k >= ceil((r_robot/res)^2 - 1e-9) (TraversabilityCheck);
 *   VoxelDownsample: voxels of side rho from the map origin, each
 *                 represented by its first node; gain = new voxels per round.
 * Rounds stop when gain <= eps_gain, after max_rounds, or at max_nodes
 * nodes. The set holds the representatives' cells in node order, without
 * repeats. p0 (the tree root, Algorithm 1's map origin) must be traversable
 * (RELOC_E_EMPTY otherwise). A host allocation that fails returns
 * RELOC_E_NOMEM.
 *   info     : counts of the run (may be NULL);
 *   nodes_xy : optional host double[2 * nodes_cap], the tree nodes (world);
 *   parent   : optional host int32[nodes_cap], each node's parent (-1 root). */
typedef struct {
  double p0_x, p0_y;        /* tree root, world */
  double rho;               /* sampling spacing (voxel side), metres (0.3);
                               at least the map resolution, else RELOC_E_INVALID */
  double robot_radius;      /* r_robot, metres (0.21) */
  double eta_max;           /* maximum expansion distance, metres (0.6) */
  int32_t eps_gain;         /* gain threshold (2) */
  int32_t max_rounds;       /* at most this many rounds (64) */
  int32_t max_nodes;        /* at most this many tree nodes (16 M) */
  uint64_t seed;
} reloc_rrt_params;

typedef struct {
  int64_t rounds, attempts, nodes, n_sampling;
} reloc_rrt_info;

/* Fills the defaults listed above (p0 = (0, 0)). */
void reloc_rrt_defaults(reloc_rrt_params* p);

int32_t reloc_sample_rrt(reloc_ctx* ctx, int32_t map_id, const reloc_rrt_params* params,
                         int32_t* set_id, int32_t* n_out, reloc_rrt_info* info,
                         double* nodes_xy, int32_t* parent, int32_t nodes_cap);

/* A caller-supplied set: cell_xy = host int32[2*n] (ix, iy) pairs of free
 * in-map cells. */
int32_t reloc_set_hypotheses(reloc_ctx* ctx, int32_t map_id, const int32_t* cell_xy,
                             int32_t n, int32_t* set_id);

/* Copies up to cap cells (host int32[2*cap]); *n_out = set size. */
int32_t reloc_read_hypotheses(reloc_ctx* ctx, int32_t set_id, int32_t* cell_xy,
                              int32_t cap, int32_t* n_out);

int32_t reloc_free_hypotheses(reloc_ctx* ctx, int32_t set_id);

/* ------------------------------------------------------------------------
 * Scans and search parameters.
 * Beam i (before downsampling) has robot-frame angle
 * angle_min + i * angle_increment. The scan is downsampled by n_skip_beam
 * (eq. 11); Ns = 2*pi / (angle_increment * n_skip_beam) must be an integer
 * (eq. 14) and angle_min a multiple of the downsampled step, both within
 * 1e-6 * Ns, else RELOC_E_BEAMGRID. Ns <= 4096.
 * FoV intervals (eq. 12) are robot-frame angle intervals [lo, hi]; a beam is
 * in the FoV iff its angle lies in one of them (all beams when n_fov == 0).
 * A FoV beam is valid iff its range is finite and range_min <= z <=
 * range_max; invalid FoV beams take the placeholder 0 in SMAD (Sec. III-B)
 * and are left out of TAM.
 * ---------------------------------------------------------------------- */
typedef struct { double lo, hi; } reloc_interval;

typedef struct {
  int32_t n_beams;
  const float* ranges;          /* host float[n_beams]; NaN = no return */
  double angle_min, angle_increment;
  int32_t n_fov;
  const reloc_interval* fov;    /* host, n_fov entries, or NULL */
  float range_min, range_max;   /* range_max < 64 m */
} reloc_scan;

typedef struct {
  int32_t n_theta;        /* TAM orientations N_theta (0: = Ns) */
  int32_t n_skip_beam;    /* eq. 11 stride (1) */
  int32_t n_skip_enum;    /* eq. 15 SMAD shift stride (1) */
  int32_t batch_k;        /* hypotheses per stage (64) */
  int32_t k_out;          /* ranked poses to return (10) */
  double tau;             /* early-termination threshold (0.95); NaN: none */
  int32_t n_hyp;          /* use the first n_hyp of the set (0: all) */
  double z_hit, sigma_hit, z_rand; /* likelihood field, eq. 23 (1, 0.2, 0) */
  double d_max;           /* eq. 29 clamp and off-map distance (2.0 m) */
  int32_t alpha_mid_pm[2];/* alpha_mid at lambda = 0 and 1, per mille (900, 700) */
  int32_t alpha_low_pm[2];/* alpha_low at lambda = 0 and 1, per mille (700, 500);
                             eq. 25 orders them: alpha_low_pm[i] <= alpha_mid_pm[i]
                             for i = 0, 1, else RELOC_E_INVALID */
  double deadline_s;      /* plain path: stop with RELOC_E_TIMEOUT after this (0: none) */
  int32_t variant;        /* ray-cast kernel: 0 default; 1 bit tiles; 2, 3, 4, 5
                             distance skipping with wavefront ray refill once 1, 8,
                             16, 32 lanes are idle. Every variant gives
                             bit-identical results. */
  /* Local refinement (Sec. III pipeline: the top-k poses of each batch are
   * refined by a local operator and re-evaluated with TAM before the
   * threshold test; Remark 2). The operator here is an exhaustive TAM
   * search over the lattice of poses next to the pose: cells (ix + dx,
   * iy + dy) with |dx|, |dy| <= refine_cells, headings g* + dg on the Ng
   * direction grid (heading index g = g* + dg mod Ng, theta = 2 pi g / Ng)
   * with |dg| <= refine_dirs, g* = (Ng / N_theta) k*. Lattice cells other
   * than the pose's own that are off the map or occupied are skipped. The
   * refined pose has the largest T; ties go to the pose itself, then to the
   * smaller raster index ((dg + s)(2h + 1) + dy + h)(2h + 1) + dx + h. The
   * refined T replaces the pose's T in the batch best and the ranking. */
  int32_t refine_k;       /* poses refined per batch (0: none; <= 64) */
  int32_t refine_cells;   /* h, lattice half-width in cells (3; <= 15) */
  int32_t refine_dirs;    /* s, heading half-width in Ng steps (-1: Ng / N_theta);
                             the lattice (2s + 1)(2h + 1)^2 holds <= 65536 points */
  /* Ablation metrics (Sec. IV, Case 3). coarse_metric orders the
   * hypotheses: 0 SMAD with prefix sums (eq. 17-20); 1 SMAD by direct sums
   * (the same values, the ablation's "without prefix-sum acceleration");
   * 2 CAER (eq. 21: mean of |z'_i - zhat_{i+m}| over the FoV beams, every
   * shift m scored, also for panoramic scans); 3 none (no ray cast, the
   * set's own order). fine_metric is the score T that picks theta*, ranks
   * poses and is tested against tau: 0 TAM (eq. 31); 1 TAM_mean (eq. 34);
   * 2 baseline (eq. 33); 3 LF (eq. 32, a sum of log-likelihoods, <= 0 up to
   * 1e-6 per beam). */
  int32_t coarse_metric;
  int32_t fine_metric;
  /* reloc_run launches the device work before its first stop-flag read (ray
   * cast, coarse metric, order, first TAM launch with refinement and stage
   * control, first ranking) kernel by kernel (0, the default), or replays
   * it as a HIP graph captured on the request's second run (1). Graphs are
   * used when a first launch of one stage ranks at most 2048 poses (its
   * ranking is then one kernel writing the rows to pinned memory) and the
   * context's stream is not the null stream; results are identical either
   * way. A
   * replayed run times only ms_total (hipEvents around the graph launch and
   * the later launches); its per-phase times read 0. The graph saves a few
   * microseconds of launch overhead per run (about 3 % on a 300-hypothesis
   * search): for serving loops that repeat one request. */
  int32_t use_graph;
  /* Launch shape of the fused ray cast + SMAD kernel (the default path:
   * coarse_metric 0, variant 0, a map with walk words): wavefronts per
   * hypothesis workgroup (1, 2 or 4) and lane refill threshold (8, 16 or 32
   * idle lanes); 0 takes the map's tuned shape or the default rule. Every
   * shape gives bit-identical results. */
  int32_t ray_waves;
  int32_t ray_refill;
} reloc_search_params;

/* Fills the defaults listed above. */
void reloc_search_defaults(reloc_search_params* p);

/* Host-only preprocessing summary of a scan (eq. 11-16, 25-26):
 * k_mid = floor(N'_Z * (A0*Ns + (A1 - A0)*N_FoV) / (1000*Ns)), likewise
 * k_low; zbar = FP64 mean of the FoV ranges with placeholders (eq. 16);
 * panoramic = (10*N_FoV >= 9*Ns), eq. 20's lambda >= 0.9. */
typedef struct {
  int32_t Ns, Ntheta, Ng;       /* Ng = lcm(Ns, Ntheta) */
  int32_t n_down;               /* beams after downsampling */
  int32_t n_fov, n_valid;       /* N_FoV (= sum |I_k|), N'_Z */
  int32_t k_full, k_mid, k_low;
  int32_t panoramic, n_runs, n_shifts, j0;
  double zbar, lambda;
} reloc_scan_info;

int32_t reloc_scan_info_get(const reloc_scan* scan, const reloc_search_params* params,
                            double resolution, reloc_scan_info* out);

/* One ranked pose hypothesis (eq. 8-9). x, y: world centre of cell (cx,
 * cy); theta: heading wrapped to [-pi, pi), k * 2*pi / N_theta, or g * 2*pi
 * / Ng for a refined pose; tam: T (eq. 31) at that pose; smad: SMAD(p) (eq.
 * 20) of the hypothesis as FP32; hyp: index in the set; k: orientation
 * index (-1 for a refined pose); rank: position in the SMAD order; stage:
 * batch index; g: heading index on the Ng direction grid; refined: 1 when
 * the pose came out of the local refinement. */
typedef struct {
  double x, y, theta;
  float tam, smad;
  int32_t hyp, k, rank, stage;
  int32_t cx, cy, g, refined;
} reloc_pose;

typedef struct {
  int64_t smad_evals;   /* N_p x shifts (1 when panoramic) */
  int64_t tam_evals;    /* hypotheses evaluated by TAM x N_theta */
  int64_t rays;         /* N_p x Ns */
  int64_t tam_lookups;  /* tam_evals x N'_Z */
  int32_t n_hyp, stages, early_stopped, n_eval;
  /* device time (hipEvents on the context's stream): whole run; ray-cast
   * kernel; SMAD kernel; SMAD order; TAM stages with refinement and stage
   * control; ranking and result copy (a run replaying its head graph sets
   * ms_total only, the others are 0) */
  float ms_total, ms_raycast, ms_sort, ms_tam, ms_rank, ms_smad;
  /* local refinement: poses refined; lattice points considered (refined
   * poses x (2s + 1)(2h + 1)^2, skipped cells included) */
  int64_t refined, refine_points;
  /* Ambiguity (Remark 1, eq. 5). best_margin = T of the top-1 pose minus
   * the best T among the evaluated poses distinct from it by the success
   * criterion of Sec. IV-C (position >= 0.5 m away or heading >= 30 deg
   * away); -1 when no evaluated pose is distinct. ambiguous: bit 0 = a
   * stage's stop decision was within 1e-4 of tau (a batch best in
   * [tau - 1e-4, tau + 1e-4]); bit 1 = best_margin <= 1e-4 |T1| + 1e-7 (the
   * top-1 is numerically tied with a distinct pose). */
  float best_margin;
  int32_t ambiguous;
} reloc_stats;

/* ------------------------------------------------------------------------
 * Relocalization.
 * A request binds a scan to a map and hypothesis set: the scan is
 * preprocessed on the host (reloc_scan_info) and its tables uploaded once.
 * reloc_run then executes the whole hot path on the device:
 *   ray cast + SMAD for every hypothesis -> stable sort by (SMAD, index) ->
 *   stages of batch_k hypotheses: TAM over N_theta orientations, theta* per
 *   hypothesis (ties: smallest k), local refinement of the batch's refine_k
 *   best poses (optional), batch best (ties: earlier rank), stop when it
 *   exceeds tau -> all evaluated poses ranked by (T desc, rank asc).
 * out: host reloc_pose[cap]; *n_out = min(cap, k_out, evaluated).
 * stats may be NULL.
 * ---------------------------------------------------------------------- */
int32_t reloc_prepare(reloc_ctx* ctx, int32_t map_id, int32_t set_id,
                      const reloc_scan* scan, const reloc_search_params* params,
                      int32_t* request_id);

int32_t reloc_run(reloc_ctx* ctx, int32_t request_id, reloc_pose* out, int32_t cap,
                  int32_t* n_out, reloc_stats* stats);

int32_t reloc_release(reloc_ctx* ctx, int32_t request_id);

/* prepare + run + release in one call. */
int32_t reloc_relocalize(reloc_ctx* ctx, int32_t map_id, int32_t set_id,
                         const reloc_scan* scan, const reloc_search_params* params,
                         reloc_pose* out, int32_t cap, int32_t* n_out, reloc_stats* stats);

/* reloc_relocalize for callers that cannot allocate device memory: code
 * under HIP stream capture, tight serving loops, hosts that forbid
 * allocation once running. It calls no hipMalloc, hipFree, hipHostMalloc,
 * hipHostFree or allocator hook: every device buffer of the request comes
 * from one 64 MiB scratch region that the library holds on each GPU it runs
 * on until the process ends (set up when a context is created on the
 * device); the host-side scan preprocessing uses ordinary host memory.
 * Arguments and results are those of reloc_relocalize, bit for bit. A
 * request whose device buffers exceed the region (about 60 bytes per
 * hypothesis plus the scan's tables; the ablation coarse metrics add a
 * 4 Ns-byte range buffer per hypothesis) fails with RELOC_E_NOMEM before any
 * device work. All calls on one GPU share its region: calls on one context
 * are serialized, calls that overlap on one GPU from different contexts
 * race. The head graph (use_graph) is not used. */
int32_t reloc_relocalize_noalloc(reloc_ctx* ctx, int32_t map_id, int32_t set_id,
                                 const reloc_scan* scan, const reloc_search_params* params,
                                 reloc_pose* out, int32_t cap, int32_t* n_out,
                                 reloc_stats* stats);

/* ------------------------------------------------------------------------
 * Dense sweeps (Sec. IV Case 1: Fig. 7's SMAD map over positions, Fig. 8's
 * metrics over a translation x rotation lattice).
 * reloc_coarse_scores runs the ray cast and the request's coarse metric for
 * every hypothesis of its set (a set of all free cells gives the coarse map
 * of Fig. 7) and returns, each optional (host, cap >= n_hyp entries, else
 * RELOC_E_INVALID): the score
 * (SMAD, or the ablation's CAER; FP64), its argmin shift m, and the stable
 * ascending (score, index) order; stats (optional) gets the counts and the
 * device time of the ray cast, the coarse kernel and the sort.
 * reloc_score_poses evaluates the request's fine metric (fine_metric: TAM,
 * TAM_mean, baseline or LF) at n explicit poses: host cell_xy[2n] (cells
 * inside the map) and heading[n] (heading index g on the request's Ng
 * direction grid, theta = 2 pi g / Ng); score: host float[n]; ms_out
 * (optional): device time of the scoring kernel. RELOC_E_INVALID for a cell
 * outside the map or a heading index outside [0, Ng).
 * ---------------------------------------------------------------------- */
int32_t reloc_coarse_scores(reloc_ctx* ctx, int32_t request_id, int32_t cap, double* score,
                            int32_t* shift, int32_t* order, reloc_stats* stats);
int32_t reloc_score_poses(reloc_ctx* ctx, int32_t request_id, const int32_t* cell_xy,
                          const int32_t* heading, int32_t n, float* score, float* ms_out);

/* ------------------------------------------------------------------------
 * Batched form: several prepared requests (any maps, scans and parameters)
 * run together. One ray-cast launch and one SMAD launch cover the
 * hypotheses of every request, one segmented sort gives every SMAD order,
 * and the TAM stages of all requests advance together: each step launches
 * TAM over a rank range of every unfinished request and one stage-control
 * kernel that reduces each of its stages on the device (Sec. III pipeline,
 * batch-wise early termination). A range covers one stage in a request's
 * first two steps, then 2, 4, ... up to 32 consecutive stages, granted
 * oldest request first out of a per-step budget of TAM workgroups (at least
 * one stage each); stages after the first whose best T exceeds tau are
 * discarded, so every request gets exactly the result of reloc_run.
 *   request_ids : host int32[n], distinct prepared requests
 *   out         : host reloc_pose[n * cap]; request i's poses at out + i*cap
 *   n_out       : host int32[n] poses written per request
 *   status      : host int32[n]: RELOC_OK, or RELOC_E_TIMEOUT when the
 *                 request's deadline_s passed (best-so-far poses returned)
 *   stats       : host reloc_stats[n] or NULL; the ms_* fields time the
 *                 batch's phases and are the same for every request.
 * Errors: RELOC_E_INVALID, RELOC_E_NOTFOUND, RELOC_E_NOMEM, RELOC_E_DEVICE.
 * ---------------------------------------------------------------------- */
int32_t reloc_run_batch(reloc_ctx* ctx, int32_t n, const int32_t* request_ids,
                        reloc_pose* out, int32_t cap, int32_t* n_out, int32_t* status,
                        reloc_stats* stats);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of requests as they arrive.
 * reloc_submit preprocesses the scan on the calling thread and queues the
 * request; a scheduler thread owned by the context repeats rounds of
 *   admission (while fewer than max_inflight requests are on the device,
 *   at most max_admit per round, and the request's device memory fits the
 *   context budget minus hbm_reserve; a request that cannot fit even on an
 *   idle device fails with RELOC_E_NOMEM) -> ray cast, SMAD and order of the
 *   admitted requests (one launch each, as in reloc_run_batch) -> one TAM
 *   step of every request in flight -> ranking of the finished ones.
 * In-flight state (ranges, SMAD, orders, per-rank best) stays on the device;
 * a request admitted while others run joins them at the next stage
 * boundary. Each result equals reloc_run's for the same inputs.
 * submit and poll may be called from any threads concurrently; other calls
 * on the context wait for the current round. The hypothesis set of a queued
 * request cannot be freed (RELOC_E_BUSY) until the request finished.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t max_inflight;   /* requests on the device at once (64) */
  size_t hbm_reserve;     /* bytes of the context budget left free (0) */
  int32_t max_admit;      /* requests admitted per round (16) */
} reloc_serve_config;

/* Replaces the scheduler configuration (takes effect at the next round). */
int32_t reloc_serve_configure(reloc_ctx* ctx, const reloc_serve_config* cfg);

/* Queues a relocalization; *ticket names it for reloc_poll. Errors of the
 * host preprocessing (RELOC_E_INVALID, RELOC_E_NOTFOUND, RELOC_E_BEAMGRID,
 * RELOC_E_EMPTY) are returned here. */
int32_t reloc_submit(reloc_ctx* ctx, int32_t map_id, int32_t set_id, const reloc_scan* scan,
                     const reloc_search_params* params, uint64_t* ticket);

/* Waits up to wait_ms (0: do not wait, < 0: no limit) for the ticket.
 * RELOC_E_PENDING: not finished (ticket stays valid). Otherwise the ticket
 * is consumed: its poses (out: host reloc_pose[cap]), *n_out and stats
 * (may be NULL; ms_total = submit to completion) are written and its status
 * returned (RELOC_OK, RELOC_E_TIMEOUT with best-so-far poses, or the error
 * that ended it). RELOC_E_NOTFOUND for an unknown or consumed ticket. */
int32_t reloc_poll(reloc_ctx* ctx, uint64_t ticket, int32_t wait_ms, reloc_pose* out,
                   int32_t cap, int32_t* n_out, reloc_stats* stats);

typedef struct {
  int64_t submitted, completed, failed, ticks;  /* ticks = scheduler rounds */
  int32_t queued, inflight;
  double busy_s;                                /* wall time spent in rounds */
  int32_t pollers;                              /* reloc_poll calls inside the library */
  int32_t reserved;
} reloc_serve_stats;

int32_t reloc_serve_stats_get(reloc_ctx* ctx, reloc_serve_stats* out);

/* ------------------------------------------------------------------------
 * Autotuning. Times the ray-cast kernel of a prepared request over a grid
 * of launch shapes, each warmed once and then launched reps times, and
 * keeps the fastest for the request's later runs (reloc_run,
 * reloc_run_batch); every shape gives bit-identical results.
 *   - Requests on the default path (coarse_metric 0, variant 0, a map with
 *     walk words) run the fused ray cast + SMAD kernel: the grid is 1, 2 or
 *     4 wavefronts per hypothesis workgroup x lane refill at 8, 16 or 32
 *     idle lanes. variant_out = 3, 4, 5 for refill 8, 16, 32; chunk_out =
 *     the wavefronts per workgroup. The choice is also kept on the map, and
 *     later requests of the map with the same beam grid (Ns) start from it.
 *   - Other requests on maps with walk words run the split ray cast: refill
 *     threshold 8 / 16 / 32 x 256, 384, 512, 768, 1024 rays per chunk;
 *     variant_out = the public variant (3, 4, 5), chunk_out = rays per
 *     chunk.
 *   - Requests on maps without walk words (above 2^28 cells) keep the
 *     bit-tile kernel and report their current settings.
 * ms_out: the chosen shape's mean kernel time. Any out pointer may be NULL.
 * Errors: RELOC_E_INVALID (reps < 1), RELOC_E_NOTFOUND, RELOC_E_DEVICE.
 * ---------------------------------------------------------------------- */
int32_t reloc_autotune(reloc_ctx* ctx, int32_t request_id, int32_t reps, int32_t* variant_out,
                       int32_t* chunk_out, float* ms_out);

/* ------------------------------------------------------------------------
 * Measured peaks of the device (the denominators of roofline fractions).
 * Runs short microbenchmarks on `device` with buffers of its own (about
 * 2.2 GiB, allocated with hipMalloc and freed before returning), each timed
 * as the best of five launches after a warm-up:
 *   valu_i32_ops : int32 lane-operations per second (adds and xors, eight
 *                  independent chains per lane, eight wavefronts per SIMD);
 *   l2_gathers   : 4-byte lane loads per second at pseudo-random offsets of
 *                  a 2 MiB table (resident in one XCD's L2);
 *   mall_gathers : the same over a 128 MiB table (beyond L2, within MALL);
 *   hbm_read     : bytes per second of a streaming read of 1 GiB;
 *   hbm_copy     : bytes read plus written per second copying 1 GiB.
 * Errors: RELOC_E_INVALID (null out), RELOC_E_DEVICE.
 * ---------------------------------------------------------------------- */
typedef struct {
  double valu_i32_ops, l2_gathers, mall_gathers, hbm_read, hbm_copy;
  int32_t compute_units, clock_khz;
} reloc_peaks;

int32_t reloc_measure_peaks(int32_t device, reloc_peaks* out);

/* ------------------------------------------------------------------------
 * Parity / inspection entry points (same kernels as reloc_run).
 * ---------------------------------------------------------------------- */

/* Panoramic synthetic scan of every hypothesis of the request (eq. 13):
 * hit_cell: host int32[n_hyp*Ns] (linear index, -1 none), range: host
 * float[n_hyp*Ns] (0 none), steps: host int32[n_hyp*Ns] traversal loop
 * iterations of the ray-cast kernel in use (the bit-tile variant makes one per
 * grid-line crossing, an exact corner counting once; the walk-word variants
 * one per free-space jump plus crossing). Any pointer may be NULL. */
int32_t reloc_debug_raycast(reloc_ctx* ctx, int32_t request_id, int32_t* hit_cell,
                            float* range, int32_t* steps);

/* SMAD(p) (FP64) and its argmin shift for every hypothesis, and the SMAD
 * order (hypothesis index per rank). Any pointer may be NULL. */
int32_t reloc_debug_smad(reloc_ctx* ctx, int32_t request_id, double* smad,
                         int32_t* argmin, int32_t* order);

/* TAM of every orientation for n ranks starting at rank r0 of the SMAD order:
 * T: host float[n*N_theta] (rank-major, may be NULL), tstar / kstar: host
 * float[n] / int32[n] (may be NULL). RELOC_E_INVALID, before any launch,
 * unless 0 <= r0, 1 <= n and r0 + n <= the request's hypothesis count. */
int32_t reloc_debug_tam(reloc_ctx* ctx, int32_t request_id, int32_t r0, int32_t n,
                        float* T, float* tstar, int32_t* kstar);

#ifdef __cplusplus
}
#endif
#endif /* RELOC_H */
