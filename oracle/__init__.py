"""FP64 CPU oracle of the relocalization hot path (arXiv 2511.01219).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the HIP library (``paper_2511_01219_amd``) and never imports it.

The arithmetic lives in ``reloc_oracle.cpp`` (plain C++17, FP64, IEEE, no
fast-math), loaded through ctypes; this module only marshals numpy arrays and
strings the C functions together in the paper's order:
scan preprocessing (eq. 11-16, 25-26) -> panoramic ray cast (eq. 13-14) ->
SMAD by direct summation (eq. 17-20) -> SMAD order and batches -> TAM over
orientations (eq. 22-31) -> early termination -> ranking (eq. 8-9).

Parity status of each part (what pins it) is listed in ``tests/test_oracle_*``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "reloc_oracle.cpp")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

# status codes shared (as numbers, by definition) with the C-ABI
E_INVALID, E_BEAMGRID, E_EMPTY = -1, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _declare(L):
    vp, i32, i64, f64, f32, u64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_float, ctypes.c_uint64)
    L.orc_edt_brute.argtypes = [i32, i32, vp, i32, vp]
    L.orc_edt.argtypes = [i32, i32, vp, i32, vp]
    L.orc_dirs.argtypes = [i32, vp]
    L.orc_dirs.restype = None
    L.orc_raycast.argtypes = [i32, i32, vp, i32, i32, i32, f64, f32, i32, vp, i32,
                              vp, vp, i32]
    L.orc_prep.argtypes = [i32, vp, f64, f64, i32, vp, vp, f32, f32, i32, i32, i32,
                           f64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.orc_smad.argtypes = [i32, i32, vp, i32, vp, f64, i32, i32, vp, vp, vp, i32]
    L.orc_tam.argtypes = [i32, i32, vp, f64, i32, i32, i32, vp, vp, i64, i64, i64,
                          f64, f64, f64, f64, i32, vp, vp, vp, i32]
    L.orc_stages.argtypes = [i32, i32, vp, f64, i32, i32, i32, vp, vp, i64, i64, i64,
                             f64, f64, f64, f64, i32, vp, vp, i32, f64, i32, i32, i32, i32,
                             vp, vp, vp, vp, vp, vp, i32]
    L.orc_refine.argtypes = [i32, i32, vp, f64, i32, i32, i32, vp, vp, i64, i64, i64,
                             f64, f64, f64, f64, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp,
                             i32]
    L.orc_caer.argtypes = [i32, i32, vp, i32, vp, vp, i32, vp, vp, vp, i32]
    L.orc_sample.argtypes = [i32, i32, vp, i32, vp, f64, f64, f64, f64, f64, i32,
                             f64, f64, u64, i32, vp, vp]
    L.orc_num_threads.argtypes = []
    L.orc_mix64.argtypes = [u64]
    L.orc_mix64.restype = u64
    L.orc_rrt.argtypes = [i32, i32, vp, i32, vp, f64, f64, f64, f64, f64, f64, f64, f64,
                          i32, u64, i32, i32, vp, vp, vp, vp]


def mix64(x: int) -> int:
    """splitmix64's output function applied to x + 0x9E3779B97F4A7C15: the
    sampler's visiting priority of cell c under seed s is mix64(s + c)."""
    return int(lib().orc_mix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
def edt(occ: np.ndarray, thr: int = 65, brute: bool = False) -> np.ndarray:
    """Exact squared EDT in cells (int64, -1 everywhere for an empty map)."""
    occ = np.ascontiguousarray(occ, dtype=np.int8)
    H, W = occ.shape
    k = np.empty((H, W), dtype=np.int64)
    f = lib().orc_edt_brute if brute else lib().orc_edt
    f(W, H, _p(occ), thr, _p(k))
    return k


def dirs(Ng: int) -> np.ndarray:
    U = np.empty((Ng, 2), dtype=np.int32)
    lib().orc_dirs(Ng, _p(U))
    return U


def raycast(occ: np.ndarray, hyp_xy: np.ndarray, Ns: int, Ng: int, res: float,
            range_max: float, thr: int = 65, brute: bool = False,
            threads: int = 0):
    """Hit cell (int32, -1 none) and range (float32, 0 none) for every
    hypothesis and panoramic direction j < Ns."""
    occ = np.ascontiguousarray(occ, dtype=np.int8)
    H, W = occ.shape
    hyp = np.ascontiguousarray(hyp_xy, dtype=np.int32).reshape(-1, 2)
    n = hyp.shape[0]
    hit = np.empty((n, Ns), dtype=np.int32)
    rng = np.empty((n, Ns), dtype=np.float32)
    st = lib().orc_raycast(W, H, _p(occ), thr, Ng, Ns, res, np.float32(range_max),
                           n, _p(hyp), int(brute), _p(hit), _p(rng), threads)
    if st != 0:
        raise ValueError("orc_raycast failed: %d" % st)
    return hit, rng


def prep(ranges: np.ndarray, angle_min: float, angle_increment: float,
         res: float, fov: Optional[Sequence] = None, range_min: float = 0.02,
         range_max: float = 30.0, n_skip_beam: int = 1, n_skip_enum: int = 1,
         n_theta: int = 0, alpha_mid_pm=(900, 700), alpha_low_pm=(700, 500)) -> Dict:
    ranges = np.ascontiguousarray(ranges, dtype=np.float32)
    n = len(ranges)
    nd = (n + n_skip_beam - 1) // n_skip_beam
    if fov:
        lo = np.array([float(a) for a, _ in fov], dtype=np.float64)
        hi = np.array([float(b) for _, b in fov], dtype=np.float64)
    else:
        lo = hi = None
    info = np.zeros(16, dtype=np.int64)
    dinfo = np.zeros(4, dtype=np.float64)
    bj = np.zeros(nd, dtype=np.int32)
    bs = np.zeros(nd, dtype=np.int32)
    bz = np.zeros(nd, dtype=np.float64)
    bq = np.zeros(nd, dtype=np.int32)
    am = np.array(alpha_mid_pm, dtype=np.int32)
    al = np.array(alpha_low_pm, dtype=np.int32)
    st = lib().orc_prep(n, _p(ranges), angle_min, angle_increment,
                        len(fov) if fov else 0, _p(lo), _p(hi),
                        np.float32(range_min), np.float32(range_max),
                        n_skip_beam, n_skip_enum, n_theta, res, _p(am), _p(al),
                        _p(info), _p(dinfo), _p(bj), _p(bs), _p(bz), _p(bq))
    out = dict(status=int(st), Ns=int(info[1]), Ntheta=int(info[2]), Ng=int(info[3]),
               N_fov=int(info[4]), N_valid=int(info[5]), k_full=int(info[6]),
               k_mid=int(info[7]), k_low=int(info[8]), panoramic=bool(info[9]),
               n_runs=int(info[10]), j0=int(info[11]), n_down=int(info[12]),
               n_shifts=int(info[13]), zbar=float(dinfo[0]), lam=float(dinfo[1]),
               beam_j=bj, beam_state=bs, beam_z=bz, beam_zq=bq,
               n_skip_enum=n_skip_enum, range_max=float(np.float32(range_max)))
    valid = bs == 2
    out["fov_j"] = np.ascontiguousarray(bj[bs >= 1])
    out["fov_z"] = np.ascontiguousarray(bz[bs >= 1])
    out["valid_j"] = np.ascontiguousarray(bj[valid])
    out["valid_zq"] = np.ascontiguousarray(bq[valid])
    return out


def smad(zhat: np.ndarray, pr: Dict, all_shifts: bool = False, threads: int = 0):
    """SMAD per hypothesis (FP64) and argmin shift m (eq. 16-20)."""
    zhat = np.ascontiguousarray(zhat, dtype=np.float32)
    n, Ns = zhat.shape
    assert Ns == pr["Ns"]
    s = np.empty(n, dtype=np.float64)
    a = np.empty(n, dtype=np.int32)
    allv = np.empty((n, pr["n_shifts"]), dtype=np.float64) if all_shifts else None
    lib().orc_smad(n, Ns, _p(zhat), len(pr["fov_j"]), _p(pr["fov_j"]), pr["zbar"],
                   pr["n_skip_enum"], int(pr["panoramic"]), _p(s), _p(a), _p(allv),
                   threads)
    return (s, a, allv) if all_shifts else (s, a)


def caer(zhat: np.ndarray, pr: Dict, all_shifts: bool = False, threads: int = 0):
    """CAER per hypothesis (FP64) and argmin shift m (eq. 21)."""
    zhat = np.ascontiguousarray(zhat, dtype=np.float32)
    n, Ns = zhat.shape
    assert Ns == pr["Ns"]
    nsh = (Ns + pr["n_skip_enum"] - 1) // pr["n_skip_enum"]
    c = np.empty(n, dtype=np.float64)
    a = np.empty(n, dtype=np.int32)
    allv = np.empty((n, nsh), dtype=np.float64) if all_shifts else None
    lib().orc_caer(n, Ns, _p(zhat), len(pr["fov_j"]), _p(pr["fov_j"]), _p(pr["fov_z"]),
                   pr["n_skip_enum"], _p(c), _p(a), _p(allv), threads)
    return (c, a, allv) if all_shifts else (c, a)


# columns of tam(); FINE_COL[m] is the score of fine metric m (0 TAM,
# 1 TAM_mean, 2 baseline, 3 LF)
TAM_COLS = ("T", "P", "s_d", "c", "Lbar", "mean_full", "mean_mid", "mean_low", "LF",
            "baseline", "T_mean")
FINE_COL = (0, 10, 9, 8)


def tam(kmap: np.ndarray, res: float, pr: Dict, q_xy: np.ndarray, q_k: np.ndarray,
        z_hit: float = 1.0, sigma_hit: float = 0.2, z_rand: float = 0.0,
        d_max: float = 2.0, threads: int = 0) -> np.ndarray:
    """[nq, 11] = T, P, s_d, c, Lbar, top-k_full / k_mid / k_low means, LF
    (eq. 32), baseline (eq. 33), T_mean (eq. 34), for each query (cell xy,
    heading k)."""
    kmap = np.ascontiguousarray(kmap, dtype=np.int64)
    H, W = kmap.shape
    q_xy = np.ascontiguousarray(q_xy, dtype=np.int32).reshape(-1, 2)
    q_k = np.ascontiguousarray(q_k, dtype=np.int32)
    out = np.empty((len(q_k), len(TAM_COLS)), dtype=np.float64)
    lib().orc_tam(W, H, _p(kmap), res, pr["Ns"], pr["Ntheta"], pr["N_valid"],
                  _p(pr["valid_j"]), _p(pr["valid_zq"]), pr["k_full"], pr["k_mid"],
                  pr["k_low"], z_hit, sigma_hit, z_rand, d_max, len(q_k), _p(q_xy),
                  _p(q_k), _p(out), threads)
    return out


def refine_span(pr: Dict, refine_dirs: int = -1) -> int:
    """Heading half-width of the refinement lattice in Ng-grid steps (-1:
    one orientation step, Ng / N_theta)."""
    return pr["Ng"] // pr["Ntheta"] if refine_dirs < 0 else int(refine_dirs)


def stages(kmap, res, pr, hyp_xy, smad_v, batch_k, tau, z_hit=1.0, sigma_hit=0.2,
           z_rand=0.0, d_max=2.0, all_T=False, threads: int = 0, refine_k: int = 0,
           refine_cells: int = 3, refine_dirs: int = -1, fine_metric: int = 0) -> Dict:
    """Batched multi-stage inference with optional local refinement of each
    batch's refine_k best poses (Sec. III pipeline text, Remark 2)."""
    kmap = np.ascontiguousarray(kmap, dtype=np.int64)
    H, W = kmap.shape
    hyp = np.ascontiguousarray(hyp_xy, dtype=np.int32).reshape(-1, 2)
    n = hyp.shape[0]
    smad_v = np.ascontiguousarray(smad_v, dtype=np.float64)
    order = np.empty(n, dtype=np.int32)
    tstar = np.zeros(n, dtype=np.float64)
    kstar = np.full(n, -1, dtype=np.int32)
    ref = np.zeros((n, 4), dtype=np.int64)
    info = np.zeros(4, dtype=np.int64)
    allT = np.zeros((n, pr["Ntheta"]), dtype=np.float64) if all_T else None
    lib().orc_stages(W, H, _p(kmap), res, pr["Ns"], pr["Ntheta"], pr["N_valid"],
                     _p(pr["valid_j"]), _p(pr["valid_zq"]), pr["k_full"], pr["k_mid"],
                     pr["k_low"], z_hit, sigma_hit, z_rand, d_max, n, _p(hyp),
                     _p(smad_v), batch_k,
                     float("nan") if tau is None else float(tau), int(fine_metric),
                     int(refine_k), int(refine_cells), refine_span(pr, refine_dirs),
                     _p(order), _p(tstar), _p(kstar), _p(ref), _p(info), _p(allT), threads)
    ne = int(info[2])
    out = dict(order=order, stages=int(info[0]), early_stopped=bool(info[1]),
               n_eval=ne, tstar=tstar[:ne], kstar=kstar[:ne],
               refined=ref[:ne, 0].astype(bool), ref_dxy=ref[:ne, 1:3].copy(),
               ref_g=ref[:ne, 3].copy())
    if all_T:
        out["all_T"] = allT[:ne]
    return out


def refine(kmap: np.ndarray, res: float, pr: Dict, q_xy: np.ndarray, q_g: np.ndarray,
           refine_cells: int = 3, refine_dirs: int = -1, z_hit: float = 1.0,
           sigma_hit: float = 0.2, z_rand: float = 0.0, d_max: float = 2.0,
           all_T: bool = False, threads: int = 0, fine_metric: int = 0):
    """Local refinement of poses (cell xy, heading index g on the Ng grid):
    refined T, (dx, dy), refined g, and optionally the T of every lattice
    point in raster order (NaN where not visited)."""
    kmap = np.ascontiguousarray(kmap, dtype=np.int64)
    H, W = kmap.shape
    q_xy = np.ascontiguousarray(q_xy, dtype=np.int32).reshape(-1, 2)
    q_g = np.ascontiguousarray(q_g, dtype=np.int64)
    nq = len(q_g)
    h, s = int(refine_cells), refine_span(pr, refine_dirs)
    L = (2 * s + 1) * (2 * h + 1) ** 2
    T = np.empty(nq, dtype=np.float64)
    dxy = np.empty((nq, 2), dtype=np.int32)
    g = np.empty(nq, dtype=np.int64)
    allv = np.empty((nq, L), dtype=np.float64) if all_T else None
    lib().orc_refine(W, H, _p(kmap), res, pr["Ns"], pr["Ntheta"], pr["N_valid"],
                     _p(pr["valid_j"]), _p(pr["valid_zq"]), pr["k_full"], pr["k_mid"],
                     pr["k_low"], z_hit, sigma_hit, z_rand, d_max, int(fine_metric), h, s,
                     nq, _p(q_xy),
                     _p(q_g), _p(T), _p(dxy), _p(g), _p(allv), threads)
    return (T, dxy, g, allv) if all_T else (T, dxy, g)


def sample(occ: np.ndarray, kmap: np.ndarray, res: float, origin=(0.0, 0.0),
           min_spacing: float = 0.3, robot_radius: float = 0.21, p0=None,
           seed: int = 0, n_target: int = 100, thr: int = 65) -> np.ndarray:
    """Hypothesis cells [n, 2] (x, y) in acceptance order."""
    occ = np.ascontiguousarray(occ, dtype=np.int8)
    kmap = np.ascontiguousarray(kmap, dtype=np.int64)
    H, W = occ.shape
    out = np.empty((n_target, 2), dtype=np.int32)
    n = np.zeros(1, dtype=np.int32)
    st = lib().orc_sample(W, H, _p(occ), thr, _p(kmap), res, origin[0], origin[1],
                          min_spacing, robot_radius, 0 if p0 is None else 1,
                          0.0 if p0 is None else p0[0], 0.0 if p0 is None else p0[1],
                          ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), n_target,
                          _p(out), _p(n))
    if st != 0:
        raise ValueError("orc_sample failed: %d" % st)
    return out[:int(n[0])].copy()


def rrt(occ: np.ndarray, kmap: np.ndarray, res: float, p0, origin=(0.0, 0.0),
        rho: float = 0.3, robot_radius: float = 0.21, eta_max: float = 0.6,
        eps_gain: int = 2, seed: int = 0, max_rounds: int = 64,
        max_nodes: int = 2_000_000, thr: int = 65) -> Dict:
    """Traversability-constrained RRT sampling (Algorithm 1): tree nodes
    [n, 2] (FP64, world), parents, representative cells [m, 2] (x, y) in node
    order, and (rounds, attempts, nodes, N_sampling)."""
    occ = np.ascontiguousarray(occ, dtype=np.int8)
    kmap = np.ascontiguousarray(kmap, dtype=np.int64)
    H, W = occ.shape
    nodes = np.empty((max_nodes, 2), dtype=np.float64)
    par = np.empty(max_nodes, dtype=np.int32)
    cells = np.empty((max_nodes, 2), dtype=np.int32)
    info = np.zeros(4, dtype=np.int64)
    nc = lib().orc_rrt(W, H, _p(occ), thr, _p(kmap), res, origin[0], origin[1], p0[0], p0[1],
                       rho, robot_radius, eta_max, eps_gain,
                       ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), max_rounds, max_nodes,
                       _p(nodes), _p(par), _p(cells), _p(info))
    if nc < 0:
        raise ValueError("orc_rrt failed: %d" % nc)
    n = int(info[2])
    return dict(nodes=nodes[:n].copy(), parent=par[:n].copy(), cells=cells[:nc].copy(),
                rounds=int(info[0]), attempts=int(info[1]), n_sampling=int(info[3]))


def ambiguity(order, tstar, ref_dxy, ref_g, hyp_xy, Ng: int, res: float, batch_k: int,
              tau) -> Dict:
    """Ambiguity of a finished search (Remark 1): the top-1 pose by (T desc,
    rank asc), the best T among the evaluated poses distinct from it by the
    success criterion of Sec. IV-C (position >= 0.5 m away, heading >= 30
    deg away on the Ng grid), best_margin = T1 - that T (-1 when none), and
    ambiguous = bit 0: some stage's best within 1e-4 of tau, bit 1:
    best_margin <= 1e-4 |T1| + 1e-7."""
    ne = len(tstar)
    hyp = np.asarray(hyp_xy).reshape(-1, 2)
    ranks = np.lexsort((np.arange(ne), -np.asarray(tstar)))
    r1 = int(ranks[0])
    cell = hyp[np.asarray(order)[:ne]] + np.asarray(ref_dxy)
    g = np.asarray(ref_g).astype(np.int64)
    best2 = None
    for r in range(ne):
        ex = int(cell[r, 0] - cell[r1, 0])
        ey = int(cell[r, 1] - cell[r1, 1])
        dg = abs(int(g[r] - g[r1]))
        if 2 * dg > Ng:
            dg = Ng - dg
        if float(ex * ex + ey * ey) * res * res >= 0.25 or 12 * dg >= Ng:
            if best2 is None or tstar[r] > best2:
                best2 = float(tstar[r])
    t1 = float(tstar[r1])
    margin = -1.0 if best2 is None else t1 - best2
    amb = 0
    if tau is not None:
        for b0 in range(0, ne, batch_k):
            tb = float(np.max(tstar[b0:b0 + batch_k]))
            if tau - 1e-4 <= tb <= tau + 1e-4:
                amb |= 1
    if best2 is not None and margin <= 1e-4 * abs(t1) + 1e-7:
        amb |= 2
    return dict(top=r1, best_margin=margin, ambiguous=amb)


def heading(k: int, Ntheta: int) -> float:
    """Heading of orientation index k, wrapped to [-pi, pi)."""
    th = (2.0 * math.pi * k) / Ntheta
    if th >= math.pi:
        th -= 2.0 * math.pi
    return th


def relocalize(occ: np.ndarray, res: float, origin, hyp_xy: np.ndarray,
               ranges: np.ndarray, angle_min: float, angle_increment: float,
               range_min: float, range_max: float, fov=None, n_theta: int = 0,
               batch_k: int = 64, tau: Optional[float] = 0.95, k_out: int = 10,
               z_hit: float = 1.0, sigma_hit: float = 0.2, z_rand: float = 0.0,
               d_max: float = 2.0, n_skip_beam: int = 1, n_skip_enum: int = 1,
               alpha_mid_pm=(900, 700), alpha_low_pm=(700, 500), thr: int = 65,
               kmap: Optional[np.ndarray] = None, threads: int = 0,
               keep: bool = False, refine_k: int = 0, refine_cells: int = 3,
               refine_dirs: int = -1, coarse_metric: int = 0,
               fine_metric: int = 0) -> Dict:
    """The whole hot path, step by step, in the paper's order."""
    if kmap is None:
        kmap = edt(occ, thr)
    pr = prep(ranges, angle_min, angle_increment, res, fov, range_min, range_max,
              n_skip_beam, n_skip_enum, n_theta, alpha_mid_pm, alpha_low_pm)
    if pr["status"] != 0:
        raise ValueError("scan rejected: %d" % pr["status"])
    hit, zhat = raycast(occ, hyp_xy, pr["Ns"], pr["Ng"], res, range_max, thr,
                        threads=threads)
    # coarse metric: 0 SMAD (prefix sums), 1 SMAD (direct sums; the same
    # values), 2 CAER, 3 none (the set's own order)
    if coarse_metric in (0, 1):
        sm, am = smad(zhat, pr, threads=threads)
    elif coarse_metric == 2:
        sm, am = caer(zhat, pr, threads=threads)
    else:
        sm, am = np.zeros(len(zhat)), np.zeros(len(zhat), np.int32)
    st = stages(kmap, res, pr, hyp_xy, sm, batch_k, tau, z_hit, sigma_hit, z_rand,
                d_max, threads=threads, refine_k=refine_k, refine_cells=refine_cells,
                refine_dirs=refine_dirs, fine_metric=fine_metric)
    ne = st["n_eval"]
    ranks = np.arange(ne)
    rank_order = np.lexsort((ranks, -st["tstar"]))     # T desc, rank asc
    hyp = np.asarray(hyp_xy).reshape(-1, 2)
    poses = []
    for r in rank_order[:k_out]:
        h = int(st["order"][r])
        k = int(st["kstar"][r])
        cx = int(hyp[h, 0] + st["ref_dxy"][r, 0])
        cy = int(hyp[h, 1] + st["ref_dxy"][r, 1])
        g = int(st["ref_g"][r])
        poses.append(dict(x=origin[0] + (cx + 0.5) * res,
                          y=origin[1] + (cy + 0.5) * res,
                          theta=(heading(g, pr["Ng"]) if st["refined"][r]
                                 else heading(k, pr["Ntheta"])),
                          tam=float(st["tstar"][r]),
                          smad=float(sm[h]), hyp=h, k=k, rank=int(r),
                          stage=int(r) // batch_k, cx=cx, cy=cy, g=g,
                          refined=bool(st["refined"][r])))
    amb = ambiguity(st["order"], st["tstar"], st["ref_dxy"], st["ref_g"], hyp, pr["Ng"], res,
                    batch_k, tau)
    out = dict(poses=poses, prep=pr, stages=st["stages"], best_margin=amb["best_margin"],
               ambiguous=amb["ambiguous"],
               early_stopped=st["early_stopped"], n_eval=ne,
               smad_evals=len(sm) * (pr["n_shifts"] if coarse_metric in (0, 1) else
                                     -(-pr["Ns"] // pr["n_skip_enum"]) if coarse_metric == 2
                                     else 0),
               tam_evals=ne * pr["Ntheta"])
    if keep:
        out.update(hit=hit, zhat=zhat, smad=sm, argm=am, order=st["order"],
                   tstar=st["tstar"], kstar=st["kstar"], kmap=kmap,
                   refined=st["refined"], ref_dxy=st["ref_dxy"], ref_g=st["ref_g"])
    return out
