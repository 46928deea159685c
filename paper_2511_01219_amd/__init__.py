"""MI355X relocalization library: Python binding of libreloc.so.

Argument marshalling only: every step of the hot path runs in the HIP
kernels behind the C ABI of ``include/reloc.h``. PyTorch supplies device
memory (its caching allocator, through the allocator hook) and the stream
work is issued on (the current torch stream).

    import paper_2511_01219_amd as reloc
    ctx = reloc.Context()
    m = ctx.load_map(occ, resolution=0.05)
    s, n = ctx.sample_hypotheses(m, n_target=20000, min_spacing=0.3)
    poses, stats = ctx.relocalize(m, s, ranges, angle_min, angle_increment,
                                  range_max=25.0, n_theta=720, batch_k=64)
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _abi
from ._abi import (E_BEAMGRID, E_BUSY, E_DEVICE, E_EMPTY, E_INVALID, E_NOMEM, E_NOTFOUND,
                   E_PENDING, E_TIMEOUT, OK, STATUS_NAMES)

__all__ = ["Context", "RelocError", "scan_info", "search_params", "lib", "version",
           "OK", "E_INVALID", "E_NOMEM", "E_NOTFOUND", "E_BEAMGRID", "E_EMPTY", "E_BUSY",
           "E_PENDING", "E_TIMEOUT", "E_DEVICE"]


class RelocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


def lib():
    return _abi.load()


def version() -> int:
    return int(lib().reloc_version())


def _check(code: int, allow=()) -> int:
    if code != OK and code not in allow:
        raise RelocError(code, lib().reloc_last_error().decode())
    return code


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def search_params(**kw) -> _abi.reloc_search_params:
    """reloc_search_params with the library defaults, overridden by ``kw``
    (tau=None means no early termination)."""
    p = _abi.reloc_search_params()
    lib().reloc_search_defaults(C.byref(p))
    for k, v in kw.items():
        if k == "tau" and v is None:
            v = float("nan")
        if k in ("alpha_mid_pm", "alpha_low_pm"):
            getattr(p, k)[0], getattr(p, k)[1] = int(v[0]), int(v[1])
            continue
        if not hasattr(p, k):
            raise TypeError("unknown search parameter %r" % k)
        setattr(p, k, v)
    return p


_POSE_FIELDS = tuple(f for f, _ in _abi.reloc_pose._fields_)
_STAT_FIELDS = tuple(f for f, _ in _abi.reloc_stats._fields_)


def _poses(out, n):
    res = []
    for i in range(n):
        o = out[i]
        res.append({f: getattr(o, f) for f in _POSE_FIELDS})
    return res


def _stats(st, code):
    d = {f: getattr(st, f) for f in _STAT_FIELDS}
    d["status"] = code
    return d


class _Scan:
    """Keeps the host buffers of a reloc_scan alive."""

    def __init__(self, ranges, angle_min, angle_increment, range_min, range_max, fov):
        self.ranges = np.ascontiguousarray(ranges, dtype=np.float32)
        self.fov = None
        n_fov = 0
        if fov:
            self.fov = (_abi.reloc_interval * len(fov))(
                *[_abi.reloc_interval(float(a), float(b)) for a, b in fov])
            n_fov = len(fov)
        self.s = _abi.reloc_scan(len(self.ranges), self.ranges.ctypes.data, float(angle_min),
                                 float(angle_increment), n_fov, self.fov, float(range_min),
                                 float(range_max))


def scan_info(ranges, angle_min, angle_increment, resolution, range_min=0.02,
              range_max=30.0, fov=None, **search) -> Dict:
    """Host-side preprocessing summary of a scan (no device needed)."""
    sc = _Scan(ranges, angle_min, angle_increment, range_min, range_max, fov)
    p = search_params(**search)
    out = _abi.reloc_scan_info()
    _check(lib().reloc_scan_info_get(C.byref(sc.s), C.byref(p), float(resolution),
                                     C.byref(out)))
    d = {f: getattr(out, f) for f, _ in out._fields_}
    d["lambda"] = d.pop("lambda_")
    return d


def measure_peaks(device: int = 0) -> Dict:
    """Measured sustainable peaks of the device (reloc_measure_peaks): int32
    VALU lane-ops/s, L2- and MALL-resident 4-byte gathers/s, HBM streaming
    read and copy bytes/s."""
    out = _abi.reloc_peaks()
    _check(lib().reloc_measure_peaks(int(device), C.byref(out)))
    return {f: getattr(out, f) for f, _ in out._fields_}


class Context:
    """A reloc_ctx on one GPU, with torch's caching allocator and stream."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, use_torch: bool = True,
                 stream=None):
        self._lib = lib()
        self._h = C.c_void_p()
        self._cb = None
        alloc_p = None
        stream_p = None
        if use_torch:
            import torch
            if not torch.cuda.is_available():
                raise RelocError(E_DEVICE, "no GPU visible to torch")
            self._torch_dev = device
            st = stream if stream is not None else torch.cuda.current_stream(device)
            if st.cuda_stream == 0:
                # the legacy default stream: give the library a stream of its
                # own (default priority) so torch's allocator can track it
                st = torch.cuda.Stream(device=device)
            self._torch_stream = st
            stream_p = C.c_void_p(st.cuda_stream)

            def _alloc(nbytes, user, _t=torch, _d=device, _s=st):
                try:
                    return int(_t.cuda.caching_allocator_alloc(int(nbytes), _d, _s))
                except Exception:
                    return None

            def _free(ptr, user, _t=torch):
                try:
                    _t.cuda.caching_allocator_delete(ptr)
                except Exception:
                    # a context left open until interpreter shutdown is torn
                    # down after torch; the process is ending, nothing to free
                    pass

            self._cb = (_abi.ALLOC_FN(_alloc), _abi.FREE_FN(_free))
            self._alloc_struct = _abi.reloc_allocator(self._cb[0], self._cb[1], None)
            alloc_p = C.byref(self._alloc_struct)
        _check(self._lib.reloc_ctx_create(int(device), alloc_p, stream_p, int(hbm_budget),
                                          C.byref(self._h)))

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if self._h:
            self._lib.reloc_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def bytes(self) -> int:
        return int(self._lib.reloc_ctx_bytes(self._h))

    # -- maps -----------------------------------------------------------------
    def load_map(self, occ: np.ndarray, resolution: float = 0.05,
                 origin: Tuple[float, float] = (0.0, 0.0), occ_threshold: int = 65) -> int:
        occ = np.ascontiguousarray(occ, dtype=np.int8)
        H, W = occ.shape
        d = _abi.reloc_map_desc(W, H, float(resolution), float(origin[0]), float(origin[1]),
                                int(occ_threshold))
        mid = C.c_int32()
        _check(self._lib.reloc_load_map(self._h, C.byref(d), _ptr(occ), C.byref(mid)))
        self._shapes = getattr(self, "_shapes", {})
        self._shapes[mid.value] = (H, W)
        return mid.value

    def unload_map(self, map_id: int):
        _check(self._lib.reloc_unload_map(self._h, int(map_id)))

    def read_edt(self, map_id: int) -> np.ndarray:
        H, W = self._shapes[map_id]
        k = np.empty((H, W), dtype=np.uint32)
        _check(self._lib.reloc_read_edt(self._h, int(map_id), _ptr(k)))
        return k

    # -- hypotheses -----------------------------------------------------------
    def sample_hypotheses(self, map_id: int, n_target: int, min_spacing: float = 0.3,
                          robot_radius: float = 0.21, p0=None, seed: int = 0):
        p = _abi.reloc_sample_params(int(n_target), float(min_spacing), float(robot_radius),
                                     0 if p0 is None else 1,
                                     0.0 if p0 is None else float(p0[0]),
                                     0.0 if p0 is None else float(p0[1]),
                                     int(seed) & 0xFFFFFFFFFFFFFFFF)
        sid, n = C.c_int32(), C.c_int32()
        _check(self._lib.reloc_sample_hypotheses(self._h, int(map_id), C.byref(p),
                                                 C.byref(sid), C.byref(n)))
        return sid.value, n.value

    def sample_rrt(self, map_id: int, p0, rho: float = 0.3, robot_radius: float = 0.21,
                   eta_max: float = 0.6, eps_gain: int = 2, seed: int = 0,
                   max_rounds: int = 64, max_nodes: int = 16 << 20, tree_cap: int = 0):
        """Traversability-constrained RRT hypothesis set (Algorithm 1): returns
        (set_id, n, info) and, with tree_cap > 0, the first tree_cap nodes
        ([n, 2] world) and parents."""
        p = _abi.reloc_rrt_params(float(p0[0]), float(p0[1]), float(rho), float(robot_radius),
                                  float(eta_max), int(eps_gain), int(max_rounds),
                                  int(max_nodes), int(seed) & 0xFFFFFFFFFFFFFFFF)
        sid, n = C.c_int32(), C.c_int32()
        info = _abi.reloc_rrt_info()
        nodes = np.empty((max(0, tree_cap), 2), dtype=np.float64) if tree_cap > 0 else None
        par = np.empty(max(0, tree_cap), dtype=np.int32) if tree_cap > 0 else None
        _check(self._lib.reloc_sample_rrt(self._h, int(map_id), C.byref(p), C.byref(sid),
                                          C.byref(n), C.byref(info), _ptr(nodes), _ptr(par),
                                          int(tree_cap)))
        inf = {f: getattr(info, f) for f, _ in info._fields_}
        if tree_cap > 0:
            k = min(tree_cap, inf["nodes"])
            return sid.value, n.value, inf, nodes[:k], par[:k]
        return sid.value, n.value, inf

    def set_hypotheses(self, map_id: int, cell_xy: np.ndarray) -> int:
        xy = np.ascontiguousarray(cell_xy, dtype=np.int32).reshape(-1, 2)
        sid = C.c_int32()
        _check(self._lib.reloc_set_hypotheses(self._h, int(map_id), _ptr(xy), len(xy),
                                              C.byref(sid)))
        return sid.value

    def read_hypotheses(self, set_id: int) -> np.ndarray:
        n = C.c_int32()
        _check(self._lib.reloc_read_hypotheses(self._h, int(set_id), None, 0, C.byref(n)))
        out = np.empty((n.value, 2), dtype=np.int32)
        _check(self._lib.reloc_read_hypotheses(self._h, int(set_id), _ptr(out), n.value,
                                               C.byref(n)))
        return out

    def free_hypotheses(self, set_id: int):
        _check(self._lib.reloc_free_hypotheses(self._h, int(set_id)))

    # -- requests -------------------------------------------------------------
    def prepare(self, map_id: int, set_id: int, ranges, angle_min: float,
                angle_increment: float, range_min: float = 0.02, range_max: float = 30.0,
                fov: Optional[Sequence] = None, **search) -> int:
        sc = _Scan(ranges, angle_min, angle_increment, range_min, range_max, fov)
        p = search_params(**search)
        rid = C.c_int32()
        _check(self._lib.reloc_prepare(self._h, int(map_id), int(set_id), C.byref(sc.s),
                                       C.byref(p), C.byref(rid)))
        return rid.value

    def run(self, request_id: int, cap: int = 64, allow_timeout: bool = False):
        out = (_abi.reloc_pose * max(1, cap))()
        n = C.c_int32()
        st = _abi.reloc_stats()
        code = _check(self._lib.reloc_run(self._h, int(request_id), out, int(cap), C.byref(n),
                                          C.byref(st)),
                      allow=(E_TIMEOUT,) if allow_timeout else ())
        return _poses(out, n.value), _stats(st, code)

    def release(self, request_id: int):
        _check(self._lib.reloc_release(self._h, int(request_id)))

    def relocalize(self, map_id: int, set_id: int, ranges, angle_min: float,
                   angle_increment: float, range_min: float = 0.02, range_max: float = 30.0,
                   fov: Optional[Sequence] = None, cap: int = 64, **search):
        """relocalize(scan, fov, beam angles) -> (ranked poses, stats): one
        reloc_relocalize call (prepare + run + release in the library)."""
        sc = _Scan(ranges, angle_min, angle_increment, range_min, range_max, fov)
        p = search_params(**search)
        out = (_abi.reloc_pose * max(1, cap))()
        n = C.c_int32()
        st = _abi.reloc_stats()
        code = _check(self._lib.reloc_relocalize(self._h, int(map_id), int(set_id),
                                                 C.byref(sc.s), C.byref(p), out, int(cap),
                                                 C.byref(n), C.byref(st)))
        return _poses(out, n.value), _stats(st, code)

    def relocalize_noalloc(self, map_id: int, set_id: int, ranges, angle_min: float,
                           angle_increment: float, range_min: float = 0.02,
                           range_max: float = 30.0, fov: Optional[Sequence] = None,
                           cap: int = 64, **search):
        """relocalize through reloc_relocalize_noalloc: no device allocation,
        the library's per-GPU scratch region instead."""
        sc = _Scan(ranges, angle_min, angle_increment, range_min, range_max, fov)
        p = search_params(**search)
        out = (_abi.reloc_pose * max(1, cap))()
        n = C.c_int32()
        st = _abi.reloc_stats()
        code = _check(self._lib.reloc_relocalize_noalloc(self._h, int(map_id), int(set_id),
                                                         C.byref(sc.s), C.byref(p), out,
                                                         int(cap), C.byref(n), C.byref(st)))
        return _poses(out, n.value), _stats(st, code)

    def coarse_scores(self, request_id: int, n_hyp: int):
        """Coarse metric of the n_hyp hypotheses of the request: (score FP64,
        argmin shift, stable order, stats)."""
        n = int(n_hyp)
        sc = np.empty(n, dtype=np.float64)
        sh = np.empty(n, dtype=np.int32)
        order = np.empty(n, dtype=np.int32)
        st = _abi.reloc_stats()
        _check(self._lib.reloc_coarse_scores(self._h, int(request_id), n, _ptr(sc), _ptr(sh),
                                             _ptr(order), C.byref(st)))
        return sc, sh, order, _stats(st, OK)

    def score_poses(self, request_id: int, cell_xy, heading):
        """Fine metric of the request at explicit poses (cells, heading index
        on the Ng grid); returns (scores float32, kernel ms)."""
        xy = np.ascontiguousarray(cell_xy, dtype=np.int32).reshape(-1, 2)
        g = np.ascontiguousarray(heading, dtype=np.int32).reshape(-1)
        if len(g) != len(xy):
            raise ValueError("cell_xy and heading differ in length")
        out = np.empty(len(g), dtype=np.float32)
        ms = C.c_float()
        _check(self._lib.reloc_score_poses(self._h, int(request_id), _ptr(xy), _ptr(g), len(g),
                                           _ptr(out), C.byref(ms)))
        return out, ms.value

    def autotune(self, request_id: int, reps: int = 3):
        """Picks the fastest ray-cast launch shape for the request; returns
        (variant, shape, mean kernel ms): shape = wavefronts per hypothesis
        workgroup for the fused kernel (the default path), else rays per
        chunk of the split ray cast."""
        v, ch, ms = C.c_int32(), C.c_int32(), C.c_float()
        _check(self._lib.reloc_autotune(self._h, int(request_id), int(reps), C.byref(v),
                                        C.byref(ch), C.byref(ms)))
        return v.value, ch.value, ms.value

    # -- batched form -------------------------------------------------------------
    def run_batch(self, request_ids: Sequence[int], cap: int = 64):
        """Runs prepared requests together; returns [(poses, stats)] in order.
        stats["status"] is OK or E_TIMEOUT per request."""
        n = len(request_ids)
        ids = np.ascontiguousarray(request_ids, dtype=np.int32)
        out = (_abi.reloc_pose * max(1, n * cap))()
        n_out = np.zeros(max(1, n), dtype=np.int32)
        status = np.zeros(max(1, n), dtype=np.int32)
        st = (_abi.reloc_stats * max(1, n))()
        _check(self._lib.reloc_run_batch(self._h, n, _ptr(ids), out, int(cap), _ptr(n_out),
                                         _ptr(status), st))
        res = []
        for i in range(n):
            poses = [{f: getattr(out[i * cap + j], f) for f, _ in out[i * cap + j]._fields_}
                     for j in range(int(n_out[i]))]
            stats = {f: getattr(st[i], f) for f, _ in st[i]._fields_}
            stats["status"] = int(status[i])
            res.append((poses, stats))
        return res

    # -- serving ----------------------------------------------------------------------
    def serve_configure(self, max_inflight: int = 64, hbm_reserve: int = 0, max_admit: int = 16):
        cfg = _abi.reloc_serve_config(int(max_inflight), int(hbm_reserve), int(max_admit))
        _check(self._lib.reloc_serve_configure(self._h, C.byref(cfg)))

    def submit(self, map_id: int, set_id: int, ranges, angle_min: float,
               angle_increment: float, range_min: float = 0.02, range_max: float = 30.0,
               fov: Optional[Sequence] = None, **search) -> int:
        sc = _Scan(ranges, angle_min, angle_increment, range_min, range_max, fov)
        p = search_params(**search)
        t = C.c_uint64()
        _check(self._lib.reloc_submit(self._h, int(map_id), int(set_id), C.byref(sc.s),
                                      C.byref(p), C.byref(t)))
        return t.value

    def poll(self, ticket: int, wait_ms: int = -1, cap: int = 64):
        """(poses, stats) when finished, None while pending."""
        out = (_abi.reloc_pose * max(1, cap))()
        n = C.c_int32()
        st = _abi.reloc_stats()
        code = _check(self._lib.reloc_poll(self._h, C.c_uint64(int(ticket)), int(wait_ms), out,
                                           int(cap), C.byref(n), C.byref(st)),
                      allow=(E_PENDING, E_TIMEOUT))
        if code == E_PENDING:
            return None
        poses = [{f: getattr(out[i], f) for f, _ in out[i]._fields_} for i in range(n.value)]
        stats = {f: getattr(st, f) for f, _ in st._fields_}
        stats["status"] = code
        return poses, stats

    def serve_stats(self) -> dict:
        s = _abi.reloc_serve_stats()
        _check(self._lib.reloc_serve_stats_get(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    # -- parity / inspection ----------------------------------------------------
    def debug_raycast(self, request_id: int, n_hyp: int, Ns: int, steps: bool = False,
                      steps_only: bool = False):
        """Hit cells and ranges of every ray (and, with steps, the traversal
        iterations per ray); steps_only returns the iterations alone."""
        hit = None if steps_only else np.empty((n_hyp, Ns), dtype=np.int32)
        rng = None if steps_only else np.empty((n_hyp, Ns), dtype=np.float32)
        stp = np.empty((n_hyp, Ns), dtype=np.int32) if (steps or steps_only) else None
        _check(self._lib.reloc_debug_raycast(self._h, int(request_id), _ptr(hit), _ptr(rng),
                                             _ptr(stp)))
        if steps_only:
            return stp
        return (hit, rng, stp) if steps else (hit, rng)

    def debug_smad(self, request_id: int, n_hyp: int):
        s = np.empty(n_hyp, dtype=np.float64)
        a = np.empty(n_hyp, dtype=np.int32)
        o = np.empty(n_hyp, dtype=np.int32)
        _check(self._lib.reloc_debug_smad(self._h, int(request_id), _ptr(s), _ptr(a), _ptr(o)))
        return s, a, o

    def debug_tam(self, request_id: int, r0: int, n: int, Ntheta: int, want_T: bool = True):
        T = np.empty((n, Ntheta), dtype=np.float32) if want_T else None
        ts = np.empty(n, dtype=np.float32)
        ks = np.empty(n, dtype=np.int32)
        _check(self._lib.reloc_debug_tam(self._h, int(request_id), int(r0), int(n), _ptr(T),
                                         _ptr(ts), _ptr(ks)))
        return T, ts, ks
