"""Multi-map workloads: the batched workload (64 queries over 8 resident maps)
and the serving workload (Poisson arrivals over 16 resident maps).

Streams: ``numpy.random.default_rng([config_id, stream, index])`` with
stream 0 = layout of map ``index``, 1 = true pose of query ``index``, 2 = its
scan noise / clutter / drop-outs, 4 = its query parameters, 5 = arrival
times. The hypothesis set of map ``m`` is drawn by the method's sampler with
seed ``1000 * config_id + m``; a query uses the first ``n_hyp`` hypotheses
of its map's set.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Any, Dict, List, Sequence

import numpy as np

from .maps import rasterize, tiled_rooms_map, warehouse_map
from .scans import ScanSpec, feasible_cells, lidar_scan, true_pose


@dataclass
class Query:
    map_index: int
    pose: tuple
    ranges: np.ndarray
    angle_min: float
    angle_increment: float
    range_min: float
    range_max: float
    n_hyp: int
    fov_deg: float
    n_beams: int
    search: Dict[str, Any]
    arrival: float = 0.0             # seconds from the start (serving)


@dataclass
class MultiWorkload:
    name: str
    maps: List[np.ndarray]           # int8 (H, W) each
    layouts: List[str]
    resolution: float
    queries: List[Query]
    sample: Dict[str, Any]           # min_spacing, robot_radius, n_target per map, seeds
    meta: Dict[str, Any] = field(default_factory=dict)


def _rng(cid: int, stream: int, index: int) -> np.random.Generator:
    return np.random.default_rng([cid, stream, index])


def _maps(cid: int, sizes: Sequence[int], layouts: Sequence[str]):
    maps, masks = [], []
    for m, (size, lay) in enumerate(zip(sizes, layouts)):
        rng = _rng(cid, 0, m)
        if lay == "warehouse":
            spec = warehouse_map(rng, size, size)
        else:
            spec = tiled_rooms_map(rng, size, size)
        occ = rasterize(spec)
        maps.append(occ)
        masks.append(feasible_cells(occ, spec.resolution, 0.21))
    return maps, masks


def _query(cid, q, occ, mask, m, res, fov, n_beams, n_hyp, r_max, sigma, drop, clutter,
           search, arrival=0.0) -> Query:
    pose = true_pose(occ, res, (0.0, 0.0), _rng(cid, 1, q), 0.21, mask=mask)
    spec = ScanSpec(float(fov), int(n_beams), float(r_max), 0.02, sigma, drop, clutter)
    ranges, amin, ainc, _ = lidar_scan(occ, res, (0.0, 0.0), pose, spec, _rng(cid, 2, q))
    return Query(m, pose, ranges, amin, ainc, spec.range_min, spec.range_max, int(n_hyp),
                 float(fov), int(n_beams), dict(search), arrival)


def make_batched(n_queries: int = 64, sizes: Sequence[int] = (500, 1000, 2000, 4000),
                 n_range=(1000, 50000), cid: int = 3) -> MultiWorkload:
    """Two maps per size (tiled rooms and warehouse); per query: a map, a
    log-uniform hypothesis count, FoV in {180, 240, 270, 360} deg with
    N in {360, 480, 540, 720, 960, 1080} beams (Ns = 360 N / FoV is then an
    integer), r_max 20 m, noise 0.02 m, 5 % drop-outs; N_theta 360, top-64
    per stage, tau 0.95."""
    msizes = [s for s in sizes for _ in range(2)]
    layouts = ["rooms", "warehouse"] * len(sizes)
    maps, masks = _maps(cid, msizes, layouts)
    res = 0.05
    fovs = (180.0, 240.0, 270.0, 360.0)
    beams = (360, 480, 540, 720, 960, 1080)
    queries = []
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    for q in range(n_queries):
        r = _rng(cid, 4, q)
        m = int(r.integers(0, len(maps)))
        fov = fovs[int(r.integers(0, len(fovs)))]
        nb = beams[int(r.integers(0, len(beams)))]
        n_hyp = int(round(math.exp(r.uniform(lo, hi))))
        queries.append(_query(cid, q, maps[m], masks[m], m, res, fov, nb, n_hyp, 20.0, 0.02,
                              0.05, 0.0, dict(n_theta=360, batch_k=64, tau=0.95)))
    n_target = [max([qq.n_hyp for qq in queries if qq.map_index == m] or [1])
                for m in range(len(maps))]
    return MultiWorkload("batched: %d queries over %d maps %s" % (n_queries, len(maps),
                                                                   list(sizes)),
                         maps, layouts, res, queries,
                         dict(min_spacing=0.3, robot_radius=0.21, n_target=n_target,
                              seeds=[1000 * cid + m for m in range(len(maps))]))


def make_serving(rate: float, n_requests: int, sizes: Sequence[int] = (1000, 2000, 3000, 4000),
                 per_size: int = 4, n_range=(2000, 40000), cid: int = 4) -> MultiWorkload:
    """``per_size`` maps of every size (alternating tiled rooms / warehouse);
    Poisson arrivals at ``rate`` per second; per request: a map, a
    log-uniform hypothesis count, FoV 270 or 360 deg with N in {540, 720,
    960, 1080, 1440} beams, r_max 20 m, noise 0.02 m, 5 % drop-outs;
    N_theta 360, top-64 per stage, tau 0.95."""
    msizes = [s for s in sizes for _ in range(per_size)]
    layouts = ["rooms" if i % 2 == 0 else "warehouse" for i in range(len(msizes))]
    maps, masks = _maps(cid, msizes, layouts)
    res = 0.05
    gaps = _rng(cid, 5, 0).exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    queries = []
    for q in range(n_requests):
        r = _rng(cid, 4, q)
        m = int(r.integers(0, len(maps)))
        fov = (270.0, 360.0)[int(r.integers(0, 2))]
        nb = (540, 720, 960, 1080, 1440)[int(r.integers(0, 5))]
        n_hyp = int(round(math.exp(r.uniform(lo, hi))))
        queries.append(_query(cid, q, maps[m], masks[m], m, res, fov, nb, n_hyp, 20.0, 0.02,
                              0.05, 0.0, dict(n_theta=360, batch_k=64, tau=0.95),
                              float(t[q])))
    n_target = [max([qq.n_hyp for qq in queries if qq.map_index == m] or [1])
                for m in range(len(maps))]
    return MultiWorkload("serving: %d requests at %.0f/s over %d maps" % (n_requests, rate,
                                                                        len(maps)),
                         maps, layouts, res, queries,
                         dict(min_spacing=0.3, robot_radius=0.21, n_target=n_target,
                              seeds=[1000 * cid + m for m in range(len(maps))]),
                         dict(rate=rate))
