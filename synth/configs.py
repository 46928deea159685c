"""The five synthetic workloads (plain-small, plain-large, batched, serving,
stress) and tiny micro-maps for brute-force checks.

Every random stream is ``numpy.random.default_rng([config_id, stream])`` with
stream 0 = map layout, 1 = true pose, 2 = scan noise/clutter/drop-outs,
3 = environment perturbation; the hypothesis sampler's own seed (a method
input) is ``config_id``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np

from .maps import (MapSpec, rooms_map, warehouse_map, tiled_rooms_map,
                   mixed_map, perturb_map, rasterize)
from .scans import ScanSpec, true_pose, lidar_scan, feasible_cells


@dataclass
class Workload:
    name: str
    occ: np.ndarray                  # int8 (H, W), the map searched
    resolution: float
    origin: tuple
    pose: tuple                      # true (x, y, theta)
    ranges: np.ndarray               # float32 [N]
    angle_min: float
    angle_increment: float
    range_min: float
    range_max: float
    sample: Dict[str, Any]           # n_target, min_spacing, robot_radius, seed
    search: Dict[str, Any]           # n_theta, batch_k, tau, ...
    scan_occ: Optional[np.ndarray] = None   # map the scan was taken in
    meta: Dict[str, Any] = field(default_factory=dict)


def _rng(cid: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cid, stream])


CONFIGS = {
    1: dict(name="plain-small rooms 200x200, 300 hypotheses, 270deg/360 beams",
            layout="rooms", size=200, n_target=300, min_spacing=0.3,
            scan=ScanSpec(270.0, 360, 12.0, 0.02, 0.02, 0.05, 0.0),
            n_theta=360, batch_k=10, tau=0.95),
    2: dict(name="plain-large warehouse 2000x2000, 20k hypotheses, 270deg/720 beams",
            layout="warehouse", size=2000, n_target=20000, min_spacing=0.3,
            scan=ScanSpec(270.0, 720, 25.0, 0.02, 0.03, 0.0, 0.10),
            n_theta=720, batch_k=64, tau=0.95),
    5: dict(name="stress mixed 8000x8000, 200k hypotheses, 360deg/1440 beams",
            layout="mixed", size=8000, n_target=200000, min_spacing=0.3,
            scan=ScanSpec(360.0, 1440, 40.0, 0.02, 0.02, 0.0, 0.15),
            n_theta=1440, batch_k=256, tau=0.95, perturb=0.2),
}


def build_map(layout: str, size: int, rng: np.random.Generator) -> MapSpec:
    if layout == "rooms":
        return rooms_map(rng, size, size)
    if layout == "warehouse":
        return warehouse_map(rng, size, size)
    if layout == "tiled":
        return tiled_rooms_map(rng, size, size)
    if layout == "mixed":
        return mixed_map(rng, size, size)
    raise ValueError(layout)


def make_config(cid: int, n_target: Optional[int] = None,
                robot_radius: float = 0.21) -> Workload:
    c = CONFIGS[cid]
    spec = build_map(c["layout"], c["size"], _rng(cid, 0))
    occ = rasterize(spec)
    scan_occ = occ
    if c.get("perturb"):
        scan_occ = rasterize(perturb_map(spec, _rng(cid, 3), c["perturb"]))
    res, origin = spec.resolution, spec.origin
    mask = feasible_cells(occ, res, robot_radius)
    if scan_occ is not occ:
        mask &= feasible_cells(scan_occ, res, robot_radius, largest_component=False)
    pose = true_pose(occ, res, origin, _rng(cid, 1), robot_radius, mask=mask)
    sc: ScanSpec = c["scan"]
    ranges, amin, ainc, _ = lidar_scan(scan_occ, res, origin, pose, sc, _rng(cid, 2))
    return Workload(
        name=c["name"], occ=occ, resolution=res, origin=origin, pose=pose,
        ranges=ranges, angle_min=amin, angle_increment=ainc,
        range_min=sc.range_min, range_max=sc.range_max,
        sample=dict(n_target=n_target or c["n_target"],
                    min_spacing=c["min_spacing"], robot_radius=robot_radius,
                    seed=cid),
        search=dict(n_theta=c["n_theta"], batch_k=c["batch_k"], tau=c["tau"]),
        scan_occ=None if scan_occ is occ else scan_occ,
        meta=dict(config=cid, layout=c["layout"], size=c["size"]))


def make_micro(seed: int, width: int = 24, height: int = 20,
               n_boxes: int = 3, wall: int = 1, p_unknown: float = 0.0) -> np.ndarray:
    """A tiny random map: one-cell outer walls, a few boxes, optionally some
    unknown (-1) cells. Used by brute-force checks."""
    rng = np.random.default_rng([1000, seed])
    occ = np.zeros((height, width), dtype=np.int8)
    occ[:wall, :] = 100
    occ[-wall:, :] = 100
    occ[:, :wall] = 100
    occ[:, -wall:] = 100
    for _ in range(n_boxes):
        w = int(rng.integers(1, max(2, width // 5)))
        h = int(rng.integers(1, max(2, height // 5)))
        x0 = int(rng.integers(wall, width - wall - w))
        y0 = int(rng.integers(wall, height - wall - h))
        occ[y0:y0 + h, x0:x0 + w] = 100
    if p_unknown > 0:
        u = rng.random((height, width)) < p_unknown
        occ[u & (occ == 0)] = -1
    return occ
