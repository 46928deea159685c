"""Seeded synthetic LiDAR scans taken from a continuous true pose.

The sensor model here is a continuous FP64 grid traversal (Amanatides-Woo
style) from an arbitrary real-valued position and heading. It simulates the
physical sensor and is independent of the fixed-point ray cast that the
relocalization method performs on its position hypotheses.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np
from scipy import ndimage


@dataclass
class ScanSpec:
    fov_deg: float = 270.0
    n_beams: int = 360
    range_max: float = 12.0
    range_min: float = 0.02
    noise_sigma: float = 0.02
    drop_frac: float = 0.05          # beams replaced by NaN (missing return)
    clutter_frac: float = 0.0        # beams replaced by U[0.3, r_true]
    clutter_min: float = 0.3

    @property
    def angle_increment(self) -> float:
        return math.radians(self.fov_deg) / self.n_beams

    @property
    def angle_min(self) -> float:
        if self.fov_deg >= 360.0:
            return -math.pi
        return -math.radians(self.fov_deg) / 2.0


def feasible_cells(occ: np.ndarray, resolution: float, robot_radius: float,
                   largest_component: bool = True) -> np.ndarray:
    """Boolean mask of free cells whose centre is at least ``robot_radius``
    from every occupied cell centre (optionally restricted to the largest
    4-connected component). Used only to draw true poses."""
    free = (occ >= 0) & (occ < 65)
    dist = ndimage.distance_transform_edt(occ < 65) * resolution
    ok = free & (dist >= robot_radius)
    if largest_component and ok.any():
        lab, n = ndimage.label(ok)
        if n > 1:
            sizes = np.bincount(lab.ravel())
            sizes[0] = 0
            ok = lab == int(np.argmax(sizes))
    return ok


def true_pose(occ: np.ndarray, resolution: float, origin: Tuple[float, float],
              rng: np.random.Generator, robot_radius: float = 0.21,
              on_grid: bool = False, mask: Optional[np.ndarray] = None):
    """Uniform pose on the feasible space: a feasible cell, a uniform point in
    it (or its centre when ``on_grid``), a uniform heading in [-pi, pi)."""
    if mask is None:
        mask = feasible_cells(occ, resolution, robot_radius)
    ys, xs = np.nonzero(mask)
    if len(xs) == 0:
        raise ValueError("map has no feasible cell")
    k = int(rng.integers(0, len(xs)))
    if on_grid:
        fx, fy = 0.5, 0.5
    else:
        fx, fy = rng.random(), rng.random()
    x = origin[0] + (xs[k] + fx) * resolution
    y = origin[1] + (ys[k] + fy) * resolution
    th = float(rng.uniform(-math.pi, math.pi))
    return float(x), float(y), th


def trace_ranges(occ: np.ndarray, resolution: float,
                 origin: Tuple[float, float], x: float, y: float,
                 angles: np.ndarray, range_max: float) -> np.ndarray:
    """Exact continuous traversal: distance from (x, y) to the boundary of the
    first occupied cell along each world angle; NaN if none within
    ``range_max`` or the ray leaves the map."""
    H, W = occ.shape
    occupied = occ >= 65
    px = (x - origin[0]) / resolution
    py = (y - origin[1]) / resolution
    n = len(angles)
    dx, dy = np.cos(angles), np.sin(angles)
    cx = np.full(n, int(math.floor(px)), dtype=np.int64)
    cy = np.full(n, int(math.floor(py)), dtype=np.int64)
    sx = np.where(dx > 0, 1, -1).astype(np.int64)
    sy = np.where(dy > 0, 1, -1).astype(np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        tdx = np.where(dx != 0, 1.0 / np.abs(dx), np.inf)
        tdy = np.where(dy != 0, 1.0 / np.abs(dy), np.inf)
        bx = np.where(dx > 0, cx + 1 - px, px - cx)
        by = np.where(dy > 0, cy + 1 - py, py - cy)
        tmx = np.where(dx != 0, bx * tdx, np.inf)
        tmy = np.where(dy != 0, by * tdy, np.inf)
    out = np.full(n, np.nan)
    active = np.ones(n, dtype=bool)
    limit = range_max / resolution
    while active.any():
        stepx = active & (tmx < tmy)
        stepy = active & ~stepx
        t = np.where(stepx, tmx, tmy)
        cx = np.where(stepx, cx + sx, cx)
        cy = np.where(stepy, cy + sy, cy)
        tmx = np.where(stepx, tmx + tdx, tmx)
        tmy = np.where(stepy, tmy + tdy, tmy)
        over = active & (t > limit)
        active &= ~over
        out_map = active & ((cx < 0) | (cx >= W) | (cy < 0) | (cy >= H))
        active &= ~out_map
        idx = np.where(active)[0]
        hit = occupied[cy[idx], cx[idx]]
        hi = idx[hit]
        out[hi] = t[hi] * resolution
        active[hi] = False
    return out


def lidar_scan(occ: np.ndarray, resolution: float,
               origin: Tuple[float, float], pose, spec: ScanSpec,
               rng: np.random.Generator):
    """Returns ``(ranges float32[N], angle_min, angle_increment, r_true)``.

    Beam i points at ``angle_min + i * angle_increment`` in the robot frame.
    Missing returns and drop-outs are NaN; clutter beams (unmapped objects)
    return U[clutter_min, r_true]; every surviving range gets N(0, sigma).
    """
    x, y, th = pose
    n = spec.n_beams
    phis = spec.angle_min + np.arange(n) * spec.angle_increment
    r_true = trace_ranges(occ, resolution, origin, x, y, th + phis,
                          spec.range_max)
    r = r_true.copy()
    if spec.clutter_frac > 0:
        cand = np.nonzero(np.isfinite(r_true) & (r_true >= spec.clutter_min))[0]
        m = int(round(spec.clutter_frac * n))
        m = min(m, len(cand))
        if m:
            pick = rng.choice(cand, size=m, replace=False)
            r[pick] = rng.uniform(spec.clutter_min, r_true[pick])
    if spec.noise_sigma > 0:
        r = r + rng.normal(0.0, spec.noise_sigma, size=n)
    if spec.drop_frac > 0:
        m = int(round(spec.drop_frac * n))
        pick = rng.choice(n, size=m, replace=False)
        r[pick] = np.nan
    return (r.astype(np.float32), float(spec.angle_min),
            float(spec.angle_increment), r_true)
