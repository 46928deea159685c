"""Seeded synthetic occupancy maps built from axis-aligned rectangles.

A map is a list of rectangles in cell coordinates (half-open
``[x0, x1) x [y0, y1)``), rasterized to an ``int8`` grid of shape ``(H, W)``
with row 0 at the minimum y: 100 = occupied, 0 = free, -1 = unknown.
Every generator takes an explicit ``numpy.random.Generator`` so that the
same seed always yields the same map.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

Rect = Tuple[int, int, int, int, str]   # x0, y0, x1, y1, kind


@dataclass
class MapSpec:
    width: int
    height: int
    resolution: float = 0.05
    origin: Tuple[float, float] = (0.0, 0.0)
    rects: List[Rect] = field(default_factory=list)

    def clip(self) -> "MapSpec":
        out = []
        for x0, y0, x1, y1, kind in self.rects:
            x0, x1 = max(0, x0), min(self.width, x1)
            y0, y1 = max(0, y0), min(self.height, y1)
            if x1 > x0 and y1 > y0:
                out.append((x0, y0, x1, y1, kind))
        return replace(self, rects=out)


def rasterize(spec: MapSpec) -> np.ndarray:
    """Rectangles -> int8 occupancy grid (100 occupied, 0 free)."""
    occ = np.zeros((spec.height, spec.width), dtype=np.int8)
    for x0, y0, x1, y1, _ in spec.clip().rects:
        occ[y0:y1, x0:x1] = 100
    return occ


def _outer_walls(W: int, H: int, t: int) -> List[Rect]:
    return [(0, 0, W, t, "wall"), (0, H - t, W, H, "wall"),
            (0, 0, t, H, "wall"), (W - t, 0, W, H, "wall")]


def _wall_with_gap(lo: int, hi: int, fixed0: int, t: int, vertical: bool,
                   gap: int, rng: np.random.Generator,
                   margin: int = 5) -> Tuple[List[Rect], Tuple[int, int]]:
    """A wall segment spanning [lo, hi) along its axis with one doorway."""
    span = hi - lo
    if span < gap + 2 * margin:
        g0 = lo + max(0, (span - gap) // 2)
    else:
        g0 = int(rng.integers(lo + margin, hi - margin - gap + 1))
    g1 = g0 + gap
    rects = []
    for a, b in ((lo, g0), (g1, hi)):
        if b > a:
            if vertical:
                rects.append((fixed0, a, fixed0 + t, b, "wall"))
            else:
                rects.append((a, fixed0, b, fixed0 + t, "wall"))
    return rects, (g0, g1)


def _place_boxes(rng, n, W, H, blocked: np.ndarray, smin=4, smax=16,
                 clearance=2, tries=2000) -> List[Rect]:
    """Axis-aligned boxes with sides in [smin, smax] cells that do not touch
    ``blocked`` (walls, doorway zones, earlier boxes) within ``clearance``."""
    out: List[Rect] = []
    for _ in range(tries):
        if len(out) >= n:
            break
        w = int(rng.integers(smin, smax + 1))
        h = int(rng.integers(smin, smax + 1))
        x0 = int(rng.integers(0, W - w))
        y0 = int(rng.integers(0, H - h))
        a0, b0 = max(0, x0 - clearance), max(0, y0 - clearance)
        a1, b1 = min(W, x0 + w + clearance), min(H, y0 + h + clearance)
        if blocked[b0:b1, a0:a1].any():
            continue
        blocked[b0:b1, a0:a1] = True
        out.append((x0, y0, x0 + w, y0 + h, "box"))
    return out


def rooms_map(rng: np.random.Generator, width: int = 200, height: int = 200,
              resolution: float = 0.05, wall: int = 3, door: int = 20,
              n_boxes: int = 10) -> MapSpec:
    """Four rooms: outer walls, one vertical and one horizontal inner wall at
    seeded 40-60 % positions, four doorways, ``n_boxes`` boxes."""
    W, H, t = width, height, wall
    vx = int(rng.integers(int(0.4 * W), int(0.6 * W) + 1))
    hy = int(rng.integers(int(0.4 * H), int(0.6 * H) + 1))
    rects = _outer_walls(W, H, t)
    doors = []
    r, g = _wall_with_gap(t, hy, vx, t, True, door, rng); rects += r; doors.append(("v", g))
    r, g = _wall_with_gap(hy + t, H - t, vx, t, True, door, rng); rects += r; doors.append(("v", g))
    r, g = _wall_with_gap(t, vx, hy, t, False, door, rng); rects += r; doors.append(("h", g))
    r, g = _wall_with_gap(vx + t, W - t, hy, t, False, door, rng); rects += r; doors.append(("h", g))
    rects.append((vx, hy, vx + t, hy + t, "wall"))     # junction block
    blocked = np.zeros((H, W), dtype=bool)
    for x0, y0, x1, y1, _ in rects:
        blocked[y0:y1, x0:x1] = True
    # keep a corridor around every doorway clear so boxes never block it
    zone = 25
    for axis, (g0, g1) in doors:
        if axis == "v":
            blocked[max(0, g0 - 4):g1 + 4, max(0, vx - zone):vx + t + zone] = True
        else:
            blocked[max(0, hy - zone):hy + t + zone, max(0, g0 - 4):g1 + 4] = True
    rects += _place_boxes(rng, n_boxes, W, H, blocked)
    return MapSpec(W, H, resolution, (0.0, 0.0), rects)


def warehouse_map(rng: np.random.Generator, width: int = 2000,
                  height: int = 2000, resolution: float = 0.05,
                  wall: int = 3, rack: int = 20, aisle: int = 50,
                  margin: int = 80, cross: int = 60,
                  cross_every: Tuple[int, int] = (400, 600),
                  x_offset: int = 0, y_offset: int = 0,
                  outer: bool = True, jitter: int = 40) -> MapSpec:
    """Rack rows ``rack`` cells wide along x separated by ``aisle``-cell aisles,
    starting ``margin`` cells inside the outer walls; seeded ``cross``-cell
    cross-aisles every 20-30 m cut the racks into segments."""
    W, H = width, height
    rects: List[Rect] = _outer_walls(W, H, wall) if outer else []
    xs = []
    x = margin + int(rng.integers(cross_every[0] // 2, cross_every[1] // 2 + 1))
    while x + cross < W - margin:
        xs.append(x)
        x += cross + int(rng.integers(cross_every[0], cross_every[1] + 1))
    cuts = [margin] + [c for c0 in xs for c in (c0, c0 + cross)] + [W - margin]
    segs = [(cuts[i], cuts[i + 1]) for i in range(0, len(cuts), 2)]
    y = margin
    while y + rack <= H - margin:
        for a, b in segs:
            # seeded jitter of the segment ends makes every aisle distinct
            a2 = a + int(rng.integers(0, jitter + 1))
            b2 = b - int(rng.integers(0, jitter + 1))
            if b2 - a2 >= rack:
                rects.append((a2 + x_offset, y + y_offset, b2 + x_offset,
                              y + rack + y_offset, "rack"))
        y += rack + aisle
    return MapSpec(W, H, resolution, (0.0, 0.0), rects)


def tiled_rooms_map(rng: np.random.Generator, width: int, height: int,
                    resolution: float = 0.05, room: Tuple[int, int] = (100, 200),
                    wall: int = 3, door: int = 20, boxes_per_room: int = 2,
                    x_offset: int = 0, y_offset: int = 0,
                    outer: bool = True) -> MapSpec:
    """A grid of rooms 5-10 m on a side; every interior wall between two
    neighbouring rooms has one doorway; a few boxes per room."""
    W, H, t = width, height, wall
    rects: List[Rect] = _outer_walls(W, H, t) if outer else []

    def splits(n):
        out, p = [0], 0
        while True:
            step = int(rng.integers(room[0], room[1] + 1))
            if p + step >= n - room[0]:
                break
            p += step
            out.append(p)
        out.append(n - t)
        return out

    xs, ys = splits(W), splits(H)
    doors = []
    for i in range(1, len(xs) - 1):               # vertical walls
        for j in range(len(ys) - 1):
            r, g = _wall_with_gap(ys[j] + t, ys[j + 1], xs[i], t, True, door, rng)
            rects += r
            doors.append(("v", xs[i], g))
    for j in range(1, len(ys) - 1):               # horizontal walls
        for i in range(len(xs) - 1):
            r, g = _wall_with_gap(xs[i] + t, xs[i + 1], ys[j], t, False, door, rng)
            rects += r
            doors.append(("h", ys[j], g))
    for i in range(1, len(xs) - 1):               # junction posts
        for j in range(1, len(ys) - 1):
            rects.append((xs[i], ys[j], xs[i] + t, ys[j] + t, "wall"))
    blocked = np.zeros((H, W), dtype=bool)
    for x0, y0, x1, y1, _ in rects:
        blocked[y0:y1, x0:x1] = True
    zone = 20
    for axis, f, (g0, g1) in doors:
        if axis == "v":
            blocked[max(0, g0 - 4):g1 + 4, max(0, f - zone):f + t + zone] = True
        else:
            blocked[max(0, f - zone):f + t + zone, max(0, g0 - 4):g1 + 4] = True
    n_rooms = (len(xs) - 1) * (len(ys) - 1)
    rects += _place_boxes(rng, boxes_per_room * n_rooms, W, H, blocked,
                          tries=20 * boxes_per_room * n_rooms + 100)
    if x_offset or y_offset:
        rects = [(a + x_offset, b + y_offset, c + x_offset, d + y_offset, k)
                 for a, b, c, d, k in rects]
    return MapSpec(W, H, resolution, (0.0, 0.0), rects)


def mixed_map(rng: np.random.Generator, width: int = 8000, height: int = 8000,
              resolution: float = 0.05, wall: int = 3, door: int = 40) -> MapSpec:
    """Left half a warehouse, right half tiled rooms, joined by a wall with
    several wide doorways."""
    W, H, t = width, height, wall
    half = W // 2
    wh = warehouse_map(rng, half, H, resolution, outer=False)
    ro = tiled_rooms_map(rng, W - half, H, resolution, outer=False,
                         x_offset=half)
    rects = _outer_walls(W, H, t) + wh.rects + ro.rects
    # dividing wall with one doorway per 20 m
    n = max(1, H // 400)
    edges = np.linspace(t, H - t, n + 1).astype(int)
    for k in range(n):
        r, _ = _wall_with_gap(int(edges[k]), int(edges[k + 1]), half - t, t,
                              True, door, rng)
        rects += r
    return MapSpec(W, H, resolution, (0.0, 0.0), rects)


def perturb_map(spec: MapSpec, rng: np.random.Generator, frac: float = 0.2,
                max_shift_m: float = 1.0) -> MapSpec:
    """Environment change: ``frac`` of the non-wall obstacles are each either
    removed (p = 1/2) or moved by U[-max_shift, max_shift] per axis."""
    rects = list(spec.rects)
    movable = [i for i, r in enumerate(rects) if r[4] != "wall"]
    if not movable:
        return replace(spec, rects=rects)
    n = int(round(frac * len(movable)))
    pick = rng.choice(np.array(movable), size=n, replace=False)
    shift = int(round(max_shift_m / spec.resolution))
    drop = set()
    for i in pick:
        x0, y0, x1, y1, kind = rects[i]
        if rng.random() < 0.5:
            drop.add(int(i))
        else:
            dx = int(rng.integers(-shift, shift + 1))
            dy = int(rng.integers(-shift, shift + 1))
            rects[i] = (x0 + dx, y0 + dy, x1 + dx, y1 + dy, kind)
    rects = [r for i, r in enumerate(rects) if i not in drop]
    return replace(spec, rects=rects).clip()
