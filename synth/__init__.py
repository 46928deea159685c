"""Seeded synthetic inputs: occupancy maps, true poses and LiDAR scans.

This package holds input generation only. It contains none of the
relocalization method's arithmetic (no ray casting on the hypothesis grid,
no SMAD, no TAM, no sampling of hypotheses); both the HIP library and the
CPU oracle consume what it produces.
"""
from .maps import (MapSpec, rooms_map, warehouse_map, tiled_rooms_map,
                   mixed_map, perturb_map, rasterize)
from .scans import ScanSpec, true_pose, lidar_scan, feasible_cells
from .configs import CONFIGS, make_config, make_micro
from .multi import MultiWorkload, Query, make_batched, make_serving

__all__ = [
    "MapSpec", "rooms_map", "warehouse_map", "tiled_rooms_map", "mixed_map",
    "perturb_map", "rasterize", "ScanSpec", "true_pose", "lidar_scan",
    "feasible_cells", "CONFIGS", "make_config", "make_micro",
    "MultiWorkload", "Query", "make_batched", "make_serving",
]
