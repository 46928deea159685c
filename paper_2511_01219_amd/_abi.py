"""ctypes mirror of include/reloc.h (structures, status codes, prototypes)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libreloc.so")

OK = 0
E_INVALID, E_NOMEM, E_NOTFOUND, E_BEAMGRID = -1, -2, -3, -4
E_EMPTY, E_BUSY, E_PENDING, E_TIMEOUT, E_DEVICE = -5, -6, -7, -8, -9
STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_NOTFOUND",
                -4: "E_BEAMGRID", -5: "E_EMPTY", -6: "E_BUSY", -7: "E_PENDING",
                -8: "E_TIMEOUT", -9: "E_DEVICE"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class reloc_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class reloc_map_desc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("resolution", C.c_double),
                ("origin_x", C.c_double), ("origin_y", C.c_double),
                ("occ_threshold", C.c_int32)]


class reloc_sample_params(C.Structure):
    _fields_ = [("n_target", C.c_int32), ("min_spacing", C.c_double),
                ("robot_radius", C.c_double), ("has_p0", C.c_int32), ("p0_x", C.c_double),
                ("p0_y", C.c_double), ("seed", C.c_uint64)]


class reloc_interval(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double)]


class reloc_scan(C.Structure):
    _fields_ = [("n_beams", C.c_int32), ("ranges", C.c_void_p), ("angle_min", C.c_double),
                ("angle_increment", C.c_double), ("n_fov", C.c_int32),
                ("fov", C.POINTER(reloc_interval)), ("range_min", C.c_float),
                ("range_max", C.c_float)]


class reloc_search_params(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("n_skip_beam", C.c_int32),
                ("n_skip_enum", C.c_int32), ("batch_k", C.c_int32), ("k_out", C.c_int32),
                ("tau", C.c_double), ("n_hyp", C.c_int32), ("z_hit", C.c_double),
                ("sigma_hit", C.c_double), ("z_rand", C.c_double), ("d_max", C.c_double),
                ("alpha_mid_pm", C.c_int32 * 2), ("alpha_low_pm", C.c_int32 * 2),
                ("deadline_s", C.c_double), ("variant", C.c_int32),
                ("refine_k", C.c_int32), ("refine_cells", C.c_int32),
                ("refine_dirs", C.c_int32), ("coarse_metric", C.c_int32),
                ("fine_metric", C.c_int32), ("use_graph", C.c_int32),
                ("ray_waves", C.c_int32), ("ray_refill", C.c_int32)]


class reloc_scan_info(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("Ns", "Ntheta", "Ng", "n_down", "n_fov", "n_valid",
                                          "k_full", "k_mid", "k_low", "panoramic", "n_runs",
                                          "n_shifts", "j0")] + \
               [("zbar", C.c_double), ("lambda_", C.c_double)]


class reloc_pose(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("theta", C.c_double),
                ("tam", C.c_float), ("smad", C.c_float), ("hyp", C.c_int32),
                ("k", C.c_int32), ("rank", C.c_int32), ("stage", C.c_int32),
                ("cx", C.c_int32), ("cy", C.c_int32), ("g", C.c_int32),
                ("refined", C.c_int32)]


class reloc_stats(C.Structure):
    _fields_ = [("smad_evals", C.c_int64), ("tam_evals", C.c_int64), ("rays", C.c_int64),
                ("tam_lookups", C.c_int64), ("n_hyp", C.c_int32), ("stages", C.c_int32),
                ("early_stopped", C.c_int32), ("n_eval", C.c_int32),
                ("ms_total", C.c_float), ("ms_raycast", C.c_float), ("ms_sort", C.c_float),
                ("ms_tam", C.c_float), ("ms_rank", C.c_float),
                ("ms_smad", C.c_float), ("refined", C.c_int64),
                ("refine_points", C.c_int64), ("best_margin", C.c_float),
                ("ambiguous", C.c_int32)]


class reloc_serve_config(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("hbm_reserve", C.c_size_t),
                ("max_admit", C.c_int32)]


class reloc_serve_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("ticks", C.c_int64), ("queued", C.c_int32), ("inflight", C.c_int32),
                ("busy_s", C.c_double), ("pollers", C.c_int32), ("reserved", C.c_int32)]


class reloc_rrt_params(C.Structure):
    _fields_ = [("p0_x", C.c_double), ("p0_y", C.c_double), ("rho", C.c_double),
                ("robot_radius", C.c_double), ("eta_max", C.c_double),
                ("eps_gain", C.c_int32), ("max_rounds", C.c_int32), ("max_nodes", C.c_int32),
                ("seed", C.c_uint64)]


class reloc_rrt_info(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("attempts", C.c_int64), ("nodes", C.c_int64),
                ("n_sampling", C.c_int64)]


class reloc_peaks(C.Structure):
    _fields_ = [("valu_i32_ops", C.c_double), ("l2_gathers", C.c_double),
                ("mall_gathers", C.c_double), ("hbm_read", C.c_double), ("hbm_copy", C.c_double),
                ("compute_units", C.c_int32), ("clock_khz", C.c_int32)]


# name -> (restype, argtypes)
PROTOS = {
    "reloc_version": (C.c_int32, []),
    "reloc_last_error": (C.c_char_p, []),
    "reloc_ctx_create": (C.c_int32, [C.c_int32, C.POINTER(reloc_allocator), C.c_void_p,
                                     C.c_size_t, C.POINTER(C.c_void_p)]),
    "reloc_ctx_destroy": (None, [C.c_void_p]),
    "reloc_ctx_bytes": (C.c_size_t, [C.c_void_p]),
    "reloc_load_map": (C.c_int32, [C.c_void_p, C.POINTER(reloc_map_desc), C.c_void_p,
                                   C.POINTER(C.c_int32)]),
    "reloc_unload_map": (C.c_int32, [C.c_void_p, C.c_int32]),
    "reloc_read_edt": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "reloc_sample_hypotheses": (C.c_int32, [C.c_void_p, C.c_int32,
                                            C.POINTER(reloc_sample_params),
                                            C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "reloc_set_hypotheses": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                         C.POINTER(C.c_int32)]),
    "reloc_read_hypotheses": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                          C.POINTER(C.c_int32)]),
    "reloc_free_hypotheses": (C.c_int32, [C.c_void_p, C.c_int32]),
    "reloc_rrt_defaults": (None, [C.POINTER(reloc_rrt_params)]),
    "reloc_sample_rrt": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(reloc_rrt_params),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(reloc_rrt_info), C.c_void_p, C.c_void_p,
                                     C.c_int32]),
    "reloc_search_defaults": (None, [C.POINTER(reloc_search_params)]),
    "reloc_scan_info_get": (C.c_int32, [C.POINTER(reloc_scan), C.POINTER(reloc_search_params),
                                        C.c_double, C.POINTER(reloc_scan_info)]),
    "reloc_prepare": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(reloc_scan),
                                  C.POINTER(reloc_search_params), C.POINTER(C.c_int32)]),
    "reloc_run": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(reloc_pose), C.c_int32,
                              C.POINTER(C.c_int32), C.POINTER(reloc_stats)]),
    "reloc_release": (C.c_int32, [C.c_void_p, C.c_int32]),
    "reloc_relocalize": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(reloc_scan),
                                     C.POINTER(reloc_search_params), C.POINTER(reloc_pose),
                                     C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(reloc_stats)]),
    "reloc_relocalize_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32,
                                             C.POINTER(reloc_scan),
                                             C.POINTER(reloc_search_params),
                                             C.POINTER(reloc_pose), C.c_int32,
                                             C.POINTER(C.c_int32), C.POINTER(reloc_stats)]),
    "reloc_run_batch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(reloc_pose),
                                    C.c_int32, C.c_void_p, C.c_void_p,
                                    C.POINTER(reloc_stats)]),
    "reloc_serve_configure": (C.c_int32, [C.c_void_p, C.POINTER(reloc_serve_config)]),
    "reloc_submit": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(reloc_scan),
                                 C.POINTER(reloc_search_params), C.POINTER(C.c_uint64)]),
    "reloc_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(reloc_pose),
                               C.c_int32, C.POINTER(C.c_int32), C.POINTER(reloc_stats)]),
    "reloc_serve_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(reloc_serve_stats)]),
    "reloc_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "reloc_coarse_scores": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(reloc_stats)]),
    "reloc_score_poses": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.c_void_p, C.POINTER(C.c_float)]),
    "reloc_measure_peaks": (C.c_int32, [C.c_int32, C.POINTER(reloc_peaks)]),
    "reloc_debug_raycast": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    "reloc_debug_smad": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "reloc_debug_tam": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
}

_lib = None


def load():
    """Loads the in-tree libreloc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (loaded by file name libamdhip64.so);
        # loading it first makes libreloc bind to that same runtime through
        # the shared soname instead of pulling in a second copy
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libreloc.so is not built; run "
                              "`python -m paper_2511_01219_amd.build` first")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
