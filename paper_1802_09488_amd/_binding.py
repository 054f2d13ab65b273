"""ctypes binding of libact.so (argument marshalling only).

Every step of the join runs in the HIP library; torch supplies device memory
(tensors) and streams. If the library is not built, importing this module
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libact.so")

ACT_OK, ACT_E_ARG, ACT_E_POLY, ACT_E_OOM, ACT_E_HIP, ACT_E_OVERFLOW, ACT_E_DEVICE, ACT_E_RANGE = \
    0, -1, -2, -3, -4, -5, -6, -7
ACT_EXACT, ACT_APPROX, ACT_AUTO = 0, 1, 2
ACT_REFINE_AUTO, ACT_REFINE_LOCAL, ACT_REFINE_FP32_FILTER, ACT_REFINE_FP64 = 0, 1, 2, 3
ACT_PENDING_AUTO, ACT_PENDING_KERNEL, ACT_PENDING_QUEUE = 0, 1, 2
ACT_GEOM_PLANE, ACT_GEOM_SPHERE = 0, 1
ACT_NCOUNTERS = 16
COUNTER_NAMES = ["points", "invalid", "false_hit", "solely_true", "cand_points", "candidates",
                 "edges", "edge_fp64", "edge_exact", "node_reads", "lut_reads"]

EXPORTS = ["act_build", "act_free", "act_join", "act_join_pairs", "act_join_ex", "act_cell_ids",
           "act_index_stats", "act_lookup_host", "act_lut_host", "act_encode_refs_host",
           "act_orient_fp32_host", "act_orient_exact_host", "act_last_error", "act_version"]


class ActError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("act error %d: %s" % (code, msg))
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("max_level", ctypes.c_int32), ("device", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("prefix_level", ctypes.c_int32),
                ("margin_deg", ctypes.c_double), ("train_points", ctypes.c_void_p),
                ("n_train", ctypes.c_int64), ("memory_budget", ctypes.c_int64),
                ("train_max_level", ctypes.c_int32), ("geometry", ctypes.c_int32),
                ("max_covering_cells", ctypes.c_int32), ("max_interior_cells", ctypes.c_int32),
                ("max_interior_level", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


class JoinArgs(ctypes.Structure):
    _fields_ = [("d_points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d_out", ctypes.c_void_p),
                ("d_pair_point", ctypes.c_void_p), ("d_pair_poly", ctypes.c_void_p),
                ("pair_capacity", ctypes.c_int64), ("d_n_pairs", ctypes.c_void_p),
                ("d_counters", ctypes.c_void_p), ("refine", ctypes.c_int32),
                ("block", ctypes.c_int32), ("lds_levels", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("pass_points", ctypes.c_int64),
                ("points_per_lane", ctypes.c_int32), ("pending", ctypes.c_int32),
                ("probe_event", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("lds_levels", ctypes.c_int32),
                ("points_per_lane", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("n_configs", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("pending", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("index_digest", ctypes.c_uint64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("max_request_points", ctypes.c_int64)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("admitted_s", ctypes.c_double),
                ("launched_s", ctypes.c_double), ("results_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("n", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("points", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("launches", ctypes.c_int64),
                ("max_pass_s", ctypes.c_double), ("max_launch_s", ctypes.c_double),
                ("max_stage_s", ctypes.c_double), ("max_finish_s", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_polys", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("n_cells_interior_only", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("node_bytes", ctypes.c_int64),
                ("lut_words", ctypes.c_int64), ("edge_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("max_depth", ctypes.c_int32),
                ("max_refs", ctypes.c_int32), ("max_cell_level", ctypes.c_int32),
                ("n_faces", ctypes.c_int32), ("face_prefix_level", ctypes.c_int32 * 6),
                ("mode", ctypes.c_int32), ("lds_nodes", ctypes.c_int32),
                ("precision_m", ctypes.c_double), ("build_seconds", ctypes.c_double),
                ("local_words", ctypes.c_int64), ("train_splits", ctypes.c_int64),
                ("train_points_used", ctypes.c_int64), ("image_bytes", ctypes.c_int64),
                ("margin_deg", ctypes.c_double), ("geometry", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["face_prefix_level"] = list(self.face_prefix_level)
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libact.so is not built (run __graft_entry__.build() or "
                          "python paper_1802_09488_amd/build_lib.py)")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "act_build": ([p, p, p, i32, i32, d, p, p], ctypes.c_int),
        "act_free": ([p], None),
        "act_save": ([p, ctypes.c_char_p], ctypes.c_int),
        "act_load": ([ctypes.c_char_p, i32, p], ctypes.c_int),
        "act_join": ([p, p, i64, p, p], ctypes.c_int),
        "act_join_pairs": ([p, p, i64, p, p, p, i64, p, p], ctypes.c_int),
        "act_join_noalloc": ([p, p, i64, p, p], ctypes.c_int),
        "act_join_count": ([p, p, i64, p, p], ctypes.c_int),
        "act_join_ids": ([p, p, p, i64, p, p], ctypes.c_int),
        "act_join_ex": ([p, p, p], ctypes.c_int),
        "act_workspace_reserve": ([p, p, i64], ctypes.c_int),
        "act_workspace_release": ([p, p], ctypes.c_int),
        "act_join_status": ([p, i64, p, p], ctypes.c_int),
        "act_cell_ids": ([p, i64, p, p], ctypes.c_int),
        "act_index_stats": ([p, p], ctypes.c_int),
        "act_lookup_host": ([p, p, p, p, i64, p], ctypes.c_int),
        "act_lut_host": ([p, p, p], ctypes.c_int),
        "act_abi_sizes": ([p], ctypes.c_int),
        "act_join_batched": ([p, p, i32, i64, p, p], ctypes.c_int),
        "act_batched_reserve": ([p, p, i32, i64], ctypes.c_int),
        "act_batched_status": ([p, p, p], ctypes.c_int),
        "act_wall_clock_hz": ([i32, p], ctypes.c_int),
        "act_tune": ([p, p, i64, p, p, ctypes.c_char_p, p], ctypes.c_int),
        "act_index_digest": ([p, p], ctypes.c_int),
        "act_server_opts_init": ([p], None),
        "act_server_create": ([p, i32, p, p], ctypes.c_int),
        "act_server_submit": ([p, i32, p, i64, p, d, p], ctypes.c_int),
        "act_server_wait": ([p, ctypes.c_uint64, p], ctypes.c_int),
        "act_server_replay": ([p, i64, p, p, p, p, i64, p], ctypes.c_int),
        "act_server_stats_get": ([p, p], ctypes.c_int),
        "act_server_clock": ([], d),
        "act_server_destroy": ([p], None),
        "act_server_last_error": ([], ctypes.c_char_p),
        "act_build_opts_init": ([p], None),
        "act_refine_local_host": ([p, i32, ctypes.c_uint32, ctypes.c_uint32, d, d, i32, p],
                                  ctypes.c_int),
        "act_encode_refs_host": ([p, i32, p, i64, p, p], ctypes.c_int),
        "act_orient_fp32_host": ([p, p, p, p, ctypes.c_float], ctypes.c_int),
        "act_orient_exact_host": ([p, p, p], ctypes.c_int),
        "act_orient_host_n": ([p, p, p, i64, i32, p], ctypes.c_int),
        "act_last_error": ([], ctypes.c_char_p),
        "act_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def check(rc: int):
    if rc != ACT_OK:
        raise ActError(rc, lib.act_last_error().decode())
    return rc
