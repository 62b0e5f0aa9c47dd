"""ctypes declarations of the C ABI in ``include/mrhash.h`` (argument marshalling only).

The shared library is loaded from this package directory.  There is no fallback: when
``libmrhash.so`` is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrhash.so")

MRH_OK = 0
ERRORS = {
    -1: "MRH_ERR_INVALID_ARG",
    -2: "MRH_ERR_OOM",
    -3: "MRH_ERR_TABLE_FULL",
    -4: "MRH_ERR_HEAP_FULL",
    -5: "MRH_ERR_BUFFER_TOO_SMALL",
    -6: "MRH_ERR_HIP",
    -7: "MRH_ERR_BLOCK_LIMIT",
}
FORM = {"range": 0, "zdiff": 1}
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}

EXPORTS = [
    "mrh_abi_version", "mrh_block_hash", "mrh_map_create", "mrh_map_destroy", "mrh_map_reset",
    "mrh_integrate_depth", "mrh_integrate_points", "mrh_sync", "mrh_query_sdf",
    "mrh_query_sdf_backward", "mrh_extract_blocks", "mrh_last_error", "mrh_profile_enable",
    "mrh_profile_collect", "mrh_batch_create", "mrh_batch_destroy", "mrh_batch_integrate", "mrh_batch_set_launch",
    "mrh_batch_get_launch", "mrh_batch_autotune", "mrh_integrate_depth_sequence", "mrh_integrate_points_sequence",
    "mrh_integrate_depth_noalloc", "mrh_extract_mesh", "mrh_heap_usage", "mrh_stream_out", "mrh_stream_in",
    "mrh_store_info", "mrh_store_extract", "mrh_load_blocks", "mrh_quadtree_create", "mrh_quadtree_destroy",
    "mrh_quadtree_build", "mrh_integrate_rgbd", "mrh_extract_color", "mrh_map_check",
    "mrh_codec_device", "mrh_codec_host",
]
KERNELS = ["reset", "alloc_depth", "integrate_depth", "finalize", "alloc_points", "rays", "apply_points",
           "query", "query_backward", "reduce", "batch_alloc", "batch_rays", "batch_update", "batch_finalize",
           "batch_step", "mesh", "color"]
FRAME_NONE, FRAME_DEPTH, FRAME_POINTS = 0, 1, 2


class MrhRegion(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("K", ctypes.c_double * 4), ("T_ws", ctypes.c_double * 16), ("radius", ctypes.c_double)]


class MrhConfig(ctypes.Structure):
    _fields_ = [
        ("voxel", ctypes.c_double), ("levels", ctypes.c_int32), ("min_obs", ctypes.c_int32),
        ("tau", ctypes.c_double), ("var_thr", ctypes.c_double), ("max_depth", ctypes.c_double),
        ("min_range", ctypes.c_double), ("max_range", ctypes.c_double), ("carve", ctypes.c_int32),
        ("form", ctypes.c_int32), ("hash_slots", ctypes.c_int64), ("max_blocks", ctypes.c_int64),
        ("heap_blocks", ctypes.c_int64 * 4), ("storage", ctypes.c_int32), ("max_probe", ctypes.c_int32),
        ("color", ctypes.c_int32),
    ]


class MrhStats(ctypes.Structure):
    _fields_ = [
        ("frames", ctypes.c_int64), ("valid_points", ctypes.c_int64), ("dropped_points", ctypes.c_int64),
        ("new_blocks", ctypes.c_int64), ("observations", ctypes.c_int64), ("merges", ctypes.c_int64 * 4),
        ("failed_inserts", ctypes.c_int64), ("fresh_observations", ctypes.c_int64),
        ("blocks", ctypes.c_int64), ("error_flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("distinct_voxels", ctypes.c_int64), ("candidate_keys", ctypes.c_int64), ("queued_blocks", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {"frames": self.frames, "valid_points": self.valid_points,
                "dropped_points": self.dropped_points, "new_blocks": self.new_blocks,
                "observations": self.observations, "merges": list(self.merges),
                "failed_inserts": self.failed_inserts, "fresh_observations": self.fresh_observations,
                "blocks": self.blocks, "distinct_voxels": self.distinct_voxels,
                "candidate_keys": self.candidate_keys, "queued_blocks": self.queued_blocks,
                "error_flags": self.error_flags}


class MrhCheck(ctypes.Structure):
    _fields_ = [
        ("blocks", ctypes.c_int64), ("live_blocks", ctypes.c_int64), ("slotless_blocks", ctypes.c_int64),
        ("gone_blocks", ctypes.c_int64), ("table_keys", ctypes.c_int64), ("tombstones", ctypes.c_int64),
        ("idless_keys", ctypes.c_int64), ("free_slots", ctypes.c_int64 * 4), ("pending_slots", ctypes.c_int64 * 4),
        ("mean_probe", ctypes.c_double), ("max_probe", ctypes.c_int32), ("consistent", ctypes.c_int32),
        ("duplicate_keys", ctypes.c_int64), ("unreachable_keys", ctypes.c_int64),
        ("bad_table_entries", ctypes.c_int64), ("slot_conflicts", ctypes.c_int64), ("lost_slots", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name.endswith("_slots") and not isinstance(v, int) else v
        out["consistent"] = bool(self.consistent)
        return out


class MrhFrame(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("data_dev", ctypes.c_void_p), ("n", ctypes.c_int64), ("K", ctypes.c_double * 4),
                ("T_ws", ctypes.c_double * 16)]


class MrhError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)}" + (f" ({detail})" if detail else ""))


_lib = None


def load():
    """Load libmrhash.so (built by ``paper_2511_21459_amd.build``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first "
                          "(the HIP library is required, there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.mrh_abi_version.restype = i32
    L.mrh_abi_version.argtypes = []
    L.mrh_block_hash.restype = ctypes.c_uint32
    L.mrh_block_hash.argtypes = [i32, i32, i32, ctypes.c_uint64]
    L.mrh_map_create.restype = i32
    L.mrh_map_create.argtypes = [ctypes.POINTER(MrhConfig), P, ctypes.POINTER(P)]
    L.mrh_map_destroy.restype = None
    L.mrh_map_destroy.argtypes = [P]
    L.mrh_map_reset.restype = i32
    L.mrh_map_reset.argtypes = [P]
    L.mrh_integrate_depth.restype = i32
    L.mrh_integrate_depth.argtypes = [P, P, i32, i32, P, P]
    L.mrh_integrate_rgbd.restype = i32
    L.mrh_integrate_rgbd.argtypes = [P, P, P, i32, i32, P, P]
    L.mrh_extract_color.restype = i32
    L.mrh_extract_color.argtypes = [P, P, i64, ctypes.POINTER(i64)]
    L.mrh_quadtree_create.restype = i32
    L.mrh_quadtree_create.argtypes = [i32, i32, P, ctypes.POINTER(P)]
    L.mrh_quadtree_destroy.restype = None
    L.mrh_quadtree_destroy.argtypes = [P]
    L.mrh_quadtree_build.restype = i32
    L.mrh_quadtree_build.argtypes = [P, P, i32, i32, ctypes.c_double, i32, P, P, i64, ctypes.POINTER(i64)]
    for fn in (L.mrh_codec_device, L.mrh_codec_host):
        fn.restype = i32
        fn.argtypes = [i32, i32, P, P, ctypes.c_int64]
    L.mrh_map_check.restype = i32
    L.mrh_map_check.argtypes = [P, ctypes.POINTER(MrhCheck)]
    L.mrh_heap_usage.restype = i32
    L.mrh_heap_usage.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.mrh_stream_out.restype = i32
    L.mrh_stream_out.argtypes = [P, ctypes.POINTER(MrhRegion), ctypes.c_double, ctypes.POINTER(i64)]
    L.mrh_stream_in.restype = i32
    L.mrh_stream_in.argtypes = [P, ctypes.POINTER(MrhRegion), ctypes.POINTER(i64)]
    L.mrh_store_info.restype = i32
    L.mrh_store_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.mrh_store_extract.restype = i32
    L.mrh_store_extract.argtypes = [P, P, P, P, P, P, P, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.mrh_load_blocks.restype = i32
    L.mrh_load_blocks.argtypes = [P, i64, P, P, P, P, P, ctypes.POINTER(i64)]
    L.mrh_extract_mesh.restype = i32
    L.mrh_extract_mesh.argtypes = [P, ctypes.c_double, P, P, P, i64, ctypes.POINTER(i64)]
    L.mrh_integrate_depth_noalloc.restype = i32
    L.mrh_integrate_depth_noalloc.argtypes = [P, P, i32, i32, P, P]
    L.mrh_integrate_points.restype = i32
    L.mrh_integrate_points.argtypes = [P, P, i64, P]
    L.mrh_integrate_depth_sequence.restype = i32
    L.mrh_integrate_depth_sequence.argtypes = [P, P, i32, i32, i32, P, P]
    L.mrh_integrate_points_sequence.restype = i32
    L.mrh_integrate_points_sequence.argtypes = [P, P, i32, i64, P]
    L.mrh_sync.restype = i32
    L.mrh_sync.argtypes = [P, ctypes.POINTER(MrhStats), ctypes.POINTER(MrhStats)]
    L.mrh_query_sdf.restype = i32
    L.mrh_query_sdf.argtypes = [P, P, i64, P, i32, P, P, P]
    L.mrh_query_sdf_backward.restype = i32
    L.mrh_query_sdf_backward.argtypes = [P, P, i64, P, i32, P, P, P]
    L.mrh_extract_blocks.restype = i32
    L.mrh_extract_blocks.argtypes = [P, P, P, P, P, P, P, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.mrh_profile_enable.restype = i32
    L.mrh_profile_enable.argtypes = [P, i32]
    L.mrh_profile_collect.restype = i32
    L.mrh_profile_collect.argtypes = [P, P, P, i32]
    L.mrh_batch_create.restype = i32
    L.mrh_batch_create.argtypes = [P, i32, ctypes.POINTER(P)]
    L.mrh_batch_destroy.restype = None
    L.mrh_batch_destroy.argtypes = [P]
    L.mrh_batch_integrate.restype = i32
    L.mrh_batch_integrate.argtypes = [P, P]
    L.mrh_batch_set_launch.restype = i32
    L.mrh_batch_set_launch.argtypes = [P, P]
    L.mrh_batch_get_launch.restype = i32
    L.mrh_batch_get_launch.argtypes = [P, P]
    L.mrh_batch_autotune.restype = i32
    L.mrh_batch_autotune.argtypes = [P, P, i32, P]
    L.mrh_last_error.restype = ctypes.c_char_p
    L.mrh_last_error.argtypes = [P]
    _ = dbl
    _lib = L
    return L
