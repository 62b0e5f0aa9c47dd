"""ctypes wrapper of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import this
package.  The HIP library never does, and the oracle never loads the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "oracle.cpp")]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP contraction off, so expressions evaluate as written)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", *SOURCES, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [P]
        L.orc_destroy.argtypes = [P]
        L.orc_integrate_depth.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, P]
        L.orc_integrate_points.argtypes = [P, P, ctypes.c_int64, P]
        L.orc_last_stats.argtypes = [P, P]
        L.orc_num_blocks.restype = ctypes.c_int64
        L.orc_num_blocks.argtypes = [P]
        L.orc_num_voxels.restype = ctypes.c_int64
        L.orc_num_voxels.argtypes = [P]
        L.orc_extract.argtypes = [P, P, P, P, P, P, P]
        L.orc_near_threshold.restype = ctypes.c_int64
        L.orc_near_threshold.argtypes = [P, P, P, P, ctypes.c_int64]
        L.orc_query.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, P, P]
        L.orc_query_backward.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P, P, P]
        L.orc_eq4_hash.restype = ctypes.c_uint32
        L.orc_eq4_hash.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
        L.orc_block_dda.restype = ctypes.c_int64
        L.orc_block_dda.argtypes = [P, P, ctypes.c_double, P, ctypes.c_int64]
        L.orc_voxel_dda.restype = ctypes.c_int64
        L.orc_voxel_dda.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P,
                                    ctypes.c_int64]
        L.orc_mesh.restype = ctypes.c_int64
        L.orc_mesh.argtypes = [P, ctypes.c_double, P, ctypes.c_int64, P, P, P, P, ctypes.c_int64]
        L.orc_set_block.restype = ctypes.c_int
        L.orc_set_block.argtypes = [P, P, ctypes.c_int32, P, P]
        L.orc_region_holds.restype = ctypes.c_int
        L.orc_region_holds.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_double, P, P]
        L.orc_quadtree.restype = ctypes.c_int64
        L.orc_quadtree.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P,
                                   ctypes.c_int64, P]
        L.orc_integrate_rgbd.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P, P]
        L.orc_extract_color.argtypes = [P, P]
        _lib = L
    return _lib


class _Config(ctypes.Structure):
    _fields_ = [("voxel", ctypes.c_double), ("levels", ctypes.c_int32), ("min_obs", ctypes.c_int32),
                ("tau", ctypes.c_double), ("var_thr", ctypes.c_double), ("max_depth", ctypes.c_double),
                ("min_range", ctypes.c_double), ("max_range", ctypes.c_double),
                ("carve", ctypes.c_int32), ("form", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("valid_points", ctypes.c_int64), ("new_blocks", ctypes.c_int64),
                ("observations", ctypes.c_int64), ("dropped_points", ctypes.c_int64),
                ("merges", ctypes.c_int64 * 4), ("near_threshold", ctypes.c_int64),
                ("distinct_voxels", ctypes.c_int64), ("candidate_keys", ctypes.c_int64),
                ("touched_blocks", ctypes.c_int64)]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Extracted:
    keys: np.ndarray  # int32[n, 3], ascending (x, y, z)
    levels: np.ndarray  # uint8[n]
    offsets: np.ndarray  # int64[n + 1]
    D: np.ndarray  # float64[v]
    W: np.ndarray  # uint32[v]
    S2: np.ndarray  # float64[v]


class OracleMap:
    """One fused map held by the oracle."""

    def __init__(self, voxel, levels=1, tau=None, var_thr=0.0, min_obs=2, max_depth=1e9,
                 min_range=0.0, max_range=1e9, carve=0, form="range"):
        self._cfg = _Config(float(voxel), int(levels), int(min_obs),
                            float(tau if tau is not None else 3.0 * voxel), float(var_thr),
                            float(max_depth), float(min_range), float(max_range), int(carve),
                            0 if form == "range" else 1)
        self._h = lib().orc_create(ctypes.byref(self._cfg))
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def integrate_depth(self, depth: np.ndarray, K, T) -> dict:
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        K = np.ascontiguousarray(K, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        lib().orc_integrate_depth(self._h, _p(depth), depth.shape[1], depth.shape[0], _p(K), _p(T))
        return self.last_stats()

    def integrate_rgbd(self, depth: np.ndarray, rgb: np.ndarray, K, T) -> dict:
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        assert rgb.shape == depth.shape + (3,)
        K = np.ascontiguousarray(K, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        lib().orc_integrate_rgbd(self._h, _p(depth), _p(rgb), depth.shape[1], depth.shape[0], _p(K), _p(T))
        return self.last_stats()

    def extract_color(self) -> np.ndarray:
        """float64 [voxels, 3] colours in the voxel order of extract()."""
        out = np.zeros((int(lib().orc_num_voxels(self._h)), 3), np.float64)
        lib().orc_extract_color(self._h, _p(out))
        return out

    def integrate_points(self, xyz: np.ndarray, T) -> dict:
        xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        lib().orc_integrate_points(self._h, _p(xyz), xyz.shape[0], _p(T))
        return self.last_stats()

    def last_stats(self) -> dict:
        s = _Stats()
        lib().orc_last_stats(self._h, ctypes.byref(s))
        return {"valid_points": s.valid_points, "new_blocks": s.new_blocks,
                "observations": s.observations, "dropped_points": s.dropped_points,
                "merges": list(s.merges), "near_threshold": s.near_threshold,
                "distinct_voxels": s.distinct_voxels, "candidate_keys": s.candidate_keys,
                "touched_blocks": s.touched_blocks}

    @property
    def num_blocks(self) -> int:
        return int(lib().orc_num_blocks(self._h))

    def extract(self) -> Extracted:
        n = self.num_blocks
        nv = int(lib().orc_num_voxels(self._h))
        keys = np.zeros((n, 3), np.int32)
        levels = np.zeros(n, np.uint8)
        offs = np.zeros(n + 1, np.int64)
        D = np.zeros(nv, np.float64)
        W = np.zeros(nv, np.uint32)
        S2 = np.zeros(nv, np.float64)
        lib().orc_extract(self._h, _p(keys), _p(levels), _p(offs), _p(D), _p(W), _p(S2))
        return Extracted(keys, levels, offs, D, W, S2)

    def near_threshold(self):
        n = int(lib().orc_near_threshold(self._h, None, None, None, 0))
        keys = np.zeros((n, 3), np.int32)
        frames = np.zeros(n, np.int64)
        margins = np.zeros(n, np.float64)
        if n:
            lib().orc_near_threshold(self._h, _p(keys), _p(frames), _p(margins), n)
        return keys, frames, margins

    def query(self, pts: np.ndarray, T=None, strict=False):
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        n = pts.shape[0]
        sdf = np.zeros(n, np.float64)
        valid = np.zeros(n, np.uint8)
        grad = np.zeros((n, 3), np.float64)
        Tp = None if T is None else np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        lib().orc_query(self._h, _p(pts), n, None if Tp is None else _p(Tp), int(strict), _p(sdf),
                        _p(valid), _p(grad))
        return sdf, valid.astype(bool), grad

    def mesh(self, collapse: float = 0.0, only_keys=None) -> Mesh:
        """Multi-resolution Marching Cubes (Sec. 3.4) of the whole map or of the listed blocks."""
        return _mesh(self._h, collapse, only_keys)

    def region_holds(self, keys, kind: str, T, K=None, width=0, height=0, radius=0.0):
        """Streaming region test per block key (Sec. 3.3): (inside bool [n], margin float64 [n] in
        metres).  kind "depth" (camera frustum; K, width, height) or "points" (ball of radius)."""
        keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3)
        Kp = np.ascontiguousarray(K if K is not None else np.ones(4), dtype=np.float64)
        Tp = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        inside = np.zeros(len(keys), bool)
        margin = np.zeros(len(keys), np.float64)
        mg = ctypes.c_double()
        kd = 1 if kind == "depth" else 2
        for i, k in enumerate(keys):
            kk = np.ascontiguousarray(k)
            inside[i] = bool(lib().orc_region_holds(self._h, kd, int(width), int(height), _p(Kp), _p(Tp), float(radius),
                                                    _p(kk), ctypes.byref(mg)))
            margin[i] = mg.value
        return inside, margin

    def set_block(self, key, level: int, D: np.ndarray, W: np.ndarray):
        """Test hook: put a level-`level` block with the given voxels (x fastest) at `key`."""
        k = np.ascontiguousarray(key, dtype=np.int32).reshape(3)
        D = np.ascontiguousarray(D, dtype=np.float64).ravel()
        W = np.ascontiguousarray(W, dtype=np.uint32).ravel()
        m = 8 >> int(level)
        if D.size != m ** 3 or W.size != m ** 3:
            raise ValueError("block arrays must hold (8 >> level)^3 voxels")
        if lib().orc_set_block(self._h, _p(k), int(level), _p(D), _p(W)) != 0:
            raise ValueError("level outside the map's levels")

    def query_backward(self, pts: np.ndarray, grad_sdf: np.ndarray, T=None, strict=False):
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, 3)
        n = pts.shape[0]
        g = np.ascontiguousarray(grad_sdf, dtype=np.float64).reshape(n)
        gp = np.zeros((n, 3), np.float64)
        gpose = np.zeros(6, np.float64)
        Tp = None if T is None else np.ascontiguousarray(T, dtype=np.float64).reshape(16)
        lib().orc_query_backward(self._h, _p(pts), n, None if Tp is None else _p(Tp), int(strict),
                                 _p(g), _p(gp), _p(gpose))
        return gp, gpose


@dataclass
class Mesh:
    verts: np.ndarray   # float64[t, 3, 3] world metres, counter-clockwise seen from outside
    blocks: np.ndarray  # int32[t, 3] block key of the triangle's cube
    codes: np.ndarray   # uint32[t] level << 30 | voxel << 15 | v0 << 10 | v1 << 5 | v2
    near: np.ndarray    # bool[t] a decision of the cube lay within rounding of its threshold


def _mesh(h, collapse: float, only_keys=None) -> Mesh:
    ok = None if only_keys is None else np.ascontiguousarray(only_keys, dtype=np.int32).reshape(-1, 3)
    okp = None if ok is None else _p(ok)
    nok = 0 if ok is None else ok.shape[0]
    n = int(lib().orc_mesh(h, float(collapse), okp, nok, None, None, None, None, 0))
    verts = np.zeros((n, 3, 3), np.float64)
    blocks = np.zeros((n, 3), np.int32)
    codes = np.zeros(n, np.uint32)
    near = np.zeros(n, np.uint8)
    if n:
        lib().orc_mesh(h, float(collapse), okp, nok, _p(verts), _p(blocks), _p(codes), _p(near), n)
    return Mesh(verts, blocks, codes, near.astype(bool))


def quadtree(rgb: np.ndarray, threshold: float, min_size: int):
    """Quadtree leaves of an 8-bit RGB image [h, w, 3] (Eq. 10, Algorithm 1): (leaves int32 [n, 4]
    as x0, y0, w, h in breadth-first order, contrast float64 [n], near-threshold decisions)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    h, w = rgb.shape[:2]
    near = ctypes.c_int64()
    n = int(lib().orc_quadtree(_p(rgb), w, h, float(threshold), int(min_size), None, None, 0, ctypes.byref(near)))
    leaves = np.zeros((n, 4), np.int32)
    con = np.zeros(n, np.float64)
    lib().orc_quadtree(_p(rgb), w, h, float(threshold), int(min_size), _p(leaves), _p(con), n, ctypes.byref(near))
    return leaves, con, int(near.value)


def eq4_hash(x: int, y: int, z: int, n_hash: int) -> int:
    return int(lib().orc_eq4_hash(x, y, z, n_hash))


def block_dda(a, e, inv_cell, cap=100000) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    out = np.zeros((cap, 3), np.int64)
    n = int(lib().orc_block_dda(_p(a), _p(e), float(inv_cell), _p(out), cap))
    return out[:min(n, cap)]


def voxel_dda(a, e, block, block_edge, inv_voxel, m, cap=1000) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    b = np.ascontiguousarray(block, dtype=np.int32)
    out = np.zeros((cap, 3), np.int32)
    n = int(lib().orc_voxel_dda(_p(a), _p(e), _p(b), float(block_edge), float(inv_voxel), int(m),
                                _p(out), cap))
    return out[:min(n, cap)]
