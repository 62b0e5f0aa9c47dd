"""MI355X-native fusion of depth frames and LiDAR scans into a spatially hashed, variance-adaptive
multi-resolution TSDF voxel-block map (MrHash, arXiv 2511.21459).

Thin Python binding over the C ABI of ``libmrhash.so`` (``include/mrhash.h``): every step of
allocation, integration, merging, querying and extraction runs in the library's HIP kernels; this
module only marshals torch tensors (device memory) and host arrays into the calls.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import FORM, STORAGE, MrhConfig, MrhError, MrhStats

__all__ = ["Map", "Batch", "SdfQuery", "block_hash", "MrhError"]


def _host_doubles(a, n):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n))
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _dev(t: torch.Tensor, dtype, shape_tail=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape (N, {', '.join(map(str, shape_tail))})")
    return ctypes.c_void_p(t.data_ptr())


def block_hash(x: int, y: int, z: int, n_hash: int) -> int:
    """Home slot of block (x, y, z) in a table of n_hash slots (Eq. 4)."""
    return int(_lib.load().mrh_block_hash(x, y, z, n_hash))


class Map:
    """One fused map living on the current GPU, bound to torch's current stream at creation."""

    def __init__(self, voxel: float, levels: int = 1, tau: float | None = None, var_thr: float = 0.0,
                 min_obs: int = 2, max_depth: float = 1e9, min_range: float = 0.0,
                 max_range: float = 1e9, carve: bool = False, form: str = "range",
                 max_blocks: int = 1 << 18, hash_slots: int | None = None, heap_blocks=None,
                 storage: str = "f32", max_probe: int = 0, color: bool = False):
        L = _lib.load()
        cfg = MrhConfig()
        cfg.voxel = float(voxel)
        cfg.levels = int(levels)
        cfg.min_obs = int(min_obs)
        cfg.tau = float(tau if tau is not None else 3.0 * voxel)
        cfg.var_thr = float(var_thr)
        cfg.max_depth = float(max_depth)
        cfg.min_range = float(min_range)
        cfg.max_range = float(max_range)
        cfg.carve = int(bool(carve))
        cfg.form = FORM[form]
        cfg.max_blocks = int(max_blocks)
        hs = hash_slots if hash_slots is not None else 1 << max(1, (2 * int(max_blocks) - 1).bit_length())
        cfg.hash_slots = int(hs)
        hb = list(heap_blocks) if heap_blocks is not None else [0, 0, 0, 0]
        for n in range(4):
            cfg.heap_blocks[n] = int(hb[n]) if n < len(hb) else 0
        cfg.storage = STORAGE[storage]
        cfg.max_probe = int(max_probe)
        cfg.color = int(bool(color))
        self.cfg = cfg
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = L.mrh_map_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise MrhError(st, "mrh_map_create")
        self._h = h

    # -- lifetime -------------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mrh_map_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            raise MrhError(st, what, _lib.load().mrh_last_error(self._h).decode())

    def reset(self):
        self._check(_lib.load().mrh_map_reset(self._h), "mrh_map_reset")

    # -- fusion ---------------------------------------------------------------------------------
    def integrate_depth(self, depth: torch.Tensor, K, T_ws):
        """Fuse one z-depth frame (float32 [H, W] metres on the GPU) seen with intrinsics
        K = (fx, fy, cx, cy) from world-from-sensor pose T_ws (4 x 4)."""
        if depth.dim() != 2:
            raise ValueError("depth must be [H, W]")
        p = _dev(depth, torch.float32, name="depth")
        Ka, Kp = _host_doubles(K, 4)
        Ta, Tp = _host_doubles(T_ws, 16)
        self._check(_lib.load().mrh_integrate_depth(self._h, p, depth.shape[1], depth.shape[0], Kp, Tp),
                    "mrh_integrate_depth")

    def integrate_rgbd(self, depth: torch.Tensor, rgb: torch.Tensor, K, T_ws):
        """Fuse one RGB-D frame with colour (a map created with color=True): depth float32 [H, W]
        and rgb uint8 [H, W, 3] on the GPU."""
        if depth.dim() != 2 or tuple(rgb.shape) != tuple(depth.shape) + (3,):
            raise ValueError("depth must be [H, W] and rgb [H, W, 3]")
        p = _dev(depth, torch.float32, name="depth")
        c = _dev(rgb, torch.uint8, name="rgb")
        Ka, Kp = _host_doubles(K, 4)
        Ta, Tp = _host_doubles(T_ws, 16)
        self._check(_lib.load().mrh_integrate_rgbd(self._h, p, c, depth.shape[1], depth.shape[0], Kp, Tp),
                    "mrh_integrate_rgbd")

    def extract_color(self) -> torch.Tensor:
        """float32 [voxels, 3] colours in the voxel order of extract()."""
        n = ctypes.c_int64()
        L = _lib.load()
        self._check(L.mrh_extract_color(self._h, None, 0, ctypes.byref(n)), "mrh_extract_color")
        out = torch.empty((n.value, 3), dtype=torch.float32, device=torch.device("cuda", torch.cuda.current_device()))
        self._check(L.mrh_extract_color(self._h, ctypes.c_void_p(out.data_ptr()), n.value, ctypes.byref(n)),
                    "mrh_extract_color")
        return out

    def integrate_depth_noalloc(self, depth: torch.Tensor, K, T_ws):
        """integrate_depth through the entry point that allocates no device memory (the per-tile
        depth summary sits in the library's fixed per-GPU array; frames of at most 65536 16 x 16
        tiles; calls overlapping on one GPU race)."""
        if depth.dim() != 2:
            raise ValueError("depth must be [H, W]")
        p = _dev(depth, torch.float32, name="depth")
        Ka, Kp = _host_doubles(K, 4)
        Ta, Tp = _host_doubles(T_ws, 16)
        self._check(_lib.load().mrh_integrate_depth_noalloc(self._h, p, depth.shape[1], depth.shape[0], Kp, Tp),
                    "mrh_integrate_depth_noalloc")

    def integrate_points(self, xyz: torch.Tensor, T_ws):
        """Fuse one LiDAR scan: float32 [N, 3] sensor-frame points on the GPU."""
        p = _dev(xyz, torch.float32, (3,), name="xyz")
        Ta, Tp = _host_doubles(T_ws, 16)
        self._check(_lib.load().mrh_integrate_points(self._h, p, xyz.shape[0], Tp), "mrh_integrate_points")

    def integrate_depth_sequence(self, depths: torch.Tensor, K, poses):
        """Fuse frames depths[0..F-1] (float32 [F, H, W] on the GPU) with poses [F, 4, 4] in order;
        the frame loop runs inside the library."""
        if depths.dim() != 3:
            raise ValueError("depths must be [F, H, W]")
        p = _dev(depths, torch.float32, name="depths")
        Ka, Kp = _host_doubles(K, 4)
        Pa, Pp = _host_doubles(poses, 16 * depths.shape[0])
        self._check(_lib.load().mrh_integrate_depth_sequence(self._h, p, depths.shape[0], depths.shape[2],
                                                             depths.shape[1], Kp, Pp), "mrh_integrate_depth_sequence")

    def integrate_points_sequence(self, xyz: torch.Tensor, poses):
        """Fuse scans xyz[0..F-1] (float32 [F, N, 3] on the GPU) with poses [F, 4, 4] in order."""
        if xyz.dim() != 3 or xyz.shape[2] != 3:
            raise ValueError("xyz must be [F, N, 3]")
        p = _dev(xyz, torch.float32, name="xyz")
        Pa, Pp = _host_doubles(poses, 16 * xyz.shape[0])
        self._check(_lib.load().mrh_integrate_points_sequence(self._h, p, xyz.shape[0], xyz.shape[1], Pp),
                    "mrh_integrate_points_sequence")

    def sync(self):
        """Wait for the map's stream; return (stats of the frames since the previous sync, totals);
        raise a latched error."""
        last, tot = MrhStats(), MrhStats()
        self._check(_lib.load().mrh_sync(self._h, ctypes.byref(last), ctypes.byref(tot)), "mrh_sync")
        return last.as_dict(), tot.as_dict()

    # -- launch profiler ------------------------------------------------------------------------
    def profile(self, on: bool = True):
        self._check(_lib.load().mrh_profile_enable(self._h, int(on)), "mrh_profile_enable")

    def profile_collect(self) -> dict:
        """{kernel name: (total ms, launches)} since the last collect (synchronises)."""
        n = len(_lib.KERNELS)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        self._check(_lib.load().mrh_profile_collect(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                                    cnt.ctypes.data_as(ctypes.c_void_p), n),
                    "mrh_profile_collect")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(_lib.KERNELS) if cnt[i]}

    # -- queries --------------------------------------------------------------------------------
    def query(self, pts: torch.Tensor, T=None, strict: bool = False, with_grad: bool = False):
        """Trilinear SDF at float32 [N, 3] points (optionally through pose T); returns
        (sdf float32 [N], valid bool [N], grad float32 [N, 3] or None)."""
        p = _dev(pts, torch.float32, (3,), name="pts")
        n = pts.shape[0]
        sdf = torch.empty(n, dtype=torch.float32, device=pts.device)
        valid = torch.empty(n, dtype=torch.uint8, device=pts.device)
        grad = torch.empty((n, 3), dtype=torch.float32, device=pts.device) if with_grad else None
        Tp = None
        if T is not None:
            Ta, Tp = _host_doubles(T, 16)
        self._check(_lib.load().mrh_query_sdf(self._h, p, n, Tp, int(strict), ctypes.c_void_p(sdf.data_ptr()),
                                              ctypes.c_void_p(valid.data_ptr()),
                                              ctypes.c_void_p(grad.data_ptr()) if grad is not None else None),
                    "mrh_query_sdf")
        return sdf, valid.bool(), grad

    def query_backward(self, pts: torch.Tensor, grad_sdf: torch.Tensor, T=None, strict: bool = False):
        """Adjoint of query: returns (dL/dp float32 [N, 3], dL/dxi float64 numpy [6])."""
        p = _dev(pts, torch.float32, (3,), name="pts")
        g = _dev(grad_sdf.contiguous(), torch.float32, name="grad_sdf")
        n = pts.shape[0]
        gp = torch.empty((n, 3), dtype=torch.float32, device=pts.device)
        pose = np.zeros(6, dtype=np.float64)
        Tp = None
        if T is not None:
            Ta, Tp = _host_doubles(T, 16)
        self._check(_lib.load().mrh_query_sdf_backward(self._h, p, n, Tp, int(strict), g,
                                                       ctypes.c_void_p(gp.data_ptr()),
                                                       pose.ctypes.data_as(ctypes.c_void_p)),
                    "mrh_query_sdf_backward")
        return gp, pose

    # -- extraction -----------------------------------------------------------------------------
    def counts(self):
        nb, nv = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.load().mrh_extract_blocks(self._h, None, None, None, None, None, None, 0, 0,
                                                   ctypes.byref(nb), ctypes.byref(nv)), "mrh_extract_blocks")
        return nb.value, nv.value

    def extract(self, voxels: bool = True) -> dict:
        """Blocks in table order: keys int32 [n, 3], levels uint8 [n] and, with voxels, offsets
        int64 [n + 1] and D float32, W int32 (bit pattern of the uint32 weights), S2 float32."""
        nb, nv = self.counts()
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty((nb, 3), dtype=torch.int32, device=dev)
        levels = torch.empty(nb, dtype=torch.uint8, device=dev)
        out = {"keys": keys, "levels": levels}
        args = [ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(levels.data_ptr())]
        if voxels:
            offs = torch.empty(nb + 1, dtype=torch.int64, device=dev)
            D = torch.empty(nv, dtype=torch.float32, device=dev)
            W = torch.empty(nv, dtype=torch.int32, device=dev)
            S2 = torch.empty(nv, dtype=torch.float32, device=dev)
            args += [ctypes.c_void_p(t.data_ptr()) for t in (offs, D, W, S2)]
            out.update(offsets=offs, D=D, W=W, S2=S2)
        else:
            args += [None, None, None, None]
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.load().mrh_extract_blocks(self._h, *args, nb, nv, ctypes.byref(a), ctypes.byref(b)),
                    "mrh_extract_blocks")
        return out


    def mesh(self, collapse: float = 0.0, codes: bool = True) -> dict:
        """Multi-resolution Marching Cubes of the map (mrh_extract_mesh): verts float32 [T, 3, 3]
        (world metres, counter-clockwise seen from outside), and with codes the block key of each
        triangle's cube (int32 [T, 3]) and its code (int32 [T], the bits of the uint32 code)."""
        n = ctypes.c_int64()
        L = _lib.load()
        self._check(L.mrh_extract_mesh(self._h, float(collapse), None, None, None, 0, ctypes.byref(n)),
                    "mrh_extract_mesh")
        t = n.value
        dev = torch.device("cuda", torch.cuda.current_device())
        verts = torch.empty((t, 3, 3), dtype=torch.float32, device=dev)
        out = {"verts": verts}
        bp = cp = None
        if codes:
            out["blocks"] = torch.empty((t, 3), dtype=torch.int32, device=dev)
            out["codes"] = torch.empty(t, dtype=torch.int32, device=dev)
            bp, cp = ctypes.c_void_p(out["blocks"].data_ptr()), ctypes.c_void_p(out["codes"].data_ptr())
        self._check(L.mrh_extract_mesh(self._h, float(collapse), ctypes.c_void_p(verts.data_ptr()), bp, cp, t,
                                       ctypes.byref(n)), "mrh_extract_mesh")
        return out


    def check(self) -> dict:
        """Consistency of the hash table, the block rows and the heaps' free stacks and pending
        lists (host copies; between frames).  'consistent' is True when no violation was found;
        'mean_probe' / 'max_probe' give the probe lengths of the present keys."""
        c = _lib.MrhCheck()
        self._check(_lib.load().mrh_map_check(self._h, ctypes.byref(c)), "mrh_map_check")
        return c.as_dict()

    # -- streaming (capacity-driven, between the heaps and the map's host store) -------------
    def heap_usage(self) -> float:
        f = ctypes.c_double()
        self._check(_lib.load().mrh_heap_usage(self._h, ctypes.byref(f)), "mrh_heap_usage")
        return f.value

    def stream_out(self, region, threshold: float = 0.85) -> int:
        """Move every block outside `region` (see depth_region / points_region) to the host store
        when the heaps are at least `threshold` full; returns the number moved."""
        n = ctypes.c_int64()
        self._check(_lib.load().mrh_stream_out(self._h, ctypes.byref(region), float(threshold), ctypes.byref(n)),
                    "mrh_stream_out")
        return n.value

    def stream_in(self, region) -> int:
        """Move every stored block inside `region` back to the GPU; returns the number moved."""
        n = ctypes.c_int64()
        self._check(_lib.load().mrh_stream_in(self._h, ctypes.byref(region), ctypes.byref(n)), "mrh_stream_in")
        return n.value

    def store_info(self):
        """(blocks, voxels, host bytes) held in the host store."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.load().mrh_store_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
                    "mrh_store_info")
        return a.value, b.value, c.value

    def store_extract(self) -> dict:
        """The host store decoded (numpy): keys int32 [n, 3] in ascending packed-key order, levels
        uint8 [n], offsets int64 [n + 1], D float32, W uint32, S2 float32 (voxels x fastest)."""
        L = _lib.load()
        nb, nv = ctypes.c_int64(), ctypes.c_int64()
        self._check(L.mrh_store_extract(self._h, None, None, None, None, None, None, 0, 0, ctypes.byref(nb),
                                        ctypes.byref(nv)), "mrh_store_extract")
        out = {"keys": np.zeros((nb.value, 3), np.int32), "levels": np.zeros(nb.value, np.uint8),
               "offsets": np.zeros(nb.value + 1, np.int64), "D": np.zeros(nv.value, np.float32),
               "W": np.zeros(nv.value, np.uint32), "S2": np.zeros(nv.value, np.float32)}
        ptr = [out[k].ctypes.data_as(ctypes.c_void_p) for k in ("keys", "levels", "offsets", "D", "W", "S2")]
        self._check(L.mrh_store_extract(self._h, *ptr, nb.value, nv.value, ctypes.byref(nb), ctypes.byref(nv)),
                    "mrh_store_extract")
        return out

    def load_blocks(self, keys, levels, D, W, S2) -> int:
        """Load caller-held blocks (numpy, the layout of store_extract / extract) into the map."""
        keys = np.ascontiguousarray(keys, dtype=np.int32).reshape(-1, 3)
        levels = np.ascontiguousarray(levels, dtype=np.uint8)
        D = np.ascontiguousarray(D, dtype=np.float32)
        W = np.ascontiguousarray(W, dtype=np.uint32)
        S2 = np.ascontiguousarray(S2, dtype=np.float32)
        nv = int(sum((8 >> int(l)) ** 3 for l in levels))
        if levels.shape[0] != keys.shape[0] or min(D.size, W.size, S2.size) < nv:
            raise ValueError("load_blocks: arrays do not match the block list")
        n = ctypes.c_int64()
        ptr = [a.ctypes.data_as(ctypes.c_void_p) for a in (keys, levels, D, W, S2)]
        self._check(_lib.load().mrh_load_blocks(self._h, keys.shape[0], *ptr, ctypes.byref(n)), "mrh_load_blocks")
        return n.value


class Quadtree:
    """Image-space quadtree by contrast (Eq. 10, Algorithm 1) for images up to max_width x max_height,
    bound to torch's current stream."""

    def __init__(self, max_width: int, max_height: int):
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = _lib.load().mrh_quadtree_create(int(max_width), int(max_height), ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(h))
        if st != 0:
            raise MrhError(st, "mrh_quadtree_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mrh_quadtree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, rgb: torch.Tensor, threshold: float, min_size: int):
        """Leaves (int32 [n, 4] as x0, y0, w, h) and contrast (float32 [n]) of a uint8 [h, w, 3] image."""
        if rgb.dim() != 3 or rgb.shape[2] != 3:
            raise ValueError("rgb must be [H, W, 3]")
        p = _dev(rgb, torch.uint8, name="rgb")
        L = _lib.load()
        n = ctypes.c_int64()
        # one build into buffers sized for the worst case (every leaf holds at least one pixel)
        cap = int(rgb.shape[0]) * int(rgb.shape[1])
        leaves = torch.empty((cap, 4), dtype=torch.int32, device=rgb.device)
        con = torch.empty(cap, dtype=torch.float32, device=rgb.device)
        st = L.mrh_quadtree_build(self._h, p, rgb.shape[1], rgb.shape[0], float(threshold), int(min_size),
                                  ctypes.c_void_p(leaves.data_ptr()), ctypes.c_void_p(con.data_ptr()), cap,
                                  ctypes.byref(n))
        if st != 0:
            raise MrhError(st, "mrh_quadtree_build")
        return leaves[: n.value].clone(), con[: n.value].clone()


def convert(values, storage: str, decode: bool = False):
    """The conversion of a 16-bit storage format ("f16" or "bf16"), element by element: float32 to
    uint16 bit patterns (decode=False) or back.  A CUDA tensor runs the device codec the fusion
    kernels use; a numpy array runs the host codec."""
    st = STORAGE[storage]
    if st == STORAGE["f32"]:
        raise ValueError("convert: storage must be 'f16' or 'bf16'")
    if isinstance(values, torch.Tensor):
        want = torch.int16 if decode else torch.float32
        if values.dtype != want or not values.is_cuda or not values.is_contiguous():
            raise ValueError(f"convert: a contiguous CUDA {want} tensor is required")
        out = torch.empty(values.shape, dtype=torch.float32 if decode else torch.int16, device=values.device)
        code = _lib.load().mrh_codec_device(st, int(decode), ctypes.c_void_p(values.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), values.numel())
    else:
        x = np.ascontiguousarray(values, dtype=np.uint16 if decode else np.float32)
        out = np.empty(x.shape, dtype=np.float32 if decode else np.uint16)
        code = _lib.load().mrh_codec_host(st, int(decode), x.ctypes.data, out.ctypes.data, x.size)
    if code != 0:
        raise MrhError(code, "convert")
    return out


def depth_region(width: int, height: int, K, T_ws) -> "_lib.MrhRegion":
    """Streaming region of an RGB-D frame: the camera frustum."""
    r = _lib.MrhRegion()
    r.kind, r.width, r.height = _lib.FRAME_DEPTH, int(width), int(height)
    for i, v in enumerate(np.asarray(K, np.float64).ravel()[:4]):
        r.K[i] = float(v)
    for i, v in enumerate(np.asarray(T_ws, np.float64).ravel()[:16]):
        r.T_ws[i] = float(v)
    return r


def points_region(T_ws, radius: float) -> "_lib.MrhRegion":
    """Streaming region of a LiDAR scan: the ball of `radius` around the sensor."""
    r = _lib.MrhRegion()
    r.kind, r.radius = _lib.FRAME_POINTS, float(radius)
    for i, v in enumerate(np.asarray(T_ws, np.float64).ravel()[:16]):
        r.T_ws[i] = float(v)
    return r


class Batch:
    """Many maps fused together: one frame per map per ``integrate`` call, at most four launches in
    total, replayed from a captured HIP graph while the frame kinds and sizes stay the same."""

    def __init__(self, maps):
        self.maps = list(maps)
        arr = (ctypes.c_void_p * len(self.maps))(*[m._h.value for m in self.maps])
        h = ctypes.c_void_p()
        st = _lib.load().mrh_batch_create(arr, len(self.maps), ctypes.byref(h))
        if st != 0:
            raise MrhError(st, "mrh_batch_create")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().mrh_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _frames(self, frames):
        """frames: one entry per map, ("depth", tensor [H, W], K, T), ("points", tensor [N, 3], T) or None."""
        if len(frames) != len(self.maps):
            raise ValueError("one frame per map")
        arr = (_lib.MrhFrame * len(frames))()
        for i, fr in enumerate(frames):
            if fr is None:
                arr[i].kind = _lib.FRAME_NONE
                continue
            T = np.asarray(fr[-1], dtype=np.float64).reshape(16)
            for k in range(16):
                arr[i].T_ws[k] = T[k]
            if fr[0] == "depth":
                d = fr[1]
                _dev(d, torch.float32, name="depth")
                arr[i].kind, arr[i].width, arr[i].height = _lib.FRAME_DEPTH, d.shape[1], d.shape[0]
                arr[i].data_dev = d.data_ptr()
                for k in range(4):
                    arr[i].K[k] = float(fr[2][k])
            elif fr[0] == "points":
                x = fr[1]
                _dev(x, torch.float32, (3,), name="xyz")
                arr[i].kind, arr[i].n, arr[i].data_dev = _lib.FRAME_POINTS, x.shape[0], x.data_ptr()
            else:
                raise ValueError(f"unknown frame kind {fr[0]}")
        return arr

    def integrate(self, frames):
        arr = self._frames(frames)
        st = _lib.load().mrh_batch_integrate(self._h, arr)
        if st != 0:
            raise MrhError(st, "mrh_batch_integrate", _lib.load().mrh_last_error(self.maps[0]._h).decode())

    def set_launch(self, update_wgs: int, cull_wgs: int, graph: bool = True, update_waves: int = 4):
        p = (ctypes.c_int32 * 4)(update_wgs, cull_wgs, int(graph), update_waves)
        st = _lib.load().mrh_batch_set_launch(self._h, p)
        if st != 0:
            raise MrhError(st, "mrh_batch_set_launch")

    def get_launch(self):
        p = (ctypes.c_int32 * 4)()
        _lib.load().mrh_batch_get_launch(self._h, p)
        return tuple(p)

    def autotune(self, frames, reps: int = 3):
        """Time every candidate launch shape on `frames` (maps are reset before and after)."""
        arr = self._frames(frames)
        best = (ctypes.c_int32 * 4)()
        st = _lib.load().mrh_batch_autotune(self._h, arr, int(reps), best)
        if st != 0:
            raise MrhError(st, "mrh_batch_autotune", _lib.load().mrh_last_error(self.maps[0]._h).decode())
        return tuple(best)


class SdfQuery(torch.autograd.Function):
    """sdf = SdfQuery.apply(map, pts, T, strict): differentiable in pts; the pose gradient of the
    last backward is kept in ``map.last_pose_grad`` (dL/dxi for a left perturbation of T)."""

    @staticmethod
    def forward(ctx, fmap: Map, pts: torch.Tensor, T=None, strict: bool = False):
        pts_c = pts.detach().contiguous()
        sdf, valid, _ = fmap.query(pts_c, T=T, strict=strict)
        ctx.fmap, ctx.T, ctx.strict = fmap, T, strict
        ctx.save_for_backward(pts_c)
        ctx.mark_non_differentiable(valid)
        return sdf, valid

    @staticmethod
    def backward(ctx, grad_sdf, grad_valid):
        (pts_c,) = ctx.saved_tensors
        if grad_sdf is None:
            return None, None, None, None
        gp, pose = ctx.fmap.query_backward(pts_c, grad_sdf.float().contiguous(), T=ctx.T, strict=ctx.strict)
        ctx.fmap.last_pose_grad = pose
        return None, gp, None, None
