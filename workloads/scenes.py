"""Analytic scenes ray-cast in closed form into depth images and LiDAR scans.

Every generator is seeded (``numpy.random.default_rng``, PCG64) and returns plain NumPy arrays:

* depth frames: ``float32[H, W]`` z-depth in metres, pixel (u, v) = (column, row) with its centre at
  integer (u, v); the camera ray of pixel (u, v) is ((u - cx)/fx, (v - cy)/fy, 1) in the sensor frame
  (x right, y down, z forward), so the ray parameter of a hit *is* its z-depth;
* LiDAR scans: ``float32[N, 3]`` points in the sensor frame (x forward, y left, z up), ring-major,
  NaN where a beam has no return inside the kept range;
* poses: ``float64[4, 4]`` world-from-sensor transforms, row-major.

The scenes stand in for the datasets the paper measures on (ScanNet / Replica rooms for RGB-D,
Newer College / Oxford Spires streets for LiDAR; Sec. 4.1), which are not available here.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


def _map_frames(fn, items):
    """Evaluate fn over frame indices on a thread pool (NumPy releases the GIL in its kernels);
    every frame draws from its own seeded generator, so the result does not depend on the pool.
    fn must not call BLAS (matrix products): concurrent BLAS calls from several threads are not
    safe in every build and have returned wrong values; use _rotate and elementwise sums."""
    workers = min(len(items), max(1, min(16, os.cpu_count() or 1)))
    if workers <= 1:
        return [fn(k) for k in items]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


@dataclass(frozen=True)
class Pinhole:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @property
    def K(self) -> np.ndarray:
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float64)

    def rays(self) -> np.ndarray:
        """float64[H, W, 3] unnormalised sensor-frame rays with z = 1."""
        u = np.arange(self.width, dtype=np.float64)
        v = np.arange(self.height, dtype=np.float64)
        uu, vv = np.meshgrid(u, v)
        return np.stack([(uu - self.cx) / self.fx, (vv - self.cy) / self.fy, np.ones_like(uu)], axis=-1)


# --------------------------------------------------------------------------------------------
# ray/primitive intersection helpers (vectorised over rays; return +inf where there is no hit)
# --------------------------------------------------------------------------------------------

def _rotate(v, R):
    """v @ R.T for float64[..., 3] vectors, by elementwise products (no BLAS)."""
    return v[..., 0:1] * R[:, 0] + v[..., 1:2] * R[:, 1] + v[..., 2:3] * R[:, 2]


def _hit_sphere(o, w, centre, radius):
    oc = o - centre
    a = np.einsum("...i,...i->...", w, w)
    b = np.einsum("...i,...i->...", w, oc)
    c = float(np.sum(oc * oc)) - radius * radius
    disc = b * b - a * c
    t = np.full(a.shape, np.inf)
    ok = disc >= 0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    t0 = (-b - sq) / a
    t1 = (-b + sq) / a
    near = np.where(t0 > 1e-9, t0, np.where(t1 > 1e-9, t1, np.inf))
    t[ok] = near[ok]
    return t


def _hit_box_outside(o, w, lo, hi):
    """Entry distance into an axis-aligned box seen from outside (inf when missed)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / w
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
    tmin = np.minimum(t1, t2)
    tmax = np.maximum(t1, t2)
    tmin = np.where(np.isnan(tmin), -np.inf, tmin)
    tmax = np.where(np.isnan(tmax), np.inf, tmax)
    tn = tmin.max(axis=-1)
    tf = tmax.min(axis=-1)
    hit = (tn <= tf) & (tn > 1e-9)
    return np.where(hit, tn, np.inf)


def _hit_box_inside(o, w, lo, hi):
    """Exit distance from an axis-aligned box that contains the ray origin."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / w
        t1 = (lo - o) * inv
        t2 = (hi - o) * inv
    tmax = np.maximum(t1, t2)
    tmax = np.where(np.isnan(tmax), np.inf, tmax)
    return tmax.min(axis=-1)


def _hit_plane_z(o, w, z0):
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (z0 - o[..., 2]) / w[..., 2]
    return np.where(t > 1e-9, t, np.inf)


# --------------------------------------------------------------------------------------------
# single frame: sphere in front of a plane (small correctness workload)
# --------------------------------------------------------------------------------------------

def sphere_plane_frame(seed: int = 0, width: int = 320, height: int = 240, f: float = 300.0,
                       radius: float = 0.5, centre_z: float = 2.5, plane_z: float = 4.0,
                       noise: float = 0.001):
    """One 320x240 RGB-D frame of a sphere (centre (0, 0, 2.5) m) in front of the plane z = 4 m.

    The sphere radius defaults to 0.5 m (a 1 m diameter) so that its silhouette stays inside the
    field of view.  Returns ``(depth f32[H, W], Pinhole, T_ws f64[4, 4])`` with an identity pose.
    """
    cam = Pinhole(width, height, f, f, width / 2.0, height / 2.0)
    r = cam.rays()
    o = np.zeros(3)
    t = np.minimum(_hit_plane_z(o, r, plane_z), _hit_sphere(o, r, np.array([0.0, 0.0, centre_z]), radius))
    rng = np.random.default_rng(seed)
    depth = t + rng.normal(0.0, noise, size=t.shape) if noise > 0 else t
    return depth.astype(np.float32), cam, np.eye(4)


def plane_frame(z0: float, width: int = 64, height: int = 48, f: float = 60.0):
    """Noise-free fronto-parallel plane z = z0 seen by an identity-pose camera."""
    cam = Pinhole(width, height, f, f, width / 2.0, height / 2.0)
    return np.full((height, width), z0, dtype=np.float32), cam, np.eye(4)


# --------------------------------------------------------------------------------------------
# RGB-D room sequence
# --------------------------------------------------------------------------------------------

@dataclass
class RoomScene:
    size: tuple = (6.0, 6.0, 3.0)
    spheres: list = field(default_factory=list)  # (centre[3], radius)
    boxes: list = field(default_factory=list)  # (lo[3], hi[3])

    def raycast(self, o, w):
        t = _hit_box_inside(o, w, np.zeros(3), np.array(self.size))
        for c, rad in self.spheres:
            t = np.minimum(t, _hit_sphere(o, w, c, rad))
        for lo, hi in self.boxes:
            t = np.minimum(t, _hit_box_outside(o, w, lo, hi))
        return t

    def sdf(self, p):
        """Signed distance of world points p [..., 3] to the room's surfaces, positive in free space:
        the minimum of the distance to the walls (from inside the room) and the signed distances of
        the spheres and cuboids.  Exact in free space; inside an obstacle it is the depth below the
        nearest face of that obstacle."""
        p = np.asarray(p, dtype=np.float64)
        size = np.array(self.size)
        d = np.minimum(p, size - p).min(axis=-1)
        for c, rad in self.spheres:
            d = np.minimum(d, np.linalg.norm(p - c, axis=-1) - rad)
        for lo, hi in self.boxes:
            q = np.abs(p - 0.5 * (lo + hi)) - 0.5 * (hi - lo)
            outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
            d = np.minimum(d, outside + np.minimum(q.max(axis=-1), 0.0))
        return d


def _orbit_clearance(centre, extent, orbit_c=(3.0, 3.0), orbit_r=1.5, z_mid=1.5, z_amp=0.2):
    rho = math.hypot(centre[0] - orbit_c[0], centre[1] - orbit_c[1])
    dz = max(0.0, abs(centre[2] - z_mid) - z_amp)
    return math.hypot(rho - orbit_r, dz) - extent


def room_scene(seed: int = 1, n_primitives: int = 20, clearance: float = 0.3) -> RoomScene:
    """A 6 x 6 x 3 m box interior holding ``n_primitives`` random spheres and axis-aligned cuboids.

    Sphere radii ~ U[0.15, 0.5] m, cuboid half-extents ~ U[0.1, 0.6] m; every primitive keeps
    ``clearance`` metres from the camera orbit (radius 1.5 m about (3, 3), height 1.5 +- 0.2 m).
    """
    rng = np.random.default_rng(seed)
    scene = RoomScene()
    size = np.array(scene.size)
    while len(scene.spheres) + len(scene.boxes) < n_primitives:
        if rng.random() < 0.5:
            rad = rng.uniform(0.15, 0.5)
            c = rng.uniform(rad, size - rad)
            if _orbit_clearance(c, rad) < clearance:
                continue
            scene.spheres.append((c, rad))
        else:
            h = rng.uniform(0.1, 0.6, size=3)
            c = rng.uniform(h, size - h)
            if _orbit_clearance(c, float(np.linalg.norm(h))) < clearance:
                continue
            scene.boxes.append((c - h, c + h))
    return scene


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-from-camera pose for a camera at ``eye`` looking at ``target`` (x right, y down, z fwd)."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = right, down, fwd, eye
    return T


def orbit_pose(k: int, n_frames: int) -> np.ndarray:
    th = 2.0 * math.pi * k / n_frames
    eye = (3.0 + 1.5 * math.cos(th), 3.0 + 1.5 * math.sin(th), 1.5 + 0.2 * math.sin(2.0 * th))
    return look_at(eye, (3.0, 3.0, 1.5))


def room_sequence(n_frames: int = 100, width: int = 640, height: int = 480, f: float = 525.0,
                  scene_seed: int = 1, noise_seed: int = 2, noise_k: float = 0.0012,
                  frames=None):
    """The 100-frame RGB-D orbit of a seeded room.

    z-depth noise is N(0, (noise_k * z^2)^2).  Pixels beyond the sensor range are left in the frame;
    the fusion's own max-depth filter drops them.  Returns ``(depths f32[F, H, W], Pinhole,
    poses f64[F, 4, 4], scene)``; ``frames`` optionally selects a subset of frame indices (the noise
    of frame k is the same whichever subset is asked for).
    """
    cam = Pinhole(width, height, f, f, width / 2.0, height / 2.0)
    scene = room_scene(scene_seed)
    r = cam.rays()
    idx = list(range(n_frames)) if frames is None else list(frames)

    def one(k):
        T = orbit_pose(k, n_frames)
        w = _rotate(r, T[:3, :3])
        z = scene.raycast(T[:3, 3], w)
        rng = np.random.default_rng([noise_seed, k])
        z = z + rng.normal(0.0, 1.0, size=z.shape) * (noise_k * z * z)
        return z.astype(np.float32), T

    out = _map_frames(one, idx)
    depths = np.stack([o[0] for o in out]) if out else np.empty((0, height, width), np.float32)
    poses = np.stack([o[1] for o in out]) if out else np.empty((0, 4, 4))
    return depths, cam, poses, scene


# --------------------------------------------------------------------------------------------
# LiDAR street sequence
# --------------------------------------------------------------------------------------------

def lidar_directions(rings: int = 64, azimuths: int = 2048, fov_lo_deg: float = -52.0,
                     fov_hi_deg: float = 52.0) -> np.ndarray:
    """float64[rings * azimuths, 3] unit beam directions, ring-major, sensor frame (x fwd, z up)."""
    el = np.deg2rad(np.linspace(fov_lo_deg, fov_hi_deg, rings))
    az = 2.0 * math.pi * np.arange(azimuths) / azimuths
    ee, aa = np.meshgrid(el, az, indexing="ij")
    d = np.stack([np.cos(ee) * np.cos(aa), np.cos(ee) * np.sin(aa), np.sin(ee)], axis=-1)
    return d.reshape(-1, 3)


@dataclass
class StreetScene:
    boxes: list = field(default_factory=list)  # (lo[3], hi[3])

    def raycast(self, o, w):
        t = _hit_plane_z(o, w, 0.0)
        for lo, hi in self.boxes:
            # skip boxes far outside any 80 m return (cheap bounding-sphere reject)
            c = 0.5 * (lo + hi)
            if math.sqrt(float(np.sum((c - o) ** 2))) - 0.5 * math.sqrt(float(np.sum((hi - lo) ** 2))) > 90.0:
                continue
            t = np.minimum(t, _hit_box_outside(o, w, lo, hi))
        return t


def street_scene(seed: int = 3, length: float = 200.0, n_street_boxes: int = 40) -> StreetScene:
    """Ground plane z = 0, facade boxes lining y = +-12 m, and street furniture boxes of 1-5 m."""
    rng = np.random.default_rng(seed)
    sc = StreetScene()
    for side in (+1.0, -1.0):
        x = -40.0
        while x < length + 40.0:
            wdt = rng.uniform(8.0, 20.0)
            hgt = rng.uniform(6.0, 25.0)
            dep = rng.uniform(8.0, 14.0)
            if side > 0:
                lo, hi = np.array([x, 12.0, 0.0]), np.array([x + wdt, 12.0 + dep, hgt])
            else:
                lo, hi = np.array([x, -12.0 - dep, 0.0]), np.array([x + wdt, -12.0, hgt])
            sc.boxes.append((lo, hi))
            x += wdt + (rng.uniform(2.0, 8.0) if rng.random() < 0.3 else 0.0)
    n = 0
    while n < n_street_boxes:
        h = rng.uniform(0.5, 2.5, size=3)
        c = np.array([rng.uniform(-10.0, length + 10.0), rng.uniform(-10.0, 10.0), h[2]])
        if abs(c[1]) - h[1] < 2.5 or abs(c[1]) + h[1] > 11.5:
            continue
        sc.boxes.append((c - h, c + h))
        n += 1
    return sc


def street_pose(k: int) -> np.ndarray:
    yaw = math.radians(3.0) * math.sin(2.0 * math.pi * k / 50.0)
    c, s = math.cos(yaw), math.sin(yaw)
    T = np.eye(4)
    T[:3, :3] = [[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]
    T[:3, 3] = [float(k), 0.0, 1.8]
    return T


def street_sequence(n_scans: int = 200, rings: int = 64, azimuths: int = 2048,
                    scene_seed: int = 3, noise_seed: int = 4, noise: float = 0.02,
                    min_range: float = 1.0, max_range: float = 80.0, scans=None):
    """LiDAR scans of a seeded street, one per metre along +x at 1.8 m height with +-3 deg yaw.

    Range noise N(0, noise^2) is added along each beam; returns outside [min_range, max_range] are
    NaN so that every scan keeps the shape (rings * azimuths, 3).  Returns ``(points f32[S, N, 3],
    poses f64[S, 4, 4], scene)``.
    """
    sc = street_scene(scene_seed)
    dirs = lidar_directions(rings, azimuths)
    idx = list(range(n_scans)) if scans is None else list(scans)

    def one(k):
        T = street_pose(k)
        w = _rotate(dirs, T[:3, :3])
        r = sc.raycast(T[:3, 3], w)
        rng = np.random.default_rng([noise_seed, k])
        r = r + rng.normal(0.0, noise, size=r.shape)
        keep = (r >= min_range) & (r <= max_range)
        with np.errstate(invalid="ignore"):
            p = dirs * r[:, None]
        p[~keep] = np.nan
        return p.astype(np.float32), T

    out = _map_frames(one, idx)
    pts = np.stack([o[0] for o in out]) if out else np.empty((0, dirs.shape[0], 3), np.float32)
    poses = np.stack([o[1] for o in out]) if out else np.empty((0, 4, 4))
    return pts, poses, sc


# --------------------------------------------------------------------------------------------
# query points near the surfaces of a room
# --------------------------------------------------------------------------------------------

def surface_query_points(scene: RoomScene, n: int, sigma: float, seed: int = 100, with_offsets: bool = False):
    """float32[n, 3] world points sampled on the room's surfaces in proportion to their area and
    offset by N(0, sigma^2) along the surface normal (towards free space); with ``with_offsets``
    also the float64[n] offsets, in the same order."""
    rng = np.random.default_rng(seed)
    sx, sy, sz = scene.size
    faces = []  # (area, sampler)
    for axis, size in ((0, sx), (1, sy), (2, sz)):
        others = [a for a in range(3) if a != axis]
        ext = [scene.size[a] for a in others]
        for val, nrm in ((0.0, 1.0), (size, -1.0)):
            faces.append((ext[0] * ext[1], ("wall", axis, val, nrm, others, ext)))
    for c, rad in scene.spheres:
        faces.append((4.0 * math.pi * rad * rad, ("sphere", c, rad)))
    for lo, hi in scene.boxes:
        e = hi - lo
        for axis in range(3):
            others = [a for a in range(3) if a != axis]
            for val, nrm in ((lo[axis], -1.0), (hi[axis], 1.0)):
                faces.append((e[others[0]] * e[others[1]],
                              ("face", axis, val, nrm, others, lo, hi)))
    area = np.array([a for a, _ in faces])
    counts = rng.multinomial(n, area / area.sum())
    out = []
    offs = []
    for cnt, (_, spec) in zip(counts, faces):
        if cnt == 0:
            continue
        if spec[0] == "wall":
            _, axis, val, nrm, others, ext = spec
            p = np.zeros((cnt, 3))
            p[:, axis] = val
            p[:, others[0]] = rng.uniform(0, ext[0], cnt)
            p[:, others[1]] = rng.uniform(0, ext[1], cnt)
            nv = np.zeros((cnt, 3))
            nv[:, axis] = nrm
        elif spec[0] == "sphere":
            _, c, rad = spec
            nv = rng.normal(size=(cnt, 3))
            nv /= np.linalg.norm(nv, axis=1, keepdims=True)
            p = c + rad * nv
        else:
            _, axis, val, nrm, others, lo, hi = spec
            p = np.zeros((cnt, 3))
            p[:, axis] = val
            p[:, others[0]] = rng.uniform(lo[others[0]], hi[others[0]], cnt)
            p[:, others[1]] = rng.uniform(lo[others[1]], hi[others[1]], cnt)
            nv = np.zeros((cnt, 3))
            nv[:, axis] = nrm
        off = rng.normal(0.0, sigma, size=(cnt, 1))
        out.append(p + nv * off)
        offs.append(off[:, 0])
    pts = np.concatenate(out, axis=0)
    perm = rng.permutation(pts.shape[0])
    if with_offsets:
        return pts[perm].astype(np.float32), np.concatenate(offs)[perm]
    return pts[perm].astype(np.float32)


def colour_image(depth, cam, T):
    """A colour per pixel from the world point it sees (a fixed function of position, so every view
    of a surface point agrees); black where the depth is invalid."""
    h, w = depth.shape
    v, u = np.mgrid[0:h, 0:w]
    x = np.stack([(u - cam.cx) / cam.fx * depth, (v - cam.cy) / cam.fy * depth, depth], axis=-1)
    p = x @ T[:3, :3].T + T[:3, 3]
    c = np.stack([128 + 100 * np.sin(7 * p[..., 0]), 128 + 100 * np.sin(5 * p[..., 1] + 1),
                  128 + 100 * np.sin(3 * p[..., 2] + 2)], axis=-1)
    c[~np.isfinite(depth) | (depth <= 0)] = 0
    return np.clip(np.nan_to_num(c), 0, 255).astype(np.uint8)
