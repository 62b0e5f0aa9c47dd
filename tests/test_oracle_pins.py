"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: exact rational geometry (the
traversals), closed-form signed distances of planes and axis-aligned rays (Eq. 1, Eq. 2), a
two-pass mean/variance over the stored observation history (Eq. 3, 5, 6), conservation laws of
the merge, the reproduction of linear fields by trilinear interpolation, and finite differences
(the query adjoint).  A plausible slip in the oracle -- a dropped term, a flipped sign, a wrong
index or a transposed operand -- breaks at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

from workloads import plane_frame, sphere_plane_frame

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------------------------------
# exact segment / cell intersection (the brute-force stand-in for the DDA walks)
# ------------------------------------------------------------------------------------------

def _seg_hits_box(A, E, lo, hi):
    """Exact test: does the segment A + t (E - A), t in [0, 1], meet the closed box [lo, hi]?"""
    t0, t1 = Fraction(0), Fraction(1)
    for k in range(3):
        a, e = Fraction(A[k]), Fraction(E[k])
        d = e - a
        if d == 0:
            if a < lo[k] or a > hi[k]:
                return False
            continue
        ta, tb = (Fraction(lo[k]) - a) / d, (Fraction(hi[k]) - a) / d
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
        if t0 > t1:
            return False
    return True


def _brute_cells(A, E):
    lo = np.floor(np.minimum(A, E)).astype(np.int64) - 1
    hi = np.floor(np.maximum(A, E)).astype(np.int64) + 1
    out = set()
    for x in range(lo[0], hi[0] + 1):
        for y in range(lo[1], hi[1] + 1):
            for z in range(lo[2], hi[2] + 1):
                if _seg_hits_box(A, E, (x, y, z), (x + 1, y + 1, z + 1)):
                    out.add((x, y, z))
    return out


def test_block_walk_equals_exact_cell_set(orc):
    """Sec. 3.2 allocates 'all intersected voxel blocks' by DDA: the walk must visit exactly the
    cells the segment meets, in order of entry, each sharing a face with the previous one."""
    rng = np.random.default_rng(7)
    for inv_cell in (1.0 / 0.16, 1.0 / 0.08, 1.0 / 0.4):
        for _ in range(120):
            a = rng.uniform(-2.0, 2.0, 3)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            e = a + d * rng.uniform(0.01, 1.6)
            cells = orc.block_dda(a, e, inv_cell)
            A, E = a * inv_cell, e * inv_cell
            assert set(map(tuple, cells.tolist())) == _brute_cells(A, E)
            assert len(cells) == len(set(map(tuple, cells.tolist())))
            steps = np.abs(np.diff(cells, axis=0)).sum(axis=1)
            assert np.all(steps == 1)
            assert tuple(cells[0]) == tuple(np.floor(A).astype(np.int64))
            assert tuple(cells[-1]) == tuple(np.floor(E).astype(np.int64))


def test_block_walk_axis_aligned_and_negative(orc):
    # along -x from 0.5 to -2.5 (unit cells): cells 0, -1, -2, -3
    cells = orc.block_dda([0.5, 0.25, 0.75], [-2.5, 0.25, 0.75], 1.0)
    assert cells.tolist() == [[0, 0, 0], [-1, 0, 0], [-2, 0, 0], [-3, 0, 0]]
    # a segment inside one cell visits only that cell
    assert orc.block_dda([0.1, 0.2, 0.3], [0.4, 0.5, 0.6], 1.0).tolist() == [[0, 0, 0]]


def test_voxel_walk_equals_exact_cells_inside_block(orc):
    """The per-block traversal on the block's own lattice visits exactly the voxels of that
    block that the segment meets."""
    rng = np.random.default_rng(11)
    B = 0.4
    for m in (8, 4, 2, 1):
        nu = B / m
        for _ in range(30):
            a = rng.uniform(-1.0, 1.0, 3)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            e = a + d * rng.uniform(0.05, 1.5)
            for b in orc.block_dda(a, e, 1.0 / B):
                vox = orc.voxel_dda(a, e, b.astype(np.int32), B, 1.0 / nu, m)
                got = set(map(tuple, vox.tolist()))
                ob = b * B
                Al = (a - ob) * (1.0 / nu)
                El = (e - ob) * (1.0 / nu)
                want = {c for c in _brute_cells(Al, El) if all(0 <= c[k] < m for k in range(3))}
                if want:  # a block the segment only grazes within rounding may have no exact cell
                    assert got == want, (m, a, e, b)
                    steps = np.abs(np.diff(vox, axis=0)).sum(axis=1)
                    assert np.all(steps == 1)


# ------------------------------------------------------------------------------------------
# Eq. 2 (projective signed distance) against closed forms
# ------------------------------------------------------------------------------------------

def _centres(ext, nu0, B):
    """World centres of every voxel of every extracted block, aligned with ext.D."""
    out = np.empty((ext.D.shape[0], 3))
    for i, (key, lvl) in enumerate(zip(ext.keys, ext.levels)):
        m = 8 >> int(lvl)
        nu = nu0 * (1 << int(lvl))
        g = (np.arange(m) + 0.5) * nu
        zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
        c = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1) + key * B
        out[ext.offsets[i]:ext.offsets[i + 1]] = c
    return out


@pytest.mark.parametrize("form", ["range", "zdiff"])
def test_plane_closed_form(orc, form):
    """A fronto-parallel plane z = Z0 seen head-on: every updated voxel holds the signed distance
    from its centre to the plane, measured along its own viewing ray (range form: the ray meets
    the plane at scale Z0 / z, so the distance is ||x|| (Z0 / z - 1)) or along z (z-difference
    form), truncated at tau; weight 1, variance 0."""
    nu, tau = 0.02, 0.06
    Z0 = float(np.float32(1.3))  # the depth image holds float32 metres
    depth, cam, T = plane_frame(Z0, 64, 48, 50.0)
    m = orc.OracleMap(nu, tau=tau, max_depth=5.0, form=form)
    st = m.integrate_depth(depth, cam.K, T)
    ext = m.extract()
    assert st["valid_points"] == 64 * 48
    c = _centres(ext, nu, 8 * nu)
    upd = ext.W > 0
    assert upd.sum() == st["observations"] > 1000
    x = c[upd]
    if form == "range":
        hit = x * (Z0 / x[:, 2:3])
        sd = np.linalg.norm(hit, axis=1) - np.linalg.norm(x, axis=1)
    else:
        sd = Z0 - x[:, 2]
    assert np.all(sd >= -tau - 1e-12)
    np.testing.assert_allclose(ext.D[upd], np.minimum(sd, tau), rtol=0, atol=1e-12)
    assert np.all(ext.W[upd] == 1) and np.all(ext.S2 == 0)
    # voxels more than tau behind the plane are never updated
    behind = (Z0 - c[:, 2]) < -tau - 1e-9
    assert not np.any(upd & behind)


def _rot(yaw, pitch, roll):
    """Rotation matrix Rz(yaw) Ry(pitch) Rx(roll) (angles in degrees)."""
    a, b, c = np.deg2rad([yaw, pitch, roll])
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
    return Rz @ Ry @ Rx


@pytest.mark.parametrize("form", ["range", "zdiff"])
def test_rotated_camera_plane_closed_form(orc, form):
    """Eq. 2 under a yawed, pitched, rolled and translated camera.  The world plane that the camera
    sees head-on (normal R e_z) has the same constant z-depth Z0 at every pixel whatever the pose,
    so the depth image is known exactly and the fused map has a closed form in the voxel's sensor
    coordinates x = R^T (c - t): D = clip(||x|| (Z0 / x_z - 1)) (range form) or clip(Z0 - x_z)
    (z-difference form), W = 1, S2 = 0.  Which voxels are updated is also fixed: those that project
    inside the image (pixel floor(u + 1/2), floor(v + 1/2)) and lie no more than tau behind the
    plane.  Allocation is checked against the world points of the pixels (each pixel's block is
    allocated) and against the plane (no allocated block lies farther than tau from it).  A pose
    applied transposed, in either direction, fails these checks."""
    nu, tau = 0.02, 0.06
    B = 8 * nu
    Z0 = float(np.float32(1.3))
    depth, cam, _ = plane_frame(Z0, 64, 48, 50.0)
    T = np.eye(4)
    R = _rot(25.0, -15.0, 10.0)
    T[:3, :3] = R
    T[:3, 3] = [0.31, -0.23, 0.47]
    t = T[:3, 3]
    m = orc.OracleMap(nu, tau=tau, max_depth=5.0, form=form)
    st = m.integrate_depth(depth, cam.K, T)
    ext = m.extract()
    assert st["valid_points"] == 64 * 48

    # allocation: the block of every pixel's world point is present ...
    keys = set(map(tuple, ext.keys.tolist()))
    rays = cam.rays()
    pw = (rays * Z0).reshape(-1, 3) @ R.T + t
    for b in np.floor(pw / B).astype(np.int64).tolist():
        assert tuple(b) in keys
    # ... and every allocated block meets the slab of points within tau of the world plane
    nw = R[:, 2]
    cplane = Z0 + float(nw @ t)
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float64)
    box = (ext.keys[:, None, :] + corners[None]) * B
    s = box @ nw - cplane
    assert np.all(s.min(axis=1) <= tau + 1e-9) and np.all(s.max(axis=1) >= -tau - 1e-9)

    # values and the set of updated voxels
    c = _centres(ext, nu, B)
    x = (c - t) @ R
    upd = ext.W > 0
    assert upd.sum() == st["observations"] > 1000
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam.fx * (x[:, 0] / x[:, 2]) + cam.cx
        v = cam.fy * (x[:, 1] / x[:, 2]) + cam.cy
        if form == "range":
            raw = np.linalg.norm(x, axis=1) * (Z0 / x[:, 2] - 1.0)
        else:
            raw = Z0 - x[:, 2]
    front = x[:, 2] > 0
    inside = front & (u >= -0.5 + 1e-6) & (u < cam.width - 0.5 - 1e-6) & (v >= -0.5 + 1e-6) & (v < cam.height - 0.5 - 1e-6)
    outside = ~front | (u < -0.5 - 1e-6) | (u >= cam.width - 0.5 + 1e-6) | (v < -0.5 - 1e-6) | (v >= cam.height - 0.5 + 1e-6)
    want = inside & (raw >= -tau + 1e-9)
    wont = outside | (front & (raw < -tau - 1e-9))
    assert want.sum() > 1000
    assert np.all(upd[want]) and not np.any(upd[wont])
    np.testing.assert_allclose(ext.D[upd], np.minimum(raw[upd], tau), rtol=0, atol=1e-12)
    assert np.all(ext.W[upd] == 1) and np.all(ext.S2 == 0)


def test_sphere_plane_truncation_and_zero_crossing(orc):
    """One noise-free frame of the sphere-and-plane scene: |D| <= tau, W = 1, S2 = 0 and the
    zero crossing on the optical axis sits on the sphere's front at z = 2.0 m."""
    depth, cam, T = sphere_plane_frame(noise=0.0)
    m = orc.OracleMap(0.02, tau=0.06, max_depth=10.0)
    m.integrate_depth(depth, cam.K, T)
    ext = m.extract()
    assert np.all(np.abs(ext.D) <= 0.06 + 1e-15)
    assert set(np.unique(ext.W)) <= {0, 1}
    sdf, valid, _ = m.query(np.array([[0.0, 0.0, 1.99], [0.0, 0.0, 2.0], [0.0, 0.0, 2.01],
                                      [0.8, -0.5, 3.99]], np.float32))
    assert valid.all()
    assert abs(sdf[1]) < 2e-3 and sdf[0] > 0 > sdf[2]
    assert abs(sdf[3] - 0.01) < 2e-3


# ------------------------------------------------------------------------------------------
# Eq. 3, 5, 6: incremental mean / Welford against a two-pass computation over the history
# ------------------------------------------------------------------------------------------

def test_running_mean_and_variance_match_two_pass_history(orc):
    """Feed noise-free planes at several depths (z-difference form, so each voxel's observation is
    Z_k - z independent of pixel rounding).  For every voxel keep the full list of observations
    it received (re-derived here from the planes and the voxel's centre) and compare the oracle's
    D, W, S2 with the two-pass mean, count and sum of squared deviations."""
    nu, tau = 0.05, 0.15
    Zs = [float(np.float32(z)) for z in (1.0, 1.07, 0.95, 1.11, 1.02, 0.99, 1.2, 1.05)]
    m = orc.OracleMap(nu, tau=tau, max_depth=5.0, form="zdiff")
    hist_frames = []
    for Z in Zs:
        depth, cam, T = plane_frame(Z, 40, 30, 30.0)
        m.integrate_depth(depth, cam.K, T)
        hist_frames.append(Z)
    ext = m.extract()
    c = _centres(ext, nu, 8 * nu)
    # which frames reached each voxel: its block existed (allocated by then) and it projects into
    # the image; the allocation frame of each block is recovered by replaying frames one by one
    first = {}
    m2 = orc.OracleMap(nu, tau=tau, max_depth=5.0, form="zdiff")
    for k, Z in enumerate(Zs):
        depth, cam, T = plane_frame(Z, 40, 30, 30.0)
        m2.integrate_depth(depth, cam.K, T)
        for key in map(tuple, m2.extract().keys.tolist()):
            first.setdefault(key, k)
    blk_first = np.repeat(np.array([first[tuple(k)] for k in ext.keys.tolist()]), np.diff(ext.offsets))
    u = np.floor(30.0 * c[:, 0] / c[:, 2] + 20 + 0.5)
    v = np.floor(30.0 * c[:, 1] / c[:, 2] + 15 + 0.5)
    inside = (c[:, 2] > 0) & (u >= 0) & (u <= 39) & (v >= 0) & (v <= 29)
    checked = 0
    for i in range(c.shape[0]):
        obs = [min(Z - c[i, 2], tau) for k, Z in enumerate(Zs)
               if k >= blk_first[i] and inside[i] and Z - c[i, 2] >= -tau]
        assert ext.W[i] == len(obs)
        if obs:
            mean = sum(obs) / len(obs)
            s2 = sum((o - mean) ** 2 for o in obs)
            assert abs(ext.D[i] - mean) < 1e-12
            assert abs(ext.S2[i] - s2) < 1e-12
            checked += 1
    assert checked > 500


# ------------------------------------------------------------------------------------------
# Eq. 1 (ray-based LiDAR update) on axis-aligned rays
# ------------------------------------------------------------------------------------------

def test_lidar_axis_ray_closed_form(orc):
    """A single beam straight up the z axis (x, y fixed inside one voxel column) to a point at
    height Zp: the voxels crossed are exactly that column from the sensor to Zp + tau, each
    holding clip(Zp - z, -tau, tau) (Eq. 1 with n = +z)."""
    nu, tau = 0.05, 0.15
    m = orc.OracleMap(nu, tau=tau, min_range=0.5, max_range=80.0, carve=1)
    x0, y0, Zp = 0.013, 0.031, 2.37
    T = np.eye(4)
    T[:3, 3] = [x0, y0, 0.011]
    st = m.integrate_points(np.array([[0.0, 0.0, Zp - 0.011]], np.float32), T)
    p_z = np.float64(np.float32(Zp - 0.011)) + 0.011
    ext = m.extract()
    c = _centres(ext, nu, 8 * nu)
    upd = ext.W > 0
    assert np.all(np.floor(c[upd, 0] / nu) == np.floor(x0 / nu))
    assert np.all(np.floor(c[upd, 1] / nu) == np.floor(y0 / nu))
    zc = np.sort(c[upd, 2])
    want = (np.arange(np.floor(0.011 / nu), np.floor((p_z + tau) / nu) + 1) + 0.5) * nu
    np.testing.assert_allclose(zc, want, atol=1e-12)
    np.testing.assert_allclose(ext.D[upd], np.clip(p_z - c[upd, 2], -tau, tau), atol=1e-12)
    assert st["observations"] == upd.sum()


def test_lidar_point_order_independence(orc):
    """Eq. 3 and 5 give the same mean and variance whatever order a frame's observations arrive
    in: permuting the points leaves W identical and D, S2 equal to rounding."""
    from workloads import street_sequence

    pts, poses, _ = street_sequence(n_scans=1, rings=8, azimuths=256, scans=[3])
    cfg = dict(voxel=0.2, tau=0.6, min_range=1.0, max_range=40.0, carve=1)
    a = orc.OracleMap(**cfg)
    b = orc.OracleMap(**cfg)
    a.integrate_points(pts[0], poses[0])
    perm = np.random.default_rng(0).permutation(pts.shape[1])
    b.integrate_points(pts[0][perm], poses[0])
    ea, eb = a.extract(), b.extract()
    assert np.array_equal(ea.keys, eb.keys)
    assert np.array_equal(ea.W, eb.W)
    np.testing.assert_allclose(ea.D, eb.D, atol=1e-12)
    np.testing.assert_allclose(ea.S2, eb.S2, atol=1e-12)
    assert ea.W.max() > 20


def test_lidar_distinct_voxels_and_candidate_keys(orc):
    """The per-scan counts: the allocation visits, per valid ray, exactly the block cells its
    segment [o, p + tau n] meets (exact rational intersection), repeats across rays included; the
    update counts a voxel once however many rays cross it -- in a fresh single-level map W after
    one scan is the number of crossings, so the distinct voxels are those with W > 0 -- and a
    block once, every block a ray's walk allocates holding at least one voxel the ray crosses.
    Sending the scan twice doubles the visits and the observations but not the distinct voxels."""
    rng = np.random.default_rng(11)
    voxel, tau = 0.2, 0.6
    B = 8 * voxel
    n = 24
    dirs = rng.normal(size=(n, 3))
    dirs[:, 2] *= 0.3
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = (dirs * rng.uniform(2.0, 9.0, size=(n, 1))).astype(np.float32)
    pts[0] = [0.1, 0.2, 0.3]  # inside min_range: not valid, not walked
    T = np.eye(4)
    T[:3, 3] = [0.37, -1.21, 0.52]
    cfg = dict(voxel=voxel, tau=tau, min_range=1.0, max_range=40.0, carve=1)
    m = orc.OracleMap(**cfg)
    st = m.integrate_points(pts, T)
    want = 0
    for q in pts[1:].astype(np.float64):
        p = q + T[:3, 3]
        nn = (p - T[:3, 3]) / np.linalg.norm(p - T[:3, 3])
        want += len(_brute_cells(T[:3, 3] / B, (p + tau * nn) / B))
    assert st["valid_points"] == n - 1
    assert st["candidate_keys"] == want
    ext = m.extract()
    assert st["distinct_voxels"] == int((ext.W > 0).sum())
    assert st["observations"] == int(ext.W.sum()) > st["distinct_voxels"]  # rays share voxels near o
    observed = np.add.reduceat((ext.W > 0).astype(np.int64), ext.offsets[:-1]) > 0
    assert st["touched_blocks"] == int(observed.sum()) == st["new_blocks"]  # every walked block is observed
    m2 = orc.OracleMap(**cfg)
    st2 = m2.integrate_points(np.concatenate([pts, pts]), T)
    assert st2["candidate_keys"] == 2 * want
    assert st2["observations"] == 2 * st["observations"]
    assert st2["distinct_voxels"] == st["distinct_voxels"]


def test_rgbd_distinct_voxels_are_the_updates(orc):
    """A depth frame gives each voxel one pixel, so its distinct voxels are its observations; its
    allocation visits the block cells of every valid pixel's band [p - tau n, p + tau n]."""
    depth, _, T = plane_frame(1.37, width=16, height=12)
    K = np.array([9.0, 9.5, 7.63, 5.29])  # off-centre: no pixel ray runs along a block face
    voxel, tau = 0.05, 0.15
    m = orc.OracleMap(voxel=voxel, tau=tau, max_depth=10.0)
    st = m.integrate_depth(depth, K, T)
    ext = m.extract()
    assert st["distinct_voxels"] == st["observations"] == int((ext.W > 0).sum()) > 0
    observed = np.add.reduceat((ext.W > 0).astype(np.int64), ext.offsets[:-1]) > 0
    assert st["touched_blocks"] == int(observed.sum()) > 0
    fx, fy, cx, cy = K
    want = 0
    for v in range(depth.shape[0]):
        for u in range(depth.shape[1]):
            d = float(depth[v, u])
            ps = np.array([((u - cx) * (1.0 / fx)) * d, ((v - cy) * (1.0 / fy)) * d, d])
            nn = ps / np.linalg.norm(ps)
            want += len(_brute_cells((ps - tau * nn) / (8 * voxel), (ps + tau * nn) / (8 * voxel)))
    assert st["candidate_keys"] == want > st["new_blocks"] > 0


# ------------------------------------------------------------------------------------------
# merging criterion (Sec. 3.2.1): conservation and the constant-field case
# ------------------------------------------------------------------------------------------

def test_merge_conserves_weight_and_weighted_tsdf(orc):
    """Two noisy frames into a never-merging map (threshold 0) and an always-merging one
    (threshold huge): each merged block keeps its total weight, its sum of W D and its sum of S2,
    and each coarse voxel holds the weighted mean of its 8 children."""
    depth, cam, T = sphere_plane_frame(seed=5)
    d2, _, _ = sphere_plane_frame(seed=6)
    kw = dict(voxel=0.02, levels=4, tau=0.06, max_depth=10.0, min_obs=2)
    a = orc.OracleMap(var_thr=0.0, **kw)
    b = orc.OracleMap(var_thr=1e9, **kw)
    for m in (a, b):
        m.integrate_depth(depth, cam.K, T)
        m.integrate_depth(d2, cam.K, T)
    ea, eb = a.extract(), b.extract()
    assert np.array_equal(ea.keys, eb.keys)
    assert np.all(ea.levels == 0)
    merged = eb.levels == 1
    assert merged.sum() > 100
    assert set(np.unique(eb.levels)) <= {0, 1}  # one level per frame at most
    for i in np.flatnonzero(merged)[:400]:
        fa = slice(ea.offsets[i], ea.offsets[i + 1])
        fb = slice(eb.offsets[i], eb.offsets[i + 1])
        Wf, Df, Sf = ea.W[fa].astype(np.float64), ea.D[fa], ea.S2[fa]
        Wc, Dc, Sc = eb.W[fb].astype(np.float64), eb.D[fb], eb.S2[fb]
        assert Wf.sum() == Wc.sum()
        assert abs((Wf * Df).sum() - (Wc * Dc).sum()) < 1e-12
        assert abs(Sf.sum() - Sc.sum()) < 1e-12
        # child (2I+a, 2J+b, 2K+c) of coarse voxel (I, J, K); x fastest in both
        Wf3, Df3 = Wf.reshape(8, 8, 8), Df.reshape(8, 8, 8)
        Wg = Wf3.reshape(4, 2, 4, 2, 4, 2).sum(axis=(1, 3, 5))
        WDg = (Wf3 * Df3).reshape(4, 2, 4, 2, 4, 2).sum(axis=(1, 3, 5))
        np.testing.assert_array_equal(Wg.ravel(), Wc)
        want = np.divide(WDg, Wg, out=np.zeros_like(WDg), where=Wg > 0).ravel()
        np.testing.assert_allclose(Dc, want, atol=1e-12)
    # blocks that stayed fine in the merging map had no voxel with two observations
    for i in np.flatnonzero(~merged)[:400]:
        fb = slice(eb.offsets[i], eb.offsets[i + 1])
        assert eb.W[fb].max() < 2


def test_constant_field_merges_down_one_level_per_frame(orc):
    """The same noise-free plane every frame gives each fine voxel the same observation every time,
    so its variance is zero: blocks merge as soon as they have two observations, and then one
    level per frame (never more), down to the coarsest level."""
    nu, tau = 0.02, 0.06
    depth, cam, T = plane_frame(2.0, 32, 24, 24.0)
    m = orc.OracleMap(nu, levels=4, tau=tau, var_thr=1e-6, max_depth=5.0, form="zdiff")
    levels_seen = []
    for _ in range(5):
        m.integrate_depth(depth, cam.K, T)
        ext = m.extract()
        levels_seen.append(int(ext.levels.max()))
    assert levels_seen == [0, 1, 2, 3, 3]
    assert np.all(np.abs(ext.D) <= tau) and np.all(ext.S2 >= 0)


@pytest.mark.parametrize("side", [-1, 1])
def test_merge_threshold_at_closed_form_variance(orc, side):
    """Eq. 6 and the merging criterion (Sec. 3.2.1) at a closed form.  Two noise-free planes delta
    apart, each seen once by the same camera (z-difference form of Eq. 2), give every voxel that
    lies inside the band on both frames W = 2, S2 = delta^2 / 2 (Eq. 5) and sigma^2 = S2 / W =
    delta^2 / 4 (Eq. 6), so a block made only of such voxels has exactly that mean variance.  It
    merges after the second frame when the threshold lies just above delta^2 / 4 (side +1) and
    stays at the finest level just below it (side -1).  A variance taken as S2 / (W - 1), or a
    comparison the other way round, fails one of the two."""
    nu, tau, z0 = 0.02, 0.3, 2.0
    d1, cam, T = plane_frame(z0, 32, 24, 24.0)
    d2, _, _ = plane_frame(z0 + 0.02, 32, 24, 24.0)
    delta = float(d2[0, 0]) - float(d1[0, 0])
    var = delta * delta / 4.0
    maps = {}
    for name, thr in (("ref", 0.0), ("test", var * (1.0 + side * 1e-6))):
        m = orc.OracleMap(nu, levels=2, tau=tau, var_thr=thr, max_depth=5.0, form="zdiff")
        for d in (d1, d2):
            m.integrate_depth(d, cam.K, T)
        maps[name] = m.extract()
    ref, ext = maps["ref"], maps["test"]
    B = 8 * nu
    zlo = ref.keys[:, 2] * B
    # every voxel centre of the block within (d - z) in (-tau, tau) for both depths
    inside = (zlo + 0.5 * nu > float(d2[0, 0]) - tau + 1e-9) & (zlo + B - 0.5 * nu < float(d1[0, 0]) + tau - 1e-9)
    # blocks allocated by the first frame hold voxels seen twice (eligible); blocks first reached
    # by the second frame hold single observations only and are not eligible
    wmax = np.array([ref.W[ref.offsets[i]:ref.offsets[i + 1]].max() for i in range(len(ref.keys))])
    eligible = inside & (wmax == 2)
    assert eligible.sum() >= 8 and set(np.unique(ref.keys[eligible, 2]).tolist()) == {11, 12, 13}
    for i in np.flatnonzero(eligible):
        sl = slice(ref.offsets[i], ref.offsets[i + 1])
        seen = ref.W[sl] > 0
        assert np.all(ref.W[sl][seen] == 2)
        np.testing.assert_allclose(ref.S2[sl][seen], delta * delta / 2.0, rtol=1e-9)
    level = {tuple(k): int(lv) for k, lv in zip(ext.keys.tolist(), ext.levels)}
    want = 1 if side > 0 else 0
    got = [level[tuple(k)] for k in ref.keys[eligible].tolist()]
    assert got == [want] * len(got), (side, np.bincount(got))
    assert all(level[tuple(k)] == 0 for k in ref.keys[inside & (wmax < 2)].tolist())


def test_free_space_merges_to_constant(orc):
    """LiDAR carving: voxels far in front of the returns see the truncated value +tau on every
    beam (Eq. 1), so blocks of free space have zero variance, merge down to the coarsest level and
    hold exactly +tau."""
    from workloads import lidar_directions

    nu, tau = 0.05, 0.15
    d = lidar_directions(16, 64, -20.0, 20.0)
    d = d[d[:, 0] > 0.5]  # a forward fan of beams to a wall at x = 6 m
    pts = (d * (6.0 / d[:, :1])).astype(np.float32)
    m = orc.OracleMap(nu, levels=4, tau=tau, var_thr=1e-6, min_range=0.5, max_range=20.0, carve=1)
    for _ in range(4):
        m.integrate_points(pts, np.eye(4))
    ext = m.extract()
    B = 8 * nu
    lo = ext.keys[:, 0] * B
    free = (lo + B < 6.0 - tau - 1e-9) & (ext.keys[:, 0] >= 1)
    assert free.sum() > 20
    assert np.all(ext.levels[free] == 3)
    for i in np.flatnonzero(free):
        sl = slice(ext.offsets[i], ext.offsets[i + 1])
        assert ext.W[sl].min() > 0
        np.testing.assert_allclose(ext.D[sl], tau, rtol=0, atol=1e-15)
        np.testing.assert_allclose(ext.S2[sl], 0.0, rtol=0, atol=1e-15)


# ------------------------------------------------------------------------------------------
# trilinear query (Sec. 3.4) and its adjoint
# ------------------------------------------------------------------------------------------

def _plane_map(orc, Z0=1.5, frames=3, levels=1):
    Z0 = float(np.float32(Z0))
    depth, cam, T = plane_frame(Z0, 96, 72, 60.0)
    m = orc.OracleMap(0.02, levels=levels, tau=0.1, max_depth=5.0, form="zdiff", var_thr=0.0)
    for _ in range(frames):
        m.integrate_depth(depth, cam.K, T)
    return m


def test_trilinear_reproduces_linear_field(orc):
    """Inside the truncation band the z-difference TSDF of a plane is the linear field Z0 - z;
    trilinear interpolation reproduces linear fields exactly, so queries return Z0 - z and at
    voxel centres return the voxel's own value."""
    Z0 = float(np.float32(1.5))
    m = _plane_map(orc, Z0)
    rng = np.random.default_rng(3)
    pts = np.stack([rng.uniform(-0.3, 0.3, 2000), rng.uniform(-0.2, 0.2, 2000),
                    rng.uniform(Z0 - 0.06, Z0 + 0.06, 2000)], axis=1).astype(np.float32)
    sdf, valid, grad = m.query(pts, strict=True)
    assert valid.mean() > 0.95
    z = pts[valid, 2].astype(np.float64)
    np.testing.assert_allclose(sdf[valid], Z0 - z, atol=1e-12)
    np.testing.assert_allclose(grad[valid], np.tile([0.0, 0.0, -1.0], (valid.sum(), 1)), atol=1e-9)


def test_trilinear_across_levels_closed_form(orc):
    """Multi-resolution interpolation (Sec. 3.4, renormalised trilinear reading): the point's own
    block fixes the lattice, and each of the 8 lattice corners takes the TSDF of the voxel, at
    whatever level, whose half-open cell holds it.  Pinned on a map with two levels side by side:
    a noise-free fronto-parallel plane (z-difference form, so every observation is Z0 - z of the
    voxel centre, a linear field) seen twice by camera A, then once by camera B shifted along x.
    After A's two frames every observed voxel holds two equal observations (variance 0), so A's
    blocks merge one level; pooling a linear field over 8 children of equal weight gives the field
    at the coarse centre.  B's frame adds the coarse centre's own value to those blocks and
    allocates fine blocks where A never looked.  So every corner value is Z0 minus the z of its
    containing voxel's centre, and a query equals the trilinear blend of those values.  Only
    corners whose voxel is known to hold exactly that value are used (a fine voxel observed at
    least once; a coarse voxel whose 8 children were each seen twice by A, or that A never saw and
    B saw once), and the test needs queries whose corners span both levels, which is where
    indexing a corner's block on the wrong level's lattice fails."""
    nu, tau = 0.02, 0.3
    B = 8 * nu
    Z0 = float(np.float32(1.5))
    depth, cam, T0 = plane_frame(Z0, 96, 72, 60.0)
    T1 = np.eye(4)
    T1[0, 3] = 0.5
    m = orc.OracleMap(nu, levels=2, tau=tau, max_depth=5.0, form="zdiff", var_thr=1e-8, min_obs=2)
    for Tk in (T0, T0, T1):
        m.integrate_depth(depth, cam.K, Tk)
    ext = m.extract()
    assert set(np.unique(ext.levels).tolist()) == {0, 1}
    idx = {tuple(k): i for i, k in enumerate(ext.keys.tolist())}

    rng = np.random.default_rng(21)
    n = 20000
    # half of the points near A's right-hand field edge, where B's fine blocks meet A's coarse ones
    xs = np.concatenate([rng.uniform(-1.1, 1.6, n // 2), rng.uniform(0.8, 1.6, n - n // 2)])
    pts = np.stack([xs, rng.uniform(-0.6, 0.6, n), rng.uniform(Z0 - 0.12, Z0 + 0.12, n)],
                   axis=1).astype(np.float32)
    sdf, valid, _ = m.query(pts, strict=True)

    def corner_value(P):
        """(value, known) of the voxel holding lattice point P under the half-open convention."""
        cb = np.floor(P / B).astype(np.int64)
        i = idx.get(tuple(cb.tolist()))
        if i is None:
            return None, False
        lv = int(ext.levels[i])
        mm, nu_l = 8 >> lv, nu * (1 << lv)
        loc = np.floor((P - cb * B) / nu_l + 1e-9).astype(np.int64)
        v = int(ext.offsets[i] + loc[0] + mm * (loc[1] + mm * loc[2]))
        zc = cb[2] * B + (loc[2] + 0.5) * nu_l
        w = int(ext.W[v])
        known = (w >= 1) if lv == 0 else (w in (1, 16, 17))
        return Z0 - zc, known

    checked = mixed = 0
    for p, s, ok in zip(pts.astype(np.float64), sdf, valid):
        hb = idx.get(tuple(np.floor(p / B).astype(np.int64).tolist()))
        if hb is None:
            continue
        lv = int(ext.levels[hb])
        nu_l = nu * (1 << lv)
        g = p / nu_l - 0.5
        i0 = np.floor(g)
        f = g - i0
        want, lvls, usable = 0.0, set(), True
        for c in range(8):
            dl = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])
            val, known = corner_value((i0 + dl + 0.5) * nu_l)
            if not known:
                usable = False
                break
            w = np.prod(np.where(dl == 1, f, 1.0 - f))
            want += w * val
            lvls.add(int(ext.levels[idx[tuple(np.floor((i0 + dl + 0.5) * nu_l / B).astype(np.int64).tolist())]]))
        if not usable:
            continue
        assert ok
        assert abs(s - want) < 1e-12, (p, s, want)
        checked += 1
        mixed += len(lvls) > 1
    assert checked > 5000 and mixed > 300, (checked, mixed)


def test_query_pose_is_applied(orc):
    Z0 = float(np.float32(1.5))
    m = _plane_map(orc, Z0)
    T = np.eye(4)
    th = 0.3
    T[:3, :3] = [[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]]
    T[:3, 3] = [0.05, -0.02, 0.01]
    rng = np.random.default_rng(4)
    xw = np.stack([rng.uniform(-0.2, 0.2, 500), rng.uniform(-0.2, 0.2, 500),
                   rng.uniform(Z0 - 0.05, Z0 + 0.05, 500)], axis=1)
    p = ((xw - T[:3, 3]) @ T[:3, :3]).astype(np.float32)
    sdf, valid, _ = m.query(p, T=T, strict=True)
    xr = p.astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    np.testing.assert_allclose(sdf[valid], Z0 - xr[valid, 2], atol=1e-12)


@pytest.mark.parametrize("strict", [True, False])
def test_query_gradient_matches_finite_differences(orc, strict):
    """Noisy sphere-and-plane map: the analytic gradient matches central differences along each
    axis (points away from cell faces).  With all 8 corners present the interpolant is linear
    along each axis inside a cell, so the difference is exact to rounding; with missing corners
    the renormalised ratio is smooth and central differences agree to O(eps^2), so a smaller
    step is used there."""
    depth, cam, T = sphere_plane_frame(seed=0)
    m = orc.OracleMap(0.02, tau=0.06, max_depth=10.0)
    m.integrate_depth(depth, cam.K, T)
    rng = np.random.default_rng(9)
    pts = np.stack([rng.uniform(-0.4, 0.4, 3000), rng.uniform(-0.3, 0.3, 3000),
                    rng.uniform(1.9, 2.3, 3000)], axis=1)
    g = pts / 0.02 - 0.5
    fr = g - np.floor(g)
    keep = np.all((fr > 0.05) & (fr < 0.95), axis=1)
    pts = pts[keep].astype(np.float32)
    _, valid, grad = m.query(pts, strict=strict)
    eps = 1e-4 if strict else 1e-6  # the renormalised ratio has curvature where weights are small
    for ax in range(3):
        dp = np.zeros(3, np.float64)
        dp[ax] = eps
        # evaluate exactly at p +- eps in float64 by a pure-translation pose
        Tp, Tm = np.eye(4), np.eye(4)
        Tp[:3, 3], Tm[:3, 3] = dp, -dp
        sp, vp, _ = m.query(pts, T=Tp, strict=strict)
        sm, vm, _ = m.query(pts, T=Tm, strict=strict)
        ok = valid & vp & vm
        assert ok.sum() > 500
        fd = (sp - sm) / (2 * eps)
        if strict:
            np.testing.assert_allclose(grad[ok, ax], fd[ok], rtol=1e-6, atol=1e-8)
        else:
            np.testing.assert_allclose(grad[ok, ax], fd[ok], rtol=1e-4, atol=1e-6)


def test_query_backward_matches_pose_finite_differences(orc):
    """dL/dxi for L = sum_i g_i sdf(exp(xi) T p_i) against central differences of the left
    perturbation, and dL/dp against the chain rule through R."""
    depth, cam, T0 = sphere_plane_frame(seed=0)
    m = orc.OracleMap(0.02, tau=0.06, max_depth=10.0)
    m.integrate_depth(depth, cam.K, T0)
    th = np.deg2rad(2.0)
    T = np.eye(4)
    T[:3, :3] = [[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]]
    T[:3, 3] = [0.02, -0.01, 0.03]
    rng = np.random.default_rng(12)
    xw = np.stack([rng.uniform(-0.3, 0.3, 4000), rng.uniform(-0.25, 0.25, 4000),
                   rng.uniform(1.95, 2.2, 4000)], axis=1)
    # keep points whose cell and corner set stay fixed under the perturbations used below
    xr = ((xw - T[:3, 3]) @ T[:3, :3]).astype(np.float32).astype(np.float64) @ T[:3, :3].T + T[:3, 3]
    g = xr / 0.02 - 0.5
    fr = g - np.floor(g)
    p = ((xw - T[:3, 3]) @ T[:3, :3]).astype(np.float32)[np.all((fr > 0.03) & (fr < 0.97), axis=1)]
    sdf, valid, gradw = m.query(p, T=T, strict=True)
    gs = rng.normal(size=p.shape[0])

    def hat(w):
        return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])

    def exp_se3(xi):
        rho, phi = xi[:3], xi[3:]
        a = np.linalg.norm(phi)
        Kx = hat(phi / a) if a > 0 else np.zeros((3, 3))
        R = np.eye(3) + np.sin(a) * Kx + (1 - np.cos(a)) * Kx @ Kx
        E = np.eye(4)
        E[:3, :3] = R
        E[:3, 3] = rho  # first order in rho is all a central difference sees
        return E

    eps = 1e-4
    evals = []
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = eps
        evals.append((m.query(p, T=exp_se3(xi) @ T, strict=True), m.query(p, T=exp_se3(-xi) @ T, strict=True)))
    ok = valid.copy()
    for (sp, vp, _), (sm, vm, _) in evals:
        ok &= vp & vm
    assert ok.sum() > 1500
    gs = np.where(ok, gs, 0.0)
    gp, gpose = m.query_backward(p, gs, T=T, strict=True)
    np.testing.assert_allclose(gp[valid], (gs[valid, None] * gradw[valid]) @ T[:3, :3], atol=1e-12)
    fd = np.array([(gs[ok] * (sp[ok] - sm[ok])).sum() / (2 * eps) for (sp, _, _), (sm, _, _) in evals])
    np.testing.assert_allclose(gpose, fd, rtol=2e-3, atol=1e-3 * np.abs(fd).max())
