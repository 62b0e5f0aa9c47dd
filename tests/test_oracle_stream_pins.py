"""Pins of the oracle's streaming-region test (Sec. 3.3), against sampled geometry rather than its
own formula: every block holding a sampled point of the region is inside (the test is
conservative: a block seen by the sensor is never streamed out); a block declared outside has no
sampled point of its bounding sphere in the region (the test is sound); closed cases straight
ahead, behind, and past the range."""
import numpy as np

from workloads import configs
from workloads.scenes import look_at


def _map(orc):
    return orc.OracleMap(**configs.oracle_kwargs(configs.ROOM))  # 1 cm voxels, B = 8 cm, tau 3 cm


def _pose():
    return look_at(np.array([1.0, -2.0, 1.5]), np.array([3.0, 2.0, 0.8]))


def _frustum_points(rng, n, W, H, K, T, zmax):
    u = rng.uniform(-0.5, W - 0.5, n)
    v = rng.uniform(-0.5, H - 0.5, n)
    z = rng.uniform(1e-3, zmax, n)
    x = np.stack([z * (u - K[2]) / K[0], z * (v - K[3]) / K[1], z], axis=1)
    return x @ T[:3, :3].T + T[:3, 3]


def _in_frustum(p, W, H, K, T, rmax):
    x = (p - T[:3, 3]) @ T[:3, :3]
    z = x[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = K[0] * x[..., 0] / z + K[2]
        v = K[1] * x[..., 1] / z + K[3]
    return (z > 0) & (u >= -0.5) & (u <= W - 0.5) & (v >= -0.5) & (v <= H - 0.5) & (np.linalg.norm(x, axis=-1) <= rmax)


def _sphere_samples(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_region_frustum_conservative_and_sound(orc):
    rng = np.random.default_rng(3)
    o = _map(orc)
    W, H, K = 320, 240, np.array([262.5, 262.5, 160.0, 120.0])
    T = _pose()
    cfg = configs.ROOM
    B = 8 * cfg["voxel"]
    zmax = cfg["max_depth"] + cfg["tau"]
    pts = _frustum_points(rng, 4000, W, H, K, T, zmax)
    keys = np.floor(pts / B).astype(np.int32)
    inside, _ = o.region_holds(keys, "depth", T, K, W, H)
    assert inside.all()
    # blocks around the frustum: those declared outside have no point of their sphere inside
    ax = [(-0.5 - K[2]) / K[0], (W - 0.5 - K[2]) / K[0]]
    ay = [(-0.5 - K[3]) / K[1], (H - 0.5 - K[3]) / K[1]]
    lam = max(np.sqrt(1 + a * a + b * b) for a in ax for b in ay)
    cand = np.unique(np.floor((_frustum_points(rng, 3000, W * 1.6, H * 1.6, np.array([K[0], K[1], K[2] * 1.6, K[3] * 1.6]),
                                                T, zmax * 1.3) + rng.normal(0, 0.3, (3000, 3))) / B).astype(np.int32), axis=0)
    inside, margin = o.region_holds(cand, "depth", T, K, W, H)
    assert (~inside).sum() > 100 and inside.sum() > 100
    rb = 0.5 * np.sqrt(3) * B
    dirs = _sphere_samples(rng, 4000)
    for k in cand[~inside]:
        c = (k + 0.5) * B
        assert not _in_frustum(c + rb * dirs, W, H, K, T, lam * zmax).any(), k


def test_region_ball_conservative_and_sound(orc):
    rng = np.random.default_rng(4)
    o = _map(orc)
    T = _pose()
    R, B = 2.5, 0.08
    d = _sphere_samples(rng, 5000) * (R * rng.uniform(0, 1, (5000, 1)) ** (1 / 3))
    keys = np.floor((T[:3, 3] + d) / B).astype(np.int32)
    inside, _ = o.region_holds(keys, "points", T, radius=R)
    assert inside.all()
    cand = np.unique(np.floor((T[:3, 3] + _sphere_samples(rng, 3000) * rng.uniform(R - 0.5, R + 0.5, (3000, 1))) / B)
                     .astype(np.int32), axis=0)
    inside, margin = o.region_holds(cand, "points", T, radius=R)
    assert (~inside).sum() > 100 and inside.sum() > 100
    rb = 0.5 * np.sqrt(3) * B
    dirs = _sphere_samples(rng, 4000)
    for k, mg in zip(cand[~inside], margin[~inside]):
        c = (k + 0.5) * B
        assert np.linalg.norm(c + rb * dirs - T[:3, 3], axis=1).min() > R
    # a clearly inside block has a point of its sphere in the ball
    for k in cand[inside & (margin > 0.01 * rb)]:
        c = (k + 0.5) * B
        assert np.linalg.norm(c + rb * dirs - T[:3, 3], axis=1).min() <= R


def test_region_closed_cases(orc):
    o = _map(orc)
    W, H, K = 320, 240, np.array([262.5, 262.5, 160.0, 120.0])
    T = np.eye(4)
    T[:3, 3] = [0.04, 0.04, 0.04]  # camera at a block centre, looking along +z
    B = 0.08
    ahead = np.array([[0, 0, 25]])        # 2 m straight ahead
    behind = np.array([[0, 0, -25]])      # 2 m behind
    far = np.array([[0, 0, 100]])         # 8 m ahead, past lambda (5 m + 3 cm)
    side = np.array([[40, 0, 5]])         # 3.2 m to the side at 0.4 m depth
    for k, want in ((ahead, True), (behind, False), (far, False), (side, False)):
        assert o.region_holds(k, "depth", T, K, W, H)[0][0] == want, k
    assert o.region_holds(np.array([[0, 0, 12]]), "points", T, radius=1.0)[0][0]
    assert not o.region_holds(np.array([[0, 0, 14]]), "points", T, radius=1.0)[0][0]
