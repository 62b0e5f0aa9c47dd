"""The synthetic room's exact signed distance, used as ground truth for query-error measurements,
checked against the scene's ray caster (the nearest hit over many directions from a free-space
point is at least the distance to the nearest surface and approaches it) and against points
sampled on the surfaces."""
import numpy as np

from workloads import surface_query_points
from workloads.scenes import room_scene


def _directions(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_room_sdf_against_ray_casting():
    scene = room_scene(1)
    rng = np.random.default_rng(11)
    dirs = _directions(40000, 12)
    pts = rng.uniform([0.2, 0.2, 0.2], [5.8, 5.8, 2.8], size=(40, 3))
    d = scene.sdf(pts)
    free = d > 0.02
    assert free.sum() >= 20
    for p, dp in zip(pts[free], d[free]):
        hit = scene.raycast(p, dirs).min()  # one origin shared by every ray
        assert hit >= dp - 1e-9, (p, hit, dp)
        assert hit <= dp * 1.01 + 1e-4, (p, hit, dp)


def test_room_sdf_on_sampled_surfaces():
    scene = room_scene(1)
    on = surface_query_points(scene, 20000, sigma=0.0, seed=5).astype(np.float64)
    d0 = scene.sdf(on)
    # a surface point is never in free space (FP32 rounding of the points aside); the few below
    # zero lie on faces buried inside another obstacle
    assert d0.max() <= 1e-6
    visible = np.abs(d0) <= 1e-6
    assert visible.mean() > 0.98
    pts, off = surface_query_points(scene, 20000, sigma=0.01, seed=5, with_offsets=True)
    d = scene.sdf(pts.astype(np.float64))
    front = visible & (off > 0)
    # moved off a visible surface into free space: no farther from the surfaces than the offset,
    # and equal to it away from edges and corners
    assert np.all(d[front] <= off[front] + 1e-6)
    assert np.mean(np.abs(d[front] - off[front]) <= 1e-5) > 0.98
