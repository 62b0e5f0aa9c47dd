"""Pins of the oracle's image quadtree (Sec. 3.5, Eq. 10, Algorithm 1): a flat image stays one leaf
of zero contrast; two flat halves give the closed-form contrast l . (a - b)^2 / 4; a checkerboard of
2 x 2 squares splits down to the minimum size everywhere; on random images the leaves tile the
image exactly, every leaf is below the threshold or at the minimum size, and each leaf's contrast
equals Eq. 10 evaluated on its pixels by NumPy."""
import numpy as np

import oracle

L = np.array([0.2989, 0.5870, 0.1140])


def _eq10(rgb, x, y, w, h):
    q = rgb[y:y + h, x:x + w].reshape(-1, 3).astype(np.float64)
    return float(L @ q.var(axis=0))


def test_flat_image():
    rgb = np.full((48, 64, 3), 77, np.uint8)
    leaves, con, near = oracle.quadtree(rgb, 1.0, 2)
    assert leaves.tolist() == [[0, 0, 64, 48]] and con[0] == 0.0 and near == 0


def test_two_halves_closed_form():
    rgb = np.zeros((32, 64, 3), np.uint8)
    rgb[:, :32] = (200, 10, 50)
    rgb[:, 32:] = (20, 110, 250)
    a, b = np.array([200, 10, 50.0]), np.array([20, 110, 250.0])
    want = float(L @ ((a - b) ** 2 / 4))
    leaves, con, _ = oracle.quadtree(rgb, want * 2, 4)  # above the root's contrast: one leaf
    assert len(leaves) == 1 and abs(con[0] - want) < 1e-9 * want
    leaves, con, _ = oracle.quadtree(rgb, want / 2, 4)  # below: split once into flat quadrants
    assert sorted(leaves.tolist()) == [[0, 0, 32, 16], [0, 16, 32, 16], [32, 0, 32, 16], [32, 16, 32, 16]]
    assert np.all(con == 0.0)


def test_checkerboard_to_minimum():
    yy, xx = np.mgrid[0:64, 0:64]
    rgb = np.where((((yy // 2) + (xx // 2)) % 2 == 0)[..., None], 255, 0).astype(np.uint8).repeat(3, axis=2)
    leaves, con, _ = oracle.quadtree(rgb, 1.0, 2)
    assert len(leaves) == 32 * 32 and np.all(leaves[:, 2:] == 2) and np.all(con == 0.0)


def test_random_images_tile_and_obey_the_rule():
    rng = np.random.default_rng(0)
    for (h, w, thr, mn) in ((37, 53, 300.0, 3), (64, 48, 800.0, 2), (100, 7, 50.0, 1)):
        smooth = rng.integers(0, 256, (h // 8 + 2, w // 8 + 2, 3)).repeat(8, 0).repeat(8, 1)[:h, :w]
        rgb = np.clip(smooth + rng.normal(0, 25, (h, w, 3)), 0, 255).astype(np.uint8)
        leaves, con, near = oracle.quadtree(rgb, thr, mn)
        assert near == 0
        cover = np.zeros((h, w), np.int32)
        for (x, y, lw, lh), c in zip(leaves.tolist(), con):
            cover[y:y + lh, x:x + lw] += 1
            assert abs(c - _eq10(rgb, x, y, lw, lh)) <= 1e-9 * max(1.0, c)
            assert c <= thr or min(lw, lh) <= mn
        assert np.all(cover == 1)
