"""Pins of the oracle's colour integration (Sec. 3: a voxel stores a colour, averaged like the TSDF):
a constant colour image leaves exactly that colour on every observed voxel; a colour image that is a
function of the pixel column leaves on each voxel the value of the column its centre projects to
(the Eq. 2 pixel rule); and sum over voxels of W C grows by each frame's observation count times its
colour and is kept by merges (a running mean with the wrong weight, or pooling with the wrong
weights, breaks it)."""
import numpy as np

from workloads import configs, room_sequence
from workloads.scenes import plane_frame


def _oracle(orc, **kw):
    return orc.OracleMap(**configs.oracle_kwargs(dict(configs.ROOM, **kw)))


def test_constant_colour(orc):
    depths, cam, poses, _ = room_sequence(width=160, height=120, f=131.25, frames=[0, 10, 20])
    o = _oracle(orc)
    rgb = np.empty(depths.shape[1:] + (3,), np.uint8)
    rgb[...] = (10, 200, 77)
    for k in range(3):
        o.integrate_rgbd(depths[k], rgb, cam.K, poses[k])
    ex = o.extract()
    col = o.extract_color()
    seen = ex.W > 0
    assert seen.sum() > 10000
    assert np.all(col[seen] == np.array([10.0, 200.0, 77.0]))


def test_colour_follows_the_pixel(orc):
    depth, cam, T = plane_frame(1.0, width=200, height=40, f=100.0)
    rgb = np.zeros((40, 200, 3), np.uint8)
    rgb[:, :, 0] = np.arange(200, dtype=np.uint8)[None, :]
    o = orc.OracleMap(voxel=0.01, levels=1, tau=0.03, max_depth=5.0, form="zdiff")
    o.integrate_rgbd(depth, rgb, cam.K, T)
    ex = o.extract()
    col = o.extract_color()
    B = 0.08
    checked = 0
    for b, (k, off) in enumerate(zip(ex.keys, ex.offsets[:-1])):
        idx = np.arange(512)
        i, j, kk = idx % 8, (idx // 8) % 8, idx // 64
        x = k[0] * B + (i + 0.5) * 0.01
        z = k[2] * B + (kk + 0.5) * 0.01
        u = np.floor(cam.fx * (x / z) + cam.cx + 0.5)
        w = ex.W[off:off + 512] > 0
        assert np.all(col[off:off + 512][w, 0] == u[w])
        checked += int(w.sum())
    assert checked > 5000


def test_weighted_colour_is_conserved_through_merges(orc):
    depth, cam, T = plane_frame(2.0, width=64, height=48, f=60.0)
    o = orc.OracleMap(voxel=0.01, levels=4, tau=0.03, var_thr=1.0, min_obs=2, max_depth=5.0)
    colours = [(250, 0, 10), (0, 128, 30), (40, 40, 255), (7, 99, 3), (200, 200, 200), (1, 2, 3)]
    want = np.zeros(3)
    merges = 0
    for c in colours:
        rgb = np.empty((48, 64, 3), np.uint8)
        rgb[...] = c
        st = o.integrate_rgbd(depth, rgb, cam.K, T)
        want += st["observations"] * np.array(c, np.float64)
        merges += sum(st["merges"])
    ex = o.extract()
    col = o.extract_color()
    got = (ex.W[:, None].astype(np.float64) * col).sum(axis=0)
    assert merges > 0 and len(set(ex.levels.tolist())) > 1
    assert np.allclose(got, want, rtol=1e-12, atol=1e-6)
