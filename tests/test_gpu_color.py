"""Colour integration on the GPU (mrh_integrate_rgbd) against the oracle's: the same blocks, levels,
weights and TSDF as without colour, and every voxel's colour within FP32 rounding of the oracle's
(running means of the pixel colours, pooled by weight when blocks merge), on the 4-level room."""
import numpy as np
import pytest
import torch

from parity_util import announce, compare_maps, excused_keys, gpu_sorted
from workloads import colour_image, configs, room_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sorted_colour(fmap):
    """gpu_sorted of the map plus its colours in the same voxel order."""
    e = fmap.extract(voxels=True)
    col = fmap.extract_color().cpu().numpy().astype(np.float64)
    keys = e["keys"].cpu().numpy()
    offs = e["offsets"].cpu().numpy()
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    sizes = np.diff(offs)[order]
    starts = offs[:-1][order]
    idx = np.repeat(starts - np.concatenate([[0], np.cumsum(sizes)[:-1]]), sizes) + np.arange(sizes.sum())
    return gpu_sorted(fmap), col[idx]


ROOM = dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)


def test_colour_matches_oracle(mrh, orc):
    announce("colour room 320x240 x12, 4 levels, against the oracle")
    frames = list(range(0, 100, 8))[:12]
    depths, cam, poses, _ = room_sequence(width=320, height=240, f=262.5, frames=frames)
    g = mrh.Map(**dict(ROOM, color=True))
    plain = mrh.Map(**ROOM)
    o = orc.OracleMap(**configs.oracle_kwargs(ROOM))
    for k in range(len(frames)):
        rgb = colour_image(depths[k], cam, poses[k])
        g.integrate_rgbd(_dev(depths[k]), _dev(rgb), cam.K, poses[k])
        plain.integrate_depth(_dev(depths[k]), cam.K, poses[k])
        o.integrate_rgbd(depths[k], rgb, cam.K, poses[k])
    g.sync()
    gs, gc = _sorted_colour(g)
    ps = gpu_sorted(plain)
    for a, b in ((gs.keys, ps.keys), (gs.levels, ps.levels), (gs.W, ps.W), (gs.D, ps.D), (gs.S2, ps.S2)):
        assert np.array_equal(a, b)  # colour does not touch the fusion
    ex = o.extract()
    excused = excused_keys(o)
    rep = compare_maps(gs, ex, tol_d=1e-5, excused=excused, tau=ROOM["tau"])
    oc = o.extract_color()
    keep = (gs.levels == ex.levels) & np.array([tuple(k) not in excused for k in ex.keys.tolist()])
    gi = np.concatenate([np.arange(gs.offsets[i], gs.offsets[i + 1]) for i in np.flatnonzero(keep)])
    oi = np.concatenate([np.arange(ex.offsets[i], ex.offsets[i + 1]) for i in np.flatnonzero(keep)])
    seen = ex.W[oi] > 0
    d = np.abs(gc[gi][seen] - oc[oi][seen])
    coarse = np.repeat(ex.levels, np.diff(ex.offsets))[oi][seen] > 0
    print(rep, "colour voxels", int(seen.sum()), "coarse", int(coarse.sum()), "max |dC|", float(d.max()))
    assert coarse.sum() > 1000
    assert d.max() <= 2e-3


def test_colour_maps_reject_other_paths(mrh):
    announce("colour maps: other fusion paths refused")
    frames = [0]
    depths, cam, poses, _ = room_sequence(width=64, height=48, f=52.5, frames=frames)
    g = mrh.Map(**dict(ROOM, color=True))
    with pytest.raises(mrh.MrhError):
        g.integrate_depth(_dev(depths[0]), cam.K, poses[0])
    with pytest.raises(mrh.MrhError):
        g.integrate_points(torch.zeros((4, 3), device="cuda"), np.eye(4))
    plain = mrh.Map(**ROOM)
    with pytest.raises(mrh.MrhError):
        plain.integrate_rgbd(_dev(depths[0]), _dev(np.zeros((48, 64, 3), np.uint8)), cam.K, poses[0])
    with pytest.raises(mrh.MrhError):
        mrh.Map(**dict(ROOM, color=True, min_obs=1))
