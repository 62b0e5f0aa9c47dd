"""Capacity-driven streaming (Sec. 3.3) on the GPU: the blocks streamed out are exactly those the
oracle's region test puts outside the sensor region; a round trip through the host store is bit
exact; fusing a sequence with every frame's region streamed in first and streamed out after gives,
over GPU and store together, the map fused without streaming (bit for bit, and against the oracle);
a LiDAR street whose heaps hold only part of the map runs through with capacity-driven streaming."""
import numpy as np
import pytest
import torch

from parity_util import Sorted, announce, compare_maps, excused_keys, gpu_sorted
from workloads import configs, room_sequence, street_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _store_raw(fmap) -> Sorted:
    s = fmap.store_extract()  # ascending packed-key order
    return Sorted(s["keys"], s["levels"], s["offsets"], s["D"].astype(np.float64), s["W"], s["S2"].astype(np.float64))


def _store_sorted(fmap) -> Sorted:
    """The host store in ascending (x, y, z) order, like gpu_sorted."""
    empty = Sorted(np.zeros((0, 3), np.int32), np.zeros(0, np.uint8), np.zeros(1, np.int64), np.zeros(0), np.zeros(0, np.uint32),
                   np.zeros(0))
    return _union(_store_raw(fmap), empty)


def _union(a: Sorted, b: Sorted) -> Sorted:
    """Blocks of two disjoint block sets, in ascending (x, y, z) order."""
    keys = np.concatenate([a.keys, b.keys])
    assert len({tuple(k) for k in keys.tolist()}) == len(keys), "a block is both on the GPU and in the store"
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    parts = []
    for src in (a, b):
        for i in range(len(src.keys)):
            sl = slice(src.offsets[i], src.offsets[i + 1])
            parts.append((src.levels[i], src.D[sl], src.W[sl], src.S2[sl]))
    parts = [parts[i] for i in order]
    sizes = np.array([len(p[1]) for p in parts], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    cat = lambda j, dt: np.concatenate([p[j] for p in parts]).astype(dt) if parts else np.zeros(0, dt)
    return Sorted(keys[order], np.array([p[0] for p in parts], np.uint8), offs, cat(1, np.float64), cat(2, np.uint32),
                  cat(3, np.float64))


def _same(a: Sorted, b: Sorted):
    assert np.array_equal(a.keys, b.keys)
    assert np.array_equal(a.levels, b.levels)
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.W, b.W)
    assert np.array_equal(a.D, b.D)
    assert np.array_equal(a.S2, b.S2)


def _room(n=12):
    frames = list(range(0, 100, 8))[:n]
    depths, cam, poses, _ = room_sequence(width=320, height=240, f=262.5, frames=frames)
    return depths, cam, poses


ROOM = dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_stream_round_trip(mrh, orc, storage):
    announce(f"stream out / in round trip, room 320x240 x12, {storage}")
    depths, cam, poses = _room()
    g = mrh.Map(**dict(ROOM, storage=storage))
    for k in range(len(poses)):
        g.integrate_depth(_dev(depths[k]), cam.K, poses[k])
    g.sync()
    before = gpu_sorted(g)
    region = mrh.depth_region(320, 240, cam.K, poses[5])
    assert g.stream_out(region, threshold=1.01) == 0  # below the threshold nothing moves
    n_out = g.stream_out(region, threshold=0.0)
    kept, stored = gpu_sorted(g), _store_sorted(g)
    assert n_out == len(stored.keys) > 100 and len(kept.keys) > 100
    _same(_union(kept, stored), before)
    # the blocks that left are those the oracle's region test puts outside
    o = orc.OracleMap(**configs.oracle_kwargs(ROOM))
    inside, margin = o.region_holds(before.keys, "depth", poses[5], cam.K, 320, 240)
    on_gpu = {tuple(k) for k in kept.keys.tolist()}
    clear = np.abs(margin) > 1e-6
    got = np.array([tuple(k) in on_gpu for k in before.keys.tolist()])
    assert np.array_equal(got[clear], inside[clear])
    _, tot = g.sync()
    assert tot["blocks"] == len(kept.keys)
    # everything back: the map as it was, the store empty
    assert g.stream_in(mrh.points_region(np.eye(4), 1e6)) == n_out
    assert g.store_info()[0] == 0
    _same(gpu_sorted(g), before)


def test_stream_sequence_is_lossless(mrh, orc):
    announce("room 320x240 x12 with per-frame stream in / out against plain fusion and the oracle")
    depths, cam, poses = _room()
    plain, streamed = mrh.Map(**ROOM), mrh.Map(**ROOM)
    o = orc.OracleMap(**configs.oracle_kwargs(ROOM))
    moved_out = moved_in = 0
    for k in range(len(poses)):
        region = mrh.depth_region(320, 240, cam.K, poses[k])
        moved_in += streamed.stream_in(region)
        d = _dev(depths[k])
        streamed.integrate_depth(d, cam.K, poses[k])
        plain.integrate_depth(d, cam.K, poses[k])
        o.integrate_depth(depths[k], cam.K, poses[k])
        moved_out += streamed.stream_out(region, threshold=0.0)
    streamed.sync()
    plain.sync()
    print("moved out", moved_out, "moved back", moved_in)
    assert moved_out > 1000 and moved_in > 1000
    union = _union(gpu_sorted(streamed), _store_sorted(streamed))
    _same(union, gpu_sorted(plain))
    rep = compare_maps(union, o.extract(), tol_d=1e-5, excused=excused_keys(o), tau=ROOM["tau"])
    print(rep)


def test_stream_lidar_capacity(mrh):
    """A 60-scan street (16 x 512 rays, returns up to 10 m) whose coarsest heap holds 60% of the
    final map's coarsest blocks: without streaming it runs out; with capacity-driven streaming
    (threshold 0.5, a 12 m ball) it does not, and GPU and store together hold the map fused with
    unlimited heaps."""
    announce("street 16x512 x60 with heaps at 60% of the map, capacity-driven streaming")
    pts, poses, _ = street_sequence(rings=16, azimuths=512, scans=range(60))
    cfg = dict(configs.STREET, max_range=10.0, max_blocks=1 << 19, hash_slots=1 << 20)
    plain = mrh.Map(**cfg)
    new_max = 0
    for k in range(60):
        plain.integrate_points(_dev(pts[k]), poses[k])
        new_max = max(new_max, plain.sync()[0]["new_blocks"])
    full = gpu_sorted(plain)
    per_level = np.bincount(full.levels, minlength=4)
    # the coarsest heap (mostly carved free space) at 60% of the final map, so the map cannot fit
    # without streaming; the finer heaps, through which every block passes one level per scan, hold
    # their final count plus two scans of new blocks
    heaps = [int(c) + 2 * new_max for c in per_level[:3]] + [int(0.6 * per_level[3])]
    small = dict(cfg, heap_blocks=heaps)
    lim = mrh.Map(**small)
    with pytest.raises(mrh.MrhError):
        for k in range(60):
            lim.integrate_points(_dev(pts[k]), poses[k])
            lim.sync()
    g = mrh.Map(**small)
    outs = 0
    for k in range(60):
        region = mrh.points_region(poses[k], 12.0)
        g.stream_in(region)
        g.integrate_points(_dev(pts[k]), poses[k])
        try:
            g.sync()  # raises on a heap overflow
        except mrh.MrhError:
            print("scan", k, "usage", g.heap_usage(), "store", g.store_info(), "heaps", heaps, "final", per_level.tolist(),
                  "live", np.bincount(gpu_sorted(g).levels, minlength=4).tolist())
            raise
        outs += g.stream_out(region, threshold=0.5)
    print("per-level blocks", per_level.tolist(), "heaps", heaps, "streamed out", outs, "store", g.store_info())
    assert outs > 0
    _same(_union(gpu_sorted(g), _store_sorted(g)), full)


def test_load_blocks(mrh):
    announce("load_blocks from a store extract into a fresh map")
    depths, cam, poses = _room(6)
    g = mrh.Map(**ROOM)
    for k in range(len(poses)):
        g.integrate_depth(_dev(depths[k]), cam.K, poses[k])
    g.stream_out(mrh.points_region(np.eye(4), 0.0), threshold=0.0)  # everything to the store
    s = g.store_extract()
    h = mrh.Map(**ROOM)
    assert h.load_blocks(s["keys"], s["levels"], s["D"], s["W"], s["S2"]) == len(s["keys"])
    assert h.load_blocks(s["keys"][:10], s["levels"][:10], s["D"], s["W"], s["S2"]) == 0  # present already
    _same(gpu_sorted(h), _store_sorted(g))
