"""Batched fusion of independent maps: results identical to fusing each map alone (the per-map
work is the same and deterministic), with and without graph replay; the autotuner resets maps."""
import numpy as np
import pytest
import torch

from parity_util import announce, compare_maps, excused_keys, gpu_sorted
from workloads import configs, room_sequence, sphere_plane_frame, street_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _streams(host=False):
    """Two RGB-D rooms of different sizes, one sphere-plane, two LiDAR streets of different sizes.
    With host=True the frames hold the numpy arrays (for the oracle) instead of device tensors."""
    dev = (lambda a: a) if host else _dev
    r1 = room_sequence(width=320, height=240, f=262.5, frames=[0, 3, 6], scene_seed=101, noise_seed=201)
    r2 = room_sequence(width=416, height=312, f=341.25, frames=[0, 3, 6], scene_seed=102, noise_seed=202)
    sp = sphere_plane_frame(seed=3)
    s1 = street_sequence(rings=16, azimuths=512, scans=[0, 1, 2], scene_seed=103, noise_seed=203)
    s2 = street_sequence(rings=8, azimuths=1024, scans=[5, 6, 7], scene_seed=104, noise_seed=204)
    room_cfg = dict(configs.ROOM, max_blocks=1 << 16, hash_slots=1 << 17)
    street_cfg = dict(configs.STREET, max_blocks=1 << 18, hash_slots=1 << 19)
    cfgs = [room_cfg, room_cfg, configs.SPHERE_PLANE, street_cfg, street_cfg]
    frames = []
    for k in range(3):
        fr = [("depth", dev(r1[0][k]), r1[1].K, r1[2][k]),
              ("depth", dev(r2[0][k]), r2[1].K, r2[2][k]),
              ("depth", dev(sp[0]), sp[1].K, sp[2]) if k != 1 else None,
              ("points", dev(s1[0][k]), s1[1][k]),
              ("points", dev(s2[0][k]), s2[1][k])]
        frames.append(fr)
    return cfgs, frames


_COUNTS = ("valid_points", "dropped_points", "new_blocks", "observations", "fresh_observations",
           "distinct_voxels", "candidate_keys", "merges")


def _single(mrh, cfg, frames_of_map, storage="f32", totals=None):
    m = mrh.Map(**dict(cfg, storage=storage))
    for fr in frames_of_map:
        if fr is None:
            continue
        if fr[0] == "depth":
            m.integrate_depth(fr[1], fr[2], fr[3])
        else:
            m.integrate_points(fr[1], fr[2])
    _, tot = m.sync()
    if totals is not None:
        totals.update(tot)
    return gpu_sorted(m)


def _same(a, b):
    assert np.array_equal(a.keys, b.keys)
    assert np.array_equal(a.levels, b.levels)
    assert np.array_equal(a.W, b.W)
    assert np.array_equal(a.D, b.D)
    assert np.array_equal(a.S2, b.S2)


@pytest.mark.parametrize("graph,waves", [(True, 4), (False, 4), (True, 1), (True, 2)])
def test_batch_equals_single_maps(mrh, graph, waves):
    """Every map of the batch equals the map fused alone, whatever the graph replay and the waves
    per update workgroup."""
    announce(f"batch of 5 maps (3 RGB-D, 2 LiDAR), graph={graph}, {waves} waves per update workgroup")
    cfgs, frames = _streams()
    maps = [mrh.Map(**c) for c in cfgs]
    b = mrh.Batch(maps)
    b.set_launch(512 * 4 // waves, 16, graph, waves)
    assert b.get_launch() == (512 * 4 // waves, 16, int(graph), waves)
    for fr in frames:
        b.integrate(fr)
    for i, c in enumerate(cfgs):
        _, tb = maps[i].sync()
        ts = {}
        _same(gpu_sorted(maps[i]), _single(mrh, c, [fr[i] for fr in frames], totals=ts))
        for name in _COUNTS:  # the batched launches keep each map's statistics
            assert tb[name] == ts[name], (i, name)


def _oracle_map(orc, cfg, frames_of_map):
    o = orc.OracleMap(**configs.oracle_kwargs(cfg))
    for fr in frames_of_map:
        if fr is None:
            continue
        if fr[0] == "depth":
            o.integrate_depth(fr[1], fr[2], fr[3])
        else:
            o.integrate_points(fr[1], fr[2])
    return o


def test_batch_maps_match_oracle(mrh, orc):
    """Every map of a batched run (graph replay, 3 calls over 3 RGB-D and 2 LiDAR maps of uneven
    sizes, one call without a sphere-plane frame) against the FP64 oracle fed the same frames: bit-exact
    block keys, equal levels (merge decisions at the threshold excused), W exact, |dD| <= 1e-5 m."""
    announce("batch of 5 maps against the oracle")
    cfgs, frames = _streams()
    _, host = _streams(host=True)
    maps = [mrh.Map(**c) for c in cfgs]
    b = mrh.Batch(maps)
    b.set_launch(512, 16, True)
    for fr in frames:
        b.integrate(fr)
    for i, c in enumerate(cfgs):
        maps[i].sync()
        o = _oracle_map(orc, c, [fr[i] for fr in host])
        rep = compare_maps(gpu_sorted(maps[i]), o.extract(), tol_d=1e-5, excused=excused_keys(o), tau=c["tau"])
        print(i, rep)
        assert rep["compared_blocks"] > 0


def test_batch_rejects_maps_on_different_streams(mrh):
    announce("batch of maps bound to different streams")
    a = mrh.Map(**configs.SPHERE_PLANE)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b = mrh.Map(**configs.SPHERE_PLANE)
    with pytest.raises(mrh.MrhError) as ei:
        mrh.Batch([a, b])
    assert ei.value.code == -1
    torch.cuda.synchronize()
    a.close()
    b.close()


def test_batch_f16_equals_single_f16(mrh):
    announce("batch f16")
    cfgs, frames = _streams()
    maps = [mrh.Map(**dict(c, storage="f16")) for c in cfgs]
    b = mrh.Batch(maps)
    for fr in frames:
        b.integrate(fr)
    for i, c in enumerate(cfgs):
        maps[i].sync()
        _same(gpu_sorted(maps[i]), _single(mrh, c, [fr[i] for fr in frames], storage="f16"))


def test_batch_autotune_resets_maps(mrh):
    announce("batch autotune")
    cfgs, frames = _streams()
    maps = [mrh.Map(**c) for c in cfgs]
    b = mrh.Batch(maps)
    best = b.autotune(frames[0], reps=2)
    assert best[3] in (1, 2, 4) and best[0] * best[3] // 4 in (256, 512, 1024, 2048, 4096)
    assert best[1] in (16, 64) and best[2] == 1
    assert b.get_launch() == best
    for m in maps:
        assert m.counts() == (0, 0)
    for fr in frames:
        b.integrate(fr)
    for i, c in enumerate(cfgs):
        maps[i].sync()
        _same(gpu_sorted(maps[i]), _single(mrh, c, [fr[i] for fr in frames]))


@pytest.mark.parametrize("graph", [True, False])
def test_batch_steps_of_one_frame_kind(mrh, graph):
    """Steps whose frames are all RGB-D, then all LiDAR, then mixed: each step launches only the
    update kernels of the kinds present (and a new graph when the kinds change)."""
    announce(f"batch steps of one frame kind, graph={graph}")
    cfgs, frames = _streams()
    kinds = [("depth",), ("points",), ("depth", "points")]
    steps = [[fr if fr is not None and fr[0] in kinds[k] else None for fr in frames[k]] for k in range(3)]
    maps = [mrh.Map(**c) for c in cfgs]
    b = mrh.Batch(maps)
    b.set_launch(256, 16, graph)
    for fr in steps:
        b.integrate(fr)
    for i, c in enumerate(cfgs):
        maps[i].sync()
        _same(gpu_sorted(maps[i]), _single(mrh, c, [fr[i] for fr in steps]))


def _device_sorted(m):
    """Block codes, levels and voxel planes of a map on the device, blocks in key order (the voxels
    of each block in their stored order)."""
    e = m.extract()
    k = e["keys"].to(torch.int64)
    code = ((k[:, 0] + (1 << 20)) << 42) | ((k[:, 1] + (1 << 20)) << 21) | (k[:, 2] + (1 << 20))
    order = torch.argsort(code)
    offs = e["offsets"]
    lens = (offs[1:] - offs[:-1])[order]
    starts = offs[:-1][order]
    first = torch.cumsum(lens, 0) - lens
    idx = torch.repeat_interleave(starts - first, lens) + torch.arange(int(lens.sum()), device=lens.device)
    return code[order], e["levels"][order], e["D"][idx], e["W"][idx], e["S2"][idx]


def _full_size_streams(L, host=False):
    from bench import LIDAR_STREAMS, RGBD_STREAMS

    dev = (lambda a: a) if host else _dev
    streams = []
    for i, (w, h) in enumerate(RGBD_STREAMS):
        d, cam, P, _ = room_sequence(width=w, height=h, f=525.0 * w / 640.0, frames=range(L), scene_seed=100 + i,
                                     noise_seed=200 + i)
        streams.append(([("depth", dev(d[k]), cam.K, P[k]) for k in range(L)],
                        dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)))
    for i, (r, a) in enumerate(LIDAR_STREAMS):
        p, P, _ = street_sequence(rings=r, azimuths=a, scans=range(L), scene_seed=108 + i, noise_seed=208 + i)
        nb = 1 << 20
        streams.append(([("points", dev(p[k]), P[k]) for k in range(L)],
                        dict(configs.STREET, max_blocks=nb, hash_slots=2 * nb, heap_blocks=[nb // 2, nb // 2, nb // 2, nb])))
    return streams


def test_batch_full_size_step_matches_oracle(mrh, orc):
    """One batched FP32 graph step of the benchmark's 16 full-size streams (8 RGB-D rooms 320x240 ..
    640x480, 8 LiDAR streets 32x1024 .. 64x2048): every map against the FP64 oracle."""
    announce("batch of the 16 full-size benchmark streams, 1 launch, against the oracle")
    streams = _full_size_streams(1)
    host = _full_size_streams(1, host=True)
    maps = [mrh.Map(**c) for _, c in streams]
    b = mrh.Batch(maps)
    b.set_launch(512, 16, True)
    b.integrate([fr[0] for fr, _ in streams])
    b.close()
    for i, (m, (frs, c)) in enumerate(zip(maps, host)):
        m.sync()
        o = _oracle_map(orc, c, frs)
        rep = compare_maps(gpu_sorted(m), o.extract(), tol_d=1e-5, excused=excused_keys(o), tau=c["tau"])
        print(i, rep)
        assert rep["compared_blocks"] > 100
        m.close()


def test_batch_full_size_streams(mrh):
    """The benchmark's 16 streams (8 RGB-D 320x240 .. 640x480 rooms, 8 LiDAR 32x1024 .. 64x2048
    streets, the same map configurations), two launches of the batched FP32 graph path: every map
    equals the same frames fused map by map, bit for bit."""
    announce("batch of the 16 full-size benchmark streams, 2 launches, FP32 graph")
    L = 2
    streams = _full_size_streams(L)
    maps = [mrh.Map(**c) for _, c in streams]
    b = mrh.Batch(maps)
    b.set_launch(512, 16, True)
    for k in range(L):
        b.integrate([fr[k] for fr, _ in streams])
    b.close()
    for m, (frs, c) in zip(maps, streams):
        m.sync()
        s = mrh.Map(**c)
        for fr in frs:
            if fr[0] == "depth":
                s.integrate_depth(fr[1], fr[2], fr[3])
            else:
                s.integrate_points(fr[1], fr[2])
        s.sync()
        got, want = _device_sorted(m), _device_sorted(s)
        assert got[0].numel() > 1000
        for a, w in zip(got, want):
            assert torch.equal(a, w)
        s.close()
        m.close()
