"""The RGB-D entry point that allocates nothing (mrh_integrate_depth_noalloc) against the ordinary
one (mrh_integrate_depth): two calls in a row, the second with a smaller frame, through the C ABI;
the two maps must be identical after each call (same kernels, the tile summary only moved)."""
import numpy as np
import pytest
import torch

from parity_util import announce, gpu_sorted
from workloads import configs, room_sequence

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert np.array_equal(a.keys, b.keys)
    assert np.array_equal(a.levels, b.levels)
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.W, b.W)
    assert np.array_equal(a.D, b.D)
    assert np.array_equal(a.S2, b.S2)


def test_noalloc_matches_integrate_depth():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    announce("no-allocation RGB-D entry point: 640x480 then 320x240 against mrh_integrate_depth")
    big = room_sequence(width=640, height=480, f=525.0, frames=[0])
    small = room_sequence(width=320, height=240, f=262.5, frames=[40])
    cfg = dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)
    ref = mrh.Map(**cfg)
    got = mrh.Map(**cfg)
    for depths, cam, poses, _ in (big, small):
        d = torch.from_numpy(np.ascontiguousarray(depths[0])).cuda()
        ref.integrate_depth(d, cam.K, poses[0])
        got.integrate_depth_noalloc(d, cam.K, poses[0])
        lr, _ = ref.sync()
        lg, _ = got.sync()
        assert lr == lg
        assert lr["observations"] > 0
        _same(gpu_sorted(got), gpu_sorted(ref))
    # a frame above the fixed tile capacity is refused before anything is launched
    with pytest.raises(mrh.MrhError) as ei:
        L = mrh._lib.load()
        import ctypes

        K = (ctypes.c_double * 4)(*big[1].K)
        T = (ctypes.c_double * 16)(*np.asarray(big[2][0], np.float64).ravel())
        st = L.mrh_integrate_depth_noalloc(got._h, ctypes.c_void_p(d.data_ptr()), 4112, 4096, K, T)
        got._check(st, "mrh_integrate_depth_noalloc")
    assert ei.value.code == -1
    assert "4096" in str(ei.value)
    got.close()
    ref.close()
