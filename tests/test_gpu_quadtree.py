"""Image quadtree by contrast on the GPU (Eq. 10, Algorithm 1) against the oracle: the same leaves
(sorted), contrast within FP32 rounding, on images of several sizes (odd, thin, and the 640x480 and
1200x680 frame sizes of the paper's RGB-D data) at several thresholds and minimum sizes."""
import numpy as np
import pytest
import torch

import oracle
from parity_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _image(rng, h, w, patch=8, noise=25.0):
    smooth = rng.integers(0, 256, (h // patch + 2, w // patch + 2, 3)).repeat(patch, 0).repeat(patch, 1)[:h, :w]
    return np.clip(smooth + rng.normal(0, noise, (h, w, 3)), 0, 255).astype(np.uint8)


CASES = [(37, 53, 300.0, 3, 8), (64, 48, 800.0, 2, 4), (100, 7, 50.0, 1, 8), (480, 640, 400.0, 4, 16),
         (680, 1200, 250.0, 8, 32), (480, 640, 1e9, 4, 16), (480, 640, 0.0, 1, 16)]


def test_quadtree_matches_oracle(mrh):
    rng = np.random.default_rng(1)
    qt = mrh.Quadtree(1200, 680)
    for h, w, thr, mn, patch in CASES:
        announce(f"quadtree {w}x{h} threshold {thr} min {mn}")
        img = _image(rng, h, w, patch)
        want, wc, near = oracle.quadtree(img, thr, mn)
        assert near == 0
        leaves, con = qt.build(torch.from_numpy(img).cuda(), thr, mn)
        got = leaves.cpu().numpy()
        gc = con.cpu().numpy().astype(np.float64)
        go, oo = np.lexsort(got.T[::-1]), np.lexsort(want.T[::-1])
        assert np.array_equal(got[go], want[oo]), (w, h, thr, len(got), len(want))
        assert np.allclose(gc[go], wc[oo], rtol=1e-5, atol=1e-3)
        print(w, h, thr, mn, "leaves", len(got))
    qt.close()


def test_quadtree_small_buffer(mrh):
    import ctypes

    announce("quadtree buffer too small")
    img = torch.from_numpy(_image(np.random.default_rng(2), 64, 64)).cuda()
    qt = mrh.Quadtree(64, 64)
    leaves, _ = qt.build(img, 100.0, 2)
    L = mrh._lib.load()
    buf = torch.empty((2, 4), dtype=torch.int32, device="cuda")
    n = ctypes.c_int64()
    st = L.mrh_quadtree_build(qt._h, ctypes.c_void_p(img.data_ptr()), 64, 64, 100.0, 2, ctypes.c_void_p(buf.data_ptr()),
                              None, 2, ctypes.byref(n))
    assert st == -5 and n.value == leaves.shape[0] > 2
    assert L.mrh_quadtree_build(qt._h, ctypes.c_void_p(img.data_ptr()), 65, 64, 100.0, 2, None, None, 0, ctypes.byref(n)) == -1
    assert L.mrh_quadtree_build(qt._h, ctypes.c_void_p(img.data_ptr()), 64, 64, 100.0, 0, None, None, 0, ctypes.byref(n)) == -1
    qt.close()
