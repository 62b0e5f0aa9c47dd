"""The map's bookkeeping (Sec. 3.1: the spatial hash of Eq. 4 from keys to blocks, the per-level
heaps whose slots the blocks hold) after fusion, merging and streaming, read back by the library's
consistency check: the counts it reports equal what the frames' statistics and the extraction say
they must be."""
import numpy as np
import pytest
import torch

from parity_util import announce, assert_consistent, gpu_sorted
from workloads import configs, room_sequence

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


ROOM = dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)


def test_check_counts_follow_the_frames(mrh):
    """Per frame: the table holds one key per block row; the slots a frame's merges free wait on
    the pending lists (merges out of level n free one level-n slot each); every other slot of a
    level is held by a block of that level or on the free stack."""
    announce("map check: room 320x240 x8 frames, 4 levels")
    frames = list(range(0, 64, 8))
    depths, cam, poses, _ = room_sequence(width=320, height=240, f=262.5, frames=frames)
    g = mrh.Map(**ROOM)
    cap = ROOM["max_blocks"]  # no per-level heap sizes: every heap holds max_blocks blocks
    merged = 0
    for k in range(len(frames)):
        g.integrate_depth(_dev(depths[k]), cam.K, poses[k])
        last, tot = g.sync()
        c = assert_consistent(g)
        assert c["blocks"] == tot["blocks"] == c["live_blocks"] == c["table_keys"], k
        assert c["tombstones"] == c["gone_blocks"] == c["slotless_blocks"] == 0, k
        for n in range(3):
            assert c["pending_slots"][n] == last["merges"][n], (k, n)
        merged += sum(last["merges"])
        held = np.bincount(gpu_sorted(g).levels, minlength=4)
        for n in range(4):
            assert held[n] + c["free_slots"][n] + c["pending_slots"][n] == cap, (k, n)
        assert 1.0 <= c["mean_probe"] <= c["max_probe"], k
    assert merged > 100


def test_check_after_streaming(mrh):
    """Streaming a block out leaves a tombstone in its table slot and its row marked gone, and
    returns its heap slot to the free stack; streaming it back inserts the key again with a new
    row (tombstones are not reused), so the map stays consistent throughout."""
    announce("map check: stream out / in, room 320x240 x6 frames")
    frames = list(range(0, 48, 8))
    depths, cam, poses, _ = room_sequence(width=320, height=240, f=262.5, frames=frames)
    g = mrh.Map(**ROOM)
    for k in range(len(frames)):
        g.integrate_depth(_dev(depths[k]), cam.K, poses[k])
    g.sync()
    c0 = assert_consistent(g)
    n_out = g.stream_out(mrh.depth_region(320, 240, cam.K, poses[2]), threshold=0.0)
    assert n_out > 100
    c1 = assert_consistent(g)
    assert c1["tombstones"] == c1["gone_blocks"] == n_out
    assert c1["table_keys"] == c0["table_keys"] - n_out
    assert c1["live_blocks"] == c0["live_blocks"] - n_out
    assert sum(c1["free_slots"]) == sum(c0["free_slots"]) + n_out
    assert g.stream_in(mrh.points_region(np.eye(4), 1e6)) == n_out
    c2 = assert_consistent(g)
    assert c2["tombstones"] == c2["gone_blocks"] == n_out
    assert c2["blocks"] == c0["blocks"] + n_out
    assert c2["table_keys"] == c0["table_keys"] and c2["live_blocks"] == c0["live_blocks"]
    assert c2["free_slots"] == c0["free_slots"]


def test_extract_blocks_buffer_too_small(mrh):
    """mrh_extract_blocks refuses buffers smaller than the map (MRH_ERR_BUFFER_TOO_SMALL, -5) before
    writing anything, with both counts still set; exact sizes succeed and match the count call."""
    import ctypes

    from workloads import sphere_plane_frame

    announce("extract: buffer-too-small path, sphere-plane frame")
    depth, cam, T = sphere_plane_frame(seed=0)
    g = mrh.Map(**configs.SPHERE_PLANE)
    g.integrate_depth(_dev(depth), cam.K, T)
    g.sync()
    nb, nv = g.counts()
    assert nb > 100 and nv == nb * 512
    L = mrh._lib.load()
    keys = torch.empty((nb, 3), dtype=torch.int32, device="cuda")
    levels = torch.empty(nb, dtype=torch.uint8, device="cuda")
    offs = torch.empty(nb + 1, dtype=torch.int64, device="cuda")
    D = torch.empty(nv, dtype=torch.float32, device="cuda")
    W = torch.empty(nv, dtype=torch.int32, device="cuda")
    S2 = torch.empty(nv, dtype=torch.float32, device="cuda")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    a, b = ctypes.c_int64(-1), ctypes.c_int64(-1)
    # one block short
    st = L.mrh_extract_blocks(g._h, ptr(keys), ptr(levels), None, None, None, None, nb - 1, 0, ctypes.byref(a),
                              ctypes.byref(b))
    assert st == -5 and (a.value, b.value) == (nb, nv)
    # one voxel short (the block capacity is enough)
    a.value = b.value = -1
    st = L.mrh_extract_blocks(g._h, ptr(keys), ptr(levels), ptr(offs), ptr(D), ptr(W), ptr(S2), nb, nv - 1,
                              ctypes.byref(a), ctypes.byref(b))
    assert st == -5 and (a.value, b.value) == (nb, nv)
    assert "extract needs" in L.mrh_last_error(g._h).decode()
    # exact sizes
    st = L.mrh_extract_blocks(g._h, ptr(keys), ptr(levels), ptr(offs), ptr(D), ptr(W), ptr(S2), nb, nv,
                              ctypes.byref(a), ctypes.byref(b))
    assert st == 0 and (a.value, b.value) == (nb, nv)
    assert int(offs[-1].item()) == nv
    e = g.extract()
    assert torch.equal(e["keys"], keys) and torch.equal(e["W"], W)
