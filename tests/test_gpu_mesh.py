"""Multi-resolution Marching Cubes on the GPU (mrh_extract_mesh) against the oracle's mesh of the
oracle's own fused map (Sec. 3.4): the same triangles cube by cube (block key, voxel and the
vertex ids of each triangle: which cube edge, collapsed corner or loop centre each vertex is on)
and vertex positions within FP32 rounding.  Cubes whose decisions the oracle took within rounding
of a threshold (a corner value within 1e-6 m of zero, a collapse within 1e-6 nu of its distance,
a crossing with corner values within 1 mm of each other) are left out on both sides, and so are
the 27-block neighbourhoods of blocks whose merge decision was excused (their levels may differ)."""
import numpy as np
import pytest
import torch

from parity_util import announce, excused_keys
from workloads import configs, room_sequence, sphere_plane_frame

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mrh():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_21459_amd as mrh

    return mrh


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _canon(blocks, codes, verts):
    """Per triangle: (bx, by, bz, level, voxel, a, b, c) with the vertex ids rotated so that the
    smallest comes first (orientation kept), and the vertices in the same rotation."""
    codes = codes.astype(np.uint64)
    ids = np.stack([(codes >> 10) & 31, (codes >> 5) & 31, codes & 31], axis=1).astype(np.int64)
    r = np.argmin(ids, axis=1)
    order = (r[:, None] + np.arange(3)[None, :]) % 3
    ids = np.take_along_axis(ids, order, axis=1)
    verts = np.take_along_axis(verts, order[:, :, None], axis=1)
    key = np.concatenate([blocks.astype(np.int64), (codes >> 30)[:, None].astype(np.int64),
                          ((codes >> 15) & 0x7FFF)[:, None].astype(np.int64), ids], axis=1)
    return key, verts


def _cube_ids(key):
    return [tuple(k) for k in key[:, :5].tolist()]


def _excluded_blocks(o, g_levels_by_key, o_ex):
    """Blocks within one block of a block whose level differs between the two maps."""
    bad = set()
    for k, lv in zip(o_ex.keys.tolist(), o_ex.levels.tolist()):
        if g_levels_by_key.get(tuple(k), lv) != lv:
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        bad.add((k[0] + dx, k[1] + dy, k[2] + dz))
    return bad


def compare_meshes(g, om, skip_blocks=frozenset(), only_blocks=None):
    gk, gv = _canon(g["blocks"].cpu().numpy(), g["codes"].cpu().numpy().view(np.uint32),
                    g["verts"].cpu().numpy().astype(np.float64))
    ok, ov = _canon(om.blocks, om.codes, om.verts)
    near_cubes = set(_cube_ids(ok[om.near]))
    def keep(key):
        cubes = _cube_ids(key)
        blocks = [c[:3] for c in cubes]
        m = np.array([c not in near_cubes and b not in skip_blocks and (only_blocks is None or b in only_blocks)
                      for c, b in zip(cubes, blocks)], bool)
        return m
    gm, omk = keep(gk), keep(ok)
    gk, gv, ok, ov = gk[gm], gv[gm], ok[omk], ov[omk]
    go = np.lexsort(gk.T[::-1])
    oo = np.lexsort(ok.T[::-1])
    gk, gv, ok, ov = gk[go], gv[go], ok[oo], ov[oo]
    assert gk.shape == ok.shape, (gk.shape, ok.shape)
    assert np.array_equal(gk, ok), "triangle sets differ"
    d = np.abs(gv - ov)
    tol = 1e-5 + 1e-6 * np.abs(ov)
    worst = np.unravel_index(np.argmax(d / tol), d.shape)
    assert np.all(d <= tol), (d[worst], ov[worst])
    return {"triangles": int(len(gk)), "near_excluded": int(om.near.sum()), "max_abs_dv": float(d.max()) if d.size else 0.0}


def _levels_by_key(fmap):
    e = fmap.extract(voxels=False)
    return {tuple(k): int(l) for k, l in zip(e["keys"].cpu().numpy().tolist(), e["levels"].cpu().numpy().tolist())}


@pytest.mark.parametrize("collapse", [0.0, 0.1])
def test_mesh_sphere_plane(mrh, orc, collapse):
    announce(f"mesh sphere_plane collapse={collapse}")
    depth, cam, T = sphere_plane_frame(seed=0)
    g = mrh.Map(**configs.SPHERE_PLANE)
    g.integrate_depth(_dev(depth), cam.K, T)
    g.sync()
    o = orc.OracleMap(**configs.oracle_kwargs(configs.SPHERE_PLANE))
    o.integrate_depth(depth, cam.K, T)
    gm = g.mesh(collapse)
    om = o.mesh(collapse)
    rep = compare_meshes(gm, om)
    print(rep)
    assert rep["triangles"] > 10000


@pytest.mark.parametrize("collapse", [0.0, 0.1])
def test_mesh_room_multires(mrh, orc, collapse):
    """12 frames of the 4-level room at 320x240: meshes across level boundaries (truncated and
    stretched cubes, corners interpolated on other levels) and collapse."""
    announce(f"mesh room 320x240 x12 4 levels collapse={collapse}")
    frames = list(range(0, 100, 8))[:12]
    depths, cam, poses, _ = room_sequence(width=320, height=240, f=262.5, frames=frames)
    cfg = dict(configs.ROOM, max_blocks=1 << 17, hash_slots=1 << 18)
    o = orc.OracleMap(**configs.oracle_kwargs(cfg))
    g = mrh.Map(**cfg)
    for k in range(len(frames)):
        o.integrate_depth(depths[k], cam.K, poses[k])
        g.integrate_depth(_dev(depths[k]), cam.K, poses[k])
    g.sync()
    ex = o.extract()
    assert len(set(ex.levels.tolist())) >= 3
    skip = _excluded_blocks(o, _levels_by_key(g), ex)
    # the oracle meshes a sample of blocks (all of it takes minutes): 1200 blocks with a face
    # neighbour on another level, 600 others
    lv = {tuple(k): int(l) for k, l in zip(ex.keys.tolist(), ex.levels.tolist())}
    trans = [k for k in lv if any(lv.get((k[0] + (a == 0), k[1] + (a == 1), k[2] + (a == 2)), lv[k]) != lv[k]
                                  for a in range(3))]
    rest = [k for k in lv if k not in set(trans)]
    rng = np.random.default_rng(11)
    pick = [trans[i] for i in rng.choice(len(trans), min(1200, len(trans)), replace=False)]
    pick += [rest[i] for i in rng.choice(len(rest), 600, replace=False)]
    om = o.mesh(collapse, only_keys=np.array(pick, np.int32))
    rep = compare_meshes(g.mesh(collapse), om, skip_blocks=skip, only_blocks=set(pick))
    print(rep, "blocks skipped", len(skip), "transition blocks", len(trans))
    assert rep["triangles"] > 20000


def test_mesh_count_and_small_buffer(mrh):
    announce("mesh buffer too small")
    depth, cam, T = sphere_plane_frame(seed=0)
    g = mrh.Map(**configs.SPHERE_PLANE)
    g.integrate_depth(_dev(depth), cam.K, T)
    full = g.mesh(0.0)
    n = full["verts"].shape[0]
    import ctypes

    L = mrh._lib.load()
    v = torch.empty((100, 3, 3), dtype=torch.float32, device="cuda")
    cnt = ctypes.c_int64()
    st = L.mrh_extract_mesh(g._h, 0.0, ctypes.c_void_p(v.data_ptr()), None, None, 100, ctypes.byref(cnt))
    assert st == -5 and cnt.value == n
    assert L.mrh_extract_mesh(g._h, 0.7, None, None, None, 0, ctypes.byref(cnt)) == -1
    e = mrh.Map(**configs.SPHERE_PLANE)
    assert e.mesh(0.0)["verts"].shape[0] == 0
