"""Pins of the oracle's multi-resolution Marching Cubes (Sec. 3.4) against what geometry fixes:

* linear fields: every vertex lies on the field's zero plane (trilinear interpolation and linear
  edge interpolation reproduce a linear field exactly), on one level and across a boundary between
  two levels in both orders (finer block after a coarser one: the coarse cubes are truncated;
  coarser after finer: the fine cubes are stretched);
* the cubes partition space: the signed area of a horizontal plane's mesh projected on the ground
  equals the area between the outermost voxel centres, with two levels side by side;
* closed surfaces: the mesh of a sphere's exact signed distance is watertight (every directed edge
  has its reverse exactly once), has Euler characteristic 2, faces outward, and its vertices lie
  within the trilinear edge-interpolation bound nu^2 / (8 (R - 2 nu)) of the sphere;
* every one of the 256 corner-sign cases: a random-sign field meshes without cracks between cubes;
* the vertex collapse: no vertex lies closer than collapse * nu to a lattice point unless it sits on
  one, and no triangle is degenerate."""
import numpy as np
import pytest


def _blocks_map(orc, levels=4, voxel=0.01, tau=0.05):
    return orc.OracleMap(voxel=voxel, levels=levels, tau=tau)


def _centres(key, level, voxel):
    m = 8 >> level
    nu = voxel * (1 << level)
    B = 8 * voxel
    idx = np.arange(m)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")  # x fastest after ravel
    return (key[0] * B + (i + 0.5) * nu, key[1] * B + (j + 0.5) * nu, key[2] * B + (k + 0.5) * nu)


def _put(o, key, level, voxel, field, tau=0.05):
    x, y, z = _centres(key, level, voxel)
    d = np.clip(field(x, y, z), -tau, tau)
    o.set_block(key, level, d.ravel(), np.ones(d.size, np.uint32))


def _edge_check(V, interior=None):
    """Directed-edge multiset of a triangle soup: edges without exactly one reverse."""
    q = np.round(V * 1e8).astype(np.int64)
    edges = {}
    for t in q:
        ks = [tuple(p) for p in t]
        for a in range(3):
            e = (ks[a], ks[(a + 1) % 3])
            edges[e] = edges.get(e, 0) + 1
    bad = []
    for e, c in edges.items():
        if interior is not None and not (interior(np.array(e[0]) / 1e8) and interior(np.array(e[1]) / 1e8)):
            continue
        if c != 1 or edges.get((e[1], e[0]), 0) != 1:
            bad.append(e)
    verts = {p for e in edges for p in e}
    return bad, len(verts), len(edges)


def test_mesh_plane_single_level(orc):
    n = np.array([0.36, -0.48, 0.8])  # unit normal
    c = 0.013
    field = lambda x, y, z: n[0] * x + n[1] * y + n[2] * z - c
    o = _blocks_map(orc)
    for bx in range(-2, 2):
        for by in range(-2, 2):
            for bz in range(-2, 2):
                _put(o, (bx, by, bz), 0, 0.01, field)
    ms = o.mesh(0.0)
    assert len(ms.codes) > 500
    V = ms.verts
    assert np.abs(V @ n - c).max() < 1e-12
    nrm = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    area2 = np.linalg.norm(nrm, axis=1)
    keep = area2 > 1e-12
    assert np.allclose(nrm[keep] / area2[keep, None], n, atol=1e-9)  # faces point to D > 0


@pytest.mark.parametrize("level", [0, 1])
def test_mesh_sphere_closed(orc, level):
    R, voxel, tau = 0.3, 0.01, 0.05
    nu = voxel * (1 << level)
    o = _blocks_map(orc, tau=tau)
    field = lambda x, y, z: np.sqrt(x * x + y * y + z * z) - R
    for bx in range(-6, 6):
        for by in range(-6, 6):
            for bz in range(-6, 6):
                _put(o, (bx, by, bz), level, voxel, field, tau)
    ms = o.mesh(0.0)
    V = ms.verts
    bad, nv, ne = _edge_check(V)
    assert not bad
    assert nv - ne // 2 + len(V) == 2
    r = np.linalg.norm(V, axis=2)
    assert np.abs(r - R).max() <= nu * nu / (8 * (R - 2 * nu)) * (1 + 1e-9)
    nrm = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    assert np.all(np.sum(nrm * V.mean(axis=1), axis=1) > 0)


def test_mesh_every_sign_case_is_crack_free(orc):
    rng = np.random.default_rng(5)
    voxel = 0.01
    o = _blocks_map(orc, tau=10.0)
    keys = [(bx, by, bz) for bx in range(2) for by in range(2) for bz in range(2)]
    cases = set()
    vals = {}
    for key in keys:
        v = np.where(rng.random(512) < 0.5, -1.0, 1.0)
        vals[key] = v.reshape(8, 8, 8)
        o.set_block(key, 0, v, np.ones(512, np.uint32))
    full = np.zeros((16, 16, 16))
    for (bx, by, bz), v in vals.items():
        full[bz * 8:bz * 8 + 8, by * 8:by * 8 + 8, bx * 8:bx * 8 + 8] = v
    for k in range(15):
        for j in range(15):
            for i in range(15):
                c = 0
                for q in range(8):
                    if full[k + (q >> 2 & 1), j + (q >> 1 & 1), i + (q & 1)] < 0:
                        c |= 1 << q
                cases.add(c)
    assert len(cases) == 256
    ms = o.mesh(0.0)
    lo, hi = 0.5 * voxel, 15.5 * voxel  # the outer faces of the meshed region are open
    interior = lambda p: np.all(p > lo + 1e-9) and np.all(p < hi - 1e-9)
    bad, _, _ = _edge_check(ms.verts, interior)
    assert not bad


@pytest.mark.parametrize("order", ["coarse_then_fine", "fine_then_coarse"])
def test_mesh_level_boundary_partition(orc, order):
    voxel, z0 = 0.01, 0.0437
    B = 8 * voxel
    o = _blocks_map(orc)
    field = lambda x, y, z: z0 - z
    xs = range(-2, 2)
    lv = {bx: (1 if (bx < 0) == (order == "coarse_then_fine") else 0) for bx in xs}
    for bx in xs:
        for by in range(0, 2):
            _put(o, (bx, by, 0), lv[bx], voxel, field)
    ms = o.mesh(0.0)
    V = ms.verts
    assert np.abs(V[:, :, 2] - z0).max() < 1e-12
    # signed area on the ground plane (faces point to D > 0, i.e. downwards)
    e1, e2 = V[:, 1] - V[:, 0], V[:, 2] - V[:, 0]
    signed = -0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    assert np.all(signed > -1e-15)
    # cubes run from the first voxel centre of the lowest block to the last of the highest; a cube
    # on a face between levels ends on the first centre plane of the next block
    nu = lambda level: voxel * (1 << level)
    area = 0.0
    for bx in xs:
        x0 = bx * B + (nu(lv[bx]) / 2 if bx == xs[0] else nu(lv[bx - 1]) / 2 * 0 + 0)
        x_lo = bx * B + nu(lv[bx]) / 2 if bx == xs[0] else bx * B + nu(lv[bx]) / 2
        x_hi = (bx + 1) * B + nu(lv[bx + 1]) / 2 if bx + 1 in lv else (bx + 1) * B - nu(lv[bx]) / 2
        y_lo, y_hi = nu(lv[bx]) / 2, 2 * B - nu(lv[bx]) / 2
        area += (x_hi - x_lo) * (y_hi - y_lo)
    assert abs(signed.sum() - area) < 1e-12


def test_mesh_collapse(orc):
    R, voxel, tau, kappa = 0.3, 0.01, 0.05, 0.2
    o = _blocks_map(orc, tau=tau)
    field = lambda x, y, z: np.sqrt(x * x + y * y + z * z) - R
    for bx in range(-6, 6):
        for by in range(-6, 6):
            for bz in range(-6, 6):
                _put(o, (bx, by, bz), 0, voxel, field, tau)
    plain = o.mesh(0.0)
    ms = o.mesh(kappa)
    V = ms.verts.reshape(-1, 3)
    g = V / voxel - 0.5  # voxel centres at integers
    frac = np.abs(g - np.round(g))
    # a vertex lies on an edge between two centres: two coordinates on the lattice, the third at
    # distance t nu from the lower centre; either on a centre or at least kappa nu from both
    off = np.sort(frac, axis=1)[:, 2] * voxel
    assert np.all(np.sort(frac, axis=1)[:, :2] < 1e-9)
    assert np.all((off < 1e-9) | (off >= kappa * voxel - 1e-12))
    assert np.any(off < 1e-9)
    T = ms.verts
    assert np.all(np.linalg.norm(T[:, 0] - T[:, 1], axis=1) > 0)
    assert np.all(np.linalg.norm(T[:, 1] - T[:, 2], axis=1) > 0)
    assert np.all(np.linalg.norm(T[:, 0] - T[:, 2], axis=1) > 0)
    assert len(ms.codes) < len(plain.codes)
