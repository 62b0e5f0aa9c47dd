"""Helpers shared by the GPU parity tests: bring a GPU map into the oracle's order and compare."""
from __future__ import annotations

import sys
from dataclasses import dataclass

import numpy as np


def announce(msg: str):
    """Name the GPU case about to run (flushed, so a dying run still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@dataclass
class Sorted:
    keys: np.ndarray
    levels: np.ndarray
    offsets: np.ndarray
    D: np.ndarray
    W: np.ndarray
    S2: np.ndarray


def assert_consistent(fmap) -> dict:
    """The map's bookkeeping checks out: every key once in the hash table and reachable from its
    home slot, table and block rows agree, and each heap's slots are held, free or pending exactly
    once."""
    c = fmap.check()
    assert c["consistent"], c
    assert c["live_blocks"] + c["slotless_blocks"] + c["gone_blocks"] == c["blocks"], c
    assert c["table_keys"] == c["blocks"] - c["gone_blocks"] + c["idless_keys"], c
    return c


def gpu_sorted(fmap) -> Sorted:
    """Extract a GPU map (after checking its bookkeeping) and order its blocks by ascending
    (x, y, z) like the oracle."""
    assert_consistent(fmap)
    e = fmap.extract(voxels=True)
    keys = e["keys"].cpu().numpy()
    levels = e["levels"].cpu().numpy()
    offs = e["offsets"].cpu().numpy()
    D = e["D"].cpu().numpy().astype(np.float64)
    W = e["W"].cpu().numpy().view(np.uint32)
    S2 = e["S2"].cpu().numpy().astype(np.float64)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    sizes = np.diff(offs)[order]
    starts = offs[:-1][order]
    idx = np.repeat(starts - np.concatenate([[0], np.cumsum(sizes)[:-1]]), sizes) + np.arange(sizes.sum())
    new_offs = np.concatenate([[0], np.cumsum(sizes)])
    return Sorted(keys[order], levels[order], new_offs, D[idx], W[idx], S2[idx])


def excused_keys(orc_map, margin: float = 1e-3) -> set:
    """Blocks whose merge decision the oracle took within `margin` (relative) of the threshold:
    FP32 state decides such blocks within rounding, 1e-3; 16-bit state within its precision."""
    keys, _, margins = orc_map.near_threshold()
    return {tuple(k) for k, mg in zip(keys.tolist(), margins.tolist()) if mg < margin}


def compare_maps(g: Sorted, o, tol_d: float = 1e-5, excused: set | None = None, tau: float = 0.15) -> dict:
    """Bit-exact block keys; equal levels except for blocks whose merge decision the oracle took
    within rounding of the threshold; on every other block W exactly equal and |dD| <= tol_d.

    S2 is checked against the FP32 accumulation bound: each of the W updates adds a term of
    magnitude at most (2 tau)^2 and rounds it at FP32 precision, so |dS2| <= 1e-5 |S2| +
    W (2 tau)^2 2^-20."""
    excused = excused or set()
    assert g.keys.shape == o.keys.shape, (g.keys.shape, o.keys.shape)
    assert np.array_equal(g.keys, o.keys), "block key sets differ"
    lv_ok = g.levels == o.levels
    bad = [tuple(k) for k in o.keys[~lv_ok].tolist() if tuple(k) not in excused]
    assert not bad, f"{len(bad)} blocks at different levels, e.g. {bad[:5]}"
    keep = lv_ok & np.array([tuple(k) not in excused for k in o.keys.tolist()], dtype=bool)
    assert np.array_equal(g.offsets[1:][keep] - g.offsets[:-1][keep], o.offsets[1:][keep] - o.offsets[:-1][keep])
    gi = np.concatenate([np.arange(g.offsets[i], g.offsets[i + 1]) for i in np.flatnonzero(keep)] or [np.zeros(0, int)])
    oi = np.concatenate([np.arange(o.offsets[i], o.offsets[i + 1]) for i in np.flatnonzero(keep)] or [np.zeros(0, int)])
    Wg, Wo = g.W[gi], o.W[oi]
    nW = int(np.count_nonzero(Wg != Wo))
    assert nW == 0, f"{nW} voxels with different weights"
    obs = Wo > 0
    dD = np.abs(g.D[gi] - o.D[oi])[obs]
    dmax = float(dD.max()) if dD.size else 0.0
    assert dmax <= tol_d, f"max |dD| = {dmax}"
    s2g, s2o = g.S2[gi][obs], o.S2[oi][obs]
    ds2 = np.abs(s2g - s2o)
    bound = 1e-5 * np.abs(s2o) + Wo[obs].astype(np.float64) * (2 * tau) ** 2 * 2.0 ** -20
    worst = int(np.argmax(ds2 / bound)) if ds2.size else 0
    assert np.all(ds2 <= bound), (f"|dS2| = {ds2[worst]} at S2 = {s2o[worst]}, W = {Wo[obs][worst]}")
    return {"blocks": int(len(o.keys)), "compared_blocks": int(keep.sum()), "excused": int((~keep).sum()),
            "observed_voxels": int(obs.sum()), "max_abs_dD": dmax,
            "rms_dD": float(np.sqrt(np.mean(dD ** 2))) if dD.size else 0.0,
            "max_abs_dS2": float(ds2.max()) if ds2.size else 0.0}
