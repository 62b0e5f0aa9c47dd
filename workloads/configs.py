"""Map parameters and input recipes of the standard workloads (configuration only).

* ``sphere_plane``: one 320x240 RGB-D frame, 2 cm voxels, single resolution, 2^16 hash slots.
* ``room``: 100-frame 640x480 RGB-D orbit of a 6 x 6 x 3 m room, 1/2/4/8 cm levels, truncation
  3 voxels, 5 m maximum depth, variance threshold (0.005 m)^2.
* ``street``: 200 LiDAR scans of 64 rings x 2048 azimuths along a 200 m street, 5/10/20/40 cm
  levels, truncation 3 voxels, carving, 1-80 m ranges, variance threshold (0.025 m)^2, 2^22 slots.
"""

SPHERE_PLANE = dict(voxel=0.02, levels=1, tau=0.06, max_depth=10.0, min_obs=2, var_thr=0.0,
                    max_blocks=1 << 15, hash_slots=1 << 16)

ROOM = dict(voxel=0.01, levels=4, tau=0.03, var_thr=0.005 ** 2, min_obs=2, max_depth=5.0,
            max_blocks=1 << 19, hash_slots=1 << 20)

STREET = dict(voxel=0.05, levels=4, tau=0.15, var_thr=0.025 ** 2, min_obs=2, min_range=1.0,
              max_range=80.0, carve=True, max_blocks=1 << 21, hash_slots=1 << 22)


def oracle_kwargs(cfg: dict) -> dict:
    """The subset of a map configuration the oracle takes."""
    keep = ("voxel", "levels", "tau", "var_thr", "min_obs", "max_depth", "min_range", "max_range",
            "carve", "form")
    out = {k: v for k, v in cfg.items() if k in keep}
    if "carve" in out:
        out["carve"] = int(out["carve"])
    return out
