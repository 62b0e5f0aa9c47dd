"""Seeded synthetic sensor workloads shared by the tests, the bench and the smoke check.

This package only *generates inputs*: depth images and LiDAR scans ray-cast in closed form from
analytic scenes, plus the sensor poses.  It holds none of the fusion method's arithmetic (no
allocation, no TSDF update, no variance rule, no interpolation), so the CPU oracle and the HIP
library can both consume its arrays without sharing any code.
"""
from .scenes import (  # noqa: F401
    Pinhole,
    sphere_plane_frame,
    room_scene,
    room_sequence,
    street_scene,
    street_sequence,
    lidar_directions,
    plane_frame,
    surface_query_points,
    colour_image,
)
