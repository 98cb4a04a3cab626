"""Seeded synthetic inputs (scenes, camera sets, ray masks) shared by the HIP
path's tests/bench and by the CPU oracle's tests.

This package holds input construction only: random draws, camera placement and
array layout.  It contains none of the method's arithmetic (no projection, no
compositing, no sensitivities, no sampling).
"""
from .scenes import (Scene, Views, make_tiny_scene, make_tiny_views,
                     make_cluster_scene, make_orbit_views, make_config,
                     look_at, ray_subsample_mask, block_subsample_mask, splitmix64, SH_C0,
                     pack_bits, unpack_bits, make_explicit_scene,
                     make_camera_set, make_batch_specs, make_batch, make_pose_region)

__all__ = ["Scene", "Views", "make_tiny_scene", "make_tiny_views",
           "make_cluster_scene", "make_orbit_views", "make_config", "look_at",
           "ray_subsample_mask", "block_subsample_mask", "splitmix64", "SH_C0", "pack_bits", "unpack_bits",
           "make_explicit_scene", "make_camera_set", "make_batch_specs", "make_batch", "make_pose_region"]
