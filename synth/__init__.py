"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package only draws random numbers and builds cameras.  It holds none of
the rendering arithmetic, so both the CPU oracle and the HIP path can take
their inputs from it without sharing any of the method's code.
"""
from .scenes import (Camera, Scene, look_at_camera, orbit_cameras,
                     tiny_scene, scene_scale, diff_scene, batched_scene,
                     serving_scenes, random_scene, WORKLOADS)

__all__ = ["Camera", "Scene", "look_at_camera", "orbit_cameras", "tiny_scene",
           "scene_scale", "diff_scene", "batched_scene", "serving_scenes",
           "random_scene", "WORKLOADS"]
