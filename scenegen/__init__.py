"""Seeded synthetic inputs (terrain, robot, poses, cameras) shared by tests and bench.

This package holds input generators only: no ray casting, no sensor model.
"""
from .rng import MASTER_SEED, substream, splitmix64
from .terrain import ProfileTerrain, TileTerrain, SlopeTile, StairsTile, StonesTile
from .robot import Robot, octasphere, quat_from_matrix, N_LINKS
from .cameras import intrinsics_from_fov, optical_axes, mounted_cameras
from .workloads import (small_plain_case, robot_scene, robots_64, robots_4096, uneven_cameras,
                        uneven_4096, CAM_DESC, RES_SET, table1, TABLE1_W, TABLE1_H,
                        TABLE1_HFOV, TABLE1_VFOV, TABLE1_POOL,
                        synthetic_frames, SENSOR, NEAR, FAR)
