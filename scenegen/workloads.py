"""Seeded synthetic workloads: scene, robot poses, cameras and sensor settings.

Each builder returns a plain dict of numpy arrays (float32 wherever the
renderer takes float32 input) that both the renderer and the oracle read.
Nothing here casts a ray.
"""
import math
import numpy as np

from .rng import substream, MASTER_SEED
from .terrain import ProfileTerrain, TileTerrain
from .robot import Robot, N_LINKS
from .cameras import intrinsics_from_fov, mounted_cameras, optical_axes
from .robot import quat_from_matrix, yaw_matrix

HFOV, VFOV = 87.0, 58.0
NEAR, FAR = 0.05, 3.0
ROOT_HEIGHT = 0.75

SENSOR = dict(sigma_abs=0.01, sigma_rel=0.0, p_drop=0.02, lat_min=1, lat_max=3,
              near=NEAR, far=FAR, fill=0.0)


def small_plain_case():
    """1 env, 1 camera 32x24, terrain profile only, no robot, no sensor model."""
    terr = ProfileTerrain()
    W, H = 32, 24
    R = optical_axes(0.0, math.radians(45.0))
    return dict(
        name="1 env x 1 cam 32x24, plane + 20deg slope + 3 stairs, no robot",
        terrain=terr.triangles(), terrain_obj=terr,
        link_tri=np.zeros((0, 3, 3), np.float32), link_off=np.zeros(1, np.int64),
        E=1, C=1, W=W, H=H,
        cam_pos=np.array([[[0.0, 0.0, 1.0]]], np.float32),
        cam_quat=quat_from_matrix(R)[None, None].astype(np.float32),
        intr=intrinsics_from_fov(W, H, HFOV, VFOV)[None, None].astype(np.float32),
        link_pos=np.zeros((1, 1, 0, 3), np.float32), link_quat=np.zeros((1, 1, 0, 4), np.float32),
        near=NEAR, far=FAR, sensor=None, optical_R=R,
    )


def env_grid(side, spacing):
    c = (np.arange(side) - (side - 1) / 2.0) * spacing
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], 1)


def robot_scene(n_tiles, env_side, spacing, n_cam, W, H, steps, seed=MASTER_SEED,
                label="scene", terrain=None, robot=None, hfov=HFOV, vfov=VFOV):
    """Envs on a tile terrain, each with the 30-link robot and mounted cameras."""
    terr = terrain if terrain is not None else TileTerrain(n_tiles, seed=seed)
    rob = robot if robot is not None else Robot(seed=seed)
    rng = substream(f"{label}/poses/{n_tiles}/{env_side}", seed)
    xy = env_grid(env_side, spacing)
    E = xy.shape[0]
    z = np.array([terr.height(x, y) for x, y in xy]) + ROOT_HEIGHT
    root_pos = np.concatenate([xy, z[:, None]], 1)
    yaw = rng.uniform(0.0, 2 * math.pi, E)
    link_pos = np.zeros((steps, E, N_LINKS, 3), np.float32)
    link_quat = np.zeros((steps, E, N_LINKS, 4), np.float32)
    for s in range(steps):
        q = rng.uniform(-0.5, 0.5, (E, N_LINKS))
        p, R = rob.forward(root_pos, yaw, q)
        link_pos[s] = p
        link_quat[s] = quat_from_matrix(R)
    cam_pos, cam_quat = mounted_cameras(root_pos, yaw_matrix(yaw), n_cam)
    intr = np.broadcast_to(intrinsics_from_fov(W, H, hfov, vfov), (E, n_cam, 4))
    link_tri, link_off = rob.link_triangles()
    return dict(
        name=f"{E} envs x {n_cam} cams {W}x{H}, {n_tiles}x{n_tiles} tiles, 30 links",
        terrain=terr.triangles(), terrain_obj=terr, robot=rob,
        link_tri=link_tri, link_off=link_off,
        E=E, C=n_cam, W=W, H=H,
        cam_pos=cam_pos.astype(np.float32), cam_quat=cam_quat.astype(np.float32),
        intr=np.ascontiguousarray(intr, dtype=np.float32),
        link_pos=link_pos, link_quat=link_quat,
        near=NEAR, far=FAR, sensor=dict(SENSOR),
    )


def robots_64():
    """64 envs x 2 cams 64x48 on a 10x10 tile terrain (about 500k triangles)."""
    return robot_scene(10, 8, 10.0, 2, 64, 48, steps=3, label="robots64")


def robots_4096(steps=100):
    """4096 envs x 2 cams 64x48 on a 20x20 tile terrain (about 2M triangles)."""
    return robot_scene(20, 64, 2.5, 2, 64, 48, steps=steps, label="robots4096")


# The paper's perception setting (Sec. 4.1, Perception Settings; Table 1):
# 1024 envs, up to 4 cameras (front, rear, left, right), 240x135 raw depth at
# 101 x 69 degrees, downsampled to 48x27.
TABLE1_W, TABLE1_H, TABLE1_HFOV, TABLE1_VFOV, TABLE1_POOL = 240, 135, 101.0, 69.0, 5


def table1(n_cam, steps=3, terrain=None, robot=None):
    """1024 envs x n_cam x 240x135 at 101x69 degrees on the 20x20 tile terrain
    (a 32 x 32 env grid at 5 m spacing)."""
    return robot_scene(20, 32, 5.0, n_cam, TABLE1_W, TABLE1_H, steps=steps, label="table1",
                       terrain=terrain, robot=robot, hfov=TABLE1_HFOV, vfov=TABLE1_VFOV)


def synthetic_frames(E, C, H, W, steps, seed=MASTER_SEED, label="frames", far=FAR):
    """Depth/inst frames for testing the sensor model alone (no rendering)."""
    rng = substream(f"{label}/{E}/{C}/{H}/{W}/{steps}", seed)
    depth = rng.uniform(0.0, far * 1.15, (steps, E, C, H, W)).astype(np.float32)
    inst = rng.integers(0, 31, (steps, E, C, H, W)).astype(np.int32)
    miss = rng.random((steps, E, C, H, W)) < 0.1
    inst[miss] = -1
    depth[miss] = np.float32(far)
    return depth, inst


# Batched uneven form: per-camera descriptors (the renderer's 64-byte layout)
CAM_DESC = np.dtype([("env", "<i4"), ("width", "<i4"), ("height", "<i4"), ("out_offset", "<u4"),
                     ("cam_uid", "<u4"), ("pos", "<f4", 3), ("quat", "<f4", 4), ("intr", "<f4", 4)])
RES_SET = [(32, 24), (64, 48), (87, 58), (106, 60)]


def uneven_cameras(scene, seed=MASTER_SEED, label="uneven", max_cams=4):
    """Descriptors for 1..max_cams cameras per env with resolutions from RES_SET.

    ``scene`` must come from robot_scene(..., n_cam=4, ...) (mounts 0..3).
    Camera uid = e * 4 + mount index (environment-local, batch independent).
    Returns (desc structured array, n_pixels).
    """
    E = scene["E"]
    rng = substream(f"{label}/{E}", seed)
    n_cams = rng.integers(1, max_cams + 1, E)
    rows = []
    off = 0
    for e in range(E):
        for c in range(int(n_cams[e])):
            W, H = RES_SET[int(rng.integers(0, len(RES_SET)))]
            K = intrinsics_from_fov(W, H, HFOV, VFOV)
            rows.append((e, W, H, off, e * 4 + c, scene["cam_pos"][e, c], scene["cam_quat"][e, c], K))
            off += W * H
    return np.array(rows, dtype=CAM_DESC), off


def uneven_4096(steps=3):
    """4096 envs on the 20x20-tile terrain, each with 1-4 cameras of mixed sizes."""
    sc = robot_scene(20, 64, 2.5, 4, 64, 48, steps=steps, label="uneven4096")
    desc, n_pix = uneven_cameras(sc)
    return sc, desc, n_pix
