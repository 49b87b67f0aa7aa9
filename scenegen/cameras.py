"""Pinhole depth cameras: intrinsics from a field of view, mounts on the robot.

Conventions (the paper leaves them open, Sec. 3.2.2): the optical frame has
x right, y down, z forward; a camera quaternion (x, y, z, w) rotates optical
vectors to world; pixel (x, y) looks through its centre (x + 0.5, y + 0.5);
the principal point is the image centre.
"""
import math
import numpy as np

from .robot import quat_from_matrix


def intrinsics_from_fov(W, H, hfov_deg, vfov_deg):
    """(fx, fy, cx, cy) with independent focal lengths for the two FOVs."""
    fx = (W / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    fy = (H / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    return np.array([fx, fy, W / 2.0, H / 2.0])


def optical_axes(forward_yaw, pitch_down):
    """Rotation matrix whose columns are the optical x, y, z axes in the parent frame.

    The camera looks along yaw ``forward_yaw`` (rad, about +z) and is pitched
    down by ``pitch_down`` (rad); image x points to the camera's right.
    """
    cy, sy = math.cos(forward_yaw), math.sin(forward_yaw)
    cp, sp = math.cos(pitch_down), math.sin(pitch_down)
    z = np.array([cp * cy, cp * sy, -sp])
    x = np.array([sy, -cy, 0.0])
    y = np.cross(z, x)
    return np.stack([x, y, z], 1)


# front, rear, left and right depth cameras (Sec. 4.1; the paper deploys the front-rear pair)
MOUNTS = [
    (np.array([0.20, 0.0, 0.25]), optical_axes(0.0, math.radians(45.0))),
    (np.array([-0.20, 0.0, 0.25]), optical_axes(math.pi, math.radians(45.0))),
    (np.array([0.0, 0.20, 0.25]), optical_axes(math.pi / 2, math.radians(45.0))),
    (np.array([0.0, -0.20, 0.25]), optical_axes(-math.pi / 2, math.radians(45.0))),
]


def mounted_cameras(root_pos, root_rot, n_cam):
    """World camera poses for cameras rigidly mounted on the root link.

    root_pos [E,3], root_rot [E,3,3] -> (pos f64 [E,C,3], quat f64 [E,C,4]).
    """
    E = root_pos.shape[0]
    pos = np.zeros((E, n_cam, 3))
    quat = np.zeros((E, n_cam, 4))
    for c in range(n_cam):
        mp, mR = MOUNTS[c]
        pos[:, c] = root_pos + np.einsum("eij,j->ei", root_rot, mp)
        quat[:, c] = quat_from_matrix(root_rot @ mR)
    return pos, quat
