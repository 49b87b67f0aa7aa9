"""Synthetic articulated robot: 30 rigid links posed by a seeded kinematic tree.

The paper ray casts against the posed link meshes of a Unitree G1 (29 DoF,
Sec. 4.1) whose meshes stay canonical in their local frames (Sec. 3.2.2).
The G1 meshes are not available, so each link is an ellipsoid tessellated
from an octahedron subdivided three times (8 * 4^3 = 512 triangles, 258
vertices), scaled by seeded semi-axes, and the tree is humanoid-like:
a floating root, two legs of 6 links, a waist of 3, two arms of 7 (29
revolute joints, 30 bodies).

Quaternions are stored (x, y, z, w) and rotate link-local vectors to world.
"""
import math
import numpy as np

from .rng import substream

N_LINKS = 30


def octasphere(levels=3):
    """Unit-sphere mesh from a subdivided octahedron: (V [258,3] f64, T [512,3])."""
    n = 1 << levels
    axes = [np.array(a, dtype=np.int64) for a in
            ((1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0), (0, -1, 0), (0, 0, -1))]
    faces = []
    for sx in (1, -1):
        for sy in (1, -1):
            for sz in (1, -1):
                A = np.array((sx, 0, 0))
                B = np.array((0, sy, 0))
                C = np.array((0, 0, sz))
                faces.append((A, B, C) if sx * sy * sz > 0 else (A, C, B))
    keys = {}
    pts = []
    tris = []

    def vid(P):
        k = tuple(int(v) for v in P)
        i = keys.get(k)
        if i is None:
            i = len(pts)
            keys[k] = i
            p = np.array(k, dtype=np.float64)
            pts.append(p / np.linalg.norm(p))
        return i

    for A, B, C in faces:
        # integer lattice points a*A + b*B + c*C with a + b + c = n
        def P(i, j):
            return (n - i - j) * A + i * B + j * C
        for i in range(n):
            for j in range(n - i):
                tris.append((vid(P(i, j)), vid(P(i + 1, j)), vid(P(i, j + 1))))
                if i + j < n - 1:
                    tris.append((vid(P(i + 1, j)), vid(P(i + 1, j + 1)), vid(P(i, j + 1))))
    del axes
    return np.asarray(pts), np.asarray(tris, dtype=np.int64)


def quat_from_matrix(R):
    """(x, y, z, w) quaternion of rotation matrix R (float64, batched [...,3,3])."""
    R = np.asarray(R, dtype=np.float64)
    m00, m11, m22 = R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]
    tr = m00 + m11 + m22
    q = np.zeros(R.shape[:-2] + (4,))
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr + 1.0, 1e-300)) * 2
    q0 = np.stack([(R[..., 2, 1] - R[..., 1, 2]) / s, (R[..., 0, 2] - R[..., 2, 0]) / s,
                   (R[..., 1, 0] - R[..., 0, 1]) / s, 0.25 * s], -1)
    c1 = (~c0) & (m00 > m11) & (m00 > m22)
    s1 = np.sqrt(np.maximum(1.0 + m00 - m11 - m22, 1e-300)) * 2
    q1 = np.stack([0.25 * s1, (R[..., 0, 1] + R[..., 1, 0]) / s1,
                   (R[..., 0, 2] + R[..., 2, 0]) / s1, (R[..., 2, 1] - R[..., 1, 2]) / s1], -1)
    c2 = (~c0) & (~c1) & (m11 > m22)
    s2 = np.sqrt(np.maximum(1.0 + m11 - m00 - m22, 1e-300)) * 2
    q2 = np.stack([(R[..., 0, 1] + R[..., 1, 0]) / s2, 0.25 * s2,
                   (R[..., 1, 2] + R[..., 2, 1]) / s2, (R[..., 0, 2] - R[..., 2, 0]) / s2], -1)
    s3 = np.sqrt(np.maximum(1.0 + m22 - m00 - m11, 1e-300)) * 2
    q3 = np.stack([(R[..., 0, 2] + R[..., 2, 0]) / s3, (R[..., 1, 2] + R[..., 2, 1]) / s3,
                   0.25 * s3, (R[..., 1, 0] - R[..., 0, 1]) / s3], -1)
    q = np.where(c0[..., None], q0, np.where(c1[..., None], q1, np.where(c2[..., None], q2, q3)))
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def axis_angle(axis, ang):
    """Rotation matrices for unit axis [3] and angles [...] (Rodrigues)."""
    ang = np.asarray(ang, dtype=np.float64)
    x, y, z = axis
    c, s = np.cos(ang), np.sin(ang)
    C = 1 - c
    R = np.empty(ang.shape + (3, 3))
    R[..., 0, 0] = c + x * x * C
    R[..., 0, 1] = x * y * C - z * s
    R[..., 0, 2] = x * z * C + y * s
    R[..., 1, 0] = y * x * C + z * s
    R[..., 1, 1] = c + y * y * C
    R[..., 1, 2] = y * z * C - x * s
    R[..., 2, 0] = z * x * C - y * s
    R[..., 2, 1] = z * y * C + x * s
    R[..., 2, 2] = c + z * z * C
    return R


def yaw_matrix(yaw):
    return axis_angle((0.0, 0.0, 1.0), yaw)


class Robot:
    """Seeded 30-link humanoid-like kinematic tree with ellipsoid link meshes."""

    def __init__(self, seed_label="robot", seed=None):
        from .rng import MASTER_SEED
        rng = substream(seed_label, MASTER_SEED if seed is None else seed)
        parent = [-1]
        direction = [np.zeros(3)]
        # legs: two chains of 6 from the root, going down
        for side in (1.0, -1.0):
            prev = 0
            for k in range(6):
                parent.append(prev)
                direction.append(np.array([0.0, side, -0.3]) if k == 0 else np.array([0.0, 0.0, -1.0]))
                prev = len(parent) - 1
        # waist: chain of 3 going up
        prev = 0
        for k in range(3):
            parent.append(prev)
            direction.append(np.array([0.0, 0.0, 1.0]))
            prev = len(parent) - 1
        waist_top = prev
        # arms: two chains of 7 from the waist top, sideways then down
        for side in (1.0, -1.0):
            prev = waist_top
            for k in range(7):
                parent.append(prev)
                direction.append(np.array([0.0, side, 0.2]) if k == 0 else np.array([0.0, 0.15 * side, -1.0]))
                prev = len(parent) - 1
        assert len(parent) == N_LINKS
        self.parent = np.array(parent)
        self.offset = np.zeros((N_LINKS, 3))
        self.axis = np.zeros((N_LINKS, 3))
        for b in range(1, N_LINKS):
            d = direction[b] + rng.normal(0.0, 0.15, 3)
            d /= np.linalg.norm(d)
            self.offset[b] = d * rng.uniform(0.05, 0.25)
            a = rng.normal(0.0, 1.0, 3)
            self.axis[b] = a / np.linalg.norm(a)
        self.semi = rng.uniform(0.03, 0.15, size=(N_LINKS, 3))
        # ellipsoid centre: half way to the link's first child (or a short stub)
        self.centre = np.zeros((N_LINKS, 3))
        for b in range(N_LINKS):
            kids = [c for c in range(N_LINKS) if self.parent[c] == b]
            self.centre[b] = 0.5 * self.offset[kids[0]] if kids else np.array([0.0, 0.0, -0.05])
        self.centre[0] = 0.0

    def link_triangles(self):
        """Link-local triangle soups: (tris f32 [30*512,3,3], offsets i64 [31])."""
        V, T = octasphere(3)
        out = []
        for b in range(N_LINKS):
            P = V * self.semi[b] + self.centre[b]
            out.append(P[T].astype(np.float32))
        off = np.arange(N_LINKS + 1, dtype=np.int64) * T.shape[0]
        return np.concatenate(out, 0), off

    def forward(self, root_pos, root_yaw, q):
        """World link poses for E envs.

        root_pos [E,3], root_yaw [E], q joint angles [E,30] (q[:,0] unused).
        Returns pos f64 [E,30,3], rotation f64 [E,30,3,3].
        """
        E = root_pos.shape[0]
        pos = np.zeros((E, N_LINKS, 3))
        rot = np.zeros((E, N_LINKS, 3, 3))
        pos[:, 0] = root_pos
        rot[:, 0] = yaw_matrix(root_yaw)
        for b in range(1, N_LINKS):
            p = self.parent[b]
            Rp = rot[:, p]
            pos[:, b] = pos[:, p] + np.einsum("eij,j->ei", Rp, self.offset[b])
            rot[:, b] = Rp @ axis_angle(self.axis[b], q[:, b])
        return pos, rot
