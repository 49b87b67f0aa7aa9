"""GPU edge cases of the ray cast (Algorithm 1) against the FP64 oracle:
degenerate (zero-area) triangles lying on pixel rays, rays with exactly zero
direction components, cameras inside a link mesh, and host-side rejection of
bad arguments (nothing is launched and outputs stay untouched)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from parity import assert_parity

pytestmark = pytest.mark.gpu

DEV = "cuda"


def rc():
    import paper_2602_03002_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def render_all(w, step=0):
    m = rc()
    sc = m.Scene(dev(w["terrain"]))
    B = int(w["link_off"].shape[0] - 1)
    if B > 0:
        sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    lp = dev(w["link_pos"][step]) if B else None
    lq = dev(w["link_quat"][step]) if B else None
    d, i, t = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                        w["far"], link_pos=lp, link_quat=lq)
    torch.cuda.synchronize()
    ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][step],
                        w["link_quat"][step], w["cam_pos"], w["cam_quat"], w["intr"], w["W"],
                        w["H"], w["far"])
    return d.cpu().numpy(), i.cpu().numpy(), t.cpu().numpy(), ref


def pixel_rays(w):
    """FP64 pixel rays (o, d) of every pixel, [E, C, H, W, 3] each."""
    E, C, H, W = w["E"], w["C"], w["H"], w["W"]
    q = np.asarray(w["cam_quat"], np.float64).reshape(E * C, 4)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    x, y, z, s = q.T
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * s), 2 * (x * z + y * s),
                  2 * (x * y + z * s), 1 - 2 * (x * x + z * z), 2 * (y * z - x * s),
                  2 * (x * z - y * s), 2 * (y * z + x * s), 1 - 2 * (x * x + y * y)], 1).reshape(-1, 3, 3)
    K = np.asarray(w["intr"], np.float64).reshape(E * C, 4)
    px = (np.arange(W) + 0.5)[None, None, :]
    py = (np.arange(H) + 0.5)[None, :, None]
    rx = (px - K[:, 2, None, None]) / K[:, 0, None, None]
    ry = (py - K[:, 3, None, None]) / K[:, 1, None, None]
    r = np.stack(np.broadcast_arrays(rx, ry, np.ones_like(rx)), -1)  # [EC, H, W, 3]
    d = np.einsum("nij,nhwj->nhwi", R, r)
    o = np.broadcast_to(np.asarray(w["cam_pos"], np.float64).reshape(E * C, 1, 1, 3), d.shape)
    return o.reshape(E, C, H, W, 3), d.reshape(E, C, H, W, 3)


def test_degenerate_triangles_on_pixel_rays():
    """Zero-area triangles (three equal vertices, two equal and a third
    elsewhere, or three distinct vertices on one line) placed on pixel rays
    halfway to the surface are never hit: a ray through them sees the terrain
    or link behind, as the oracle says."""
    say("[edge] degenerate triangles on pixel rays")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="degenerate")
    ref0 = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                         w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"], w["W"], w["H"],
                         w["far"])
    o, d = pixel_rays(w)
    o, d = o.reshape(-1, 3), d.reshape(-1, 3)
    rng = np.random.default_rng(5)
    hits = np.nonzero(ref0["inst"] >= 0)[0]
    pick = rng.choice(hits, 400, replace=False)
    extra = []
    u = np.float32([2.0 ** -6, 0.0, 0.0])
    for k, p in enumerate(pick):
        pt = (o[p] + 0.5 * ref0["depth"][p] * d[p]).astype(np.float32)
        q = (pt + rng.normal(0, 0.05, 3)).astype(np.float32)
        # exactly collinear in FP32: pt -+ u differ from pt in x only, exactly
        extra.append([[pt, pt, pt], [pt, pt, q], [pt - u, pt, pt + u]][k % 3])
    extra = np.asarray(extra, np.float32)
    w["terrain"] = np.concatenate([w["terrain"], extra], 0)
    dd, ii, tt, ref = render_all(w)
    assert_parity(dd, ii, tt, ref, w["far"], label="degenerate triangles on rays")
    # none of the degenerate triangles is reported
    n0 = w["terrain"].shape[0] - extra.shape[0]
    B = int(w["link_off"].shape[0] - 1)
    assert not np.any((ii == B) & (tt >= n0))


def test_degenerate_link_triangles():
    """A link mesh with zero-area triangles at its own vertices renders like
    the oracle."""
    say("[edge] degenerate link triangles")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="degenlink")
    lt = w["link_tri"].reshape(-1, 3, 3)
    off = w["link_off"].copy()
    last0, last1 = int(off[-2]), int(off[-1])
    V = lt[last0:last1].reshape(-1, 3)
    rng = np.random.default_rng(6)
    a = V[rng.choice(V.shape[0], 40)]
    b = V[rng.choice(V.shape[0], 40)]
    deg = np.concatenate([np.stack([a, a, a], 1), np.stack([a, a, b], 1), np.stack([a, b, a], 1)], 0)
    w["link_tri"] = np.concatenate([lt, deg.astype(np.float32)], 0)
    off[-1] = last1 + deg.shape[0]
    w["link_off"] = off
    dd, ii, tt, ref = render_all(w)
    assert_parity(dd, ii, tt, ref, w["far"], label="degenerate link triangles")


# optical -> world quaternions (x, y, z, w) with exactly representable rotations:
# down: optical z -> -z; along_x: optical z -> +x; along_y: optical z -> +y
QUATS = {"down": (1.0, 0.0, 0.0, 0.0), "along_x": (-0.5, 0.5, -0.5, 0.5),
         "along_y": (-0.5, -0.5, -0.5, 0.5)}


def _cam(E, pos, quat, W, H):
    K = np.array([3.0 * W / 4, 3.0 * W / 4, (W - 1) / 2 + 0.5, (H - 1) / 2 + 0.5])
    return (np.asarray(pos, np.float32).reshape(E, 1, 3),
            np.broadcast_to(np.float32(quat), (E, 1, 4)).copy(),
            np.broadcast_to(K, (E, 1, 4)).astype(np.float32).copy())


@pytest.mark.parametrize("view", ["down", "along_x", "along_y"])
def test_axis_aligned_rays(view):
    """Cameras looking straight down or horizontally along an axis, with odd
    image sizes so the centre rays have exactly zero components, over stairs
    and stepping stones (faces parallel to those rays)."""
    say(f"[edge] axis-aligned rays: {view}")
    w = sg.robot_scene(2, 3, 2.5, 1, 17, 13, steps=1, label="axis")
    E = w["E"]
    terr = w["terrain_obj"]
    xy = w["link_pos"][0, :, 0, :2].astype(np.float64)
    lift = 1.2 if view == "down" else 0.15
    pos = np.concatenate([xy + 0.37, [[terr.height(x + 0.37, y + 0.37) + lift] for x, y in xy]], 1)
    w["cam_pos"], w["cam_quat"], w["intr"] = _cam(E, pos, QUATS[view], 17, 13)
    w["C"], w["W"], w["H"] = 1, 17, 13
    dd, ii, tt, ref = render_all(w)
    assert_parity(dd, ii, tt, ref, w["far"], label=f"axis-aligned {view}")
    o, d = pixel_rays(w)
    c = d[:, 0, 6, 8]
    assert np.count_nonzero(c == 0.0) == 2 * E  # two exact zeros per centre ray


def test_camera_inside_a_link():
    """A camera at a link's origin sees the link's inside (faces are
    two-sided)."""
    say("[edge] camera inside a link")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="inside")
    E = w["E"]
    lp = w["link_pos"][0]
    cp = w["cam_pos"].copy()
    cp[:, 0] = lp[:, 0]  # the root link's origin: inside its ellipsoid
    w["cam_pos"] = cp
    dd, ii, tt, ref = render_all(w)
    assert_parity(dd, ii, tt, ref, w["far"], label="camera inside a link")
    assert np.all(ii[:, 0] >= 0) and np.mean(ii[:, 0] == 0) > 0.5


def test_render_rejects_bad_arguments_and_leaves_outputs():
    say("[edge] argument validation")
    m = rc()
    w = sg.robot_scene(1, 1, 4.0, 1, 16, 12, steps=1, label="validate")
    sc = m.Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    lp, lq = dev(w["link_pos"][0]), dev(w["link_quat"][0])
    cp, cq, K = dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"])
    depth = torch.full((1, 1, 12, 16), 123.0, device=DEV)
    inst = torch.full((1, 1, 12, 16), 77, dtype=torch.int32, device=DEV)
    tri = torch.full_like(inst, 77)
    a, _, ws = sc._plain_args(cp, cq, K, 16, 12, 3.0, lp, lq, 0, (depth, inst, tri), True)
    L = m.lib()

    def call(**changes):
        b = type(a).from_buffer_copy(a)
        for k, v in changes.items():
            setattr(b, k, v)
        return L.rc_render(sc.handle, ctypes.byref(b), ctypes.c_void_p(ws.ptr), ws.nbytes, None)

    bad = [dict(width=0), dict(height=0), dict(n_env=0), dict(n_cam=-1), dict(width=65536),
           dict(n_env=1 << 20, width=65535, height=65535), dict(cam_pos=None), dict(intr=None),
           dict(depth=None), dict(link_pos=None), dict(far_plane=0.0), dict(far_plane=float("nan")),
           dict(far_plane=float("inf")), dict(far_plane=1e21), dict(depth_mode=2)]
    for ch in bad:
        assert call(**ch) == -1, ch
    assert L.rc_render(sc.handle, ctypes.byref(a), ctypes.c_void_p(ws.ptr), 64, None) == -2
    assert L.rc_render(sc.handle, ctypes.byref(a), ctypes.c_void_p(ws.ptr + 8), ws.nbytes - 8,
                       None) == -2
    torch.cuda.synchronize()
    assert torch.all(depth == 123.0) and torch.all(inst == 77) and torch.all(tri == 77)
    # and the good call renders
    assert call() == 0
    torch.cuda.synchronize()
    assert not torch.all(depth == 123.0)


def test_largest_width_and_many_envs():
    """The largest image width (65535, three rows: a ragged tile row) and
    16,384 environments (a grid far beyond one block per compute unit, an
    uneven last run per XCD), sampled against the oracle."""
    say("[edge] width 65535 and 16384 envs")
    w = sg.robot_scene(2, 1, 4.0, 1, 16, 12, steps=1, label="widest")
    W, H = 65535, 3
    w["intr"] = np.array([[sg.intrinsics_from_fov(W, H, 120.0, 0.01)]], np.float32)
    w["W"], w["H"] = W, H
    dd, ii, tt = _render_only(w)
    rays = np.sort(np.random.default_rng(3).choice(W * H, 300, replace=False))
    ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                        w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"], W, H, w["far"],
                        rays=rays)
    assert_parity(dd.ravel()[rays], ii.ravel()[rays], tt.ravel()[rays], ref, w["far"], label="width 65535")

    w = sg.robot_scene(2, 128, 0.06, 1, 8, 8, steps=1, label="manyenvs")
    assert w["E"] == 16384
    dd, ii, tt = _render_only(w)
    rays = np.sort(np.random.default_rng(4).choice(dd.size, 400, replace=False))
    ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                        w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"], 8, 8, w["far"],
                        rays=rays)
    assert_parity(dd.ravel()[rays], ii.ravel()[rays], tt.ravel()[rays], ref, w["far"], label="16384 envs")


def _render_only(w):
    m = rc()
    sc = m.Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    d, i, t = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                        w["far"], link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
    torch.cuda.synchronize()
    return d.cpu().numpy(), i.cpu().numpy(), t.cpu().numpy()
