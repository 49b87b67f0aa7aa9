"""GPU: the privileged height map (Sec. 3.1: the terrain experts' 17 x 11 grid
at 0.1 m around the base) against the oracle's brute-force vertical rays."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL = 1e-5  # metres: FP32 output of an FP64 decision on both sides


def rc():
    import paper_2602_03002_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def say(msg):
    print(msg, flush=True)


def gpu_heightmap(sc, base, yaw, **kw):
    out = sc.heightmap(dev(base), dev(yaw), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def agree(got, ref, terrain, base, yaw, kw):
    """Element-wise parity; a point where the two differ must sit on a vertical
    step, where moving the base by 1e-5 m makes the oracle give the GPU's value."""
    same = (np.abs(got - ref) <= TOL) | (np.isnan(got) & np.isnan(ref))
    bad = np.argwhere(~same)
    for e in np.unique(bad[:, 0]) if bad.size else []:
        alts = []
        for ddx, ddy in ((1e-5, 0), (-1e-5, 0), (0, 1e-5), (0, -1e-5)):
            b = np.array(base[e], np.float64)
            b[0] += ddx
            b[1] += ddy
            alts.append(oracle.heightmap(terrain, b[None], [yaw[e]], **kw)[0])
        for _, j, i in bad[bad[:, 0] == e]:
            assert any(abs(a[j, i] - got[e, j, i]) <= 1e-4 for a in alts), \
                (e, j, i, got[e, j, i], ref[e, j, i])
    return int(len(bad))


def test_heightmap_tile_terrain_all_points():
    say("[heightmap] 2x2 tiles, 24 random bases, all 17x11 points")
    terr = sg.TileTerrain(2, seed=sg.MASTER_SEED)
    tri = terr.triangles()
    rng = np.random.default_rng(3)
    E = 24
    xy = np.stack([rng.uniform(-4.5, 4.5, E), rng.uniform(-4.5, 4.5, E)], 1)
    base = np.concatenate([xy, [[terr.height(x, y) + 0.6] for x, y in xy]], 1).astype(np.float32)
    yaw = rng.uniform(0, 2 * np.pi, E).astype(np.float32)
    kw = dict(nx=17, ny=11, dx=0.1, dy=0.1, top=1.0, depth=3.0)
    sc = rc().Scene(dev(tri))
    got = gpu_heightmap(sc, base, yaw, **kw)
    ref = oracle.heightmap(tri, base, yaw, **kw)
    assert got.shape == (E, 11, 17)
    assert np.isfinite(ref).all()
    n_bad = agree(got, ref, tri, base, yaw, kw)
    assert n_bad <= 0.01 * got.size


@pytest.mark.parametrize("cap", [1, 2])
def test_heightmap_stack_cap_falls_back_to_the_binary_walk(cap):
    """With the 4-wide walk's stack capped, columns whose pushes are dropped
    are walked again over the binary records: the map is bit-identical to the
    uncapped one, and still agrees with the oracle."""
    say(f"[heightmap] 2x2 tiles, 24 bases, 4-wide walk stack capped at {cap}")
    terr = sg.TileTerrain(2, seed=sg.MASTER_SEED)
    tri = terr.triangles()
    rng = np.random.default_rng(5)
    E = 24
    xy = np.stack([rng.uniform(-4.5, 4.5, E), rng.uniform(-4.5, 4.5, E)], 1)
    base = np.concatenate([xy, [[terr.height(x, y) + 0.6] for x, y in xy]], 1).astype(np.float32)
    yaw = rng.uniform(0, 2 * np.pi, E).astype(np.float32)
    kw = dict(nx=17, ny=11, dx=0.1, dy=0.1, top=1.0, depth=3.0)
    sc = rc().Scene(dev(tri))
    full = gpu_heightmap(sc, base, yaw, **kw)
    sc.set_walk_stack_limit(cap)
    try:
        capped = gpu_heightmap(sc, base, yaw, **kw)
    finally:
        sc.set_walk_stack_limit(16)
    assert np.array_equal(full.view(np.uint64), capped.view(np.uint64))
    ref = oracle.heightmap(tri, base, yaw, **kw)
    assert agree(capped, ref, tri, base, yaw, kw) <= 0.01 * capped.size


def test_heightmap_grid_vertices_watertight():
    """Grid points on the vertices and edges of a triangulated tilted plane
    (yaw 0, base on a vertex): every vertical ray finds the plane."""
    say("[heightmap] tilted plane, points on shared vertices and edges")
    n, h = 40, 0.1
    g = (np.arange(n + 1) - n / 2) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    Z = 0.3 * X - 0.2 * Y
    V = np.stack([X, Y, Z], -1)
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = V[i, j], V[i + 1, j], V[i + 1, j + 1], V[i, j + 1]
            tris += [[a, b, c], [a, c, d]] if (i + j) % 2 else [[a, b, d], [b, c, d]]
    tri = np.array(tris, np.float32)
    base = np.array([[0.0, 0.0, 0.5], [0.05, 0.1, 0.5], [-1.0, 1.0, 0.9]], np.float32)
    yaw = np.array([0.0, 0.0, np.pi / 2], np.float32)
    kw = dict(nx=17, ny=11, dx=0.1, dy=0.05, top=1.0, depth=4.0)
    sc = rc().Scene(dev(tri))
    got = gpu_heightmap(sc, base, yaw, **kw)
    ref = oracle.heightmap(tri, base, yaw, **kw)
    assert not np.isnan(got).any()
    assert np.max(np.abs(got - ref)) <= TOL
    # the plane itself: z = 0.3 x - 0.2 y
    for e in range(3):
        c, s = np.cos(float(yaw[e])), np.sin(float(yaw[e]))
        for j in range(11):
            for i in range(17):
                gx, gy = (i - 8) * 0.1, (j - 5) * 0.05
                x, y = base[e, 0] + c * gx - s * gy, base[e, 1] + s * gx + c * gy
                assert got[e, j, i] == pytest.approx(0.3 * x - 0.2 * y - base[e, 2], abs=1e-5)


def test_heightmap_miss_depth_and_grid_shapes():
    """Outside the terrain and below `depth` the miss value comes back; odd
    and even grid sizes, including a single point, follow the oracle."""
    say("[heightmap] miss, depth cut, grid shapes")
    tri = np.array([[[-1.0, -1.0, 0.2], [3.0, -1.0, 0.2], [-1.0, 3.0, 0.2]],
                    [[5.0, 5.0, -2.5], [7.0, 5.0, -2.5], [5.0, 7.0, -2.5]]], np.float32)
    base = np.array([[0.0, 0.0, 1.0], [2.0, 2.0, 1.0], [6.0, 5.5, 1.0], [10.0, 10.0, 1.0]], np.float32)
    yaw = np.array([0.3, -1.2, 0.0, 2.0], np.float32)
    sc = rc().Scene(dev(tri))
    for nx, ny, dx, dy in ((17, 11, 0.1, 0.1), (1, 1, 0.1, 0.1), (16, 4, 0.25, 0.3), (33, 21, 0.05, 0.05)):
        for depth in (3.0, 4.0, 4.6):
            kw = dict(nx=nx, ny=ny, dx=dx, dy=dy, top=1.0, depth=depth)
            got = gpu_heightmap(sc, base, yaw, miss=-7.0, **kw)
            ref = oracle.heightmap(tri, base, yaw, miss=-7.0, **kw)
            assert got.shape == (4, ny, nx)
            assert np.max(np.abs(got - ref)) <= TOL, (nx, ny, depth)
    # base 3 is off the terrain: all miss; base 2's ray starts at z 2.0 and needs
    # depth >= 4.5 to reach the low triangle at z -2.5
    assert np.all(got[3] == -7.0)
    got3 = gpu_heightmap(sc, base, yaw, nx=1, ny=1, top=1.0, depth=3.0, miss=-7.0)
    assert got3[2, 0, 0] == -7.0
    got4 = gpu_heightmap(sc, base, yaw, nx=1, ny=1, top=1.0, depth=4.6, miss=-7.0)
    assert got4[2, 0, 0] == pytest.approx(-3.5, abs=1e-6)


def test_heightmap_rejects_bad_args():
    m = rc()
    sc = m.Scene(dev(sg.small_plain_case()["terrain"]))
    b, y = dev(np.zeros((2, 3))), dev(np.zeros(2))
    for kw in (dict(nx=0), dict(ny=5000), dict(dx=0.0), dict(dy=-0.1), dict(depth=0.0),
               dict(depth=float("inf")), dict(top=float("nan"))):
        with pytest.raises(m.RcError):
            sc.heightmap(b, y, **kw)


def test_heightmap_4096_envs_sampled():
    """The measured workload: 4096 bases of the 4096-env scene on the 20 x 20
    tile terrain, all 17 x 11 points on the GPU; 3 whole envs against the
    oracle and 64 envs against the analytic tile surface."""
    say("[heightmap] 4096 envs x 187 points on 20x20 tiles")
    w = sg.robots_4096(steps=1)
    terr = w["terrain_obj"]
    base = w["link_pos"][0, :, 0].astype(np.float32)  # the base link's origin
    yaw = sg.substream("heightmap/yaw").uniform(0, 2 * np.pi, w["E"]).astype(np.float32)
    kw = dict(nx=17, ny=11, dx=0.1, dy=0.1, top=1.0, depth=3.0)
    sc = rc().Scene(dev(w["terrain"]))
    got = gpu_heightmap(sc, base, yaw, **kw)
    assert np.isfinite(got).all()
    pick = np.array([0, 2049, 4095])
    ref = oracle.heightmap(w["terrain"], base[pick], yaw[pick], **kw)
    agree(got[pick], ref, w["terrain"], base[pick], yaw[pick], kw)
    rng = np.random.default_rng(9)
    checked = 0
    for e in rng.choice(w["E"], 64, replace=False):
        c, s = np.cos(float(yaw[e])), np.sin(float(yaw[e]))
        for j in range(11):
            for i in range(17):
                gx, gy = (i - 8) * 0.1, (j - 5) * 0.1
                x = float(base[e, 0]) + c * gx - s * gy
                y = float(base[e, 1]) + s * gx + c * gy
                near = [terr.height(x + a, y + b) for a in (-1e-5, 1e-5) for b in (-1e-5, 1e-5)]
                if max(near) - min(near) > 1e-4:
                    continue  # a vertical step
                assert got[e, j, i] == pytest.approx(terr.height(x, y) - float(base[e, 2]), abs=2e-5)
                checked += 1
    assert checked > 0.8 * 64 * 187
