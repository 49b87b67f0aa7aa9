"""Invariants of the seeded input generators (no ray casting involved)."""
import collections
import numpy as np

import scenegen as sg


def edge_use(tris):
    v = np.ascontiguousarray(tris, np.float32).view(np.uint32).reshape(-1, 3, 3)
    cnt = collections.Counter()
    for t in v:
        a, b, c = tuple(t[0]), tuple(t[1]), tuple(t[2])
        for e in ((a, b), (b, c), (c, a)):
            cnt[tuple(sorted(e))] += 1
    return cnt


def test_tiles_are_conforming_and_meet_at_borders():
    tt = sg.TileTerrain(3, seed=12345)
    assert {t.kind for t in tt.tiles} == {"slope", "stairs", "stones"}
    cnt = edge_use(tt.triangles())
    assert set(cnt.values()) == {1, 2}
    ones = [e for e, c in cnt.items() if c == 1]
    # every single-use edge lies on the outer border of the 3x3 tile block (|x| or |y| = 12)
    for e in ones:
        p = np.array(e, np.uint32).view(np.float32).reshape(2, 3)
        assert np.all(np.isclose(np.abs(p[:, 0]), 12.0)) or np.all(np.isclose(np.abs(p[:, 1]), 12.0))
    assert len(ones) == 4 * 3 * sg.terrain.BORDER_SEG


def test_no_degenerate_triangles():
    tri = sg.TileTerrain(2).triangles().astype(np.float64)
    area = np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    assert area.min() > 1e-4
    lt, off = sg.Robot().link_triangles()
    lt = lt.astype(np.float64)
    area = np.linalg.norm(np.cross(lt[:, 1] - lt[:, 0], lt[:, 2] - lt[:, 0]), axis=1)
    assert area.min() > 1e-7


def test_octasphere_and_links_closed():
    V, T = sg.octasphere(3)
    assert V.shape == (258, 3) and T.shape == (512, 3)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
    lt, off = sg.Robot().link_triangles()
    assert off.tolist() == list(range(0, 30 * 512 + 1, 512))
    for b in (0, 7, 29):
        assert set(edge_use(lt[off[b]:off[b + 1]]).values()) == {2}


def test_profile_terrain_size_and_conformity():
    w = sg.small_plain_case()
    assert 2000 <= w["terrain"].shape[0] <= 2600
    assert set(edge_use(w["terrain"]).values()) == {1, 2}


def test_scene_shapes_and_determinism():
    a = sg.robot_scene(2, 2, 4.0, 2, 16, 12, steps=2, label="t")
    b = sg.robot_scene(2, 2, 4.0, 2, 16, 12, steps=2, label="t")
    for k in ("terrain", "link_pos", "link_quat", "cam_pos", "cam_quat", "intr"):
        assert np.array_equal(a[k], b[k])
    assert a["link_pos"].shape == (2, 4, 30, 3) and a["cam_quat"].shape == (4, 2, 4)
    # cameras sit 1.0 m above the terrain under the root (0.75 m root + 0.25 m mount)
    terr = a["terrain_obj"]
    for e in range(4):
        x, y = a["link_pos"][0, e, 0, :2]
        assert abs(a["link_pos"][0, e, 0, 2] - terr.height(x, y) - 0.75) < 1e-5
