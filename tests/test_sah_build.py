"""CPU tests of the binned-SAH terrain hierarchy (rc_sah_build_host, the
builder behind rc_scene_rebuild_sah): structure, containment, leaf order,
zero-area triangles, determinism, and a lower surface-area cost than the
Morton build's (the reason for it)."""
import numpy as np
import pytest

import paper_2602_03002_amd as m
import scenegen as sg
from oracle import lbvh

FAR = np.float32(1e30)


def walk(rec):
    """Leaves below the root and, per internal record, the leaves below each
    child (recursion over the child words)."""
    ri = rec.view(np.int32)
    below = {}

    def leaves(c):
        if c < 0:
            return [~c]
        if c not in below:
            below[c] = (leaves(ri[c, 12]), leaves(ri[c, 13]))
        return below[c][0] + below[c][1]

    return leaves(0), below


def sah_cost(rec):
    """C_trav = C_tri = 1, one triangle per leaf: every child box weighs 1."""
    b = rec[:, :12].astype(np.float64).reshape(-1, 2, 6)
    ok = b[..., 0] < 1e29
    ext = np.clip(b[..., 1::2] - b[..., 0::2], 0, None)
    area = np.where(ok, 2 * (ext[..., 0] * ext[..., 1] + ext[..., 1] * ext[..., 2] + ext[..., 2] * ext[..., 0]), 0)
    lo = np.min(np.where(ok[..., None], b[..., 0::2], np.inf), axis=(0, 1))
    hi = np.max(np.where(ok[..., None], b[..., 1::2], -np.inf), axis=(0, 1))
    e = hi - lo
    return float((2 * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0]) + area.sum()) / (2 * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0])))


def check_structure(tri, rec, tris, ids, depth, degenerate=()):
    n = tri.shape[0]
    t = np.asarray(tri, np.float32).reshape(-1, 9)
    assert np.array_equal(np.sort(ids), np.arange(n)), "ids are a permutation"
    assert np.array_equal(tris, t[ids]), "leaf-order triangles"
    ri = rec.view(np.int32)
    if n == 1:
        assert ri[0, 12] == ~0 and ri[0, 13] == ~0 and np.all(rec[0, 6:12] == FAR)
        return
    order, below = walk(rec)
    assert sorted(order) == list(range(n)), "every leaf once"
    assert order == list(range(n)), "leaves numbered left to right"
    assert len(below) == n - 1 and ri[0, 14] == -1 and ri[0, 15] == -1
    deg = set(int(k) for k in np.nonzero(np.isin(ids, list(degenerate)))[0])
    v = tris.reshape(-1, 3, 3)
    d = {0: 0}
    for i in range(n - 1):
        for h in (0, 1):
            c = ri[i, 12 + h]
            lo, hi = rec[i, 6 * h:6 * h + 6:2], rec[i, 6 * h + 1:6 * h + 6:2]
            good = [k for k in (below[c][0] + below[c][1] if c >= 0 else [~c]) if k not in deg]
            if not good:
                assert np.all(lo == FAR) and np.all(hi == FAR), (i, h)
            else:
                assert np.all(v[good].min((0, 1)) > lo) and np.all(v[good].max((0, 1)) < hi), (i, h)
            if c >= 0:
                assert ri[c, 14] == i and ri[c, 15] == ri[i, 13 - h], "parent and sibling words"
                d[int(c)] = d[i] + 1
    assert depth == max(d.values())


@pytest.mark.parametrize("n", [1, 2, 3, 17, 3000])
def test_structure_and_containment(n):
    tri = sg.TileTerrain(1).triangles()[:n]
    rec, tris, ids, depth = m.sah_build_host(tri)
    check_structure(tri, rec, tris, ids, depth)


def test_zero_area_triangles_are_unreachable():
    t = sg.TileTerrain(1).triangles()[:400].copy()
    p = t[::37, 0]
    u = np.float32([2.0 ** -6, 0.0, 0.0])
    deg = np.concatenate([np.stack([p, p, p], 1), np.stack([p - u, p, p + u], 1)], 0).astype(np.float32)
    tri = np.concatenate([t, deg], 0)
    rec, tris, ids, depth = m.sah_build_host(tri)
    check_structure(tri, rec, tris, ids, depth, degenerate=range(400, tri.shape[0]))


def test_coincident_centroids_are_halved():
    one = np.float32([[0, 0, 0], [1, 0, 0], [0, 1, 0]])
    tri = np.repeat(one[None], 9, 0)
    rec, tris, ids, depth = m.sah_build_host(tri)
    check_structure(tri, rec, tris, ids, depth)
    assert depth == 3  # 9 leaves halved: 4 + 5, ...


def test_deterministic_and_cheaper_than_the_morton_build():
    tri = sg.TileTerrain(2).triangles()[:6000]
    a = m.sah_build_host(tri)
    b = m.sah_build_host(tri)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
    morton = lbvh.build(tri)["records"]
    assert sah_cost(a[0]) < 0.95 * sah_cost(morton)


def test_rejects_bad_arguments():
    import ctypes
    L = m.lib()
    d = ctypes.c_int32()
    x = np.zeros((2, 9), np.float32)
    p = x.ctypes.data_as(ctypes.c_void_p)
    assert L.rc_sah_build_host(p, 0, p, p, p, ctypes.byref(d)) == -1
    assert L.rc_sah_build_host(None, 1, p, p, p, ctypes.byref(d)) == -1
    assert L.rc_sah_build_host(p, 1, p, p, p, ctypes.byref(d)) == -1  # tris_out aliases tri
    assert L.rc_scene_rebuild_sah(None, 1, None) == -1


def test_non_finite_coordinates_do_not_break_the_build():
    """A vertex that is NaN or infinite must not derail the binning: the
    build still places every triangle once and boxes the finite ones."""
    tri = sg.TileTerrain(1).triangles()[:500].copy()
    tri[7, 1, 0] = np.nan
    tri[11, 2, 2] = np.inf
    tri[13, 0, 1] = -np.inf
    rec, tris, ids, depth = m.sah_build_host(tri)
    assert np.array_equal(np.sort(ids), np.arange(500)) and 0 < depth < 64
    order, below = walk(rec)
    assert order == list(range(500))
    ri = rec.view(np.int32)
    finite = np.isfinite(tris.reshape(-1, 9)).all(1)
    v = tris.reshape(-1, 3, 3)
    for i in range(499):
        for h in (0, 1):
            c = ri[i, 12 + h]
            ks = [k for k in (below[c][0] + below[c][1] if c >= 0 else [~c]) if finite[k]]
            if ks and np.all(np.isfinite(rec[i, 6 * h:6 * h + 6])) and rec[i, 6 * h] != FAR:
                lo, hi = rec[i, 6 * h:6 * h + 6:2], rec[i, 6 * h + 1:6 * h + 6:2]
                assert np.all(v[ks].min((0, 1)) > lo) and np.all(v[ks].max((0, 1)) < hi), (i, h)
