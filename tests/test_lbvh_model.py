"""Pins for the CPU LBVH model: brute-force bit interleaving, the defining
properties of the Karras hierarchy, and box containment."""
import numpy as np
import pytest

from oracle import lbvh
import scenegen as sg


def test_morton_matches_bit_by_bit_interleave():
    rng = np.random.default_rng(0)
    q = rng.integers(0, 2 ** 21, size=(200, 3)).astype(np.uint32)
    fast = (lbvh._spread3(q[:, 0]) << np.uint64(2)) | (lbvh._spread3(q[:, 1]) << np.uint64(1)) | \
        lbvh._spread3(q[:, 2])
    for i in range(200):
        assert int(fast[i]) == lbvh.interleave_bits(q[i])


def test_morton_quantisation_is_isotropic_and_clamped():
    # centroids on a line along x from 0 to 8 and a tiny z range: x uses all 21
    # bits, z uses few (one scale for all axes)
    lo = np.zeros((3, 3), np.float32)
    lo[:, 0] = [0.0, 4.0, 8.0]
    lo[:, 2] = [0.0, 0.001, 0.002]
    keys = lbvh.morton_keys(lo, lo)
    qx = [sum(((int(k) >> (3 * b + 2)) & 1) << b for b in range(21)) for k in keys]
    qz = [sum(((int(k) >> (3 * b)) & 1) << b for b in range(21)) for k in keys]
    assert qx == [0, 2 ** 20, 2 ** 21 - 1]
    assert qz[2] == int(np.float32(0.002) * np.float32(2 ** 21 / 8.0))


def _leaf_ranges(c0, c1, n):
    """Leaves under every internal node, by explicit descent."""
    out = {}

    def leaves(ref):
        if ref < 0:
            return [~ref]
        if ref not in out:
            out[ref] = leaves(c0[ref]) + leaves(c1[ref])
        return out[ref]
    leaves(0)
    return out


def test_karras_hierarchy_properties():
    rng = np.random.default_rng(1)
    for n in (2, 3, 17, 64, 257):
        keys = np.sort(rng.integers(0, 2 ** 12, size=n).astype(np.uint64))  # many duplicates
        c0, c1, parent, sibling = lbvh.karras(keys)
        rng_of = _leaf_ranges(c0, c1, n)
        assert sorted(rng_of[0]) == list(range(n)), "every leaf reached exactly once"
        assert len(rng_of) == n - 1, "every internal node reachable from the root"
        for i, lv in rng_of.items():
            assert lv == list(range(lv[0], lv[-1] + 1)), "internal nodes cover contiguous ranges"
            left = rng_of[c0[i]] if c0[i] >= 0 else [~c0[i]]
            # split at the highest differing bit of (key, index) between the halves
            a, b = left[-1], left[-1] + 1

            def kd(u, v):
                if keys[u] != keys[v]:
                    return 64 - int(int(keys[u]) ^ int(keys[v])).bit_length()
                return 64 + 32 - int(u ^ v).bit_length()
            inside = min(kd(lv[0], lv[-1]), 1000)
            assert kd(a, b) == inside, "split at the node's common-prefix boundary"
            for c in (c0[i], c1[i]):
                if c >= 0:
                    assert parent[c] == i
                    assert sibling[c] == (c1[i] if c == c0[i] else c0[i])


def test_boxes_contain_children_and_leaves():
    tri = sg.TileTerrain(1).triangles()[:3000]
    m = lbvh.build(tri)
    rec = m["records"]
    ints = rec.view(np.int32)
    t = tri.reshape(-1, 9)[m["tri_id"]].reshape(-1, 3, 3)
    for i in range(rec.shape[0]):
        for h in (0, 1):
            lo, hi = rec[i, 6 * h:6 * h + 6:2], rec[i, 6 * h + 1:6 * h + 6:2]
            c = ints[i, 12 + h]
            if c < 0:
                assert np.all(t[~c].min(0) > lo) and np.all(t[~c].max(0) < hi)
            else:
                clo = np.minimum(rec[c, 0:6:2], rec[c, 6:12:2])
                chi = np.maximum(rec[c, 1:6:2], rec[c, 7:12:2])
                assert np.all(clo >= lo) and np.all(chi <= hi), "parents contain their children"


def _with_degenerate(n_good=400, seed=2):
    tri = sg.TileTerrain(1).triangles()[:n_good].copy()
    rng = np.random.default_rng(seed)
    p = tri[rng.choice(n_good, 30), 0]  # existing vertices
    q = tri[rng.choice(n_good, 30), 1]
    u = np.float32([2.0 ** -6, 0.0, 0.0])
    deg = np.concatenate([np.stack([p, p, p], 1), np.stack([p, q, p], 1),
                          np.stack([p - u, p, p + u], 1)], 0).astype(np.float32)
    return np.concatenate([tri, deg], 0), n_good


def test_degenerate_triangles_are_unreachable():
    """Zero-area triangles (three equal vertices, two equal, three on one
    line) keep their Morton codes, but their leaf boxes become the far point
    and every other box is the padded union of the non-degenerate leaves."""
    tri, n_good = _with_degenerate()
    assert np.array_equal(np.nonzero(lbvh.degenerate(tri))[0], np.arange(n_good, tri.shape[0]))
    m = lbvh.build(tri)
    lo, hi = lbvh.prim_boxes(tri)
    assert np.array_equal(m["keys"], np.sort(lbvh.morton_keys(lo, hi)))
    rec, ints = m["records"], m["records"].view(np.int32)
    t = tri.reshape(-1, 9)[m["tri_id"]].reshape(-1, 3, 3)
    is_deg = m["tri_id"] >= n_good

    def leaves(c):  # leaf indices below child c
        if c < 0:
            return [~c]
        return leaves(ints[c, 12]) + leaves(ints[c, 13])

    far = np.full(3, lbvh.FAR_POINT, np.float32)
    for i in range(rec.shape[0]):
        for h in (0, 1):
            blo, bhi = rec[i, 6 * h:6 * h + 6:2], rec[i, 6 * h + 1:6 * h + 6:2]
            good = [k for k in leaves(ints[i, 12 + h]) if not is_deg[k]]
            if not good:
                assert np.array_equal(blo, far) and np.array_equal(bhi, far)
                continue
            ulo, uhi = t[good].min((0, 1)), t[good].max((0, 1))
            plo, phi = lbvh._pad(ulo, uhi)
            assert np.array_equal(blo, plo) and np.array_equal(bhi, phi)


def test_single_degenerate_triangle():
    m = lbvh.build(np.array([[[0, 0, 0], [1, 1, 1], [2, 2, 2]]], np.float32))
    assert np.all(m["records"][0, :12] == lbvh.FAR_POINT)


# ---------------------------------------------------------------------------
# top level over the link instances
# ---------------------------------------------------------------------------

def _tlas_inputs(B=30, seed=7):
    rng = np.random.default_rng(seed)
    lp = rng.uniform(-0.6, 0.6, (B, 3)).astype(np.float32) + np.float32([3.0, -2.0, 0.8])
    lq = rng.normal(size=(B, 4)).astype(np.float32)
    half = rng.uniform(0.03, 0.15, (B, 3))
    root = np.stack([-half[:, 0], half[:, 0], -half[:, 1], half[:, 1], -half[:, 2], half[:, 2]],
                    1).astype(np.float32)
    return lp, lq, root


def test_tlas_transforms_match_scipy_and_boxes_hold_the_posed_link():
    from scipy.spatial.transform import Rotation
    lp, lq, root = _tlas_inputs()
    xf, rec = lbvh.tlas(lp, lq, root)
    for b in range(len(lp)):
        R = Rotation.from_quat(lq[b].astype(np.float64)).as_matrix()
        assert np.max(np.abs(xf[b, :9].reshape(3, 3) - R.T)) < 1e-6
        assert np.array_equal(xf[b, 9:], lp[b])
        corners = np.array([[root[b, i], root[b, 2 + j], root[b, 4 + k]]
                            for i in (0, 1) for j in (0, 1) for k in (0, 1)], np.float64)
        world = corners @ R.T + lp[b].astype(np.float64)
        lo, hi = lbvh.instance(lp[b], lq[b], root[b])[1][0::2], lbvh.instance(lp[b], lq[b], root[b])[1][1::2]
        assert np.all(world >= lo) and np.all(world <= hi)


@pytest.mark.parametrize("B", [2, 3, 30, 64])
def test_tlas_hierarchy_properties(B):
    lp, lq, root = _tlas_inputs(B, seed=B)
    xf, rec = lbvh.tlas(lp, lq, root)
    ints = rec.view(np.int32)
    c0, c1, par, sib = ints[:, 12], ints[:, 13], ints[:, 14], ints[:, 15]
    leaves = sorted(~c for c in np.concatenate([c0, c1]) if c < 0)
    assert leaves == list(range(B))  # every instance exactly once
    assert par[0] == -1
    for i in range(B - 1):
        for h, c in enumerate((c0[i], c1[i])):
            other = (c1[i], c0[i])[h]
            if c >= 0:
                assert par[c] == i and sib[c] == other
                child = rec[c, :12].reshape(2, 6)
                box = rec[i, 6 * h:6 * h + 6]
                assert np.all(child[:, 0::2] >= box[0::2]) and np.all(child[:, 1::2] <= box[1::2])
            else:
                box = rec[i, 6 * h:6 * h + 6]
                assert np.array_equal(box, lbvh.instance(lp[~c], lq[~c], root[~c])[1])


def test_tlas_absent_instances():
    lp, lq, root = _tlas_inputs(8, seed=3)
    lp[2, 1] = np.nan
    lq[5] = 0.0
    lq[6, 0] = np.inf
    xf, rec = lbvh.tlas(lp, lq, root)
    ints = rec.view(np.int32)
    for b in (2, 5, 6):
        assert np.array_equal(xf[b], np.float32([1, 0, 0, 0, 1, 0, 0, 0, 1, 1e30, 1e30, 1e30]))
    for i in range(7):
        for h, c in enumerate((ints[i, 12], ints[i, 13])):
            if c < 0 and ~c in (2, 5, 6):
                assert np.all(rec[i, 6 * h:6 * h + 6] == np.float32(1e30))


@pytest.mark.parametrize("case", ["terrain", "degenerate", "single"])
def test_collapse4_records_cover_every_leaf_once(case):
    """4-wide records: walking them from the root (internal slots only)
    reaches every leaf exactly once; every slot's box holds the triangles of
    the leaves below it (the far point only when all of them have zero area),
    and a record has two slots per child that it expands, one per child that
    it keeps, far-point empty slots after them."""
    if case == "terrain":
        tri, n_good = sg.TileTerrain(1).triangles()[:2000], 2000
    elif case == "degenerate":
        tri, n_good = _with_degenerate()
    else:
        tri, n_good = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), 1
    m = lbvh.build(tri)
    rec, ints = m["records"], m["records"].view(np.int32)
    w = lbvh.collapse4(rec)
    wi = w.view(np.int32)
    assert w.shape == (rec.shape[0], 32) and np.all(wi[:, 28:32] == 0)
    t = tri.reshape(-1, 9)[m["tri_id"]].reshape(-1, 3, 3)
    is_deg = m["tri_id"] >= n_good
    n = t.shape[0]

    def leaves(c):
        if c < 0:
            return [~c]
        return leaves(ints[c, 12]) + leaves(ints[c, 13])

    far = np.full(3, lbvh.FAR_POINT, np.float32)
    seen = []
    stack = [0]
    while stack:
        r = stack.pop()
        used = 0
        for h in (0, 1):
            c = ints[r, 12 + h]
            keep = c < 0 or rec[r, 6 * h] == lbvh.FAR_POINT
            used += 1 if keep else 2
        for k in range(4):
            lo, hi, c = w[r, k:24:4][0::2], w[r, k:24:4][1::2], wi[r, 24 + k]
            if k >= used:
                assert np.array_equal(lo, far) and np.array_equal(hi, far) and c == 0
                continue
            if n == 1 and k == 1:  # a one-leaf hierarchy's second child: the far point
                assert np.array_equal(lo, far) and c == ~0
                continue
            good = [i for i in leaves(c) if not is_deg[i]]
            if not good:
                assert np.array_equal(lo, far) and np.array_equal(hi, far)
                seen += leaves(c)
                continue
            assert np.all(t[good].min((0, 1)) > lo) and np.all(t[good].max((0, 1)) < hi)
            if c < 0:
                seen.append(~c)
            else:
                stack.append(c)
    assert sorted(seen) == list(range(n)), "every leaf reached once"
