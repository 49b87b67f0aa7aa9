"""Pins for the FP64 oracle against facts fixed outside the oracle itself.

Closed-form depths of the terrain profile (plane, 20 degree slope, treads,
risers), the published Philox known-answer vectors, PyTorch's independent
Philox source, SciPy rotations for the body transform, convex-solid
watertightness, permutation invariance and sensor-model statistics.
"""
import math
import os
import subprocess
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def look_quat(direction, up=(0.0, 0.0, 1.0)):
    """Quaternion (x,y,z,w) of a camera whose optical z is ``direction``."""
    z = np.asarray(direction, float)
    z = z / np.linalg.norm(z)
    up = np.asarray(up, float)
    if abs(np.dot(up, z)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return Rotation.from_matrix(np.stack([x, y, z], 1)).as_quat()


def render_points(tris, cams, far=10.0, link=None):
    """One 1x1 camera per env at cams[i] = (pos, dir): the ray goes along dir."""
    E = len(cams)
    pos = np.array([[c[0]] for c in cams], np.float32)
    quat = np.array([[look_quat(c[1])] for c in cams], np.float32)
    intr = np.tile(np.array([1.0, 1.0, 0.5, 0.5], np.float32), (E, 1, 1))
    if link is None:
        lt, lo = np.zeros((0, 3, 3), np.float32), np.zeros(1, np.int64)
        lp, lq = np.zeros((E, 0, 3), np.float32), np.zeros((E, 0, 4), np.float32)
    else:
        lt, lo, lp, lq = link
    return oracle.render(tris, lt, lo, lp, lq, pos, quat, intr, 1, 1, far)


def profile_closed_form(w):
    """Independent closed-form depth for every pixel of the small plain case.

    The ray is built from the optical axes stated for this camera (1 m above
    the ground, pitched 45 degrees down), not from its quaternion.
    Returns (depth, piece index, near_boundary flag).
    """
    terr = w["terrain_obj"]
    K = w["intr"][0, 0].astype(np.float64)
    s2 = 1.0 / math.sqrt(2.0)
    ax = np.array([0.0, -1.0, 0.0])
    ay = np.array([-s2, 0.0, -s2])
    az = np.array([s2, 0.0, -s2])
    o = np.array([0.0, 0.0, 1.0])
    H, W = w["H"], w["W"]
    depth = np.full((H, W), w["far"])
    piece = np.full((H, W), -1)
    nearb = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            a = (x + 0.5 - K[2]) / K[0]
            b = (y + 0.5 - K[3]) / K[1]
            d = az + a * ax + b * ay
            best = math.inf
            for k, (xa, za, xb, zb, yh) in enumerate(terr.pieces()):
                n = np.array([-(zb - za), 0.0, xb - xa])
                den = n @ d
                if den == 0.0:
                    continue
                lam = n @ (np.array([xa, 0.0, za]) - o) / den
                if not (lam > 0):
                    continue
                P = o + lam * d
                L2 = (xb - xa) ** 2 + (zb - za) ** 2
                s = ((P[0] - xa) * (xb - xa) + (P[2] - za) * (zb - za)) / L2
                L = math.sqrt(L2)
                if -1e-12 <= s <= 1 + 1e-12 and abs(P[1]) <= yh and lam < best:
                    best = lam
                    piece[y, x] = k
                    nearb[y, x] = min(s * L, (1 - s) * L, yh - abs(P[1])) < 1e-6
            if best <= w["far"]:
                depth[y, x] = best
    return depth, piece, nearb


# ---------------------------------------------------------------------------
# ray generation, intersection and depth semantics
# ---------------------------------------------------------------------------

def small_render(depth_mode=0):
    w = sg.small_plain_case()
    r = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                      w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"],
                      w["W"], w["H"], w["far"], depth_mode=depth_mode)
    return w, r


def test_plane_closed_form_rows():
    """Ground z = 0 seen from h = 1 m at 45 deg: depth(y) = sqrt(2) h / (1 + b)."""
    w, r = small_render()
    d = r["depth"].reshape(w["H"], w["W"])
    fy, cy = float(w["intr"][0, 0, 1]), float(w["intr"][0, 0, 3])
    checked = 0
    for y in range(w["H"]):
        b = (y + 0.5 - cy) / fy
        lam = math.sqrt(2.0) / (1.0 + b)
        xhit = lam * (1.0 / math.sqrt(2.0) - b / math.sqrt(2.0))  # along +x
        if xhit < 0.79:
            assert np.all(np.abs(d[y] - lam) <= 1e-6), (y, d[y] - lam)
            checked += 1
    assert checked >= 6


def test_profile_closed_form_all_pixels():
    w, r = small_render()
    d = r["depth"].reshape(w["H"], w["W"])
    cf, piece, nearb = profile_closed_form(w)
    ok = ~nearb
    assert np.max(np.abs(d - cf)[ok]) <= 1e-6
    # the image must see the plane, the slope, a riser and a tread
    seen = set(np.unique(piece[ok]).tolist())
    assert {0, 1}.issubset(seen)            # ground and 20 degree slope
    assert seen & {3, 5, 7}                  # a riser
    assert seen & {4, 6, 8}                  # a tread or the top landing
    assert np.all(r["inst"] == 0)            # terrain is inst B = 0 with no robot


def test_range_mode_scales_planar_depth():
    w, rp = small_render(0)
    _, rr = small_render(1)
    K = w["intr"][0, 0].astype(np.float64)
    y, x = np.divmod(np.arange(w["H"] * w["W"]), w["W"])
    a = (x + 0.5 - K[2]) / K[0]
    b = (y + 0.5 - K[3]) / K[1]
    norm = np.sqrt(1 + a * a + b * b)
    hit = rr["depth"] < w["far"] - 1e-9
    np.testing.assert_allclose(rr["depth"][hit], rp["depth"][hit] * norm[hit], rtol=1e-12)


def test_single_triangle_and_far_plane():
    tri = np.array([[[-1, -1, 0], [3, -1, 0], [-1, 3, 0]]], np.float32)
    r = render_points(tri, [((0, 0, 2), (0, 0, -1)), ((0, 0, 5), (0, 0, -1))], far=3.0)
    assert r["depth"][0] == pytest.approx(2.0, abs=1e-12) and r["inst"][0] == 0 and r["tri"][0] == 0
    assert r["depth"][1] == 3.0 and r["inst"][1] == -1 and r["tri"][1] == -1
    # a hit exactly behind the origin does not count (lambda > 0)
    r = render_points(tri, [((0, 0, -1), (0, 0, -1))], far=3.0)
    assert r["inst"][0] == -1


def test_tie_rules():
    A = [[-1, -1, 0], [3, -1, 0], [-1, 3, 0]]
    tri = np.array([A, A], np.float32)
    r = render_points(tri, [((0, 0, 2), (0, 0, -1))])
    assert r["tri"][0] == 0
    # the same triangle as link 0 (identity pose) and as terrain: the link wins
    link = (np.array([A], np.float32), np.array([0, 1], np.int64),
            np.zeros((1, 1, 3), np.float32), np.array([[[0, 0, 0, 1]]], np.float32))
    r = render_points(np.array([A], np.float32), [((0, 0, 2), (0, 0, -1))], link=link)
    assert r["inst"][0] == 0 and r["tri"][0] == 0
    assert r["flags"][0] & oracle.FLAG_TIE


def flat_tri(z, shift=-1.0):
    """A horizontal right triangle at height z whose edge x = shift passes at
    lateral distance |shift| from the vertical ray through (0, 0): at that ray
    its barycentrics are (-shift/4, 1/4, 3/4 + shift/4), so the default
    contains the ray well inside (1/4 from every edge)."""
    s = np.float32(shift)
    return [[s, -1, z], [s + 4, -1, z], [s, 3, z]]


def test_candidate_list_contents_and_order():
    """The band candidates (what the weak check may accept) of a hit ray are
    exactly the closed-enough surfaces within 1e-4 m beyond the hit, nearest
    first: the depths come from the triangles' heights (ray from z = 2 going
    straight down), the ids from their input order."""
    z_b = np.float32(-0.5e-4)   # 2.00005 m: inside the 1e-4 m band
    z_c = np.float32(-2e-4)     # 2.0002 m: beyond it
    z_e = np.float32(-0.3e-4)   # 2.00003 m, but min barycentric -5e-7 (edge band)
    z_m = np.float32(-0.2e-4)   # 2.00002 m, min barycentric -2e-6 (outside the edge band)
    tris = np.array([flat_tri(z_c),            # 0: too deep
                     flat_tri(z_b),            # 1: candidate, second nearest
                     flat_tri(z_m, 8e-6),      # 2: misses by more than the band
                     flat_tri(0.0),            # 3: the hit
                     flat_tri(z_e, 2e-6),      # 4: edge-band candidate
                     flat_tri(3.0)],           # 5: behind the origin (lambda < 0)
                    np.float32)
    r = render_points(tris, [((0, 0, 2), (0, 0, -1))], far=10.0)
    assert r["inst"][0] == 0 and r["tri"][0] == 3 and r["depth"][0] == pytest.approx(2.0, abs=1e-12)
    cand, cd = r["cand"][0], r["cand_depth"][0]
    got = [tuple(c) for c in cand if c[0] >= 0]
    assert got == [(0, 3), (0, 4), (0, 1)]
    np.testing.assert_allclose(cd[:3], [2.0, 2.0 - float(z_e), 2.0 - float(z_b)], rtol=0, atol=1e-12)
    assert np.all(np.isnan(cd[3:])) and np.all(cand[3:] == -1)
    # the edge-band candidate sets EDGE; no TIE (1e-5 m) and no FAR
    assert r["flags"][0] == oracle.FLAG_EDGE
    # without the edge-band triangle the ray is unflagged and keeps two candidates
    r = render_points(tris[[0, 1, 2, 3, 5]], [((0, 0, 2), (0, 0, -1))], far=10.0)
    assert r["flags"][0] == 0
    assert [tuple(c) for c in r["cand"][0] if c[0] >= 0] == [(0, 3), (0, 1)]
    # a candidate list holds the K nearest only
    r = oracle.render(tris, np.zeros((0, 3, 3), np.float32), np.zeros(1, np.int64),
                      np.zeros((1, 0, 3)), np.zeros((1, 0, 4)), np.float32([[[0, 0, 2]]]),
                      np.float32([[look_quat((0, 0, -1))]]), np.float32([[[1, 1, .5, .5]]]),
                      1, 1, 10.0, K=2)
    assert [tuple(c) for c in r["cand"][0]] == [(0, 3), (0, 4)]


def test_candidate_list_of_a_link_hit_lists_links_before_terrain():
    """Equal depths: the link's candidate comes first (links precede the
    terrain in the order of Algorithm 1's queries), and the pair is a TIE."""
    A = flat_tri(0.0)
    link = (np.array([A], np.float32), np.array([0, 1], np.int64),
            np.zeros((1, 1, 3), np.float32), np.array([[[0, 0, 0, 1]]], np.float32))
    r = render_points(np.array([A, flat_tri(np.float32(-0.5e-4))], np.float32),
                      [((0, 0, 2), (0, 0, -1))], link=link)
    assert r["inst"][0] == 0 and r["tri"][0] == 0
    assert [tuple(c) for c in r["cand"][0] if c[0] >= 0] == [(0, 0), (1, 0), (1, 1)]
    assert r["flags"][0] == oracle.FLAG_TIE


@pytest.mark.parametrize("dz,hit,flag", [
    (0.0, True, True),          # a hit exactly at the far plane counts and is in the band
    (-0.5e-5, True, True),      # 0.5e-5 m before it: a hit, in the band
    (+0.5e-5, False, True),     # 0.5e-5 m beyond it: a miss, in the band
    (-2e-5, True, False),       # 2e-5 m before: a plain hit
    (+2e-5, False, False),      # 2e-5 m beyond: a plain miss
])
def test_far_band_flag(dz, hit, flag):
    far = 2.0
    z = np.float32(-np.float32(dz))    # the ray goes down from z = 2: depth = 2 - z
    # quaternion (1, 0, 0, 0): a half turn about x, so optical z is exactly -z
    r = oracle.render(np.array([flat_tri(z)], np.float32), np.zeros((0, 3, 3), np.float32),
                      np.zeros(1, np.int64), np.zeros((1, 0, 3)), np.zeros((1, 0, 4)),
                      np.float32([[[0, 0, 2]]]), np.float32([[[1, 0, 0, 0]]]),
                      np.float32([[[1, 1, .5, .5]]]), 1, 1, far)
    depth = 2.0 - float(z)
    assert (r["inst"][0] == 0) == hit
    assert r["depth"][0] == (depth if hit else far)
    assert bool(r["flags"][0] & oracle.FLAG_FAR) == flag
    assert r["flags"][0] & ~oracle.FLAG_FAR == 0
    # the band's surface is a candidate; a plain miss has none
    cands = [tuple(c) for c in r["cand"][0] if c[0] >= 0]
    assert cands == ([(0, 0)] if (hit or flag) else [])


def test_far_band_not_set_for_a_miss_into_empty_space():
    tri = np.array([flat_tri(0.0)], np.float32)
    r = render_points(tri, [((0, 0, 2), (0, 0, 1))], far=3.0)   # looking up, away from it
    assert r["inst"][0] == -1 and r["depth"][0] == 3.0 and r["flags"][0] == 0
    assert np.all(r["cand"][0] == -1)


def random_scene(seed, n_tri=40, E=2, C=2, W=9, H=7):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, (n_tri, 1, 3)) * [2, 2, 0.3] + [2.0, 0, 0]
    terr = (c + rng.normal(0, 0.4, (n_tri, 3, 3))).astype(np.float32)
    V, T = sg.octasphere(3)
    link = (V[T] * 0.35).astype(np.float32)
    lp = rng.uniform(-0.3, 0.3, (E, 1, 3)).astype(np.float32) + np.float32([1.2, 0, 0.3])
    lq = rng.normal(size=(E, 1, 4)).astype(np.float32)
    cp = np.zeros((E, C, 3), np.float32) + np.float32([0, 0, 1.0])
    cq = np.array([[look_quat((1.0, rng.uniform(-.3, .3), -0.6)) for _ in range(C)] for _ in range(E)],
                  np.float32)
    intr = np.tile(np.float32([6, 6, W / 2, H / 2]), (E, C, 1))
    return terr, link, lp, lq, cp, cq, intr, W, H


def test_zero_area_triangles_are_never_hit():
    """A triangle with no interior (equal or collinear vertices) is met by no
    ray, also by a ray through its points; a proper triangle through the same
    point is hit there."""
    p = np.array([0.25, -0.5, 1.0], np.float32)
    q = np.array([0.75, 0.5, 1.25], np.float32)
    u = np.float32([2.0 ** -6, 0.0, 0.0])
    tris = {"point": [p, p, p], "pair": [p, q, p], "line": [p - u, p, p + u],
            "slanted line": [p - 2 * (q - p), p, q]}
    good = np.array([[[-1, -1, 1], [2, -1, 1], [-1, 2, 1]]], np.float32)
    cam_pos = np.zeros((1, 1, 3), np.float32)
    # optical axis through p: a 1x1 image whose pixel centre ray is (0.25, -0.5, 1)
    intr = np.array([[[1.0, 1.0, 0.25, 1.0]]], np.float32)
    quat = np.array([[[0.0, 0.0, 0.0, 1.0]]], np.float32)
    empty = (np.zeros((0, 3, 3), np.float32), np.zeros(1, np.int64),
             np.zeros((1, 0, 3), np.float32), np.zeros((1, 0, 4), np.float32))
    for name, t in tris.items():
        t = np.asarray(t, np.float32)[None]
        r = oracle.render(t, *empty, cam_pos, quat, intr, 1, 1, 3.0)
        assert r["inst"][0] == -1 and r["depth"][0] == 3.0, name
        r = oracle.render(np.concatenate([t, good], 0), *empty, cam_pos, quat, intr, 1, 1, 3.0)
        assert r["inst"][0] == 0 and r["tri"][0] == 1 and r["depth"][0] == pytest.approx(1.0), name


def test_permutation_invariance():
    terr, link, lp, lq, cp, cq, intr, W, H = random_scene(1)
    off = np.array([0, link.shape[0]], np.int64)
    r0 = oracle.render(terr, link, off, lp, lq, cp, cq, intr, W, H, 5.0)
    perm = np.random.default_rng(2).permutation(terr.shape[0])
    r1 = oracle.render(terr[perm], link, off, lp, lq, cp, cq, intr, W, H, 5.0)
    assert np.array_equal(r0["depth"], r1["depth"])
    assert np.array_equal(r0["inst"], r1["inst"])
    terr_hit = r0["inst"] == 1
    assert terr_hit.sum() > 10 and (r0["inst"] == 0).sum() > 5
    assert np.array_equal(r0["tri"][terr_hit], perm[r1["tri"][terr_hit]])


def test_body_transform_matches_world_placement():
    """A posed link equals its triangles placed in the world by SciPy's rotation."""
    terr, link, lp, lq, cp, cq, intr, W, H = random_scene(3, n_tri=1)
    E = lp.shape[0]
    empty = np.zeros((0, 3, 3), np.float32)
    off = np.array([0, link.shape[0]], np.int64)
    r_link = oracle.render(empty, link, off, lp, lq, cp, cq, intr, W, H, 5.0)
    for e in range(E):
        R = Rotation.from_quat(lq[e, 0].astype(np.float64)).as_matrix()
        world = (link.astype(np.float64) @ R.T + lp[e, 0]).astype(np.float64)
        sl = slice(e * 2 * W * H, (e + 1) * 2 * W * H)
        r_w = oracle.render(world, np.zeros((0, 3, 3), np.float32), np.zeros(1, np.int64),
                            np.zeros((1, 0, 3)), np.zeros((1, 0, 4)), cp[e:e + 1], cq[e:e + 1],
                            intr[e:e + 1], W, H, 5.0)
        hit = r_w["inst"] >= 0
        assert hit.sum() > 5
        # world vertices were rounded to float32, so allow that rounding only
        assert np.max(np.abs(r_w["depth"] - r_link["depth"][sl])) < 2e-6
        same = (r_w["flags"] == 0) & (r_link["flags"][sl] == 0)
        assert np.array_equal(r_w["tri"][same], r_link["tri"][sl][same])


@pytest.mark.parametrize("bad", ["nan_pos", "inf_pos", "nan_quat", "inf_quat", "zero_quat"])
def test_link_with_non_finite_pose_is_absent(bad):
    """A link whose pose places it nowhere (a non-finite component, a zero
    quaternion) is absent: env 0 renders as the scene without that link
    (instance ids of the later links and the terrain shift down by one), env 1
    is unchanged."""
    terr, link, lp, lq, cp, cq, intr, W, H = random_scene(5)
    lp2 = np.concatenate([lp, lp + np.float32([0.1, 0.25, 0.0])], 1)
    lq2 = np.concatenate([lq, lq[:, :, [1, 0, 3, 2]]], 1)
    links = np.concatenate([link, link], 0)
    off2 = np.array([0, link.shape[0], 2 * link.shape[0]], np.int64)
    full = oracle.render(terr, links, off2, lp2, lq2, cp, cq, intr, W, H, 5.0)
    assert (full["inst"] == 0).sum() > 5
    bp, bq = lp2.copy(), lq2.copy()
    if bad == "nan_pos":
        bp[0, 0, 1] = np.nan
    elif bad == "inf_pos":
        bp[0, 0, 0] = np.inf
    elif bad == "nan_quat":
        bq[0, 0, 2] = np.nan
    elif bad == "inf_quat":
        bq[0, 0, 3] = -np.inf
    else:
        bq[0, 0] = 0.0
    r = oracle.render(terr, links, off2, bp, bq, cp, cq, intr, W, H, 5.0)
    off1 = np.array([0, link.shape[0]], np.int64)
    one = oracle.render(terr, link, off1, lp2[:, 1:], lq2[:, 1:], cp, cq, intr, W, H, 5.0)
    n0 = 2 * W * H  # env 0's rays come first
    exp_inst = np.where(one["inst"][:n0] >= 0, one["inst"][:n0] + 1, -1)
    assert np.array_equal(r["inst"][:n0], exp_inst)
    assert np.array_equal(r["tri"][:n0], one["tri"][:n0])
    assert np.array_equal(r["depth"][:n0], one["depth"][:n0])
    for k in ("inst", "tri", "depth", "flags"):
        assert np.array_equal(r[k][n0:], full[k][n0:])


def test_quaternion_sign_invariance():
    terr, link, lp, lq, cp, cq, intr, W, H = random_scene(4)
    off = np.array([0, link.shape[0]], np.int64)
    a = oracle.render(terr, link, off, lp, lq, cp, cq, intr, W, H, 5.0)
    b = oracle.render(terr, link, off, lp, -lq, cp, -cq, intr, W, H, 5.0)
    assert np.array_equal(a["inst"], b["inst"]) and np.array_equal(a["tri"], b["tri"])
    assert np.max(np.abs(a["depth"] - b["depth"])) < 1e-12


def test_watertight_closed_convex_mesh():
    """Rays aimed at every vertex and edge midpoint of a convex closed mesh hit it
    at the aimed point (the solid is convex, so that point is the first hit)."""
    V, T = sg.octasphere(3)
    tris = V[T].astype(np.float32)
    Vf = tris.reshape(-1, 3).astype(np.float64)
    targets = {tuple(v) for v in Vf}
    for t in tris.astype(np.float64):
        for i in range(3):
            targets.add(tuple(0.5 * (t[i] + t[(i + 1) % 3])))
    targets = np.array(sorted(targets))
    cams = [(3.0 * p / np.linalg.norm(p), -p) for p in targets]
    r = render_points(tris, cams, far=10.0)
    assert np.all(r["inst"] == 0)
    expect = np.array([np.linalg.norm(3.0 * p / np.linalg.norm(p) - p) for p in targets])
    assert np.max(np.abs(r["depth"] - expect)) < 1e-5
    assert np.mean((r["flags"] & oracle.FLAG_EDGE) > 0) > 0.99


# ---------------------------------------------------------------------------
# counter-based generator
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        assert oracle.philox(v[0:4], v[4:6]).tolist() == v[6:10]


TORCH_PHILOX_PROBE = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  for (int i = 1; i + 2 < argc; i += 3) {
    unsigned long long seed = strtoull(argv[i], 0, 0), sub = strtoull(argv[i+1], 0, 0),
                       off = strtoull(argv[i+2], 0, 0);
    at::Philox4_32 eng(seed, sub, off);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


def test_philox_matches_pytorch_source(tmp_path):
    """PyTorch ships an independent Philox4x32-10 (header source); compare words.

    at::Philox4_32(seed, subsequence, offset) encrypts the counter
    (offset_lo, offset_hi, subsequence_lo, subsequence_hi) with key (seed_lo, seed_hi).
    """
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(TORCH_PHILOX_PROBE)
    subprocess.check_call(["g++", "-O1", "-std=c++17", f"-I{inc}", str(src), "-o", str(exe)])
    rng = np.random.default_rng(7)
    cases = [(int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63)), int(rng.integers(0, 2**63)))
             for _ in range(20)]
    args = [str(x) for c in cases for x in c]
    out = subprocess.check_output([str(exe)] + args).decode().split("\n")
    for (seed, sub, off), line in zip(cases, out):
        ctr = [off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        assert oracle.philox(ctr, key).tolist() == [int(x) for x in line.split()]


# ---------------------------------------------------------------------------
# sensor model
# ---------------------------------------------------------------------------

def test_post_identity_when_everything_off():
    depth, inst = sg.synthetic_frames(2, 2, 5, 7, 3)
    p = oracle.make_params(seed=5, near=0.05, far=3.0)
    out, drop, lat = oracle.post(depth, inst, p)
    near, far = float(np.float32(0.05)), float(np.float32(3.0))  # parameters are FP32
    expect = np.where(inst >= 0, np.clip(depth.astype(np.float64), near, far), far)
    assert np.array_equal(out, expect)
    assert not drop.any() and not lat.any()


def test_post_dropout_rate_and_fill():
    depth, inst = sg.synthetic_frames(4, 2, 48, 64, 4)
    p = oracle.make_params(seed=11, p_drop=0.02, fill=-1.0)
    out, drop, _ = oracle.post(depth, inst, p)
    n = drop.size
    rate = drop.mean()
    assert abs(rate - 0.02) < 5 * math.sqrt(0.02 * 0.98 / n)
    assert np.all(out[drop == 1] == -1.0)
    p0 = oracle.make_params(seed=11, p_drop=0.0, flags=oracle.POST_DROPOUT)
    assert not oracle.post(depth, inst, p0)[1].any()
    p1 = oracle.make_params(seed=11, p_drop=1.0)
    assert oracle.post(depth, inst, p1)[1].all()


def test_post_noise_statistics():
    S, E, C, H, W = 2, 4, 2, 48, 64
    depth = np.full((S, E, C, H, W), 1.5, np.float32)
    inst = np.zeros((S, E, C, H, W), np.int32)
    p = oracle.make_params(seed=3, sigma_abs=0.01, near=0.05, far=3.0)
    out, _, _ = oracle.post(depth, inst, p)
    g = (out - 1.5) / 0.01
    n = g.size
    assert abs(g.mean()) < 5 / math.sqrt(n)
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    # kurtosis of a Gaussian is 3
    assert abs(np.mean(g ** 4) / g.var() ** 2 - 3.0) < 0.1
    # relative noise scales with depth
    p2 = oracle.make_params(seed=3, sigma_rel=0.1, near=0.0, far=100.0)
    out2, _, _ = oracle.post(depth, inst, p2)
    assert abs(np.std(out2 - 1.5) / 0.15 - 1.0) < 0.02
    # misses get no noise
    inst[:] = -1
    out3, _, _ = oracle.post(depth, inst, p)
    assert np.all(out3 == 3.0)


def test_post_latency_semantics_and_histogram():
    S, E, C, H, W = 12, 3, 2, 2, 3
    vals = 0.5 + 0.1 * np.arange(S)
    depth = np.broadcast_to(vals[:, None, None, None, None], (S, E, C, H, W)).astype(np.float32).copy()
    inst = np.zeros((S, E, C, H, W), np.int32)
    s0 = 40
    p = oracle.make_params(seed=9, lat_min=1, lat_max=3)
    out, _, lat = oracle.post(depth, inst, p, s0=s0)
    for si in range(S):
        for ec in range(E * C):
            k = int(lat[si].ravel()[ec])
            assert 1 <= k <= 3
            src = max(si - k, 0)
            assert np.all(out[si].reshape(E * C, -1)[ec] == np.float64(np.float32(vals[src])))
    ks = np.array([oracle.latency(p, u, s) for u in range(200) for s in range(30)])
    counts = np.bincount(ks, minlength=4)[1:]
    expect = ks.size / 3
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 13.8  # chi-square, 2 dof, p = 0.001


# ---------------------------------------------------------------------------
# block pooling of frames (240x135 -> 48x27, Sec. 4.1)
# ---------------------------------------------------------------------------

def test_downsample_worked_example():
    far = 3.0
    depth = np.array([[1.0, 2.0, 5.0, 5.0],
                      [3.0, 9.0, 5.0, 5.0]])
    inst = np.array([[0, 4, -1, -1],
                     [30, -1, -1, -1]])
    out = oracle.downsample(depth[None], inst[None], 2, far)[0]
    # block 0: hits 1, 2, 3 (the 9 is a miss), block 1: no hit -> far
    assert out.shape == (1, 2)
    assert out[0, 0] == pytest.approx(2.0, abs=0) and out[0, 1] == far


def test_downsample_constant_all_hit_and_all_miss():
    d = np.full((2, 3, 10, 15), 1.25)
    hit = np.zeros(d.shape, np.int32)
    assert np.all(oracle.downsample(d, hit, 5, 3.0) == 1.25)
    assert np.all(oracle.downsample(d, hit - 1, 5, 3.0) == 3.0)


def test_downsample_brute_force_and_trailing_pixels():
    rng = np.random.default_rng(4)
    H, W, f = 7, 11, 3
    d = rng.uniform(0.1, 3.0, (2, H, W))
    inst = rng.integers(-1, 3, (2, H, W))
    got = oracle.downsample(d, inst, f, 3.0)
    assert got.shape == (2, H // f, W // f)
    for i in range(2):
        for y in range(H // f):
            for x in range(W // f):
                vals = [d[i, yy, xx] for yy in range(y * f, y * f + f) for xx in range(x * f, x * f + f)
                        if inst[i, yy, xx] >= 0]
                want = sum(vals) / len(vals) if vals else 3.0
                assert got[i, y, x] == pytest.approx(want, rel=1e-15, abs=1e-15)


# ---------------------------------------------------------------------------
# perception randomisation of the cameras (the paper's Table 6)
# ---------------------------------------------------------------------------

def _cams(n, seed=3):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-5, 5, (n, 3))
    quat = Rotation.random(n, random_state=seed).as_quat()
    intr = np.tile([33.72, 43.30, 32.0, 24.0], (n, 1))
    return pos, quat, intr


def test_cam_randomize_zero_ranges_is_identity():
    pos, quat, intr = _cams(50)
    c = oracle.cam_randomize(pos, quat, intr, np.arange(50), 7, 0, [0, 0, 0], [0, 0, 0], 0.0)
    R0 = Rotation.from_quat(quat).as_matrix()
    assert np.allclose(c[:, :9].reshape(-1, 3, 3), R0, atol=1e-14)
    assert np.array_equal(c[:, 9:12], pos)
    assert np.array_equal(c[:, 12:], intr)


def test_cam_randomize_offsets_within_ranges_and_uniform():
    from scipy import stats
    n = 4000
    pos, quat, intr = _cams(n)
    tr, eu, fov = [0.025, 0.025, 0.025], [2.5, 3.0, 2.5], 2.0
    c = oracle.cam_randomize(pos, quat, intr, np.arange(n), 11, 5, tr, eu, fov)
    R0 = Rotation.from_quat(quat).as_matrix()
    # translation in the camera's own frame
    t_local = np.einsum("nji,nj->ni", R0, c[:, 9:12] - pos)
    assert np.all(np.abs(t_local) <= 0.025 + 1e-12)
    # rotation: R0^T R = Rx(phi) Ry(theta) Rz(psi), an intrinsic x-y-z sequence
    rel = np.einsum("nji,njk->nik", R0, c[:, :9].reshape(-1, 3, 3))
    ang = Rotation.from_matrix(rel).as_euler("XYZ", degrees=True)
    assert np.all(np.abs(ang) <= np.array(eu) + 1e-9)
    # field of view: both axes widened or narrowed by the same offset
    dh = np.degrees(2 * np.arctan(intr[:, 2] / c[:, 12]) - 2 * np.arctan(intr[:, 2] / intr[:, 0]))
    dv = np.degrees(2 * np.arctan(intr[:, 3] / c[:, 13]) - 2 * np.arctan(intr[:, 3] / intr[:, 1]))
    assert np.allclose(dh, dv, atol=1e-9) and np.all(np.abs(dh) <= fov + 1e-9)
    for x, a in ((t_local[:, 0], 0.025), (ang[:, 1], 3.0), (dh, 2.0)):
        assert stats.kstest(x, "uniform", args=(-a, 2 * a)).pvalue > 1e-3
    # independent per camera uid and per epoch
    c2 = oracle.cam_randomize(pos, quat, intr, np.arange(n), 11, 6, tr, eu, fov)
    assert not np.allclose(c2[:, 9:12], c[:, 9:12])


# ---------------------------------------------------------------------------
# random side masking (Sec. 3.2)
# ---------------------------------------------------------------------------

def _masked(frac, p, E=200, W=16, types=None, epoch=0):
    out = np.full((1, E, 1, 2, W), 1.5)
    drop = np.ones(out.shape, np.uint8)
    modes = oracle.side_mask(out, drop, 9, 0.05, 3.0, 0, frac, p, epoch, types)
    return out, drop, modes


def test_side_mask_certain_modes_and_bands():
    for p, mode, m in (((1, 0, 0), 0, 0), ((0, 1, 0), 1, 2), ((0, 0, 1), 2, 4)):
        out, drop, modes = _masked((0.125, 0.25), [p] * 4, E=5)
        assert np.all(modes == mode)
        band = np.zeros(16, bool)
        band[:m] = True
        band[16 - m:] = True
        assert np.all(out[..., band] != 1.5) and np.all(out[..., ~band] == 1.5)
        assert np.all(drop[..., band] == 0) and np.all(drop[..., ~band] == 1)


def test_side_mask_mode_rates_fill_range_and_types():
    from scipy import stats
    out, drop, modes = _masked((0.125, 0.25), [(0.5, 0.2, 0.3)] * 4, E=3000)
    for k, pk in enumerate((0.5, 0.2, 0.3)):
        n = int(np.sum(modes == k))
        assert stats.binomtest(n, 3000, pk).pvalue > 1e-4
    vals = out[out != 1.5]
    assert np.all((vals >= 0.05) & (vals < 3.0))
    assert stats.kstest(vals, "uniform", args=(0.05, 2.95)).pvalue > 1e-3
    # terrain type selects the probabilities
    types = np.array([0, 1] * 50)
    _, _, modes = _masked((0.125, 0.25), [(0, 1, 0), (0, 0, 1), (1, 0, 0), (1, 0, 0)], E=100,
                          types=types)
    assert np.all(modes[types == 0] == 1) and np.all(modes[types == 1] == 2)


# ---------------------------------------------------------------------------
# privileged height map (Sec. 3.1)
# ---------------------------------------------------------------------------

def test_heightmap_against_analytic_terrain():
    """Vertical rays against the meshed tile terrain equal the tiles' analytic
    surface heights except next to a vertical step (riser or stone edge)."""
    terr = sg.TileTerrain(2, seed=sg.MASTER_SEED)
    tri = terr.triangles()
    rng = np.random.default_rng(12)
    E = 6
    xy = np.stack([rng.uniform(-6, 6, E), rng.uniform(-6, 6, E)], 1)
    base = np.concatenate([xy, [[terr.height(x, y) + 0.75] for x, y in xy]], 1)
    yaw = rng.uniform(0, 2 * np.pi, E)
    hm = oracle.heightmap(tri, base, yaw, 17, 11, 0.1, 0.1, 2.0, 5.0)
    base32, yaw32 = base.astype(np.float32).astype(np.float64), yaw.astype(np.float32).astype(np.float64)
    checked = 0
    for e in range(E):
        c, s = np.cos(yaw32[e]), np.sin(yaw32[e])
        for j in range(11):
            for i in range(17):
                gx, gy = (i - 8) * 0.1, (j - 5) * 0.1
                x, y = base32[e, 0] + c * gx - s * gy, base32[e, 1] + s * gx + c * gy
                near = [terr.height(x + a, y + b) for a in (-1e-6, 0, 1e-6) for b in (-1e-6, 0, 1e-6)]
                if max(near) - min(near) > 1e-6:
                    continue  # a vertical step: either side is a valid answer
                assert hm[e, j, i] == pytest.approx(near[4] - base32[e, 2], abs=2e-6)
                checked += 1
    assert checked > 0.8 * E * 17 * 11


def test_heightmap_grid_geometry_and_miss():
    """A single flat triangle: heights are z - base_z inside, `miss` outside,
    and the grid is centred on the base and turned by the yaw."""
    tri = np.array([[[-1.0, -1.0, 0.2], [3.0, -1.0, 0.2], [-1.0, 3.0, 0.2]]], np.float32)
    hm = oracle.heightmap(tri, [[0.0, 0.0, 1.0]], [np.pi / 2], 17, 11, 0.1, 0.1, 1.0, 3.0, miss=-9.0)
    assert hm.shape == (1, 11, 17)
    assert hm[0, 5, 8] == pytest.approx(-0.8, abs=1e-7)
    # yaw 90 degrees: the heading is +y, so grid x maps to world y
    # world point of (i, j) = (-(j - 5) 0.1, (i - 8) 0.1); inside the triangle iff x + y <= 2
    inside = np.array([[(-(j - 5) * 0.1) + ((i - 8) * 0.1) <= 2 and (-(j - 5) * 0.1) >= -1
                        and ((i - 8) * 0.1) >= -1 for i in range(17)] for j in range(11)])
    assert np.all(hm[0][inside] == pytest.approx(-0.8, abs=1e-7))
    assert np.all(hm[0][~inside] == -9.0)
