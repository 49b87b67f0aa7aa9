"""Synthetic static terrain meshes shaped like the paper's terrain families.

The paper trains on slopes, stairs and stepping stones (Sec. 3.1.1) and its
real course has a 20 degree slope, stairs with 20 cm rise and 22/25/30 cm
treads and 25 cm stones with 60 cm gaps (Sec. 4.1).  No terrain files ship with
the paper, so these generators build seeded stand-ins.

Every mesh is conforming: a vertex shared by several triangles is one entry
of a per-tile vertex table (so its FP32 coordinates are bit-identical in every
triangle that uses it), there are no T-junctions, and tiles meet along borders
at z = 0 whose vertices are computed by the same expression on both sides.

Output is a triangle soup, float32 [T][3][3] (x, y, z per vertex), in world
metres, z up.
"""
import math
import numpy as np

from .rng import substream

TILE = 8.0            # tile edge length (m)
HALF = TILE / 2.0
BORDER_SEG = 50       # segments per tile side along the shared z = 0 border


def side_coord(a, m, j):
    """Canonical coordinate of point j (0..m) along a side of half-length a."""
    return -a + (2.0 * a * j) / m


class VertexTable:
    """Per-tile vertex table keyed by a logical key so shared vertices are unique."""

    def __init__(self):
        self.index = {}
        self.pts = []

    def get(self, key, xyz):
        i = self.index.get(key)
        if i is None:
            i = len(self.pts)
            self.index[key] = i
            self.pts.append(xyz)
        return i

    def array(self):
        return np.asarray(self.pts, dtype=np.float64).reshape(-1, 3)


def zipper(outer, inner, s_outer, s_inner):
    """Triangulate the strip between two polylines given their params in [0,1]."""
    tris = []
    i = j = 0
    no, ni = len(outer) - 1, len(inner) - 1
    while i < no or j < ni:
        adv_outer = j >= ni or (i < no and s_outer[i + 1] <= s_inner[j + 1])
        if adv_outer:
            tris.append((outer[i], inner[j], outer[i + 1]))
            i += 1
        else:
            tris.append((outer[i], inner[j], inner[j + 1]))
            j += 1
    return tris


def square_loop(vt, tag, a, m, z, coords=None):
    """Vertex ids of the closed square loop of half-size a at height z.

    Returns a list of 4 sides; each side is the list of m+1 vertex ids from
    one corner to the next, counter-clockwise seen from +z, starting at the
    corner (-a, -a).  ``coords`` optionally gives the breakpoints (length m+1,
    increasing from -a to a) used instead of a uniform subdivision.
    """
    if coords is None:
        coords = [side_coord(a, m, j) for j in range(m + 1)]
    sides = []
    # bottom: y = -a, x increasing; right: x = +a, y increasing;
    # top: y = +a, x decreasing; left: x = -a, y decreasing.
    spec = [
        (lambda c: (c, -a), range(m + 1)),
        (lambda c: (a, c), range(m + 1)),
        (lambda c: (c, a), range(m, -1, -1)),
        (lambda c: (-a, c), range(m, -1, -1)),
    ]
    for xy, order in spec:
        ids = []
        for j in order:
            x, y = xy(coords[j])
            ids.append(vt.get((tag, round(x, 9), round(y, 9)), (x, y, z)))
        sides.append(ids)
    return sides


def _side_params(n):
    return [k / n for k in range(n + 1)]


def ring_between(outer_sides, inner_sides):
    tris = []
    for so, si in zip(outer_sides, inner_sides):
        tris += zipper(so, si, _side_params(len(so) - 1), _side_params(len(si) - 1))
    return tris


def wall_between(lower_sides, upper_sides):
    """Quads between two loops with identical xy (a riser or a vertical wall)."""
    tris = []
    for lo, up in zip(lower_sides, upper_sides):
        for k in range(len(lo) - 1):
            tris.append((lo[k], lo[k + 1], up[k + 1]))
            tris.append((lo[k], up[k + 1], up[k]))
    return tris


# ----------------------------------------------------------------------------
# tile families
# ----------------------------------------------------------------------------

class SlopeTile:
    """Pyramid slope rising from the z = 0 border to a central platform."""

    kind = "slope"

    def __init__(self, theta_deg, plat_cells=6):
        self.theta = math.radians(theta_deg)
        self.n = BORDER_SEG
        self.p = plat_cells * TILE / self.n

    def height(self, lx, ly):
        d = max(abs(lx), abs(ly))
        return math.tan(self.theta) * (HALF - max(d, self.p))

    def mesh(self):
        n = self.n
        c = np.array([side_coord(HALF, n, j) for j in range(n + 1)])
        X, Y = np.meshgrid(c, c, indexing="ij")
        D = np.maximum(np.abs(X), np.abs(Y))
        Z = math.tan(self.theta) * (HALF - np.maximum(D, self.p))
        V = np.stack([X, Y, Z], -1).reshape(-1, 3)
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        i, j = i.ravel(), j.ravel()
        v00 = i * (n + 1) + j
        v10 = (i + 1) * (n + 1) + j
        v01 = i * (n + 1) + j + 1
        v11 = (i + 1) * (n + 1) + j + 1
        cx = 0.5 * (c[i] + c[i + 1])
        cy = 0.5 * (c[j] + c[j + 1])
        main = (cx * cy) > 0  # split along the crease direction of the pyramid
        t_main = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
        t_anti = np.concatenate([np.stack([v00, v10, v01], 1), np.stack([v10, v11, v01], 1)])
        mm = np.concatenate([main, main])
        T = np.where(mm[:, None], t_main, t_anti)
        return V, T


class StairsTile:
    """Pyramid of square stair rings (up or down) around a central platform."""

    kind = "stairs"

    def __init__(self, tread, riser, up=True, seg=0.2, min_plat=1.0):
        self.tread, self.riser, self.sgn = tread, riser, (1.0 if up else -1.0)
        self.n_s = int((HALF - min_plat) // tread)
        self.a = [HALF - k * tread for k in range(self.n_s + 1)]
        self.seg = seg

    def height(self, lx, ly):
        d = max(abs(lx), abs(ly))
        k = min(self.n_s, max(0, int((HALF - d) // self.tread)))
        return self.sgn * k * self.riser

    def mesh(self):
        vt = VertexTable()
        tris = []
        h = [self.sgn * k * self.riser for k in range(self.n_s + 1)]
        m = [BORDER_SEG] + [max(1, int(round(2 * a / self.seg))) for a in self.a[1:]]
        outer = square_loop(vt, ("b", 0, 0), self.a[0], m[0], 0.0)
        for k in range(self.n_s):
            inner_lo = square_loop(vt, ("b", k + 1, 0), self.a[k + 1], m[k + 1], h[k])
            tris += ring_between(outer, inner_lo)
            inner_hi = square_loop(vt, ("b", k + 1, 1), self.a[k + 1], m[k + 1], h[k + 1])
            tris += wall_between(inner_lo, inner_hi)
            outer = inner_hi
        centre = vt.get(("centre",), (0.0, 0.0, h[self.n_s]))
        for side in outer:
            for q in range(len(side) - 1):
                tris.append((side[q], side[q + 1], centre))
        return vt.array(), np.asarray(tris, dtype=np.int64)


class StonesTile:
    """Square stepping stones standing in a pit, with a z = 0 rim."""

    kind = "stones"

    def __init__(self, tops, pit_half=3.7, stone=0.25, gap=0.6, n_stones=8,
                 depth=0.5, gap_pieces=2, stone_pieces=2, wall_pieces=2):
        self.tops = np.asarray(tops, dtype=np.float64).reshape(n_stones, n_stones)
        self.ph, self.stone, self.gap, self.ns, self.depth = pit_half, stone, gap, n_stones, depth
        lines = [-pit_half]
        self.stone_lo = []
        x = -pit_half
        for k in range(n_stones + 1):
            for q in range(1, gap_pieces + 1):
                lines.append(x + gap * q / gap_pieces)
            x = x + gap
            if k == n_stones:
                break
            self.stone_lo.append(x)
            for q in range(1, stone_pieces + 1):
                lines.append(x + stone * q / stone_pieces)
            x = x + stone
        lines[-1] = pit_half
        self.lines = lines
        self.sp, self.wp = stone_pieces, wall_pieces

    def _stone_at(self, c):
        for k, lo in enumerate(self.stone_lo):
            if lo <= c <= lo + self.stone:
                return k
        return -1

    def height(self, lx, ly):
        if max(abs(lx), abs(ly)) > self.ph:
            return 0.0
        i, j = self._stone_at(lx), self._stone_at(ly)
        if i >= 0 and j >= 0:
            return float(self.tops[i, j])
        return -self.depth

    def mesh(self):
        vt = VertexTable()
        tris = []
        L = self.lines
        nl = len(L) - 1
        fz = -self.depth
        # floor grid at the pit bottom; cells under a stone are left out
        fid = {}
        for i in range(nl + 1):
            for j in range(nl + 1):
                fid[i, j] = vt.get(("g", i, j, "floor"), (L[i], L[j], fz))
        under = np.zeros((nl, nl), dtype=bool)
        stone_cells = []
        for si, lo in enumerate(self.stone_lo):
            ci = L.index(lo)
            stone_cells.append(ci)
        for si, ci in enumerate(stone_cells):
            for sj, cj in enumerate(stone_cells):
                under[ci:ci + self.sp, cj:cj + self.sp] = True
        for i in range(nl):
            for j in range(nl):
                if under[i, j]:
                    continue
                a, b, c, d = fid[i, j], fid[i + 1, j], fid[i + 1, j + 1], fid[i, j + 1]
                tris += [(a, b, c), (a, c, d)]
        # stones: vertical walls (floor -> top) and the top face
        wp = self.wp
        for si, ci in enumerate(stone_cells):
            for sj, cj in enumerate(stone_cells):
                zt = float(self.tops[si, sj])
                zl = [fz + (zt - fz) * q / wp for q in range(wp + 1)]
                # perimeter of the footprint as grid indices, counter-clockwise
                per = [(ci + q, cj) for q in range(self.sp)] + \
                      [(ci + self.sp, cj + q) for q in range(self.sp)] + \
                      [(ci + self.sp - q, cj + self.sp) for q in range(self.sp)] + \
                      [(ci, cj + self.sp - q) for q in range(self.sp)]
                per.append(per[0])

                def sv(gi, gj, lev):
                    if lev == 0:
                        return fid[gi, gj]
                    return vt.get(("s", si, sj, gi, gj, lev), (L[gi], L[gj], zl[lev]))
                for k in range(len(per) - 1):
                    (i0, j0), (i1, j1) = per[k], per[k + 1]
                    for lev in range(wp):
                        a, b = sv(i0, j0, lev), sv(i1, j1, lev)
                        c, d = sv(i1, j1, lev + 1), sv(i0, j0, lev + 1)
                        tris += [(a, b, c), (a, c, d)]
                for gi in range(ci, ci + self.sp):
                    for gj in range(cj, cj + self.sp):
                        a, b = sv(gi, gj, wp), sv(gi + 1, gj, wp)
                        c, d = sv(gi + 1, gj + 1, wp), sv(gi, gj + 1, wp)
                        tris += [(a, b, c), (a, c, d)]
        # pit walls from the rim (z = 0) down to the floor, along the pit edge
        zl = [fz + (0.0 - fz) * q / wp for q in range(wp + 1)]
        per = [(q, 0) for q in range(nl)] + [(nl, q) for q in range(nl)] + \
              [(nl - q, nl) for q in range(nl)] + [(0, nl - q) for q in range(nl)]
        per.append(per[0])

        def pv(gi, gj, lev):
            if lev == 0:
                return fid[gi, gj]
            return vt.get(("p", gi, gj, lev), (L[gi], L[gj], zl[lev]))
        for k in range(len(per) - 1):
            (i0, j0), (i1, j1) = per[k], per[k + 1]
            for lev in range(wp):
                a, b = pv(i0, j0, lev), pv(i1, j1, lev)
                c, d = pv(i1, j1, lev + 1), pv(i0, j0, lev + 1)
                tris += [(a, b, c), (a, c, d)]
        # rim: zipper between the z = 0 tile border and the pit edge at z = 0
        border = square_loop(vt, ("rim",), HALF, BORDER_SEG, 0.0)
        bottom = [pv(q, 0, wp) for q in range(nl + 1)]
        right = [pv(nl, q, wp) for q in range(nl + 1)]
        top = [pv(q, nl, wp) for q in range(nl, -1, -1)]
        left = [pv(0, q, wp) for q in range(nl, -1, -1)]
        s_inc = [(c + self.ph) / (2 * self.ph) for c in L]
        s_dec = s_inc[::-1]
        s_dec = [1.0 - s for s in s_dec]
        sb = _side_params(BORDER_SEG)
        for so, si, ss in zip(border, [bottom, right, top, left], [s_inc, s_inc, s_dec, s_dec]):
            tris += zipper(so, si, sb, ss)
        return vt.array(), np.asarray(tris, dtype=np.int64)


# ----------------------------------------------------------------------------
# terrains
# ----------------------------------------------------------------------------

class TileTerrain:
    """A seeded n x n grid of tiles centred on the world origin."""

    def __init__(self, n, seed_label="terrain", seed=None):
        from .rng import MASTER_SEED
        rng = substream(f"{seed_label}/{n}", MASTER_SEED if seed is None else seed)
        self.n = n
        self.tiles = []
        for _ in range(n * n):
            kind = int(rng.integers(0, 3))
            if kind == 0:
                t = SlopeTile(theta_deg=float(rng.uniform(0.0, 20.0)))
            elif kind == 1:
                t = StairsTile(tread=float(rng.choice([0.22, 0.25, 0.30])),
                               riser=float(rng.uniform(0.05, 0.20)),
                               up=bool(rng.integers(0, 2)))
            else:
                t = StonesTile(tops=rng.uniform(-0.05, 0.05, size=64))
            self.tiles.append(t)

    def centre(self, i, j):
        return (-self.n * HALF + TILE * i + HALF, -self.n * HALF + TILE * j + HALF)

    def tile_index(self, x, y):
        i = min(self.n - 1, max(0, int(math.floor((x + self.n * HALF) / TILE))))
        j = min(self.n - 1, max(0, int(math.floor((y + self.n * HALF) / TILE))))
        return i, j

    def tile_at(self, x, y):
        i, j = self.tile_index(x, y)
        return self.tiles[i * self.n + j]

    def height(self, x, y):
        i, j = self.tile_index(x, y)
        cx, cy = self.centre(i, j)
        return self.tiles[i * self.n + j].height(x - cx, y - cy)

    def triangles(self):
        out = []
        cache = {}
        for i in range(self.n):
            for j in range(self.n):
                t = self.tiles[i * self.n + j]
                key = id(t)
                if key not in cache:
                    cache[key] = t.mesh()
                V, T = cache[key]
                cx, cy = self.centre(i, j)
                G = V.copy()
                G[:, 0] += cx
                G[:, 1] += cy
                out.append(G[T].astype(np.float32))
        return np.concatenate(out, 0)


class ProfileTerrain:
    """Plane, 20 degree slope and a 3-step staircase, extruded along y.

    Profile in the x-z plane (m): ground z = 0 on [-2, 0.8]; a 20 degree ramp
    over [0.8, 1.3]; a landing to x = 1.6; three 0.15 m risers at x = 1.60,
    1.85 and 2.10 with 0.25 m treads; a top landing to x = 6.  y spans [-4, 4].
    """

    def __init__(self, piece=0.25, y_half=4.0):
        h1 = 0.5 * math.tan(math.radians(20.0))
        r = 0.15
        self.profile = [(-2.0, 0.0), (0.8, 0.0), (1.3, h1), (1.6, h1),
                        (1.6, h1 + r), (1.85, h1 + r), (1.85, h1 + 2 * r),
                        (2.1, h1 + 2 * r), (2.1, h1 + 3 * r), (6.0, h1 + 3 * r)]
        self.piece, self.y_half = piece, y_half

    def pieces(self):
        """Planar rectangles of the analytic surface: (xa, za, xb, zb, y_half)."""
        P = self.profile
        return [(P[k][0], P[k][1], P[k + 1][0], P[k + 1][1], self.y_half) for k in range(len(P) - 1)]

    def triangles(self):
        pts = []
        P = self.profile
        for k in range(len(P) - 1):
            (xa, za), (xb, zb) = P[k], P[k + 1]
            ln = math.hypot(xb - xa, zb - za)
            m = max(1, int(math.ceil(ln / self.piece - 1e-9)))
            start = 0 if k == 0 else 1
            for q in range(start, m + 1):
                s = q / m
                pts.append((xa + (xb - xa) * s, za + (zb - za) * s))
        ny = int(round(2 * self.y_half / self.piece))
        ys = [side_coord(self.y_half, ny, j) for j in range(ny + 1)]
        V = np.array([[x, y, z] for (x, z) in pts for y in ys], dtype=np.float64)
        tris = []
        for a in range(len(pts) - 1):
            for b in range(ny):
                v00 = a * (ny + 1) + b
                v10 = (a + 1) * (ny + 1) + b
                v01 = v00 + 1
                v11 = v10 + 1
                tris += [(v00, v10, v11), (v00, v11, v01)]
        T = np.asarray(tris, dtype=np.int64)
        return V[T].astype(np.float32)


def flat_height(x, y):
    return 0.0
