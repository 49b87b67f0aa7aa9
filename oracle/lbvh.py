"""CPU model of the linear BVH the renderer builds (TEST INFRASTRUCTURE ONLY).

Only tests may use it.  It restates, in plain numpy and Python loops, the
published construction the renderer follows so its output can be compared
bit for bit: Morton codes of quantised box centres (Lauterbach et al. 2009),
a stable sort of (code, index), the Karras (2012) hierarchy with duplicate
codes broken by leaf index, boxes as unions of children, then an outward
padding of every child box.  All floating-point steps are single FP32
operations in the stated order, so the results are exact replicas.

A triangle of zero area (edge vectors with an all-zero FP64 cross product)
is met by no ray: it keeps its Morton code, but its leaf box is empty for
the unions, and an empty child box is stored as the far point.
"""
import math

import numpy as np

PAD_REL = np.float32(2.0 ** -20)
PAD_ABS = np.float32(1e-5)
FAR_POINT = np.float32(1e30)


def _spread3(v):
    x = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    x = (x | (x << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    x = (x | (x << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    x = (x | (x << np.uint64(2))) & np.uint64(0x1249249249249249)
    return x


def interleave_bits(q):
    """Reference bit interleave by loops: bit k of axis a -> bit 3k + (2 - a)."""
    out = 0
    for k in range(21):
        for a in range(3):
            out |= ((int(q[a]) >> k) & 1) << (3 * k + (2 - a))
    return out


def prim_boxes(tri):
    t = np.ascontiguousarray(tri, np.float32).reshape(-1, 3, 3)
    return t.min(axis=1), t.max(axis=1)


def morton_keys(lo, hi):
    """Box centres quantised to 21 bits with one scale for all axes
    (2^21 / largest centroid extent), then bit-interleaved."""
    c = (lo + hi) * np.float32(0.5)
    cmin, cmax = c.min(axis=0), c.max(axis=0)
    ext = np.float32((cmax - cmin).max())
    s = np.float32(2097152.0) / ext if ext > 0 else np.float32(0)
    f = (c - cmin) * np.float32(s)
    f = np.minimum(np.maximum(f, np.float32(0)), np.float32(2097151.0))
    q = f.astype(np.uint32)
    return (_spread3(q[:, 0]) << np.uint64(2)) | (_spread3(q[:, 1]) << np.uint64(1)) | _spread3(q[:, 2])


def _clz64(x):
    return 64 - int(x).bit_length()


def _clz32(x):
    return 32 - int(x).bit_length()


def karras(keys):
    """Children (ref: >= 0 internal, < 0 leaf ~i), parent and sibling per internal node."""
    n = len(keys)
    k = [int(x) for x in keys]

    def delta(i, j):
        if j < 0 or j >= n:
            return -1
        if k[i] != k[j]:
            return _clz64(k[i] ^ k[j])
        return 64 + _clz32(i ^ j)

    m = n - 1
    c0 = np.zeros(m, np.int32)
    c1 = np.zeros(m, np.int32)
    parent = np.full(m, -1, np.int32)
    sibling = np.full(m, -1, np.int32)
    for i in range(m):
        d = 1 if delta(i, i + 1) - delta(i, i - 1) > 0 else -1
        dmin = delta(i, i - d)
        lmax = 2
        while delta(i, i + lmax * d) > dmin:
            lmax *= 2
        l = 0
        t = lmax // 2
        while t >= 1:
            if delta(i, i + (l + t) * d) > dmin:
                l += t
            t //= 2
        j = i + l * d
        dnode = delta(i, j)
        s = 0
        div = 2
        while True:
            t = (l + div - 1) // div
            if delta(i, i + (s + t) * d) > dnode:
                s += t
            if t <= 1:
                break
            div *= 2
        g = i + s * d + (-1 if d < 0 else 0)
        lo, hi = min(i, j), max(i, j)
        a = ~g if lo == g else g
        b = ~(g + 1) if hi == g + 1 else g + 1
        c0[i], c1[i] = a, b
        if a >= 0:
            parent[a], sibling[a] = i, b
        if b >= 0:
            parent[b], sibling[b] = i, a
    return c0, c1, parent, sibling


def _pad(lo, hi):
    if np.any(lo > hi):  # empty: only zero-area triangles below
        far = np.full(3, FAR_POINT, np.float32)
        return far, far.copy()
    lo = lo - (np.abs(lo) * PAD_REL + PAD_ABS)
    hi = hi + (np.abs(hi) * PAD_REL + PAD_ABS)
    return lo.astype(np.float32), hi.astype(np.float32)


def degenerate(tri):
    """Zero-area triangles: the FP64 cross product of their edges is zero."""
    t = np.asarray(tri, np.float32).reshape(-1, 3, 3).astype(np.float64)
    c = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    return np.all(c == 0.0, axis=1)


def build(tri):
    """Returns dict(keys u64 sorted, tri_id i32, records f32 [m,16] view, and parts)."""
    lo, hi = prim_boxes(tri)
    n = lo.shape[0]
    rec = np.zeros((max(n - 1, 1), 16), np.float32)
    ints = rec.view(np.int32)
    deg = degenerate(tri)
    if n == 1:
        if deg[0]:
            lo, hi = np.full_like(lo, np.inf), np.full_like(hi, -np.inf)
        plo, phi = _pad(lo[0], hi[0])
        rec[0, 0:6:2], rec[0, 1:6:2] = plo, phi
        rec[0, 6:12] = FAR_POINT
        ints[0, 12:16] = [~0, ~0, -1, -1]
        return dict(keys=np.zeros(1, np.uint64), tri_id=np.zeros(1, np.int32), records=rec, depth=0)
    keys = morton_keys(lo, hi)
    lo, hi = lo.copy(), hi.copy()
    lo[deg], hi[deg] = np.float32(np.inf), np.float32(-np.inf)
    order = np.argsort(keys, kind="stable").astype(np.int32)
    skeys = keys[order]
    c0, c1, parent, sibling = karras(skeys)
    slo, shi = lo[order], hi[order]
    m = n - 1
    blo = np.zeros((m, 3), np.float32)
    bhi = np.zeros((m, 3), np.float32)
    done = np.zeros(m, bool)
    stack = [0]
    while stack:  # post-order: a node's box is the union of its children's
        i = stack[-1]
        pending = [c for c in (c0[i], c1[i]) if c >= 0 and not done[c]]
        if pending:
            stack.extend(pending)
            continue
        stack.pop()
        parts = [(blo[c], bhi[c]) if c >= 0 else (slo[~c], shi[~c]) for c in (c0[i], c1[i])]
        blo[i] = np.minimum(parts[0][0], parts[1][0])
        bhi[i] = np.maximum(parts[0][1], parts[1][1])
        done[i] = True
    for i in range(m):
        for h, c in enumerate((c0[i], c1[i])):
            clo, chi = (blo[c], bhi[c]) if c >= 0 else (slo[~c], shi[~c])
            plo, phi = _pad(clo, chi)
            rec[i, 6 * h + 0:6 * h + 6:2] = plo
            rec[i, 6 * h + 1:6 * h + 6:2] = phi
    ints[:, 12], ints[:, 13], ints[:, 14], ints[:, 15] = c0, c1, parent, sibling
    depth = np.zeros(m, np.int64)
    for i in range(1, m):
        p, d = parent[i], 0
        while p >= 0:
            d += 1
            p = parent[p]
        depth[i] = d
    return dict(keys=skeys, tri_id=order, records=rec, depth=int(depth.max()))


# ---------------------------------------------------------------------------
# Per-environment top level over the link instances (rebuilt every step)
# ---------------------------------------------------------------------------

INST_PAD_REL = np.float32(2.0 ** -20)
INST_PAD_ABS = np.float32(1e-4)


def _spread10(v):
    x = int(v) & 0x3FF
    x = (x | (x << 16)) & 0x030000FF
    x = (x | (x << 8)) & 0x0300F00F
    x = (x | (x << 4)) & 0x030C30C3
    x = (x | (x << 2)) & 0x09249249
    return x


def _f(x):
    return np.float32(x)


def instance(pos, quat, root):
    """Transform (R^T row-major, t) and padded world box (lo.x, hi.x, ...) of
    one link instance, or None for a pose that places the link nowhere (a
    non-finite component or a zero quaternion).  The rotation is evaluated in
    FP64 and rounded once to FP32; every other step is one FP32 operation in
    the order written."""
    q64 = [float(np.float32(v)) for v in quat]
    t = [_f(v) for v in pos]
    with np.errstate(over="ignore", invalid="ignore"):
        nn = math.sqrt(((q64[0] * q64[0] + q64[1] * q64[1]) + q64[2] * q64[2]) + q64[3] * q64[3]) \
            if all(math.isfinite(v) for v in q64) else float("nan")
    if not (all(np.isfinite(t)) and nn > 0 and math.isfinite(nn)):
        return None
    qx, qy, qz, qw = (v / nn for v in q64)
    R = [_f(1.0 - 2.0 * (qy * qy + qz * qz)), _f(2.0 * (qx * qy - qz * qw)), _f(2.0 * (qx * qz + qy * qw)),
         _f(2.0 * (qx * qy + qz * qw)), _f(1.0 - 2.0 * (qx * qx + qz * qz)), _f(2.0 * (qy * qz - qx * qw)),
         _f(2.0 * (qx * qz - qy * qw)), _f(2.0 * (qy * qz + qx * qw)), _f(1.0 - 2.0 * (qx * qx + qy * qy))]
    one, two, half = _f(1), _f(2), _f(0.5)
    m = [R[3 * c + r] for r in range(3) for c in range(3)]
    box, cw = [], []
    for a in range(3):
        c, h = _f(0), _f(0)
        for k in range(3):
            lc = (_f(root[2 * k]) + _f(root[2 * k + 1])) * half
            lh = (_f(root[2 * k + 1]) - _f(root[2 * k])) * half
            c = c + R[3 * a + k] * lc
            h = h + abs(R[3 * a + k]) * lh
        w = c + t[a]
        pad = abs(w) * INST_PAD_REL + INST_PAD_ABS
        box += [(w - h) - pad, (w + h) + pad]
        cw.append(w)
    return np.array(m + t, np.float32), np.array(box, np.float32), np.array(cw, np.float32)


def tlas(link_pos, link_quat, root):
    """Top level of one environment: link_pos [B, 3], link_quat [B, 4] (x, y,
    z, w), root [B, 6] padded local root boxes of the link meshes.  Returns
    (xf [B, 12] f32: R^T row-major then t; records [max(B - 1, 1), 16] f32
    with the int32 refs in the last four words).  Instance boxes come from the
    local box's centre and half extents under the pose, padded outward; keys
    are 30-bit Morton codes of the box centres quantised per axis over the
    environment's centre bounds, ranked by (key, instance); the hierarchy is
    Karras's over the ranked keys, a node's box the union of its leaf range.
    An absent instance (see instance()) gets the identity rotation, t at the
    far point, a box that is the far point, and the largest key."""
    B = len(link_pos)
    xf = np.zeros((B, 12), np.float32)
    box = np.zeros((B, 6), np.float32)
    cw = np.zeros((B, 3), np.float32)
    ok = np.zeros(B, bool)
    for b in range(B):
        r = instance(link_pos[b], link_quat[b], root[b])
        if r is None:
            xf[b] = [1, 0, 0, 0, 1, 0, 0, 0, 1, FAR_POINT, FAR_POINT, FAR_POINT]
            box[b] = FAR_POINT
        else:
            xf[b], box[b], cw[b] = r
            ok[b] = True
    m = max(B - 1, 1)
    rec = np.zeros((m, 16), np.float32)
    ints = rec.view(np.int32)
    if B == 1:
        rec[0, 0:6] = box[0]
        rec[0, 6:12] = FAR_POINT
        ints[0, 12:16] = [~0, ~0, -1, -1]
        return xf, rec
    keys = np.full(B, 0xFFFFFFFF, np.uint64)
    if ok.any():
        cmin, cmax = cw[ok].min(0), cw[ok].max(0)
        for b in np.nonzero(ok)[0]:
            q = []
            for a in range(3):
                ext = cmax[a] - cmin[a]
                s = _f(1024) / ext if ext > 0 else _f(0)
                f = min(max((cw[b, a] - cmin[a]) * s, _f(0)), _f(1023))
                q.append(int(f))
            keys[b] = (_spread10(q[0]) << 2) | (_spread10(q[1]) << 1) | _spread10(q[2])
    order = np.lexsort((np.arange(B), keys))
    # 30-bit keys in 64-bit words: every prefix length shifts by the same 32,
    # so the hierarchy is the one over the 32-bit words
    c0, c1, parent, sibling = karras(keys[order])
    sbox = box[order]
    for i in range(B - 1):
        for h, c in enumerate((c0[i], c1[i])):
            if c < 0:
                rec[i, 6 * h:6 * h + 6] = sbox[~c]
            else:
                lo, hi = _leaf_range(c0, c1, c)
                u = sbox[lo:hi + 1]
                rec[i, 6 * h:6 * h + 6] = [u[:, 0].min(), u[:, 1].max(), u[:, 2].min(),
                                           u[:, 3].max(), u[:, 4].min(), u[:, 5].max()]
        ints[i, 12] = ~order[~c0[i]] if c0[i] < 0 else c0[i]
        ints[i, 13] = ~order[~c1[i]] if c1[i] < 0 else c1[i]
    ints[:, 14] = parent
    # a leaf sibling is stored by its instance; the root has none (-1)
    ints[:, 15] = [-1 if i == 0 else (~order[~c] if c < 0 else c) for i, c in enumerate(sibling)]
    return xf, rec


def collapse4(records):
    """4-wide records [m, 32] f32 of binary records [m, 16]: for node n, its two
    children in order, each internal child (one whose box is not the far point)
    replaced by that child's two children; unused slots get the far-point box
    and child word 0.  Columns: lo.x[4], hi.x[4], lo.y[4], hi.y[4], lo.z[4],
    hi.z[4], int32 child[4], four zero words."""
    m = len(records)
    ints = records.view(np.int32)
    out = np.zeros((m, 32), np.float32)
    oi = out.view(np.int32)
    for n in range(m):
        slots = []
        for h in range(2):
            c = int(ints[n, 12 + h])
            bx = records[n, 6 * h:6 * h + 6]
            if c < 0 or c >= m or bx[0] == FAR_POINT:
                slots.append((bx, c))
            else:
                slots.append((records[c, 0:6], int(ints[c, 12])))
                slots.append((records[c, 6:12], int(ints[c, 13])))
        while len(slots) < 4:
            slots.append((np.full(6, FAR_POINT, np.float32), 0))
        for k, (bx, c) in enumerate(slots):
            out[n, k:24:4] = bx
            oi[n, 24 + k] = c
    return out


def _leaf_range(c0, c1, i):
    """First and last sorted leaf below internal node i."""
    lo, hi = i, i
    while lo >= 0:
        lo = c0[lo]
    while hi >= 0:
        hi = c1[hi]
    return ~lo, ~hi
