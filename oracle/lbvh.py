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
