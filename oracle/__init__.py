"""Oracle for the multi-camera depth path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package.  It is a plain FP64 brute-force reference written from the
paper (Sec. 3.2.2, Algorithm 1; sensor model in Sec. 1, Sec. 4.1 and Table
6) and shares no code with the GPU renderer.  The C part is built by
``oracle/build.py`` (gcc, OpenMP) into ``oracle/liboracle.so``.
"""
import ctypes
import math
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FLAG_EDGE, FLAG_FAR, FLAG_TIE = 1, 2, 4
POST_NOISE, POST_DROPOUT, POST_LATENCY = 1, 2, 4


class PostParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64),
                ("sigma_abs", ctypes.c_float), ("sigma_rel", ctypes.c_float),
                ("p_drop", ctypes.c_float), ("near", ctypes.c_float),
                ("far", ctypes.c_float), ("fill", ctypes.c_float),
                ("lat_min", ctypes.c_int32), ("lat_max", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build
            build.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.oracle_render.restype = ctypes.c_int
        _lib.oracle_post.restype = ctypes.c_int
        _lib.oracle_latency.restype = ctypes.c_int
    return _lib


def set_threads(n):
    """Host threads the oracle's parallel loops use (for timing it)."""
    lib().oracle_set_threads(int(n))


def get_threads():
    return int(lib().oracle_get_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def render(terrain, link_tri, link_off, link_pos, link_quat, cam_pos, cam_quat, intr,
           W, H, far, depth_mode=0, rays=None, K=8, cam64=None):
    """Brute-force FP64 render.

    terrain [T,3,3]; link_tri [LT,3,3] with link_off [B+1]; link_pos [E,B,3];
    link_quat [E,B,4]; cam_pos [E,C,3]; cam_quat [E,C,4]; intr [E,C,4].
    cam64: optional FP64 cameras [E,C,16] (R row-major, p, fx, fy, cx, cy)
    replacing cam_pos / cam_quat / intr (see cam_randomize).
    rays: optional int64 linear pixel ids into [E,C,H,W].
    Returns dict(depth f64, inst i32, tri i32, flags i32, cand i32 [n,K,2],
    cand_depth f64 [n,K]); flat over ``rays`` (or all pixels).
    """
    terrain = _f32(terrain).reshape(-1, 9)
    link_tri = _f32(link_tri).reshape(-1, 9)
    link_off = np.ascontiguousarray(link_off, dtype=np.int64)
    B = int(link_off.shape[0] - 1)
    cam_pos = _f32(cam_pos)
    E, C = cam_pos.shape[0], cam_pos.shape[1]
    link_pos = _f32(link_pos).reshape(E, B, 3)
    link_quat = _f32(link_quat).reshape(E, B, 4)
    cam_quat = _f32(cam_quat).reshape(E, C, 4)
    intr = _f32(intr).reshape(E, C, 4)
    if rays is not None:
        rays = np.ascontiguousarray(rays, dtype=np.int64)
        n = rays.shape[0]
    else:
        n = E * C * H * W
    depth = np.empty(n, np.float64)
    inst = np.empty(n, np.int32)
    tri = np.empty(n, np.int32)
    flags = np.empty(n, np.int32)
    cand = np.empty((n, K, 2), np.int32)
    cand_d = np.empty((n, K), np.float64)
    c64 = None if cam64 is None else np.ascontiguousarray(cam64, dtype=np.float64).reshape(E, C, 16)
    rc = lib().oracle_render(
        _p(terrain), ctypes.c_int64(terrain.shape[0]), _p(link_tri), _p(link_off), ctypes.c_int(B),
        _p(link_pos), _p(link_quat), _p(cam_pos), _p(cam_quat), _p(intr),
        ctypes.c_int(E), ctypes.c_int(C), ctypes.c_int(W), ctypes.c_int(H),
        ctypes.c_double(far), ctypes.c_int(depth_mode),
        _p(rays), ctypes.c_int64(n),
        _p(depth), _p(inst), _p(tri), _p(flags), _p(cand), _p(cand_d), ctypes.c_int(K), _p(c64))
    if rc != 0:
        raise ValueError("oracle_render: bad arguments")
    return dict(depth=depth, inst=inst, tri=tri, flags=flags, cand=cand, cand_depth=cand_d)


def philox(ctr, key):
    """Philox4x32-10 of one 4-word counter and 2-word key -> 4 uint32 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def make_params(seed=0, sigma_abs=0.0, sigma_rel=0.0, p_drop=0.0, near=0.05, far=3.0,
                fill=0.0, lat_min=0, lat_max=0, flags=None):
    if flags is None:
        flags = (POST_NOISE if (sigma_abs or sigma_rel) else 0) | \
                (POST_DROPOUT if p_drop else 0) | (POST_LATENCY if lat_max else 0)
    return PostParams(seed, sigma_abs, sigma_rel, p_drop, near, far, fill, lat_min, lat_max, flags)


def latency(params, cam_uid, step):
    return lib().oracle_latency(ctypes.byref(params), ctypes.c_uint32(cam_uid), ctypes.c_uint64(step))


def post(depth, inst, params, s0=0, cam_uid=None):
    """Sensor model over frames depth/inst [S,E,C,H,W] starting at step s0.

    Returns (out f64 [S,E,C,H,W], drop u8 [S,E,C,H,W], lat u8 [S,E,C]).
    """
    depth = _f32(depth)
    inst = np.ascontiguousarray(inst, dtype=np.int32)
    S, E, C, H, W = depth.shape
    out = np.empty(depth.shape, np.float64)
    drop = np.empty(depth.shape, np.uint8)
    lat = np.empty((S, E, C), np.uint8)
    uid = None if cam_uid is None else np.ascontiguousarray(cam_uid, dtype=np.uint32)
    rc = lib().oracle_post(_p(depth), _p(inst), ctypes.c_int(E), ctypes.c_int(C), ctypes.c_int(H),
                           ctypes.c_int(W), ctypes.c_int(S), ctypes.c_uint64(s0), _p(uid),
                           ctypes.byref(params), _p(out), _p(drop), _p(lat))
    if rc != 0:
        raise ValueError("oracle_post: bad arguments")
    return out, drop, lat


def downsample(depth, inst, factor, far):
    """Block pooling of frames [..., H, W] into [..., H // f, W // f]: the mean
    depth (FP64) of the block's hit pixels (inst >= 0), or far when none hit.
    The paper downsamples its 240x135 depth to 48x27 (Sec. 4.1) without naming
    the pooling rule; this is the reading used."""
    depth = np.asarray(depth, dtype=np.float64)
    inst = np.asarray(inst)
    f = int(factor)
    H, W = depth.shape[-2], depth.shape[-1]
    Ho, Wo = H // f, W // f
    lead = depth.shape[:-2]
    d = depth[..., :Ho * f, :Wo * f].reshape(lead + (Ho, f, Wo, f))
    hit = (inst[..., :Ho * f, :Wo * f] >= 0).reshape(lead + (Ho, f, Wo, f))
    s = np.where(hit, d, 0.0).sum(axis=(-3, -1))
    n = hit.sum(axis=(-3, -1))
    return np.where(n > 0, s / np.maximum(n, 1), float(far))


def cam_randomize(cam_pos, cam_quat, intr, cam_uid, seed, epoch, trans_m, euler_deg, dfov_deg):
    """Per-camera perception randomisation (the paper's Table 6: depth camera
    translation, rotation as Euler angles and field of view, each uniform in a
    symmetric range) as FP64 cameras [N,16] (R row-major, p, fx, fy, cx, cy).

    Draws: Philox4x32-10 with key = seed and counter (uid, 0xFFFFFFFE,
    epoch_lo32, (epoch_hi16 << 16) | stream), stream 2 -> (tx, ty, tz, phi),
    stream 3 -> (theta, psi, dfov, -); u = (w >> 8) 2^-24, offset = a (2u - 1).
    The translation is taken in the camera's own (unperturbed) frame, the
    rotation is R0 Rx(phi) Ry(theta) Rz(psi) (about the camera's x, y, z),
    and the field of view widens both axes: f' = c / tan(atan(c / f) + dfov / 2)
    (no change when the FOV range is 0)."""
    pos = np.asarray(cam_pos, np.float64).reshape(-1, 3)
    quat = np.asarray(cam_quat, np.float64).reshape(-1, 4)
    K = np.asarray(intr, np.float64).reshape(-1, 4)
    uid = np.asarray(cam_uid, np.uint64).reshape(-1)
    out = np.zeros((pos.shape[0], 16))
    e_lo = int(epoch) & 0xFFFFFFFF
    e_hi = (int(epoch) >> 32) & 0xFFFF
    key = np.array([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF], np.uint32)

    def offsets(w, a):
        u = (np.asarray(w, np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
        return np.asarray(a, np.float64) * (2.0 * u - 1.0)

    for i in range(pos.shape[0]):
        w2 = philox(np.array([uid[i], 0xFFFFFFFE, e_lo, (e_hi << 16) | 2], np.uint32), key)
        w3 = philox(np.array([uid[i], 0xFFFFFFFE, e_lo, (e_hi << 16) | 3], np.uint32), key)
        t = offsets(w2[:3], trans_m)
        ang = np.radians(offsets([w2[3], w3[0], w3[1]], euler_deg))
        dfov = math.radians(float(offsets([w3[2]], [dfov_deg])[0]))
        x, y, z, w = quat[i] / np.linalg.norm(quat[i])
        R0 = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                       [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                       [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
        c, s_ = np.cos(ang), np.sin(ang)
        Rx = np.array([[1, 0, 0], [0, c[0], -s_[0]], [0, s_[0], c[0]]])
        Ry = np.array([[c[1], 0, s_[1]], [0, 1, 0], [-s_[1], 0, c[1]]])
        Rz = np.array([[c[2], -s_[2], 0], [s_[2], c[2], 0], [0, 0, 1]])
        R = R0 @ Rx @ Ry @ Rz
        fx, fy, cx, cy = K[i]
        if float(dfov_deg) != 0.0:
            fx = cx / math.tan(math.atan(cx / fx) + dfov / 2)
            fy = cy / math.tan(math.atan(cy / fy) + dfov / 2)
        out[i, :9] = R.ravel()
        out[i, 9:12] = pos[i] + R0 @ t
        out[i, 12:] = (fx, fy, cx, cy)
    return out


def side_mask(out, drop, seed, near, far, s0, mask_frac, mask_p, mask_epoch=0, mask_type=None,
              cam_uid=None):
    """Random side masking (the paper's RSM, Sec. 3.2) applied to the sensor
    model's outputs out / drop [S,E,C,H,W] of steps s0.. (modified in place).

    Per env e and mask epoch: u = (w0 >> 8) 2^-24 of Philox with counter
    (e, 0xFFFFFFFD, epoch_lo32, (epoch_hi16 << 16) | 4); mode none if
    u < p0, small if u < p0 + p1, else large (decided in FP32, with the FP32
    sum p0 + p1); m = floor(frac * W + 0.5) in FP32.  Columns x < m and
    x >= W - m of every camera of the env show near + (far - near) u3, u3 from
    word 3 of the pixel's draw (pix, uid, s_lo32, s_hi16 << 16) at step s, and
    their dropout mask is 0."""
    S, E, C, H, W = out.shape
    key = np.array([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF], np.uint32)
    e_lo, e_hi = int(mask_epoch) & 0xFFFFFFFF, (int(mask_epoch) >> 32) & 0xFFFF
    f24 = np.float32(2.0 ** -24)
    modes = np.zeros(E, np.int32)
    for e in range(E):
        typ = min(int(mask_type[e]), 3) if mask_type is not None else 0
        w0 = philox(np.array([e, 0xFFFFFFFD, e_lo, (e_hi << 16) | 4], np.uint32), key)[0]
        u = np.float32(int(w0) >> 8) * f24
        p0, p1 = np.float32(mask_p[typ][0]), np.float32(mask_p[typ][1])
        if u < p0:
            continue
        mode = 1 if u < np.float32(p0 + p1) else 2
        modes[e] = mode
        m = int(np.floor(np.float32(np.float32(mask_frac[mode - 1]) * np.float32(W)) + np.float32(0.5)))
        cols = [x for x in range(W) if x < m or x >= W - m]
        for i in range(S):
            s = int(s0) + i
            for c in range(C):
                uid = int(cam_uid[e * C + c]) if cam_uid is not None else e * C + c
                for y in range(H):
                    for x in cols:
                        w = philox(np.array([y * W + x, uid, s & 0xFFFFFFFF,
                                             ((s >> 32) & 0xFFFF) << 16], np.uint32), key)
                        u3 = float(int(w[3]) >> 8) * 2.0 ** -24
                        out[i, e, c, y, x] = near + (far - near) * u3
                        drop[i, e, c, y, x] = 0
    return modes


def heightmap(terrain, base_pos, base_yaw, nx=17, ny=11, dx=0.1, dy=0.1, top=1.0, depth=3.0,
              miss=float("nan")):
    """Brute-force FP64 privileged height map [E, ny, nx] (terrain z minus base
    z under each grid point; see oracle_heightmap in oracle.c)."""
    terrain = _f32(terrain).reshape(-1, 9)
    base_pos = _f32(base_pos).reshape(-1, 3)
    base_yaw = _f32(base_yaw).reshape(-1)
    # the grid parameters are FP32 numbers, as every input of the method is
    dx, dy, top, depth = (float(np.float32(v)) for v in (dx, dy, top, depth))
    E = base_pos.shape[0]
    out = np.empty((E, ny, nx), np.float64)
    lib().oracle_heightmap(_p(terrain), ctypes.c_int64(terrain.shape[0]), _p(base_pos), _p(base_yaw),
                           ctypes.c_int(E), ctypes.c_int(nx), ctypes.c_int(ny), ctypes.c_double(dx),
                           ctypes.c_double(dy), ctypes.c_double(top), ctypes.c_double(depth),
                           ctypes.c_double(miss), _p(out))
    return out
