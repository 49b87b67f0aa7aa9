"""Python binding of librc's C-ABI (include/rc.h): argument marshalling only.

Torch tensors provide device memory and streams; every step of the path runs
in librc's HIP kernels.  If librc.so is missing this module raises: there is
no fallback implementation.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librc.so")

RC_OK = 0
RC_DEPTH_PLANAR, RC_DEPTH_RANGE = 0, 1
RC_POST_NOISE, RC_POST_DROPOUT, RC_POST_LATENCY = 1, 2, 4

EXPORTED = [
    "rc_version", "rc_status_string", "rc_last_error",
    "rc_scene_size", "rc_scene_create", "rc_scene_destroy",
    "rc_robot_size", "rc_robot_meshes",
    "rc_render_size", "rc_render", "rc_render_exact_count",
    "rc_post_size", "rc_post_create", "rc_post_reset", "rc_postprocess", "rc_post_destroy",
    "rc_bvh_layout_of",
]


class RcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librc status {status}: {msg}")
        self.status = status


class RenderArgs(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("n_cam", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("link_pos", ctypes.c_void_p), ("link_quat", ctypes.c_void_p),
                ("cam_pos", ctypes.c_void_p), ("cam_quat", ctypes.c_void_p),
                ("intr", ctypes.c_void_p), ("far_plane", ctypes.c_float),
                ("depth_mode", ctypes.c_int32), ("depth", ctypes.c_void_p),
                ("inst", ctypes.c_void_p), ("tri", ctypes.c_void_p)]


class PostParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("sigma_abs", ctypes.c_float),
                ("sigma_rel", ctypes.c_float), ("p_drop", ctypes.c_float),
                ("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float),
                ("fill", ctypes.c_float), ("lat_min", ctypes.c_int32),
                ("lat_max", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class BvhLayout(ctypes.Structure):
    _fields_ = [("n_prim", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("node_offset", ctypes.c_int64), ("tri_offset", ctypes.c_int64),
                ("tri_id_offset", ctypes.c_int64), ("key_offset", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load librc.so (built by ``paper_2602_03002_amd/build.py``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.rc_version.restype = i32
        L.rc_status_string.restype = ctypes.c_char_p
        L.rc_status_string.argtypes = [i32]
        L.rc_last_error.restype = ctypes.c_char_p
        L.rc_scene_size.argtypes = [i64, ctypes.POINTER(sz)]
        L.rc_scene_create.argtypes = [vp, i64, vp, sz, vp, ctypes.POINTER(vp)]
        L.rc_scene_destroy.argtypes = [vp]
        L.rc_robot_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
        L.rc_robot_meshes.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        L.rc_render_size.argtypes = [vp, i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.rc_render_exact_count.argtypes = [vp, i32, i32, i32, i32, vp, ctypes.POINTER(i64), vp]
        L.rc_render.argtypes = [vp, ctypes.POINTER(RenderArgs), vp, sz, vp]
        L.rc_post_size.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.rc_post_create.argtypes = [i32, i32, i32, i32, i32, vp, sz, ctypes.POINTER(vp)]
        L.rc_post_reset.argtypes = [vp]
        L.rc_postprocess.argtypes = [vp, vp, vp, ctypes.POINTER(PostParams), ctypes.c_uint64, vp,
                                     vp, vp, vp, vp]
        L.rc_post_destroy.argtypes = [vp]
        L.rc_bvh_layout_of.argtypes = [vp, i32, ctypes.POINTER(BvhLayout)]
        for name in EXPORTED:
            if name not in ("rc_version", "rc_status_string", "rc_last_error"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def check(status):
    if status != RC_OK:
        raise RcError(status, lib().rc_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, shape, name):
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    return t


class Workspace:
    """Caller-owned device bytes with a 256-byte aligned base pointer."""

    def __init__(self, nbytes, device):
        self.buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
        base = self.buf.data_ptr()
        self.offset = (-base) % 256
        self.nbytes = int(nbytes)
        self.ptr = base + self.offset

    def view(self):
        return self.buf[self.offset:self.offset + self.nbytes]


class Scene:
    """Terrain hierarchy (+ optional robot link hierarchies) resident on the device."""

    def __init__(self, terrain, stream=None):
        terrain = _dev_f32(terrain, (terrain.shape[0], 3, 3), "terrain")
        L = lib()
        self.device = terrain.device
        n = terrain.shape[0]
        size = ctypes.c_size_t()
        check(L.rc_scene_size(n, ctypes.byref(size)))
        self.ws = Workspace(size.value, self.device)
        h = ctypes.c_void_p()
        check(L.rc_scene_create(_ptr(terrain), n, ctypes.c_void_p(self.ws.ptr), size.value,
                                _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_links = 0
        self.robot_ws = None
        self._render_ws = {}

    def set_robot(self, link_tri, tri_offset, stream=None):
        L = lib()
        off = (ctypes.c_int64 * len(tri_offset))(*[int(x) for x in tri_offset])
        nb = len(tri_offset) - 1
        size = ctypes.c_size_t()
        check(L.rc_robot_size(off, nb, ctypes.byref(size)))
        if nb > 0:
            link_tri = _dev_f32(link_tri, (int(tri_offset[-1]), 3, 3), "link_tri")
            self.robot_ws = Workspace(size.value, self.device)
            check(L.rc_robot_meshes(self.handle, _ptr(link_tri), off, nb,
                                    ctypes.c_void_p(self.robot_ws.ptr), size.value,
                                    _stream(stream)))
        else:
            check(L.rc_robot_meshes(self.handle, None, off, 0, None, 0, _stream(stream)))
            self.robot_ws = None
        self.n_links = nb
        self._render_ws = {}

    def render_workspace(self, n_env, n_cam, width, height):
        key = (n_env, n_cam, width, height)
        ws = self._render_ws.get(key)
        if ws is None:
            size = ctypes.c_size_t()
            check(lib().rc_render_size(self.handle, n_env, n_cam, width, height, ctypes.byref(size)))
            ws = Workspace(size.value, self.device)
            self._render_ws[key] = ws
        return ws

    def exact_count(self, n_env, n_cam, width, height, stream=None):
        """Rays the last render with these sizes sent to the exact pass."""
        ws = self.render_workspace(n_env, n_cam, width, height)
        c = ctypes.c_int64()
        check(lib().rc_render_exact_count(self.handle, n_env, n_cam, width, height,
                                          ctypes.c_void_p(ws.ptr), ctypes.byref(c), _stream(stream)))
        return c.value

    def render(self, cam_pos, cam_quat, intr, width, height, far_plane, link_pos=None,
               link_quat=None, depth_mode=RC_DEPTH_PLANAR, out=None, ids=True, stream=None):
        """Returns (depth [E,C,H,W] f32, inst i32 or None, tri i32 or None)."""
        E, C = cam_pos.shape[0], cam_pos.shape[1]
        _dev_f32(cam_pos, (E, C, 3), "cam_pos")
        _dev_f32(cam_quat, (E, C, 4), "cam_quat")
        _dev_f32(intr, (E, C, 4), "intr")
        if self.n_links > 0:
            _dev_f32(link_pos, (E, self.n_links, 3), "link_pos")
            _dev_f32(link_quat, (E, self.n_links, 4), "link_quat")
        if out is None:
            depth = torch.empty((E, C, height, width), dtype=torch.float32, device=self.device)
            inst = torch.empty_like(depth, dtype=torch.int32) if ids else None
            tri = torch.empty_like(depth, dtype=torch.int32) if ids else None
        else:
            depth, inst, tri = out
        ws = self.render_workspace(E, C, width, height)
        a = RenderArgs(E, C, width, height, _ptr(link_pos) if self.n_links else None,
                       _ptr(link_quat) if self.n_links else None, _ptr(cam_pos), _ptr(cam_quat),
                       _ptr(intr), float(far_plane), depth_mode, _ptr(depth), _ptr(inst), _ptr(tri))
        check(lib().rc_render(self.handle, ctypes.byref(a), ctypes.c_void_p(ws.ptr), ws.nbytes,
                              _stream(stream)))
        return depth, inst, tri

    def bvh_layout(self, which=-1):
        out = BvhLayout()
        check(lib().rc_bvh_layout_of(self.handle, which, ctypes.byref(out)))
        return out

    def close(self):
        if self.handle:
            lib().rc_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def post_params(seed=0, sigma_abs=0.0, sigma_rel=0.0, p_drop=0.0, near=0.05, far=3.0, fill=0.0,
                lat_min=0, lat_max=0, flags=None):
    if flags is None:
        flags = (RC_POST_NOISE if (sigma_abs or sigma_rel) else 0) | \
                (RC_POST_DROPOUT if p_drop else 0) | (RC_POST_LATENCY if lat_max else 0)
    return PostParams(seed, sigma_abs, sigma_rel, p_drop, near, far, fill, lat_min, lat_max, flags)


class Post:
    """Sensor-model state (device ring of max_latency + 1 frames)."""

    def __init__(self, n_env, n_cam, height, width, max_latency, device="cuda"):
        L = lib()
        size = ctypes.c_size_t()
        check(L.rc_post_size(n_env, n_cam, height, width, max_latency, ctypes.byref(size)))
        self.ws = Workspace(size.value, device)
        h = ctypes.c_void_p()
        check(L.rc_post_create(n_env, n_cam, height, width, max_latency,
                               ctypes.c_void_p(self.ws.ptr), size.value, ctypes.byref(h)))
        self.handle = h
        self.shape = (n_env, n_cam, height, width)
        self.device = device

    def reset(self):
        check(lib().rc_post_reset(self.handle))

    def process(self, depth, inst, params, step, cam_uid=None, out=None, stream=None):
        """Returns (depth_out f32, drop u8, lat u8 [E,C])."""
        _dev_f32(depth, self.shape, "depth")
        if out is None:
            d = torch.empty(self.shape, dtype=torch.float32, device=depth.device)
            drop = torch.empty(self.shape, dtype=torch.uint8, device=depth.device)
            lat = torch.empty(self.shape[:2], dtype=torch.uint8, device=depth.device)
        else:
            d, drop, lat = out
        check(lib().rc_postprocess(self.handle, _ptr(depth), _ptr(inst), ctypes.byref(params),
                                   int(step), _ptr(cam_uid), _ptr(d), _ptr(drop), _ptr(lat),
                                   _stream(stream)))
        return d, drop, lat

    def close(self):
        if self.handle:
            lib().rc_post_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
