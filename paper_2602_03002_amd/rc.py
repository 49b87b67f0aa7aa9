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
RC_POST_NOISE, RC_POST_DROPOUT, RC_POST_LATENCY, RC_POST_SIDEMASK = 1, 2, 4, 8

# Random side masking defaults (the paper gives neither the band widths nor the
# probabilities): bands of 1/8 and 1/4 of the width per side; terrain type 0
# (slopes, stairs) favours large masks, type 1 (stepping stones) small ones.
SIDEMASK_FRAC = (0.125, 0.25)
SIDEMASK_P = ((0.4, 0.2, 0.4), (0.4, 0.4, 0.2), (1.0, 0.0, 0.0), (1.0, 0.0, 0.0))

EXPORTED = [
    "rc_version", "rc_status_string", "rc_last_error",
    "rc_scene_size", "rc_scene_create", "rc_scene_destroy",
    "rc_robot_size", "rc_robot_meshes",
    "rc_render_size", "rc_render", "rc_render_exact_count", "rc_render_counts", "rc_render_noalloc",
    "rc_post_size", "rc_post_create", "rc_post_reset", "rc_postprocess", "rc_post_destroy",
    "rc_postprocess_words",
    "rc_downsample", "rc_heightmap",
    "rc_bvh_layout_of", "rc_scene_rebuild_sah", "rc_sah_build_host",
    "rc_render_batched_size", "rc_render_batched", "rc_render_batched_status",
    "rc_get_render_config", "rc_set_render_config", "rc_autotune", "rc_set_walk_stack_limit",
    "rc_graph_capture_batched", "rc_graph_launch", "rc_graph_destroy",
    "rc_post_size_packed", "rc_post_create_packed", "rc_postprocess_batched",
    "rc_server_arena_size", "rc_server_create", "rc_server_create_simulated", "rc_server_submit",
    "rc_server_poll", "rc_server_next_result", "rc_server_release", "rc_server_stats_get",
    "rc_server_fail_next",
    "rc_server_destroy",
]

import numpy as np  # noqa: E402

# rc_cam_desc, 64 bytes
CAM_DESC = np.dtype([("env", "<i4"), ("width", "<i4"), ("height", "<i4"), ("out_offset", "<u4"),
                     ("cam_uid", "<u4"), ("pos", "<f4", 3), ("quat", "<f4", 4), ("intr", "<f4", 4)])
assert CAM_DESC.itemsize == 64


class RcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librc status {status}: {msg}")
        self.status = status


class CamRand(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("epoch", ctypes.c_uint64),
                ("trans_m", ctypes.c_float * 3), ("euler_deg", ctypes.c_float * 3),
                ("dfov_deg", ctypes.c_float), ("reserved", ctypes.c_float)]


def cam_rand(seed=0, epoch=0, trans_m=(0.025, 0.025, 0.025), euler_deg=(2.5, 3.0, 2.5),
             dfov_deg=2.0):
    """Perception randomisation of the cameras (defaults: the paper's Table 6 ranges)."""
    return CamRand(int(seed), int(epoch), (ctypes.c_float * 3)(*trans_m),
                   (ctypes.c_float * 3)(*euler_deg), float(dfov_deg), 0.0)


class RenderArgs(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("n_cam", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("link_pos", ctypes.c_void_p), ("link_quat", ctypes.c_void_p),
                ("cam_pos", ctypes.c_void_p), ("cam_quat", ctypes.c_void_p),
                ("intr", ctypes.c_void_p), ("far_plane", ctypes.c_float),
                ("depth_mode", ctypes.c_int32), ("depth", ctypes.c_void_p),
                ("inst", ctypes.c_void_p), ("tri", ctypes.c_void_p),
                ("timing", ctypes.c_void_p), ("cam_rand", ctypes.POINTER(CamRand))]


class HeightmapArgs(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("base_pos", ctypes.c_void_p),
                ("base_yaw", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("top", ctypes.c_float),
                ("depth", ctypes.c_float), ("miss", ctypes.c_float), ("heights", ctypes.c_void_p)]


class PostParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("sigma_abs", ctypes.c_float),
                ("sigma_rel", ctypes.c_float), ("p_drop", ctypes.c_float),
                ("near_plane", ctypes.c_float), ("far_plane", ctypes.c_float),
                ("fill", ctypes.c_float), ("lat_min", ctypes.c_int32),
                ("lat_max", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("mask_frac", ctypes.c_float * 2), ("mask_p", (ctypes.c_float * 3) * 4),
                ("mask_epoch", ctypes.c_uint64), ("mask_type", ctypes.c_void_p)]


class BatchArgs(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("n_desc", ctypes.c_int32),
                ("link_pos", ctypes.c_void_p), ("link_quat", ctypes.c_void_p),
                ("desc", ctypes.c_void_p), ("n_pixels", ctypes.c_int64),
                ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32),
                ("far_plane", ctypes.c_float), ("depth_mode", ctypes.c_int32),
                ("depth", ctypes.c_void_p), ("inst", ctypes.c_void_p), ("tri", ctypes.c_void_p),
                ("timing", ctypes.c_void_p), ("cam_rand", ctypes.POINTER(CamRand))]


class RenderConfig(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("rays_per_lane", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("terrain_packet", ctypes.c_int32),
                ("bodies_flat", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("max_batch_rays", ctypes.c_int64),
                ("out_pixels", ctypes.c_int64), ("far_plane", ctypes.c_float),
                ("depth_mode", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("n_cam", ctypes.c_int32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("link_pos", ctypes.c_void_p),
                ("link_quat", ctypes.c_void_p), ("cam_pos", ctypes.c_void_p),
                ("cam_quat", ctypes.c_void_p), ("intr", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_pixels", ctypes.c_int64), ("depth", ctypes.c_void_p), ("inst", ctypes.c_void_p),
                ("tri", ctypes.c_void_p), ("arrival_s", ctypes.c_double),
                ("launch_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "rejected", "queued",
                                               "in_flight", "batches", "rays_completed")] + \
               [(k, ctypes.c_double) for k in ("p50_s", "p99_s", "mean_s", "max_s",
                                                "first_arrival_s", "last_done_s")]


class BvhLayout(ctypes.Structure):
    _fields_ = [("n_prim", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("node_offset", ctypes.c_int64), ("tri_offset", ctypes.c_int64),
                ("tri_id_offset", ctypes.c_int64), ("key_offset", ctypes.c_int64),
                ("max_depth", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("wide_offset", ctypes.c_int64)]


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
        L.rc_render_exact_count.argtypes = [vp, i32, i32, i32, i32, vp, ctypes.POINTER(i64),
                                            ctypes.POINTER(i64), vp]
        L.rc_render.argtypes = [vp, ctypes.POINTER(RenderArgs), vp, sz, vp]
        L.rc_render_noalloc.argtypes = [vp, ctypes.POINTER(RenderArgs), vp]
        L.rc_render_counts.argtypes = [vp, ctypes.POINTER(RenderArgs), vp, vp, sz, vp]
        L.rc_post_size.argtypes = [i32, i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.rc_post_create.argtypes = [i32, i32, i32, i32, i32, vp, sz, ctypes.POINTER(vp)]
        L.rc_post_reset.argtypes = [vp]
        L.rc_downsample.argtypes = [vp, vp, i64, i32, i32, i32, ctypes.c_float, vp, vp]
        L.rc_heightmap.argtypes = [vp, ctypes.POINTER(HeightmapArgs), vp]
        L.rc_postprocess.argtypes = [vp, vp, vp, ctypes.POINTER(PostParams), ctypes.c_uint64, vp,
                                     vp, vp, vp, vp]
        L.rc_postprocess_words.argtypes = [vp, vp, vp, ctypes.POINTER(PostParams), ctypes.c_uint64, vp,
                                     vp, vp, vp, vp, vp]
        L.rc_post_destroy.argtypes = [vp]
        L.rc_bvh_layout_of.argtypes = [vp, i32, ctypes.POINTER(BvhLayout)]
        L.rc_scene_rebuild_sah.argtypes = [vp, i32, vp]
        L.rc_sah_build_host.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(i32)]
        L.rc_render_batched_size.argtypes = [vp, i32, i32, i64, ctypes.POINTER(sz)]
        L.rc_render_batched.argtypes = [vp, ctypes.POINTER(BatchArgs), vp, sz, vp]
        L.rc_render_batched_status.argtypes = [vp, ctypes.POINTER(BatchArgs), vp,
                                               ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(i64), vp]
        L.rc_get_render_config.argtypes = [vp, i32, ctypes.POINTER(RenderConfig)]
        L.rc_set_render_config.argtypes = [vp, i32, ctypes.POINTER(RenderConfig)]
        L.rc_set_walk_stack_limit.argtypes = [vp, i32]
        L.rc_autotune.argtypes = [vp, ctypes.POINTER(RenderArgs), ctypes.POINTER(BatchArgs), vp, sz,
                                  i32, vp, ctypes.POINTER(RenderConfig), ctypes.POINTER(ctypes.c_float)]
        L.rc_graph_capture_batched.argtypes = [vp, ctypes.POINTER(BatchArgs), vp, sz, vp,
                                               ctypes.POINTER(vp)]
        L.rc_graph_launch.argtypes = [vp, vp]
        L.rc_graph_destroy.argtypes = [vp]
        L.rc_post_size_packed.argtypes = [i64, i32, ctypes.POINTER(sz)]
        L.rc_post_create_packed.argtypes = [i64, i32, vp, sz, ctypes.POINTER(vp)]
        L.rc_postprocess_batched.argtypes = [vp, vp, vp, ctypes.POINTER(PostParams), ctypes.c_uint64,
                                             vp, i32, vp, vp, vp, vp]
        L.rc_server_arena_size.argtypes = [ctypes.POINTER(ServerConfig), sz, ctypes.POINTER(sz)]
        L.rc_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), vp, sz, ctypes.POINTER(vp)]
        L.rc_server_create_simulated.argtypes = [ctypes.POINTER(ServerConfig), sz, ctypes.c_double,
                                                 ctypes.c_double, ctypes.POINTER(vp)]
        L.rc_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.c_double,
                                       ctypes.POINTER(i64)]
        L.rc_server_poll.argtypes = [vp, ctypes.c_double, ctypes.POINTER(i32)]
        L.rc_server_fail_next.argtypes = [vp, i32]
        L.rc_server_next_result.argtypes = [vp, ctypes.POINTER(Result)]
        L.rc_server_release.argtypes = [vp, i64]
        L.rc_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.rc_server_destroy.argtypes = [vp]
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


def _events(timing):
    """Host array of the two raw hipEvent_t handles of a pair of torch events."""
    if timing is None:
        return None
    handles = []
    for ev in timing:
        if ev.cuda_event == 0:  # torch creates the event on its first record
            ev.record()
        handles.append(ev.cuda_event)
    return (ctypes.c_void_p * 2)(*handles)


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


def sah_build_host(tri):
    """rc_sah_build_host on a host array [n][3][3] float32: (records [m][16]
    float32 with int32 child/parent/sibling words, leaf-order triangles
    [n][9], input ids [n], depth)."""
    import numpy as np
    t = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    n = t.shape[0]
    rec = np.zeros((max(n - 1, 1), 16), np.float32)
    tris = np.zeros((n, 9), np.float32)
    ids = np.zeros(n, np.int32)
    d = ctypes.c_int32()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    check(lib().rc_sah_build_host(p(t), n, p(rec), p(tris), p(ids), ctypes.byref(d)))
    return rec, tris, ids, d.value


class Scene:
    """Terrain hierarchy (+ optional robot link hierarchies) resident on the device."""

    def __init__(self, terrain, stream=None, sah=True):
        """sah: rebuild the terrain's (and later the links') hierarchies with
        the binned SAH after the Morton build (rc_scene_rebuild_sah); False
        keeps the Morton ones."""
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
        self.sah = sah
        if sah:
            check(L.rc_scene_rebuild_sah(h, 1, _stream(stream)))

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
            if self.sah:
                check(L.rc_scene_rebuild_sah(self.handle, 2, _stream(stream)))
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

    def exact_count(self, n_env, n_cam, width, height, stream=None, recast=False):
        """Rays the last render with these sizes sent to the exact pass (and, with
        recast=True, also how many of them it re-cast in full)."""
        ws = self.render_workspace(n_env, n_cam, width, height)
        c = ctypes.c_int64()
        r = ctypes.c_int64()
        check(lib().rc_render_exact_count(self.handle, n_env, n_cam, width, height,
                                          ctypes.c_void_p(ws.ptr), ctypes.byref(c), ctypes.byref(r),
                                          _stream(stream)))
        return (c.value, r.value) if recast else c.value

    def _plain_args(self, cam_pos, cam_quat, intr, width, height, far_plane, link_pos, link_quat,
                    depth_mode, out, ids, timing=None, rand=None, want_ws=True):
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
        ev = _events(timing)
        a = RenderArgs(E, C, width, height, _ptr(link_pos) if self.n_links else None,
                       _ptr(link_quat) if self.n_links else None, _ptr(cam_pos), _ptr(cam_quat),
                       _ptr(intr), float(far_plane), depth_mode, _ptr(depth), _ptr(inst), _ptr(tri),
                       ctypes.cast(ev, ctypes.c_void_p) if ev is not None else None,
                       ctypes.pointer(rand) if rand is not None else None)
        a._ev = ev  # keep the event array and randomisation alive with the argument block
        a._rand = rand
        return a, (depth, inst, tri), (self.render_workspace(E, C, width, height) if want_ws else None)

    def render(self, cam_pos, cam_quat, intr, width, height, far_plane, link_pos=None,
               link_quat=None, depth_mode=RC_DEPTH_PLANAR, out=None, ids=True, stream=None,
               timing=None, rand=None):
        """Returns (depth [E,C,H,W] f32, inst i32 or None, tri i32 or None).
        timing: optional pair of recorded torch.cuda.Event(enable_timing=True) placed
        around the fast-pass kernel.  rand: optional cam_rand(...) randomisation."""
        a, outs, ws = self._plain_args(cam_pos, cam_quat, intr, width, height, far_plane, link_pos,
                                       link_quat, depth_mode, out, ids, timing, rand)
        check(lib().rc_render(self.handle, ctypes.byref(a), ctypes.c_void_p(ws.ptr), ws.nbytes,
                              _stream(stream)))
        return outs

    def render_noalloc(self, cam_pos, cam_quat, intr, width, height, far_plane, link_pos=None,
                       link_quat=None, depth_mode=RC_DEPTH_PLANAR, out=None, ids=True, stream=None):
        """rc_render_noalloc: render() without a workspace (the library's static
        per-GPU scratch; calls on one GPU must not overlap).  Pass `out` to
        allocate nothing here either."""
        a, outs, _ = self._plain_args(cam_pos, cam_quat, intr, width, height, far_plane, link_pos,
                                      link_quat, depth_mode, out, ids, want_ws=False)
        check(lib().rc_render_noalloc(self.handle, ctypes.byref(a), _stream(stream)))
        return outs

    def render_counts(self, cam_pos, cam_quat, intr, width, height, far_plane, link_pos=None,
                      link_quat=None, depth_mode=RC_DEPTH_PLANAR, out=None, stream=None):
        """rc_render plus per-ray work counts.  Returns ((depth, inst, tri),
        counts int32 [E,C,H,W,4] = (node records, triangles, instances, link node records))."""
        a, outs, ws = self._plain_args(cam_pos, cam_quat, intr, width, height, far_plane, link_pos,
                                       link_quat, depth_mode, out, True)
        counts = torch.empty((cam_pos.shape[0], cam_pos.shape[1], height, width, 4),
                             dtype=torch.int32, device=self.device)
        check(lib().rc_render_counts(self.handle, ctypes.byref(a), _ptr(counts),
                                     ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
        return outs, counts

    def heightmap(self, base_pos, base_yaw, nx=17, ny=11, dx=0.1, dy=0.1, top=1.0, depth=3.0,
                  miss=float("nan"), out=None, stream=None):
        """Terrain height minus base height on a local grid [E, ny, nx] around
        each base (the paper's privileged height map: 17 x 11 at 0.1 m)."""
        E = base_pos.shape[0]
        _dev_f32(base_pos, (E, 3), "base_pos")
        _dev_f32(base_yaw, (E,), "base_yaw")
        if out is None:
            out = torch.empty((E, ny, nx), dtype=torch.float32, device=self.device)
        a = HeightmapArgs(E, _ptr(base_pos), _ptr(base_yaw), nx, ny, dx, dy, top, depth, miss,
                          _ptr(out))
        check(lib().rc_heightmap(self.handle, ctypes.byref(a), _stream(stream)))
        return out

    # -- batched uneven form -------------------------------------------------

    def batch(self, desc, n_pixels, max_width, max_height, far_plane, link_pos=None,
              link_quat=None, depth_mode=RC_DEPTH_PLANAR, out=None, ids=True, rand=None):
        """Argument block of a batched render.  desc: uint8 CUDA tensor holding
        n_desc rc_cam_desc records (see CAM_DESC)."""
        if desc.device.type != "cuda" or desc.dtype != torch.uint8 or desc.numel() % 64:
            raise ValueError("desc: need a uint8 CUDA tensor of 64-byte rc_cam_desc records")
        n_desc = desc.numel() // 64
        E = link_pos.shape[0] if link_pos is not None else 1
        if self.n_links > 0:
            _dev_f32(link_pos, (E, self.n_links, 3), "link_pos")
            _dev_f32(link_quat, (E, self.n_links, 4), "link_quat")
        if out is None:
            depth = torch.empty(n_pixels, dtype=torch.float32, device=self.device)
            inst = torch.empty(n_pixels, dtype=torch.int32, device=self.device) if ids else None
            tri = torch.empty(n_pixels, dtype=torch.int32, device=self.device) if ids else None
        else:
            depth, inst, tri = out
        a = BatchArgs(E, n_desc, _ptr(link_pos) if self.n_links else None,
                      _ptr(link_quat) if self.n_links else None, _ptr(desc), int(n_pixels),
                      int(max_width), int(max_height), float(far_plane), depth_mode, _ptr(depth),
                      _ptr(inst), _ptr(tri), None, ctypes.pointer(rand) if rand is not None else None)
        a._rand = rand
        key = ("batch", E, n_desc, int(n_pixels))
        ws = self._render_ws.get(key)
        if ws is None:
            size = ctypes.c_size_t()
            check(lib().rc_render_batched_size(self.handle, E, n_desc, int(n_pixels), ctypes.byref(size)))
            ws = Workspace(size.value, self.device)
            self._render_ws[key] = ws
        return Batch(self, a, (depth, inst, tri), ws, (desc, link_pos, link_quat))

    def config(self, batched=False):
        c = RenderConfig()
        check(lib().rc_get_render_config(self.handle, int(batched), ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, batched=False, **kw):
        c = RenderConfig(**{**self.config(batched), **kw})
        check(lib().rc_set_render_config(self.handle, int(batched), ctypes.byref(c)))

    def set_walk_stack_limit(self, entries):
        """Cap the fast pass's per-lane terrain-walk stack (1..16) to exercise
        its overflow path; results do not depend on it."""
        check(lib().rc_set_walk_stack_limit(self.handle, int(entries)))

    def autotune(self, reps=3, stream=None, batch=None, **plain):
        """Time every schedule on one launch (plain keyword args as for render(),
        or batch=Batch) and keep the fastest.  Returns (config dict, ms)."""
        best, ms = RenderConfig(), ctypes.c_float()
        if batch is not None:
            check(lib().rc_autotune(self.handle, None, ctypes.byref(batch.args),
                                    ctypes.c_void_p(batch.ws.ptr), batch.ws.nbytes, reps,
                                    _stream(stream), ctypes.byref(best), ctypes.byref(ms)))
        else:
            a, _, ws = self._plain_args(plain["cam_pos"], plain["cam_quat"], plain["intr"],
                                        plain["width"], plain["height"], plain["far_plane"],
                                        plain.get("link_pos"), plain.get("link_quat"),
                                        plain.get("depth_mode", RC_DEPTH_PLANAR), plain.get("out"),
                                        True)
            check(lib().rc_autotune(self.handle, ctypes.byref(a), None, ctypes.c_void_p(ws.ptr),
                                    ws.nbytes, reps, _stream(stream), ctypes.byref(best),
                                    ctypes.byref(ms)))
        return best.as_dict(), ms.value

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


class Batch:
    """A batched render's arguments, outputs and workspace (keeps tensors alive)."""

    def __init__(self, scene, args, outs, ws, keep):
        self.scene, self.args, self.outs, self.ws, self._keep = scene, args, outs, ws, keep

    def render(self, stream=None):
        check(lib().rc_render_batched(self.scene.handle, ctypes.byref(self.args),
                                      ctypes.c_void_p(self.ws.ptr), self.ws.nbytes, _stream(stream)))
        return self.outs

    def status(self, stream=None):
        """(status word, rays re-cast exactly) of the last render; synchronises."""
        st, n = ctypes.c_uint32(), ctypes.c_int64()
        check(lib().rc_render_batched_status(self.scene.handle, ctypes.byref(self.args),
                                             ctypes.c_void_p(self.ws.ptr), ctypes.byref(st),
                                             ctypes.byref(n), _stream(stream)))
        return st.value, n.value

    def capture(self, stream=None):
        """Capture this render into a graph; replay with Graph.launch().  The
        legacy null stream cannot capture, so a side stream is used by default."""
        s = stream if stream is not None else torch.cuda.Stream()
        g = ctypes.c_void_p()
        check(lib().rc_graph_capture_batched(self.scene.handle, ctypes.byref(self.args),
                                             ctypes.c_void_p(self.ws.ptr), self.ws.nbytes,
                                             ctypes.c_void_p(s.cuda_stream), ctypes.byref(g)))
        return Graph(g, self)


class Graph:
    def __init__(self, handle, batch):
        self.handle, self.batch = handle, batch

    def launch(self, stream=None):
        check(lib().rc_graph_launch(self.handle, _stream(stream)))
        return self.batch.outs

    def close(self):
        if self.handle:
            lib().rc_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def downsample(depth, inst, factor, far_plane, out=None, stream=None):
    """Block pooling of frames [..., H, W] (mean of hit pixels, else far_plane)
    into [..., H // factor, W // factor]."""
    H, W = depth.shape[-2], depth.shape[-1]
    lead = depth.shape[:-2]
    n_img = 1
    for d in lead:
        n_img *= d
    _dev_f32(depth, depth.shape, "depth")
    if out is None and 1 <= factor <= min(H, W):  # other factors: the library reports the error
        out = torch.empty(tuple(lead) + (H // factor, W // factor), dtype=torch.float32,
                          device=depth.device)
    check(lib().rc_downsample(_ptr(depth), _ptr(inst), n_img, H, W, factor, float(far_plane),
                              _ptr(out), _stream(stream)))
    return out


def post_params(seed=0, sigma_abs=0.0, sigma_rel=0.0, p_drop=0.0, near=0.05, far=3.0, fill=0.0,
                lat_min=0, lat_max=0, flags=None, side_mask=False, mask_frac=SIDEMASK_FRAC,
                mask_p=SIDEMASK_P, mask_epoch=0, mask_type=None):
    """mask_type: optional uint8 CUDA tensor [n_env] of terrain types (0..3)."""
    if flags is None:
        flags = (RC_POST_NOISE if (sigma_abs or sigma_rel) else 0) | \
                (RC_POST_DROPOUT if p_drop else 0) | (RC_POST_LATENCY if lat_max else 0) | \
                (RC_POST_SIDEMASK if side_mask else 0)
    p = PostParams(seed, sigma_abs, sigma_rel, p_drop, near, far, fill, lat_min, lat_max, flags,
                   (ctypes.c_float * 2)(*mask_frac),
                   ((ctypes.c_float * 3) * 4)(*[(ctypes.c_float * 3)(*row) for row in mask_p]),
                   int(mask_epoch), _ptr(mask_type))
    p._mask_type = mask_type  # keep the device table alive with the parameters
    return p


class Post:
    """Sensor-model state (device ring of max_latency + 1 frames).  Post(E, C, H, W,
    L) for the plain layout; Post.packed(n_pixels, L) for batched outputs."""

    def __init__(self, n_env, n_cam, height, width, max_latency, device="cuda", _packed=None):
        L = lib()
        size = ctypes.c_size_t()
        h = ctypes.c_void_p()
        if _packed is None:
            check(L.rc_post_size(n_env, n_cam, height, width, max_latency, ctypes.byref(size)))
            self.ws = Workspace(size.value, device)
            check(L.rc_post_create(n_env, n_cam, height, width, max_latency,
                                   ctypes.c_void_p(self.ws.ptr), size.value, ctypes.byref(h)))
            self.shape = (n_env, n_cam, height, width)
        else:
            check(L.rc_post_size_packed(_packed, max_latency, ctypes.byref(size)))
            self.ws = Workspace(size.value, device)
            check(L.rc_post_create_packed(_packed, max_latency, ctypes.c_void_p(self.ws.ptr),
                                          size.value, ctypes.byref(h)))
            self.shape = (_packed,)
        self.handle = h
        self.device = device

    @classmethod
    def packed(cls, n_pixels, max_latency, device="cuda"):
        return cls(0, 0, 0, 0, max_latency, device=device, _packed=int(n_pixels))

    def process_batched(self, depth, inst, params, step, desc, out=None, stream=None):
        """Packed outputs: returns (depth_out [n_pixels], drop [n_pixels], lat [n_desc])."""
        n_desc = desc.numel() // 64
        if out is None:
            d = torch.empty(self.shape, dtype=torch.float32, device=depth.device)
            drop = torch.empty(self.shape, dtype=torch.uint8, device=depth.device)
            lat = torch.empty(n_desc, dtype=torch.uint8, device=depth.device)
        else:
            d, drop, lat = out
        check(lib().rc_postprocess_batched(self.handle, _ptr(depth), _ptr(inst), ctypes.byref(params),
                                           int(step), _ptr(desc), n_desc, _ptr(d), _ptr(drop),
                                           _ptr(lat), _stream(stream)))
        return d, drop, lat

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

    def process_words(self, depth, inst, params, step, cam_uid=None, stream=None):
        """process() plus the raw Philox words of every pixel's draw: returns
        (depth_out, drop, lat, words uint32 [E,C,H,W,4] as int32 storage)."""
        _dev_f32(depth, self.shape, "depth")
        d = torch.empty(self.shape, dtype=torch.float32, device=depth.device)
        drop = torch.empty(self.shape, dtype=torch.uint8, device=depth.device)
        lat = torch.empty(self.shape[:2], dtype=torch.uint8, device=depth.device)
        words = torch.empty(tuple(self.shape) + (4,), dtype=torch.int32, device=depth.device)
        check(lib().rc_postprocess_words(self.handle, _ptr(depth), _ptr(inst), ctypes.byref(params),
                                         int(step), _ptr(cam_uid), _ptr(d), _ptr(drop), _ptr(lat),
                                         _ptr(words), _stream(stream)))
        return d, drop, lat, words

    def close(self):
        if self.handle:
            lib().rc_post_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over a resident scene (or, with simulated(), over a timing model).

    submit() queues a request at the caller's clock time; poll() collects finished
    batches and starts new ones; next_result() hands back finished requests whose
    outputs stay valid until release()."""

    def __init__(self, scene, n_streams=8, max_batch_rays=1 << 22, out_pixels=1 << 26,
                 scratch_bytes=1 << 30, far_plane=3.0, depth_mode=RC_DEPTH_PLANAR, _sim=None):
        L = lib()
        self.cfg = ServerConfig(n_streams, int(max_batch_rays), int(out_pixels), float(far_plane),
                                depth_mode)
        size = ctypes.c_size_t()
        check(L.rc_server_arena_size(ctypes.byref(self.cfg), int(scratch_bytes), ctypes.byref(size)))
        h = ctypes.c_void_p()
        self.arena = None
        if _sim is None:
            self.arena = Workspace(size.value, scene.device)
            check(L.rc_server_create(scene.handle, ctypes.byref(self.cfg),
                                     ctypes.c_void_p(self.arena.ptr), size.value, ctypes.byref(h)))
        else:
            check(L.rc_server_create_simulated(ctypes.byref(self.cfg), size.value, _sim[0], _sim[1],
                                               ctypes.byref(h)))
        self.handle = h
        self.scene = scene
        self._inputs = {}

    @classmethod
    def simulated(cls, launch_s, s_per_ray, **kw):
        return cls(None, _sim=(float(launch_s), float(s_per_ray)), **kw)

    def submit(self, now, n_env, n_cam, width, height, link_pos=None, link_quat=None,
               cam_pos=None, cam_quat=None, intr=None):
        r = Request(n_env, n_cam, width, height, _ptr(link_pos), _ptr(link_quat), _ptr(cam_pos),
                    _ptr(cam_quat), _ptr(intr))
        i = ctypes.c_int64()
        check(lib().rc_server_submit(self.handle, ctypes.byref(r), float(now), ctypes.byref(i)))
        self._inputs[i.value] = (link_pos, link_quat, cam_pos, cam_quat, intr)
        return i.value

    def fail_next(self, n_batches=1):
        """Report the next n_batches completed batches as failed (testing aid)."""
        check(lib().rc_server_fail_next(self.handle, int(n_batches)))

    def poll(self, now):
        n = ctypes.c_int32()
        check(lib().rc_server_poll(self.handle, float(now), ctypes.byref(n)))
        return n.value

    def next_result(self):
        r = Result()
        if lib().rc_server_next_result(self.handle, ctypes.byref(r)) != RC_OK:
            return None
        return {k: getattr(r, k) for k, _ in Result._fields_}

    def outputs(self, res, shape):
        """(depth, inst, tri) tensor views of a result inside the arena."""
        n = res["n_pixels"]
        base = self.arena.ptr
        views = []
        for key, dt in (("depth", torch.float32), ("inst", torch.int32), ("tri", torch.int32)):
            off = res[key] - base
            views.append(self.arena.buf[self.arena.offset + off:self.arena.offset + off + 4 * n]
                         .view(dt).view(shape))
        return tuple(views)

    def release(self, rid):
        check(lib().rc_server_release(self.handle, int(rid)))
        self._inputs.pop(rid, None)

    def stats(self):
        st = ServerStats()
        check(lib().rc_server_stats_get(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            h, self.handle = self.handle, None
            check(lib().rc_server_destroy(h))  # freed either way; raises on a device error

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
