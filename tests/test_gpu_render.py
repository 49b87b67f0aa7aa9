"""GPU parity: librc (through its C-ABI) against the FP64 oracle and the CPU LBVH model."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from oracle import lbvh
import scenegen as sg
from parity import assert_parity

pytestmark = pytest.mark.gpu

DEV = "cuda"


def rc():
    import paper_2602_03002_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def make_scene(w, step=0, sah=True):
    m = rc()
    sc = m.Scene(dev(w["terrain"]), sah=sah)
    B = int(w["link_off"].shape[0] - 1)
    if B > 0:
        sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    return sc


def render(sc, w, step=0, depth_mode=0):
    B = sc.n_links
    lp = dev(w["link_pos"][step]) if B else None
    lq = dev(w["link_quat"][step]) if B else None
    d, i, t = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                        w["far"], link_pos=lp, link_quat=lq, depth_mode=depth_mode)
    torch.cuda.synchronize()
    return d.cpu().numpy(), i.cpu().numpy(), t.cpu().numpy()


def oracle_render(w, step=0, depth_mode=0, rays=None):
    return oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][step],
                         w["link_quat"][step], w["cam_pos"], w["cam_quat"], w["intr"], w["W"],
                         w["H"], w["far"], depth_mode=depth_mode, rays=rays)


# ---------------------------------------------------------------------------
# hierarchy build: bit-exact against the CPU model
# ---------------------------------------------------------------------------

def ws_bytes(ws):
    torch.cuda.synchronize()
    return ws.view().cpu().numpy()


def check_bvh(buf, lay, tri):
    model = lbvh.build(tri)
    n, m = lay.n_prim, lay.n_nodes
    rec = buf[lay.node_offset:lay.node_offset + 64 * m].view(np.float32).reshape(m, 16)
    ids = buf[lay.tri_id_offset:lay.tri_id_offset + 4 * n].view(np.int32)
    assert np.array_equal(ids, model["tri_id"]), "leaf order differs"
    if n > 1:
        keys = buf[lay.key_offset:lay.key_offset + 8 * n].view(np.uint64)
        assert np.array_equal(keys, model["keys"]), "Morton keys differ"
    assert np.array_equal(rec.view(np.uint32), model["records"].view(np.uint32)), "node records differ"
    wide = buf[lay.wide_offset:lay.wide_offset + 128 * m].view(np.uint32).reshape(m, 32)
    assert np.array_equal(wide, lbvh.collapse4(model["records"]).view(np.uint32)), "4-wide records differ"
    tris = buf[lay.tri_offset:lay.tri_offset + 36 * n].view(np.float32).reshape(n, 9)
    assert np.array_equal(tris, np.asarray(tri, np.float32).reshape(-1, 9)[model["tri_id"]])
    assert lay.max_depth == model["depth"]


@pytest.mark.parametrize("which", ["profile", "tiles2", "single", "degenerate", "single_degenerate"])
def test_terrain_bvh_bit_exact(which):
    say(f"[bvh] terrain {which}")
    if which == "profile":
        tri = sg.small_plain_case()["terrain"]
    elif which == "tiles2":
        tri = sg.TileTerrain(2).triangles()
    elif which == "degenerate":
        # zero-area triangles among proper ones: unreachable leaves
        t = sg.TileTerrain(1).triangles()[:5000]
        p = t[::97, 0]
        u = np.float32([2.0 ** -6, 0.0, 0.0])
        tri = np.concatenate([t, np.stack([p, p, p], 1), np.stack([p - u, p, p + u], 1)], 0)
    elif which == "single_degenerate":
        tri = np.array([[[0, 0, 0], [1, 1, 1], [2, 2, 2]]], np.float32)
    else:
        tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    sc = rc().Scene(dev(tri), sah=False)
    check_bvh(ws_bytes(sc.ws), sc.bvh_layout(-1), tri)


@pytest.mark.parametrize("which", ["tiles2", "single", "degenerate"])
def test_sah_rebuild_matches_the_host_builder(which):
    """rc_scene_rebuild_sah: the terrain's records, leaf-order triangles, ids
    and 4-wide records equal the host builder's output over the Morton
    build's leaf order (ids mapped through it), bit for bit."""
    say(f"[bvh] SAH rebuild {which}")
    if which == "tiles2":
        tri = sg.TileTerrain(2).triangles()
    elif which == "degenerate":
        t = sg.TileTerrain(1).triangles()[:5000]
        p = t[::97, 0]
        tri = np.concatenate([t, np.stack([p, p, p], 1)], 0).astype(np.float32)
    else:
        tri = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
    m = rc()
    s0 = m.Scene(dev(tri), sah=False)
    b0, l0 = ws_bytes(s0.ws), s0.bvh_layout(-1)
    n, nn = l0.n_prim, l0.n_nodes
    t0 = b0[l0.tri_offset:l0.tri_offset + 36 * n].view(np.float32).reshape(n, 9)
    i0 = b0[l0.tri_id_offset:l0.tri_id_offset + 4 * n].view(np.int32)
    rec, tris, ids, depth = m.sah_build_host(t0.reshape(n, 3, 3))
    s1 = m.Scene(dev(tri))
    b1, l1 = ws_bytes(s1.ws), s1.bvh_layout(-1)
    assert (l1.node_offset, l1.wide_offset, l1.tri_offset) == (l0.node_offset, l0.wide_offset, l0.tri_offset)
    got = b1[l1.node_offset:l1.node_offset + 64 * nn].view(np.uint32).reshape(nn, 16)
    assert np.array_equal(got, rec.view(np.uint32)), "records"
    assert np.array_equal(b1[l1.tri_offset:l1.tri_offset + 36 * n].view(np.float32).reshape(n, 9), tris)
    assert np.array_equal(b1[l1.tri_id_offset:l1.tri_id_offset + 4 * n].view(np.int32), i0[ids])
    wide = b1[l1.wide_offset:l1.wide_offset + 128 * nn].view(np.uint32).reshape(nn, 32)
    assert np.array_equal(wide, lbvh.collapse4(rec).view(np.uint32)), "4-wide records"
    assert l1.max_depth == depth


def test_link_bvh_bit_exact():
    say("[bvh] 30 link meshes")
    rob = sg.Robot()
    lt, off = rob.link_triangles()
    sc = rc().Scene(dev(sg.small_plain_case()["terrain"]), sah=False)
    sc.set_robot(dev(lt), off.tolist())
    buf = ws_bytes(sc.robot_ws)
    for b in (0, 13, 29):
        check_bvh(buf, sc.bvh_layout(b), lt[off[b]:off[b + 1]])


def test_link_sah_rebuild_matches_the_host_builder():
    """The link meshes' hierarchies after rc_scene_rebuild_sah (which = 2, as
    Scene.set_robot does with sah=True) against the host builder over the
    Morton build's leaf order, bit for bit."""
    say("[bvh] SAH rebuild of 30 link meshes")
    rob = sg.Robot()
    lt, off = rob.link_triangles()
    terr = dev(sg.small_plain_case()["terrain"])
    m = rc()
    s0 = m.Scene(terr, sah=False)
    s0.set_robot(dev(lt), off.tolist())
    s1 = m.Scene(terr)
    s1.set_robot(dev(lt), off.tolist())
    b0, b1 = ws_bytes(s0.robot_ws), ws_bytes(s1.robot_ws)
    for b in (0, 13, 29):
        l0, l1 = s0.bvh_layout(b), s1.bvh_layout(b)
        n, nn = l0.n_prim, l0.n_nodes
        t0 = b0[l0.tri_offset:l0.tri_offset + 36 * n].view(np.float32).reshape(n, 3, 3)
        i0 = b0[l0.tri_id_offset:l0.tri_id_offset + 4 * n].view(np.int32)
        rec, tris, ids, depth = m.sah_build_host(t0)
        assert np.array_equal(b1[l1.node_offset:l1.node_offset + 64 * nn].view(np.uint32).reshape(nn, 16),
                              rec.view(np.uint32)), f"link {b} records"
        assert np.array_equal(b1[l1.tri_offset:l1.tri_offset + 36 * n].view(np.float32).reshape(n, 9), tris)
        assert np.array_equal(b1[l1.tri_id_offset:l1.tri_id_offset + 4 * n].view(np.int32), i0[ids])
        assert l1.max_depth == depth


def _align(x, a=256):
    return (x + a - 1) // a * a


@pytest.mark.parametrize("bodies_flat", [0, 1])
def test_tlas_bit_exact(bodies_flat):
    """The per-step top level (instance transforms, and with the top-level walk
    schedule the node records) against the CPU model, for given poses,
    including absent links (non-finite poses, a zero quaternion)."""
    say(f"[tlas] 64 envs x 30 links, bodies_flat {bodies_flat}")
    w = sg.robot_scene(2, 8, 2.5, 2, 16, 12, steps=1, label="tlas")
    lp, lq = w["link_pos"][0].copy(), w["link_quat"][0].copy()
    lp[3, 7, 0] = np.nan
    lq[5, 0] = 0.0
    lq[9, 29, 2] = np.inf
    lp[9, 12, 2] = -np.inf
    sc = make_scene(w)
    sc.set_config(batched=False, bodies_flat=bodies_flat)
    E, B = lp.shape[0], lp.shape[1]
    sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"], w["far"],
              link_pos=dev(lp), link_quat=dev(lq))
    buf = ws_bytes(sc.render_workspace(E, 2, w["W"], w["H"]))
    meta = ws_bytes(sc.robot_ws)[:64 * B].view(np.float32).reshape(B, 16)
    root = meta[:, 4:10]
    n_rec = B - 1
    nodes = buf[:E * n_rec * 64].view(np.float32).reshape(E, n_rec, 16)
    x0 = _align(E * n_rec * 64)
    xf = buf[x0:x0 + E * B * 64].view(np.float32).reshape(E, B, 16)
    lo, hi = root[:, 0::2].astype(np.float64), root[:, 1::2].astype(np.float64)
    corners = np.stack([np.where([(k >> a) & 1 for a in range(3)], hi, lo) for k in range(8)], 1)
    for e in range(E):
        mx, mrec = lbvh.tlas(lp[e], lq[e], root)
        assert np.array_equal(xf[e, :, :12].view(np.uint32), mx.view(np.uint32)), f"transforms of env {e}"
        # bounding spheres: an absent link's is the far point with radius 0;
        # otherwise it holds the posed local box (corners under the model's
        # R, t) and its radius is the half-diagonal widened by 1% + 1 mm
        for b in range(B):
            sph = xf[e, b, 12:16].astype(np.float64)
            if mx[b, 9] == lbvh.FAR_POINT:
                assert np.array_equal(xf[e, b, 12:16], np.float32([1e30, 1e30, 1e30, 0])), (e, b)
                continue
            R, t = mx[b, :9].astype(np.float64).reshape(3, 3).T, mx[b, 9:12].astype(np.float64)
            w = corners[b] @ R.T + t
            half = 0.5 * np.linalg.norm(hi[b] - lo[b])
            assert abs(sph[3] - (half * 1.01 + 1e-3)) <= 1e-6 * sph[3], (e, b)
            assert np.max(np.linalg.norm(w - sph[:3], axis=1)) <= sph[3], (e, b)
            ctr = R @ (0.5 * (lo[b] + hi[b])) + t
            assert np.max(np.abs(ctr - sph[:3])) <= 1e-6 * (1 + np.abs(t).max()), (e, b)
        if bodies_flat == 0:
            g, mm = nodes[e].view(np.uint32), mrec.view(np.uint32)
            bad = np.argwhere(g != mm)
            assert bad.size == 0, (f"top level of env {e}: {len(bad)} words differ, first "
                                   f"{[(int(r), int(c), nodes[e][r, c], mrec[r, c], g[r, c], mm[r, c]) for r, c in bad[:6]]}")


def test_non_finite_link_poses_render_as_absent_links():
    """Links with a non-finite pose or a zero quaternion are absent from their
    environment (the oracle's reading); every schedule agrees."""
    say("[render] 4 envs x 2 cams 37x29, links with non-finite poses")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="parity-ragged")
    w["link_pos"] = w["link_pos"].copy()
    w["link_quat"] = w["link_quat"].copy()
    w["link_pos"][0, 0, 0:30:3, 1] = np.nan
    w["link_quat"][0, 1, 1:30:2] = 0.0
    w["link_quat"][0, 2, :, 3] = np.inf
    sc = make_scene(w)
    ref = oracle_render(w)
    for flat in (1, 0):
        sc.set_config(batched=False, bodies_flat=flat)
        d, i, t = render(sc, w)
        assert_parity(d, i, t, ref, w["far"], label=f"non-finite poses, bodies_flat {flat}")
    assert not np.any((i.reshape(4, -1)[2] >= 0) & (i.reshape(4, -1)[2] < 30))


# ---------------------------------------------------------------------------
# rendering parity
# ---------------------------------------------------------------------------

def test_small_plain_case_full_frame():
    say("[render] 1 env x 1 cam 32x24, terrain profile")
    w = sg.small_plain_case()
    sc = make_scene(w)
    d, i, t = render(sc, w)
    ref = oracle_render(w)
    assert_parity(d, i, t, ref, w["far"], label="small plain case")
    assert np.all(i == 0)


@pytest.mark.parametrize("depth_mode,sah", [(0, True), (1, True), (0, False)])
def test_robot_scene_full_frame_ragged(depth_mode, sah):
    say(f"[render] 4 envs x 2 cams 37x29 (ragged tiles), 2x2 tiles, 30 links, mode {depth_mode}, "
        f"{'SAH' if sah else 'Morton'} terrain hierarchy")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=2, label="parity-ragged")
    sc = make_scene(w, sah=sah)
    for step in (0, 1):
        d, i, t = render(sc, w, step, depth_mode)
        ref = oracle_render(w, step, depth_mode)
        r = assert_parity(d, i, t, ref, w["far"], label=f"ragged step {step} mode {depth_mode}")
        assert (i >= 0).mean() > 0.5
        assert ((i >= 0) & (i < 30)).sum() > 20, "the cameras should see the robot"
        del r


def test_single_link_and_single_triangle():
    say("[render] one link, one-triangle terrain")
    w = sg.robot_scene(1, 1, 4.0, 2, 16, 12, steps=1, label="single")
    w["link_tri"] = w["link_tri"][:512]
    w["link_off"] = np.array([0, 512], np.int64)
    w["link_pos"] = np.ascontiguousarray(w["link_pos"][:, :, 10:11])  # a leg link in view
    w["link_quat"] = np.ascontiguousarray(w["link_quat"][:, :, 10:11])
    w["terrain"] = np.array([[[-5, -5, 0], [5, -5, 0], [0, 5, 0]]], np.float32) + \
        np.float32([w["cam_pos"][0, 0, 0], w["cam_pos"][0, 0, 1], w["cam_pos"][0, 0, 2] - 1.0])
    sc = make_scene(w)
    d, i, t = render(sc, w)
    ref = oracle_render(w)
    assert_parity(d, i, t, ref, w["far"], label="single link + single triangle")


def test_far_plane_misses():
    say("[render] everything beyond the far plane")
    w = sg.small_plain_case()
    w["far"] = 0.5
    sc = make_scene(w)
    d, i, t = render(sc, w)
    assert np.all(i == -1) and np.all(t == -1) and np.all(d == np.float32(0.5))


def test_render_is_deterministic():
    say("[render] determinism")
    w = sg.robot_scene(2, 2, 4.0, 2, 64, 48, steps=1, label="det")
    sc = make_scene(w)
    a = render(sc, w)
    b = render(sc, w)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_packet_terrain_walk_gives_identical_results():
    say("[render] terrain walked per lane vs as a wavefront packet, 16 envs x 2 cams 64x48")
    w = sg.robot_scene(2, 4, 2.5, 2, 64, 48, steps=1, label="packet")
    sc = make_scene(w)
    lane = render(sc, w)
    sc.set_config(batched=False, terrain_packet=1)
    for rpl in (1, 2):
        sc.set_config(batched=False, rays_per_lane=rpl)
        got = render(sc, w)
        for g, r in zip(got, lane):
            assert np.array_equal(g, r)
    _, counts = sc.render_counts(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"],
                                 w["H"], w["far"], link_pos=dev(w["link_pos"][0]),
                                 link_quat=dev(w["link_quat"][0]))
    torch.cuda.synchronize()
    c = counts.cpu().numpy().reshape(-1, 4)
    say(f"  packet walk: mean nodes {c[:, 0].mean():.1f}, triangles {c[:, 1].mean():.2f}")
    assert np.all(c[lane[1].ravel() >= 0, 1] >= 1)


def test_render_counts_matches_render():
    say("[render] diagnostic work counts: same outputs as rc_render, plausible counts")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="counts")
    sc = make_scene(w)
    ref = render(sc, w)
    args = (dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"], w["far"])
    kw = dict(link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
    outs, counts = sc.render_counts(*args, **kw)
    torch.cuda.synchronize()
    for g, r in zip(outs, ref):
        assert np.array_equal(g.cpu().numpy(), r)
    c = counts.cpu().numpy().reshape(-1, 4)
    inst = ref[1].ravel()
    assert np.all(c[:, 3] <= c[:, 0]), "link node records are part of all node records"
    assert np.all(c[c[:, 2] == 0, 3] == 0), "no link nodes without an entered link"
    assert np.all(c[:, 0] >= 1), "every ray reads at least one node record"
    assert np.all(c[:, 2] <= sc.n_links), "a link is entered at most once per ray"
    assert np.all(c[inst >= 0, 1] >= 1), "a hit needs a triangle test"
    assert np.all(c[(inst >= 0) & (inst < sc.n_links), 2] >= 1), "a link hit needs its instance"
    _, again = sc.render_counts(*args, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy().reshape(-1, 4), c)
    m = rc()
    a, _, ws = sc._plain_args(*args, kw["link_pos"], kw["link_quat"], 0, None, True)
    st = m.lib().rc_render_counts(sc.handle, ctypes.byref(a), None, ctypes.c_void_p(ws.ptr),
                                  ws.nbytes, None)
    assert st == -1


def sampled(w, n, seed):
    total = w["E"] * w["C"] * w["H"] * w["W"]
    return np.sort(np.random.default_rng(seed).choice(total, size=n, replace=False))


def test_64_envs_sampled():
    say("[render] 64 envs x 2 cams 64x48, 10x10 tiles (~500k tris), 2048 sampled rays")
    w = sg.robots_64()
    sc = make_scene(w)
    for step in (0, 2):
        d, i, t = render(sc, w, step)
        rays = sampled(w, 2048, 100 + step)
        ref = oracle_render(w, step, rays=rays)
        assert_parity(d.ravel()[rays], i.ravel()[rays], t.ravel()[rays], ref, w["far"],
                      label=f"64 envs step {step}")


def test_4096_envs_sampled():
    """The bench's workload at full size (4096 envs x 2 cams 64x48 on the
    ~1.98M-triangle terrain, poses of steps 0, 50 and 99 of the 100-step
    sequence), 4096 sampled rays per step against the oracle."""
    say("[render] 4096 envs x 2 cams 64x48, 20x20 tiles (~2M tris), steps 0/50/99, 4096 rays each")
    w = sg.robots_4096(steps=100)
    sc = make_scene(w)
    for step in (0, 50, 99):
        d, i, t = render(sc, w, step)
        assert (i >= 0).mean() > 0.9
        rays = sampled(w, 4096, 200 + step)
        ref = oracle_render(w, step, rays=rays)
        assert_parity(d.ravel()[rays], i.ravel()[rays], t.ravel()[rays], ref, w["far"],
                      label=f"4096 envs step {step}")


# ---------------------------------------------------------------------------
# sensor model
# ---------------------------------------------------------------------------

def run_post(depth, inst, params_kw, s0=0, cam_uid=None, max_latency=3):
    m = rc()
    S, E, C, H, W = depth.shape
    post = m.Post(E, C, H, W, max_latency)
    p = m.post_params(**params_kw)
    uid = dev(cam_uid) if cam_uid is not None else None
    outs, drops, lats = [], [], []
    for s in range(S):
        o, dr, la = post.process(dev(depth[s]), dev(inst[s]), p, s0 + s, cam_uid=uid)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        drops.append(dr.cpu().numpy())
        lats.append(la.cpu().numpy())
    return np.stack(outs), np.stack(drops), np.stack(lats)


@pytest.mark.parametrize("s0,with_uid,hw", [(0, False, (29, 37)), (5, True, (29, 37)),
                                             (0, False, (24, 36)), (5, True, (24, 36))])
def test_post_matches_oracle(s0, with_uid, hw):
    """Odd image sizes take the one-pixel-per-thread form, sizes divisible by
    four the four-pixel form."""
    say(f"[post] 3 envs x 2 cams {hw[0]}x{hw[1]}, 9 steps from {s0}, uid table {with_uid}")
    depth, inst = sg.synthetic_frames(3, 2, hw[0], hw[1], 9)
    kw = dict(seed=0x1234_5678_9ABC, sigma_abs=0.01, sigma_rel=0.02, p_drop=0.02, near=0.05,
              far=3.0, fill=0.0, lat_min=1, lat_max=3)
    uid = (np.arange(6, dtype=np.uint32) * 7 + 100) if with_uid else None
    out, drop, lat = run_post(depth, inst, kw, s0=s0, cam_uid=uid)
    ro, rd, rl = oracle.post(depth, inst, oracle.make_params(**kw), s0=s0, cam_uid=uid)
    assert np.array_equal(lat, rl), "latency draws differ"
    assert np.array_equal(drop, rd), "dropout masks differ"
    assert np.max(np.abs(out - ro)) <= 1e-5


@pytest.mark.parametrize("hw", [(29, 37), (24, 36)])
def test_post_raw_draws_bit_exact(hw):
    """The raw Philox4x32-10 words of every pixel's draw (rc_postprocess_words,
    the same code that makes the outputs) equal the oracle's Philox at the
    documented counter (pixel, camera uid, step low 32 bits, step bits 32-47
    shifted up 16, stream 0 in the low bits) with key = seed, at steps above
    2^40; the outputs equal rc_postprocess's.  Odd sizes take the one-pixel
    form, sizes divisible by four the four-pixel form."""
    m = rc()
    H, W = hw
    say(f"[post] raw draws, 3 envs x 2 cams {H}x{W}")
    depth, inst = sg.synthetic_frames(3, 2, H, W, 3)
    kw = dict(seed=0x1234_5678_9ABC, sigma_abs=0.01, sigma_rel=0.02, p_drop=0.02, near=0.05,
              far=3.0, fill=0.0, lat_min=1, lat_max=3)
    uid = np.arange(6, dtype=np.uint32) * 11 + 7
    s0 = (1 << 40) + (1 << 33) + 5
    a, b = m.Post(3, 2, H, W, 3), m.Post(3, 2, H, W, 3)
    p = m.post_params(**kw)
    key = np.array([kw["seed"] & 0xFFFFFFFF, kw["seed"] >> 32], np.uint32)
    for s in range(3):
        step = s0 + s
        o, dr, la, words = a.process_words(dev(depth[s]), dev(inst[s]), p, step, cam_uid=dev(uid))
        o2, dr2, la2 = b.process(dev(depth[s]), dev(inst[s]), p, step, cam_uid=dev(uid))
        torch.cuda.synchronize()
        assert torch.equal(o, o2) and torch.equal(dr, dr2) and torch.equal(la, la2)
        got = words.cpu().numpy().view(np.uint32).reshape(6, H * W, 4)
        hi = ((step >> 32) & 0xFFFF) << 16
        for ec in range(6):
            for pix in range(H * W):
                want = oracle.philox([pix, uid[ec], step & 0xFFFFFFFF, hi], key)
                assert np.array_equal(got[ec, pix], want), (s, ec, pix)


def test_post_reset_starts_a_new_sequence():
    """After rc_post_reset the next step starts a new sequence: frames captured
    before the reset are never shown (the oracle started at that step)."""
    say("[post] reset between two sequences")
    m = rc()
    depth, inst = sg.synthetic_frames(2, 2, 12, 16, 8)
    kw = dict(seed=99, sigma_abs=0.01, p_drop=0.05, near=0.05, far=3.0, lat_min=1, lat_max=3)
    post = m.Post(2, 2, 12, 16, 3)
    p = m.post_params(**kw)
    for s in range(4):  # first sequence, steps 0..3
        post.process(dev(depth[s]), dev(inst[s]), p, s)
    post.reset()
    outs, drops = [], []
    for k, s in enumerate(range(20, 24)):  # new sequence from step 20, frames 4..7
        o, dr, _ = post.process(dev(depth[4 + k]), dev(inst[4 + k]), p, s)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        drops.append(dr.cpu().numpy())
    ro, rd, _ = oracle.post(depth[4:], inst[4:], oracle.make_params(**kw), s0=20)
    assert np.array_equal(np.stack(drops), rd)
    assert np.max(np.abs(np.stack(outs) - ro)) <= 1e-5


def test_post_identity_and_errors():
    say("[post] everything off; out-of-order step")
    depth, inst = sg.synthetic_frames(2, 1, 8, 8, 2)
    out, drop, lat = run_post(depth, inst, dict(seed=1, near=0.05, far=3.0))
    near, far = np.float32(0.05), np.float32(3.0)
    expect = np.where(inst >= 0, np.clip(depth, near, far), far)
    assert np.array_equal(out, expect) and not drop.any() and not lat.any()
    m = rc()
    post = m.Post(2, 1, 8, 8, 3)
    p = m.post_params(seed=1)
    post.process(dev(depth[0]), dev(inst[0]), p, 10)
    with pytest.raises(m.RcError):
        post.process(dev(depth[1]), dev(inst[1]), p, 12)


def test_render_then_post_end_to_end():
    say("[render+post] 4 envs x 2 cams 32x24, 4 steps")
    w = sg.robot_scene(2, 2, 4.0, 2, 32, 24, steps=4, label="e2e")
    sc = make_scene(w)
    m = rc()
    kw = dict(seed=77, sigma_abs=0.01, p_drop=0.02, near=0.05, far=3.0, lat_min=1, lat_max=3)
    post = m.Post(w["E"], w["C"], w["H"], w["W"], 3)
    p = m.post_params(**kw)
    frames_d, frames_i, outs, refs = [], [], [], []
    for s in range(4):
        lp, lq = dev(w["link_pos"][s]), dev(w["link_quat"][s])
        d, i, _ = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                            w["far"], link_pos=lp, link_quat=lq)
        o, _, _ = post.process(d, i, p, s)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        ref = oracle_render(w, s)
        refs.append(ref)
        frames_d.append(ref["depth"].astype(np.float32).reshape(w["E"], w["C"], w["H"], w["W"]))
        frames_i.append(ref["inst"].reshape(w["E"], w["C"], w["H"], w["W"]))
    ro, _, rl = oracle.post(np.stack(frames_d), np.stack(frames_i), oracle.make_params(**kw))
    # compare pixels whose shown capture comes from an unflagged oracle ray
    for s in range(4):
        for ec in range(w["E"] * w["C"]):
            k = int(rl[s].ravel()[ec])
            src = max(s - k, 0)
            fl = refs[src]["flags"].reshape(w["E"] * w["C"], -1)[ec]
            ok = fl == 0
            a = outs[s].reshape(w["E"] * w["C"], -1)[ec][ok]
            b = ro[s].reshape(w["E"] * w["C"], -1)[ec][ok]
            assert np.max(np.abs(a - b)) <= 1e-4


def look_quat(direction):
    from scipy.spatial.transform import Rotation
    z = np.asarray(direction, float)
    z = z / np.linalg.norm(z)
    up = np.array([0.0, 0.0, 1.0]) if abs(z[2]) < 0.99 else np.array([1.0, 0.0, 0.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    return Rotation.from_matrix(np.stack([x, np.cross(z, x), z], 1)).as_quat()


def watertight_scene(as_link, repeat=1):
    """Rays aimed exactly at every vertex and edge midpoint of a closed convex
    mesh (one 1x1 camera per ray), the set repeated `repeat` times."""
    V, T = sg.octasphere(3)
    mesh = (V[T] * 0.3).astype(np.float32)
    centre = np.array([5.0, -3.0, 1.5])
    pts = {tuple(v) for v in mesh.reshape(-1, 3).astype(np.float64)}
    for t in mesh.astype(np.float64):
        for i in range(3):
            pts.add(tuple(0.5 * (t[i] + t[(i + 1) % 3])))
    pts = np.tile(np.array(sorted(pts)), (repeat, 1))
    E = pts.shape[0]
    dirs = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    cam_pos = (centre + 2.0 * dirs)[:, None, :].astype(np.float32)
    cam_quat = np.array([[look_quat(-p)] for p in dirs], np.float32)
    intr = np.tile(np.float32([1, 1, 0.5, 0.5]), (E, 1, 1))
    far_tri = np.array([[[50, 50, 50], [51, 50, 50], [50, 51, 50]]], np.float32)
    if as_link:
        w = dict(terrain=far_tri, link_tri=mesh, link_off=np.array([0, mesh.shape[0]], np.int64),
                 link_pos=np.tile(centre.astype(np.float32), (1, E, 1, 1)),
                 link_quat=np.tile(np.float32([0, 0, 0, 1]), (1, E, 1, 1)))
    else:
        w = dict(terrain=(mesh + centre).astype(np.float32), link_tri=np.zeros((0, 3, 3), np.float32),
                 link_off=np.zeros(1, np.int64), link_pos=np.zeros((1, E, 0, 3), np.float32),
                 link_quat=np.zeros((1, E, 0, 4), np.float32))
    w.update(E=E, C=1, W=1, H=1, cam_pos=cam_pos, cam_quat=cam_quat, intr=intr, far=10.0)
    return w


@pytest.mark.parametrize("as_link", [False, True])
def test_watertight_vertices_and_edges(as_link):
    """Decisions FP32 cannot make: the exact pass must take them (edge rays by
    deciding the two undecided triangles, vertex rays by a full re-cast)."""
    say(f"[render] watertight vertex/edge rays, mesh as {'link' if as_link else 'terrain'}")
    w = watertight_scene(as_link)
    sc = make_scene(w)
    d, i, t = render(sc, w)
    n_exact, n_full = sc.exact_count(w["E"], 1, 1, 1, recast=True)
    say(f"  {w['E']} rays, {n_exact} sent to the exact pass, {n_full} of them re-cast in full")
    assert np.all(i.ravel() == 0), "a ray slipped through an edge or vertex"
    ref = oracle_render(w)
    assert_parity(d, i, t, ref, w["far"], label="watertight")
    assert n_exact > 0


def test_grid_edge_rays_decided_by_listed_triangles():
    """Rays through edge midpoints of a flat triangulated grid leave two
    FP32-undecided triangles, which the exact pass decides without a re-cast;
    rays through vertices leave more and are re-cast in full."""
    say("[render] grid edge-midpoint and vertex rays")
    n, h = 12, 0.25
    xs = np.arange(n + 1) * h
    V = np.array([[x, y, 0.0] for y in xs for x in xs])
    idx = lambda i, j: j * (n + 1) + i
    T = []
    for j in range(n):
        for i in range(n):
            T.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)])
            T.append([idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)])
    tri = V[np.array(T)].astype(np.float32)
    pts = set()
    for t in tri.astype(np.float64):
        for i in range(3):
            m = 0.5 * (t[i] + t[(i + 1) % 3])
            if 0 < m[0] < n * h and 0 < m[1] < n * h:
                pts.add(("e",) + tuple(m))
        for v in t:
            if 0 < v[0] < n * h and 0 < v[1] < n * h:
                pts.add(("v",) + tuple(v))
    pts = sorted(pts)
    kind = np.array([p[0] for p in pts])
    P = np.array([p[1:] for p in pts])
    E = P.shape[0]
    rng = np.random.default_rng(11)
    off = np.stack([rng.uniform(-0.4, 0.4, E), rng.uniform(-0.4, 0.4, E), np.full(E, 1.0)], 1)
    cam_pos = (P + off)[:, None, :].astype(np.float32)
    cam_quat = np.array([[look_quat(-o)] for o in off], np.float32)
    intr = np.tile(np.float32([1, 1, 0.5, 0.5]), (E, 1, 1))
    w = dict(terrain=tri, link_tri=np.zeros((0, 3, 3), np.float32), link_off=np.zeros(1, np.int64),
             link_pos=np.zeros((1, E, 0, 3), np.float32), link_quat=np.zeros((1, E, 0, 4), np.float32),
             E=E, C=1, W=1, H=1, cam_pos=cam_pos, cam_quat=cam_quat, intr=intr, far=10.0)
    sc = make_scene(w)
    d, i, t = render(sc, w)
    n_exact, n_full = sc.exact_count(E, 1, 1, 1, recast=True)
    say(f"  {E} rays ({int((kind == 'e').sum())} edge, {int((kind == 'v').sum())} vertex), "
        f"{n_exact} sent to the exact pass, {n_full} re-cast in full")
    assert np.all(i.ravel() == 0), "a ray slipped through the grid"
    assert_parity(d, i, t, oracle_render(w), w["far"], label="grid edges")
    assert n_full > 0 and n_exact - n_full > 0


@pytest.mark.parametrize("cap", [1, 3])
def test_walk_stack_cap_sends_rays_to_the_full_recast(cap):
    """The fast pass's 4-wide terrain walk with its stack capped at `cap`
    entries: a ray whose push is dropped is re-cast in full by the exact pass,
    so the ids stay bit-identical to the uncapped render and the depths agree
    (to the FP32 rounding of an FP64 depth) and meet the oracle's bar."""
    say(f"[render] 4 envs x 2 cams 37x29, walk stack capped at {cap}")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="parity-ragged")
    sc = make_scene(w)
    E, C, W, H = w["E"], w["C"], w["W"], w["H"]
    d0, i0, t0 = render(sc, w)
    _, full0 = sc.exact_count(E, C, W, H, recast=True)
    sc.set_walk_stack_limit(cap)
    try:
        d1, i1, t1 = render(sc, w)
        _, full1 = sc.exact_count(E, C, W, H, recast=True)
    finally:
        sc.set_walk_stack_limit(16)
    say(f"  full re-casts: {full0} uncapped, {full1} capped")
    assert full1 > full0 + 100
    assert np.array_equal(i0, i1) and np.array_equal(t0, t1)
    assert np.max(np.abs(d0 - d1)) <= 2e-5
    assert_parity(d1, i1, t1, oracle_render(w), w["far"], label=f"stack cap {cap}")
    for bad in (0, 17):
        with pytest.raises(RuntimeError):
            sc.set_walk_stack_limit(bad)


def test_exact_list_overflow_recasts_everything():
    """More listed rays than the exact pass's list holds (4096 entries here):
    every pixel is re-cast, with the same results."""
    say("[render] exact-pass list overflow")
    w = watertight_scene(False, repeat=5)
    sc = make_scene(w)
    d, i, t = render(sc, w)
    n_exact = sc.exact_count(w["E"], 1, 1, 1)
    say(f"  {w['E']} rays, {n_exact} listed")
    assert n_exact > 4096
    assert np.all(i.ravel() == 0)
    ref = oracle_render(w)
    assert_parity(d, i, t, ref, w["far"], label="overflow")
