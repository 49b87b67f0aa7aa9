"""GPU: batched uneven form (descriptor table, schedules, graph replay,
autotuner) against the plain per-camera path and the oracle; packed sensor model."""
import numpy as np
import pytest
import torch

import oracle
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


def uneven_scene(tiles=2, side=3, steps=3, label="b"):
    w = sg.robot_scene(tiles, side, 3.0, 4, 16, 12, steps=steps, label=label)
    desc, n_pix = sg.uneven_cameras(w, label=label)
    return w, desc, n_pix


def make_scene(w):
    sc = rc().Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    return sc


def batch_of(sc, w, desc, n_pix, step=0, lp=None, lq=None):
    lp = dev(w["link_pos"][step]) if lp is None else lp
    lq = dev(w["link_quat"][step]) if lq is None else lq
    d = dev(desc.view(np.uint8))
    return sc.batch(d, n_pix, 106, 60, w["far"], link_pos=lp, link_quat=lq)


def plain_per_camera(sc, w, desc, n_pix, step=0):
    """Each camera through rc_render as its own one-env, one-camera launch."""
    depth = np.zeros(n_pix, np.float32)
    inst = np.zeros(n_pix, np.int32)
    tri = np.zeros(n_pix, np.int32)
    for d in desc:
        e = int(d["env"])
        W, H, o = int(d["width"]), int(d["height"]), int(d["out_offset"])
        r = sc.render(dev(d["pos"].reshape(1, 1, 3)), dev(d["quat"].reshape(1, 1, 4)),
                      dev(d["intr"].reshape(1, 1, 4)), W, H, w["far"],
                      link_pos=dev(w["link_pos"][step][e:e + 1]), link_quat=dev(w["link_quat"][step][e:e + 1]))
        torch.cuda.synchronize()
        depth[o:o + W * H] = r[0].cpu().numpy().ravel()
        inst[o:o + W * H] = r[1].cpu().numpy().ravel()
        tri[o:o + W * H] = r[2].cpu().numpy().ravel()
    return depth, inst, tri


def host(outs):
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in outs)


def test_batched_equals_plain_per_camera_and_oracle():
    say("[batched] 9 envs, 1-4 cameras of mixed sizes vs plain per camera and oracle")
    w, desc, n_pix = uneven_scene()
    sc = make_scene(w)
    b = batch_of(sc, w, desc, n_pix)
    got = host(b.render())
    status, n_exact = b.status()
    assert status == 0
    ref = plain_per_camera(sc, w, desc, n_pix)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r), "batched and plain per-camera results differ"
    # oracle on a sample of pixels of every camera
    rng = np.random.default_rng(5)
    for d in desc[:6]:
        e, W, H, o = int(d["env"]), int(d["width"]), int(d["height"]), int(d["out_offset"])
        rays = np.sort(rng.choice(W * H, size=min(200, W * H), replace=False))
        oref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0][e:e + 1],
                             w["link_quat"][0][e:e + 1], d["pos"].reshape(1, 1, 3),
                             d["quat"].reshape(1, 1, 4), d["intr"].reshape(1, 1, 4), W, H, w["far"],
                             rays=rays)
        assert_parity(got[0][o + rays], got[1][o + rays], got[2][o + rays], oref, w["far"],
                      label=f"batched camera {W}x{H}")


@pytest.mark.parametrize("cfg", [
    dict(tile_w=8, tile_h=8, rays_per_lane=1, waves=6, persistent=1, terrain_packet=0, bodies_flat=0),
    dict(tile_w=16, tile_h=4, rays_per_lane=2, waves=7, persistent=1, terrain_packet=1, bodies_flat=1),
    dict(tile_w=4, tile_h=16, rays_per_lane=1, waves=8, persistent=0, terrain_packet=0, bodies_flat=1),
    dict(tile_w=32, tile_h=2, rays_per_lane=2, waves=6, persistent=0, terrain_packet=1, bodies_flat=0),
    dict(tile_w=8, tile_h=8, rays_per_lane=1, waves=6, persistent=0, terrain_packet=1, bodies_flat=1),
    dict(tile_w=8, tile_h=8, rays_per_lane=1, waves=7, persistent=0, terrain_packet=0, bodies_flat=1),
])
def test_every_schedule_gives_identical_results(cfg):
    say(f"[batched] schedule {cfg}")
    w, desc, n_pix = uneven_scene(label="sched")
    sc = make_scene(w)
    base = host(batch_of(sc, w, desc, n_pix).render())
    sc.set_config(batched=True, **cfg)
    got = host(batch_of(sc, w, desc, n_pix).render())
    for g, r in zip(got, base):
        assert np.array_equal(g, r)
    # the plain path under the same tile schedule
    plain = dict(cfg)
    plain.pop("persistent")
    sc.set_config(batched=False, **plain)
    r = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"], w["far"],
                  link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
    sc.set_config(batched=False, tile_w=8, tile_h=8, rays_per_lane=1, waves=6, terrain_packet=0,
                  bodies_flat=0)
    r0 = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"], w["far"],
                   link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
    for g, h in zip(host(r), host(r0)):
        assert np.array_equal(g, h)


def test_invalid_descriptor_is_skipped_and_reported():
    say("[batched] an out-of-range descriptor")
    w, desc, n_pix = uneven_scene(label="bad")
    sc = make_scene(w)
    good = host(batch_of(sc, w, desc, n_pix).render())
    bad = desc.copy()
    bad[1]["env"] = 999
    b = batch_of(sc, w, bad, n_pix)
    b.outs[0].fill_(-7.0)
    got = host(b.render())
    status, _ = b.status()
    assert status & 1
    o, np1 = int(bad[1]["out_offset"]), int(bad[1]["width"] * bad[1]["height"])
    assert np.all(got[0][o:o + np1] == -7.0)
    mask = np.ones(n_pix, bool)
    mask[o:o + np1] = False
    assert np.array_equal(got[0][mask], good[0][mask])


def test_graph_replay_tracks_pose_updates():
    say("[batched] graph capture and replay with in-place pose updates")
    w, desc, n_pix = uneven_scene(steps=3, label="graph")
    sc = make_scene(w)
    lp = dev(w["link_pos"][0]).clone()
    lq = dev(w["link_quat"][0]).clone()
    b = batch_of(sc, w, desc, n_pix, lp=lp, lq=lq)
    g = b.capture()
    for step in (1, 2, 0, 1):
        lp.copy_(dev(w["link_pos"][step]))
        lq.copy_(dev(w["link_quat"][step]))
        replay = host(g.launch())
        replay = tuple(x.copy() for x in replay)
        eager = host(batch_of(sc, w, desc, n_pix, step=step).render())
        for x, y in zip(replay, eager):
            assert np.array_equal(x, y), f"replay differs from eager at step {step}"
    g.close()


def test_autotune_keeps_results():
    say("[autotune] plain and batched")
    w, desc, n_pix = uneven_scene(label="tune")
    sc = make_scene(w)
    b = batch_of(sc, w, desc, n_pix)
    before = host(b.render())
    cfg, ms = sc.autotune(reps=1, batch=b)
    assert ms > 0 and cfg["tile_w"] * cfg["tile_h"] == 64
    assert sc.config(batched=True) == cfg
    after = host(b.render())
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    kw = dict(cam_pos=dev(w["cam_pos"]), cam_quat=dev(w["cam_quat"]), intr=dev(w["intr"]),
              width=w["W"], height=w["H"], far_plane=w["far"], link_pos=dev(w["link_pos"][0]),
              link_quat=dev(w["link_quat"][0]))
    cfg2, ms2 = sc.autotune(reps=1, **kw)
    assert ms2 > 0 and cfg2["persistent"] == 0


def test_packed_post_matches_oracle():
    say("[post] packed batch vs oracle per camera")
    rng = np.random.default_rng(3)
    w, desc, n_pix = uneven_scene(label="post")
    S = 5
    depth = rng.uniform(0, 3.4, (S, n_pix)).astype(np.float32)
    inst = rng.integers(-1, 31, (S, n_pix)).astype(np.int32)
    m = rc()
    kw = dict(seed=99, sigma_abs=0.01, sigma_rel=0.01, p_drop=0.05, near=0.05, far=3.0,
              lat_min=1, lat_max=3)
    post = m.Post.packed(n_pix, 3)
    p = m.post_params(**kw)
    d_dev = dev(desc.view(np.uint8))
    outs, drops, lats = [], [], []
    for s in range(S):
        o, dr, la = post.process_batched(dev(depth[s]), dev(inst[s]), p, s, d_dev)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        drops.append(dr.cpu().numpy())
        lats.append(la.cpu().numpy())
    op = oracle.make_params(**kw)
    for k, d in enumerate(desc):
        W, H, o = int(d["width"]), int(d["height"]), int(d["out_offset"])
        fr = depth[:, o:o + W * H].reshape(S, 1, 1, H, W)
        fi = inst[:, o:o + W * H].reshape(S, 1, 1, H, W)
        ro, rd, rl = oracle.post(fr, fi, op, cam_uid=np.array([d["cam_uid"]], np.uint32))
        for s in range(S):
            assert lats[s][k] == rl[s, 0, 0]
            assert np.array_equal(drops[s][o:o + W * H], rd[s].ravel())
            assert np.max(np.abs(outs[s][o:o + W * H] - ro[s].ravel())) <= 1e-5


def test_batched_4096_uneven_sampled():
    """The measured uneven workload at its full size (4096 envs, 1-4 cameras of
    mixed sizes, ~39M rays), autotuned and replayed from a captured graph as the
    bench runs it: sampled pixels of 48 cameras against the oracle, and two
    whole cameras against rc_render of that camera alone."""
    say("[batched] 4096 envs uneven, graph replay, sampled against the oracle")
    w, desc, n_pix = sg.uneven_4096(steps=1)
    sc = make_scene(w)
    lp, lq = dev(w["link_pos"][0]), dev(w["link_quat"][0])
    b = batch_of(sc, w, desc, n_pix, lp=lp, lq=lq)
    sc.autotune(reps=1, batch=b)
    g = b.capture()
    g.launch()
    g.launch()  # a second replay: results must not depend on leftover state
    got = host(b.outs)
    status, _ = b.status()
    assert status == 0
    rng = np.random.default_rng(11)
    for k in rng.choice(len(desc), 48, replace=False):
        d = desc[k]
        e, W, H, o = int(d["env"]), int(d["width"]), int(d["height"]), int(d["out_offset"])
        rays = np.sort(rng.choice(W * H, size=12, replace=False))
        oref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0][e:e + 1],
                             w["link_quat"][0][e:e + 1], d["pos"].reshape(1, 1, 3),
                             d["quat"].reshape(1, 1, 4), d["intr"].reshape(1, 1, 4), W, H, w["far"],
                             rays=rays)
        assert_parity(got[0][o + rays], got[1][o + rays], got[2][o + rays], oref, w["far"],
                      label=f"4096-env batch, camera {k} {W}x{H}")
    for k in (0, len(desc) - 1):
        d = desc[k]
        e, W, H, o = int(d["env"]), int(d["width"]), int(d["height"]), int(d["out_offset"])
        r = sc.render(dev(d["pos"].reshape(1, 1, 3)), dev(d["quat"].reshape(1, 1, 4)),
                      dev(d["intr"].reshape(1, 1, 4)), W, H, w["far"], link_pos=lp[e:e + 1],
                      link_quat=lq[e:e + 1])
        for x, y in zip(host(r), got):
            assert np.array_equal(x.ravel(), y[o:o + W * H])


def test_batched_range_depth():
    """Range depth (distance along the ray) in the batched form: equal to each
    camera rendered alone in range mode, and to the oracle's range depth."""
    say("[batched] range depth")
    w, desc, n_pix = uneven_scene(label="range")
    sc = make_scene(w)
    d = dev(desc.view(np.uint8))
    b = sc.batch(d, n_pix, 106, 60, w["far"], link_pos=dev(w["link_pos"][0]),
                 link_quat=dev(w["link_quat"][0]), depth_mode=1)
    got = host(b.render())
    rng = np.random.default_rng(8)
    for k in (0, len(desc) // 2, len(desc) - 1):
        dk = desc[k]
        e, W, H, o = int(dk["env"]), int(dk["width"]), int(dk["height"]), int(dk["out_offset"])
        r = sc.render(dev(dk["pos"].reshape(1, 1, 3)), dev(dk["quat"].reshape(1, 1, 4)),
                      dev(dk["intr"].reshape(1, 1, 4)), W, H, w["far"],
                      link_pos=dev(w["link_pos"][0][e:e + 1]), link_quat=dev(w["link_quat"][0][e:e + 1]),
                      depth_mode=1)
        for x, y in zip(host(r), got):
            assert np.array_equal(x.ravel(), y[o:o + W * H])
        rays = np.sort(rng.choice(W * H, size=min(150, W * H), replace=False))
        oref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0][e:e + 1],
                             w["link_quat"][0][e:e + 1], dk["pos"].reshape(1, 1, 3),
                             dk["quat"].reshape(1, 1, 4), dk["intr"].reshape(1, 1, 4), W, H, w["far"],
                             depth_mode=1, rays=rays)
        assert_parity(got[0][o + rays], got[1][o + rays], got[2][o + rays], oref, w["far"],
                      label=f"batched range camera {k}")


def test_batched_terrain_only_scene():
    """A scene without robot links (terrain only): cameras of different sizes
    in one batched launch equal each camera rendered alone, and the oracle."""
    say("[batched] terrain-only scene")
    w = sg.small_plain_case()
    sc = rc().Scene(dev(w["terrain"]))
    rows, off = [], 0
    for k, (W, H) in enumerate(((32, 24), (17, 13), (64, 48))):
        K = sg.intrinsics_from_fov(W, H, 87.0, 58.0)
        rows.append((0, W, H, off, k, w["cam_pos"][0, 0], w["cam_quat"][0, 0], K))
        off += W * H
    desc = np.array(rows, dtype=sg.CAM_DESC)
    b = sc.batch(dev(desc.view(np.uint8)), off, 64, 48, w["far"])
    got = host(b.render())
    assert b.status()[0] == 0
    none3 = np.zeros((0, 3, 3), np.float32)
    for dk in desc:
        W, H, o = int(dk["width"]), int(dk["height"]), int(dk["out_offset"])
        r = sc.render(dev(dk["pos"].reshape(1, 1, 3)), dev(dk["quat"].reshape(1, 1, 4)),
                      dev(dk["intr"].reshape(1, 1, 4)), W, H, w["far"])
        for x, y in zip(host(r), got):
            assert np.array_equal(x.ravel(), y[o:o + W * H])
        oref = oracle.render(w["terrain"], none3, np.zeros(1, np.int64), np.zeros((1, 0, 3), np.float32),
                             np.zeros((1, 0, 4), np.float32), dk["pos"].reshape(1, 1, 3),
                             dk["quat"].reshape(1, 1, 4), dk["intr"].reshape(1, 1, 4), W, H, w["far"])
        assert_parity(got[0][o:o + W * H], got[1][o:o + W * H], got[2][o:o + W * H], oref, w["far"],
                      label=f"terrain-only batched {W}x{H}")
