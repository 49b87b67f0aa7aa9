"""rc_render_noalloc (no workspace argument, no allocation) against rc_render
on the same inputs: two calls in a row on the library's static scratch, the
second smaller, each bit-identical to rc_render, plus the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_noalloc_matches_render_twice_second_smaller():
    import paper_2602_03002_amd as m
    print("[noalloc] 64 envs x 2 cams 64x48, then 4 envs x 1 cam 37x29", flush=True)
    big = sg.robot_scene(2, 8, 2.5, 2, 64, 48, steps=1, label="noalloc-big")
    small = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="noalloc-small",
                           terrain=big["terrain_obj"], robot=big["robot"])
    sc = m.Scene(dev(big["terrain"]))
    sc.set_robot(dev(big["link_tri"]), big["link_off"].tolist())
    for w, C in ((big, 2), (small, 1)):
        args = (dev(w["cam_pos"][:, :C]), dev(w["cam_quat"][:, :C]), dev(w["intr"][:, :C]), w["W"],
                w["H"], w["far"])
        kw = dict(link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
        ref = sc.render(*args, **kw)
        E = w["E"]
        out = (torch.full((E, C, w["H"], w["W"]), -7.0, device="cuda"),
               torch.full((E, C, w["H"], w["W"]), -7, dtype=torch.int32, device="cuda"),
               torch.full((E, C, w["H"], w["W"]), -7, dtype=torch.int32, device="cuda"))
        got = sc.render_noalloc(*args, **kw, out=out)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert torch.equal(g, r)
        assert (ref[1] >= 0).float().mean().item() > 0.5
        print(f"[noalloc] {E} envs x {C} cams {w['W']}x{w['H']}: identical", flush=True)


def test_noalloc_rejects_renders_beyond_its_scratch():
    import paper_2602_03002_amd as m
    w = sg.robot_scene(1, 1, 4.0, 1, 16, 12, steps=1, label="noalloc-limit")
    sc = m.Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    E = 16384  # 16,384 top levels of 30 links need about 62 MB
    cam = dev(np.broadcast_to(w["cam_pos"], (E, 1, 3)))
    q = dev(np.broadcast_to(w["cam_quat"], (E, 1, 4)))
    K = dev(np.broadcast_to(w["intr"], (E, 1, 4)))
    lp = dev(np.broadcast_to(w["link_pos"][0], (E, 30, 3)))
    lq = dev(np.broadcast_to(w["link_quat"][0], (E, 30, 4)))
    depth = torch.full((E, 1, 12, 16), 5.0, device="cuda")
    with pytest.raises(m.RcError) as ei:
        sc.render_noalloc(cam, q, K, 16, 12, w["far"], link_pos=lp, link_quat=lq,
                          out=(depth, None, None), ids=False)
    assert ei.value.status == -2 and b"static scratch" in m.lib().rc_last_error()
    torch.cuda.synchronize()
    assert torch.all(depth == 5.0)  # nothing was enqueued
