"""GPU: perception randomisation of the cameras (the paper's Table 6) drawn on
the device, against the oracle's randomisation of the same cameras."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from parity import assert_parity

pytestmark = pytest.mark.gpu

DEV = "cuda"
TABLE6 = dict(trans_m=(0.025, 0.025, 0.025), euler_deg=(2.5, 3.0, 2.5), dfov_deg=2.0)


def rc():
    import paper_2602_03002_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def scene(w):
    sc = rc().Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    return sc


def render(sc, w, rand=None):
    d, i, t = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                        w["far"], link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]),
                        rand=rand)
    torch.cuda.synchronize()
    return d.cpu().numpy(), i.cpu().numpy(), t.cpu().numpy()


def test_zero_ranges_change_nothing():
    say("[camrand] zero ranges: bit-identical to no randomisation")
    w = sg.robot_scene(2, 2, 4.0, 2, 37, 29, steps=1, label="camrand0")
    sc = scene(w)
    base = render(sc, w)
    got = render(sc, w, rc().cam_rand(seed=5, epoch=1, trans_m=(0, 0, 0), euler_deg=(0, 0, 0),
                                      dfov_deg=0.0))
    for g, b in zip(got, base):
        assert np.array_equal(g, b)


@pytest.mark.parametrize("epoch", [0, 3])
def test_table6_ranges_match_oracle(epoch):
    say(f"[camrand] 64 envs x 2 cams 64x48, Table 6 ranges, epoch {epoch}, 2048 sampled rays")
    w = sg.robots_64()
    sc = scene(w)
    r = rc().cam_rand(seed=0x2602, epoch=epoch, **TABLE6)
    d, i, t = render(sc, w, r)
    cam64 = oracle.cam_randomize(w["cam_pos"], w["cam_quat"], w["intr"],
                                 np.arange(w["E"] * w["C"]), 0x2602, epoch, **TABLE6)
    rays = np.sort(np.random.default_rng(epoch).choice(d.size, size=2048, replace=False))
    ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                        w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"], w["W"], w["H"],
                        w["far"], rays=rays, cam64=cam64)
    assert_parity(d.ravel()[rays], i.ravel()[rays], t.ravel()[rays], ref, w["far"],
                  label=f"camrand epoch {epoch}")
    base = render(sc, w)
    assert not np.array_equal(d, base[0]), "randomisation changed nothing"
    again = render(sc, w, r)
    assert np.array_equal(again[0], d)


def test_batched_randomisation_uses_descriptor_uids():
    say("[camrand] batched uneven cameras with randomisation vs oracle")
    w = sg.robot_scene(2, 3, 3.0, 4, 16, 12, steps=1, label="camrandb")
    desc, n_pix = sg.uneven_cameras(w, label="camrandb")
    sc = scene(w)
    r = rc().cam_rand(seed=77, epoch=2, **TABLE6)
    b = sc.batch(dev(desc.view(np.uint8)), n_pix, 106, 60, w["far"], link_pos=dev(w["link_pos"][0]),
                 link_quat=dev(w["link_quat"][0]), rand=r)
    d, i, t = (x.cpu().numpy() for x in b.render())
    torch.cuda.synchronize()
    for k in range(min(6, len(desc))):
        D = desc[k]
        e, W, H, o = int(D["env"]), int(D["width"]), int(D["height"]), int(D["out_offset"])
        cam64 = oracle.cam_randomize(D["pos"][None], D["quat"][None], D["intr"][None],
                                     [int(D["cam_uid"])], 77, 2, **TABLE6)
        ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0][e:e + 1],
                            w["link_quat"][0][e:e + 1], D["pos"].reshape(1, 1, 3),
                            D["quat"].reshape(1, 1, 4), D["intr"].reshape(1, 1, 4), W, H, w["far"],
                            cam64=cam64)
        assert_parity(d[o:o + W * H], i[o:o + W * H], t[o:o + W * H], ref, w["far"],
                      label=f"batched camrand camera {k}")


def test_bad_ranges_rejected():
    m = rc()
    w = sg.robot_scene(1, 1, 4.0, 1, 8, 8, steps=1, label="camrandbad")
    sc = scene(w)
    with pytest.raises(m.RcError):
        render(sc, w, m.cam_rand(trans_m=(-1.0, 0, 0)))
    with pytest.raises(m.RcError):
        render(sc, w, m.cam_rand(dfov_deg=95.0))
