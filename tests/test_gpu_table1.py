"""GPU: the paper's perception setting (Sec. 4.1) - 1024 envs x 1-4 cameras x
240x135 at 101 x 69 degrees - against the oracle on sampled rays, and the
block pooling to 48x27 against the oracle's pooling."""
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


@pytest.mark.parametrize("shape,f", [((3, 135, 240), 5), ((2, 2, 37, 29), 4), ((1, 6, 6), 6),
                                     ((4, 5, 7), 1)])
def test_downsample_matches_oracle(shape, f):
    say(f"[downsample] {shape} by {f}")
    rng = np.random.default_rng(sum(shape) + f)
    depth = rng.uniform(0.05, 3.0, shape).astype(np.float32)
    inst = rng.integers(-1, 31, shape).astype(np.int32)
    inst[..., :f, :f] = -1  # a block with no hit
    got = rc().downsample(dev(depth), dev(inst), f, 3.0)
    torch.cuda.synchronize()
    ref = oracle.downsample(depth, inst, f, 3.0)
    g = got.cpu().numpy()
    assert g.shape == ref.shape
    assert np.max(np.abs(g - ref)) <= 1e-5
    assert np.all(g[..., 0, 0] == 3.0)


def test_downsample_rejects_bad_sizes():
    m = rc()
    d = torch.zeros((1, 4, 4), device=DEV)
    with pytest.raises(m.RcError):
        m.downsample(d, None, 5, 3.0)
    with pytest.raises(m.RcError):
        m.downsample(d, None, 0, 3.0)


@pytest.mark.parametrize("n_cam", [1, 4])
def test_table1_sampled_and_pooled(n_cam):
    say(f"[table1] 1024 envs x {n_cam} cams x 240x135, 101x69 degrees, 512 sampled rays + pooling")
    w = sg.table1(n_cam, steps=1)
    m = rc()
    sc = m.Scene(dev(w["terrain"]))
    sc.set_robot(dev(w["link_tri"]), w["link_off"].tolist())
    d, i, t = sc.render(dev(w["cam_pos"]), dev(w["cam_quat"]), dev(w["intr"]), w["W"], w["H"],
                        w["far"], link_pos=dev(w["link_pos"][0]), link_quat=dev(w["link_quat"][0]))
    pooled = m.downsample(d, i, sg.TABLE1_POOL, w["far"])
    torch.cuda.synchronize()
    dn, inn, tn = d.cpu().numpy(), i.cpu().numpy(), t.cpu().numpy()
    assert pooled.shape == (w["E"], n_cam, 27, 48)
    total = dn.size
    rays = np.sort(np.random.default_rng(7 + n_cam).choice(total, size=512, replace=False))
    ref = oracle.render(w["terrain"], w["link_tri"], w["link_off"], w["link_pos"][0],
                        w["link_quat"][0], w["cam_pos"], w["cam_quat"], w["intr"], w["W"], w["H"],
                        w["far"], rays=rays)
    assert_parity(dn.ravel()[rays], inn.ravel()[rays], tn.ravel()[rays], ref, w["far"],
                  label=f"table1 {n_cam} cams")
    # pooling of the rendered frames against the oracle's pooling of the same frames
    sel = np.random.default_rng(n_cam).choice(w["E"], size=16, replace=False)
    ref_pool = oracle.downsample(dn[sel], inn[sel], sg.TABLE1_POOL, w["far"])
    assert np.max(np.abs(pooled.cpu().numpy()[sel] - ref_pool)) <= 1e-5
