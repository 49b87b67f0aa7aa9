"""Write the reference visit counts behind the roofline's algorithmic bytes.

MEASUREMENT AID (test/bench infrastructure).  Runs oracle/refcount.c (a CPU
binned-SAH BVH2 with ordered closest-first traversal) over a seeded sample of
65,536 pixel rays of step 0 of the 4096-env x 2-camera x 64x48 workload and
stores the mean counts in tests/golden/ref_visits_4096x2_64x48.json.

    python oracle/ref_visits.py
"""
import ctypes
import json
import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
OUT = os.path.join(ROOT, "tests", "golden", "ref_visits_4096x2_64x48.json")


def lib():
    so = os.path.join(HERE, "librefcount.so")
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", so,
                           os.path.join(HERE, "refcount.c"), "-lm"])
    L = ctypes.CDLL(so)
    L.ref_counts.restype = ctypes.c_int
    L.ref_sah_cost.restype = ctypes.c_double
    return L


def counts(w, rays):
    L = lib()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    f = lambda a: np.ascontiguousarray(a, np.float32)
    terr = f(w["terrain"]).reshape(-1, 9)
    lt = f(w["link_tri"]).reshape(-1, 9)
    off = np.ascontiguousarray(w["link_off"], np.int64)
    lp, lq = f(w["link_pos"][0]), f(w["link_quat"][0])
    cp, cq, K = f(w["cam_pos"]), f(w["cam_quat"]), f(w["intr"])
    rays = np.ascontiguousarray(rays, np.int64)
    out = np.zeros((rays.size, 6))
    L.ref_counts(p(terr), ctypes.c_int64(terr.shape[0]), p(lt), p(off), ctypes.c_int(off.size - 1),
                 p(lp), p(lq), p(cp), p(cq), p(K), w["E"], w["C"], w["W"], w["H"],
                 ctypes.c_double(w["far"]), p(rays), ctypes.c_int64(rays.size), p(out))
    return out


def sah_cost(tri):
    """Surface-area cost of the reference hierarchy over these triangles."""
    t = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    return float(lib().ref_sah_cost(t.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(t.shape[0])))


def main():
    import scenegen as sg
    w = sg.robots_4096(steps=1)
    total = w["E"] * w["C"] * w["H"] * w["W"]
    rays = np.sort(np.random.default_rng(2602_03002).choice(total, size=65536, replace=False))
    t0 = time.time()
    c = counts(w, rays)
    m = c.mean(axis=0)
    res = {
        "description": "mean per-ray reference counts: binned-SAH BVH2 (32 bins, leaf <= 4, "
                       "C_trav = C_tri = 1), SAH top level per env, ordered closest-first "
                       "traversal under the render bound; 65,536 seeded rays of step 0",
        "workload": w["name"], "n_rays": int(rays.size), "seed": 260203002,
        "mean_counts": {"node": float(m[0] + m[1]), "tri": float(m[2] + m[3]), "inst": float(m[4])},
        "split": {"robot_nodes": float(m[0]), "terrain_nodes": float(m[1]),
                  "link_tris": float(m[2]), "terrain_tris": float(m[3]), "hit_fraction": float(m[5])},
        "sah_cost_terrain": sah_cost(w["terrain"]),
        "bytes_per_ray_formula": "12 + 13 + 56 node + 36 tri + 28 inst",
        "seconds": round(time.time() - t0, 1),
    }
    c_ = res["mean_counts"]
    res["bytes_per_ray"] = 12 + 13 + 56 * c_["node"] + 36 * c_["tri"] + 28 * c_["inst"]
    json.dump(res, open(OUT, "w"), indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
