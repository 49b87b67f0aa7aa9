"""Element-wise comparison of renderer output with the FP64 oracle.

Bar (per pixel): depth within 1e-4 m and bit-exact (inst, tri) for every ray
the oracle does not flag.  A flagged ray (edge band, far band or tie band:
decisions FP32 cannot resolve) must still report one of the oracle's band
candidates with that candidate's depth within 1e-4 m, or a miss when it is in
the far band.  The counts of each band are reported apart (a ray can be in
more than one band).
"""
import numpy as np

DEPTH_TOL = 1e-4
FLAG_EDGE, FLAG_FAR, FLAG_TIE = 1, 2, 4


def compare(depth, inst, tri, ref, tol=DEPTH_TOL, far=None):
    depth = np.asarray(depth, np.float64).ravel()
    inst = np.asarray(inst).ravel()
    tri = np.asarray(tri).ravel()
    flags = ref["flags"]
    strict = flags == 0
    d_err = np.abs(depth - ref["depth"])
    id_ok = (inst == ref["inst"]) & (tri == ref["tri"])
    bad_strict = strict & ~(id_ok & (d_err <= tol))
    bad_weak = np.zeros_like(strict)
    weak_by_cand = 0
    for i in np.nonzero(~strict)[0]:
        if id_ok[i] and d_err[i] <= tol:
            continue
        cand = ref["cand"][i]
        cd = ref["cand_depth"][i]
        hit = (cand[:, 0] == inst[i]) & (cand[:, 1] == tri[i])
        if hit.any() and np.min(np.abs(cd[hit] - depth[i])) <= tol:
            weak_by_cand += 1
            continue
        if inst[i] == -1 and (flags[i] & FLAG_FAR) and far is not None and depth[i] == np.float32(far):
            weak_by_cand += 1
            continue
        bad_weak[i] = True
    return dict(
        n=int(depth.size), n_flagged=int((~strict).sum()),
        n_edge=int(((flags & FLAG_EDGE) != 0).sum()),
        n_tie=int(((flags & FLAG_TIE) != 0).sum()),
        n_far=int(((flags & FLAG_FAR) != 0).sum()),
        # flagged rays whose answer differs from the oracle's own pick but is
        # one of its band candidates (or a far-band miss)
        n_flagged_other_candidate=int(weak_by_cand),
        strict_fail=int(bad_strict.sum()), weak_fail=int(bad_weak.sum()),
        id_mismatch_strict=int((strict & ~id_ok).sum()),
        max_depth_err=float(d_err[strict].max()) if strict.any() else 0.0,
        bad_idx=np.nonzero(bad_strict | bad_weak)[0][:20].tolist(),
    )


def assert_parity(depth, inst, tri, ref, far, tol=DEPTH_TOL, label=""):
    r = compare(depth, inst, tri, ref, tol=tol, far=far)
    msg = f"{label}: {r}"
    print(msg, flush=True)
    assert r["strict_fail"] == 0 and r["weak_fail"] == 0, msg
    return r
