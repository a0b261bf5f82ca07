"""The parity helpers themselves, pinned on the CPU against the oracle.

The parity tests compare transported vectors of rays that end in a face next
to the oracle's (an endpoint on their shared edge, where either face is a
correct answer) after unfolding the GPU's vectors about that edge.  Here the
unfolding is checked against the oracle's own transport: a ray stopped just
before an edge and the same ray stopped just after it differ exactly by the
unfolding (a vector is constant inside a face and rotated with the hinge).
"""
import numpy as np

import oracle
from parity import _unfold_about_edge, report
from workloads import configs as CF
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len


def test_unfold_matches_oracle_transport_across_an_edge():
    X, F = CF.mesh_config(1)
    X, F = M.canonical(M.sh_displace(X.astype(np.float64), 6, 0.2, np.random.default_rng(7)), F)
    om = oracle.Mesh(X, F)
    r = random_rays(X, F, 200, np.random.default_rng(8), uniform_len(0.3, 0.6), K=2)
    checked = 0
    for i in range(200):
        t = om.trace(r["f"][i], r["b"][i], r["v"][i])
        if len(t["kind"]) < 2 or t["kind"][0] != 0:   # the first event must be an edge crossing
            continue
        # the traced length at the first crossing, by bisection on the length
        L = np.linalg.norm(r["v"][i].astype(np.float64))
        lo, hi = 0.0, L
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            o = om.exp(r["f"][i:i + 1], r["b"][i:i + 1], r["v"][i:i + 1] * (mid / L))
            if o["n_cross"][0] == 0:
                lo = mid
            else:
                hi = mid
        s = lo
        a = om.exp(r["f"][i:i + 1], r["b"][i:i + 1], r["v"][i:i + 1] * ((s - 1e-9) / L), r["W"][i:i + 1])
        b = om.exp(r["f"][i:i + 1], r["b"][i:i + 1], r["v"][i:i + 1] * ((s + 1e-9) / L), r["W"][i:i + 1])
        if a["n_cross"][0] != 0 or b["n_cross"][0] != 1 or b["min_vdist"][0] < 1e-4:
            continue
        w = np.concatenate([a["v"][0:1], a["W"][0]])
        got = _unfold_about_edge(X, F, a["f"][0], b["f"][0], w)
        want = np.concatenate([b["v"][0:1], b["W"][0]])
        # v' grows by 2e-9 in length between the two; directions and W are otherwise equal
        ang = np.arctan2(np.linalg.norm(np.cross(got, want), axis=1), (got * want).sum(1))
        assert ang.max() < 1e-12, (i, ang)
        assert np.abs(np.linalg.norm(got[1:], axis=1) - np.linalg.norm(want[1:], axis=1)).max() < 1e-12
        checked += 1
    assert checked >= 20


def test_unfold_is_identity_on_a_plane():
    X, F = M.canonical(*M.flat_grid(6, 0.2, np.random.default_rng(2), size=6.0))
    w = np.array([[0.3, -0.2, 0.0], [1.0, 2.0, 0.0]])
    done = 0
    for f in range(F.shape[0]):
        for g in range(f + 1, F.shape[0]):
            if len(set(F[f]) & set(F[g])) == 2:
                assert np.allclose(_unfold_about_edge(X, F, f, g, w), w, atol=1e-12)
                done += 1
        if done > 20:
            break
    assert done > 20


def test_report_counts_slid_rays_and_excuses_only_ties():
    """Oracle against itself with hole avoidance: everything matches, slid rays
    are compared (not excused), and a planted error on a slid ray is caught."""
    from test_oracle_holes import holed_sphere
    X, F = holed_sphere()
    om = oracle.Mesh(X, F)
    r = random_rays(X, F, 3000, np.random.default_rng(21), uniform_len(0.0, 4.0), K=2)
    o = om.exp(r["f"], r["b"], r["v"], r["W"], boundary_mode=1)
    g = {k: o[k].copy() for k in ("f", "b", "p", "v", "W", "status", "n_cross")}
    g["hash"] = o["hash"].copy()
    s = report(o, g, om.mean_edge, K=2, mesh=(X, F))
    assert s["n_slid"] > 300 and s["n_slid_compared"] >= 0.9 * s["n_slid"], s
    assert s["bad_not_near"] == 0 and s["W_angle_max"] == 0.0
    i = np.where((o["n_bnd"] > 0) & (o["bnd_margin"] > 1e-3) & (o["min_vdist"] > 1e-3))[0][0]
    g["p"][i] += 10 * s["tol"]
    g["W"][i, 0] = -g["W"][i, 0]
    s2 = report(o, g, om.mean_edge, K=2, mesh=(X, F))
    assert s2["bad_not_near"] == 1 and s2["W_angle_max"] > 1.0
