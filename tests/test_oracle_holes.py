"""Pins of the oracle's hole avoidance (Sec. 4; the hole branches of the
appendix algorithms transport_over_edge and transport_over_vertex).

Reading: a ray that reaches a boundary edge slides along it toward the end
its direction leans to; at a boundary vertex it resumes straight in the fan
face whose corner holds the projection of the direction recorded at the
boundary (least out-of-plane deviation); when no face's corner holds it, it
slides on along the next boundary edge.  On a flat plane these moves have
closed forms, checked here; on curved meshes the invariants are checked.
"""
import numpy as np
import pytest

import oracle
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len
from test_oracle_pins import locate

HOLE = dict(boundary_mode=1)


def plane():
    # [-2, 3]^2, spacing 0.25, square hole [0, 1]^2 (sides on grid lines)
    X, F = M.canonical(*M.plane_with_hole(20, 5.0, -2.0, 0.0, 1.0))
    return X, F, oracle.Mesh(X, F)


def shoot(X, F, m, p0, d, L, **kw):
    f, b = locate(X, F, np.array([p0[0], p0[1], 0.0]))
    v = L * np.array([d[0], d[1], 0.0]) / np.hypot(d[0], d[1])
    W = np.array([[[0.3, -0.7, 0.0]]])
    return m.exp(np.array([f]), b[None], v[None], W, **kw), v, W


def test_slide_to_corner_then_resume():
    """Hits the hole's left side at (0, 0.3), slides up past the side's grid
    vertices (0, 0.5), (0, 0.75), where the recorded direction points into the
    hole, to the corner (0, 1), where it points out of it: resumes straight."""
    X, F, m = plane()
    d = np.array([1.0, 0.2]) / np.hypot(1.0, 0.2)
    seg = 0.5 / d[0]
    o, v, W = shoot(X, F, m, (-0.5, 0.2), d, 2.0, **HOLE)
    assert o["status"][0] == 0
    rest = 2.0 - seg - 0.7
    want = np.array([0.0, 1.0]) + rest * d
    assert np.abs(o["p"][0, :2] - want).max() < 1e-12
    assert abs(o["p"][0, 2]) < 1e-15
    assert abs(o["traced"][0] - 2.0) < 1e-12
    assert o["n_bnd"][0] == 4                        # three slides, one resumption
    assert np.abs(o["v"][0] - v).max() < 1e-12      # flat: the direction is unchanged
    assert np.abs(o["W"][0] - W[0]).max() < 1e-12   # and so are transported vectors
    # without hole avoidance the ray stops on the hole's side
    o0, _, _ = shoot(X, F, m, (-0.5, 0.2), d, 2.0)
    assert o0["status"][0] == oracle.RAY_BOUNDARY
    assert np.abs(o0["p"][0, :2] - [0.0, 0.2 + 0.5 * 0.2]).max() < 1e-12


def test_slide_down_when_leaning_down():
    """Direction leaning down: the slide goes to the lower corner (0, 0)."""
    X, F, m = plane()
    d = np.array([1.0, -0.4]) / np.hypot(1.0, -0.4)
    seg = 0.5 / d[0]
    o, _, _ = shoot(X, F, m, (-0.5, 0.8), d, 1.5, **HOLE)
    hit = 0.8 - 0.5 * 0.4
    rest = 1.5 - seg - hit
    assert np.abs(o["p"][0, :2] - (np.array([0.0, 0.0]) + rest * d)).max() < 1e-12
    assert o["status"][0] == 0 and o["n_bnd"][0] == 4   # 0.6 -> 0.5 -> 0.25 -> 0, resume


def test_length_ends_during_slide():
    X, F, m = plane()
    d = np.array([1.0, 0.2]) / np.hypot(1.0, 0.2)
    seg = 0.5 / d[0]
    o, v, _ = shoot(X, F, m, (-0.5, 0.2), d, seg + 0.3, **HOLE)
    assert o["status"][0] == 0
    assert np.abs(o["p"][0, :2] - [0.0, 0.6]).max() < 1e-12
    assert np.abs(o["v"][0] - v).max() < 1e-12     # the recorded direction is reported
    assert o["n_bnd"][0] == 2                      # one whole slide (to (0, 0.5)), then part of the next
    assert abs(o["traced"][0] - (seg + 0.3)) < 1e-12
    # the closest call of its decisions: the slide's end (|cos| of d to the vertical side), which
    # equals the corner test's margin against the horizontal fan edge at (0, 0.5)
    assert abs(o["bnd_margin"][0] - 0.2 / np.hypot(1.0, 0.2)) < 1e-12


def test_slide_around_outer_corner():
    """Hits the mesh's right border x = 3, slides up to the corner (3, 3); no
    face there holds the direction (it points off the mesh), so the ray slides
    on along the top border y = 3, to the left."""
    X, F, m = plane()
    d = np.array([1.0, 0.5]) / np.hypot(1.0, 0.5)
    seg = 0.5 / d[0]
    L = 2.0
    o, _, _ = shoot(X, F, m, (2.5, 2.1), d, L, **HOLE)
    rest = L - seg - 0.65
    assert o["status"][0] == 0
    assert np.abs(o["p"][0, :2] - [3.0 - rest, 3.0]).max() < 1e-12
    assert o["n_bnd"][0] == 3 + int(rest / 0.25) + 1   # three side slides, whole top edges, a partial one
    assert abs(o["traced"][0] - L) < 1e-12


def test_max_steps_during_slides():
    X, F, m = plane()
    d = np.array([1.0, 0.5]) / np.hypot(1.0, 0.5)
    o, _, _ = shoot(X, F, m, (2.5, 2.1), d, 2.0, max_steps=3, **HOLE)
    assert o["status"][0] == oracle.RAY_MAXSTEPS
    assert o["n_cross"][0] <= 3


def holed_sphere():
    X, F = M.icosphere(3)
    X = M.sh_displace(X, 6, 0.1, np.random.default_rng(12))
    rng = np.random.default_rng(13)
    c = X[F].mean(1)
    dead = set()
    for cen in rng.normal(size=(5, 3)):          # five holes of ~6 faces
        cen /= np.linalg.norm(cen)
        dead.update(np.argsort(np.linalg.norm(c / np.linalg.norm(c, axis=1)[:, None] - cen, axis=1))[:6].tolist())
    return M.canonical(*M.remove_faces(X, F, sorted(dead)))


def test_invariants_on_sphere_with_holes():
    """Traced length = |v_t|, |W'| = |W|, the angle of W' to v' is kept, no
    ray ends on the boundary, and rays that never reach the boundary are
    unchanged by the option."""
    X, F = holed_sphere()
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 3000, np.random.default_rng(14), uniform_len(0.0, 4.0), K=2)
    o = m.exp(r["f"], r["b"], r["v"], r["W"], **HOLE)
    o0 = m.exp(r["f"], r["b"], r["v"], r["W"])
    assert np.all(o["status"] == 0)
    assert (o["n_bnd"] > 0).sum() > 300
    L = np.linalg.norm(o["v"], axis=1)
    assert np.allclose(o["traced"], L, rtol=0, atol=1e-12)
    n0 = np.linalg.norm(r["W"].astype(np.float64), axis=2)
    n1 = np.linalg.norm(o["W"], axis=2)
    # W is projected onto the start face first; compare against that norm
    Xd = X.astype(np.float64)
    nf = np.cross(Xd[F[r["f"], 1]] - Xd[F[r["f"], 0]], Xd[F[r["f"], 2]] - Xd[F[r["f"], 0]])
    nf /= np.linalg.norm(nf, axis=1)[:, None]
    Wt = r["W"] - (r["W"] * nf[:, None, :]).sum(2)[:, :, None] * nf[:, None, :]
    assert np.allclose(n1, np.linalg.norm(Wt, axis=2), rtol=1e-12, atol=1e-12)
    vt = r["v"] - (r["v"] * nf).sum(1)[:, None] * nf
    cos0 = (Wt * vt[:, None, :]).sum(2) / (np.linalg.norm(Wt, axis=2) * np.linalg.norm(vt, axis=1)[:, None])
    cos1 = (o["W"] * o["v"][:, None, :]).sum(2) / (n1 * L[:, None])
    assert np.abs(cos0 - cos1).max() < 1e-10
    same = o0["status"] == 0
    assert same.sum() > 1000
    for k in ("f", "p", "v", "W", "n_cross"):
        assert np.array_equal(o[k][same], o0[k][same]), k
    assert np.all(o["n_bnd"][same] == 0)
    # every ray that met the boundary reports the margin of its closest decision, the others none;
    # the straight parts of slid rays keep their own distance to vertices
    slid = o["n_bnd"] > 0
    assert np.all(np.isinf(o["bnd_margin"][~slid])) and np.all(np.isfinite(o["bnd_margin"][slid]))
    assert np.all(o["bnd_margin"][slid] >= 0.0)
    assert np.median(o["min_vdist"][slid]) > 1e-4 * m.mean_edge


def test_gradx_excludes_boundary_rays():
    X, F = holed_sphere()
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 400, np.random.default_rng(15), uniform_len(0.0, 3.0))
    o = m.exp(r["f"], r["b"], r["v"], **HOLE)
    g = np.random.default_rng(16).normal(size=(400, 3))
    _, nvx = m.gradx(r["f"], r["b"], r["v"], g, **HOLE)
    assert np.all(nvx[o["n_bnd"] > 0] == -1)
