"""Pins of the oracle's projection-integration (PI) exponential map (appendix
"Projection Integration Exp Map", Alg. projection-exp) against facts other
than itself: the nearest point of a mesh by brute-force sampling, the flat
plane (each step lands where it was aimed), a folded plane (the vector turns
about the fold by the dihedral angle), the sphere's closed form, and the
invariants of rotating from normal to normal.  The extrinsic proxy and the
geodesic finite differences run over PI as over the straightest map.
"""
import numpy as np
import pytest

import oracle
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len


def _p0(X, F, f, b):
    b = np.asarray(b, np.float64)
    return (b[:, :, None] * X.astype(np.float64)[F[f]]).sum(1) / b.sum(1)[:, None]


def _normals(X, F):
    Xd = X.astype(np.float64)
    n = np.cross(Xd[F[:, 1]] - Xd[F[:, 0]], Xd[F[:, 2]] - Xd[F[:, 0]])
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def _roof(n, beta, size=4.0):
    """A plane folded along the y axis: x <= 0 stays in z = 0, x >= 0 turns up
    by the dihedral angle beta about the y axis."""
    X, F = M.flat_grid(n, 0.0, None, size=size)
    X = X - np.array([size / 2, size / 2, 0.0])
    x = X[:, 0].copy()
    up = x > 0
    X[up, 0] = x[up] * np.cos(beta)
    X[up, 2] = x[up] * np.sin(beta)
    return M.canonical(X, F)


def test_pi_project_is_nearest_point():
    """project_to_mesh returns the nearest point of the mesh: no sample of any
    triangle is nearer, the point lies on the returned face, and where it is
    inside the face, q - c is along the face normal."""
    rng = np.random.default_rng(3)
    X, F = M.canonical(*M.icosphere(1))
    X = X.astype(np.float64)
    m = oracle.Mesh(X.astype(np.float32), F)
    Xd = X.astype(np.float32).astype(np.float64)
    q = rng.normal(size=(300, 3))
    q *= rng.uniform(0.5, 1.5, (300, 1)) / np.linalg.norm(q, axis=1, keepdims=True)
    f, c, bc, mg = m.pi_project(q)
    # dense barycentric samples of every triangle
    t = np.linspace(0.0, 1.0, 41)
    u, v = np.meshgrid(t, t, indexing="ij")
    keep = u + v <= 1.0 + 1e-12
    u, v = u[keep], v[keep]
    P = (Xd[F[:, 0]][:, None] * (1 - u - v)[None, :, None] + Xd[F[:, 1]][:, None] * u[None, :, None]
         + Xd[F[:, 2]][:, None] * v[None, :, None]).reshape(-1, 3)
    hmax = np.linalg.norm(Xd[F[:, 1]] - Xd[F[:, 0]], axis=1).max() / 40.0
    d = np.linalg.norm(q - c, axis=1)
    ds = np.sqrt(((q[:, None, :] - P[None]) ** 2).sum(-1)).min(1)
    assert np.all(d <= ds + 1e-12)
    assert np.all(d >= ds - hmax)
    assert np.all(bc >= 0.0) and np.allclose(bc.sum(1), 1.0, atol=1e-14)
    assert np.allclose((bc[:, :, None] * Xd[F[f]]).sum(1), c, atol=1e-14)
    N = _normals(Xd.astype(np.float32), F)
    inside = bc.min(1) > 1e-9
    r = q[inside] - c[inside]
    cosang = np.abs((r * N[f[inside]]).sum(1)) / np.linalg.norm(r, axis=1)
    assert np.all(cosang > 1 - 1e-12)
    assert np.all(mg >= 0.0)


@pytest.mark.parametrize("step", [0.05, 0.01])
def test_pi_flat_plane(step):
    """On a plane every step lands where it was aimed: p' = p + N s v with N the
    number of steps, the smallest with N s |v| >= |v| (the loop runs while the
    traced length is short of |v|); vectors are unchanged."""
    X, F = M.canonical(*M.flat_grid(12, 0.3, np.random.default_rng(1), size=12.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    inner = [f for f in range(F.shape[0]) if np.all(np.abs(Xd[F[f]][:, :2] - 6.0).max(1) < 2.5)]
    r = random_rays(X, F, 60, np.random.default_rng(2), uniform_len(0.1, 3.0), K=2, faces=inner)
    o = m.pi_exp(r["f"], r["b"], r["v"], r["W"], step=step)
    p0 = _p0(X, F, r["f"], r["b"])
    v = r["v"].astype(np.float64)
    assert np.all(o["status"] == 0)
    N = o["n_steps"]
    n_min = int(np.ceil(1.0 / step - 1e-9))
    assert np.all((N == n_min) | (N == n_min + 1))
    assert np.abs(o["p"] - (p0 + (N * step)[:, None] * v)).max() < 1e-12
    assert np.abs(o["v"] - v).max() < 1e-14
    assert np.abs(o["W"] - r["W"].astype(np.float64)).max() < 1e-14
    L = np.linalg.norm(v, axis=1)
    assert np.allclose(o["traced"], N * step * L, rtol=1e-12)


@pytest.mark.parametrize("beta", [0.3, -0.5])
def test_pi_folded_plane_rotation(beta):
    """Across a fold of dihedral angle beta the vector turns about the fold by
    beta (the rotation taking one normal to the other), keeping its angle to
    the fold; the end point stays within two steps of the unfolded straight
    line at the traced length."""
    X, F = _roof(16, beta)
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    rng = np.random.default_rng(5)
    cen = Xd[F].mean(1)
    start = np.where((cen[:, 0] < -0.6) & (cen[:, 0] > -1.2) & (np.abs(cen[:, 1]) < 0.6))[0]
    n = 40
    f = start[rng.integers(0, start.size, n)]
    b = rng.dirichlet([1, 1, 1], n)
    gam = rng.uniform(0.35 * np.pi, 0.65 * np.pi, n)   # angle to the fold direction (+y)
    L = rng.uniform(1.5, 2.0, n)
    v = L[:, None] * np.stack([np.sin(gam), np.cos(gam), np.zeros(n)], 1)
    W = np.stack([np.zeros(n), np.ones(n), np.zeros(n)], 1)[:, None, :]   # along the fold
    step = 0.01
    o = m.pi_exp(f, b, v, W, step=step)
    assert np.all(o["status"] == 0)
    assert np.all(o["p"][:, 0] > 0.05)   # every ray ended beyond the fold
    ca, sa = np.cos(beta), np.sin(beta)
    R = np.array([[ca, 0, -sa], [0, 1, 0], [sa, 0, ca]])   # about +y, taking (0,0,1) to the folded normal
    Nf = _normals(X, F)
    assert np.allclose(R @ np.array([0, 0, 1.0]), Nf[o["f"][0]], atol=1e-6)
    # (the float32 mesh's folded faces carry beta to about 1e-7)
    assert np.abs(o["v"] - v @ R.T).max() < 1e-6
    assert np.abs(o["W"][:, 0] - W[:, 0] @ R.T).max() < 1e-6
    # the unfolded line: develop the end point back into z = 0 and compare with p0 + traced * d
    p0 = _p0(X, F, f, b)
    pe = o["p"].copy()
    dev = np.stack([pe[:, 0] / ca if abs(ca) > 0 else pe[:, 0], pe[:, 1], np.zeros(n)], 1)
    dev[:, 0] = np.hypot(pe[:, 0], pe[:, 2])
    line = p0 + (o["traced"] / L)[:, None] * v
    assert np.abs(dev - line).max() < 2 * step * L.max()


def test_pi_sphere_closed_form():
    """On a fine icosphere PI follows the great circle: its end point is close to
    Exp_p on the unit sphere at the traced length, within the mesh's own
    deviation from the sphere plus the integrator's."""
    X, F = M.canonical(*M.icosphere(4))
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 12, np.random.default_rng(9), uniform_len(0.3, 1.2))
    o = m.pi_exp(r["f"], r["b"], r["v"], step=0.02)
    assert np.all(o["status"] == 0)
    p0 = _p0(X, F, r["f"], r["b"])
    v = r["v"].astype(np.float64)
    ph = p0 / np.linalg.norm(p0, axis=1, keepdims=True)
    L = np.linalg.norm(v, axis=1)
    d = v - (v * ph).sum(1, keepdims=True) * ph
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = o["traced"]
    ps = np.cos(t)[:, None] * ph + np.sin(t)[:, None] * d
    err = np.linalg.norm(o["p"] - ps, axis=1)
    assert err.max() < 0.01, err
    # the transported vector is the great circle's tangent there, to the same order
    ts = -np.sin(t)[:, None] * ph + np.cos(t)[:, None] * d
    cosv = (o["v"] * ts).sum(1) / L
    assert np.all(cosv > 0.999)


def test_pi_invariants():
    """Rotations keep |v|, keep each extra vector's angle to v and leave v in
    the end face's plane; the end point is on its face; the traced length
    passes |v| by at most two steps."""
    X0, F = M.icosphere(2)
    X, F = M.canonical(M.sh_displace(X0, 4, 0.1, np.random.default_rng(4)), F)
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 64, np.random.default_rng(6), uniform_len(0.0, 1.5), K=2)
    step = 0.02
    o = m.pi_exp(r["f"], r["b"], r["v"], r["W"], step=step)
    assert np.all(o["status"] == 0)
    Nf = _normals(X, F)
    N0 = Nf[r["f"]]
    v0 = r["v"].astype(np.float64)
    vt = v0 - (v0 * N0).sum(1, keepdims=True) * N0
    W0 = r["W"].astype(np.float64)
    Wt = W0 - (W0 * N0[:, None]).sum(-1, keepdims=True) * N0[:, None]
    L = np.linalg.norm(vt, axis=1)
    assert np.allclose(np.linalg.norm(o["v"], axis=1), L, rtol=1e-12, atol=1e-15)
    assert np.abs((o["v"] * Nf[o["f"]]).sum(1)).max() < 1e-12
    assert np.allclose((o["W"] * o["v"][:, None]).sum(-1), (Wt * vt[:, None]).sum(-1), atol=1e-12)
    assert np.allclose(np.linalg.norm(o["W"], axis=-1), np.linalg.norm(Wt, axis=-1), atol=1e-12)
    assert np.all(o["b"] >= 0.0) and np.allclose(o["b"].sum(1), 1.0)
    Xd = X.astype(np.float64)
    assert np.allclose((o["b"][:, :, None] * Xd[F[o["f"]]]).sum(1), o["p"], atol=1e-14)
    moved = L > 0
    assert np.all(o["traced"][moved] >= L[moved])
    assert np.all(o["traced"][moved] <= L[moved] * (1 + 2 * step) + 1e-12)
    assert np.all(o["n_steps"][~moved] == 0)


def test_pi_bad_input_and_max_steps():
    X, F = M.canonical(*M.icosphere(1))
    m = oracle.Mesh(X, F)
    f = np.array([0, 3, -1, 2], np.int32)
    b = np.array([[1, 1, 1], [np.nan, 1, 1], [1, 1, 1], [1, 0, 0]], np.float64)
    v = np.array([[0.5, 0.1, 0.0], [0.1, 0, 0], [0.1, 0, 0], [0.0, 0.0, 0.0]])
    o = m.pi_exp(f, b, v, step=0.1, max_steps=3)
    assert list(o["status"]) == [oracle.RAY_MAXSTEPS, oracle.RAY_BADINPUT, oracle.RAY_BADINPUT, oracle.RAY_OK]
    assert o["n_steps"][0] == 3 and o["n_steps"][3] == 0
    assert np.all(np.isnan(o["p"][1])) and np.all(np.isnan(o["p"][2]))


@pytest.mark.parametrize("beta", [0.4])
def test_pi_ep_folded_plane(beta):
    """The extrinsic proxy over PI: R = M_{p'} M_p^T is the rotation about the
    fold by beta, so grad_v = R^T g."""
    X, F = _roof(16, beta)
    m = oracle.Mesh(X, F)
    rng = np.random.default_rng(8)
    Xd = X.astype(np.float64)
    cen = Xd[F].mean(1)
    start = np.where((cen[:, 0] < -0.6) & (cen[:, 0] > -1.2) & (np.abs(cen[:, 1]) < 0.6))[0]
    n = 20
    f = start[rng.integers(0, start.size, n)]
    b = rng.dirichlet([1, 1, 1], n)
    gam = rng.uniform(0.4 * np.pi, 0.6 * np.pi, n)
    L = rng.uniform(1.5, 2.0, n)
    v = L[:, None] * np.stack([np.sin(gam), np.cos(gam), np.zeros(n)], 1)
    g = rng.normal(size=(n, 3))
    gv, gb = m.pi_ep(f, b, v, g, step=0.02)
    ca, sa = np.cos(beta), np.sin(beta)
    R = np.array([[ca, 0, -sa], [0, 1, 0], [sa, 0, ca]])
    assert np.abs(gv - g @ R).max() < 1e-6   # R^T g, row-wise (beta to float32 rounding)
    assert np.all(gb == 0.0)


def test_pi_gfd_flat_plane():
    """Geodesic finite differences over PI on a plane.  With 1/s not an integer
    every trace takes N = ceil(1/s) steps and lands at p + N s v, so every
    finite difference is exact: J^v = J^p = N s times the identity, hence
    grad_v = N s g and grad_b_k = N s g . x_k (g projected onto the plane)."""
    X, F = M.canonical(*M.flat_grid(12, 0.3, np.random.default_rng(1), size=12.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    inner = [f for f in range(F.shape[0]) if np.all(np.abs(Xd[F[f]][:, :2] - 6.0).max(1) < 2.5)]
    r = random_rays(X, F, 30, np.random.default_rng(12), uniform_len(0.5, 3.0), faces=inner)
    g = np.random.default_rng(13).normal(size=(30, 3))
    step = 0.03
    c = np.ceil(1.0 / step) * step   # 34 steps of 0.03
    eps = 5e-3 * m.mean_edge
    out = m.pi_gfd(r["f"], r["b"], r["v"], g, eps, eps, step=step)
    gin = g.copy()
    gin[:, 2] = 0.0
    assert np.abs(out["grad_v"] - c * gin).max() < 1e-8
    gb_exact = c * (gin[:, None, :] * Xd[F[r["f"]]]).sum(-1)
    assert np.abs(out["grad_b"] - gb_exact).max() < 1e-7
    o = m.pi_exp(r["f"], r["b"], r["v"], step=step)
    assert np.all(o["n_steps"] == 34) and o["margin"].min() > 0.0
