"""Pins of the oracle's K-step exponential map (eq. fmobj, Sec. "MeshFlow"):
p^(k+1) = Exp_{p^(k)}(v(p^(k)) / K), the field re-evaluated at every
intermediate point.

* Flat plane: Exp_p(v) = p + P v (P the projection onto the plane), so the
  K-step map is explicit Euler integration of the projected field with step
  1/K.  The composition and its derivatives in a field parameter and in the
  start point have closed forms (the Euler recursion and its linearisation).
* Curved mesh, away from vertices: each step's Jacobian in both its start
  point and its vector is the hinge product R (the frame rotation of the
  extrinsic proxy, pinned against the hinge product elsewhere), so the
  derivative of the composition follows the chain rule
      dp^(k+1) = R_k (dp^(k) + P_k dv_k / K),
      dv_k = dv/dtheta . dtheta + dv/dp . dp^(k).
  Central differences (h = 1e-6) of the composed map must agree with it.

The field is v(p) = t0 c1 + t1 (c2 x (p - o)), one (t0, t1) per query.
"""
import numpy as np

import oracle
from workloads import configs as CF
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len

H = 1e-6


def field_factory(theta, c1, c2, o):
    def field(p, f, b):
        return theta[:, 0:1] * c1[None, :] + theta[:, 1:2] * np.cross(c2[None, :], p - o[None, :])
    return field


def test_flat_plane_is_explicit_euler():
    X, F = M.canonical(*M.flat_grid(12, 0.3, np.random.default_rng(1), size=12.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    inner = [f for f in range(F.shape[0]) if np.all(np.abs(Xd[F[f]][:, :2] - 6.0).max(1) < 1.5)]
    rng = np.random.default_rng(31)
    r = random_rays(X, F, 300, rng, uniform_len(0.0, 1.0), faces=inner)
    n = r["f"].shape[0]
    theta = rng.normal(size=(n, 2)) * [0.8, 0.4]
    c1 = np.array([0.6, -0.3, 0.5])           # has a normal part: the step projects it away
    c2 = np.array([0.0, 0.0, 1.0])            # e_z x (p - o): a rotation about o
    o = np.array([6.0, 6.0, 0.0])
    P = np.diag([1.0, 1.0, 0.0])
    K = 4
    it = m.exp_iterated(r["f"], r["b"], field_factory(theta, c1, c2, o), K)
    assert np.all(it["status"] == 0)
    b = r["b"].astype(np.float64)
    p = (b[:, :, None] * Xd[F[r["f"]]]).sum(1) / b.sum(1)[:, None]
    for k in range(K):
        p = p + (field_factory(theta, c1, c2, o)(p, None, None) @ P) / K
        assert np.abs(it["pts"][k] - p).max() < 1e-12, k
    # derivatives: central differences of the composition against the Euler recursion's linearisation
    J = np.zeros((n, 3, 2))   # dp/dtheta
    p = (b[:, :, None] * Xd[F[r["f"]]]).sum(1) / b.sum(1)[:, None]
    for k in range(K):
        dv = np.stack([np.broadcast_to(c1, (n, 3)), np.cross(c2[None, :], p - o[None, :])], 2)
        dv = dv + theta[:, 1, None, None] * np.cross(c2[None, :, None], J, axis=1)
        p = p + (field_factory(theta, c1, c2, o)(p, None, None) @ P) / K
        J = J + np.einsum("ij,njq->niq", P, dv) / K
    for q in range(2):
        tp, tm = theta.copy(), theta.copy()
        tp[:, q] += H
        tm[:, q] -= H
        fd = (m.exp_iterated(r["f"], r["b"], field_factory(tp, c1, c2, o), K)["p"]
              - m.exp_iterated(r["f"], r["b"], field_factory(tm, c1, c2, o), K)["p"]) / (2 * H)
        assert np.abs(fd - J[:, :, q]).max() < 1e-8, q


def _chain_rule(m, X, F, r, theta, c1, c2, o, K, db):
    """dp^(K)/dtheta [n,3,2] and the derivative along start-barycentric direction db [n,3],
    by the chain rule through each step's hinge product R (from the oracle's extrinsic proxy:
    grad_v = R^T g, so g = e_j gives row j of R)."""
    n = r["f"].shape[0]
    Xd = X.astype(np.float64)
    f = r["f"].copy()
    b = r["b"].astype(np.float64)
    b = b / b.sum(1)[:, None]
    p = (b[:, :, None] * Xd[F[f]]).sum(1)
    J = np.zeros((n, 3, 3))   # columns: dtheta0, dtheta1, d(start point along db)
    J[:, :, 2] = (db[:, :, None] * Xd[F[f]]).sum(1)
    fld = field_factory(theta, c1, c2, o)
    for _ in range(K):
        v = fld(p, f, b) / K
        R = np.stack([m.ep(f, b, v, np.broadcast_to(e, (n, 3)).copy())[0] for e in np.eye(3)], 1)
        nf = np.cross(Xd[F[f, 1]] - Xd[F[f, 0]], Xd[F[f, 2]] - Xd[F[f, 0]])
        nf /= np.linalg.norm(nf, axis=1)[:, None]
        Pk = np.eye(3)[None] - nf[:, :, None] * nf[:, None, :]
        dv = np.zeros((n, 3, 3))
        dv[:, :, 0] = c1
        dv[:, :, 1] = np.cross(c2[None, :], p - o[None, :])
        dv = dv + theta[:, 1, None, None] * np.cross(c2[None, :, None], J, axis=1)
        J = np.einsum("nij,njq->niq", R, J + np.einsum("nij,njq->niq", Pk, dv) / K)
        out = m.exp(f, b, v)
        f, b, p = out["f"], out["b"], out["p"]
    return J


def test_curved_mesh_chain_rule_matches_central_differences():
    X, F = CF.mesh_config(1)
    X, F = M.canonical(M.sh_displace(X.astype(np.float64), 6, 0.15, np.random.default_rng(33)), F)
    m = oracle.Mesh(X, F)
    rng = np.random.default_rng(34)
    r = random_rays(X, F, 400, rng, uniform_len(0.0, 1.0))
    n = r["f"].shape[0]
    theta = rng.normal(size=(n, 2)) * [0.5, 0.5]
    c1 = rng.normal(size=3)
    c2 = rng.normal(size=3)
    c2 /= np.linalg.norm(c2)
    o = np.zeros(3)
    K = 3
    db = rng.normal(size=(n, 3))
    db -= db.mean(1)[:, None]          # keeps sum(b) = 1
    it = m.exp_iterated(r["f"], r["b"], field_factory(theta, c1, c2, o), K)
    keep = (it["status"] == 0) & (it["min_vdist"] > 1e-3 * m.mean_edge) & (r["b"].min(1) > 1e-3)
    assert keep.sum() > 150
    J = _chain_rule(m, X, F, r, theta, c1, c2, o, K, db)
    fd = np.zeros((n, 3, 3))
    for q in range(2):
        tp, tm = theta.copy(), theta.copy()
        tp[:, q] += H
        tm[:, q] -= H
        fd[:, :, q] = (m.exp_iterated(r["f"], r["b"], field_factory(tp, c1, c2, o), K)["p"]
                       - m.exp_iterated(r["f"], r["b"], field_factory(tm, c1, c2, o), K)["p"]) / (2 * H)
    b0 = r["b"].astype(np.float64) / r["b"].astype(np.float64).sum(1)[:, None]
    fld = field_factory(theta, c1, c2, o)
    fd[:, :, 2] = (m.exp_iterated(r["f"], b0 + H * db, fld, K)["p"] - m.exp_iterated(r["f"], b0 - H * db, fld, K)["p"]) / (2 * H)
    rel = np.linalg.norm(fd - J, axis=1) / np.maximum(np.linalg.norm(J, axis=1), 1e-12)
    assert np.quantile(rel[keep], 0.99) < 1e-7, np.quantile(rel[keep], [0.5, 0.99, 1.0])
    # a composition that evaluated the field at the start point only would fail this pin
    assert np.abs(J[keep][:, :, 1]).max() > 1e-2


def test_one_step_is_one_exp():
    X, F = CF.mesh_config(1)
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 200, np.random.default_rng(35), uniform_len(0.0, 1.0))
    c1 = np.array([0.3, 0.2, -0.4])
    theta = np.ones((200, 2))
    fld = field_factory(theta, c1, np.array([0.0, 1.0, 0.0]), np.zeros(3))
    it = m.exp_iterated(r["f"], r["b"], fld, 1)
    p0 = m.exp(r["f"], r["b"], np.zeros((200, 3)))["p"]
    o = m.exp(r["f"], r["b"], fld(p0, None, None))
    # (the composition starts from the renormalised barycentrics: equal up to rounding)
    assert np.abs(it["p"] - o["p"]).max() < 1e-13 and np.array_equal(it["f"], o["f"])
