"""Pins of the float64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
(flat plane, developable prism, cube corner, sphere), brute-force planar
unfolding, the hinge-composition identity and the invariants of the
straightest rule (Sec. 4).  A plausible mistake in the oracle (dropped term,
wrong sign, wrong side of the fan, transposed rotation) fails at least one.
"""
import numpy as np
import pytest

import oracle
from workloads import configs as CF
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len, face_frames
from unfold_bruteforce import unfold_path


def bary_of(X, F, f, p):
    x0, x1, x2 = (X[F[f, k]].astype(np.float64) for k in range(3))
    A = np.column_stack([x1 - x0, x2 - x0])
    l, *_ = np.linalg.lstsq(A, p - x0, rcond=None)
    return np.array([1 - l.sum(), l[0], l[1]])


def locate(X, F, p, faces=None):
    faces = range(F.shape[0]) if faces is None else faces
    for f in faces:
        b = bary_of(X, F, f, p)
        x = (b[:, None] * X[F[f]].astype(np.float64)).sum(0)
        if b.min() >= -1e-12 and np.linalg.norm(x - p) < 1e-12:
            return f, np.clip(b, 0, None) / np.clip(b, 0, None).sum()
    raise AssertionError("point not on mesh")


# ---------------------------------------------------------------- P1 flat plane
def test_flat_plane_straight_lines(rng):
    """theta = 2 pi everywhere: Exp_p(v) = p + v and vectors are unchanged (Sec. 4)."""
    X, F = M.canonical(*M.flat_grid(12, 0.3, np.random.default_rng(1), size=12.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    inner = [f for f in range(F.shape[0]) if np.all(np.abs(Xd[F[f]][:, :2] - 6.0).max(1) < 2.5)]
    r = random_rays(X, F, 400, rng, uniform_len(0.0, 3.0), K=2, faces=inner)
    b = r["b"].astype(np.float64)
    v = r["v"].astype(np.float64)
    W = r["W"].astype(np.float64)
    p0 = (b[:, :, None] * Xd[F[r["f"]]]).sum(1) / b.sum(1)[:, None]
    # add rays aimed exactly through interior vertices
    vids = np.resize([i for i in range(X.shape[0]) if np.abs(Xd[i, :2] - 6.0).max() < 2.0], 60)
    fa = r["f"][:60]
    va = (Xd[vids] - p0[:60]) * 1.3
    f_all = np.concatenate([r["f"], fa])
    b_all = np.concatenate([b, b[:60]])
    v_all = np.concatenate([v, va])
    W_all = np.concatenate([W, W[:60]])
    p_all = np.concatenate([p0, p0[:60]])
    o = m.exp(f_all, b_all, v_all, W_all)
    assert np.all(o["status"] == 0)
    assert np.abs(o["p"] - (p_all + v_all)).max() < 1e-12
    assert np.abs(o["v"] - v_all).max() < 1e-12
    assert np.abs(o["W"] - W_all).max() < 1e-12
    # the aimed rays really went through vertices
    assert np.all(o["min_vdist"][-60:] == 0.0)


# ---------------------------------------------------------------- P2 prism
def _prism_dev(X, nsides, nr):
    Xd = X.astype(np.float64)
    P = Xd[np.arange(nsides) * (nr + 1)][:, :2]
    nxt = np.roll(P, -1, axis=0)
    w = np.linalg.norm(nxt - P, axis=1)
    u = (nxt - P) / w[:, None]
    S = np.concatenate([[0.0], np.cumsum(w)])
    return P, u, S


def _facet(F, f, nsides, nr):
    ks = sorted(set(int(i) // (nr + 1) for i in F[f]))
    if ks == [0, nsides - 1]:
        return nsides - 1
    return ks[0]


def test_prism_unrolled_helix(rng):
    """Developable cylinder: the geodesic is the straight line of the development."""
    nsides, nr, h = 7, 6, 3.0
    X, F, meta = M.prism(nsides, nr, radius=1.0, height=h)
    X, F = M.canonical(X, F)
    m = oracle.Mesh(X, F)
    P, u, S = _prism_dev(X, nsides, nr)
    n = 300
    f = rng.integers(0, F.shape[0], n)
    b = rng.dirichlet([1, 1, 1], n)
    Xd = X.astype(np.float64)
    p0 = (b[:, :, None] * Xd[F[f]]).sum(1)
    ang = rng.uniform(0, 2 * np.pi, n)
    wang = rng.uniform(0, 2 * np.pi, n)
    k0 = np.array([_facet(F, fi, nsides, nr) for fi in f])
    s0 = S[k0] + np.einsum("ij,ij->i", p0[:, :2] - P[k0], u[k0])
    z0 = p0[:, 2]
    ds, dz = np.cos(ang), np.sin(ang)
    # longest length that keeps the line inside the open strip (margin 0.05)
    lim = np.where(dz > 0, (h / 2 - 0.05 - z0) / np.maximum(dz, 1e-12), (z0 + h / 2 - 0.05) / np.maximum(-dz, 1e-12))
    L = np.minimum(rng.uniform(0, 6.0, n), np.maximum(lim, 0))
    d3 = ds[:, None] * np.column_stack([u[k0], np.zeros(n)]) + dz[:, None] * np.array([0, 0, 1.0])
    v = L[:, None] * d3
    W = np.cos(wang)[:, None] * np.column_stack([u[k0], np.zeros(n)]) + np.sin(wang)[:, None] * np.array([0, 0, 1.0])
    o = m.exp(f, b, v, W[:, None, :])
    assert np.all(o["status"] == 0)
    se = np.mod(s0 + L * ds, S[-1])
    ke = np.clip(np.searchsorted(S, se, side="right") - 1, 0, nsides - 1)
    t = se - S[ke]
    pe = np.column_stack([P[ke] + t[:, None] * u[ke], z0 + L * dz])
    assert np.abs(o["p"] - pe).max() < 1e-11
    ws, wz = np.cos(wang), np.sin(wang)
    We = ws[:, None] * np.column_stack([u[ke], np.zeros(n)]) + wz[:, None] * np.array([0, 0, 1.0])
    assert np.abs(o["W"][:, 0] - We).max() < 1e-11
    ve = L[:, None] * (ds[:, None] * np.column_stack([u[ke], np.zeros(n)]) + dz[:, None] * np.array([0, 0, 1.0]))
    assert np.abs(o["v"] - ve).max() < 1e-11
    assert o["n_cross"].max() > 10   # the paths really wrap around facets


# ---------------------------------------------------------------- P3 cube corner
@pytest.mark.parametrize("a", [0.1, 0.4, 0.7, np.pi / 4 - 0.05, np.pi / 4 + 0.05, 1.2, 1.45])
def test_cube_corner_half_angle(a):
    """A ray through a cube corner (theta = 3 pi / 2) leaves 3 pi / 4 from -d on both sides."""
    X, F = M.canonical(*M.cube_grid(2, 1.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    c = np.array([1.0, 1.0, 1.0])
    d = np.array([np.cos(a), np.sin(a), 0.0])
    D, r = 0.8, 0.6
    p = c - D * d
    ztop = [f for f in range(F.shape[0]) if np.all(Xd[F[f], 2] == 1.0)]
    f, b = locate(Xd, F, p, ztop)
    o = m.exp([f], [b], [(D + r) * d])
    if a <= np.pi / 4:
        out = np.cos(np.pi / 4 + a) * np.array([0, -1.0, 0]) + np.sin(np.pi / 4 + a) * np.array([0, 0, -1.0])
    else:
        out = np.cos(3 * np.pi / 4 - a) * np.array([-1.0, 0, 0]) + np.sin(3 * np.pi / 4 - a) * np.array([0, 0, -1.0])
    assert o["status"][0] == 0
    assert o["min_vdist"][0] == 0.0
    assert np.abs(o["p"][0] - (c + r * out)).max() < 1e-12
    assert np.abs(o["v"][0] / (D + r) - out).max() < 1e-12


def test_cube_corner_reversible():
    """The vertex rule is symmetric: tracing back with -v' returns to the start."""
    X, F = M.canonical(*M.cube_grid(2, 1.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    c = np.array([1.0, 1.0, 1.0])
    ztop = [f for f in range(F.shape[0]) if np.all(Xd[F[f], 2] == 1.0)]
    for a in (0.2, 0.9, 1.3):
        d = np.array([np.cos(a), np.sin(a), 0.0])
        p = c - 0.7 * d
        f, b = locate(Xd, F, p, ztop)
        o = m.exp([f], [b], [1.2 * d])
        back = m.exp(o["f"], o["b"], -o["v"])
        assert np.abs(back["p"][0] - p).max() < 1e-12


# ---------------------------------------------------------------- P4 invariants
def _test_meshes():
    out = [M.canonical(*M.icosphere(3))]
    X, F = M.icosphere(3)
    out.append(M.canonical(M.sh_displace(X, 6, 0.15, np.random.default_rng(7)), F))
    out.append(M.canonical(*M.torus_grid(36, 12, 0.2, np.random.default_rng(8))))
    out.append(M.canonical(*M.klein_bottle(96, 48)))   # non-orientable: the carried normal flips
    return out


@pytest.mark.parametrize("mi", [0, 1, 2, 3])
def test_invariants(mi, rng):
    X, F = _test_meshes()[mi]
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 2000, rng, uniform_len(0.0, 2.0), K=2)
    o = m.exp(r["f"], r["b"], r["v"], r["W"])
    assert np.all(o["status"] == 0)
    _, _, n0 = face_frames(X, F, r["f"])
    v = r["v"].astype(np.float64)
    vt = v - np.einsum("ij,ij->i", v, n0)[:, None] * n0
    L = np.linalg.norm(vt, axis=1)
    # I1: traced length equals |v_t|
    assert np.abs(o["traced"] - L).max() < 1e-12 * max(1.0, L.max()) * 10
    assert np.abs(np.linalg.norm(o["v"], axis=1) - L).max() < 1e-12
    # I2 / I3: norms and signed angles to the tangent are kept
    _, _, n1 = face_frames(X, F, o["f"])
    n1 = n1 * o["sigma"][:, None]
    for k in range(2):
        W = r["W"][:, k].astype(np.float64)
        Wt = W - np.einsum("ij,ij->i", W, n0)[:, None] * n0
        assert np.abs(np.linalg.norm(o["W"][:, k], axis=1) - np.linalg.norm(Wt, axis=1)).max() < 1e-12
        a0 = np.arctan2(np.einsum("ij,ij->i", np.cross(vt, Wt), n0), np.einsum("ij,ij->i", vt, Wt))
        a1 = np.arctan2(np.einsum("ij,ij->i", np.cross(o["v"], o["W"][:, k]), n1),
                        np.einsum("ij,ij->i", o["v"], o["W"][:, k]))
        da = np.angle(np.exp(1j * (a1 - a0)))
        assert np.abs(da).max() < 1e-9
    # I4: reversal returns to the start, away from vertices
    sel = np.where(o["min_vdist"] > 1e-6)[0][:500]
    back = m.exp(o["f"][sel], o["b"][sel], -o["v"][sel])
    b0 = r["b"][sel].astype(np.float64)
    p0 = (b0[:, :, None] * X.astype(np.float64)[F[r["f"][sel]]]).sum(1) / b0.sum(1)[:, None]
    assert np.abs(back["p"] - p0).max() < 1e-10
    assert np.all(back["n_cross"] == o["n_cross"][sel])


def test_klein_bottle_is_non_orientable():
    """Walks on the Klein bottle come back with the carried normal reversed
    (sigma = -1) as often as not: no consistent face orientation exists."""
    X, F = M.canonical(*M.klein_bottle(96, 48))
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 2000, np.random.default_rng(3), uniform_len(2.0, 8.0))
    o = m.exp(r["f"], r["b"], r["v"])
    assert np.all(o["status"] == 0)
    assert 0.2 < np.mean(o["sigma"] < 0) < 0.8


def test_reversal_reverses_face_sequence(rng):
    X, F = _test_meshes()[1]
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 50, rng, uniform_len(0.2, 1.5))
    for i in range(50):
        t = m.trace(r["f"][i], r["b"][i], r["v"][i])
        if t["status"] or len(t["kind"]) == 0 or np.any(t["kind"] == 1):
            continue
        o = m.exp([r["f"][i]], [r["b"][i]], [r["v"][i]])
        tb = m.trace(o["f"][0], o["b"][0], -o["v"][0])
        fwd = [int(r["f"][i])] + list(t["face"])
        bwd = [int(o["f"][0])] + list(tb["face"])
        assert fwd == bwd[::-1]


def test_hash_is_fnv1a_of_face_sequence(rng):
    X, F = _test_meshes()[0]
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 20, rng, uniform_len(0.5, 1.5))
    o = m.exp(r["f"], r["b"], r["v"])
    for i in range(20):
        t = m.trace(r["f"][i], r["b"][i], r["v"][i])
        h = 14695981039346656037
        for fid in [int(r["f"][i])] + [int(q) for q in t["face"]]:
            for byte in int(fid & 0xFFFFFFFF).to_bytes(4, "little"):
                h = ((h ^ byte) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
        assert int(o["hash"][i]) == h


# ---------------------------------------------------------------- P5 brute force
@pytest.mark.parametrize("name", ["tetra", "octa", "cube", "ico0", "ico1", "torus"])
def test_bruteforce_unfolding(name, rng):
    if name == "tetra":
        X, F = M.tetrahedron()
    elif name == "octa":
        X, F = M.octahedron()
    elif name == "cube":
        X, F = M.cube_grid(1)
    elif name == "ico0":
        X, F = M.icosahedron()
    elif name == "ico1":
        X, F = M.icosphere(1)
    else:
        X, F = M.torus_grid(12, 4, 0.2, np.random.default_rng(3))
    X, F = M.canonical(X, F)
    m = oracle.Mesh(X, F)
    me = m.mean_edge
    r = random_rays(X, F, 60, rng, uniform_len(0.0, 3.5 * me))
    o = m.exp(r["f"], r["b"], r["v"])
    checked = 0
    for i in range(60):
        if o["min_vdist"][i] < 1e-6 or o["n_cross"][i] > 12:
            continue
        t = m.trace(r["f"][i], r["b"][i], r["v"][i])
        paths = unfold_path(X, F, int(r["f"][i]), r["b"][i].astype(np.float64), r["v"][i].astype(np.float64))
        assert len(paths) == 1
        faces, pe = paths[0]
        assert faces == [int(r["f"][i])] + [int(q) for q in t["face"]]
        assert np.abs(pe - o["p"][i]).max() < 1e-12
        checked += 1
    assert checked >= 30


# ---------------------------------------------------------------- P6 hinge identity
def _rodrigues(x, axis, ang):
    return x * np.cos(ang) + np.cross(axis, x) * np.sin(ang) + axis * np.dot(axis, x) * (1 - np.cos(ang))


def _hinge_chain(X, F, f0, vt, p, events):
    """p' = H_m o ... o H_1(p + v_t); each H_j rotates by the signed dihedral angle about edge j."""
    Xd = X.astype(np.float64)

    def normal(f):
        x0, x1, x2 = Xd[F[f]]
        n = np.cross(x1 - x0, x2 - x0)
        return n / np.linalg.norm(n)

    y = p + vt
    R = np.eye(3)
    prev = f0
    for face, a, c in events:
        xa = Xd[a]
        axis = (Xd[c] - xa) / np.linalg.norm(Xd[c] - xa)
        n0, n1 = normal(prev), normal(face)
        ang = np.arctan2(np.dot(np.cross(n0, n1), axis), np.dot(n0, n1))
        y = xa + _rodrigues(y - xa, axis, ang)
        R = np.column_stack([_rodrigues(R[:, k], axis, ang) for k in range(3)])
        prev = face
    return y, R


def test_hinge_identity_and_ep_rotation(rng):
    X, F = _test_meshes()[1]
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 300, rng, uniform_len(0.0, 2.0))
    g = rng.normal(size=(300, 3))
    o = m.exp(r["f"], r["b"], r["v"])
    gv, gb = m.ep(r["f"], r["b"], r["v"], g)
    assert np.all(gb == 0)
    _, _, n0 = face_frames(X, F, r["f"])
    checked = 0
    for i in range(300):
        t = m.trace(r["f"][i], r["b"][i], r["v"][i])
        if np.any(t["kind"] == 1):
            continue
        v = r["v"][i].astype(np.float64)
        vt = v - np.dot(v, n0[i]) * n0[i]
        b = r["b"][i].astype(np.float64)
        p = (b[:, None] * X.astype(np.float64)[F[r["f"][i]]]).sum(0) / b.sum()
        ev = list(zip(t["face"], t["e0"], t["e1"]))
        y, R = _hinge_chain(X, F, int(r["f"][i]), vt, p, ev)
        assert np.abs(y - o["p"][i]).max() < 1e-12
        # extrinsic proxy: R = M_{p'} M_p^T equals the hinge product away from vertices
        assert np.abs(gv[i] - R.T @ g[i]).max() < 1e-10 * (1 + np.abs(g[i]).max())
        checked += 1
    assert checked > 250


# ---------------------------------------------------------------- P7 sphere
def test_sphere_convergence():
    """The mean error against the sphere's closed form falls as the mesh refines."""
    errs = []
    for lev in (2, 3, 4, 5):
        X, F = M.canonical(*M.icosphere(lev))
        m = oracle.Mesh(X, F)
        r = random_rays(X, F, 2000, np.random.default_rng(lev), uniform_len(0.0, np.pi / 2))
        o = m.exp(r["f"], r["b"], r["v"])
        b = r["b"].astype(np.float64)
        p0 = (b[:, :, None] * X.astype(np.float64)[F[r["f"]]]).sum(1) / b.sum(1)[:, None]
        v = r["v"].astype(np.float64)
        L = np.linalg.norm(v, axis=1)
        ph = p0 / np.linalg.norm(p0, axis=1, keepdims=True)
        ps = np.cos(L)[:, None] * ph + np.sin(L)[:, None] * v / L[:, None]
        errs.append(np.linalg.norm(o["p"] - ps, axis=1).mean())
    assert all(errs[i + 1] < 0.6 * errs[i] for i in range(3)), errs
    assert errs[-1] < 5e-3   # first-order convergence: about 0.11 mean edge at every level


# ---------------------------------------------------------------- mesh checks
def test_mesh_validation():
    X, F = M.canonical(*M.octahedron())
    with pytest.raises(oracle.OracleError) as e:   # edge with three faces
        oracle.Mesh(np.concatenate([X, [[2, 2, 2]]]).astype(np.float32),
                    np.concatenate([F, [[F[0, 0], F[0, 1], 6]]]).astype(np.int32))
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError) as e:   # repeated vertex
        oracle.Mesh(X, np.concatenate([F, [[0, 0, 1]]]).astype(np.int32))
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:   # index out of range
        oracle.Mesh(X, np.concatenate([F, [[0, 1, 99]]]).astype(np.int32))
    assert e.value.code == -1
    # two tetrahedra sharing one vertex: the shared vertex has two fans
    Xt, Ft = M.tetrahedron()
    X2 = np.concatenate([Xt, Xt[1:] + np.array([3.0, 0, 0]) + (Xt[0] - Xt[0])]).astype(np.float32)
    X2[4:] = (Xt[1:] - Xt[0]) * -1 + Xt[0]
    F2 = np.concatenate([Ft, np.where(Ft == 0, 0, Ft + 3)])
    with pytest.raises(oracle.OracleError) as e:
        oracle.Mesh(X2, F2.astype(np.int32))
    assert e.value.code == -2


def test_status_codes(rng):
    X, F = M.canonical(*M.icosphere(2))
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 64, rng, uniform_len(0.5, 1.5))
    o = m.exp(r["f"], r["b"], r["v"], max_steps=1)
    assert np.all((o["status"] == 1) | (o["n_cross"] <= 1))
    assert np.any(o["status"] == 1)
    # invalid inputs
    bad = m.exp([10**6, 0, 0], [[1, 1, 1], [np.nan, 1, 1], [1, 1, 1]], [[0.1, 0, 0], [0.1, 0, 0], [np.nan, 0, 0]])
    assert np.all(bad["status"] == 3)
    # |v| = 0 is the identity
    z = m.exp(r["f"][:4], r["b"][:4], np.zeros((4, 3)))
    assert np.all(z["f"] == r["f"][:4]) and np.all(z["n_cross"] == 0)
    # a hole: rays that reach it stop on the boundary
    Xh, Fh = M.remove_faces(X, F, np.where((F == 0).any(1) | (F == 7).any(1))[0])
    mh = oracle.Mesh(Xh, Fh)
    rh = random_rays(Xh, Fh, 300, rng, uniform_len(1.0, 3.0))
    oh = mh.exp(rh["f"], rh["b"], rh["v"])
    assert np.any(oh["status"] == 2)
    assert np.all(oh["traced"][oh["status"] == 2] < np.linalg.norm(rh["v"][oh["status"] == 2], axis=1))


# ---------------------------------------------------------------- P8 gradients
def test_gfd_flat_is_projection(rng):
    """On a plane Exp_p(v) = p + v: GFD gives J^v = J^p = identity on the tangent plane."""
    X, F = M.canonical(*M.flat_grid(10, 0.3, np.random.default_rng(2), size=10.0))
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    inner = [f for f in range(F.shape[0]) if np.all(np.abs(Xd[F[f]][:, :2] - 5.0).max(1) < 2.0)]
    r = random_rays(X, F, 200, rng, uniform_len(0.1, 2.0), faces=inner)
    g = rng.normal(size=(200, 3))
    out = m.gfd(r["f"], r["b"], r["v"], g, 1e-3, 1e-3)
    gp = g.copy()
    gp[:, 2] = 0
    assert np.abs(out["grad_v"] - gp).max() < 1e-9
    Gb = np.einsum("ic,ikc->ik", gp, Xd[F[r["f"]]])
    assert np.abs(out["grad_b"] - Gb).max() < 1e-8
    gv, _ = m.ep(r["f"], r["b"], r["v"], g)
    assert np.abs(gv - g).max() < 1e-12


def test_gfd_matches_central_differences(rng):
    """Away from vertices the map is a rigid motion of p + v_t (hinge composition),
    so GFD at small eps equals the FP64 central difference (h = 1e-6)."""
    X, F = _test_meshes()[1]
    m = oracle.Mesh(X, F)
    Xd = X.astype(np.float64)
    me = m.mean_edge
    eps = 5e-3 * me
    r = random_rays(X, F, 400, rng, uniform_len(0.1, 1.5))
    o = m.exp(r["f"], r["b"], r["v"])
    # the stencil paths deviate by about eps * |J| from the base path, so the
    # vertex margin must exceed that; stencil endpoints must also stay in the
    # end face of p' (else GFD sees the fold of the chord, a finite-step effect)
    sel = np.where((o["min_vdist"] > 2e-2 * me) & (r["b"].min(1) > 0.05) & (o["b"].min(1) > 0.05))[0][:80]
    f, b, v = r["f"][sel], r["b"][sel].astype(np.float64), r["v"][sel].astype(np.float64)
    g = rng.normal(size=(len(sel), 3))
    out = m.gfd(f, b, v, g, eps, eps)
    e1, e2, n = face_frames(X, F, f)
    vt = v - np.einsum("ij,ij->i", v, n)[:, None] * n
    epar = vt / np.linalg.norm(vt, axis=1, keepdims=True)
    eperp = np.cross(n, epar)
    h = 1e-6
    x0, x1, x2 = Xd[F[f, 0]], Xd[F[f, 1]], Xd[F[f, 2]]
    l1, l2 = np.linalg.norm(x1 - x0, axis=1), np.linalg.norm(x2 - x0, axis=1)
    db_u = np.column_stack([-1 / l1, 1 / l1, np.zeros_like(l1)])
    db_v = np.column_stack([-1 / l2, np.zeros_like(l2), 1 / l2])
    bn = b / b.sum(1, keepdims=True)

    def cd_v(e):
        return (m.exp(f, b, vt + h * e)["p"] - m.exp(f, b, vt - h * e)["p"]) / (2 * h)

    def cd_p(db):
        return (m.exp(f, bn + h * db, vt)["p"] - m.exp(f, bn - h * db, vt)["p"]) / (2 * h)

    cols = [cd_v(epar), cd_v(eperp), cd_p(db_u), cd_p(db_v)]
    fe = o["f"][sel]
    y0, y1, y2 = Xd[F[fe, 0]], Xd[F[fe, 1]], Xd[F[fe, 2]]
    eu = (y1 - y0) / np.linalg.norm(y1 - y0, axis=1, keepdims=True)
    ev = (y2 - y0) / np.linalg.norm(y2 - y0, axis=1, keepdims=True)
    for i in range(len(sel)):
        Mq = np.column_stack([eu[i], ev[i]])
        Mp = np.linalg.pinv(Mq)
        Jv = Mp @ np.column_stack([cols[0][i], cols[1][i]])
        Jp = Mp @ np.column_stack([cols[2][i], cols[3][i]])
        assert np.abs(Jv - out["Jv"][i]).max() < 1e-6 * max(1, np.abs(Jv).max())
        assert np.abs(Jp - out["Jp"][i]).max() < 1e-6 * max(1, np.abs(Jp).max())


def test_gfd_sphere_jacobian_sanity():
    """Sanity only (not parity): GFD with a large step follows the sphere's J_v."""
    X, F = M.canonical(*M.icosphere(5))
    m = oracle.Mesh(X, F)
    r = random_rays(X, F, 300, np.random.default_rng(5), uniform_len(0.3, 1.2))
    g = np.random.default_rng(6).normal(size=(300, 3))
    out = m.gfd(r["f"], r["b"], r["v"], g, 0.05, 0.05)
    b = r["b"].astype(np.float64)
    p = (b[:, :, None] * X.astype(np.float64)[F[r["f"]]]).sum(1) / b.sum(1)[:, None]
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    v = r["v"].astype(np.float64)
    cos = []
    for i in range(300):
        L = np.linalg.norm(v[i])
        vv = np.outer(v[i], v[i])
        Jv = ((np.eye(3) - np.outer(p[i], v[i])) / L - vv / L ** 3) * np.sin(L) + vv / L ** 2 * np.cos(L)
        gv = Jv.T @ g[i]
        gv -= np.dot(gv, p[i]) * p[i]
        cos.append(np.dot(gv, out["grad_v"][i]) / np.linalg.norm(gv) / np.linalg.norm(out["grad_v"][i]))
    assert np.median(cos) > 0.98


def test_orientation_invariance(rng):
    """Reversing the vertex order of some faces describes the same surface: the
    orientation-free unfolding must return the same points and vectors."""
    X, F = M.icosphere(3)
    X, F = M.canonical(M.sh_displace(X, 6, 0.1, np.random.default_rng(3)), F)
    r = random_rays(X, F, 3000, rng, uniform_len(0.0, 2.0), K=2)
    flip = np.random.default_rng(5).random(F.shape[0]) < 0.4
    F2 = F.copy()
    F2[flip] = F2[flip][:, [0, 2, 1]]
    b2 = r["b"].astype(np.float64).copy()
    sel = flip[r["f"]]
    b2[sel] = b2[sel][:, [0, 2, 1]]
    o = oracle.Mesh(X, F).exp(r["f"], r["b"], r["v"], r["W"])
    o2 = oracle.Mesh(X, F2).exp(r["f"], b2, r["v"], r["W"])
    far = o["min_vdist"] > 1e-9
    assert np.abs(o2["p"] - o["p"])[far].max() < 1e-12
    assert np.abs(o2["v"] - o["v"])[far].max() < 1e-12
    assert np.abs(o2["W"] - o["W"])[far].max() < 1e-12


@pytest.mark.parametrize("mixed", [False, True])
def test_gradx_matches_central_differences(rng, mixed):
    """dL/dX for L = sum g . p' against central differences of the float64
    forward in the vertex positions (h = 1e-6), on rays that keep a margin
    from every vertex (frozen combinatorics); also with faces of disagreeing
    orientation (the unfolding is orientation-free)."""
    X, F = CF.mesh_config(1)
    if mixed:
        F = F.copy()
        flip = rng.random(F.shape[0]) < 0.3
        F[flip] = F[flip][:, ::-1]
    X64 = X.astype(np.float64)
    n = 200
    r = random_rays(X, F, n, rng, uniform_len(0.0, 1.5))
    g = rng.standard_normal((n, 3))
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"])
    keep = (o["min_vdist"] > 1e-2 * om.mean_edge) & (o["status"] == 0)
    g[~keep] = 0.0
    gx, nvx = om.gradx(r["f"], r["b"], r["v"], g)
    assert np.all(nvx[keep] == 0)
    assert keep.sum() > 100

    def loss(Xp):
        oo = oracle.Mesh(Xp, F, exact64=True).exp(r["f"], r["b"], r["v"])
        return float((g * oo["p"]).sum())

    h = 1e-6
    for _ in range(2):
        dX = rng.standard_normal(X.shape)
        dX /= np.linalg.norm(dX, axis=1).max()
        cd = (loss(X64 + h * dX) - loss(X64 - h * dX)) / (2 * h)
        assert abs(cd - float((gx * dX).sum())) <= 1e-6 * abs(cd)
    for vtx in np.argsort(-np.linalg.norm(gx, axis=1))[:2]:
        for c in range(3):
            dX = np.zeros_like(X64)
            dX[vtx, c] = 1.0
            cd = (loss(X64 + h * dX) - loss(X64 - h * dX)) / (2 * h)
            assert abs(cd - gx[vtx, c]) <= 1e-6 * np.linalg.norm(gx[vtx])


def test_gradx_translation(rng):
    """Translating the whole mesh (v held fixed) translates every p': the
    vertex gradients sum to the sum of the upstream gradients."""
    X, F = CF.mesh_config(1)
    n = 300
    r = random_rays(X, F, n, rng, uniform_len(0.0, 1.5))
    g = rng.standard_normal((n, 3))
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"])
    keep = (o["min_vdist"] > 1e-2 * om.mean_edge) & (o["status"] == 0)
    g[~keep] = 0.0
    gx, _ = om.gradx(r["f"], r["b"], r["v"], g)
    assert np.allclose(gx.sum(0), g.sum(0), rtol=1e-7, atol=1e-7)


# ---------------------------------------------------------------- transported outputs (backward extension)
def test_transport_vjp_against_central_differences():
    """dL/dv from dL/dv' and dL/dW from dL/dW' (W'_k = R W_k, v' = R v_t, R the
    frame the walk carries): directional derivatives of the float64 forward,
    by central differences in v (margin rays) and in W (linear: every ray)."""
    X, F = M.canonical(M.sh_displace(M.icosphere(3)[0], 6, 0.1, np.random.default_rng(81)), M.icosphere(3)[1])
    m = oracle.Mesh(X, F)
    rng = np.random.default_rng(82)
    r = random_rays(X, F, 300, rng, uniform_len(0.0, 2.0), K=2)
    f, b = r["f"], r["b"].astype(np.float64)
    v, W = r["v"].astype(np.float64), r["W"].astype(np.float64)
    o = m.exp(f, b, v, W)
    gv_out = rng.normal(size=(300, 3))
    gW_out = rng.normal(size=(300, 2, 3))
    gv, gW = m.transport_vjp(f, b, v, gv_out, gW_out)
    dv = rng.normal(size=(300, 3))
    dW = rng.normal(size=(300, 2, 3))
    h = 1e-6
    vp = m.exp(f, b, v + h * dv, W)["v"]
    vm = m.exp(f, b, v - h * dv, W)["v"]
    fd_v = ((vp - vm) / (2 * h) * gv_out).sum(1)
    margin = (o["min_vdist"] > 1e-3 * m.mean_edge) & (o["status"] == 0)
    assert margin.sum() > 150
    an_v = (dv * gv).sum(1)
    scale = np.linalg.norm(dv, axis=1) * np.linalg.norm(gv_out, axis=1)
    assert np.abs(fd_v - an_v)[margin].max() < 1e-6 * scale[margin].max()
    Wp = m.exp(f, b, v, W + h * dW)["W"]
    Wm = m.exp(f, b, v, W - h * dW)["W"]
    fd_W = ((Wp - Wm) / (2 * h) * gW_out).sum((1, 2))
    ok = o["status"] == 0
    an_W = (dW * gW).sum((1, 2))
    assert np.abs(fd_W - an_W)[ok].max() < 1e-7 * np.abs(an_W[ok]).max()
    # a wrong frame (transposed map, dropped orientation) would fail the checks above;
    # a zero-length ray transports nothing: the projection onto the start plane
    z = np.zeros((3, 3))
    gz, gWz = m.transport_vjp(f[:3], b[:3], z, gv_out[:3], gW_out[:3])
    Xd = X.astype(np.float64)
    n0 = np.cross(Xd[F[f[:3], 1]] - Xd[F[f[:3], 0]], Xd[F[f[:3], 2]] - Xd[F[f[:3], 0]])
    n0 /= np.linalg.norm(n0, axis=1)[:, None]
    assert np.allclose(gz, gv_out[:3] - (gv_out[:3] * n0).sum(1)[:, None] * n0, atol=1e-15)
    assert np.allclose(gWz, gW_out[:3] - (gW_out[:3] * n0[:, None, :]).sum(2)[:, :, None] * n0[:, None, :], atol=1e-15)
