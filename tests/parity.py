"""Parity criteria between the GPU float32 walk and the float64 oracle.

Tolerances (endpoint 1e-4 x mean edge for at least 99.9% of rays; face and
face-sequence divergence only where the float64 path passes within 1e-6 of a
vertex; transported-vector angle 1e-4 rad) are the parity bar for the
float32 tracer.  Where several answers are correct (an endpoint on a shared
edge may be reported in either face; paths through a vertex neighbourhood may
split) the unique part is compared and the rest is checked for validity.
"""
from __future__ import annotations

import numpy as np

NEAR_VERTEX = 1e-6
# A hole-avoidance decision (which end of a boundary edge to slide to, which
# fan face to resume in) taken with a margin below this may go either way in
# float32: the float64 oracle reports the smallest margin per ray.
BOUNDARY_TIE = 1e-5


def _angle(a, b):
    """Angle between vectors along the last axis, float64, accurate near 0."""
    c = np.cross(a, b)
    return np.arctan2(np.linalg.norm(c, axis=-1), np.einsum("...c,...c->...", a, b))


def _unfold_about_edge(X, F, fg, fo, w):
    """Vectors w (K x 3) tangent to face fg, unfolded about the edge fg shares
    with face fo into fo's plane (the rotation about the edge that takes fg's
    inward edge normal to fo's outward one); None if the faces share no edge."""
    common = [v for v in F[fg] if v in F[fo]]
    if len(common) != 2:
        return None
    a, b = X[common[0]].astype(np.float64), X[common[1]].astype(np.float64)
    u = (b - a) / np.linalg.norm(b - a)

    def inward(f):
        c = X[[v for v in F[f] if v not in common][0]].astype(np.float64) - a
        m = c - (c @ u) * u
        return m / np.linalg.norm(m)
    mg, mo = inward(fg), -inward(fo)
    src = np.stack([u, mg, np.cross(u, mg)])
    dst = np.stack([u, mo, np.cross(u, mo)])
    return (w @ src.T) @ dst


def report(o, g, me, K=0, mesh=None):
    """Returns a dict of parity statistics (o: oracle dict, g: GPU dict of numpy
    arrays).  With mesh = (X, F), transported vectors of rays that end in a
    face next to the oracle's (an endpoint on their shared edge) are compared
    after unfolding the GPU's vector about that edge."""
    err = np.linalg.norm(g["p"].astype(np.float64) - o["p"], axis=1)
    tol = 1e-4 * me
    near = o["min_vdist"] < NEAR_VERTEX
    if "bnd_margin" in o:
        near = near | (o["bnd_margin"] < BOUNDARY_TIE)
    bad = err > tol
    face_mis = g["f"] != o["f"]
    # an endpoint within tolerance of an edge may be reported in either face
    on_edge = (np.min(o["b"], axis=1) * me < 2 * tol) | (np.min(g["b"], axis=1) * me < 2 * tol)
    out = dict(n=len(err), tol=tol, frac_ok=1.0 - bad.mean(), n_near=int(near.sum()),
               bad_not_near=int(np.sum(bad & ~near)),
               face_mis_unexplained=int(np.sum(face_mis & ~near & ~(on_edge & ~bad))),
               status_mis=int(np.sum((g["status"] != o["status"]) & ~near)),
               err_max_far=float(err[~near].max()) if np.any(~near) else 0.0,
               err_p999=float(np.percentile(err, 99.9)), err_median=float(np.median(err)))
    if "n_bnd" in o:
        out["n_slid"] = int(np.sum(o["n_bnd"] > 0))
        out["n_slid_compared"] = int(np.sum((o["n_bnd"] > 0) & ~near))
    # an endpoint on an edge may sit in either face: the sequences then differ by that last crossing
    edge_ok = on_edge & ~bad
    if "n_cross" in g and g["n_cross"] is not None:
        dc = np.abs(g["n_cross"].astype(np.int64) - o["n_cross"])
        out["cross_mis_far"] = int(np.sum((dc != 0) & ~near & ~(edge_ok & (dc <= 1))))
        edge_ok = edge_ok & (dc <= 1)
    if "hash" in g and g["hash"] is not None:
        out["hash_mis_far"] = int(np.sum((g["hash"].astype(np.uint64) != o["hash"]) & ~near & ~edge_ok))
    # vectors: same end face, or (with the mesh) the GPU's unfolded into the oracle's face
    gv = g["v"].astype(np.float64)
    gw = g["W"].astype(np.float64) if K else None
    same = (g["f"] == o["f"]) & ~near
    unfolded = np.zeros(len(err), bool)
    skipped = 0
    if mesh is not None:
        X, F = mesh
        for i in np.where((g["f"] != o["f"]) & ~near & ~bad)[0]:
            w = np.concatenate([gv[i:i + 1], gw[i] if K else np.zeros((0, 3))])
            r = _unfold_about_edge(X, F, g["f"][i], o["f"][i], w)
            if r is None:
                skipped += 1
                continue
            gv[i] = r[0]
            if K:
                gw[i] = r[1:]
            unfolded[i] = True
        out["vec_unfolded"] = int(unfolded.sum())
        out["vec_skipped"] = skipped
    cmp = same | unfolded
    if K:
        ow = o["W"]
        ang = _angle(gw, ow)
        out["W_angle_max"] = float(ang[cmp].max()) if cmp.any() else 0.0
        out["W_angle_max_unfolded"] = float(ang[unfolded].max()) if unfolded.any() else 0.0
        out["W_norm_err"] = float(np.abs(np.linalg.norm(gw, axis=2) - np.linalg.norm(ow, axis=2))[cmp].max()) if cmp.any() else 0.0
    vang = _angle(gv, o["v"])
    sel = cmp & (np.linalg.norm(o["v"], axis=1) > 0)
    out["v_angle_max"] = float(vang[sel].max()) if sel.any() else 0.0
    return out


def assert_parity(o, g, me, K=0, label="", mesh=None):
    s = report(o, g, me, K, mesh)
    msg = f"{label}: {s}"
    assert s["frac_ok"] >= 0.999, msg
    assert s["bad_not_near"] == 0, msg
    assert s["face_mis_unexplained"] == 0, msg
    assert s["status_mis"] == 0, msg
    if "hash_mis_far" in s:
        assert s["hash_mis_far"] == 0, msg
    if "cross_mis_far" in s:
        assert s["cross_mis_far"] == 0, msg
    if K:
        assert s["W_angle_max"] <= 1e-4, msg
    assert s["v_angle_max"] <= 1e-4, msg
    if mesh is not None:
        assert s["vec_skipped"] == 0, msg
    return s


def grad_report(o_exp, og_v, og_b, gg_v, gg_b, me, margin=2e-2, tol=1e-3, near=None):
    """Backward parity: relative errors of grad_v (norm) and of the barycentric
    gradient differences (grad_b[1] - grad_b[0], grad_b[2] - grad_b[0]), which
    carry the in-plane start-point gradient (grad_b[k] = G . x_k; its common
    part G . x_0 is ill-conditioned against |G| |x| on curved meshes and is
    checked against that scale).  `margin` rays keep at least margin * mean edge
    from every vertex along the oracle's base walk: finite differences of
    geodesics that pass a vertex closer than their step are not smooth.

    near = (radius, tol_near), for geodesic finite differences: margin rays whose
    base walk passes within radius * mean edge of a vertex are held to tol_near.
    Both sides take the same difference quotient, but the float32 stencil ends
    differ from the float64 ones by rounding, and the quotient amplifies that by
    the map's second derivative, which grows as the walk nears a cone vertex
    (on the 327,680-face mesh, with step eps = 5e-3 mean edge, the b-gradient
    error has median 9e-5 and maximum 1.9e-3 for rays that pass 4-6 eps from a
    vertex, and median 3e-5, maximum 6e-4 for rays that stay beyond 20 eps).
    """
    def d(x):
        return np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]], 1)

    def rel(a, b):
        den = np.linalg.norm(b, axis=1)
        return np.linalg.norm(a - b, axis=-1 if a.ndim == 2 else (1, 2)) / np.maximum(den, 1e-30)

    ev = rel(gg_v, og_v)
    zb = np.linalg.norm(og_b, axis=1) == 0
    eb = np.where(zb, np.linalg.norm(gg_b, axis=1), 0.0)
    nz = ~zb
    if nz.any():
        eb[nz] = np.linalg.norm(d(gg_b[nz]) - d(og_b[nz]), axis=1) / np.maximum(
            np.linalg.norm(d(og_b[nz]), axis=1), 1e-30)
    m = o_exp["min_vdist"] > margin * me
    if "n_bnd" in o_exp:   # a boundary slide is not a smooth part of the map
        m = m & (o_exp["n_bnd"] == 0)
    t = np.full(len(ev), tol)
    if near is not None:
        t[o_exp["min_vdist"] <= near[0] * me] = near[1]
    return dict(n=len(ev), n_margin=int(m.sum()), v_ok=float(np.mean(ev[m] <= t[m])) if m.any() else 1.0,
                b_ok=float(np.mean(eb[m] <= t[m])) if m.any() else 1.0, v_med=float(np.median(ev)),
                b_med=float(np.median(eb)), v_all_ok=float(np.mean(ev <= tol)), finite=bool(
                    np.isfinite(gg_v).all() and np.isfinite(gg_b).all()))


def gradx_report(ref, got, floor=0.1, tol=1e-3):
    """Vertex-gradient parity: per-vertex error against max(|ref_v|, floor * rms)
    (each vertex sums float32 per-crossing terms of size ~ |v| |g| / edge that
    largely cancel between neighbouring hinges, so a vertex whose gradient
    cancels to near zero is judged against the field's scale) and the global
    relative error."""
    nrm = np.linalg.norm(ref, axis=1)
    err = np.linalg.norm(got - ref, axis=1)
    nz = nrm > 0
    rms = float(np.sqrt((nrm[nz] ** 2).mean())) if nz.any() else 0.0
    rel = err / np.maximum(nrm, max(floor * rms, 1e-300))
    return dict(n_verts=int(nz.sum()), rms=rms, global_rel=float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)),
                frac_ok=float(np.mean(rel[nz] <= tol)) if nz.any() else 1.0, max_rel=float(rel.max()),
                finite=bool(np.isfinite(got).all()))
