"""Seeded synthetic triangle meshes.

Every generator builds its geometry in float64 and returns the *canonical*
mesh: vertex positions rounded once to float32 and int32 faces, outward
counter-clockwise.  Both the GPU path and the float64 oracle consume exactly
these float32 values (the oracle upcasts them exactly), so neither side sees a
different surface.  Nothing in this module knows how a geodesic is traced.

Mesh families (paper: synthetic stand-ins for the benchmark meshes of the
accuracy/performance section, F from about 10^3 to 10^6 faces):
  * icosphere(level)            -- midpoint-subdivided icosahedron on the unit sphere
  * geodesic_sphere(freq)       -- icosahedron with each face split into freq^2
  * sh_displace(...)            -- radial displacement by random real spherical harmonics
  * normal_noise(...)           -- i.i.d. offsets along area-weighted vertex normals
  * torus_grid(nu, nv, ...)     -- jittered (u, v) grid torus, R:r = 3:1
  * mobius_strip, klein_bottle  -- non-orientable surfaces (no consistent face orientation exists)
  * tiny test meshes            -- tetrahedron, octahedron, cube grid, flat grid,
                                   polygonal prism (developable cylinder)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "icosahedron", "icosphere", "geodesic_sphere", "sh_displace", "normal_noise",
    "torus_grid", "mobius_strip", "klein_bottle", "tetrahedron", "octahedron", "cube_grid", "flat_grid", "prism",
    "canonical", "mean_edge", "orient_outward", "remove_faces", "plane_with_hole", "slim_faces",
]


def canonical(X, F):
    """Round positions once to float32 and faces to int32 (the shared mesh)."""
    return np.ascontiguousarray(X, dtype=np.float32), np.ascontiguousarray(F, dtype=np.int32)


def mean_edge(X, F):
    """Mean length of the unique undirected edges, in float64."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(X[e[:, 1]] - X[e[:, 0]], axis=1).mean())


def orient_outward(X, F, center=None):
    """Flip faces whose normal points towards `center` (star-shaped meshes only)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.array(F, dtype=np.int64)
    c = X.mean(axis=0) if center is None else np.asarray(center, dtype=np.float64)
    x0, x1, x2 = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    n = np.cross(x1 - x0, x2 - x0)
    flip = np.einsum("ij,ij->i", n, (x0 + x1 + x2) / 3.0 - c) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return F


def icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = []
    for a in (-1.0, 1.0):
        for b in (-t, t):
            V += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    V = np.array(V, dtype=np.float64)
    # the 20 faces are the vertex triples whose pairwise distances are all 2
    d = np.linalg.norm(V[:, None] - V[None], axis=2)
    adj = np.abs(d - 2.0) < 1e-9
    F = [(i, j, k) for i in range(12) for j in range(i + 1, 12) for k in range(j + 1, 12)
         if adj[i, j] and adj[j, k] and adj[i, k]]
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = orient_outward(V, np.array(F), center=np.zeros(3))
    return V, F


def _midpoint_split(X, F):
    F = np.asarray(F, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    key = np.sort(e, axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    nv = X.shape[0]
    Xm = 0.5 * (X[uniq[:, 0]] + X[uniq[:, 1]])
    nf = F.shape[0]
    m01 = nv + inv[0 * nf:1 * nf]
    m12 = nv + inv[1 * nf:2 * nf]
    m20 = nv + inv[2 * nf:3 * nf]
    a, b, c = F[:, 0], F[:, 1], F[:, 2]
    Fn = np.concatenate([
        np.stack([a, m01, m20], 1), np.stack([b, m12, m01], 1),
        np.stack([c, m20, m12], 1), np.stack([m01, m12, m20], 1)])
    return np.concatenate([X, Xm]), Fn


def icosphere(level: int):
    """Unit icosphere: icosahedron, `level` midpoint splits, each projected to the sphere.

    level 3 -> 642 vertices / 1,280 faces; level 7 -> 163,842 / 327,680;
    level 8 -> 655,362 / 1,310,720.
    """
    X, F = icosahedron()
    for _ in range(level):
        X, F = _midpoint_split(X, F)
        X = X / np.linalg.norm(X, axis=1, keepdims=True)
    return X, F


def geodesic_sphere(freq: int):
    """Unit geodesic sphere with F = 20 freq^2 faces (each icosahedron face split freq x freq)."""
    V, F0 = icosahedron()
    n = int(freq)
    ij = [(i, j) for i in range(n + 1) for j in range(n + 1 - i)]
    ij = np.array(ij, dtype=np.int64)                     # weights of corners 1 and 2
    w = np.stack([n - ij[:, 0] - ij[:, 1], ij[:, 0], ij[:, 1]], 1)
    local = {tuple(p): q for q, p in enumerate(ij)}
    tris = []
    for i in range(n):
        for j in range(n - i):
            tris.append((local[(i, j)], local[(i + 1, j)], local[(i, j + 1)]))
            if i + j < n - 1:
                tris.append((local[(i + 1, j)], local[(i + 1, j + 1)], local[(i, j + 1)]))
    tris = np.array(tris, dtype=np.int64)
    npt = ij.shape[0]
    # global key of every lattice point: (vertex id, weight) pairs sorted by id
    keys = np.zeros((F0.shape[0] * npt, 6), dtype=np.int64)
    pos = np.zeros((F0.shape[0] * npt, 3))
    for fi, (a, b, c) in enumerate(F0):
        ids = np.array([a, b, c])
        ww = w.copy()
        idm = np.broadcast_to(ids, ww.shape).copy()
        idm[ww == 0] = -1
        ww[ww == 0] = 0
        order = np.argsort(idm, axis=1, kind="stable")
        idm = np.take_along_axis(idm, order, 1)
        ww = np.take_along_axis(ww, order, 1)
        keys[fi * npt:(fi + 1) * npt] = np.stack(
            [idm[:, 0], ww[:, 0], idm[:, 1], ww[:, 1], idm[:, 2], ww[:, 2]], 1)
        pos[fi * npt:(fi + 1) * npt] = (w[:, :1] * V[a] + w[:, 1:2] * V[b] + w[:, 2:] * V[c]) / n
    uniq, first, inv = np.unique(keys, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    X = pos[first]
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    F = np.concatenate([inv[fi * npt + tris] for fi in range(F0.shape[0])])
    F = orient_outward(X, F, center=np.zeros(3))
    return X, F


def _real_sph_harm(lmax, theta, phi):
    """Orthonormal real spherical harmonics Y_lm for l = 1..lmax (rows), points (cols)."""
    from scipy.special import sph_harm_y
    out = []
    for l in range(1, lmax + 1):
        m = np.arange(0, l + 1)
        Y = sph_harm_y(l, m[:, None], theta[None, :], phi[None, :])   # complex, m >= 0
        sgn = ((-1.0) ** m)[:, None]
        rows = [np.sqrt(2.0) * sgn[mm] * Y[mm].imag for mm in range(l, 0, -1)]   # m = -l..-1
        rows.append(Y[0].real)
        rows += [np.sqrt(2.0) * sgn[mm] * Y[mm].real for mm in range(1, l + 1)]
        out.append(np.stack(rows))
    return np.concatenate(out)


def _real_sph_harm_rec(lmax, theta, phi):
    """The same functions as _real_sph_harm (same row order and signs), from the
    standard three-term recurrences for fully normalised associated Legendre
    functions; vectorised over points, for high degrees."""
    x = np.cos(theta)
    sx = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    # Pbar[l][m] = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(x), without the Condon-Shortley phase
    P = {(0, 0): np.full_like(x, np.sqrt(1.0 / (4.0 * np.pi)))}
    for m in range(1, lmax + 1):
        P[(m, m)] = np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx * P[(m - 1, m - 1)]
    for m in range(0, lmax):
        P[(m + 1, m)] = np.sqrt(2.0 * m + 3.0) * x * P[(m, m)]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[(l, m)] = a * (x * P[(l - 1, m)] - b * P[(l - 2, m)])
    cm = [np.cos(m * phi) for m in range(lmax + 1)]
    sm = [np.sin(m * phi) for m in range(lmax + 1)]
    out = []
    for l in range(1, lmax + 1):
        rows = [np.sqrt(2.0) * P[(l, mm)] * sm[mm] for mm in range(l, 0, -1)]
        rows.append(P[(l, 0)])
        rows += [np.sqrt(2.0) * P[(l, mm)] * cm[mm] for mm in range(1, l + 1)]
        out.append(np.stack(rows))
    return np.concatenate(out)


def sh_displace(X, lmax: int, amplitude: float, rng):
    """r = 1 + amplitude * sum_{l=1..lmax} sum_m c_lm Y_lm(x_hat), c_lm ~ N(0, 1/l^2)."""
    X = np.asarray(X, dtype=np.float64)
    u = X / np.linalg.norm(X, axis=1, keepdims=True)
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.arctan2(u[:, 1], u[:, 0])
    ls = np.concatenate([np.full(2 * l + 1, l) for l in range(1, lmax + 1)])
    c = rng.normal(0.0, 1.0, ls.shape[0]) / ls
    r = np.ones(X.shape[0])
    chunk = 1 << 16
    sh = _real_sph_harm if lmax <= 8 else _real_sph_harm_rec   # the recurrence for high degrees (speed)
    for s in range(0, X.shape[0], chunk):
        Y = sh(lmax, theta[s:s + chunk], phi[s:s + chunk])
        r[s:s + chunk] += amplitude * (c @ Y)
    return u * r[:, None]


def vertex_normals(X, F):
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    n = np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]])   # 2 * area * unit normal
    vn = np.zeros_like(X)
    for k in range(3):
        np.add.at(vn, F[:, k], n)
    return vn / np.linalg.norm(vn, axis=1, keepdims=True)


def normal_noise(X, F, sigma_rel_edge: float, rng):
    """Offsets N(0, sigma_rel_edge * mean edge) along unit area-weighted vertex normals."""
    X = np.asarray(X, dtype=np.float64)
    sig = sigma_rel_edge * mean_edge(X, F)
    return X + rng.normal(0.0, sig, X.shape[0])[:, None] * vertex_normals(X, F)


def slim_faces(X, F, frac: float, rng, lo: float = 0.6, hi: float = 0.9):
    """Slim triangles: a fraction `frac` of the vertices (no two adjacent) each
    move a fraction U[lo, hi] of the way toward the midpoint of the opposite
    edge of one incident face, which becomes a sliver (its height shrinks by
    that fraction) while the faces around stretch."""
    X = np.asarray(X, dtype=np.float64).copy()
    F = np.asarray(F)
    inc = [[] for _ in range(X.shape[0])]
    for fi, (a, b, c) in enumerate(F):
        inc[a].append((b, c)); inc[b].append((c, a)); inc[c].append((a, b))
    taken = np.zeros(X.shape[0], bool)
    for v in rng.permutation(X.shape[0]):
        if rng.uniform() >= frac or taken[v] or any(taken[u] for e in inc[v] for u in e):
            continue
        a, b = inc[v][rng.integers(len(inc[v]))]
        X[v] += rng.uniform(lo, hi) * (0.5 * (X[a] + X[b]) - X[v])
        taken[v] = True
    return X


def _twisted_grid(nu, nv, periodic_v):
    """Faces of an nu x nv grid, periodic in u with the v index reflected across the
    seam ((u + period, v) ~ (u, -v)); periodic or open in v."""
    def vid(i, j):
        if i == nu:
            i, j = 0, (nv - 1 - j) if not periodic_v else (-j) % nv
        return i * nv + (j % nv)
    F = []
    for i in range(nu):
        for j in range(nv if periodic_v else nv - 1):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            F += [(a, b, c), (a, c, d)]
    return np.array(F, dtype=np.int64)


def mobius_strip(nu: int, nw: int, R=1.0, width=0.6):
    """Moebius strip: centre circle of radius R, a half twist along it, boundary on w = +-1."""
    u = np.arange(nu) * (2 * np.pi / nu)
    w = np.linspace(-1.0, 1.0, nw)
    U, Wg = np.meshgrid(u, w, indexing="ij")
    h = 0.5 * width * Wg
    X = np.stack([(R + h * np.cos(U / 2)) * np.cos(U), (R + h * np.cos(U / 2)) * np.sin(U), h * np.sin(U / 2)], -1)
    return X.reshape(-1, 3), _twisted_grid(nu, nw, periodic_v=False)


def klein_bottle(nu: int, nv: int, r=2.0):
    """Klein bottle, figure-8 immersion in R^3 (self-intersecting in space, a closed
    non-orientable manifold as a mesh: the walk is intrinsic)."""
    u = np.arange(nu) * (2 * np.pi / nu)
    v = np.arange(nv) * (2 * np.pi / nv)
    U, V = np.meshgrid(u, v, indexing="ij")
    a = r + np.cos(U / 2) * np.sin(V) - np.sin(U / 2) * np.sin(2 * V)
    X = np.stack([a * np.cos(U), a * np.sin(U), np.sin(U / 2) * np.sin(V) + np.cos(U / 2) * np.sin(2 * V)], -1)
    return X.reshape(-1, 3), _twisted_grid(nu, nv, periodic_v=True)


def torus_grid(nu: int, nv: int, jitter: float, rng, R=0.75, r=0.25):
    """Torus on an (nu x nv) periodic grid with (u, v) jitter U(-jitter, jitter) * cell.

    Quads (i, j), (i+1, j), (i+1, j+1), (i, j+1) are split on the (i,j)-(i+1,j+1) diagonal.
    """
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    u = (i + rng.uniform(-jitter, jitter, i.shape)) * (2 * np.pi / nu)
    v = (j + rng.uniform(-jitter, jitter, j.shape)) * (2 * np.pi / nv)
    X = np.stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)], -1)
    X = X.reshape(-1, 3)
    idx = lambda a, b: (a % nu) * nv + (b % nv)
    i, j = i.reshape(-1), j.reshape(-1)
    p00, p10, p11, p01 = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
    F = np.concatenate([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)])
    # outward: normal must point away from the tube's core circle
    x0, x1, x2 = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    cen = (x0 + x1 + x2) / 3.0
    core = cen.copy()
    core[:, 2] = 0.0
    core = R * core / np.linalg.norm(core, axis=1, keepdims=True)
    n = np.cross(x1 - x0, x2 - x0)
    flip = np.einsum("ij,ij->i", n, cen - core) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return X, F


def tetrahedron():
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    F = orient_outward(V, np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]]))
    return V, F


def octahedron():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
    F = [(a, b, c) for a in (0, 1) for b in (2, 3) for c in (4, 5)]
    return V, orient_outward(V, np.array(F))


def cube_grid(n: int, half: float = 1.0):
    """Surface of the cube [-half, half]^3, each face an n x n grid of split squares.

    Corner vertices have total angle 3*pi/2; every other vertex is flat (2*pi).
    """
    pts = {}
    X = []
    F = []

    def vid(p):
        key = tuple(int(round(c)) for c in p)
        if key not in pts:
            pts[key] = len(X)
            X.append(key)
        return pts[key]

    for axis in range(3):
        for side in (-n, n):
            a1, a2 = [a for a in range(3) if a != axis]
            for i in range(-n, n, 2):
                for j in range(-n, n, 2):
                    def P(di, dj):
                        p = [0, 0, 0]
                        p[axis] = side
                        p[a1] = i + di
                        p[a2] = j + dj
                        return vid(p)
                    q00, q10, q11, q01 = P(0, 0), P(2, 0), P(2, 2), P(0, 2)
                    F += [(q00, q10, q11), (q00, q11, q01)]
    X = np.array(X, dtype=np.float64) * (half / n)
    return X, orient_outward(X, np.array(F), center=np.zeros(3))


def flat_grid(n: int, jitter: float, rng, size: float = 1.0):
    """Planar (z = 0) n x n grid of split squares with interior vertices jittered in-plane."""
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    x = i.astype(np.float64)
    y = j.astype(np.float64)
    inner = (i > 0) & (i < n) & (j > 0) & (j < n)
    if jitter > 0:
        x[inner] += rng.uniform(-jitter, jitter, inner.sum())
        y[inner] += rng.uniform(-jitter, jitter, inner.sum())
    X = np.stack([x, y, np.zeros_like(x)], -1).reshape(-1, 3) * (size / n)
    idx = lambda a, b: a * (n + 1) + b
    F = []
    for a in range(n):
        for b in range(n):
            p00, p10, p11, p01 = idx(a, b), idx(a + 1, b), idx(a + 1, b + 1), idx(a, b + 1)
            if (a + b) % 2 == 0:
                F += [(p00, p10, p11), (p00, p11, p01)]
            else:
                F += [(p00, p10, p01), (p10, p11, p01)]
    return X, np.array(F, dtype=np.int64)


def prism(nsides: int, nrings: int, radius: float = 1.0, height: float = 2.0):
    """Open polygonal prism (developable cylinder), vertices on nsides x (nrings+1) rings.

    Returns (X, F, meta) where meta gives the facet width and ring spacing for
    the development (unrolled) coordinates (s, z).
    """
    k, r = np.meshgrid(np.arange(nsides), np.arange(nrings + 1), indexing="ij")
    ang = 2 * np.pi * k / nsides
    z = -height / 2 + height * r / nrings
    X = np.stack([radius * np.cos(ang), radius * np.sin(ang), z], -1).reshape(-1, 3)
    idx = lambda a, b: (a % nsides) * (nrings + 1) + b
    F = []
    for a in range(nsides):
        for b in range(nrings):
            p00, p10, p11, p01 = idx(a, b), idx(a + 1, b), idx(a + 1, b + 1), idx(a, b + 1)
            F += [(p00, p10, p11), (p00, p11, p01)]
    F = np.array(F, dtype=np.int64)
    x0, x1, x2 = X[F[:, 0]], X[F[:, 1]], X[F[:, 2]]
    cen = (x0 + x1 + x2) / 3.0
    cen[:, 2] = 0
    n = np.cross(x1 - x0, x2 - x0)
    flip = np.einsum("ij,ij->i", n, cen) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    meta = dict(facet=2 * radius * np.sin(np.pi / nsides), dz=height / nrings,
                nsides=nsides, radius=radius, height=height)
    return X, F, meta


def plane_with_hole(n: int, size: float, origin, hole_lo, hole_hi):
    """Flat n x n grid of split squares over [origin, origin + size]^2 with the
    faces whose centroids lie inside the square [hole_lo, hole_hi]^2 removed
    (a square hole when its sides fall on grid lines)."""
    X, F = flat_grid(n, 0.0, None, size=size)
    X = X + np.array([origin, origin, 0.0])
    c = X[F].mean(1)
    inside = np.all((c[:, :2] > hole_lo) & (c[:, :2] < hole_hi), axis=1)
    return remove_faces(X, F, np.where(inside)[0])


def remove_faces(X, F, faces):
    """Drop the listed faces (used to punch holes for boundary tests)."""
    keep = np.ones(F.shape[0], dtype=bool)
    keep[np.asarray(faces, dtype=np.int64)] = False
    return X, F[keep]
