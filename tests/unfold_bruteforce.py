"""Brute-force planar unfolding: an independent check of straight paths on tiny meshes.

Uses only edge lengths (intrinsic data).  From the start face, every face path
is explored by laying the next triangle out in the plane from its three edge
lengths; a path is kept if the straight 2D segment crosses its shared edges in
order and ends inside its last triangle.  Both non-entry edges of every face
are tried, so the search does not rely on any exit formula.  Valid away from
vertices (the segment must not pass through a vertex), which is where a
straightest geodesic coincides with the unfolded straight line.
"""
from __future__ import annotations

import numpy as np


def _edge_faces(F):
    ef = {}
    for f, t in enumerate(F):
        for k in range(3):
            a, b = int(t[k]), int(t[(k + 1) % 3])
            ef.setdefault((min(a, b), max(a, b)), []).append(f)
    return ef


def _place(A, B, la, lb, side):
    """2D point C with |AC| = la, |BC| = lb on `side` (+1 left, -1 right) of A->B."""
    d = np.linalg.norm(B - A)
    ex = (B - A) / d
    ey = np.array([-ex[1], ex[0]])
    x = (la * la - lb * lb + d * d) / (2 * d)
    y = np.sqrt(max(la * la - x * x, 0.0))
    return A + x * ex + side * y * ey


def _cross2(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _hit(P0, D, A, B):
    """Segment P0 + t D against edge A + s (B - A): returns (t, s) or None if parallel."""
    E = B - A
    den = _cross2(D, E)
    if abs(den) < 1e-300:
        return None
    w = A - P0
    return _cross2(w, E) / den, _cross2(w, D) / den


def unfold_path(X, F, f0, b, v, max_depth=14):
    """All face paths whose development contains the straight segment of (f0, b, v).

    Returns a list of (faces, endpoint3d).  A well-posed ray away from
    vertices has exactly one.
    """
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    ef = _edge_faces(F)
    lens = lambda i, j: float(np.linalg.norm(X[i] - X[j]))
    t0 = F[f0]
    l01, l02, l12 = lens(t0[0], t0[1]), lens(t0[0], t0[2]), lens(t0[1], t0[2])
    P = {int(t0[0]): np.zeros(2), int(t0[1]): np.array([l01, 0.0])}
    P[int(t0[2])] = _place(P[int(t0[0])], P[int(t0[1])], l02, l12, +1)
    x0, x1, x2 = X[t0[0]], X[t0[1]], X[t0[2]]
    e1 = (x1 - x0) / np.linalg.norm(x1 - x0)
    n = np.cross(x1 - x0, x2 - x0)
    n /= np.linalg.norm(n)
    e2 = np.cross(n, e1)
    D = np.array([np.dot(v, e1), np.dot(v, e2)])
    L = float(np.linalg.norm(D))
    D = D / L
    bb = np.asarray(b, dtype=np.float64) / np.sum(b)
    p0 = bb[0] * P[int(t0[0])] + bb[1] * P[int(t0[1])] + bb[2] * P[int(t0[2])]
    found = []

    def inside(face_layout, q):
        A, B, Cc = face_layout
        M = np.column_stack([B - A, Cc - A])
        l1, l2 = np.linalg.solve(M, q - A)
        return min(1 - l1 - l2, l1, l2) >= -1e-12, np.array([1 - l1 - l2, l1, l2])

    def rec(face, layout, entry, t_in, path):
        tri = F[face]
        A, B, Cc = layout[int(tri[0])], layout[int(tri[1])], layout[int(tri[2])]
        end = p0 + L * D
        ok, bar = inside((A, B, Cc), end)
        exits = []
        for k in range(3):
            a, c = int(tri[k]), int(tri[(k + 1) % 3])
            key = (min(a, c), max(a, c))
            if key == entry:
                continue
            h = _hit(p0, D, layout[a], layout[c])
            if h is None:
                continue
            t, s = h
            if t > t_in + 1e-14 and 0.0 <= s <= 1.0:
                exits.append((t, key, a, c))
        if ok and all(t >= L for t, *_ in exits):
            found.append((list(path), bar[0] * X[tri[0]] + bar[1] * X[tri[1]] + bar[2] * X[tri[2]]))
        if len(path) > max_depth:
            return
        for t, key, a, c in exits:
            if t >= L:
                continue
            nb = [g for g in ef[key] if g != face]
            if not nb:
                continue
            g = nb[0]
            tg = F[g]
            z = [int(q) for q in tg if int(q) not in key][0]
            # the new triangle goes on the far side of the crossed edge
            third_old = [int(q) for q in tri if int(q) not in key][0]
            side_old = np.sign(_cross2(layout[c] - layout[a], layout[third_old] - layout[a]))
            lay = dict(layout)
            lay[z] = _place(layout[a], layout[c], lens(a, z), lens(c, z), -side_old)
            rec(g, lay, key, t, path + [g])

    rec(f0, P, None, 0.0, [f0])
    return found
