"""Seeded ray batches (start face, barycentric point, tangent vector, extra vectors).

The law follows the benchmark configurations: start faces uniform by index,
barycentrics Dirichlet(1,1,1), tangent angle uniform in [0, 2 pi) measured in
the start face from e1 = unit(x1 - x0) towards e2 = n x e1, and a length drawn
by a caller-supplied law.  Vectors are built in float64 from the canonical
float32 mesh and rounded once to float32.  Draw order is fixed (faces,
barycentrics, angle, length, extra-vector angles) so a seed names a batch.
"""
from __future__ import annotations

import numpy as np

__all__ = ["face_frames", "random_rays", "uniform_len", "loguniform_len"]


def face_frames(X, F, f):
    """(e1, e2, n) per face in float64: e1 = unit(x1-x0), n = unit normal, e2 = n x e1."""
    X = np.asarray(X, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    x0, x1, x2 = X[F[f, 0]], X[F[f, 1]], X[F[f, 2]]
    e1 = x1 - x0
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    n = np.cross(x1 - x0, x2 - x0)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    e2 = np.cross(n, e1)
    return e1, e2, n


def uniform_len(lo, hi):
    return lambda rng, n: rng.uniform(lo, hi, n)


def loguniform_len(lo, hi):
    return lambda rng, n: np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def random_rays(X, F, n, rng, length_law, K=0, frame_vectors=False, faces=None):
    """Returns dict(f int32[n], b f32[n,3], v f32[n,3], W f32[n,K,3], angle, length).

    With frame_vectors=True, K must be 2 and W is the start frame (e1, e2).
    `faces`, if given, restricts start faces to that index set (uniform over it).
    """
    nf = F.shape[0]
    if faces is None:
        f = rng.integers(0, nf, n)
    else:
        faces = np.asarray(faces)
        f = faces[rng.integers(0, faces.shape[0], n)]
    b = rng.dirichlet([1.0, 1.0, 1.0], n)
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    L = length_law(rng, n)
    e1, e2, _ = face_frames(X, F, f)
    v = L[:, None] * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
    if frame_vectors:
        assert K == 2
        W = np.stack([e1, e2], 1)
    elif K > 0:
        a = rng.uniform(0.0, 2.0 * np.pi, (n, K))
        W = np.cos(a)[..., None] * e1[:, None] + np.sin(a)[..., None] * e2[:, None]
    else:
        W = np.zeros((n, 0, 3))
    return dict(
        f=f.astype(np.int32),
        b=b.astype(np.float32),
        v=v.astype(np.float32),
        W=np.ascontiguousarray(W, dtype=np.float32),
        angle=ang,
        length=L,
    )
