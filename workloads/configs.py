"""The five benchmark workloads (synthetic stand-ins for the paper's meshes).

Seeds are numpy default_rng(1000*c + s) with s = 0 (mesh), 1 (rays),
2 (upstream gradient), 3 (vertex perturbation).

  1  icosphere level 3 (1,280 faces), 8,192 rays, |v| ~ U[0, pi/2], K = 1
  2  icosphere level 7 (327,680 faces) with SH displacement (l <= 8, amplitude 0.1),
     1,048,576 rays, |v| ~ U[0, pi/2], K = 2
  3  64 meshes (displaced geodesic spheres and 3:1 jittered tori), F log-uniform in
     [5e3, 5e5], rays per mesh log-uniform in [16k, 256k], lengths log-uniform in
     [0.01, 1] x mesh diameter, K = 0
  4  config-2 mesh and rays with K = 0, upstream gradient g ~ N(0, I3)
  5  icosphere level 8 (1,310,720 faces), SH l <= 32 plus normal noise 0.1 x mean edge,
     16,777,216 rays, |v| ~ U[0, pi], K = 2 (start frame)
"""
from __future__ import annotations

import numpy as np

from . import meshes as M
from .rays import random_rays, uniform_len, loguniform_len

__all__ = ["rng", "mesh_config", "rays_config", "config3_meshes", "upstream_grad"]


def rng(c: int, s: int):
    return np.random.default_rng(1000 * c + s)


def mesh_config(c: int):
    """Canonical (X f32, F i32) of configs 1, 2 (= 4) and 5."""
    if c == 1:
        X, F = M.icosphere(3)
    elif c in (2, 4):
        X, F = M.icosphere(7)
        X = M.sh_displace(X, 8, 0.1, rng(2, 0))
    elif c == 5:
        X, F = M.icosphere(8)
        g = rng(5, 0)
        X = M.sh_displace(X, 32, 0.1, g)
        X = M.normal_noise(X, F, 0.1, g)
    else:
        raise ValueError(c)
    return M.canonical(X, F)


def rays_config(c: int, X, F, n=None, seed_offset=0):
    """Rays of configs 1, 2, 4, 5 (n overrides the count; same law)."""
    g = np.random.default_rng(1000 * c + 1 + 100 * seed_offset)
    if c == 1:
        return random_rays(X, F, n or 8192, g, uniform_len(0.0, np.pi / 2), K=1)
    if c == 2:
        return random_rays(X, F, n or 1 << 20, g, uniform_len(0.0, 0.5 * np.pi), K=2)
    if c == 4:
        return random_rays(X, F, n or 1 << 20, g, uniform_len(0.0, 0.5 * np.pi), K=0)
    if c == 5:
        return random_rays(X, F, n or 1 << 24, g, uniform_len(0.0, np.pi), K=2, frame_vectors=True)
    raise ValueError(c)


def upstream_grad(c: int, n: int):
    return rng(c, 2).normal(0.0, 1.0, (n, 3)).astype(np.float32)


def config3_meshes(n_meshes: int = 64, scale: float = 1.0):
    """Specs and canonical meshes of config 3 (scale < 1 shrinks face and ray counts)."""
    g = rng(3, 0)
    out = []
    for i in range(n_meshes):
        Fi = float(np.exp(g.uniform(np.log(5e3), np.log(5e5)))) * scale
        kind = "sphere" if g.uniform() < 0.5 else "torus"
        if kind == "sphere":
            freq = max(2, int(round(np.sqrt(Fi / 20.0))))
            X, F = M.geodesic_sphere(freq)
            X = M.sh_displace(X, 8, 0.1, g)
        else:
            nv = max(3, int(round(np.sqrt(Fi / 6.0))))
            X, F = M.torus_grid(3 * nv, nv, 0.2, g)
        X, F = M.canonical(X, F)
        c = X.astype(np.float64).mean(0)
        D = 2.0 * float(np.linalg.norm(X.astype(np.float64) - c, axis=1).max())
        R = int(np.exp(g.uniform(np.log(16384), np.log(262144))) * scale)
        out.append(dict(kind=kind, X=X, F=F, n_rays=max(R, 1), diameter=D))
    return out


def config3_rays(spec, i: int):
    g = np.random.default_rng(1000 * 3 + 1 + 7919 * i)
    D = spec["diameter"]
    return random_rays(spec["X"], spec["F"], spec["n_rays"], g, loguniform_len(0.01 * D, D), K=0)


def config3_batch(n_meshes: int = 64, scale: float = 1.0):
    """Config 3 as one batch: concatenated vertices, faces with local vertex ids,
    vertex / face offsets (prefix sums), faces with global vertex ids, and the
    rays of all meshes with global face ids; `slices` gives each mesh's rays."""
    specs = config3_meshes(n_meshes, scale)
    vo, fo, ro = [0], [0], [0]
    for s in specs:
        vo.append(vo[-1] + s["X"].shape[0])
        fo.append(fo[-1] + s["F"].shape[0])
        ro.append(ro[-1] + s["n_rays"])
    X = np.concatenate([s["X"] for s in specs])
    F_local = np.concatenate([s["F"] for s in specs])
    F_global = np.concatenate([s["F"] + vo[i] for i, s in enumerate(specs)]).astype(np.int32)
    rays = [config3_rays(s, i) for i, s in enumerate(specs)]
    r = {k: np.concatenate([ri[k] + (fo[i] if k == "f" else 0) for i, ri in enumerate(rays)]).astype(rays[0][k].dtype)
         for k in ("f", "b", "v")}
    r["W"] = np.zeros((r["f"].shape[0], 0, 3), np.float32)
    return dict(specs=specs, X=X, F_local=F_local, F_global=F_global, vert_offsets=np.array(vo, np.int64),
                face_offsets=np.array(fo, np.int64), rays=r,
                slices=[slice(ro[i], ro[i + 1]) for i in range(len(specs))])
