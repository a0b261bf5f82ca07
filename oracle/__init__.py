"""Float64 CPU oracle for the straightest-geodesic exponential map.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.  The
tracer is plain C (sg_oracle.c) following the paper's extrinsic algorithms
(geodesic_step, transport_over_edge, transport_over_vertex, Alg. gpu_parallel)
and its two backward schemes (eq. proxy_func, eqs. jv/jp).  This module only
marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

RAY_OK, RAY_MAXSTEPS, RAY_BOUNDARY, RAY_BADINPUT = 0, 1, 2, 3
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        L.or_mesh_build.argtypes = [P, C.c_int64, P, C.c_int64, C.POINTER(C.c_void_p)]
        L.or_mesh_build.restype = C.c_int
        L.or_mesh_build64.argtypes = [P, C.c_int64, P, C.c_int64, C.POINTER(C.c_void_p)]
        L.or_mesh_build64.restype = C.c_int
        L.or_mesh_free.argtypes = [P]
        L.or_mesh_mean_edge.argtypes = [P]
        L.or_mesh_mean_edge.restype = C.c_double
        L.or_mesh_theta.argtypes = [P, P]
        L.or_last_error.restype = C.c_char_p
        L.or_exp_batch.argtypes = [P, C.c_int64, P, P, P, C.c_int32, P, P] + [P] * 13 + [C.c_int32]
        L.or_exp_batch.restype = C.c_int
        L.or_exp_trace.argtypes = [P, C.c_int32, P, P, P, C.c_int32] + [P] * 8
        L.or_exp_trace.restype = C.c_int32
        L.or_ep_batch.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, C.c_int32]
        L.or_ep_batch.restype = C.c_int
        L.or_gfd_batch.argtypes = [P, C.c_int64, P, P, P, P, C.c_double, C.c_double, P, P, P, P, P, C.c_int32]
        L.or_gfd_batch.restype = C.c_int
        L.or_transport_vjp.argtypes = [P, C.c_int64, P, P, P, P, C.c_int32, P, P, P, P, C.c_int32]
        L.or_transport_vjp.restype = C.c_int
        L.or_gradx_batch.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, C.c_int32]
        L.or_gradx_batch.restype = C.c_int
        L.or_pi_exp_batch.argtypes = [P, C.c_int64, P, P, P, C.c_int32, P, P] + [P] * 9 + [C.c_int32]
        L.or_pi_exp_batch.restype = C.c_int
        L.or_pi_project.argtypes = [P, C.c_int64, P, P, P, P, P]
        L.or_pi_project.restype = C.c_int
        L.or_pi_ep_batch.argtypes = [P, C.c_int64, P, P, P, P, P, P, P, C.c_int32]
        L.or_pi_ep_batch.restype = C.c_int
        L.or_pi_gfd_batch.argtypes = [P, C.c_int64, P, P, P, P, C.c_double, C.c_double, P, P, P, P, P, C.c_int32]
        L.or_pi_gfd_batch.restype = C.c_int
        _lib = L
    return _lib


class Opts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("vertex_snap", C.c_double), ("boundary_mode", C.c_int32)]


class PiOpts(C.Structure):
    _fields_ = [("step", C.c_double), ("max_steps", C.c_int32)]


PI_STEP = 0.01   # default s of the projection-integration Exp


def pi_max_steps(step):
    """Default step cap of the projection-integration Exp: 8 / s."""
    return int(np.ceil(8.0 / step))


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Mesh:
    """Oracle mesh built from the canonical float32 (X, F); exact64=True keeps
    float64 positions as given (used for central differences in X)."""

    def __init__(self, X, F, exact64=False):
        L = lib()
        self.X = np.ascontiguousarray(X, dtype=np.float64 if exact64 else np.float32)
        self.F = np.ascontiguousarray(F, dtype=np.int32)
        h = C.c_void_p()
        build = L.or_mesh_build64 if exact64 else L.or_mesh_build
        rc = build(_p(self.X), self.X.shape[0], _p(self.F), self.F.shape[0], C.byref(h))
        if rc != 0:
            raise OracleError(rc, L.or_last_error().decode())
        self._h = h
        self.nv, self.nf = self.X.shape[0], self.F.shape[0]

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_mesh_free(self._h)
            self._h = None

    @property
    def mean_edge(self):
        return lib().or_mesh_mean_edge(self._h)

    def theta(self):
        t = np.zeros(self.nv)
        lib().or_mesh_theta(self._h, _p(t))
        return t

    @staticmethod
    def opts(max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0):
        return Opts(max_steps, vertex_snap, boundary_mode)

    def exp(self, f, b, v, W=None, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0, nthreads=0):
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        if W is None:
            W = np.zeros((n, 0, 3))
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(n, -1, 3)
        K = W.shape[1]
        out = dict(
            f=np.zeros(n, np.int32), b=np.zeros((n, 3)), p=np.zeros((n, 3)), v=np.zeros((n, 3)),
            W=np.zeros((n, K, 3)), status=np.zeros(n, np.int32), n_cross=np.zeros(n, np.int32),
            hash=np.zeros(n, np.uint64), min_vdist=np.zeros(n), traced=np.zeros(n),
            sigma=np.zeros(n, np.int8), n_bnd=np.zeros(n, np.int32), bnd_margin=np.zeros(n))
        o = Opts(max_steps, vertex_snap, boundary_mode)
        rc = lib().or_exp_batch(
            self._h, n, _p(f), _p(b), _p(v), K, _p(W) if K else None, C.byref(o),
            _p(out["f"]), _p(out["b"]), _p(out["p"]), _p(out["v"]), _p(out["W"]) if K else None,
            _p(out["status"]), _p(out["n_cross"]), _p(out["hash"]), _p(out["min_vdist"]),
            _p(out["traced"]), _p(out["sigma"]), _p(out["n_bnd"]), _p(out["bnd_margin"]), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return out

    def trace(self, f, b, v, cap=100000, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0):
        kind = np.zeros(cap, np.int8)
        face = np.zeros(cap, np.int32)
        e0 = np.zeros(cap, np.int32)
        e1 = np.zeros(cap, np.int32)
        pt = np.zeros((cap, 3))
        fo = C.c_int32()
        st = C.c_int32()
        po = np.zeros(3)
        b = np.ascontiguousarray(b, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        o = Opts(max_steps, vertex_snap, boundary_mode)
        k = lib().or_exp_trace(self._h, int(f), _p(b), _p(v), C.byref(o), cap, _p(kind), _p(face),
                               _p(e0), _p(e1), _p(pt), C.byref(fo), _p(po), C.byref(st))
        return dict(kind=kind[:k], face=face[:k], e0=e0[:k], e1=e1[:k], point=pt[:k],
                    f=fo.value, p=po, status=st.value)

    def ep(self, f, b, v, g, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0, nthreads=0):
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(n, 3)
        gv = np.zeros((n, 3))
        gb = np.zeros((n, 3))
        o = Opts(max_steps, vertex_snap, boundary_mode)
        rc = lib().or_ep_batch(self._h, n, _p(f), _p(b), _p(v), C.byref(o), _p(g), _p(gv), _p(gb), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return gv, gb

    def gfd(self, f, b, v, g, eps_v, eps_p, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0, nthreads=0):
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(n, 3)
        gv = np.zeros((n, 3))
        gb = np.zeros((n, 3))
        Jv = np.zeros((n, 2, 2))
        Jp = np.zeros((n, 2, 2))
        o = Opts(max_steps, vertex_snap, boundary_mode)
        rc = lib().or_gfd_batch(self._h, n, _p(f), _p(b), _p(v), C.byref(o), float(eps_v), float(eps_p),
                                _p(g), _p(gv), _p(gb), _p(Jv), _p(Jp), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return dict(grad_v=gv, grad_b=gb, Jv=Jv, Jp=Jp)

    def transport_vjp(self, f, b, v, g_v=None, g_W=None, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0,
                      nthreads=0):
        """(dL/dv from g_v = dL/dv', dL/dW [n,K,3] from g_W = dL/dW') through the transport."""
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        gv_in = None if g_v is None else np.ascontiguousarray(g_v, dtype=np.float64).reshape(n, 3)
        gW = np.zeros((n, 0, 3)) if g_W is None else np.ascontiguousarray(g_W, dtype=np.float64).reshape(n, -1, 3)
        K = gW.shape[1]
        gv = np.zeros((n, 3))
        gWo = np.zeros((n, K, 3))
        o = Opts(max_steps, vertex_snap, boundary_mode)
        rc = lib().or_transport_vjp(self._h, n, _p(f), _p(b), _p(v), C.byref(o), K, _p(gv_in),
                                    _p(gW) if K else None, _p(gv), _p(gWo) if K else None, nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return gv, gWo

    def gradx(self, f, b, v, g, max_steps=1 << 20, vertex_snap=1e-10, boundary_mode=0, nthreads=0):
        """(dL/dX [nv,3] float64, vertex passages per ray (-1: status not OK)) for L = sum g . p'."""
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(n, 3)
        gx = np.zeros((self.nv, 3))
        nvx = np.zeros(n, np.int32)
        o = Opts(max_steps, vertex_snap, boundary_mode)
        rc = lib().or_gradx_batch(self._h, n, _p(f), _p(b), _p(v), C.byref(o), _p(g), _p(gx), _p(nvx), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return gx, nvx

    def exp_iterated(self, f, b, field, steps, **kw):
        """The K-step exponential map of the paper's flow-matching objective (eq. fmobj, Sec. "MeshFlow"):
        p^(k+1) = Exp_{p^(k)}(field(p^(k)) / K) for k = 0 .. K-1, the field re-evaluated at every
        intermediate point.  Composed from `exp` alone; field(p [n,3], f [n], b [n,3]) -> v [n,3]
        (float64).  Returns the last step's f, b, p, v, status, every intermediate point (`pts`, K of
        them, with their faces `fs` and barycentrics `bs`, and the start point's face and barycentrics
        first in `fs`, `bs`) and the smallest vertex distance over all steps (`min_vdist`)."""
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        o = self.exp(f, b, np.zeros((n, 3)), **kw)   # p^(0) = sum_k b_k x_k
        p, b = o["p"], o["b"]
        pts, mvd, status = [], np.full(n, np.inf), np.zeros(n, np.int32)
        fs, bs = [f.copy()], [b.copy()]
        for _ in range(int(steps)):
            v = np.asarray(field(p, f, b), dtype=np.float64) / float(steps)
            o = self.exp(f, b, v, **kw)
            f, b, p = o["f"], o["b"], o["p"]
            mvd = np.minimum(mvd, o["min_vdist"])
            status = np.where(status != 0, status, o["status"])
            pts.append(p)
            fs.append(f.copy())
            bs.append(b.copy())
        return dict(f=f, b=b, p=p, v=o["v"], status=status, pts=pts, fs=fs, bs=bs, min_vdist=mvd)

    # ---- projection integration (appendix "Projection Integration Exp Map", Alg. projection-exp)
    def _pi_opts(self, step, max_steps):
        return PiOpts(float(step), int(pi_max_steps(step) if max_steps is None else max_steps))

    def pi_exp(self, f, b, v, W=None, step=PI_STEP, max_steps=None, nthreads=0):
        """The PI exponential map: f, b, p, v, W, status, n_steps, traced, margin (float64)."""
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        if W is None:
            W = np.zeros((n, 0, 3))
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(n, -1, 3)
        K = W.shape[1]
        out = dict(f=np.zeros(n, np.int32), b=np.zeros((n, 3)), p=np.zeros((n, 3)), v=np.zeros((n, 3)),
                   W=np.zeros((n, K, 3)), status=np.zeros(n, np.int32), n_steps=np.zeros(n, np.int32),
                   traced=np.zeros(n), margin=np.zeros(n))
        o = self._pi_opts(step, max_steps)
        rc = lib().or_pi_exp_batch(self._h, n, _p(f), _p(b), _p(v), K, _p(W) if K else None, C.byref(o),
                                   _p(out["f"]), _p(out["b"]), _p(out["p"]), _p(out["v"]),
                                   _p(out["W"]) if K else None, _p(out["status"]), _p(out["n_steps"]),
                                   _p(out["traced"]), _p(out["margin"]), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return out

    def pi_project(self, q):
        """project_to_mesh of points q [n,3]: (face, nearest point, barycentrics, margin)."""
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
        n = q.shape[0]
        f = np.zeros(n, np.int32)
        c = np.zeros((n, 3))
        bc = np.zeros((n, 3))
        mg = np.zeros(n)
        rc = lib().or_pi_project(self._h, n, _p(q), _p(f), _p(c), _p(bc), _p(mg))
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return f, c, bc, mg

    def pi_ep(self, f, b, v, g, step=PI_STEP, max_steps=None, nthreads=0):
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(n, 3)
        gv = np.zeros((n, 3))
        gb = np.zeros((n, 3))
        o = self._pi_opts(step, max_steps)
        rc = lib().or_pi_ep_batch(self._h, n, _p(f), _p(b), _p(v), C.byref(o), _p(g), _p(gv), _p(gb), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return gv, gb

    def pi_gfd(self, f, b, v, g, eps_v, eps_p, step=PI_STEP, max_steps=None, nthreads=0):
        f = np.ascontiguousarray(f, dtype=np.int32).reshape(-1)
        n = f.shape[0]
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(n, 3)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(n, 3)
        gv = np.zeros((n, 3))
        gb = np.zeros((n, 3))
        Jv = np.zeros((n, 2, 2))
        Jp = np.zeros((n, 2, 2))
        o = self._pi_opts(step, max_steps)
        rc = lib().or_pi_gfd_batch(self._h, n, _p(f), _p(b), _p(v), C.byref(o), float(eps_v), float(eps_p),
                                   _p(g), _p(gv), _p(gb), _p(Jv), _p(Jp), nthreads)
        if rc != 0:
            raise OracleError(rc, lib().or_last_error().decode())
        return dict(grad_v=gv, grad_b=gb, Jv=Jv, Jp=Jp)
