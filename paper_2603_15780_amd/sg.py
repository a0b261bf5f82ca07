"""Python binding of libsg.so (include/sg.h): argument marshalling only.

Every step of the exponential map runs in the library's gfx950 kernels.
PyTorch supplies device memory and the current HIP stream.  If the library
is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

SG_OK = 0
SG_E_ARG, SG_E_NONMANIFOLD, SG_E_DEGENERATE, SG_E_HIP, SG_E_OOM = -1, -2, -3, -4, -5
RAY_OK, RAY_MAXSTEPS, RAY_BOUNDARY, RAY_BADINPUT = 0, 1, 2, 3
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_PERSISTENT, KERNEL_PARTITIONED = 0, 1, 2, 3
BWD_EP, BWD_GFD = 0, 1
BOUNDARY_STOP, BOUNDARY_AVOID = 0, 1
PI_GRID, PI_SCAN = 0, 1

_lib = None


class SgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sg error {code}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("max_steps", C.c_int32), ("vertex_snap", C.c_float), ("eps_v", C.c_float),
                ("eps_p", C.c_float), ("kernel", C.c_int32), ("debug", C.c_uint32),
                ("refill_min", C.c_int32), ("walk_blocks", C.c_int32), ("rays_per_lane", C.c_int32),
                ("ray_queues", C.c_int32), ("boundary_mode", C.c_int32), ("gradx_records", C.c_int32),
                ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64)]


class PiOpts(C.Structure):
    _fields_ = [("step", C.c_float), ("max_steps", C.c_int32), ("search", C.c_int32)]


def lib_path() -> str:
    return _build.LIB


def lib():
    """Loads libsg.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise ImportError(f"libsg.so not built at {_build.LIB}; run __graft_entry__.build()")
        L = C.CDLL(_build.LIB)
        P, I64, I32 = C.c_void_p, C.c_int64, C.c_int32
        L.sg_last_error.restype = C.c_char_p
        L.sg_opts_default.argtypes = [C.POINTER(Opts)]
        L.sg_mesh_create.argtypes = [P, I64, P, I64, P, P, I32, C.POINTER(C.c_void_p)]
        L.sg_mesh_create.restype = C.c_int
        L.sg_mesh_destroy.argtypes = [P]
        L.sg_mesh_update_vertices.argtypes = [P, P, I64]
        L.sg_mesh_update_vertices.restype = C.c_int
        L.sg_mesh_info.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
        L.sg_mesh_info.restype = C.c_int
        L.sg_exp.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P, C.POINTER(Opts), P]
        L.sg_exp.restype = C.c_int
        L.sg_exp_transport.argtypes = [P, I64, P, P, P, I32, P, P, P, P, P, P, P, P, P, C.POINTER(Opts), P]
        L.sg_exp_transport.restype = C.c_int
        L.sg_exp_transport_noalloc.argtypes = L.sg_exp_transport.argtypes
        L.sg_exp_transport_noalloc.restype = C.c_int
        L.sg_exp_backward.argtypes = [P, I32, I64, P, P, P, P, P, P, P, P, P, P, P, C.POINTER(Opts), P]
        L.sg_exp_backward.restype = C.c_int
        L.sg_exp_backward_transport.argtypes = [P, I32, I64, P, P, P, I32, P, P, P, P, P, P, P, P, P, P, P, P,
                                                C.POINTER(Opts), P]
        L.sg_exp_backward_transport.restype = C.c_int
        L.sg_exp_workspace_size.argtypes = [P, I64, I32, C.POINTER(Opts), C.POINTER(C.c_size_t)]
        L.sg_exp_workspace_size.restype = C.c_int
        L.sg_backward_workspace_size.argtypes = [P, I32, I64, I32, I32, C.POINTER(Opts), C.POINTER(C.c_size_t)]
        L.sg_backward_workspace_size.restype = C.c_int
        L.sg_autotune.argtypes = [P, I64, P, P, P, I32, P, C.POINTER(Opts), C.POINTER(C.c_double), P]
        L.sg_autotune.restype = C.c_int
        L.sg_pi_opts_default.argtypes = [C.POINTER(PiOpts)]
        L.sg_pi_exp.argtypes = [P, I64, P, P, P, I32, P, P, P, P, P, P, P, P, C.POINTER(PiOpts), P]
        L.sg_pi_exp.restype = C.c_int
        L.sg_pi_backward.argtypes = [P, I32, I64, P, P, P, P, P, P, P, P, C.POINTER(PiOpts), C.POINTER(Opts), P]
        L.sg_pi_backward.restype = C.c_int
        L.sg_pi_backward_workspace_size.argtypes = [P, I32, I64, C.POINTER(C.c_size_t)]
        L.sg_pi_backward_workspace_size.restype = C.c_int
        L.sg_mesh_walk_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.sg_mesh_walk_time.restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != SG_OK:
        raise SgError(rc, lib().sg_last_error().decode())


def opts(**kw) -> Opts:
    o = Opts()
    lib().sg_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def pi_opts(step=None, max_steps=None, search=None) -> PiOpts:
    o = PiOpts()
    lib().sg_pi_opts_default(C.byref(o))
    if step is not None:
        o.step = step
    if max_steps is not None:
        o.max_steps = max_steps
    if search is not None:
        o.search = search
    return o


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A packed mesh handle (one or several meshes batched by offsets)."""

    def __init__(self, X, F, vert_offsets=None, face_offsets=None):
        L = lib()
        X = np.ascontiguousarray(X, dtype=np.float32)
        F = np.ascontiguousarray(F, dtype=np.int32)
        h = C.c_void_p()
        if vert_offsets is None:
            rc = L.sg_mesh_create(_np_ptr(X), X.shape[0], _np_ptr(F), F.shape[0], None, None, 1, C.byref(h))
        else:
            vo = np.ascontiguousarray(vert_offsets, dtype=np.int64)
            fo = np.ascontiguousarray(face_offsets, dtype=np.int64)
            rc = L.sg_mesh_create(_np_ptr(X), X.shape[0], _np_ptr(F), F.shape[0], _np_ptr(vo), _np_ptr(fo),
                                  vo.shape[0] - 1, C.byref(h))
        _check(rc)
        self._h = h
        self.n_verts, self.n_faces = X.shape[0], F.shape[0]

    def close(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and _lib is not None:
            _lib.sg_mesh_destroy(h)

    __del__ = close

    def update_vertices(self, X):
        """New vertex positions (numpy or torch [n_verts, 3], same connectivity);
        synchronous (waits for the device to be idle)."""
        if hasattr(X, "detach"):
            X = X.detach().cpu().numpy()
        X = np.ascontiguousarray(X, dtype=np.float32)
        if X.shape != (self.n_verts, 3):
            raise ValueError(f"X must be [{self.n_verts}, 3]")
        _check(lib().sg_mesh_update_vertices(self._h, _np_ptr(X), X.shape[0]))

    def info(self):
        me = C.c_double()
        nh = C.c_int64()
        nb = C.c_size_t()
        _check(lib().sg_mesh_info(self._h, C.byref(me), C.byref(nh), C.byref(nb)))
        return dict(mean_edge=me.value, n_half_edges=nh.value, device_bytes=nb.value)

    def exp_workspace_size(self, n, K=0, o: Opts | None = None, **kw):
        o = o if o is not None else opts(**kw)
        nb = C.c_size_t()
        _check(lib().sg_exp_workspace_size(self._h, n, int(K), C.byref(o), C.byref(nb)))
        return nb.value

    def backward_workspace_size(self, mode, n, want_vjp=True, want_grad_X=False, o: Opts | None = None, **kw):
        o = o if o is not None else opts(**kw)
        nb = C.c_size_t()
        _check(lib().sg_backward_workspace_size(self._h, int(mode), n, int(want_vjp), int(want_grad_X), C.byref(o),
                                                C.byref(nb)))
        return nb.value

    def autotune(self, f, b, v, W=None, o: Opts | None = None, **kw):
        """Opts with the fastest forward schedule for this batch, and its time per call (ms)."""
        o = o if o is not None else opts(**kw)
        K = 0 if W is None else W.shape[1]
        ms = C.c_double()
        _check(lib().sg_autotune(self._h, f.shape[0], _dptr(f), _dptr(b), _dptr(v), K, _dptr(W), C.byref(o),
                                 C.byref(ms), _stream()))
        return o, ms.value

    def walk_time(self):
        """(summed ms, launches) of walk kernels timed with debug bit 2 since the last call."""
        ms = C.c_double()
        cnt = C.c_int64()
        _check(lib().sg_mesh_walk_time(self._h, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def exp(self, f, b, v, W=None, *, out=None, want_status=True, want_cross=False, want_hash=False,
            noalloc=False, o: Opts | None = None, **kw):
        """Exp_p(v) for torch CUDA tensors f[n] int32, b[n,3], v[n,3] (float32), W[n,K,3].

        noalloc=True calls sg_exp_transport_noalloc (the library's fixed
        scratch instead of a workspace allocation; pass `out` to allocate
        nothing here either)."""
        import torch
        n = f.shape[0]
        dev = f.device
        assert f.dtype == torch.int32 and b.dtype == torch.float32 and v.dtype == torch.float32
        assert f.is_contiguous() and b.is_contiguous() and v.is_contiguous()
        assert b.shape == (n, 3) and v.shape == (n, 3)
        K = 0 if W is None else W.shape[1]
        if W is not None:
            assert W.dtype == torch.float32 and W.is_contiguous() and W.shape == (n, K, 3)
        if o is None:
            o = opts(**kw)
        if want_cross:
            o.debug |= 1
        if want_hash:
            o.debug |= 2
        if out is None:
            out = dict(
                f=torch.empty(n, dtype=torch.int32, device=dev),
                b=torch.empty(n, 3, dtype=torch.float32, device=dev),
                p=torch.empty(n, 3, dtype=torch.float32, device=dev),
                v=torch.empty(n, 3, dtype=torch.float32, device=dev),
                W=torch.empty(n, K, 3, dtype=torch.float32, device=dev) if K else None,
                status=torch.empty(n, dtype=torch.int32, device=dev) if want_status else None,
                n_cross=torch.empty(n, dtype=torch.int32, device=dev) if want_cross else None,
                hash=torch.empty(n, dtype=torch.int64, device=dev) if want_hash else None,
            )
        call = lib().sg_exp_transport_noalloc if noalloc else lib().sg_exp_transport
        rc = call(
            self._h, n, _dptr(f), _dptr(b), _dptr(v), K, _dptr(W), _dptr(out["f"]), _dptr(out["b"]),
            _dptr(out["p"]), _dptr(out["v"]), _dptr(out.get("W")), _dptr(out.get("status")),
            _dptr(out.get("n_cross")), _dptr(out.get("hash")), C.byref(o), _stream())
        _check(rc)
        return out

    def pi_exp(self, f, b, v, W=None, *, step=None, max_steps=None, search=None, want_steps=False):
        """The projection-integration Exp (sg_pi_exp) for torch CUDA tensors as in exp()."""
        import torch
        n = f.shape[0]
        dev = f.device
        assert f.dtype == torch.int32 and b.dtype == torch.float32 and v.dtype == torch.float32
        assert f.is_contiguous() and b.is_contiguous() and v.is_contiguous()
        assert b.shape == (n, 3) and v.shape == (n, 3)
        K = 0 if W is None else W.shape[1]
        if W is not None:
            assert W.dtype == torch.float32 and W.is_contiguous() and W.shape == (n, K, 3)
        out = dict(
            f=torch.empty(n, dtype=torch.int32, device=dev),
            b=torch.empty(n, 3, dtype=torch.float32, device=dev),
            p=torch.empty(n, 3, dtype=torch.float32, device=dev),
            v=torch.empty(n, 3, dtype=torch.float32, device=dev),
            W=torch.empty(n, K, 3, dtype=torch.float32, device=dev) if K else None,
            status=torch.empty(n, dtype=torch.int32, device=dev),
            n_steps=torch.empty(n, dtype=torch.int32, device=dev) if want_steps else None,
        )
        po = pi_opts(step, max_steps, search)
        _check(lib().sg_pi_exp(self._h, n, _dptr(f), _dptr(b), _dptr(v), K, _dptr(W), _dptr(out["f"]),
                               _dptr(out["b"]), _dptr(out["p"]), _dptr(out["v"]), _dptr(out["W"]),
                               _dptr(out["status"]), _dptr(out["n_steps"]), C.byref(po), _stream()))
        return out

    def pi_backward(self, mode, f, b, v, g, *, f_out=None, v_out=None, step=None, max_steps=None, search=None,
                    o: Opts | None = None, **kw):
        """(grad_v, grad_b) of the PI map for upstream g = dL/dp' [n,3] (sg_pi_backward)."""
        import torch
        n = f.shape[0]
        dev = f.device
        assert f.dtype == torch.int32 and b.dtype == torch.float32 and v.dtype == torch.float32
        assert g.dtype == torch.float32 and g.is_contiguous() and g.shape == (n, 3)
        if o is None:
            o = opts(**kw)
        po = pi_opts(step, max_steps, search)
        gv = torch.empty(n, 3, dtype=torch.float32, device=dev)
        gb = torch.empty(n, 3, dtype=torch.float32, device=dev)
        _check(lib().sg_pi_backward(self._h, int(mode), n, _dptr(f), _dptr(b), _dptr(v), _dptr(f_out), _dptr(v_out),
                                    _dptr(g), _dptr(gv), _dptr(gb), C.byref(po), C.byref(o), _stream()))
        return gv, gb

    def pi_backward_workspace_size(self, mode, n):
        nb = C.c_size_t()
        _check(lib().sg_pi_backward_workspace_size(self._h, int(mode), n, C.byref(nb)))
        return nb.value

    def backward(self, mode, f, b, v, g, *, f_out=None, b_out=None, v_out=None, status=None, out=None, grad_X=None,
                 want_vjp=True, g_b=None, g_v=None, g_W=None, o: Opts | None = None, **kw):
        """(grad_v, grad_b) for upstream g = dL/dp' [n,3]; mode BWD_EP or BWD_GFD.

        f_out, b_out, v_out, status: the forward's saved outputs (EP reads f_out
        and v_out; with f_out, v_out and status the vertex gradient, and with
        f_out, b_out and v_out GFD, skip walking the base geodesic again).

        grad_X: a float64 [n_verts, 3] tensor to accumulate dL/dX into (or None).
        want_vjp=False skips grad_v / grad_b (returns (None, None)).
        g_b = dL/db' [n,3], g_v = dL/dv' [n,3] and g_W = dL/dW' [n,K,3] (optional; g
        may then be None) add the other outputs' cotangents; with g_W the result
        is (grad_v, grad_b, grad_W).
        """
        import torch
        n = f.shape[0]
        dev = f.device
        assert f.dtype == torch.int32 and b.dtype == torch.float32 and v.dtype == torch.float32
        assert f.is_contiguous() and b.is_contiguous() and v.is_contiguous()
        for t, shape in ((g, (n, 3)), (g_b, (n, 3)), (g_v, (n, 3))):
            assert t is None or (t.dtype == torch.float32 and t.is_contiguous() and t.shape == shape)
        if g_b is not None or g_v is not None or g_W is not None:
            K = 0 if g_W is None else g_W.shape[1]
            assert g_W is None or (g_W.dtype == torch.float32 and g_W.is_contiguous() and g_W.shape == (n, K, 3))
            if o is None:
                o = opts(**kw)
            gv_ = torch.empty(n, 3, dtype=torch.float32, device=dev)
            gb_ = torch.empty(n, 3, dtype=torch.float32, device=dev)
            gW_ = torch.empty(n, K, 3, dtype=torch.float32, device=dev) if g_W is not None else None
            if grad_X is not None:
                assert grad_X.dtype == torch.float64 and grad_X.is_contiguous() and grad_X.shape == (self.n_verts, 3)
            _check(lib().sg_exp_backward_transport(
                self._h, int(mode), n, _dptr(f), _dptr(b), _dptr(v), K, _dptr(f_out), _dptr(b_out), _dptr(v_out),
                _dptr(status),
                _dptr(g),
                _dptr(g_b), _dptr(g_v), _dptr(g_W), _dptr(gv_), _dptr(gb_), _dptr(gW_), _dptr(grad_X), C.byref(o),
                _stream()))
            return (gv_, gb_, gW_) if g_W is not None else (gv_, gb_)
        assert g is not None
        if grad_X is not None:
            assert grad_X.dtype == torch.float64 and grad_X.is_contiguous() and grad_X.shape == (self.n_verts, 3)
        if o is None:
            o = opts(**kw)
        if not want_vjp:
            out = (None, None)
        elif out is None:
            out = (torch.empty(n, 3, dtype=torch.float32, device=dev), torch.empty(n, 3, dtype=torch.float32, device=dev))
        _check(lib().sg_exp_backward(self._h, int(mode), n, _dptr(f), _dptr(b), _dptr(v), _dptr(f_out), _dptr(b_out),
                                     _dptr(v_out), _dptr(status), _dptr(g), _dptr(out[0]), _dptr(out[1]), _dptr(grad_X), C.byref(o),
                                     _stream()))
        return out


def _autograd_function():
    import torch

    class ExpFunction(torch.autograd.Function):
        """p' = Exp_p(v) with the library's backward (Sec. 4 "Differentiation").

        Inputs: f [n] int32, b [n,3], v [n,3] float32 (cuda); X [V,3] (the
        mesh's vertex positions as a tensor, or None) receives dL/dX from the
        float64 vertex-gradient pass.  mode: BWD_EP or BWD_GFD for dL/dv and
        dL/db.  The end point p', its barycentrics b', the end tangent v' and
        the transported vectors W' (when W [n,K,3] is given) are
        differentiated; dL/dX takes the p' and b' terms.
        """

        @staticmethod
        def forward(ctx, mesh, mode, f, b, v, W, X, opts_kw):
            Wc = None if W is None else W.contiguous().float()
            out = mesh.exp(f.contiguous(), b.contiguous(), v.contiguous(), Wc, **(opts_kw or {}))
            ctx.mesh, ctx.mode, ctx.opts_kw = mesh, mode, opts_kw or {}
            ctx.want_x = X is not None and X.requires_grad
            ctx.x_dtype = X.dtype if X is not None else None
            ctx.K = 0 if W is None else W.shape[1]
            ctx.save_for_backward(f, b, v, out["f"], out["b"], out["v"], out["status"])
            ctx.mark_non_differentiable(out["f"], out["status"])
            if W is None:
                return out["p"], out["f"], out["b"], out["v"], out["status"]
            return out["p"], out["f"], out["b"], out["v"], out["W"], out["status"]

        @staticmethod
        def backward(ctx, g_p, g_f, g_b, g_vo, *rest):
            f, b, v, f_out, b_out, v_out, status = ctx.saved_tensors
            g_Wo = rest[0] if ctx.K else None
            g = g_p.contiguous().float()
            gX = torch.zeros(ctx.mesh.n_verts, 3, dtype=torch.float64, device=g.device) if ctx.want_x else None
            res = ctx.mesh.backward(ctx.mode, f.contiguous(), b.contiguous(), v.contiguous(), g, f_out=f_out,
                                    b_out=b_out, v_out=v_out, status=status, grad_X=gX,
                                    g_b=g_b.contiguous().float(),
                                    g_v=g_vo.contiguous().float(),
                                    g_W=None if g_Wo is None else g_Wo.contiguous().float(), **ctx.opts_kw)
            gv, gb = res[0], res[1]
            gW = res[2] if g_Wo is not None else None
            return (None, None, None, gb, gv, gW, gX.to(ctx.x_dtype) if gX is not None else None, None)

    return ExpFunction


_ExpFunction = None


def exp_with_grad(mesh, f, b, v, X=None, mode=BWD_GFD, W=None, **opts_kw):
    """Differentiable Exp: returns (p', f', b', v', status), or (p', f', b', v', W', status) when
    W [n,K,3] is given.  p', v' and W' carry the library's backward to b, v and W (mode BWD_EP
    or BWD_GFD for p'), and p' to X when X is a tensor that requires grad."""
    global _ExpFunction
    if _ExpFunction is None:
        _ExpFunction = _autograd_function()
    return _ExpFunction.apply(mesh, mode, f, b, v, W, X, opts_kw)


def exp_iterated(mesh, f, b, field, steps, **opts_kw):
    """Exp applied `steps` times with a vector field re-evaluated at each intermediate point:
    p_{k+1} = Exp_{p_k}(field(p_k, f_k, b_k) / steps) (the K-step map of the paper's flow
    matching, eq. fmobj in Sec. "MeshFlow").  field(p [n,3], f [n], b [n,3]) -> v [n,3] float32
    tensor.  Differentiable (exp_with_grad, mode BWD_GFD by default): gradients flow through the
    field's outputs and, step to step, through the start points (the end barycentrics'
    cotangents); p_0 = sum_k b_k x_k is itself a library call (a zero-length Exp), so with
    BWD_GFD the field's dependence on the start point reaches b.
    Returns (p, f, b) of the last step and the list of intermediate points."""
    import torch
    mode = opts_kw.pop("mode", BWD_GFD)
    n = f.shape[0]
    zero = torch.zeros(n, 3, dtype=torch.float32, device=f.device)
    p, f, b, _, _ = exp_with_grad(mesh, f, b.contiguous(), zero, mode=mode, **opts_kw)
    pts = []
    for _ in range(int(steps)):
        v = field(p, f, b) / float(steps)
        p, f, b, _, _ = exp_with_grad(mesh, f, b.contiguous(), v.contiguous().float(), mode=mode, **opts_kw)
        pts.append(p)
    return (p, f, b), pts


def transport_back(mesh, f_out, b_out, v_out, W, **opts_kw):
    """Adjoint (inverse) of the parallel transport of an earlier call: carries vectors W [n,K,3]
    at p' back along the same geodesic to p, by walking from (f', b') with -v' (a walk reversed
    from its end retraces its path).  Returns (W at p [n,K,3], status)."""
    out = mesh.exp(f_out.contiguous(), b_out.contiguous(), (-v_out).contiguous(), W.contiguous(), **opts_kw)
    return out["W"], out["status"]
