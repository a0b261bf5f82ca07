"""Host-side checks of the C ABI library (no GPU compute).

The library must load and export every function include/sg.h declares, and
mesh validation (which runs on the host before any HIP call) must reject the
same bad meshes the manifold condition of Sec. 4 excludes.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from workloads import meshes as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", src)))


def test_header_declares_the_three_calls():
    names = _declared()
    for n in ("sg_exp", "sg_exp_transport", "sg_mesh_create", "sg_mesh_destroy", "sg_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_15780_amd import sg
    L = sg.lib()
    for n in _declared():
        assert hasattr(L, n), n


def _create(X, F):
    from paper_2603_15780_amd import sg
    L = sg.lib()
    X = np.ascontiguousarray(X, dtype=np.float32)
    F = np.ascontiguousarray(F, dtype=np.int32)
    h = C.c_void_p()
    rc = L.sg_mesh_create(X.ctypes.data_as(C.c_void_p), X.shape[0], F.ctypes.data_as(C.c_void_p), F.shape[0],
                          None, None, 1, C.byref(h))
    return rc, L.sg_last_error().decode()


def test_mesh_validation_errors():
    X, F = M.canonical(*M.octahedron())
    # an edge shared by three faces
    X3 = np.concatenate([X, [[2, 2, 2]]]).astype(np.float32)
    F3 = np.concatenate([F, [[F[0, 0], F[0, 1], 6]]])
    rc, msg = _create(X3, F3)
    assert rc == -2 and "faces" in msg
    rc, _ = _create(X, np.concatenate([F, [[0, 0, 1]]]))
    assert rc == -3
    rc, _ = _create(X, np.concatenate([F, [[0, 1, 99]]]))
    assert rc == -1
    Xz = np.concatenate([X, [[0.5, 0, 0]]]).astype(np.float32)   # collinear with vertices 0 and 1
    rc, _ = _create(Xz, np.concatenate([F, [[0, 1, 6]]]))
    assert rc in (-2, -3)
    Xn = X.copy()
    Xn[2, 0] = np.nan
    rc, _ = _create(Xn, F)
    assert rc == -1
    # two tetrahedra glued at one vertex: that vertex has two fans
    Xt, Ft = M.tetrahedron()
    X2 = np.concatenate([Xt, -(Xt[1:] - Xt[0]) + Xt[0]]).astype(np.float32)
    F2 = np.concatenate([Ft, np.where(Ft == 0, 0, Ft + 3)])
    rc, msg = _create(X2, F2)
    assert rc == -2 and "fan" in msg


def test_null_arguments_fail_before_launch():
    from paper_2603_15780_amd import sg
    L = sg.lib()
    h = C.c_void_p()
    assert L.sg_mesh_create(None, 0, None, 0, None, None, 1, C.byref(h)) == -1
    assert L.sg_mesh_create(None, 0, None, 0, None, None, 1, None) == -1
    o = sg.opts()
    assert L.sg_exp(None, 1, None, None, None, None, None, None, None, None, None, None, C.byref(o), None) == -1
    assert L.sg_mesh_info(None, None, None, None) == -1


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message before touching a device."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "4"], capture_output=True, text=True,
                       timeout=60)
    assert p.returncode == 2 and "one GPU" in p.stderr
