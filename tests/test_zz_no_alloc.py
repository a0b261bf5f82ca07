"""The allocation-free forward (sg_exp_transport_noalloc) against
sg_exp_transport: the same kernels on the library's fixed device scratch
instead of a workspace allocation, so every output must agree bit for bit.
Two calls in a row, the second smaller (the scratch keeps the first call's
contents), then the size limit and the rejected options."""
import numpy as np
import pytest
import torch

from paper_2603_15780_amd import sg
from workloads import configs as CF
from workloads.rays import random_rays, uniform_len

pytestmark = pytest.mark.gpu


def _dev(r, n):
    return {k: torch.from_numpy(np.ascontiguousarray(r[k][:n])).cuda() for k in ("f", "b", "v", "W")}


def _same(a, b):
    for k in ("f", "b", "p", "v", "W", "status", "n_cross", "hash"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("cfg,n1,n2", [(1, 8192, 3001), (2, 1 << 20, 100_003)])
def test_noalloc_matches_workspace_call(cfg, n1, n2):
    X, F = CF.mesh_config(cfg)
    r = random_rays(X, F, n1, np.random.default_rng(7000 + cfg), uniform_len(0.0, np.pi / 2), K=2)
    mesh = sg.Mesh(X, F)
    print(f"noalloc parity: config {cfg}, n = {n1} then {n2}", flush=True)
    for n in (n1, n2):
        t = _dev(r, n)
        # the persistent walk (the default for batches beyond its resident lanes) runs on the scratch
        kw = dict(kernel=sg.KERNEL_PERSISTENT, want_cross=True, want_hash=True)
        ref = mesh.exp(t["f"], t["b"], t["v"], t["W"], **kw)
        got = mesh.exp(t["f"], t["b"], t["v"], t["W"], noalloc=True, **kw)
        torch.cuda.synchronize()
        _same(ref, got)
        assert (got["status"] == sg.RAY_OK).float().mean().item() > 0.99


def test_noalloc_limits():
    X, F = CF.mesh_config(1)
    mesh = sg.Mesh(X, F)
    r = random_rays(X, F, 64, np.random.default_rng(1), uniform_len(0.0, 1.0), K=2)
    t = _dev(r, 64)
    # the plain kernel needs no scratch and is accepted
    ref = mesh.exp(t["f"], t["b"], t["v"], t["W"], kernel=sg.KERNEL_PLAIN)
    got = mesh.exp(t["f"], t["b"], t["v"], t["W"], kernel=sg.KERNEL_PLAIN, noalloc=True)
    torch.cuda.synchronize()
    for k in ("f", "b", "p", "v", "W", "status"):
        assert torch.equal(ref[k], got[k]), k
    for kw in (dict(kernel=sg.KERNEL_PARTITIONED), dict(debug=4)):
        with pytest.raises(sg.SgError) as e:
            mesh.exp(t["f"], t["b"], t["v"], t["W"], noalloc=True, **kw)
        assert e.value.code == sg.SG_E_ARG
    ws = torch.empty(mesh.exp_workspace_size(64, 2, kernel=sg.KERNEL_PERSISTENT), dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SgError):
        mesh.exp(t["f"], t["b"], t["v"], t["W"], noalloc=True, workspace=ws.data_ptr(), workspace_bytes=ws.numel())
    # a batch beyond the scratch is refused before any launch: the size check
    # comes first, so the (small) arrays are never indexed past 64 rays
    big = 2_000_000
    assert mesh.exp_workspace_size(big, 2) > 128 << 20
    out = {k: v for k, v in ref.items()}
    with pytest.raises(sg.SgError) as e:
        sg.lib()
        rc = sg.lib().sg_exp_transport_noalloc(
            mesh._h, big, sg._dptr(t["f"]), sg._dptr(t["b"]), sg._dptr(t["v"]), 2, sg._dptr(t["W"]),
            sg._dptr(out["f"]), sg._dptr(out["b"]), sg._dptr(out["p"]), sg._dptr(out["v"]), sg._dptr(out["W"]),
            None, None, None, sg.opts(), sg._stream())
        sg._check(rc)
    assert e.value.code == sg.SG_E_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
