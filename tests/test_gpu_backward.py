"""GPU parity of the backward (sg_exp_backward) against the oracle.

Extrinsic proxy (eq. proxy_func) and geodesic finite differences (eqs. jv,
jp, chain) through the C ABI on cuda:0, compared with the float64 oracle at
the same step sizes.  Gradients are compared on rays that keep a margin from
every vertex (finite differences of geodesics are not smooth across a vertex);
the bar is a relative error of 1e-3, and 5e-3 for finite differences whose
base walk passes within ten steps (10 eps) of a vertex.
"""
import numpy as np
import pytest

import oracle
from parity import grad_report
from workloads import configs as CF
from workloads import meshes as M
from workloads.rays import random_rays, uniform_len

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU test needs a HIP device"
    return T


def dev_inputs(torch, r, g):
    dev = torch.device("cuda:0")
    t = dict(f=torch.from_numpy(np.ascontiguousarray(r["f"], np.int32)).to(dev),
             b=torch.from_numpy(np.ascontiguousarray(r["b"], np.float32)).to(dev),
             v=torch.from_numpy(np.ascontiguousarray(r["v"], np.float32)).to(dev),
             g=torch.from_numpy(np.ascontiguousarray(g, np.float32)).to(dev))
    return t


def gpu_bwd(torch, gm, mode, r, g, saved=False, **kw):
    """The backward on the GPU; EP reads the forward's f' and v'; with saved=True
    every mode is also given b' and the status (GFD then takes the base
    geodesic's end from the forward instead of walking it)."""
    from paper_2603_15780_amd import sg
    t = dev_inputs(torch, r, g)
    fo = bo = vo = st = None
    if mode == sg.BWD_EP or saved:
        out = gm.exp(t["f"], t["b"], t["v"], **{k: v for k, v in kw.items() if k in ("max_steps", "boundary_mode")})
        fo, vo = out["f"], out["v"]
        if saved:
            bo, st = out["b"], out["status"]
    gv, gb = gm.backward(mode, t["f"], t["b"], t["v"], t["g"], f_out=fo, b_out=bo, v_out=vo, status=st, **kw)
    torch.cuda.synchronize()
    return gv.cpu().numpy(), gb.cpu().numpy()


def check(torch, X, F, r, g, mode, rows=None, min_margin_rays=100, saved=False, **kw):
    from paper_2603_15780_amd import sg
    om = oracle.Mesh(X, F)
    gm = sg.Mesh(X, F)
    eps = np.float32(5e-3 * om.mean_edge)
    gv, gb = gpu_bwd(torch, gm, mode, r, g, saved=saved, eps_v=float(eps), eps_p=float(eps), **kw)
    sel = slice(None) if rows is None else rows
    rf, rb, rv, gs = r["f"][sel], r["b"][sel], r["v"][sel], g[sel]
    okw = dict(boundary_mode=kw["boundary_mode"]) if "boundary_mode" in kw else {}
    o = om.exp(rf, rb, rv, **okw)
    if mode == sg.BWD_EP:
        ogv, ogb = om.ep(rf, rb, rv, gs, **okw)
    else:
        od = om.gfd(rf, rb, rv, gs, float(eps), float(eps), **okw)
        ogv, ogb = od["grad_v"], od["grad_b"]
    # GFD: rays whose base walk passes within 10 eps of a vertex are held to 5e-3 (see grad_report)
    near = None if mode == sg.BWD_EP else (10 * float(eps) / om.mean_edge, 5e-3)
    s = grad_report(o, ogv, ogb, gv[sel], gb[sel], om.mean_edge, near=near)
    print(s)
    assert s["finite"], s
    assert s["n_margin"] >= min_margin_rays, s
    assert s["v_ok"] >= 0.999 and s["b_ok"] >= 0.999, s
    return s, gv, gb


@pytest.mark.parametrize("mode", [0, 1])
def test_config1(torch, mode):
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    s, _, gb = check(torch, X, F, r, g, mode)
    if mode == 0:
        assert s["v_all_ok"] >= 0.99 and np.all(gb == 0)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n", [1, 255, 257, 4097])
def test_ragged(torch, mode, n):
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(100 + n)
    r = random_rays(X, F, n, rng, uniform_len(0.0, 1.0))
    g = rng.standard_normal((n, 3)).astype(np.float32)
    check(torch, X, F, r, g, mode, min_margin_rays=min(n, 100) // 2)


@pytest.mark.parametrize("mode,saved", [(0, False), (1, False), (1, True)])
def test_config2_full_batch_sampled(torch, mode, saved):
    """Backward over all 1,048,576 rays on the 327,680-face mesh; 16,384 sampled
    rows (every 64th) vs the oracle.  saved: GFD takes the base geodesic's end
    from the forward's outputs (six walks per query instead of seven)."""
    X, F = CF.mesh_config(2)
    r = CF.rays_config(2, X, F)
    g = CF.upstream_grad(2, r["f"].shape[0])
    rows = np.arange(0, r["f"].shape[0], 64)
    check(torch, X, F, r, g, mode, rows=rows, saved=saved)



@pytest.mark.parametrize("mode,saved", [(0, False), (1, False), (1, True)])
def test_config5_full_batch_sampled(torch, config5, mode, saved):
    """Backward over all 16,777,216 rays on the 1,310,720-face noisy mesh (641
    crossings per ray on average, lengths up to pi); every 512th row vs the
    oracle.  GFD runs with and without the forward's outputs (its long walks
    three or four to a query in one pass)."""
    X, F, r = config5
    g = CF.upstream_grad(5, r["f"].shape[0])
    rows = np.arange(0, r["f"].shape[0], 512)
    check(torch, X, F, r, g, mode, rows=rows, saved=saved, min_margin_rays=600)

@pytest.mark.parametrize("mixed", [False, True])
def test_gfd_from_saved_forward(torch, mixed):
    """GFD given the forward's f', b', v' and status walks six geodesics per
    query; it matches the oracle like the seven-walk form and agrees with it
    (relative 1e-3 on the margin rays: the base end point enters through the
    float32 b' instead of the walk's chart state).  On a mesh whose faces
    disagree in orientation the saved outputs are not used: bit for bit the
    seven-walk result."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    if mixed:
        F = F.copy()
        flip = np.random.default_rng(5).random(F.shape[0]) < 0.3
        F[flip] = F[flip][:, ::-1]
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    s7, gv7, gb7 = check(torch, X, F, r, g, sg.BWD_GFD)
    s6, gv6, gb6 = check(torch, X, F, r, g, sg.BWD_GFD, saved=True)
    if mixed:
        assert np.array_equal(gv6, gv7) and np.array_equal(gb6, gb7)
        return
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"])
    keep = (o["min_vdist"] > 1e-4 * om.mean_edge) & (o["status"] == 0)
    rel = np.linalg.norm(gv6 - gv7, axis=1) / np.maximum(np.linalg.norm(gv7, axis=1), 1e-12)
    assert np.quantile(rel[keep], 0.999) < 1e-3, np.quantile(rel[keep], 0.999)


@pytest.mark.parametrize("mode", [0, 1])
def test_torus_and_mixed_orientation(torch, mode):
    rng = np.random.default_rng(3)
    X, F = M.torus_grid(40, 20, 0.2, rng)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 1.5))
    g = rng.standard_normal((4096, 3)).astype(np.float32)
    check(torch, X, F, r, g, mode)
    # faces with disagreeing orientation: the extrinsic proxy re-walks the geodesic
    X, F = CF.mesh_config(1)
    F2 = F.copy()
    flip = np.random.default_rng(5).random(F.shape[0]) < 0.3
    F2[flip] = F2[flip][:, ::-1]
    r = random_rays(X, F2, 4096, rng, uniform_len(0.0, 1.5))
    check(torch, X, F2, r, g, mode)


def test_zero_length_and_short(torch):
    """|v| = 0: the extrinsic proxy is the identity; GFD differentiates Exp at 0 (projection)."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(9)
    r = random_rays(X, F, 2048, rng, uniform_len(0.0, 0.0))
    g = rng.standard_normal((2048, 3)).astype(np.float32)
    gm = sg.Mesh(X, F)
    gv, gb = gpu_bwd(torch, gm, sg.BWD_EP, r, g)
    assert np.array_equal(gv, g) and np.all(gb == 0)
    s, gv, gb = check(torch, X, F, r, g, sg.BWD_GFD)
    # Exp_p(w) = p + w for small in-face w: grad_v is g projected on the start face
    om = oracle.Mesh(X, F)
    N = np.cross(X[F[r["f"], 1]] - X[F[r["f"], 0]], X[F[r["f"], 2]] - X[F[r["f"], 0]])
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    proj = g - (g * N).sum(1, keepdims=True) * N
    far = r["b"].min(1) > 0.05
    err = np.linalg.norm(gv - proj, axis=1) / np.linalg.norm(proj, axis=1)
    assert np.quantile(err[far], 0.999) < 1e-3
    r = random_rays(X, F, 2048, rng, uniform_len(0.0, 0.02 * om.mean_edge))
    for mode in (0, 1):
        check(torch, X, F, r, g, mode)


def test_edge_cases(torch):
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    gm = sg.Mesh(X, F)
    dev = torch.device("cuda:0")
    e = torch.empty(0, dtype=torch.int32, device=dev)
    e3 = torch.empty(0, 3, device=dev)
    for mode in (0, 1):
        gv, gb = gm.backward(mode, e, e3, e3, e3, f_out=e, v_out=e3)
        assert gv.shape == (0, 3)
    f = torch.tensor([0, -1, F.shape[0], 1], dtype=torch.int32, device=dev)
    b = torch.tensor([[1, 1, 1], [1, 1, 1], [1, 1, 1], [float("nan"), 1, 1]], dtype=torch.float32, device=dev)
    v = torch.full((4, 3), 0.1, device=dev)
    g = torch.ones(4, 3, device=dev)
    for mode in (0, 1):
        out = gm.exp(f, b, v)
        gv, gb = gm.backward(mode, f, b, v, g, f_out=out["f"], v_out=out["v"])
        torch.cuda.synchronize()
        gv = gv.cpu().numpy()
        assert np.isfinite(gv[0]).all() and np.isnan(gv[1:]).all()
    with pytest.raises(sg.SgError):
        gm.backward(7, f, b, v, g)
    with pytest.raises(sg.SgError):   # the saved-output extrinsic proxy needs the forward's outputs
        gm.backward(0, f, b, v, g)


def test_deterministic_and_schedules(torch):
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(11)
    r = random_rays(X, F, 20000, rng, uniform_len(0.0, 1.5))
    g = rng.standard_normal((20000, 3)).astype(np.float32)
    gm = sg.Mesh(X, F)
    ref = gpu_bwd(torch, gm, sg.BWD_GFD, r, g)
    for kw in ({}, dict(refill_min=1), dict(refill_min=64), dict(walk_blocks=7), dict(walk_blocks=3000, refill_min=32),
               dict(ray_queues=64, walk_blocks=5)):
        out = gpu_bwd(torch, gm, sg.BWD_GFD, r, g, **kw)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), kw


# ---------------------------------------------------------------- vertex-position gradient
def margin_mask(om, r, margin=1e-2):
    o = om.exp(r["f"], r["b"], r["v"])
    return (o["min_vdist"] > margin * om.mean_edge) & (o["status"] == 0)


def gpu_gradx(torch, gm, r, g, mode=0, want_vjp=False, **kw):
    from paper_2603_15780_amd import sg
    t = dev_inputs(torch, r, g)
    gX = torch.zeros(gm.n_verts, 3, dtype=torch.float64, device=t["f"].device)
    fo = vo = None
    if want_vjp and mode == sg.BWD_EP:
        out = gm.exp(t["f"], t["b"], t["v"], **{k: v for k, v in kw.items() if k in ("max_steps", "boundary_mode")})
        fo, vo = out["f"], out["v"]
    res = gm.backward(mode, t["f"], t["b"], t["v"], t["g"], f_out=fo, v_out=vo, grad_X=gX, want_vjp=want_vjp, **kw)
    torch.cuda.synchronize()
    return gX.cpu().numpy(), res


@pytest.mark.parametrize("mixed", [False, True])
def test_gradx_config1(torch, mixed):
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = CF.mesh_config(1)
    if mixed:
        F = F.copy()
        flip = np.random.default_rng(5).random(F.shape[0]) < 0.3
        F[flip] = F[flip][:, ::-1]
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, nvx = om.gradx(r["f"], r["b"], r["v"], g)
    assert np.all(nvx[keep] == 0)
    gm = sg.Mesh(X, F)
    got, _ = gpu_gradx(torch, gm, r, g)
    s = gradx_report(ref, got)
    print(s)
    assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s
    # the same sums come out of the combined calls (base walk shared with EP / GFD)
    for mode in (sg.BWD_EP, sg.BWD_GFD):
        got2, (gv, gb) = gpu_gradx(torch, gm, r, g, mode=mode, want_vjp=True)
        assert gradx_report(ref, got2)["global_rel"] < 1e-4
        assert np.allclose(got2, got, rtol=1e-9, atol=1e-9 * np.abs(got).max())
        assert np.isfinite(gv.cpu().numpy()[keep]).all()


@pytest.mark.parametrize("mixed", [False, True])
def test_gradx_from_saved_outputs(torch, mixed):
    """With the forward's f_out, v_out and status the vertex gradient takes its
    end frame from them instead of re-walking the geodesic: the same sums up to
    the float32 rounding of v' (global relative 1e-6), and the oracle's within
    1e-4, for EP + grad_X and for grad_X alone.  On a mesh whose faces disagree
    in orientation the end normal's sign needs the walk: the call re-walks and
    gives the walked sums bit for bit."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = CF.mesh_config(1)
    if mixed:
        F = F.copy()
        flip = np.random.default_rng(5).random(F.shape[0]) < 0.3
        F[flip] = F[flip][:, ::-1]
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    gm = sg.Mesh(X, F)
    t = dev_inputs(torch, r, g)
    out = gm.exp(t["f"], t["b"], t["v"])
    res = {}
    for name, st, vjp in (("walked", None, True), ("saved", out["status"], True), ("saved_x_only", out["status"], False)):
        gX = torch.zeros(gm.n_verts, 3, dtype=torch.float64, device=t["f"].device)
        gm.backward(sg.BWD_EP, t["f"], t["b"], t["v"], t["g"], f_out=out["f"], v_out=out["v"], status=st, grad_X=gX,
                    want_vjp=vjp)
        torch.cuda.synchronize()
        res[name] = gX.cpu().numpy()
    scale = np.abs(res["walked"]).max()
    for name in ("saved", "saved_x_only"):
        s = gradx_report(ref, res[name])
        print(name, s)
        assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s
        if mixed:
            assert np.allclose(res[name], res["walked"], rtol=1e-9, atol=1e-9 * scale)
        else:
            assert np.linalg.norm(res[name] - res["walked"]) <= 1e-6 * np.linalg.norm(res["walked"])



@pytest.mark.parametrize("mixed", [False, True])
def test_gfd_gradx_from_saved_outputs(torch, mixed):
    """GFD and the vertex gradient in one call, given all of the forward's
    saved outputs (f', b', v', status).  On consistently oriented faces
    neither walks the base geodesic: GFD's three long walks share one pass and
    the adjoint walk starts from the saved end frame.  On a mesh whose faces
    disagree in orientation both re-walk it.  Either way the GFD gradients
    equal those of the same call without grad_X bit for bit, and grad_X
    equals EP + grad_X's from the same outputs up to the float64 summation
    order and the oracle's within 1e-4."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = CF.mesh_config(1)
    if mixed:
        F = F.copy()
        flip = np.random.default_rng(5).random(F.shape[0]) < 0.3
        F[flip] = F[flip][:, ::-1]
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    gm = sg.Mesh(X, F)
    t = dev_inputs(torch, r, g)
    out = gm.exp(t["f"], t["b"], t["v"])
    eps = float(np.float32(5e-3 * om.mean_edge))
    kw = dict(f_out=out["f"], b_out=out["b"], v_out=out["v"], status=out["status"])
    args = (t["f"], t["b"], t["v"], t["g"])
    gv0, gb0 = gm.backward(sg.BWD_GFD, *args, eps_v=eps, eps_p=eps, **kw)
    gX = torch.zeros(gm.n_verts, 3, dtype=torch.float64, device=t["f"].device)
    gv1, gb1 = gm.backward(sg.BWD_GFD, *args, grad_X=gX, want_vjp=True, eps_v=eps, eps_p=eps, **kw)
    gXe = torch.zeros_like(gX)
    gm.backward(sg.BWD_EP, *args, grad_X=gXe, want_vjp=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(gv0, gv1) and torch.equal(gb0, gb1)
    assert np.isfinite(gv1.cpu().numpy()[keep]).all()
    got, got_ep = gX.cpu().numpy(), gXe.cpu().numpy()
    s = gradx_report(ref, got)
    print(s)
    assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s
    assert np.allclose(got, got_ep, rtol=1e-9, atol=1e-9 * np.abs(got_ep).max())

def test_gradx_config2_full_batch(torch):
    """All 1,048,576 rays on the 327,680-face mesh.  (1) Upstream g on every
    margin ray: translating the mesh translates each p', so the vertex
    gradients sum to sum g.  (2) g on 16,384 sampled margin rays only: the
    gradient field is compared with the oracle's on those rays."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = CF.mesh_config(2)
    r = CF.rays_config(2, X, F)
    n = r["f"].shape[0]
    g = CF.upstream_grad(2, n)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    gm = sg.Mesh(X, F)
    got, _ = gpu_gradx(torch, gm, r, g)
    assert np.isfinite(got).all()
    tot = got.sum(0)
    assert np.allclose(tot, g.astype(np.float64).sum(0), rtol=1e-5, atol=1e-5 * np.abs(g).sum() / np.sqrt(n)), tot
    idx = np.flatnonzero(keep)[:: max(1, keep.sum() // 16384)][:16384]
    gs = np.zeros_like(g)
    gs[idx] = g[idx]
    got_s, _ = gpu_gradx(torch, gm, r, gs)
    sub = {k: r[k][idx] for k in ("f", "b", "v")}
    ref, _ = om.gradx(sub["f"], sub["b"], sub["v"], g[idx])
    s = gradx_report(ref, got_s)
    print(s)
    assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


def test_gradx_zero_length_and_torus(torch):
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    rng = np.random.default_rng(21)
    X, F = CF.mesh_config(1)
    r = random_rays(X, F, 2048, rng, uniform_len(0.0, 0.0))
    g = rng.standard_normal((2048, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    got, _ = gpu_gradx(torch, sg.Mesh(X, F), r, g)
    s = gradx_report(ref, got)
    assert s["global_rel"] < 1e-5 and s["frac_ok"] >= 0.999, s
    X, F = M.torus_grid(60, 20, 0.2, rng)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 1.5))
    g = rng.standard_normal((4096, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    got, _ = gpu_gradx(torch, sg.Mesh(X, F), r, g)
    s = gradx_report(ref, got)
    print(s)
    assert s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


def test_gradx_records_spill_and_atomics_agree(torch):
    """The per-half-edge sums come out the same whether the crossings go through
    the binned records (default), partly spill to float64 atomics (a record
    budget far below the crossings, few walking waves) or all use atomics."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F)
    g = CF.upstream_grad(1, r["f"].shape[0])
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    gm = sg.Mesh(X, F)
    runs = {"records": {}, "spill": dict(gradx_records=1, walk_blocks=2), "atomics": dict(gradx_records=-1)}
    got = {k: gpu_gradx(torch, gm, r, g, **kw)[0] for k, kw in runs.items()}
    scale = np.abs(got["atomics"]).max()
    for k, x in got.items():
        s = gradx_report(ref, x)
        print(k, s)
        assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, (k, s)
        assert np.allclose(x, got["atomics"], rtol=1e-9, atol=1e-11 * scale), k
    # sizes: records take 48 bytes each on top of the atomics-only workspace
    n = r["f"].shape[0]
    w_rec = gm.backward_workspace_size(sg.BWD_EP, n, want_vjp=False, want_grad_X=True)
    w_atm = gm.backward_workspace_size(sg.BWD_EP, n, want_vjp=False, want_grad_X=True, gradx_records=-1)
    assert w_rec - w_atm >= 48 * 256 * n


def test_gradx_records_large_mesh(torch):
    """A mesh of more than 4M half-edges: the record bins span 2048 half-edges
    and the reduce pass sums each bin in two LDS windows."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    rng = np.random.default_rng(31)
    X, F = M.flat_grid(860, 0.2, rng)
    assert 3 * F.shape[0] > 4096 * 1024
    X = (X - np.array([0.5, 0.5, 0.0])).astype(np.float32)
    # rays in a patch around the origin, where float32 positions resolve the
    # 1.2e-3 edges as finely as on the other test meshes
    near = np.flatnonzero(np.linalg.norm(X[F].mean(1)[:, :2], axis=1) < 0.04)
    r = random_rays(X, F, 8192, rng, uniform_len(0.0, 0.03), faces=near)
    g = rng.standard_normal((8192, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    g[~keep] = 0.0
    ref, _ = om.gradx(r["f"], r["b"], r["v"], g)
    gm = sg.Mesh(X, F)
    got = gpu_gradx(torch, gm, r, g)[0]
    atm = gpu_gradx(torch, gm, r, g, gradx_records=-1)[0]
    assert np.allclose(got, atm, rtol=1e-9, atol=1e-11 * np.abs(atm).max())
    s = gradx_report(ref, got)
    print(s)
    assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


def test_gradx_config5_sliced_records(torch, config5):
    """16,777,216 queries on the 1,310,720-face mesh (641 crossings per ray): the
    vertex gradient in 16 calls of 2^20 queries with 800 records each, accumulated
    into one grad_X, equals one call on float64 atomics alone; on every 1024th
    margin ray the records path matches the oracle."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F, r = config5
    n = r["f"].shape[0]
    g = CF.upstream_grad(5, n)
    gm = sg.Mesh(X, F)
    t = dev_inputs(torch, r, g)
    rec = torch.zeros(gm.n_verts, 3, dtype=torch.float64, device=t["f"].device)
    for a in range(0, n, 1 << 20):
        z = slice(a, a + (1 << 20))
        gm.backward(sg.BWD_EP, t["f"][z], t["b"][z], t["v"][z], t["g"][z], grad_X=rec, want_vjp=False,
                    gradx_records=800)
    atm = torch.zeros_like(rec)
    gm.backward(sg.BWD_EP, t["f"], t["b"], t["v"], t["g"], grad_X=atm, want_vjp=False, gradx_records=-1)
    torch.cuda.synchronize()
    rec, atm = rec.cpu().numpy(), atm.cpu().numpy()
    assert np.isfinite(rec).all()
    assert np.allclose(rec, atm, rtol=1e-9, atol=1e-11 * np.abs(atm).max())
    rows = np.arange(0, n, 1024)
    sub = {k: r[k][rows] for k in ("f", "b", "v")}
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, sub)
    gs = np.zeros_like(g)
    gs[rows[keep]] = g[rows[keep]]
    got, _ = gpu_gradx(torch, gm, r, gs)
    ref, _ = om.gradx(sub["f"], sub["b"], sub["v"], np.where(keep[:, None], g[rows], 0.0).astype(np.float32))
    s = gradx_report(ref, got)
    print(s)
    assert s["finite"] and s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


def test_autograd_function(torch):
    """torch.autograd through exp_with_grad gives the library's gradients (and the oracle's)."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report, grad_report
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F)
    n = r["f"].shape[0]
    gup = CF.upstream_grad(1, n)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    gup[~keep] = 0.0
    gm = sg.Mesh(X, F)
    dev = torch.device("cuda:0")
    f = torch.from_numpy(r["f"]).to(dev)
    b = torch.from_numpy(r["b"]).to(dev).requires_grad_(True)
    v = torch.from_numpy(r["v"]).to(dev).requires_grad_(True)
    Xt = torch.from_numpy(X).to(dev).requires_grad_(True)
    eps = float(np.float32(5e-3 * om.mean_edge))
    p, fo, bo, vo, st = sg.exp_with_grad(gm, f, b, v, Xt, mode=sg.BWD_GFD, eps_v=eps, eps_p=eps)
    loss = (p * torch.from_numpy(gup).to(dev)).sum()
    loss.backward()
    torch.cuda.synchronize()
    od = om.gfd(r["f"], r["b"], r["v"], gup, eps, eps)
    o = om.exp(r["f"], r["b"], r["v"])
    s = grad_report(o, od["grad_v"], od["grad_b"], v.grad.cpu().numpy(), b.grad.cpu().numpy(), om.mean_edge)
    assert s["v_ok"] >= 0.999 and s["b_ok"] >= 0.999, s
    ref, _ = om.gradx(r["f"], r["b"], r["v"], gup)
    sx = gradx_report(ref, Xt.grad.double().cpu().numpy(), tol=1e-3)
    # the tensor gradient is float32 (the dtype of X): compare at float32's resolution
    assert sx["frac_ok"] >= 0.999 and sx["global_rel"] < 1e-4, sx


def test_gradx_unreferenced_vertex_and_batched_meshes(torch):
    """The vertex pass sums per vertex over its corner list: a vertex no face
    uses gets exactly zero and the others what they get without it; two meshes
    batched in one handle get each mesh's own gradient (global vertex ids)."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F, n=2048)
    g = CF.upstream_grad(1, 2048)
    ref, _ = gpu_gradx(torch, sg.Mesh(X, F), r, g)
    assert np.abs(ref).max() > 0
    X2 = np.vstack([X, np.array([[2.0, 0.5, -0.25]], np.float32)])
    got, _ = gpu_gradx(torch, sg.Mesh(X2, F), r, g)
    assert np.all(got[-1] == 0.0)
    assert np.allclose(got[:-1], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # a second, displaced mesh after the first in one handle
    XB = M.sh_displace(X, 4, 0.05, np.random.default_rng(77)).astype(np.float32)
    rB = CF.rays_config(1, XB, F, n=2048, seed_offset=1)
    gB = CF.upstream_grad(1, 4096)[2048:]
    refB, _ = gpu_gradx(torch, sg.Mesh(XB, F), rB, gB)
    nv, nf = X.shape[0], F.shape[0]
    gm = sg.Mesh(np.vstack([X, XB]), np.vstack([F, F]), [0, nv, 2 * nv], [0, nf, 2 * nf])
    rr = {k: np.concatenate([r[k], rB[k] + (nf if k == "f" else 0)]) for k in ("f", "b", "v")}
    both, _ = gpu_gradx(torch, gm, rr, np.concatenate([g, gB]))
    want = np.vstack([ref, refB])
    assert np.allclose(both, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("mode", [0, 1])
def test_backward_mesh_with_holes(torch, mode):
    """A mesh with holes: rays that stop on the boundary are left out of the
    vertex gradient (both sides); the others match the oracle."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = M.icosphere(3)
    X, F = M.remove_faces(X, F, np.where((F == 0).any(1) | (F == 7).any(1) | (F == 100).any(1))[0])
    X, F = M.canonical(X, F)
    rng = np.random.default_rng(31)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 2.0))
    g = rng.standard_normal((4096, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"])
    assert np.any(o["status"] == 2)
    keep = margin_mask(om, r)
    gk = np.where(keep[:, None], g, 0.0).astype(np.float32)
    check(torch, X, F, r, gk, mode)
    ref, nvx = om.gradx(r["f"], r["b"], r["v"], gk)
    got, _ = gpu_gradx(torch, sg.Mesh(X, F), r, gk)
    s = gradx_report(ref, got)
    assert s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


@pytest.mark.parametrize("mode", [0, 1])
def test_backward_klein_bottle(torch, mode):
    """Extrinsic proxy, GFD and the vertex gradient on a non-orientable surface."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    X, F = M.canonical(*M.klein_bottle(96, 48))
    rng = np.random.default_rng(43)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 3.0))
    g = rng.standard_normal((4096, 3)).astype(np.float32)
    check(torch, X, F, r, g, mode)
    om = oracle.Mesh(X, F)
    keep = margin_mask(om, r)
    gk = np.where(keep[:, None], g, 0.0).astype(np.float32)
    ref, _ = om.gradx(r["f"], r["b"], r["v"], gk)
    got, _ = gpu_gradx(torch, sg.Mesh(X, F), r, gk, mode=mode, want_vjp=True)
    s = gradx_report(ref, got)
    assert s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


@pytest.mark.parametrize("mode", [0, 1])
def test_backward_hole_avoidance(torch, mode):
    """EP and GFD with hole avoidance against the oracle's (same boundary mode);
    the vertex gradient leaves out rays that slid, on both sides."""
    from paper_2603_15780_amd import sg
    from parity import gradx_report
    from test_oracle_holes import holed_sphere
    X, F = holed_sphere()
    rng = np.random.default_rng(61)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 3.0))
    g = rng.standard_normal((4096, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"], boundary_mode=1)
    assert (o["n_bnd"] > 0).sum() > 300
    check(torch, X, F, r, g, mode, boundary_mode=1)
    keep = (o["min_vdist"] > 1e-2 * om.mean_edge) & (o["status"] == 0) & (o["n_bnd"] == 0)
    gk = np.where(keep[:, None], g, 0.0).astype(np.float32)
    ref, nvx = om.gradx(r["f"], r["b"], r["v"], gk, boundary_mode=1)
    assert np.all(nvx[o["n_bnd"] > 0] == -1)
    got, _ = gpu_gradx(torch, sg.Mesh(X, F), r, gk, mode=mode, want_vjp=True, boundary_mode=1)
    s = gradx_report(ref, got)
    assert s["global_rel"] < 1e-4 and s["frac_ok"] >= 0.999, s


# ---------------------------------------------------------------- cotangents of b', v', W'; iterated Exp; adjoint transport
@pytest.mark.parametrize("mode", [0, 1])
def test_transport_cotangents(torch, mode):
    """dL/dv' and dL/dW' through the transport (R^T in the start plane) against
    the oracle's, in both modes (the p' term left out: g_p = None)."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(91)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 2.0), K=2)
    gvo = rng.standard_normal((4096, 3)).astype(np.float32)
    gWo = rng.standard_normal((4096, 2, 3)).astype(np.float32)
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"])
    ref_v, ref_W = om.transport_vjp(r["f"], r["b"], r["v"], gvo, gWo)
    gm = sg.Mesh(X, F)
    t = dev_inputs(torch, r, gvo)
    out = gm.exp(t["f"], t["b"], t["v"])
    gv, gb, gW = gm.backward(mode, t["f"], t["b"], t["v"], None, f_out=out["f"], v_out=out["v"], g_v=t["g"],
                             g_W=torch.from_numpy(gWo).cuda())
    torch.cuda.synchronize()
    gv, gb, gW = gv.cpu().numpy(), gb.cpu().numpy(), gW.cpu().numpy()
    ok = o["status"] == 0
    scale = np.linalg.norm(gvo, axis=1)
    ev = np.linalg.norm(gv - ref_v, axis=1) / scale
    eW = np.linalg.norm(gW - ref_W, axis=2) / np.linalg.norm(gWo, axis=2)
    assert np.mean(ev[ok] < 1e-4) >= 0.999 and np.mean(eW[ok] < 1e-4) >= 0.999, (ev.max(), eW.max())
    assert np.abs(gb).max() == 0.0   # no p' cotangent: nothing for the start point


@pytest.mark.parametrize("mode", [0, 1])
def test_end_barycentric_cotangent(torch, mode):
    """dL/db' enters as dL/dp' = sum_k g_bk grad b'_k inside the end face."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(92)
    r = random_rays(X, F, 2048, rng, uniform_len(0.0, 2.0))
    gbo = rng.standard_normal((2048, 3)).astype(np.float32)
    gm = sg.Mesh(X, F)
    t = dev_inputs(torch, r, gbo)
    out = gm.exp(t["f"], t["b"], t["v"])
    fo = out["f"].cpu().numpy()
    Xd = X.astype(np.float64)
    y0, y1, y2 = (Xd[F[fo, k]] for k in range(3))
    c = np.cross(y1 - y0, y2 - y0)
    c2 = (c * c).sum(1)[:, None]
    grads = [np.cross(c, y2 - y1) / c2, np.cross(c, y0 - y2) / c2, np.cross(c, y1 - y0) / c2]
    gp = sum(gbo[:, k:k + 1] * grads[k] for k in range(3)).astype(np.float32)
    a = gm.backward(mode, t["f"], t["b"], t["v"], None, f_out=out["f"], v_out=out["v"], g_b=t["g"])
    b_ = gm.backward(mode, t["f"], t["b"], t["v"], torch.from_numpy(gp).cuda(), f_out=out["f"], v_out=out["v"])
    torch.cuda.synchronize()
    for x, y in zip(a, b_):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.abs(x - y).max() <= 1e-4 * np.abs(y).max()


def test_autograd_all_outputs_and_iterated(torch):
    """exp_with_grad differentiates p', b', v' and W' (the library's backward,
    checked against explicit calls), and exp_iterated chains steps."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(93)
    r = random_rays(X, F, 1024, rng, uniform_len(0.0, 1.0), K=2)
    gm = sg.Mesh(X, F)
    dev = torch.device("cuda:0")
    f = torch.from_numpy(r["f"]).to(dev)
    b = torch.from_numpy(r["b"].astype(np.float32)).to(dev).requires_grad_(True)
    v = torch.from_numpy(r["v"].astype(np.float32)).to(dev).requires_grad_(True)
    W = torch.from_numpy(r["W"].astype(np.float32)).to(dev).requires_grad_(True)
    cs = [torch.from_numpy(rng.standard_normal(s).astype(np.float32)).to(dev) for s in ((1024, 3), (1024, 3), (1024, 3), (1024, 2, 3))]
    p, fo, bo, vo, Wo, st = sg.exp_with_grad(gm, f, b, v, mode=sg.BWD_EP, W=W)
    loss = (p * cs[0]).sum() + (bo * cs[1]).sum() + (vo * cs[2]).sum() + (Wo * cs[3]).sum()
    loss.backward()
    out = gm.exp(f, b.detach(), v.detach(), W.detach())
    gv, gb, gW = gm.backward(sg.BWD_EP, f, b.detach().contiguous(), v.detach().contiguous(), cs[0], f_out=out["f"],
                             v_out=out["v"], g_b=cs[1], g_v=cs[2], g_W=cs[3])
    torch.cuda.synchronize()
    assert torch.allclose(v.grad, gv) and torch.allclose(b.grad, gb) and torch.allclose(W.grad, gW)


def test_iterated_exp_against_oracle(torch):
    """The K-step map of eq. fmobj (Sec. "MeshFlow"), K = 3, through exp_iterated
    (GFD): end points against the oracle's composition (tests/test_oracle_iterated.py
    pins it), and the autograd gradients in the field's per-query parameters and
    in the start barycentrics against float64 central differences (h = 1e-6) of
    that composition, at relative error 1e-3 on queries whose paths keep
    2e-2 mean edges from every vertex at every step and whose start and
    intermediate points lie farther than 2 eps from their faces' edges.
    The second condition keeps every GFD stencil inside one face: a stencil
    walk of length eps that crosses an edge makes the difference a chord bent
    by the dihedral angle (eqs. jv and jp take the literal 3D chord), an error
    of order dihedral^2 (about 1e-2 on this coarse mesh) that central
    differences of the map do not have."""
    from paper_2603_15780_amd import sg
    from test_oracle_iterated import field_factory
    X, F = CF.mesh_config(1)
    X, F = M.canonical(M.sh_displace(X.astype(np.float64), 6, 0.15, np.random.default_rng(33)), F)
    om = oracle.Mesh(X, F)
    gm = sg.Mesh(X, F)
    rng = np.random.default_rng(95)
    n, K, H = 4096, 3, 1e-6
    r = random_rays(X, F, n, rng, uniform_len(0.0, 1.0))
    theta = (rng.normal(size=(n, 2)) * [0.5, 0.5]).astype(np.float32).astype(np.float64)
    c1 = rng.normal(size=3).astype(np.float32).astype(np.float64)
    c2 = rng.normal(size=3)
    c2 = (c2 / np.linalg.norm(c2)).astype(np.float32).astype(np.float64)
    o0 = np.zeros(3)
    gup = rng.standard_normal((n, 3))
    # GPU: loss = sum_i g_i . p_K,i
    dev = torch.device("cuda:0")
    th = torch.tensor(theta, dtype=torch.float32, device=dev, requires_grad=True)
    tc1 = torch.tensor(c1, dtype=torch.float32, device=dev)
    tc2 = torch.tensor(c2, dtype=torch.float32, device=dev)
    field = lambda pp, ff, bb: th[:, 0:1] * tc1 + th[:, 1:2] * torch.cross(tc2.expand_as(pp), pp, dim=1)
    f = torch.from_numpy(r["f"]).to(dev)
    b = torch.from_numpy(r["b"].astype(np.float32)).to(dev).requires_grad_(True)
    eps = float(np.float32(5e-3 * om.mean_edge))
    (pK, fK, bK), pts = sg.exp_iterated(gm, f, b, field, K, eps_v=eps, eps_p=eps)
    assert len(pts) == K
    (pK * torch.tensor(gup, dtype=torch.float32, device=dev)).sum().backward()
    torch.cuda.synchronize()
    g_theta = th.grad.double().cpu().numpy()
    g_b = b.grad.double().cpu().numpy()
    # oracle composition (same float32 start barycentrics, same field)
    fld = field_factory(theta, c1, c2, o0)
    it = om.exp_iterated(r["f"], r["b"].astype(np.float32), fld, K)
    err = np.linalg.norm(pK.detach().double().cpu().numpy() - it["p"], axis=1)
    far = it["min_vdist"] > 1e-6
    assert np.mean(err <= 1e-4 * om.mean_edge) >= 0.999 and np.all(err[far] <= 1e-4 * om.mean_edge), err.max()
    assert np.array_equal(fK.cpu().numpy()[far & (err < 1e-6)], it["f"][far & (err < 1e-6)])
    keep = (it["status"] == 0) & (it["min_vdist"] > 2e-2 * om.mean_edge) & (r["b"].min(1) > 1e-3)
    # distance of each start and intermediate point to its face's edges: b_j times the altitude onto edge j
    Xd = X.astype(np.float64)
    for fk, bk in zip(it["fs"], it["bs"]):
        x = Xd[F[fk]]
        area2 = np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)
        opp = np.stack([np.linalg.norm(x[:, (j + 2) % 3] - x[:, (j + 1) % 3], axis=1) for j in range(3)], 1)
        keep &= (bk * (area2[:, None] / opp)).min(1) > 2 * eps
    assert keep.sum() > 1000, keep.sum()
    # central differences of the oracle's composition, per query (queries are independent)
    fd_theta = np.zeros((n, 2))
    for q in range(2):
        tp, tm = theta.copy(), theta.copy()
        tp[:, q] += H
        tm[:, q] -= H
        dp = (om.exp_iterated(r["f"], r["b"].astype(np.float32), field_factory(tp, c1, c2, o0), K)["p"]
              - om.exp_iterated(r["f"], r["b"].astype(np.float32), field_factory(tm, c1, c2, o0), K)["p"]) / (2 * H)
        fd_theta[:, q] = (dp * gup).sum(1)
    # the start-point gradient in the face plane, as its components along the
    # constraint-preserving barycentric directions (-1, 1, 0) and (-1, 0, 1)
    b0 = r["b"].astype(np.float32).astype(np.float64)
    b0 /= b0.sum(1)[:, None]
    fd_b = np.zeros((n, 2))
    for q, d in enumerate(([-1.0, 1.0, 0.0], [-1.0, 0.0, 1.0])):
        d = np.asarray(d)[None, :]
        dp = (om.exp_iterated(r["f"], b0 + H * d, fld, K)["p"] - om.exp_iterated(r["f"], b0 - H * d, fld, K)["p"]) / (2 * H)
        fd_b[:, q] = (dp * gup).sum(1)
    rel_t = np.linalg.norm(g_theta - fd_theta, axis=1) / np.maximum(np.linalg.norm(fd_theta, axis=1), 1e-12)
    got_b = np.stack([g_b[:, 1] - g_b[:, 0], g_b[:, 2] - g_b[:, 0]], 1)
    rel_b = np.linalg.norm(got_b - fd_b, axis=1) / np.maximum(np.linalg.norm(fd_b, axis=1), 1e-12)
    print(dict(n_keep=int(keep.sum()), t_med=float(np.median(rel_t[keep])), t_ok=float(np.mean(rel_t[keep] <= 1e-3)),
               b_med=float(np.median(rel_b[keep])), b_ok=float(np.mean(rel_b[keep] <= 1e-3))))
    assert np.mean(rel_t[keep] <= 1e-3) >= 0.999
    assert np.mean(rel_b[keep] <= 1e-3) >= 0.999


def test_transport_back_inverts_transport(torch):
    """Carrying W' back along the same geodesic (from p' with -v') returns W."""
    from paper_2603_15780_amd import sg
    X, F = CF.mesh_config(1)
    rng = np.random.default_rng(94)
    r = random_rays(X, F, 4096, rng, uniform_len(0.0, 2.0), K=2)
    om = oracle.Mesh(X, F)
    o = om.exp(r["f"], r["b"], r["v"], r["W"])
    gm = sg.Mesh(X, F)
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(r[k])).to(dev) for k in ("f", "b", "v", "W")}
    out = gm.exp(t["f"], t["b"], t["v"], t["W"])
    Wb, st = sg.transport_back(gm, out["f"], out["b"], out["v"], out["W"])
    torch.cuda.synchronize()
    Wb = Wb.cpu().numpy()
    ok = (o["status"] == 0) & (o["min_vdist"] > 1e-3 * om.mean_edge) & (st.cpu().numpy() == 0)
    Xd = X.astype(np.float64)
    n0 = np.cross(Xd[F[r["f"], 1]] - Xd[F[r["f"], 0]], Xd[F[r["f"], 2]] - Xd[F[r["f"], 0]])
    n0 /= np.linalg.norm(n0, axis=1)[:, None]
    Wt = r["W"] - (r["W"] * n0[:, None, :]).sum(2)[:, :, None] * n0[:, None, :]
    err = np.linalg.norm(Wb - Wt, axis=2) / np.linalg.norm(Wt, axis=2)
    assert ok.sum() > 1000 and np.quantile(err[ok], 0.999) < 1e-4, np.quantile(err[ok], 0.999)
