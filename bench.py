"""Benchmark of the batched exponential map on one MI355X.

Workload (default, --config 2): 1,048,576 rays on the 327,680-face
SH-displaced icosphere (level 7, l <= 8, amplitude 0.1), |v| ~ U[0, pi/2],
two extra vectors transported (K = 2).  --config 3: 64 meshes of uneven size
(displaced spheres and jittered tori, 6.8M faces in all) and 5.6M rays of
uneven length in one persistent call.  Inputs are synthetic and resident in
HBM before timing.  A step is one sg_exp_transport call over the whole batch
with the library's default schedule (--autotune: the schedule the library's
autotuner picks for this batch, tuned untimed).

The forward + backward forms are timed on the same batch and reported
beside it; each backward takes the forward's saved outputs: the extrinsic
proxy walks nothing, geodesic finite differences walk six geodesics per
query (the base geodesic's end is the forward's), and the float64
vertex-position gradient adds one adjoint walk.  `gfd-no-outputs` times GFD
without the forward's outputs (seven walks per query).

With the default config the 64-mesh batch (--config 3) is also run, in a
child process, as HIP-graph replays of one call with the autotuner's
schedule, and reported as `config3` (--no-config3 skips it).

The projection-integration Exp map (the paper's comparison Exp) is timed on
the same batch (`pi`), with its extrinsic proxy and geodesic finite
differences.

Prints one JSON line.  `value` is face-crossings per second (the crossing
count is the float64 oracle's when the CPU-baseline leg traces the whole
batch, else the GPU's).  The roofline object prices the walk kernel against
HBM bandwidth with 16 algorithmic bytes per crossing plus 64 bytes per ray
(its 32-byte state in and out); `whole_call` prices the whole forward call
(16 bytes per crossing plus the queries' 144 + 24 K bytes), and each
fwd_bwd form carries the algorithmic bytes of its backward and their
fraction of the HBM peak over the backward's time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CROSSING = 16
METRIC = "face-crossings/s & queries/s, fwd and fwd+bwd, 327k-face mesh, 1M rays"
WORKLOADS = {
    1: "icosphere level 3 (1,280 faces); 8,192 rays, |v|~U[0,pi/2], K=1; forward",
    2: ("icosphere level 7, SH-displaced (l<=8, amp 0.1), 327,680 faces; 1,048,576 rays, |v|~U[0,pi/2], "
        "K=2 transported; forward (fwd+bwd forms in fwd_bwd)"),
    3: ("64 meshes (displaced geodesic spheres and 3:1 jittered tori, faces log-U[5k,500k]) in one handle; "
        "rays per mesh log-U[16k,256k], |v| log-U[0.01,1] x diameter, K=0; one persistent forward call"),
    5: ("icosphere level 8 (1,310,720 faces), SH-displaced (l<=32, amp 0.1) plus N(0, 0.1 mean edge) normal noise; "
        "16,777,216 rays, |v|~U[0,pi], K=2 (the start frame); forward (fwd+bwd forms in fwd_bwd)"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WALK_SOURCES = ("paper_2603_15780_amd/csrc/sg_kernels.hip", "paper_2603_15780_amd/csrc/sg_internal.h",
                "paper_2603_15780_amd/csrc/sg_launch.h", "paper_2603_15780_amd/csrc/sg_host.cpp",
                "paper_2603_15780_amd/build.py")
TRAFFIC_NOTE = "profiles/k_walk_icosphere7_1M_rays.md"


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (empty if unreadable)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def measured_traffic():
    """HBM bytes per walk launch from the committed counter summary, if it was taken on these sources."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in WALK_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        note = open(os.path.join(ROOT, TRAFFIC_NOTE)).read()
    except OSError:
        return None
    vals = dict(line.strip().split(": ", 1) for line in note.splitlines() if line.strip().startswith("walk_"))
    if vals.get("walk_sources_sha256") != h.hexdigest():
        return None
    return int(vals["walk_traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--kernel", type=int, default=0, help="0 library default (persistent), 1 plain, 2 persistent, 3 partitioned")
    ap.add_argument("--autotune", action="store_true", help="time the autotuner's pick instead of the library defaults")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=0,
                    help="oracle sample size (0: whole batch; 1/4 of it for config 3, 1/64 for config 5)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain kernel for comparison")
    ap.add_argument("--no-bwd", action="store_true", help="skip timing the backward forms")
    ap.add_argument("--bwd-forms", default="ep,gfd,gfd-no-outputs,ep+gradX,gfd+gradX",
                    help="comma-separated backward forms to time (ep, gfd, gfd-no-outputs, ep+gradX, gfd+gradX); "
                         "gfd-no-outputs is GFD without the forward's outputs (it walks the base geodesic too)")
    ap.add_argument("--refill", type=int, default=0, help="persistent kernel refill threshold (0: library default)")
    ap.add_argument("--walk-blocks", type=int, default=0, help="persistent kernel blocks (0: library default, three per CU)")
    ap.add_argument("--queues", type=int, default=0, help="persistent kernel ray queues (0: library default, 8)")
    ap.add_argument("--calib-copy", type=int, default=0, help="MiB copied once to calibrate byte counters")
    ap.add_argument("--graph", type=int, default=-1,
                    help="1: time HIP-graph replays of the call (caller workspace); 0: eager calls; "
                         "-1: graph for the 64-mesh batch, eager otherwise")
    ap.add_argument("--no-pi", action="store_true", help="skip timing the projection-integration map")
    ap.add_argument("--no-config3", action="store_true", help="skip the 64-mesh batch leg of the default run")
    ap.add_argument("--pi-rays", type=int, default=0, help="rays for the PI leg (0: the whole batch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(rays are independent: a multi-GPU run would shard rays and replicate the mesh)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_15780_amd import sg
    from workloads import configs as CF

    t0 = time.time()
    if args.config == 3:
        B = CF.config3_batch(64)
        X, F_or, r = B["X"], B["F_global"], B["rays"]
        mesh_args = (B["X"], B["F_local"], B["vert_offsets"], B["face_offsets"])
    else:
        X, F_or = CF.mesh_config(args.config)
        r = CF.rays_config(args.config, X, F_or)
        mesh_args = (X, F_or)
    n = r["f"].shape[0]
    K = r["W"].shape[1]
    log(f"workload ready in {time.time() - t0:.1f}s: {F_or.shape[0]} faces, {n} rays, K={K}")
    dev = torch.device("cuda:0")
    t1 = time.time()
    mesh = sg.Mesh(*mesh_args)
    pack_s = time.time() - t1
    info = mesh.info()
    log(f"mesh packed in {pack_s:.2f}s ({info['device_bytes'] / 2**20:.1f} MiB on the device)")
    t = {k: torch.from_numpy(np.ascontiguousarray(r[k])).to(dev) for k in ("f", "b", "v")}
    t["W"] = torch.from_numpy(np.ascontiguousarray(r["W"])).to(dev) if K else None
    out = dict(
        f=torch.empty(n, dtype=torch.int32, device=dev), b=torch.empty(n, 3, device=dev),
        p=torch.empty(n, 3, device=dev), v=torch.empty(n, 3, device=dev),
        W=torch.empty(n, K, 3, device=dev) if K else None, status=torch.empty(n, dtype=torch.int32, device=dev),
        n_cross=torch.empty(n, dtype=torch.int32, device=dev), hash=None)

    base = sg.opts(kernel=args.kernel, refill_min=args.refill, walk_blocks=args.walk_blocks, ray_queues=args.queues)
    tuned = None
    if args.graph < 0:
        args.graph = 1 if args.config == 3 else 0
    if args.config == 3 and args.kernel == 0 and not (args.refill or args.walk_blocks or args.queues):
        args.autotune = True   # the 64-mesh batch runs the schedule the autotuner picks for it
    if args.kernel == 0 and args.autotune:
        t1 = time.time()
        base, tune_ms = mesh.autotune(t["f"], t["b"], t["v"], t["W"], o=base)
        tuned = {"kernel": ["auto", "plain", "persistent", "partitioned"][base.kernel], "refill_min": base.refill_min,
                 "walk_blocks": base.walk_blocks, "rays_per_lane": base.rays_per_lane, "ray_queues": base.ray_queues,
                 "tuned_ms": tune_ms, "tuning_s": time.time() - t1}
        log(f"autotuner: {tuned}")

    def opts_for(kernel=None, debug=0):
        o = sg.opts(kernel=base.kernel if kernel is None else kernel, refill_min=base.refill_min,
                    walk_blocks=base.walk_blocks, rays_per_lane=base.rays_per_lane, ray_queues=base.ray_queues)
        o.debug = debug
        return o

    # a caller workspace, allocated once outside the timed region: the calls allocate nothing
    ws_bytes = mesh.exp_workspace_size(n, K, o=opts_for(debug=1))
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)

    def with_ws(o):
        o.workspace = ws.data_ptr()
        o.workspace_bytes = ws.numel()
        return o

    def timed(o, steps, warmup):
        """(wall ms per call, event ms per call, walk-kernel event ms per launch or None,
        median event ms of one call)."""
        for _ in range(warmup):
            mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=o)
        torch.cuda.synchronize()
        mesh.walk_time()   # drop the warm-up launches
        stream = torch.cuda.current_stream()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]   # one between every two calls
        w0 = time.perf_counter()
        evs[0].record(stream)
        for j in range(steps):
            mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=o)
            evs[j + 1].record(stream)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        wms, wn = mesh.walk_time()
        per = sorted(evs[j].elapsed_time(evs[j + 1]) for j in range(steps))
        return ((w1 - w0) * 1e3 / steps, evs[0].elapsed_time(evs[-1]) / steps, (wms / wn if wn else None),
                per[steps // 2] if steps % 2 else 0.5 * (per[steps // 2 - 1] + per[steps // 2]))

    main_o = with_ws(opts_for(debug=1 | (4 if base.kernel != sg.KERNEL_PLAIN else 0)))
    ms_step, ms_call, ms_walk, ms_call_median = timed(main_o, args.steps, args.warmup)
    graph = None
    if args.graph:
        # the same call captured once in a HIP graph and replayed (launch-bound meshes gain most)
        go = with_ws(opts_for(debug=1))
        mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=go)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=go)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        ms_graph = (time.perf_counter() - w0) * 1e3 / args.steps
        graph = {"ms_per_step": ms_graph, "eager_ms_per_step": ms_step}
        log(f"graph replay: {ms_graph:.3f} ms/step (eager {ms_step:.3f})")
        ms_step = ms_graph
    # dominant kernel: the persistent walk (events the library records around it), or the plain kernel
    ms_kernel = ms_walk if ms_walk is not None else ms_call
    gpu_cross = int(out["n_cross"].sum().item())
    n_ok = int((out["status"] == 0).sum().item())
    log(f"timed {args.steps} steps ({tuned or 'kernel %d' % base.kernel}): {ms_step:.3f} ms/step "
        f"(events {ms_kernel:.3f} ms), GPU crossings {gpu_cross}, status ok {n_ok}/{n}")
    plain = None
    if base.kernel != sg.KERNEL_PLAIN and not args.no_plain:
        ms_p, ms_pk, _, _ = timed(opts_for(kernel=sg.KERNEL_PLAIN, debug=1), max(3, args.steps // 4), 1)
        plain = {"ms_per_call": ms_p, "events_ms": ms_pk}
        log(f"plain one-ray-per-lane kernel: {ms_p:.3f} ms/call")

    bwd = None
    if not args.no_bwd and args.config != 3:
        # forward + backward on the same batch: the forward's saved outputs feed the extrinsic
        # proxy; geodesic finite differences re-walk seven geodesics per query (recompute, no paths)
        g_up = torch.from_numpy(CF.upstream_grad(args.config, n)).to(dev)
        gv = torch.empty(n, 3, device=dev)
        gb = torch.empty(n, 3, device=dev)
        gX = torch.zeros(X.shape[0], 3, dtype=torch.float64, device=dev)
        bwd = {}
        fo = opts_for()
        persistent = base.kernel == sg.KERNEL_PERSISTENT
        bo = sg.opts(refill_min=base.refill_min if persistent else 0, walk_blocks=base.walk_blocks if persistent else 0)
        want = set(args.bwd_forms.split(","))
        forms = tuple(fm for fm in (("ep", sg.BWD_EP, False), ("gfd", sg.BWD_GFD, False),
                                    ("gfd-no-outputs", sg.BWD_GFD, False), ("ep+gradX", sg.BWD_EP, True),
                                    ("gfd+gradX", sg.BWD_GFD, True)) if fm[0] in want)
        # The vertex gradient reserves gradx_records records per query (at most 2^30 per call); config 5's
        # 1.1e10 crossings (641 per ray) go through it in slices of 2^20 queries with 800 records each,
        # accumulating into one grad_X.
        gx_slice, gx_records = {5: (1 << 20, 800)}.get(args.config, (n, 0))
        bo_x = sg.opts(refill_min=bo.refill_min, walk_blocks=bo.walk_blocks, gradx_records=gx_records)
        for name, mode, with_x in forms:
            steps = max(3, args.steps // 2)

            def call():
                mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=fo)
                if name == "gfd-no-outputs":
                    mesh.backward(mode, t["f"], t["b"], t["v"], g_up, out=(gv, gb), o=bo)
                    return
                if not with_x:
                    mesh.backward(mode, t["f"], t["b"], t["v"], g_up, f_out=out["f"], b_out=out["b"], v_out=out["v"],
                                  status=out["status"], out=(gv, gb), o=bo)
                    return
                gX.zero_()
                for a in range(0, n, gx_slice):
                    z = slice(a, min(n, a + gx_slice))
                    mesh.backward(mode, t["f"][z], t["b"][z], t["v"][z], g_up[z], f_out=out["f"][z],
                                  b_out=out["b"][z], v_out=out["v"][z], status=out["status"][z],
                                  out=(gv[z], gb[z]), grad_X=gX,
                                  o=bo_x)
            for _ in range(max(1, args.warmup)):
                call()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - w0) * 1e3 / steps
            bwd[name] = {"ms_fwd_plus_bwd": ms, "ms_bwd": ms - ms_step, "queries_per_s": n / (ms * 1e-3),
                         "finite": bool(torch.isfinite(gv).all().item()) and bool(torch.isfinite(gX).all().item()),
                         "mode": name}
            log(f"forward + {name} backward: {ms:.3f} ms/step ({n / (ms * 1e-3):.3e} queries/s)")
    if args.calib_copy:
        # a plain copy of known size, profiled beside the walk to scale the HBM byte counters
        src = torch.empty(args.calib_copy << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy} MiB read + {args.calib_copy} MiB written")

    cross = gpu_cross
    cross_src = "gpu"
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nc = args.cpu_rays or {3: n // 4, 5: n // 64}.get(args.config, n)
        rows = np.arange(n) if nc >= n else np.linspace(0, n - 1, nc).astype(np.int64)
        om = oracle.Mesh(X, F_or)
        # the machine's CPU share is given by OMP_NUM_THREADS when set
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        c0 = time.perf_counter()
        oo = om.exp(r["f"][rows], r["b"][rows], r["v"][rows], r["W"][rows] if K else None, nthreads=cores)
        c1 = time.perf_counter()
        ocross = int(oo["n_cross"].sum())
        if rows.shape[0] == n:
            cross, cross_src = ocross, "oracle"
        cpu = {"value": ocross / (c1 - c0), "unit": "face-crossings/s", "cores": cores, "kind": "oracle",
               "sample": f"{rows.shape[0]} of the {n} rays (K={K}), float64 C oracle, {cores} threads, "
                         f"{c1 - c0:.2f} s",
               "queries_per_s": rows.shape[0] / (c1 - c0), "cpu_model": cpu_model(),
               "host_cpus": os.cpu_count()}
        log(f"oracle: {ocross} crossings in {c1 - c0:.2f}s on {cores} threads; GPU/oracle crossing ratio "
            f"{gpu_cross / max(ocross, 1) if rows.shape[0] == n else float('nan'):.6f}")
    if bwd:
        # algorithmic bytes of each backward (the paper's schemes, counted per query and per crossing):
        # EP streams ~152 B per query (query, saved f' and v', g, both gradients, start and end
        # faces' vertices) and walks nothing; GFD walks three long geodesics (the e_perp-perturbed
        # one and the two start-shifted ones; the base geodesic is the forward's, and the three
        # short ones cross almost nothing) at 16 B per crossing, with 64 B of chart state in and
        # out per walk and query (without the forward's outputs it walks the base geodesic as well);
        # the vertex gradient adds one adjoint walk (16 B per crossing), the float64 sums (6 per
        # half-edge) and grad_X (24 B per vertex).
        n_he = 3 * int(F_or.shape[0])
        per_q = 152
        algo = {"ep": n * per_q,
                "gfd": 3 * cross * BYTES_PER_CROSSING + n * (per_q + 6 * 64),
                "gfd-no-outputs": 4 * cross * BYTES_PER_CROSSING + n * (per_q + 7 * 64)}
        gx_extra = cross * BYTES_PER_CROSSING + n * 64 + n_he * 6 * 8 + int(X.shape[0]) * 24
        algo["ep+gradX"] = algo["ep"] + gx_extra
        algo["gfd+gradX"] = algo["gfd"] + gx_extra
        for name, b in bwd.items():   # forward-path crossings per second of the whole fwd + bwd step
            b["crossings_per_s"] = cross / (b["ms_fwd_plus_bwd"] * 1e-3)
            b["algorithmic_bytes_bwd"] = algo[name]
            b["frac_bwd"] = algo[name] / (b["ms_bwd"] * 1e-3) / 1e9 / HBM_PEAK_GBS if b["ms_bwd"] > 0 else None
            b.pop("mode", None)

    pi = None
    if not args.no_pi and args.config in (1, 2):
        # the projection-integration Exp (float64 steps of s = 0.01, grid search for the nearest
        # point), its EP from the saved outputs and its GFD (seven PI maps per query), on the same
        # batch or its first --pi-rays rays
        npi = min(n, args.pi_rays) if args.pi_rays else n
        tp = {k: (vv[:npi].contiguous() if vv is not None else None) for k, vv in t.items()}
        g_pi = torch.from_numpy(CF.upstream_grad(args.config, npi)).to(dev)

        def pi_timed(fn, steps):
            fn()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - w0) * 1e3 / steps
        po = {}
        ms_pi = pi_timed(lambda: po.update(mesh.pi_exp(tp["f"], tp["b"], tp["v"], tp["W"], want_steps=True)), 3)
        psteps = int(po["n_steps"].sum().item())
        ms_pi_ep = pi_timed(lambda: mesh.pi_backward(sg.BWD_EP, tp["f"], tp["b"], tp["v"], g_pi, f_out=po["f"],
                                                     v_out=po["v"]), 3)
        ms_pi_gfd = pi_timed(lambda: mesh.pi_backward(sg.BWD_GFD, tp["f"], tp["b"], tp["v"], g_pi), 2)
        ms_sg = ms_step * npi / n   # the straightest map on the same rays (per-ray share of the timed call)
        pi = {"rays": npi, "step": 0.01, "search": "grid", "precision": "f64",
              "ms_per_call": ms_pi, "queries_per_s": npi / (ms_pi * 1e-3), "projection_steps": psteps,
              "steps_per_s": psteps / (ms_pi * 1e-3), "ms_ep_bwd": ms_pi_ep, "ms_gfd_bwd": ms_pi_gfd,
              "slowdown_vs_straightest": ms_pi / ms_sg}
        log(f"PI exp map: {ms_pi:.2f} ms for {npi} rays ({psteps} projection steps), EP {ms_pi_ep:.2f} ms, "
            f"GFD {ms_pi_gfd:.2f} ms; {ms_pi / ms_sg:.1f}x the straightest map's time")

    # algorithmic bytes: 16 per crossing (next face's shape in the crossed edge's frame and its two
    # onward links); per ray the walk kernel reads and writes a 32-byte chart state, while the whole
    # forward call reads the query and writes the answer (144 + 24 K bytes)
    walk_bytes = cross * BYTES_PER_CROSSING + n * 64
    call_bytes = cross * BYTES_PER_CROSSING + n * (144 + 24 * K)
    algo_bytes = walk_bytes if ms_walk is not None else call_bytes
    achieved = algo_bytes / (ms_kernel * 1e-3) / 1e9
    res = {
        "metric": METRIC,
        "value": cross / (ms_step * 1e-3),
        "unit": "face-crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median_events": ms_call_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config],
            "faces": int(F_or.shape[0]), "rays": n, "K": K, "crossings": cross, "crossings_from": cross_src,
            "schedule": tuned or {"kernel": ["default", "plain", "persistent", "partitioned"][args.kernel]},
        },
        "plain_kernel": plain,
        "speedup_over_plain": (plain["ms_per_call"] / ms_step) if plain else None,
        "queries_per_s": n / (ms_step * 1e-3),
        "fwd_bwd": bwd,
        "pi": pi,
        "graph": graph,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if (args.config == 2 and ms_walk is not None and not tuned
                                                       and args.kernel in (0, 2) and not args.refill
                                                       and not args.walk_blocks and not args.queues) else None,
                     "kernel": "k_walk (persistent walk)" if ms_walk is not None else "k_exp_plain",
                     "algorithmic_bytes_per_launch": algo_bytes, "kernel_ms": ms_kernel,
                     # what the walk's loads request from the cache hierarchy per crossing (its 32-byte
                     # face record), over the same time: an L2 request rate, not HBM traffic
                     "l2_request_GBs_at_32B": (32 * cross + (algo_bytes - 16 * cross)) / (ms_kernel * 1e-3) / 1e9,
                     "whole_call": {"ms": ms_step, "algorithmic_bytes": call_bytes,
                                    "achieved_GBs": call_bytes / (ms_step * 1e-3) / 1e9,
                                    "frac": call_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                    "target_frac": 0.40,
                                    "meets_target": call_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS >= 0.40}},
        "cpu_baseline": cpu,
        "mesh_device_bytes": info["device_bytes"],
        "mesh_pack_s": pack_s,
        "config3": None,
    }
    if args.config == 2 and not args.no_config3:
        res["config3"] = config3_leg()
    print(json.dumps(res), flush=True)


def config3_leg():
    """The 64-mesh batch as HIP-graph replays with the autotuner's schedule, run by
    this script in a child process (its own workload and device memory)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--config", "3", "--steps", "20", "--warmup", "3",
           "--no-cpu-baseline", "--no-plain", "--no-bwd", "--no-pi"]
    log("64-mesh batch leg: " + " ".join(cmd[1:]))
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600)
    except subprocess.TimeoutExpired:
        return {"error": "timed out"}
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": f"exit status {p.returncode}"}
    r = json.loads(lines[-1])
    rf = r["roofline"]
    return {"workload": r["config"]["workload"], "faces": r["config"]["faces"], "rays": r["config"]["rays"],
            "crossings": r["config"]["crossings"], "schedule": r["config"]["schedule"],
            "graph_replay": True, "ms_per_step": r["ms_per_step"], "eager_ms_per_step": r["graph"]["eager_ms_per_step"],
            "crossings_per_s": r["value"], "queries_per_s": r["queries_per_s"],
            "walk_ms": rf["kernel_ms"], "walk_frac": rf["frac"], "whole_call_frac": rf["whole_call"]["frac"]}


if __name__ == "__main__":
    main()
