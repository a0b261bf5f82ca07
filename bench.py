"""Benchmark of the batched exponential map on one MI355X.

Workload (default): 1,048,576 rays on the 327,680-face SH-displaced
icosphere (level 7, l <= 8, amplitude 0.1), |v| ~ U[0, pi/2], two extra
vectors transported (K = 2).  Inputs are synthetic and resident in HBM
before timing.  A step is one sg_exp_transport call over the whole batch.

The forward + backward forms (extrinsic proxy from the saved outputs, and
geodesic finite differences, which re-walk seven geodesics per query) are
timed on the same batch and reported beside it.

Prints one JSON line.  `value` is face-crossings per second (the crossing
count is the float64 oracle's, computed on the same batch in the CPU-baseline
leg).  The roofline object prices the walk kernel against HBM bandwidth with
16 algorithmic bytes per crossing plus 144 + 24 K bytes per query.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2])
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 plain, 2 persistent")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=0, help="oracle sample size (0: whole batch)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain kernel for comparison")
    ap.add_argument("--refill", type=int, default=0, help="persistent kernel refill threshold (0: library default)")
    ap.add_argument("--walk-blocks", type=int, default=0, help="persistent kernel blocks (0: fill the GPU)")
    ap.add_argument("--no-bwd", action="store_true", help="skip timing the backward (EP and GFD)")
    ap.add_argument("--calib-copy", type=int, default=0, help="MiB copied once to calibrate byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(rays are independent: a multi-GPU run would shard rays and replicate the mesh)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_15780_amd import sg
    from workloads import configs as CF

    t0 = time.time()
    X, F = CF.mesh_config(args.config)
    r = CF.rays_config(args.config, X, F)
    n = r["f"].shape[0]
    K = r["W"].shape[1]
    log(f"workload ready in {time.time() - t0:.1f}s: {F.shape[0]} faces, {n} rays, K={K}")
    dev = torch.device("cuda:0")
    mesh = sg.Mesh(X, F)
    info = mesh.info()
    t = {k: torch.from_numpy(np.ascontiguousarray(r[k])).to(dev) for k in ("f", "b", "v", "W")}
    out = dict(
        f=torch.empty(n, dtype=torch.int32, device=dev), b=torch.empty(n, 3, device=dev),
        p=torch.empty(n, 3, device=dev), v=torch.empty(n, 3, device=dev),
        W=torch.empty(n, K, 3, device=dev), status=torch.empty(n, dtype=torch.int32, device=dev),
        n_cross=torch.empty(n, dtype=torch.int32, device=dev), hash=None)
    def timed(kernel, steps, warmup):
        """(wall ms per call, event ms per call, walk-kernel event ms per launch or None)."""
        o = sg.opts(kernel=kernel, debug=1 | (4 if kernel != 1 else 0), refill_min=args.refill,
                    walk_blocks=args.walk_blocks)
        for _ in range(warmup):
            mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=o)
        torch.cuda.synchronize()
        mesh.walk_time()   # drop the warm-up launches
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=o)
        ev1.record(stream)
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        wms, wn = mesh.walk_time()
        return (w1 - w0) * 1e3 / steps, ev0.elapsed_time(ev1) / steps, (wms / wn if wn else None)

    ms_step, ms_call, ms_walk = timed(args.kernel, args.steps, args.warmup)
    # dominant kernel: the persistent walk (events the library records around it), or the plain kernel
    ms_kernel = ms_walk if ms_walk is not None else ms_call
    gpu_cross = int(out["n_cross"].sum().item())
    n_ok = int((out["status"] == 0).sum().item())
    log(f"timed {args.steps} steps (kernel {args.kernel}): {ms_step:.3f} ms/step (events {ms_kernel:.3f} ms), "
        f"GPU crossings {gpu_cross}, status ok {n_ok}/{n}")
    plain = None
    if args.kernel != 1 and not args.no_plain:
        ms_p, ms_pk, _ = timed(1, max(3, args.steps // 4), 1)
        plain = {"ms_per_call": ms_p, "events_ms": ms_pk}
        log(f"plain one-ray-per-lane kernel: {ms_p:.3f} ms/call")
    bwd = None
    if not args.no_bwd:
        # forward + backward on the same batch: the forward's saved outputs feed the extrinsic
        # proxy; geodesic finite differences re-walk seven geodesics per query (recompute, no paths)
        g_up = torch.from_numpy(CF.upstream_grad(args.config, n)).to(dev)
        gv = torch.empty(n, 3, device=dev)
        gb = torch.empty(n, 3, device=dev)
        bwd = {}
        fo = sg.opts(kernel=args.kernel, refill_min=args.refill, walk_blocks=args.walk_blocks)
        for name, mode in (("ep", sg.BWD_EP), ("gfd", sg.BWD_GFD)):
            steps = max(3, args.steps // 2)
            def call():
                mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=fo)
                mesh.backward(mode, t["f"], t["b"], t["v"], g_up, f_out=out["f"], v_out=out["v"], out=(gv, gb), o=fo)
            for _ in range(max(1, args.warmup)):
                call()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - w0) * 1e3 / steps
            bwd[name] = {"ms_fwd_plus_bwd": ms, "ms_bwd": ms - ms_step, "queries_per_s": n / (ms * 1e-3),
                         "finite": bool(torch.isfinite(gv).all().item())}
            log(f"forward + {name} backward: {ms:.3f} ms/step ({n / (ms * 1e-3):.3e} queries/s)")
    if args.calib_copy:
        # a plain copy of known size, profiled beside the walk to scale the HBM byte counters
        src = torch.empty(args.calib_copy << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy} MiB read + {args.calib_copy} MiB written")

    cross = gpu_cross
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nc = args.cpu_rays or n
        om = oracle.Mesh(X, F)
        # the machine's CPU share is given by OMP_NUM_THREADS when set
        cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        c0 = time.perf_counter()
        oo = om.exp(r["f"][:nc], r["b"][:nc], r["v"][:nc], r["W"][:nc], nthreads=cores)
        c1 = time.perf_counter()
        ocross = int(oo["n_cross"].sum())
        if nc == n:
            cross = ocross
        cpu = {"value": ocross / (c1 - c0), "unit": "face-crossings/s", "cores": cores, "kind": "oracle",
               "sample": f"{nc} of the {n} rays (K={K}), float64 C oracle, {cores} threads, {c1 - c0:.2f} s",
               "queries_per_s": nc / (c1 - c0)}
        log(f"oracle: {ocross} crossings in {c1 - c0:.2f}s on {cores} threads; GPU/oracle crossing ratio "
            f"{gpu_cross / max(ocross, 1) if nc == n else float('nan'):.6f}")

    if bwd:
        for b in bwd.values():   # forward-path crossings per second of the whole fwd + bwd step
            b["crossings_per_s"] = cross / (b["ms_fwd_plus_bwd"] * 1e-3)
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("icosphere level 7, SH-displaced (l<=8, amp 0.1), 327,680 faces; 1,048,576 rays, "
                         "|v|~U[0,pi/2], K=2 transported; forward only" if args.config == 2 else
                         "icosphere level 3 (1,280 faces); 8,192 rays, |v|~U[0,pi/2], K=1; forward only"),
            "faces": int(F.shape[0]), "rays": n, "K": K, "crossings": cross,
            "kernel": ["persistent (auto)", "plain", "persistent"][args.kernel],
        },
        "plain_kernel": plain,
        "fwd_bwd": bwd,
        "speedup_over_plain": (plain["ms_per_call"] / ms_step) if plain else None,
        "queries_per_s": n / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_walk (persistent walk)" if ms_walk is not None else "k_exp_plain",
                     "algorithmic_bytes_per_launch": algo_bytes, "kernel_ms": ms_kernel,
                     "whole_call": {"ms": ms_call, "algorithmic_bytes": call_bytes,
                                    "achieved_GBs": call_bytes / (ms_call * 1e-3) / 1e9}},
        "cpu_baseline": cpu,
        "mesh_device_bytes": info["device_bytes"],
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
