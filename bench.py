"""Benchmark of the batched exponential map on one MI355X.

Workload (default): 1,048,576 rays on the 327,680-face SH-displaced
icosphere (level 7, l <= 8, amplitude 0.1), |v| ~ U[0, pi/2], two extra
vectors transported (K = 2).  Inputs are synthetic and resident in HBM
before timing.  A step is one sg_exp_transport call over the whole batch.

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
    o = sg.opts(kernel=args.kernel, debug=1)

    def step():
        mesh.exp(t["f"], t["b"], t["v"], t["W"], out=out, o=o)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ms_step = (w1 - w0) * 1e3 / args.steps
    ms_kernel = ev0.elapsed_time(ev1) / args.steps
    gpu_cross = int(out["n_cross"].sum().item())
    n_ok = int((out["status"] == 0).sum().item())
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (events {ms_kernel:.3f} ms), "
        f"GPU crossings {gpu_cross}, status ok {n_ok}/{n}")

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

    algo_bytes = cross * BYTES_PER_CROSSING + n * (144 + 24 * K)
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
            "kernel": ["auto", "plain", "persistent"][args.kernel],
        },
        "queries_per_s": n / (ms_step * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": algo_bytes, "kernel_ms": ms_kernel},
        "cpu_baseline": cpu,
        "mesh_device_bytes": info["device_bytes"],
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
