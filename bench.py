"""Benchmark of the directional-distance-field hot path on one MI355X.

Primary line (``value``): DDF queries/s of the batched network query in bfloat16 on the
precision workload -- 2^24 uniform rays (origin U([-1,1]^3), direction uniform on S^2,
seed 3) through the 4 x 128 Fourier-encoded network (Xavier init, seed 0).  One step is
the whole query path for the batch: ray assembly (direction -> angles) and the network
forward (encoding, 4 hidden MFMA layers, head).  Inputs are resident in HBM before the
timed region starts.

Also reported (``extra``): the same workload in float32 and fp8 (e4m3, static per-layer
scales), each with its distance abs-err / hit agreement against the float64 oracle on a
sample, the labeller's rays/s on the training workload (2^20 rays x 20,480 triangles),
the roofline of the dominant kernel and the float64 CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK = {"bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}   # dense TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0
W, D = 128, 4


def flop_per_query(width, depth):
    macs = 65 * width + (depth - 1) * width * width + 2 * width
    return 2 * macs


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="primary line only (no secondary workloads)")
    ap.add_argument("--n-log2", type=int, default=24)
    return ap.parse_args()


def event_timer(torch):
    class T:
        def __init__(self):
            self.pairs = []

        def start(self):
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.pairs.append([e, None])

        def stop(self):
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            self.pairs[-1][1] = e

        def mean_ms(self):
            return float(np.mean([a.elapsed_time(b) for a, b in self.pairs]))
    return T()


def error_stats(logit, dist, ref_logit, ref_dist):
    hit_ref = ref_logit > 0
    agree = float(np.mean((logit > 0) == hit_ref)) * 100.0
    e = np.abs(dist[hit_ref] - ref_dist[hit_ref])
    return {"hit_agreement_pct": round(agree, 4), "dist_abs_err_mean": float(e.mean()),
            "dist_abs_err_p99": float(np.quantile(e, 0.99)), "dist_abs_err_max": float(e.max())}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X here "
              "(--gpus %d requested). See DESIGN.md for how it would shard." % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synthetic
    from paper_2306_16142_amd import api

    dev = torch.device("cuda:0")
    n = 1 << args.n_log2
    o, d = synthetic.uniform_cube_rays(n, 3)
    p = synthetic.xavier_params(W, D, 0)
    o_g = torch.from_numpy(o).to(dev)
    d_g = torch.from_numpy(d).to(dev)
    p_g = torch.from_numpy(p).to(dev)
    rays = torch.empty((5, n), device=dev)
    logit = torch.empty(n, device=dev)
    dist = torch.empty(n, device=dev)
    calib_o, calib_d = synthetic.uniform_cube_rays(1 << 16, 4)
    calib = api.assemble_rays(torch.from_numpy(calib_o).to(dev), torch.from_numpy(calib_d).to(dev))
    nets = {"bf16": api.Network(p_g, W, D, "bf16"), "fp32": api.Network(p_g, W, D, "fp32")}
    nets["fp8"] = api.Network(p_g, W, D, "fp8", scales=api.fp8_scales(p_g, W, D, calib, nets["fp32"]))
    torch.cuda.synchronize()

    def step(net, timer=None):
        api.assemble_rays(o_g, d_g, out=rays)
        if timer:
            timer.start()
        net.forward(rays, logit, dist)
        if timer:
            timer.stop()

    results = {}
    for prec in (["bf16"] if args.quick else ["bf16", "fp32", "fp8"]):
        net = nets[prec]
        steps = args.steps if prec != "fp32" else max(3, args.steps // 4)
        # cold: first call after packing (the paper notes the first render is slower)
        t0 = time.perf_counter()
        step(net)
        torch.cuda.synchronize()
        cold_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(args.warmup):
            step(net)
        torch.cuda.synchronize()
        timer = event_timer(torch)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(net, timer)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kern_ms = timer.mean_ms()
        results[prec] = {"ms_per_step": ms, "queries_per_s": n / (ms * 1e-3), "forward_kernel_ms": kern_ms,
                         "forward_tflops": flop_per_query(W, D) * n / (kern_ms * 1e-3) / 1e12,
                         "cold_first_step_ms": cold_ms, "steps": steps}
        # accuracy against the float64 oracle on a fixed sample of the batch
        if not args.quick:
            from oracle import mlp
            idx = np.arange(0, n, max(1, n // 65536))[:65536]
            sub = rays[:, idx].cpu().numpy()
            if "ref" not in results:
                results["ref"] = mlp.forward(p, W, D, sub.astype(np.float64))
            rl, rd = results["ref"]
            results[prec]["error_vs_fp64"] = error_stats(logit[idx].cpu().numpy(), dist[idx].cpu().numpy(), rl, rd)
    results.pop("ref", None)

    bf = results["bf16"]
    line = {
        "metric": "DDF queries/s (bf16 MFMA forward incl. ray assembly)",
        "value": bf["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic: seeded uniform rays; Xavier-initialised network (no trained weights)",
        "config": {"workload": "precision query: 2^%d uniform rays, DDF MLP 65->128x4->2 (Fourier 6 freq)" % args.n_log2,
                   "rays": n, "width": W, "depth": D, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": bf["forward_tflops"], "peak": PEAK["bf16"], "unit": "TFLOP/s",
                     "frac": bf["forward_tflops"] / PEAK["bf16"], "traffic": None,
                     "kernel": "forward_kernel<bf16,128,2,lds>",
                     "algorithmic_flop_per_query": flop_per_query(W, D)},
    }
    extra = {k: v for k, v in results.items() if k != "bf16"}
    extra["bf16"] = {k: v for k, v in bf.items() if k not in ("queries_per_s",)}

    if not args.quick:
        # labeller on the training workload
        v, f = synthetic.training_mesh(1)
        tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)
        lo, ld, _ = synthetic.training_rays(v, f, 1 << 20, 1)
        lo_g, ld_g = torch.from_numpy(lo).to(dev), torch.from_numpy(ld).to(dev)
        api.label_rays(lo_g, ld_g, tris)
        torch.cuda.synchronize()
        timer = event_timer(torch)
        for _ in range(3):
            timer.start()
            api.label_rays(lo_g, ld_g, tris)
            timer.stop()
        torch.cuda.synchronize()
        lms = timer.mean_ms()
        extra["label"] = {"rays": 1 << 20, "triangles": int(f.shape[0]), "kernel_ms": lms,
                          "rays_per_s": (1 << 20) / (lms * 1e-3),
                          "tests_per_s": (1 << 20) * f.shape[0] / (lms * 1e-3)}
        # the float64 oracle on the host cores, bounded sample of the same query workload
        from oracle import mlp
        from threadpoolctl import threadpool_info
        ns = 1 << 18
        sub = rays[:, :ns].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        mlp.forward(p, W, D, sub)
        cpu_s = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line["cpu_baseline"] = {"value": ns / cpu_s, "unit": "queries/s", "cores": threads, "kind": "oracle",
                                "sample": "float64 NumPy forward of the first 2^18 rays of the batch (%.1f s)" % cpu_s}
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
