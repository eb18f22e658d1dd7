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
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK = {"bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3}   # dense TFLOP/s, MI355X
HBM_PEAK_GBS = 8000.0
W, D = 128, 4


def cosine_lr(i, n, hi=1e-3, lo=1e-5):
    """Adam step size of step i of n: a cosine from hi down to lo."""
    return lo + 0.5 * (hi - lo) * (1.0 + math.cos(math.pi * i / n))


def flop_per_query(width, depth):
    macs = 65 * width + (depth - 1) * width * width + 2 * width
    return 2 * macs


PROFILE = os.path.join(ROOT, "profiles", "forward_bf16_w128d4_2e24rays.md")
KERNEL_SOURCES = ("mlp.hip", "mlp_device.hpp", "mlp_layout.hpp", "rays_device.hpp")


def committed_profile_field(name):
    """A figure of the committed rocprofv3 counter summary of the forward kernel (HBM bytes per
    launch, the clock under load), or None when the kernel sources have changed since those
    counters were taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines() if l.startswith((name, "kernel_source_sha256")))
    src = "".join(open(os.path.join(ROOT, "paper_2306_16142_amd", "csrc", f)).read() for f in KERNEL_SOURCES)
    if fields.get("kernel_source_sha256", "").strip() != hashlib.sha256(src.encode()).hexdigest() or name not in fields:
        return None
    return float(fields[name])


def committed_traffic():
    return committed_profile_field("traffic_bytes_per_launch")


def progress(msg):
    """One line per workload on stderr (the JSON result line is the only stdout output)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for l in open("/proc/cpuinfo"):
            if l.startswith("model name"):
                return l.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def issued_flop_per_query(width, depth, precision):
    """MFMA work the kernel issues per query: layer 0's 65 features padded to the operand's
    K slots (80 in bf16, 128 in fp8), and the head's one 32-row output block (two rows used)."""
    k0 = {"bf16": 80, "fp8": 128}[precision]
    macs = k0 * width + (depth - 1) * width * width + 32 * width
    return 2 * macs


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--quick", action="store_true", help="primary line only (no secondary workloads)")
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--render-spp", type=int, default=64)
    ap.add_argument("--multi-spp", type=int, default=16)
    ap.add_argument("--icosphere-train-steps", type=int, default=1500)
    ap.add_argument("--render-train-steps", type=int, default=5000)
    ap.add_argument("--multi-train-steps", type=int, default=100)
    ap.add_argument("--dataset-s", type=int, default=10, help="s_fc = s_dr = s_p of the dataset sampler workload")
    ap.add_argument("--only", default=None,
                    help="comma list of the workloads to run besides the bf16 primary line (for profiling): "
                         "fp32, fp8, render (labeller, training and render), multi, dataset, udf, paper, eikonal; "
                         "no CPU baseline is taken then")
    ap.add_argument("--save-params", default=None,
                    help="write the in-run trained 4 x 128 icosphere network's float32 parameters to this .npy file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
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


def train_network(torch, api, dev, v, f, tris, width, depth, seed, steps, n_rays=1 << 20, batch=65536, lr=1e-3):
    """Xavier init (seed), then `steps` Adam steps on labeller-labelled training rays of the mesh."""
    import synthetic
    params = torch.from_numpy(synthetic.xavier_params(width, depth, seed)).to(dev)
    if steps == 0:
        return params, {"steps": 0}
    o, d, _ = synthetic.training_rays(v, f, n_rays, seed + 1)
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    t, tri, cr = api.label_rays(og, dg, tris)
    keep = (cr % 2) == 0
    rays = api.assemble_rays(og, dg)[:, keep].contiguous()
    t = t[keep].contiguous()
    tr = api.Trainer(params, width, depth, batch, lr=lr)
    nb = rays.shape[1] // batch
    batches = [(rays[:, i * batch:(i + 1) * batch].contiguous(), t[i * batch:(i + 1) * batch].contiguous()) for i in range(nb)]
    first = float(tr.step(*batches[0]))
    for i in range(1, steps):
        tr.step(*batches[i % nb])
    torch.cuda.synchronize()
    return params, {"steps": steps, "loss_first": first, "loss_last": float(tr.loss)}


def bench_udf(args, torch, api, dev, net, radius):
    """Unsigned distance field (Eq. 5) of the icosphere network on a 32^3 grid x 512 directions."""
    import synthetic
    x_np = synthetic.grid_points(32)
    _, d_np = synthetic.uniform_cube_rays(512, 38)
    x, d = torch.from_numpy(x_np).to(dev), torch.from_numpy(d_np).to(dev)
    n, nd = x.shape[1], d.shape[1]
    ws = torch.empty(api.udf_workspace_bytes(n, nd), device=dev, dtype=torch.uint8)
    u, a = api.udf(net, x, d, workspace=ws)
    torch.cuda.synchronize()
    timer = event_timer(torch)
    for _ in range(5):
        timer.start()
        api.udf(net, x, d, out=u, arg=a, workspace=ws)
        timer.stop()
    torch.cuda.synchronize()
    ms = timer.mean_ms()
    uh = u.cpu().numpy()
    fin = np.isfinite(uh)
    # the icosphere's own unsigned distance, for context on the network's fit
    # (the network was trained on rays from outside the object: points inside are off its data)
    r = np.linalg.norm(x_np.astype(np.float64), axis=0)
    true_u = np.abs(r - radius)
    out = fin & (r > radius)
    return {"udf": {"workload": "32^3 grid points x 512 directions, bf16 4 x 128 icosphere network",
                    "ms": ms, "points_per_s": n / (ms * 1e-3), "queries_per_s": n * nd / (ms * 1e-3),
                    "finite_fraction": float(fin.mean()),
                    "abs_err_vs_icosphere_udf_mean_outside": float(np.abs(uh[out] - true_u[out]).mean()),
                    "abs_err_vs_icosphere_udf_mean_all": float(np.abs(uh[fin] - true_u[fin]).mean())}}


def bench_eikonal(torch, api, dev, net, o_g, d_g, rays):
    """How far the trained network is from the directed Eikonal equation (Sec. III-A, Eq. 2):
    along its own ray the distance falls at unit rate, grad_x phi . d = -1 where the ray hits.
    The input gradient of the distance comes from ddf_backward; sampled rays, hits only."""
    idx = torch.arange(0, rays.shape[1], max(1, rays.shape[1] // 65536), device=dev)[:65536]
    sub = rays[:, idx].contiguous()
    logit, _ = net(sub)
    g_rays, _ = api.backward(net, sub, None, torch.ones(sub.shape[1], device=dev))
    d = d_g[:, idx]
    d = d / d.norm(dim=0, keepdim=True)
    r = (g_rays[:3] * d).sum(dim=0) + 1.0
    hit = logit > 0
    ra = r[hit].abs()
    return {"rays": int(hit.sum()), "abs_residual_mean": float(ra.mean()), "abs_residual_median": float(ra.median()),
            "fraction_below_0.1": float((ra < 0.1).float().mean())}


def bench_eikonal_training(args, torch, api, dev, steps=1500, lam=1.0, h=0.02, batch=65536):
    """The 4 x 128 icosphere network trained with and without the directed Eikonal penalty
    (Eq. 2, forward difference with step h): residual |grad_x phi . d + 1|, distance error and
    hit agreement on held-out rays, and the time per step."""
    import synthetic
    v, f = synthetic.icosphere(2, 0.8)
    tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)

    def labelled(n, seed):
        o, d, _ = synthetic.training_rays(v, f, n, seed)
        og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
        t, _, cr = api.label_rays(og, dg, tris)
        k = (cr % 2) == 0
        og, dg, t = og[:, k].contiguous(), dg[:, k].contiguous(), t[k].contiguous()
        return og, dg, t, api.assemble_rays(og, dg)

    og, dg, t, rays = labelled(1 << 20, 1)
    ho, hd, ht, hrays = labelled(1 << 16, 7)
    nb = rays.shape[1] // batch
    out = {}
    for name, weight in (("plain", 0.0), ("eikonal", lam)):
        tr = api.Trainer(torch.from_numpy(synthetic.xavier_params(128, 4, 0)).to(dev), 128, 4, batch)
        timer = event_timer(torch)
        for s in range(steps):
            sl = slice((s % nb) * batch, (s % nb + 1) * batch)
            batch_args = ((og[:, sl].contiguous(), dg[:, sl].contiguous(), t[sl].contiguous()) if weight
                          else (rays[:, sl].contiguous(), t[sl].contiguous()))
            if s == steps - 20:
                torch.cuda.synchronize()
            if s >= steps - 20:
                timer.start()
            if weight:
                tr.step_eikonal(*batch_args, h=h, lam=weight)
            else:
                tr.step(*batch_args)
            if s >= steps - 20:
                timer.stop()
        torch.cuda.synchronize()
        lg, ds = tr.net(hrays)
        g, _ = api.backward(tr.net, hrays, None, torch.ones(hrays.shape[1], device=dev))
        r = ((g[:3] * (hd / hd.norm(dim=0, keepdim=True))).sum(0) + 1).abs()
        hit = (lg > 0) & torch.isfinite(ht)
        out[name] = {"lambda": weight, "eikonal_abs_residual_mean": float(r[hit].mean()),
                     "dist_abs_err_mean_hits": float((ds[hit] - ht[hit]).abs().mean()),
                     "hit_agreement": float(((lg > 0) == torch.isfinite(ht)).float().mean()),
                     "ms_per_step": timer.mean_ms()}
    out["workload"] = "4 x 128 fp32, icosphere labels, batch %d, %d Adam steps, h = %g; held-out rays" % (
        batch, steps, h)
    return {"eikonal_training": out}


def paper_flop_per_query(depth, width=512):
    return 2 * (5 * width + (depth - 1) * width * width + width)


def bench_paper_network(args, torch, api, dev, depth=8):
    """The paper's own network (Sec. V-A: 8 weight-normalised hidden layers of 512 on the raw
    ray, one distance output): bf16 and float32 queries, bf16 input gradients (normals) and the
    float32 training step with the clamp loss (Eq. 7) on icosphere labels.  Weights: the
    weight-norm start (g = |v|) from a seed, untrained (throughput)."""
    import synthetic
    p = torch.from_numpy(synthetic.paper_params(depth, 81)).to(dev)
    nets = {pr: api.PaperNetwork(p, depth, pr) for pr in ("bf16", "fp32")}
    out = {"workload": "paper network %d x 512 (weight norm folded, raw 5-value input, one output), "
                       "uniform rays; training: batch 65,536, clamp loss delta 1, dropout 0.5 (Sec. V-A)" % depth,
           "flop_per_query": paper_flop_per_query(depth)}
    sizes = {"bf16": 1 << 22, "fp32": 1 << 20}
    for pr, n in sizes.items():
        o, d = synthetic.uniform_cube_rays(n, 82)
        rays = api.assemble_rays(torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev))
        dist = torch.empty(n, device=dev)
        nets[pr](rays, dist)
        torch.cuda.synchronize()
        timer = event_timer(torch)
        for _ in range(5 if pr == "bf16" else 3):
            timer.start()
            nets[pr](rays, dist)
            timer.stop()
        torch.cuda.synchronize()
        ms = timer.mean_ms()
        tf = paper_flop_per_query(depth) * n / (ms * 1e-3) / 1e12
        out[pr] = {"rays": n, "forward_ms": ms, "queries_per_s": n / (ms * 1e-3), "tflops": tf,
                   "roofline_frac": tf / PEAK[pr]}
        if pr == "bf16":
            g = torch.ones(n, device=dev)
            nets[pr].backward(rays, g)
            torch.cuda.synchronize()
            timer = event_timer(torch)
            for _ in range(3):
                timer.start()
                nets[pr].backward(rays, g)
                timer.stop()
            torch.cuda.synchronize()
            gms = timer.mean_ms()
            out[pr]["input_gradient_ms"] = gms
            out[pr]["input_gradients_per_s"] = n / (gms * 1e-3)
            out[pr]["input_gradient_tflops"] = 2 * paper_flop_per_query(depth) * n / (gms * 1e-3) / 1e12
            if not args.quick:
                from oracle import paper
                idx = np.arange(0, n, n // 2048)[:2048]
                sub = rays[:, idx].cpu().numpy().astype(np.float64)
                ref = paper.forward(p.cpu().numpy(), 512, depth, sub)
                got = dist[idx].cpu().numpy()
                e = np.abs(got - ref)
                out[pr]["abs_err_vs_fp64"] = {"mean": float(e.mean()), "p99": float(np.quantile(e, 0.99)),
                                              "max": float(e.max()), "ref_rms": float(np.sqrt(np.mean(ref ** 2)))}
    # float32 training step (clamp loss) on icosphere labels
    v, f = synthetic.icosphere(2, 0.8)
    tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)
    batch = 65536
    o, d, _ = synthetic.training_rays(v, f, batch, 83)
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    t, _, _ = api.label_rays(og, dg, tris)
    rays = api.assemble_rays(og, dg)
    tr = api.PaperTrainer(p.clone(), depth, batch, lr=1e-4, loss="clamp", delta=1.0, dropout=0.5, seed=1)
    first = float(tr.step(rays, t))
    torch.cuda.synchronize()
    steps = 5
    timer = event_timer(torch)
    for _ in range(steps):
        timer.start()
        tr.step(rays, t)
        timer.stop()
    torch.cuda.synchronize()
    ms = timer.mean_ms()
    out["train"] = {"batch": batch, "ms_per_step": ms, "steps_per_s": 1e3 / ms,
                    "tflops": 3 * paper_flop_per_query(depth) * batch / (ms * 1e-3) / 1e12,
                    "loss_first": first, "loss_after": float(tr.loss), "steps": 1 + steps}
    out["train"]["roofline_frac_fp32"] = out["train"]["tflops"] / PEAK["fp32"]
    return {"paper_network": out}


def bench_dataset(args, torch, api, dev):
    """Training-data sampler of Sec. V-B (Eqs. 8-12) on the 20,480-triangle mesh."""
    import synthetic
    from oracle import dataset
    v, f = synthetic.training_mesh(1)
    tris_np = synthetic.tri_soup(v, f)
    tris = torch.from_numpy(tris_np).to(dev)
    m, s, eps = f.shape[0], args.dataset_s, 1e-4
    fu_np, du_np = synthetic.dataset_uniforms(m, s, s, 25)
    fu, du = torch.from_numpy(fu_np).to(dev), torch.from_numpy(du_np).to(dev)
    smp = api.DatasetSampler(tris, s, s, s, eps)
    smp.run(fu, du)
    torch.cuda.synchronize()
    timer = event_timer(torch)
    for _ in range(3):
        timer.start()
        smp.run(fu, du)
        timer.stop()
    torch.cuda.synchronize()
    ms = timer.mean_ms()
    n = int(smp.count.item())
    kept = int(torch.isfinite(smp.t[:n]).sum().item()) // s   # one finite label per marching step
    pairs = m * s * s
    rays = pairs + 2 * kept * s                               # pair rays + perpendicular rays
    out = {"workload": "20,480-triangle mesh, s_fc = s_dr = s_p = %d (%d pairs), eps %g" % (s, pairs, eps),
           "ms": ms, "samples": n, "samples_per_s": n / (ms * 1e-3), "pairs_per_s": pairs / (ms * 1e-3),
           "kept_fraction": kept / pairs, "labeller_rays": rays,
           "ray_triangle_tests_per_s": rays * m / (ms * 1e-3)}
    if not args.quick:
        # the float64 oracle on the host: the pairs of faces 0 and 1, against every triangle
        t0 = time.perf_counter()
        ref = dataset.sample_dataset(tris_np, fu_np, du_np, s, s, s, eps, 0, 2)
        cpu_s = time.perf_counter() - t0
        out["oracle"] = {"pairs_per_s": ref["keep"].size / cpu_s, "samples_per_s": ref["t"].size / cpu_s,
                         "sample": "faces 0-1 (%d pairs), %.1f s" % (ref["keep"].size, cpu_s)}
    del smp
    return {"dataset": out}


def bench_label_train_render(args, torch, api, dev):
    """Labeller and training on the 20,480-triangle workload; render with the trained network."""
    import synthetic
    out = {}
    v, f = synthetic.training_mesh(1)
    tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)
    nl = 1 << 20
    lo, ld, _ = synthetic.training_rays(v, f, nl, 1)
    lo_g, ld_g = torch.from_numpy(lo).to(dev), torch.from_numpy(ld).to(dev)
    t, tri, cr = api.label_rays(lo_g, ld_g, tris)
    torch.cuda.synchronize()
    timer = event_timer(torch)
    for _ in range(3):
        timer.start()
        api.label_rays(lo_g, ld_g, tris)
        timer.stop()
    torch.cuda.synchronize()
    lms = timer.mean_ms()
    out["label"] = {"workload": "2^20 training rays x 20,480-triangle mesh", "kernel_ms": lms,
                    "rays_per_s": nl / (lms * 1e-3), "tests_per_s": nl * f.shape[0] / (lms * 1e-3),
                    "hit_fraction": float((tri >= 0).float().mean())}
    # training set: drop rays whose origin is inside the mesh (odd crossing count)
    keep = (cr % 2) == 0
    rays_all = api.assemble_rays(lo_g, ld_g)[:, keep].contiguous()
    t_all = t[keep].contiguous()
    nvalid = rays_all.shape[1]
    width, depth, batch = 256, 6, 65536
    params = torch.from_numpy(synthetic.xavier_params(width, depth, 1)).to(dev)
    trainer = api.Trainer(params, width, depth, batch, lr=1e-3)
    nb = nvalid // batch
    batches = [(rays_all[:, i * batch:(i + 1) * batch].contiguous(), t_all[i * batch:(i + 1) * batch].contiguous())
               for i in range(nb)]
    losses = []
    for i in range(3):
        losses.append(float(trainer.step(*batches[i % nb])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.train_steps):
        trainer.step(*batches[i % nb])
    torch.cuda.synchronize()
    tms = (time.perf_counter() - t0) * 1e3 / args.train_steps
    losses.append(float(trainer.loss))
    # keep training (untimed) so the rendered network has learned the object; Adam's step size
    # follows a cosine from 1e-3 down to 1e-5 over this stretch
    for i in range(args.render_train_steps):
        trainer.lr = cosine_lr(i, args.render_train_steps)
        trainer.step(*batches[i % nb])
    losses.append(float(trainer.loss))
    torch.cuda.synchronize()
    step_flop = 3 * flop_per_query(width, depth) * batch   # forward, adjoints and weight gradients
    out["train"] = {"workload": "6x256 fp32, batch 65,536, Adam 1e-3, labels from the labeller (%d valid rays)" % nvalid,
                    "ms_per_step": tms, "steps_per_s": 1e3 / tms,
                    "algorithmic_flop_per_step": step_flop, "tflops": step_flop / (tms * 1e-3) / 1e12,
                    "roofline_frac_fp32": step_flop / (tms * 1e-3) / 1e12 / PEAK["fp32"],
                    "loss_first_step": losses[0], "loss_after_%d_steps" % (3 + args.train_steps): losses[-2],
                    "loss_after_%d_steps" % (3 + args.train_steps + args.render_train_steps): losses[-1]}
    # the rendered network: trained as many steps on the rays a renderer asks (cube-entry,
    # surface-leaving and training rays) with the directed Eikonal penalty (Eq. 2, lam 1,
    # h 0.02); the plain network above is its comparison
    ro, rd = synthetic.render_rays(v, f, nl, 1)
    ro_g, rd_g = torch.from_numpy(ro).to(dev), torch.from_numpy(rd).to(dev)
    rt, _, rcr = api.label_rays(ro_g, rd_g, tris)
    rkeep = (rcr % 2) == 0
    ro_g, rd_g, rt = ro_g[:, rkeep].contiguous(), rd_g[:, rkeep].contiguous(), rt[rkeep].contiguous()
    rparams = torch.from_numpy(synthetic.xavier_params(width, depth, 1)).to(dev)
    rtrainer = api.Trainer(rparams, width, depth, batch, lr=1e-3)
    rnb = ro_g.shape[1] // batch
    rbatches = [(ro_g[:, i * batch:(i + 1) * batch].contiguous(), rd_g[:, i * batch:(i + 1) * batch].contiguous(),
                 rt[i * batch:(i + 1) * batch].contiguous()) for i in range(rnb)]
    rsteps = 3 + args.train_steps + args.render_train_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(rsteps):
        rtrainer.lr = cosine_lr(i, rsteps)
        rtrainer.step_eikonal(*rbatches[i % rnb], h=0.02, lam=1.0)
    torch.cuda.synchronize()
    eik_ms = (time.perf_counter() - t0) * 1e3 / rsteps
    # render: 1920 x 1080, spp samples, 4 bounces, Russian roulette after bounce 2, bf16 queries
    cfg = synthetic.full_render(args.render_spp)
    net16 = api.Network(rparams, width, depth, "bf16")
    r = api.Renderer(cfg, net=net16)
    r.capture()   # the frame as one HIP graph; path samples/s from its warm replays
    r.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        r.replay()
    torch.cuda.synchronize()
    rs = (time.perf_counter() - t0) / reps
    paths = cfg.width * cfg.height * cfg.spp
    entering, shadows, hits, queries, _ = r.path_stats()
    entering, shadows = [int(x) for x in entering], [int(x) for x in shadows]
    hits, queries = [int(x) for x in hits], [int(x) for x in queries]
    # network work of the frame from the device queue counts: every ray of a bounce that enters
    # the cube is one query, every hit one input gradient for its normal (the transposed
    # product, the same multiply-adds as the forward), every shadow ray one query.  The kernel
    # runs the reverse sweep for every wave of 32 queries that holds a hit, so it issues more.
    frame_flop = (sum(queries) + sum(hits) + sum(shadows)) * flop_per_query(width, depth)
    # shading normals against the mesh normal at the brute-force hit point (primary hits), and
    # primary-hit agreement, for the rendered network and the plain one
    cfg1 = synthetic.full_render(1)
    cfg1.bounces = 1
    rm = api.Renderer(cfg1, tris=tris)
    rm.render()

    def quality(p16):
        rn = api.Renderer(cfg1, net=p16)
        rn.render()
        torch.cuda.synchronize()
        both = torch.isfinite(rm.depth) & torch.isfinite(rn.depth)
        cosang = (rm.normal * rn.normal).sum(0)[both].clamp(-1, 1)
        ang = torch.rad2deg(torch.acos(cosang)).cpu().numpy()
        agree = float((torch.isfinite(rm.depth) == torch.isfinite(rn.depth)).float().mean()) * 100
        return {"normal_angle_err_deg_mean": float(ang.mean()) if ang.size else None,
                "normal_angle_err_deg_median": float(np.median(ang)) if ang.size else None,
                "primary_hit_agreement_vs_mesh_pct": agree}

    q_render = quality(net16)
    q_plain = quality(api.Network(params, width, depth, "bf16"))
    out["render"] = {"workload": "1920x1080, %d spp, 4 bounces, RR after bounce 2, bf16 6x256 network trained %d "
                                 "directed-Eikonal steps (lam 1, h 0.02, Adam step size cosine 1e-3 -> 1e-5) on render rays"
                                 % (cfg.spp, rsteps),
                     "seconds_per_frame": rs, "path_samples_per_s": paths / rs, "timing": "warm hipGraph replay of the whole frame",
                     "paths_per_bounce": entering, "queries_per_bounce": queries, "hits_per_bounce": hits,
                     "shadow_rays_per_bounce": shadows,
                     "network_flop_per_frame": frame_flop, "network_tflops": frame_flop / rs / 1e12,
                     "roofline_frac_bf16": frame_flop / rs / 1e12 / PEAK["bf16"],
                     **q_render,
                     "render_network_training": {"rays": "render_rays: 1/3 entering the cube, 1/3 leaving the surface, "
                                                         "1/3 training rays (%d kept)" % ro_g.shape[1],
                                                 "eikonal_ms_per_step": eik_ms, "loss_last": float(rtrainer.loss)},
                     "plain_network": {"training": "%d plain steps on training rays (the train workload's network; "
                                                   "the untimed ones with the same cosine step size)" % rsteps,
                                       **q_plain}}
    return out


def bench_multi(args, torch, api, dev):
    """Multi-object scene: 8 procedural objects (seeds 2-9), each with its own network (width
    128 or 256, depth 4-8, briefly trained on labeller output), 16 rigid instances, 1280 x 720,
    16 spp, 3 bounces, bf16 queries."""
    import synthetic
    nets, shapes, tris_counts = [], [], []
    for seed in range(2, 10):
        v, f = synthetic.multi_object_mesh(seed)
        tris_counts.append(int(f.shape[0]))
        width, depth = synthetic.multi_object_network_shape(seed)
        shapes.append((width, depth))
        tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)
        o, d, _ = synthetic.training_rays(v, f, 1 << 18, seed)
        og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
        t, tri, cr = api.label_rays(og, dg, tris)
        keep = (cr % 2) == 0
        rays = api.assemble_rays(og, dg)[:, keep].contiguous()
        t = t[keep].contiguous()
        params = torch.from_numpy(synthetic.xavier_params(width, depth, seed)).to(dev)
        batch = 32768
        tr = api.Trainer(params, width, depth, batch)
        nb = rays.shape[1] // batch
        for i in range(args.multi_train_steps):
            j = i % nb
            tr.step(rays[:, j * batch:(j + 1) * batch].contiguous(), t[j * batch:(j + 1) * batch].contiguous())
        nets.append(api.Network(params, width, depth, "bf16"))
    inst = synthetic.instance_layout(16, 8, seed=10)
    cfg = synthetic.multi_object_render(args.multi_spp)
    r = api.Renderer(cfg, nets=nets, instances=inst)

    def frame():
        r.render()
        return [r.radiance, r.depth, r.normal, r.stats]

    # launch shapes of the persistent network kernel and of the culling, chosen by the
    # autotuner on this scene (outputs checked bit for bit per candidate), then captured
    from paper_2306_16142_amd import autotune
    tuned = autotune.tune("multi_object_%dx%d_%dspp" % (cfg.width, cfg.height, cfg.spp), frame,
                          ["stream_wg_per_cu", "cull_rays_per_block"], reps=5, use_cache=False)
    r.capture()   # one HIP graph per frame (every launch of every bounce and chunk)
    r.replay()
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        r.replay()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    paths, _, _, _, per_net = r.path_stats()
    per_net = per_net.astype(np.float64)
    imb = [float(row.max() / row.mean()) if row.mean() > 0 else None for row in per_net]
    # network work of the nearest-hit passes alone, from the device pair counts: every (ray,
    # instance) pair is one query of its instance's network.  The normals of the hits and the
    # shadow pairs come on top (not counted on the device for these scenes), so the rate is
    # a lower bound on the frame's network work
    main_flop = float(sum(per_net[b][k] * flop_per_query(*shapes[k]) for b in range(per_net.shape[0])
                          for k in range(per_net.shape[1])))
    return {"multi_object": {
        "workload": "8 objects (seeds 2-9, %s triangles), 16 instances, 1280x720, %d spp, 3 bounces, bf16 networks "
                    "(width, depth) = %s trained %d steps each" % (tris_counts, cfg.spp, shapes, args.multi_train_steps),
        "seconds_per_frame": sec, "path_samples_per_s": cfg.width * cfg.height * cfg.spp / sec,
        "timing": "warm hipGraph replay of the whole frame",
        "autotune": {"chosen": tuned["chosen"],
                     "median_ms": {k: {str(v): round(ms, 3) for v, ms in t.items()} for k, t in tuned["median_ms"].items()}},
        "paths_per_bounce": [int(x) for x in paths],
        "pairs_per_network_per_bounce": per_net.astype(np.int64).tolist(),
        "nearest_hit_pass_flop_per_frame": main_flop, "nearest_hit_pass_tflops": main_flop / sec / 1e12,
        "roofline_frac_bf16_lower_bound": main_flop / sec / 1e12 / PEAK["bf16"],
        "queue_imbalance_max_over_mean": imb}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus %d requested): every ray is independent, so the "
              "path would shard by rays, one process per GPU, with no collective in the query or render "
              "loops; that multi-GPU launch is not built." % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synthetic
    from paper_2306_16142_amd import api

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n = 1 << args.n_log2
    o, d = synthetic.uniform_cube_rays(n, 3)
    o_g = torch.from_numpy(o).to(dev)
    d_g = torch.from_numpy(d).to(dev)
    # the precision workload queries the 4 x 128 network trained on the icosphere (labels from
    # the labeller, the training recipe of the 20k-triangle workload, fixed step count)
    ico_v, ico_f = synthetic.icosphere(2, 0.8)
    ico_tris = torch.from_numpy(synthetic.tri_soup(ico_v, ico_f)).to(dev)
    progress("training the icosphere network")
    p_g, train_info = train_network(torch, api, dev, ico_v, ico_f, ico_tris, W, D, seed=0,
                                    steps=0 if args.quick else args.icosphere_train_steps)
    p = p_g.cpu().numpy()
    if args.save_params:
        np.save(args.save_params, p)
    rays = torch.empty((5, n), device=dev)
    logit = torch.empty(n, device=dev)
    dist = torch.empty(n, device=dev)
    calib_o, calib_d = synthetic.uniform_cube_rays(1 << 16, 4)
    calib = api.assemble_rays(torch.from_numpy(calib_o).to(dev), torch.from_numpy(calib_d).to(dev))
    nets = {"bf16": api.Network(p_g, W, D, "bf16"), "fp32": api.Network(p_g, W, D, "fp32")}
    nets["fp8"] = api.Network(p_g, W, D, "fp8", scales=api.fp8_scales(p_g, W, D, calib, nets["fp32"]))
    torch.cuda.synchronize()

    api.assemble_rays(o_g, d_g, out=rays)   # the assembled batch, for the oracle comparisons

    def step(net, timer=None):
        # bf16 / fp8 networks held in LDS: ray assembly fused into the query kernel (ddf_query);
        # float32: ddf_assemble_rays, then ddf_forward
        fused = net.precision != "fp32"
        if not fused:
            api.assemble_rays(o_g, d_g, out=rays)
        if timer:
            timer.start()
        if fused:
            net.query(o_g, d_g, logit, dist)
        else:
            net.forward(rays, logit, dist)
        if timer:
            timer.stop()

    results = {}
    only = None if args.only is None else set(args.only.split(","))
    want = (lambda name: not args.quick and (only is None or name in only))
    for prec in ["bf16"] + [pr for pr in ("fp32", "fp8") if want(pr)]:
        progress("precision workload, %s" % prec)
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
        if not args.quick and only is None:
            from oracle import mlp
            idx = np.arange(0, n, max(1, n // 65536))[:65536]
            sub = rays[:, idx].cpu().numpy()
            if "ref" not in results:
                results["ref"] = mlp.forward(p, W, D, sub.astype(np.float64))
            rl, rd = results["ref"]
            results[prec]["error_vs_fp64"] = error_stats(logit[idx].cpu().numpy(), dist[idx].cpu().numpy(), rl, rd)
            # against the mesh: brute-force labels of the same rays (the query starts at the ray origin)
            if "mesh" not in results:
                mt, mtri, mcr = api.label_rays(o_g[:, idx].contiguous(), d_g[:, idx].contiguous(), ico_tris)
                results["mesh"] = (mt.cpu().numpy(), mtri.cpu().numpy(), mcr.cpu().numpy())
            mt, mtri, mcr = results["mesh"]
            lg, ds = logit[idx].cpu().numpy(), dist[idx].cpu().numpy()
            ml, md = np.where(mtri >= 0, 1.0, -1.0), np.where(mtri >= 0, mt, 0.0)
            out = mcr % 2 == 0   # origin outside the mesh (the training distribution)
            results[prec]["error_vs_mesh"] = {"all_rays": error_stats(lg, ds, ml, md),
                                              "outside_origins": error_stats(lg[out], ds[out], ml[out], md[out])}
    results.pop("ref", None)
    results.pop("mesh", None)

    bf = results["bf16"]
    clock = committed_profile_field("clock_under_load_GHz")
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
        "data": "synthetic: seeded uniform rays; network trained in-run on the icosphere (%d steps)" % train_info["steps"],
        "config": {"workload": "precision query: 2^%d uniform rays, DDF MLP 65->128x4->2 (Fourier 6 freq), "
                               "trained on the 320-triangle icosphere" % args.n_log2,
                   "rays": n, "width": W, "depth": D, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": bf["forward_tflops"], "peak": PEAK["bf16"], "unit": "TFLOP/s",
                     "frac": bf["forward_tflops"] / PEAK["bf16"], "traffic": committed_traffic(),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": 32 * n,
                     "kernel": "forward_kernel<bf16,128,2,lds> with ray assembly fused (ddf_query)",
                     "algorithmic_flop_per_query": flop_per_query(W, D),
                     "issued_flop_per_query": issued_flop_per_query(W, D, "bf16"),
                     # the dense peak scales with the clock, which drops under this load
                     # (GRBM_GUI_ACTIVE per XCD over the kernel time, committed profile)
                     "clock_under_load_GHz": clock,
                     "frac_at_measured_clock": (bf["forward_tflops"] / (PEAK["bf16"] * clock / 2.4)) if clock else None},
    }
    extra = {k: v for k, v in results.items() if k != "bf16"}
    extra["icosphere_training"] = train_info
    extra["bf16"] = {k: v for k, v in bf.items() if k not in ("queries_per_s",)}

    if want("render"):
        progress("labeller, training and render workloads")
        extra.update(bench_label_train_render(args, torch, api, dev))
    if want("multi"):
        progress("multi-object render")
        extra.update(bench_multi(args, torch, api, dev))
    if want("dataset"):
        progress("training-data sampler")
        extra.update(bench_dataset(args, torch, api, dev))
    if want("udf"):
        progress("unsigned distance field")
        extra.update(bench_udf(args, torch, api, dev, nets["bf16"], 0.8))
    if want("paper"):
        progress("the paper's 8 x 512 network")
        extra.update(bench_paper_network(args, torch, api, dev))
    if want("eikonal"):
        progress("Eikonal residual and Eikonal training")
        extra["eikonal_fp32"] = bench_eikonal(torch, api, dev, nets["fp32"], o_g, d_g, rays)
        extra.update(bench_eikonal_training(args, torch, api, dev))
    if not args.quick and only is None:
        # the float64 oracle on the host cores, bounded sample of the same query workload
        from oracle import mlp
        from threadpoolctl import threadpool_info
        ns, nc = 1 << 22, 1 << 19   # evaluated in chunks to bound host memory
        sub = rays[:, :ns].cpu().numpy()
        t0 = time.perf_counter()
        for c0 in range(0, ns, nc):
            mlp.forward(p, W, D, sub[:, c0:c0 + nc].astype(np.float64))
        cpu_s = time.perf_counter() - t0
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        line["cpu_baseline"] = {"value": ns / cpu_s, "unit": "queries/s", "cores": threads, "kind": "oracle",
                                "sample": "float64 NumPy forward of the first 2^22 rays of the batch, in chunks "
                                          "of 2^19 (%.1f s)" % cpu_s,
                                "cores_note": "BLAS threads used by the oracle's matrix products",
                                "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
                                "cpu_model": cpu_model()}
    line["extra"] = extra
    print(json.dumps(line))


if __name__ == "__main__":
    main()
