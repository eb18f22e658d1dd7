"""GPU parity of the hand-written backward (input and parameter gradients), the loss seeds,
Adam and a whole training step, against the float64 oracle."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import mlp
from paper_2306_16142_amd import api

from gpu_common import banner, cuda, host, rays5_from

pytestmark = pytest.mark.gpu


def _rays(n, seed):
    o, d = synthetic.uniform_cube_rays(n, seed)
    return rays5_from(o, d)


def _away_from_kinks(p, width, depth, rays, tol=1e-4):
    """Rays whose every hidden pre-activation is at least `tol` from the ReLU kink (float64):
    float32 and float64 then take the same branch, so gradients can be compared tightly."""
    _, _, _, pres = mlp.forward(p, width, depth, rays, return_acts=True)
    m = np.ones(rays.shape[1], dtype=bool)
    for z in pres[:-1]:
        m &= np.abs(z).min(axis=0) > tol
    return np.ascontiguousarray(rays[:, m])


def _rel(g, r):
    scale = max(np.sqrt(np.mean(r ** 2)), 1e-30)
    return np.abs(g - r) / np.maximum(np.abs(r), scale)


def _robust_batch(p, width, depth, rays, t, loss="bce_l1", delta=1.0, extra_rays=(), tol=1e-4):
    """Mask of rays on which float32 and float64 take every branch of the step the same way:
    each hidden pre-activation at least `tol` from the ReLU kink (also on `extra_rays`, the
    moved copies of an Eikonal step), and the loss's own branch points clear of the distance
    (the L1 sign, the clamp window's edges and sign, the squish sign)."""
    m = np.ones(rays.shape[1], dtype=bool)
    for r in (rays,) + tuple(extra_rays):
        _, _, _, pres = mlp.forward(p, width, depth, r, return_acts=True)
        for z in pres[:-1]:
            m &= np.abs(z).min(axis=0) > tol
    _, ds = mlp.forward(p, width, depth, rays)
    tt = t.astype(np.float64)
    hit = np.isfinite(tt)
    if loss == "bce_l1":
        m &= ~hit | (np.abs(ds - np.where(hit, tt, 0.0)) > tol)
    elif loss == "clamp":
        m &= (np.abs(np.abs(ds) - delta) > tol) & (np.abs(np.clip(ds, -delta, delta) - np.clip(tt, -delta, delta)) > tol)
    else:
        m &= np.abs(np.tanh(ds) - np.tanh(tt)) > tol
    return m


def _per_layer_close(g, ref, width, depth, tol):
    """Every affine layer's weight and bias gradients separately: max |g - ref| within `tol`
    of that slice's largest reference component (a fault confined to one layer, the head or
    a chunk edge cannot hide behind the other layers)."""
    off, worst = 0, 0.0
    for o, i in synthetic.layer_shapes(width, depth):
        for cnt in (o * i, o):
            sl = slice(off, off + cnt)
            off += cnt
            big = np.abs(ref[sl]).max()
            if big == 0.0:
                assert not g[sl].any()
                continue
            worst = max(worst, np.abs(g[sl] - ref[sl]).max() / big)
    assert off == ref.size
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("width,depth,n", [(128, 4, 4096 + 21), (256, 6, 1024 + 3), (128, 1, 64)])
def test_input_gradient_fp32(width, depth, n):
    banner("input gradient fp32 %dx%d n=%d" % (depth, width, n))
    p = synthetic.random_params(width, depth, 31)
    rays = _away_from_kinks(p, width, depth, _rays(n, 32))
    n = rays.shape[1]
    rng = np.random.default_rng(0)
    gl, gd = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    net = api.Network(cuda(p), width, depth, "fp32")
    g_rays, _ = api.backward(net, cuda(rays), cuda(gl), cuda(gd))
    ref, _ = mlp.backward(p, width, depth, rays, gl, gd)
    err = _rel(host(g_rays), ref)
    assert err.max() < 1e-4
    assert np.median(err) < 1e-6


@pytest.mark.parametrize("width,depth,n", [(128, 4, 8192), (256, 6, 2048 + 7), (128, 1, 100), (256, 8, 512 + 1),
                                           (128, 7, 1000)])
def test_input_gradient_bf16_normals(width, depth, n):
    """bf16 input gradients (the streamed kernel at every width, odd and even depths, ragged n)."""
    banner("input gradient bf16 %dx%d n=%d (distance seed = normals)" % (depth, width, n))
    p = synthetic.random_params(width, depth, 33)
    rays = _rays(n, 34)
    net = api.Network(cuda(p), width, depth, "bf16")
    ones = np.ones(n, np.float32)
    g_rays, _ = api.backward(net, cuda(rays), None, cuda(ones))
    ref, _ = mlp.backward(p, width, depth, rays, np.zeros(n), ones)
    g = host(g_rays)
    emu = mlp.backward_input_bf16(p, width, depth, rays, np.zeros(n), ones)

    def angle(x, y):
        a = x[:3] / np.linalg.norm(x[:3], axis=0)
        b = y[:3] / np.linalg.norm(y[:3], axis=0)
        return np.degrees(np.arccos(np.clip(np.sum(a * b, axis=0), -1, 1)))

    # the kernel must sit much closer to the bf16 emulation than the emulation sits to float64
    own = angle(emu, ref)
    gap = angle(g, emu)
    assert np.median(gap) < 0.2 * np.median(own)
    assert np.quantile(gap, 0.9) < 0.5 * np.quantile(own, 0.9)
    assert np.mean(angle(g, ref)) < 1.2 * np.mean(own)


@pytest.mark.parametrize("width,depth,n", [(128, 4, 8192 + 5), (256, 6, 4096)])
def test_parameter_gradient_fp32(width, depth, n):
    banner("parameter gradient fp32 %dx%d n=%d" % (depth, width, n))
    p = synthetic.random_params(width, depth, 35)
    rays = _away_from_kinks(p, width, depth, _rays(n, 36))
    n = rays.shape[1]
    rng = np.random.default_rng(1)
    gl, gd = rng.normal(size=n).astype(np.float32) / n, rng.normal(size=n).astype(np.float32) / n
    net = api.Network(cuda(p), width, depth, "fp32")
    g_rays, g_params = api.backward(net, cuda(rays), cuda(gl), cuda(gd), want_params=True)
    ref_r, ref_p = mlp.backward(p, width, depth, rays, gl, gd)
    gp = host(g_params)
    scale = np.sqrt(np.mean(ref_p ** 2))
    assert np.max(np.abs(gp - ref_p)) < 1e-5 * np.abs(ref_p).max()
    assert np.median(np.abs(gp - ref_p) / np.maximum(np.abs(ref_p), scale)) < 1e-5
    assert np.quantile(_rel(host(g_rays), ref_r), 0.999) < 1e-4
    # accumulate flag adds, and a second identical call is bitwise identical
    _, g2 = api.backward(net, cuda(rays), cuda(gl), cuda(gd), want_params=True)
    assert torch.equal(g_params, g2)
    _, g3 = api.backward(net, cuda(rays), cuda(gl), cuda(gd), want_params=True, g_params=g2.clone(), accumulate=True)
    torch.testing.assert_close(g3, 2 * g2, rtol=1e-6, atol=0)


@pytest.mark.parametrize("width,depth,n", [(128, 4, 4096 + 37), (256, 6, 2048 + 5), (256, 1, 50), (128, 8, 64 * 3)])
def test_parameter_gradient_fp32_training_sweep(width, depth, n):
    """Parameter gradients without the input gradient run the LDS training sweep: they match
    the float64 oracle, and those of the per-wave kernel (which also returns the input
    gradient; its layer products run over the same tiles in the same order, only the head is
    summed in another order) to float32 rounding."""
    banner("parameter gradient fp32 (training sweep) %dx%d n=%d" % (depth, width, n))
    p = synthetic.random_params(width, depth, 37)
    rays = _away_from_kinks(p, width, depth, _rays(n, 38))
    n = rays.shape[1]
    rng = np.random.default_rng(3)
    gl, gd = rng.normal(size=n).astype(np.float32) / n, rng.normal(size=n).astype(np.float32) / n
    net = api.Network(cuda(p), width, depth, "fp32")
    g_none, g_sweep = api.backward(net, cuda(rays), cuda(gl), cuda(gd), want_rays=False, want_params=True)
    assert g_none is None
    _, g_wave = api.backward(net, cuda(rays), cuda(gl), cuda(gd), want_rays=True, want_params=True)
    gw = host(g_wave)
    assert np.max(np.abs(host(g_sweep) - gw)) <= 1e-6 * np.abs(gw).max()
    _, ref_p = mlp.backward(p, width, depth, rays, gl, gd)
    gp = host(g_sweep)
    scale = np.sqrt(np.mean(ref_p ** 2))
    assert np.max(np.abs(gp - ref_p)) < 1e-5 * np.abs(ref_p).max()
    assert np.median(np.abs(gp - ref_p) / np.maximum(np.abs(ref_p), scale)) < 1e-5


def test_loss_seeds_and_adam():
    banner("loss seeds + adam")
    rng = np.random.default_rng(2)
    n = 10000 + 7
    z = (rng.normal(size=n) * 3).astype(np.float32)
    d = rng.normal(size=n).astype(np.float32)
    t = np.where(rng.random(n) < 0.4, rng.uniform(0, 2, n), np.inf).astype(np.float32)
    loss, gl, gd = api.loss_seeds(cuda(z), cuda(d), cuda(t))
    rl, rgl, rgd = mlp.loss_and_seeds(z, d, t < np.inf, t)
    assert abs(host(loss)[0] - rl) < 1e-5 * abs(rl)
    np.testing.assert_allclose(host(gl), rgl, rtol=1e-5, atol=1e-10)
    np.testing.assert_array_equal(host(gd), rgd.astype(np.float32))
    P = 5000
    p0 = rng.normal(size=P).astype(np.float32)
    pg, mg, vg = cuda(p0), torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    pr, mr, vr = p0.astype(np.float64), np.zeros(P), np.zeros(P)
    for s in range(1, 4):
        g = rng.normal(size=P).astype(np.float32)
        api.adam_step(pg, cuda(g), mg, vg, s)
        pr, mr, vr = mlp.adam_step(pr, g, mr, vr, s)
    np.testing.assert_allclose(host(pg), pr, rtol=1e-6, atol=1e-7)


def test_train_step_matches_oracle():
    banner("train step 128x4 batch 4096")
    width, depth, n = 128, 4, 4096
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, n, 3)
    from oracle import geometry
    lab = geometry.nearest_hit(o, d, tris)
    t = lab["t"].astype(np.float32)
    rays = rays5_from(o, d)
    p = synthetic.xavier_params(width, depth, 0)
    keep = _robust_batch(p, width, depth, rays, t)
    rays, t = np.ascontiguousarray(rays[:, keep]), t[keep]
    n = t.size
    pg = cuda(p)
    tr = api.Trainer(pg, width, depth, n, lr=1e-3)
    loss = host(tr.step(cuda(rays), cuda(t)))[0]
    # oracle step
    lg, ds = mlp.forward(p, width, depth, rays)
    rl, sl, sd = mlp.loss_and_seeds(lg, ds, t < np.inf, t)
    _, gref = mlp.backward(p, width, depth, rays, sl, sd)
    pnew, _, _ = mlp.adam_step(p, gref, np.zeros_like(gref), np.zeros_like(gref), 1)
    assert abs(loss - rl) < 1e-5 * abs(rl)
    g = host(tr.g)
    scale = np.sqrt(np.mean(gref ** 2))
    assert np.median(np.abs(g - gref) / np.maximum(np.abs(gref), scale)) < 1e-5
    banner("  worst per-layer gradient error %.3g" % _per_layer_close(g, gref, width, depth, 1e-5))
    # the first Adam step moves every parameter by lr * sign(g) (up to eps): compare moves
    moved = host(pg) - p
    ref_moved = pnew - p
    agree = np.abs(moved - ref_moved) < 1e-6
    assert agree.mean() > 0.999
    # the repacked network reflects the update
    lg2, _ = tr.net.forward(cuda(rays))
    lref, _ = mlp.forward(host(pg).astype(np.float64), width, depth, rays)
    assert np.max(_rel(host(lg2), lref)) < 1e-4


@pytest.mark.parametrize("width,depth,n,chunk", [(128, 4, 4096 + 100, 1000), (256, 3, 3000, 64 * 7 + 5)])
def test_chunked_train_step_equals_full_batch(width, depth, n, chunk):
    """A batch swept in column ranges (each recomputing its forward pass in a workspace sized
    for one range) gives the full batch's loss and gradient: the seeds use the whole batch's
    normalisation, only the float32 summation order differs."""
    banner("chunked train step %dx%d n=%d chunk=%d" % (depth, width, n, chunk))
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, n, 5)
    from oracle import geometry
    t = geometry.nearest_hit(o, d, tris)["t"].astype(np.float32)
    rays = cuda(rays5_from(o, d))
    p = synthetic.xavier_params(width, depth, 4)
    full = api.Trainer(cuda(p), width, depth, n)
    part = api.Trainer(cuda(p), width, depth, n, chunk=chunk)
    assert part.ws.numel() < full.ws.numel()
    lf = host(full.step(rays, cuda(t)))[0]
    lp = host(part.step(rays, cuda(t)))[0]
    assert abs(lp - lf) <= 1e-6 * abs(lf)
    gf, gp = host(full.g), host(part.g)
    assert np.max(np.abs(gp - gf)) <= 1e-5 * np.abs(gf).max()
    # the first Adam step moves by lr * sign(g): signs of near-zero components may differ
    moved_f, moved_p = host(full.params) - p, host(part.params) - p
    assert np.mean(np.abs(moved_f - moved_p) < 1e-6) > 0.999
    # a second step runs on the repacked network
    lf2 = host(full.step(rays, cuda(t)))[0]
    lp2 = host(part.step(rays, cuda(t)))[0]
    assert abs(lp2 - lf2) <= 1e-3 * abs(lf2)


def test_autograd_function_matches_backward():
    banner("autograd.Function")
    width, depth, n = 128, 2, 512
    p = synthetic.random_params(width, depth, 37)
    rays = cuda(_rays(n, 38)).requires_grad_(True)
    pg = cuda(p).requires_grad_(True)
    net = api.Network(pg.detach(), width, depth, "fp32")
    logit, dist = api.DDFQuery.apply(rays, pg, net)
    (logit.sum() * 0.5 + (dist ** 2).sum()).backward()
    lg, ds = mlp.forward(p, width, depth, host(rays.detach()))
    ref_r, ref_p = mlp.backward(p, width, depth, host(rays.detach()), np.full(n, 0.5), 2 * ds)
    assert np.quantile(_rel(host(rays.grad), ref_r), 0.99) < 1e-4
    assert np.median(_rel(host(pg.grad), ref_p)) < 1e-4


@pytest.mark.parametrize("loss,delta", [("clamp", 0.7), ("squish", 1.0)])
def test_paper_loss_seeds(loss, delta):
    """ddf_loss_seeds_ex with the clamp loss (Eq. 7) and the squish loss (Eq. 6, tanh) against
    the oracle: no logit gradient, distance seeds sign(c(d) - c(t)) c'(d) / N."""
    banner("loss seeds: %s (delta %g)" % (loss, delta))
    rng = np.random.default_rng(12)
    n = 20000 + 3
    z = rng.normal(size=n).astype(np.float32)
    d = (rng.normal(size=n) * 1.2).astype(np.float32)
    t = np.where(rng.random(n) < 0.5, rng.uniform(0, 2, n), np.inf).astype(np.float32)
    out, gl, gd = api.loss_seeds(cuda(z), cuda(d), cuda(t), loss=loss, delta=delta)
    rl, rgd = mlp.paper_loss_and_seeds(d, t, loss, delta)
    assert abs(host(out)[0] - rl) < 1e-5 * abs(rl)
    assert not host(gl).any()
    # 1 - tanh(d)^2 cancels in float32 where |d| is large: its absolute error is about two
    # float32 ulps of 1, i.e. 2.4e-7 / N in the seed
    np.testing.assert_allclose(host(gd), rgd, rtol=1e-5, atol=2.4e-7 / n)


@pytest.mark.parametrize("loss,delta,chunk", [("clamp", 0.5, 0), ("squish", 1.0, 0), ("clamp", 0.5, 1500)])
def test_train_step_paper_loss(loss, delta, chunk):
    """A training step with the paper's loss (whole batch and in chunks) against the oracle's
    seeds pushed through its backward pass."""
    banner("train step %s delta %g chunk %d, 128x4 batch 4096" % (loss, delta, chunk))
    width, depth, n = 128, 4, 4096
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, n, 5)
    from oracle import geometry
    t = geometry.nearest_hit(o, d, tris)["t"].astype(np.float32)
    rays = rays5_from(o, d)
    p = synthetic.xavier_params(width, depth, 2)
    keep = _robust_batch(p, width, depth, rays, t, loss, delta)
    rays, t = np.ascontiguousarray(rays[:, keep]), t[keep]
    n = t.size
    tr = api.Trainer(cuda(p), width, depth, n, lr=1e-3, chunk=chunk or None, loss=loss, delta=delta)
    out = host(tr.step(cuda(rays), cuda(t)))[0]
    lg, ds = mlp.forward(p, width, depth, rays)
    rl, sd = mlp.paper_loss_and_seeds(ds, t, loss, delta)
    _, gref = mlp.backward(p, width, depth, rays, np.zeros(n), sd)
    assert abs(out - rl) < 1e-5 * abs(rl)
    g = host(tr.g)
    scale = np.sqrt(np.mean(gref ** 2))
    assert np.median(np.abs(g - gref) / np.maximum(np.abs(gref), scale)) < 1e-5
    banner("  worst per-layer gradient error %.3g" % _per_layer_close(g, gref, width, depth, 1e-5))
    # the logit head's parameters (the head's first row and bias) get no gradient
    head_w = slice(g.size - 2 * width - 2, g.size - width - 2)
    assert not g[head_w].any() and g[-2] == 0.0


@pytest.mark.parametrize("chunk", [None, 1500])
def test_train_step_graph_replay_matches_eager(chunk):
    """A training step captured into a HIP graph: four replays equal four eager steps bit for
    bit (parameters, Adam moments, loss).  Adam's step number is a host argument, so both
    sides run step 2 four times; eager forward queries run between the replays."""
    banner("train step graph replay, 128x4 batch 4096, chunk %s" % chunk)
    width, depth, n = 128, 4, 4096
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, n, 7)
    from oracle import geometry
    t = cuda(geometry.nearest_hit(o, d, tris)["t"].astype(np.float32))
    rays = cuda(rays5_from(o, d))
    p = synthetic.xavier_params(width, depth, 3)
    eager = api.Trainer(cuda(p), width, depth, n, chunk=chunk)
    graph = api.Trainer(cuda(p), width, depth, n, chunk=chunk)
    for tr in (eager, graph):   # step 1, eager on both (one-time launch setup outside the capture)
        tr.step(rays, t)
    torch.cuda.synchronize()
    graph.step_count = 1
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        graph.step(rays, t)
    torch.cuda.synchronize()
    for rep in range(4):
        eager.step_count = 1
        eager.step(rays, t)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(eager.params, graph.params), rep
        assert torch.equal(eager.m, graph.m) and torch.equal(eager.v, graph.v), rep
        assert torch.equal(eager.loss, graph.loss), rep
        eager.net.forward(rays)   # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("loss,h,lam", [("bce_l1", 0.02, 0.1), ("clamp", 0.05, 0.5), ("bce_l1", 0.1, 100.0)])
def test_train_step_eikonal_matches_oracle(loss, h, lam):
    """The directed Eikonal training step (Eq. 2 as a forward difference along each ray) against
    the oracle: primary loss seeds on the rays, the penalty's seeds on the rays and on their
    moved copies, one backward pass of the doubled batch.  With lam = 100 the penalty's seeds
    set the gradient almost alone, so the moved half of the batch is checked by itself.
    The seeds divide float32 distance differences by h (an error of ~1e-6 of the distance
    becomes ~5e-5 of the residual at h = 0.02), so the per-layer bound is 5e-4 (measured: up
    to 5e-5), and the penalty-dominated case takes h = 0.1."""
    banner("train step eikonal: %s h=%g lam=%g, 128x4 batch 4096" % (loss, h, lam))
    width, depth, n = 128, 4, 4096
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, n, 9)
    from oracle import geometry
    t = geometry.nearest_hit(o, d, tris)["t"].astype(np.float32)
    p = synthetic.xavier_params(width, depth, 4)
    # the rays at x and at x + h d (moved in float32 like the kernel), angles of d
    ra = rays5_from(o, d)
    dn = (d / np.linalg.norm(d, axis=0)).astype(np.float32)
    rb = ra.copy()
    rb[:3] = (o.astype(np.float32) + np.float32(h) * dn).astype(np.float32)
    keep = _robust_batch(p, width, depth, ra, t, loss, 0.5, extra_rays=(rb,))
    o, d, t = np.ascontiguousarray(o[:, keep]), np.ascontiguousarray(d[:, keep]), t[keep]
    ra, rb = np.ascontiguousarray(ra[:, keep]), np.ascontiguousarray(rb[:, keep])
    n = t.size
    tr = api.Trainer(cuda(p), width, depth, n, lr=1e-3, loss=loss, delta=0.5)
    out = host(tr.step_eikonal(cuda(o), cuda(d), cuda(t), h=h, lam=lam))[0]
    la, da = mlp.forward(p, width, depth, ra)
    _, db = mlp.forward(p, width, depth, rb)
    if loss == "bce_l1":
        l0, gl, gd = mlp.loss_and_seeds(la, da, t < np.inf, t)
    else:
        l0, gd = mlp.paper_loss_and_seeds(da, t, loss, 0.5)
        gl = np.zeros(n)
    le, ga, gb = mlp.eikonal_loss_and_seeds(da, db, t, h, lam)
    rays2 = np.concatenate([ra, rb], axis=1)
    _, gref = mlp.backward(p, width, depth, rays2, np.concatenate([gl, np.zeros(n)]), np.concatenate([gd + ga, gb]))
    assert le > 0 and abs(out - (l0 + le)) < 1e-4 * abs(l0 + le)
    if lam > 10:
        assert le > 10 * l0
    g = host(tr.g)
    scale = np.sqrt(np.mean(gref ** 2))
    assert np.median(np.abs(g - gref) / np.maximum(np.abs(gref), scale)) < 1e-4
    banner("  worst per-layer gradient error %.3g" % _per_layer_close(g, gref, width, depth, 5e-4))
