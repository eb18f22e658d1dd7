"""GPU parity of the paper's own network (Sec. V-A: weight-normalised 512-wide ReLU layers on
the raw ray, one distance output) against the float64 oracle and its bf16 emulation."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import paper
from paper_2306_16142_amd import api

from gpu_common import banner, cuda, host, rays5_from

pytestmark = pytest.mark.gpu

W = 512


def _rays(n, seed):
    o, d = synthetic.uniform_cube_rays(n, seed)
    return rays5_from(o, d)


def _scaled_err(gpu, ref):
    scale = np.maximum(np.abs(ref), np.sqrt(np.mean(ref ** 2)))
    return np.abs(gpu - ref) / scale


@pytest.mark.parametrize("depth,n", [(8, 40000 + 7), (3, 5000 + 3), (1, 300), (2, 129)])
def test_paper_forward_bf16_matches_emulation(depth, n):
    """bf16 query of the paper's network (several 128-ray tiles per workgroup at the largest n,
    a ragged tail everywhere) against the emulated bf16 forward, and its error against float64
    no larger than the emulation's own."""
    banner("paper forward bf16: depth %d, n=%d" % (depth, n))
    p = synthetic.paper_params(depth, 51)
    rays = _rays(n, 52)
    net = api.PaperNetwork(cuda(p), depth, "bf16")
    d = host(net(cuda(rays)))
    e = paper.forward_bf16(p, W, depth, rays)
    r = paper.forward(p, W, depth, rays)
    err, own = _scaled_err(d, e), _scaled_err(e, r)
    banner("  kernel vs emulation: median %.3g p99 %.3g max %.3g; emulation vs float64: median %.3g p99 %.3g"
           % (np.median(err), np.quantile(err, 0.99), err.max(), np.median(own), np.quantile(own, 0.99)))
    assert np.median(err) < 1e-5
    assert np.quantile(err, 0.99) < (0.3 if depth <= 6 else 0.6) * np.quantile(own, 0.99)
    assert err.max() <= own.max()
    assert _scaled_err(d, r).mean() <= 1.1 * own.mean() + 1e-6


@pytest.mark.parametrize("depth,n", [(8, 3000 + 11), (3, 1000), (1, 77)])
def test_paper_input_gradient_bf16_matches_emulation(depth, n):
    """bf16 input gradient (the normal's direction, Eq. 3) against the emulated bf16 backward."""
    banner("paper input gradient bf16: depth %d, n=%d" % (depth, n))
    p = synthetic.paper_params(depth, 53)
    rays = _rays(n, 54)
    gd = np.random.default_rng(55).normal(size=n).astype(np.float32)
    net = api.PaperNetwork(cuda(p), depth, "bf16")
    g, _ = net.backward(cuda(rays), cuda(gd))
    g = host(g)
    e = paper.backward_input_bf16(p, W, depth, rays, gd)
    r, _ = paper.backward(p, W, depth, rays, gd)
    err, own = _scaled_err(g, e), _scaled_err(e, r)
    banner("  kernel vs emulation: median %.3g p99 %.3g max %.3g; emulation vs float64: median %.3g p99 %.3g"
           % (np.median(err), np.quantile(err, 0.99), err.max(), np.median(own), np.quantile(own, 0.99)))
    assert np.median(err) < 0.2 * np.median(own)
    assert np.quantile(err, 0.99) < 0.6 * np.quantile(own, 0.99)
    assert _scaled_err(g, r).mean() <= 1.2 * own.mean()


def test_paper_edge_cases():
    banner("paper network: n = 0, NaN ray, bad arguments")
    p = synthetic.paper_params(2, 56)
    net = api.PaperNetwork(cuda(p), 2, "bf16")
    assert net(torch.zeros((5, 0), device="cuda")).numel() == 0
    rays = _rays(200, 57)
    rays[3, 150] = np.nan
    d = host(net(cuda(rays)))
    assert np.isnan(d[150]) and np.all(np.isfinite(np.delete(d, 150)))
    g, _ = net.backward(cuda(rays), cuda(np.ones(200, np.float32)))
    g = host(g)
    assert np.all(np.isnan(g[:, 150])) and np.all(np.isfinite(np.delete(g, 150, axis=1)))
    with pytest.raises(Exception):
        api.PaperNetwork(cuda(p[:-1]), 2, "bf16")


def _kink_free(p, depth, rays, tol=1e-4, extra=None):
    """Rays whose every hidden pre-activation is at least `tol` from the ReLU kink (float64)."""
    _, _, pres = paper.forward(p, W, depth, rays, return_acts=True)
    m = np.ones(rays.shape[1], dtype=bool)
    for z in pres[:-1]:
        m &= np.abs(z).min(axis=0) > tol
    return m


def _slices(depth):
    """(name, slice) of every parameter block: v, g, b per hidden layer, then the output row and bias."""
    out, off = [], 0
    for l, (o, i) in enumerate(paper.shapes(W, depth)[:-1]):
        for name, cnt in (("v%d" % l, o * i), ("g%d" % l, o), ("b%d" % l, o)):
            out.append((name, slice(off, off + cnt)))
            off += cnt
    out += [("w_out", slice(off, off + W)), ("b_out", slice(off + W, off + W + 1))]
    return out


def _per_block_close(g, ref, depth, tol):
    worst = 0.0
    for name, sl in _slices(depth):
        big = np.abs(ref[sl]).max()
        assert big > 0, name
        worst = max(worst, np.abs(g[sl] - ref[sl]).max() / big)
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("depth,n", [(8, 9000 + 5), (2, 333)])
def test_paper_forward_fp32_matches_float64(depth, n):
    """float32 query (the training sweep's forward; several 32-ray tiles per workgroup)."""
    banner("paper forward fp32: depth %d, n=%d" % (depth, n))
    p = synthetic.paper_params(depth, 71)
    rays = _rays(n, 72)
    d = host(api.PaperNetwork(cuda(p), depth, "fp32")(cuda(rays)))
    r = paper.forward(p, W, depth, rays)
    err = _scaled_err(d, r)
    banner("  scaled error vs float64: median %.3g max %.3g" % (np.median(err), err.max()))
    # float32 sums of 512 products per unit, eight layers deep, and an output small next to
    # the terms that form it (measured: median 3.4e-6, max 2.5e-5 at depth 8)
    assert np.median(err) < 1e-5 and err.max() < 1e-4


@pytest.mark.parametrize("depth,n", [(8, 2000 + 3), (3, 500)])
def test_paper_gradients_fp32_match_oracle(depth, n):
    """float32 input and parameter gradients (through the weight normalisation) against the
    float64 oracle on rays clear of ReLU kinks: per parameter block (v, g, b of every layer,
    the output row) the max error within 1e-5 of the block's largest component.  The
    accumulate flag adds, and a second call is bitwise identical."""
    banner("paper gradients fp32: depth %d, n=%d" % (depth, n))
    p = synthetic.paper_params(depth, 73)
    rays = _rays(n, 74)
    rays = np.ascontiguousarray(rays[:, _kink_free(p, depth, rays)])
    n = rays.shape[1]
    gd = (np.random.default_rng(75).normal(size=n) / n).astype(np.float32)
    net = api.PaperNetwork(cuda(p), depth, "fp32")
    g_rays, g_p = net.backward(cuda(rays), cuda(gd), want_params=True)
    ref_r, ref_p = paper.backward(p, W, depth, rays, gd)
    worst = _per_block_close(host(g_p), ref_p, depth, 1e-5)
    err_r = _scaled_err(host(g_rays), ref_r)
    banner("  worst per-block parameter error %.3g; input gradient max %.3g" % (worst, err_r.max()))
    assert err_r.max() < 1e-4
    g_only, _ = net.backward(cuda(rays), cuda(gd))   # input gradient without the parameter sweep
    assert torch.equal(g_only, g_rays)
    _, g2 = net.backward(cuda(rays), cuda(gd), want_params=True)
    assert torch.equal(g_p, g2)
    _, g3 = net.backward(cuda(rays), cuda(gd), want_params=True, g_params=g2.clone(), accumulate=True)
    torch.testing.assert_close(g3, 2 * g2, rtol=1e-6, atol=0)


def _clear_batch(p, depth, rays, t, n, loss, delta, masks, tol=2e-5):
    """A batch of n rays (from the candidates `rays`, `t`) in which every ray, under the dropout
    masks of its position (masks: per position, or None), keeps every hidden pre-activation at
    least `tol` from the ReLU kink (20 x the float32 error of a pre-activation) and its distance
    away from the loss's branch points.  A
    ray that fails at a position is replaced there by the next candidate, so the positions and
    with them the masks stay fixed."""
    m = rays.shape[1]
    pick = np.arange(n) % m
    good = np.zeros(n, dtype=bool)
    for rnd in range(m // n):   # every position tries distinct candidates
        cand = np.where(good, pick, (np.arange(n) + rnd * n) % m)
        r = np.ascontiguousarray(rays[:, cand])
        ds, _, pres = paper.forward(p, W, depth, r, return_acts=True, masks=masks)
        ok = np.ones(n, dtype=bool)
        for z in pres[:-1]:
            ok &= np.abs(z).min(axis=0) > tol
        tt = t[cand].astype(np.float64)
        if loss == "clamp":
            ok &= (np.abs(np.abs(ds) - delta) > tol) & (np.abs(np.clip(ds, -delta, delta) - np.clip(tt, -delta, delta)) > tol)
        else:
            ok &= np.abs(np.tanh(ds) - np.tanh(tt)) > tol
        pick = np.where(good, pick, cand)
        good |= ok
        if good.all():
            break
    assert good.all()
    return np.ascontiguousarray(rays[:, pick]), np.ascontiguousarray(t[pick])


@pytest.mark.parametrize("loss,delta,p_drop", [("clamp", 0.5, 0.0), ("squish", 1.0, 0.0), ("clamp", 0.5, 0.5),
                                               ("squish", 1.0, 0.3)])
def test_paper_train_step_matches_oracle(loss, delta, p_drop):
    """One training step of the paper's network (Sec. V-A) with the clamp (Eq. 7) or squish
    (Eq. 6) loss on labeller labels, without and with dropout (the paper: 0.5; the GPU and the
    oracle draw the same counter-based masks), on a batch clear of ReLU kinks and of the loss's
    branch points under those masks: loss, per-block gradient, the Adam move and the repacked
    network against the oracle."""
    banner("paper train step fp32: %s delta %g dropout %g, depth 8, batch 1024" % (loss, delta, p_drop))
    depth, n, seed = 8, 1024, 5
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, _ = synthetic.training_rays(v, f, 16384, 76)
    from oracle import geometry
    t = geometry.nearest_hit(o, d, tris)["t"].astype(np.float32)
    p = synthetic.paper_params(depth, 77)
    masks = paper.dropout_masks(seed, 1, W, depth, n, p_drop)
    rays, t = _clear_batch(p, depth, rays5_from(o, d), t, n, loss, delta, masks)
    pg = cuda(p)
    tr = api.PaperTrainer(pg, depth, n, lr=1e-3, loss=loss, delta=delta, dropout=p_drop, seed=seed)
    out = host(tr.step(cuda(rays), cuda(t)))[0]
    z = np.zeros(p.size)
    rl, gref, pnew, _, _ = paper.train_step(p.astype(np.float64), W, depth, rays, t, z, z, 1, loss, delta, lr=1e-3,
                                            dropout=p_drop, seed=seed)
    assert abs(out - rl) < 1e-5 * abs(rl)
    worst = _per_block_close(host(tr.g), gref, depth, 1e-4)
    banner("  loss %.6g (oracle %.6g); worst per-block gradient error %.3g" % (out, rl, worst))
    moved, ref_moved = host(pg) - p, pnew - p
    assert np.mean(np.abs(moved - ref_moved) < 1e-6) > 0.999
    # the repacked network is the updated one
    d2 = host(tr.net(cuda(rays)))
    r2 = paper.forward(host(pg).astype(np.float64), W, depth, rays)
    assert _scaled_err(d2, r2).max() < 2e-5
