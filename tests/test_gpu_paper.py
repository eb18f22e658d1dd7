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
