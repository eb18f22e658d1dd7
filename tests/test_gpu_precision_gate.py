"""Accuracy of the reduced-precision queries against the float64 oracle on the trained 4 x 128
icosphere network of the benchmark's precision workload: bf16 must keep the mean absolute
distance error at or below 1e-3 and the hit agreement at or above 99.5% (the accuracy targets
of the bf16 query); float32 must agree to float32 rounding; fp8 is held to its measured level
(e4m3's three mantissa bits cannot reach the bf16 targets on this network)."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import mlp
from paper_2306_16142_amd import api

from gpu_common import banner

pytestmark = pytest.mark.gpu

W, D = 128, 4


@pytest.fixture(scope="module")
def trained():
    """Xavier init (seed 0), 1,500 Adam steps (lr 1e-3, batch 65,536) on 2^20 labeller-labelled
    training rays of the 320-triangle icosphere (seed 1), origins inside the mesh dropped."""
    banner("precision gate: training the 4 x 128 icosphere network, 1500 steps")
    dev = torch.device("cuda:0")
    v, f = synthetic.icosphere(2, 0.8)
    tris = torch.from_numpy(synthetic.tri_soup(v, f)).to(dev)
    params = torch.from_numpy(synthetic.xavier_params(W, D, 0)).to(dev)
    o, d, _ = synthetic.training_rays(v, f, 1 << 20, 1)
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    t, _, cr = api.label_rays(og, dg, tris)
    keep = (cr % 2) == 0
    rays = api.assemble_rays(og, dg)[:, keep].contiguous()
    t = t[keep].contiguous()
    batch = 65536
    tr = api.Trainer(params, W, D, batch, lr=1e-3)
    nb = rays.shape[1] // batch
    batches = [(rays[:, i * batch:(i + 1) * batch].contiguous(), t[i * batch:(i + 1) * batch].contiguous())
               for i in range(nb)]
    for i in range(1500):
        tr.step(*batches[i % nb])
    torch.cuda.synchronize()
    assert float(tr.loss) < 0.3
    # 2^20 uniform rays (seed 3), every 16th compared with the oracle
    o, d = synthetic.uniform_cube_rays(1 << 20, 3)
    og, dg = torch.from_numpy(o).to(dev), torch.from_numpy(d).to(dev)
    idx = np.arange(0, 1 << 20, 16)
    sub = api.assemble_rays(og, dg)[:, idx].cpu().numpy().astype(np.float64)
    ref = mlp.forward(params.cpu().numpy(), W, D, sub)
    return params, og, dg, idx, ref


def _errors(net, og, dg, idx, ref):
    """Hit agreement, and the distance error on the rays the oracle says hit (mean, p99)."""
    if net.precision == "fp32":
        logit, dist = net.forward(api.assemble_rays(og, dg))
    else:
        logit, dist = net.query(og, dg)   # the benchmarked fused kernel
    torch.cuda.synchronize()
    lg, ds = logit.cpu().numpy()[idx], dist.cpu().numpy()[idx]
    rl, rd = ref
    hit_agree = np.mean((lg > 0) == (rl > 0))
    err = np.abs(ds[rl > 0] - rd[rl > 0])
    return hit_agree, err.mean(), np.quantile(err, 0.99)


def test_bf16_meets_the_accuracy_targets(trained):
    params, og, dg, idx, ref = trained
    agree, mean, p99 = _errors(api.Network(params, W, D, "bf16"), og, dg, idx, ref)
    banner("  bf16: hit agreement %.4f%%, distance error mean %.3g p99 %.3g" % (100 * agree, mean, p99))
    assert agree >= 0.995 and mean <= 1e-3


def test_fp32_agrees_to_rounding(trained):
    params, og, dg, idx, ref = trained
    agree, mean, p99 = _errors(api.Network(params, W, D, "fp32"), og, dg, idx, ref)
    banner("  fp32: hit agreement %.4f%%, distance error mean %.3g p99 %.3g" % (100 * agree, mean, p99))
    assert agree >= 0.9999 and mean <= 1e-6


def test_fp8_holds_its_measured_level(trained):
    params, og, dg, idx, ref = trained
    calib_o, calib_d = synthetic.uniform_cube_rays(1 << 16, 4)
    calib = api.assemble_rays(torch.from_numpy(calib_o).to(og.device), torch.from_numpy(calib_d).to(og.device))
    net = api.Network(params, W, D, "fp8", scales=api.fp8_scales(params, W, D, calib))
    agree, mean, p99 = _errors(net, og, dg, idx, ref)
    banner("  fp8: hit agreement %.4f%%, distance error mean %.3g p99 %.3g" % (100 * agree, mean, p99))
    assert agree >= 0.99 and mean <= 2e-2
