"""GPU parity of ddf_forward (and the fp8 calibration) against the float64 network oracle
and its emulated bfloat16 / fp8 forms."""
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


def _scaled_err(gpu, ref):
    """|gpu - ref| divided by max(|ref|, rms(ref)) (relative error that ignores tiny outputs)."""
    scale = np.maximum(np.abs(ref), np.sqrt(np.mean(ref ** 2)))
    return np.abs(gpu - ref) / scale


@pytest.mark.parametrize("width,depth,n", [(128, 4, 16384 + 37), (256, 6, 4096 + 5), (128, 1, 999), (256, 2, 64)])
def test_forward_fp32_matches_float64(width, depth, n):
    banner("forward fp32: %dx%d, n=%d" % (depth, width, n))
    p = synthetic.random_params(width, depth, 11)
    rays = _rays(n, 12)
    net = api.Network(cuda(p), width, depth, "fp32")
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    rl, rd = mlp.forward(p, width, depth, rays)
    assert _scaled_err(lg, rl).max() < 1e-5
    assert _scaled_err(ds, rd).max() < 1e-5


@pytest.mark.parametrize("width,depth,n", [(128, 4, 16384 + 37), (256, 6, 4096 + 5), (128, 2, 100), (256, 8, 1000),
                                           (128, 6, 3000 + 1), (256, 1, 77)])
def test_forward_bf16_matches_emulation(width, depth, n):
    banner("forward bf16: %dx%d, n=%d" % (depth, width, n))
    p = synthetic.random_params(width, depth, 13)
    rays = _rays(n, 14)
    net = api.Network(cuda(p), width, depth, "bf16")
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    el, ed = mlp.forward_bf16(p, width, depth, rays)
    # Rare bfloat16 rounding flips of an activation (the kernel and the emulation round
    # float32 sums taken in a different order, and the kernel's higher Fourier
    # frequencies come from a double-angle recurrence) move an output by about one bf16
    # ulp of one term: bound the typical error tightly and the worst case loosely, and
    # require the kernel's error against float64 to match the emulation's.
    # The gap between kernel and emulation must stay well inside the emulation's own error.
    # Every layer is another chance for such a flip, so the tail of the gap grows with depth
    # faster than the emulation's own error does: the 99th-percentile bound is 0.3 of the
    # emulation's error up to six hidden layers and 0.6 at eight.
    rl, rd = mlp.forward(p, width, depth, rays)
    tail = 0.3 if depth <= 6 else 0.6
    for g, e, r in ((lg, el, rl), (ds, ed, rd)):
        err = _scaled_err(g, e)
        own = _scaled_err(e, r)
        assert np.median(err) < 1e-5
        assert np.quantile(err, 0.99) < tail * np.quantile(own, 0.99)
        assert err.max() <= own.max()
        assert _scaled_err(g, r).mean() <= 1.1 * own.mean() + 1e-6


@pytest.mark.parametrize("width,depth,n", [(128, 4, 8192 + 3), (256, 6, 4096 + 17)])
def test_forward_bf16_keeps_head_remainder(width, depth, n):
    """bf16 head rows travel as two bf16 rows (the rounded row and its rounded remainder).
    With every other weight bf16-representable the kernel must sit far closer to that
    emulation than to one with plainly rounded head rows (the LDS-resident kernel at
    width 128, the streamed kernel at 256)."""
    banner("forward bf16 head remainder: %dx%d, n=%d" % (depth, width, n))
    layers = mlp.unpack(synthetic.random_params(width, depth, 17), width, depth)
    for W, _ in layers[:-1]:
        W[:] = mlp.round_bf16(W)
    p = mlp.pack(layers).astype(np.float32)
    rays = _rays(n, 18)
    net = api.Network(cuda(p), width, depth, "bf16")
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    el, ed = mlp.forward_bf16(p, width, depth, rays)
    layers[-1][0][:] = mlp.round_bf16(layers[-1][0])
    nl, nd = mlp.forward_bf16(mlp.pack(layers), width, depth, rays)   # remainder dropped
    for out, emu, plain in ((lg, el, nl), (ds, ed, nd)):
        shift = np.median(np.abs(plain - emu))
        assert shift > 0
        assert np.median(np.abs(out - emu)) < 0.1 * shift


@pytest.mark.parametrize("width,depth", [(128, 4), (256, 3)])
def test_fp8_scales_and_forward_match_emulation(width, depth):
    banner("forward fp8: %dx%d" % (depth, width))
    p = synthetic.random_params(width, depth, 15)
    calib = _rays(8192, 4)
    rays = _rays(8192 + 3, 16)
    scales_gpu = api.fp8_scales(cuda(p), width, depth, cuda(calib))
    sg = host(scales_gpu)
    so = mlp.fp8_scales(p, width, depth, calib)
    np.testing.assert_allclose(sg, so, rtol=1e-5)
    net = api.Network(cuda(p), width, depth, "fp8", scales=scales_gpu)
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    el, ed = mlp.forward_fp8(p, width, depth, rays, so)
    rl, rd = mlp.forward(p, width, depth, rays)
    # e4m3 keeps 3 mantissa bits: a requantisation flip moves an output by up to ~6% of one
    # term, so the kernel-vs-emulation gap is bounded against the emulation's own error
    for g, e, r in ((lg, el, rl), (ds, ed, rd)):
        err = _scaled_err(g, e)
        own = _scaled_err(e, r)
        assert np.median(err) < 1e-4
        assert np.quantile(err, 0.99) < 0.5 * np.quantile(own, 0.99)
        assert _scaled_err(g, r).mean() <= 1.1 * own.mean() + 1e-5


def test_forward_full_size_sampled():
    """2^24 uniform rays (the precision workload) in bf16: sampled outputs against float64."""
    n = 1 << 24
    banner("forward bf16 full size n=2^24 (sampled check)")
    o, d = synthetic.uniform_cube_rays(n, 3)
    p = synthetic.xavier_params(128, 4, 0)
    rays_gpu = cuda(rays5_from(o, d))
    net32 = api.Network(cuda(p), 128, 4, "fp32")
    net16 = api.Network(cuda(p), 128, 4, "bf16")
    l32, d32 = net32(rays_gpu)
    l16, d16 = net16(rays_gpu)
    torch.cuda.synchronize()
    idx = np.random.default_rng(0).choice(n, 4096, replace=False)
    idx.sort()
    sub = rays5_from(o[:, idx], d[:, idx])
    rl, rd = mlp.forward(p, 128, 4, sub)
    assert _scaled_err(host(l32)[idx], rl).max() < 1e-5
    assert _scaled_err(host(d32)[idx], rd).max() < 1e-5
    el, ed = mlp.forward_bf16(p, 128, 4, sub)
    for g, e, r in ((host(l16)[idx], el, rl), (host(d16)[idx], ed, rd)):
        err, own = _scaled_err(g, e), _scaled_err(e, r)
        assert np.median(err) < 1e-5
        assert np.quantile(err, 0.99) < 5e-4
        assert err.max() <= own.max()
    # hit decisions: the kernel takes the emulation's decision where the emulation's logit is
    # clear of zero (a rare activation rounding flip may move a logit by a few bf16 ulps of
    # one term), and agrees with float64 about as well as the emulation does
    clear = np.abs(el) > 5e-3 * np.sqrt(np.mean(el ** 2))
    assert np.mean((host(l16)[idx] > 0)[clear] == (el > 0)[clear]) >= 0.999
    assert np.mean((host(l16)[idx] > 0) == (rl > 0)) >= np.mean((el > 0) == (rl > 0)) - 0.002
    # the tail is written too (no stale values past the last full tile)
    assert np.all(np.isfinite(host(l16)[-100:]))


@pytest.mark.parametrize("width,depth", [(128, 4), (256, 6)])
def test_forward_bf16_large_coordinates(width, depth):
    """Encoding arguments beyond the fast sin/cos range (|v| > 1024) send their whole wave to
    the general reduction; the result still matches the emulation like any other ray."""
    banner("forward bf16 with coordinates beyond the fast sin/cos range: %dx%d" % (depth, width))
    p = synthetic.random_params(width, depth, 13)
    rays = _rays(256 + 19, 14)
    rays[0, 5:40] = rays[0, 5:40] * 3000.0   # rays 5..39: the first wave and part of the second
    rays[1, 200] = -1500.25
    net = api.Network(cuda(p), width, depth, "bf16")
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    el, ed = mlp.forward_bf16(p, width, depth, rays)
    rl, rd = mlp.forward(p, width, depth, rays)
    for g, e, r in ((lg, el, rl), (ds, ed, rd)):
        err = _scaled_err(g, e)
        own = _scaled_err(e, r)
        assert np.median(err) < 1e-5
        assert err.max() <= own.max()


@pytest.mark.parametrize("width,depth,prec", [(128, 1, "fp32"), (128, 1, "bf16"), (256, 1, "bf16"), (256, 3, "bf16")])
def test_encoding_layout_one_hot(width, depth, prec):
    """Layout pin of the Fourier encoding (65 features, their order and the packing of layer 0):
    units 0 and 1 of the first layer copy +feature i and -feature i, later hidden layers pass
    units 0 and 1 on unchanged, and the distance head takes their difference, so the network
    outputs exactly feature i, for every i (3 x 256 runs on the streamed kernel, the others on
    the per-wave kernels).  float32 must match the oracle's encoding to float32 accuracy; bf16
    must equal the bf16 rounding of it (up to the rare feature whose float32 value sits on the
    other side of a rounding tie)."""
    banner("encoding layout one-hot: %dx%d, %s" % (depth, width, prec))
    n = 1000
    rays = _rays(n, 21)
    feat = mlp.encode(rays)   # [65, n]
    worst = 0.0
    inexact = 0
    for i in range(mlp.IN_DIM):
        W1 = np.zeros((width, mlp.IN_DIM), np.float32)
        W1[0, i], W1[1, i] = 1.0, -1.0
        parts = [W1.ravel(), np.zeros(width, np.float32)]
        for _ in range(depth - 1):
            Wh = np.zeros((width, width), np.float32)
            Wh[0, 0], Wh[1, 1] = 1.0, 1.0   # relu(+f_i), relu(-f_i) pass through
            parts += [Wh.ravel(), np.zeros(width, np.float32)]
        W2 = np.zeros((2, width), np.float32)
        W2[0, 0] = 1.0                   # logit = relu(+f_i)
        W2[1, 0], W2[1, 1] = 1.0, -1.0   # dist = relu(+f_i) - relu(-f_i) = f_i
        p = np.concatenate(parts + [W2.ravel(), np.zeros(2, np.float32)])
        net = api.Network(cuda(p), width, depth, prec)
        lg, ds = net(cuda(rays))
        ds = host(ds).astype(np.float64)
        if prec == "fp32":
            worst = max(worst, np.abs(ds - feat[i]).max())
        else:
            ref = mlp.round_bf16(feat[i])
            ulp = np.abs(mlp.round_bf16(feat[i] * (1 + 2.0 ** -7)) - ref) + 1e-30
            assert np.all(np.abs(ds - ref) <= ulp * 1.01), i
            inexact += int(np.sum(ds != ref))
    if prec == "fp32":
        assert worst < 2e-6, worst
    else:
        assert inexact <= 0.001 * n * mlp.IN_DIM, inexact


def test_forward_edge_cases():
    banner("forward: n = 0, NaN ray")
    p = synthetic.random_params(128, 2, 17)
    net = api.Network(cuda(p), 128, 2, "bf16")
    lg, ds = net(torch.zeros((5, 0), device="cuda"))
    assert lg.numel() == 0
    rays = _rays(70, 18)
    rays[1, 3] = np.nan
    lg, ds = net(cuda(rays))
    lg, ds = host(lg), host(ds)
    assert np.isnan(lg[3]) and np.isnan(ds[3])
    assert np.all(np.isfinite(np.delete(lg, 3))) and np.all(np.isfinite(np.delete(ds, 3)))
    # float32 at width 256 (the sweep's forward) propagates NaN inputs too
    net32 = api.Network(cuda(synthetic.random_params(256, 2, 17)), 256, 2, "fp32")
    lg, ds = net32(cuda(rays))
    lg, ds = host(lg), host(ds)
    assert np.isnan(lg[3]) and np.isnan(ds[3])
    assert np.all(np.isfinite(np.delete(lg, 3))) and np.all(np.isfinite(np.delete(ds, 3)))


def test_fp8_scales_not_powers_of_two_give_nan():
    """The fp8 kernels rescale through the MFMA's power-of-two operand scale: a blob packed with
    other scales is rejected by writing NaN (both the LDS and the L2 kernel)."""
    for width, depth in ((128, 4), (256, 3)):
        banner("forward fp8 non-power-of-two scales: %dx%d" % (depth, width))
        p = synthetic.random_params(width, depth, 15)
        rays = _rays(257, 16)
        good = mlp.fp8_scales(p, width, depth, _rays(4096, 4))
        bad = good.copy()
        bad[3] *= 1.5
        out = api.Network(cuda(p), width, depth, "fp8", scales=cuda(bad))(cuda(rays))
        assert np.all(np.isnan(host(out[0]))) and np.all(np.isnan(host(out[1])))
        out = api.Network(cuda(p), width, depth, "fp8", scales=cuda(good))(cuda(rays))
        assert np.all(np.isfinite(host(out[0]))) and np.all(np.isfinite(host(out[1])))


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_query_from_directions_equals_assembly_then_forward(prec):
    """ddf_query (ray assembly fused into the network kernel) gives exactly the outputs of
    ddf_assemble_rays followed by ddf_forward, ragged tail and NaN rays included."""
    banner("query from directions (%s 4x128), n=70000" % prec)
    n = 70000
    o, d = synthetic.uniform_cube_rays(n, 21)
    d[:, 17] = np.nan   # a NaN direction gives NaN outputs on both paths
    p = synthetic.random_params(128, 4, 22)
    og, dg = cuda(o), cuda(d)
    scales = api.fp8_scales(cuda(p), 128, 4, api.assemble_rays(og, dg)[:, :4096].contiguous()) if prec == "fp8" else None
    net = api.Network(cuda(p), 128, 4, prec, scales=scales)
    l1, d1 = net(api.assemble_rays(og, dg))
    l2, d2 = net.query(og, dg)
    assert torch.equal(torch.nan_to_num(l1, nan=7.0), torch.nan_to_num(l2, nan=7.0))
    assert torch.equal(torch.nan_to_num(d1, nan=7.0), torch.nan_to_num(d2, nan=7.0))
    assert torch.isnan(l2[17]) and torch.isfinite(l2[:17]).all()
    # networks that do not fit in LDS are refused
    wide = api.Network(cuda(synthetic.random_params(256, 2, 23)), 256, 2, "bf16")
    with pytest.raises(Exception):
        wide.query(og, dg)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_query_full_size_several_tiles_per_wave(prec):
    """ddf_query at 2^20 + 37 rays: with one workgroup per CU every wave runs about eight
    64-ray tiles, so the rays of each next tile are loaded while the current one is computed,
    and the last tile is ragged.  Outputs equal ddf_assemble_rays + ddf_forward bit for bit,
    and sampled rays (spread over the batch, plus the whole tail) match the emulated forward
    on both outputs."""
    n = (1 << 20) + 37
    banner("query full size (%s 4x128), n=2^20+37" % prec)
    o, d = synthetic.uniform_cube_rays(n, 25)
    p = synthetic.random_params(128, 4, 26)
    og, dg = cuda(o), cuda(d)
    calib = _rays(8192, 4)
    scales = api.fp8_scales(cuda(p), 128, 4, cuda(calib)) if prec == "fp8" else None
    net = api.Network(cuda(p), 128, 4, prec, scales=scales)
    l1, d1 = net(api.assemble_rays(og, dg))
    l2, d2 = net.query(og, dg)
    torch.cuda.synchronize()
    assert torch.equal(l1, l2) and torch.equal(d1, d2)
    rng = np.random.default_rng(27)
    idx = np.union1d(rng.choice(n, 4096, replace=False), np.arange(n - 200, n))
    sub = rays5_from(o[:, idx], d[:, idx])
    rl, rd = mlp.forward(p, 128, 4, sub)
    if prec == "bf16":
        el, ed = mlp.forward_bf16(p, 128, 4, sub)
        med, tail = 1e-5, 0.3
    else:
        so = mlp.fp8_scales(p, 128, 4, calib)
        np.testing.assert_array_equal(host(scales), so)
        el, ed = mlp.forward_fp8(p, 128, 4, sub, so)
        med, tail = 1e-4, 0.5
    lg, ds = host(l2)[idx], host(d2)[idx]
    for g, e, r in ((lg, el, rl), (ds, ed, rd)):
        err, own = _scaled_err(g, e), _scaled_err(e, r)
        assert np.median(err) < med
        assert np.quantile(err, 0.99) < tail * np.quantile(own, 0.99)
        assert _scaled_err(g, r).mean() <= 1.1 * own.mean() + 1e-5
    clear = np.abs(el) > (5e-3 if prec == "bf16" else 0.05) * np.sqrt(np.mean(el ** 2))
    assert np.mean((lg > 0)[clear] == (el > 0)[clear]) >= 0.999
