"""Pins of the network oracle: closed-form encoding, library forward/autograd, finite differences,
reduced-precision rounding against torch's casts, Adam against torch.optim.Adam, plane-field normals."""
import json
import os

import numpy as np
import pytest
import torch

import synthetic
from oracle import mlp

from conftest import GOLDEN


def _val(x):
    return {"pi/2": np.pi / 2, "-pi/2": -np.pi / 2, "pi": np.pi}.get(x, x) if isinstance(x, str) else float(x)


def test_encoding_closed_form():
    cases = json.load(open(os.path.join(GOLDEN, "encoding_closed_form.json")))["cases"]
    for c in cases:
        ray = np.array([_val(x) for x in c["ray"]])[:, None]
        g = mlp.encode(ray)[:, 0]
        e = c["expect"]
        np.testing.assert_allclose(g[:5], [_val(x) for x in e["raw"]], atol=1e-15)
        np.testing.assert_allclose(g[5:35], np.array(e["sin"], dtype=np.float64).ravel(), atol=1e-12)
        np.testing.assert_allclose(g[35:65], np.array(e["cos"], dtype=np.float64).ravel(), atol=1e-12)


def _torch_net(params, width, depth):
    layers = mlp.unpack(params, width, depth)
    mods = []
    for l, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if l < depth:
            mods.append(torch.nn.ReLU())
    return torch.nn.Sequential(*mods)


def _torch_encode(r):
    feats = [r] + [torch.sin((2.0 ** k) * r) for k in range(6)] + [torch.cos((2.0 ** k) * r) for k in range(6)]
    return torch.cat(feats, dim=0)


def _rays(n, seed):
    from oracle import geometry
    o, d = synthetic.uniform_cube_rays(n, seed)
    th, ph = geometry.angles_from_dirs(d)
    return np.concatenate([o.astype(np.float64), th[None], ph[None]]).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("width,depth", [(128, 4), (32, 3)])
def test_forward_matches_torch_linear_layers(width, depth):
    p = synthetic.random_params(width, depth, 3).astype(np.float64)
    rays = _rays(512, 1)
    lg, ds = mlp.forward(p, width, depth, rays)
    net = _torch_net(p, width, depth)
    with torch.no_grad():
        out = net(_torch_encode(torch.from_numpy(rays)).T).numpy()
    np.testing.assert_allclose(lg, out[:, 0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ds, out[:, 1], rtol=1e-12, atol=1e-12)


def test_forward_zero_weights_gives_bias_and_one_hot_path():
    width, depth = 16, 3
    layers = mlp.unpack(np.zeros(synthetic.param_count(width, depth)), width, depth)
    layers = [(W.copy(), b.copy()) for W, b in layers]
    layers[-1][1][:] = [0.25, -1.5]
    rays = _rays(10, 2)
    lg, ds = mlp.forward(mlp.pack(layers), width, depth, rays)
    assert np.all(lg == 0.25) and np.all(ds == -1.5)
    # one-hot chain: feature 35 (cos(ox)) -> unit 0 -> ... -> dist; logit reads unit 0 with weight -2
    for W, _ in layers:
        W[:] = 0
    layers[0][0][0, 35] = 1.0
    for l in range(1, depth):
        layers[l][0][0, 0] = 1.0
    layers[-1][0][1, 0] = 1.0
    layers[-1][0][0, 0] = -2.0
    lg, ds = mlp.forward(mlp.pack(layers), width, depth, rays)
    np.testing.assert_allclose(ds, np.cos(rays[0]) + (-1.5), rtol=0, atol=1e-15)   # cos > 0 on [-1, 1]
    np.testing.assert_allclose(lg, -2.0 * np.cos(rays[0]) + 0.25, atol=1e-15)


def test_backward_matches_torch_autograd():
    width, depth = 32, 3
    p = synthetic.random_params(width, depth, 4).astype(np.float64)
    rays = _rays(256, 3)
    rng = np.random.default_rng(0)
    gl, gd = rng.normal(size=256), rng.normal(size=256)
    g_rays, g_params = mlp.backward(p, width, depth, rays, gl, gd)
    net = _torch_net(p, width, depth)
    r = torch.from_numpy(rays).requires_grad_(True)
    out = net(_torch_encode(r).T)
    (out[:, 0] @ torch.from_numpy(gl) + out[:, 1] @ torch.from_numpy(gd)).backward()
    np.testing.assert_allclose(g_rays, r.grad.numpy(), rtol=1e-10, atol=1e-12)
    tg = np.concatenate([torch.cat([m.weight.grad.ravel(), m.bias.grad.ravel()]).numpy()
                         for m in net if isinstance(m, torch.nn.Linear)])
    np.testing.assert_allclose(g_params, tg, rtol=1e-10, atol=1e-12)


def test_backward_central_differences():
    """Central differences (h = 1e-4, float64) on 64 parameters and on all 5 inputs of 64 rays; kinks skipped."""
    width, depth = 48, 3
    p = synthetic.random_params(width, depth, 5).astype(np.float64)
    rays = _rays(64, 4)
    rng = np.random.default_rng(1)
    gl, gd = rng.normal(size=64), rng.normal(size=64)
    g_rays, g_params = mlp.backward(p, width, depth, rays, gl, gd)
    h = 1e-4

    def f(pp, rr):
        a, b = mlp.forward(pp, width, depth, rr)
        return a @ gl + b @ gd

    def pattern(pp, rr):
        _, _, _, pres = mlp.forward(pp, width, depth, rr, return_acts=True)
        return [z > 0 for z in pres[:-1]]

    base = pattern(p, rays)
    idx = rng.choice(p.size, 64, replace=False)
    n_ok = 0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        if any((a != b).any() for a, b in zip(pattern(pp, rays), base)) or \
           any((a != b).any() for a, b in zip(pattern(pm, rays), base)):
            continue
        fd = (f(pp, rays) - f(pm, rays)) / (2 * h)
        assert abs(fd - g_params[i]) <= 1e-6 * max(1.0, abs(fd))
        n_ok += 1
    assert n_ok >= 48
    for j in range(64):
        for c in range(5):
            rp, rm = rays.copy(), rays.copy()
            rp[c, j] += h
            rm[c, j] -= h
            if any((a[:, j] != b[:, j]).any() for a, b in zip(pattern(p, rp), base)) or \
               any((a[:, j] != b[:, j]).any() for a, b in zip(pattern(p, rm), base)):
                continue
            # the 2^5 frequency makes the O(h^2) truncation term large for the inputs:
            # Richardson-extrapolate the central differences at h and h / 2 (error O(h^4))
            rp2, rm2 = rays.copy(), rays.copy()
            rp2[c, j] += h / 2
            rm2[c, j] -= h / 2
            d1 = (f(p, rp) - f(p, rm)) / (2 * h)
            d2 = (f(p, rp2) - f(p, rm2)) / h
            fd = (4 * d2 - d1) / 3
            assert abs(fd - g_rays[c, j]) <= 1e-6 * max(1.0, abs(fd)), (c, j)


def test_loss_seeds_central_differences():
    rng = np.random.default_rng(2)
    n = 200
    z, d = rng.normal(size=n) * 3, rng.normal(size=n)
    y = rng.random(n) < 0.4
    t = np.where(y, rng.uniform(0, 2, n), np.inf)
    loss, gl, gd = mlp.loss_and_seeds(z, d, y, t)
    h = 1e-6
    for i in rng.choice(n, 30, replace=False):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        fd = (mlp.loss_and_seeds(zp, d, y, t)[0] - mlp.loss_and_seeds(zm, d, y, t)[0]) / (2 * h)
        assert abs(fd - gl[i]) < 1e-8
        dp, dm = d.copy(), d.copy()
        dp[i] += h
        dm[i] -= h
        fd = (mlp.loss_and_seeds(z, dp, y, t)[0] - mlp.loss_and_seeds(z, dm, y, t)[0]) / (2 * h)
        assert abs(fd - gd[i]) < 1e-8
    # against torch's BCE-with-logits and L1 means
    tl = torch.nn.functional.binary_cross_entropy_with_logits(torch.from_numpy(z), torch.from_numpy(y.astype(np.float64)))
    tl = tl + torch.nn.functional.l1_loss(torch.from_numpy(d[y]), torch.from_numpy(t[y]))
    assert abs(tl.item() - loss) < 1e-12


def test_round_bf16_matches_torch_cast():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000) * 10 ** rng.uniform(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 3.3, 1e-40, 65504.0]]).astype(np.float32)
    ours = mlp.round_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_split_bf16_two_terms():
    """hi + lo reproduces values of up to 16 significant bits exactly; both parts are bfloat16
    and hi is the plain bfloat16 rounding; in general hi + lo is within 2^-16 relative."""
    rng = np.random.default_rng(3)
    m = rng.integers(1 << 15, 1 << 16, size=4096).astype(np.float64)
    x = m * 2.0 ** rng.integers(-30, 10, size=m.size) * rng.choice([-1.0, 1.0], size=m.size)
    hi, lo = mlp.split_bf16(x)
    np.testing.assert_array_equal(hi + lo, x)
    np.testing.assert_array_equal(mlp.round_bf16(hi), hi)
    np.testing.assert_array_equal(mlp.round_bf16(lo), lo)
    np.testing.assert_array_equal(hi, torch.from_numpy(x).float().bfloat16().double().numpy())
    y = rng.standard_normal(4096).astype(np.float32).astype(np.float64)
    hi, lo = mlp.split_bf16(y)
    assert np.all(np.abs(hi + lo - y) <= 2.0 ** -16 * np.abs(y))
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(y))


def test_round_e4m3_matches_torch_cast():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(size=20000) * 10 ** rng.uniform(-4, 3, 20000),
                        [0.0, 448.0, 449.0, 464.0, 1e6, -1e6, 2 ** -10, 1.5 * 2 ** -9, 1.0625, 1.1875]]).astype(np.float32)
    ours = mlp.round_e4m3(x)
    xc = np.clip(x, -448.0, 448.0)
    ref = torch.from_numpy(xc).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_emulated_precisions_exact_on_representable_inputs():
    """With weights, biases and every layer input exactly representable, the emulations equal float64."""
    width, depth = 8, 2
    layers = mlp.unpack(np.zeros(synthetic.param_count(width, depth)), width, depth)
    layers = [(W.copy(), b.copy()) for W, b in layers]
    # first layer reads only the raw inputs (features 0..4), which are small dyadic values
    rng = np.random.default_rng(5)
    layers[0][0][:, :5] = rng.integers(-2, 3, size=(width, 5)) * 0.25
    layers[1][0][:] = rng.integers(-2, 3, size=(width, width)) * 0.5
    layers[2][0][:] = rng.integers(-2, 3, size=(2, width)) * 0.5
    rays = (rng.integers(-4, 5, size=(5, 64)) * 0.25).astype(np.float64)
    p = mlp.pack(layers)
    ref = mlp.forward(p, width, depth, rays)
    np.testing.assert_array_equal(mlp.forward_bf16(p, width, depth, rays), ref)
    # head weights with 9 to 16 significant bits: not bfloat16, but the sum of two; the
    # emulation stays exact only if it keeps the remainder of the head rows
    head = layers[2][0].copy()
    layers[2][0][:] = head * (1.0 + 2.0 ** -10) + np.sign(head) * 2.0 ** -14
    p = mlp.pack(layers)
    ref = mlp.forward(p, width, depth, rays)
    assert np.any(mlp.round_bf16(layers[2][0]) != layers[2][0])
    np.testing.assert_array_equal(mlp.forward_bf16(p, width, depth, rays), ref)
    layers[2][0][:] = head
    # e4m3 keeps 3 mantissa bits: signed permutations scaled by powers of two keep every
    # layer input representable
    for l, (W, b) in enumerate(layers):
        W[:] = 0
        b[:] = 0
        for r in range(W.shape[0]):
            W[r, int(rng.integers(0, 5 if l == 0 else W.shape[1]))] = rng.choice([-1.0, 1.0]) * 2.0 ** int(rng.integers(-1, 2))
    p = mlp.pack(layers)
    ref = mlp.forward(p, width, depth, rays)
    scales = np.ones(2 * (depth + 1))
    np.testing.assert_array_equal(mlp.forward_fp8(p, width, depth, rays, scales), ref)
    # power-of-two scales are exact too
    scales = 2.0 ** rng.integers(-3, 3, size=2 * (depth + 1)).astype(np.float64)
    np.testing.assert_array_equal(mlp.forward_fp8(p, width, depth, rays, scales), ref)


def test_bf16_input_gradient_exact_on_representable_inputs():
    """With every operand representable in bfloat16 the emulated input gradient equals float64."""
    width, depth = 8, 3
    rng = np.random.default_rng(8)
    layers = mlp.unpack(np.zeros(synthetic.param_count(width, depth)), width, depth)
    layers = [(W.copy(), b.copy()) for W, b in layers]
    layers[0][0][:, :5] = rng.integers(-2, 3, size=(width, 5)) * 0.25
    for l in range(1, depth + 1):
        layers[l][0][:] = rng.integers(-2, 3, size=layers[l][0].shape) * 0.5
    for l in range(depth):
        layers[l][1][:] = 0.125
    rays = (rng.integers(-4, 5, size=(5, 40)) * 0.25).astype(np.float64)
    p = mlp.pack(layers)
    gl, gd = rng.integers(-2, 3, size=40) * 0.5, rng.integers(-2, 3, size=40) * 0.25
    ref, _ = mlp.backward(p, width, depth, rays, gl, gd)
    np.testing.assert_array_equal(mlp.backward_input_bf16(p, width, depth, rays, gl, gd), ref)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(5)]
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=1e-3)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s, g in enumerate(grads, start=1):
        p, m, v = mlp.adam_step(p, g, m, v, s)
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_normals_on_analytic_plane_field():
    """Plane n_p . x = c: the field is (c - n_p . x) / (n_p . d), so d(field)/dx = -n_p / (n_p . d)
    and the directed Eikonal equation (Eq. 2) holds exactly: grad . d = -1."""
    rng = np.random.default_rng(7)
    n_p = rng.normal(size=3)
    n_p /= np.linalg.norm(n_p)
    d = rng.normal(size=(3, 500))
    d /= np.linalg.norm(d, axis=0)
    keep = np.abs(n_p @ d) > 1e-3
    d = d[:, keep]
    g = -n_p[:, None] / (n_p @ d)[None]
    np.testing.assert_allclose(np.sum(g * d, axis=0), -1.0, rtol=1e-12)
    n = mlp.normals(g, d)
    facing = np.where((n_p @ d) > 0, -1.0, 1.0)
    np.testing.assert_allclose(n, n_p[:, None] * facing[None], atol=1e-12)
    assert np.all(np.sum(n * d, axis=0) < 0)
    # degenerate cases
    z = mlp.normals(np.zeros((3, 1)), np.array([[0.0], [0.0], [2.0]]))
    np.testing.assert_array_equal(z[:, 0], [0.0, 0.0, -1.0])


def test_fp8_scales_closed_form():
    """Per-layer scales are the smallest powers of two that map the absmax into [-448, 448]:
    weight absmax from the matrix, input absmax over the calibration rays (layer 0: the
    Fourier features, whose largest magnitude here is the raw azimuth; deeper layers: ReLU
    outputs of the one-hot chain)."""
    width, depth = 8, 2
    layers = mlp.unpack(np.zeros(synthetic.param_count(width, depth)), width, depth)
    layers = [(W.copy(), b.copy()) for W, b in layers]
    layers[0][0][0, 4] = -3.0          # unit 0 = -3 * phi (ReLU keeps it only for phi < 0: never)
    layers[0][0][1, 0] = 2.0           # unit 1 = 2 * ox
    layers[1][0][2, 1] = 0.5           # unit 2 = 0.5 * relu(2 ox)
    layers[2][0][1, 2] = 4.0
    rays = np.array([[0.5, -0.25], [0, 0], [0, 0], [1.0, 2.0], [6.0, 3.0]], dtype=np.float64)
    s = mlp.fp8_scales(mlp.pack(layers), width, depth, rays)
    # absmax values 3, 6, 0.5, 1, 4, 0.5: 3 / 2^-7 = 384, 6 / 2^-6 = 384, 0.5 / 2^-9 = 256,
    # 1 / 2^-8 = 256, 4 / 2^-6 = 256
    np.testing.assert_array_equal(s, 2.0 ** np.array([-7, -6, -9, -8, -6, -9]))


def test_pow2_scale_edges():
    """The scale is the smallest power of two with absmax / s <= 448: exact at 448 * 2^k, one
    binade up just above it; zero tensors get 1."""
    for k in (-12, -3, 0, 5):
        a = 448.0 * 2.0 ** k
        assert mlp.pow2_scale(a) == 2.0 ** k
        assert mlp.pow2_scale(np.nextafter(a, np.inf)) == 2.0 ** (k + 1)
        assert mlp.pow2_scale(np.nextafter(a, 0.0)) == 2.0 ** k
        assert mlp.pow2_scale(a / 2 + 1e-9 * a) == 2.0 ** k
    assert mlp.pow2_scale(0.0) == 1.0
    rng = np.random.default_rng(11)
    for a in rng.uniform(1e-6, 1e6, size=200):
        s = mlp.pow2_scale(a)
        assert np.log2(s) == np.round(np.log2(s))
        assert 224.0 < a / s <= 448.0


def test_paper_losses_closed_form_and_differences():
    """Eq. 7 clamp and Eq. 6 squish losses: hand-computed values, then central differences of
    the loss against the seeds away from the clamp edges and from d = c(t)."""
    d = np.array([0.5, -2.0, 0.2, 3.0])
    t = np.array([np.inf, 0.1, 0.2, np.inf])
    loss, g = mlp.paper_loss_and_seeds(d, t, "clamp", 1.0)
    # |1 - 0.5| + |0.1 - (-1)| + 0 + |1 - 1| over 4
    assert abs(loss - (0.5 + 1.1 + 0.0 + 0.0) / 4) < 1e-15
    np.testing.assert_array_equal(g, [-0.25, 0.0, 0.0, 0.0])
    loss, g = mlp.paper_loss_and_seeds(d, t, "squish")
    want = (abs(1 - np.tanh(0.5)) + abs(np.tanh(0.1) - np.tanh(-2.0)) + 0 + abs(1 - np.tanh(3.0))) / 4
    assert abs(loss - want) < 1e-15
    np.testing.assert_allclose(g, [-(1 - np.tanh(0.5) ** 2) / 4, -(1 - np.tanh(-2.0) ** 2) / 4, 0.0,
                                   -(1 - np.tanh(3.0) ** 2) / 4], rtol=1e-14)
    rng = np.random.default_rng(8)
    n = 200
    d = rng.normal(size=n) * 1.5
    t = np.where(rng.random(n) < 0.5, rng.uniform(0, 2, n), np.inf)
    h = 1e-6
    for kind, delta in (("clamp", 0.8), ("squish", 1.0)):
        _, g = mlp.paper_loss_and_seeds(d, t, kind, delta)
        for i in range(0, n, 7):
            c_t = min(t[i], delta) if kind == "clamp" else np.tanh(t[i])
            c_d = np.clip(d[i], -delta, delta) if kind == "clamp" else np.tanh(d[i])
            if kind == "clamp" and (abs(abs(d[i]) - delta) < 1e-3 or abs(c_d - c_t) < 1e-3):
                continue
            dp, dm = d.copy(), d.copy()
            dp[i] += h
            dm[i] -= h
            fd = (mlp.paper_loss_and_seeds(dp, t, kind, delta)[0] - mlp.paper_loss_and_seeds(dm, t, kind, delta)[0]) / (2 * h)
            assert abs(fd - g[i]) < 1e-7, (kind, i, fd, g[i])


def test_eikonal_penalty_plane_field_and_differences():
    """Eq. 2 on an analytic field: for the plane z = 0 seen from above, phi(x, d) = -x_z / d_z
    for d_z < 0, and phi(x + h d) - phi(x) = -h exactly, so the residual vanishes; then
    central differences of the penalty against its seeds."""
    rng = np.random.default_rng(9)
    n, h = 500, 0.05
    x = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0.2, 1, n)])
    d = rng.normal(size=(3, n))
    d[2] = -np.abs(d[2]) - 0.2
    d /= np.linalg.norm(d, axis=0)
    phi = lambda p: -p[2] / d[2]
    t = phi(x)
    loss, ga, gb = mlp.eikonal_loss_and_seeds(phi(x), phi(x + h * d), t, h, 0.3)
    assert loss < 1e-24 and np.abs(ga).max() < 1e-12
    # rays whose label is a miss or closer than h do not count
    a = rng.normal(size=n)
    b = a - h + rng.normal(size=n) * 0.01
    t = np.where(rng.random(n) < 0.3, np.inf, rng.uniform(0, 0.1, n))
    loss, ga, gb = mlp.eikonal_loss_and_seeds(a, b, t, h, 0.3)
    off = ~(np.isfinite(t) & (t > h))
    assert not ga[off].any() and not gb[off].any()
    eps = 1e-6
    for i in range(0, n, 23):
        ap, am = a.copy(), a.copy()
        ap[i] += eps
        am[i] -= eps
        fd = (mlp.eikonal_loss_and_seeds(ap, b, t, h, 0.3)[0] - mlp.eikonal_loss_and_seeds(am, b, t, h, 0.3)[0]) / (2 * eps)
        assert abs(fd - ga[i]) < 1e-7
        bp, bm = b.copy(), b.copy()
        bp[i] += eps
        bm[i] -= eps
        fd = (mlp.eikonal_loss_and_seeds(a, bp, t, h, 0.3)[0] - mlp.eikonal_loss_and_seeds(a, bm, t, h, 0.3)[0]) / (2 * eps)
        assert abs(fd - gb[i]) < 1e-7
