"""Pins of the paper-network oracle (Sec. V-A): weight normalisation, forward and gradients
against torch's own weight-norm parametrisation and central differences, and hand-worked
cases for every rounding step of the bfloat16 emulation."""
import numpy as np
import pytest
import torch

from oracle import mlp, paper


def _params(width, depth, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in paper.shapes(width, depth)[:-1]:
        parts += [rng.normal(size=o * i), rng.uniform(0.5, 2.0, size=o) * rng.choice([-1, 1], size=o),
                  rng.uniform(-0.2, 0.2, size=o)]
    parts += [rng.normal(size=width) / np.sqrt(width), rng.uniform(-0.2, 0.2, size=1)]
    return np.concatenate(parts).astype(np.float32)


def _rays(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(-1, 1, size=(3, n))
    th = rng.uniform(0, np.pi, size=(1, n))
    ph = rng.uniform(0, 2 * np.pi, size=(1, n))
    return np.concatenate([o, th, ph]).astype(np.float32)


def _torch_model(params, width, depth):
    """The paper's network built from torch modules: weight-normalised Linear layers (torch's
    parametrisation, g over the output dimension), ReLU and Dropout(0.5), then a Linear."""
    hidden, head = paper.unpack(params, width, depth)
    mods = []
    for (v, g, b), (o, i) in zip(hidden, paper.shapes(width, depth)[:-1]):
        lin = torch.nn.Linear(i, o).double()
        lin = torch.nn.utils.parametrizations.weight_norm(lin, dim=0)
        with torch.no_grad():
            lin.parametrizations.weight.original0.copy_(torch.from_numpy(g).reshape(o, 1))
            lin.parametrizations.weight.original1.copy_(torch.from_numpy(v))
            lin.bias.copy_(torch.from_numpy(b))
        mods += [lin, torch.nn.ReLU(), torch.nn.Dropout(0.5)]
    out = torch.nn.Linear(width, 1).double()
    with torch.no_grad():
        out.weight.copy_(torch.from_numpy(head[0]))
        out.bias.copy_(torch.from_numpy(head[1]))
    model = torch.nn.Sequential(*mods, out)
    model.eval()
    return model


def test_shapes_and_count():
    assert paper.shapes(512, 8)[0] == (512, 5) and paper.shapes(512, 8)[-1] == (1, 512)
    # 8 x 512 paper network: 5*512 + 7*512*512 weights, 8*512 gains and biases, a 512-wide output
    assert paper.param_count(512, 8) == 5 * 512 + 7 * 512 * 512 + 2 * 8 * 512 + 512 + 1
    p = _params(4, 3, 0)
    hidden, head = paper.unpack(p, 4, 3)
    np.testing.assert_array_equal(paper.pack(hidden, head), p.astype(np.float64))


def test_fold_closed_form_and_invariants():
    # rows (3, 4, 0, 0, 0) with g = 2 and (0, 0, 0, 0, -2) with g = -1.5
    v = np.array([[3, 4, 0, 0, 0], [0, 0, 0, 0, -2]], dtype=np.float64)
    p = np.concatenate([v.ravel(), [2.0, -1.5], [0.1, 0.2], [1.0, 1.0], [0.0]])
    (W, b), _ = paper.fold(p, 2, 1)
    np.testing.assert_allclose(W, [[1.2, 1.6, 0, 0, 0], [0, 0, 0, 0, 1.5]], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(b, [0.1, 0.2])
    # |W_i| = |g_i|, and scaling any row of v by a positive factor changes nothing
    p = _params(8, 3, 1)
    hidden, head = paper.unpack(p, 8, 3)
    layers = paper.fold(p, 8, 3)
    for (v, g, _), (W, _) in zip(hidden, layers):
        np.testing.assert_allclose(np.linalg.norm(W, axis=1), np.abs(g), rtol=1e-14)
    scaled = [(v * np.arange(1, v.shape[0] + 1)[:, None] * 3.7, g, b) for v, g, b in hidden]
    for (W1, _), (W2, _) in zip(layers, paper.fold(paper.pack(scaled, head), 8, 3)):
        np.testing.assert_allclose(W1, W2, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("width,depth", [(16, 3), (32, 8)])
def test_forward_matches_torch_weight_norm(width, depth):
    p = _params(width, depth, 2)
    rays = _rays(300, 3)
    ref = _torch_model(p, width, depth)(torch.from_numpy(rays.T.astype(np.float64))).detach().numpy()[:, 0]
    out = paper.forward(p, width, depth, rays)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("width,depth", [(16, 3), (24, 8)])
def test_backward_matches_torch_autograd(width, depth):
    p = _params(width, depth, 4)
    rays = _rays(200, 5)
    gd = np.random.default_rng(6).normal(size=200)
    model = _torch_model(p, width, depth)
    x = torch.from_numpy(rays.T.astype(np.float64)).requires_grad_(True)
    (model(x)[:, 0] * torch.from_numpy(gd)).sum().backward()
    ref = []
    for mod in model:
        if isinstance(mod, torch.nn.Linear):
            if hasattr(mod, "parametrizations"):
                ref += [mod.parametrizations.weight.original1.grad.numpy().ravel(),
                        mod.parametrizations.weight.original0.grad.numpy().ravel(), mod.bias.grad.numpy()]
            else:
                ref += [mod.weight.grad.numpy().ravel(), mod.bias.grad.numpy()]
    g_rays, g_p = paper.backward(p, width, depth, rays, gd)
    np.testing.assert_allclose(g_p, np.concatenate(ref), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g_rays, x.grad.numpy().T, rtol=1e-10, atol=1e-12)


def test_backward_central_differences():
    width, depth = 6, 3
    p = _params(width, depth, 7).astype(np.float64)
    rays = _rays(40, 8).astype(np.float64)
    gd = np.random.default_rng(9).normal(size=40)
    g_rays, g_p = paper.backward(p, width, depth, rays, gd)
    h = 1e-6

    def loss(pp, rr):
        return np.sum(gd * paper.forward(pp, width, depth, rr))

    def kinks(pp, rr):
        _, _, pres = paper.forward(pp, width, depth, rr, return_acts=True)
        return min(np.abs(z).min() for z in pres[:-1])

    rng = np.random.default_rng(10)
    checked = 0
    for i in rng.choice(p.size, 60, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        if kinks(p + e, rays) < 1e-4 or kinks(p - e, rays) < 1e-4:
            continue
        fd = (loss(p + e, rays) - loss(p - e, rays)) / (2 * h)
        assert abs(fd - g_p[i]) <= 1e-6 * max(1.0, abs(fd)), i
        checked += 1
    assert checked > 30
    for j in range(5):
        e = np.zeros_like(rays)
        e[j] = h
        fd = (np.sum(gd * paper.forward(p, width, depth, rays + e)) - np.sum(gd * paper.forward(p, width, depth, rays - e))) / (2 * h)
        assert abs(fd - g_rays[j].sum()) <= 1e-6 * max(1.0, abs(fd))


def _tiny(first_row, g0, b0, hidden=(), head_w=1.0, head_b=0.0):
    """Width-1 network: first-layer row v0 (5 values) with gain g0 and bias b0, then hidden
    layers given as (v, g, b) scalars, then the output weight and bias."""
    parts = [np.asarray(first_row, dtype=np.float64), [g0], [b0]]
    for v, g, b in hidden:
        parts += [[v], [g], [b]]
    parts += [[head_w], [head_b]]
    return np.concatenate(parts), 1 + len(hidden)


def _ray(x0=0.0):
    return np.array([[x0], [0.0], [0.0], [0.0], [0.0]])


def test_bf16_first_layer_reads_unrounded_inputs():
    # x = 1 + 2^-8 - 2^-20 (float32, rounds to 1 in bf16) times a weight of 255: the true
    # pre-activation 255.9958 rounds to 256; from a rounded input it would be 255
    x = 1 + 2.0 ** -8 - 2.0 ** -20
    assert np.float32(x) == x and mlp.round_bf16(x) == 1.0
    p, d = _tiny([1, 0, 0, 0, 0], 255.0, 0.0)
    assert paper.forward_bf16(p, 1, d, _ray(x))[0] == 256.0


def test_bf16_hidden_activation_is_rounded():
    # h1 = 1, hidden layer z = 1 + 2^-9 -> bf16 1 (the float64 network gives 1 + 2^-9)
    p, d = _tiny([1, 0, 0, 0, 0], 1.0, 0.0, hidden=[(1.0, 1.0, 2.0 ** -9)])
    assert paper.forward(p, 1, d, _ray(1.0))[0] == 1 + 2.0 ** -9
    assert paper.forward_bf16(p, 1, d, _ray(1.0))[0] == 1.0


def test_bf16_hidden_weights_are_rounded():
    # hidden weight 1 + 2^-8 - 2^-20 rounds to 1: 255 * 1 = 255 (unrounded: 255.9958 -> 256)
    w = 1 + 2.0 ** -8 - 2.0 ** -20
    p, d = _tiny([1, 0, 0, 0, 0], 1.0, 0.0, hidden=[(1.0, w, 0.0)])
    assert paper.forward_bf16(p, 1, d, _ray(255.0))[0] == 255.0


def test_bf16_hidden_bias_is_not_rounded():
    # h1 = 1, weight -1, bias 1 + 2^-8 - 2^-20 (bf16 would make it 1): z = 2^-8 - 2^-20 -> 2^-8
    p, d = _tiny([1, 0, 0, 0, 0], 1.0, 0.0, hidden=[(1.0, -1.0, 1 + 2.0 ** -8 - 2.0 ** -20)])
    assert paper.forward_bf16(p, 1, d, _ray(1.0))[0] == 2.0 ** -8


def test_bf16_output_row_carries_its_remainder_and_bias_is_exact():
    # output weight 1 + 2^-10 + 2^-20: bf16 hi = 1, lo = 2^-10 (16 significant bits kept);
    # the output bias 2^-12 + 3 is added unrounded
    p, d = _tiny([1, 0, 0, 0, 0], 1.0, 0.0, head_w=1 + 2.0 ** -10 + 2.0 ** -20, head_b=3 + 2.0 ** -12)
    assert paper.forward_bf16(p, 1, d, _ray(1.0))[0] == 1 + 2.0 ** -10 + 3 + 2.0 ** -12


def test_bf16_input_gradient_rounds_weights_and_adjoints():
    # first-layer weight 1 + 2^-10 and seed 1 + 2^-10: both round to 1 in the transposed product
    s = 1 + 2.0 ** -10
    p, d = _tiny([1, 0, 0, 0, 0], s, 0.0)
    g = paper.backward_input_bf16(p, 1, d, _ray(1.0), np.array([s]))
    assert g[0, 0] == 1.0 and np.all(g[1:] == 0.0)
    g64, _ = paper.backward(p, 1, d, _ray(1.0), np.array([s]))
    assert g64[0, 0] == s * s


def test_bf16_input_gradient_rounds_hidden_transposed_weights():
    # output weight 255, hidden weight 1 + 2^-8 - 2^-20 (bf16: 1): the adjoint reaching the
    # first layer is 255 (unrounded weight: 255.9958, which would round to 256)
    w = 1 + 2.0 ** -8 - 2.0 ** -20
    p, d = _tiny([1, 0, 0, 0, 0], 1.0, 0.0, hidden=[(1.0, w, 0.0)], head_w=255.0)
    g = paper.backward_input_bf16(p, 1, d, _ray(1.0), np.array([1.0]))
    assert g[0, 0] == 255.0


def test_bf16_emulation_exact_on_representable_operands():
    """With every weight, bias and activation bfloat16-representable the emulations equal the
    float64 network (forward and input gradient)."""
    width, depth = 8, 3
    rng = np.random.default_rng(11)
    parts = []
    for o, i in paper.shapes(width, depth)[:-1]:
        # rows of one or four entries +-1: |v| = 1 or 2, and W = g v / |v| is exact
        v = np.zeros((o, i))
        for r in range(o):
            k = 1 if (r % 2 or i < 4) else 4
            v[r, rng.choice(i, k, replace=False)] = rng.choice([-1.0, 1.0], k)
        parts += [v.ravel(), rng.choice([0.5, 1.0], o), rng.integers(-2, 3, size=o) / 8.0]
    parts += [rng.integers(-3, 4, size=width) / 8.0, [0.25]]
    p = np.concatenate(parts)
    rays = rng.integers(-4, 5, size=(5, 50)) / 4.0
    layers = paper.fold(p, width, depth)
    for W, b in layers:
        assert np.array_equal(mlp.round_bf16(W), W) and np.array_equal(mlp.round_bf16(b), b)
    _, acts, pres = paper.forward(p, width, depth, rays, return_acts=True)
    for a in acts[1:] + pres:
        assert np.array_equal(mlp.round_bf16(a), a)   # precondition: every value representable
    assert sum(np.count_nonzero(a) for a in acts[1:]) > 100
    np.testing.assert_array_equal(paper.forward_bf16(p, width, depth, rays), paper.forward(p, width, depth, rays))
    gd = np.ones(50)
    np.testing.assert_array_equal(paper.backward_input_bf16(p, width, depth, rays, gd),
                                  paper.backward(p, width, depth, rays, gd)[0])


def test_train_step_is_loss_backward_adam():
    width, depth = 8, 2
    p = _params(width, depth, 12).astype(np.float64)
    rays = _rays(64, 13).astype(np.float64)
    t = np.where(np.arange(64) % 3 == 0, np.inf, np.linspace(0.1, 1.5, 64))
    z = np.zeros_like(p)
    loss, grad, p1, m, v = paper.train_step(p, width, depth, rays, t, z, z, 1, "clamp", 0.7, lr=1e-3)
    l_ref, seeds = mlp.paper_loss_and_seeds(paper.forward(p, width, depth, rays), t, "clamp", 0.7)
    assert loss == l_ref
    np.testing.assert_array_equal(grad, paper.backward(p, width, depth, rays, seeds)[1])
    # first Adam step: every parameter with a non-zero gradient moves by lr (up to eps)
    big = np.abs(grad) > 1e-5
    assert big.mean() > 0.5
    np.testing.assert_allclose(np.abs(p1 - p)[big], 1e-3, rtol=1e-3)


# ---------------------------------------------------------------------------- training dropout
class _FixedMask(torch.nn.Module):
    """Multiplies by a fixed tensor: torch's Dropout in training mode with a given mask."""

    def __init__(self, m):
        super().__init__()
        self.m = m

    def forward(self, x):
        return x * self.m


def _torch_train_model(params, width, depth, masks):
    """The torch model of the paper's network with each Dropout replaced by its training-mode
    action under the given masks (kept units scaled by 1 / (1 - p))."""
    model = _torch_model(params, width, depth)
    mods, l = [], 0
    for mod in model:
        if isinstance(mod, torch.nn.Dropout):
            mods.append(_FixedMask(torch.from_numpy(masks[l].T.copy())))
            l += 1
        else:
            mods.append(mod)
    return torch.nn.Sequential(*mods)


@pytest.mark.parametrize("p_drop", [0.25, 0.5, 0.9])
def test_dropout_keep_rate_and_independence(p_drop):
    """Each unit of each ray is kept with probability 1 - p: the keep rate of a layer, of every
    unit and of every ray lies within binomial bounds; layers, steps and seeds draw different
    masks, with the agreement of independent draws, p^2 + (1 - p)^2."""
    w, n = 256, 2048
    k = paper.dropout_keep(11, 5, 1, w, n, p_drop)
    q = 1.0 - p_drop
    sd = np.sqrt(q * (1 - q))
    assert abs(k.mean() - q) < 5 * sd / np.sqrt(w * n)
    assert np.all(np.abs(k.mean(axis=1) - q) < 6 * sd / np.sqrt(n))
    assert np.all(np.abs(k.mean(axis=0) - q) < 6 * sd / np.sqrt(w))
    agree = p_drop ** 2 + q ** 2
    for other in (paper.dropout_keep(11, 5, 2, w, n, p_drop), paper.dropout_keep(11, 6, 1, w, n, p_drop),
                  paper.dropout_keep(12, 5, 1, w, n, p_drop)):
        assert abs(np.mean(k == other) - agree) < 6 * np.sqrt(agree * (1 - agree) / (w * n))
    # neighbouring units and rays are independent too
    assert abs(np.mean(k[1:] == k[:-1]) - agree) < 6 * np.sqrt(agree * (1 - agree) / (w * n))
    assert abs(np.mean(k[:, 1:] == k[:, :-1]) - agree) < 6 * np.sqrt(agree * (1 - agree) / (w * n))


def test_dropout_keep_boundary():
    """The draw is a 24-bit uniform u on {0, 2^-24, ..., 1 - 2^-24}; keeping u >= p keeps a unit
    with probability exactly 1 - p for every p on that grid, and so keeps every unit at p = 0.
    This sample of 2^24 draws holds a draw in the lowest bin (u = 0: dropped at p = 2^-24), so a
    strict comparison, which drops it at p = 0, fails here."""
    w, n = 512, 32768
    assert paper.dropout_keep(1, 0, 0, w, n, 0.0).all()
    low = ~paper.dropout_keep(1, 0, 0, w, n, 2.0 ** -24)
    assert 1 <= low.sum() <= 8   # about one draw per 2^24 lands in the lowest bin


def test_dropout_zero_is_the_query_network():
    width, depth = 16, 3
    p = _params(width, depth, 21).astype(np.float64)
    rays = _rays(50, 22).astype(np.float64)
    t = np.linspace(0.1, 1.0, 50)
    z = np.zeros_like(p)
    a = paper.train_step(p, width, depth, rays, t, z, z, 3, "clamp", 0.5, dropout=0.0, seed=9)
    b = paper.train_step(p, width, depth, rays, t, z, z, 3, "clamp", 0.5)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_dropout_expected_activation_is_the_query():
    """Inverted dropout: the mean over many training steps' masks of the dropout network's
    first-layer output is the query network's (the 1 / (1 - p) scale makes it unbiased)."""
    width, depth = 32, 1
    p = _params(width, depth, 23).astype(np.float64)
    rays = _rays(8, 24).astype(np.float64)
    _, acts, _ = paper.forward(p, width, depth, rays, return_acts=True)
    steps = 4000
    s = np.zeros_like(acts[1])
    for step in range(1, steps + 1):
        m = paper.dropout_masks(3, step, width, depth, 8, 0.5)
        s += paper.forward(p, width, depth, rays, return_acts=True, masks=m)[1][1]
    mean = s / steps
    # each entry is h x 2 or 0 with equal probability: standard deviation h / sqrt(steps)
    assert np.all(np.abs(mean - acts[1]) <= 5 * acts[1] / np.sqrt(steps) + 1e-12)


@pytest.mark.parametrize("p_drop", [0.5, 0.3])
def test_dropout_forward_and_gradients_match_torch(p_drop):
    """Forward, input and parameter gradients with one step's dropout masks against torch float64
    autograd on the weight-normalised model whose Dropout layers apply the same masks."""
    width, depth = 16, 4
    p = _params(width, depth, 25)
    rays = _rays(120, 26)
    masks = paper.dropout_masks(7, 4, width, depth, 120, p_drop)
    model = _torch_train_model(p, width, depth, masks)
    x = torch.from_numpy(rays.T.astype(np.float64)).requires_grad_(True)
    out = model(x)[:, 0]
    np.testing.assert_allclose(paper.forward(p, width, depth, rays, masks=masks), out.detach().numpy(),
                               rtol=1e-12, atol=1e-12)
    gd = np.random.default_rng(27).normal(size=120)
    (out * torch.from_numpy(gd)).sum().backward()
    ref = []
    for mod in model:
        if isinstance(mod, torch.nn.Linear):
            if hasattr(mod, "parametrizations"):
                ref += [mod.parametrizations.weight.original1.grad.numpy().ravel(),
                        mod.parametrizations.weight.original0.grad.numpy().ravel(), mod.bias.grad.numpy()]
            else:
                ref += [mod.weight.grad.numpy().ravel(), mod.bias.grad.numpy()]
    g_rays, g_p = paper.backward(p, width, depth, rays, gd, masks=masks)
    np.testing.assert_allclose(g_p, np.concatenate(ref), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g_rays, x.grad.numpy().T, rtol=1e-10, atol=1e-12)


def test_dropout_train_step_uses_the_step_masks():
    width, depth = 8, 2
    p = _params(width, depth, 28).astype(np.float64)
    rays = _rays(64, 29).astype(np.float64)
    t = np.where(np.arange(64) % 4 == 0, np.inf, np.linspace(0.1, 1.5, 64))
    z = np.zeros_like(p)
    loss, grad, _, _, _ = paper.train_step(p, width, depth, rays, t, z, z, 2, "clamp", 0.7, dropout=0.5, seed=31)
    masks = paper.dropout_masks(31, 2, width, depth, 64, 0.5)
    l_ref, seeds = mlp.paper_loss_and_seeds(paper.forward(p, width, depth, rays, masks=masks), t, "clamp", 0.7)
    assert loss == l_ref
    np.testing.assert_array_equal(grad, paper.backward(p, width, depth, rays, seeds, masks=masks)[1])
    other = paper.train_step(p, width, depth, rays, t, z, z, 3, "clamp", 0.7, dropout=0.5, seed=31)[1]
    assert not np.array_equal(grad, other)   # the next step draws other masks
