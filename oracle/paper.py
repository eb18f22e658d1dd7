"""Oracle of the paper's own network (Sec. V-A): weight-normalised ReLU layers on the raw
oriented point, one distance output, trained on the clamp loss (Eq. 7) or the squish loss
(Eq. 6).

Test infrastructure only (see the package docstring).

The network MLP_w : (R^3, R^2) -> R of Sec. IV-A takes the oriented point (x, theta) as the
5 raw values (ox, oy, oz, polar angle, azimuth) and returns the field value.  Sec. V-A gives
its shape: ``depth`` (8 in the paper) weight-normalised hidden layers of ``width`` (512)
units, each followed by ReLU and dropout with p = 0.5.  Readings taken here:

* weight normalisation (Salimans and Kingma, 2016) per output unit of every hidden layer:
  W[i, :] = g[i] v[i, :] / |v[i, :]|; the output layer is a plain affine map (the paper
  normalises the hidden layers); a row of v must not be all zero (its W is undefined);
* dropout is the identity when the network is queried; while training (inverted dropout,
  the paper's p = 0.5) each hidden unit's ReLU output is kept with probability 1 - p and
  scaled by 1 / (1 - p), so the expected activation is the query's.  The keep decisions come
  from a counter-based generator, so that the forward and reverse sweeps (and the GPU) draw
  the same masks without storing them: with H(x) the first output of a SplitMix64 generator
  whose state is x (Steele, Lea and Flood, 2014), layer l of training step `step` has the key
  K = H(H(H(seed) ^ step) ^ l), unit u of ray r is kept when the top 24 bits of
  H(K ^ (u << 32 | r)), read as a fraction of 2^24, are >= p;
* the single output is the distance; the paper's losses act on it directly.

Flat parameter vector (float32), per hidden layer l: v_l [width][in_l] row-major, g_l
[width], b_l [width] (in_0 = 5, in_l = width); then the output layer's weight [1][width]
and bias [1].
"""
import numpy as np

from . import mlp

IN_RAW = 5


def shapes(width, depth):
    """Per hidden layer (out, in), then the output layer's (1, width)."""
    dims = [IN_RAW] + [width] * depth
    return [(dims[l + 1], dims[l]) for l in range(depth)] + [(1, width)]


def param_count(width, depth):
    hid = sum(o * i + 2 * o for o, i in shapes(width, depth)[:-1])
    return hid + width + 1


def unpack(params, width, depth):
    """Split the flat vector: ``[(v, g, b)] * depth`` and the output layer ``(W, b)``, float64."""
    p = np.asarray(params, dtype=np.float64)
    hidden, off = [], 0
    for o, i in shapes(width, depth)[:-1]:
        v = p[off:off + o * i].reshape(o, i)
        off += o * i
        g = p[off:off + o]
        off += o
        b = p[off:off + o]
        off += o
        hidden.append((v, g, b))
    W = p[off:off + width].reshape(1, width)
    off += width
    b = p[off:off + 1]
    off += 1
    if off != p.size:
        raise ValueError("parameter vector has %d values, the network needs %d" % (p.size, off))
    return hidden, (W, b)


def pack(hidden, head):
    parts = []
    for v, g, b in hidden:
        parts += [v.ravel(), g.ravel(), b.ravel()]
    return np.concatenate(parts + [head[0].ravel(), head[1].ravel()])


def fold(params, width, depth):
    """Weight normalisation written out: W = g v / |v| per row (Salimans and Kingma, 2016).

    Returns the plain affine layers ``[(W [out, in], b [out])] * (depth + 1)`` in float64.
    Pinned by closed-form rows, by |W_i| = |g_i|, by the invariance to scaling v, and by
    torch's own weight-norm parametrisation in the tests.
    """
    hidden, head = unpack(params, width, depth)
    layers = []
    for v, g, b in hidden:
        norm = np.sqrt(np.sum(v * v, axis=1))
        layers.append((g[:, None] * v / norm[:, None], b))
    layers.append(head)
    return layers


def dropout_keep(seed, step, layer, width, n, p):
    """Keep decisions [width, n] of hidden layer ``layer`` at training step ``step`` for rays
    0 .. n - 1 (the counter-based draw described in the module docstring)."""
    from .render import _h, _h_np
    key = _h(_h(_h(seed) ^ step) ^ layer)
    u = np.arange(width, dtype=np.uint64)[:, None]
    r = np.arange(n, dtype=np.uint64)[None, :]
    k = _h_np(np.uint64(key) ^ ((u << np.uint64(32)) | r))
    return (k >> np.uint64(40)).astype(np.float64) * 2.0 ** -24 >= p


def dropout_masks(seed, step, width, depth, n, p):
    """Scaled masks [depth][width, n] (0 or 1 / (1 - p)) of one training step; None for p = 0."""
    if p == 0:
        return None
    return [dropout_keep(seed, step, l, width, n, p) / (1.0 - p) for l in range(depth)]


def forward(params, width, depth, rays, return_acts=False, masks=None):
    """Float64 forward of the paper's network on the raw rays [5, N]: h_0 = ray,
    h_l = max(0, W_l h_{l-1} + b_l), times the scaled dropout mask of layer l when training
    (``masks``: ``dropout_masks``; None: dropout is the identity), distance = W h_D + b.

    Returns dist [N] (and, with ``return_acts``, the layer inputs and pre-activations).
    Pinned against torch float64 (weight_norm Linear layers, ReLU, Dropout in eval mode; in
    training mode with the same masks applied as fixed factors).
    """
    layers = fold(params, width, depth)
    h = np.asarray(rays, dtype=np.float64)
    acts, pres = [h], []
    for l, (W, b) in enumerate(layers):
        z = W @ h + b[:, None]
        pres.append(z)
        if l < depth:
            h = np.maximum(z, 0.0)
            if masks is not None:
                h = h * masks[l]
            acts.append(h)
        else:
            h = z
    if return_acts:
        return h[0], acts, pres
    return h[0]


def forward_bf16(params, width, depth, rays):
    """Forward with the hidden layers' products in bfloat16 operands and float64 sums.

    The first layer takes the raw rays and its weights unrounded (a raw coordinate
    rounded to bfloat16 would move by up to 2^-9 of its size); its output and every
    later layer input are rounded to bfloat16 after the ReLU; the weights of the hidden
    layers are the folded weights rounded to bfloat16; biases are added unrounded; the
    output row is carried as a sum of two bfloat16 values (``mlp.split_bf16``).
    Pinned by hand-worked cases where each of these choices changes the result.
    """
    layers = fold(params, width, depth)
    W0, b0 = layers[0]
    h = mlp.round_bf16(np.maximum(W0 @ np.asarray(rays, dtype=np.float64) + b0[:, None], 0.0))
    for W, b in layers[1:depth]:
        h = mlp.round_bf16(np.maximum(mlp.round_bf16(W) @ h + b[:, None], 0.0))
    hi, lo = mlp.split_bf16(layers[depth][0])
    return ((hi + lo) @ h + layers[depth][1][:, None])[0]


def backward(params, width, depth, rays, g_dist, masks=None):
    """Reverse-mode gradient of sum(g_dist * dist): returns (g_rays [5, N], g_params [P]);
    ``masks``: the training step's dropout masks (``dropout_masks``), or None.

    The input gradient is the derivative with respect to the query point and angles that
    Sec. IV-B takes by automatic differentiation (its origin part gives the normal of
    Eq. 3).  Parameter gradients are taken for the folded weights G = dL/dW and carried
    back through the weight normalisation of each hidden row (u = v / |v|):
    dL/dg = G . u and dL/dv = (g / |v|) (G - (G . u) u).  ReLU'(0) = 0.
    Pinned by torch float64 autograd through its weight-norm parametrisation and by central
    differences in the tests.
    """
    hidden, _ = unpack(params, width, depth)
    layers = fold(params, width, depth)
    _, acts, pres = forward(params, width, depth, rays, return_acts=True, masks=masks)
    delta = np.asarray(g_dist, dtype=np.float64)[None, :]
    g_layers = [None] * (depth + 1)
    for l in range(depth, -1, -1):
        W = layers[l][0]
        g_layers[l] = (delta @ acts[l].T, delta.sum(axis=1))
        g_in = W.T @ delta
        if l > 0:
            delta = g_in * (pres[l - 1] > 0.0)
            if masks is not None:
                delta = delta * masks[l - 1]
    g_hidden = []
    for (v, g, _), (G, gb) in zip(hidden, g_layers[:depth]):
        norm = np.sqrt(np.sum(v * v, axis=1))
        u = v / norm[:, None]
        gg = np.sum(G * u, axis=1)
        gv = (g / norm)[:, None] * (G - gg[:, None] * u)
        g_hidden.append((gv, gg, gb))
    return g_in, pack(g_hidden, g_layers[depth])


def backward_input_bf16(params, width, depth, rays, g_dist):
    """Input gradient with bfloat16 operands in the hidden layers' products, float64 sums.

    The forward pass (and its ReLU masks) is ``forward_bf16``'s; the adjoint of the last
    hidden layer is the unrounded output row times the seed; every transposed product,
    the first layer's included, rounds its weights and its incoming adjoint to bfloat16.
    Returns g_rays [5, N].  Pinned: equals ``backward`` when every operand is
    representable, and by a hand-worked case where the adjoint's rounding decides.
    """
    layers = fold(params, width, depth)
    W0, b0 = layers[0]
    z = W0 @ np.asarray(rays, dtype=np.float64) + b0[:, None]
    pres = [z]
    h = mlp.round_bf16(np.maximum(z, 0.0))
    for W, b in layers[1:depth]:
        z = mlp.round_bf16(W) @ h + b[:, None]
        pres.append(z)
        h = mlp.round_bf16(np.maximum(z, 0.0))
    delta = (layers[depth][0].T @ np.asarray(g_dist, dtype=np.float64)[None, :]) * (pres[-1] > 0.0)
    for l in range(depth - 1, 0, -1):
        delta = (mlp.round_bf16(layers[l][0]).T @ mlp.round_bf16(delta)) * (pres[l - 1] > 0.0)
    return mlp.round_bf16(W0).T @ mlp.round_bf16(delta)


def train_step(params, width, depth, rays, t, m, v, step, kind="clamp", delta=1.0, lr=1e-3, dropout=0.0,
               seed=0):
    """One training step of Sec. V-A: the paper's loss (``mlp.paper_loss_and_seeds``: the
    clamp loss of Eq. 7 or the squish loss of Eq. 6) on the distance of the network with
    dropout ``dropout`` (the paper: 0.5; masks of this step from ``seed``), its gradient with
    respect to (v, g, b) of every layer, and one Adam update of those parameters.
    Returns (loss, grad, params, m, v)."""
    masks = dropout_masks(seed, step, width, depth, np.asarray(rays).shape[1], dropout)
    dist = forward(params, width, depth, rays, masks=masks)
    loss, seeds = mlp.paper_loss_and_seeds(dist, t, kind, delta)
    _, grad = backward(params, width, depth, rays, seeds, masks=masks)
    p, m, v = mlp.adam_step(params, grad, m, v, step, lr)
    return loss, grad, p, m, v
