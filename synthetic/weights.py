"""Network parameters: the flat float32 parameter vector and its layer order.

The network has ``depth`` hidden layers of ``width`` ReLU units on a 65-value
input and a 2-value output (hit logit, distance), so ``depth + 1`` affine
layers.  The flat vector stores, layer after layer, the weight matrix in
row-major ``[out][in]`` order followed by the bias ``[out]`` (the order of
``torch.nn.Linear`` parameters).

Xavier-uniform initialisation: ``U(-a, a)`` with ``a = sqrt(6 / (fan_in + fan_out))``,
gain 1, biases zero; drawn layer after layer from ``default_rng(seed)``.
"""
import numpy as np

IN_DIM = 65
OUT_DIM = 2


def layer_shapes(width, depth, in_dim=IN_DIM, out_dim=OUT_DIM):
    dims = [in_dim] + [width] * depth + [out_dim]
    return [(dims[i + 1], dims[i]) for i in range(depth + 1)]


def param_count(width, depth, in_dim=IN_DIM, out_dim=OUT_DIM):
    return sum(o * i + o for o, i in layer_shapes(width, depth, in_dim, out_dim))


def xavier_params(width, depth, seed, in_dim=IN_DIM, out_dim=OUT_DIM):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in layer_shapes(width, depth, in_dim, out_dim):
        a = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=(o, i)).ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def random_params(width, depth, seed, bias_scale=0.1, in_dim=IN_DIM, out_dim=OUT_DIM):
    """Xavier weights with non-zero uniform biases (exercises the bias path in tests)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in layer_shapes(width, depth, in_dim, out_dim):
        a = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=(o, i)).ravel())
        parts.append(rng.uniform(-bias_scale, bias_scale, size=o))
    return np.concatenate(parts).astype(np.float32)


def multi_object_network_shape(seed):
    """Width in {128, 256} and depth in 4..8 of the network of one multi-object scene object,
    drawn from ``default_rng(seed)`` (width first)."""
    rng = np.random.default_rng(seed)
    width = int(rng.choice([128, 256]))
    depth = int(rng.integers(4, 9))
    return width, depth


PAPER_WIDTH = 512


def paper_params(depth, seed, width=PAPER_WIDTH, bias_scale=0.1):
    """Parameters of the paper's network (weight-normalised hidden layers on the 5 raw ray
    values, one output): per hidden layer v [width][in] Xavier-uniform, g = |v| per row (the
    weight-norm start, so W = v), b uniform in +-bias_scale; then the output row
    (Xavier-uniform) and a zero bias.  Drawn layer after layer from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    dims = [5] + [width] * depth
    parts = []
    for l in range(depth):
        i, o = dims[l], dims[l + 1]
        a = np.sqrt(6.0 / (i + o))
        v = rng.uniform(-a, a, size=(o, i)).astype(np.float32)
        parts += [v.ravel(), np.sqrt(np.sum(v.astype(np.float64) ** 2, axis=1)).astype(np.float32),
                  rng.uniform(-bias_scale, bias_scale, size=o).astype(np.float32)]
    a = np.sqrt(6.0 / (width + 1))
    parts += [rng.uniform(-a, a, size=width).astype(np.float32), np.zeros(1, np.float32)]
    return np.concatenate(parts).astype(np.float32)
