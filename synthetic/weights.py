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
