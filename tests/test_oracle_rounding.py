"""Hand-derived pins of where the reduced-precision emulations round, and of the tie rule of the
nearest-hit search.

Each network here is built by hand so that one rounding step (of the encoding, a weight, a
hidden activation, an adjoint, an fp8 quantisation or saturation) decides the answer: the
network subtracts 1 from a value that is 1 + 2^-9 in float64 but exactly 1 after bfloat16
rounding (1 + 2^-4 and e4m3 for fp8), so the output is 0 where the emulation rounds in the
stated place and the unrounded remainder where it does not.  Expected values are worked out in
the comments; none is produced by the oracle itself.

bfloat16 has 8 significant bits: near 1 its spacing is 2^-7, so 1 + 2^-9 rounds to 1.
e4m3 has 4 significant bits: near 1 its spacing is 2^-3, so 1 + 2^-4 is a tie and rounds to the
even neighbour 1; its largest finite value is 448.
"""
import numpy as np

import synthetic
from oracle import geometry, mlp

E9 = 2.0 ** -9
E4 = 2.0 ** -4


def _net(width, depth):
    layers = mlp.unpack(np.zeros(synthetic.param_count(width, depth)), width, depth)
    return [(W.copy(), b.copy()) for W, b in layers]


def _ray(ox):
    """One ray (ox, 0, 0, 0, 0): its raw feature 0 is ox; only feature 0 carries weight below."""
    r = np.zeros((5, 1))
    r[0, 0] = ox
    return r


def _bf16(layers, width, depth, rays):
    lg, ds = mlp.forward_bf16(mlp.pack(layers), width, depth, rays)
    return lg[0], ds[0]


# ----------------------------------------------------------------------------- bfloat16 forward
def test_bf16_forward_rounds_the_encoding():
    # ox = 1 + 2^-9 -> feature 0 rounds to 1; unit 0 = relu(f0 - 1) = 0; dist = unit 0 + 0.5.
    # Without rounding the encoding, unit 0 = 2^-9 (exact in bf16) and dist = 0.5 + 2^-9.
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0, -1.0
    L[1][0][1, 0], L[1][1][1] = 1.0, 0.5
    L[1][0][0, 0], L[1][1][0] = -1.0, 0.25
    lg, ds = _bf16(L, 2, 1, _ray(1.0 + E9))
    assert ds == 0.5 and lg == 0.25


def test_bf16_forward_rounds_hidden_activations():
    # depth 2: unit 0 of layer 1 = relu(ox + 2^-9) = 1 + 2^-9 in float64, stored as bf16 1;
    # unit 0 of layer 2 = relu(h - 1) = 0; dist = that + 0.5.  Without the rounding: 0.5 + 2^-9.
    L = _net(2, 2)
    L[0][0][0, 0], L[0][1][0] = 1.0, E9
    L[1][0][0, 0], L[1][1][0] = 1.0, -1.0
    L[2][0][1, 0], L[2][1][1] = 1.0, 0.5
    _, ds = _bf16(L, 2, 2, _ray(1.0))
    assert ds == 0.5
    # the last hidden layer's output is rounded before the head too: depth 1, h = bf16(1 + 2^-9)
    # = 1, dist = h - 1 = 0 (unrounded: 2^-9)
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0, E9
    L[1][0][1, 0], L[1][1][1] = 1.0, -1.0
    _, ds = _bf16(L, 2, 1, _ray(1.0))
    assert ds == 0.0


def test_bf16_forward_rounds_hidden_weights_but_not_biases():
    # W = 1 + 2^-9 rounds to 1: unit 0 = relu(1 * 1 - 1) = 0, dist = 0.5 (unrounded W: 0.5 + 2^-9)
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0 + E9, -1.0
    L[1][0][1, 0], L[1][1][1] = 1.0, 0.5
    _, ds = _bf16(L, 2, 1, _ray(1.0))
    assert ds == 0.5
    # the head's bias is added unrounded: 0.5 + 2^-12 survives (bf16 would make it 0.5)
    L[1][1][1] = 0.5 + 2.0 ** -12
    _, ds = _bf16(L, 2, 1, _ray(1.0))
    assert ds == 0.5 + 2.0 ** -12


def test_bf16_head_rows_keep_their_remainder():
    # h = 1 exactly; the distance row's weight 1 + 2^-9 + 2^-13 (14 significant bits) is carried as
    # bf16(w) + bf16(w - bf16(w)) = (1) + (2^-9 + 2^-13), so dist = w exactly; a single bf16
    # weight would give 1.
    L = _net(2, 1)
    L[0][0][0, 0] = 1.0
    w = 1.0 + E9 + 2.0 ** -13
    L[1][0][1, 0] = w
    _, ds = _bf16(L, 2, 1, _ray(1.0))
    assert ds == w


# ----------------------------------------------------------------------------- bfloat16 input gradient
def _gin(layers, width, depth, rays, gl, gd):
    return mlp.backward_input_bf16(mlp.pack(layers), width, depth, rays, np.array([gl]), np.array([gd]))[:, 0]


def test_bf16_input_gradient_rounds_the_first_layer_adjoint():
    # depth 1, ray ox = 0.5: pre-activations (0.5 + 1, -0.5 + 1) = (1.5, 0.5) > 0.  The head's
    # distance row (1 + 2^-9, 1) is unrounded, so the adjoint at the hidden layer is (1 + 2^-9, 1);
    # rounded to bf16 it is (1, 1), and the first-layer product gives d/d(ox) = 1 * 1 - 1 * 1 = 0.
    # Without rounding the adjoint: 2^-9.
    L = _net(2, 1)
    L[0][0][0, 0], L[0][0][1, 0] = 1.0, -1.0
    L[0][1][:] = 1.0
    L[1][0][1, :] = (1.0 + E9, 1.0)
    g = _gin(L, 2, 1, _ray(0.5), 0.0, 1.0)
    np.testing.assert_array_equal(g, np.zeros(5))


def test_bf16_input_gradient_rounds_the_first_layer_weights():
    # first-layer weights (1 + 2^-9, -1) in column 0 round to (1, -1); adjoint (1, 1):
    # d/d(ox) = 1 - 1 = 0 (unrounded weights: 2^-9).  Pre-activations 1 * 0.5 + 1 and -0.5 + 1 > 0.
    L = _net(2, 1)
    L[0][0][0, 0], L[0][0][1, 0] = 1.0 + E9, -1.0
    L[0][1][:] = 1.0
    L[1][0][1, :] = (1.0, 1.0)
    g = _gin(L, 2, 1, _ray(0.5), 0.0, 1.0)
    np.testing.assert_array_equal(g, np.zeros(5))


def test_bf16_input_gradient_rounds_hidden_adjoints():
    # depth 2, ox = 0.5.  Layer 1: unit 0 = 0.5 + 1 = 1.5, unit 1 = 1.  Layer 2 (biases 3):
    # (1.5 + 3, -1.5 + 3) = (4.5, 1.5) > 0.  Head distance row (1 + 2^-9, 1): adjoint at layer 2 =
    # (1 + 2^-9, 1) -> bf16 (1, 1); through layer 2's weights (column 0 = (1, -1)) the adjoint of
    # unit 0 of layer 1 is 1 - 1 = 0, so d/d(ox) = 0 (unrounded: 2^-9).
    L = _net(2, 2)
    L[0][0][0, 0] = 1.0
    L[0][1][:] = 1.0
    L[1][0][0, 0], L[1][0][1, 0] = 1.0, -1.0
    L[1][1][:] = 3.0
    L[2][0][1, :] = (1.0 + E9, 1.0)
    g = _gin(L, 2, 2, _ray(0.5), 0.0, 1.0)
    np.testing.assert_array_equal(g, np.zeros(5))


def test_bf16_input_gradient_takes_its_masks_from_the_bf16_forward():
    # first-layer weight 1 + 2^-9 -> 1, ox = 1, bias -1: the bf16 pre-activation is exactly 0, so
    # the ReLU passes nothing back (ReLU'(0) = 0) and the gradient is 0.  In float64 the
    # pre-activation is 2^-9 > 0 and d/d(ox) would be 1 (the bf16 weight times the head's 1).
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0 + E9, -1.0
    L[1][0][1, 0] = 1.0
    g = _gin(L, 2, 1, _ray(1.0), 0.0, 1.0)
    np.testing.assert_array_equal(g, np.zeros(5))
    L[0][1][0] = -0.5      # pre-activation 0.5 > 0 in both: d/d(ox) = bf16(1 + 2^-9) * 1 = 1
    g = _gin(L, 2, 1, _ray(1.0), 0.0, 1.0)
    np.testing.assert_array_equal(g, [1.0, 0, 0, 0, 0])


# ----------------------------------------------------------------------------- fp8 e4m3 forward
def _fp8(layers, width, depth, rays, scales):
    lg, ds = mlp.forward_fp8(mlp.pack(layers), width, depth, rays, np.asarray(scales, np.float64))
    return lg[0], ds[0]


def test_fp8_quantises_layer_inputs():
    # ox = 1 + 2^-4 quantises to 1 (a tie, to even): unit 0 = relu(1 - 1) = 0, dist = 0 + 0.5.
    # Without quantising the input: unit 0 = 2^-4 (representable), dist = 0.5625.
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0, -1.0
    L[1][0][1, 0], L[1][1][1] = 1.0, 0.5
    _, ds = _fp8(L, 2, 1, _ray(1.0 + E4), np.ones(4))
    assert ds == 0.5
    # the head's input is quantised too: unit 0 = 1 + 2^-4 (bias 2^-4, ox = 1), seen as 1 by the
    # head, dist = 1 - 1 = 0 (unquantised: 2^-4)
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0, E4
    L[1][0][1, 0], L[1][1][1] = 1.0, -1.0
    _, ds = _fp8(L, 2, 1, _ray(1.0), np.ones(4))
    assert ds == 0.0


def test_fp8_saturates_at_448():
    # ox = 500 saturates to 448 (scale 1); unit 0 = relu(448 - 448) = 0; dist = 0.5.
    # Without saturation: relu(500 - 448) = 52 (representable) and dist = 52.5.
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0, -448.0
    L[1][0][1, 0], L[1][1][1] = 1.0, 0.5
    _, ds = _fp8(L, 2, 1, _ray(500.0), np.ones(4))
    assert ds == 0.5


def test_fp8_quantises_weights_and_applies_both_scales():
    # weight 1 + 2^-4 -> 1, ox = 1, bias -1: unit 0 = 0, dist = 0.5 (unquantised: 0.5625)
    L = _net(2, 1)
    L[0][0][0, 0], L[0][1][0] = 1.0 + E4, -1.0
    L[1][0][1, 0], L[1][1][1] = 1.0, 0.5
    _, ds = _fp8(L, 2, 1, _ray(1.0), np.ones(4))
    assert ds == 0.5
    # scales s_w = 2, s_a = 4 on the first layer: weight 2 (q = 1), ox = 4.25 (q = 4.25 / 4 =
    # 1 + 2^-4 -> 1): 1 * 1 * 2 * 4 - 8 = 0 -> dist 0.5 (unquantised: 2 * 4.25 - 8 = 0.5 -> 1.0)
    L[0][0][0, 0], L[0][1][0] = 2.0, -8.0
    _, ds = _fp8(L, 2, 1, _ray(4.25), [2.0, 4.0, 1.0, 1.0])
    assert ds == 0.5


# ----------------------------------------------------------------------------- nearest hit ties
def _soup(tris):
    """[[v0, v1, v2], ...] -> [9][m] float32 soup."""
    t = np.asarray(tris, dtype=np.float64)
    return t.reshape(len(tris), 9).T.astype(np.float32)


def test_nearest_hit_exact_ties_go_to_the_lowest_index():
    far = [(5, 5, 5), (6, 5, 5), (5, 6, 5)]
    a = [(0, 0, 0), (1, 0, 0), (0, 1, 0)]
    b = [(-1, -1, 0), (2, -1, 0), (-1, 2, 0)]   # same plane z = 0, also contains (0.25, 0.25, 0)
    o = np.array([[0.25], [0.25], [1.0]])
    d = np.array([[0.0], [0.0], [-1.0]])
    for tris, want in (([far, a, a], 1), ([far, a, b], 1), ([far, b, a], 1), ([a, far, a], 0),
                       ([far, far, b, a, b], 2)):
        r = geometry.nearest_hit(o, d, _soup(tris))
        assert r["t"][0] == 1.0 and r["tri"][0] == want, (tris, r["tri"][0])
        assert r["crossings"][0] == sum(1 for x in tris if x is not far)
