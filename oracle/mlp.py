"""Network oracle: encoding, forward, emulated low precision, loss, backward, Adam, normals.

Test infrastructure only (see the package docstring).

The network is the paper's MLP_w over an oriented point (x, theta) (Sec. IV-A)
with two changes of this workload: the 5-value ray (ox, oy, oz, theta, phi) is
Fourier-encoded to 65 values, and the output is a pair (hit logit, distance)
instead of a single squished distance.  ``depth`` hidden layers of ``width``
ReLU units, ``depth + 1`` affine layers; parameters are the flat vector of
``synthetic.weights`` (per layer: weight ``[out][in]`` row-major, then bias).
"""
import numpy as np

N_FREQ = 6
IN_RAW = 5
IN_DIM = IN_RAW * (1 + 2 * N_FREQ)   # 65
FP8_MAX = 448.0


# ----------------------------------------------------------------------------- parameters
def unpack(params, width, depth, in_dim=IN_DIM, out_dim=2):
    """Split the flat parameter vector into ``[(W [out, in], b [out]), ...]`` in float64."""
    p = np.asarray(params, dtype=np.float64)
    dims = [in_dim] + [width] * depth + [out_dim]
    layers, off = [], 0
    for l in range(depth + 1):
        o, i = dims[l + 1], dims[l]
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        layers.append((W, b))
    if off != p.size:
        raise ValueError("parameter vector has %d values, the network needs %d" % (p.size, off))
    return layers


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# ----------------------------------------------------------------------------- encoding
def encode(rays):
    """Fourier features of the 5-value rays ``[5, N]`` -> ``[65, N]``.

    Order: the 5 raw values; then sin(2^k v_j) for k = 0..5 (outer), j = 0..4
    (inner); then cos(2^k v_j) in the same order.  Frequencies 2^k without a
    factor pi.  (Not in the paper; the workload's input encoding.)  Pinned by
    closed-form values in the tests.
    """
    v = np.asarray(rays, dtype=np.float64)
    feats = [v]
    sins, coss = [], []
    for k in range(N_FREQ):
        a = (2.0 ** k) * v
        sins.append(np.sin(a))
        coss.append(np.cos(a))
    return np.concatenate(feats + sins + coss, axis=0)


def encode_grad(rays, g_feat):
    """Chain rule through ``encode``: d/dv of sum(g_feat * encode(v)), ``[65, N]`` -> ``[5, N]``."""
    v = np.asarray(rays, dtype=np.float64)
    g = np.array(g_feat[:IN_RAW], dtype=np.float64)
    for k in range(N_FREQ):
        f = 2.0 ** k
        gs = g_feat[IN_RAW + IN_RAW * k: IN_RAW + IN_RAW * (k + 1)]
        gc = g_feat[IN_RAW + IN_RAW * N_FREQ + IN_RAW * k: IN_RAW + IN_RAW * N_FREQ + IN_RAW * (k + 1)]
        g = g + f * (gs * np.cos(f * v) - gc * np.sin(f * v))
    return g


# ----------------------------------------------------------------------------- forward
def forward(params, width, depth, rays, return_acts=False):
    """Float64 forward: h_0 = encode(ray); h_l = max(0, W_l h_{l-1} + b_l); out = W h_D + b.

    Sec. IV-A (MLP_w approximating the field) and Sec. V-A (fully connected ReLU
    layers).  Returns ``(logit [N], dist [N])``; a ray is a hit when logit > 0.
    Pinned against an explicit-loop evaluation, zero weights (output = bias)
    and torch float64 in the tests.
    """
    layers = unpack(params, width, depth)
    h = encode(rays)
    acts, pres = [h], []
    for l, (W, b) in enumerate(layers):
        z = W @ h + b[:, None]
        pres.append(z)
        if l < depth:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    if return_acts:
        return h[0], h[1], acts, pres
    return h[0], h[1]


# ----------------------------------------------------------------------------- emulated precision
def round_bf16(x):
    """Round to bfloat16 (nearest, ties to even) via float32, returned as float64.

    The value is first rounded to float32, the precision in which the kernel
    holds it before conversion.  Pinned bit-exactly against torch's CPU cast.
    """
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def round_e4m3(x):
    """Saturating round to OCP fp8 e4m3fn (nearest, ties to even; |x| <= 448).

    4 exponent bits (bias 7), 3 mantissa bits, subnormal step 2^-9, no
    infinities.  The value is first rounded to float32 (the kernel's precision).
    Pinned bit-exactly against torch's CPU ``float8_e4m3fn`` cast after clamping.
    """
    f = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    a = np.minimum(np.abs(f), FP8_MAX)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    quantum = 2.0 ** (e - 3.0)
    q = np.round(a / quantum) * quantum   # numpy rounds half to even
    q = np.minimum(q, FP8_MAX)
    return np.sign(f) * q


def split_bf16(x):
    """``x`` (a float32 value) as ``hi + lo`` with both parts bfloat16.

    hi = bf16(x); lo = bf16(x - hi), where x - hi is exact in float32 (hi is x with
    its low mantissa bits rounded off).  hi + lo keeps 16 significant bits of x.
    """
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    hi = round_bf16(x32)
    return hi, round_bf16(x32 - hi)


def forward_bf16(params, width, depth, rays):
    """Forward with every layer's operands rounded to bfloat16 and float64 sums.

    Weights and layer inputs (the encoding and each hidden activation) are
    rounded to bfloat16; products and sums are exact-ish (float64, standing in
    for the kernel's float32 accumulation); the bias is added unrounded.  The
    head's two weight rows are carried as a sum of two bfloat16 values: the
    rounded row plus the rounded remainder (``split_bf16``), since a rounding
    error there moves the outputs directly rather than through later layers.
    """
    layers = unpack(params, width, depth)
    h = round_bf16(encode(rays))
    for l, (W, b) in enumerate(layers):
        if l < depth:
            Wq = round_bf16(W)
        else:
            hi, lo = split_bf16(W)
            Wq = hi + lo
        z = Wq @ h + b[:, None]
        if l < depth:
            h = round_bf16(np.maximum(z, 0.0))
        else:
            h = z
    return h[0], h[1]


def pow2_scale(absmax):
    """Smallest power of two s with absmax / s <= 448 (1 for an all-zero tensor).

    A power-of-two scale makes every rescaling between layers exact: the ratio
    s_w s_a / s_next is itself a power of two.
    """
    a = float(absmax)
    if not a > 0.0:
        return 1.0
    e = int(np.ceil(np.log2(a / FP8_MAX)))
    # the guess can be one off where a / 448 rounds; comparisons with 448 * 2^e are exact
    while a > FP8_MAX * 2.0 ** e:
        e += 1
    while a <= FP8_MAX * 2.0 ** (e - 1):
        e -= 1
    return float(2.0 ** e)


def fp8_scales(params, width, depth, calib_rays):
    """Per-layer static power-of-two scales for the weight and for the layer input.

    s_w covers the weight absmax and s_a the layer-input absmax over the
    calibration rays (float64 forward), each as ``pow2_scale``.  Returns an
    array ``[2 * (depth + 1)]``: (s_w, s_a) per layer.
    """
    layers = unpack(params, width, depth)
    _, _, acts, _ = forward(params, width, depth, calib_rays, return_acts=True)
    s = []
    for l, (W, _) in enumerate(layers):
        s.append(pow2_scale(np.abs(W).max()))
        s.append(pow2_scale(np.abs(acts[l]).max()))
    return np.array(s)


def forward_fp8(params, width, depth, rays, scales):
    """Forward with e4m3 operands: y = (sum q_w q_a) s_w s_a + b, q = sat(RNE(x / s)).

    Every affine layer (first, hidden and head) is quantised with its own
    per-tensor weight scale and activation scale.
    """
    layers = unpack(params, width, depth)
    h = encode(rays)
    for l, (W, b) in enumerate(layers):
        sw, sa = scales[2 * l], scales[2 * l + 1]
        qw = round_e4m3(W / sw)
        qa = round_e4m3(h / sa)
        z = (qw @ qa) * (sw * sa) + b[:, None]
        h = np.maximum(z, 0.0) if l < depth else z
    return h[0], h[1]


# ----------------------------------------------------------------------------- loss and gradients
def loss_and_seeds(logit, dist, hit, t):
    """Binary cross-entropy on the hit logit plus L1 on the distance over hit rays.

    BCE with logits, mean over the N rays: max(z,0) - z y + log(1 + exp(-|z|));
    L1 mean over rays with y = 1: |dist - t|; weights 1:1.  Returns
    ``(loss, g_logit, g_dist)`` with g_logit = (sigmoid(z) - y) / N and
    g_dist = sign(dist - t) / n_hit on hit rays (sign(0) = 0), zero elsewhere.
    (The paper's own loss is the clamp loss of Eq. 7; this is the workload's.)
    Pinned by central finite differences of ``loss`` in the tests.
    """
    z = np.asarray(logit, dtype=np.float64)
    y = np.asarray(hit, dtype=np.float64)
    d = np.asarray(dist, dtype=np.float64)
    tt = np.where(y > 0, np.asarray(t, dtype=np.float64), 0.0)
    n = z.size
    n_hit = int(y.sum())
    bce = np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z))))
    l1 = (np.abs(d - tt) * y).sum() / n_hit if n_hit else 0.0
    g_logit = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g_dist = np.sign(d - tt) * y / n_hit if n_hit else np.zeros_like(d)
    return bce + l1, g_logit, g_dist


def paper_loss_and_seeds(dist, t, kind, delta=1.0):
    """The paper's losses on the distance output alone (Sec. IV-A Eq. 6, Sec. V-A Eq. 7).

    kind "clamp" (Eq. 7): mean over the N rays of |c(t) - c(d)|, c(x) = min(delta,
    max(-delta, x)); a miss (t = +inf) clamps to delta.  kind "squish" (Eq. 6, reading:
    the absolute value of the difference, sigma = tanh): mean of |tanh(t) - tanh(d)|, with
    tanh(+inf) = 1.  Returns ``(loss, g_dist)``: g_dist = sign(c(d) - c(t)) c'(d) / N with
    sign(0) = 0 and c' the derivative (1 strictly inside the clamp window, 0 outside and
    on its edges; 1 - tanh^2 for the squish).  The logit gets no gradient.
    Pinned by closed-form values and central finite differences in the tests.
    """
    d = np.asarray(dist, dtype=np.float64)
    tt = np.asarray(t, dtype=np.float64)
    n = d.size
    if kind == "clamp":
        cd, ct = np.clip(d, -delta, delta), np.clip(tt, -delta, delta)
        dc = ((d > -delta) & (d < delta)).astype(np.float64)
    elif kind == "squish":
        cd, ct = np.tanh(d), np.tanh(tt)
        dc = 1.0 - cd * cd
    else:
        raise ValueError("kind must be 'clamp' or 'squish'")
    loss = np.abs(ct - cd).mean() if n else 0.0
    return loss, np.sign(cd - ct) * dc / n


def eikonal_loss_and_seeds(dist_a, dist_b, t, h, lam):
    """Directed Eikonal penalty (Sec. III-A, Eq. 2) with the derivative along the ray taken as
    a forward difference: r = (phi(x + h d) - phi(x)) / h + 1, which Eq. 2 makes 0.

    dist_a, dist_b: the network's distances at x and at x + h d (same direction); the penalty
    lam / N * sum r^2 runs over the N rays, counting those whose label is a hit farther than h
    (t finite, t > h: x + h d is still in front of the surface).  Returns (loss, g_a, g_b) with
    g_a = -2 lam r / (N h), g_b = +2 lam r / (N h) on counted rays, 0 elsewhere.
    Pinned by an analytic plane field (r = 0 exactly) and central differences in the tests.
    """
    a = np.asarray(dist_a, dtype=np.float64)
    b = np.asarray(dist_b, dtype=np.float64)
    tt = np.asarray(t, dtype=np.float64)
    n = a.size
    on = np.isfinite(tt) & (tt > h)
    r = np.where(on, (b - a) / h + 1.0, 0.0)
    loss = lam * np.sum(r * r) / n if n else 0.0
    g = 2.0 * lam * r / (n * h)
    return loss, -g, g


def backward(params, width, depth, rays, g_logit, g_dist):
    """Reverse-mode gradient of sum(g_logit * logit + g_dist * dist).

    Returns ``(g_rays [5, N], g_params [P])``.  The input gradient is the
    derivative with respect to the query point and angles that Sec. IV-B takes
    with automatic differentiation for normals; the parameter gradient is the
    usual training backward.  ReLU'(0) = 0.  Pinned by central finite
    differences and by torch float64 autograd in the tests.
    """
    layers = unpack(params, width, depth)
    _, _, acts, pres = forward(params, width, depth, rays, return_acts=True)
    delta = np.stack([np.asarray(g_logit, np.float64), np.asarray(g_dist, np.float64)])
    grads = [None] * len(layers)
    for l in range(depth, -1, -1):
        W, _ = layers[l]
        grads[l] = (delta @ acts[l].T, delta.sum(axis=1))
        g_in = W.T @ delta
        if l > 0:
            delta = g_in * (pres[l - 1] > 0.0)
    g_rays = encode_grad(rays, g_in)
    return g_rays, pack(grads)


def backward_input_bf16(params, width, depth, rays, g_logit, g_dist):
    """Input gradient with bfloat16 operands in every product, float64 sums.

    The forward pass is ``forward_bf16``; the ReLU masks come from its
    pre-activations; the head rows stay unrounded; every transposed product rounds
    its weights and its incoming adjoint to bfloat16.  Returns g_rays [5, N].
    Pinned: equals ``backward`` when every operand is representable.
    """
    layers = unpack(params, width, depth)
    h = round_bf16(encode(rays))
    pres = []
    for l, (W, b) in enumerate(layers[:-1]):
        z = round_bf16(W) @ h + b[:, None]
        pres.append(z)
        h = round_bf16(np.maximum(z, 0.0))
    Wh = layers[-1][0]
    delta = (Wh.T @ np.stack([np.asarray(g_logit, np.float64), np.asarray(g_dist, np.float64)])) * (pres[-1] > 0.0)
    for l in range(depth - 1, 0, -1):
        delta = (round_bf16(layers[l][0]).T @ round_bf16(delta)) * (pres[l - 1] > 0.0)
    g_feat = round_bf16(layers[0][0]).T @ round_bf16(delta)
    return encode_grad(rays, g_feat)


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction and no weight decay.

    The paper optimises with Adam (Sec. V-A).  ``step`` is the 1-based index of
    this update.  Returns new ``(params, m, v)``.  Pinned against
    ``torch.optim.Adam`` in float64 in the tests.
    """
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def normals(g_origin, d):
    """Shading normal from the distance gradient (Eq. 3): n = kappa g / |g| with n . d < 0.

    kappa = -sign(g . d); kappa = +1 when g . d = 0; n = -d when |g| = 0.
    ``g_origin`` and ``d`` are ``[3, N]``.  Pinned with the analytic plane field.
    """
    g = np.asarray(g_origin, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    gn = np.linalg.norm(g, axis=0)
    gd = np.sum(g * d, axis=0)
    kappa = np.where(gd > 0.0, -1.0, 1.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        n = kappa * g / gn
    dn = d / np.linalg.norm(d, axis=0)
    return np.where(gn > 0.0, n, -dn)
