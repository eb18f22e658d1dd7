"""Seeded ray sets: origins and unit directions, float32, structure of arrays ``[3][N]``.

Directions are drawn uniformly on the unit sphere as normalised Gaussian
triples (Muller's method) and stored as float32 vectors; converting them to the
(polar, azimuth) angles the network takes is a step of the method and is not
done here.

* ``uniform_cube_rays``: origin ~ U([-1,1]^3), direction uniform on S^2.  Draw
  order: origins (N x 3), then Gaussian directions (N x 3).
* ``unit_ball_rays``: origin uniform in the unit ball (radius u^(1/3) times a
  uniform direction), direction uniform on S^2.
* ``training_rays``: the training-ray recipe, half surface-anchored and half
  uniform in the unit ball.  A surface-anchored ray picks a triangle with
  probability proportional to its area, a point with barycentrics
  (1 - sqrt(u1), sqrt(u1) (1 - u2), sqrt(u1) u2), a direction uniform on S^2,
  and backs the origin off along the ray by s ~ U(0.05, 2), shortened where
  needed so that the origin stays inside the cube [-1,1]^3.  Rays whose origin
  lies inside the mesh are not removed here: the labeller's crossing count
  decides that, and the training loop drops them.
* ``render_rays``: the rays a renderer asks of an object's network, for training
  a network that is rendered: a third enter the cube [-1,1]^3 from a point
  uniform on its surface (a face, then a point on it) in a direction uniform over
  the inward hemisphere (a camera ray starts its query where it enters the cube);
  a third leave the surface (an area-weighted point moved 1e-3 off the surface
  along its face normal, to a side chosen at random, in a direction uniform over
  that side's hemisphere: the bounce and shadow rays); the rest follow
  ``training_rays``.  Origins inside the mesh are left to the labeller's crossing
  count, as there.
"""
import numpy as np


def _unit_dirs(rng, n):
    g = rng.normal(size=(n, 3))
    nrm = np.linalg.norm(g, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return g / nrm


def _soa(o, d):
    return (np.ascontiguousarray(o.T.astype(np.float32)), np.ascontiguousarray(d.T.astype(np.float32)))


def uniform_cube_rays(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(-1.0, 1.0, size=(n, 3))
    d = _unit_dirs(rng, n)
    return _soa(o, d)


def _ball_points(rng, n):
    r = rng.random(n) ** (1.0 / 3.0)
    return _unit_dirs(rng, n) * r[:, None]


def unit_ball_rays(n, seed):
    rng = np.random.default_rng(seed)
    o = _ball_points(rng, n)
    d = _unit_dirs(rng, n)
    return _soa(o, d)


def area_weighted_surface_points(v, f, n, rng):
    """Points on the mesh surface: triangle chosen with probability proportional to area."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    p = area / area.sum()
    tri = rng.choice(len(f), size=n, p=p)
    u1, u2 = rng.random(n), rng.random(n)
    s1 = np.sqrt(u1)
    w0, w1, w2 = 1.0 - s1, s1 * (1.0 - u2), s1 * u2
    q = w0[:, None] * a[tri] + w1[:, None] * b[tri] + w2[:, None] * c[tri]
    return q, tri


def _max_backoff(q, d):
    """Largest s >= 0 with q - s d inside [-1,1]^3 (q is inside the cube)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        lim = np.where(d > 0, (q + 1.0) / d, np.where(d < 0, (q - 1.0) / d, np.inf))
    return lim.min(axis=1)


def training_rays(v, f, n, seed):
    """Returns ``(orig [3][n], dirs [3][n], anchored bool [n])``; the first half is surface-anchored."""
    rng = np.random.default_rng(seed)
    n_s = n // 2
    q, _ = area_weighted_surface_points(v, f, n_s, rng)
    d_s = _unit_dirs(rng, n_s)
    s = rng.uniform(0.05, 2.0, size=n_s)
    s = np.minimum(s, _max_backoff(q, d_s))
    o_s = q - s[:, None] * d_s
    o_u = _ball_points(rng, n - n_s)
    d_u = _unit_dirs(rng, n - n_s)
    o = np.concatenate([o_s, o_u])
    d = np.concatenate([d_s, d_u])
    o = np.clip(o, -1.0, 1.0)
    anchored = np.zeros(n, dtype=bool)
    anchored[:n_s] = True
    oo, dd = _soa(o, d)
    return oo, dd, anchored


def dataset_uniforms(m, s_fc, s_dr, seed):
    """Uniforms of the face-point and direction samplers, float32 in [0, 1).

    Returns ``face_uv`` [2, m * s_fc] (column f * s_fc + j: the (a, b) pair of
    point j of face f) and ``dir_uv`` [2, m * s_dr] (column f * s_dr + j: the
    (a, b) pair of direction j of face f).  Draw order: face pairs, then direction
    pairs, each row-major over (column, component).
    """
    rng = np.random.default_rng(seed)
    face_uv = np.ascontiguousarray(rng.random((m * s_fc, 2), dtype=np.float32).T)
    dir_uv = np.ascontiguousarray(rng.random((m * s_dr, 2), dtype=np.float32).T)
    return face_uv, dir_uv


def grid_points(n_side, half=0.95):
    """Regular grid of n_side^3 points in [-half, half]^3, float32 [3, n_side^3] (x fastest)."""
    c = np.linspace(-half, half, n_side)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()]).astype(np.float32))


def render_rays(v, f, n, seed):
    """Returns ``(orig [3][n], dirs [3][n])``: cube-entry rays, surface-leaving rays, training rays."""
    rng = np.random.default_rng(seed)
    n_c = n // 3
    n_b = n // 3
    # entering the cube: face (axis k, side sg), point on it, inward hemisphere
    k = rng.integers(0, 3, n_c)
    sg = np.where(rng.random(n_c) < 0.5, -1.0, 1.0)
    o_c = rng.uniform(-1.0, 1.0, size=(n_c, 3))
    o_c[np.arange(n_c), k] = sg
    d_c = _unit_dirs(rng, n_c)
    out = d_c[np.arange(n_c), k] * sg > 0
    d_c[np.arange(n_c)[out], k[out]] *= -1.0
    # leaving the surface: point, side of its face, that side's hemisphere
    q, tri = area_weighted_surface_points(v, f, n_b, rng)
    a, b, c = v[f[tri, 0]], v[f[tri, 1]], v[f[tri, 2]]
    nrm = np.cross(b - a, c - a)
    nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-30)
    side = np.where(rng.random(n_b) < 0.5, -1.0, 1.0)[:, None] * nrm
    o_b = np.clip(q + 1e-3 * side, -1.0, 1.0)
    d_b = _unit_dirs(rng, n_b)
    d_b = np.where(np.sum(d_b * side, axis=1, keepdims=True) < 0, -d_b, d_b)
    o_t, d_t, _ = training_rays(v, f, n - n_c - n_b, int(rng.integers(0, 2 ** 31)))
    o = np.concatenate([o_c, o_b, o_t.T.astype(np.float64)])
    d = np.concatenate([d_c, d_b, d_t.T.astype(np.float64)])
    return _soa(o, d)
