"""Pins of the UDF oracle (Sec. III-A, Eq. 5) against fields with closed forms."""
import numpy as np

import synthetic
from oracle import geometry, udf


def _sphere_field(r):
    """Analytic directional distance to the sphere |x| = r (closed-form ray/sphere distance)."""
    def field(rays):
        o = rays[:3]
        d = geometry.dirs_from_angles(rays[3], rays[4])
        b = np.sum(o * d, 0)
        c = np.sum(o * o, 0) - r * r
        disc = b * b - c
        sq = np.sqrt(np.maximum(disc, 0.0))
        t0, t1 = -b - sq, -b + sq
        t = np.where(t0 > 0, t0, t1)
        hit = (disc >= 0) & (t > 0)
        return hit, np.where(hit, t, np.inf)
    return field


def test_udf_of_a_sphere_is_the_unsigned_distance():
    r = 0.6
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(3, 500))
    x = x[:, np.abs(np.linalg.norm(x, axis=0) - r) > 1e-3]
    _, d = synthetic.uniform_cube_rays(256, 3)
    d = d.astype(np.float64)
    d /= np.linalg.norm(d, axis=0)
    u_all = []
    for k in range(x.shape[1]):   # one set per point, holding the direction to its nearest surface point at 100
        xs = x[:, k:k + 1]
        toward = -np.sign(np.linalg.norm(xs) - r) * xs[:, 0] / np.linalg.norm(xs)
        dk = d.copy()
        dk[:, 100] = toward
        u, arg = udf.udf(_sphere_field(r), xs, dk)
        u_all.append(u[0])
        assert arg[0] == 100
    np.testing.assert_allclose(u_all, np.abs(np.linalg.norm(x, axis=0) - r), rtol=1e-12, atol=1e-12)


def test_udf_misses_give_infinity_and_ties_the_lowest_index():
    r = 0.3
    x = np.array([[0.9], [0.0], [0.0]])
    away = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]).T          # both miss the sphere
    u, arg = udf.udf(_sphere_field(r), x, away)
    assert np.isinf(u[0]) and arg[0] == -1
    toward = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]]).T
    u, arg = udf.udf(_sphere_field(r), x, toward)
    np.testing.assert_allclose(u[0], 0.6, rtol=1e-12)
    assert arg[0] == 1
    # the query grid is point-major with the angles of Eq. 1
    g = udf.query_grid(np.zeros((3, 2)), toward)
    assert g.shape == (5, 6)
    np.testing.assert_allclose(geometry.dirs_from_angles(g[3], g[4])[:, :3], toward, atol=1e-15)


def test_network_field_is_the_hit_masked_distance():
    width, depth = 8, 1
    p = synthetic.random_params(width, depth, 4)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, size=(3, 7))
    _, d = synthetic.uniform_cube_rays(9, 6)
    u, arg = udf.udf(udf.network_field(p, width, depth), x, d)
    from oracle import mlp
    logit, dist = mlp.forward(p, width, depth, udf.query_grid(x, d))
    D = np.where(logit > 0, dist, np.inf).reshape(7, 9)
    for k in range(7):   # brute force, one point at a time
        best, bi = np.inf, -1
        for j in range(9):
            if D[k, j] < best:
                best, bi = D[k, j], j
        assert u[k] == best and arg[k] == bi
