"""Pins of the geometry oracle: closed forms, the icosphere sandwich, exact rational brute force."""
from fractions import Fraction

import numpy as np
import pytest

import synthetic
from oracle import geometry


def test_dirs_closed_form():
    d = geometry.dirs_from_angles([0.0, np.pi / 2, np.pi / 2, np.pi], [0.0, 0.0, np.pi / 2, 1.234])
    expect = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [0, 0, -1]], dtype=np.float64).T
    np.testing.assert_allclose(d, expect, atol=1e-15)


def test_angles_round_trip_and_ranges():
    o, d = synthetic.uniform_cube_rays(4096, 11)
    th, ph = geometry.angles_from_dirs(d)
    assert np.all((th >= 0) & (th <= np.pi))
    assert np.all((ph >= 0) & (ph < 2 * np.pi))
    dd = geometry.dirs_from_angles(th, ph)
    dn = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=0)
    np.testing.assert_allclose(dd, dn, atol=1e-14)
    # poles: azimuth 0; negative-y half plane maps into (pi, 2 pi)
    # columns: +z, -z, -y, (1, -1, 0)
    th, ph = geometry.angles_from_dirs(np.array([[0.0, 0.0, 0.0, 1.0], [0.0, 0.0, -1.0, -1.0], [1.0, -1.0, 0.0, 0.0]]))
    assert ph[0] == 0.0 and th[0] == 0.0 and th[1] == np.pi and ph[1] == 0.0
    assert th[2] == np.pi / 2 and ph[2] == 3 * np.pi / 2
    np.testing.assert_allclose(ph[3], 7 * np.pi / 4, rtol=1e-15)


def test_cube_entry_closed_form():
    o = np.array([[-3.0, 0.0, 0.0], [0.2, 0.0, 0.0], [0.0, 5.0, 0.0], [3.0, 0.0, 0.0]]).T
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]).T
    t_in, t_out, hit = geometry.cube_entry(o, d)
    assert hit.tolist() == [True, True, False, False]
    assert t_in[0] == 2.0 and t_out[0] == 4.0
    assert t_in[1] == -1.0 and t_out[1] == 1.0


def _quad():
    v = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], dtype=np.float64)
    f = np.array([[0, 1, 2], [0, 2, 3]])
    return synthetic.tri_soup(v, f)


def test_quad_closed_form():
    rng = np.random.default_rng(5)
    n = 2000
    o = np.stack([rng.uniform(-2, 2, n), rng.uniform(-2, 2, n), rng.uniform(0.1, 2, n)])
    d = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), -rng.uniform(0.2, 1, n)])
    d /= np.linalg.norm(d, axis=0)
    o, d = o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)
    r = geometry.nearest_hit(o, d, _quad())
    t_plane = -o[2] / d[2]
    x = o + t_plane * d
    inside = (np.abs(x[0]) <= 1) & (np.abs(x[1]) <= 1)
    ok = ~r["ambiguous"]
    assert ok.mean() > 0.99
    np.testing.assert_array_equal((r["tri"] >= 0)[ok], inside[ok])
    np.testing.assert_allclose(r["t"][ok & inside], t_plane[ok & inside], rtol=1e-13)
    # the diagonal x = y is shared by both triangles; away from it the id follows the half
    side = np.where(x[1] < x[0], 0, 1)
    far = ok & inside & (np.abs(x[0] - x[1]) > 1e-6)
    np.testing.assert_array_equal(r["tri"][far], side[far])
    assert np.all(r["crossings"][ok] == inside[ok])


def test_single_triangle_barycentric():
    rng = np.random.default_rng(6)
    v = rng.normal(size=(3, 3))
    tris = synthetic.tri_soup(v, np.array([[0, 1, 2]]))
    V = tris.astype(np.float64).reshape(3, 3, 1)[:, :, 0]   # corners as rows
    for _ in range(200):
        a, b = rng.random(2)
        if a + b > 1:
            a, b = 1 - a, 1 - b
        P = (1 - a - b) * V[0] + a * V[1] + b * V[2]
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        t = rng.uniform(0.1, 3)
        o = P - t * d
        r = geometry.nearest_hit(o[:, None], d[:, None], tris)
        if r["ambiguous"][0]:
            continue
        assert r["tri"][0] == 0
        assert abs(r["t"][0] - t) < 1e-10 * (1 + t)
        # the opposite direction misses (origin behind), t_max before the hit misses
        assert geometry.nearest_hit(o[:, None], -d[:, None], tris)["tri"][0] == -1
        assert geometry.nearest_hit(o[:, None], d[:, None], tris, 0.0, t * 0.999)["tri"][0] == -1


@pytest.fixture(scope="module")
def ico():
    v, f = synthetic.icosphere(2, 0.8)
    return v, f, synthetic.tri_soup(v, f)


def test_icosphere_counts(ico):
    v, f, _ = ico
    assert v.shape == (162, 3) and f.shape == (320, 3)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 0.8, rtol=1e-15)


def _plane_dist(tris):
    v0, v1, v2 = geometry.triangles_from_soup(tris)
    n = np.cross(v1 - v0, v2 - v0, axis=0)
    n /= np.linalg.norm(n, axis=0)
    return np.abs(np.sum(n * v0, axis=0))


def test_icosphere_sandwich(ico):
    v, f, tris = ico
    r_in = _plane_dist(tris).min()
    assert 0.7857 < r_in < 0.7859
    # from the centre: t between the inscribed radius and 0.8; one crossing
    o, d = synthetic.uniform_cube_rays(3000, 21)
    z = np.zeros_like(o)
    r = geometry.nearest_hit(z, d, tris)
    ok = ~r["ambiguous"]
    assert ok.mean() > 0.99
    assert np.all((r["t"][ok] >= r_in - 1e-12) & (r["t"][ok] <= 0.8 + 1e-12))
    assert np.all(r["crossings"][ok] == 1)
    # towards the vertices: t = 0.8 exactly up to rounding; towards face centroids: |centroid|
    vv = tris.astype(np.float64)
    cen = (vv[0:3] + vv[3:6] + vv[6:9]) / 3
    r = geometry.nearest_hit(np.zeros_like(cen), cen, tris)
    # direction = centroid (not unit), so the hit parameter is t = 1
    np.testing.assert_allclose(r["t"], 1.0, rtol=1e-12)
    np.testing.assert_array_equal(r["tri"], np.arange(320))
    dv = np.ascontiguousarray(vv[0:3, :40])
    r = geometry.nearest_hit(np.zeros_like(dv), dv / np.linalg.norm(dv, axis=0), tris)
    np.testing.assert_allclose(r["t"], np.linalg.norm(dv, axis=0), rtol=1e-12)


def test_icosphere_outside_rays_and_parity(ico):
    _, _, tris = ico
    r_in = _plane_dist(tris).min()
    o, d = synthetic.uniform_cube_rays(20000, 22)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    r = geometry.nearest_hit(o64, d64, tris)
    ok = ~r["ambiguous"]
    on = np.linalg.norm(o64, axis=0)
    # odd-even rule: inside the inscribed ball -> odd, outside the circumscribed ball -> even
    assert np.all(r["crossings"][ok & (on < r_in)] % 2 == 1)
    assert np.all(r["crossings"][ok & (on > 0.8)] % 2 == 0)

    def ball_entry(rad):
        b = np.sum(o64 * d64, axis=0)
        c = on ** 2 - rad ** 2
        disc = b * b - c
        return -b - np.sqrt(np.maximum(disc, 0)), disc

    t_in_r, disc_r = ball_entry(r_in)
    t_out_08, disc_08 = ball_entry(0.8)
    outside = on > 0.8
    hits_inner = outside & (disc_r > 0) & (t_in_r > 0)
    sel = ok & hits_inner
    assert sel.sum() > 1000
    assert np.all(r["t"][sel] >= t_out_08[sel] - 1e-12)
    assert np.all(r["t"][sel] <= t_in_r[sel] + 1e-12)
    misses_outer = outside & ((disc_08 < 0) | (t_out_08 < 0))
    assert np.all(r["tri"][ok & misses_outer] == -1)


def _exact_hits(o, d, V):
    """Exact rational nearest hit and crossing count by Cramer's rule on o + t d = v0 + u e1 + v e2."""
    best, best_i, cross = None, -1, 0
    for i, (a, b, c) in enumerate(V):
        e1 = [b[k] - a[k] for k in range(3)]
        e2 = [c[k] - a[k] for k in range(3)]
        s = [o[k] - a[k] for k in range(3)]
        # columns: [-d, e1, e2] [t u v]^T = s
        M = [[-d[k], e1[k], e2[k]] for k in range(3)]

        def det3(m):
            return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                    - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                    + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))

        D = det3(M)
        if D == 0:
            continue
        sol = []
        for col in range(3):
            Mc = [row[:] for row in M]
            for k in range(3):
                Mc[k][col] = s[k]
            sol.append(det3(Mc) / D)
        t, u, v = sol
        if u >= 0 and v >= 0 and u + v <= 1 and t > 0:
            cross += 1
            if best is None or t < best:
                best, best_i = t, i
    return best, best_i, cross


def test_exact_rational_brute_force():
    rng = np.random.default_rng(23)
    v, f = synthetic.icosphere(0, 0.7)           # 20 triangles -> keep 12 of them
    f = f[:12]
    tris = synthetic.tri_soup(v, f)
    o, d = synthetic.uniform_cube_rays(600, 24)
    r = geometry.nearest_hit(o, d, tris)
    tv = tris.astype(np.float64)
    V = [[[Fraction(float(tv[3 * c + k, i])) for k in range(3)] for c in range(3)] for i in range(tris.shape[1])]
    checked = 0
    for j in range(o.shape[1]):
        if r["ambiguous"][j]:
            continue
        oj = [Fraction(float(x)) for x in o[:, j]]
        dj = [Fraction(float(x)) for x in d[:, j]]
        t, i, c = _exact_hits(oj, dj, V)
        assert r["crossings"][j] == c
        if t is None:
            assert r["tri"][j] == -1
        else:
            assert r["tri"][j] == i
            assert abs(r["t"][j] - float(t)) <= 1e-12 * (1 + float(t))
        checked += 1
    assert checked > 590
    assert (r["tri"] >= 0).sum() > 50
