"""Pins of the dataset oracle (Sec. V-B, Eqs. 8-12) against geometry it does not compute itself:
points on their faces and uniform, the angle kinds as directions, a quad whose perpendicular
hits have a closed form, the convex-mesh rejection rule and the labelling rules of Fig. 2b."""
import numpy as np
import pytest

import synthetic
from oracle import dataset, geometry


def _barycentric(pts, v0, v1, v2):
    """Barycentric coordinates of points in the planes of their triangles (least squares)."""
    e1, e2, r = v1 - v0, v2 - v0, pts - v0
    d11, d12, d22 = np.sum(e1 * e1, 0), np.sum(e1 * e2, 0), np.sum(e2 * e2, 0)
    r1, r2 = np.sum(r * e1, 0), np.sum(r * e2, 0)
    den = d11 * d22 - d12 * d12
    a = (d22 * r1 - d12 * r2) / den
    b = (d11 * r2 - d12 * r1) / den
    off_plane = np.linalg.norm(r - a * e1 - b * e2, axis=0)
    return a, b, off_plane


def test_face_points_on_faces_and_uniform():
    rng = np.random.default_rng(1)
    m, s_fc = 64, 2048
    tris = rng.uniform(-0.9, 0.9, size=(9, m)).astype(np.float32)
    face_uv, _ = synthetic.dataset_uniforms(m, s_fc, 1, 2)
    pts = dataset.face_points(tris, face_uv, s_fc)
    v0, v1, v2 = geometry.triangles_from_soup(tris)
    f = np.repeat(np.arange(m), s_fc)
    a, b, off = _barycentric(pts, v0[:, f], v1[:, f], v2[:, f])
    assert off.max() < 1e-12
    assert a.min() >= -1e-12 and b.min() >= -1e-12 and (a + b).max() <= 1 + 1e-12
    # uniform over the triangle: each of the four midpoint sub-triangles holds a quarter
    centre = (a > 0.5).astype(int) + 2 * (b > 0.5) + 3 * ((a <= 0.5) & (b <= 0.5) & (a + b > 0.5))
    frac = np.bincount(centre, minlength=4) / centre.size
    assert np.all(np.abs(frac - 0.25) < 0.01), frac
    # a face subrange gives the same points
    sub = dataset.face_points(tris, face_uv, s_fc, face_first=5, n_faces=3)
    np.testing.assert_array_equal(sub, pts[:, 5 * s_fc:8 * s_fc])


def test_direction_angles_closed_form():
    uv = np.array([[0.0, 0.5, 0.25], [0.0, 0.25, 0.75]])
    th0, th1 = dataset.direction_angles(uv)
    np.testing.assert_allclose(th0, [0.0, np.pi / 2, np.pi / 4])
    np.testing.assert_allclose(th1, [0.0, np.pi / 2, 1.5 * np.pi])
    d = geometry.dirs_from_angles(th0, th1)
    np.testing.assert_allclose(d[:, 0], [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(d[:, 1], [0, 1, 0], atol=1e-15)


def test_sample_angle_kinds_are_the_stated_directions():
    rng = np.random.default_rng(3)
    th0 = np.concatenate([rng.uniform(0, np.pi, 4000), [0.0, np.pi / 2, np.pi - 1e-9]])
    th1 = np.concatenate([rng.uniform(0, 2 * np.pi, 4000), [0.3, 6.0, 2 * np.pi - 1e-9]])
    d = geometry.dirs_from_angles(th0, th1)
    z = np.array([0.0, 0.0, 1.0])[:, None]
    for kind in range(4):
        theta, phi = dataset.sample_angles(th0, th1, kind)
        assert theta.min() >= 0 and theta.max() <= np.pi and phi.min() >= 0 and phi.max() < 2 * np.pi
        e = geometry.dirs_from_angles(theta, phi)
        if kind == 0:
            np.testing.assert_allclose(e, -d, atol=1e-12)
        elif kind == 1:
            np.testing.assert_allclose(e, d, atol=1e-12)
        else:
            # perpendicular to d, in the plane of d and the z axis, and the two kinds opposite
            assert np.abs(np.sum(e * d, 0)).max() < 1e-12
            assert np.abs(np.sum(e * np.cross(z, d, axis=0), 0)).max() < 1e-12
            # +pi/2 on the polar angle turns d towards -z (the polar angle grows)
            sgn = 1.0 if kind == 2 else -1.0
            dtheta = np.stack([np.cos(th0) * np.cos(th1), np.cos(th0) * np.sin(th1), -np.sin(th0)])
            np.testing.assert_allclose(e, sgn * dtheta, atol=1e-12)


def _quad(z0=0.1, half=0.5):
    v = np.array([[-half, -half, z0], [half, -half, z0], [half, half, z0], [-half, half, z0]])
    f = np.array([[0, 1, 2], [0, 2, 3]])
    return synthetic.tri_soup(v, f)


def test_quad_closed_form():
    """Every ray leaves a flat quad without meeting it again, so every pair is kept; the
    marching points and the perpendicular samples follow from plane geometry alone."""
    z0, half = 0.1, 0.5
    tris = _quad(z0, half)
    s_fc, s_dr, s_p = 3, 5, 4
    face_uv, dir_uv = synthetic.dataset_uniforms(2, s_fc, s_dr, 7)
    out = dataset.sample_dataset(tris, face_uv, dir_uv, s_fc, s_dr, s_p, eps=1e-4)
    P = 2 * s_fc * s_dr
    assert out["keep"].all() and out["keep"].size == P
    o, th0, th1, t_exit = out["origin"], out["theta0"], out["theta1"], out["t_exit"]
    np.testing.assert_allclose(o[2], z0, atol=1e-7)
    d = geometry.dirs_from_angles(th0, th1)
    # t_exit: the exit point lies on the cube's surface
    x = o + t_exit * d
    np.testing.assert_allclose(np.abs(x).max(axis=0), 1.0, atol=1e-12)
    # expected samples from plane geometry: the perpendicular ray from q meets the quad iff it
    # heads towards the plane and crosses it inside the square
    exp_count = 0
    rays, t, pair, kind = out["rays"], out["t"], out["pair"], out["kind"]
    col = 0
    for i in range(P):
        dp = np.array([np.cos(th0[i]) * np.cos(th1[i]), np.cos(th0[i]) * np.sin(th1[i]), -np.sin(th0[i])])
        for k in range(1, s_p + 1):
            q = o[:, i] + (k / s_p) * t_exit[i] * d[:, i]
            want = [(0, -d[:, i], k / s_p * t_exit[i]), (1, d[:, i], np.inf)]
            for kk, e in ((2, dp), (3, -dp)):
                s = (z0 - q[2]) / e[2] if e[2] != 0 else -1.0
                hit = s > 0 and np.all(np.abs((q + s * e)[:2]) <= half)
                if not hit:
                    want.append((kk, e, np.inf))
            for kk, e, tt in want:
                assert pair[col] == i and kind[col] == kk
                np.testing.assert_allclose(rays[:3, col], q, atol=1e-12)
                np.testing.assert_allclose(geometry.dirs_from_angles(rays[3, col], rays[4, col]), e, atol=1e-12)
                if np.isinf(tt):
                    assert np.isinf(t[col])
                else:
                    np.testing.assert_allclose(t[col], tt, rtol=1e-12)
                col += 1
            exp_count += len(want)
    assert col == exp_count == t.size


def test_convex_mesh_keeps_exactly_the_outward_rays():
    """On a closed convex mesh a ray from a face point leaves without a hit iff it points out
    of the face (and enters the solid, so meets another face, iff it points in)."""
    v, f = synthetic.icosphere(1, 0.8)
    tris = synthetic.tri_soup(v, f)
    m = f.shape[0]
    s_fc, s_dr = 2, 6
    face_uv, dir_uv = synthetic.dataset_uniforms(m, s_fc, s_dr, 11)
    out = dataset.sample_dataset(tris, face_uv, dir_uv, s_fc, s_dr, 2, eps=1e-5)
    n = geometry.face_normals(tris)
    centroid = synthetic.tri_soup(v, f).reshape(3, 3, -1).mean(axis=0)
    n = n * np.sign(np.sum(n * centroid, 0))               # outward (the sphere is centred at 0)
    face = np.arange(out["keep"].size) // (s_fc * s_dr)
    d = geometry.dirs_from_angles(out["theta0"], out["theta1"])
    cosn = np.sum(d * n[:, face], 0)
    clear = np.abs(cosn) > 1e-6
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(out["keep"][clear], cosn[clear] > 0)


def test_every_sample_is_a_correct_label():
    """Fig. 2b's labelling rules on a concave mesh: looking back from q the first surface is
    the face point at t_k (up to the offset eps), looking on along the ray or to either
    perpendicular side that was sampled, nothing is hit."""
    v, f = synthetic.torus(0.5, 0.2, 12, 8)
    tris = synthetic.tri_soup(v, f)
    m = f.shape[0]
    s_fc, s_dr, s_p, eps = 2, 4, 3, 1e-4
    face_uv, dir_uv = synthetic.dataset_uniforms(m, s_fc, s_dr, 5)
    out = dataset.sample_dataset(tris, face_uv, dir_uv, s_fc, s_dr, s_p, eps)
    keep = out["keep"]
    assert 0.2 < keep.mean() < 0.6                        # concave: outward rays are occluded too
    rays = out["rays"]
    d = geometry.dirs_from_angles(rays[3], rays[4])
    h = geometry.nearest_hit(rays[:3], d, tris)
    back = out["kind"] == 0
    ok = ~h["ambiguous"]
    np.testing.assert_allclose(h["t"][back & ok], out["t"][back & ok], atol=eps)
    assert np.all(h["tri"][~back & ok] < 0)
    assert ok.mean() > 0.99
    # sample count: two per marching step of a kept pair, plus the free perpendiculars
    assert out["t"].size == keep.sum() * s_p * 2 + out["perp_free"].sum()


def test_empty_inputs():
    tris = _quad()
    face_uv, dir_uv = synthetic.dataset_uniforms(2, 2, 2, 1)
    out = dataset.sample_dataset(tris, face_uv, dir_uv, 2, 2, 3, 1e-4, face_first=1, n_faces=0)
    assert out["rays"].shape == (5, 0) and out["t"].size == 0 and out["keep"].size == 0
