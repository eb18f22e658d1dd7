"""Statistical and structural checks of the seeded input generators."""
import numpy as np

import synthetic
from oracle import geometry, render


def test_ray_sets_shapes_and_ranges():
    o, d = synthetic.uniform_cube_rays(10000, 0)
    assert o.dtype == np.float32 and o.shape == (3, 10000) and d.shape == (3, 10000)
    assert np.all(np.abs(o) <= 1)
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=0), 1, atol=1e-6)
    assert np.all(np.abs(d.mean(axis=1)) < 0.03)
    o2, d2 = synthetic.uniform_cube_rays(10000, 0)
    assert np.array_equal(o, o2) and np.array_equal(d, d2)
    o, d = synthetic.unit_ball_rays(10000, 1)
    assert np.all(np.linalg.norm(o.astype(np.float64), axis=0) <= 1 + 1e-6)


def test_area_weighted_face_frequencies_chi2():
    v, f = synthetic.icosphere(1, 0.8)
    v = v * np.array([1.0, 0.5, 2.0])         # unequal areas
    rng = np.random.default_rng(0)
    n = 200000
    _, tri = synthetic.area_weighted_surface_points(v, f, n, rng)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    expect = n * area / area.sum()
    obs = np.bincount(tri, minlength=len(f))
    chi2 = ((obs - expect) ** 2 / expect).sum()
    dof = len(f) - 1
    assert chi2 < dof + 5 * np.sqrt(2 * dof)


def test_training_rays_surface_anchored_hit_the_mesh():
    v, f = synthetic.icosphere(2, 0.8)
    tris = synthetic.tri_soup(v, f)
    o, d, anchored = synthetic.training_rays(v, f, 4000, 1)
    assert anchored[:2000].all() and not anchored[2000:].any()
    r = geometry.nearest_hit(o[:, :2000], d[:, :2000], tris)
    ok = ~r["ambiguous"]
    assert (r["tri"][ok] >= 0).mean() > 0.999
    assert np.all(np.abs(o) <= 1)


def test_training_mesh_size_and_disjoint_parts():
    v, f = synthetic.training_mesh(1)
    assert f.shape == (20480, 3)
    assert np.abs(v).max() < 1.0
    # uniform rays from far outside the parts see an even crossing count (closed, disjoint parts)
    tris = synthetic.tri_soup(v, f)
    o = np.tile(np.array([[0.0], [0.0], [5.0]]), (1, 64)).astype(np.float32)
    rng = np.random.default_rng(2)
    tgt = rng.uniform(-0.5, 0.5, size=(3, 64))
    d = (tgt - o).astype(np.float64)
    d /= np.linalg.norm(d, axis=0)
    r = geometry.nearest_hit(o, d.astype(np.float32), tris)
    ok = ~r["ambiguous"]
    assert np.all(r["crossings"][ok] % 2 == 0)


def test_render_oracle_network_backend_runs():
    p = synthetic.random_params(32, 2, 0)
    cfg = synthetic.RenderConfig(12, 10, 2, 3, 1, 5)
    out = render.render(render.NetworkScene(p, 32, 2), cfg)
    assert out["radiance"].shape == (3, 10, 12)
    assert np.all(np.isfinite(out["radiance"])) and np.all(out["radiance"] >= 0)
    assert out["active"][0] == 240


def test_render_rays_mix():
    """Cube-entry rays start on the cube's surface and point into it; surface-leaving rays start
    1e-3 off a face of the mesh and leave to that side; all directions are unit; the draw is
    fixed by the seed."""
    v, f = synthetic.icosphere(2, 0.8)
    n = 3000
    o, d = synthetic.render_rays(v, f, n, 5)
    o2, d2 = synthetic.render_rays(v, f, n, 5)
    np.testing.assert_array_equal(o, o2)
    np.testing.assert_array_equal(d, d2)
    assert o.shape == d.shape == (3, n) and o.dtype == np.float32
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=0), 1.0, atol=1e-6)
    c = n // 3
    oc, dc = o[:, :c].astype(np.float64), d[:, :c].astype(np.float64)
    k = np.argmax(np.abs(oc), axis=0)
    face = oc[k, np.arange(c)]
    assert np.all(np.abs(face) == 1.0)
    assert np.all(dc[k, np.arange(c)] * face <= 0)   # into the cube
    # surface-leaving rays of a mesh of one triangle in the plane z = 0: the origin is 1e-3 off
    # the plane, over the triangle, and the direction leaves to the origin's side
    tv = np.array([[-0.5, -0.5, 0.0], [0.5, -0.5, 0.0], [0.0, 0.5, 0.0]])
    o, d = synthetic.render_rays(tv, np.array([[0, 1, 2]]), n, 6)
    ob, db = o[:, c:2 * c].astype(np.float64), d[:, c:2 * c].astype(np.float64)
    np.testing.assert_allclose(np.abs(ob[2]), 1e-3, rtol=1e-4)
    assert np.all(ob[2] * db[2] >= 0)
    assert 0.4 < np.mean(ob[2] > 0) < 0.6   # both sides
    assert np.all((ob[1] >= -0.5) & (ob[1] <= 0.5) & (np.abs(ob[0]) <= 0.5))
