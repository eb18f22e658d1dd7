"""Pins of the render oracle: published SplitMix64 outputs, sampling invariants, and the
closed-form single-bounce image of a lit quad (ray/plane intersection, no triangle test)."""
import json
import os

import numpy as np

import synthetic
from oracle import render

from conftest import GOLDEN


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    for s in g["streams"]:
        out = render.splitmix64_stream(s["seed"], len(s.get("outputs_hex", s.get("outputs", []))))
        if "outputs_hex" in s:
            assert [int(x, 16) for x in s["outputs_hex"]] == out
        else:
            assert s["outputs"] == out


def test_counter_uniforms_vectorised_equal_scalar():
    pix = np.arange(50, dtype=np.int64)
    smp = (pix * 7) % 5
    keys = render.path_keys(9, pix, smp)
    u = render.uniform(keys, 2, 3)
    for i in range(50):
        assert u[i] == render.uniform_scalar(9, int(pix[i]), int(smp[i]), 2, 3)
    # exact multiples of 2^-24 in [0, 1)
    big = render.uniform(render.path_keys(1, np.arange(100000), np.zeros(100000, np.int64)), 0, 0)
    assert np.all((big >= 0) & (big < 1))
    assert np.all(big * 2 ** 24 == np.floor(big * 2 ** 24))
    assert abs(big.mean() - 0.5) < 0.005


def test_onb_and_cosine_sampling():
    rng = np.random.default_rng(0)
    n = rng.normal(size=(3, 20000))
    n /= np.linalg.norm(n, axis=0)
    b1, b2 = render.onb_duff(n)
    for a, b in [(b1, b2), (b1, n), (b2, n)]:
        np.testing.assert_allclose(np.sum(a * b, axis=0), 0, atol=1e-12)
    for a in (b1, b2):
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 1, rtol=1e-12)
    # right-handed: b1 x b2 = n
    np.testing.assert_allclose(np.cross(b1, b2, axis=0), n, atol=1e-12)
    # Malley's method: E[cos] = 2/3 for cosine-weighted directions
    u1, u2 = rng.random(200000), rng.random(200000)
    lz = np.sqrt(1 - u1)
    assert abs(lz.mean() - 2.0 / 3.0) < 0.003


def test_camera_rays_field_of_view():
    cfg = synthetic.small_render()
    W, H = cfg.width, cfg.height
    pix = np.array([0, W - 1, (H - 1) * W, H * W - 1], dtype=np.int64)
    o, d = render.camera_rays(cfg, pix, np.zeros(4, np.int64), None)
    f = -np.asarray(cfg.camera.eye) / np.linalg.norm(cfg.camera.eye)
    th = np.tan(np.radians(cfg.camera.vfov_deg) / 2)
    # corner pixel centres sit at (1 - 1/W) and (1 - 1/H) of the half extents
    expect = 1.0 / np.sqrt(1 + (th * (1 - 1 / H)) ** 2 + (th * (1 - 1 / W) * W / H) ** 2)
    np.testing.assert_allclose(f @ d, expect, rtol=1e-12)
    assert np.all(o == np.asarray(cfg.camera.eye)[:, None])


def test_single_bounce_quad_closed_form():
    """One bounce, one sample: every pixel is (albedo / pi) I cos / r^2 at the ray/plane hit."""
    big = 50.0
    v = np.array([[-big, -big, 0], [big, -big, 0], [big, big, 0], [-big, big, 0]], dtype=np.float64)
    tris = synthetic.tri_soup(v, np.array([[0, 1, 2], [0, 2, 3]]))
    cfg = synthetic.RenderConfig(24, 16, 1, 1, 3, 0)
    cfg.camera.eye = (0.0, -3.0, 2.0)
    out = render.render(render.MeshScene(tris), cfg)
    P = cfg.width * cfg.height
    o, d = render.camera_rays(cfg, np.arange(P), np.zeros(P, np.int64), None)
    t = -o[2] / d[2]
    hit = t > 0
    x = o + t * d
    xs = x + cfg.eps * np.array([0, 0, 1.0])[:, None]
    lv = np.asarray(cfg.light.position)[:, None] - xs
    r2 = np.sum(lv * lv, axis=0)
    cos = lv[2] / np.sqrt(r2)
    expect = np.where(hit, 0.7 / np.pi * 10.0 * np.maximum(cos, 0) / r2, 0.0).reshape(cfg.height, cfg.width)
    ok = out["robust"]
    assert ok.mean() > 0.95
    for c in range(3):
        np.testing.assert_allclose(out["radiance"][c][ok], expect[ok], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["depth"][ok & hit.reshape(ok.shape)], t.reshape(ok.shape)[ok & hit.reshape(ok.shape)], rtol=1e-12)
    nz = out["normal"][2][ok & hit.reshape(ok.shape)]
    np.testing.assert_allclose(nz, 1.0)


def test_shadowed_quad_is_dark_under_occluder():
    """A small quad between the light and the floor casts a shadow: the NEE term vanishes there."""
    big = 50.0
    floor = np.array([[-big, -big, 0], [big, -big, 0], [big, big, 0], [-big, big, 0]], dtype=np.float64)
    light = np.array([0.0, 0.0, 3.0])
    occ = np.array([[-0.3, -0.3, 1.5], [0.3, -0.3, 1.5], [0.3, 0.3, 1.5], [-0.3, 0.3, 1.5]])
    v = np.concatenate([floor, occ])
    f = np.array([[0, 1, 2], [0, 2, 3], [4, 5, 6], [4, 6, 7]])
    cfg = synthetic.RenderConfig(32, 32, 1, 1, 3, 0)
    cfg.camera.eye = (0.0, -0.01, 6.0)
    cfg.camera.vfov_deg = 30.0
    cfg.light.position = tuple(light)
    out = render.render(render.MeshScene(synthetic.tri_soup(v, f)), cfg)
    P = cfg.width * cfg.height
    o, d = render.camera_rays(cfg, np.arange(P), np.zeros(P, np.int64), None)
    # floor points whose segment to the light crosses the occluder (the occluder hides some pixels too)
    tf = -o[2] / d[2]
    x = o + tf * d
    s = (1.5 - x[2]) / (light[2] - x[2])
    y = x + s * (light[:, None] - x)
    shadow = (np.abs(y[0]) < 0.3) & (np.abs(y[1]) < 0.3)
    to = (1.5 - o[2]) / d[2]
    xo = o + to * d
    sees_occluder = (np.abs(xo[0]) <= 0.3) & (np.abs(xo[1]) <= 0.3)
    sel = (shadow & ~sees_occluder).reshape(32, 32) & out["robust"]
    assert sel.sum() > 5
    assert np.all(out["radiance"][0][sel] == 0.0)
    lit = (~shadow & ~sees_occluder).reshape(32, 32) & out["robust"]
    assert np.all(out["radiance"][0][lit] > 0.0)


def _hitting(width, depth, seed):
    p = synthetic.random_params(width, depth, seed, bias_scale=0.3)
    p[-2], p[-1] = 0.5, 1.0
    return p


def test_multi_single_identity_instance_equals_network_scene():
    from oracle import multi
    p = _hitting(32, 2, 3)
    cfg = synthetic.RenderConfig(16, 12, 2, 3, 1, 4)
    a = render.render(render.NetworkScene(p, 32, 2), cfg)
    b = render.render(multi.MultiScene([(p, 32, 2)], [{"R": np.eye(3), "T": np.zeros(3), "net": 0}]), cfg)
    ok = a["robust"] & b["robust"]
    assert ok.mean() > 0.8
    # the multi scene treats negative predicted distances as misses; compare where both agree
    np.testing.assert_allclose(a["radiance"][:, ok], b["radiance"][:, ok], rtol=1e-12, atol=1e-15)


def _moved_render(nets, inst, M, c, bounces):
    from oracle import multi
    cfg = synthetic.RenderConfig(20, 14, 1, bounces, 3, 2)
    cfg.camera.eye = (0.0, -6.0, 1.0)
    a = render.render(multi.MultiScene(nets, inst), cfg)
    inst2 = [{"R": M @ d["R"], "T": M @ d["T"] + c, "net": d["net"]} for d in inst]
    cfg2 = synthetic.RenderConfig(20, 14, 1, bounces, 3, 2)
    cfg2.camera.eye = tuple(M @ np.array(cfg.camera.eye) + c)
    cfg2.camera.target = tuple(M @ np.array(cfg.camera.target) + c)
    cfg2.camera.up = tuple(M @ np.array(cfg.camera.up))
    cfg2.light.position = tuple(M @ np.array(cfg.light.position) + c)
    b = render.render(multi.MultiScene(nets, inst2), cfg2)
    ok = a["robust"] & b["robust"]
    assert ok.mean() > 0.8 and np.isfinite(a["depth"]).mean() > 0.1
    np.testing.assert_allclose(a["radiance"][:, ok], b["radiance"][:, ok], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(a["depth"][ok], b["depth"][ok], rtol=1e-9)


def test_multi_rigid_motion_of_the_whole_scene_leaves_the_image_unchanged():
    """Direct lighting is invariant under any rigid motion of scene + camera + light; with more
    bounces only under translations (the scatter basis of Duff et al. is tied to world z)."""
    nets = [(_hitting(32, 2, 5), 32, 2), (_hitting(32, 3, 6), 32, 3)]
    r0 = np.array([0.1, 0.3, -0.2, 0.9])
    inst = [{"R": synthetic.scenes._rotation_from_quaternion(r0 / np.linalg.norm(r0)), "T": np.array([-1.2, 0.3, 0.1]),
             "net": 0},
            {"R": np.eye(3), "T": np.array([1.3, -0.2, 0.0]), "net": 1}]
    q = np.array([0.2, -0.4, 0.3, 0.8])
    M = synthetic.scenes._rotation_from_quaternion(q / np.linalg.norm(q))
    _moved_render(nets, inst, M, np.array([0.5, -1.0, 2.0]), 1)
    _moved_render(nets, inst, np.eye(3), np.array([0.5, -1.0, 2.0]), 3)


def test_pixel_subset_equals_whole_frame():
    """Tracing only listed pixels gives those pixels' values of the whole frame bit for bit
    (paths are independent and every random number is keyed by pixel and sample), with
    jitter, several bounces and Russian roulette."""
    v, f = synthetic.icosphere(1, 0.8)
    cfg = synthetic.RenderConfig(20, 14, 3, 4, 1, 5)
    scene = render.MeshScene(synthetic.tri_soup(v, f))
    whole = render.render(scene, cfg)
    pix = np.array([279, 0, 141, 150, 151, 37, 200, 141])   # any order, repeats allowed
    part = render.render(scene, cfg, pixels=pix)
    r, c = pix // cfg.width, pix % cfg.width
    np.testing.assert_array_equal(part["radiance"], whole["radiance"][:, r, c])
    np.testing.assert_array_equal(part["depth"], whole["depth"][r, c])
    np.testing.assert_array_equal(part["normal"], whole["normal"][:, r, c])
    np.testing.assert_array_equal(part["robust"], whole["robust"][r, c])
    assert whole["radiance"][:, r, c].max() > 0 and np.isfinite(whole["depth"][r, c]).any()


def test_shadow_ray_counts():
    """Shadow rays are traced exactly for hits whose normal faces the light: with the light at
    the centre of the closed convex icosphere every outward normal faces away from it (no
    shadow rays, a black image), with the light outside some hits face it; a split of the
    pixels into two sets splits both counts."""
    from synthetic.scenes import Light
    v, f = synthetic.icosphere(1, 0.8)
    scene = render.MeshScene(synthetic.tri_soup(v, f))
    cfg = synthetic.RenderConfig(16, 12, 2, 3, 1, 2)
    out = render.render(scene, cfg)
    assert out["shadow"][0] > 0 and all(s <= a for s, a in zip(out["shadow"], out["active"]))
    inside = synthetic.RenderConfig(16, 12, 2, 3, 1, 2, light=Light(position=(0.0, 0.0, 0.0)))
    dark = render.render(scene, inside)
    assert dark["active"][0] == 16 * 12 * 2 and dark["active"][1] > 0
    assert sum(dark["shadow"]) == 0 and dark["radiance"].max() == 0
    pix = np.arange(16 * 12)
    a, b = render.render(scene, cfg, pixels=pix[::2]), render.render(scene, cfg, pixels=pix[1::2])
    pad = lambda c: c + [0] * (cfg.bounces - len(c))
    assert [x + y for x, y in zip(pad(a["shadow"]), pad(b["shadow"]))] == pad(out["shadow"])
    assert [x + y for x, y in zip(pad(a["active"]), pad(b["active"]))] == pad(out["active"])


def test_hit_counts():
    """Hits per bounce: at bounce 0 exactly the camera rays that the brute-force labeller finds
    hitting the mesh; a bounce ray leaves a closed convex object through the hemisphere of its
    outward normal, so with the light inside the icosphere (no shadow rays) nothing is hit
    again; every continuing path was a hit, and before Russian roulette every hit continues;
    a split of the pixels splits the counts."""
    from synthetic.scenes import Light
    from oracle import geometry
    v, f = synthetic.icosphere(1, 0.8)
    tris = synthetic.tri_soup(v, f)
    scene = render.MeshScene(tris)
    cfg = synthetic.RenderConfig(16, 12, 2, 3, 1, 2)
    out = render.render(scene, cfg)
    P = 16 * 12 * 2
    pid = np.arange(P)
    pixel, sample = pid // 2, pid % 2
    o, d = render.camera_rays(cfg, pixel, sample, render.path_keys(cfg.seed, pixel, sample))
    assert out["hits"][0] == int((geometry.nearest_hit(o, d, tris)["tri"] >= 0).sum()) > 0
    pad = lambda c: c + [0] * (cfg.bounces - len(c))
    hits, active, shadow = pad(out["hits"]), pad(out["active"]), pad(out["shadow"])
    assert all(s <= h <= a for s, h, a in zip(shadow, hits, active))
    assert all(active[b + 1] <= hits[b] for b in range(cfg.bounces - 1))
    assert active[1] == hits[0]   # Russian roulette starts after bounce 1
    inside = synthetic.RenderConfig(16, 12, 2, 3, 1, 2, light=Light(position=(0.0, 0.0, 0.0)))
    dark = render.render(scene, inside)
    assert dark["hits"][0] == out["hits"][0] and sum(pad(dark["hits"])[1:]) == 0
    pix = np.arange(16 * 12)
    a, b = render.render(scene, cfg, pixels=pix[::2]), render.render(scene, cfg, pixels=pix[1::2])
    assert [x + y for x, y in zip(pad(a["hits"]), pad(b["hits"]))] == hits


def test_queried_rays_of_a_network_scene():
    """A network scene queries only the rays that enter the domain cube: at bounce 0 the count
    lies between brute-force counts of camera rays that pass through a slightly smaller and a
    slightly larger cube (points sampled along each ray, no slab test); the mesh scene traces
    every path; no count exceeds the paths of its bounce."""
    p = _hitting(32, 2, 11)
    cfg = synthetic.RenderConfig(20, 14, 2, 3, 1, 5)
    cfg.camera.eye = (0.3, -4.5, 1.2)   # the cube fills part of the view
    out = render.render(render.NetworkScene(p, 32, 2), cfg)
    P = 20 * 14 * 2
    pid = np.arange(P)
    o, d = render.camera_rays(cfg, pid // 2, pid % 2, render.path_keys(cfg.seed, pid // 2, pid % 2))
    t = np.linspace(0.0, 9.0, 9001)
    pts = o[:, :, None] + d[:, :, None] * t[None, None, :]
    inner = int(np.any(np.all(np.abs(pts) <= 1.0 - 2e-3, axis=0), axis=1).sum())
    outer = int(np.any(np.all(np.abs(pts) <= 1.0 + 2e-3, axis=0), axis=1).sum())
    assert 0 < inner <= out["queried"][0] <= outer < P
    assert all(qn <= a for qn, a in zip(out["queried"], out["active"]))
    v, f = synthetic.icosphere(1, 0.8)
    mesh = render.render(render.MeshScene(synthetic.tri_soup(v, f)), cfg)
    assert mesh["queried"] == mesh["active"]
