"""GPU parity of ddf_udf (Eq. 5: the minimum of the field over a direction set) against the UDF
oracle evaluated through the float64 network (float32 networks) or the bf16 emulation."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import udf
from paper_2306_16142_amd import api

from gpu_common import banner, cuda, host

pytestmark = pytest.mark.gpu


def _inputs(n_points, n_dirs, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.95, 0.95, size=(3, n_points)).astype(np.float32)
    _, d = synthetic.uniform_cube_rays(n_dirs, seed + 1)
    return x, d


def _check(u, a, ref_u, ref_a, D, rtol):
    """u, a: GPU udf and argmin; ref_*: oracle; D [n, d]: the oracle's masked distances."""
    fin = np.isfinite(ref_u)
    np.testing.assert_array_equal(np.isfinite(u), fin)
    np.testing.assert_array_equal(a[~fin], -1)
    scale = np.maximum(1.0, np.abs(ref_u[fin]))
    assert np.all(np.abs(u[fin] - ref_u[fin]) <= rtol * scale)
    # the argument: the oracle's own, or a direction the oracle puts within the tolerance
    rows = np.flatnonzero(fin)
    other = a[rows] != ref_a[rows]
    if other.any():
        r = rows[other]
        assert np.all(D[r, a[r]] - ref_u[r] <= 2 * rtol * np.maximum(1.0, np.abs(ref_u[r])))


@pytest.mark.parametrize("width,depth,n_points,n_dirs", [(128, 2, 301, 77), (256, 3, 65, 130), (128, 4, 5, 1)])
def test_udf_fp32_matches_float64(width, depth, n_points, n_dirs):
    banner("udf fp32: %dx%d, %d points x %d dirs" % (depth, width, n_points, n_dirs))
    p = synthetic.random_params(width, depth, 31)
    x, d = _inputs(n_points, n_dirs, 32)
    net = api.Network(cuda(p), width, depth, "fp32")
    u, a = api.udf(net, cuda(x), cuda(d))
    u, a = host(u), host(a)
    field = udf.network_field(p, width, depth)
    ref_u, ref_a = udf.udf(field, x, d)
    hit, dist = field(udf.query_grid(x, d))
    D = np.where(hit, dist, np.inf).reshape(n_points, n_dirs)
    _check(u, a, ref_u, ref_a, D, 2e-5)


@pytest.mark.parametrize("width,depth", [(128, 4), (256, 6)])
def test_udf_bf16_matches_emulation(width, depth):
    """The LDS-resident kernel (128 x 4) and the streamed one (256 x 6): away from ReLU and
    logit sign flips the kernel and the bf16 emulation agree to a few bf16 ulps."""
    banner("udf bf16: %dx%d, 200 points x 96 dirs" % (depth, width))
    p = synthetic.random_params(width, depth, 33)
    x, d = _inputs(200, 96, 34)
    net = api.Network(cuda(p), width, depth, "bf16")
    u, a = api.udf(net, cuda(x), cuda(d))
    u, a = host(u), host(a)
    field = udf.network_field(p, width, depth, "bf16")
    ref_u, ref_a = udf.udf(field, x, d)
    fin = np.isfinite(ref_u) & np.isfinite(u)
    assert np.mean(np.isfinite(ref_u) == np.isfinite(u)) >= 0.99
    err = np.abs(u[fin] - ref_u[fin]) / np.maximum(1.0, np.abs(ref_u[fin]))
    assert np.quantile(err, 0.99) < 2e-2 and np.median(err) < 2e-3
    # where the argument agrees the minimum is the same query, so the gap is one query's error
    same = fin & (a == ref_a)
    assert same.mean() > 0.9
    assert np.median(np.abs(u[same] - ref_u[same])) < 2e-3


def test_udf_chunks_and_edges():
    banner("udf: workspace chunking (fp32, unfused), no directions, no points")
    width, depth = 128, 2
    p = synthetic.random_params(width, depth, 35)
    x, d = _inputs(37, 50, 36)
    net = api.Network(cuda(p), width, depth, "fp32")
    xg, dg = cuda(x), cuda(d)
    u1, a1 = [t.clone() for t in api.udf(net, xg, dg)]
    # a workspace for five points' queries: eight chunks, bit-identical results
    ws = torch.empty(512 + 768 + 5 * 28 * 50, device="cuda", dtype=torch.uint8)   # angles, alignment, 5 points
    u2, a2 = api.udf(net, xg, dg, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2) and torch.equal(a1, a2)
    # no directions: +inf and -1 everywhere; no points: nothing (fused and unfused networks)
    for prec in ("fp32", "bf16"):
        net = api.Network(cuda(p), width, depth, prec)
        u3, a3 = api.udf(net, xg, torch.empty((3, 0), device="cuda"))
        torch.cuda.synchronize()
        assert torch.isinf(u3).all() and (a3 == -1).all()
        u4, _ = api.udf(net, torch.empty((3, 0), device="cuda"), dg)
        assert u4.numel() == 0


@pytest.mark.parametrize("prec,n_points,n_dirs", [("bf16", 333, 70), ("bf16", 50, 7), ("fp8", 129, 96)])
def test_udf_fused_equals_forward_then_minimum(prec, n_points, n_dirs):
    """4 x 128 bf16 / fp8 networks take the fused kernel (grid, network and minimum in one
    launch); its answer equals, bit for bit, the minimum over ddf_forward's outputs for the
    same grid assembled by ddf_assemble_rays (the same angle code), ties to the lowest index."""
    banner("udf fused %s: %d points x %d dirs" % (prec, n_points, n_dirs))
    width, depth = 128, 4
    p = synthetic.random_params(width, depth, 41)
    x, d = _inputs(n_points, n_dirs, 42)
    pg, xg, dg = cuda(p), cuda(x), cuda(d)
    if prec == "fp8":
        co, cd = synthetic.uniform_cube_rays(1 << 14, 4)
        calib = api.assemble_rays(cuda(co), cuda(cd))
        net = api.Network(pg, width, depth, "fp8",
                          scales=api.fp8_scales(pg, width, depth, calib, api.Network(pg, width, depth, "fp32")))
    else:
        net = api.Network(pg, width, depth, prec)
    u, a = api.udf(net, xg, dg)
    og = xg.repeat_interleave(n_dirs, dim=1).contiguous()
    og_d = dg.repeat(1, n_points).contiguous()
    lg, ds = net(api.assemble_rays(og, og_d))
    torch.cuda.synchronize()
    L, Dd = lg.view(n_points, n_dirs), ds.view(n_points, n_dirs)
    masked = torch.where((L > 0) & (Dd < float("inf")), Dd, torch.full_like(Dd, float("inf")))
    ref_u = masked.min(dim=1).values
    ref_a = torch.where(torch.isinf(ref_u), torch.full_like(ref_u, -1, dtype=torch.int64),
                        masked.argmin(dim=1)).to(torch.int32)
    assert torch.isfinite(ref_u).float().mean() > 0.3
    assert torch.equal(u, ref_u) and torch.equal(a, ref_a)


def test_udf_full_size_sampled():
    """32^3 grid points x 512 directions through the 4 x 128 bf16 network (the benchmark's UDF
    workload): 64 sampled points against the emulation."""
    banner("udf: 32^3 grid x 512 dirs, bf16 4x128, 64 sampled points")
    width, depth = 128, 4
    p = synthetic.random_params(width, depth, 37)
    x = synthetic.grid_points(32)
    _, d = synthetic.uniform_cube_rays(512, 38)
    net = api.Network(cuda(p), width, depth, "bf16")
    u, a = api.udf(net, cuda(x), cuda(d))
    u, a = host(u), host(a)
    idx = np.random.default_rng(39).choice(x.shape[1], 64, replace=False)
    ref_u, ref_a = udf.udf(udf.network_field(p, width, depth, "bf16"), x[:, idx], d)
    fin = np.isfinite(ref_u) & np.isfinite(u[idx])
    assert np.mean(np.isfinite(ref_u) == np.isfinite(u[idx])) >= 0.95
    err = np.abs(u[idx][fin] - ref_u[fin]) / np.maximum(1.0, np.abs(ref_u[fin]))
    assert np.median(err) < 2e-3


def test_udf_nan_points_are_misses():
    """A point with a NaN coordinate gives NaN network outputs, which no direction counts as a
    hit: +inf and -1, on the fused (bf16) and the unfused (fp32) path alike."""
    banner("udf: NaN points")
    p = synthetic.random_params(128, 2, 43)
    x, d = _inputs(70, 40, 44)
    x[1, 5] = np.nan
    x[0, 66] = np.nan
    for prec in ("bf16", "fp32"):
        net = api.Network(cuda(p), 128, 2, prec)
        u, a = api.udf(net, cuda(x), cuda(d))
        u, a = host(u), host(a)
        assert np.isinf(u[[5, 66]]).all() and (a[[5, 66]] == -1).all()
        ok = np.ones(70, bool)
        ok[[5, 66]] = False
        ref_u, _ = udf.udf(udf.network_field(p, 128, 2, "bf16" if prec == "bf16" else "fp64"), x[:, ok], d)
        assert np.mean(np.isfinite(u[ok]) == np.isfinite(ref_u)) >= 0.95


def test_sampler_and_udf_graph_replay_matches_eager():
    """ddf_sample_dataset and the fused ddf_udf captured into one HIP graph: every replay, with
    eager work and synchronisations between replays, equals the eager results bit for bit
    (no host synchronisation and no memset inside either call)."""
    banner("graph replay: dataset sampler (icosphere 80 tris) + fused udf (bf16 4x128)")
    v, f = synthetic.icosphere(1, 0.8)
    tris = cuda(synthetic.tri_soup(v, f))
    fu, du = [cuda(a) for a in synthetic.dataset_uniforms(f.shape[0], 2, 4, 45)]
    sampler = api.DatasetSampler(tris, 2, 4, 3, 1e-4)
    p = synthetic.random_params(128, 4, 46)
    net = api.Network(cuda(p), 128, 4, "bf16")
    x, d = _inputs(300, 64, 47)
    xg, dg = cuda(x), cuda(d)
    ws = torch.empty(api.udf_workspace_bytes(300, 64), device="cuda", dtype=torch.uint8)
    u = torch.empty(300, device="cuda")
    a = torch.empty(300, device="cuda", dtype=torch.int32)

    def work():
        sampler.run(fu, du)
        api.udf(net, xg, dg, out=u, arg=a, workspace=ws)

    work()   # eager, also keeps one-time launch setup outside the capture
    torch.cuda.synchronize()
    n = int(sampler.count.item())
    ref = [sampler.rays[:, :n].clone(), sampler.t[:n].clone(), sampler.pair[:n].clone(), u.clone(), a.clone()]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        work()
    torch.cuda.synchronize()
    for rep in range(3):
        sampler.rays.fill_(-1.0)
        u.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(sampler.count.item()) == n
        got = [sampler.rays[:, :n], sampler.t[:n], sampler.pair[:n], u, a]
        for r_, g_ in zip(ref, got):
            assert torch.equal(r_, g_), rep
        work()   # eager work between replays
        torch.cuda.synchronize()
