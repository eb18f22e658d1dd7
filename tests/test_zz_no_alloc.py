"""The allocation-free UDF entry point (ddf_udf_noalloc, scratch in a fixed device array)
against ddf_udf with a caller workspace: bit-identical results on two calls in a row, the
second smaller, for the fused form (a bf16 network held in LDS), the chunked form (a float32
network), and a point count beyond the fused form's key capacity."""
import ctypes

import numpy as np
import pytest
import torch

import synthetic
from paper_2306_16142_amd import _lib, api

from gpu_common import banner, cuda

pytestmark = pytest.mark.gpu


def _noalloc(net, points, dirs):
    n, d = points.shape[1], dirs.shape[1]
    out = torch.full((n,), 7.0, device="cuda")
    arg = torch.full((n,), -7, device="cuda", dtype=torch.int32)
    _lib.call("ddf_udf_noalloc", ctypes.byref(net.desc), ctypes.c_void_p(points.data_ptr()), n,
              ctypes.c_void_p(dirs.data_ptr()), d, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(arg.data_ptr()),
              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return out, arg


@pytest.mark.parametrize("width,depth,prec,sizes", [
    (128, 4, "bf16", [(3000, 257), (1000, 64)]),          # fused: keys of all points fit
    (256, 2, "fp32", [(700, 300), (150, 33)]),             # chunks of points through ddf_forward
    (128, 2, "bf16", [((1 << 20) + 3000, 5), (10, 4)]),    # beyond the keys' capacity: chunked
])
def test_udf_noalloc_equals_udf(width, depth, prec, sizes):
    p = synthetic.random_params(width, depth, 61, bias_scale=0.3)
    p[-2], p[-1] = 0.3, 0.5   # logit and distance biases: plenty of hits
    net = api.Network(cuda(p), width, depth, prec)
    for call, (n, d) in enumerate(sizes):
        banner("udf noalloc %dx%d %s call %d: %d points x %d directions" % (depth, width, prec, call, n, d))
        rng = np.random.default_rng(62 + call)
        pts = cuda(rng.uniform(-0.9, 0.9, size=(3, n)).astype(np.float32))
        _, dirs_np = synthetic.uniform_cube_rays(d, 63 + call)
        dirs = cuda(dirs_np)
        ref, ref_arg = api.udf(net, pts, dirs)
        out, arg = _noalloc(net, pts, dirs)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(arg, ref_arg)
        assert torch.isfinite(ref).float().mean() > 0.25 and (ref_arg >= 0).float().mean() > 0.25


def test_udf_noalloc_rejects_too_many_directions():
    banner("udf noalloc: direction count beyond the scratch")
    p = synthetic.random_params(128, 2, 64)
    net = api.Network(cuda(p), 128, 2, "bf16")
    pts = torch.zeros((3, 4), device="cuda")
    dirs = torch.zeros((3, 65537), device="cuda")
    dirs[2] = 1.0
    with pytest.raises(_lib.DdfError) as e:
        _noalloc(net, pts, dirs)
    assert e.value.status == _lib.DDF_ERR_UNSUPPORTED and "65536" in str(e.value)
