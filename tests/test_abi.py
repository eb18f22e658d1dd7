"""C-ABI checks that run without a GPU: the library loads, exports every entry point that
include/ddf.h declares, and validates arguments before touching the device."""
import ctypes
import math
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ddf.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ddf_status|int32_t|const char \*)\s*(ddf_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_16142_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libddf.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_hot_path():
    names = _declared()
    for required in ("ddf_label_rays", "ddf_forward", "ddf_backward", "ddf_render_wavefront", "ddf_pack_net",
                     "ddf_train_step", "ddf_train_step_chunked", "ddf_assemble_rays", "ddf_query",
                     "ddf_set_tuning", "ddf_sample_dataset", "ddf_dataset_workspace_size", "ddf_udf", "ddf_udf_workspace_size", "ddf_loss_seeds_ex", "ddf_train_step_ex", "ddf_train_step_eikonal", "ddf_eikonal_workspace_size"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2306_16142_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, "binding lacks " + name


def test_version_and_error_string(lib):
    assert lib.ddf_abi_version() == 1
    assert isinstance(lib.ddf_last_error(), bytes)


def test_validation_before_launch(lib):
    from paper_2306_16142_amd import _lib
    # NULL arrays with n > 0, negative sizes, empty windows: rejected with a message
    assert lib.ddf_label_rays(None, None, 5, None, 3, 0.0, 1.0, None, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    assert b"NULL" in lib.ddf_last_error()
    assert lib.ddf_label_rays(None, None, -1, None, 3, 0.0, 1.0, None, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_label_rays(None, None, 5, None, 3, 1.0, 1.0, None, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_label_rays(None, None, 5, None, 3, 0.0, math.nan, None, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    # n == 0 is a no-op even with NULL arrays
    assert lib.ddf_label_rays(None, None, 0, None, 3, 0.0, 1.0, None, None, None, None) == _lib.DDF_OK
    assert lib.ddf_assemble_rays(None, None, 0, None, None) == _lib.DDF_OK
    assert lib.ddf_assemble_rays(None, None, 4, None, None) == _lib.DDF_ERR_INVALID_ARG
    # unsupported shapes and precisions
    b = ctypes.c_size_t(0)
    assert lib.ddf_packed_bytes(96, 4, 1, ctypes.byref(b)) == _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_packed_bytes(128, 9, 1, ctypes.byref(b)) == _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_packed_bytes(128, 4, 7, ctypes.byref(b)) == _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_packed_bytes(128, 4, 1, ctypes.byref(b)) == _lib.DDF_OK and b.value > 0
    net = _lib.DdfNet(128, 4, 1, None)
    assert lib.ddf_forward(ctypes.byref(net), None, 10, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_forward(None, None, 10, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    # fused query: NULL arrays rejected, n == 0 a no-op, networks beyond LDS or fp32 refused
    assert lib.ddf_query(ctypes.byref(net), None, None, 10, None, None, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_query(ctypes.byref(net), None, None, 0, None, None, None) == _lib.DDF_OK
    wide = _lib.DdfNet(256, 4, 1, 1)
    assert lib.ddf_query(ctypes.byref(wide), 1, 1, 10, 1, 1, None) == _lib.DDF_ERR_UNSUPPORTED
    f32 = _lib.DdfNet(128, 4, 0, 1)
    assert lib.ddf_query(ctypes.byref(f32), 1, 1, 10, 1, 1, None) == _lib.DDF_ERR_UNSUPPORTED
    # parameter gradients need a float32 network; fp8 cannot give input gradients
    net = _lib.DdfNet(128, 4, 1, 1)
    assert lib.ddf_backward(ctypes.byref(net), 1, 10, None, None, None, 1, 0, None, 0, None) == _lib.DDF_ERR_UNSUPPORTED
    net = _lib.DdfNet(128, 4, 2, 1)
    assert lib.ddf_backward(ctypes.byref(net), 1, 10, None, None, 1, None, 0, None, 0, None) == _lib.DDF_ERR_UNSUPPORTED
    # chunked training step: float32 only, chunk >= 1, workspace sized for one chunk
    f32 = _lib.DdfNet(128, 4, 0, 1)
    bf = _lib.DdfNet(128, 4, 1, 1)
    big = 1 << 40
    assert lib.ddf_train_step_chunked(ctypes.byref(bf), 1, 1, 1, 1, 1e-3, 1, 1, 1000, 100, 1, 1, 1, big, None) == \
        _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_train_step_chunked(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 1000, 0, 1, 1, 1, big, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_chunked(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 1000, 100, 1, 1, 1, 16, None) == \
        _lib.DDF_ERR_WORKSPACE
    assert b"workspace" in lib.ddf_last_error()
    # fp8 packing needs scales, the others must not get any
    assert lib.ddf_pack_net(1, 128, 4, 2, None, 1, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_pack_net(1, 128, 4, 1, 1, 1, None) == _lib.DDF_ERR_INVALID_ARG


def test_dataset_sampler_validation(lib):
    from paper_2306_16142_amd import _lib
    P = _lib.DdfDatasetParams
    b = ctypes.c_size_t(0)
    assert lib.ddf_dataset_workspace_size(ctypes.byref(P(10, 10, 10, 1e-4, 0, 20480)), ctypes.byref(b)) == _lib.DDF_OK
    # pair data, perpendicular lines (origin, direction, a flag per side) and two scans, at least
    pairs = 20480 * 100
    assert b.value >= pairs * 36 + pairs * 10 * (24 + 8 + 8)
    assert lib.ddf_dataset_workspace_size(None, ctypes.byref(b)) == _lib.DDF_ERR_INVALID_ARG
    for bad in (P(0, 1, 1, 1e-4, 0, 1), P(1, 0, 1, 1e-4, 0, 1), P(1, 1, 0, 1e-4, 0, 1), P(1, 1, 1, -1.0, 0, 1),
                P(1, 1, 1, math.nan, 0, 1), P(1, 1, 1, 1e-4, -1, 1), P(1, 1, 1, 1e-4, 0, -1)):
        assert lib.ddf_dataset_workspace_size(ctypes.byref(bad), ctypes.byref(b)) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_dataset_workspace_size(ctypes.byref(P(64, 64, 64, 1e-4, 0, 1 << 20)), ctypes.byref(b)) == \
        _lib.DDF_ERR_UNSUPPORTED
    ok = P(2, 2, 2, 1e-4, 0, 4)
    # face range beyond the mesh, NULL count, NULL outputs with capacity, negative capacity
    assert lib.ddf_sample_dataset(1, 3, ctypes.byref(ok), 1, 1, 1, 1, None, 8, 1, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert b"beyond" in lib.ddf_last_error()
    assert lib.ddf_sample_dataset(1, 4, ctypes.byref(ok), 1, 1, 1, 1, None, 8, None, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_sample_dataset(1, 4, ctypes.byref(ok), 1, 1, None, None, None, 8, 1, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_sample_dataset(1, 4, ctypes.byref(ok), 1, 1, 1, 1, None, -1, 1, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    # NULL triangles or uniforms, too small a workspace
    assert lib.ddf_sample_dataset(None, 4, ctypes.byref(ok), 1, 1, 1, 1, None, 8, 1, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_sample_dataset(1, 4, ctypes.byref(ok), 1, 1, 1, 1, None, 8, 1, 1, 16, None) == \
        _lib.DDF_ERR_WORKSPACE
    assert b"workspace" in lib.ddf_last_error()


def test_udf_validation(lib):
    from paper_2306_16142_amd import _lib
    b = ctypes.c_size_t(0)
    assert lib.ddf_udf_workspace_size(1000, 100, ctypes.byref(b)) == _lib.DDF_OK and b.value >= 1000 * 100 * 28
    assert lib.ddf_udf_workspace_size(1 << 20, 512, ctypes.byref(b)) == _lib.DDF_OK
    assert b.value < (1 << 24) * 29 + 8 * 512 + 1024   # one pass holds at most 2^24 queries
    assert lib.ddf_udf_workspace_size(-1, 100, ctypes.byref(b)) == _lib.DDF_ERR_INVALID_ARG
    net = _lib.DdfNet(128, 4, 1, 1)
    assert lib.ddf_udf(None, 1, 10, 1, 10, 1, None, 1, 1 << 30, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_udf(ctypes.byref(_lib.DdfNet(96, 4, 1, 1)), 1, 10, 1, 10, 1, None, 1, 1 << 30, None) == \
        _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_udf(ctypes.byref(net), None, 10, 1, 10, 1, None, 1, 1 << 30, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_udf(ctypes.byref(net), 1, -1, 1, 10, 1, None, 1, 1 << 30, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_udf(ctypes.byref(net), 1, 0, None, 10, None, None, None, 0, None) == _lib.DDF_OK
    assert lib.ddf_udf(ctypes.byref(net), 1, 10, 1, 10, 1, None, 1, 64, None) == _lib.DDF_ERR_WORKSPACE
    assert b"workspace" in lib.ddf_last_error()


def test_paper_loss_validation(lib):
    from paper_2306_16142_amd import _lib
    L = _lib.DdfLoss
    big = 1 << 20
    for bad in (L(3, 1.0), L(-1, 1.0), L(1, 0.0), L(1, -1.0), L(1, math.inf), L(1, math.nan)):
        assert lib.ddf_loss_seeds_ex(1, 1, 1, 10, ctypes.byref(bad), 1, 1, 1, 1, big, None) == _lib.DDF_ERR_INVALID_ARG
    assert b"loss" in lib.ddf_last_error() or b"delta" in lib.ddf_last_error()
    f32 = _lib.DdfNet(128, 4, 0, 1)
    assert lib.ddf_train_step_ex(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 100, 0, ctypes.byref(L(7, 1.0)), 1, 1, 1,
                                 1 << 40, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_ex(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 100, -1, None, 1, 1, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    # the squish loss ignores delta; the default loss is taken for NULL
    assert lib.ddf_loss_seeds_ex(None, 1, 1, 10, ctypes.byref(L(2, math.nan)), 1, 1, 1, 1, big, None) == \
        _lib.DDF_ERR_INVALID_ARG   # (NULL logit)
    assert lib.ddf_train_step_ex(ctypes.byref(_lib.DdfNet(128, 4, 1, 1)), 1, 1, 1, 1, 1e-3, 1, 1, 100, 0, None, 1, 1,
                                 1, 1 << 40, None) == _lib.DDF_ERR_UNSUPPORTED


def test_eikonal_step_validation(lib):
    from paper_2306_16142_amd import _lib
    b = ctypes.c_size_t(0)
    assert lib.ddf_eikonal_workspace_size(128, 4, 1000, ctypes.byref(b)) == _lib.DDF_OK and b.value > 2000 * 4 * 9
    f32 = _lib.DdfNet(128, 4, 0, 1)
    args = lambda h, lam, ws: (ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 1, 100, h, lam, None, 1, 1, 1, ws, None)
    assert lib.ddf_train_step_eikonal(*args(0.0, 0.1, 1 << 40)) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_eikonal(*args(math.nan, 0.1, 1 << 40)) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_eikonal(*args(0.01, -1.0, 1 << 40)) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_eikonal(*args(0.01, 0.1, 16)) == _lib.DDF_ERR_WORKSPACE
    bf = _lib.DdfNet(128, 4, 1, 1)
    assert lib.ddf_train_step_eikonal(ctypes.byref(bf), 1, 1, 1, 1, 1e-3, 1, 1, 1, 100, 0.01, 0.1, None, 1, 1, 1,
                                      1 << 40, None) == _lib.DDF_ERR_UNSUPPORTED


def test_workspace_sizes(lib):
    from paper_2306_16142_amd import _lib
    b = ctypes.c_size_t(0)
    assert lib.ddf_train_workspace_size(256, 6, 65536, ctypes.byref(b)) == _lib.DDF_OK
    # features + activations + adjoints + chunk partials, at least
    assert b.value >= (65 + 2 * 6 * 256) * 65536 * 4
    p = _lib.DdfRenderParams()
    p.width, p.height, p.spp, p.bounces = 64, 64, 1, 3
    scene = _lib.DdfScene(_lib.BACKEND_MESH, 1, 3, None, 0, None, 0, None)
    assert lib.ddf_render_workspace_size(ctypes.byref(scene), ctypes.byref(p), ctypes.byref(b)) == _lib.DDF_OK
    assert b.value > 64 * 64 * 40
    p.bounces = 0
    assert lib.ddf_render_workspace_size(ctypes.byref(scene), ctypes.byref(p), ctypes.byref(b)) == _lib.DDF_ERR_INVALID_ARG
    # a multi-object scene sizes its (ray, instance) pair buffers by the instance count
    p.bounces = 3
    nets = (_lib.DdfNet * 1)(_lib.DdfNet(128, 4, 1, 1))
    inst = (_lib.DdfInstance * 4)(*[_lib.DdfInstance() for _ in range(4)])
    multi = _lib.DdfScene(_lib.BACKEND_MULTI, None, 0, None, 1, nets, 4, inst)
    b2 = ctypes.c_size_t(0)
    assert lib.ddf_render_workspace_size(ctypes.byref(multi), ctypes.byref(p), ctypes.byref(b2)) == _lib.DDF_OK
    assert b2.value > b.value + 4 * 64 * 64 * 60
    # an instance naming a missing network is rejected before launching
    inst[2].net = 3
    assert lib.ddf_render_wavefront(ctypes.byref(multi), ctypes.byref(p), 1, None, None, None, 1, b2.value, None) == \
        _lib.DDF_ERR_INVALID_ARG
    # a too-small workspace is rejected before launching
    p.bounces = 3
    assert lib.ddf_render_wavefront(ctypes.byref(scene), ctypes.byref(p), 1, None, None, None, 1, 16, None) == \
        _lib.DDF_ERR_WORKSPACE


def test_tuning_knobs_validate_and_round_trip(lib):
    from paper_2306_16142_amd import _lib
    v = ctypes.c_int32(0)
    defaults = {"stream_wg_per_cu": 2, "cull_rays_per_block": 2048, "grad_wg_per_cu": 2}
    for name, knob in _lib.TUNE_KNOBS.items():
        assert lib.ddf_get_tuning(knob, ctypes.byref(v)) == _lib.DDF_OK
        assert v.value == defaults[name]
    assert lib.ddf_set_tuning(99, 1) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_set_tuning(_lib.TUNE_KNOBS["stream_wg_per_cu"], 3) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_set_tuning(_lib.TUNE_KNOBS["cull_rays_per_block"], 3000) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_set_tuning(_lib.TUNE_KNOBS["grad_wg_per_cu"], 3) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_get_tuning(0, None) == _lib.DDF_ERR_INVALID_ARG
    k = _lib.TUNE_KNOBS["cull_rays_per_block"]
    assert lib.ddf_set_tuning(k, 4096) == _lib.DDF_OK
    assert lib.ddf_get_tuning(k, ctypes.byref(v)) == _lib.DDF_OK and v.value == 4096
    assert lib.ddf_set_tuning(k, 2048) == _lib.DDF_OK


def test_empty_batch_is_rejected_where_a_loss_is_formed(lib):
    """The header's exception to "n == 0 is a no-op": every entry point that forms a loss
    rejects an empty batch before launching anything."""
    from paper_2306_16142_amd import _lib
    big = 1 << 40
    f32 = _lib.DdfNet(128, 4, 0, 1)
    clamp = _lib.DdfLoss(1, 1.0)
    assert lib.ddf_loss_seeds(1, 1, 1, 0, 1, 1, 1, 1, big, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_loss_seeds_ex(1, 1, 1, 0, None, 1, 1, 1, 1, big, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 0, 1, 1, 1, big, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_chunked(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 0, 10, 1, 1, 1, big, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_ex(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 0, 0, None, 1, 1, 1, big, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_train_step_eikonal(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 1, 0, 0.01, 0.1, None, 1, 1, 1, big,
                                      None) == _lib.DDF_ERR_INVALID_ARG
    paper = _lib.DdfPaperNet(8, 0, 1)
    assert lib.ddf_paper_train_step(ctypes.byref(paper), 1, 1, 1, 1, 1e-3, 1, 1, 0, ctypes.byref(clamp), 0.5, 0, 1, 1,
                                    1, big, None) == _lib.DDF_ERR_INVALID_ARG
    # the queries and gradients stay no-ops on an empty batch
    assert lib.ddf_forward(ctypes.byref(f32), None, 0, None, None, None) == _lib.DDF_OK
    assert lib.ddf_paper_forward(ctypes.byref(_lib.DdfPaperNet(8, 1, 1)), None, 0, None, None) == _lib.DDF_OK
    assert lib.ddf_paper_backward(ctypes.byref(paper), None, None, 0, None, None, None, 0, None, 0, None) == _lib.DDF_OK


def test_paper_network_validation(lib):
    from paper_2306_16142_amd import _lib
    c, b = ctypes.c_int64(0), ctypes.c_size_t(0)
    assert lib.ddf_paper_param_count(8, ctypes.byref(c)) == _lib.DDF_OK
    assert c.value == 5 * 512 + 7 * 512 * 512 + 2 * 8 * 512 + 512 + 1
    assert lib.ddf_paper_param_count(9, ctypes.byref(c)) == _lib.DDF_ERR_UNSUPPORTED
    assert lib.ddf_paper_packed_bytes(8, 2, ctypes.byref(b)) == _lib.DDF_ERR_UNSUPPORTED   # no fp8 form
    assert lib.ddf_paper_packed_bytes(8, 1, ctypes.byref(b)) == _lib.DDF_OK and b.value > 7 * 512 * 512 * 2
    bf = _lib.DdfPaperNet(8, 1, 1)
    # parameter gradients need float32 and the parameters
    assert lib.ddf_paper_backward(ctypes.byref(bf), 1, 1, 10, None, None, 1, 0, 1, 1 << 40, None) == \
        _lib.DDF_ERR_UNSUPPORTED
    f32 = _lib.DdfPaperNet(8, 0, 1)
    assert lib.ddf_paper_backward(ctypes.byref(f32), None, 1, 10, None, None, 1, 0, 1, 1 << 40, None) == \
        _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_paper_backward(ctypes.byref(f32), 1, 1, 10, None, None, 1, 0, 1, 16, None) == _lib.DDF_ERR_WORKSPACE
    # the paper's network trains on its own losses only (clamp, squish)
    assert lib.ddf_paper_train_step(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 10, ctypes.byref(_lib.DdfLoss(0, 1.0)),
                                    0.5, 0, 1, 1, 1, 1 << 40, None) == _lib.DDF_ERR_INVALID_ARG
    assert lib.ddf_paper_train_step(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 10, None, 0.5, 0, 1, 1, 1, 1 << 40,
                                    None) == _lib.DDF_ERR_INVALID_ARG
    # dropout must lie in [0, 1)
    clamp = ctypes.byref(_lib.DdfLoss(_lib.LOSSES["clamp"], 1.0))
    for bad in (1.0, -0.1, float("nan")):
        assert lib.ddf_paper_train_step(ctypes.byref(f32), 1, 1, 1, 1, 1e-3, 1, 1, 10, clamp, bad, 0, 1, 1, 1, 1 << 40,
                                        None) == _lib.DDF_ERR_INVALID_ARG


def test_udf_noalloc_validation(lib):
    from paper_2306_16142_amd import _lib
    net = _lib.DdfNet(128, 4, 1, 1)
    assert lib.ddf_udf_noalloc(ctypes.byref(net), 1, 10, 1, 65537, 1, 1, None) == _lib.DDF_ERR_UNSUPPORTED
    assert b"65536" in lib.ddf_last_error()
