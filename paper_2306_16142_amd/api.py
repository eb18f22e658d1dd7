"""Thin PyTorch binding of libddf: allocates outputs as torch CUDA tensors and passes
raw device pointers and the current HIP stream to the C ABI.  Every step of the hot
path runs in the library's kernels; nothing here computes."""
import ctypes
import math

import torch

from . import _lib

PRECISIONS = {"fp32": _lib.PREC_FP32, "bf16": _lib.PREC_BF16, "fp8": _lib.PREC_FP8}


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, rows=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if rows is not None and (t.dim() != 2 or t.shape[0] != rows):
        raise ValueError("%s must have shape [%d, n], got %s" % (name, rows, tuple(t.shape)))
    return t


def label_rays(orig, dirs, tris, t_min=0.0, t_max=math.inf, crossings=True):
    """Nearest triangle hit of every ray: returns (t [n], tri [n] int32, crossings [n] int32 or None)."""
    _dev(orig, torch.float32, "orig", 3)
    _dev(dirs, torch.float32, "dirs", 3)
    _dev(tris, torch.float32, "tris", 9)
    n, m = orig.shape[1], tris.shape[1]
    t = torch.empty(n, device=orig.device, dtype=torch.float32)
    tri = torch.empty(n, device=orig.device, dtype=torch.int32)
    cr = torch.empty(n, device=orig.device, dtype=torch.int32) if crossings else None
    _lib.call("ddf_label_rays", _p(orig), _p(dirs), n, _p(tris), m, t_min, t_max, _p(t), _p(tri), _p(cr), _stream())
    return t, tri, cr


def assemble_rays(orig, dirs, out=None):
    """(origins [3][n], directions [3][n]) -> rays [5][n] = (ox, oy, oz, theta, phi)."""
    _dev(orig, torch.float32, "orig", 3)
    _dev(dirs, torch.float32, "dirs", 3)
    n = orig.shape[1]
    out = torch.empty((5, n), device=orig.device, dtype=torch.float32) if out is None else out
    _lib.call("ddf_assemble_rays", _p(orig), _p(dirs), n, _p(out), _stream())
    return out


def packed_bytes(width, depth, precision):
    b = ctypes.c_size_t(0)
    _lib.call("ddf_packed_bytes", width, depth, PRECISIONS[precision], ctypes.byref(b))
    return b.value


class Network:
    """A packed network (weights in MFMA-tile order) for one precision.

    ``params``: flat float32 CUDA tensor (per layer weight [out][in] then bias).
    For ``precision='fp8'`` give ``scales`` ([2 (depth + 1)] CUDA float32), e.g. from
    :func:`fp8_scales`.
    """

    def __init__(self, params, width, depth, precision="bf16", scales=None):
        _dev(params, torch.float32, "params")
        self.params, self.width, self.depth, self.precision = params, width, depth, precision
        self.scales = scales
        nbytes = packed_bytes(width, depth, precision)
        self.blob = torch.empty(nbytes, device=params.device, dtype=torch.uint8)
        _lib.call("ddf_pack_net", _p(params), width, depth, PRECISIONS[precision],
                  _p(scales) if scales is not None else ctypes.c_void_p(0), _p(self.blob), _stream())
        self.desc = _lib.DdfNet(width, depth, PRECISIONS[precision], self.blob.data_ptr())

    def forward(self, rays, logit=None, dist=None):
        """rays [5][n] -> (logit [n], dist [n])."""
        _dev(rays, torch.float32, "rays", 5)
        n = rays.shape[1]
        logit = torch.empty(n, device=rays.device, dtype=torch.float32) if logit is None else logit
        dist = torch.empty(n, device=rays.device, dtype=torch.float32) if dist is None else dist
        _lib.call("ddf_forward", ctypes.byref(self.desc), _p(rays), n, _p(logit), _p(dist), _stream())
        return logit, dist

    __call__ = forward


def fp8_scales(params, width, depth, calib_rays, net_fp32=None):
    """Static per-layer fp8 scales (weight absmax / 448, input absmax over calib rays / 448)."""
    _dev(calib_rays, torch.float32, "calib_rays", 5)
    net_fp32 = net_fp32 or Network(params, width, depth, "fp32")
    out = torch.empty(2 * (depth + 1), device=params.device, dtype=torch.float32)
    _lib.call("ddf_fp8_scales", ctypes.byref(net_fp32.desc), _p(params), _p(calib_rays), calib_rays.shape[1],
              _p(out), _stream())
    return out
