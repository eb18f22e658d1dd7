"""Shared helpers of the GPU parity tests (inputs come from ``synthetic``; expected values
from ``oracle``; the device path goes through the C ABI via the package binding)."""
import numpy as np
import torch

from oracle import geometry


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def rays5_from(o, d):
    """Oracle-side ray assembly (float64 angles of the float32 directions), cast to float32."""
    th, ph = geometry.angles_from_dirs(d)
    return np.concatenate([o.astype(np.float64), th[None], ph[None]]).astype(np.float32)


def banner(msg):
    print("[gpu-case] " + msg, flush=True)
