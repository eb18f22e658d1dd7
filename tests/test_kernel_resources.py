"""Register budgets of the hot kernels, from the compiler's resource report for gfx950 (runs
on the CPU: hipcc cross-compiles).  The query, normal and training kernels on the measured
paths must not spill to scratch; in particular every fp8 kernel (variants that spilled gave
wrong results on MI355X, cause not found: see the design notes), with one allowance: the
width-128 training sweep keeps four waves per SIMD and spills 176 bytes per lane, measured
faster than its spill-free form."""
import concurrent.futures
import os
import re
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2306_16142_amd", "csrc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "--cuda-device-only", "-c", "-o", os.devnull, "-Rpass-analysis=kernel-resource-usage"]


def _report(src):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    r = subprocess.run([hipcc] + FLAGS + [os.path.join(CSRC, src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    return out


@pytest.fixture(scope="module")
def scratch():
    if not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    srcs = ["mlp.hip", "stream.hip", "paper.hip", "sweep.hip"]
    with concurrent.futures.ThreadPoolExecutor(4) as ex:
        reports = list(ex.map(_report, srcs))
    merged = {}
    for rep in reports:
        merged.update(rep)
    return merged


def _pick(scratch, pattern):
    names = [n for n in scratch if re.search(pattern, n)]
    assert names, pattern
    return {n: scratch[n] for n in names}


def test_fp8_kernels_do_not_spill(scratch):
    k = _pick(scratch, r"forward_kernelILi2E")   # every fp8 instantiation of the query kernel
    assert all(v == 0 for v in k.values()), k


def test_measured_kernels_do_not_spill(scratch):
    for pattern in (r"forward_kernelILi1ELi128ELi2ELb1E",   # bf16 query with the weights in LDS
                    r"stream_kernel",                       # streamed bf16 queries and normals
                    r"paper_stream_kernel", r"paper_sweep_kernel",
                    r"sweep_kernelILi256E"):
        k = _pick(scratch, pattern)
        assert all(v == 0 for v in k.values()), k


def test_width_128_training_sweep_spill_stays_small(scratch):
    k = _pick(scratch, r"sweep_kernelILi128E")
    assert all(v <= 256 for v in k.values()), k
