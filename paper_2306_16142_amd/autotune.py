"""Autotuner of the launch-shape knobs (``ddf_set_tuning``).

A workload is a callable that launches GPU work on the current stream and returns its
output tensors.  For each knob, every candidate value is timed (median of ``reps`` runs
after one warm-up run, HIP events on the stream) and its outputs are compared bit for bit
with those of the configuration the tuner started from: a knob only spreads work
differently, so any difference is an error.  The fastest value is kept and the knob is
left set to it.  Results are cached as JSON keyed by GPU architecture and workload name
(path: argument, else ``DDF_AUTOTUNE_CACHE``, else ``~/.cache/ddf/autotune.json``).
"""
import json
import os
import statistics

import torch

from . import api

CANDIDATES = {
    "stream_wg_per_cu": [1, 2],
    "cull_rays_per_block": [512, 1024, 2048, 4096, 8192],
    "grad_wg_per_cu": [1, 2, 4],
}


def cache_path(path=None):
    return path or os.environ.get("DDF_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ddf",
                                                                         "autotune.json")


def _arch():
    return getattr(torch.cuda.get_device_properties(torch.cuda.current_device()), "gcnArchName", "unknown")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time_ms(run, reps):
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(name, run, knobs, reps=20, path=None, use_cache=True):
    """Tune `knobs` (names from CANDIDATES) on the workload `run`; returns
    {"chosen": {knob: value}, "median_ms": {knob: {value: ms}}, "cached": bool}."""
    path = cache_path(path)
    key = "%s/%s" % (_arch(), name)
    cache = _load(path)
    if use_cache and key in cache:
        for k, v in cache[key]["chosen"].items():
            api.set_tuning(k, v)
        return dict(cache[key], cached=True)
    ref = [t.clone() for t in run()]
    torch.cuda.synchronize()
    chosen, table = {}, {}
    for knob in knobs:
        start = api.get_tuning(knob)
        best, table[knob] = None, {}
        for v in CANDIDATES[knob]:
            api.set_tuning(knob, v)
            out = run()   # warm-up, and the result check
            torch.cuda.synchronize()
            if not all(torch.equal(a, b) for a, b in zip(out, ref)):
                api.set_tuning(knob, start)
                raise RuntimeError("autotune: knob %s = %d changed the result of %s" % (knob, v, name))
            ms = _time_ms(run, reps)
            table[knob][v] = ms
            if best is None or ms < best[1]:
                best = (v, ms)
        api.set_tuning(knob, best[0])
        chosen[knob] = best[0]
    result = {"chosen": chosen, "median_ms": table}
    cache[key] = result
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return dict(result, cached=False)
