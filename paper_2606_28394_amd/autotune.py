"""Pack-size tuner for batched stepping.

The step kernel gives each workgroup a pack of whole towers.  A larger pack fills more of
a wave's 64 lanes in every colour of the coloured Gauss-Seidel sweep, but needs more LDS,
so fewer workgroups share a compute unit.  The library picks the largest pack that keeps
eight workgroups per CU (``pack_bodies = 0``); this tuner times a few pack sizes on the
batch itself and keeps the fastest.

It runs the batch for ``lead_in`` steps first (the tilted towers are falling by then, so
the contacts are those of the collapse, not of the intact towers), then builds one world
per candidate pack size from that state and times ``steps`` steps of each in one launch,
with HIP events on the world's stream.  Packing changes which towers share a workgroup,
not what any tower computes, so every candidate advances the same state.

Results can be kept in a JSON file keyed by the device, the library's kernel sources, the
batch (tower sizes, friction, parameters) and the tuning settings, so a later run on the
same batch skips the timing.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from . import jenga as J

DEFAULT_CANDIDATES = (0, 64, 80, 96, 112, 128)
_SOURCES = ("csrc/jenga_step.hip", "csrc/jenga_device.h", "csrc/jenga_world.hip")


def batch_key(scene: dict, warm_start: int, candidates, steps: int, lead_in: int, device: str,
              margin: float = 0.02) -> str:
    """Cache key: device name, kernel sources, the batch's shape and parameters, tuning settings."""
    h = hashlib.sha256()
    h.update(device.encode())
    here = os.path.dirname(os.path.abspath(__file__))
    for s in _SOURCES:
        with open(os.path.join(here, s), "rb") as f:
            h.update(f.read())
    h.update(np.ascontiguousarray(np.diff(np.asarray(scene["tower_ptr"], np.int64))).tobytes())
    h.update(np.ascontiguousarray(np.asarray(scene["mu"], np.float64)).tobytes())
    h.update(json.dumps(scene["params"], sort_keys=True, default=float).encode())
    h.update(json.dumps([int(warm_start), [int(c) for c in candidates], int(steps), int(lead_in),
                         float(margin)]).encode())
    return h.hexdigest()[:24]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, entry):
    table = _load(path)
    table[key] = entry
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_pack_bodies(scene: dict, candidates=DEFAULT_CANDIDATES, steps: int = 40, lead_in: int = 60,
                     warm_start: int = 0, cache: str | None = None, margin: float = 0.02, log=None) -> dict:
    """Time ``steps`` steps of the batch for each pack size in ``candidates`` (0 = the library's
    own choice) and return ``{"pack_bodies": best, "tower_steps_per_s": {size: rate}, ...}``.
    The library's choice is kept unless another candidate is faster by more than ``margin``
    (run-to-run noise of a short timing is about 1 %).  Needs a GPU; the worlds run on
    torch's current stream."""
    cands = [int(c) for c in candidates]
    if not cands or any(c < 0 or c > 256 for c in cands):
        raise ValueError("candidate pack sizes must lie in [0, 256] (0 = the library's choice)")
    if steps < 1 or lead_in < 0:
        raise ValueError("steps must be positive and lead_in non-negative")
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the pack-size tuner times the step kernel and needs a GPU")
    device = torch.cuda.get_device_name()
    key = batch_key(scene, warm_start, cands, steps, lead_in, device, margin)
    if cache:
        hit = _load(cache).get(key)
        if hit is not None:
            return dict(hit, cached=True)
    stream = torch.cuda.current_stream()
    start = J.World(scene, warm_start=warm_start, stream=stream.cuda_stream)
    if lead_in > 0:
        start.step(lead_in)
    state = start.state()
    start.close()
    rates = {}
    T = int(scene["n_towers"])
    for c in cands:
        w = J.World(scene, warm_start=warm_start, stream=stream.cuda_stream, pack_bodies=c)
        w.set_state(*state)
        w.step(0)          # upload before the timed launch
        w.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        w.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        err = int(w.stats().error_word)
        w.close()
        rates[c] = T * steps / (ms * 1e-3) if err == 0 else 0.0
        if log:
            log(f"  pack_bodies {c}: {rates[c]:.4g} tower-steps/s" + (f" (error word {err})" if err else ""))
    best = max(cands, key=lambda c: rates[c])
    if 0 in rates and rates[best] <= rates[0] * (1.0 + margin):
        best = 0
    entry = {"pack_bodies": best, "tower_steps_per_s": {str(c): rates[c] for c in cands},
             "steps": steps, "lead_in": lead_in, "margin": margin, "device": device}
    if cache:
        _store(cache, key, entry)
    return dict(entry, cached=False)
