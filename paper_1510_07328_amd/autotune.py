"""Autotuner for the launch shapes of the library: the tile shape of the batched
tube sweep (columns per tile S, halo / steps per round H, threads per
workgroup) and the workgroup size of the plain field step.

Candidates are timed on the GPU through the library's own entry points and the
fastest is kept in a JSON cache, keyed by the device, the built library and a
digest of the workload, so that later runs reuse it.  The cache file is
$LBM_AUTOTUNE_CACHE if set, else ~/.cache/paper_1510_07328_amd/autotune.json.

Batched sweep: the time of one sweep is the longest tube's chain of rounds plus
the rounds' synchronisation, and the tile shape trades halo work (2H redundant
columns per S useful ones), round count (steps / H) and parallelism in the
tail, where only the longest tubes are active.  Each candidate is therefore
timed on the real tube set with every tube's step count scaled by `fraction`,
which keeps the shape of the schedule.
"""
from __future__ import annotations

import functools
import hashlib
import json
import os
import time

import numpy as np

MAX_WINDOW = 512  # LDS window of the batched round kernel (columns, tile + 2 halo)
HALOS = (16, 24, 32, 48, 64)
WINDOWS = (256, 512)
BLOCKS = (256, 512, 1024)
FIELD_BLOCKS = (128, 256, 512, 1024)


def cache_path() -> str:
    p = os.environ.get("LBM_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1510_07328_amd", "autotune.json")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def batch_candidates(halos=HALOS, windows=WINDOWS, blocks=BLOCKS):
    """(tile_cols, halo, block) triples with tile + 2 halo within the LDS window."""
    out = []
    for w in windows:
        for h in halos:
            s = w - 2 * h
            if s < 1 or w > MAX_WINDOW:
                continue
            for b in blocks:
                if b % 64 == 0 and 64 <= b <= 1024:
                    out.append((s, h, b))
    return out


def batch_key(device: str, tubes, opt) -> str:
    """Digest of what decides the best shape: device, the (nx, steps) multiset,
    precision and truncation order."""
    pairs = sorted((int(t.nx), int(t.steps)) for t in tubes)
    h = hashlib.sha256(json.dumps(pairs).encode()).hexdigest()[:16]
    return f"batch|{device}|p{int(opt.precision)}|o{int(opt.order)}|n{len(pairs)}|{h}"


def field_key(device: str, cfg) -> str:
    return (f"field|{device}|l{cfg.lattice}|{cfg.nx}x{cfg.ny}x{cfg.nz}|p{cfg.precision}|o{cfg.order}"
            f"|s{cfg.scheme}")


def pick_best(timings: dict) -> tuple:
    """Fastest candidate (ties: the first in sorted order, so the choice is
    deterministic)."""
    if not timings:
        raise ValueError("no timings")
    return min(sorted(timings), key=lambda k: timings[k])


def device_name() -> str:
    """Architecture and CU count of the current device, plus a digest of the built
    library, so that a rebuilt kernel is tuned again rather than served an
    optimum measured on the previous one."""
    import torch

    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch.split(':')[0]}x{p.multi_processor_count}|lib{library_digest()}"


@functools.lru_cache(maxsize=1)
def library_digest() -> str:
    from . import lbm

    h = hashlib.sha256()
    with open(lbm.library_path(), "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:12]


def _scaled_tubes(tubes, fraction: float):
    from . import batch as B

    nx = np.array([t.nx for t in tubes])
    steps = np.array([max(1, int(round(t.steps * fraction))) if t.steps > 0 else 0 for t in tubes])
    return B.make_tubes(nx, [t.tau for t in tubes], [t.n_left for t in tubes], [t.n_right for t in tubes], steps)


def time_batch_shape(tubes, opt, shape, repeats: int = 2) -> float:
    """Milliseconds of one lbm_batch_run of `tubes` with the tile shape `shape`
    (best of `repeats`, after a warm-up run that also captures the graph)."""
    import copy

    import torch

    from . import batch as B

    o = copy.copy(opt)
    o.tile_cols, o.halo, o.block = shape
    bt = B.Batch(tubes, o)
    try:
        bt.run()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(bt.stream)
            bt.run()
            e1.record(bt.stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
    finally:
        bt.free()
    return best


def tune_batch(tubes, opt, fraction: float = 0.125, candidates=None, cache: dict | None = None,
               path: str | None = None, timer=None, device: str | None = None):
    """Best (tile_cols, halo, block) for this tube set, from the cache or by
    timing every candidate on the tube set with steps scaled by `fraction`.
    Returns (shape, record); record holds the timings and the tuning time."""
    device = device or device_name()
    key = batch_key(device, tubes, opt)
    own_cache = cache is None
    cache = load_cache(path) if own_cache else cache
    if key in cache:
        rec = cache[key]
        return (rec["tile_cols"], rec["halo"], rec["block"]), dict(rec, cached=True)
    cands = candidates or batch_candidates()
    probe = _scaled_tubes(tubes, fraction)
    timer = timer or time_batch_shape
    t0 = time.perf_counter()
    timings = {tuple(c): timer(probe, opt, tuple(c)) for c in cands}
    best = pick_best(timings)
    rec = {"tile_cols": best[0], "halo": best[1], "block": best[2], "ms_probe": timings[best],
           "fraction": fraction, "tuning_s": round(time.perf_counter() - t0, 3),
           "timings": {f"{s}/{h}/{b}": round(v, 4) for (s, h, b), v in sorted(timings.items())}}
    cache[key] = rec
    if own_cache:
        save_cache(cache, path)
    return best, dict(rec, cached=False)


def batch_options(tubes, opt, **kw):
    """A copy of opt with the autotuned tile shape filled in."""
    import copy

    (s, h, b), rec = tune_batch(tubes, opt, **kw)
    o = copy.copy(opt)
    o.tile_cols, o.halo, o.block = s, h, b
    return o, rec


# -- plain field step ----------------------------------------------------------

def time_field_block(cfg, n0, u0, block: int, steps: int = 100) -> float:
    """Microseconds per step of the field step with `block` threads per workgroup."""
    import copy

    import torch

    from . import lbm

    c = copy.copy(cfg)
    c.block = block
    lat = lbm.Lattice.create(c, n0, u0)
    try:
        lat.step(10)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / steps
    finally:
        lat.free()


def tune_field(cfg, n0, u0, blocks=FIELD_BLOCKS, cache: dict | None = None, path: str | None = None, timer=None,
               device: str | None = None):
    """Best workgroup size for the field step of cfg (cached like tune_batch)."""
    device = device or device_name()
    key = field_key(device, cfg)
    own_cache = cache is None
    cache = load_cache(path) if own_cache else cache
    if key in cache:
        return cache[key]["block"], dict(cache[key], cached=True)
    timer = timer or time_field_block
    timings = {b: timer(cfg, n0, u0, b) for b in blocks}
    best = pick_best(timings)
    rec = {"block": best, "us_per_step": timings[best], "timings": {str(b): round(v, 3) for b, v in timings.items()}}
    cache[key] = rec
    if own_cache:
        save_cache(cache, path)
    return best, dict(rec, cached=False)
