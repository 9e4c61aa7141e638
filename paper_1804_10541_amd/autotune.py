"""Tile autotuner for the voxel-tile kernels.

Picks the work-group shape (bx x by threads) and the z split (the number of
work-groups the split aims for) for one problem size by timing the
Hessian-vector kernel -- the one the conjugate-gradient iterations repeat --
with HIP events on the device, and keeps the winner in a JSON cache keyed by
GPU architecture, kernel and problem size.  The choice only changes the
schedule: every configuration computes the same quantities (the fixed-order
float64 partial sums follow the tiling, so results agree to rounding).

Cache file: ``$MFR_TUNE_CACHE`` if set, else ``~/.cache/mfr/tiles.json``.
"""
from __future__ import annotations

import json
import os
import tempfile

import torch

from . import mfr

SHAPES = ((32, 16), (64, 8), (32, 32), (64, 16))
GROUP_TARGETS = (1024, 2048, 4096)
# explicit z-chunk lengths (planes per work-group), tried besides the derived
# splits: small volumes run fastest with chunks shorter than the derived minimum
CHUNK_LENS = (4, 6, 12, 24)
KERNEL = "tile_hv"


def cache_path():
    p = os.environ.get("MFR_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "mfr", "tiles.json")


def arch(device):
    props = torch.cuda.get_device_properties(torch.device(device))
    return getattr(props, "gcnArchName", props.name)


def size_key(spec):
    m = "x".join(str(int(k)) for k in spec.m)
    my = "x".join(str(int(k)) for k in spec.my)
    mT = getattr(spec, "mT", None)
    t = "" if mT is None else "/T" + "x".join(str(int(k)) for k in mT)
    return f"m={m}/my={my}{t}"


def cache_key(device, spec, kernel=KERNEL):
    return f"{arch(device)}|{kernel}|{size_key(spec)}"


def _load(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tiles.", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)   # atomic: concurrent readers see the old or the new file


def lookup(spec, device="cuda:0", path=None):
    """The cached configuration for this size on this GPU, or None."""
    entry = _load(path or cache_path()).get(cache_key(device, spec))
    return None if entry is None else dict(entry["config"])


def candidates():
    return ([dict(bx=bx, by=by, chunk_len=0, target_groups=g) for (bx, by) in SHAPES for g in GROUP_TARGETS]
            + [dict(bx=bx, by=by, chunk_len=c, target_groups=0) for (bx, by) in SHAPES for c in CHUNK_LENS])


def time_config(cfg, spec, R, T, u, p, device, reps):
    """Average Hessian-vector kernel time (ms, HIP events) under one configuration."""
    mfr.set_tile_config(**cfg)
    ctx = mfr.Context(spec, device)
    try:
        ctx.set_images(R, T)
        q = torch.empty_like(p)
        ctx.hess_vec(u, p, out=q)   # warm-up (code object load, caches)
        ctx.profile(True)
        ctx.profile_read(reset=True)
        for _ in range(reps):
            ctx.hess_vec(u, p, out=q)
        launches, ms = ctx.profile_read(reset=True)[KERNEL]
        ctx.profile(False)
    finally:
        ctx.close()
    return ms / max(launches, 1)


def tune(spec, R, T, u, device="cuda:0", reps=5, configs=None, path=None, seed=0):
    """Times every candidate on (R, T, u) with a seeded N(0,1) direction,
    stores the fastest in the cache, makes it the process-wide configuration
    and returns {"config", "ms", "timings"}."""
    device = torch.device(device)
    gen = torch.Generator(device=device).manual_seed(seed)
    p = torch.randn(u.shape, generator=gen, device=device, dtype=torch.float32)
    prev = mfr.get_tile_config()
    timings = []
    try:
        for cfg in (configs or candidates()):
            timings.append((time_config(cfg, spec, R, T, u, p, device, reps), cfg))
    except Exception:
        mfr.set_tile_config(**prev)
        raise
    ms, best = min(timings, key=lambda t: t[0])
    path = path or cache_path()
    data = _load(path)
    data[cache_key(device, spec)] = {"config": best, "ms": ms,
                                     "timings": [{"config": c, "ms": t} for t, c in timings]}
    _store(path, data)
    mfr.set_tile_config(**best)
    return {"config": best, "ms": ms, "timings": timings}


def apply(spec, R, T, u, device="cuda:0", path=None, reps=5):
    """Cached configuration for this size if there is one, else tune; the
    result becomes the process-wide configuration.  Returns the config."""
    cfg = lookup(spec, device, path)
    if cfg is None:
        return tune(spec, R, T, u, device=device, reps=reps, path=path)["config"]
    mfr.set_tile_config(**cfg)
    return cfg
