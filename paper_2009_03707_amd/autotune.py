"""Autotuner for the launch parameters of the hot path.

It picks, per GPU architecture and size class:
  * the gradient workgroup tile shape (MS_OPT_GRADIENT_TILE), timed on the
    gradient stage alone;
  * the path-counting schedule (MS_OPT_PATH_SCHEDULE: the ready frontier
    with column merges, the ready frontier with entry-parallel merges, or
    the paper's power iteration, the last only below 2^26 voxels) and the
    ready schedule's column-merge parameters (MS_OPT_MERGE_LIGHT,
    MS_OPT_MERGE_CHUNK), timed on the path stage.

None of these options changes any result (the library is bit-exact for every
setting); only the time does.  Choices are cached as JSON in
$MSC_TUNE_CACHE (default ~/.cache/msc_tune.json) keyed by
"<arch>|<size class>", where the size class is the power-of-two bucket of
the voxel count and of the number of fields.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import msc

DEFAULT = {"tile": 0, "schedule": msc.MS_PATHS_READY, "light": 32, "chunk": 4096}
TILES = (0, 1, 2, 3, 4, 5, 6)
SCHEDULES = (msc.MS_PATHS_READY, msc.MS_PATHS_ENTRY, msc.MS_PATHS_POWER)
LIGHTS = (8, 16, 32, 64, 128)
CHUNKS = (2048, 4096)
# the power iteration materialises every frontier (about four times the
# entries of A* at 512^3); beyond this many voxels it is not tried
POWER_MAX_VOXELS = 1 << 26


def cache_path() -> str:
    return os.environ.get("MSC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "msc_tune.json"))


def size_class(fields) -> str:
    vox = sum(int(f.numel()) for f in fields)
    return f"v{int(math.log2(max(vox, 1)))}-n{int(math.log2(len(fields)))}"


def arch() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def apply(ctx: msc.Context, cfg: dict) -> None:
    ctx.set_option(msc.MS_OPT_GRADIENT_TILE, cfg["tile"])
    ctx.set_option(msc.MS_OPT_PATH_SCHEDULE, cfg["schedule"])
    ctx.set_option(msc.MS_OPT_MERGE_LIGHT, cfg["light"])
    ctx.set_option(msc.MS_OPT_MERGE_CHUNK, cfg["chunk"])


def _run(ctx, fields):
    if len(fields) == 1:
        ctx.complex_raw(fields[0])
    else:
        ctx.complex_batch_raw(fields)


def _measure(ctx, fields, cfg, stage, reps):
    apply(ctx, cfg)
    try:
        _run(ctx, fields)  # warm the workspace for this setting
        ctx.set_timing(True)
        for _ in range(reps):
            _run(ctx, fields)
    except msc.MscError as e:
        if e.status != msc.MS_ERR_OOM:
            raise
        ctx.set_timing(False)
        ctx.release()  # drop what the failed setting allocated
        return float("inf")
    t = ctx.timing()
    ctx.set_timing(False)
    return t[stage] / max(t["calls"], 1)


def tune(ctx: msc.Context, fields, reps: int = 2, use_cache: bool = True, log=None) -> dict:
    """Coordinate descent over the options; returns (and caches) the best
    setting for this architecture and size class, and applies it to ctx."""
    key = f"{arch()}|{size_class(fields)}"
    path = cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        cfg = dict(DEFAULT, **cache[key])
        apply(ctx, cfg)
        return cfg
    cfg = dict(DEFAULT)
    trace = {}
    best = None
    for t in TILES:
        c = dict(cfg, tile=t)
        ms = _measure(ctx, fields, c, "gradient_ms", reps)
        trace[f"tile={t}"] = ms
        if best is None or ms < best[0]:
            best = (ms, t)
    cfg["tile"] = best[1]
    best = None
    vox = sum(int(f.numel()) for f in fields)
    for sch in SCHEDULES:
        if sch == msc.MS_PATHS_POWER and vox > POWER_MAX_VOXELS:
            continue
        for light in (LIGHTS if sch == msc.MS_PATHS_READY else (32,)):
            for chunk in (CHUNKS if sch == msc.MS_PATHS_READY else (4096,)):
                c = dict(cfg, schedule=sch, light=light, chunk=chunk)
                ms = _measure(ctx, fields, c, "paths_ms", reps)
                trace[f"schedule={sch},light={light},chunk={chunk}"] = ms
                if best is None or ms < best[0]:
                    best = (ms, sch, light, chunk)
    cfg.update(schedule=best[1], light=best[2], chunk=best[3])
    ctx.release()  # keep only what the chosen setting needs
    apply(ctx, cfg)
    if log:
        log(f"autotune {key}: {cfg} from {trace}")
    cache[key] = cfg
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        json.dump(cache, open(path, "w"), indent=1, sort_keys=True)
    except OSError:
        pass
    return cfg
