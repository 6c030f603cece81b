"""Autotuner for the launch shape of the LDS-tiled a-trous kernels.

A 5x5 level's tile is 64 columns by 4 x rows lattice rows, with rows (the
lattice rows each thread computes) 1 or 2; it runs one tile per workgroup
or with persistent workgroups that prefetch their next tile, at a chosen
number of workgroups per CU.  The fused separable level's wave walks a band
of 6 or 16 output rows.  Which is fastest depends on the step (the LDS
halo grows with it and sets how many workgroups fit a CU), the storage type
and the image size, so the choice is measured: each candidate is timed with
HIP events on synthetic planes of the target size, and the fastest kept.
Results do not depend on the launch shape (the tests check that bitwise),
only the time does.

A choice is (persistent, workgroups per CU, tile rows), the per-level
fields of the frame parameters.  Choices are cached as JSON, keyed by
device, image size, storage type, filter form and level.
"""

from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import lib

# 5x5 levels: (persistent, workgroups per CU, lattice rows per thread);
# (0, 0, r) = one tile per workgroup
CANDIDATES: Sequence[Tuple[int, int, int]] = tuple(
    (per, bpc, rows) for rows in (1, 2)
    for per, bpc in ((0, 0), (1, 2), (1, 3), (1, 4), (1, 6), (1, 8)))
# fused separable levels: output rows per wave
SEP_CANDIDATES: Sequence[Tuple[int, int, int]] = ((0, 0, 6), (0, 0, 16))

_DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def _key(dev: str, W: int, H: int, dtype: torch.dtype, separable: bool, level: int) -> str:
    return f"{dev}|{W}x{H}|{str(dtype).split('.')[-1]}|{'sep' if separable else '2d'}|L{level}"


def _planes(H: int, W: int, dtype: torch.dtype, seed: int = 7):
    """Synthetic planes for timing: smooth depth and normals, noisy colour."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    ys = torch.arange(H, dtype=torch.float32)[:, None]
    xs = torch.arange(W, dtype=torch.float32)[None, :]
    z = 10.0 + 2.0 * torch.sin(0.01 * xs) * torch.cos(0.013 * ys)
    dzdx = 0.02 * torch.cos(0.01 * xs) * torch.cos(0.013 * ys)
    dzdy = -0.026 * torch.sin(0.01 * xs) * torch.sin(0.013 * ys)
    n = torch.stack([-dzdx, torch.ones_like(z), -dzdy])
    n = n / n.norm(dim=0, keepdim=True)
    c = torch.rand((3, H, W), generator=g) * 0.8
    var = torch.rand((H, W), generator=g) * 0.02
    dev = lambda t, dt=dtype: t.to(dt).cuda().contiguous()
    return (dev(c), dev(var, torch.float32),
            lib.GBuf(dev(z), dev(dzdx), dev(dzdy), dev(n)))


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(H: int, W: int, dtype: torch.dtype = torch.float32, separable: bool = False,
         levels: int = 5, params: Optional[lib.AtrousParams] = None, reps: int = 10,
         candidates: Optional[Sequence[Tuple[int, int, int]]] = None
         ) -> Tuple[List[Tuple[int, int, int]], Dict]:
    """Time every candidate for each level; returns the per-level choice and
    the measured times (ms) per level and candidate."""
    params = params or lib.AtrousParams()
    if candidates is None:
        candidates = SEP_CANDIDATES if separable else CANDIDATES
    c, var, g = _planes(H, W, dtype)
    out = torch.empty_like(c)
    vout = torch.empty_like(var)
    best, times = [], {}
    for i in range(levels):
        step = 1 << i
        last = i == levels - 1
        row = {}
        for per, bpc, rows in candidates:
            p = lib.AtrousParams(**{**params.__dict__, "persistent": per, "blocks_per_cu": bpc,
                                    "tile_rows": rows, "inv_tonemap": last})
            vo = None if last else vout
            if separable:  # the fused form (no scratch)
                fn = lambda p=p, vo=vo: lib.sv_atrous_sep(c, var, g, None, out, vo, step, p)
            else:
                fn = lambda p=p, vo=vo: lib.sv_atrous(c, var, g, out, vo, step, p)
            row[(per, bpc, rows)] = _time(fn, reps)
        times[i] = row
        best.append(min(row, key=row.get))
    return best, times


def tiles_for(H: int, W: int, dtype: torch.dtype = torch.float32, separable: bool = False,
              levels: int = 5, cache: Optional[str] = _DEFAULT_CACHE,
              retune: bool = False) -> List[Tuple[int, int, int]]:
    """Per-level launch shapes (persistent, workgroups per CU, tile rows)
    for this device and size, from the cache or measured now (and
    cached)."""
    dev = torch.cuda.get_device_name()
    keys = [_key(dev, W, H, dtype, separable, i) for i in range(levels)]
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if not retune and all(k in table and len(table[k]) == 3 for k in keys):
        return [tuple(table[k]) for k in keys]
    best, _ = tune(H, W, dtype, separable, levels)
    for k, b in zip(keys, best):
        table[k] = list(b)
    if cache:
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best
