"""Launch-shape autotuner.

For a grid and a batch size, times a few band shapes (pixel rows x columns
per workgroup) of the forward kernel with HIP events on the current stream
and installs the fastest with ``set_launch_shape``.  Results are cached in a
JSON file keyed by the grid geometry, component set and batch size.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Tuple

import torch

from . import Grid, GalkinError

CACHE = os.environ.get("GALKIN_TUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), ".tune_cache.json"))


def _key(grid: Grid, B: int) -> str:
    s = grid.spec
    return (f"{s.nx}x{s.ny}/s{s.supersample}/sig{float(s.psf_sigma_px):.5f}/"
            f"b{s.bulge}d{s.n_discs}h{s.halo}/B{B}")


def candidates(nx: int, ny: int, B: int, n_cu: int = 256) -> List[Tuple[int, int]]:
    out = set()
    widths = sorted({nx, (nx + 1) // 2, min(nx, 64), min(nx, 32), min(nx, 16)})
    heights = sorted({ny, (ny + 1) // 2, min(ny, 32), min(ny, 16), min(ny, 8), min(ny, 4)})
    for w in widths:
        for h in heights:
            nb = math.ceil(nx / w) * math.ceil(ny / h)
            if nb > 1024:
                continue
            # enough workgroups to fill the chip, not far more bands than needed
            if B * nb < n_cu and nb < 1024:
                pass
            out.add((h, w))
    return sorted(out)


def _time(grid: Grid, th: torch.Tensor, out: torch.Tensor, reps: int) -> float:
    grid.loglike(th, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        grid.loglike(th, out)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(grid: Grid, th: torch.Tensor, reps: int = 3, use_cache: bool = True,
         shapes: Optional[List[Tuple[int, int]]] = None) -> Tuple[int, int, float]:
    """Pick the fastest band shape for batches of th.shape[0] vectors and install
    it for batch sizes >= that B.  Returns (band_h, band_w, ms)."""
    B = th.shape[0]
    key = _key(grid, B)
    cache: Dict[str, list] = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        h, w, ms = cache[key]
        grid.set_launch_shape(B, h, w)
        return h, w, ms
    out = torch.empty(B, dtype=torch.float64, device=th.device)
    best = None
    for (h, w) in (shapes or candidates(grid.nx, grid.ny, B)):
        try:
            grid.set_launch_shape(B, h, w)
        except GalkinError:
            continue
        ms = _time(grid, th, out, reps)
        if best is None or ms < best[2]:
            best = (h, w, ms)
    grid.set_launch_shape(B, best[0], best[1])
    if use_cache:
        cache[key] = list(best)
        try:
            json.dump(cache, open(CACHE, "w"), indent=1)
        except OSError:
            pass
    return best
