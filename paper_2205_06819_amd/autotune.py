"""Launch-shape autotuner.

For a grid and a batch size, times a few band shapes (pixel rows x columns
per workgroup) of the forward kernel with HIP events on the current stream
and installs the fastest with ``set_launch_shape`` (``tune``); likewise for
the gradient's adjoint kernel (``tune_adjoint``, ``set_adjoint_shape``) and
for the band policy of a many-grid launch (``tune_multi``).  The library's
own shape is always one of the candidates, so tuning never installs a slower
one.  Results of ``tune`` are cached in a JSON file keyed by everything that
changes the kernel's work: grid geometry, lattice, PSF and its mode, the
component set, the centre frame and the batch size.
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
            f"b{s.bulge}d{s.n_discs}h{s.halo}/psf{int(getattr(s, 'psf_mode', 0))}/"
            f"frame{float(getattr(s, 'frame_px_kpc', 0.0)):.6g},{float(getattr(s, 'frame_dx', 0.0)):.6g},"
            f"{float(getattr(s, 'frame_dy', 0.0)):.6g}/B{B}")


def candidates(nx: int, ny: int, B: int) -> List[Tuple[int, int]]:
    """Band shapes (rows, columns) tried by tune: whole, half and fixed-size
    splits, at most 1024 bands."""
    out = set()
    widths = sorted({nx, (nx + 1) // 2, min(nx, 64), min(nx, 32), min(nx, 16)})
    heights = sorted({ny, (ny + 1) // 2, min(ny, 32), min(ny, 16), min(ny, 8), min(ny, 4)})
    for w in widths:
        for h in heights:
            if math.ceil(nx / w) * math.ceil(ny / h) <= 1024:
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
         shapes: Optional[List[Tuple[int, int]]] = None) -> Tuple[int, int, int, float]:
    """Pick the fastest band shape and pixel rows per model phase for batches of
    th.shape[0] vectors and install it for batch sizes >= that B.  Band shapes
    are timed with the automatic row count, then the three best shapes with
    every row count.  Returns (band_h, band_w, steps, ms)."""
    B = th.shape[0]
    key = _key(grid, B)
    cache: Dict[str, list] = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache and len(cache[key]) == 4:
        h, w, st, ms = cache[key]
        try:
            grid.set_launch_shape(B, h, w, st)
            return h, w, st, ms
        except GalkinError:
            pass            # a shape this build rejects (e.g. a stale cache): tune again
    out = torch.empty(B, dtype=torch.float64, device=th.device)
    # the library's own shape for this batch size is a candidate too, so the
    # result is never slower than not tuning
    h0, w0, st0 = grid.launch_shape(B)
    grid.set_launch_shape(B, h0, w0, st0)
    timed = [(_time(grid, th, out, reps), h0, w0, st0)]
    for (h, w) in (shapes or candidates(grid.nx, grid.ny, B)):
        try:
            grid.set_launch_shape(B, h, w, 0)
        except GalkinError:
            continue
        timed.append((_time(grid, th, out, reps), h, w, 0))
    if not timed:
        raise GalkinError(-1, "no launch shape fits this grid")
    timed.sort()
    best = timed[0]
    for (_, h, w, st_t) in timed[:3]:
        for st in (1, 2, 3, 4):
            if st == st_t:
                continue
            try:
                grid.set_launch_shape(B, h, w, st)
            except GalkinError:
                continue
            ms = _time(grid, th, out, reps)
            if ms < best[0]:
                best = (ms, h, w, st)
    ms, h, w, st = best
    grid.set_launch_shape(B, h, w, st)
    if use_cache:
        cache[key] = [h, w, st, ms]
        try:
            json.dump(cache, open(CACHE, "w"), indent=1)
        except OSError:
            pass
    return h, w, st, ms


def multi_policies(n_x: int, n_y: int) -> List[Tuple[int, int]]:
    """Band shapes tried for one grid of a many-grid launch (band_w <= 64)."""
    w = min(n_x, 64)
    if n_x > 64:
        w = (n_x + 1) // 2 if (n_x + 1) // 2 <= 64 else 64
    return [(n_y, w), (min(n_y, 32), w), (min(n_y, 16), w), (min(n_y, 8), w)]


def tune_multi(grids: List[Grid], th: torch.Tensor, offsets, reps: int = 3) -> Tuple[int, int, float]:
    """Pick one band policy (index into multi_policies) and row count for all
    grids of a many-grid launch by timing the whole launch; installs it on
    every grid for its own row count.  Returns (policy, steps, ms)."""
    from . import loglike_multi
    handles = [g.handle for g in grids]
    rows = [int(offsets[k + 1]) - int(offsets[k]) for k in range(len(grids))]
    out = torch.empty(int(offsets[-1]), dtype=torch.float64, device=th.device)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for pol in range(4):
        for st in (0, 1, 2):
            try:
                for g, r in zip(grids, rows):
                    h, w = multi_policies(g.nx, g.ny)[pol]
                    g.set_launch_shape(max(1, r), h, w, st)
                loglike_multi(handles, th, offsets, out)
            except GalkinError:
                continue
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                loglike_multi(handles, th, offsets, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if best is None or ms < best[2]:
                best = (pol, st, ms)
    if best is None:
        raise GalkinError(-1, "no band policy fits every grid of this catalogue")
    pol, st, ms = best
    for g, r in zip(grids, rows):
        h, w = multi_policies(g.nx, g.ny)[pol]
        g.set_launch_shape(max(1, r), h, w, st)
    return best


def adjoint_candidates(nx: int, ny: int) -> List[Tuple[int, int, int]]:
    """Adjoint shapes (rows, columns, lattice rows per phase; 0 = automatic)
    tried by tune_adjoint: columns split evenly into bands of at most 80, 64,
    40 or 32 pixels, bands of at most 64 or 128 rows."""
    def split(n, m):
        k = (n + m - 1) // m
        return (n + k - 1) // k
    out = set()
    for wmax in (80, 64, 40, 32):
        for hmax in (64, 128):
            for rows in (0, 2, 3, 4):
                out.add((split(ny, hmax), split(nx, wmax), rows))
    return sorted(out)


def tune_adjoint(grid: Grid, th: torch.Tensor, reps: int = 2,
                 shapes: Optional[List[Tuple[int, int, int]]] = None) -> Tuple[int, int, int, float]:
    """Pick the fastest adjoint shape for gradients of batches like th by
    timing loglike_grad_batch, and install it (set_adjoint_shape).  The
    library's current shape is a candidate.  Returns (band_h, band_w, rows, ms)."""
    B = th.shape[0]
    out = torch.empty(B, dtype=torch.float64, device=th.device)
    gbuf = torch.empty(B, th.shape[1], dtype=torch.float64, device=th.device)

    def timed_grad():
        grid.loglike_grad(th, out, gbuf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            grid.loglike_grad(th, out, gbuf)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    h0, w0, r0 = grid.adjoint_shape()
    best = (timed_grad(), h0, w0, r0)
    for (h, w, r) in (shapes or adjoint_candidates(grid.nx, grid.ny)):
        try:
            grid.set_adjoint_shape(h, w, r)
        except GalkinError:
            continue
        ms = timed_grad()
        if ms < best[0]:
            best = (ms, *grid.adjoint_shape())
    ms, h, w, r = best
    grid.set_adjoint_shape(h, w, r)
    return h, w, r, ms
