"""Benchmark of the batched likelihood (and gradient) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload stress]

One step = one batched likelihood call over the whole batch of parameter
vectors of the workload.  The default workload is the largest single-GPU
configuration: the 300x300 high-resolution stress grid (5x5 lattice per pixel,
4 px FWHM PSF, bulge + 2 discs + NFW halo, 8192 parameter vectors).  Inputs
(parameters, data maps, errors) are resident in device memory before the
timed region; the timed region is K back-to-back calls bracketed by HIP
events on the stream the kernels run on.  Prints one JSON line.

Also measured: gradient evaluations/s (loglike_grad_batch over the same
batch), one HIP-graph-captured leapfrog trajectory (32 steps on the stress
grid), the plain form (the same kernels called once per parameter vector),
the roofline position of the forward and the adjoint kernel, the CPU oracle
on a bounded sample of the same workload (worker processes on the host
cores), and, as secondary keys, the realistic 80x80 IFU cube.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector (packed FMA), vendor figure
PEAK_FP32_NONPACKED = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
WORKLOAD_TEXT = {
    "realistic": "realistic IFU cube: 80x80 spaxels, ~4000 valid in an elliptical mask, "
                 "3x3 supersampling, PSF FWHM 2.5 px, bulge + inner disc + outer disc + NFW halo "
                 "(17 params), 1024 parameter vectors",
    "tiny": "tiny: 40x40 spaxels, no supersampling, PSF sigma 1.5 px, bulge + disc + NFW "
            "(13 params), 64 parameter vectors",
    "adjoint": "100x100 spaxels, 3x3 supersampling, PSF FWHM 2.5 px, 4 components (17 params), "
               "4096 parameter vectors",
    "stress": "300x300 spaxels, 5x5 supersampling, PSF FWHM 4 px, 4 components (17 params), "
              "8192 parameter vectors",
    "jaffe": "realistic IFU cube with a Jaffe bulge (Appendix B): 80x80 spaxels, 3x3 supersampling, "
             "PSF FWHM 2.5 px, Jaffe bulge + 2 discs + NFW halo (17 params), 1024 parameter vectors",
    "lw": "realistic IFU cube with the PSF applied to the luminosity-weighted moments (B, B v, "
          "B (sigma^2 + v^2), mass): 80x80 spaxels, 3x3 supersampling, PSF FWHM 2.5 px, 4 components "
          "(17 params), 1024 parameter vectors",
}


# ----------------------------------------------------------------------------
# algorithmic work of the forward pass (FP32 flops; FMA = 2, each
# transcendental / reciprocal / square root = 1)
# ----------------------------------------------------------------------------
def flops_per_point(spec) -> int:
    f = 13                                   # frame: rotate, deproject, r, cos(phi)
    if spec.bulge:
        f += 42 if spec.bulge == 1 else 40   # R, s, g and h polynomials, B, B sigma^2, mass, v_c^2
    f += 32 * spec.n_discs                   # exp, B, light sums, phi polynomial, v_c^2
    f += {0: 0, 1: 6, 2: 19}[spec.halo]      # Hernquist / NFW v_c^2
    f += 13                                  # v_int, light-weighted v, sigma, <L/M>
    if getattr(spec, "psf_mode", 0) == 1:
        f += 6                               # moments B v, B (sigma^2 + v^2), B / <L/M>
    return f


def flops_per_point_light(spec) -> int:
    """The light-only body (grids whose only valid map is B): the surface
    brightness alone, no halo or kinematics."""
    f = 7 + (5 if spec.n_discs else 0)       # rotate; deprojected radius for the discs
    if spec.bulge:
        f += 19                              # R, s, g polynomial, B
    f += 5 * spec.n_discs                    # exp and the weighted sum
    if not spec.bulge and spec.n_discs:
        f += 3                               # reference exponential
    return f + 1


def light_only(data, err) -> bool:
    """True when B is the only map with a valid pixel (the library then runs
    its light-only forward body in the log-likelihood passes)."""
    valid = np.isfinite(data) & np.isfinite(err) & (err > 0)
    return bool(valid[0].any()) and not bool(valid[1:].any())


def stencil_pad(spec) -> int:
    return int(math.floor(3.0 * spec.psf_sigma_px * spec.supersample))


def flops_per_pixel(spec, n_maps: int = 4) -> int:
    """Separable circular stencil: per map, s lattice rows of incremental
    horizontal sums (1 + 3 pad) plus (2 pad + 1) weighted pushes (2 each),
    then the residual and FP64 chi^2 term (~5); the moment ratios of the
    luminosity-weighted mode add ~7 per pixel."""
    s, pad = spec.supersample, stencil_pad(spec)
    lw = 7 if getattr(spec, "psf_mode", 0) == 1 else 0
    return n_maps * (s * (1 + 3 * pad) + 2 * (2 * pad + 1) + 5) + 1 + lw


def adjoint_tap_pairs(spec) -> int:
    """The adjoint kernel variant: horizontal tap pairs per table row (4 for a
    lag depth D = floor(2 pad / s) <= 6, else 6)."""
    return 4 if 2 * stencil_pad(spec) // spec.supersample <= 6 else 6


def flops_adjoint_per_point(spec) -> int:
    """Adjoint kernel, per needed lattice point: the point model recomputed
    with the derivatives of its special functions, its reverse sweep into the
    27 constant adjoints, and the transposed stencil (D + 1 horizontal taps of
    4 FMAs, the 1/W scaling, and the vertical group sums, 4 FMAs per lag per
    pixel column, shared by the s lattice columns of that pixel column)."""
    f = 13 + 36                               # frame: forward, reverse
    if spec.bulge == 1:
        f += 69 + 36                          # Hernquist: g, h and derivatives; reverse
    elif spec.bulge == 2:
        f += 67 + 29                          # Jaffe
    f += (43 + 29) * spec.n_discs             # exp, phi and phi'; reverse
    f += {0: 0, 1: 6 + 14, 2: 32 + 8}[spec.halo]
    f += 7 + 37                               # v_int, combination; reverse of the combination
    if getattr(spec, "psf_mode", 0) == 1:
        f += flops_per_point(spec) + 12       # moments need the forward model and their own reverse
    s, pad = spec.supersample, stencil_pad(spec)
    D = 2 * pad // s
    f += 8 * (D + 1) + 4 + round(8 * (D + 1) / s)
    return f


def needed_points(spec, mask) -> int:
    """Lattice points inside the union of the 3-sigma stencils of valid pixels."""
    s, pad = spec.supersample, stencil_pad(spec)
    sig = spec.psf_sigma_px * s
    nfy, nfx = spec.ny * s + 2 * pad, spec.nx * s + 2 * pad
    need = np.zeros((nfy, nfx), bool)
    jj, ii = np.nonzero(mask)
    h = (s - 1) // 2
    for b in range(-pad, pad + 1):
        for a in range(-pad, pad + 1):
            if a * a + b * b <= 9.0 * sig * sig:
                need[jj * s + h + pad + b, ii * s + h + pad + a] = True
    return int(need.sum())


# the sources the forward kernel is compiled from (the traffic records are
# counters of that kernel, valid only for the code they were taken on)
FWD_SOURCES = ("fwd_inst.hip", "gk_fwd.h", "gk_kern.h", "gk_device.h", "gk_tables.h")


def source_hash() -> str:
    """Hash of the forward kernel's HIP sources."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2205_06819_amd", "csrc")
    for f in FWD_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# CPU baseline: the oracle, unchanged, on a bounded sample (worker processes)
# ----------------------------------------------------------------------------
def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    spec_d, data, err, thetas = args
    import workloads as W
    from oracle import model as M
    spec = W.GridSpec(**spec_d)
    t0 = time.perf_counter()
    out = [M.loglike(spec, data, err, t) for t in thetas]
    return out, time.perf_counter() - t0


def _oracle_items_worker(items):
    """items: list of (spec dict, data, err, theta); returns (values, CPU seconds)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import workloads as W
    from oracle import model as M
    t0 = time.perf_counter()
    out = [M.loglike(W.GridSpec(**sd), d, e, t) for sd, d, e, t in items]
    return out, time.perf_counter() - t0


def _host_cores() -> int:
    """Worker processes for the oracle: the CPUs this process may run on,
    capped at 16 (the host CPU share that goes with one GPU on the
    benchmark machines)."""
    return max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                      else os.cpu_count() or 1))


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"nproc": os.cpu_count(), "affinity_cpus": aff, "cpu_model": model,
            "worker_cap": 16, "worker_cap_reason": "host CPU share of one GPU on the benchmark machines"}


def device_info() -> dict:
    """The GPU the numbers were taken on: name, compute units, memory and the
    highest shader clock level the driver lists (the peaks above assume 256
    CUs at 2.4 GHz)."""
    info = {}
    try:
        import torch
        p = torch.cuda.get_device_properties(0)
        info = {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "compute_units": p.multi_processor_count,
                "memory_gib": round(p.total_memory / 2 ** 30, 1)}
    except Exception as exc:  # report, do not hide
        info = {"error": str(exc)}
    sclk = None
    try:
        import glob
        for f in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
            levels = [int(l.split(":")[1].strip().lower().rstrip("mhz").strip()) for l in open(f) if ":" in l]
            if levels:
                sclk = max(levels) if sclk is None else max(sclk, max(levels))
    except (OSError, ValueError):
        pass
    info["max_sclk_mhz"] = sclk
    return info


def cpu_baseline(spec, data, err, thetas, budget_s: float = 20.0, min_n: int = 0):
    """The oracle's log-likelihood on a bounded sample of the batch: about
    budget_s of CPU work per worker, at least min_n vectors."""
    import dataclasses
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    cores = _host_cores()
    spec_d = dataclasses.asdict(spec)
    # calibrate on one vector in this process, then size the sample
    sys.path.insert(0, ROOT)
    from oracle import model as M
    t0 = time.perf_counter()
    M.loglike(spec, data, err, thetas[0])
    per = time.perf_counter() - t0
    n = int(max(cores, min(len(thetas), budget_s / max(per, 1e-4))))
    n = (n // cores) * cores or cores
    n = max(n, min_n)
    workers = min(cores, n)
    sample = thetas[:n]
    chunks = [sample[i::workers] for i in range(workers)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_worker, [(spec_d, data, err, c) for c in chunks]))
    wall = time.perf_counter() - t0
    cpu_work = sum(r[1] for r in res)
    vals = []
    for i in range(n):
        vals.append(res[i % workers][0][i // workers])
    return {"value": n / wall, "unit": "likelihood evals/s", "cores": workers, "kind": "oracle",
            "sample": f"first {n} parameter vectors of the benchmark batch, {workers} worker processes "
                      f"(one vector per worker and round), {cpu_work:.1f} s of CPU work in {wall:.1f} s "
                      f"wall ({cpu_work / n:.2f} s per vector per core); the rate is n / wall and "
                      f"extrapolates linearly in the batch (vectors are independent)",
            "per_core_evals_per_s": n / cpu_work, **host_info()}, np.array(vals), n


# ----------------------------------------------------------------------------
# many galaxies in one launch (loglike_multi)
# ----------------------------------------------------------------------------
def bench_uneven(args):
    import dataclasses
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    import torch
    import workloads as W
    import paper_2205_06819_amd as gk

    wls = W.uneven_galaxies()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stride = max(w.spec.n_params for w in wls)
    grids, datas, rows = [], [], []
    for w in wls:
        rng = np.random.default_rng(w.seed)
        g = gk.Grid(w.spec, max_batch=w.batch)
        truth = W.draw_thetas(w.spec, 1, rng)
        maps = g.maps(torch.tensor(truth, dtype=torch.float64, device=dev))[0].cpu().numpy()
        mask = w.mask()
        err = W.error_maps(maps, mask)
        data = W.noisy_data(maps, err, rng)
        g.set_data(data, err)
        th = np.zeros((w.batch, stride))
        th[:, :w.spec.n_params] = W.draw_thetas(w.spec, w.batch, rng)
        grids.append(g)
        datas.append((data, err, mask))
        rows.append(th)
    offs = np.concatenate([[0], np.cumsum([w.batch for w in wls])]).astype(np.int32)
    th = torch.tensor(np.vstack(rows), device=dev)
    total = int(offs[-1])
    out = torch.empty(total, dtype=torch.float64, device=dev)
    handles = [g.handle for g in grids]
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_tune:
        from paper_2205_06819_amd import autotune
        tuned = autotune.tune_multi(grids, th, offs, reps=2)
    gk.loglike_multi(handles, th, offs, out)              # builds the work plan
    for _ in range(args.warmup):
        gk.loglike_multi(handles, th, offs, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        gk.loglike_multi(handles, th, offs, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    evals = total / (ms_step * 1e-3)
    multi_vals = out.cpu().numpy()
    # the same work as one launch per galaxy
    outs = [out[offs[k]:offs[k + 1]] for k in range(len(wls))]
    ths = [th[offs[k]:offs[k + 1], :wls[k].spec.n_params].contiguous() for k in range(len(wls))]
    for k, g in enumerate(grids):
        g.loglike(ths[k], outs[k])
    torch.cuda.synchronize()
    e0.record(stream)
    reps = max(1, args.steps // 4)
    for _ in range(reps):
        for k, g in enumerate(grids):
            g.loglike(ths[k], outs[k])
    e1.record(stream)
    torch.cuda.synchronize()
    per_grid_evals = reps * total / (e0.elapsed_time(e1) * 1e-3)
    assert np.allclose(out.cpu().numpy(), multi_vals, rtol=1e-9, atol=1e-6)

    flop = 0
    for w, (_, _, mask), r in zip(wls, datas, rows):
        flop += len(r) * (needed_points(w.spec, mask) * flops_per_point(w.spec)
                          + int(mask.sum()) * flops_per_pixel(w.spec))
    achieved = flop / (ms_step * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "frac_of_nonpacked_fp32": round(achieved / PEAK_FP32_NONPACKED, 4),
            "kernel": "gk::multi_kernel", "flop_per_step": flop}

    cpu = None
    if not args.no_cpu:
        cores = _host_cores()
        items, idx = [], []
        t_est = 0.0
        from oracle import model as M
        k = 0
        while t_est < args.cpu_budget * cores and k < 4 * len(wls):
            gi, ri = k % len(wls), k // len(wls)
            w = wls[gi]
            data, err, _ = datas[gi]
            items.append((dataclasses.asdict(w.spec), data.astype(np.float32).astype(np.float64),
                          err.astype(np.float32).astype(np.float64), rows[gi][ri, :w.spec.n_params]))
            idx.append(int(offs[gi]) + ri)
            t_est += 0.07 * (w.spec.nx * w.spec.ny) / 6400.0 * (w.spec.n_params / 17.0) * 3
            k += 1
        chunks = [items[i::cores] for i in range(cores)]
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_items_worker, chunks))
        wall = time.perf_counter() - t0
        vals = np.array([res[i % cores][0][i // cores] for i in range(len(items))])
        work = sum(r[1] for r in res)
        rel = np.abs(vals - multi_vals[idx]) / np.maximum(1.0, np.abs(vals))
        cpu = {"value": round(len(items) / wall, 3), "unit": "likelihood evals/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{len(items)} (galaxy, parameter vector) pairs, galaxies in order, "
                         f"{cores} worker processes, {work:.1f} s CPU in {wall:.1f} s wall",
               "max_rel_diff_vs_gpu": float(rel.max())}
    line = {
        "metric": "likelihood evals/s and gradient evals/s (params×spaxels/s), batched vs plain",
        "value": round(evals, 1), "unit": "likelihood evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256 galaxies, square grids of side U{30..120}, 2-4 components, "
                               "3x3 supersampling, PSF FWHM 2.5 px, 128 parameter vectors each, "
                               "one launch", "batch": total, "galaxies": len(wls),
                   "band_policy": list(tuned[:2]) if tuned else None},
        "one_launch_per_galaxy_evals_per_s": round(per_grid_evals, 1),
        "speedup_vs_launch_per_galaxy": round(evals / per_grid_evals, 3),
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    for g in grids:
        g.close()


def time_hmc(gk, grid, th, n_steps: int, eps: float = 1e-9) -> dict:
    """One leapfrog trajectory of n_steps for every row, captured once in a
    HIP graph and replayed once (a one-step eager trajectory first loads the
    kernels; the start is restored outside the timing).  The rows are prior
    draws far from the data's truth, where |d logL / d theta| reaches ~1e10:
    the small step keeps every row inside the valid domain, so no row is
    frozen and every step does the full work."""
    import torch
    B, P = th.shape
    dev = th.device
    g = torch.Generator(device="cpu").manual_seed(5)
    mom0 = torch.randn(B, P, generator=g, dtype=torch.float64).to(dev)
    theta, mom = th.clone(), mom0.clone()
    inv_mass = torch.ones(P, dtype=torch.float64, device=dev)
    logL = torch.empty(B, dtype=torch.float64, device=dev)
    grad = torch.empty(B, P, dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gk.hmc_leapfrog(grid.handle, theta, mom, inv_mass, eps, 1, logL, grad)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gk.hmc_leapfrog(grid.handle, theta, mom, inv_mass, eps, n_steps, logL, grad)
    theta.copy_(th)
    mom.copy_(mom0)
    torch.cuda.synchronize()
    print(f"hmc: graph of {n_steps} leapfrog steps captured, replaying", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    frozen = int((~torch.isfinite(logL)).sum())
    del graph
    return {"hmc_steps": n_steps, "ms_per_hmc_trajectory": ms,
            "hmc_grad_evals_per_s": B * (n_steps + 1) / (ms * 1e-3), "hmc_rows_frozen": frozen}


# ----------------------------------------------------------------------------
# nested sampling driven by the batched likelihood (throughput of the sampler)
# ----------------------------------------------------------------------------
def bench_nested(args):
    import torch
    import workloads as W
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd.nested import nested_sampling

    wl = W.workload("realistic")
    spec = wl.spec
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rng = np.random.default_rng(wl.seed)
    mask = wl.mask()
    truth = W.draw_thetas(spec, 1, rng)
    n_live, k = 8192, 1024
    grid = gk.Grid(spec, max_batch=n_live)
    maps = grid.maps(torch.tensor(truth, dtype=torch.float64, device=dev))[0].cpu().numpy()
    err = W.error_maps(maps, mask)
    grid.set_data(W.noisy_data(maps, err, rng), err)
    bounds = W.prior_bounds(spec)
    lo, hi = bounds[:, 0], bounds[:, 1]

    def loglike(th):
        return grid.loglike(th.contiguous())

    iters = max(2, args.steps)
    rates = {}
    for mode in ("eager", "graph"):
        g = torch.Generator(device=dev).manual_seed(7)
        nested_sampling(loglike, lo, hi, n_live=n_live, k=k, walk_steps=2, max_iter=2, device=dev, generator=g,
                        graph=mode == "graph")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = nested_sampling(loglike, lo, hi, n_live=n_live, k=k, walk_steps=10, max_iter=iters, device=dev,
                              generator=g, graph=mode == "graph", check_every=8)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rates[mode] = (res.n_like / wall, wall / res.n_iter * 1e3, res.n_like)
        print(f"bench: nested sampling ({mode}) {rates[mode][0]:.0f} likelihood evals/s", file=sys.stderr, flush=True)
    line = {
        "metric": "likelihood evals/s and gradient evals/s (params×spaxels/s), batched vs plain",
        "value": round(rates["graph"][0], 1), "unit": "likelihood evals/s",
        "n_gpus": 1, "steps": iters, "warmup": 2, "ms_per_step": round(rates["graph"][1], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched nested sampling (Sec. 2.5) on the realistic IFU cube: 8192 live "
                               "points over the 17-parameter prior box, 1024 replaced per iteration by "
                               "10-step constrained random walks (each step one 1024-vector likelihood "
                               "launch); each iteration captured once in a HIP graph and replayed; "
                               "throughput inside the sampler, the run's setup included",
                   "live_points": n_live, "replaced_per_iteration": k, "iterations": iters},
        "likelihood_evaluations": rates["graph"][2],
        "eager_evals_per_s": round(rates["eager"][0], 1),
        "eager_ms_per_iteration": round(rates["eager"][1], 3),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    grid.close()


# ----------------------------------------------------------------------------
# one galaxy on two pixelisations: joint likelihood over two grids
# ----------------------------------------------------------------------------
def bench_multires(args):
    import torch
    import workloads as W
    import paper_2205_06819_amd as gk

    wp, wk = W.multires_pair()
    B = wp.batch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rng = np.random.default_rng(wp.seed)
    truth = W.draw_thetas(wk.spec, 1, rng)
    thetas = W.draw_thetas(wk.spec, B, rng)
    th = torch.tensor(thetas, dtype=torch.float64, device=dev)
    t0 = torch.tensor(truth, dtype=torch.float64, device=dev)
    grids, datas, carried = [], [], [(0,), (1, 2, 3)]
    for w, maps_kept in zip((wp, wk), carried):
        g = gk.Grid(w.spec, max_batch=B)
        maps = g.maps(t0)[0].cpu().numpy()
        err = W.error_maps(maps, w.mask())
        for m in range(4):
            if m not in maps_kept:
                err[m] = 0.0          # this pixelisation does not carry map m
        data = W.noisy_data(maps, err, rng)
        g.set_data(data, err)
        grids.append(g)
        datas.append((data, err))
    hs = [g.handle for g in grids]
    out = torch.empty(B, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tuned = None
    if args.tune:
        from paper_2205_06819_amd import autotune
        tuned = [list(autotune.tune(g, th, reps=2)[:3]) for g in grids]

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_step = timed(lambda: gk.loglike_joint(hs, th, out), args.steps)
    logl = out.cpu().numpy()
    # per-grid launches (the same kernels the joint call enqueues), for the roofline
    per = [timed(lambda g=g: g.loglike(th, out), args.steps) for g in grids]
    grad_info = {}
    if not args.no_grad:
        gbuf = torch.empty(B, th.shape[1], dtype=torch.float64, device=dev)
        msg = timed(lambda: gk.loglike_joint(hs, th, out, grad=gbuf), max(1, args.steps // 2))
        grad_info = {"grad_ms_per_step": round(msg, 4), "grad_evals_per_s": round(B / (msg * 1e-3), 1)}
    flops, light = [], []
    for w, maps_kept, (d_w, e_w) in zip((wp, wk), carried, datas):
        n_need = needed_points(w.spec, w.mask())
        lo = light_only(d_w, e_w) and not w.spec.psf_mode
        light.append(int(lo))
        fp = flops_per_point_light(w.spec) if lo else flops_per_point(w.spec)
        flops.append(n_need * fp + int(w.mask().sum()) * flops_per_pixel(w.spec, len(maps_kept)))
    dom = int(np.argmax(per))
    wd = (wp, wk)[dom]
    achieved = flops[dom] * B / (per[dom] * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": f"gk::fwd_kernel<{wd.spec.bulge},{wd.spec.n_discs},{0 if light[dom] else wd.spec.halo},0,"
                      f"{wd.spec.psf_mode},{light[dom]}> ({wd.name})",
            "flop_per_vector": flops[dom], "per_grid_ms": [round(x, 4) for x in per]}
    cpu = None
    if not args.no_cpu:
        # the oracle's joint likelihood on a bounded sample of the batch
        from oracle import model as M
        n, t_start = 0, time.perf_counter()
        specs = [wp.spec, wk.spec]
        dd = [d.astype(np.float32).astype(np.float64) for d, _ in datas]
        ee = [e.astype(np.float32).astype(np.float64) for _, e in datas]
        vals = []
        while n < B and time.perf_counter() - t_start < args.cpu_budget:
            vals.append(M.loglike_joint(specs, dd, ee, thetas[n]))
            n += 1
        wall = time.perf_counter() - t_start
        rel = np.abs(np.array(vals) - logl[:n]) / np.maximum(1.0, np.abs(np.array(vals)))
        cpu = {"value": round(n / wall, 3), "unit": "likelihood evals/s", "cores": 1, "kind": "oracle",
               "sample": f"first {n} of the {B} parameter vectors, one process",
               "max_rel_diff_vs_gpu": float(rel.max())}
    line = {
        "metric": "likelihood evals/s and gradient evals/s (params×spaxels/s), batched vs plain",
        "value": round(B / (ms_step * 1e-3), 1), "unit": "likelihood evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one galaxy on two pixelisations (joint likelihood): B on 160x160 pixels "
                               "of 0.25 arcsec, no supersampling, PSF FWHM 4 px; v, sigma, M/L on the "
                               "realistic 80x80 IFU grid (3x3 supersampling, PSF FWHM 2.5 px); 4 "
                               "components (17 params), 1024 parameter vectors",
                   "batch": B, "launch_shapes": tuned or "library default"},
        **grad_info,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    for g in grids:
        g.close()


# ----------------------------------------------------------------------------
# data preparation (colour-M/L maps): an HBM-bound elementwise kernel
# ----------------------------------------------------------------------------
def bench_prep(args):
    import torch
    import paper_2205_06819_amd as gk
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = 4096 * 4096
    g = torch.Generator(device=dev).manual_seed(3)
    mb = 15 + 7 * torch.rand(n, device=dev, generator=g)
    mg = mb - 1.8 * torch.rand(n, device=dev, generator=g) + 0.2
    eb = 0.01 + 0.3 * torch.rand(n, device=dev, generator=g)
    eg = 0.01 + 0.3 * torch.rand(n, device=dev, generator=g)
    ml = torch.empty_like(mb)
    err = torch.empty_like(mb)
    stream = torch.cuda.current_stream()

    def call():
        gk._check(gk._lib.ml_from_colour(mb.data_ptr(), mg.data_ptr(), eb.data_ptr(), eg.data_ptr(), n,
                                         -0.70, 0.89, 0.07, ml.data_ptr(), err.data_ptr(), gk._stream(stream)))
    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    byts = 24 * n                                  # 4 float32 maps in, 2 out
    gbs = byts / (ms * 1e-3) / 1e9
    line = {
        "metric": "likelihood evals/s and gradient evals/s (params×spaxels/s), batched vs plain",
        "value": round(n / (ms * 1e-3), 1), "unit": "pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "colour-M/L data preparation (Sec. 2.5.1 relation, Appendix C errors) on a "
                               "4096x4096 map", "pixels": n},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(gbs / 8000.0, 4), "traffic": None, "kernel": "gk::ml_colour_kernel4",
                     "bytes_per_launch": byts},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


# ----------------------------------------------------------------------------
# one grid, one batch: forward, gradient, plain form, roofline, oracle
# ----------------------------------------------------------------------------
def _events(stream):
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_calls(fn, steps, warmup, stream):
    """Mean milliseconds per call of fn over `steps` calls (after `warmup`),
    HIP events recorded on the stream the calls enqueue on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(stream)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def run_single(args, name, *, steps, warmup, grad_steps, hmc_steps, plain, with_cpu, cpu_min_n=0):
    import torch
    import workloads as W
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd import autotune

    wl = W.workload(name)
    spec, B = wl.spec, wl.batch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rng = np.random.default_rng(wl.seed)
    mask = wl.mask()
    truth = W.draw_thetas(spec, 1, rng)
    thetas = W.draw_thetas(spec, B, rng)
    grid = gk.Grid(spec, max_batch=B)
    # synthetic data: the model at a seeded truth (this GPU path) plus seeded noise
    maps = grid.maps(torch.tensor(truth, dtype=torch.float64, device=dev))[0].cpu().numpy()
    err = W.error_maps(maps, mask)
    data = W.noisy_data(maps, err, rng)
    grid.set_data(data, err)
    th = torch.tensor(thetas, dtype=torch.float64, device=dev)
    out = torch.empty(B, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    print(f"bench: {name} grid ready ({spec.nx}x{spec.ny}, s = {spec.supersample}, B = {B})",
          file=sys.stderr, flush=True)

    tuned = None
    if args.tune:
        tuned = autotune.tune(grid, th, reps=2)
    # ---- batched forward (one launch of the forward kernel per step)
    ms_step = _time_calls(lambda: grid.loglike(th, out), steps, warmup, stream)
    evals = B / (ms_step * 1e-3)
    logl_gpu = out.cpu().numpy()
    print(f"bench: {name} forward {ms_step:.3f} ms per step", file=sys.stderr, flush=True)

    # ---- gradient (forward kernel in its adjoint-seed mode + the adjoint kernel)
    grad_info, ms_grad = {}, None
    if grad_steps > 0:
        gbuf = torch.empty(B, th.shape[1], dtype=torch.float64, device=dev)
        ms_grad = _time_calls(lambda: grid.loglike_grad(th, out, gbuf), grad_steps, 1, stream)
        grad_info = {"grad_evals_per_s": round(B / (ms_grad * 1e-3), 1), "ms_per_grad_step": round(ms_grad, 4),
                     "adjoint_launch_shape": list(grid.adjoint_shape())}
        print(f"bench: {name} gradient {ms_grad:.3f} ms per step", file=sys.stderr, flush=True)
        if hmc_steps > 0:
            h = time_hmc(gk, grid, th, hmc_steps)
            grad_info.update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in h.items()})

    # ---- plain form: one call (one launch sequence) per parameter vector
    n_plain = min(plain, B)
    one = [th[i:i + 1] for i in range(n_plain)]
    outs = [torch.empty(1, dtype=torch.float64, device=dev) for _ in range(n_plain)]

    def plain_loop():
        for i in range(n_plain):
            grid.loglike(one[i], outs[i])
    plain_loop_evals = n_plain / (_time_calls(plain_loop, 1, 1, stream) * 1e-3)
    plain_vals = torch.cat(outs).cpu().numpy()
    assert np.allclose(plain_vals, logl_gpu[:n_plain], rtol=1e-9, atol=1e-6)
    # the same per-vector calls captured once in a HIP graph (no host overhead per call)
    plain_graph_evals = None
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plain_loop()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plain_loop()
        plain_graph_evals = n_plain / (_time_calls(graph.replay, 3, 1, stream) * 1e-3)
        assert np.allclose(torch.cat(outs).cpu().numpy(), logl_gpu[:n_plain], rtol=1e-9, atol=1e-6)
        del graph
    except Exception as exc:  # report, do not hide
        print(f"plain-graph timing skipped: {exc}", file=sys.stderr)
    plain_evals = max(plain_loop_evals, plain_graph_evals or 0.0)

    # ---- roofline: forward kernel (one launch per step) and adjoint kernel
    n_need = needed_points(spec, mask)
    n_valid = int(mask.sum())
    flop_theta = n_need * flops_per_point(spec) + n_valid * flops_per_pixel(spec)
    achieved = flop_theta * B / (ms_step * 1e-3) / 1e12
    traffic = None
    shape = list(tuned[:3]) if tuned else None
    tpath = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if os.path.exists(tpath):
        try:
            t = json.load(open(tpath))
            # counters are valid only for this kernel source and launch shape
            if t.get("source_hash") == source_hash() and t.get("launch_shape") == shape:
                traffic = t.get("bytes_per_launch")
        except (OSError, ValueError):
            pass
    lw = spec.psf_mode
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "frac_of_nonpacked_fp32": round(achieved / PEAK_FP32_NONPACKED, 4),
            "kernel": f"gk::fwd_kernel<{spec.bulge},{spec.n_discs},{spec.halo},0,{lw},0>",
            "kernel_ms": round(ms_step, 4),
            "flop_per_vector": flop_theta,
            "per_unit": {"lattice_points": n_need, "flop_per_point": flops_per_point(spec),
                         "valid_spaxels": n_valid, "flop_per_spaxel": flops_per_pixel(spec)}}
    roof_adj = None
    if ms_grad is not None:
        # the gradient step is the forward kernel in its seed mode (the forward
        # plus 16 B of stores per pixel) followed by the adjoint kernel
        ms_adj = ms_grad - ms_step
        fa = flops_adjoint_per_point(spec)
        a_ach = n_need * fa * B / (ms_adj * 1e-3) / 1e12
        roof_adj = {"bound": "alu", "achieved": round(a_ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(a_ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
                    "frac_of_nonpacked_fp32": round(a_ach / PEAK_FP32_NONPACKED, 4),
                    "kernel": f"gk::adj_kernel<{spec.bulge},{spec.n_discs},{spec.halo},{lw},{adjoint_tap_pairs(spec)},0>",
                    "kernel_ms": round(ms_adj, 4),
                    "kernel_ms_from": "gradient step minus forward step (HIP events)",
                    "flop_per_vector": n_need * fa,
                    "per_unit": {"lattice_points": n_need, "flop_per_point": fa}}

    # ---- CPU baseline (oracle, unchanged)
    cpu = None
    if with_cpu:
        print(f"bench: {name} oracle leg", file=sys.stderr, flush=True)
        cpu, cvals, n = cpu_baseline(spec, data.astype(np.float32).astype(np.float64),
                                     err.astype(np.float32).astype(np.float64), thetas,
                                     args.cpu_budget, cpu_min_n)
        rel = np.abs(cvals - logl_gpu[:n]) / np.maximum(1.0, np.abs(cvals))
        cpu["max_rel_diff_vs_gpu"] = float(rel.max())
    grid.close()
    P = spec.n_params
    spax = spec.nx * spec.ny
    res = {
        "value": round(evals, 1), "ms_per_step": round(ms_step, 4),
        "config": {"workload": WORKLOAD_TEXT.get(name, name), "batch": B,
                   "spaxels": spax, "valid_spaxels": n_valid, "params": P,
                   "supersample": spec.supersample, "psf_sigma_px": round(spec.psf_sigma_px, 5),
                   "launch_shape": list(tuned[:3]) if tuned else "library default"},
        "params_x_spaxels_per_s": round(evals * P * spax, 1),
        "fine_points_per_s": round(evals * n_need, 1),
        "plain_evals_per_s": round(plain_evals, 1),
        "plain_host_loop_evals_per_s": round(plain_loop_evals, 1),
        "plain_graph_evals_per_s": round(plain_graph_evals, 1) if plain_graph_evals else None,
        "speedup_vs_plain": round(evals / plain_evals, 2),
        **grad_info,
        "roofline": roof, "roofline_adjoint": roof_adj, "cpu_baseline": cpu,
    }
    if "grad_evals_per_s" in grad_info:
        res["grad_params_x_spaxels_per_s"] = round(grad_info["grad_evals_per_s"] * P * spax, 1)
    return res


# ----------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="stress",
                    help="stress (default: 300x300, 5x5 lattice, B = 8192), realistic, tiny, adjoint, jaffe, "
                         "lw (luminosity-weighted PSF), uneven (many galaxies), multires (one galaxy on two "
                         "pixelisations), nested (the nested sampler driving the likelihood) or prep "
                         "(colour-M/L maps)")
    ap.add_argument("--hmc-steps", type=int, default=None,
                    help="time one graph-captured leapfrog trajectory of this many steps "
                         "(default: 32 on the stress workload, none elsewhere)")
    ap.add_argument("--grad-steps", type=int, default=None,
                    help="gradient calls timed (default: 3 on the stress workload, --steps elsewhere)")
    ap.add_argument("--plain", type=int, default=256, help="number of single-vector calls timed")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="stress workload: skip the secondary realistic-cube measurement")
    ap.add_argument("--no-tune", action="store_true", help="many-galaxy workload: skip the band-policy search")
    ap.add_argument("--tune", action="store_true",
                    help="single-grid workloads: autotune the launch shape (default: the library's defaults)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run one 512 MiB device copy (the traffic-counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(every (galaxy, parameter vector) pair is independent; see the design notes "
              "on sharding). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.copy_calib:
        import torch
        src_buf = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        print("copied 512 MiB", flush=True)
        return
    if args.workload == "uneven":
        return bench_uneven(args)
    if args.workload == "nested":
        return bench_nested(args)
    if args.workload == "prep":
        return bench_prep(args)
    if args.workload == "multires":
        return bench_multires(args)

    stress = args.workload == "stress"
    hmc = args.hmc_steps if args.hmc_steps is not None else (32 if stress else 0)
    gsteps = 0 if args.no_grad else (args.grad_steps if args.grad_steps is not None else (3 if stress else args.steps))
    res = run_single(args, args.workload, steps=args.steps, warmup=args.warmup, grad_steps=gsteps,
                     hmc_steps=hmc, plain=args.plain, with_cpu=not args.no_cpu,
                     cpu_min_n=8 if stress else 0)
    secondary = None
    if stress and not args.no_secondary:
        r2 = run_single(args, "realistic", steps=args.steps, warmup=args.warmup,
                        grad_steps=0 if args.no_grad else args.steps, hmc_steps=0, plain=args.plain,
                        with_cpu=False)
        secondary = {"realistic": {k: r2[k] for k in (
            "value", "ms_per_step", "config", "fine_points_per_s", "plain_evals_per_s", "speedup_vs_plain",
            "grad_evals_per_s", "ms_per_grad_step", "roofline", "roofline_adjoint") if k in r2}}
    line = {
        "metric": "likelihood evals/s and gradient evals/s (params×spaxels/s), batched vs plain",
        "value": res.pop("value"),
        "unit": "likelihood evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        **res,
    }
    if secondary:
        line["secondary"] = secondary
    line["device"] = device_info()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
