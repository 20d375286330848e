"""Host logic of bench.py (no GPU): the one-GPU contract and the algorithmic
work counts that the roofline figures divide by."""
import os
import subprocess
import sys

import numpy as np

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        e = dict(os.environ, **env)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True,
                           text=True, env=e, timeout=120)
        assert r.returncode == 2, (args, env, r.stdout, r.stderr)
        assert "one GPU" in r.stderr
        assert r.stdout.strip() == ""


def test_realistic_work_counts():
    wl = W.workload("realistic")
    spec, mask = wl.spec, wl.mask()
    assert int(mask.sum()) == 4008
    # frame 13 + Hernquist bulge 42 + 2 discs x 32 + NFW 19 + combination 13
    assert bench.flops_per_point(spec) == 151
    assert bench.stencil_pad(spec) == 9
    # 4 maps x [s (1 + 3 pad) + 2 (2 pad + 1) + 5] + 1 at s = 3, pad = 9
    assert bench.flops_per_pixel(spec) == 4 * (3 * 28 + 38 + 5) + 1 == 509
    assert bench.needed_points(spec, mask) == 42116


def test_needed_points_by_brute_force():
    """The union of the valid pixels' 3-sigma lattice discs, counted point by
    point on a small grid."""
    spec = W.GridSpec(9, 7, 0.2, 3, 0.8, 1, 1, W.HALO_NFW)
    mask = W.elliptical_mask(9, 7, 3.5, 2.5)
    s, pad = spec.supersample, bench.stencil_pad(spec)
    r2 = 9.0 * (spec.psf_sigma_px * s) ** 2
    pts = set()
    for j, i in zip(*np.nonzero(mask)):
        cy, cx = j * s + (s - 1) // 2 + pad, i * s + (s - 1) // 2 + pad
        for b in range(-pad, pad + 1):
            for a in range(-pad, pad + 1):
                if a * a + b * b <= r2:
                    pts.add((cy + b, cx + a))
    assert bench.needed_points(spec, mask) == len(pts)


def test_luminosity_weighted_and_single_map_counts():
    lw = W.workload("lw").spec
    assert bench.flops_per_point(lw) == 151 + 6
    assert bench.flops_per_pixel(lw) == 509 + 7
    wp, _ = W.multires_pair()
    assert bench.flops_per_pixel(wp.spec, 1) == 1 * (1 * (1 + 3 * 5) + 2 * 11 + 5) + 1


def test_adjoint_work_counts():
    """Per needed lattice point: frame 49, Hernquist bulge 105, two discs 2 x 72,
    NFW 40, combination 44 (= 382), plus the transposed stencil 8 (D + 1) + 4
    + 8 (D + 1) / s."""
    spec = W.workload("realistic").spec          # s = 3, pad = 9, D = 6
    assert bench.flops_adjoint_per_point(spec) == 382 + 56 + 4 + 19
    st = W.workload("stress").spec               # s = 5, pad = 25, D = 10
    assert bench.stencil_pad(st) == 25
    assert bench.flops_adjoint_per_point(st) == 382 + 88 + 4 + 18
    lw = W.workload("lw").spec
    assert bench.flops_adjoint_per_point(lw) == 382 + 157 + 12 + 56 + 4 + 19


def test_traffic_records_match_the_forward_sources():
    """The committed HBM-traffic records (from the FETCH_SIZE / WRITE_SIZE
    counters) are keyed to the forward kernel's sources: the bench line only
    reports them while the hash still matches, so a record left behind by a
    kernel change shows up here, and its byte count follows from its raw
    counters and calibration scales."""
    import json
    for name in ("stress", "realistic"):
        with open(os.path.join(ROOT, "profiles", f"traffic_{name}.json")) as f:
            t = json.load(f)
        assert t["source_hash"] == bench.source_hash(), f"traffic_{name}.json is stale: re-run the counters"
        assert tuple(t["source_files"]) == tuple(bench.FWD_SOURCES)
        got = t["fetch_size_kib_raw"] * 1024 * t["fetch_scale"] + t["write_size_kib_raw"] * 1024 * t["write_scale"]
        assert abs(got - t["bytes_per_launch"]) <= 1e-3 * t["bytes_per_launch"]
