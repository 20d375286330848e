"""The allocation-free entry point (loglike_batch_noalloc, scratch in a fixed
device array) against loglike_batch through the C ABI: two calls in a row,
the second with a smaller batch, must give the same log-likelihoods bit for
bit (same kernel, same launch shape, same FP64 band order), and requests
beyond the scratch limit are rejected."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _grid(gk, spec, mask, max_batch, rng):
    dev = torch.device("cuda:0")
    g = gk.Grid(spec, max_batch=max_batch)
    truth = W.draw_thetas(spec, 1, rng)
    maps = g.maps(torch.tensor(truth, dtype=torch.float64, device=dev))[0].cpu().numpy()
    err = W.error_maps(maps, mask)
    g.set_data(W.noisy_data(maps, err, rng), err)
    return g, truth


def _call(gk, fn, g, th):
    B, stride = th.shape
    out = torch.full((B,), float("nan"), dtype=torch.float64, device=th.device)
    stream = torch.cuda.current_stream()
    rc = fn(g.handle, ctypes.c_void_p(th.data_ptr()), B, stride, ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(stream.cuda_stream))
    assert rc == gk.GK_OK, gk.last_error()
    torch.cuda.synchronize()
    return out.cpu()


def test_noalloc_equals_loglike_batch_on_two_calls():
    import paper_2205_06819_amd as gk
    print("case: realistic cube, B = 1024 then B = 37, loglike_batch_noalloc vs loglike_batch", flush=True)
    torch.cuda.set_device(0)
    wl = W.workload("realistic")
    rng = np.random.default_rng(7101)
    g, truth = _grid(gk, wl.spec, wl.mask(), 1024, rng)
    dev = torch.device("cuda:0")
    th1 = W.draw_thetas(wl.spec, 1024, rng)
    th1[0] = truth[0]
    th1[5, 3] = 95.0                       # outside the domain: -inf on both paths
    th2 = W.draw_thetas(wl.spec, 37, rng)  # the second call is smaller
    for th_np in (th1, th2):
        th = torch.tensor(th_np, dtype=torch.float64, device=dev)
        ref = _call(gk, gk._lib.loglike_batch, g, th)
        got = _call(gk, gk._lib.loglike_batch_noalloc, g, th)
        assert torch.equal(got, ref), (got - ref).abs().max()
        assert np.isfinite(got.numpy()).sum() == len(th_np) - (1 if th_np is th1 else 0)
    assert got.numel() == 37
    g.close()


def test_noalloc_single_band_and_limit():
    import paper_2205_06819_amd as gk
    print("case: 12x10 grid (one band), then 80x80 grid with 4x4-px bands beyond the scratch limit", flush=True)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(7102)
    spec = W.GridSpec(12, 10, W.PK_50MPC, 3, 1.0, W.BULGE_HERNQUIST, 2, W.HALO_NFW)
    g, _ = _grid(gk, spec, np.ones((10, 12), bool), 64, rng)
    for bm in (1, 32):                     # one band: no tickets, no partials
        g.set_launch_shape(bm, 10, 12)
    th = torch.tensor(W.draw_thetas(spec, 64, rng), dtype=torch.float64, device=dev)
    assert torch.equal(_call(gk, gk._lib.loglike_batch_noalloc, g, th), _call(gk, gk._lib.loglike_batch, g, th))
    g.close()
    wl = W.workload("realistic")
    g, _ = _grid(gk, wl.spec, wl.mask(), 8192, rng)
    for bm in (1, 32, 512, 4096):          # 400 bands: 8192 x (4 + 8 x 400) B > 16 MiB
        g.set_launch_shape(bm, 4, 4)
    th = torch.tensor(W.draw_thetas(wl.spec, 8192, rng), dtype=torch.float64, device=dev)
    out = torch.empty(8192, dtype=torch.float64, device=dev)
    rc = gk._lib.loglike_batch_noalloc(g.handle, ctypes.c_void_p(th.data_ptr()), 8192, th.shape[1],
                                       ctypes.c_void_p(out.data_ptr()), None)
    assert rc == gk.GK_EINVAL and "scratch" in gk.last_error()
    # within the limit with the same shape: 512 x (4 + 3200) B
    assert torch.equal(_call(gk, gk._lib.loglike_batch_noalloc, g, th[:512]), _call(gk, gk._lib.loglike_batch, g, th[:512]))
    g.close()
