"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "galkin.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("create_grid", "set_data", "loglike_batch", "loglike_grad_batch", "eval_maps",
              "n_params", "destroy_grid", "loglike_multi", "last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2205_06819_amd as gk
    lib = ctypes.CDLL(gk.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) <= set(gk.EXPORTS)


def test_argument_errors_without_device():
    import paper_2205_06819_amd as gk
    lib = gk._lib
    h = ctypes.c_void_p()
    assert lib.create_grid(None, 4, ctypes.byref(h)) == gk.GK_EINVAL
    assert "NULL" in gk.last_error()
    bad = [dict(nx=0), dict(supersample=2), dict(supersample=0), dict(psf_sigma_px=-1.0),
           dict(n_discs=3), dict(halo=5), dict(bulge=0, n_discs=0), dict(pixel_kpc=0.0), dict(bulge=3),
           dict(psf_mode=2), dict(psf_mode=-1), dict(frame_px_kpc=-0.1), dict(frame_dx=float("nan")),
           dict(frame_dy=float("inf"))]
    for over in bad:
        d = dict(nx=10, ny=10, pixel_kpc=0.1, supersample=3, psf_sigma_px=1.0, bulge=1,
                 n_discs=1, halo=2, hubble_h=0.7)
        d.update(over)
        desc = gk.GridDesc(**d)
        assert lib.create_grid(ctypes.byref(desc), 4, ctypes.byref(h)) == gk.GK_EINVAL, over
    desc = gk.GridDesc(10, 10, 0.1, 3, 1.0, 1, 1, 2, 0.7)
    assert lib.create_grid(ctypes.byref(desc), 0, ctypes.byref(h)) == gk.GK_EINVAL
    assert lib.n_params(None) == gk.GK_EINVAL
    assert lib.loglike_batch(None, None, 1, 13, None, None) == gk.GK_EINVAL
    assert lib.loglike_grad_batch(None, None, 1, 13, None, None, None) == gk.GK_EINVAL
    assert lib.eval_maps(None, None, 1, 13, None, None) == gk.GK_EINVAL
    assert lib.set_data(None, None, None, 0, None) == gk.GK_EINVAL
    assert lib.destroy_grid(None) == gk.GK_EINVAL
    assert lib.loglike_joint(None, 1, None, 1, 13, None, None, None) == gk.GK_EINVAL
    assert lib.get_launch_shape(None, 1, None, None, None) == gk.GK_EINVAL
    assert lib.loglike_joint(None, 0, None, 1, 13, None, None, None) == gk.GK_EINVAL
    assert lib.set_launch_shape(None, 1, 1, 1, 0) == gk.GK_EINVAL
    assert lib.set_adjoint_shape(None, 40, 40, 0) == gk.GK_EINVAL
    assert lib.get_adjoint_shape(None, None, None, None) == gk.GK_EINVAL
    assert lib.loglike_multi(None, -1, None, None, 13, None, None, None) == gk.GK_EINVAL
    assert lib.loglike_multi(None, 0, None, None, 13, None, None, None) == gk.GK_OK
    assert lib.loglike_multi(None, 2, None, None, 13, None, None, None) == gk.GK_EINVAL
    nulls = (ctypes.c_void_p * 2)()
    offs = (ctypes.c_int * 3)(0, 1, 2)
    assert lib.loglike_multi(nulls, 2, None, offs, 13, None, None, None) == gk.GK_EINVAL
    assert "NULL" in gk.last_error()
    assert lib.ml_from_colour(None, None, None, None, 4, 0.0, 1.0, 0.1, None, None, None) == gk.GK_EINVAL
    assert lib.ml_from_colour(None, None, None, None, 0, 0.0, 1.0, 0.1, None, None, None) == gk.GK_OK
    assert lib.brightness_errors(None, 4, 0.05, 0.1, None, None) == gk.GK_EINVAL
    assert lib.brightness_errors(None, -1, 0.05, 0.1, None, None) == gk.GK_EINVAL


def test_binding_has_no_cpu_fallback():
    # the product package must not import the oracle
    pkg = os.path.join(ROOT, "paper_2205_06819_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
