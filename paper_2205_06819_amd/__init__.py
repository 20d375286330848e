"""galkin: MI355X-native batched likelihood of the bulge + disc(s) + halo
disc-galaxy model of Rigamonti et al. 2022 (arXiv 2205.06819).

Thin Python binding of the C-ABI library ``libgalkin.so`` (declared in
``include/galkin.h``).  The functions below carry the same names as the C
entry points and only marshal arguments: every step of the likelihood runs
in the HIP kernels.  PyTorch supplies device memory and streams.

If the library has not been built (``python paper_2205_06819_amd/build.py``),
importing this package raises an error: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgalkin.so")

GK_OK, GK_EINVAL, GK_ENOMEM, GK_EHIP, GK_ESTATE = 0, -1, -2, -3, -4
GK_BULGE_NONE, GK_BULGE_HERNQUIST, GK_BULGE_JAFFE = 0, 1, 2
GK_HALO_NONE, GK_HALO_HERNQUIST, GK_HALO_NFW = 0, 1, 2
GK_PSF_MAPS, GK_PSF_LUMINOSITY = 0, 1

EXPORTS = ("create_grid", "destroy_grid", "n_params", "set_data", "loglike_batch",
           "loglike_grad_batch", "eval_maps", "set_launch_shape", "hmc_leapfrog", "loglike_multi", "loglike_joint", "get_launch_shape", "ml_from_colour",
           "brightness_errors", "set_adjoint_shape", "get_adjoint_shape", "loglike_batch_noalloc",
           "last_error")


class GalkinError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"galkin error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("pixel_kpc", ctypes.c_double),
                ("supersample", ctypes.c_int), ("psf_sigma_px", ctypes.c_double),
                ("bulge", ctypes.c_int), ("n_discs", ctypes.c_int), ("halo", ctypes.c_int),
                ("hubble_h", ctypes.c_double), ("psf_mode", ctypes.c_int),
                ("frame_px_kpc", ctypes.c_double), ("frame_dx", ctypes.c_double),
                ("frame_dy", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2205_06819_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in EXPORTS if not hasattr(lib, n)]
    if missing:
        raise ImportError(f"{LIB_PATH} lacks {missing}: rebuild it with `python paper_2205_06819_amd/build.py`")
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.create_grid.argtypes = [ctypes.POINTER(GridDesc), i, ctypes.POINTER(vp)]
    lib.destroy_grid.argtypes = [vp]
    lib.n_params.argtypes = [vp]
    lib.set_data.argtypes = [vp, vp, vp, i, vp]
    lib.loglike_batch.argtypes = [vp, vp, i, i, vp, vp]
    lib.loglike_batch_noalloc.argtypes = [vp, vp, i, i, vp, vp]
    lib.loglike_grad_batch.argtypes = [vp, vp, i, i, vp, vp, vp]
    lib.eval_maps.argtypes = [vp, vp, i, i, vp, vp]
    lib.set_launch_shape.argtypes = [vp, i, i, i, i]
    lib.hmc_leapfrog.argtypes = [vp, vp, vp, vp, d, i, i, i, vp, vp, vp]
    lib.loglike_multi.argtypes = [vp, i, vp, vp, i, vp, vp, vp]
    lib.loglike_joint.argtypes = [vp, i, vp, i, i, vp, vp, vp]
    lib.get_launch_shape.argtypes = [vp, i, vp, vp, vp]
    lib.set_adjoint_shape.argtypes = [vp, i, i, i]
    lib.get_adjoint_shape.argtypes = [vp, vp, vp, vp]
    lib.ml_from_colour.argtypes = [vp, vp, vp, vp, i, d, d, d, vp, vp, vp]
    lib.brightness_errors.argtypes = [vp, i, d, d, vp, vp]
    lib.last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "last_error":
            getattr(lib, name).restype = i
    return lib


_lib = _load()


def _check(rc: int) -> int:
    if rc < 0:
        raise GalkinError(rc, _lib.last_error().decode())
    return rc


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def make_desc(spec) -> GridDesc:
    """GridDesc from any object with the descriptor's attribute names."""
    return GridDesc(int(spec.nx), int(spec.ny), float(spec.pixel_kpc), int(spec.supersample),
                    float(spec.psf_sigma_px), int(spec.bulge), int(spec.n_discs), int(spec.halo),
                    float(getattr(spec, "hubble_h", 0.7)), int(getattr(spec, "psf_mode", 0)),
                    float(getattr(spec, "frame_px_kpc", 0.0)), float(getattr(spec, "frame_dx", 0.0)),
                    float(getattr(spec, "frame_dy", 0.0)))


# --- C-ABI names -------------------------------------------------------------
def create_grid(spec, max_batch: int) -> int:
    desc = make_desc(spec)
    h = ctypes.c_void_p()
    _check(_lib.create_grid(ctypes.byref(desc), int(max_batch), ctypes.byref(h)))
    return h.value


def destroy_grid(handle: int) -> None:
    _check(_lib.destroy_grid(handle))


def n_params(handle: int) -> int:
    return _check(_lib.n_params(handle))


def set_data(handle: int, value, err, stream=None) -> None:
    """value, err: [4, ny, nx] (numpy or torch); converted to float32."""
    if isinstance(value, torch.Tensor) and value.is_cuda:
        v = value.to(torch.float32).contiguous()
        e = err.to(device=v.device, dtype=torch.float32).contiguous()
        _check(_lib.set_data(handle, v.data_ptr(), e.data_ptr(), 1, _stream(stream)))
        return
    v = np.ascontiguousarray(np.asarray(value.cpu() if isinstance(value, torch.Tensor) else value,
                                        dtype=np.float32))
    e = np.ascontiguousarray(np.asarray(err.cpu() if isinstance(err, torch.Tensor) else err,
                                        dtype=np.float32))
    _check(_lib.set_data(handle, v.ctypes.data, e.ctypes.data, 0, _stream(stream)))


def _theta(theta: torch.Tensor, P: int) -> torch.Tensor:
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.dim() == 2):
        raise ValueError("theta must be a 2-D float64 CUDA tensor [B, stride]")
    if theta.stride(1) != 1:
        theta = theta.contiguous()
    if theta.shape[1] < P:
        raise ValueError(f"theta has {theta.shape[1]} columns, the model has {P} parameters")
    return theta


def loglike_batch(handle: int, theta: torch.Tensor, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    theta = _theta(theta, n_params(handle))
    B = theta.shape[0]
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=theta.device)
    _check(_lib.loglike_batch(handle, theta.data_ptr(), B, theta.stride(0), out.data_ptr(),
                              _stream(stream)))
    return out


def loglike_batch_noalloc(handle: int, theta: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """loglike_batch with the launch's scratch in the library's fixed device
    array (nothing is allocated: out must be given, float64 [B] on the device)."""
    theta = _theta(theta, n_params(handle))
    B = theta.shape[0]
    if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= B):
        raise ValueError("out must be a contiguous float64 CUDA tensor of at least B elements")
    _check(_lib.loglike_batch_noalloc(handle, theta.data_ptr(), B, theta.stride(0), out.data_ptr(),
                                      _stream(stream)))
    return out


def loglike_grad_batch(handle: int, theta: torch.Tensor, out: Optional[torch.Tensor] = None,
                       grad: Optional[torch.Tensor] = None, stream=None
                       ) -> Tuple[torch.Tensor, torch.Tensor]:
    theta = _theta(theta, n_params(handle))
    B = theta.shape[0]
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=theta.device)
    if grad is None:
        grad = torch.empty(B, theta.stride(0), dtype=torch.float64, device=theta.device)
    _check(_lib.loglike_grad_batch(handle, theta.data_ptr(), B, theta.stride(0), out.data_ptr(),
                                   grad.data_ptr(), _stream(stream)))
    return out, grad[:, :theta.shape[1]]


def eval_maps(handle: int, theta: torch.Tensor, ny: int, nx: int,
              out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    theta = _theta(theta, n_params(handle))
    B = theta.shape[0]
    if out is None:
        out = torch.empty(B, 4, ny, nx, dtype=torch.float32, device=theta.device)
    _check(_lib.eval_maps(handle, theta.data_ptr(), B, theta.stride(0), out.data_ptr(),
                          _stream(stream)))
    return out


def hmc_leapfrog(handle: int, theta: torch.Tensor, momentum: torch.Tensor, inv_mass: torch.Tensor,
                 eps: float, n_steps: int, logL: torch.Tensor, grad: torch.Tensor, stream=None) -> None:
    """In-place leapfrog trajectory (see include/galkin.h); all tensors on the device."""
    P = n_params(handle)
    for t, nm in ((theta, "theta"), (momentum, "momentum"), (grad, "grad")):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError(f"{nm} must be a contiguous-row float64 CUDA tensor [B, stride]")
    if momentum.stride(0) != theta.stride(0) or grad.stride(0) != theta.stride(0):
        raise ValueError("theta, momentum and grad must share the row stride")
    if inv_mass.numel() < P or inv_mass.dtype != torch.float64 or not inv_mass.is_cuda:
        raise ValueError("inv_mass must be a float64 CUDA tensor with P entries")
    _check(_lib.hmc_leapfrog(handle, theta.data_ptr(), momentum.data_ptr(), inv_mass.data_ptr(),
                             float(eps), int(n_steps), theta.shape[0], theta.stride(0),
                             logL.data_ptr(), grad.data_ptr(), _stream(stream)))


def loglike_multi(handles, theta: torch.Tensor, theta_offset, out: Optional[torch.Tensor] = None,
                  grad: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Log-likelihoods of many grids in one launch.  Rows theta_offset[g] ..
    theta_offset[g+1]-1 of theta belong to grid handles[g]; theta has as many
    columns as the largest parameter count.  With grad given (float64
    [rows, stride]) the gradient is written too."""
    n = len(handles)
    offs = np.ascontiguousarray(np.asarray(theta_offset, dtype=np.int32))
    if offs.shape != (n + 1,):
        raise ValueError("theta_offset needs len(handles) + 1 entries")
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.dim() == 2 and theta.stride(1) == 1):
        raise ValueError("theta must be a contiguous-row float64 CUDA tensor [rows, stride]")
    if theta.shape[0] < int(offs[-1]):
        raise ValueError("theta has fewer rows than theta_offset[-1]")
    hs = (ctypes.c_void_p * max(1, n))(*[ctypes.c_void_p(h) for h in handles])
    if out is None:
        out = torch.empty(int(offs[-1]), dtype=torch.float64, device=theta.device)
    if grad is not None and (grad.stride(0) != theta.stride(0) or grad.stride(1) != 1 or grad.dtype != torch.float64):
        raise ValueError("grad must be float64 with theta's row stride")
    _check(_lib.loglike_multi(hs, n, theta.data_ptr(), offs.ctypes.data, theta.stride(0), out.data_ptr(),
                              _ptr(grad), _stream(stream)))
    return out


def loglike_joint(handles, theta: torch.Tensor, out: Optional[torch.Tensor] = None,
                  grad: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Joint log-likelihood of one galaxy observed on several grids (one per
    pixelisation, sharing the parameter vector): logL[b] = sum over the
    grids.  With grad given (float64, theta's shape) the summed gradient is
    written too."""
    n = len(handles)
    if not (theta.is_cuda and theta.dtype == torch.float64 and theta.dim() == 2 and theta.stride(1) == 1):
        raise ValueError("theta must be a contiguous-row float64 CUDA tensor [B, stride]")
    hs = (ctypes.c_void_p * max(1, n))(*[ctypes.c_void_p(h) for h in handles])
    B = theta.shape[0]
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=theta.device)
    if grad is not None and (grad.stride(0) != theta.stride(0) or grad.stride(1) != 1 or grad.dtype != torch.float64
                             or grad.shape[0] < B):
        raise ValueError("grad must be float64 [B, stride] with theta's row stride")
    _check(_lib.loglike_joint(hs, n, theta.data_ptr(), B, theta.stride(0), out.data_ptr(), _ptr(grad),
                              _stream(stream)))
    return out


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32):
        raise ValueError(f"{name} must be a float32 CUDA tensor")
    return t.contiguous()


def ml_from_colour(m_beta, m_gamma, dm_beta, dm_gamma, a: float, b: float, sigma_a: float,
                   stream=None) -> Tuple[torch.Tensor, torch.Tensor]:
    """M/L map and its error from two magnitude maps (see include/galkin.h)."""
    xs = [_dev_f32(t, nm) for t, nm in ((m_beta, "m_beta"), (m_gamma, "m_gamma"),
                                        (dm_beta, "dm_beta"), (dm_gamma, "dm_gamma"))]
    n = xs[0].numel()
    if any(x.numel() != n for x in xs):
        raise ValueError("magnitude maps differ in size")
    ml = torch.empty_like(xs[0])
    err = torch.empty_like(xs[0])
    _check(_lib.ml_from_colour(*[x.data_ptr() for x in xs], n, float(a), float(b), float(sigma_a),
                               ml.data_ptr(), err.data_ptr(), _stream(stream)))
    return ml, err


def brightness_errors(B, rel: float = 0.05, floor_frac: float = 0.1, stream=None) -> torch.Tensor:
    """Surface-brightness errors: relative part plus a floor from the faintest pixel."""
    B = _dev_f32(B, "B")
    err = torch.empty_like(B)
    _check(_lib.brightness_errors(B.data_ptr(), B.numel(), float(rel), float(floor_frac), err.data_ptr(),
                                  _stream(stream)))
    return err


def set_launch_shape(handle: int, batch_min: int, band_h: int, band_w: int, steps: int = 0) -> None:
    _check(_lib.set_launch_shape(handle, int(batch_min), int(band_h), int(band_w), int(steps)))


def get_launch_shape(handle: int, B: int):
    """(band_h, band_w, steps) that calls with B vectors use on this grid."""
    h, w, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.get_launch_shape(handle, int(B), ctypes.byref(h), ctypes.byref(w), ctypes.byref(st)))
    return h.value, w.value, st.value


def set_adjoint_shape(handle: int, band_h: int, band_w: int, rows: int = 0) -> None:
    _check(_lib.set_adjoint_shape(handle, int(band_h), int(band_w), int(rows)))


def get_adjoint_shape(handle: int):
    """(band_h, band_w, rows) of the gradient's adjoint launch."""
    h, w, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(_lib.get_adjoint_shape(handle, ctypes.byref(h), ctypes.byref(w), ctypes.byref(st)))
    return h.value, w.value, st.value


def last_error() -> str:
    return _lib.last_error().decode()


# --- convenience wrapper -------------------------------------------------------
class Grid:
    """Owns one grid handle (device buffers for one galaxy's maps)."""

    def __init__(self, spec, max_batch: int):
        self.spec = spec
        self.nx, self.ny = int(spec.nx), int(spec.ny)
        self.handle = create_grid(spec, max_batch)
        self.P = n_params(self.handle)
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "handle", None):
            destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, value, err, stream=None):
        set_data(self.handle, value, err, stream)

    def loglike(self, theta, out=None, stream=None):
        return loglike_batch(self.handle, theta, out, stream)

    def loglike_grad(self, theta, out=None, grad=None, stream=None):
        return loglike_grad_batch(self.handle, theta, out, grad, stream)

    def maps(self, theta, out=None, stream=None):
        return eval_maps(self.handle, theta, self.ny, self.nx, out, stream)

    def set_launch_shape(self, batch_min, band_h, band_w, steps=0):
        set_launch_shape(self.handle, batch_min, band_h, band_w, steps)

    def set_adjoint_shape(self, band_h, band_w, rows=0):
        set_adjoint_shape(self.handle, band_h, band_w, rows)

    def adjoint_shape(self):
        return get_adjoint_shape(self.handle)

    def launch_shape(self, B):
        return get_launch_shape(self.handle, B)


class LogLike(torch.autograd.Function):
    """logL = LogLike.apply(theta, grid): float64 [B]; backward uses the
    hand-written adjoint kernel (d logL / d theta)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, grid: Grid):
        if theta.requires_grad:
            logL, g = grid.loglike_grad(theta.detach())
            ctx.save_for_backward(g.clone())
        else:
            logL = grid.loglike(theta)
        return logL

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout[:, None] * g, None
