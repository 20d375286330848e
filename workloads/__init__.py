"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the galaxy model. It only defines

* the grid descriptor (``GridSpec``) and the parameter-vector layout, which are
  the interface both implementations agree on;
* the five benchmark workloads (IFU-shaped synthetic stand-ins for the paper's
  CALIFA/SDSS maps of NGC 7683, which are not available);
* seeded draws: parameter vectors from uniform priors, elliptical masks and
  Gaussian noise added to model maps produced by whichever implementation the
  caller chooses.

Parameter layout (all float64, sampling coordinates, not the paper's
log-radius / sin-i coordinates of its Table 2):

====================  =====================================================
group                 entries
====================  =====================================================
frame                 x0 [px], y0 [px], PA [deg], i [deg]
bulge (if present)    log10 Mb [Msun], Rb [kpc], (M/L)b
each disc j           log10 Mdj [Msun], Rdj [kpc], (M/L)dj, kj
halo (if present)     log10 Mh [Msun], then c (NFW) or Rh [kpc] (Hernquist)
====================  =====================================================

The galaxy centre sits at the grid centre plus (x0, y0) pixels (pixels of a
shared frame, possibly offset, when ``GridSpec.frame_px_kpc`` is set).  x is the
column index (fastest varying), y the row index, maps are stored [ny][nx].
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# Components
BULGE_NONE, BULGE_HERNQUIST, BULGE_JAFFE = 0, 1, 2
PSF_MAPS, PSF_LUMINOSITY = 0, 1
HALO_NONE, HALO_HERNQUIST, HALO_NFW = 0, 1, 2

ARCSEC_PER_RAD = 180.0 * 3600.0 / math.pi
FWHM_PER_SIGMA = 2.0 * math.sqrt(2.0 * math.log(2.0))


def pixel_kpc(arcsec_per_px: float, distance_mpc: float) -> float:
    """Small-angle pixel size in kpc."""
    return distance_mpc * 1.0e3 * arcsec_per_px / ARCSEC_PER_RAD


@dataclasses.dataclass(frozen=True)
class GridSpec:
    nx: int
    ny: int
    pixel_kpc: float
    supersample: int          # odd, >= 1
    psf_sigma_px: float       # Gaussian sigma in pixels; stencil radius 3 sigma
    bulge: int = BULGE_HERNQUIST
    n_discs: int = 1
    halo: int = HALO_NFW
    hubble_h: float = 0.7
    psf_mode: int = 0         # PSF_MAPS (each map averaged) or PSF_LUMINOSITY (moments)
    # shared frame of the centre parameters when several grids (one per
    # pixelisation) see the same galaxy: x0, y0 are in pixels of size
    # frame_px_kpc (0: this grid's own pixels), and the frame's centre sits
    # frame_dx, frame_dy pixels of this grid from this grid's centre
    frame_px_kpc: float = 0.0
    frame_dx: float = 0.0
    frame_dy: float = 0.0

    @property
    def n_params(self) -> int:
        return (4 + 3 * (self.bulge != BULGE_NONE) + 4 * self.n_discs
                + 2 * (self.halo != HALO_NONE))


def param_names(spec: GridSpec) -> List[str]:
    names = ["x0", "y0", "PA", "incl"]
    if spec.bulge:
        names += ["logMb", "Rb", "MLb"]
    for j in range(1, spec.n_discs + 1):
        names += [f"logMd{j}", f"Rd{j}", f"MLd{j}", f"k{j}"]
    if spec.halo == HALO_NFW:
        names += ["logMh", "c"]
    elif spec.halo == HALO_HERNQUIST:
        names += ["logMh", "Rh"]
    return names


# Uniform prior ranges of the benchmark workloads (k in [0, 1] as in the
# paper's Table 2; a Hernquist halo scale radius range is added for that kind).
PRIORS = {
    "x0": (-2.0, 2.0), "y0": (-2.0, 2.0), "PA": (0.0, 180.0), "incl": (10.0, 80.0),
    "logMb": (8.0, 11.0), "Rb": (0.1, 3.0), "MLb": (0.5, 10.0),
    "logMd": (9.0, 11.5), "Rd": (0.5, 10.0), "MLd": (0.5, 10.0), "k": (0.0, 1.0),
    "logMh": (11.0, 13.0), "c": (5.0, 20.0), "Rh": (10.0, 100.0),
}


def _prior_key(name: str) -> str:
    for key in ("logMd", "Rd", "MLd"):
        if name.startswith(key):
            return key
    if name[0] == "k" and name[1:].isdigit():
        return "k"
    return name


def prior_bounds(spec: GridSpec) -> np.ndarray:
    """[P, 2] array of (low, high) for each parameter."""
    return np.array([PRIORS[_prior_key(n)] for n in param_names(spec)], dtype=np.float64)


def draw_thetas(spec: GridSpec, n: int, rng: np.random.Generator) -> np.ndarray:
    """n parameter vectors drawn uniformly from the priors, [n, P] float64.

    Disc scale radii are sorted so that disc 1 is the inner disc (R_d1 < R_d2).
    """
    b = prior_bounds(spec)
    th = b[:, 0] + (b[:, 1] - b[:, 0]) * rng.random((n, b.shape[0]))
    if spec.n_discs == 2:
        names = param_names(spec)
        i1, i2 = names.index("Rd1"), names.index("Rd2")
        lo = np.minimum(th[:, i1], th[:, i2])
        hi = np.maximum(th[:, i1], th[:, i2])
        th[:, i1], th[:, i2] = lo, hi
    return th


def elliptical_mask(nx: int, ny: int, a_px: float, b_px: float,
                    cx: Optional[float] = None, cy: Optional[float] = None) -> np.ndarray:
    """Boolean [ny, nx] mask, True inside the axis-aligned ellipse."""
    cx = (nx - 1) / 2.0 if cx is None else cx
    cy = (ny - 1) / 2.0 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx]
    return ((x - cx) / a_px) ** 2 + ((y - cy) / b_px) ** 2 <= 1.0


# Noise recipe of the benchmark workloads: 5 % on surface brightness,
# 10 km/s on velocity and dispersion, 10 % on M/L.
NOISE_REL_B, NOISE_ABS_V, NOISE_ABS_S, NOISE_REL_ML = 0.05, 10.0, 10.0, 0.10


def error_maps(maps: np.ndarray, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-pixel 1-sigma errors [4, ny, nx] for maps [4, ny, nx] = (B, v, sigma, M/L).

    Masked pixels get error 0, which marks them invalid at the boundary.
    """
    maps = np.asarray(maps, dtype=np.float64)
    err = np.empty_like(maps)
    err[0] = NOISE_REL_B * np.abs(maps[0])
    err[1] = NOISE_ABS_V
    err[2] = NOISE_ABS_S
    err[3] = NOISE_REL_ML * np.abs(maps[3])
    if mask is not None:
        err[:, ~mask] = 0.0
    return err


def noisy_data(maps: np.ndarray, err: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """maps + N(0, err^2), float64 [4, ny, nx]; masked pixels keep the map value."""
    maps = np.asarray(maps, dtype=np.float64)
    return maps + err * rng.standard_normal(maps.shape)


@dataclasses.dataclass
class Workload:
    name: str
    spec: GridSpec
    batch: int
    mask_axes: Optional[Sequence[float]] = None   # (a, b) px of the elliptical mask
    seed: int = 0
    gradient: bool = False

    def mask(self) -> np.ndarray:
        if self.mask_axes is None:
            return np.ones((self.spec.ny, self.spec.nx), dtype=bool)
        return elliptical_mask(self.spec.nx, self.spec.ny, *self.mask_axes)


PK_50MPC = pixel_kpc(0.5, 50.0)          # 0.121203 kpc/px
SIGMA_FWHM_2P5 = 2.5 / FWHM_PER_SIGMA    # 1.06165 px
SIGMA_FWHM_4 = 4.0 / FWHM_PER_SIGMA      # 1.69864 px
SEED0 = 20220505


def workload(name: str) -> Workload:
    """The benchmark workloads, by name: tiny, realistic, adjoint, stress, jaffe, lw."""
    if name == "tiny":
        spec = GridSpec(40, 40, PK_50MPC, 1, 1.5, BULGE_HERNQUIST, 1, HALO_NFW)
        return Workload(name, spec, 64, None, SEED0 + 0)
    if name == "realistic":
        spec = GridSpec(80, 80, PK_50MPC, 3, SIGMA_FWHM_2P5, BULGE_HERNQUIST, 2, HALO_NFW)
        return Workload(name, spec, 1024, (38.0, 33.6), SEED0 + 1)
    if name == "adjoint":
        spec = GridSpec(100, 100, PK_50MPC, 3, SIGMA_FWHM_2P5, BULGE_HERNQUIST, 2, HALO_NFW)
        return Workload(name, spec, 4096, None, SEED0 + 3, gradient=True)
    if name == "jaffe":
        # the realistic IFU cube with the Appendix-B (Jaffe) bulge
        spec = GridSpec(80, 80, PK_50MPC, 3, SIGMA_FWHM_2P5, BULGE_JAFFE, 2, HALO_NFW)
        return Workload(name, spec, 1024, (38.0, 33.6), SEED0 + 5)
    if name == "lw":
        # the realistic IFU cube, PSF applied to the luminosity-weighted moments
        spec = GridSpec(80, 80, PK_50MPC, 3, SIGMA_FWHM_2P5, BULGE_HERNQUIST, 2, HALO_NFW,
                        psf_mode=PSF_LUMINOSITY)
        return Workload(name, spec, 1024, (38.0, 33.6), SEED0 + 6)
    if name == "stress":
        spec = GridSpec(300, 300, PK_50MPC, 5, SIGMA_FWHM_4, BULGE_HERNQUIST, 2, HALO_NFW)
        return Workload(name, spec, 8192, None, SEED0 + 4, gradient=True)
    raise KeyError(name)


COMPONENT_SETS = [  # (bulge, n_discs, halo) for the uneven multi-galaxy workload
    (BULGE_HERNQUIST, 1, HALO_NONE),
    (BULGE_HERNQUIST, 1, HALO_NFW),
    (BULGE_HERNQUIST, 2, HALO_NFW),
]


def uneven_galaxies(n_gal: int = 256, theta_per_gal: int = 128,
                    seed: int = SEED0 + 2) -> List[Workload]:
    """Many galaxies with square grids of side U{30..120} and 2-4 components."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(n_gal):
        n = int(rng.integers(30, 121))
        bulge, nd, halo = COMPONENT_SETS[int(rng.integers(0, 3))]
        spec = GridSpec(n, n, PK_50MPC, 3, SIGMA_FWHM_2P5, bulge, nd, halo)
        out.append(Workload(f"gal{g}", spec, theta_per_gal, None, seed * 1000 + g))
    return out


def multires_pair():
    """One galaxy seen on two pixelisations: photometry (B) on a 160x160 grid
    of 0.25 arcsec pixels with 1 arcsec seeing and no supersampling, and the
    kinematic and M/L maps on the realistic 80x80 IFU grid.  The centre
    parameters are in the IFU grid's pixels.  Returns (photometry workload,
    IFU workload); the photometric grid's mask is the IFU mask scaled by 2."""
    phot = GridSpec(160, 160, PK_50MPC / 2.0, 1, SIGMA_FWHM_4, BULGE_HERNQUIST, 2, HALO_NFW,
                    frame_px_kpc=PK_50MPC)
    kin = GridSpec(80, 80, PK_50MPC, 3, SIGMA_FWHM_2P5, BULGE_HERNQUIST, 2, HALO_NFW)
    return (Workload("multires-phot", phot, 1024, (76.0, 67.2), SEED0 + 7),
            Workload("multires-ifu", kin, 1024, (38.0, 33.6), SEED0 + 7))
