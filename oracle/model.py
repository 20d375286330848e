"""Plain FP64 CPU oracle of the bulge + disc(s) + halo likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP implementation.

What it computes (paper Sec. 2 and Appendix A), for one parameter vector:

1. Frame (Sec. 2.1): translate the sky coordinates to the model centre,
   rotate by the position angle so the projected major axis lies on +x
   (PA counter-clockwise from +x), and deproject by the inclination onto the
   razor-thin disc plane:
   x' = dx cos PA + dy sin PA,  y' = -dx sin PA + dy cos PA,
   R = |(x', y')| (sky-plane radius), r = |(x', y'/cos i)| (disc-plane radius),
   cos(phi) = x'/r (azimuth from the major axis; 0 at r = 0).
2. Bulge (Sec. 2.2): Hernquist projected density and isotropic projected
   dispersion at s = R/R_b (s clamped below at 1e-6); circular velocity
   sqrt(G M r)/(r + R_b) at the disc-plane radius.  The bulge dispersion uses
   only its own potential.
3. Discs (Sec. 2.3): exponential, razor thin; projected density
   M/(2 pi R_d^2) exp(-r/R_d) / cos i; Freeman circular velocity (see
   ``special``); Satoh decomposition v_j = -k_j sin i cos(phi) v_int(r),
   sigma_j^2 = (1 - k_j^2) v_int^2 / 3, with v_int^2 the sum of the squared
   circular velocities of every component present.
4. Halo: Hernquist (paper, Sec. 2.2: circular velocity as for the bulge) or
   NFW (M200 at 200 times the critical density, concentration c); it only
   adds to v_int.
5. Observables (Sec. 2.4 and the likelihood section 2.5.1): surface brightness
   B = sum Sigma_x/(M/L)_x, light-weighted l.o.s. velocity (bulge not
   rotating), light-weighted sigma_los^2, and <L/M> = B / Sigma_tot.
6. PSF (Sec. 3.1, PSF convolution equation): each of B, v_los, sigma_los and
   <L/M> is averaged with normalised Gaussian weights over the points of a
   lattice of spacing 1/s pixel lying within 3 sigma of the pixel centre.
   Here the model is evaluated once on a padded fine lattice shared by all
   pixels (``psf_maps``); ``psf_maps_alg1`` evaluates, for every pixel, its
   own K sub-grid points (the two nested loops of Appendix A, Algorithm 1).
   Both give the same numbers up to rounding.
7. Likelihood (Sec. 2.5.1): sum of four Gaussian log terms (B, v, sigma, M/L),
   each over its own valid pixels, with model M/L = 1 / <L/M>_PSF; the
   normalisation -1/2 ln(2 pi e^2) is included.

Units: kpc, km/s, Msun; G = 4.300917270e-6 kpc (km/s)^2 / Msun; surface
densities in Msun/kpc^2 inside, brightness in Lsun/pc^2 (factor 1e-6).

The parameter layout and the grid descriptor come from ``workloads``.
Gradients: ``grad_complex_step`` (forward mode, one complex evaluation per
parameter, exact to rounding) and ``grad_central_fd`` (central differences).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

from workloads import (BULGE_JAFFE, BULGE_NONE, HALO_HERNQUIST, HALO_NFW, HALO_NONE, GridSpec,
                       param_names)
from . import special

G_KPC = 4.300917270e-6          # kpc (km/s)^2 / Msun
S_CLAMP = 1.0e-6                # lower clamp of s = R / R_b at the centre


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def unpack(spec: GridSpec, theta) -> Dict[str, object]:
    names = param_names(spec)
    theta = np.asarray(theta)
    if theta.shape[-1] < len(names):
        raise ValueError("theta has fewer entries than the model has parameters")
    return {n: theta[..., k] for k, n in enumerate(names)}


def is_valid(spec: GridSpec, theta) -> bool:
    """Physical domain of the parameters; outside it log L = -inf."""
    p = {k: float(np.real(v)) for k, v in unpack(spec, theta).items()}
    if not all(math.isfinite(v) for v in p.values()):
        return False
    if not (0.0 < p["incl"] < 90.0):
        return False
    if spec.bulge != BULGE_NONE and not (p["Rb"] > 0.0 and p["MLb"] > 0.0):
        return False
    for j in range(1, spec.n_discs + 1):
        if not (p[f"Rd{j}"] > 0.0 and p[f"MLd{j}"] > 0.0 and abs(p[f"k{j}"]) <= 1.0):
            return False
    if spec.halo == HALO_NFW and not p["c"] > 0.0:
        return False
    if spec.halo == HALO_HERNQUIST and not p["Rh"] > 0.0:
        return False
    return True


def rho_crit(hubble_h: float) -> float:
    """Critical density 3 H^2 / (8 pi G) in Msun/kpc^3, H = 100 h km/s/Mpc."""
    H = 0.1 * hubble_h          # km/s/kpc
    return 3.0 * H * H / (8.0 * math.pi * G_KPC)


# ---------------------------------------------------------------------------
# the model at arbitrary sky positions
# ---------------------------------------------------------------------------
def frame_scale(spec: GridSpec) -> float:
    """This grid's pixels per pixel of the frame the centre parameters use."""
    f = getattr(spec, "frame_px_kpc", 0.0)
    return f / spec.pixel_kpc if f > 0.0 else 1.0


def point_model(spec: GridSpec, theta, x_px, y_px):
    """(B, v_los, sigma_los, <L/M>) at sky positions given in pixel coordinates.

    x_px, y_px: arrays (any shape) of column / row coordinates; pixel (i, j)
    has its centre at (i, j).  Works for complex theta (complex step).
    """
    p = unpack(spec, theta)
    cplx = np.iscomplexobj(np.asarray(theta))
    dt = np.complex128 if cplx else np.float64
    x_px = np.asarray(x_px, dtype=np.float64)
    y_px = np.asarray(y_px, dtype=np.float64)

    # 1. frame; (x0, y0) may be given in a shared frame of another pixel size
    fs = frame_scale(spec)
    xc = 0.5 * (spec.nx - 1) + getattr(spec, "frame_dx", 0.0) + fs * p["x0"]
    yc = 0.5 * (spec.ny - 1) + getattr(spec, "frame_dy", 0.0) + fs * p["y0"]
    dx = (x_px - xc) * spec.pixel_kpc
    dy = (y_px - yc) * spec.pixel_kpc
    pa = p["PA"] * (math.pi / 180.0)
    inc = p["incl"] * (math.pi / 180.0)
    cpa, spa = np.cos(pa), np.sin(pa)
    xp = dx * cpa + dy * spa
    yp = -dx * spa + dy * cpa
    R = np.sqrt(xp * xp + yp * yp)
    yd = yp / np.cos(inc)
    r = np.sqrt(xp * xp + yd * yd)
    at_centre = np.real(r) == 0.0
    r_safe = np.where(at_centre, 1.0, r)
    cosphi = np.where(at_centre, 0.0, xp / r_safe)
    sin_i, cos_i = np.sin(inc), np.cos(inc)

    zeros = np.zeros(np.broadcast(x_px, y_px).shape, dtype=dt)
    B_tot = zeros.copy()          # Lsun/pc^2
    Sig_tot = zeros.copy()        # Msun/pc^2
    BV = zeros.copy()             # sum_j B_j v_j
    BS2 = zeros.copy()            # sum_x B_x sigma_x^2
    vint2 = zeros.copy()

    # 2. bulge
    if spec.bulge != BULGE_NONE:
        Mb = 10.0 ** p["logMb"]
        Rb = p["Rb"]
        MLb = p["MLb"]
        s = R / Rb
        s = np.where(np.real(s) < S_CLAMP, S_CLAMP + 0.0 * s, s)
        if spec.bulge == BULGE_JAFFE:
            # Appendix B: Sigma_b = Mb g / Rb^2, Sigma_b sigma_b^2 = G Mb^2 h / (4 pi Rb^3),
            # v_c^2 = G Mb / (r + Rb)
            Sig_b = 1.0e-6 * Mb * special.jf_g(s) / (Rb * Rb)
            BS2 = BS2 + 1.0e-6 * G_KPC * Mb * Mb * special.jf_h(s) / (4.0 * math.pi * Rb ** 3 * MLb)
            vint2 = vint2 + G_KPC * Mb / (r + Rb)
        else:
            Sig_b = 1.0e-6 * Mb * special.hq_g(s) / (2.0 * math.pi * Rb * Rb)
            # B_b sigma_b^2 = (Sigma_b / ML) G Mb^2 h / (12 pi Rb^3 Sigma_b)
            BS2 = BS2 + 1.0e-6 * G_KPC * Mb * Mb * special.hq_h(s) / (12.0 * math.pi * Rb ** 3 * MLb)
            vint2 = vint2 + G_KPC * Mb * r / (r + Rb) ** 2
        B_b = Sig_b / MLb
        B_tot = B_tot + B_b
        Sig_tot = Sig_tot + Sig_b

    # 3. discs (densities now; kinematics need the total v_int first)
    discs = []
    for j in range(1, spec.n_discs + 1):
        Md = 10.0 ** p[f"logMd{j}"]
        Rd = p[f"Rd{j}"]
        MLd = p[f"MLd{j}"]
        k = p[f"k{j}"]
        Sig_d = 1.0e-6 * Md * np.exp(-r / Rd) / (2.0 * math.pi * Rd * Rd * cos_i)
        B_d = Sig_d / MLd
        y = r / (2.0 * Rd)
        vint2 = vint2 + (2.0 * G_KPC * Md / Rd) * special.freeman_phi(y)
        B_tot = B_tot + B_d
        Sig_tot = Sig_tot + Sig_d
        discs.append((B_d, k))

    # 4. halo
    if spec.halo == HALO_NFW:
        M200 = 10.0 ** p["logMh"]
        c = p["c"]
        r200 = (3.0 * M200 / (4.0 * math.pi * 200.0 * rho_crit(spec.hubble_h))) ** (1.0 / 3.0)
        rs = r200 / c
        x = r_safe / rs
        vh2 = G_KPC * M200 * special.nfw_mu(x) / (r_safe * special.nfw_mu(c))
        vint2 = vint2 + np.where(at_centre, 0.0, vh2)
    elif spec.halo == HALO_HERNQUIST:
        Mh = 10.0 ** p["logMh"]
        Rh = p["Rh"]
        vint2 = vint2 + G_KPC * Mh * r / (r + Rh) ** 2

    # 5. disc kinematics (Satoh) and light-weighted observables
    vint = np.sqrt(vint2)
    for B_d, k in discs:
        BV = BV + B_d * (-k * sin_i * cosphi * vint)
        BS2 = BS2 + B_d * (1.0 - k * k) * vint2 / 3.0
    V = BV / B_tot
    S = np.sqrt(BS2 / B_tot)
    LM = B_tot / Sig_tot
    return np.stack([B_tot, V, S, LM])


# ---------------------------------------------------------------------------
# PSF stencil and lattice
# ---------------------------------------------------------------------------
def stencil(spec: GridSpec):
    """Offsets (a, b) in fine-lattice units within 3 sigma, their Gaussian
    weights w, and the sum W; pad = largest |offset|."""
    s = spec.supersample
    sig = spec.psf_sigma_px * s
    rad2 = (3.0 * sig) ** 2
    pad = int(math.floor(3.0 * sig))
    taps = []
    for b in range(-pad, pad + 1):
        for a in range(-pad, pad + 1):
            if a * a + b * b <= rad2:
                # sigma = 0 is the limit of a vanishing PSF: the single central tap
                w = 1.0 if sig == 0.0 else math.exp(-(a * a + b * b) / (2.0 * sig * sig))
                taps.append((a, b, w))
    W = sum(t[2] for t in taps)
    return taps, W, pad


def lattice_coords(spec: GridSpec):
    """Pixel coordinates of the padded fine lattice: x(u) = (u - pad - (s-1)/2) / s."""
    s = spec.supersample
    _, _, pad = stencil(spec)
    nfx, nfy = spec.nx * s + 2 * pad, spec.ny * s + 2 * pad
    u = np.arange(nfx)
    v = np.arange(nfy)
    x = (u - pad - 0.5 * (s - 1)) / s
    y = (v - pad - 0.5 * (s - 1)) / s
    return x, y, pad


def model_lattice(spec: GridSpec, theta) -> np.ndarray:
    """[4, nfy, nfx] model (B, v, sigma, <L/M>) on the padded fine lattice."""
    x, y, _ = lattice_coords(spec)
    X, Y = np.meshgrid(x, y)
    return point_model(spec, theta, X, Y)


def convolve_lattice(spec: GridSpec, f: np.ndarray) -> np.ndarray:
    """PSF average at every pixel centre of lattice maps f [..., nfy, nfx]:
    F(p) = sum over taps of w f(centre(p) + offset) / W."""
    taps, W, pad = stencil(spec)
    s = spec.supersample
    h = (s - 1) // 2
    out = np.zeros(f.shape[:-2] + (spec.ny, spec.nx), dtype=f.dtype)
    for a, b, w in taps:
        v0 = pad + h + b
        u0 = pad + h + a
        out += w * f[..., v0: v0 + spec.ny * s: s, u0: u0 + spec.nx * s: s]
    return out / W


def psf_maps(spec: GridSpec, theta) -> np.ndarray:
    """[4, ny, nx] PSF-averaged (B, v, sigma, <L/M>) at every pixel centre.

    psf_mode 0 (Sec. 3.1): each of the four model maps is averaged over the
    PSF.  psf_mode 1 (luminosity-weighted moments): the PSF averages the
    light B, the first moment B v, the second moment B (sigma^2 + v^2) and
    the mass density B / <L/M>; the observed velocity is their ratio to the
    averaged light, the dispersion the square root of the second moment minus
    v^2, and <L/M> the averaged light over the averaged mass."""
    f = model_lattice(spec, theta)
    if getattr(spec, "psf_mode", 0) == 0:
        return convolve_lattice(spec, f)
    B, V, S, LM = f
    q = convolve_lattice(spec, np.stack([B, B * V, B * (S * S + V * V), B / LM]))
    v = q[1] / q[0]
    s2 = q[2] / q[0] - v * v
    sig = np.sqrt(np.where(np.real(s2) > 0, s2, 0.0 * s2))
    return np.stack([q[0], v, sig, q[0] / q[3]])


def psf_pixels(spec: GridSpec, theta, pixels) -> np.ndarray:
    """PSF-averaged (B, v, sigma, <L/M>) at the listed pixels [(i, j), ...],
    [4, n], with the structure of Appendix A, Algorithm 1: each pixel
    evaluates the model at its K own sub-grid points and averages them.
    Cost is K model evaluations per pixel, so it serves grids too large for
    the whole-lattice path."""
    taps, W, _ = stencil(spec)
    s = spec.supersample
    offs = np.array([(a / s, b / s) for a, b, _ in taps])
    wts = np.array([w for _, _, w in taps])
    out = np.zeros((4, len(pixels)))
    lw = getattr(spec, "psf_mode", 0) == 1
    for n, (i, j) in enumerate(pixels):
        vals = point_model(spec, theta, i + offs[:, 0], j + offs[:, 1])
        if lw:          # luminosity-weighted moments, combined as in psf_maps
            B, V, S, LM = vals
            q = np.stack([B, B * V, B * (S * S + V * V), B / LM]) @ wts / W
            v = q[1] / q[0]
            out[:, n] = [q[0], v, math.sqrt(max(q[2] / q[0] - v * v, 0.0)), q[0] / q[3]]
        else:
            out[:, n] = vals @ wts / W
    return out


def psf_maps_alg1(spec: GridSpec, theta) -> np.ndarray:
    """Same as ``psf_maps`` with the structure of Appendix A, Algorithm 1: for
    every pixel, evaluate the model at its K own sub-grid points and average."""
    pix = [(i, j) for j in range(spec.ny) for i in range(spec.nx)]
    return psf_pixels(spec, theta, pix).reshape(4, spec.ny, spec.nx)


# ---------------------------------------------------------------------------
# likelihood
# ---------------------------------------------------------------------------
def valid_masks(data: np.ndarray, err: np.ndarray) -> np.ndarray:
    """Per-map validity: finite data and finite error > 0."""
    return np.isfinite(data) & np.isfinite(err) & (err > 0.0)


def loglike_terms(spec: GridSpec, data: np.ndarray, err: np.ndarray, theta):
    """(chi2 per map [4], normalisation sum ln(2 pi e^2) over valid pixels)."""
    F = psf_maps(spec, theta)
    return _terms_from_maps(F, data, err)


def _terms_from_maps(F, data, err):
    ok = valid_masks(data, err)
    model = [F[0], F[1], F[2], 1.0 / F[3]]       # model M/L = 1 / <L/M>
    chi2 = []
    norm = 0.0
    for m in range(4):
        d = data[m][ok[m]]
        e = err[m][ok[m]]
        res = (model[m][ok[m]] - d) / e
        chi2.append(np.sum(res * res))
        norm += float(np.sum(np.log(2.0 * math.pi * e * e)))
    return chi2, norm


def loglike(spec: GridSpec, data: np.ndarray, err: np.ndarray, theta):
    """log L = sum over the four maps of -1/2 [chi^2 + sum ln(2 pi e^2)]."""
    if not is_valid(spec, theta):
        return -math.inf
    chi2, norm = loglike_terms(spec, data, err, theta)
    total = chi2[0] + chi2[1] + chi2[2] + chi2[3]
    return -0.5 * (total + norm)


def grad_complex_step(spec: GridSpec, data, err, theta, h: float = 1e-30) -> np.ndarray:
    """d log L / d theta by complex step: Im L(theta + i h e_k) / h."""
    theta = np.asarray(theta, dtype=np.float64)
    P = spec.n_params
    g = np.zeros_like(theta)
    if not is_valid(spec, theta):
        return g
    for k in range(P):
        tc = theta.astype(np.complex128)
        tc[k] += 1j * h
        chi2, _ = loglike_terms(spec, data, err, tc)
        g[k] = -0.5 * np.imag(chi2[0] + chi2[1] + chi2[2] + chi2[3]) / h
    return g


def grad_central_fd(spec: GridSpec, data, err, theta, rel: float = 1e-6) -> np.ndarray:
    """Central differences with step h_k = rel * max(|theta_k|, 1)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(spec.n_params):
        hk = rel * max(abs(theta[k]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[k] += hk
        tm[k] -= hk
        g[k] = (loglike(spec, data, err, tp) - loglike(spec, data, err, tm)) / (tp[k] - tm[k])
    return g


def loglike_joint(specs, datas, errs, theta):
    """Several observations of one galaxy, each map set on its own pixel grid
    (the method takes observables mapped on different numbers of pixels, as
    the comparison with DYNAMITE in Sec. 3.2 points out): the
    Gaussian terms of the likelihood simply add over the grids, each grid
    contributing the maps it carries (a map it does not carry has zero
    errors, hence no valid pixels)."""
    return sum(loglike(sp, d, e, theta) for sp, d, e in zip(specs, datas, errs))


def grad_joint_complex_step(specs, datas, errs, theta) -> np.ndarray:
    return sum(grad_complex_step(sp, d, e, theta) for sp, d, e in zip(specs, datas, errs))


def loglike_batch(spec: GridSpec, data, err, thetas) -> np.ndarray:
    return np.array([loglike(spec, data, err, t) for t in np.atleast_2d(thetas)])


def synthetic_data(spec: GridSpec, theta_true, mask, rng) -> Tuple[np.ndarray, np.ndarray]:
    """(data, err) from the noise recipe of ``workloads`` applied to this oracle's maps."""
    import workloads
    F = psf_maps(spec, theta_true)
    maps = np.stack([F[0], F[1], F[2], 1.0 / F[3]])
    err = workloads.error_maps(maps, mask)
    data = workloads.noisy_data(maps, err, rng)
    return data, err
