"""CPU check of the adjoint's lattice-block scheme (the index arithmetic of
`adj.hip`, restated in Python): the blocks that the bands own tile the padded
lattice, each block's frame holds every pixel that reaches it, the separable
transposed stencil streamed through the pixel-adjoint ring (vertical group
sums, then horizontal taps from the host-built tables) equals the direct
transposed stencil (Sec. 3.1, the PSF average, transposed), and every index
stays inside the LDS layout that the host sizes the launch with.  No GPU."""
import math

import numpy as np
import pytest

DSTRIDE = 11          # vertical table entries per row phase (lag depth <= 10)


def stencil(s, sigma_px):
    """1-D weights g(|k|), half-widths A(|b|) of the circular 3-sigma disc and
    the lag depth D, on the lattice (s points per pixel)."""
    sig = sigma_px * s
    pad = int(math.floor(3.0 * sig))
    rad2 = 9.0 * sig * sig
    gw = [math.exp(-k * k / (2.0 * sig * sig)) if sig > 0 else float(k == 0) for k in range(pad + 1)]
    aof = [max((a for a in range(pad + 1) if a * a + b * b <= rad2), default=-1) for b in range(pad + 1)]
    if sig == 0:
        aof[0] = 0
    return pad, gw, aof, 2 * pad // s, rad2


def adjoint_tables(s, pad, gw, aof, D):
    """Vertical table per row phase: the lags in reach sorted by decreasing
    half-width, grouped by equal half-width ((lag, group, last-of-group),
    weight); horizontal table per (row phase, column phase): per pixel
    column in reach the S offset (-k nlev + groups with A >= |t| - 1) and
    g(|t|).  Zero entries pad both to fixed widths."""
    vt = [[(0, 0, 0, 0.0)] * DSTRIDE for _ in range(s)]
    groups = []
    for ph in range(s):
        lags = sorted(((aof[abs(d * s + ph - pad)], d) for d in range(D + 1) if abs(d * s + ph - pad) <= pad),
                      key=lambda t: (-t[0], t[1]))
        gA, grp = [], -1
        for n, (A, d) in enumerate(lags):
            if n == 0 or A != lags[n - 1][0]:
                grp += 1
                gA.append(A)
            last = int(n + 1 == len(lags) or lags[n + 1][0] != A)
            vt[ph][n] = (d, grp, last, gw[abs(d * s + ph - pad)])
        groups.append(gA)
    nlev = max(1, max(len(g) for g in groups))
    KP = 8 if D <= 6 else 12
    ht = [[(0, 0.0)] * KP for _ in range(s * s)]
    for ph in range(s):
        for i in range(s):
            for k in range(D + 1):
                at = abs(k * s + i - pad)
                l = sum(1 for A in groups[ph] if A >= at)
                if l:
                    ht[ph * s + i][k] = (-k * nlev + l - 1, gw[at])
    return vt, ht, nlev, KP


def ceil_div(a, b):
    return -((-a) // b)


def run_blocks(ny, nx, s, sigma_px, bh, bw, R, mask, rng, end_slip=0):
    pad, gw, aof, D, rad2 = stencil(s, sigma_px)
    vt, ht, nlev, KP = adjoint_tables(s, pad, gw, aof, D)
    rbar = rng.standard_normal((ny, nx)) * mask
    spans = []
    for j in range(ny):
        c = np.nonzero(mask[j])[0]
        spans.append((int(c[0]), int(c[-1])) if len(c) else (1, 0))
    NLR, NLC = (ny - 1) * s + 2 * pad + 1, (nx - 1) * s + 2 * pad + 1
    direct = np.zeros((NLR, NLC))
    for j in range(ny):
        for i in range(nx):
            if rbar[j, i] != 0.0:
                for b in range(-pad, pad + 1):
                    for a in range(-pad, pad + 1):
                        if a * a + b * b <= rad2:
                            direct[j * s + pad + b, i * s + pad + a] += gw[abs(a)] * gw[abs(b)] * rbar[j, i]
    bh, bw = min(bh, ny), min(bw, nx)
    RB = D + 1 + ceil_div(R - 1, s)
    # the host's LDS layout bounds (frame of at most band + D + 1 pixels)
    nrf, ncf = bh + D + 1, bw + D + 1
    nph_max = ceil_div(bh * s + 2 * pad + 1, R) + 1
    out = np.zeros((NLR, NLC))
    owner = np.zeros((NLR, NLC), int)
    own = pad - s // 2
    for j0 in range(0, ny, bh):
        for c0 in range(0, nx, bw):
            j1, c1 = min(ny, j0 + bh), min(nx, c0 + bw)
            Lr0, Lr1 = (0 if j0 == 0 else j0 * s + own), (NLR if j1 == ny else j1 * s + own)
            Lc0, Lc1 = (0 if c0 == 0 else c0 * s + own), (NLC if c1 == nx else c1 * s + own - end_slip)
            jf0, jf1 = max(0, ceil_div(Lr0 - 2 * pad, s)), min(ny, (Lr1 - 1) // s + 1)
            cf0, cf1 = max(0, ceil_div(Lc0 - 2 * pad, s)), min(nx, (Lc1 - 1) // s + 1)
            NR, NC = jf1 - jf0, cf1 - cf0
            assert 1 <= NR <= nrf and 1 <= NC <= ncf
            # the frame holds every pixel whose disc (lattice rows j s .. j s + 2 pad)
            # reaches the block: the pixels just outside it do not
            assert jf0 == 0 or (jf0 - 1) * s + 2 * pad < Lr0
            assert jf1 == ny or jf1 * s > Lr1 - 1
            assert cf0 == 0 or (cf0 - 1) * s + 2 * pad < Lc0
            assert cf1 == nx or cf1 * s > Lc1 - 1
            # rows / columns of the block before the frame's first lattice row /
            # column are reached by no pixel (pad < s / 2); the kernel divides
            # with C semantics, so every index it divides must be non-negative
            rbeg, rend = max(0, Lr0 - jf0 * s), Lr1 - jf0 * s
            xbeg, xend = max(0, Lc0 - cf0 * s), Lc1 - cf0 * s
            assert rbeg >= 0 and xbeg >= 0
            NCP = NC + 2 * D
            nph = ceil_div(rend - rbeg, R)
            assert nph <= nph_max
            ranges = []
            for k in range(nph):
                lo, hi = 1 << 30, -(1 << 30)
                for r in range(rbeg + k * R, min(rend, rbeg + (k + 1) * R)):
                    for jj in range(max(0, ceil_div(r - 2 * pad, s)), min(NR - 1, r // s) + 1):
                        sx, sy = spans[jf0 + jj]
                        cl, ch = max(cf0, sx), min(cf1 - 1, sy)
                        if cl <= ch:
                            A = aof[abs(r - jj * s - pad)]
                            lo = min(lo, (cl - cf0) * s + pad - A)
                            hi = max(hi, (ch - cf0) * s + pad + A)
                lo, hi = max(lo, xbeg), min(hi, xend - 1)
                ranges.append((lo, hi - lo + 1) if hi >= lo else (0, 0))
            ring = np.zeros((RB, NC))
            S = np.zeros((R, NCP, nlev))
            loaded = max(-1, rbeg // s - D - 1)

            def load(rA):
                nonlocal loaded
                qlo, qhi = rA // s, (rA + min(R, rend - rA) - 1) // s
                base = (qlo - D) % RB
                for jj in range(loaded + 1, qhi + 1):
                    slot = base + jj - (qlo - D)
                    assert jj >= 0 and 0 <= slot < 2 * RB
                    ring[slot - RB if slot >= RB else slot] = rbar[jf0 + jj, cf0:cf1] if jj < NR else 0.0
                loaded = max(loaded, qhi)

            load(rbeg)
            for ph_i, rA in enumerate(range(rbeg, rend, R)):
                nrow, qlo = min(R, rend - rA), rA // s
                base = (qlo - D) % RB
                for rl in range(nrow):
                    r = rA + rl
                    assert r >= 0
                    qr, ph = r // s, r % s
                    acc = np.zeros(NC)
                    for (d, grp, last, w) in vt[ph]:
                        slot = base + qr - qlo + D - d
                        assert 0 <= slot < 2 * RB
                        acc = acc + w * ring[slot - RB if slot >= RB else slot]
                        if last:
                            assert grp < nlev
                            S[rl, D:D + NC, grp] = acc
                lo, pw = ranges[ph_i]
                for rl in range(nrow):
                    r = rA + rl
                    flat = S[rl].reshape(-1)
                    for x in range(lo, lo + pw):
                        assert x >= 0
                        qx, ix = x // s, x % s
                        f = 0.0
                        for (off, w) in ht[(r % s) * s + ix]:
                            idx = (qx + D) * nlev + off
                            assert 0 <= idx < NCP * nlev
                            f += w * flat[idx]
                        out[jf0 * s + r, cf0 * s + x] += f
                        owner[jf0 * s + r, cf0 * s + x] += 1
                if rA + R < rend:
                    load(rA + R)
    assert owner.max() <= 1, "a lattice point was evaluated by two blocks"
    done = owner == 1
    assert np.all(direct[~done] == 0.0), "a lattice point that some pixel reaches was skipped"
    scale = max(np.abs(direct).max(), 1e-300)
    return np.abs(out - direct)[done].max() / scale


CASES = [  # (ny, nx, s, PSF sigma in pixels, band_h, band_w, lattice rows per phase)
    (9, 8, 3, 1.0617, 4, 3, 2),
    (12, 11, 5, 1.6986, 5, 4, 1),
    (12, 11, 5, 1.6986, 3, 3, 3),
    (7, 9, 1, 1.5, 2, 3, 4),
    (6, 6, 3, 0.0, 2, 2, 2),
    (20, 21, 3, 0.0, 3, 3, 2),
    (7, 6, 7, 0.05, 2, 3, 1),
    (5, 7, 7, 0.3, 2, 3, 3),
    (8, 9, 5, 1.70, 8, 2, 16),
    (11, 10, 3, 1.0617, 4, 10, 3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}s{c[2]}b{c[4]}x{c[5]}R{c[6]}" for c in CASES])
@pytest.mark.parametrize("maskkind", ["full", "ellipse", "holes"])
def test_blocks_tile_the_lattice_and_match_the_transposed_stencil(case, maskkind):
    ny, nx, s, sig, bh, bw, R = case
    rng = np.random.default_rng(hash((case, maskkind)) % 2 ** 32)
    yy, xx = np.mgrid[0:ny, 0:nx]
    if maskkind == "full":
        mask = np.ones((ny, nx))
    elif maskkind == "ellipse":
        mask = (((yy - ny / 2) / (ny / 2.5)) ** 2 + ((xx - nx / 2) / (nx / 3)) ** 2 <= 1).astype(float)
    else:
        mask = (rng.random((ny, nx)) > 0.4).astype(float)
        mask[0, :] = 0.0
        mask[:, -1] = 0.0
    assert run_blocks(ny, nx, s, sig, bh, bw, R, mask, rng) < 1e-12


@pytest.mark.parametrize("slip,message", [(1, "skipped"), (-1, "two blocks")])
def test_a_planted_tiling_slip_is_caught(slip, message):
    """Ending each inner block's columns one lattice column early (a gap) or
    late (an overlap) fails the tiling check."""
    rng = np.random.default_rng(7)
    with pytest.raises(AssertionError, match=message):
        run_blocks(9, 8, 3, 1.0617, 4, 3, 2, np.ones((9, 8)), rng, end_slip=slip)
