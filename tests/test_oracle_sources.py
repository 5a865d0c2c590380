"""Pins of the oracle's extended sources: the top-hat disc (the 0.3 cm beam
of Sec. 3.2, the 0.1 cm collimated beam of the curved-vs-voxelised case)
and the uniform rectangle (uniform incidence, Sec. 3.1 and Sec. 4).

A source above a clear, index-matched plate shines straight down through
it: there is no refraction, no Fresnel loss and (mu_a = 1e-9 /cm) no
interaction, so each packet leaves the bottom face at its emission (x, y)
with unit weight.  The escape image of that face is then the source's
spatial distribution binned on the pixels: pixel k holds N A_k / A_src
packets on average, where A_k is
the area the pixel shares with the source.  The areas come from geometry
written here (an exact rectangle overlap; a disc overlap integrated along
one axis in closed form), so a mistake in the sampling -- r = R xi instead
of R sqrt(xi), a half side taken as a full side, a shifted centre -- moves
whole rings or rows of pixels by many standard errors.  Each pixel count is
binomial; every pixel must pass an exact binomial test at 1e-5 and the
chi-square over pixels lie within its 4-sigma band."""
import math

import numpy as np
import pytest


def _plate_with_source(W, source, mua=1e-9, L=0.4, half=2.0):
    prims = [{"kind": "box", "c": [0.0, 0.0, -0.5 * L], "half": [half, half, 0.5 * L]}]
    regions = [W._region([0], mua, 0.0, 0.0, 1.0)]   # index matched with the air
    sc = W._scene("source_plate", prims, regions, source, None, pad=0.05)
    return sc


def _disc_area_in_rect(R, x0, x1, y0, y1):
    """Area of the disc x^2 + y^2 <= R^2 inside [x0, x1] x [y0, y1]: the
    integral over x of the chord's overlap with [y0, y1], the chord running
    over |y| <= sqrt(R^2 - x^2).  With x = R sin(t) the integrand is smooth
    between its kinks (where a chord end crosses y0 or y1), so
    Gauss-Legendre panels split there integrate it to rounding."""
    a, b = max(x0, -R), min(x1, R)
    if a >= b:
        return 0.0
    cuts = {math.asin(a / R), math.asin(b / R)}
    for y in (y0, y1):           # a chord end crosses y where x = +-sqrt(R^2 - y^2)
        if abs(y) < R:
            for x in (-math.sqrt(R * R - y * y), math.sqrt(R * R - y * y)):
                if a < x < b:
                    cuts.add(math.asin(x / R))
    pts = sorted(cuts)
    tg, wg = np.polynomial.legendre.leggauss(40)
    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        t = 0.5 * (hi - lo) * tg + 0.5 * (hi + lo)
        h = R * np.cos(t)                       # chord half-length at x = R sin t
        f = np.clip(np.minimum(h, y1) - np.maximum(-h, y0), 0.0, None) * R * np.cos(t)
        total += 0.5 * (hi - lo) * float(np.dot(wg, f))
    return total


def _rect_area_in_rect(hx, hy, x0, x1, y0, y1):
    return max(0.0, min(x1, hx) - max(x0, -hx)) * max(0.0, min(y1, hy) - max(y0, -hy))


def _check_image(img, expect, N):
    """Exact binomial test per pixel (two-sided tail probability at least
    1e-5, about 4.4 sigma where the normal limit holds) and the chi-square
    over the pixels expecting at least 5 packets, within 4 of its sigma."""
    from scipy.stats import binom
    p = expect / N
    inside = expect > 0
    assert np.all(img[~inside] == 0.0), "counts in pixels the source does not reach"
    k_obs, p_in = img[inside], p[inside]
    tail = 2 * np.minimum(binom.cdf(k_obs, N, p_in), binom.sf(k_obs - 1, N, p_in))
    assert tail.min() >= 1e-5, tail.min()
    big = expect >= 5
    k = int(big.sum())
    chi2 = float(np.sum(((img - expect)[big]) ** 2 / (N * p * (1 - p))[big]))
    assert abs(chi2 - k) <= 4.0 * math.sqrt(2.0 * k), (chi2, k)


def _pixel_edges(lo, hi, n):
    return np.linspace(lo, hi, n + 1)


@pytest.mark.parametrize("R,centre", [(0.3, (0.0, 0.0)), (0.17, (0.05, -0.08))])
def test_disc_source_fills_its_area_uniformly(orc, W, R, centre):
    cx, cy = centre
    src = {"kind": "disc", "c": [cx, cy, 0.02], "r": R, "u": [0.0, 0.0, -1.0]}
    sc = _plate_with_source(W, src)
    n_pix, lo, hi = 12, -0.36, 0.36
    sc["detector"] = {"face": 4, "lo": [lo + cx, lo + cy], "hi": [hi + cx, hi + cy], "dims": [n_pix, n_pix]}
    N = 200_000
    r = orc.run(sc, 2024, N)
    assert r["escaped_face"][4] == N and r["interactions"] == 0   # every packet leaves downward
    e = _pixel_edges(lo, hi, n_pix)
    area = np.array([[_disc_area_in_rect(R, e[i], e[i + 1], e[j], e[j + 1]) for i in range(n_pix)]
                     for j in range(n_pix)])
    assert area.sum() == pytest.approx(math.pi * R * R, rel=1e-10)
    _check_image(r["image"], N * area / (math.pi * R * R), N)


@pytest.mark.parametrize("half,centre", [((0.3, 0.17), (0.0, 0.0)), ((0.11, 0.25), (-0.04, 0.07))])
def test_rect_source_fills_its_area_uniformly(orc, W, half, centre):
    hx, hy = half
    cx, cy = centre
    src = {"kind": "rect", "c": [cx, cy, 0.02], "half": [hx, hy], "u": [0.0, 0.0, -1.0]}
    sc = _plate_with_source(W, src)
    n_pix, lo, hi = 10, -0.35, 0.35
    sc["detector"] = {"face": 4, "lo": [lo + cx, lo + cy], "hi": [hi + cx, hi + cy], "dims": [n_pix, n_pix]}
    N = 200_000
    r = orc.run(sc, 77, N)
    assert r["escaped_face"][4] == N and r["interactions"] == 0
    e = _pixel_edges(lo, hi, n_pix)
    area = np.array([[_rect_area_in_rect(hx, hy, e[i], e[i + 1], e[j], e[j + 1]) for i in range(n_pix)]
                     for j in range(n_pix)])
    assert area.sum() == pytest.approx(4 * hx * hy, rel=1e-12)
    _check_image(r["image"], N * area / (4 * hx * hy), N)


def test_disc_overlap_geometry():
    # the overlap integrator against cases with known areas: a full disc, a
    # half plane, a quadrant, and a square inscribed in the disc
    R = 0.7
    assert _disc_area_in_rect(R, -1, 1, -1, 1) == pytest.approx(math.pi * R * R, rel=1e-12)
    assert _disc_area_in_rect(R, 0, 1, -1, 1) == pytest.approx(0.5 * math.pi * R * R, rel=1e-12)
    assert _disc_area_in_rect(R, 0, 1, 0, 1) == pytest.approx(0.25 * math.pi * R * R, rel=1e-12)
    s = R / math.sqrt(2.0)
    assert _disc_area_in_rect(R, -s, s, -s, s) == pytest.approx(2 * R * R, rel=1e-12)
    # a circular segment: the part beyond x = R/2 is R^2 (theta - sin theta)/2, theta = 2 acos(1/2)
    th = 2 * math.acos(0.5)
    assert _disc_area_in_rect(R, R / 2, 1, -1, 1) == pytest.approx(0.5 * R * R * (th - math.sin(th)), rel=1e-12)


def test_disc_sampling_mutation_is_caught(orc, W):
    # the check above rejects a disc sampled with r = R xi: emulate that
    # distribution's pixel counts (density 1/(2 pi R r)) by drawing it here
    # and binning it like the image; the same check must fail
    R, n_pix, lo, hi, N = 0.3, 12, -0.36, 0.36, 200_000
    rng = np.random.default_rng(5)
    rr, ph = R * rng.uniform(size=N), 2 * math.pi * rng.uniform(size=N)
    img, _, _ = np.histogram2d(rr * np.sin(ph), rr * np.cos(ph), bins=[n_pix, n_pix], range=[[lo, hi], [lo, hi]])
    e = _pixel_edges(lo, hi, n_pix)
    area = np.array([[_disc_area_in_rect(R, e[i], e[i + 1], e[j], e[j + 1]) for i in range(n_pix)]
                     for j in range(n_pix)])
    with pytest.raises(AssertionError):
        _check_image(img, N * area / (math.pi * R * R), N)
