"""CPU pins of the oracle's transmitted (unscattered) beam: each neutron's
straight flight from its source point through its slit point to the
detector, weighted by the slab's transmission exp(-mu chord).

- A pencil beam along the axis: every event lands in the centre pixel with
  weight exp(-mu d), d the slab thickness (normal incidence).
- A divergent beam through a wide slab: the mean weight equals
  E[exp(-mu d / cos theta)] over the beam's directions, the expectation by
  deterministic quadrature over the trapezoidal densities of the
  source-to-slit offsets (each the difference of two uniforms).
- The detector image: the hit abscissa is -(r - 1) x_src + r x_slit with
  r = (z_det - z_src)/(z_slit - z_src), a sum of two uniforms, so the
  column marginal is a trapezoid; the histogram of columns matches its
  integral over each pixel (chi^2), which pins the pixel layout (x along
  the row index, y along the column of rows).
- A beam wider than the slab: with an opaque slab only the neutrons that
  miss it arrive, with weight 1, at the rate the trapezoidal beam profile
  at the slab gives.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import oracle
from paper_2501_06054_amd import workloads as W


def _trapezoid_pdf_nodes(a, b, n=64):
    """Nodes and weights for E[g(Z)], Z = U1 + U2 with U1 ~ U(-a/2, a/2) and
    U2 ~ U(-b/2, b/2): the density is piecewise linear with knots at
    +-(a + b)/2 and +-|a - b|/2; Gauss-Legendre on each of the three pieces."""
    lo, hi = abs(a - b) / 2, (a + b) / 2
    peak = 1.0 / max(a, b)
    knots = [-hi, -lo, lo, hi]
    gx, gw = leggauss(n)
    xs, ws = [], []
    for k in range(3):
        x0, x1 = knots[k], knots[k + 1]
        if x1 <= x0:
            continue
        x = 0.5 * (x1 - x0) * gx + 0.5 * (x1 + x0)
        dens = np.where(np.abs(x) <= lo, peak, peak * (hi - np.abs(x)) / (hi - lo) if hi > lo else peak)
        xs.append(x)
        ws.append(0.5 * (x1 - x0) * gw * dens)
    return np.concatenate(xs), np.concatenate(ws)


def test_pencil_beam_hits_the_centre_with_slab_transmission():
    mu, d = 150.0, 0.002
    p = W.params(src_w=1e-9, src_h=1e-9, slit_w=1e-9, slit_h=1e-9, sample_d=d, mu_att=mu, nx=129, ny=129)
    pix, w = oracle.transmitted_debug(p, 2000, 3)
    assert np.all(pix == 64 * 129 + 64)
    np.testing.assert_allclose(w, math.exp(-mu * d), rtol=1e-12)
    det = oracle.trace(p, 2000, 3, transmitted=True) - oracle.trace(p, 2000, 3)
    assert det.sum() == pytest.approx(2000 * math.exp(-mu * d), rel=1e-12)


def test_divergent_beam_mean_transmission():
    mu, d = 400.0, 0.003
    p = W.params(sample_w=0.05, sample_h=0.05, sample_d=d, mu_att=mu, src_w=0.03, src_h=0.02,
                 slit_w=0.012, slit_h=0.008, src_z=-1.0, nx=257, ny=257, det_w=1.0, det_h=1.0)
    n = 400_000
    _, w = oracle.transmitted_debug(p, n, 11)
    L = p["slit_z"] - p["src_z"]
    x, wx = _trapezoid_pdf_nodes(p["src_w"], p["slit_w"])
    y, wy = _trapezoid_pdf_nodes(p["src_h"], p["slit_h"])
    X, Y = np.meshgrid(x, y, indexing="ij")
    cos_t = L / np.sqrt(X * X + Y * Y + L * L)
    want = float(np.einsum("i,j,ij->", wx, wy, np.exp(-mu * d / cos_t)))
    assert abs(w.mean() - want) <= 4.0 * w.std() / math.sqrt(n) + 1e-12
    # the divergence matters at this size: the normal-incidence value is off
    assert abs(math.exp(-mu * d) - want) > 20.0 * w.std() / math.sqrt(n)


def test_direct_beam_image_is_the_trapezoid():
    p = W.params(src_w=0.03, src_h=0.004, slit_w=0.01, slit_h=0.004, src_z=-2.0, det_z=6.0,
                 det_w=0.2, det_h=0.2, nx=100, ny=100, sample_w=0.2, sample_h=0.2)
    n = 300_000
    pix, w = oracle.transmitted_debug(p, n, 5)
    assert np.all(pix >= 0)
    cols = pix % p["nx"]
    counts = np.bincount(cols, minlength=p["nx"]).astype(float)
    r = (p["det_z"] - p["src_z"]) / (p["slit_z"] - p["src_z"])
    a, b = (r - 1.0) * p["src_w"], r * p["slit_w"]
    edges = np.linspace(-p["det_w"] / 2, p["det_w"] / 2, p["nx"] + 1)

    def cdf(z):
        # CDF of U(-a/2, a/2) + U(-b/2, b/2) by integrating the trapezoid
        zz = np.linspace(-(a + b) / 2, (a + b) / 2, 200001)
        lo, hi = abs(a - b) / 2, (a + b) / 2
        dens = np.where(np.abs(zz) <= lo, 1 / max(a, b), (hi - np.abs(zz)) / (hi - lo) / max(a, b))
        c = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(zz))])
        return np.interp(z, zz, c, left=0.0, right=1.0)

    expect = n * np.diff(cdf(edges))
    used = expect > 5
    chi2 = float(np.sum((counts[used] - expect[used]) ** 2 / expect[used]))
    dof = int(used.sum()) - 1
    assert dof > 10
    assert chi2 / dof < 1.5
    # rows: the vertical extent is the narrower trapezoid of the heights
    rows = pix // p["nx"]
    hy = ((r - 1.0) * p["src_h"] + r * p["slit_h"]) / 2
    ylo, yhi = (rows.min() + 1) * p["det_h"] / p["ny"] - p["det_h"] / 2, rows.max() * p["det_h"] / p["ny"] - p["det_h"] / 2
    assert -hy <= ylo and yhi <= hy
    assert hy < 0.3 * (a + b) / 2


def test_beam_wider_than_slab_passes_around_it():
    # an opaque slab narrower than the beam in x (it spans the beam in y)
    p = W.params(src_w=0.02, src_h=0.004, slit_w=0.02, slit_h=0.004, src_z=-4.0, slit_z=-2.0,
                 sample_w=0.03, sample_h=0.1, sample_d=0.001, mu_att=1e7, det_w=0.3, det_h=0.3)
    n = 400_000
    pix, w = oracle.transmitted_debug(p, n, 9)
    assert np.all(pix >= 0)
    # rays that cut only a corner of the slab (chords of a few micrometres)
    # keep part of their weight; they are rare
    partial = (w > 0.0) & (w < 1.0)
    assert partial.mean() < 1e-3
    # abscissa at the slab: -(r - 1) x_src + r x_slit, r = z_src/(z_src - z_slit) = 2
    r = (0.0 - p["src_z"]) / (p["slit_z"] - p["src_z"])
    a, b = (r - 1.0) * p["src_w"], r * p["slit_w"]
    lo, hi = abs(a - b) / 2, (a + b) / 2
    hw = p["sample_w"] / 2
    # P(|Z| > hw) for the trapezoid with hw inside its sloped part
    assert lo < hw < hi
    tail = (hi - hw) ** 2 / (2 * (hi - lo) * max(a, b))
    want = 2 * tail
    frac = w.mean()
    assert abs(frac - want) <= 4 * math.sqrt(want * (1 - want) / n)
