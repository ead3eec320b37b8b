"""CPU pins of the oracle's neutron guide (a straight supermirror channel
upstream of the source aperture, followed back wall by wall).

- The reflection count: the oracle's bounce-by-bounce backward flight gives
  R(Q_x)^n_x R(Q_y)^n_y with n_x, n_y the number of wall planes the
  unfolded straight line crosses between the exit and the entrance
  (|floor((x_entrance + w/2)/w)|), computed here independently.
- Perfect mirrors whose exit covers the beam leave every weight 1, so the
  detector equals the one without a guide; a guide whose exit is narrower
  than the beam's backward footprint zeroes exactly the neutrons that miss
  its exit.
- The reflectivity: R0 up to Qc, then falling monotonically; never above 1
  or below 0; no guide: weight 1.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_06054_amd import workloads as W


def _refl(p, q):
    r0, qc, m, a, wc = p["guide_r0"], p["guide_qc"], p["guide_m"], p["guide_alpha"], p["guide_wc"]
    if q <= qc:
        return r0
    return max(0.0, 0.5 * r0 * (1 - math.tanh((q - m * qc) / wc)) * (1 - a * (q - qc)))


def test_reflection_count_matches_the_unfolded_line():
    p = W.params(guide_len=12.0, guide_w=0.02, guide_h=0.015, guide_gap=0.3, guide_m=3.0)
    rng = np.random.default_rng(4)
    hw, hh = p["guide_w"] / 2, p["guide_h"] / 2
    seen = set()
    for _ in range(3000):
        src = np.array([rng.uniform(-0.005, 0.005), rng.uniform(-0.005, 0.005), p["src_z"]])
        ang = rng.uniform(-6e-3, 6e-3, size=2)
        ki = np.array([ang[0], ang[1], 1.0])
        ki /= np.linalg.norm(ki)
        lam = rng.uniform(4.0, 8.0)
        got = oracle.guide_weight(p, src, ki, lam)
        t = p["guide_gap"] / ki[2]
        ex, ey = src[0] - t * ki[0], src[1] - t * ki[1]
        if abs(ex) > hw or abs(ey) > hh:
            assert got == 0.0
            continue
        xu = ex - ki[0] / ki[2] * p["guide_len"]
        yu = ey - ki[1] / ki[2] * p["guide_len"]
        nx = abs(math.floor((xu + hw) / p["guide_w"]))
        ny = abs(math.floor((yu + hh) / p["guide_h"]))
        seen.add((nx, ny))
        qx, qy = 4 * math.pi * abs(ki[0]) / lam, 4 * math.pi * abs(ki[1]) / lam
        want = _refl(p, qx) ** nx * _refl(p, qy) ** ny
        assert got == pytest.approx(want, rel=1e-12, abs=1e-300)
    # the sample covers no, one and several reflections on both axes
    assert {0, 1, 2} <= {a for a, _ in seen} and {0, 1, 2} <= {b for _, b in seen}


def test_reflectivity_shape():
    p = W.params(guide_len=5.0, guide_m=2.0)
    qs = np.linspace(0.0, 0.2, 2001)
    r = np.array([_refl(p, q) for q in qs])
    assert np.all((r >= 0) & (r <= 1))
    assert np.all(r[qs <= p["guide_qc"]] == p["guide_r0"])
    above = qs > p["guide_qc"]
    assert np.all(np.diff(r[above]) <= 1e-15)
    # a single reflection: the ray leaves the axis at the exit and meets one wall
    src = np.array([0.0, 0.0, p["src_z"]])
    for ang in (3e-3, 5e-3, 7e-3):
        ki = np.array([ang, 0.0, 1.0])
        ki /= np.linalg.norm(ki)
        t = p["guide_gap"] / ki[2]
        ex = -t * ki[0]
        xu = ex - ki[0] / ki[2] * p["guide_len"]
        assert abs(math.floor((xu + p["guide_w"] / 2) / p["guide_w"])) == 1
        q = 4 * math.pi * abs(ki[0]) / 6.0
        assert oracle.guide_weight(p, src, ki, 6.0) == pytest.approx(_refl(p, q), rel=1e-13)
    assert oracle.guide_weight(W.params(), src, np.array([0.0, 0.0, 1.0]), 6.0) == 1.0


def test_perfect_guide_leaves_the_detector_unchanged():
    base = W.workload("tiny_sphere")["params"]
    perfect = dict(base, guide_len=10.0, guide_w=0.2, guide_h=0.2, guide_r0=1.0, guide_qc=1e3)
    n = 50_000
    a = oracle.trace(base, n, 3, transmitted=True)
    b = oracle.trace(perfect, n, 3, transmitted=True)
    assert np.array_equal(a, b)


def test_narrow_exit_cuts_the_beam():
    p = W.params(guide_len=4.0, guide_w=0.006, guide_h=0.2, guide_gap=2.0, guide_r0=1.0, guide_qc=1e3)
    n = 20_000
    _, w = oracle.transmitted_debug(p, n, 21)
    # the backward footprint at the exit plane, 2 m behind the source aperture
    st = np.zeros(n * 4, dtype=np.uint32)
    oracle.lib().orc_philox_stream(21, 0, n, 1, 0, st.ctypes.data_as(oracle.C.POINTER(oracle.C.c_uint32)))
    u = (st.reshape(n, 4).astype(np.float64) + 0.5) * 2.0**-32
    sx = (u[:, 0] - 0.5) * p["src_w"]
    tx = (u[:, 2] - 0.5) * p["slit_w"]
    dz = p["slit_z"] - p["src_z"]
    ex = sx - p["guide_gap"] * (tx - sx) / dz
    inside = np.abs(ex) <= p["guide_w"] / 2
    assert 0.2 < inside.mean() < 0.9
    assert np.array_equal(w > 0, inside)
    np.testing.assert_allclose(w[inside], 1.0, rtol=0, atol=0)
