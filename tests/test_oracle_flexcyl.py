"""CPU pins of the oracle's flexible cylinder with an elliptical cross-section
(named in Table II of the paper without a formula; the reading: Kholodenko's
closed form for the wormlike chain times the angle-averaged elliptical
cross-section, both by the model's own Gauss-Legendre rule).

- The rigid-rod limit (Kuhn length far above the contour length): the
  chain factor is the thin rod's 2 Si(qL)/(qL) - 2 (1 - cos qL)/(qL)^2
  (SciPy's sine integral).
- The Gaussian-coil limit (contour length far above the Kuhn length, q b
  small): the Debye function of Rg^2 = L b/6, to (q b)^2/20 + 10 b/(3L).
- The two branches of the chain factor join continuously at q b = 3.
- The circular cross-section (eps = 1) is [2 J1(qR)/(qR)]^2 (SciPy's J1);
  the elliptical average against SciPy's adaptive quadrature of the angle
  integral; eps and 1/eps with R scaled give the same ellipse.
- The rule: 48 points against 256 on the workload's parameters.
- The plain flexible cylinder (circular section): the elliptical one at
  eps = 1, the chain times SciPy's [2 J1(qR)/(qR)]^2, forward value and
  mean volume.
- F^2(q -> 0) = (drho pi eps R^2 L)^2 and <V> = pi eps R^2 L (moments of the
  size draw for the mask's sizes).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from paper_2501_06054_amd import workloads as W


@pytest.mark.parametrize("q", [1e-3, 1e-2, 3e-2, 0.1])
def test_rigid_rod_limit(q):
    L = 400.0
    x = q * L
    si, _ = special.sici(x)
    rod = 2 * si / x - 2 * (1 - math.cos(x)) / x**2
    assert oracle.flexcyl_chain(q, L, 1e7, 128) == pytest.approx(rod, rel=1e-8)


@pytest.mark.parametrize("L,b", [(2e5, 20.0), (2e4, 20.0)])
@pytest.mark.parametrize("qrg", [0.1, 0.5, 1.0, 2.0, 5.0])
def test_gaussian_coil_limit(L, b, qrg):
    rg = math.sqrt(L * b / 6)
    q, u = qrg / rg, qrg**2
    debye = 2 * (math.expm1(-u) + u) / u**2
    tol = (q * b) ** 2 / 20 + 10 * b / (3 * L)
    assert abs(oracle.flexcyl_chain(q, L, b, 256) / debye - 1) <= tol


def test_branches_join_at_qb_3():
    L, b = 1000.0, 100.0
    q0 = 3.0 / b
    mid = oracle.flexcyl_chain(q0, L, b, 128)
    lo = oracle.flexcyl_chain(q0 * (1 - 1e-7), L, b, 128)
    hi = oracle.flexcyl_chain(q0 * (1 + 1e-7), L, b, 128)
    assert math.isfinite(mid)
    assert lo == pytest.approx(mid, rel=1e-6) and hi == pytest.approx(mid, rel=1e-6)


@pytest.mark.parametrize("q", [1e-3, 0.02, 0.055, 0.3])
def test_cross_section(q):
    R = 20.0
    lam = (2 * special.j1(q * R) / (q * R)) ** 2
    assert oracle.flexcyl_section(q, R, 1.0, 24) == pytest.approx(lam, rel=1e-12)
    eps = 2.0

    def f(psi):
        r = R * math.sqrt(math.sin(psi) ** 2 + eps**2 * math.cos(psi) ** 2)
        return (2 * special.j1(q * r) / (q * r)) ** 2

    want = integrate.quad(f, 0, math.pi / 2, epsabs=0, epsrel=1e-12)[0] / (math.pi / 2)
    assert oracle.flexcyl_section(q, R, eps, 64) == pytest.approx(want, rel=1e-9)
    # the same ellipse described from its other axis
    assert oracle.flexcyl_section(q, R * eps, 1 / eps, 64) == pytest.approx(want, rel=1e-9)


def test_rule_converges():
    p = W.workload("flexible_cylinder_elliptical")["params"]
    R, L, b, eps, n = p["size"][0], p["size"][1], p["extra"][0], p["extra"][1], p["quad_n"]
    for q in np.geomspace(1e-3, 0.06, 25):
        assert oracle.flexcyl_chain(q, L, b, n) == pytest.approx(oracle.flexcyl_chain(q, L, b, 256), rel=1e-7)
        assert oracle.flexcyl_section(q, R, eps, n) == pytest.approx(oracle.flexcyl_section(q, R, eps, 256),
                                                                     rel=1e-10)


def test_forward_value_and_volume():
    p = W.workload("flexible_cylinder_elliptical")["params"]
    R, L, eps = p["size"][0], p["size"][1], p["extra"][1]
    v = math.pi * eps * R * R * L
    f2 = oracle.form_f2(p, 1e-7, (1e-7, 0.0, 0.0))
    assert f2 == pytest.approx(((p["sld"][0] - p["sld"][2]) * v) ** 2, rel=1e-6)
    assert oracle.mean_volume(p) == pytest.approx(v, rel=1e-14)
    pp = dict(p, poly=0.2, poly_mask=3)
    a = 1 / 0.2**2
    m3 = (a + 1) * (a + 2) / a**2      # <y^3> of the Schulz draw: R^2 L scale together
    assert oracle.mean_volume(pp) == pytest.approx(v * m3, rel=1e-12)


def test_round_section_is_the_ellipse_at_axis_ratio_one():
    """The plain flexible cylinder (circular section) is the elliptical one at
    eps = 1, whose section average reduces to [2 J1(qR)/(qR)]^2 (pinned above
    against SciPy's J1); the forward value is (drho pi R^2 L)^2 and the mean
    volume pi R^2 L with the size moments of the draw."""
    base = dict(W.workload("flexible_cylinder_elliptical")["params"], quad_n=40)
    round_ = dict(base, kind="flexible_cylinder", extra=(base["extra"][0], 0.0, 0, 0))
    ell = dict(base, extra=(base["extra"][0], 1.0, 0, 0))
    R, L, b = base["size"][0], base["size"][1], base["extra"][0]
    for q in np.geomspace(1e-4, 0.3, 30):
        got = oracle.form_f2(round_, q, (q, 0.0, 0.0))
        assert got == pytest.approx(oracle.form_f2(ell, q, (q, 0.0, 0.0)), rel=1e-12)
        lam = (2 * special.j1(q * R) / (q * R)) ** 2
        v = (base["sld"][0] - base["sld"][2]) * math.pi * R * R * L
        assert got == pytest.approx(v * v * oracle.flexcyl_chain(q, L, b, 40) * lam, rel=1e-12)
    assert oracle.form_f2(round_, 1e-8, (1e-8, 0, 0)) == pytest.approx(
        ((base["sld"][0] - base["sld"][2]) * math.pi * R * R * L) ** 2, rel=1e-6)
    for mask, k in ((1, 2), (2, 1), (3, 3)):
        pp = dict(round_, poly=0.2, poly_mask=mask)
        a = 1 / 0.2**2
        mk = {1: 1.0, 2: (a + 1) / a, 3: (a + 1) * (a + 2) / a**2}[k]     # <y^k> of the Schulz draw
        assert oracle.mean_volume(pp) == pytest.approx(math.pi * R * R * L * mk, rel=1e-12)
