"""CPU pins of the oracle's Hayter-Penfold structure factor (charged hard
spheres with a screened Coulomb tail in the mean spherical approximation;
named in Tables I-II of the paper without a formula):

- no charge: the mean spherical approximation of hard spheres is the
  Percus-Yevick one, so S is the oracle's pinned Percus-Yevick closed form;
- low density: S - 1 = rho c^(K) + O(rho^2) with c the zero-density direct
  correlation function, -1 in the core and -beta U outside: the core's
  transform -4 pi (sin K - K cos K)/K^3 and the tail's by SciPy's adaptive
  quadrature of 4 pi/K int_1^inf x (-beta U) sin(K x) dx;
- the grid: twice as fine gives the same S;
- the C tracer's S is the solver's.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import msa


@pytest.mark.parametrize("eta", [0.05, 0.2, 0.35])
def test_uncharged_is_percus_yevick(eta):
    R = 50.0
    q = np.geomspace(1e-4, 0.3, 40)
    got = msa.s_of_q(q, R, eta, 0.0, 2.0)
    want = np.array([oracle.py_sq(x, R, eta) for x in q])
    # the grid's O(h^2) error (h = sigma/1024) is largest at the deep minimum
    assert np.max(np.abs(got / want - 1)) < 1e-5


@pytest.mark.parametrize("uc,ks", [(1.0, 1.0), (3.0, 3.0), (0.5, 0.5)])
def test_low_density_limit(uc, ks):
    eta = 1e-5
    rho = 6 * eta / math.pi
    K = np.array([0.05, 0.5, 2.0, 5.0, 9.0])
    s = msa.s_of_q(K / 2.0, 1.0, eta, uc, ks)       # radius 1: q sigma = K

    def tail(k):
        f = lambda x: x * (-uc * math.exp(-ks * (x - 1)) / x)
        a = integrate.quad(f, 1.0, 200.0, weight="sin", wvar=k, limit=400)[0]
        return 4 * math.pi / k * a

    want = [-4 * math.pi * (math.sin(k) - k * math.cos(k)) / k**3 + tail(k) for k in K]
    got = (s - 1.0) / rho
    assert np.allclose(got, want, rtol=2e-3, atol=2e-3), (got, want)


def test_grid_refinement():
    q = np.geomspace(1e-3, 0.2, 25)
    a = msa.s_of_q(q, 40.0, 0.15, 4.0, 1.2)
    b = msa.s_of_q(q, 40.0, 0.15, 4.0, 1.2, nin=2048, n=131072)
    assert np.max(np.abs(a / b - 1)) < 2e-6


def test_c_tracer_evaluates_the_solver():
    eta, uc, ks = 0.12, 6.0, 1.8
    oracle.set_msa(eta, uc, ks)
    q = np.geomspace(1e-3, 0.1, 15)
    got = [oracle.msa_sq(x, 45.0, eta, uc, ks) for x in q]
    assert np.allclose(got, msa.s_of_q(q, 45.0, eta, uc, ks), rtol=1e-13, atol=0)
    # a repulsive tail lowers the forward structure factor below the
    # uncharged (Percus-Yevick) one
    assert msa.s_of_q(1e-4, 45.0, eta, uc, ks)[0] < oracle.py_sq(1e-4, 45.0, eta)
