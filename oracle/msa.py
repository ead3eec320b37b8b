"""The Hayter-Penfold structure factor of the oracle (TEST INFRASTRUCTURE,
with the rest of oracle/): charged hard spheres of diameter sigma with the
screened Coulomb (hard-core Yukawa) interaction

    beta U(r) = inf (r < sigma),  beta U(r) = U_c (sigma/r) exp(-kappa (r - sigma)) (r > sigma),

in the mean spherical approximation of Hayter and Penfold (Mol. Phys. 42,
109 (1981)): the Ornstein-Zernike equation h = c + rho c * h closed by
h(r) = -1 inside the core and c(r) = -beta U(r) outside it.  (For a charge
Z on spheres of diameter sigma in a medium of Bjerrum length l_B, U_c =
Z^2 l_B / (sigma (1 + kappa sigma / 2)^2).)

Solved plainly on a radial grid (units of sigma): x_i = i h, h = 1/1024,
i < N = 65536 (to x = 64), the three-dimensional Fourier transforms as
sine transforms (SciPy's DST-I), iterating on gamma = h - c: c = -1 - gamma
inside the core, -beta U outside, the mean of the two at x = 1 (the jump);
c^ = transform of c; gamma^ = rho c^2 / (1 - rho c^); gamma = inverse
transform of gamma^.  The fixed point is followed from the uncharged
spheres (U_c = 0, the Percus-Yevick hard spheres) up to the given U_c in
equal steps of at most 1 in U_c, each solved by Anderson mixing (6
differences, mixing 0.3) from the previous stage's gamma, to 1e-8 on the
way and until gamma changes by less than 1e-12 at the end; every iterate
must keep 1 - rho c^ > 0 (the physical branch), else the solver fails.
The structure factor at any K = q sigma is then S = 1 / (1 - rho c^(K))
with c^ = 4 pi / K int_0^1 x c(x) sin(K x) dx (Simpson on the grid's 1024
intervals) plus the tail's closed form
-4 pi U_c (kappa sigma sin K + K cos K) / (K ((kappa sigma)^2 + K^2)).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy import fft

N = 65536          # grid points (x < 64 sigma)
NIN = 1024         # grid intervals inside the core (h = 1/1024)


def _tail(x, uc, ks):
    return uc * np.exp(-ks * (x - 1.0)) / x


@lru_cache(maxsize=16)
def inside_c(eta: float, uc: float, ks: float, tol: float = 1e-12, max_iter: int = 400,
             nin: int = NIN, n: int = N) -> np.ndarray:
    """c(x) on the core's grid x_i = i/nin, i = 0..nin (the value at x = 1
    is the inside limit, -1 - gamma(1)); the solver's grid has n points of
    spacing 1/nin."""
    NIN, N = nin, n
    h = 1.0 / NIN
    L = N * h
    rho = 6.0 * eta / math.pi
    i = np.arange(1, N)
    x = i * h
    dk = math.pi / L
    K = np.arange(1, N) * dk
    inside, at1 = x < 1.0 - 0.5 * h, np.abs(x - 1.0) < 0.5 * h
    u = np.where(x > 1.0, _tail(x, uc, ks), 0.0)

    def closure(g, us):
        c = np.where(inside, -1.0 - g, -us * u)
        c[at1] = 0.5 * ((-1.0 - g[at1]) + (-us * uc))
        return c

    def step(g, us):
        """gamma -> the next gamma at the contact potential us * U_c, or None
        when 1 - rho c^ <= 0 somewhere (off the physical branch)."""
        c = closure(g, us)
        ch = 4.0 * math.pi * h / K * 0.5 * fft.dst(x * c, type=1)
        d = 1.0 - rho * ch
        if not np.all(d > 0.0):
            return None
        gh = rho * ch * ch / d
        return dk / (2.0 * math.pi**2 * x) * 0.5 * fft.dst(K * gh, type=1)

    def anderson(g, us, stage_tol):
        hist_g, hist_f = [], []
        m, beta = 6, 0.3
        for _ in range(max_iter):
            gn = step(g, us)
            if gn is None:
                raise RuntimeError(f"MSA iterate left the physical branch (eta={eta}, U_c={uc}, kappa sigma={ks})")
            f = gn - g
            err = float(np.max(np.abs(f)))
            if not math.isfinite(err):
                break
            if err < stage_tol:
                return gn
            hist_g.append(g.copy())
            hist_f.append(f.copy())
            if len(hist_g) > m:
                hist_g.pop(0)
                hist_f.pop(0)
            if len(hist_f) > 1:
                dF = np.array([hist_f[k + 1] - hist_f[k] for k in range(len(hist_f) - 1)]).T
                dG = np.array([hist_g[k + 1] - hist_g[k] for k in range(len(hist_g) - 1)]).T
                coef, *_ = np.linalg.lstsq(dF, f, rcond=None)
                g = g + beta * f - (dG + beta * dF) @ coef
            else:
                g = g + beta * f
        raise RuntimeError(f"MSA iteration did not converge (eta={eta}, U_c={uc}, kappa sigma={ks})")

    # continuation in the contact potential: U_c s / S for s = 1..S
    stages = max(1, math.ceil(uc))
    g = np.zeros(N - 1)
    for s_ in range(1, stages + 1):
        g = anderson(g, s_ / stages, tol if s_ == stages else max(tol, 1e-8))
    # gamma at x = 0 (the transform's limit) and on the core's grid
    c = closure(g, 1.0)
    ch = 4.0 * math.pi * h / K * 0.5 * fft.dst(x * c, type=1)
    if not np.all(1.0 - rho * ch > 0.0):
        raise RuntimeError(f"MSA solution unphysical (1 - rho c^ <= 0; eta={eta}, U_c={uc}, kappa sigma={ks})")
    gh_final = rho * ch * ch / (1.0 - rho * ch)
    g0 = dk / (2.0 * math.pi**2) * float(np.sum(K * K * gh_final))
    gin = np.concatenate([[g0], g[:NIN]])          # x = 0, h, ..., 1
    return -1.0 - gin


def c_hat(K, eta: float, uc: float, ks: float, nin: int = NIN, n: int = N) -> np.ndarray:
    """The direct correlation function's transform at K = q sigma (array)."""
    K = np.atleast_1d(np.asarray(K, dtype=np.float64))
    cin = inside_c(eta, uc, ks, nin=nin, n=n)
    x = np.linspace(0.0, 1.0, nin + 1)
    w = np.full(nin + 1, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    w *= (1.0 / nin) / 3.0
    s = np.sin(np.outer(K, x))
    inner = 4.0 * math.pi / K * (s @ (w * x * cin))
    tail = -4.0 * math.pi * uc * (ks * np.sin(K) + K * np.cos(K)) / (K * (ks * ks + K * K))
    return inner + tail


def s_of_q(q, radius: float, eta: float, uc: float, ks: float, nin: int = NIN, n: int = N) -> np.ndarray:
    """S(q) of spheres of radius `radius` (A), q in 1/A."""
    K = 2.0 * radius * np.atleast_1d(np.asarray(q, dtype=np.float64))
    return 1.0 / (1.0 - 6.0 * eta / math.pi * c_hat(K, eta, uc, ks, nin=nin, n=n))
