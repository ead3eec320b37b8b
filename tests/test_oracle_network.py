"""CPU pins of the oracle's surrogate network and of its surrogate mode.

- The FP64 network's gradient (orc_mlp_backward, no operand rounding) against
  central finite differences of its forward pass (orc_mlp_forward), on a few
  hundred parameters sampled from every block: a wrong index, a transposed
  weight, a missing SiLU derivative or a dropped bias term fails it.
- The first layer's [in][out] layout on a network with one active path,
  where a transposed W0 would move the gradient to another row.
- The surrogate mode's domain: a size distribution that does not scale all
  three axes together (poly > 0, poly_mask != 7) was never seen in training,
  so the weight is the exact quadrature average throughout, bit for bit the
  quadrature mode's.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2501_06054_amd import workloads as W

NP = 199_937
# offsets of the parameter blocks: W0[8][256] b0 W1[256][256] b1 W2 b2 W3 b3 W4[256] b4
BLOCKS = {"W0": (0, 2048), "b0": (2048, 2304)}
_o = 2304
for _l in (1, 2, 3):
    BLOCKS[f"W{_l}"] = (_o, _o + 65536)
    BLOCKS[f"b{_l}"] = (_o + 65536, _o + 65792)
    _o += 65792
BLOCKS["W4"] = (_o, _o + 256)
BLOCKS["b4"] = (_o + 256, _o + 257)
assert _o + 257 == NP


def random_network(seed, bias=0.2):
    """He-normal weights and N(0, bias^2) biases, so that every block carries
    gradient."""
    rng = np.random.default_rng(seed)
    w = np.zeros(NP)
    fan = {"W0": 8, "W1": 256, "W2": 256, "W3": 256, "W4": 256}
    for name, (a, b) in BLOCKS.items():
        if name.startswith("W"):
            w[a:b] = rng.normal(0.0, math.sqrt((1.0 if name == "W4" else 2.0) / fan[name]), size=b - a)
        else:
            w[a:b] = rng.normal(0.0, bias, size=b - a)
    return w


def test_parameter_count():
    assert oracle.mlp_param_count() == NP


def test_gradient_against_central_differences():
    w = random_network(21)
    rng = np.random.default_rng(22)
    n = 9
    x = rng.uniform(-1.0, 1.0, size=(n, 8))
    dy = rng.normal(size=n)
    g = oracle.mlp_backward(w, x, dy, round_bf16=False)
    # 40 parameters of every block (all of the small ones)
    picks = []
    for name, (a, b) in BLOCKS.items():
        k = min(40, b - a)
        picks.extend(rng.choice(np.arange(a, b), size=k, replace=False).tolist())
    gmax = np.abs(g).max()
    for j in picks:
        h = 1e-5 * max(1.0, abs(w[j]))
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        fp = float(dy @ oracle.mlp_forward(wp, x))
        fm = float(dy @ oracle.mlp_forward(wm, x))
        fd = (fp - fm) / (2.0 * h)
        # central differences: O(h^2) truncation, O(eps |f| / h) rounding
        assert abs(fd - g[j]) <= 1e-7 * gmax + 1e-6 * abs(g[j]), (j, fd, g[j])


def test_first_layer_layout():
    """W0 is stored [in][out]: on a network with a single path (hidden unit 0
    of every layer, large biases keep it in SiLU's increasing range), only
    column 0 of W0 carries gradient, and each of its entries matches a
    central difference; a transposed W0 would put it in row 0."""
    w = np.zeros(NP)
    a0, _ = BLOCKS["W0"]
    # one path: input k -> unit 0 of every layer -> output, all in SiLU's
    # near-linear positive range (large bias keeps z > 0, SiLU'(z) > 0)
    for l in (1, 2, 3):
        a, _ = BLOCKS[f"W{l}"]
        w[a + 0 * 256 + 0] = 1.0
        b, _ = BLOCKS[f"b{l}"]
        w[b] = 4.0
    w[BLOCKS["b0"][0]] = 4.0
    w[BLOCKS["W4"][0]] = 1.0
    rng = np.random.default_rng(5)
    x = rng.uniform(-1.0, 1.0, size=(6, 8))
    dy = np.ones(6)
    g = oracle.mlp_backward(w, x, dy, round_bf16=False)
    gw0 = g[a0:a0 + 2048].reshape(8, 256)
    # only column 0 (hidden unit 0) carries gradient
    assert np.all(gw0[:, 1:] == 0.0)
    col = gw0[:, 0]
    for k in range(8):
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[a0 + k * 256] += h
        wm[a0 + k * 256] -= h
        fd = (oracle.mlp_forward(wp, x).sum() - oracle.mlp_forward(wm, x).sum()) / (2 * h)
        assert abs(fd - col[k]) <= 1e-7 * np.abs(col).max(), (k, fd, col[k])
    # a transposed W0 ([out][in]) would put the gradient in row 0 instead
    assert np.count_nonzero(gw0[0, :]) == 1


@pytest.mark.parametrize("mask", [1, 3, 4])
def test_partial_size_mask_takes_the_exact_average(mask):
    """An untrained network with large biases changes the weight wherever it
    is used: with poly_mask 7 the surrogate detector differs from the
    quadrature detector, with any other mask it equals it exactly."""
    w = random_network(7, bias=0.5) * 0.3
    wl = W.workload("surrogate_spheroid")
    lo, hi = W.SURROGATE_BOX["spheroid"]
    oracle.set_surrogate(w, lo, hi)
    n, seed = 3001, 17
    p_sur = dict(wl["params"], poly=0.2, poly_mask=mask, quad_n=24)
    p_quad = dict(p_sur, mode="quad")
    d_sur = oracle.trace(p_sur, n, seed, nthreads=4)
    d_quad = oracle.trace(p_quad, n, seed, nthreads=4)
    assert np.array_equal(d_sur, d_quad)
    p7 = dict(p_sur, poly_mask=7)
    d7 = oracle.trace(p7, n, seed, nthreads=4)
    d7q = oracle.trace(dict(p7, mode="quad"), n, seed, nthreads=4)
    assert not np.allclose(d7, d7q, rtol=1e-3)


# ---------------------------------------------------------------- the in-domain judge

def _judged_setup(seed=11):
    p = dict(W.workload("quad_parallelepiped")["params"], mode="surrogate", quad_n=24)
    w = random_network(seed, bias=0.05) * 0.2
    lo, hi = W.SURROGATE_BOX["parallelepiped"]
    return p, w, lo, hi


def test_judge_everywhere_gives_the_exact_average():
    """tol = 0 flags every bin: the surrogate mode's weights are then the
    quadrature mode's, bit for bit; tol = infinity flags none and leaves the
    unjudged surrogate."""
    p, w, lo, hi = _judged_setup()
    n, seed = 600, 5
    oracle.set_surrogate(w, lo, hi)
    _, w_free, _ = oracle.trace_debug(p, n, seed)
    k, _ = oracle.surrogate_judge(p, 0.0, 64)
    assert k == 64
    pix, w_all, _ = oracle.trace_debug(p, n, seed)
    qpix, w_quad, _ = oracle.trace_debug(dict(p, mode="quad"), n, seed)
    assert np.array_equal(pix, qpix)
    assert np.array_equal(w_all, w_quad)
    k, _ = oracle.surrogate_judge(p, math.inf, 64)
    assert k == 0
    _, w_none, _ = oracle.trace_debug(p, n, seed)
    assert np.array_equal(w_none, w_free)
    assert not np.allclose(w_free, w_quad, rtol=1e-3)   # the untrained network is far off


def test_judge_bounds_the_error_of_what_it_keeps():
    """A finite tolerance: neutrons of flagged bins take the exact weight;
    the others keep the network's, within the tolerance at their bin's edges
    and midpoint (and, the bins being fine, within twice it anywhere)."""
    p, w, lo, hi = _judged_setup()
    oracle.set_surrogate(w, lo, hi)
    nb = 256
    _, err = oracle.surrogate_judge(p, math.inf, nb)
    tol = float(np.quantile(err, 0.5))
    k, _ = oracle.surrogate_judge(p, tol, nb)
    assert 0 < k < nb
    n, seed = 1500, 6
    pix, w_j, q = oracle.trace_debug(p, n, seed)
    _, w_x, _ = oracle.trace_debug(dict(p, mode="quad"), n, seed)
    hit = pix >= 0
    x0 = np.log(q[hit] * p["size"][0])
    b = np.clip(np.floor((x0 - lo[0]) / (hi[0] - lo[0]) * nb).astype(int), 0, nb - 1)
    bin_err = np.maximum.reduce([err[2 * b], err[2 * b + 1], err[2 * b + 2]])
    flagged = bin_err > tol
    r = np.abs(np.log(w_j[hit] / w_x[hit]))
    assert np.all(r[flagged] == 0.0)
    assert np.all(r[~flagged] <= 2.0 * tol), float(np.max(r[~flagged]))
    assert flagged.any() and (~flagged).any()
