"""CPU pins of the oracle's independent size draws: each size with its own
width draws its own relative factor y_k ~ N(1, p_k^2) kept where positive
(the paper's Gaussian rule, Methods "Polydispersity and orientational
distributions", Eq. (8); the cylinder's parameter vector carries separate
spreads of r and L, Results "Small angle scattering models").

- one width on the sphere is the paper's single Gaussian draw (same word,
  same table, same weight);
- <V> against moments of SciPy's truncated normal, size by size;
- the drawn factors against SciPy's truncated normal (Kolmogorov-Smirnov),
  mutually uncorrelated and uncorrelated with the geometry draws;
- the words: y_0 from (block 2, x), y_1 and y_2 from (block 3, x) and
  (block 3, y), looked up in the width's table; enabling them shifts no other
  draw;
- the weight is the one of the drawn sizes: l dOmega (phi/<V>) F^2 S.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2501_06054_amd import workloads as W


def truncnorm(p):
    return stats.truncnorm(a=-1.0 / p, b=np.inf, loc=1.0, scale=p)


def test_one_width_is_the_papers_single_draw():
    base = W.params(kind="sphere", size=(50.0, 0, 0), poly_kind="gaussian")
    a = dict(base, poly=0.2, poly_mask=1)
    b = dict(base, poly_sep=(0.2, 0.0, 0.0))
    pa, wa, _ = oracle.trace_debug(a, 3000, 5)
    pb, wb, _ = oracle.trace_debug(b, 3000, 5)
    assert np.array_equal(pa, pb)
    assert np.allclose(wa, wb, rtol=1e-14, atol=0)
    assert oracle.mean_volume(a) == pytest.approx(oracle.mean_volume(b), rel=1e-14)


@pytest.mark.parametrize("kind,size,widths,power,vol", [
    ("sphere", (50.0, 0, 0), (0.2, 0, 0), (3, 0, 0), lambda s: 4 / 3 * math.pi * s[0] ** 3),
    ("cylinder", (20.0, 400.0, 0), (0.15, 0.25, 0), (2, 1, 0), lambda s: math.pi * s[0] ** 2 * s[1]),
    ("ellipsoid", (20.0, 40.0, 120.0), (0.1, 0.2, 0.3), (1, 1, 1),
     lambda s: 4 / 3 * math.pi * s[0] * s[1] * s[2]),
    ("parallelepiped", (20.0, 40.0, 120.0), (0.3, 0.0, 0.1), (1, 1, 1), lambda s: s[0] * s[1] * s[2]),
    ("elliptical_cylinder", (20.0, 30.0, 200.0), (0.0, 0.2, 0.25), (1, 1, 1),
     lambda s: math.pi * s[0] * s[1] * s[2]),
])
def test_mean_volume_from_truncated_normal_moments(kind, size, widths, power, vol):
    p = W.params(kind=kind, size=size, poly_kind="gaussian", poly_sep=widths)
    want = vol(size)
    for w, e in zip(widths, power):
        if w > 0 and e > 0:
            want *= truncnorm(w).moment(e)
    assert oracle.mean_volume(p) == pytest.approx(want, rel=1e-9)


@pytest.fixture(scope="module")
def sep_draws():
    p = W.workload("poly_sep_parallelepiped")["params"]
    return p, oracle.trace_debug_ex(p, 20000, 9)


def test_factors_follow_their_distributions(sep_draws):
    p, ex = sep_draws
    for k, width in enumerate(p["poly_sep"]):
        y = ex[:, 11 + k]
        d, pval = stats.kstest(y, truncnorm(width).cdf)
        assert pval > 1e-3, (k, d, pval)
        assert y.mean() == pytest.approx(truncnorm(width).mean(), abs=4 * width / math.sqrt(y.size))


def test_factors_are_independent(sep_draws):
    _, ex = sep_draws
    cols = [ex[:, 11], ex[:, 12], ex[:, 13], ex[:, 2], ex[:, 7]]   # y_0, y_1, y_2, q, theta
    r = np.corrcoef(np.vstack(cols))
    lim = 4.0 / math.sqrt(ex.shape[0])
    for i in range(3):
        for j in range(i + 1, len(cols)):
            assert abs(r[i, j]) < lim, (i, j, r[i, j])


def test_words_of_the_draws():
    p = W.workload("poly_sep_parallelepiped")["params"]
    n, seed, first = 500, 7, 123456789
    ex = oracle.trace_debug_ex(p, n, seed, first=first)
    words = oracle.philox_stream(seed, first, n, 4).reshape(n, 4, 4)
    M = p["table_size"]
    picks = [(2, 0), (3, 0), (3, 1)]
    for k, (b, wd) in enumerate(picks):
        tab = oracle.table_truncnorm(M, p["poly_sep"][k])
        want = [max(0.0, oracle.table_lookup(tab, oracle.uniform(int(x)))) for x in words[:, b, wd]]
        assert np.allclose(ex[:, 11 + k], want, rtol=0, atol=0), k
    # with the second and third widths off, block 3 is not drawn: nothing else moves
    ex1 = oracle.trace_debug_ex(dict(p, poly_sep=(p["poly_sep"][0], 0.0, 0.0)), n, seed, first=first)
    assert np.array_equal(ex1[:, 11], ex[:, 11])
    assert np.array_equal(ex1[:, 2:11], ex[:, 2:11])
    assert np.all(ex1[:, 12:14] == 1.0)


def test_weight_is_that_of_the_drawn_sizes():
    wl = W.workload("poly_sep_cylinder")
    p = wl["params"]
    ex = oracle.trace_debug_ex(p, 400, wl["seed"])
    mv = oracle.mean_volume(p)
    omc = 1.0 - math.cos(p["cone_alpha"])
    for row in ex:
        pix, w, q = int(row[0]), row[1], row[2]
        if pix < 0:
            continue
        sizes = tuple(s * y for s, y in zip(p["size"], row[11:14]))
        fixed = dict(p, size=sizes, poly_sep=(0.0, 0.0, 0.0))
        f2 = oracle.form_f2(fixed, q, row[3:6], 1.0, row[7:10])
        want = row[10] * 1e10 * 2 * math.pi * omc * p["phi"] / mv * f2
        assert w == pytest.approx(want, rel=1e-12)
