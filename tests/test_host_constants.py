"""CPU checks of the library's host set-up against the oracle, through the
C ABI's host-only entry (no GPU): the number-averaged particle volume of
every parameter set the GPU parity tests use, and the weight's scale."""
import importlib.util
import math
import os

import pytest

import oracle
from paper_2501_06054_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _parity_sets():
    spec = importlib.util.spec_from_file_location("gpu_parity_sets", os.path.join(HERE, "test_gpu_parity.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.PER_NEUTRON


SETS = _parity_sets()
SHAPE_INDEPENDENT = set(W.SHAPE_INDEPENDENT_KINDS)


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    return sans


@pytest.mark.parametrize("name", sorted(SETS))
def test_mean_volume_and_weight_scale_match_the_oracle(S, name):
    p, _ = SETS[name]
    if p["mode"] == "surrogate":
        pytest.skip("the surrogate needs an attached network")
    mv, ws = S.sans_debug_weight_scale(p)
    omc = 2 * math.sin(0.5 * p["cone_alpha"]) ** 2
    domega = 2 * math.pi * omc
    if p["kind"] in SHAPE_INDEPENDENT:
        assert ws == pytest.approx(1e10 * domega * 1e-8, rel=1e-13)
        return
    want = oracle.mean_volume(p)
    assert mv == pytest.approx(want, rel=1e-10), name
    assert ws == pytest.approx(1e10 * domega * p["phi"] / want, rel=1e-10), name
