"""GPU test of sans_trace_noalloc, the entry point that allocates nothing
(its per-XCD replicas live in a fixed device array inside the library),
against sans_trace_ex on the same handle, seed and neutron range: same hit
pattern, total within 1e-6 and every hit pixel within 1e-4 relative.  Two
calls in a row share the array, the second on a smaller detector and fewer
neutrons, then an accumulating call and a detector over the limit."""
import sys

import numpy as np
import pytest
import torch

from paper_2501_06054_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sans


def same_detector(a, b, where):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a != 0, b != 0), f"{where}: hit patterns differ"
    assert abs(a.sum() - b.sum()) <= 1e-6 * abs(b.sum()), f"{where}: totals {a.sum()} vs {b.sum()}"
    nz = b != 0
    rel = np.abs(a[nz] - b[nz]) / np.abs(b[nz])
    assert rel.max() <= 1e-4, f"{where}: worst pixel {rel.max():.3g}"


def test_noalloc_matches_trace_ex_on_two_calls(S):
    runs = [("coreshell_py", 3_000_000, 2, 7), ("tiny_sphere", 400_000, 1, 0)]
    for name, n, seed, first in runs:
        log(f"noalloc: {name} n={n} seed={seed} first={first}")
        p = dict(W.workload(name)["params"])
        m = S.Model(p)
        ref = m.trace(n, seed, first=first)
        det = torch.full((p["ny"], p["nx"]), 7.0, dtype=torch.float64, device="cuda")   # overwritten
        S.sans_trace_noalloc(m.handle, first, n, seed, 0, 0, det)
        torch.cuda.synchronize()
        same_detector(det, ref, f"{name} overwrite")
        # accumulate a second range onto the first
        S.sans_trace_noalloc(m.handle, first + n, n, seed, 0, S.SANS_ACCUMULATE, det)
        m.trace(n, seed, det=ref, first=first + n, accumulate=True)
        torch.cuda.synchronize()
        same_detector(det, ref, f"{name} accumulate")
        m.close()


def test_noalloc_rejects_a_detector_over_the_limit(S):
    log("noalloc: 1024 x 1024 detector is refused")
    p = dict(W.workload("tiny_sphere")["params"])
    p["nx"] = p["ny"] = 1024
    m = S.Model(p)
    det = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SansError) as e:
        S.sans_trace_noalloc(m.handle, 0, 1000, 1, 0, 0, det)
    assert e.value.status == S.SANS_E_INVALID_ARG
    m.close()
