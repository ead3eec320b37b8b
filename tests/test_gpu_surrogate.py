"""GPU tests of the surrogate network: the MFMA forward/backward kernels and
Adam against the FP64 oracle network (same BF16 operand rounding), the
training targets against the oracle's quadrature, and the surrogate tracer
(including its exact fallback queue) against the oracle's surrogate mode."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2501_06054_amd import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    return sans


@pytest.fixture(scope="module")
def SG():
    from paper_2501_06054_amd import surrogate
    return surrogate


def bf16_weights(SG, seed, scale=1.0):
    w = SG.init_params(seed) * scale
    wt = torch.from_numpy(w.astype(np.float32)).to(torch.bfloat16)
    return wt.cuda(), wt.float().numpy().astype(np.float64)


def test_forward_matches_oracle(S, SG):
    wb, w64 = bf16_weights(SG, 1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(100, 8)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty(100, dtype=torch.float32, device="cuda")
    ws = torch.empty(S.sans_mlp_workspace_bytes(100) // 4, dtype=torch.float32, device="cuda")
    S.sans_mlp_forward(wb, xt, y, ws)
    torch.cuda.synchronize()
    ref = oracle.mlp_forward(w64, x.astype(np.float64), round_bf16=True)
    err = np.abs(y.cpu().numpy() - ref)
    assert err.max() <= 2e-3 * max(1.0, np.abs(ref).max()), err.max()


def test_backward_matches_oracle(S, SG):
    wb, w64 = bf16_weights(SG, 3)
    rng = np.random.default_rng(4)
    n = 67
    x = rng.uniform(-1, 1, size=(n, 8)).astype(np.float32)
    dy = rng.normal(size=n).astype(np.float32)
    xt, dyt = torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    dw = torch.empty(S.sans_mlp_param_count(), dtype=torch.float32, device="cuda")
    ws = torch.empty(S.sans_mlp_workspace_bytes(n) // 4, dtype=torch.float32, device="cuda")
    S.sans_mlp_forward(wb, xt, y, ws)
    S.sans_mlp_backward(wb, xt, dyt, dw, ws)
    torch.cuda.synchronize()
    g = dw.cpu().numpy().astype(np.float64)
    ref = oracle.mlp_backward(w64, x.astype(np.float64), dy.astype(np.float64), round_bf16=True)
    # block by block: W0 b0 W1 b1 W2 b2 W3 b3 W4 b4
    bounds = [0, 2048, 2304]
    for l in range(3):
        bounds += [bounds[-1] + 65536, bounds[-1] + 65536 + 256]
    bounds += [bounds[-1] + 256, bounds[-1] + 257]
    for a, b in zip(bounds[:-1], bounds[1:]):
        num = np.linalg.norm(g[a:b] - ref[a:b])
        den = max(np.linalg.norm(ref[a:b]), 1e-12)
        assert num / den <= 1e-2, (a, b, num / den)


def test_adam_matches_formula(S):
    rng = np.random.default_rng(5)
    n = 1000
    w = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    m = rng.normal(size=n).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=n)).astype(np.float32) * 0.1
    wt, gt, mt, vt = (torch.from_numpy(a.copy()).cuda() for a in (w, g, m, v))
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    S.sans_adam_step(wt, wb, gt, mt, vt, 1e-3, 7)
    torch.cuda.synchronize()
    b1, b2, eps = 0.9, 0.999, 1e-8
    m2 = b1 * m + (1 - b1) * g
    v2 = b2 * v + (1 - b2) * g * g
    w2 = w - 1e-3 * (m2 / (1 - b1**7)) / (np.sqrt(v2 / (1 - b2**7)) + eps)
    assert np.allclose(wt.cpu().numpy(), w2, rtol=1e-5, atol=1e-7)
    assert np.allclose(wb.float().cpu().numpy(), torch.from_numpy(w2).to(torch.bfloat16).float().numpy())


def test_mse_gradient(S):
    y = torch.tensor([1.0, 2.0, 3.0], device="cuda")
    t = torch.tensor([0.5, 2.5, 3.0], device="cuda")
    dy = torch.empty(3, device="cuda")
    loss = torch.zeros(1, device="cuda")
    S.sans_mse_grad(y, t, dy, loss)
    torch.cuda.synchronize()
    assert np.allclose(dy.cpu().numpy(), [1 / 3, -1 / 3, 0.0])
    assert abs(float(loss) - 0.5 / 3) < 1e-7


@pytest.mark.parametrize("model", ["parallelepiped", "spheroid"])
def test_dataset_targets_match_oracle(S, SG, model):
    x = W.surrogate_inputs(model, 40, seed=11)
    xt = torch.from_numpy(x).cuda()
    t = torch.empty(40, dtype=torch.float32, device="cuda")
    rc = S.lib.sans_pq_dataset(SG.KIND[model], S.C.c_void_p(xt.data_ptr()), 40,
                               S.C.c_void_p(t.data_ptr()), 76,
                               S.C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    got = t.cpu().numpy()
    kind = "parallelepiped" if model == "parallelepiped" else "ellipsoid"
    for i in range(40):
        s = (1.0, math.exp(x[i, 1]), math.exp(x[i, 2]))
        p = W.params(kind=kind, mode="quad", size=s, poly=float(x[i, 3]), poly_mask=7,
                     orient_kind="isotropic", quad_n=76)
        q = math.exp(float(x[i, 0]))
        ref = math.log(oracle.pq_avg(p, q) / oracle.pq_avg(p, 0.0))
        assert abs(got[i] - ref) <= 2e-4 + 1e-5 * abs(ref), (i, got[i], ref)


@pytest.mark.parametrize("model,box_hi0", [("parallelepiped", None), ("spheroid", None),
                                           ("parallelepiped", math.log(0.5))])
def test_surrogate_tracer_matches_oracle(S, SG, model, box_hi0):
    # an untrained network with small weights: the check is the plumbing
    # (inputs, network, weight, fallback queue), not the accuracy
    wb, w64 = bf16_weights(SG, 7, scale=0.3)
    wl = W.workload("surrogate_" + model)
    p = wl["params"]
    sg = SG.Surrogate(model)
    sg.wb.copy_(wb)
    if box_hi0 is not None:
        lo, hi = list(sg.lo), list(sg.hi)
        hi[0] = box_hi0
        sg.lo, sg.hi = tuple(lo), tuple(hi)
    m = S.Model(p)
    sg.attach(m.handle)
    n, seed = 20011, 13
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    oracle.set_surrogate(w64, sg.lo, sg.hi)
    ref = oracle.trace(p, n, seed, nthreads=NTHREADS)
    d = det.cpu().numpy()
    assert np.array_equal(d != 0, ref != 0)
    assert abs(d.sum() - ref.sum()) <= 1e-4 * abs(ref.sum())
    nz = ref != 0
    assert np.max(np.abs(d[nz] - ref[nz]) / np.abs(ref[nz])) <= 2e-3
    m.close()


def test_training_reduces_loss(S, SG):
    u, t = SG.make_dataset("spheroid", 200_000, seed=21)
    sg = SG.Surrogate("spheroid", seed=1)
    hist = sg.train(u, t, steps=1500, batch=4096, lr=2e-3, log_every=100)
    first, last = hist[0][1], hist[-1][1]
    assert last < first / 20, (first, last)
