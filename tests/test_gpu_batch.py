"""GPU tests of the batched path (sans_trace_batch): every experiment equals
the plain per-experiment trace on the same random streams; a subset matches
the oracle; graph replays and the tuning cache behave."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2501_06054_amd import workloads as W
from tests.parity_bars import check_detector, oracle_detector_sparse

pytestmark = pytest.mark.gpu

# The batched kernel and the plain per-experiment kernels inline the same
# per-neutron code, but each is compiled on its own, so FMA contraction may
# differ in the last bit of an FP32 weight: the two agree per pixel to 1e-6,
# far below any error a wrong parameter, table or random stream would make.
SAME_EXPERIMENT_RTOL = 1e-6

NTHREADS = max(1, min(16, os.cpu_count() or 1))


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    return sans


def _small_batch(n_exp=48, n_lo=2e4, n_hi=3e5):
    return W.batch_experiments(n_exp=n_exp, seed=4096, nx=128, n_lo=n_lo, n_hi=n_hi)


def _run_batch(S, exps, tune_cache=None, seeds=None):
    out = torch.empty((len(exps), 128, 128), dtype=torch.float64, device="cuda")
    S.sans_trace_batch([x["params"] for x in exps], [x["n"] for x in exps],
                       seeds if seeds is not None else [x["seed"] for x in exps], out,
                       tune_cache=tune_cache)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_batch_equals_plain(S):
    exps = _small_batch()
    got = _run_batch(S, exps)
    for e, x in enumerate(exps):
        m = S.Model(x["params"])
        ref = m.trace(x["n"], x["seed"], exp_id=e).cpu().numpy()
        m.close()
        assert np.array_equal(got[e] != 0, ref != 0), e
        assert np.allclose(got[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0), e


def test_batch_matches_oracle_subset(S):
    # Pixel parity is judged where pixels hold many neutrons (about 100 per
    # pixel of the 128x128 detector at 1e6 neutrons); with a handful per
    # pixel a pixel can be one neutron whose amplitude sits near a zero of
    # F, which only the per-neutron bar (with its w_max term) governs.
    exps = _small_batch(n_lo=6e5, n_hi=2e6)
    got = _run_batch(S, exps)
    for e in (0, 1, 2, 3, 5, 8, 13, 21):
        x = exps[e]
        ref = oracle.trace(x["params"], x["n"], x["seed"], exp_id=e, nthreads=NTHREADS)
        g = got[e]
        assert np.array_equal(g != 0, ref != 0), e
        assert abs(g.sum() - ref.sum()) <= 1e-6 * abs(ref.sum()), e
        nz = ref != 0
        assert np.max(np.abs(g[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-4, e


def test_batch_graph_replay_and_new_values(S):
    exps = _small_batch(n_exp=16)
    a = _run_batch(S, exps)
    b = _run_batch(S, exps)                       # graph replay, same inputs
    assert np.allclose(a, b, rtol=1e-12, atol=0)
    seeds = [x["seed"] + 100 for x in exps]       # same shape, new values
    c = _run_batch(S, exps, seeds=seeds)
    for e in (0, 7, 15):
        x = exps[e]
        m = S.Model(x["params"])
        ref = m.trace(x["n"], seeds[e], exp_id=e).cpu().numpy()
        m.close()
        assert np.allclose(c[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0)


def test_batch_zero_and_ragged_counts(S):
    exps = _small_batch(n_exp=6)
    exps[2]["n"] = 0
    exps[4]["n"] = 1
    exps[5]["n"] = (1 << 18) + 3
    got = _run_batch(S, exps)
    assert float(np.abs(got[2]).sum()) == 0.0
    for e in (4, 5):
        x = exps[e]
        ref = oracle.trace(x["params"], x["n"], x["seed"], exp_id=e, nthreads=NTHREADS)
        assert np.array_equal(got[e] != 0, ref != 0)
        if x["n"] == 1:
            # one neutron: the per-neutron bar, |dw| <= 1e-5 w_max + 1e-4 |w|, w_max = |w|
            assert abs(got[e].sum() - ref.sum()) <= 1.1e-4 * abs(ref.sum())
        else:
            assert abs(got[e].sum() - ref.sum()) <= 1e-6 * abs(ref.sum())


def test_batch_tuning_cache(S, tmp_path):
    exps = _small_batch(n_exp=8)
    path = str(tmp_path / "tune.json")
    a = _run_batch(S, exps, tune_cache=path)
    assert os.path.exists(path)
    entries = json.load(open(path))
    assert len(entries) == 1
    (entry,) = entries.values()
    # the tile searched over 2^16 .. 2^20 (and halved or doubled for the
    # cost-weighted split), the split and the workgroups per compute unit
    assert entry["tile"] in [1 << k for k in range(15, 22)]
    assert entry["split"] in (0, 1)
    assert entry["occ"] == 1          # a 128 x 128 histogram leaves room for one workgroup per CU
    b = _run_batch(S, exps, tune_cache=path)   # read back
    assert np.allclose(a, b, rtol=SAME_EXPERIMENT_RTOL, atol=0)


@pytest.mark.parametrize("tile,split,occ", [(1 << 16, 0, 1), (1 << 15, 1, 1), (1 << 17, 1, 2), (1 << 16, 0, 4)])
def test_batch_schedules_give_the_same_detectors(S, tmp_path, tile, split, occ):
    """Any schedule read from the tuning cache (tile size, split, workgroups
    per CU) traces the same experiments: every detector equals its plain
    trace.  64 x 64 detectors, whose LDS histogram lets four workgroups share
    a compute unit."""
    exps = W.batch_experiments(n_exp=24, seed=4096, nx=64, n_lo=2e4, n_hi=3e5)
    total = float(sum(x["n"] for x in exps))
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    key = f"E{len(exps)}_S{int(round(np.log2(total)))}_D64x64_CU{cu}"
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        json.dump({key: {"tile": tile, "split": split, "occ": occ, "ms": 0.0}}, f)
    out = torch.empty((len(exps), 64, 64), dtype=torch.float64, device="cuda")
    S.sans_trace_batch([x["params"] for x in exps], [x["n"] for x in exps], [x["seed"] for x in exps], out,
                       tune_cache=path)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert json.load(open(path))[key]["split"] == split       # read, not re-tuned
    for e, x in enumerate(exps):
        m = S.Model(x["params"])
        ref = m.trace(x["n"], x["seed"], exp_id=e).cpu().numpy()
        m.close()
        assert np.array_equal(got[e] != 0, ref != 0), e
        assert np.allclose(got[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0), e


def test_batch_rejects_mismatched_detectors(S):
    exps = _small_batch(n_exp=2)
    p1 = dict(exps[1]["params"], nx=64, ny=64)
    out = torch.empty((2, 128, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SansError):
        S.sans_trace_batch([exps[0]["params"], p1], [10, 10], [1, 1], out)


def test_batch_rejects_attenuation_and_guides(S):
    exps = _small_batch(n_exp=2)
    p1 = dict(exps[1]["params"], mu_att=50.0)
    out = torch.empty((2, 128, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(S.SansError):
        S.sans_trace_batch([exps[0]["params"], p1], [10, 10], [1, 1], out)
    p2 = dict(exps[1]["params"], guide_len=10.0)
    with pytest.raises(S.SansError):
        S.sans_trace_batch([exps[0]["params"], p2], [10, 10], [1, 1], out)


def test_batch_gaussian_sizes(S):
    """Experiments with the paper's Gaussian size rule mixed with Schulz ones:
    each equals its plain trace, and two match the oracle."""
    exps = _small_batch(n_exp=12, n_lo=2e5, n_hi=6e5)
    for e in range(0, 12, 2):
        exps[e]["params"] = dict(exps[e]["params"], poly_kind="gaussian",
                                 poly=max(exps[e]["params"]["poly"], 0.05))
    got = _run_batch(S, exps)
    for e, x in enumerate(exps):
        m = S.Model(x["params"])
        ref = m.trace(x["n"], x["seed"], exp_id=e).cpu().numpy()
        m.close()
        assert np.allclose(got[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0), e
    for e in (0, 2):
        x = exps[e]
        ref = oracle.trace(x["params"], x["n"], x["seed"], exp_id=e, nthreads=NTHREADS)
        assert np.array_equal(got[e] != 0, ref != 0), e
        assert abs(got[e].sum() - ref.sum()) <= 1e-6 * abs(ref.sum()), e


def test_batch_extra_models(S):
    """Barbells and capped cylinders (each experiment with its own cap rule),
    hollow and core-shell bodies, polymer micelles and shape-independent
    models mixed with the other models: each equals its plain trace, and the
    extra models match the oracle."""
    exps = _small_batch(n_exp=42, n_lo=2e5, n_hi=5e5)
    caps = {1: dict(kind="barbell", size=(20.0, 300.0, 35.0), poly_mask=7, quad_n=40),
            4: dict(kind="capped_cylinder", size=(30.0, 120.0, 45.0), poly=0.1, poly_mask=7, quad_n=23),
            7: dict(kind="barbell", size=(15.0, 80.0, 15.0), poly_mask=7, quad_n=76),
            8: dict(kind="hollow_prism", size=(30.0, 50.0, 150.0), shell=2.0, poly_mask=7),
            9: dict(kind="micelle", size=(40.0, 25.0, 0.0), sld=(1e-6, 0.5e-6, 6.3e-6),
                    extra=(60.0, 4000.0, 3500.0, 1.0), poly_mask=3),
            10: dict(kind="hollow_cylinder", size=(20.0, 150.0, 0.0), shell=6.0, poly_mask=3),
            11: dict(kind="core_shell_cylinder", size=(25.0, 90.0, 0.0), shell=5.0, extra=(2.0, 0.0, 0.0, 0.0),
                     sld=(1e-6, 4e-6, 6.3e-6), poly_mask=3),
            12: dict(kind="core_shell_ellipsoid", size=(20.0, 30.0, 70.0), shell=4.0,
                     sld=(1e-6, 4e-6, 6.3e-6), poly_mask=7),
            13: dict(kind="hollow_prism_thick", size=(40.0, 60.0, 150.0), shell=5.0, poly_mask=0),
            14: dict(kind="teubner_strey", size=(60.0, 150.0, 0.0), extra=(5.0, 0.0, 0.0, 0.0), poly=0.0,
                     sq_phi=0.0),
            15: dict(kind="poly_gauss_coil", size=(60.0, 0.0, 0.0), extra=(20.0, 1.0, 0.0, 0.0), poly=0.0,
                     sq_phi=0.0),
            16: dict(kind="guinier", size=(45.0, 0.0, 0.0), extra=(3.0, 0.0, 0.0, 0.0), poly=0.0, sq_phi=0.0),
            17: dict(kind="power_law", extra=(1e-4, 3.2, 0.0, 0.0), poly=0.0, sq_phi=0.0),
            18: dict(kind="star_polymer", size=(70.0, 0.0, 0.0), extra=(3.0, 6.0, 0.0, 0.0), poly=0.0,
                     sq_phi=0.0),
            19: dict(kind="linear_pearls", size=(25.0, 12.0, 0.0), extra=(6.0, 0.0, 0.0, 0.0), poly_mask=1),
            20: dict(kind="guinier_porod", size=(60.0, 0.0, 0.0), extra=(7.0, 1.0, 3.5, 0.0), poly=0.0,
                     sq_phi=0.0),
            21: dict(kind="fractal_core_shell", size=(20.0, 250.0, 0.0), shell=5.0, sld=(1e-6, 3e-6, 6.3e-6),
                     extra=(0.0, 2.5, 0.0, 0.0), poly_mask=1),
            22: dict(kind="polymer_excl_volume", size=(80.0, 0.0, 0.0), extra=(10.0, 0.588, 0.0, 0.0), poly=0.0,
                     sq_phi=0.0),
            23: dict(kind="core_shell_bicelle", size=(30.0, 40.0, 0.0), shell=8.0, sld=(1e-6, 4e-6, 6.3e-6),
                     extra=(6.0, 2.5e-6, 0.0, 0.0), poly_mask=3),
            24: dict(kind="core_shell_parallelepiped", size=(30.0, 50.0, 90.0), sld=(1e-6, 3e-6, 6.3e-6),
                     extra=(4.0, 6.0, 3.0, 0.0), poly_mask=7),
            25: dict(kind="stacked_disks", size=(80.0, 25.0, 0.0), shell=8.0, sld=(1e-6, 4e-6, 6.3e-6),
                     extra=(5.0, 4.0, 0.0, 0.0), poly_mask=1),
            26: dict(kind="sc_paracrystal", size=(30.0, 150.0, 0.0), extra=(0.08, 0.0, 0.0, 0.0), poly_mask=1),
            27: dict(kind="core_shell", size=(30.0, 0.0, 0.0), shell=8.0, sld=(1e-6, 3e-6, 6.3e-6), poly_mask=1,
                     sq_phi=0.1, sq_radius=38.0, sq_kind="sticky_hard_sphere", sq_extra=(0.25, 0.0)),
            28: dict(kind="sphere", size=(35.0, 0.0, 0.0), poly_mask=1, sq_phi=0.15, sq_radius=36.0,
                     sq_kind="square_well", sq_extra=(0.8, 1.5)),
            29: dict(kind="mass_surface_fractal", size=(200.0, 20.0, 0.0), extra=(30.0, 2.0, 2.4, 0.0), poly=0.0,
                     sq_phi=0.0),
            30: dict(kind="gel_fit", size=(35.0, 120.0, 0.0), extra=(3.0, 0.6, 2.2, 0.0), poly=0.0, sq_phi=0.0),
            31: dict(kind="superball", size=(25.0, 0.0, 0.0), extra=(3.0, 0.0, 0.0, 0.0), quad_n=12, poly_mask=1,
                     sq_phi=0.0),
            32: dict(kind="lamellar_hg_stack_caille", size=(14.0, 8.0, 70.0), sld=(-0.4e-6, 3e-6, 6.3e-6),
                     extra=(15.0, 0.1, 0.0, 0.0), poly=0.0, sq_phi=0.0),
            33: dict(kind="lamellar_stack_paracrystal", size=(30.0, 75.0, 0.0), sld=(1e-6, 0.0, 6.3e-6),
                     extra=(10.0, 5.0, 0.0, 0.0), poly=0.0, sq_phi=0.0),
            34: dict(kind="core_shell_bicelle_elliptical_belt_rough", size=(25.0, 40.0, 0.0), shell=6.0,
                     sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 2.5e-6, 1.7, 3.0), poly_mask=3),
            35: dict(kind="raspberry", size=(60.0, 12.0, 0.0), sld=(1e-6, 4e-6, 6.3e-6), extra=(30.0, 0.2, 0.0, 0.0),
                     poly_mask=1),
            36: dict(kind="pearl_necklace", size=(25.0, 40.0, 6.0), sld=(1e-6, 3e-6, 6.3e-6), extra=(8.0, 0, 0, 0),
                     quad_n=16, poly_mask=1),
            37: dict(kind="binary_hard_sphere", size=(45.0, 15.0, 0.0), sld=(1e-6, 4e-6, 6.3e-6), phi=0.25,
                     extra=(0.08, 0, 0, 0), poly=0.0, sq_phi=0.0),
            38: dict(kind="adsorbed_layer", size=(1500.0, 0.0, 0.0), shell=2.0, sld=(1.5e-6, 0.0, 6.3e-6),
                     extra=(10.0, 0, 0, 0), poly=0.0, sq_phi=0.0),
            39: dict(kind="pringle", size=(40.0, 8.0, 0.0), extra=(0.002, 0.015, 0, 0), quad_n=10, poly_mask=3),
            40: dict(kind="sphere", size=(40.0, 0.0, 0.0), poly_mask=1, sq_phi=0.12, sq_radius=44.0,
                     sq_kind="hayter_msa", sq_extra=(6.0, 1.8)),
            41: dict(kind="flexible_cylinder", size=(15.0, 800.0, 0.0), extra=(80.0, 0, 0, 0), quad_n=24,
                     poly_mask=3)}
    for e, over in caps.items():
        exps[e]["params"] = dict(exps[e]["params"], **over)
    got = _run_batch(S, exps)
    for e, x in enumerate(exps):
        m = S.Model(x["params"])
        ref = m.trace(x["n"], x["seed"], exp_id=e).cpu().numpy()
        m.close()
        assert np.allclose(got[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0), e
    for e in (1, 4, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32, 33, 34, 35, 36, 37, 38, 39, 40, 41):
        x = exps[e]
        ref = oracle.trace(x["params"], x["n"], x["seed"], exp_id=e, nthreads=NTHREADS)
        assert np.array_equal(got[e] != 0, ref != 0), e
        assert abs(got[e].sum() - ref.sum()) <= 1e-6 * abs(ref.sum()), e


def test_full_batch_4096(S):
    """The whole set of 4096 experiments (sum of N about 8.7e9) in one
    batched launch, in the launch configuration the benchmark times: every
    experiment equals its plain trace on the same streams (1e-6 per pixel),
    and 128 of them -- 64 drawn with a seeded generator and the 64 smallest
    -- match the oracle (hit patterns identical, totals within 1e-6, pixels
    within 1e-4 or, where the pixels hold few neutrons, the summed
    per-neutron bar)."""
    exps = W.batch_experiments()
    assert len(exps) == 4096
    log(f"full batch: {len(exps)} experiments, sum N = {sum(x['n'] for x in exps):.4g}")
    got = _run_batch(S, exps)
    for e, x in enumerate(exps):
        m = S.Model(x["params"])
        ref = m.trace(x["n"], x["seed"], exp_id=e).cpu().numpy()
        m.close()
        assert np.array_equal(got[e] != 0, ref != 0), e
        assert np.allclose(got[e], ref, rtol=SAME_EXPERIMENT_RTOL, atol=0), e
    log("full batch: every experiment equals its plain trace")
    rng = np.random.default_rng(4096)
    picked = set(rng.choice(len(exps), size=64, replace=False).tolist())
    picked |= set(np.argsort([x["n"] for x in exps], kind="stable")[:64].tolist())
    for e in sorted(picked):
        x = exps[e]
        ref, bar = oracle_detector_sparse(x["params"], x["n"], x["seed"], exp_id=e)
        check_detector(got[e], ref, f"experiment {e} ({x['params']['kind']}, n={x['n']})", **bar)
    log(f"full batch: {len(picked)} experiments match the oracle")
