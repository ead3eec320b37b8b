"""Host logic of bench.py (CPU): the per-neutron slot model, the lookup of
counter-measured HBM traffic, and the one-GPU guard.  No GPU is touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2501_06054_amd import workloads as W  # noqa: E402


def test_every_workload_has_a_work_count():
    """Each Monte Carlo or quadrature workload carries an algorithmic count
    (the roofline's numerator); the surrogate ones are timed against MFMA."""
    for name in W.WORKLOADS:
        mode = W.workload(name)["params"]["mode"]
        algo = bench.algo_per_neutron(name)
        if mode == "surrogate":
            assert algo is None, name
            continue
        assert algo is not None, name
        slots, flops = algo
        assert slots > 0 and flops >= 0, name
        if mode == "quad":
            assert name in bench.QUAD_NODE and name in bench.QUAD_MU, name


def test_paths_name_only_counted_steps():
    for name, steps in bench.PATHS.items():
        for s in steps:
            assert s in bench.STEP, (name, s)
        # every Monte Carlo path flies, scatters, weights and tallies its neutron
        for s in bench.COMMON:
            assert s in steps, (name, s)


@pytest.mark.parametrize("cls", bench._CLASSES)
def test_step_slots_is_linear_in_the_class_costs(cls):
    unit = tuple(1 if c == cls else 0 for c in bench._CLASSES)
    assert bench.step_slots(unit) == pytest.approx(bench.SLOT_COST[cls])
    assert bench.step_slots(tuple(3 * u for u in unit)) == pytest.approx(3 * bench.SLOT_COST[cls])
    assert bench.step_slots((0,) * len(bench._CLASSES)) == 0.0


def test_quadrature_count_scales_with_its_nodes():
    """The quadrature workloads' count is the Monte Carlo base plus the
    per-node and per-mu-node costs times 76 x 76 and 76 nodes."""
    base = sum(bench.step_slots(bench.STEP[x][0]) for x in bench.QUAD_BASE)
    for name in bench.QUAD_NODE:
        slots, _ = bench.algo_per_neutron(name)
        node = bench.step_slots(bench.QUAD_NODE[name][0])
        mu = bench.step_slots(bench.QUAD_MU[name][0])
        assert slots == pytest.approx(base + bench.QUAD_NODES * node + 76 * mu, abs=0.1)
        assert slots > bench.QUAD_NODES * node


def test_peak_follows_the_unit_counts():
    # 256 CUs x 2.4 GHz x 128 FP32 FMA lanes per clock x 2 flops
    assert bench.CUS * bench.CLOCK_GHZ * 128 * 2 / 1e3 == pytest.approx(bench.PEAK_FP32_TFLOPS, rel=2e-3)
    assert bench.PEAK_VALU_TSLOTS == pytest.approx(bench.PEAK_FP32_TFLOPS / 2)


def test_measured_traffic_needs_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic.md").write_text(
        "| workload | kernel | sources | fetch B/neutron | write B/neutron |\n"
        "|---|---|---|---|---|\n"
        "| wl_a | trace_call | 0123456789abcdef | 9.5 | 10.25 |\n"
        "| wl_b | trace_call | fedcba9876543210 | 1.0 | 2.0 |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    assert bench.measured_traffic("wl_a", "trace_call", 1000) == (9500.0, 10250.0)
    assert bench.measured_traffic("wl_b", "trace_call", 1000) is None     # other sources
    assert bench.measured_traffic("wl_a", "other_kernel", 1000) is None
    assert bench.measured_traffic("wl_c", "trace_call", 1000) is None


def test_measured_traffic_without_a_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("coreshell_py", "trace_call", 10) is None


def test_kernel_source_hash_tracks_the_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2501_06054_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("x")
    (csrc / "notes.txt").write_text("ignored")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h1 = bench.kernel_source_hash()
    (csrc / "notes.txt").write_text("still ignored")
    assert bench.kernel_source_hash() == h1
    (csrc / "a.hip").write_text("y")
    assert bench.kernel_source_hash() != h1
    assert len(h1) == 16 and int(h1, 16) >= 0


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
