"""Host logic of bench.py (CPU): the per-neutron FP32 flop counts behind the
roofline, the lookup of counter-measured HBM traffic and VALU work, the host
thread count of the CPU baseline, and the one-GPU guard.  No GPU is
touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2501_06054_amd import workloads as W  # noqa: E402


def test_every_workload_has_a_flop_count():
    """Each Monte Carlo or quadrature workload carries an algorithmic FP32
    count (the roofline's numerator); the surrogate ones are timed against
    the exact-average trace instead."""
    for name in W.WORKLOADS:
        mode = W.workload(name)["params"]["mode"]
        algo = bench.algo_flops(name)
        if mode == "surrogate":
            assert algo is None, name
            continue
        assert algo is not None, name
        flops, source = algo
        assert flops > 0 and source, name
        if mode == "quad":
            assert name in bench.QUAD_NODE and name in bench.QUAD_MU, name


def test_reference_configurations_take_the_reference_budget():
    # the four reference configurations
    assert bench.algo_flops("coreshell_py")[0] == 110
    assert bench.algo_flops("tiny_sphere")[0] == 35
    assert bench.algo_flops("oriented_cylinder")[0] == 80
    assert bench.algo_flops("oriented_ellipsoid")[0] == 80
    assert bench.algo_flops("quad_parallelepiped")[0] == bench.own_flops("quad_parallelepiped")
    # the step counts stay a lower bound of them (series forms)
    for name in bench.REFERENCE_FLOPS:
        assert bench.own_flops(name) <= bench.REFERENCE_FLOPS[name], name


def test_paths_name_only_counted_steps():
    for name, steps in bench.PATHS.items():
        for s in steps:
            assert s in bench.STEP, (name, s)
        # every Monte Carlo path flies, scatters, weights and tallies its neutron
        for s in bench.COMMON:
            assert s in steps, (name, s)


def test_quadrature_count_scales_with_its_nodes():
    """The quadrature workloads' count is the weight plus the per-node and
    per-mu-node flops times 76 x 76 and 76 nodes."""
    for name in bench.QUAD_NODE:
        flops = bench.own_flops(name)
        assert flops == bench.STEP["weight"] + bench.QUAD_NODES * bench.QUAD_NODE[name] + 76 * bench.QUAD_MU[name]


def test_peak_follows_the_unit_counts():
    # 256 CUs x 2.4 GHz x 128 FP32 FMA lanes per clock x 2 flops
    assert bench.CUS * bench.CLOCK_GHZ * 128 * 2 / 1e3 == pytest.approx(bench.PEAK_FP32_TFLOPS, rel=2e-3)


def test_roofline_is_the_fp32_fraction(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda *a: None)
    r = bench.roofline_of("coreshell_py", 10**8, 2.0)
    # 110 flops x 1e8 neutrons in 2 ms = 5.5 TFLOP/s
    assert r["achieved"] == pytest.approx(5.5)
    assert r["peak"] == bench.PEAK_FP32_TFLOPS and r["unit"] == "TFLOP/s"
    assert r["frac"] == pytest.approx(5.5 / 157.3, abs=1e-5)
    assert bench.roofline_of("surrogate_parallelepiped", 10, 1.0) is None


def test_host_threads_respects_the_cpu_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.host_threads() == min(3, len(os.sched_getaffinity(0)))
    monkeypatch.setenv("OMP_NUM_THREADS", "")
    assert bench.host_threads() == len(os.sched_getaffinity(0))
    assert bench.cpu_model()


def test_measured_valu_needs_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "valu_counters.md").write_text(
        "| workload | kernel | sources | VALU/neutron | FP32 flops/neutron | FP64/neutron | busy | MHz |\n"
        "|---|---|---|---|---|---|---|---|\n"
        "| wl_a | k_emit<1, 0> | 0123456789abcdef | 11.5 | 201 | 2.2 | 0.93 | 2100 |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    v = bench.measured_valu("wl_a")
    assert v["kernel"] == "k_emit<1, 0>" and v["valu_instr_per_neutron"] == 11.5 and v["clock_mhz"] == 2100
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "fedcba9876543210")
    assert bench.measured_valu("wl_a") is None


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
