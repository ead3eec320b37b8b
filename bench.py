"""Benchmark of the SANS sample tracer on one MI355X.

One step = one pass of the whole hot path over one batch: the detector is
cleared and n neutrons are traced (Philox draws, source/slit/slab geometry,
cone sampling, Schulz size draw from the LDS table, core-shell amplitude,
Percus-Yevick S(Q), weight, detector pixel, FP64 tally).  The default workload
is the polydisperse core-shell sphere with hard-sphere S(Q) on a 256x256
detector, 1e8 neutrons per step.

Prints one JSON line (rank 0, one GPU):
  metric/value/unit       neutrons traced per second (whole job)
  roofline                the trace kernel against the VALU issue ceiling
                          (algorithmic lane-op slots per neutron x neutrons per
                          launch / launch time from HIP events on its stream)
  fp32_valu               the same kernel's algorithmic FP32 flops against the
                          FP32 vector peak
  cpu_baseline            the FP64 CPU oracle on a bounded sample of the same
                          workload, on this host's cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
PEAK_FP32_TFLOPS = 157.3
CUS, CLOCK_GHZ = 256, 2.4
# VALU issue ceiling: 4 SIMDs of 16 lanes per CU, one lane-operation per lane
# per clock (a wave64 instruction every 4 clocks per SIMD): 64 lane-slots per
# clock per CU.  FP64 add/mul/fma issue at this rate on MI355X, as unpacked
# FP32 does.
PEAK_VALU_TSLOTS = CUS * CLOCK_GHZ * 1e9 * 64 / 1e12

# Algorithmic work per neutron, counted from the method's steps (the
# derivation is tabulated in the design notes).  Counting rules, per lane:
#   slots: 1 per FP64/FP32/integer add, mul, fma, min/max, compare/select or
#          conversion; 4 per quarter-rate op (32x32->64 integer multiply, FP32
#          reciprocal/sqrt/exp/log); 8 per FP64 reciprocal, divide or sqrt;
#          where a function has a short series below a threshold, the cheaper
#          (series) cost is counted, so the totals are lower bounds.
#   fp32:  FP32 flops of the weight (add/mul 1, fma 2, reciprocal/sqrt 1).
STEP = {
    # step                slots  fp32
    "philox_block":      (100,   0),   # 10 rounds x (2 multiplies x 4 + 2 xor3); key schedule is scalar
    "uniform":           (2,     0),   # u32 -> f64, fma
    "source_slit":       (39,    0),   # A3: points, direction (sqrt, rcp), lambda, k = 2 pi/lambda
    "slab":              (51,    0),   # A4: 3 axes x (rcp 8, 2 fma-pairs, min/max 4), length
    "scatter_point":     (4,     0),   # A5
    "cone_q":            (85,    0),   # A6: t, sqrt, sincospi(psi), Duff basis, k_f, |Q|
    "qvec":              (6,     0),   # Q vector (anisotropic models)
    "size_draw":         (10,    0),   # A7: FP64 table lerp
    "orient_angle":      (31,    0),   # A8 per Gaussian angle: lerp, small-angle sincos, rotation
    "project_c":         (5,     0),   # Q . C
    "project_abc":       (27,    0),   # Q . A, Q . B, Q . C
    "sphere_F":          (13,   21),   # A9: 3 j1(x)/x (series) and volume
    "core_shell_F":      (32,   44),
    "cylinder_F":        (32,   39),   # sinc (series), 2 J1(x)/x (series), Q_AB
    "ellipsoid_F":       (26,   25),
    "py_sq":             (17,   25),   # A10: series in x^2, 1/(1 + 24 phi G/x)
    "weight":            (5,     3),   # A11
    "detector":          (26,    0),   # A12: plane crossing (divide), pixel
    "tally":             (2,     0),   # A13: address; the atomic is a memory op
}
COMMON = ["source_slit", "slab", "scatter_point", "cone_q", "weight", "detector", "tally"]
PATHS = {
    "tiny_sphere": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["sphere_F"],
    "coreshell_py": COMMON + ["philox_block"] * 3 + ["uniform"] * 9
                    + ["size_draw", "core_shell_F", "py_sq"],
    "oriented_cylinder": COMMON + ["philox_block"] * 3 + ["uniform"] * 10
                         + ["qvec"] + ["orient_angle"] * 2 + ["project_c", "cylinder_F"],
    "oriented_ellipsoid": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                          + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "ellipsoid_F"],
}
# Exact-average paths: per quadrature node (76 x 76 = 5776 nodes per neutron)
# parallelepiped: 2 in-plane projections (2), three sinc (series, 7 each),
# product and accumulation (5); spheroid: sin(theta) (sqrt, 6), projections (2),
# argument (3 mul + 2 fma + sqrt = 9), 3 j1(x)/x (series, 9), volume (4),
# accumulation (2).  FP32 flops per node: 2 + 3 x 11 + 5 = 40 and 6 + 2 + 11 +
# 17 + 4 + 3 = 43.
QUAD_NODE = {"quad_parallelepiped": (28, 40), "quad_spheroid": (32, 43)}
QUAD_NODES = 76 * 76
QUAD_BASE = COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["qvec"]


def algo_per_neutron(workload: str):
    """(VALU slots, FP32 flops) per neutron of a workload, or None."""
    if workload in PATHS:
        steps = PATHS[workload]
        return sum(STEP[s][0] for s in steps), sum(STEP[s][1] for s in steps)
    if workload in QUAD_NODE:
        base = sum(STEP[s][0] for s in QUAD_BASE)
        slots, flops = QUAD_NODE[workload]
        return base + QUAD_NODES * slots, STEP["weight"][1] + QUAD_NODES * flops
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="coreshell_py")
    ap.add_argument("--n", type=float, default=None, help="neutrons per step (default: workload's)")
    ap.add_argument("--tally", default="auto", choices=["auto", "global", "lds", "xcd", "binned"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample (0 = skip)")
    return ap.parse_args()


def cpu_baseline(params, seed, target_s):
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    n = 200_000
    t0 = time.perf_counter()
    oracle.trace(params, n, seed, nthreads=threads)
    dt = time.perf_counter() - t0
    rate = n / max(dt, 1e-9)
    n_s = int(max(n, min(rate * target_s, 2e9)))
    t0 = time.perf_counter()
    oracle.trace(params, n_s, seed, nthreads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n_s / dt, unit="neutrons/s", cores=threads, kind="oracle",
                sample=f"first {n_s} neutrons of the same workload and seed "
                       f"(FP64 C oracle, {threads} threads, {dt:.1f} s)")


def bench_copy(a):
    """A plain device copy of 256 MiB per step (torch's copy kernel): the HBM
    reference that the traffic counters (FETCH_SIZE, WRITE_SIZE) are scaled
    by, and a check of the achievable copy bandwidth."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    nbytes = 2 * src.numel() * 8
    return {"metric": "device copy bandwidth", "value": round(nbytes / dt / 1e9, 1), "unit": "GB/s",
            "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(dt * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "copy", "bytes_read": nbytes // 2,
                                            "bytes_written": nbytes // 2}}


def bench_batch(a):
    """The batched high-throughput set: 4096 experiments, one persistent
    graph-captured launch per step; compared with plain per-experiment
    traces of a subset on the same GPU."""
    import torch
    from paper_2501_06054_amd import sans, workloads as W

    exps = W.batch_experiments()
    plist = [x["params"] for x in exps]
    ns = [x["n"] for x in exps]
    seeds = [x["seed"] for x in exps]
    total = float(sum(ns))
    torch.cuda.set_device(0)
    out = torch.empty((len(exps), 128, 128), dtype=torch.float64, device="cuda")
    tune = os.path.join(ROOT, "profiles", "batch_tuning.json")
    sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)   # tunes once (cached file)
    for _ in range(a.warmup):
        sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = total * a.steps / elapsed
    # plain path on the first 256 experiments (model set-up outside the timing)
    sub = range(256)
    models = [sans.Model(exps[e]["params"]) for e in sub]
    dets = [m.detector() for m in models]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in sub:
        models[e].trace(ns[e], seeds[e], det=dets[e], exp_id=e)
    torch.cuda.synchronize()
    plain_rate = sum(ns[e] for e in sub) / (time.perf_counter() - t0)
    for m in models:
        m.close()
    return {
        "metric": "neutrons traced/s at 1 GPU",
        "value": round(value, 1),
        "unit": "neutrons/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 weights, f64 geometry and tallies",
        "data": "synthetic (seeded experiment generator, Philox streams)",
        "config": {"workload": "batch", "experiments": len(exps), "total_neutrons": total,
                   "detector": "128x128 each", "parallelism": "none (1 GPU)"},
        "plain_same_gpu": {"value": round(plain_rate, 1), "unit": "neutrons/s",
                           "sample": "first 256 experiments, one sans_trace_ex each"},
        "batched_over_plain": round(value / plain_rate, 3),
    }


def kernel_source_hash() -> str:
    """Hash of the HIP sources: HBM traffic measured with rocprofv3 counters
    is valid only for the kernels it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2501_06054_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str, n: int):
    """HBM bytes of one trace call from the committed counter summary (sum
    over its dispatches of FETCH_SIZE and WRITE_SIZE, each scaled by the
    copy-kernel calibration, per neutron), or None when the summary was taken
    on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 5 and cells[0] == workload and cells[1] == kernel and cells[2] == src:
            try:
                return float(cells[3]) * n, float(cells[4]) * n
            except ValueError:
                return None
    return None


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(sharding design: neutron ranges per GPU, one reduce of the detector)",
              file=sys.stderr)
        sys.exit(2)

    if a.workload == "batch":
        print(json.dumps(bench_batch(a)), flush=True)
        return
    if a.workload == "copy":
        print(json.dumps(bench_copy(a)), flush=True)
        return

    import torch
    from paper_2501_06054_amd import sans, workloads as W

    wl = W.workload(a.workload)
    p = wl["params"]
    n = int(a.n) if a.n else int(wl["n"])
    seed = wl["seed"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    m = sans.Model(p, tally=a.tally)
    if p["mode"] == "surrogate":
        from paper_2501_06054_amd import surrogate as SG
        model = "parallelepiped" if p["kind"] == "parallelepiped" else "spheroid"
        SG.Surrogate.load(model).attach(m.handle)
    det = m.detector()

    def step(record=None):
        det.zero_()
        if record is not None:
            record[0].record(stream)
        m.trace(n, seed, det=det, accumulate=True)
        if record is not None:
            record[1].record(stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # the trace call's kernels, timed with events on the stream they run on
    kernel_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / a.steps
    total = float(det.sum())
    value = n * a.steps / elapsed
    kernel_rate = n / (kernel_ms * 1e-3)

    algo = algo_per_neutron(a.workload)
    roofline = fp32 = None
    if algo:
        slots, flops = algo
        ach = slots * kernel_rate / 1e12
        traffic = measured_traffic(a.workload, "trace_call", n)
        roofline = dict(bound="alu", achieved=round(ach, 3), peak=round(PEAK_VALU_TSLOTS, 3),
                        unit="Tslot/s (VALU lane-op issue)", frac=round(ach / PEAK_VALU_TSLOTS, 4),
                        traffic=(None if traffic is None else round(traffic[0] + traffic[1])),
                        timed="one sans_trace call: all of its kernels (trace kernel launches and "
                              "tally reduction), HIP events on its stream",
                        call_ms=round(kernel_ms, 4), slots_per_neutron=slots, neutrons_per_call=n)
        fach = flops * kernel_rate / 1e12
        fp32 = dict(achieved=round(fach, 4), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=round(fach / PEAK_FP32_TFLOPS, 5), flops_per_neutron=flops)

    out = {
        "metric": "neutrons traced/s at 1 GPU",
        "value": round(value, 1),
        "unit": "neutrons/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry, f32 weight, f64 tally",
        "data": "synthetic (seeded Philox streams; synthetic instrument)",
        "config": {"workload": a.workload, "neutrons_per_step": n, "seed": seed,
                   "model": p["kind"], "mode": p["mode"], "detector": f"{p['nx']}x{p['ny']}",
                   "tally": a.tally, "parallelism": "none (1 GPU)"},
        "detector_total": total,
        "roofline": roofline,
        "fp32_valu": fp32,
    }
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, seed, a.cpu_seconds)
    m.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
