"""Benchmark of the SANS sample tracer on one MI355X.

One step = one pass of the whole hot path over one batch: the detector is
cleared and n neutrons are traced (Philox draws, source/slit/slab geometry,
cone sampling, Schulz size draw from the LDS table, core-shell amplitude,
Percus-Yevick S(Q), weight, detector pixel, FP64 tally).  The default workload
is the polydisperse core-shell sphere with hard-sphere S(Q) on a 256x256
detector, 1e8 neutrons per step.

Prints one JSON line (rank 0, one GPU):
  metric/value/unit       neutrons traced per second (whole job)
  roofline                FP32 VALU fraction of the dominant kernel (k_trace),
                          timed with HIP events on its stream
  valu                    the same kernel against the VALU issue rate, counting
                          every algorithmic lane operation (integer, FP32, FP64)
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
# one wave64 VALU instruction per 4 clocks on each of the 4 SIMDs of a CU:
# 64 lane-operations per clock per CU
PEAK_VALU_TOPS = CUS * CLOCK_GHZ * 1e9 * 64 / 1e12

# Algorithmic operations per traced neutron, per workload (counted from the
# method's steps; the counting rules are stated in the design notes):
#   fp32: FP32 flops of the weight (add/mul = 1, fma = 2, each sin, cos, rcp,
#         sqrt, acos = 1);
#   slots: VALU lane-op issue slots of the whole step (integer, FP64, FP32;
#          full-rate ops 1 slot, quarter-rate ops - 32-bit integer multiplies,
#          FP64/FP32 transcendentals - 4 slots).
ALGO_OPS = {
    "coreshell_py": dict(fp32=80, slots=1180),
    "tiny_sphere": dict(fp32=30, slots=860),
    "oriented_cylinder": dict(fp32=120, slots=1260),
    "oriented_ellipsoid": dict(fp32=125, slots=1270),
    "quad_parallelepiped": dict(fp32=5776 * 21, slots=5776 * 33 + 860),
    "quad_spheroid": dict(fp32=5776 * 17, slots=5776 * 28 + 860),
}


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

    import torch
    from paper_2501_06054_amd import sans, workloads as W

    wl = W.workload(a.workload)
    p = wl["params"]
    n = int(a.n) if a.n else int(wl["n"])
    seed = wl["seed"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    m = sans.Model(p, tally=a.tally)
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
    kernel_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / a.steps
    total = float(det.sum())

    value = n * a.steps / elapsed
    ops = ALGO_OPS.get(a.workload)
    kernel_rate = n / (kernel_ms * 1e-3)
    roofline = valu = None
    if ops:
        ach = ops["fp32"] * kernel_rate / 1e12
        roofline = dict(bound="alu", achieved=round(ach, 4), peak=PEAK_FP32_TFLOPS,
                        unit="TFLOP/s", frac=round(ach / PEAK_FP32_TFLOPS, 5), traffic=None,
                        kernel="k_trace", kernel_ms=round(kernel_ms, 4),
                        fp32_flops_per_neutron=ops["fp32"])
        vach = ops["slots"] * kernel_rate / 1e12
        valu = dict(achieved=round(vach, 3), peak=round(PEAK_VALU_TOPS, 2), unit="Tlane-op/s",
                    frac=round(vach / PEAK_VALU_TOPS, 4), slots_per_neutron=ops["slots"])

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
        "dtype": "f32 weights, f64 geometry and tallies",
        "data": "synthetic (seeded Philox streams; synthetic instrument)",
        "config": {"workload": a.workload, "neutrons_per_step": n, "seed": seed,
                   "model": p["kind"], "mode": p["mode"], "detector": f"{p['nx']}x{p['ny']}",
                   "tally": a.tally, "parallelism": "none (1 GPU)"},
        "detector_total": total,
        "roofline": roofline,
        "valu": valu,
    }
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, seed, a.cpu_seconds)
    m.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
