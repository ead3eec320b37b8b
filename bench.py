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
# The VALU ceiling in FP32-FMA lane slots: 157.3 TFLOP/s = 256 CUs x 2.4 GHz
# x 128 FMA lanes per clock (two wave64 FP32 FMAs per clock per CU).
PEAK_VALU_TSLOTS = PEAK_FP32_TFLOPS / 2.0

# Issue cost of each operation class in FP32-FMA slots, from the rates
# measured on MI355X by sans_debug_valu_rates (bench.py --workload
# valu_rates; wave64 instructions per clock per CU: FP32 FMA 1.49, 32-bit
# integer 1.54, 32x32->64 multiply with an xor 0.86, FP64 FMA 0.79, FP32
# reciprocal 0.45, FP64 reciprocal 0.24).  A GPU test keeps the measured
# costs within 30 % of these.
SLOT_COST = {"fp32": 1.0, "int32": 1.0, "mul64": 2.5, "fp64": 1.9, "trans32": 3.3, "trans64": 6.3}

# Algorithmic work per neutron, counted from the method's steps (tabulated in
# the design notes): operations per lane by class -- fp32 and fp64 add, mul,
# fma, min/max, compare or conversion; int32 add, xor, logic or select;
# mul64 a 32x32->64 multiply; trans32 an FP32 reciprocal/sqrt/exp/log; trans64
# the FP64 reciprocal or rsq estimate (the Newton steps that refine it are
# fp64 ops).  Where a function has a short series below a threshold, the
# cheaper (series) form is counted, so the totals are lower bounds.  The last
# column is the FP32 flops of the weight (fma 2).
#           step               fp32 int32 mul64 fp64 trans32 trans64 | fp32 flops
STEP = {
    "philox_block":  ((0,  40, 20,  0, 0, 0), 0),   # 10 rounds: 2 multiplies, 4 xor
    "uniform":       ((0,   0,  0,  2, 0, 0), 0),   # u32 -> f64, fma
    "source_slit":   ((0,   0,  0, 30, 0, 3), 0),   # A3: points, |d| (sqrt), 1/|d|, lambda, 2 pi/lambda
    "slab":          ((0,   2,  0, 38, 0, 3), 0),   # A4: 3 axes x (1/k_c, 2 planes, min/max), chord
    "scatter_point": ((0,   0,  0,  4, 0, 0), 0),   # A5
    "cone_q":        ((0,   8,  0, 69, 0, 3), 0),   # A6: t, sqrt, sincospi(psi), Duff basis, k_f, |Q|
    "qvec":          ((0,   0,  0,  6, 0, 0), 0),   # Q vector (anisotropic models)
    "size_draw":     ((0,   2,  0, 10, 0, 0), 0),   # A7: FP64 table lerp
    "orient_angle":  ((0,   2,  0, 31, 0, 0), 0),   # A8 per Gaussian angle: lerp, Taylor sincos, rotation
    "project_c":     ((0,   0,  0,  5, 0, 0), 0),   # Q . C
    "project_abc":   ((0,   0,  0, 27, 0, 0), 0),   # Q . A, Q . B, Q . C
    "sphere_F":      ((15,  0,  0,  4, 0, 0), 21),  # A9: phase, 3 j1(x)/x series, volume
    "core_shell_F":  ((29,  0,  0, 10, 0, 0), 44),
    "cylinder_F":    ((24,  0,  0, 13, 0, 1), 39),  # Q_AB (sqrt), sinc and 2 J1(x)/x series
    "ellipsoid_F":   ((15,  0,  0, 15, 0, 1), 25),  # |(aQ_A, bQ_B, cQ_C)| (sqrt), series
    "caps_phase":    ((16,  6,  0,  8, 0, 0), 26),  # cap centre phase: FP64 reduction, sincos polynomials
    "cap_node":      ((37,  6,  0,  0, 0, 0), 58),  # per cap node: sincos of B t, angle sum, 2 J1(x)/x series
    "hollow_F":      ((62, 18,  0, 21, 3, 0), 93),  # 3 x (FP64 phase reduction, sincos, sin/x), 3 faces
    "micelle_F":     ((59,  0,  0,  9, 0, 0), 96),  # core 3 j1(x)/x, sinc, two chain series, the sum
    "cs_cyl_F":      ((50,  0,  0, 28, 0, 2), 80),  # two cylinders (core, outer), contrasts
    "cs_ell_F":      ((31,  0,  0, 32, 0, 2), 52),  # two ellipsoids (core, outer), contrasts
    "thick_box_F":   ((68,  0,  0, 15, 0, 0), 122), # box minus cavity: six sinc series
    "iso_orient":    ((0,   4,  0, 70, 0, 1), 0),   # cos theta = 2u - 1, sin theta (sqrt), two sincospi
    "ts_I":          ((6,   0,  0,  2, 1, 0), 8),   # Teubner-Strey: q^2 + c, square + e, reciprocal, scale
    "pcoil_I":       ((2,   0,  0, 35, 0, 2), 0),   # polydisperse coil: FP64 power (log, exp), quotient
    "mfrac_I":       ((40,  0,  0,  1, 4, 0), 60),  # mass fractal: atan, sin, log2, exp2, reciprocal
    "shell_F":       ((32,  0,  0,  8, 0, 0), 44),  # one vesicle shell: two 3 j1(x)/x (FP64 phases), volumes
    "ellcyl_F":      ((24,  0,  0, 15, 0, 1), 39),  # elliptical cylinder: |(a Q_A, b Q_B)| (sqrt), sinc, 2 J1(x)/x
    "paracrystal_Z": ((54,  6,  0, 60, 1, 3), 60),  # 3 x (Q.v_k, FP64 half-phase reduction, sin^2, quotient), e
    "pev_I":         ((196, 0,  0,  4, 64, 0), 256),  # excluded-volume chain: two 32-node rules of t^(s-1) exp(-U t)
                                                      # (a multiply, an exp and an fma per node)
    "py_sq":         ((15,  0,  0,  0, 1, 0), 25),  # A10: series in x^2, 1/(1 + 24 phi G/x)
    "sticky_sq":     ((27,  0,  0,  0, 1, 0), 50),  # adhesive spheres: two series in k^2, A^2 + B^2, reciprocal
    "msf_I":         ((8,   0,  0,  3, 3, 0), 10),  # mass-surface fractal: two log2, one exp2
    "sb_row":        ((16,  3,  0,  0, 0, 0), 22),  # superball, per x node: cos(Q_A R x), the row's sum
    "sb_node":       ((32,  6,  0,  0, 0, 0), 44),  # superball, per (x, y) node: cos(Q_B R y), sin(Q_C R zm)/Q_C R
    "lam_hg_F":      ((24,  0,  0,  4, 0, 1), 30),  # head-tail bilayer: two sinc (FP64 phases), 2 pi/delta, 1/q^2
    "caille_term":   ((18,  3,  0,  6, 1, 0), 24),  # one sheet pair of a Caille stack: FP64 phase reduction, cos, exp
    "neck_node":     ((34,  6,  0,  6, 2, 0), 44),  # necklace rod rule node: two sinc (one FP64 phase), two fma
    "neck_unit":     ((8,   0,  0,  0, 0, 0), 12),  # necklace pair-sum step: power, three fma
    "bhs_node":      ((16,  3,  0,  0, 0, 0), 20),  # binary spheres, one node of a Qhat_ij integral: sincos, two fma
    "bhs_mat":       ((24,  0,  0,  0, 1, 0), 40),  # binary spheres: Qhat^H Qhat, its inverse, v^T S v
    "rasp_F":        ((36,  0,  0, 12, 0, 0), 60),  # raspberry: two sphere amplitudes, sinc(qD), the pair sum
    "belt_F":        ((56,  0,  0, 34, 1, 2), 80),  # belt bicelle: two 2 J1(x)/x, two sinc, roughness exp
    "ads_I":         ((6,   0,  0,  2, 1, 1), 8),   # adsorbed layer: (drho t)^2 exp(-(q sigma)^2) / q^2
    "pr_node":       ((30,  6,  0,  0, 0, 0), 40),  # pringle, one polar node: two sincos, three fma
    "attenuation":   ((1,   4,  0, 44, 0, 3), 1),   # exit distance (3 axes: quotient, min), FP64 exp, damp
    "weight":        ((3,   0,  0,  2, 0, 0), 3),   # A11
    "detector":      ((0,   5,  0, 23, 0, 1), 0),   # A12: plane crossing (quotient), pixel
    "tally":         ((0,   2,  0,  0, 0, 0), 0),   # A13: address; the add itself is a memory op
}
_CLASSES = ("fp32", "int32", "mul64", "fp64", "trans32", "trans64")


def step_slots(ops) -> float:
    return sum(n * SLOT_COST[c] for n, c in zip(ops, _CLASSES))


COMMON = ["source_slit", "slab", "scatter_point", "cone_q", "weight", "detector", "tally"]
PATHS = {
    "tiny_sphere": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["sphere_F"],
    "coreshell_py": COMMON + ["philox_block"] * 3 + ["uniform"] * 9
                    + ["size_draw", "core_shell_F", "py_sq"],
    "attenuated_coreshell": COMMON + ["philox_block"] * 3 + ["uniform"] * 9
                            + ["size_draw", "core_shell_F", "py_sq", "attenuation"],
    "oriented_cylinder": COMMON + ["philox_block"] * 3 + ["uniform"] * 10
                         + ["qvec"] + ["orient_angle"] * 2 + ["project_c", "cylinder_F"],
    "oriented_ellipsoid": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                          + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "ellipsoid_F"],
    # barbell: the cylinder's amplitude plus the caps' 76-node integral
    "oriented_barbell": COMMON + ["philox_block"] * 3 + ["uniform"] * 10
                        + ["qvec"] + ["orient_angle"] * 2 + ["project_c", "cylinder_F", "caps_phase"]
                        + ["cap_node"] * 76,
    "oriented_hollow_prism": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                             + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "hollow_F"],
    "micelle_py": COMMON + ["philox_block"] * 3 + ["uniform"] * 9 + ["size_draw", "micelle_F", "py_sq"],
    "oriented_core_shell_cylinder": COMMON + ["philox_block"] * 3 + ["uniform"] * 10
                                    + ["qvec"] + ["orient_angle"] * 2 + ["project_c", "cs_cyl_F"],
    "iso_core_shell_ellipsoid": COMMON + ["philox_block"] * 3 + ["uniform"] * 12
                                + ["size_draw", "qvec", "iso_orient", "project_abc", "cs_ell_F"],
    "oriented_hollow_prism_thick": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                                   + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "thick_box_F"],
    "teubner_strey": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["ts_I"],
    "poly_gauss_coil": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["pcoil_I"],
    "mass_fractal": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["mfrac_I"],
    "multilayer_vesicle": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["shell_F"] * 5,
    "polymer_excl_volume": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["pev_I"],
    "oriented_elliptical_cylinder": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                                    + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "ellcyl_F"],
    "oriented_fcc_paracrystal": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                                + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "sphere_F", "paracrystal_Z"],
    "sticky_coreshell": COMMON + ["philox_block"] * 3 + ["uniform"] * 9
                        + ["size_draw", "core_shell_F", "sticky_sq"],
    "mass_surface_fractal": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["msf_I"],
    # superball: the 24 x 24 rule of the workload
    "oriented_superball": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                          + ["qvec"] + ["orient_angle"] * 3 + ["project_abc"] + ["sb_row"] * 24 + ["sb_node"] * 576,
    # lamellae: 30 sheets, 29 pair terms
    "lamellar_caille": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["lam_hg_F"] + ["caille_term"] * 29,
    # pearl necklace: pearl amplitude, 24 rule nodes, 9 pair-sum steps
    "pearl_necklace": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["sphere_F"] + ["neck_node"] * 24
                      + ["neck_unit"] * 9,
    "binary_hard_sphere": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["sphere_F"] * 2 + ["bhs_node"] * 64
                          + ["bhs_mat"],
    "raspberry": COMMON + ["philox_block"] * 3 + ["uniform"] * 9 + ["size_draw", "rasp_F"],
    "oriented_belt_bicelle": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                             + ["qvec"] + ["orient_angle"] * 3 + ["project_abc", "belt_F"],
    "adsorbed_layer": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["ads_I"],
    "oriented_pringle": COMMON + ["philox_block"] * 3 + ["uniform"] * 11
                        + ["qvec", "iso_orient", "project_abc"] + ["pr_node"] * 512,
}
# Exact-average paths, per quadrature node (76 x 76 = 5776 nodes per neutron),
# all FP32:
#   parallelepiped (amplitude = product of one factor per axis; the C factor
#   depends on mu only and is taken once per mu node): 2 arguments, two sinc
#   series (5 each), product, square, weighted sum: 15 ops, 24 flops; per mu
#   node the C sinc and its weight: 12 ops, 20 flops;
#   spheroid (mu x size nodes): q mu, q st, 3 mul, 2 fma, sqrt (trans32), the
#   3 j1(x)/x series (9), square and weighted sum: 18 ops + 1 trans32, 35 flops.
#   capped cylinder (mu x cap nodes): per cap node as in the Monte Carlo path
#   (cap_node); per mu node Q_AB (sqrt), the cylinder's sinc and 2 J1(x)/x
#   series, the FP32-reduced cap-centre phase, F^2 and its weight: 57 ops +
#   6 int + 1 trans32, 83 flops;
#   thin-walled hollow prism (mu x beta nodes; the C axis' sinc and cos per mu
#   node): 2 arguments, 2 x (FP32 reduction, sincos polynomials, sin/x), the
#   three faces, F^2 and its weight: 54 ops + 12 int + 2 trans32, 82 flops;
#   per mu node 25 ops + 6 int + 1 trans32, 37 flops;
#   hollow cylinder (size x mu nodes): Q_AB (sqrt), two 2 J1(x)/x series, the
#   sinc series, the ring, F^2 and its weight: 52 ops + 1 trans32, 79 flops;
#   per size node 4 ops.
QUAD_NODE = {"quad_parallelepiped": ((15, 0, 0, 0, 0, 0), 24), "quad_spheroid": ((18, 0, 0, 0, 1, 0), 35),
             "quad_capped_cylinder": STEP["cap_node"], "quad_hollow_prism": ((54, 12, 0, 0, 2, 0), 82),
             "quad_hollow_cylinder": ((52, 0, 0, 0, 1, 0), 79)}
QUAD_MU = {"quad_parallelepiped": ((12, 0, 0, 0, 0, 0), 20), "quad_spheroid": ((0, 0, 0, 0, 0, 0), 0),
           "quad_capped_cylinder": ((57, 6, 0, 0, 1, 0), 83), "quad_hollow_prism": ((25, 6, 0, 0, 1, 0), 37),
           "quad_hollow_cylinder": ((4, 0, 0, 0, 0, 0), 4)}
QUAD_NODES = 76 * 76
QUAD_BASE = COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["qvec"]


def algo_per_neutron(workload: str):
    """(FP32-FMA slots, FP32 flops) per neutron of a workload, or None."""
    if workload in PATHS:
        steps = PATHS[workload]
        return (round(sum(step_slots(STEP[x][0]) for x in steps), 1), sum(STEP[x][1] for x in steps))
    if workload in QUAD_NODE:
        base = sum(step_slots(STEP[x][0]) for x in QUAD_BASE)
        (nops, nflops), (mops, mflops) = QUAD_NODE[workload], QUAD_MU[workload]
        return (round(base + QUAD_NODES * step_slots(nops) + 76 * step_slots(mops), 1),
                STEP["weight"][1] + QUAD_NODES * nflops + 76 * mflops)
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="coreshell_py")
    ap.add_argument("--n", type=float, default=None, help="neutrons per step (default: workload's)")
    ap.add_argument("--tally", default="auto", choices=["auto", "global", "lds", "xcd", "binned"])
    ap.add_argument("--sweep", action="store_true",
                    help="time one trace call per neutron count 1e5 .. 1e10 instead")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample (0 = skip)")
    return ap.parse_args()


def cpu_baseline(params, seed, target_s):
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    # calibrate the sample size on a probe long enough to hide thread start-up
    n = 200_000
    while True:
        t0 = time.perf_counter()
        oracle.trace(params, n, seed, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.5 or n >= 1 << 27:
            break
        n *= 4
    rate = n / max(dt, 1e-9)
    n_s = int(max(n, min(rate * target_s, 2e9)))
    t0 = time.perf_counter()
    oracle.trace(params, n_s, seed, nthreads=threads)
    dt = time.perf_counter() - t0
    # one thread, the paper's single-core reference scheme (about 3 s of work)
    n1 = int(max(20_000, min(rate / threads * 3.0, 5e8)))
    t0 = time.perf_counter()
    oracle.trace(params, n1, seed, nthreads=1)
    dt1 = time.perf_counter() - t0
    return dict(value=n_s / dt, unit="neutrons/s", cores=threads, kind="oracle",
                sample=f"first {n_s} neutrons of the same workload and seed "
                       f"(FP64 C oracle, {threads} threads, {dt:.1f} s)",
                single_thread=dict(value=n1 / dt1, sample=f"first {n1} neutrons, 1 thread, {dt1:.1f} s"))


def bench_valu_rates(a):
    """Issue rates of the VALU operation classes the slot costs rest on."""
    import torch
    from paper_2501_06054_amd import sans
    torch.cuda.set_device(0)
    rates = sans.sans_debug_valu_rates()
    return {"metric": "VALU issue rate", "unit": "wave64 instructions per clock per CU",
            "rates": {k: round(v, 3) for k, v in rates.items()},
            "slot_cost_vs_fp32_fma": {k: round(rates["fp32 fma"] / v, 2) for k, v in rates.items()},
            "note": "the mul 32x32->64 class is a multiply plus an xor (two instructions)"}


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
    # the autotuner's cache (one entry per batch shape) lives outside the tree
    import tempfile
    tune = os.path.join(tempfile.gettempdir(), "sans_batch_tuning.json")
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


def sweep(m, p, seed, workload):
    """Wall time of one trace call (detector cleared, events on the stream)
    for N = 1e5 .. 1e10: the shape of the paper's time-versus-N curves."""
    import torch
    det = m.detector()
    rows = []
    for e in range(5, 11):
        n = 10 ** e
        m.trace(min(n, 10 ** 7), seed, det=det)          # warm
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        m.trace(n, seed, det=det)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rows.append({"n": n, "wall_ms": round(wall * 1e3, 4), "gpu_ms": round(e0.elapsed_time(e1), 4),
                     "neutrons_per_s": round(n / wall, 1)})
    return {"metric": "trace time versus neutron count", "workload": workload,
            "detector": f"{p['nx']}x{p['ny']}", "rows": rows}


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
    if a.workload == "valu_rates":
        print(json.dumps(bench_valu_rates(a)), flush=True)
        return

    import torch
    from paper_2501_06054_amd import sans, workloads as W

    wl = W.workload(a.workload)
    p = wl["params"]
    n = int(a.n) if a.n else int(wl["n"])
    seed = wl["seed"]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    m = sans.Model(p, tally=a.tally)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    if a.sweep:
        print(json.dumps(sweep(m, p, seed, a.workload)), flush=True)
        m.close()
        return
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
                        unit="T FP32-FMA lane slots/s (VALU issue, 157.3 TFLOP/s / 2)",
                        frac=round(ach / PEAK_VALU_TSLOTS, 4),
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
        "setup_ms": round(setup_ms, 3),
        "roofline": roofline,
        "fp32_valu": fp32,
    }
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, seed, a.cpu_seconds)
    m.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
