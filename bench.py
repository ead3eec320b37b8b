"""Benchmark of the SANS sample tracer on one MI355X.

One step = one pass of the whole hot path over one batch: the detector is
cleared and n neutrons are traced (Philox draws, source/slit/slab geometry,
cone sampling, Schulz size draw from the LDS table, core-shell amplitude,
Percus-Yevick S(Q), weight, detector pixel, FP64 tally).  The default workload
is the polydisperse core-shell sphere with hard-sphere S(Q) on a 256x256
detector, 1e8 neutrons per step.

Prints one JSON line (rank 0, one GPU):
  metric/value/unit       neutrons traced per second (whole job)
  roofline                the trace call against the FP32 vector peak:
                          algorithmic FP32 flops per neutron x neutrons per
                          call / the call's time from HIP events on its stream
  valu                    counter-measured VALU work of the trace kernel
                          (instructions and FP32 flops per neutron, VALU busy,
                          clock), when measured on the current kernel sources
  cpu_baseline            the FP64 CPU oracle on a bounded sample of the same
                          workload, built for and run on this host's cores
  other_configs           the other configurations timed on the same GPU: the
                          oriented cylinder and ellipsoid at 1e9 neutrons, the
                          4096-experiment batch against plain traces, and the
                          surrogate against the exact-average trace
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

# Algorithmic FP32 flops per neutron (FMA = 2) of the four reference
# configurations: the per-neutron budget of the method's FP32 steps (A9-A11)
# with the amplitudes in their closed forms -- tiny sphere: 3 j1(x)/x and the
# weight; core-shell: two sphere amplitudes, the Percus-Yevick S(Q) and the
# weight; oriented cylinder and triaxial ellipsoid: the projected amplitude
# (sinc and 2 J1(x)/x, or 3 j1(x)/x of the scaled radius) and the weight.
# Other workloads use the step counts below.
REFERENCE_FLOPS = {"tiny_sphere": 35, "coreshell_py": 110, "oriented_cylinder": 80,
                   "oriented_ellipsoid": 80}

# FP32 flops of each step of the per-neutron work (FMA = 2), counted from the
# method's steps with the cheaper series forms where a function has one below
# a threshold (so these are lower bounds).  The geometry (A3-A6, A12) is FP64
# and contributes none.
STEP = {
    "philox_block": 0, "uniform": 0, "source_slit": 0, "slab": 0, "scatter_point": 0, "cone_q": 0,
    "qvec": 0, "size_draw": 0, "orient_angle": 0, "project_c": 0, "project_abc": 0,
    "sphere_F": 21,      # phase, 3 j1(x)/x series, volume
    "core_shell_F": 44,
    "cylinder_F": 39,    # Q_AB (sqrt), sinc and 2 J1(x)/x series
    "ellipsoid_F": 25,   # |(aQ_A, bQ_B, cQ_C)| (sqrt), series
    "caps_phase": 26,    # cap centre phase: FP64 reduction, sincos polynomials
    "cap_node": 58,      # per cap node: sincos of B t, angle sum, 2 J1(x)/x series
    "hollow_F": 93,      # 3 x (FP64 phase reduction, sincos, sin/x), 3 faces
    "micelle_F": 96,     # core 3 j1(x)/x, sinc, two chain series, the sum
    "cs_cyl_F": 80, "cs_ell_F": 52, "thick_box_F": 122,
    "box_F": 33,         # parallelepiped: three sinc series, their product, volume
    "iso_orient": 0,
    "ts_I": 8, "pcoil_I": 0, "mfrac_I": 60, "shell_F": 44, "ellcyl_F": 39,
    "paracrystal_Z": 60,
    "pev_I": 256,        # excluded-volume chain: two 32-node rules
    "py_sq": 25,         # A10: series in x^2, 1/(1 + 24 phi G/x)
    "sticky_sq": 50, "msf_I": 10, "sb_row": 22, "sb_node": 44, "lam_hg_F": 30, "caille_term": 24,
    "neck_node": 44, "neck_unit": 12, "bhs_node": 20, "bhs_mat": 40, "rasp_F": 60, "belt_F": 80,
    "ads_I": 8, "pr_node": 40, "attenuation": 1,
    "fc_chain_node": 28,  # flexible cylinder, one node of the chain rule: exp, expm1, the two sums
    "cyl_section": 20,    # [2 J1(qR)/(qR)]^2, series or asymptotic form
    "msa_sq": 12,        # Hayter-Penfold S: knot index, cubic Hermite between two knots
    "fc_node": 40,       # flexible cylinder, one node of the chain and section rules: exp, expm1, a sine,
                         # the two chain sums; the section's radius (sqrt) and 2 J1(x)/x series
    "weight": 3,         # A11
    "detector": 0, "tally": 0,
}
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
    # independent size draws: a fourth Philox block, one table lerp per size
    "poly_sep_cylinder": COMMON + ["philox_block"] * 4 + ["uniform"] * 12
                         + ["size_draw"] * 2 + ["qvec"] + ["orient_angle"] * 2 + ["project_c", "cylinder_F"],
    "poly_sep_parallelepiped": COMMON + ["philox_block"] * 4 + ["uniform"] * 14
                               + ["size_draw"] * 3 + ["qvec", "iso_orient", "project_abc", "box_F"],
    # flexible elliptical cylinder: 48-point chain and section rules
    "flexible_cylinder_elliptical": COMMON + ["philox_block"] * 2 + ["uniform"] * 8 + ["fc_node"] * 48,
    "flexible_cylinder": COMMON + ["philox_block"] * 3 + ["uniform"] * 9 + ["size_draw"]
                         + ["fc_chain_node"] * 48 + ["cyl_section"],
    "charged_spheres": COMMON + ["philox_block"] * 3 + ["uniform"] * 9 + ["size_draw", "sphere_F", "msa_sq"],
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
QUAD_NODE = {"quad_parallelepiped": 24, "quad_spheroid": 35, "quad_capped_cylinder": STEP["cap_node"],
             "quad_hollow_prism": 82, "quad_hollow_cylinder": 79}
QUAD_MU = {"quad_parallelepiped": 20, "quad_spheroid": 0, "quad_capped_cylinder": 83,
           "quad_hollow_prism": 37, "quad_hollow_cylinder": 4}
QUAD_NODES = 76 * 76


def own_flops(workload: str):
    """FP32 flops per neutron of a workload from the step counts, or None."""
    if workload in PATHS:
        return sum(STEP[x] for x in PATHS[workload])
    if workload in QUAD_NODE:
        return STEP["weight"] + QUAD_NODES * QUAD_NODE[workload] + 76 * QUAD_MU[workload]
    return None


def algo_flops(workload: str):
    """(FP32 flops per neutron, where the figure comes from) or None."""
    if workload in REFERENCE_FLOPS:
        return REFERENCE_FLOPS[workload], "per-neutron budget of the reference configurations"
    f = own_flops(workload)
    return None if f is None else (f, "step counts (series forms; lower bound)")


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
    ap.add_argument("--others", type=int, default=1,
                    help="1: also time the other configurations (default workload only)")
    return ap.parse_args()


def host_threads() -> int:
    """Threads the CPU baseline uses: the cores this process may run on,
    capped by OMP_NUM_THREADS where the host sets it (the GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(params, seed, target_s):
    """The FP64 oracle, compiled here for this host (-O3 -march=native), on
    the first neutrons of the same workload: all allowed threads (about
    target_s of work) and one thread (the paper's single-core scheme)."""
    import tempfile
    import oracle
    threads = host_threads()
    with tempfile.TemporaryDirectory() as tmp:
        so = oracle.build_native(tmp)
        # calibrate the sample size on a probe long enough to hide thread start-up
        n = 200_000
        while True:
            t0 = time.perf_counter()
            oracle.trace_native(so, params, n, seed, nthreads=threads)
            dt = time.perf_counter() - t0
            if dt >= 0.5 or n >= 1 << 27:
                break
            n *= 4
        rate = n / max(dt, 1e-9)
        n_s = int(max(n, min(rate * target_s, 2e9)))
        t0 = time.perf_counter()
        oracle.trace_native(so, params, n_s, seed, nthreads=threads)
        dt = time.perf_counter() - t0
        n1 = int(max(20_000, min(rate / threads * 3.0, 5e8)))
        t0 = time.perf_counter()
        oracle.trace_native(so, params, n1, seed, nthreads=1)
        dt1 = time.perf_counter() - t0
    return dict(value=n_s / dt, unit="neutrons/s", cores=threads, kind="oracle",
                sample=f"first {n_s} neutrons of the same workload and seed "
                       f"(FP64 C oracle, gcc -O3 -march=native, {threads} threads, {dt:.1f} s)",
                cpu=cpu_model(),
                single_thread=dict(value=n1 / dt1, sample=f"first {n1} neutrons, 1 thread, {dt1:.1f} s"))


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


def batch_rates(steps: int, warmup: int):
    """The 4096-experiment set in one persistent graph-captured launch per
    step, against plain per-experiment traces of its first 256 experiments on
    the same GPU."""
    import tempfile
    import torch
    from paper_2501_06054_amd import sans, workloads as W

    exps = W.batch_experiments()
    # the experiments' parameter array, built once (as a caller tracing the
    # same set repeatedly holds it), so that the timed calls do not convert
    # 4096 dicts each
    plist = sans.batch_params([x["params"] for x in exps])
    ns = [x["n"] for x in exps]
    seeds = [x["seed"] for x in exps]
    total = float(sum(ns))
    torch.cuda.set_device(0)
    out = torch.empty((len(exps), 128, 128), dtype=torch.float64, device="cuda")
    # the autotuner's cache (one entry per batch shape) lives outside the tree
    tune = os.path.join(tempfile.gettempdir(), "sans_batch_tuning.json")
    t0 = time.perf_counter()
    sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)   # tunes once (cached file)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    for _ in range(warmup):
        sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sans.sans_trace_batch(plist, ns, seeds, out, tune_cache=tune)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = total * steps / elapsed
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
    return dict(experiments=len(exps), total_neutrons=total, ms_per_call=round(elapsed / steps * 1e3, 3),
                value=round(value, 1), unit="neutrons/s", first_call_s=round(first_s, 3),
                plain_same_gpu=dict(value=round(plain_rate, 1), unit="neutrons/s",
                                    sample="first 256 experiments, one sans_trace_ex each"),
                batched_over_plain=round(value / plain_rate, 3))


def bench_batch(a):
    """The batched set as the bench line (--workload batch)."""
    r = batch_rates(a.steps, a.warmup)
    return {
        "metric": "neutrons traced/s at 1 GPU",
        "value": r["value"],
        "unit": "neutrons/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 weights, f64 geometry and tallies",
        "data": "synthetic (seeded experiment generator, Philox streams)",
        "config": {"workload": "batch", "experiments": r["experiments"], "total_neutrons": r["total_neutrons"],
                   "detector": "128x128 each", "parallelism": "none (1 GPU)"},
        "plain_same_gpu": r["plain_same_gpu"],
        "batched_over_plain": r["batched_over_plain"],
    }


def sweep(m, p, seed, workload):
    """Wall time of one trace call (detector cleared, events on the stream)
    for N = 1e5 .. 1e10: the shape of the paper's time-versus-N curves."""
    import torch
    det = m.detector()
    rows = []
    for e in range(5, 11):
        n = 10 ** e
        m.trace(min(n, 10 ** 9), seed, det=det)          # warm: workspaces sized for this n
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


def roofline_of(workload: str, n: int, call_ms: float):
    """The trace call against the FP32 vector peak (the call's kernels timed
    together with HIP events on their stream)."""
    algo = algo_flops(workload)
    if algo is None:
        return None
    flops, source = algo
    ach = flops * n / (call_ms * 1e-3) / 1e12
    traffic = measured_traffic(workload, "trace_call", n)
    return dict(bound="alu", achieved=round(ach, 4), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(ach / PEAK_FP32_TFLOPS, 5),
                traffic=(None if traffic is None else round(traffic[0] + traffic[1])),
                flops_per_neutron=flops, flops_source=source, own_count=own_flops(workload),
                timed="one sans_trace call: all of its kernels (trace launches and tally "
                      "reduction), HIP events on its stream",
                call_ms=round(call_ms, 4), neutrons_per_call=n)


def measured_valu(workload: str):
    """Counter-measured VALU work of the workload's trace kernel from the
    committed summary (profiles/valu_counters.md), or None when it was taken
    on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "valu_counters.md")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    keys = ("kernel", "valu_instr_per_neutron", "fp32_flops_per_neutron", "fp64_instr_per_neutron",
            "valu_busy", "clock_mhz")
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 8 and cells[0] == workload and cells[2] == src:
            try:
                vals = [cells[1]] + [float(c) for c in cells[3:]]
            except ValueError:
                return None
            return dict(zip(keys, vals), source="rocprofv3 counters, profiles/valu_counters.md")
    return None


def time_calls(m, n, seed, steps, warm_n=None):
    """Mean time (ms) of `steps` trace calls of n neutrons on a warm model,
    HIP events on the stream its kernels run on; the detector."""
    import torch
    stream = torch.cuda.current_stream()
    det = m.detector()
    m.trace(warm_n or n, seed, det=det)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        m.trace(n, seed, det=det)
        e1.record(stream)
    torch.cuda.synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) / steps, det


def other_configs():
    """The other configurations on the same GPU: oriented cylinder and
    ellipsoid (1e9 neutrons each), the 4096-experiment batch against plain
    per-experiment traces, and each surrogate against the exact-average trace
    of the same workload."""
    import torch
    from paper_2501_06054_amd import sans, surrogate as SG, workloads as W
    out = {}
    for name in ("oriented_cylinder", "oriented_ellipsoid"):
        wl = W.workload(name)
        m = sans.Model(wl["params"])
        ms, _ = time_calls(m, int(wl["n"]), wl["seed"], 3)
        m.close()
        n = int(wl["n"])
        out[name] = dict(neutrons_per_call=n, ms_per_call=round(ms, 3), value=round(n / (ms * 1e-3), 1),
                         unit="neutrons/s", roofline=roofline_of(name, n, ms))
    b = batch_rates(steps=4, warmup=1)
    out["batch"] = b
    for model in ("parallelepiped", "spheroid"):
        sw, qw = W.workload(f"surrogate_{model}"), W.workload(f"quad_{model}")
        ms_ = sans.Model(sw["params"])
        SG.Surrogate.load(model).attach(ms_.handle)
        n_s = 10 ** 9
        t_s, _ = time_calls(ms_, n_s, sw["seed"], 1, warm_n=10 ** 8)
        ms_.close()
        mq = sans.Model(qw["params"])
        n_q = 10 ** 8
        t_q, _ = time_calls(mq, n_q, qw["seed"], 1, warm_n=10 ** 7)
        mq.close()
        r_s, r_q = n_s / (t_s * 1e-3), n_q / (t_q * 1e-3)
        out[f"surrogate_{model}"] = dict(neutrons_per_call=n_s, ms_per_call=round(t_s, 3), value=round(r_s, 1),
                                         unit="neutrons/s",
                                         exact_average=dict(workload=f"quad_{model}", neutrons_per_call=n_q,
                                                            value=round(r_q, 1),
                                                            roofline=roofline_of(f"quad_{model}", n_q, t_q)),
                                         surrogate_over_exact=round(r_s / r_q, 3))
    torch.cuda.synchronize()
    return out


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

    roofline = roofline_of(a.workload, n, kernel_ms)
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
        "valu": measured_valu(a.workload),
    }
    m.close()
    if a.others and a.workload == "coreshell_py" and not a.n:
        out["other_configs"] = other_configs()
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(p, seed, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
