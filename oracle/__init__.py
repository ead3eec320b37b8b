"""Python access to the FP64 CPU oracle (``sans_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product package never imports it.

``build()`` compiles ``liboracle.so`` with gcc (plain C99 + pthreads,
``-O2 -ffp-contract=off``); ``lib()`` loads it, building it when missing.
``build_native()`` compiles a copy for the host it runs on (``-O3
-march=native``), which the benchmark's CPU baseline times.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sans_oracle.c")
SO = os.path.join(HERE, "liboracle.so")

KIND = {"sphere": 0, "core_shell": 1, "cylinder": 2, "ellipsoid": 3, "parallelepiped": 4,
        "barbell": 5, "capped_cylinder": 6, "hollow_prism": 7,
        "micelle": 8, "hollow_cylinder": 9, "core_shell_cylinder": 10, "core_shell_ellipsoid": 11,
        "hollow_prism_thick": 12, "guinier": 13, "ornstein_zernike": 14, "dab": 15, "gauss_coil": 16,
        "poly_gauss_coil": 17, "teubner_strey": 18, "power_law": 19, "gaussian_peak": 20,
        "lorentz_peak": 21, "mass_fractal": 22, "star_polymer": 23, "gauss_lorentz_gel": 24,
        "fuzzy_sphere": 25, "vesicle": 26, "multilayer_vesicle": 27, "linear_pearls": 28,
        "surface_fractal": 29, "two_power_law": 30, "guinier_porod": 31, "spinodal": 32, "porod": 33,
        "line": 34, "two_lorentzian": 35, "correlation_length": 36, "broad_peak": 37, "fractal": 38,
        "fractal_core_shell": 39, "polymer_excl_volume": 40, "elliptical_cylinder": 41,
        "core_shell_bicelle": 42, "core_shell_parallelepiped": 43, "core_shell_bicelle_elliptical": 44,
        "stacked_disks": 45, "sc_paracrystal": 46, "bcc_paracrystal": 47, "fcc_paracrystal": 48,
        "mass_surface_fractal": 49, "gel_fit": 50, "superball": 51,
        "lamellar_hg": 52, "lamellar_stack_caille": 53, "lamellar_hg_stack_caille": 54,
        "lamellar_stack_paracrystal": 55, "core_shell_bicelle_elliptical_belt_rough": 56,
        "raspberry": 57, "pearl_necklace": 58, "binary_hard_sphere": 59, "adsorbed_layer": 60,
        "pringle": 61,
        "flexible_cylinder_elliptical": 62, "flexible_cylinder": 63}
SQ_KIND = {"hard_sphere": 0, "sticky_hard_sphere": 1, "square_well": 2, "hayter_msa": 3}
ORIENT = {"fixed": 0, "gaussian": 1, "isotropic": 2, "uniform_angles": 3}
MODE = {"mc": 0, "quad": 1, "surrogate": 2}
POLY_KIND = {"schulz": 0, "gaussian": 1}


class OrcParams(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("mode", C.c_int32),
        ("size", C.c_double * 3), ("shell", C.c_double), ("sld", C.c_double * 3),
        ("phi", C.c_double), ("sq_phi", C.c_double), ("sq_radius", C.c_double),
        ("poly", C.c_double), ("poly_mask", C.c_int32), ("orient_kind", C.c_int32),
        ("orient_mean", C.c_double * 3), ("orient_sigma", C.c_double * 3),
        ("src_w", C.c_double), ("src_h", C.c_double), ("src_z", C.c_double),
        ("slit_w", C.c_double), ("slit_h", C.c_double), ("slit_z", C.c_double),
        ("lambda0", C.c_double), ("dlambda_rel", C.c_double), ("cone_alpha", C.c_double),
        ("sample_w", C.c_double), ("sample_h", C.c_double), ("sample_d", C.c_double),
        ("det_w", C.c_double), ("det_h", C.c_double), ("det_z", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("table_size", C.c_int32), ("quad_n", C.c_int32),
        ("poly_kind", C.c_int32), ("sq_kind", C.c_int32),
        ("extra", C.c_double * 4), ("sq_extra", C.c_double * 2), ("mu_att", C.c_double),
        ("poly_sep", C.c_double * 3), ("guide", C.c_double * 9),
    ]


def _compile(out: str, opt) -> None:
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *opt, "-std=c99", "-D_GNU_SOURCE", "-ffp-contract=off",
                           "-fPIC", "-shared", "-o", tmp, SRC, "-lm", "-lpthread"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        _compile(SO, ["-O2"])
    return SO


def build_native(out_dir: str) -> str:
    """A copy of the oracle compiled for the CPU it runs on (-O3
    -march=native, still without FMA contraction), for timing it on that
    host; built on the spot, never shipped to another machine."""
    so = os.path.join(out_dir, "liboracle_native.so")
    _compile(so, ["-O3", "-march=native"])
    return so


_NATIVE = {}


def trace_native(so_path: str, p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0,
                 nthreads: int = 1) -> np.ndarray:
    """trace() through the library at so_path (a build_native() copy)."""
    L = _NATIVE.get(so_path)
    if L is None:
        L = C.CDLL(so_path)
        P = C.POINTER
        L.orc_trace.argtypes = [P(OrcParams), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int32,
                                P(C.c_double), P(C.c_double), P(C.c_uint64)]
        L.orc_trace.restype = C.c_int32
        L.orc_set_msa.argtypes = [P(C.c_double), C.c_double, C.c_double, C.c_double]
        _NATIVE[so_path] = L
    if p.get("sq_kind") == "hayter_msa" and p.get("sq_phi", 0.0) > 0.0:
        from oracle import msa
        c = np.ascontiguousarray(msa.inside_c(float(p["sq_phi"]), float(p["sq_extra"][0]), float(p["sq_extra"][1])))
        L.orc_set_msa(_ptr(c, C.c_double), float(p["sq_phi"]), float(p["sq_extra"][0]), float(p["sq_extra"][1]))
    o = to_params(p)
    det = np.zeros((p["ny"], p["nx"]))
    rc = L.orc_trace(C.byref(o), first, n, seed, exp_id, nthreads, _ptr(det, C.c_double), None, None)
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc})")
    return det


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(SO)
        d, u32, u64, i32 = C.c_double, C.c_uint32, C.c_uint64, C.c_int32
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.orc_philox_stream.argtypes = [u64, u64, u64, u32, u32, P(u32)]
        L.orc_uniform.argtypes = [u32]
        L.orc_uniform.restype = d
        for f in ("orc_normal_quantile",):
            getattr(L, f).argtypes = [d]
            getattr(L, f).restype = d
        for f in ("orc_schulz_quantile", "orc_truncnorm_quantile", "orc_gamma_p", "orc_py_g_over_x_direct",
                  "orc_gamma_q", "orc_schulz_quantile_upper"):
            getattr(L, f).argtypes = [d, d]
            getattr(L, f).restype = d
        for f in ("orc_sph", "orc_lambda1", "orc_sinc"):
            getattr(L, f).argtypes = [d]
            getattr(L, f).restype = d
        L.orc_py_sq.argtypes = [d, d, d]
        L.orc_py_sq.restype = d
        L.orc_flexcyl_chain.argtypes = [d, d, d, i32]
        L.orc_flexcyl_chain.restype = d
        L.orc_flexcyl_section.argtypes = [d, d, d, i32]
        L.orc_flexcyl_section.restype = d
        L.orc_set_msa.argtypes = [P(d), d, d, d]
        L.orc_msa_sq.argtypes = [d, d, d, d, d]
        L.orc_msa_sq.restype = d
        L.orc_sticky_lambda.argtypes = [d, d]
        L.orc_sticky_lambda.restype = d
        L.orc_sticky_sq.argtypes = [d, d, d, d]
        L.orc_sticky_sq.restype = d
        L.orc_square_well_sq.argtypes = [d, d, d, d, d]
        L.orc_square_well_sq.restype = d
        L.orc_bhs_inverse_s.argtypes = [d, d, d, d, d, P(d), P(d)]
        L.orc_py_series.argtypes = [d, i32, P(d)]
        L.orc_table_normal.argtypes = [i32, P(d)]
        L.orc_table_truncnorm.argtypes = [i32, d, P(d)]
        L.orc_size_moment.argtypes = [P(OrcParams), i32]
        L.orc_size_moment.restype = d
        L.orc_table_schulz.argtypes = [i32, d, P(d)]
        L.orc_table_lookup.argtypes = [P(d), i32, d]
        L.orc_table_lookup.restype = d
        L.orc_table_lookup_u.argtypes = [P(d), i32, d]
        L.orc_table_lookup_u.restype = d
        L.orc_mean_volume.argtypes = [P(OrcParams)]
        L.orc_mean_volume.restype = d
        L.orc_gauss_legendre.argtypes = [i32, P(d), P(d)]
        L.orc_pq_avg.argtypes = [P(OrcParams), d, P(d)]
        L.orc_pq_avg.restype = d
        L.orc_amplitude.argtypes = [P(OrcParams), d, P(d), d, P(d)]
        L.orc_amplitude.restype = d
        L.orc_form_f2.argtypes = [P(OrcParams), d, P(d), d, P(d)]
        L.orc_form_f2.restype = d
        L.orc_trace.argtypes = [P(OrcParams), u64, u64, u64, u32, i32, P(d), P(d), P(u64)]
        L.orc_trace.restype = i32
        L.orc_trace_debug.argtypes = [P(OrcParams), u64, u64, u64, u32, P(i32), P(d), P(d)]
        L.orc_trace_debug.restype = i32
        L.orc_mlp_param_count.restype = C.c_int64
        L.orc_bf16_round.argtypes = [d]
        L.orc_bf16_round.restype = d
        L.orc_mlp_forward.argtypes = [P(d), P(d), i32, P(d), i32, P(d), P(d)]
        L.orc_mlp_backward.argtypes = [P(d), P(d), P(d), i32, P(d), i32, P(d)]
        L.orc_set_surrogate.argtypes = [P(d), P(d), P(d)]
        L.orc_surrogate_judge.argtypes = [P(OrcParams), d, i32, P(d)]
        L.orc_surrogate_judge.restype = i32
        L.orc_trace_debug_ex.argtypes = [P(OrcParams), u64, u64, u64, u32, P(d)]
        L.orc_trace_debug_ex.restype = i32
        L.orc_transmitted_debug.argtypes = [P(OrcParams), u64, u64, u64, u32, P(i32), P(d)]
        L.orc_transmitted_debug.restype = i32
        L.orc_transmitted_add.argtypes = [P(OrcParams), u64, u64, u64, u32, P(d), P(d), P(u64)]
        L.orc_transmitted_add.restype = i32
        L.orc_guide_weight.argtypes = [P(OrcParams), P(d), P(d), d]
        L.orc_guide_weight.restype = d
        _LIB = L
    return _LIB


GUIDE_FIELDS = ("guide_len", "guide_w", "guide_h", "guide_gap", "guide_m", "guide_r0", "guide_qc",
                "guide_alpha", "guide_wc")


def guide_weight(p: dict, src, ki, lam: float) -> float:
    """The guide's weight of a neutron reaching the source aperture at src
    (m) along the unit vector ki with wavelength lam (A)."""
    o = to_params(p)
    a = np.ascontiguousarray(src, dtype=np.float64)
    b = np.ascontiguousarray(ki, dtype=np.float64)
    return lib().orc_guide_weight(C.byref(o), _ptr(a, C.c_double), _ptr(b, C.c_double), float(lam))


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def to_params(p: dict) -> OrcParams:
    """Workload parameter dict -> the oracle's own parameter struct."""
    o = OrcParams()
    o.kind = KIND[p["kind"]]
    o.mode = MODE[p["mode"]]
    for k in range(3):
        o.size[k] = p["size"][k]
        o.sld[k] = p["sld"][k]
        o.orient_mean[k] = p["orient_mean"][k]
        o.orient_sigma[k] = p["orient_sigma"][k]
    for f in ("shell", "phi", "sq_phi", "sq_radius", "poly", "src_w", "src_h", "src_z",
              "slit_w", "slit_h", "slit_z", "lambda0", "dlambda_rel", "cone_alpha",
              "sample_w", "sample_h", "sample_d", "det_w", "det_h", "det_z"):
        setattr(o, f, float(p[f]))
    o.poly_mask = int(p["poly_mask"])
    o.orient_kind = ORIENT[p["orient_kind"]]
    o.nx, o.ny = int(p["nx"]), int(p["ny"])
    o.table_size = int(p["table_size"])
    o.quad_n = int(p["quad_n"])
    o.poly_kind = POLY_KIND[p.get("poly_kind", "schulz")]
    for k, v in enumerate(p.get("extra", (0.0, 0.0, 0.0, 0.0))):
        o.extra[k] = float(v)
    o.sq_kind = SQ_KIND[p.get("sq_kind", "hard_sphere")]
    o.mu_att = float(p.get("mu_att", 0.0))
    for k, v in enumerate(p.get("sq_extra", (0.0, 0.0))):
        o.sq_extra[k] = float(v)
    for k, v in enumerate(p.get("poly_sep", (0.0, 0.0, 0.0))):
        o.poly_sep[k] = float(v)
    for k, f in enumerate(GUIDE_FIELDS):
        o.guide[k] = float(p.get(f, 0.0))
    return o


# ---------------------------------------------------------------- wrappers

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def philox_stream(seed: int, first: int, n: int, nblocks: int, exp_id: int = 0) -> np.ndarray:
    out = np.zeros((n, nblocks, 4), dtype=np.uint32)
    lib().orc_philox_stream(seed, first, n, nblocks, exp_id, _ptr(out, C.c_uint32))
    return out


def uniform(x: int) -> float:
    return lib().orc_uniform(x)


def normal_quantile(u: float) -> float:
    return lib().orc_normal_quantile(u)


def schulz_quantile(u: float, p: float) -> float:
    return lib().orc_schulz_quantile(u, p)


def truncnorm_quantile(u: float, p: float) -> float:
    """Quantile of N(1, p^2) restricted to positive values."""
    return lib().orc_truncnorm_quantile(u, p)


def table_truncnorm(M: int, p: float) -> np.ndarray:
    out = np.zeros(M)
    lib().orc_table_truncnorm(M, p, _ptr(out, C.c_double))
    return out


def size_moment(p: dict, k: int) -> float:
    """<y^k> of the parameter set's size distribution."""
    o = to_params(p)
    return lib().orc_size_moment(C.byref(o), k)


def gamma_p(a: float, x: float) -> float:
    return lib().orc_gamma_p(a, x)


def gamma_q(a: float, x: float) -> float:
    return lib().orc_gamma_q(a, x)


def schulz_quantile_upper(v: float, p: float) -> float:
    """The Schulz size whose upper tail holds probability v."""
    return lib().orc_schulz_quantile_upper(v, p)


def table_dt(M: int) -> float:
    """Knot spacing in t = -ln(2 min(u, 1 - u)) of an M-knot table."""
    return 32.0 * np.log(2.0) / (M // 2 - 1)


def table_normal(M: int) -> np.ndarray:
    out = np.zeros(M)
    lib().orc_table_normal(M, _ptr(out, C.c_double))
    return out


def table_schulz(M: int, p: float) -> np.ndarray:
    out = np.zeros(M)
    lib().orc_table_schulz(M, p, _ptr(out, C.c_double))
    return out


def table_lookup_u(knots: np.ndarray, u: float) -> float:
    """Lookup in the orientation's normal table (knots at (k + 1/2)/M)."""
    k = np.ascontiguousarray(knots, dtype=np.float64)
    return lib().orc_table_lookup_u(_ptr(k, C.c_double), len(k), u)


def table_lookup(knots: np.ndarray, u: float) -> float:
    k = np.ascontiguousarray(knots, dtype=np.float64)
    return lib().orc_table_lookup(_ptr(k, C.c_double), len(k), u)


def sph(x: float) -> float:
    return lib().orc_sph(x)


def lambda1(x: float) -> float:
    return lib().orc_lambda1(x)


def sinc(x: float) -> float:
    return lib().orc_sinc(x)


def py_sq(q: float, radius: float, phi: float) -> float:
    return lib().orc_py_sq(q, radius, phi)


def sticky_lambda(eta: float, tau: float) -> float:
    """Baxter's lambda of adhesive hard spheres (NaN inside the two-phase region)."""
    return lib().orc_sticky_lambda(eta, tau)


def sticky_sq(q: float, radius: float, eta: float, tau: float) -> float:
    return lib().orc_sticky_sq(q, radius, eta, tau)


def square_well_sq(q: float, radius: float, eta: float, depth: float, width: float) -> float:
    return lib().orc_square_well_sq(q, radius, eta, depth, width)


def bhs_inverse_s(r1: float, r2: float, phi1: float, phi2: float, q: float):
    """I - C(q) of a binary hard-sphere mixture (Percus-Yevick) as a complex 2x2 matrix."""
    re = np.zeros(4)
    im = np.zeros(4)
    lib().orc_bhs_inverse_s(r1, r2, phi1, phi2, q, _ptr(re, C.c_double), _ptr(im, C.c_double))
    return (re + 1j * im).reshape(2, 2)


def py_series(phi: float, nterms: int) -> np.ndarray:
    out = np.zeros(nterms)
    lib().orc_py_series(phi, nterms, _ptr(out, C.c_double))
    return out


def py_g_over_x_direct(x: float, phi: float) -> float:
    return lib().orc_py_g_over_x_direct(x, phi)


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _ptr(x, C.c_double), _ptr(w, C.c_double))
    return x, w


def mean_volume(p: dict) -> float:
    o = to_params(p)
    return lib().orc_mean_volume(C.byref(o))


def pq_avg(p: dict, q: float, qvec=(0.0, 0.0, 0.0)) -> float:
    o = to_params(p)
    qv = np.asarray(qvec, dtype=np.float64).copy()
    return lib().orc_pq_avg(C.byref(o), q, _ptr(qv, C.c_double))


def amplitude(p: dict, q: float, qvec, y: float = 1.0, angles=None) -> float:
    o = to_params(p)
    qv = np.asarray(qvec, dtype=np.float64).copy()
    ang = np.asarray(p["orient_mean"] if angles is None else angles, dtype=np.float64).copy()
    return lib().orc_amplitude(C.byref(o), q, _ptr(qv, C.c_double), y, _ptr(ang, C.c_double))


def form_f2(p: dict, q: float, qvec, y: float = 1.0, angles=None) -> float:
    """F^2 of one particle at one event (the micelle: its scattering per
    particle, which has incoherent chain terms)."""
    o = to_params(p)
    qv = np.asarray(qvec, dtype=np.float64).copy()
    ang = np.asarray(p["orient_mean"] if angles is None else angles, dtype=np.float64).copy()
    return lib().orc_form_f2(C.byref(o), q, _ptr(qv, C.c_double), y, _ptr(ang, C.c_double))


def _prepare(p: dict) -> None:
    """Per-parameter-set set-up outside the C tracer: the Hayter-Penfold
    direct correlation function inside the core."""
    if p.get("sq_kind") == "hayter_msa" and p.get("sq_phi", 0.0) > 0.0:
        set_msa(p["sq_phi"], p["sq_extra"][0], p["sq_extra"][1])


def set_msa(eta: float, uc: float, ks: float) -> None:
    from oracle import msa
    c = np.ascontiguousarray(msa.inside_c(float(eta), float(uc), float(ks)))
    lib().orc_set_msa(_ptr(c, C.c_double), float(eta), float(uc), float(ks))


def msa_sq(q: float, radius: float, eta: float, uc: float, ks: float) -> float:
    """The Hayter-Penfold S(q) of the C oracle (after set_msa)."""
    return lib().orc_msa_sq(q, radius, eta, uc, ks)


def trace(p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0, nthreads: int = 1,
          with_w2: bool = False, with_count: bool = False, transmitted: bool = False):
    """Detector (ny, nx) FP64 of neutrons first..first+n-1; optionally the
    sum of w^2 and the hit counts; with transmitted, the unscattered beam
    is added (each neutron's straight flight, weight exp(-mu_att chord))."""
    _prepare(p)
    o = to_params(p)
    det = np.zeros((p["ny"], p["nx"]))
    w2 = np.zeros_like(det) if with_w2 else None
    cnt = np.zeros(det.shape, dtype=np.uint64) if with_count else None
    rc = lib().orc_trace(C.byref(o), first, n, seed, exp_id, nthreads, _ptr(det, C.c_double),
                         _ptr(w2, C.c_double) if w2 is not None else None,
                         _ptr(cnt, C.c_uint64) if cnt is not None else None)
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc})")
    if transmitted:
        lib().orc_transmitted_add(C.byref(o), first, n, seed, exp_id, _ptr(det, C.c_double),
                                  _ptr(w2, C.c_double) if w2 is not None else None,
                                  _ptr(cnt, C.c_uint64) if cnt is not None else None)
    if with_w2 or with_count:
        return det, w2, cnt
    return det


def transmitted(p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0) -> np.ndarray:
    """The transmitted beam alone: detector (ny, nx) FP64."""
    o = to_params(p)
    det = np.zeros((p["ny"], p["nx"]))
    lib().orc_transmitted_add(C.byref(o), first, n, seed, exp_id, _ptr(det, C.c_double), None, None)
    return det


def transmitted_debug(p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0):
    """Per-neutron transmitted events (pixel, w): pixel -1 and w 0 off the
    detector."""
    o = to_params(p)
    pix = np.zeros(n, dtype=np.int32)
    w = np.zeros(n)
    lib().orc_transmitted_debug(C.byref(o), first, n, seed, exp_id, _ptr(pix, C.c_int32), _ptr(w, C.c_double))
    return pix, w


def trace_debug(p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0):
    """Per-neutron (pixel, w, q): pixel -1 and w 0 when nothing is tallied."""
    _prepare(p)
    o = to_params(p)
    pix = np.zeros(n, dtype=np.int32)
    w = np.zeros(n)
    q = np.zeros(n)
    rc = lib().orc_trace_debug(C.byref(o), first, n, seed, exp_id, _ptr(pix, C.c_int32),
                               _ptr(w, C.c_double), _ptr(q, C.c_double))
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc})")
    return pix, w, q


def trace_debug_ex(p: dict, n: int, seed: int, first: int = 0, exp_id: int = 0) -> np.ndarray:
    """Per-neutron intermediates [n, 14]: pixel, w, q, Q_x, Q_y, Q_z, y,
    theta, phi, Psi, path length (m), and the independent size factors
    y_0, y_1, y_2 (1 where a size has no width of its own)."""
    _prepare(p)
    o = to_params(p)
    out = np.zeros((n, 14))
    rc = lib().orc_trace_debug_ex(C.byref(o), first, n, seed, exp_id, _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc})")
    return out


def bf16_round(v: float) -> float:
    return lib().orc_bf16_round(v)


def mlp_param_count() -> int:
    return int(lib().orc_mlp_param_count())


def mlp_forward(w: np.ndarray, x: np.ndarray, round_bf16: bool = False, hidden: bool = False):
    """Outputs y [n]; with hidden, also the pre-activations and activations
    of the four hidden layers, each [4, n, 256]."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    y = np.zeros(n)
    z = np.zeros((4, n, 256)) if hidden else None
    h = np.zeros((4, n, 256)) if hidden else None
    lib().orc_mlp_forward(_ptr(w, C.c_double), _ptr(x, C.c_double), n, _ptr(y, C.c_double),
                          int(round_bf16), _ptr(z, C.c_double) if hidden else None,
                          _ptr(h, C.c_double) if hidden else None)
    return (y, z, h) if hidden else y


def mlp_backward(w: np.ndarray, x: np.ndarray, dy: np.ndarray, round_bf16: bool = False,
                 with_abs: bool = False):
    """Gradient of sum(dy * y) over the parameters; with_abs, also the sum of
    the absolute values of the terms of each element."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    dy = np.ascontiguousarray(dy, dtype=np.float64)
    dw = np.zeros(mlp_param_count())
    da = np.zeros(mlp_param_count()) if with_abs else None
    lib().orc_mlp_backward(_ptr(w, C.c_double), _ptr(x, C.c_double), _ptr(dy, C.c_double), x.shape[0],
                           _ptr(dw, C.c_double), int(round_bf16), _ptr(da, C.c_double) if with_abs else None)
    return (dw, da) if with_abs else dw


def set_surrogate(w: np.ndarray, lo, hi) -> None:
    """Network (FP64 copy of the BF16 parameters) and input box of the
    surrogate mode."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    lib().orc_set_surrogate(_ptr(w, C.c_double), _ptr(lo, C.c_double), _ptr(hi, C.c_double))


def surrogate_judge(p: dict, tol: float, nbins: int):
    """The in-domain judge of the surrogate set by set_surrogate for the
    parameter set p: (number of flagged bins, the ln-errors at the bins'
    edges and midpoints [2 nbins + 1]).  Later surrogate-mode traces send the
    neutrons of flagged bins to the exact average."""
    o = to_params(p)
    err = np.zeros(2 * nbins + 1)
    k = lib().orc_surrogate_judge(C.byref(o), tol, nbins, _ptr(err, C.c_double))
    if k < 0:
        raise ValueError("surrogate judge: no network set or bad arguments")
    return int(k), err


def flexcyl_chain(q: float, L: float, b: float, n: int) -> float:
    """Kholodenko's wormlike-chain factor of the flexible cylinder (n-point rule)."""
    return lib().orc_flexcyl_chain(q, L, b, n)


def flexcyl_section(q: float, R: float, eps: float, n: int) -> float:
    """The elliptical cross-section factor averaged over its in-plane angle."""
    return lib().orc_flexcyl_section(q, R, eps, n)
