"""Thin ctypes binding of libsans (see include/sans.h).

Argument marshalling only: every step of the trace runs in the library's
HIP kernels.  PyTorch supplies device memory and streams.  The names follow
the C ABI one to one (sans_model_create, sans_trace, ...).  If the library is
missing the import fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # loaded first so that libsans shares PyTorch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsans.so")

SANS_ABI_VERSION = 7
SANS_OK = 0
SANS_E_INVALID_ARG = -1
SANS_E_UNSUPPORTED = -2
SANS_E_NOMEM = -3
SANS_E_HIP = -4
SANS_E_DOMAIN = -5
GUIDE_FIELDS = ("guide_len", "guide_w", "guide_h", "guide_gap", "guide_m", "guide_r0", "guide_qc",
                "guide_alpha", "guide_wc")
SANS_ACCUMULATE = 1
SANS_TRANSMITTED = 2

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
        "raspberry": 57, "pearl_necklace": 58, "binary_hard_sphere": 59,
        "adsorbed_layer": 60, "pringle": 61,
        "flexible_cylinder_elliptical": 62, "flexible_cylinder": 63}
SQ_KIND = {"hard_sphere": 0, "sticky_hard_sphere": 1, "square_well": 2, "hayter_msa": 3}
MODE = {"mc": 0, "quad": 1, "surrogate": 2}
ORIENT = {"fixed": 0, "gaussian": 1, "isotropic": 2, "uniform_angles": 3}
POLY_KIND = {"schulz": 0, "gaussian": 1}
TALLY = {"auto": 0, "global": 1, "lds": 2, "xcd": 3, "binned": 4}


class SansError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class sans_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("kind", C.c_int32), ("mode", C.c_int32),
        ("orient_kind", C.c_int32),
        ("size", C.c_double * 3), ("shell", C.c_double), ("sld", C.c_double * 3),
        ("phi", C.c_double), ("sq_phi", C.c_double), ("sq_radius", C.c_double),
        ("poly", C.c_double), ("poly_mask", C.c_int32), ("table_size", C.c_int32),
        ("orient_mean", C.c_double * 3), ("orient_sigma", C.c_double * 3),
        ("src_w", C.c_double), ("src_h", C.c_double), ("src_z", C.c_double),
        ("slit_w", C.c_double), ("slit_h", C.c_double), ("slit_z", C.c_double),
        ("lambda0", C.c_double), ("dlambda_rel", C.c_double), ("cone_alpha", C.c_double),
        ("sample_w", C.c_double), ("sample_h", C.c_double), ("sample_d", C.c_double),
        ("det_w", C.c_double), ("det_h", C.c_double), ("det_z", C.c_double),
        ("nx", C.c_int32), ("ny", C.c_int32), ("quad_n", C.c_int32), ("tally", C.c_int32),
        ("poly_kind", C.c_int32), ("sq_kind", C.c_int32),
        ("extra", C.c_double * 4), ("sq_extra", C.c_double * 2), ("mu_att", C.c_double),
        ("poly_sep", C.c_double * 3), ("guide", C.c_double * 9),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsans.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2501_06054_amd.build` (or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, u32, u64, i64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_int64
    L.sans_model_create.argtypes = [P(sans_params), P(vp)]
    L.sans_model_destroy.argtypes = [vp]
    L.sans_trace.argtypes = [vp, u64, u64, P(sans_params), vp, vp]
    L.sans_trace_ex.argtypes = [vp, u64, u64, u64, u32, u32, vp, vp, vp, vp]
    L.sans_trace_noalloc.argtypes = [vp, u64, u64, u64, u32, u32, vp, vp]
    L.sans_debug_trace.argtypes = [vp, u64, u64, u64, u32, vp, vp, vp, vp]
    L.sans_debug_transmitted.argtypes = [vp, u64, u64, u64, u32, vp, vp, vp]
    L.sans_debug_philox.argtypes = [u64, u64, u64, u32, u32, vp, vp]
    L.sans_debug_table.argtypes = [vp, i32, P(C.c_double), i32]
    L.sans_debug_weight_scale.argtypes = [P(sans_params), P(C.c_double), P(C.c_double)]
    L.sans_pq_avg.argtypes = [vp, vp, vp, i64, vp, vp]
    L.sans_model_constants.argtypes = [vp, P(C.c_double)]
    L.sans_trace_batch.argtypes = [C.c_int, P(sans_params), P(u64), P(u64), vp, C.c_char_p, vp]
    L.sans_batch_release.argtypes = []
    L.sans_model_attach_surrogate.argtypes = [vp, vp, P(C.c_float), P(C.c_float)]
    L.sans_model_attach_surrogate.restype = C.c_int
    L.sans_model_judge_surrogate.argtypes = [vp, C.c_double, i32, P(C.c_float), P(C.c_uint8)]
    L.sans_model_judge_surrogate.restype = C.c_int
    L.sans_pq_dataset.argtypes = [i32, vp, i64, vp, i32, vp]
    L.sans_pq_dataset.restype = C.c_int
    L.sans_mlp_param_count.restype = i64
    L.sans_mlp_workspace_bytes.argtypes = [i64]
    L.sans_mlp_workspace_bytes.restype = u64
    L.sans_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    L.sans_mlp_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.sans_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float,
                                 C.c_float, C.c_int, vp]
    L.sans_mse_grad.argtypes = [vp, vp, i64, vp, vp, vp]
    L.sans_f32_to_bf16.argtypes = [vp, vp, i64, vp]
    L.sans_mlp_last_error.restype = C.c_char_p
    for f in ("sans_mlp_forward", "sans_mlp_backward", "sans_adam_step", "sans_mse_grad",
              "sans_f32_to_bf16"):
        getattr(L, f).restype = C.c_int
    L.sans_abi_params_size.restype = u32
    L.sans_status_string.argtypes = [C.c_int]
    L.sans_status_string.restype = C.c_char_p
    L.sans_last_error.restype = C.c_char_p
    for f in ("sans_model_create", "sans_model_destroy", "sans_trace", "sans_trace_ex", "sans_trace_noalloc",
              "sans_debug_trace", "sans_debug_transmitted", "sans_debug_philox", "sans_debug_table",
              "sans_debug_weight_scale", "sans_pq_avg",
              "sans_model_constants", "sans_trace_batch", "sans_batch_release"):
        getattr(L, f).restype = C.c_int
    return L


lib = _load()


def _check(rc: int, where: str):
    if rc != SANS_OK:
        raise SansError(rc, where, lib.sans_last_error().decode())


def _dev(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def to_params(p: dict, tally: str = "auto") -> sans_params:
    """Workload parameter dict (paper_2501_06054_amd.workloads) -> sans_params."""
    s = sans_params()
    s.abi_version = SANS_ABI_VERSION
    s.kind = KIND[p["kind"]]
    s.mode = MODE[p["mode"]]
    s.orient_kind = ORIENT[p["orient_kind"]]
    for k in range(3):
        s.size[k] = p["size"][k]
        s.sld[k] = p["sld"][k]
        s.orient_mean[k] = p["orient_mean"][k]
        s.orient_sigma[k] = p["orient_sigma"][k]
    for f in ("shell", "phi", "sq_phi", "sq_radius", "poly", "src_w", "src_h", "src_z",
              "slit_w", "slit_h", "slit_z", "lambda0", "dlambda_rel", "cone_alpha",
              "sample_w", "sample_h", "sample_d", "det_w", "det_h", "det_z"):
        setattr(s, f, float(p[f]))
    s.poly_mask = int(p["poly_mask"])
    s.table_size = int(p["table_size"])
    s.nx, s.ny = int(p["nx"]), int(p["ny"])
    s.quad_n = int(p["quad_n"])
    s.tally = TALLY[p.get("tally", tally)]
    s.poly_kind = POLY_KIND[p.get("poly_kind", "schulz")]
    for k, v in enumerate(p.get("extra", (0.0, 0.0, 0.0, 0.0))):
        s.extra[k] = float(v)
    s.sq_kind = SQ_KIND[p.get("sq_kind", "hard_sphere")]
    s.mu_att = float(p.get("mu_att", 0.0))
    for k, v in enumerate(p.get("sq_extra", (0.0, 0.0))):
        s.sq_extra[k] = float(v)
    for k, v in enumerate(p.get("poly_sep", (0.0, 0.0, 0.0))):
        s.poly_sep[k] = float(v)
    for k, f in enumerate(GUIDE_FIELDS):
        s.guide[k] = float(p.get(f, 0.0))
    return s


# ---------------------------------------------------------------- C ABI mirror

def sans_model_create(params) -> C.c_void_p:
    sp = params if isinstance(params, sans_params) else to_params(params)
    h = C.c_void_p()
    _check(lib.sans_model_create(C.byref(sp), C.byref(h)), "sans_model_create")
    return h


def sans_model_destroy(h) -> None:
    _check(lib.sans_model_destroy(h), "sans_model_destroy")


def sans_trace(h, n_neutrons: int, seed: int, params, detector_out, stream=None) -> None:
    sp = None
    if params is not None:
        sp = params if isinstance(params, sans_params) else to_params(params)
    _check(lib.sans_trace(h, n_neutrons, seed, C.byref(sp) if sp is not None else None,
                          _dev(detector_out, torch.float64, "detector_out"), _stream(stream)),
           "sans_trace")


def sans_trace_ex(h, first: int, n: int, seed: int, exp_id: int, flags: int, det,
                  det_w2=None, det_count=None, stream=None) -> None:
    _check(lib.sans_trace_ex(h, first, n, seed, exp_id, flags, _dev(det, torch.float64, "det"),
                             _dev(det_w2, torch.float64, "det_w2"),
                             _dev(det_count, torch.int64, "det_count"), _stream(stream)),
           "sans_trace_ex")


def sans_trace_noalloc(h, first: int, n: int, seed: int, exp_id: int, flags: int, det,
                       stream=None) -> None:
    _check(lib.sans_trace_noalloc(h, first, n, seed, exp_id, flags, _dev(det, torch.float64, "det"),
                                  _stream(stream)), "sans_trace_noalloc")


def sans_debug_trace(h, first: int, n: int, seed: int, exp_id: int, pixel=None, w=None, q=None,
                     stream=None) -> None:
    _check(lib.sans_debug_trace(h, first, n, seed, exp_id, _dev(pixel, torch.int32, "pixel"),
                                _dev(w, torch.float32, "w"), _dev(q, torch.float32, "q"),
                                _stream(stream)), "sans_debug_trace")


def sans_debug_transmitted(h, first: int, n: int, seed: int, exp_id: int, pixel, w, stream=None) -> None:
    _check(lib.sans_debug_transmitted(h, first, n, seed, exp_id, _dev(pixel, torch.int32, "pixel"),
                                      _dev(w, torch.float64, "w"), _stream(stream)), "sans_debug_transmitted")


def sans_debug_philox(seed: int, first: int, n: int, n_blocks: int, exp_id: int, out,
                      stream=None) -> None:
    _check(lib.sans_debug_philox(seed, first, n, n_blocks, exp_id, _dev(out, torch.int32, "out"),
                                 _stream(stream)), "sans_debug_philox")


def sans_debug_weight_scale(params):
    """(<V>, weight scale per metre) of a parameter set, computed on the host."""
    sp = params if isinstance(params, sans_params) else to_params(params)
    mv, ws = C.c_double(), C.c_double()
    _check(lib.sans_debug_weight_scale(C.byref(sp), C.byref(mv), C.byref(ws)), "sans_debug_weight_scale")
    return mv.value, ws.value


def sans_debug_table(h, which: int, n: int):
    import numpy as np
    out = np.zeros(n, dtype=np.float64)
    _check(lib.sans_debug_table(h, which, out.ctypes.data_as(C.POINTER(C.c_double)), n),
           "sans_debug_table")
    return out


def sans_pq_avg(h, q, qvec, out, stream=None) -> None:
    _check(lib.sans_pq_avg(h, _dev(q, torch.float32, "q"), _dev(qvec, torch.float32, "qvec"),
                           q.numel(), _dev(out, torch.float32, "out"), _stream(stream)),
           "sans_pq_avg")


def sans_model_constants(h):
    out = (C.c_double * 3)()
    _check(lib.sans_model_constants(h, out), "sans_model_constants")
    return tuple(out)


def batch_params(params_list):
    """The sans_params array of a batch (list of dicts or sans_params), built
    once: a caller that traces the same experiments repeatedly passes it to
    sans_trace_batch instead of the list, which is otherwise converted at
    every call."""
    arr = (sans_params * len(params_list))()
    for e, p in enumerate(params_list):
        arr[e] = p if isinstance(p, sans_params) else to_params(p)
    return arr


def sans_trace_batch(params_list, n_neutrons, seeds, detectors_out, tune_cache=None,
                     stream=None) -> None:
    """params_list: list of dicts or sans_params, or the array of
    batch_params; detectors_out: device float64 tensor [n_exp, ny, nx]
    (overwritten)."""
    n = len(params_list)
    arr = params_list if isinstance(params_list, C.Array) and params_list._type_ is sans_params \
        else batch_params(params_list)
    nn = (C.c_uint64 * n)(*[int(x) for x in n_neutrons])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    tc = tune_cache.encode() if tune_cache else None
    _check(lib.sans_trace_batch(n, arr, nn, sd, _dev(detectors_out, torch.float64, "detectors_out"),
                                tc, _stream(stream)), "sans_trace_batch")


def sans_batch_release() -> None:
    _check(lib.sans_batch_release(), "sans_batch_release")


def _mcheck(rc: int, where: str):
    if rc != SANS_OK:
        raise SansError(rc, where, lib.sans_mlp_last_error().decode())


def sans_mlp_param_count() -> int:
    return int(lib.sans_mlp_param_count())


def sans_mlp_workspace_bytes(n: int) -> int:
    return int(lib.sans_mlp_workspace_bytes(n))


def sans_mlp_forward(w_bf16, x, y, ws, stream=None) -> None:
    _mcheck(lib.sans_mlp_forward(_dev(w_bf16, torch.bfloat16, "w_bf16"), _dev(x, torch.float32, "x"),
                                 x.shape[0], _dev(y, torch.float32, "y"), _dev(ws, None, "ws"),
                                 _stream(stream)), "sans_mlp_forward")


def sans_mlp_backward(w_bf16, x, dy, dw, ws, stream=None) -> None:
    _mcheck(lib.sans_mlp_backward(_dev(w_bf16, torch.bfloat16, "w_bf16"), _dev(x, torch.float32, "x"),
                                  _dev(dy, torch.float32, "dy"), x.shape[0],
                                  _dev(dw, torch.float32, "dw"), _dev(ws, None, "ws"),
                                  _stream(stream)), "sans_mlp_backward")


def sans_adam_step(w32, w_bf16, dw, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8,
                   stream=None) -> None:
    _mcheck(lib.sans_adam_step(_dev(w32, torch.float32, "w32"), _dev(w_bf16, torch.bfloat16, "w_bf16"),
                               _dev(dw, torch.float32, "dw"), _dev(m, torch.float32, "m"),
                               _dev(v, torch.float32, "v"), w32.numel(), lr, beta1, beta2, eps, step,
                               _stream(stream)), "sans_adam_step")


def sans_mse_grad(y, t, dy, loss=None, stream=None) -> None:
    _mcheck(lib.sans_mse_grad(_dev(y, torch.float32, "y"), _dev(t, torch.float32, "t"), y.numel(),
                              _dev(dy, torch.float32, "dy"), _dev(loss, torch.float32, "loss"),
                              _stream(stream)), "sans_mse_grad")


def sans_f32_to_bf16(x, y, stream=None) -> None:
    _mcheck(lib.sans_f32_to_bf16(_dev(x, torch.float32, "x"), _dev(y, torch.bfloat16, "y"), x.numel(),
                                 _stream(stream)), "sans_f32_to_bf16")


def sans_pq_dataset(kind: str, x, out, quad_n: int = 76, stream=None) -> None:
    """Exact training targets ln(<V^2 P>/<V^2>) for surrogate inputs x [n][8]."""
    _check(lib.sans_pq_dataset(KIND[kind], _dev(x, torch.float32, "x"), x.shape[0],
                               _dev(out, torch.float32, "out"), quad_n, _stream(stream)),
           "sans_pq_dataset")


def sans_model_attach_surrogate(h, w_bf16, lo, hi) -> None:
    lo4 = (C.c_float * 4)(*lo)
    hi4 = (C.c_float * 4)(*hi)
    _check(lib.sans_model_attach_surrogate(h, _dev(w_bf16, torch.bfloat16, "w_bf16"), lo4, hi4),
           "sans_model_attach_surrogate")


def sans_model_judge_surrogate(h, tol: float, nbins: int):
    """Runs the in-domain judge; returns (errors [2 nbins + 1], flags [nbins])
    as NumPy arrays."""
    import numpy as np
    err = np.zeros(2 * nbins + 1, dtype=np.float32)
    flags = np.zeros(nbins, dtype=np.uint8)
    _check(lib.sans_model_judge_surrogate(h, float(tol), nbins, err.ctypes.data_as(C.POINTER(C.c_float)),
                                          flags.ctypes.data_as(C.POINTER(C.c_uint8))),
           "sans_model_judge_surrogate")
    return err, flags


def sans_abi_params_size() -> int:
    return int(lib.sans_abi_params_size())


# ---------------------------------------------------------------- convenience

class Model:
    """Owns a model handle; destroyed on close() / garbage collection."""

    def __init__(self, params: dict, tally: str = "auto"):
        self.params = dict(params)
        self.handle = sans_model_create(to_params(params, tally))

    def close(self):
        if self.handle is not None:
            sans_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def detector(self):
        return torch.zeros((self.params["ny"], self.params["nx"]), dtype=torch.float64,
                           device="cuda")

    def trace(self, n: int, seed: int, det=None, first: int = 0, exp_id: int = 0,
              accumulate: bool = False, det_w2=None, det_count=None, stream=None,
              transmitted: bool = False):
        if det is None:
            det = self.detector()
        flags = (SANS_ACCUMULATE if accumulate else 0) | (SANS_TRANSMITTED if transmitted else 0)
        sans_trace_ex(self.handle, first, n, seed, exp_id, flags, det, det_w2, det_count, stream)
        return det

    def debug_transmitted(self, n: int, seed: int, first: int = 0, exp_id: int = 0):
        pix = torch.empty(n, dtype=torch.int32, device="cuda")
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        sans_debug_transmitted(self.handle, first, n, seed, exp_id, pix, w)
        return pix, w

    def debug_trace(self, n: int, seed: int, first: int = 0, exp_id: int = 0):
        pix = torch.empty(n, dtype=torch.int32, device="cuda")
        w = torch.empty(n, dtype=torch.float32, device="cuda")
        q = torch.empty(n, dtype=torch.float32, device="cuda")
        sans_debug_trace(self.handle, first, n, seed, exp_id, pix, w, q)
        return pix, w, q

    def pq_avg(self, q, qvec=None):
        out = torch.empty_like(q)
        sans_pq_avg(self.handle, q, qvec, out)
        return out

    def constants(self):
        return sans_model_constants(self.handle)
