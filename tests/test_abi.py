"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/sans.h, agrees with the binding on the parameter layout,
and rejects invalid parameters before touching the GPU."""
import ctypes as C
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sans.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(sans_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    return sans


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sans_model_create", "sans_model_destroy", "sans_trace", "sans_trace_ex",
                 "sans_debug_trace", "sans_debug_philox", "sans_pq_avg", "sans_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(S):
    for name in declared_functions():
        assert hasattr(S.lib, name), name


def test_params_layout_matches(S):
    assert S.sans_abi_params_size() == C.sizeof(S.sans_params)


def test_status_strings(S):
    assert S.lib.sans_status_string(0) == b"ok"
    assert S.lib.sans_status_string(S.SANS_E_INVALID_ARG) == b"invalid argument"


def _create_status(S, p):
    h = C.c_void_p()
    sp = S.to_params(p)
    return S.lib.sans_model_create(C.byref(sp), C.byref(h)), sp


@pytest.mark.parametrize("over,status", [
    (dict(size=(-1.0, 0, 0)), -1),
    (dict(phi=1.5), -1),
    (dict(sq_phi=0.7), -1),
    (dict(poly=-0.1), -1),
    (dict(table_size=10), -1),
    (dict(nx=0), -1),
    (dict(cone_alpha=0.0), -1),
    (dict(kind="cylinder", size=(20.0, 0.0, 0.0)), -1),
    (dict(mode="surrogate"), -2),
    (dict(kind="cylinder", size=(20.0, 40.0, 0.0), mode="quad", orient_kind="gaussian"), -2),
    # independent size widths: the models, mode, distribution and sizes that take them
    (dict(kind="core_shell", size=(40.0, 0, 0), shell=10.0, poly_kind="gaussian", poly_sep=(0.2, 0, 0)), -2),
    (dict(kind="cylinder", size=(20.0, 40.0, 0.0), poly_kind="gaussian", poly_sep=(0.1, 0.1, 0.1)), -1),
    (dict(kind="cylinder", size=(20.0, 40.0, 0.0), poly_kind="gaussian", poly_sep=(0.1, 0.1, 0), poly=0.1), -1),
    (dict(kind="cylinder", size=(20.0, 40.0, 0.0), poly_sep=(0.1, 0.1, 0)), -2),
    (dict(kind="cylinder", size=(20.0, 40.0, 0.0), poly_kind="gaussian", poly_sep=(0.1, 0.1, 0),
          mode="quad", orient_kind="isotropic"), -2),
    (dict(kind="sphere", poly_kind="gaussian", poly_sep=(-0.1, 0, 0)), -1),
    (dict(kind="sphere", poly_kind="gaussian", poly_sep=(1.5, 0, 0)), -1),
    # flexible elliptical cylinder: Kuhn length, axis ratio, Monte Carlo mode only
    (dict(kind="flexible_cylinder_elliptical", size=(20.0, 1000.0, 0), extra=(0.0, 1.5, 0, 0)), -1),
    (dict(kind="flexible_cylinder_elliptical", size=(20.0, 1000.0, 0), extra=(100.0, -1.0, 0, 0)), -1),
    (dict(kind="flexible_cylinder_elliptical", size=(20.0, 1000.0, 0), extra=(100.0, 1.5, 0, 0), mode="quad"), -2),
])
def test_invalid_params_rejected_without_gpu(S, over, status):
    from paper_2501_06054_amd import workloads as W
    p = W.params(**over)
    rc, _ = _create_status(S, p)
    assert rc == status
    assert len(S.lib.sans_last_error()) > 0


def test_abi_version_checked(S):
    from paper_2501_06054_amd import workloads as W
    sp = S.to_params(W.params())
    sp.abi_version = 99
    h = C.c_void_p()
    assert S.lib.sans_model_create(C.byref(sp), C.byref(h)) == S.SANS_E_INVALID_ARG


def test_null_arguments(S):
    assert S.lib.sans_model_create(None, None) == S.SANS_E_INVALID_ARG
    assert S.lib.sans_trace(None, 10, 1, None, None, None) == S.SANS_E_INVALID_ARG
    assert S.lib.sans_debug_philox(1, 0, 10, 2, 0, None, None) == S.SANS_E_INVALID_ARG
    assert S.lib.sans_model_destroy(None) == S.SANS_OK


def test_batch_params_array_matches_per_experiment_conversion(S):
    """The prebuilt parameter array of a batch holds, byte for byte, what the
    per-call conversion of the same experiments gives."""
    from paper_2501_06054_amd import workloads as W
    plist = [x["params"] for x in W.batch_experiments()[:17]]
    arr = S.batch_params(plist)
    assert isinstance(arr, C.Array) and arr._type_ is S.sans_params and len(arr) == 17
    for e, p in enumerate(plist):
        assert bytes(arr[e]) == bytes(S.to_params(p)), e
    # already-converted entries pass through unchanged
    again = S.batch_params(list(arr))
    assert bytes(again) == bytes(arr)


def test_unknown_poly_kind_rejected_without_gpu(S):
    from paper_2501_06054_amd import workloads as W
    sp = S.to_params(W.params(poly=0.1))
    sp.poly_kind = 7
    h = C.c_void_p()
    assert S.lib.sans_model_create(C.byref(sp), C.byref(h)) == S.SANS_E_UNSUPPORTED


@pytest.mark.parametrize("over,code", [
    (dict(kind="barbell", size=(40.0, 400.0, 20.0)), "SANS_E_INVALID_ARG"),         # cap radius < R
    (dict(kind="capped_cylinder", size=(20.0, 400.0, 0.0)), "SANS_E_INVALID_ARG"),  # no cap radius
    (dict(kind="barbell", size=(20.0, 400.0, 40.0), poly=0.1, poly_mask=3), "SANS_E_UNSUPPORTED"),
    (dict(kind="capped_cylinder", size=(20.0, 400.0, 40.0), quad_n=0), "SANS_E_INVALID_ARG"),
    (dict(kind="barbell", size=(20.0, 400.0, 40.0), quad_n=257), "SANS_E_INVALID_ARG"),
    (dict(kind="hollow_prism", size=(20.0, 40.0, 60.0), shell=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="hollow_prism", size=(20.0, 40.0, 60.0), shell=1.0, quad_n=0, mode="quad",
          orient_kind="isotropic"), "SANS_E_INVALID_ARG"),
    (dict(kind="micelle", size=(40.0, 25.0, 0.0), extra=(0.5, 4000.0, 3500.0, 1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="micelle", size=(40.0, 25.0, 0.0), extra=(60.0, -1.0, 3500.0, 1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="micelle", size=(40.0, 0.0, 0.0), extra=(60.0, 4000.0, 3500.0, 1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="micelle", size=(40.0, 25.0, 0.0), extra=(60.0, 0.0, 0.0, 1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="hollow_cylinder", size=(20.0, 100.0, 0.0), shell=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_cylinder", size=(20.0, 100.0, 0.0), shell=2.0, extra=(-1.0, 0.0, 0.0, 0.0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_ellipsoid", size=(20.0, 30.0, 40.0), shell=-1.0), "SANS_E_INVALID_ARG"),
    (dict(kind="hollow_prism_thick", size=(20.0, 30.0, 40.0), shell=10.0), "SANS_E_INVALID_ARG"),
    (dict(kind="hollow_prism_thick", size=(20.0, 30.0, 40.0), shell=2.0, poly=0.1, poly_mask=1),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="guinier", size=(20.0, 0.0, 0.0), extra=(-1.0, 0.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="teubner_strey", size=(20.0, 0.0, 0.0), extra=(1.0, 0.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="poly_gauss_coil", size=(20.0, 0.0, 0.0), extra=(1.0, -0.5, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="dab", size=(20.0, 0.0, 0.0), extra=(1.0, 0.0, 0.0, 0.0), poly=0.1), "SANS_E_UNSUPPORTED"),
    (dict(kind="gauss_coil", size=(20.0, 0.0, 0.0), extra=(1.0, 0.0, 0.0, 0.0), sq_phi=0.1, sq_radius=30.0),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="power_law", extra=(1.0, 11.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="gaussian_peak", extra=(1.0, 0.03, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="lorentz_peak", extra=(1.0, -0.01, 0.01, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="mass_fractal", size=(100.0, 0.0, 0.0), extra=(1.0, 1.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="star_polymer", size=(100.0, 0.0, 0.0), extra=(1.0, 0.5, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="gauss_lorentz_gel", size=(100.0, 0.0, 0.0), extra=(1.0, 1.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="vesicle", size=(50.0, 0.0, 0.0), shell=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="linear_pearls", size=(20.0, 5.0, 0.0), extra=(2.5, 0.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="multilayer_vesicle", size=(50.0, 5.0, 0.0), shell=3.0, extra=(3.0, 0, 0, 0), poly=0.1),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="surface_fractal", size=(50.0, 0.0, 0.0), extra=(1.0, 1.5, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="two_power_law", extra=(1.0, 1.0, 0.0, 3.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="guinier_porod", size=(50.0, 0.0, 0.0), extra=(1.0, 2.0, 1.5, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="spinodal", extra=(1.0, 0.0, 3.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="line", extra=(1.0, -2.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="two_lorentzian", size=(10.0, 20.0, 0.0), extra=(1.0, 0.0, 1.0, 2.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="broad_peak", size=(10.0, -0.1, 0.0), extra=(1.0, 2.0, 1.0, 2.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="fractal", size=(10.0, 100.0, 0.0), extra=(0.0, 3.5, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="polymer_excl_volume", size=(10.0, 0.0, 0.0), extra=(1.0, 0.2, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="elliptical_cylinder", size=(10.0, 20.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_bicelle", size=(10.0, 20.0, 0.0), shell=2.0, extra=(-1.0, 1e-6, 0, 0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_parallelepiped", size=(10.0, 20.0, 30.0), extra=(1.0, -1.0, 1.0, 0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_bicelle_elliptical", size=(10.0, 20.0, 0.0), shell=1.0, extra=(1.0, 1e-6, 0.0, 0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="stacked_disks", size=(10.0, 20.0, 0.0), shell=1.0, extra=(2.5, 1.0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="fcc_paracrystal", size=(10.0, 50.0, 0.0), extra=(0.0, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="mass_surface_fractal", size=(100.0, 5.0, 0.0), extra=(1.0, 3.0, 3.0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="mass_surface_fractal", size=(100.0, -5.0, 0.0), extra=(1.0, 2.0, 2.0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="gel_fit", size=(30.0, 100.0, 0.0), extra=(1.0, 0.5, 0.0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="gel_fit", size=(30.0, 100.0, 0.0), extra=(1.0, -0.5, 2.0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", sq_phi=0.2, sq_radius=50.0, sq_kind="sticky_hard_sphere", sq_extra=(0.0, 0.0)),
     "SANS_E_INVALID_ARG"),
    # below Baxter's two-phase boundary: no real adhesion parameter
    (dict(kind="sphere", sq_phi=0.12, sq_radius=50.0, sq_kind="sticky_hard_sphere", sq_extra=(0.05, 0.0)),
     "SANS_E_DOMAIN"),
    (dict(kind="sphere", sq_phi=0.2, sq_radius=50.0, sq_kind="square_well", sq_extra=(1.0, 0.9)),
     "SANS_E_INVALID_ARG"),
    # a deep, wide well drives 1/S(0) below zero
    (dict(kind="sphere", sq_phi=0.2, sq_radius=50.0, sq_kind="square_well", sq_extra=(3.0, 2.0)),
     "SANS_E_DOMAIN"),
    (dict(kind="sphere", poly=0.1, table_size=1001), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", guide_len=-1.0), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", guide_len=5.0, guide_w=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", guide_len=5.0, guide_r0=1.2), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", guide_len=5.0, guide_wc=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="flexible_cylinder", size=(10.0, 500.0, 0.0), extra=(0.0, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="flexible_cylinder", size=(10.0, 500.0, 0.0), extra=(50.0, 0, 0, 0), mode="quad",
          orient_kind="isotropic"), "SANS_E_UNSUPPORTED"),
    (dict(kind="sphere", sq_phi=0.1, sq_radius=50.0, sq_kind="hayter_msa", sq_extra=(-1.0, 2.0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", sq_phi=0.1, sq_radius=50.0, sq_kind="hayter_msa", sq_extra=(60.0, 2.0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", sq_phi=0.1, sq_radius=50.0, sq_kind="hayter_msa", sq_extra=(3.0, 0.0)),
     "SANS_E_INVALID_ARG"),
    (dict(kind="superball", size=(30.0, 0.0, 0.0), extra=(0.2, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="superball", size=(30.0, 0.0, 0.0), extra=(2.0, 0, 0, 0), quad_n=0), "SANS_E_INVALID_ARG"),
    (dict(kind="superball", size=(30.0, 0.0, 0.0), extra=(2.0, 0, 0, 0), mode="quad", orient_kind="isotropic"),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="superball", size=(30.0, 0.0, 0.0), extra=(2.0, 0, 0, 0), poly=0.1, poly_mask=3),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="lamellar_hg", size=(10.0, 0.0, 0.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="lamellar_stack_caille", size=(30.0, 60.0, 0.0), extra=(2.5, 0.1, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="lamellar_hg_stack_caille", size=(10.0, 5.0, 60.0), extra=(10.0, 1.5, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="lamellar_stack_paracrystal", size=(30.0, 60.0, 0.0), extra=(10.0, -1.0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="lamellar_hg", size=(10.0, 5.0, 0.0), poly=0.1), "SANS_E_UNSUPPORTED"),
    (dict(kind="lamellar_stack_caille", size=(30.0, 60.0, 0.0), extra=(5.0, 0.1, 0, 0), sq_phi=0.1,
          sq_radius=30.0), "SANS_E_UNSUPPORTED"),
    (dict(kind="core_shell_bicelle_elliptical_belt_rough", size=(25.0, 40.0, 0.0), shell=6.0,
          extra=(5.0, 2.5e-6, 1.7, -1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="core_shell_bicelle_elliptical_belt_rough", size=(25.0, 40.0, 0.0), shell=6.0,
          extra=(5.0, 2.5e-6, 0.0, 1.0)), "SANS_E_INVALID_ARG"),
    (dict(kind="raspberry", size=(50.0, 10.0, 0.0), extra=(10.0, 1.5, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="raspberry", size=(50.0, 0.0, 0.0), extra=(10.0, 0.5, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="raspberry", size=(50.0, 10.0, 0.0), extra=(10.0, 0.5, 0, 0), poly=0.1, poly_mask=3),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="pearl_necklace", size=(20.0, 50.0, 4.0), extra=(0.0, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="pearl_necklace", size=(20.0, 0.0, 4.0), extra=(5.0, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="pearl_necklace", size=(20.0, 50.0, -1.0), extra=(5.0, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="binary_hard_sphere", size=(50.0, 20.0, 0.0), phi=0.2, extra=(0.3, 0, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="binary_hard_sphere", size=(50.0, 20.0, 0.0), phi=0.2, extra=(0.1, 0, 0, 0), poly=0.1),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="binary_hard_sphere", size=(50.0, 20.0, 0.0), phi=0.2, extra=(0.1, 0, 0, 0), sq_phi=0.1,
          sq_radius=50.0), "SANS_E_UNSUPPORTED"),
    (dict(kind="adsorbed_layer", size=(1000.0, 0.0, 0.0), shell=0.0), "SANS_E_INVALID_ARG"),
    (dict(kind="adsorbed_layer", size=(1000.0, 0.0, 0.0), shell=2.0, poly=0.1), "SANS_E_UNSUPPORTED"),
    (dict(kind="pringle", size=(60.0, 10.0, 0.0), extra=(0.001, 0.02, 0, 0), mode="quad", orient_kind="isotropic"),
     "SANS_E_UNSUPPORTED"),
    (dict(kind="pringle", size=(60.0, 0.0, 0.0), extra=(0.001, 0.02, 0, 0)), "SANS_E_INVALID_ARG"),
    (dict(kind="sphere", mu_att=-1.0), "SANS_E_INVALID_ARG"),
    (dict(kind="parallelepiped", size=(20.0, 40.0, 120.0), mode="surrogate", orient_kind="isotropic", mu_att=10.0),
     "SANS_E_UNSUPPORTED"),
])
def test_capped_body_params_rejected_without_gpu(S, over, code):
    from paper_2501_06054_amd import workloads as W
    sp = S.to_params(W.params(**over))
    h = C.c_void_p()
    assert S.lib.sans_model_create(C.byref(sp), C.byref(h)) == getattr(S, code)


def test_unknown_kind_rejected_without_gpu(S):
    from paper_2501_06054_amd import workloads as W
    sp = S.to_params(W.params(kind="hollow_prism", size=(20.0, 40.0, 60.0), shell=1.0))
    sp.kind = max(S.KIND.values()) + 1
    h = C.c_void_p()
    assert S.lib.sans_model_create(C.byref(sp), C.byref(h)) == S.SANS_E_UNSUPPORTED


def test_unknown_structure_factor_rejected_without_gpu(S):
    from paper_2501_06054_amd import workloads as W
    sp = S.to_params(W.params(kind="sphere", sq_phi=0.1, sq_radius=50.0))
    sp.sq_kind = max(S.SQ_KIND.values()) + 1
    h = C.c_void_p()
    assert S.lib.sans_model_create(C.byref(sp), C.byref(h)) == S.SANS_E_UNSUPPORTED
