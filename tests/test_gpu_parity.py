"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs and the same Philox streams.

Tolerances (the build's stated bar):
  - random streams, pixel indices, hit patterns: bit-exact;
  - per-neutron weight: |dw| <= 1e-5 * w_max + 1e-4 * |w|;
  - total detected intensity: 1e-6 relative;
  - every nonzero pixel: 1e-4 relative.
"""
import math
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2501_06054_amd import workloads as W
from tests.parity_bars import (NTHREADS, SUMMED_BAR, check_detector, check_weights, oracle_detector,  # noqa: F401
                                oracle_detector_sparse)

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    from paper_2501_06054_amd import sans
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sans


# ------------------------------------------------------------------ streams

@pytest.mark.parametrize("seed,first,n,nb,e", [
    (1, 0, 5000, 3, 0),
    (2**63 + 12345, 2**32 - 100, 300, 3, 4095),
    (0xFFFFFFFFFFFFFFFF, 2**40 + 7, 257, 2, 7),
])
def test_philox_streams_bit_exact(S, seed, first, n, nb, e):
    log(f"philox seed={seed} first={first} n={n}")
    out = torch.empty((n, nb, 4), dtype=torch.int32, device="cuda")
    S.sans_debug_philox(seed, first, n, nb, e, out)
    torch.cuda.synchronize()
    g = out.cpu().numpy().view(np.uint32)
    ref = oracle.philox_stream(seed, first, n, nb, e)
    assert np.array_equal(g, ref)


# ------------------------------------------------------------------ tables

@pytest.mark.parametrize("poly", [0.05, 0.2, 0.3])
def test_tables_match_oracle(S, poly):
    p = W.params(kind="cylinder", size=(20, 400, 0), poly=poly, poly_mask=1,
                 orient_kind="gaussian", orient_sigma=(0.1, 0.1, 0.1))
    m = S.Model(p)
    M = p["table_size"]
    tn = S.sans_debug_table(m.handle, 0, M)
    ts = S.sans_debug_table(m.handle, 1, M)
    on = oracle.table_normal(M)
    os_ = oracle.table_schulz(M, poly)
    assert np.allclose(tn, on, rtol=1e-12, atol=1e-13)
    assert np.allclose(ts, os_, rtol=1e-12, atol=1e-14)
    m.close()


@pytest.mark.parametrize("poly", [0.05, 0.2, 0.35])
def test_gaussian_size_table_matches_oracle(S, poly):
    p = W.params(kind="sphere", size=(50, 0, 0), poly=poly, poly_kind="gaussian")
    m = S.Model(p)
    M = p["table_size"]
    ts = S.sans_debug_table(m.handle, 1, M)
    ref = oracle.table_truncnorm(M, poly)
    assert np.allclose(ts, ref, rtol=1e-12, atol=1e-14)
    m.close()


# ------------------------------------------------------------------ per neutron

PER_NEUTRON = {
    "tiny_sphere": (W.workload("tiny_sphere")["params"], 50021),
    "coreshell_py": (W.workload("coreshell_py")["params"], 50021),
    "oriented_cylinder": (W.workload("oriented_cylinder")["params"], 50021),
    "oriented_ellipsoid": (W.workload("oriented_ellipsoid")["params"], 50021),
    "iso_parallelepiped": (W.params(kind="parallelepiped", size=(20, 40, 120),
                                    orient_kind="isotropic"), 30011),
    "poly_cylinder_uniform_angles": (W.params(kind="cylinder", size=(30, 200, 0), poly=0.1,
                                              poly_mask=3, orient_kind="uniform_angles"), 30011),
    "fixed_cylinder": (W.params(kind="cylinder", size=(120, 200, 0),
                                orient_mean=(math.pi / 3, math.pi / 3, 0)), 30011),
    "poly_ellipsoid_py": (W.params(kind="ellipsoid", size=(30, 50, 90), poly=0.25, poly_mask=7,
                                   sq_phi=0.3, sq_radius=45.0, phi=0.3,
                                   orient_kind="isotropic"), 30011),
    "big_sphere_py": (W.params(kind="sphere", size=(300, 0, 0), poly=0.3, sq_phi=0.45,
                               sq_radius=300.0, phi=0.45), 30011),
    "quad_parallelepiped": (dict(W.workload("quad_parallelepiped")["params"]), 601),
    "quad_spheroid": (dict(W.workload("quad_spheroid")["params"]), 601),
    "quad_coreshell": (W.params(kind="core_shell", mode="quad", size=(40, 0, 0), shell=10,
                                sld=(1e-6, 3e-6, 6.3e-6), poly=0.2, sq_phi=0.2,
                                sq_radius=50.0, phi=0.2), 2003),
    "quad_fixed_cylinder": (W.params(kind="cylinder", mode="quad", size=(20, 400, 0), poly=0.1,
                                     orient_mean=(math.pi / 2, 0, 0)), 2003),
    # the paper's own size rule: Gaussian, positive sizes only
    "gauss_coreshell_py": (W.params(kind="core_shell", size=(40, 0, 0), shell=10,
                                    sld=(1e-6, 3e-6, 6.3e-6), poly=0.3, poly_kind="gaussian",
                                    sq_phi=0.2, sq_radius=50.0, phi=0.2, nx=256, ny=256), 50021),
    "gauss_cylinder_uniform_angles": (W.params(kind="cylinder", size=(30, 200, 0), poly=0.35,
                                               poly_kind="gaussian", poly_mask=3,
                                               orient_kind="uniform_angles"), 30011),
    "quad_gauss_sphere": (W.params(kind="sphere", mode="quad", size=(50, 0, 0), poly=0.25,
                                   poly_kind="gaussian"), 2003),
    # bodies with spherical end caps (the caps' integral by quad_n-point
    # Gauss-Legendre in every mode; 23 nodes leave a ragged unrolled tail)
    "oriented_barbell": (W.workload("oriented_barbell")["params"], 30011),
    "poly_capped_cylinder_iso": (W.params(kind="capped_cylinder", size=(20, 200, 25), poly=0.15,
                                          poly_mask=7, orient_kind="isotropic"), 30011),
    "gauss_barbell_uniform_angles": (W.params(kind="barbell", size=(30, 150, 45), poly=0.1,
                                              poly_kind="gaussian", poly_mask=7, quad_n=23,
                                              orient_kind="uniform_angles"), 30011),
    "hemisphere_capped_cylinder": (W.params(kind="capped_cylinder", size=(40, 120, 40),
                                            orient_mean=(math.pi / 4, math.pi / 6, 0)), 30011),
    "quad_capped_cylinder": (dict(W.workload("quad_capped_cylinder")["params"]), 601),
    "quad_poly_barbell_fixed": (W.params(kind="barbell", mode="quad", size=(20, 400, 40), poly=0.1,
                                         poly_mask=7, orient_mean=(math.pi / 2, 0, 0)), 2003),
    # thin-walled hollow prism
    "oriented_hollow_prism": (W.workload("oriented_hollow_prism")["params"], 50021),
    "iso_poly_hollow_prism": (W.params(kind="hollow_prism", size=(40, 60, 200), shell=3.0, poly=0.2,
                                       poly_mask=7, orient_kind="isotropic"), 30011),
    "gauss_hollow_prism_uniform_angles": (W.params(kind="hollow_prism", size=(25, 25, 90), shell=1.0,
                                                   poly=0.15, poly_kind="gaussian", poly_mask=4,
                                                   orient_kind="uniform_angles"), 30011),
    "quad_hollow_prism": (dict(W.workload("quad_hollow_prism")["params"]), 601),
    "quad_poly_hollow_prism_fixed": (W.params(kind="hollow_prism", mode="quad", size=(30, 50, 150),
                                              shell=2.0, poly=0.2, poly_mask=7,
                                              orient_mean=(0.4, 1.2, 0.3)), 2003),
    # polymer micelle (isotropic; the chain functions' series/closed-form
    # switch at (q Rg)^2 = 1 falls inside the Q range)
    "micelle_py": (W.workload("micelle_py")["params"], 50021),
    "gauss_micelle_big_rg": (W.params(kind="micelle", size=(60, 45, 0), sld=(2e-6, 0.5e-6, 6.3e-6),
                                      extra=(120.0, 9000.0, 5000.0, 1.5), poly=0.25, poly_mask=3,
                                      poly_kind="gaussian", orient_kind="isotropic"), 30011),
    "quad_micelle_poly": (W.params(kind="micelle", mode="quad", size=(40, 25, 0),
                                   sld=(1e-6, 0.5e-6, 6.3e-6), extra=(60.0, 4000.0, 3500.0, 1.0),
                                   poly=0.2, poly_mask=3), 2003),
    # hollow and layered bodies
    "oriented_core_shell_cylinder": (W.workload("oriented_core_shell_cylinder")["params"], 50021),
    "iso_poly_hollow_cylinder": (W.params(kind="hollow_cylinder", size=(15, 120, 0), shell=10.0, poly=0.2,
                                          poly_mask=3, orient_kind="isotropic"), 30011),
    "quad_hollow_cylinder": (dict(W.workload("quad_hollow_cylinder")["params"]), 601),
    "iso_core_shell_ellipsoid": (W.workload("iso_core_shell_ellipsoid")["params"], 30011),
    "quad_core_shell_spheroid_poly": (W.params(kind="core_shell_ellipsoid", mode="quad", size=(25, 25, 70),
                                               shell=6.0, sld=(1e-6, 4e-6, 6.3e-6), poly=0.15, poly_mask=7,
                                               orient_kind="isotropic"), 601),
    "oriented_hollow_prism_thick": (W.workload("oriented_hollow_prism_thick")["params"], 30011),
    "quad_hollow_prism_thick": (W.params(kind="hollow_prism_thick", mode="quad", size=(30, 50, 120),
                                         shell=4.0, orient_kind="isotropic"), 601),
    "fixed_gauss_core_shell_cylinder": (W.params(kind="core_shell_cylinder", size=(40, 80, 0), shell=10.0,
                                                 extra=(0.0, 0.0, 0.0, 0.0), sld=(6e-6, 1e-6, 3e-6),
                                                 poly=0.3, poly_kind="gaussian", poly_mask=1,
                                                 orient_mean=(0.7, 0.2, 0.0)), 30011),
    # shape-independent models (cross-sections in 1/cm)
    "guinier": (W.params(kind="guinier", size=(45, 0, 0), extra=(3.0, 0, 0, 0)), 30011),
    "ornstein_zernike": (W.params(kind="ornstein_zernike", size=(80, 0, 0), extra=(3.0, 0, 0, 0)), 30011),
    "dab": (W.params(kind="dab", size=(120, 0, 0), extra=(3.0, 0, 0, 0)), 30011),
    "gauss_coil": (W.params(kind="gauss_coil", size=(70, 0, 0), extra=(3.0, 0, 0, 0)), 30011),
    "poly_gauss_coil": (W.workload("poly_gauss_coil")["params"], 50021),
    "poly_gauss_coil_broad": (W.params(kind="poly_gauss_coil", size=(150, 0, 0), extra=(1.0, 4.0, 0, 0)),
                              30011),
    "teubner_strey": (W.workload("teubner_strey")["params"], 50021),
    "quad_teubner_strey": (W.params(kind="teubner_strey", mode="quad", size=(60, 150, 0),
                                    extra=(5.0, 0, 0, 0)), 2003),
    "power_law": (W.params(kind="power_law", extra=(1e-4, 3.2, 0, 0)), 30011),
    "gaussian_peak": (W.params(kind="gaussian_peak", extra=(4.0, 0.03, 0.004, 0)), 30011),
    "lorentz_peak": (W.params(kind="lorentz_peak", extra=(4.0, 0.025, 0.006, 0)), 30011),
    "mass_fractal": (W.workload("mass_fractal")["params"], 50021),
    "mass_fractal_thin": (W.params(kind="mass_fractal", size=(40, 0, 0), extra=(2.0, 1.4, 0, 0)), 30011),
    "star_polymer": (W.params(kind="star_polymer", size=(70, 0, 0), extra=(3.0, 6.0, 0, 0)), 30011),
    "gauss_lorentz_gel": (W.params(kind="gauss_lorentz_gel", size=(25, 120, 0), extra=(2.0, 0.8, 0, 0)), 30011),
    # sphere family
    "fuzzy_sphere_poly": (W.params(kind="fuzzy_sphere", size=(60, 0, 0), shell=8.0, poly=0.15), 30011),
    "vesicle_poly_py": (W.params(kind="vesicle", size=(80, 0, 0), shell=12.0, sld=(6.3e-6, 1e-6, 6.3e-6),
                                 poly=0.2, sq_phi=0.1, sq_radius=95.0, phi=0.1), 30011),
    "multilayer_vesicle": (W.workload("multilayer_vesicle")["params"], 50021),
    "linear_pearls_poly": (W.params(kind="linear_pearls", size=(25, 12, 0), extra=(6.0, 0, 0, 0), poly=0.1),
                           30011),
    "quad_linear_pearls": (W.params(kind="linear_pearls", mode="quad", size=(25, 12, 0), extra=(6.0, 0, 0, 0),
                                    poly=0.1), 2003),
    # more shape-independent models
    "surface_fractal": (W.params(kind="surface_fractal", size=(150, 0, 0), extra=(2.0, 2.4, 0, 0)), 30011),
    "two_power_law": (W.params(kind="two_power_law", extra=(3e-5, 1.5, 0.02, 4.0)), 30011),
    "guinier_porod": (W.params(kind="guinier_porod", size=(60, 0, 0), extra=(7.0, 1.0, 3.5, 0)), 30011),
    "spinodal": (W.params(kind="spinodal", extra=(9.0, 0.02, 4.0, 0)), 30011),
    "porod": (W.params(kind="porod", extra=(1e-7, 0, 0, 0)), 30011),
    "line": (W.params(kind="line", extra=(0.5, 40.0, 0, 0)), 30011),
    "two_lorentzian": (W.params(kind="two_lorentzian", size=(80.0, 15.0, 0), extra=(3.0, 2.6, 0.5, 1.7)), 30011),
    "correlation_length": (W.params(kind="correlation_length", size=(50.0, 0, 0), extra=(2e-4, 2.5, 1.5, 2.2)),
                           30011),
    "broad_peak": (W.params(kind="broad_peak", size=(120.0, 0.025, 0), extra=(2e-4, 2.5, 1.5, 2.0)), 30011),
    "fractal_poly": (W.params(kind="fractal", size=(20.0, 300.0, 0), sld=(1e-6, 0, 0), extra=(0, 2.2, 0, 0),
                              poly=0.1, phi=0.05), 30011),
    "fractal_core_shell": (W.params(kind="fractal_core_shell", size=(20.0, 250.0, 0), shell=5.0,
                                    sld=(1e-6, 3e-6, 6.3e-6), extra=(0, 2.5, 0, 0), phi=0.05), 30011),
    "polymer_excl_volume": (W.workload("polymer_excl_volume")["params"], 50021),
    "polymer_excl_volume_compact": (W.params(kind="polymer_excl_volume", size=(150.0, 0, 0),
                                             extra=(3.0, 0.34, 0, 0)), 30011),
    # oriented: elliptical cylinder, bicelle, core-shell box
    "oriented_elliptical_cylinder": (W.workload("oriented_elliptical_cylinder")["params"], 50021),
    "quad_elliptical_cylinder": (W.params(kind="elliptical_cylinder", mode="quad", size=(15, 40, 150),
                                          orient_kind="isotropic"), 601),
    "bicelle_poly_iso": (W.params(kind="core_shell_bicelle", size=(30, 40, 0), shell=8.0,
                                  sld=(1e-6, 4e-6, 6.3e-6), extra=(6.0, 2.5e-6, 0, 0), poly=0.15, poly_mask=3,
                                  orient_kind="isotropic"), 30011),
    "quad_bicelle": (W.params(kind="core_shell_bicelle", mode="quad", size=(30, 40, 0), shell=8.0,
                              sld=(1e-6, 4e-6, 6.3e-6), extra=(6.0, 2.5e-6, 0, 0), orient_kind="isotropic"),
                     601),
    "cs_parallelepiped_gauss": (W.params(kind="core_shell_parallelepiped", size=(30, 50, 90),
                                         sld=(1e-6, 3e-6, 6.3e-6), extra=(4.0, 6.0, 3.0, 0),
                                         orient_kind="gaussian", orient_mean=(0.5, 1.0, 0.2),
                                         orient_sigma=(0.2, 0.2, 0.2)), 30011),
    # elliptical bicelle, stacked disks, paracrystals
    "bicelle_elliptical_gauss": (W.params(kind="core_shell_bicelle_elliptical", size=(25, 40, 0), shell=6.0,
                                          sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 2.5e-6, 1.8, 0),
                                          orient_kind="gaussian", orient_mean=(1.2, 0.3, 0.5),
                                          orient_sigma=(0.15, 0.15, 0.3)), 30011),
    "stacked_disks_gauss": (W.params(kind="stacked_disks", size=(80, 25, 0), shell=8.0,
                                     sld=(1e-6, 4e-6, 6.3e-6), extra=(8.0, 4.0, 0, 0), orient_kind="gaussian",
                                     orient_mean=(1.4, 0.2, 0.0), orient_sigma=(0.1, 0.1, 0.0)), 30011),
    "quad_stacked_disks": (W.params(kind="stacked_disks", mode="quad", size=(80, 25, 0), shell=8.0,
                                    sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 4.0, 0, 0), orient_kind="isotropic"),
                           601),
    "oriented_fcc_paracrystal": (W.workload("oriented_fcc_paracrystal")["params"], 50021),
    "sc_paracrystal_fixed": (W.params(kind="sc_paracrystal", size=(30, 150, 0), extra=(0.08, 0, 0, 0),
                                      orient_mean=(0.3, 0.7, 0.2)), 30011),
    "bcc_paracrystal_iso": (W.params(kind="bcc_paracrystal", size=(30, 160, 0), extra=(0.1, 0, 0, 0),
                                     orient_kind="isotropic", poly=0.1), 30011),
    "quad_bcc_paracrystal": (W.params(kind="bcc_paracrystal", mode="quad", size=(30, 160, 0),
                                      extra=(0.1, 0, 0, 0), orient_kind="isotropic", quad_n=40), 301),
    # the last shape-independent models; adhesive and square-well structure factors
    "mass_surface_fractal": (W.workload("mass_surface_fractal")["params"], 50021),
    "gel_fit": (W.params(kind="gel_fit", size=(40.0, 150.0, 0), extra=(3.0, 0.5, 1.7, 0)), 30011),
    "sticky_coreshell": (W.workload("sticky_coreshell")["params"], 50021),
    "square_well_poly_sphere": (W.params(kind="sphere", size=(40.0, 0, 0), sld=(1e-6, 0, 0), phi=0.15, poly=0.1,
                                         sq_phi=0.15, sq_radius=42.0, sq_kind="square_well",
                                         sq_extra=(1.0, 1.4)), 30011),
    "quad_sticky_cylinder": (W.params(kind="cylinder", mode="quad", size=(20.0, 80.0, 0), orient_kind="isotropic",
                                      sq_phi=0.1, sq_radius=30.0, sq_kind="sticky_hard_sphere",
                                      sq_extra=(0.3, 0.0)), 601),
    "repulsive_shoulder_cylinder": (W.params(kind="cylinder", size=(20.0, 120.0, 0), orient_kind="isotropic",
                                             sq_phi=0.2, sq_radius=35.0, sq_kind="square_well",
                                             sq_extra=(-0.8, 1.6)), 30011),
    # superball: a 2-D Gauss-Legendre rule per event
    "oriented_superball": (W.workload("oriented_superball")["params"], 20021),
    "superball_iso_poly": (W.params(kind="superball", size=(30.0, 0, 0), extra=(1.5, 0, 0, 0), quad_n=20,
                                    orient_kind="isotropic", poly=0.1, poly_mask=1), 10011),
    "superball_octahedron": (W.params(kind="superball", size=(50.0, 0, 0), extra=(0.5, 0, 0, 0), quad_n=30,
                                      orient_mean=(0.4, 0.9, 0.3)), 10011),
    "superball_cubic_small_q": (W.params(kind="superball", size=(8.0, 0, 0), extra=(40.0, 0, 0, 0), quad_n=7,
                                         orient_kind="uniform_angles"), 10011),
    # lamellae
    "lamellar_caille": (W.workload("lamellar_caille")["params"], 50021),
    "lamellar_hg": (W.params(kind="lamellar_hg", size=(12.0, 9.0, 0), sld=(-0.3e-6, 2.5e-6, 6.3e-6), phi=0.05),
                    30011),
    "lamellar_stack_caille": (W.params(kind="lamellar_stack_caille", size=(35.0, 90.0, 0), sld=(1e-6, 0, 6.3e-6),
                                       extra=(12.0, 0.3, 0, 0), phi=0.2), 30011),
    "lamellar_stack_paracrystal": (W.params(kind="lamellar_stack_paracrystal", size=(30.0, 75.0, 0),
                                            sld=(1e-6, 0, 6.3e-6), extra=(20.0, 6.0, 0, 0), phi=0.2), 30011),
    "quad_lamellar_paracrystal": (W.params(kind="lamellar_stack_paracrystal", mode="quad", size=(30.0, 75.0, 0),
                                           sld=(1e-6, 0, 6.3e-6), extra=(5.0, 3.0, 0, 0), phi=0.2), 3011),
    # elliptical bicelle with a belt and rough interfaces
    "belt_bicelle_gauss": (W.params(kind="core_shell_bicelle_elliptical_belt_rough", size=(25, 40, 0), shell=6.0,
                                    sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 2.5e-6, 1.7, 3.0), orient_kind="gaussian",
                                    orient_mean=(1.1, 0.4, 0.6), orient_sigma=(0.15, 0.15, 0.3), poly=0.1,
                                    poly_mask=3), 30011),
    "quad_belt_bicelle": (W.params(kind="core_shell_bicelle_elliptical_belt_rough", mode="quad", size=(25, 40, 0),
                                   shell=6.0, sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 2.5e-6, 1.7, 3.0),
                                   orient_kind="isotropic", quad_n=40), 301),
    # raspberry
    "raspberry_poly": (W.params(kind="raspberry", size=(80.0, 15.0, 0), sld=(1e-6, 4e-6, 6.3e-6),
                                extra=(40.0, 0.3, 0, 0), poly=0.1, poly_mask=1, phi=0.05), 30011),
    "raspberry_py": (W.params(kind="raspberry", size=(50.0, 10.0, 0), sld=(1e-6, 4e-6, 6.3e-6),
                              extra=(12.0, 0.0, 0, 0), sq_phi=0.15, sq_radius=62.0, phi=0.15), 30011),
    # pearl necklace
    "pearl_necklace": (W.workload("pearl_necklace")["params"], 50021),
    "pearl_necklace_long_poly": (W.params(kind="pearl_necklace", size=(15.0, 120.0, 5.0), sld=(2e-6, 1e-6, 6.3e-6),
                                          extra=(60.0, 0, 0, 0), quad_n=40, poly=0.1, poly_mask=1), 30011),
    "pearl_single": (W.params(kind="pearl_necklace", size=(30.0, 10.0, 4.0), extra=(1.0, 0, 0, 0), quad_n=8), 10011),
    # binary hard spheres
    "binary_hard_sphere": (W.params(kind="binary_hard_sphere", size=(50.0, 20.0, 0), sld=(1e-6, 4e-6, 6.3e-6),
                                    phi=0.3, extra=(0.1, 0, 0, 0)), 30011),
    "binary_hard_sphere_dilute_small": (W.params(kind="binary_hard_sphere", size=(80.0, 12.0, 0),
                                                 sld=(3e-6, 0.5e-6, 6.3e-6), phi=0.25, extra=(0.01, 0, 0, 0)), 30011),
    "adsorbed_layer": (W.params(kind="adsorbed_layer", size=(2000.0, 0, 0), shell=2.5, sld=(1.5e-6, 0, 6.3e-6),
                                extra=(12.0, 0, 0, 0), phi=0.05), 30011),
    # independent positive-Gaussian widths per size (the paper's Eq. (8))
    "poly_sep_cylinder": (W.workload("poly_sep_cylinder")["params"], 30011),
    "poly_sep_parallelepiped": (W.workload("poly_sep_parallelepiped")["params"], 30011),
    "poly_sep_sphere": (W.params(kind="sphere", size=(60.0, 0, 0), poly_kind="gaussian",
                                 poly_sep=(0.3, 0.0, 0.0)), 20011),
    "poly_sep_ellipsoid_gauss": (W.params(kind="ellipsoid", size=(20.0, 40.0, 120.0), poly_kind="gaussian",
                                          poly_sep=(0.2, 0.1, 0.05), orient_kind="gaussian",
                                          orient_mean=(1.2, 0.4, 0.8), orient_sigma=(0.2, 0.1, 0.3)), 20011),
    "poly_sep_ellcyl_iso": (W.params(kind="elliptical_cylinder", size=(20.0, 35.0, 300.0), poly_kind="gaussian",
                                     poly_sep=(0.1, 0.0, 0.2), orient_kind="isotropic"), 20011),
    # flexible cylinder with an elliptical cross-section
    "flexible_cylinder_elliptical": (W.workload("flexible_cylinder_elliptical")["params"], 20011),
    "flexcyl_poly_stiff": (W.params(kind="flexible_cylinder_elliptical", size=(15.0, 600.0, 0),
                                    extra=(2000.0, 1.0, 0, 0), quad_n=32, poly=0.2, poly_mask=3), 20011),
    "flexcyl_flexible_flat": (W.params(kind="flexible_cylinder_elliptical", size=(10.0, 3000.0, 0),
                                       extra=(40.0, 3.0, 0, 0), quad_n=64, poly=0.15, poly_mask=1,
                                       poly_kind="gaussian"), 20011),
    "flexible_cylinder": (W.workload("flexible_cylinder")["params"], 20011),
    "flexcyl_round_long_len_poly": (W.params(kind="flexible_cylinder", size=(8.0, 4000.0, 0),
                                             extra=(60.0, 0, 0, 0), quad_n=64, poly=0.2, poly_mask=2,
                                             poly_kind="gaussian"), 20011),
    # sample attenuation
    "attenuated_coreshell": (dict(W.workload("coreshell_py")["params"], mu_att=150.0), 30011),
    "attenuated_wide_cone_cylinder": (W.params(kind="cylinder", size=(20.0, 200.0, 0), orient_kind="isotropic",
                                               cone_alpha=1.0, sample_d=0.003, mu_att=400.0), 30011),
    # monodisperse spheres whose q R crosses the first zero of j1 (4.49) and
    # the long series' bound (4.3): the weight near the zero ring
    "sphere_through_first_zero": (W.params(kind="sphere", size=(100.0, 0, 0), sld=(1e-6, 0, 0)), 30011),
    # Hayter-Penfold charged spheres (the Ornstein-Zernike solve at set-up,
    # S tabulated over the instrument's q range)
    "charged_spheres": (W.workload("charged_spheres")["params"], 30011),
    "hayter_strong_cylinder": (W.params(kind="cylinder", size=(20.0, 90.0, 0), orient_kind="isotropic",
                                        sq_phi=0.3, sq_radius=30.0, sq_kind="hayter_msa", sq_extra=(20.0, 3.0)),
                               20011),
    "hayter_weak_screening_poly": (W.params(kind="core_shell", size=(40.0, 0, 0), shell=8.0,
                                            sld=(1e-6, 3e-6, 6.3e-6), phi=0.05, poly=0.15, poly_mask=1,
                                            sq_phi=0.05, sq_radius=48.0, sq_kind="hayter_msa",
                                            sq_extra=(3.0, 0.4)), 20011),
    # a supermirror guide upstream of the source aperture (reflections
    # counted on the unfolded line; the oracle bounces wall by wall)
    "guided_coreshell": (dict(W.workload("coreshell_py")["params"], guide_len=14.0, guide_w=0.012,
                              guide_h=0.012, guide_gap=0.4, guide_m=1.5), 30011),
    "guided_oriented_cylinder_attenuated": (dict(W.workload("oriented_cylinder")["params"], guide_len=20.0,
                                                 guide_w=0.008, guide_h=0.02, guide_gap=1.0, guide_m=3.0,
                                                 lambda0=10.0, dlambda_rel=0.1, mu_att=120.0), 30011),
    # pringle (complex amplitude, a polar rule per event)
    "pringle_iso": (W.params(kind="pringle", size=(60.0, 10.0, 0), extra=(0.001, 0.02, 0, 0), quad_n=16,
                             orient_kind="isotropic"), 10011),
    "pringle_gauss_poly": (W.params(kind="pringle", size=(45.0, 8.0, 0), extra=(0.01, 0.004, 0, 0), quad_n=12,
                                    orient_kind="gaussian", orient_mean=(0.7, 0.3, 1.1),
                                    orient_sigma=(0.2, 0.2, 0.2), poly=0.1, poly_mask=3), 10011),
}


@pytest.mark.parametrize("name", sorted(PER_NEUTRON))
@pytest.mark.parametrize("first", [0, 2**33 + 5])
def test_per_neutron_parity(S, name, first):
    p, n = PER_NEUTRON[name]
    seed = 77
    log(f"per-neutron {name} first={first} n={n}")
    m = S.Model(p)
    pix, w, q = m.debug_trace(n, seed, first=first)
    torch.cuda.synchronize()
    opix, ow, oq = oracle.trace_debug(p, n, seed, first=first)
    assert np.array_equal(pix.cpu().numpy(), opix)
    check_weights(w.cpu().numpy(), ow, name)
    assert np.allclose(q.cpu().numpy(), oq, rtol=2e-7, atol=0)
    m.close()


# ------------------------------------------------------------------ detectors

DET_CASES = ["tiny_sphere", "coreshell_py", "oriented_cylinder", "oriented_ellipsoid",
             "iso_parallelepiped", "poly_ellipsoid_py", "gauss_coreshell_py", "oriented_barbell",
             "poly_capped_cylinder_iso", "oriented_hollow_prism", "iso_poly_hollow_prism", "micelle_py",
             "oriented_core_shell_cylinder", "iso_poly_hollow_cylinder", "iso_core_shell_ellipsoid",
             "oriented_hollow_prism_thick", "teubner_strey", "poly_gauss_coil", "dab", "mass_fractal",
             "star_polymer", "gaussian_peak", "multilayer_vesicle", "linear_pearls_poly", "spinodal",
             "fractal_poly", "polymer_excl_volume", "broad_peak", "oriented_elliptical_cylinder",
             "bicelle_poly_iso", "cs_parallelepiped_gauss", "stacked_disks_gauss", "oriented_fcc_paracrystal",
             "mass_surface_fractal", "gel_fit", "sticky_coreshell", "square_well_poly_sphere",
             "oriented_superball", "lamellar_caille", "lamellar_hg", "lamellar_stack_paracrystal",
             "belt_bicelle_gauss", "raspberry_poly", "pearl_necklace", "binary_hard_sphere",
             "adsorbed_layer", "pringle_iso", "attenuated_coreshell", "poly_sep_cylinder",
             "poly_sep_parallelepiped", "poly_sep_ellipsoid_gauss", "flexible_cylinder_elliptical",
             "flexcyl_flexible_flat", "charged_spheres", "hayter_strong_cylinder", "flexible_cylinder",
             "guided_coreshell", "sphere_through_first_zero"]


@pytest.mark.parametrize("name", DET_CASES)
@pytest.mark.parametrize("tally", ["auto", "global", "lds", "xcd", "binned"])
def test_detector_parity(S, name, tally):
    p, _ = PER_NEUTRON[name]
    n, seed = 300_007, 5
    log(f"detector {name} tally={tally} n={n}")
    m = S.Model(p, tally=tally)
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref, bar = oracle_detector(p, n, seed)
    check_detector(det.cpu().numpy(), ref, f"{name}/{tally}", **bar)
    m.close()


# Detector shapes for the binned tally's row-band tiles: a tile size that is
# not a power of two (the tile index is an FP32 quotient corrected by its
# remainder), a band count that does not divide the rows, wide and flat
# detectors, and the largest band count (64 tiles of 8 rows).
BINNED_SHAPES = [(300, 301), (1000, 37), (257, 1024), (2048, 512), (64, 2000)]


@pytest.mark.parametrize("nx,ny", BINNED_SHAPES)
def test_binned_tally_detector_shapes(S, nx, ny):
    p = dict(PER_NEUTRON["coreshell_py"][0], nx=nx, ny=ny)
    n, seed = 400_009, 8
    log(f"binned tally {nx}x{ny} n={n}")
    m = S.Model(p, tally="binned")
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref, bar = oracle_detector_sparse(p, n, seed)
    check_detector(det.cpu().numpy(), ref, f"binned {nx}x{ny}", **bar)
    m.close()


def test_uncharged_hayter_penfold_is_percus_yevick(S):
    """With no charge (U_c = 0) the mean spherical approximation of charged
    hard spheres is the Percus-Yevick closure: the detector of the Hayter-
    Penfold table equals that of the closed-form hard-sphere S(Q) to FP32
    rounding of the weights."""
    base = W.params(kind="sphere", size=(40.0, 0, 0), sld=(1e-6, 0, 6.3e-6), phi=0.25, poly=0.1,
                    sq_phi=0.25, sq_radius=40.0, nx=128, ny=128)
    n, seed = 300_007, 8
    log(f"uncharged Hayter-Penfold vs Percus-Yevick n={n}")
    dets = []
    for over in (dict(sq_kind="hard_sphere"), dict(sq_kind="hayter_msa", sq_extra=(0.0, 1.0))):
        m = S.Model(dict(base, **over))
        dets.append(m.trace(n, seed).cpu().numpy())
        m.close()
    hs, msa = dets
    assert np.array_equal(hs != 0, msa != 0)
    nz = hs != 0
    assert np.max(np.abs(msa[nz] - hs[nz]) / hs[nz]) < 2e-5
    assert abs(msa.sum() - hs.sum()) <= 2e-6 * hs.sum()


@pytest.mark.parametrize("name", ["quad_parallelepiped", "quad_capped_cylinder", "quad_hollow_prism",
                                  "quad_hollow_cylinder"])
def test_quad_detector_parity(S, name):
    """Exact-average mode (5776 orientation nodes per neutron), 1e5 neutrons
    on the 128 x 128 detector."""
    p = W.workload(name)["params"]
    n, seed = 100_003, 6
    log(f"quad detector {name} n={n}")
    m = S.Model(p)
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref, bar = oracle_detector(p, n, seed)
    check_detector(det.cpu().numpy(), ref, name, **bar)
    m.close()


def test_pq_avg_matches_oracle(S):
    for name in ("quad_parallelepiped", "quad_spheroid", "quad_coreshell", "quad_capped_cylinder",
                 "quad_hollow_prism", "quad_micelle_poly", "quad_hollow_cylinder",
                 "quad_core_shell_spheroid_poly", "quad_hollow_prism_thick", "quad_linear_pearls",
                 "quad_elliptical_cylinder", "quad_bicelle", "quad_stacked_disks", "quad_bcc_paracrystal"):
        p, _ = PER_NEUTRON[name]
        m = S.Model(p)
        qs = np.concatenate([np.linspace(0.0, 0.06, 61), np.geomspace(1e-4, 0.3, 40)])
        qt = torch.tensor(qs, dtype=torch.float32, device="cuda")
        out = m.pq_avg(qt).cpu().numpy()
        ref = np.array([oracle.pq_avg(p, float(np.float32(x))) for x in qs])
        check_weights(out, ref, name)
        m.close()


# ------------------------------------------------------------------ transmitted beam

TRANSMIT_CASES = {
    "attenuated_coreshell": dict(W.workload("coreshell_py")["params"], mu_att=150.0),
    "divergent_thick": W.params(sample_w=0.05, sample_h=0.05, sample_d=0.003, mu_att=400.0, src_w=0.03,
                                src_h=0.02, slit_w=0.012, slit_h=0.008, src_z=-1.0, nx=257, ny=257,
                                det_w=1.0, det_h=1.0),
    "around_opaque_slab": W.params(src_w=0.02, src_h=0.004, slit_w=0.02, slit_h=0.004, src_z=-4.0,
                                   slit_z=-2.0, sample_w=0.03, sample_h=0.1, sample_d=0.001, mu_att=1e7,
                                   det_w=0.3, det_h=0.3),
    "no_attenuation_cylinder": W.params(kind="cylinder", size=(20.0, 80.0, 0), orient_kind="isotropic"),
    "guided_divergent": W.params(sample_w=0.05, sample_h=0.05, sample_d=0.003, mu_att=400.0, src_w=0.03,
                                 src_h=0.02, slit_w=0.012, slit_h=0.008, src_z=-1.0, nx=257, ny=257,
                                 det_w=1.0, det_h=1.0, guide_len=12.0, guide_w=0.02, guide_h=0.015,
                                 guide_gap=0.3, guide_m=2.5, lambda0=5.0),
}


@pytest.mark.parametrize("name", sorted(TRANSMIT_CASES))
def test_transmitted_per_neutron(S, name):
    p = TRANSMIT_CASES[name]
    n, seed = 200_003, 13
    for first in (0, 2**35 + 7):
        log(f"transmitted per-neutron {name} first={first} n={n}")
        m = S.Model(p)
        pix, w = m.debug_transmitted(n, seed, first=first, exp_id=3)
        torch.cuda.synchronize()
        opix, ow = oracle.transmitted_debug(p, n, seed, first=first, exp_id=3)
        assert np.array_equal(pix.cpu().numpy(), opix)
        # w <= 1; the chord's rounding (a few 1e-16 m, from crossing points
        # metres away) enters as exp(-mu delta) and is visible in relative
        # terms only where w is negligible (opaque slabs, corner cuts)
        np.testing.assert_allclose(w.cpu().numpy(), ow, rtol=1e-12, atol=1e-15)
        m.close()


@pytest.mark.parametrize("name", sorted(TRANSMIT_CASES))
@pytest.mark.parametrize("tally", ["auto", "global", "lds", "xcd", "binned"])
def test_transmitted_detector(S, name, tally):
    """The detector with the transmitted beam minus the one without it is the
    oracle's transmitted beam (FP64 weights; only the order of the atomic
    sums differs), and the hit counts add exactly."""
    p = TRANSMIT_CASES[name]
    n, seed = 300_007, 17
    log(f"transmitted detector {name} tally={tally} n={n}")
    m = S.Model(p, tally=tally)
    det = m.trace(n, seed)
    both = m.trace(n, seed, transmitted=True)
    torch.cuda.synchronize()
    ref = oracle.transmitted(p, n, seed)
    got = both.cpu().numpy() - det.cpu().numpy()
    scale = float(np.abs(both.cpu().numpy()).max())
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * scale)
    m.close()


def test_transmitted_with_w2_counts_and_accumulate(S):
    p = TRANSMIT_CASES["attenuated_coreshell"]
    n, seed = 200_003, 19
    log("transmitted w2/count/accumulate")
    m = S.Model(p)
    det = m.detector()
    w2 = torch.zeros_like(det)
    cnt = torch.zeros(det.shape, dtype=torch.int64, device="cuda")
    half = n // 2
    m.trace(half, seed, det=det, det_w2=w2, det_count=cnt, transmitted=True)
    m.trace(n - half, seed, det=det, det_w2=w2, det_count=cnt, first=half, accumulate=True, transmitted=True)
    torch.cuda.synchronize()
    rdet, rw2, rcnt = oracle.trace(p, n, seed, nthreads=NTHREADS, with_w2=True, with_count=True, transmitted=True)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), rcnt)
    beam = rcnt > 1000
    np.testing.assert_allclose(det.cpu().numpy()[beam], rdet[beam], rtol=1e-9)
    np.testing.assert_allclose(w2.cpu().numpy()[beam], rw2[beam], rtol=1e-9)
    # the total: FP64 transmitted weights (1e-9) plus the scattered ones,
    # FP32 weights held to the detector bar (1e-6 of their total)
    scat = oracle.trace(p, n, seed, nthreads=NTHREADS).sum()
    assert abs(det.cpu().numpy().sum() - rdet.sum()) <= 1e-9 * (rdet.sum() - scat) + 1e-6 * scat
    m.close()


def test_transmitted_rejects_unknown_flags(S):
    m = S.Model(W.workload("tiny_sphere")["params"])
    det = m.detector()
    with pytest.raises(RuntimeError):
        S.sans_trace_ex(m.handle, 0, 10, 1, 0, 4, det)
    m.close()


# ------------------------------------------------------------------ edge cases

def test_zero_neutrons_clears_detector(S):
    p = W.workload("tiny_sphere")["params"]
    m = S.Model(p)
    det = torch.full((128, 128), 3.0, dtype=torch.float64, device="cuda")
    m.trace(0, 1, det=det)
    torch.cuda.synchronize()
    assert float(det.abs().sum()) == 0.0
    # accumulate with zero neutrons leaves the detector alone
    det.fill_(2.0)
    m.trace(0, 1, det=det, accumulate=True)
    torch.cuda.synchronize()
    assert float(det.sum()) == 2.0 * 128 * 128
    m.close()


@pytest.mark.parametrize("n", [1, 255, 257, 1000003])
def test_ragged_counts(S, n):
    p = W.workload("coreshell_py")["params"]
    m = S.Model(p)
    det = m.trace(n, 9)
    torch.cuda.synchronize()
    ref = oracle.trace(p, n, 9, nthreads=NTHREADS)
    check_detector(det.cpu().numpy(), ref, f"n={n}")
    m.close()


def test_chunked_and_far_ranges(S):
    p = W.workload("oriented_cylinder")["params"]
    m = S.Model(p)
    first = 2**40 - 12345
    whole = m.trace(200_000, 3, first=first)
    parts = m.trace(70_000, 3, first=first)
    m.trace(130_000, 3, first=first + 70_000, det=parts, accumulate=True)
    torch.cuda.synchronize()
    a, b = whole.cpu().numpy(), parts.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-12, atol=0)
    # 3 neutrons per pixel: the summed per-neutron bar
    ref, bar = oracle_detector_sparse(p, 200_000, 3, first=first)
    check_detector(a, ref, "far range", **bar)
    m.close()


def test_experiment_id_and_w2_count(S):
    p = W.workload("coreshell_py")["params"]
    m = S.Model(p)
    det = m.detector()
    w2 = m.detector()
    cnt = torch.zeros_like(det, dtype=torch.int64)
    m.trace(100_003, 11, det=det, exp_id=17, det_w2=w2, det_count=cnt)
    torch.cuda.synchronize()
    r, rw2, rc = oracle.trace(p, 100_003, 11, exp_id=17, nthreads=NTHREADS, with_w2=True,
                              with_count=True)
    check_detector(det.cpu().numpy(), r, "exp 17")
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), rc)
    nz = rw2 != 0
    assert np.allclose(w2.cpu().numpy()[nz], rw2[nz], rtol=2e-4)
    m.close()


def test_params_update_in_trace(S):
    p = W.workload("tiny_sphere")["params"]
    m = S.Model(p)
    p2 = dict(p, kind="ellipsoid", size=(20.0, 40.0, 60.0), orient_kind="isotropic")
    det = m.detector()
    S.sans_trace(m.handle, 50_000, 4, p2, det)
    torch.cuda.synchronize()
    ref = oracle.trace(p2, 50_000, 4, nthreads=NTHREADS)
    check_detector(det.cpu().numpy(), ref, "params replaced")
    m.close()


# ------------------------------------------------------------------ full sizes

def test_full_size_coreshell(S):
    """The core-shell + Percus-Yevick workload at its full 1e8 neutrons, in
    the launch configuration the benchmark times, against the oracle."""
    wl = W.workload("coreshell_py")
    p, n, seed = wl["params"], wl["n"], wl["seed"]
    log(f"full-size coreshell n={n} oracle threads={NTHREADS}")
    m = S.Model(p)
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref = oracle.trace(p, n, seed, nthreads=NTHREADS)
    check_detector(det.cpu().numpy(), ref, "coreshell 1e8")
    m.close()


@pytest.mark.parametrize("name", ["oriented_cylinder", "oriented_ellipsoid"])
def test_full_size_oriented(S, name):
    """The oriented cylinder and triaxial ellipsoid at their full 1e9
    neutrons, in the launch configuration the benchmark times: the whole
    256 x 256 detector against the oracle's."""
    wl = W.workload(name)
    p, n, seed = wl["params"], wl["n"], wl["seed"]
    log(f"full-size {name} n={n} oracle threads={NTHREADS}")
    m = S.Model(p)
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref = oracle.trace(p, n, seed, nthreads=NTHREADS)
    check_detector(det.cpu().numpy(), ref, f"{name} 1e9")
    m.close()


@pytest.mark.parametrize("name", ["poly_sep_cylinder", "poly_sep_parallelepiped"])
def test_full_size_independent_widths(S, name):
    """The independent-width workloads at their full 1e8 neutrons: the whole
    detector against the oracle's."""
    wl = W.workload(name)
    p, n, seed = wl["params"], wl["n"], wl["seed"]
    log(f"full-size {name} n={n}")
    m = S.Model(p)
    det = m.trace(n, seed)
    torch.cuda.synchronize()
    ref = oracle.trace(p, n, seed, nthreads=NTHREADS)
    check_detector(det.cpu().numpy(), ref, f"{name} 1e8")
    m.close()


@pytest.mark.parametrize("name", ["oriented_cylinder", "oriented_ellipsoid", "oriented_barbell",
                                  "oriented_hollow_prism", "micelle_py", "oriented_core_shell_cylinder",
                                  "teubner_strey", "sticky_coreshell", "mass_surface_fractal", "lamellar_caille",
                                  "pearl_necklace", "polymer_excl_volume", "binary_hard_sphere",
                                  "raspberry", "oriented_belt_bicelle", "adsorbed_layer",
                                  "attenuated_coreshell", "flexible_cylinder_elliptical", "charged_spheres",
                                  "flexible_cylinder"])
def test_full_size_sampled(S, name):
    """1e9- and 1e8-neutron workloads: the full run equals the sum of its chunks, and
    windows spread over the whole index range match the oracle neutron by
    neutron."""
    wl = W.workload(name)
    p, n, seed = wl["params"], wl["n"], wl["seed"]
    log(f"full-size sampled {name} n={n}")
    m = S.Model(p)
    full = m.trace(n, seed)
    parts = m.detector()
    step = n // 8
    for c in range(8):
        m.trace(step, seed, first=c * step, det=parts, accumulate=True)
    torch.cuda.synchronize()
    a, b = full.cpu().numpy(), parts.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-9, atol=0)
    rng = np.random.default_rng(1)
    for first in rng.integers(0, n - 4096, size=8):
        pix, w, _ = m.debug_trace(4096, seed, first=int(first))
        opix, ow, _ = oracle.trace_debug(p, 4096, seed, first=int(first))
        assert np.array_equal(pix.cpu().numpy(), opix)
        check_weights(w.cpu().numpy(), ow, f"{name}@{first}")
    # the first 5e6 neutrons as a whole detector
    head = m.trace(5_000_000, seed)
    torch.cuda.synchronize()
    ref, bar = oracle_detector(p, 5_000_000, seed)
    check_detector(head.cpu().numpy(), ref, f"{name} head", **bar)
    m.close()
