"""Seeded synthetic workloads for the SANS sample tracer.

This module only *describes* inputs: parameter sets of the instrument and the
sample, neutron counts, seeds and the seeded generator of the batched
high-throughput experiment set.  It holds none of the method's arithmetic, so
that the HIP library's binding and the CPU oracle can both consume the same
inputs without sharing code.

Units: instrument geometry in metres, wavelength and sample sizes in
Angstrom, scattering-length densities in 1/Angstrom^2, angles in radians.

The paper's own instrument (the KWS-1 model, a monochromatic source, guides,
slits, the sample and a 2D position-sensitive detector; Methods, end of
"Form factor and structure factor models") is not published with it, so a
synthetic stand-in of the same structure is used: a square source 8 m
upstream, a square slit at the sample face, a 1 mm slab sample and a square
area detector 5 m downstream.
"""
from __future__ import annotations

import copy
import math

import numpy as np

KINDS = ("sphere", "core_shell", "cylinder", "ellipsoid", "parallelepiped")
#: models beyond the five of the batched experiment generator: bodies of
#: revolution with spherical caps, hollow and core-shell bodies and the
#: polymer micelle (Tables I-II)
EXTRA_KINDS = ("barbell", "capped_cylinder", "hollow_prism", "micelle", "hollow_cylinder",
               "core_shell_cylinder", "core_shell_ellipsoid", "hollow_prism_thick", "fuzzy_sphere",
               "vesicle", "multilayer_vesicle", "linear_pearls", "fractal", "fractal_core_shell",
               "elliptical_cylinder", "core_shell_bicelle", "core_shell_parallelepiped",
               "core_shell_bicelle_elliptical", "stacked_disks", "sc_paracrystal", "bcc_paracrystal",
               "fcc_paracrystal", "superball", "core_shell_bicelle_elliptical_belt_rough", "raspberry",
               "pearl_necklace", "binary_hard_sphere", "pringle")
#: randomly oriented lamellae (weight per unit volume fraction phi)
LAMELLAR_KINDS = ("lamellar_hg", "lamellar_stack_caille", "lamellar_hg_stack_caille", "lamellar_stack_paracrystal",
                  "adsorbed_layer")
#: shape-independent models: a cross-section in 1/cm, extra[0] = I(0)
SHAPE_INDEPENDENT_KINDS = ("guinier", "ornstein_zernike", "dab", "gauss_coil", "poly_gauss_coil",
                           "teubner_strey", "power_law", "gaussian_peak", "lorentz_peak", "mass_fractal",
                           "star_polymer", "gauss_lorentz_gel", "surface_fractal", "two_power_law",
                           "guinier_porod", "spinodal", "porod", "line", "two_lorentzian", "correlation_length",
                           "broad_peak", "polymer_excl_volume", "mass_surface_fractal", "gel_fit")
ORIENT_KINDS = ("fixed", "gaussian", "isotropic", "uniform_angles")
MODES = ("mc", "quad", "surrogate")
POLY_KINDS = ("schulz", "gaussian")
#: structure factors (when sq_phi > 0): Percus-Yevick hard spheres, Baxter's
#: adhesive hard spheres (sq_extra[0] = stickiness), square-well fluid in the
#: mean spherical approximation (sq_extra = depth in kT, width in diameters)
SQ_KINDS = ("hard_sphere", "sticky_hard_sphere", "square_well", "hayter_msa")

DEG = math.pi / 180.0

#: The common instrument: 10x10 mm source at z = -8 m, 5x5 mm slit on the
#: sample front face, wavelength uniform in 6 A +- 5 %, scattering directions
#: uniform inside a 0.05 rad cone, 10x10x1 mm slab, 0.6x0.6 m detector at 5 m.
INSTRUMENT = dict(
    src_w=0.010, src_h=0.010, src_z=-8.0,
    slit_w=0.005, slit_h=0.005, slit_z=-0.0005,
    lambda0=6.0, dlambda_rel=0.05, cone_alpha=0.05,
    sample_w=0.010, sample_h=0.010, sample_d=0.001,
    det_w=0.6, det_h=0.6, det_z=5.0,
    nx=128, ny=128,
    # straight supermirror guide upstream of the source aperture (length 0:
    # none); reflectivity R0, Qc (1/A), alpha (A), W (1/A) of common m-coated
    # mirrors
    guide_len=0.0, guide_w=0.03, guide_h=0.03, guide_gap=0.5, guide_m=2.0,
    guide_r0=0.99, guide_qc=0.0219, guide_alpha=6.07, guide_wc=0.003,
)

SAMPLE_DEFAULTS = dict(
    kind="sphere", mode="mc",
    size=(50.0, 0.0, 0.0), shell=0.0, sld=(1e-6, 0.0, 0.0),
    phi=0.01, sq_phi=0.0, sq_radius=0.0, sq_kind="hard_sphere", sq_extra=(0.0, 0.0),
    poly=0.0, poly_mask=1, poly_kind="schulz",
    orient_kind="fixed", orient_mean=(0.0, 0.0, 0.0), orient_sigma=(0.0, 0.0, 0.0),
    table_size=4096, quad_n=76,
    extra=(0.0, 0.0, 0.0, 0.0),
    mu_att=0.0,
    poly_sep=(0.0, 0.0, 0.0),
)


def params(**over) -> dict:
    """A full parameter dict: defaults, then the instrument, then overrides."""
    p = dict(SAMPLE_DEFAULTS)
    p.update(INSTRUMENT)
    for k, v in over.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    for k in ("size", "sld", "orient_mean", "orient_sigma", "extra", "sq_extra", "poly_sep"):
        p[k] = tuple(float(x) for x in p[k])
    return p


# --------------------------------------------------------------------------
# The named workloads.  n is the neutron count the workload is quoted on.

def tiny_sphere() -> dict:
    """Monodisperse sphere R = 50 A, contrast 1e-6 /A^2, volume fraction 0.01,
    no structure factor, 128x128 detector, 1e6 neutrons, seed 1."""
    return dict(name="tiny_sphere", n=10**6, seed=1, exp_id=0,
                params=params(kind="sphere", size=(50.0, 0, 0), sld=(1e-6, 0, 0), phi=0.01))


def coreshell_py() -> dict:
    """Core-shell sphere: Schulz core radius (mean 40 A, sigma/mean 0.2) with a
    10 A shell, SLD core/shell/solvent 1e-6/3e-6/6.3e-6, hard-sphere
    Percus-Yevick S(Q) at volume fraction 0.2 (effective radius 50 A),
    256x256 detector, 1e8 neutrons, seed 2."""
    return dict(name="coreshell_py", n=10**8, seed=2, exp_id=0,
                params=params(kind="core_shell", size=(40.0, 0, 0), shell=10.0,
                              sld=(1e-6, 3e-6, 6.3e-6), phi=0.2, sq_phi=0.2, sq_radius=50.0,
                              poly=0.2, poly_mask=1, nx=256, ny=256))


def oriented_cylinder() -> dict:
    """Cylinders R = 20 A, L = 400 A, axis along the beam-perpendicular x axis
    with Gaussian angular spread 10 deg, 256x256 detector, 1e9 neutrons."""
    return dict(name="oriented_cylinder", n=10**9, seed=3, exp_id=0,
                params=params(kind="cylinder", size=(20.0, 400.0, 0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="gaussian",
                              orient_mean=(90 * DEG, 0.0, 0.0),
                              orient_sigma=(10 * DEG, 10 * DEG, 0.0), nx=256, ny=256))


def oriented_ellipsoid() -> dict:
    """Triaxial ellipsoids with semi-axes 20/40/120 A (A along y, B along z,
    C along x), Gaussian angular spread 10 deg, 256x256, 1e9 neutrons."""
    return dict(name="oriented_ellipsoid", n=10**9, seed=4, exp_id=0,
                params=params(kind="ellipsoid", size=(20.0, 40.0, 120.0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="gaussian",
                              orient_mean=(90 * DEG, 0.0, 90 * DEG),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def quad_parallelepiped() -> dict:
    """Isotropically oriented parallelepipeds 20x40x120 A whose orientation
    average is taken by 76x76 Gauss-Legendre quadrature per neutron (exact
    average mode), 128x128 detector, seed 6."""
    return dict(name="quad_parallelepiped", n=10**8, seed=6, exp_id=0,
                params=params(kind="parallelepiped", mode="quad", size=(20.0, 40.0, 120.0),
                              sld=(1e-6, 0, 0), phi=0.01, orient_kind="isotropic"))


def quad_spheroid() -> dict:
    """Polydisperse, isotropically oriented spheroids (a = b = 20 A, c = 60 A,
    Schulz width 0.2 on all axes) averaged by 76x76 (mu, size) quadrature."""
    return dict(name="quad_spheroid", n=10**8, seed=7, exp_id=0,
                params=params(kind="ellipsoid", mode="quad", size=(20.0, 20.0, 60.0),
                              sld=(1e-6, 0, 0), phi=0.01, poly=0.2, poly_mask=7,
                              orient_kind="isotropic"))


def oriented_barbell() -> dict:
    """Barbells: cylinder R = 20 A, L = 400 A with spherical end caps of radius
    40 A, axis along x with Gaussian angular spread 10 deg; the caps' integral
    by 76-point Gauss-Legendre per neutron; 256x256 detector, 1e8 neutrons."""
    return dict(name="oriented_barbell", n=10**8, seed=8, exp_id=0,
                params=params(kind="barbell", size=(20.0, 400.0, 40.0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="gaussian",
                              orient_mean=(90 * DEG, 0.0, 0.0),
                              orient_sigma=(10 * DEG, 10 * DEG, 0.0), nx=256, ny=256))


def quad_capped_cylinder() -> dict:
    """Isotropically oriented capped cylinders (R = 20 A, L = 400 A, cap
    radius 25 A), exact average over 76 orientation nodes, each with the
    76-node cap integral, 128x128 detector, 1e7 neutrons."""
    return dict(name="quad_capped_cylinder", n=10**7, seed=9, exp_id=0,
                params=params(kind="capped_cylinder", mode="quad", size=(20.0, 400.0, 25.0),
                              sld=(1e-6, 0, 0), phi=0.01, orient_kind="isotropic"))


def oriented_hollow_prism() -> dict:
    """Thin-walled hollow rectangular prisms, outer edges 30/50/150 A (A along
    y, B along z, C along x), walls 2 A, Gaussian angular spread 10 deg on all
    three angles, 256x256 detector, 1e9 neutrons."""
    return dict(name="oriented_hollow_prism", n=10**9, seed=10, exp_id=0,
                params=params(kind="hollow_prism", size=(30.0, 50.0, 150.0), shell=2.0,
                              sld=(1e-6, 0, 0), phi=0.01, orient_kind="gaussian",
                              orient_mean=(90 * DEG, 0.0, 90 * DEG),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def quad_hollow_prism() -> dict:
    """Isotropically oriented thin-walled hollow prisms 30x50x150 A (walls
    2 A), exact 76x76 orientation average per neutron, 128x128, 1e7 neutrons."""
    return dict(name="quad_hollow_prism", n=10**7, seed=11, exp_id=0,
                params=params(kind="hollow_prism", mode="quad", size=(30.0, 50.0, 150.0), shell=2.0,
                              sld=(1e-6, 0, 0), phi=0.01, orient_kind="isotropic"))


def micelle_py() -> dict:
    """Polymer micelles: polystyrene-like core R = 40 A (Schulz 0.1) with 60
    Gaussian chains of Rg = 25 A (core block 4000 A^3, corona chain 3500 A^3,
    d = 1), SLD core/corona/solvent 1.0e-6/0.5e-6/6.3e-6, hard-sphere S(Q)
    at volume fraction 0.15 (effective radius 80 A), 256x256, 1e9 neutrons."""
    return dict(name="micelle_py", n=10**9, seed=12, exp_id=0,
                params=params(kind="micelle", size=(40.0, 25.0, 0.0), sld=(1.0e-6, 0.5e-6, 6.3e-6),
                              extra=(60.0, 4000.0, 3500.0, 1.0), phi=0.15, sq_phi=0.15,
                              sq_radius=80.0, poly=0.1, poly_mask=1, nx=256, ny=256))


def oriented_core_shell_cylinder() -> dict:
    """Core-shell cylinders: core R = 20 A, L = 300 A, shell 5 A (faces 3 A),
    SLD core/shell/solvent 1e-6/4e-6/6.3e-6, axis along x with Gaussian
    spread 10 deg, 256x256, 1e9 neutrons."""
    return dict(name="oriented_core_shell_cylinder", n=10**9, seed=13, exp_id=0,
                params=params(kind="core_shell_cylinder", size=(20.0, 300.0, 0.0), shell=5.0,
                              extra=(3.0, 0.0, 0.0, 0.0), sld=(1e-6, 4e-6, 6.3e-6), phi=0.01,
                              orient_kind="gaussian", orient_mean=(90 * DEG, 0.0, 0.0),
                              orient_sigma=(10 * DEG, 10 * DEG, 0.0), nx=256, ny=256))


def quad_hollow_cylinder() -> dict:
    """Isotropic hollow cylinders (bore 20 A, wall 6 A, L = 200 A, Schulz 0.15
    on bore and length), exact average over 76 mu x 76 size nodes, 128x128,
    1e7 neutrons."""
    return dict(name="quad_hollow_cylinder", n=10**7, seed=14, exp_id=0,
                params=params(kind="hollow_cylinder", mode="quad", size=(20.0, 200.0, 0.0), shell=6.0,
                              sld=(1e-6, 0, 0), phi=0.01, poly=0.15, poly_mask=3,
                              orient_kind="isotropic"))


def iso_core_shell_ellipsoid() -> dict:
    """Isotropic triaxial core-shell ellipsoids (core 20/30/80 A, shell 5 A,
    SLD 1e-6/4e-6/6.3e-6, Schulz 0.1 on the core), 256x256, 1e9 neutrons."""
    return dict(name="iso_core_shell_ellipsoid", n=10**9, seed=15, exp_id=0,
                params=params(kind="core_shell_ellipsoid", size=(20.0, 30.0, 80.0), shell=5.0,
                              sld=(1e-6, 4e-6, 6.3e-6), phi=0.01, poly=0.1, poly_mask=7,
                              orient_kind="isotropic", nx=256, ny=256))


def oriented_hollow_prism_thick() -> dict:
    """Hollow prisms with 5 A walls, outer edges 40/60/150 A, Gaussian spread
    10 deg on three angles, 256x256, 1e9 neutrons."""
    return dict(name="oriented_hollow_prism_thick", n=10**9, seed=16, exp_id=0,
                params=params(kind="hollow_prism_thick", size=(40.0, 60.0, 150.0), shell=5.0,
                              sld=(1e-6, 0, 0), phi=0.01, orient_kind="gaussian",
                              orient_mean=(90 * DEG, 0.0, 90 * DEG),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def teubner_strey() -> dict:
    """Microemulsion (Teubner-Strey): correlation length 60 A, period 150 A
    (peak at q = 0.042 / A inside the cone), I(0) = 5 / cm, 256x256, 1e9
    neutrons."""
    return dict(name="teubner_strey", n=10**9, seed=17, exp_id=0,
                params=params(kind="teubner_strey", size=(60.0, 150.0, 0.0), extra=(5.0, 0.0, 0.0, 0.0),
                              nx=256, ny=256))


def poly_gauss_coil() -> dict:
    """Polymer coils with Schulz-Zimm masses (Mw/Mn = 2, z-average Rg = 60 A),
    I(0) = 20 / cm, 256x256, 1e9 neutrons (the power in FP64)."""
    return dict(name="poly_gauss_coil", n=10**9, seed=18, exp_id=0,
                params=params(kind="poly_gauss_coil", size=(60.0, 0.0, 0.0), extra=(20.0, 1.0, 0.0, 0.0),
                              nx=256, ny=256))


def mass_fractal() -> dict:
    """Mass fractal aggregates, dimension 2.3, cut-off length 300 A, I(0) =
    50 / cm, 256x256, 1e9 neutrons."""
    return dict(name="mass_fractal", n=10**9, seed=19, exp_id=0,
                params=params(kind="mass_fractal", size=(300.0, 0.0, 0.0), extra=(50.0, 2.3, 0.0, 0.0),
                              nx=256, ny=256))


def multilayer_vesicle() -> dict:
    """Multilamellar vesicles: 5 lipid shells of 10 A around an 80 A solvent
    core, 20 A water layers between them, SLD shell/solvent 0.4e-6/6.3e-6,
    volume fraction 0.05, 256x256, 1e9 neutrons."""
    return dict(name="multilayer_vesicle", n=10**9, seed=20, exp_id=0,
                params=params(kind="multilayer_vesicle", size=(80.0, 20.0, 0.0), shell=10.0,
                              sld=(6.3e-6, 0.4e-6, 6.3e-6), extra=(5.0, 0.0, 0.0, 0.0), phi=0.05,
                              nx=256, ny=256))


def polymer_excl_volume() -> dict:
    """Swollen polymer chains (Flory exponent 0.588, Rg = 80 A), I(0) =
    10 / cm, 256x256, 1e9 neutrons (incomplete gamma functions in FP64)."""
    return dict(name="polymer_excl_volume", n=10**9, seed=21, exp_id=0,
                params=params(kind="polymer_excl_volume", size=(80.0, 0.0, 0.0), extra=(10.0, 0.588, 0.0, 0.0),
                              nx=256, ny=256))


def oriented_elliptical_cylinder() -> dict:
    """Elliptical cylinders (semi-axes 15 and 40 A, length 300 A) with the
    axis along x and Gaussian spread 10 deg on all three angles, 256x256,
    1e9 neutrons."""
    return dict(name="oriented_elliptical_cylinder", n=10**9, seed=22, exp_id=0,
                params=params(kind="elliptical_cylinder", size=(15.0, 40.0, 300.0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="gaussian", orient_mean=(90 * DEG, 0.0, 0.0),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def oriented_fcc_paracrystal() -> dict:
    """Spheres of radius 40 A on a face-centred cubic paracrystal (nearest
    neighbours 220 A, distortion 0.06), cube axes tilted by 30/20/10 deg with
    Gaussian spread 3 deg, volume fraction 0.2, 256x256, 1e9 neutrons."""
    return dict(name="oriented_fcc_paracrystal", n=10**9, seed=23, exp_id=0,
                params=params(kind="fcc_paracrystal", size=(40.0, 220.0, 0.0), sld=(1e-6, 0, 0),
                              extra=(0.06, 0, 0, 0), phi=0.2, orient_kind="gaussian",
                              orient_mean=(30 * DEG, 20 * DEG, 10 * DEG),
                              orient_sigma=(3 * DEG, 3 * DEG, 3 * DEG), nx=256, ny=256))


def sticky_coreshell() -> dict:
    """The core-shell spheres of the default workload (Schulz core radius 40
    A, sigma/mean 0.2, 10 A shell) as adhesive spheres: Baxter's S(Q) at
    volume fraction 0.1, radius 50 A, stickiness 0.2; 256x256, 1e8 neutrons."""
    return dict(name="sticky_coreshell", n=10**8, seed=24, exp_id=0,
                params=params(kind="core_shell", size=(40.0, 0, 0), shell=10.0,
                              sld=(1e-6, 3e-6, 6.3e-6), phi=0.1, sq_phi=0.1, sq_radius=50.0,
                              sq_kind="sticky_hard_sphere", sq_extra=(0.2, 0.0),
                              poly=0.2, poly_mask=1, nx=256, ny=256))


def mass_surface_fractal() -> dict:
    """Mass-surface fractal: clusters of mass dimension 1.8 and radius of
    gyration 300 A made of primary particles of radius of gyration 25 A with
    surface dimension 2.3, I(0) = 40 / cm, 256x256, 1e9 neutrons."""
    return dict(name="mass_surface_fractal", n=10**9, seed=25, exp_id=0,
                params=params(kind="mass_surface_fractal", size=(300.0, 25.0, 0.0), extra=(40.0, 1.8, 2.3, 0.0),
                              nx=256, ny=256))


def oriented_superball() -> dict:
    """Superballs of half-edge 40 A and exponent parameter 2.5 (a rounded
    cube), axes tilted 30/20/10 deg with Gaussian spread 10 deg, their
    transform by a 24 x 24 Gauss-Legendre rule per event, 256x256, 1e8
    neutrons."""
    return dict(name="oriented_superball", n=10**8, seed=26, exp_id=0,
                params=params(kind="superball", size=(40.0, 0.0, 0.0), sld=(1e-6, 0, 0), extra=(2.5, 0, 0, 0),
                              quad_n=24, phi=0.01, orient_kind="gaussian",
                              orient_mean=(30 * DEG, 20 * DEG, 10 * DEG),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def lamellar_caille() -> dict:
    """Multilamellar phase: head-tail bilayers (tails 14 A, SLD -0.4e-6;
    heads 8 A, 3e-6; solvent 6.3e-6) stacked 30 at a time with repeat
    distance 70 A and Caille parameter 0.1, volume fraction 0.1, 256x256,
    1e9 neutrons."""
    return dict(name="lamellar_caille", n=10**9, seed=27, exp_id=0,
                params=params(kind="lamellar_hg_stack_caille", size=(14.0, 8.0, 70.0), sld=(-0.4e-6, 3e-6, 6.3e-6),
                              extra=(30.0, 0.1, 0.0, 0.0), phi=0.1, nx=256, ny=256))


def pearl_necklace() -> dict:
    """Pearl necklaces: 10 pearls of radius 40 A (SLD 1e-6) joined by 60 A
    rods 8 A thick (SLD 3e-6) into freely jointed chains, solvent 6.3e-6,
    the rods' integrals by a 24-point rule, volume fraction 0.02, 256x256,
    1e9 neutrons."""
    return dict(name="pearl_necklace", n=10**9, seed=28, exp_id=0,
                params=params(kind="pearl_necklace", size=(40.0, 60.0, 8.0), sld=(1e-6, 3e-6, 6.3e-6),
                              extra=(10.0, 0.0, 0.0, 0.0), quad_n=24, phi=0.02, nx=256, ny=256))


def binary_hard_sphere() -> dict:
    """Binary hard-sphere mixture: spheres of 50 A (SLD 1e-6) at volume
    fraction 0.2 and of 20 A (4e-6) at 0.1 in 6.3e-6 solvent, with their
    Percus-Yevick partial structure factors, 256x256, 1e9 neutrons."""
    return dict(name="binary_hard_sphere", n=10**9, seed=29, exp_id=0,
                params=params(kind="binary_hard_sphere", size=(50.0, 20.0, 0.0), sld=(1e-6, 4e-6, 6.3e-6),
                              phi=0.3, extra=(0.1, 0.0, 0.0, 0.0), nx=256, ny=256))


def raspberry() -> dict:
    """Raspberries: 80 A spheres (SLD 1e-6, Schulz 0.1) carrying 40 spheres of
    15 A (4e-6) sunk 0.3 of their diameter, solvent 6.3e-6, volume fraction
    0.05, 256x256, 1e9 neutrons."""
    return dict(name="raspberry", n=10**9, seed=30, exp_id=0,
                params=params(kind="raspberry", size=(80.0, 15.0, 0.0), sld=(1e-6, 4e-6, 6.3e-6),
                              extra=(40.0, 0.3, 0.0, 0.0), poly=0.1, poly_mask=1, phi=0.05, nx=256, ny=256))


def oriented_belt_bicelle() -> dict:
    """Elliptical bicelles with a belt and rough interfaces (core 25 x 42.5 A,
    length 40 A; faces 5 A; belt 6 A; roughness 3 A), Gaussian spread 10 deg
    on three angles, 256x256, 1e9 neutrons."""
    return dict(name="oriented_belt_bicelle", n=10**9, seed=31, exp_id=0,
                params=params(kind="core_shell_bicelle_elliptical_belt_rough", size=(25.0, 40.0, 0.0), shell=6.0,
                              sld=(1e-6, 4e-6, 6.3e-6), extra=(5.0, 2.5e-6, 1.7, 3.0), phi=0.01,
                              orient_kind="gaussian", orient_mean=(60 * DEG, 20 * DEG, 30 * DEG),
                              orient_sigma=(10 * DEG, 10 * DEG, 10 * DEG), nx=256, ny=256))


def adsorbed_layer() -> dict:
    """A 2.5 A (excess) polymer layer (SLD 1.5e-6) on contrast-matched 2000 A
    particles at volume fraction 0.05, smeared by 12 A, 256x256, 1e9
    neutrons."""
    return dict(name="adsorbed_layer", n=10**9, seed=32, exp_id=0,
                params=params(kind="adsorbed_layer", size=(2000.0, 0.0, 0.0), shell=2.5, sld=(1.5e-6, 0.0, 6.3e-6),
                              extra=(12.0, 0.0, 0.0, 0.0), phi=0.05, nx=256, ny=256))


def oriented_pringle() -> dict:
    """Pringles: 60 A plates 10 A thick bent into the saddle 0.001 x^2 - 0.02
    y^2, isotropic orientation, a 16 x 32 polar rule per event, 256x256, 1e8
    neutrons."""
    return dict(name="oriented_pringle", n=10**8, seed=33, exp_id=0,
                params=params(kind="pringle", size=(60.0, 10.0, 0.0), sld=(1e-6, 0, 6.3e-6),
                              extra=(0.001, 0.02, 0.0, 0.0), quad_n=16, phi=0.01, orient_kind="isotropic",
                              nx=256, ny=256))


def attenuated_coreshell() -> dict:
    """The core-shell sphere of coreshell_py in a 1 mm slab that attenuates
    5.6 1/cm (of the order of light water's total cross-section), every
    neutron damped along its path in and out; 256x256, 1e8 neutrons."""
    wl = coreshell_py()
    return dict(name="attenuated_coreshell", n=10**8, seed=34, exp_id=0,
                params=dict(wl["params"], mu_att=560.0))


def poly_sep_cylinder() -> dict:
    """The paper's own polydispersity on the oriented cylinder: radius and
    length each drawn from their own N(1, p^2) kept where positive (Methods,
    Eq. (8); Results: the cylinder's parameter vector carries separate
    spreads of r and L), relative widths 0.15 and 0.25, R = 20 A, L = 400 A,
    axis Gaussian-spread 10 deg about x, 256x256, 1e8 neutrons."""
    return dict(name="poly_sep_cylinder", n=10**8, seed=36, exp_id=0,
                params=params(kind="cylinder", size=(20.0, 400.0, 0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="gaussian", poly_kind="gaussian",
                              poly_sep=(0.15, 0.25, 0.0),
                              orient_mean=(90 * DEG, 0.0, 0.0),
                              orient_sigma=(10 * DEG, 10 * DEG, 0.0), nx=256, ny=256))


def poly_sep_parallelepiped() -> dict:
    """Isotropic parallelepipeds 20 x 40 x 120 A, each edge with its own
    positive-Gaussian width (0.1, 0.2, 0.3), 128x128, 1e8 neutrons."""
    return dict(name="poly_sep_parallelepiped", n=10**8, seed=37, exp_id=0,
                params=params(kind="parallelepiped", size=(20.0, 40.0, 120.0), sld=(1e-6, 0, 0),
                              phi=0.01, orient_kind="isotropic", poly_kind="gaussian",
                              poly_sep=(0.1, 0.2, 0.3)))


def flexible_cylinder_elliptical() -> dict:
    """Flexible cylinders with an elliptical cross-section (one of the models
    the paper's GPU runs fastest against MPI): contour length 1000 A, Kuhn
    length 100 A, minor radius 20 A, axis ratio 1.5, the chain and section
    integrals by 48-point rules, 256x256, 1e8 neutrons."""
    return dict(name="flexible_cylinder_elliptical", n=10**8, seed=38, exp_id=0,
                params=params(kind="flexible_cylinder_elliptical", size=(20.0, 1000.0, 0), sld=(1e-6, 0, 0),
                              phi=0.01, extra=(100.0, 1.5, 0, 0), quad_n=48, nx=256, ny=256))


def flexible_cylinder() -> dict:
    """Flexible cylinders with a circular cross-section: contour length 1000
    A, Kuhn length 100 A, radius 20 A (Schulz, sigma/mean 0.1), the chain
    integrals by a 48-point rule, 256x256, 1e8 neutrons."""
    return dict(name="flexible_cylinder", n=10**8, seed=35, exp_id=0,
                params=params(kind="flexible_cylinder", size=(20.0, 1000.0, 0), sld=(1e-6, 0, 0),
                              phi=0.01, extra=(100.0, 0, 0, 0), quad_n=48, poly=0.1, poly_mask=1,
                              nx=256, ny=256))


def charged_spheres() -> dict:
    """Charged spheres (Schulz radius 45 A, sigma/mean 0.1) at volume fraction
    0.12 with the Hayter-Penfold S(Q) of radius 45 A: contact potential 6 kT,
    screening kappa sigma = 1.8; 256x256, 1e8 neutrons."""
    return dict(name="charged_spheres", n=10**8, seed=39, exp_id=0,
                params=params(kind="sphere", size=(45.0, 0, 0), sld=(1e-6, 0, 6.3e-6), phi=0.12, poly=0.1,
                              sq_phi=0.12, sq_radius=45.0, sq_kind="hayter_msa", sq_extra=(6.0, 1.8),
                              nx=256, ny=256))


WORKLOADS = {
    "tiny_sphere": tiny_sphere,
    "coreshell_py": coreshell_py,
    "oriented_cylinder": oriented_cylinder,
    "oriented_ellipsoid": oriented_ellipsoid,
    "quad_parallelepiped": quad_parallelepiped,
    "quad_spheroid": quad_spheroid,
    "oriented_barbell": oriented_barbell,
    "quad_capped_cylinder": quad_capped_cylinder,
    "oriented_hollow_prism": oriented_hollow_prism,
    "quad_hollow_prism": quad_hollow_prism,
    "micelle_py": micelle_py,
    "oriented_core_shell_cylinder": oriented_core_shell_cylinder,
    "quad_hollow_cylinder": quad_hollow_cylinder,
    "iso_core_shell_ellipsoid": iso_core_shell_ellipsoid,
    "oriented_hollow_prism_thick": oriented_hollow_prism_thick,
    "teubner_strey": teubner_strey,
    "poly_gauss_coil": poly_gauss_coil,
    "mass_fractal": mass_fractal,
    "multilayer_vesicle": multilayer_vesicle,
    "polymer_excl_volume": polymer_excl_volume,
    "oriented_elliptical_cylinder": oriented_elliptical_cylinder,
    "oriented_fcc_paracrystal": oriented_fcc_paracrystal,
    "sticky_coreshell": sticky_coreshell,
    "mass_surface_fractal": mass_surface_fractal,
    "oriented_superball": oriented_superball,
    "lamellar_caille": lamellar_caille,
    "pearl_necklace": pearl_necklace,
    "binary_hard_sphere": binary_hard_sphere,
    "raspberry": raspberry,
    "oriented_belt_bicelle": oriented_belt_bicelle,
    "adsorbed_layer": adsorbed_layer,
    "oriented_pringle": oriented_pringle,
    "attenuated_coreshell": attenuated_coreshell,
    "poly_sep_cylinder": poly_sep_cylinder,
    "flexible_cylinder_elliptical": flexible_cylinder_elliptical,
    "poly_sep_parallelepiped": poly_sep_parallelepiped,
    "charged_spheres": charged_spheres,
    "flexible_cylinder": flexible_cylinder,
}


def workload(name: str) -> dict:
    return copy.deepcopy(WORKLOADS[name]())


# --------------------------------------------------------------------------
# The batched high-throughput set: 4096 virtual experiments.

def batch_experiments(n_exp: int = 4096, seed: int = 4096, nx: int = 128,
                      n_lo: float = 1e5, n_hi: float = 1e7) -> list[dict]:
    """Seeded experiment list (NumPy PCG64).  Model uniform over the five
    kinds; characteristic size log-uniform in [10, 200] A; secondary sizes are
    the size times a log-uniform aspect ratio in [1, 10]; core-shell shell =
    0.25 size; Schulz width uniform in [0, 0.3] applied to all sizes; volume
    fraction uniform in [0, 0.3] for both the number density and the
    hard-sphere S(Q), whose radius is the equal-volume sphere radius;
    isotropic orientation; neutron count log-uniform in [n_lo, n_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for e in range(n_exp):
        kind = KINDS[int(rng.integers(0, 5))]
        s = float(np.exp(rng.uniform(math.log(10.0), math.log(200.0))))
        r1 = float(np.exp(rng.uniform(0.0, math.log(10.0))))
        r2 = float(np.exp(rng.uniform(0.0, math.log(10.0))))
        poly = float(rng.uniform(0.0, 0.3))
        phi = float(rng.uniform(0.0, 0.3))
        n = int(round(float(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))))
        shell = 0.0
        sld = (1e-6, 0.0, 0.0)
        if kind == "sphere":
            size = (s, 0.0, 0.0)
            mask = 1
            req = s
        elif kind == "core_shell":
            size = (s, 0.0, 0.0)
            shell = 0.25 * s
            sld = (1e-6, 3e-6, 6.3e-6)
            mask = 1
            req = s + shell
        elif kind == "cylinder":
            size = (s, s * r1, 0.0)
            mask = 3
            req = (0.75 * s * s * s * r1) ** (1.0 / 3.0)
        elif kind == "ellipsoid":
            size = (s, s * r1, s * r2)
            mask = 7
            req = (s * s * r1 * s * r2) ** (1.0 / 3.0)
        else:
            size = (s, s * r1, s * r2)
            mask = 7
            req = (s * s * r1 * s * r2 * 3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
        p = params(kind=kind, size=size, shell=shell, sld=sld, phi=phi, sq_phi=phi,
                   sq_radius=req, poly=poly, poly_mask=mask,
                   orient_kind="isotropic" if kind in ("cylinder", "ellipsoid",
                                                       "parallelepiped") else "fixed",
                   nx=nx, ny=nx)
        out.append(dict(exp_id=e, n=n, seed=5, params=p))
    return out


# --------------------------------------------------------------------------
# The learned surrogate: training inputs and their box.
#
# Physical inputs x = (ln(q s0), ln(s1/s0), ln(s2/s0), poly, 0, 0, 0, 0):
#   parallelepiped: s0 = A (edge), B/A and C/A uniform in [1, 10], no
#                   polydispersity (orientation average 76 x 76);
#   spheroid:       ellipsoid of revolution a = b = s0, c/a uniform in
#                   [1, 10], Schulz width uniform in [0, 0.3] on all axes
#                   (orientation x size average 76 x 76).
# q s0 log-uniform in [1e-3, 20].
SURROGATE_BOX = {
    "parallelepiped": ((math.log(1e-3), 0.0, 0.0, 0.0), (math.log(20.0), math.log(10.0), math.log(10.0), 0.0)),
    "spheroid": ((math.log(1e-3), 0.0, 0.0, 0.0), (math.log(20.0), 0.0, math.log(10.0), 0.3)),
}


def surrogate_inputs(model: str, n: int, seed: int) -> np.ndarray:
    """Seeded training/validation inputs [n, 8] (float32) in the box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = SURROGATE_BOX[model]
    x = np.zeros((n, 8), dtype=np.float64)
    x[:, 0] = rng.uniform(lo[0], hi[0], size=n)
    if model == "parallelepiped":
        x[:, 1] = np.log(rng.uniform(1.0, 10.0, size=n))
        x[:, 2] = np.log(rng.uniform(1.0, 10.0, size=n))
    else:
        x[:, 2] = np.log(rng.uniform(1.0, 10.0, size=n))
        x[:, 3] = rng.uniform(0.0, 0.3, size=n)
    return x.astype(np.float32)


def surrogate_parallelepiped() -> dict:
    """Tracing workload of the surrogate: isotropic parallelepipeds
    20 x 40 x 120 A, 128x128 detector (as quad_parallelepiped)."""
    wl = quad_parallelepiped()
    wl["name"] = "surrogate_parallelepiped"
    wl["params"] = dict(wl["params"], mode="surrogate")
    return wl


def surrogate_spheroid() -> dict:
    wl = quad_spheroid()
    wl["name"] = "surrogate_spheroid"
    wl["params"] = dict(wl["params"], mode="surrogate")
    return wl


WORKLOADS["surrogate_parallelepiped"] = surrogate_parallelepiped
WORKLOADS["surrogate_spheroid"] = surrogate_spheroid
