/*
 * sans.h -- C ABI of libsans, the MI355X (gfx950) small-angle neutron
 * scattering sample tracer.
 *
 * The library traces independent neutrons through a small-angle scattering
 * sample and tallies them on an area detector, one neutron per GPU lane.
 * The physics is that of arXiv 2501.06054 ("Small Angle Neutron Scattering in
 * McStas: optimization for high throughput virtual experiments"):
 *   - per scattering event the intensity is n (drho)^2 V^2 P(Q) S(Q), Eq. (3),
 *     with n = phi/<V>, built from the particle amplitude of Eq. (1) (|A|^2,
 *     Eqs. (2) and (4));
 *   - isotropic amplitudes depend on |Q| (Eq. (5)); particles without a
 *     symmetry axis on the projections Q_A, Q_B, Q_C (Eq. (6)); particles with
 *     one symmetry axis on Q_AB and Q_C (Eq. (7)); the cylinder amplitude is
 *     Eq. (9) (read with the sinc factor on the axis projection);
 *   - size (polydispersity) and orientation are drawn anew at every
 *     scattering event (Methods, "Polydispersity and orientational
 *     distributions");
 *   - neutrons are independent and the detector is summed with atomic
 *     updates (Methods, "Acceleration schemes").
 * Instrument, weight, random numbers (Philox4x32-10), tables, the model
 * formulas (the paper names its models but gives few formulas) and the
 * structure factors are the library's own readings where the paper is
 * silent; they are documented field by field below.
 *
 * Conventions for every entry point
 *   - Return value: SANS_OK (0) or a negative SANS_E_* status; the text of
 *     the last error of the calling thread is returned by sans_last_error().
 *     No entry point throws, aborts or exits.
 *   - Pointers documented as "device" are HIP device pointers (for instance
 *     the data of a PyTorch CUDA/HIP tensor); they are owned by the caller and
 *     must stay valid until the work queued on the stream has finished.  The
 *     library never frees caller memory.  Pointers documented as "host" are
 *     read (or written) before the call returns.
 *   - stream is a hipStream_t (NULL: the default stream).  All GPU work is
 *     queued asynchronously on it; nothing synchronises the device.
 *   - Detectors are FP64, row-major [ny][nx], pixel p = iy*nx + ix.
 *   - A neutron count of 0 is a successful no-op (an overwritten detector is
 *     still cleared).
 *   - The random stream of neutron i of experiment e is a pure function of
 *     (seed, e, i): results do not depend on the launch shape, the chunking of
 *     [first, first+n) or the tally strategy, apart from the order of FP64
 *     summation.
 */
#ifndef SANS_H
#define SANS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SANS_ABI_VERSION 7u

/* Status codes. */
#define SANS_OK 0
#define SANS_E_INVALID_ARG (-1) /* null pointer, bad size, value out of range  */
#define SANS_E_UNSUPPORTED (-2) /* mode/model/option combination not provided  */
#define SANS_E_NOMEM (-3)       /* device or host allocation failed            */
#define SANS_E_HIP (-4)         /* a HIP runtime call failed (see last error)  */
#define SANS_E_DOMAIN (-5)      /* inputs outside a model's valid domain        */

/* Scattering models (Tables I and II of the paper): particles, lamellae and
 * shape-independent cross-sections, 62 kinds; the structure factors are
 * selected separately (sans_sq_kind). */
typedef enum {
    SANS_SPHERE = 0,           /* size[0] = R                                   */
    SANS_CORE_SHELL_SPHERE = 1,/* size[0] = core R, shell = thickness            */
    SANS_CYLINDER = 2,         /* size[0] = R, size[1] = L; axis = particle C    */
    SANS_ELLIPSOID = 3,        /* semi-axes size[0..2] along particle A, B, C    */
    SANS_PARALLELEPIPED = 4,   /* edges size[0..2] along particle A, B, C        */
    SANS_BARBELL = 5,          /* cylinder R = size[0], L = size[1] (axis C) with
                                  two spherical end caps of radius r = size[2]
                                  >= R whose centres lie outside the cylinder   */
    SANS_CAPPED_CYLINDER = 6,  /* the same cylinder and cap radius, cap centres
                                  inside the cylinder (lens-shaped end caps)    */
    SANS_HOLLOW_PRISM = 7,     /* hollow rectangular prism, outer edges size[0..2]
                                  along A, B, C, thin walls of thickness shell
                                  (> 0): the faces as sheets (Tables I-II)     */
    SANS_POLYMER_MICELLE = 8,  /* spherical core of radius size[0] carrying
                                  extra[0] Gaussian chains of radius of gyration
                                  size[1] (Tables I-II; the model of Pedersen
                                  and Gerstenberg): sld = core, corona, solvent;
                                  extra[1], extra[2]: volume of one core block
                                  and one corona chain (A^3); extra[3]: the
                                  chains' penetration factor d (their centres
                                  at size[0] + d size[1]); isotropic           */
    SANS_HOLLOW_CYLINDER = 9,  /* bore radius size[0], length size[1], wall of
                                  thickness shell (> 0) around the bore; axis C */
    SANS_CORE_SHELL_CYLINDER = 10, /* core radius size[0] and length size[1] in
                                  a shell of radial thickness shell and end-face
                                  thickness extra[0]; sld = core, shell, solvent */
    SANS_CORE_SHELL_ELLIPSOID = 11, /* core semi-axes size[0..2] along A, B, C,
                                  each grown by shell for the outer surface;
                                  sld = core, shell, solvent                    */
    SANS_HOLLOW_PRISM_THICK = 12, /* box with outer edges size[0..2] less the
                                  cavity whose edges are 2 shell shorter
                                  (0 < 2 shell < every edge; monodisperse)      */
    /* Shape-independent models (Tables I-II): the weight is the macroscopic
     * cross-section dSigma/dOmega(q) in 1/cm, extra[0] its value at q = 0
     * (unless stated otherwise),
     * L = size[0] (phi, poly and the structure factor unused: poly > 0 or
     * sq_phi > 0 is SANS_E_UNSUPPORTED). */
    SANS_GUINIER = 13,           /* exp(-(q L)^2 / 3), L the radius of gyration */
    SANS_ORNSTEIN_ZERNIKE = 14,  /* 1 / (1 + (q L)^2), L the correlation length */
    SANS_DAB = 15,               /* Debye-Anderson-Brumberger 1/(1 + (q L)^2)^2  */
    SANS_GAUSS_COIL = 16,        /* Debye function of (q L)^2, L the coil's Rg  */
    SANS_POLY_GAUSS_COIL = 17,   /* coils with Schulz-Zimm masses, U = Mw/Mn - 1
                                    = extra[1] in [0, 100], L the z-average Rg  */
    SANS_TEUBNER_STREY = 18,     /* microemulsion: correlation length L, period
                                    size[1]                                    */
    SANS_POWER_LAW = 19,         /* extra[0] q^-m, m = extra[1] in [0, 10]
                                    (q in 1/A; no length)                      */
    SANS_GAUSSIAN_PEAK = 20,     /* exp(-(q - q0)^2/(2 w^2)), q0 = extra[1],
                                    w = extra[2] > 0; extra[0] at q0            */
    SANS_LORENTZ_PEAK = 21,      /* 1/(1 + ((q - q0)/w)^2), q0, w as above      */
    SANS_MASS_FRACTAL = 22,      /* the transform of r^(D-3) exp(-r/L), D =
                                    extra[1] in (1, 3]                         */
    SANS_STAR_POLYMER = 23,      /* f = extra[1] >= 1 Gaussian arms, L the star's
                                    radius of gyration                         */
    SANS_GAUSS_LORENTZ_GEL = 24, /* extra[0] exp(-(q L)^2/2) + extra[1] /
                                    (1 + (q size[1])^2)                        */
    /* Isotropic sphere-based particles (Tables I-II, group F); R = size[0]. */
    SANS_FUZZY_SPHERE = 25,      /* sphere smeared by a Gaussian of width shell */
    SANS_VESICLE = 26,           /* solvent-filled shell of thickness shell > 0
                                    around a bore of radius R; sld[1] the
                                    shell, sld[2] the solvent inside and out;
                                    the particle volume is the shell's         */
    SANS_MULTILAYER_VESICLE = 27,/* extra[0] (integer) such shells, a solvent
                                    layer size[1] between them; monodisperse   */
    SANS_LINEAR_PEARLS = 28,     /* extra[0] (integer) spheres of radius R in a
                                    line, gaps size[1]; orientation averaged   */
    /* More shape-independent models (cross-sections in 1/cm, as above). */
    SANS_SURFACE_FRACTAL = 29,   /* transform of r^(3-Ds) exp(-r/L), Ds =
                                    extra[1] in (2, 3]                         */
    SANS_TWO_POWER_LAW = 30,     /* extra[0] q^-m1 up to qc, continued as q^-m2;
                                    m1 = extra[1], qc = extra[2], m2 = extra[3] */
    SANS_GUINIER_POROD = 31,     /* Guinier (dimension s = extra[1], Rg = L)
                                    joined smoothly to Porod q^-m, m = extra[2] */
    SANS_SPINODAL = 32,          /* Furukawa: peak extra[0] at q_max = extra[1],
                                    exponent gamma = extra[2]                  */
    SANS_POROD = 33,             /* extra[0] q^-4                               */
    SANS_LINE = 34,              /* extra[0] + extra[1] q (slope >= 0)           */
    SANS_TWO_LORENTZIAN = 35,    /* extra[0]/(1 + (q size[0])^extra[1]) +
                                    extra[2]/(1 + (q size[1])^extra[3])        */
    SANS_CORRELATION_LENGTH = 36,/* extra[0] q^-extra[1] + extra[2]/(1 + (q L)^extra[3]) */
    SANS_BROAD_PEAK = 37,        /* extra[0] q^-extra[1] + extra[2]/(1 + (|q - size[1]| L)^extra[3]) */
    SANS_FRACTAL = 38,           /* particle: fractal aggregate of spheres of
                                    radius size[0] (Teixeira; cut-off size[1],
                                    dimension extra[1] in (1, 3])              */
    SANS_FRACTAL_CORE_SHELL = 39,/* the same with core-shell blocks (shell,
                                    sld = core, shell, solvent)                */
    SANS_POLYMER_EXCL_VOLUME = 40, /* chain with excluded volume, Flory exponent
                                    extra[1] in [1/3, 1], L its Rg              */
    /* Oriented particles (as SANS_CYLINDER .. SANS_HOLLOW_PRISM_THICK). */
    SANS_ELLIPTICAL_CYLINDER = 41, /* semi-axes size[0] along A, size[1] along B,
                                    length size[2] along C                     */
    SANS_CORE_SHELL_BICELLE = 42,/* core radius size[0], length size[1]; face
                                    layers of thickness extra[0] (SLD extra[1])
                                    on the ends; a rim of thickness shell (SLD
                                    sld[1]) around core and faces; axis C       */
    SANS_CORE_SHELL_PARALLELEPIPED = 43, /* core edges size[0..2]; on each pair of
                                    faces a slab of thickness extra[0..2] that
                                    covers just that face, SLD sld[1]          */
    SANS_CORE_SHELL_BICELLE_ELLIPTICAL = 44, /* the bicelle with core semi-axes
                                    size[0] (A) and extra[2] size[0] (B); the
                                    rim adds shell to both                     */
    SANS_STACKED_DISKS = 45,     /* extra[0] (integer) disks along C: core radius
                                    size[0], thickness size[1], face layers shell
                                    (SLD sld[1]); spacing spread extra[1] (A),
                                    accumulating                               */
    SANS_SC_PARACRYSTAL = 46,    /* spheres of radius size[0] on a simple cubic
                                    paracrystal, nearest neighbours size[1],
                                    distortion factor extra[0] in (0, 1); the
                                    cubic axes along A, B, C                   */
    SANS_BCC_PARACRYSTAL = 47,   /* the same, body-centred cubic               */
    SANS_FCC_PARACRYSTAL = 48,   /* the same, face-centred cubic               */
    /* The last shape-independent models (cross-sections in 1/cm, as above). */
    SANS_MASS_SURFACE_FRACTAL = 49, /* clusters (mass dimension Dm = extra[1],
                                    radius of gyration L) of primary particles
                                    with surface dimension Ds = extra[2] and
                                    radius of gyration size[1] >= 0:
                                    (1 + (qL)^2/(3 pm))^-pm (1 + (q size[1])^2/(3 ps))^-ps,
                                    pm = Dm/2 > 0, ps = (6 - Ds - Dm)/2 > 0    */
    SANS_GEL_FIT = 50,           /* network of mesh size L and dimension D =
                                    extra[2] in (0, 6]:
                                    extra[0] (1 + (D + 1)/3 (qL)^2)^(-D/2),
                                    plus frozen inhomogeneities extra[1]
                                    exp(-(q size[1])^2/3), size[1] >= 0       */
    /* Oriented superball (Tables I-II, group F): |x|^2p + |y|^2p + |z|^2p <=
     * R^2p with x, y, z along A, B, C; R = size[0], p = extra[0] in
     * [0.25, 10000] (1/2 octahedron, 1 sphere, large p a cube of edge 2R).
     * Its transform is integrated over x and y by quad_n-point Gauss-Legendre
     * rules (quad_n^2 nodes per event, in every mode), over z exactly;
     * SANS_MODE_QUAD is not provided (quad_n^2 nodes per orientation node). */
    SANS_SUPERBALL = 51,
    /* Randomly oriented lamellae (Tables I-II, group C): flat sheets at
     * volume fraction phi, the weight phi (2 pi / delta) F1(q)^2 S(q) / q^2
     * with F1 the transform of the sheet's transverse contrast profile and
     * S the stacking factor of extra[0] (integer, 1..1000) sheets;
     * monodisperse, no structure factor (poly > 0 or sq_phi > 0 is
     * SANS_E_UNSUPPORTED). */
    SANS_LAMELLAR_HG = 52,       /* bilayer: tails (sld[0]) over |z| < size[0],
                                    heads (sld[1]) out to size[0] + size[1];
                                    delta = 2 (size[0] + size[1]); S = 1    */
    SANS_LAMELLAR_STACK_CAILLE = 53, /* slabs of thickness size[0] (sld[0]),
                                    repeat distance size[1], Caille parameter
                                    extra[1] in [0, 1]                        */
    SANS_LAMELLAR_HG_STACK_CAILLE = 54, /* head-tail bilayers (size[0],
                                    size[1], as SANS_LAMELLAR_HG) in a Caille
                                    stack of repeat distance size[2]          */
    SANS_LAMELLAR_STACK_PARACRYSTAL = 55, /* slabs of thickness size[0], spacings
                                    Gaussian of mean size[1] and width
                                    extra[1] >= 0 (A)                         */
    SANS_CORE_SHELL_BICELLE_ELLIPTICAL_BELT_ROUGH = 56, /* oriented: elliptic
                                    core (semi-axes size[0] along A,
                                    extra[2] size[0] along B; length size[1]
                                    along C); face layers extra[0] thick (SLD
                                    extra[1]) over the core's cross-section; a
                                    belt of thickness shell (SLD sld[1])
                                    around the core's length only; interface
                                    roughness extra[3] >= 0 (A) damps F by
                                    exp(-(q extra[3])^2 / 2)                  */
    SANS_RASPBERRY = 57,         /* isotropic: a large sphere (radius size[0],
                                    sld[0]) carrying extra[0] >= 0 small
                                    spheres (radius size[1], sld[1]) centred
                                    size[0] + size[1] (1 - 2 extra[1]) from
                                    its centre (extra[1] in [0, 1]: the depth
                                    of penetration in small-sphere diameters),
                                    at independent uniform positions;
                                    polydispersity scales size[0] only       */
    SANS_PEARL_NECKLACE = 58,    /* isotropic: extra[0] (integer, 1..1000)
                                    pearls of radius size[0] (sld[0]) joined
                                    by rods of length size[1] > 0 between
                                    pearl surfaces and diameter size[2] >= 0
                                    (sld[1]) into a freely jointed chain; the
                                    rods' integrals by quad_n-point
                                    Gauss-Legendre; polydispersity scales
                                    size[0] only                              */
    SANS_BINARY_HARD_SPHERE = 59, /* isotropic: spheres of radius size[0]
                                    (sld[0]) and size[1] (sld[1]) at volume
                                    fractions phi - extra[0] and extra[0]
                                    (0 <= extra[0] <= phi < 0.6), with their
                                    Percus-Yevick partial structure factors
                                    (Baxter's factorisation for mixtures);
                                    monodisperse, no separate structure
                                    factor                                    */
    SANS_ADSORBED_LAYER = 60,    /* a layer of excess thickness shell > 0
                                    (adsorbed amount over its bulk density;
                                    SLD sld[0]) on large contrast-matched
                                    particles of radius size[0] at volume
                                    fraction phi, locally flat (3 phi / R of
                                    sheet per volume), smeared by extra[0] >= 0
                                    (A): phi (3/R) 2 pi (drho shell)^2
                                    exp(-(q extra[0])^2) / q^2; monodisperse,
                                    no structure factor                       */
    SANS_PRINGLE = 61,           /* oriented: a plate of thickness size[1] over
                                    the disc of radius size[0] in the AB plane,
                                    bent into the saddle z = extra[0] x^2 -
                                    extra[1] y^2 (1/A); its disc integral by a
                                    quad_n-point radial Gauss-Legendre times
                                    2 quad_n-point angular midpoint rule per
                                    event; no quadrature mode; poly_mask bits
                                    0 (radius) and 1 (thickness)              */
    SANS_FLEXIBLE_CYLINDER_ELLIPTICAL = 62, /* isotropic: a semiflexible chain
                                    of contour length size[1] and Kuhn length
                                    extra[0] > 0 whose cross-section is an
                                    ellipse of semi-axes size[0] and extra[1]
                                    size[0] (extra[1] > 0); F^2 = (drho pi
                                    extra[1] size[0]^2 size[1])^2 P_chain
                                    P_cs, P_chain Kholodenko's closed form for
                                    the wormlike chain (Macromolecules 26,
                                    4179 (1993)), P_cs the ellipse's
                                    [2 J1(q r)/(q r)]^2 averaged over the
                                    in-plane angle, both integrals by
                                    quad_n-point Gauss-Legendre per event;
                                    Monte Carlo mode only; poly_mask bits 0
                                    (radius) and 1 (length)                   */
    SANS_FLEXIBLE_CYLINDER = 63, /* isotropic: the same chain with a circular
                                    cross-section of radius size[0]
                                    (extra[1] unused): F^2 = (drho pi
                                    size[0]^2 size[1])^2 P_chain
                                    [2 J1(q R)/(q R)]^2; chain integrals by
                                    quad_n-point Gauss-Legendre per event;
                                    Monte Carlo mode only; poly_mask bits 0
                                    (radius) and 1 (length)                   */
} sans_kind;

/* Structure factor S(q) of the particles (when sq_phi > 0): volume fraction
 * sq_phi, particle radius sq_radius (diameter sigma = 2 sq_radius). */
typedef enum {
    SANS_SQ_HARD_SPHERE = 0,     /* Percus-Yevick hard spheres                  */
    SANS_SQ_STICKY_HARD_SPHERE = 1, /* Baxter's adhesive hard spheres (Percus-
                                    Yevick closure), stickiness tau =
                                    sq_extra[0] > 0; SANS_E_DOMAIN where no
                                    solution exists (tau below the two-phase
                                    boundary)                                  */
    SANS_SQ_SQUARE_WELL = 2,     /* square-well fluid, mean spherical
                                    approximation: well depth sq_extra[0] (kT,
                                    attractive when > 0) from sigma out to
                                    sq_extra[1] sigma (width in [1, 4]);
                                    SANS_E_DOMAIN where 1/S(q) <= 0 inside the
                                    instrument's q range                       */
    SANS_SQ_HAYTER_MSA = 3       /* Hayter-Penfold charged spheres: hard core
                                    plus the screened Coulomb repulsion
                                    U_c (sigma/r) exp(-kappa (r - sigma)) in
                                    the mean spherical approximation, contact
                                    potential U_c = sq_extra[0] (kT, in
                                    [0, 50]) and screening kappa sigma =
                                    sq_extra[1] (in (0, 50]).  The Ornstein-
                                    Zernike equation is solved on a radial
                                    grid when the parameters are set (about a
                                    second per U_c = 5; cached by eta, U_c,
                                    kappa sigma) and S tabulated over the
                                    instrument's q range; SANS_E_DOMAIN where
                                    the solver finds no physical solution     */
} sans_sq_kind;

/* How the particle size and orientation enter the weight. */
typedef enum {
    SANS_MODE_MC = 0,        /* drawn per event (the paper's method)             */
    SANS_MODE_QUAD = 1,      /* exact Gauss-Legendre average per event           */
    SANS_MODE_SURROGATE = 2  /* learned average (needs an attached network)      */
} sans_mode;

/* Orientation distribution of anisotropic particles.  The particle axes are
 * A = R x, B = R y, C = R z with R = Rz(phi) Ry(theta) Rz(Psi): theta and phi
 * place the C axis, Psi turns the particle about it (the angles that come
 * with Eq. (6)). */
typedef enum {
    SANS_ORIENT_FIXED = 0,          /* angles = orient_mean                      */
    SANS_ORIENT_GAUSSIAN = 1,       /* angle_k = mean_k + sigma_k N(0,1)         */
    SANS_ORIENT_ISOTROPIC = 2,      /* cos theta ~ U[-1,1], phi, Psi ~ U[0,2pi]  */
    SANS_ORIENT_UNIFORM_ANGLES = 3  /* the paper's literal rule: theta ~ U[0,pi],
                                       phi, Psi ~ U[0,2pi] (not isotropic)       */
} sans_orient;

/* Size distribution of the polydisperse sizes (relative size y, mean 1 for
 * Schulz; the mode at 1 for the Gaussian). */
typedef enum {
    SANS_POLY_SCHULZ = 0,   /* Schulz (Gamma) of relative width poly             */
    SANS_POLY_GAUSSIAN = 1  /* the paper's rule (Methods, "Polydispersity and
                               orientational distributions", Eq. (8)): y ~
                               N(1, poly^2) redrawn until positive, i.e. the
                               normal restricted to y > 0, drawn by inverse CDF */
} sans_poly;

/* Tally strategies (all give the same detector up to FP64 summation order).
 * AUTO takes LDS when the whole detector (plus the tables) fits in a
 * workgroup's 160 KiB of LDS, else BINNED.  Requests for det_w2/det_count use
 * the atomic path (GLOBAL, or XCD when asked for). */
typedef enum {
    SANS_TALLY_AUTO = 0,   /* library choice: GLOBAL in quadrature mode, else LDS
                              when the detector fits in 128 KiB, else BINNED     */
    SANS_TALLY_GLOBAL = 1, /* one FP64 global atomic per detected neutron          */
    SANS_TALLY_LDS = 2,    /* workgroup-private FP64 histogram of the detector in
                              LDS; partial histograms summed by a second kernel   */
    SANS_TALLY_XCD = 3,    /* one detector replica per XCD, summed at the end      */
    SANS_TALLY_BINNED = 4  /* two passes per chunk of neutrons: events sorted into
                              row bands of the detector, then each band summed in
                              LDS (detectors too large for LDS)                    */
} sans_tally;

/* Flags. */
#define SANS_ACCUMULATE 1u /* add to the detector instead of overwriting it     */
#define SANS_TRANSMITTED 2u /* sans_trace_ex: also tally the unscattered beam  */

/* All parameters of one virtual experiment.  Plain data; set abi_version to
 * SANS_ABI_VERSION.  Geometry in metres, wavelength and sizes in Angstrom,
 * scattering-length densities in 1/Angstrom^2, angles in radians.
 *
 * Instrument (a synthetic stand-in for the paper's KWS-1 model): a neutron
 * leaves a uniform point of the src_w x src_h source at z = src_z and flies to
 * a uniform point of the slit_w x slit_h slit at z = slit_z; its wavelength is
 * uniform in lambda0 (1 +- dlambda_rel).  The sample is the slab
 * |x| < sample_w/2, |y| < sample_h/2, |z| < sample_d/2; the scattering point is
 * uniform along the path inside it (length l).  The scattered direction is
 * uniform in solid angle inside the cone of half-angle cone_alpha about the
 * incident direction.  The detector is the plane z = det_z, |x| < det_w/2,
 * |y| < det_h/2, with nx x ny pixels.
 *
 * Weight of a detected neutron (forced single scattering, unit initial weight):
 *   w = l[A] * dOmega * (phi / <V>) * F^2 * S(q),
 * dOmega = 2 pi (1 - cos cone_alpha), F the particle amplitude in Angstrom
 * (F^2 = (drho V)^2 P), <V> the number-averaged particle volume, S the
 * structure factor sq_kind (sans_sq_kind) of radius sq_radius and volume
 * fraction sq_phi (S = 1 when sq_phi = 0; fixed radius, decoupled from the
 * drawn size).  Misses of the sample or the detector are not tallied. */
typedef struct {
    uint32_t abi_version;
    int32_t kind;            /* sans_kind                                      */
    int32_t mode;            /* sans_mode                                      */
    int32_t orient_kind;     /* sans_orient                                    */
    double size[3];
    double shell;
    double sld[3];           /* particle (core), shell, solvent                */
    double phi;              /* particle volume fraction (number density phi/<V>) */
    double sq_phi;           /* hard-sphere volume fraction, in [0, 0.6)       */
    double sq_radius;        /* hard-sphere radius                             */
    double poly;             /* relative width sigma of the size draw y (see
                                poly_kind); 0 = monodisperse                   */
    int32_t poly_mask;       /* bit k set: size[k] is multiplied by y (the core-
                                shell shell never is)                          */
    int32_t table_size;      /* knots of the inverse-CDF tables (even, 64..8192) */
    double orient_mean[3];   /* theta, phi, Psi                                */
    double orient_sigma[3];  /* Gaussian spreads (SANS_ORIENT_GAUSSIAN)        */
    double src_w, src_h, src_z;
    double slit_w, slit_h, slit_z;
    double lambda0, dlambda_rel, cone_alpha;
    double sample_w, sample_h, sample_d;
    double det_w, det_h, det_z;
    int32_t nx, ny;
    int32_t quad_n;          /* Gauss-Legendre order of SANS_MODE_QUAD (<= 256);
                                also the order of the end-cap integral of
                                SANS_BARBELL / SANS_CAPPED_CYLINDER in every
                                mode                                           */
    int32_t tally;           /* sans_tally                                     */
    int32_t poly_kind;       /* sans_poly                                      */
    int32_t sq_kind;         /* sans_sq_kind                                   */
    double extra[4];         /* model parameters beyond size and shell (see
                                sans_kind; unused entries 0)                   */
    double sq_extra[2];      /* structure-factor parameters (sans_sq_kind)     */
    double mu_att;           /* attenuation coefficient of the sample (1/m,
                                >= 0): the weight is damped by exp(-mu_att
                                (path inside the slab before the scattering
                                point + path after it to where the scattered
                                neutron leaves the slab)); 0 = none.
                                Attenuated Monte Carlo runs take any tally
                                (their own kernel instances); attenuated
                                exact-average runs tally with atomics
                                (GLOBAL, or XCD when asked for); the batched
                                launch and the surrogate mode refuse them
                                (SANS_E_UNSUPPORTED)                        */
    double poly_sep[3];      /* independent relative widths (the paper's rule,
                                Methods, "Polydispersity and orientational
                                distributions", Eq. (8): each radius or
                                length drawn from its own Gaussian; the
                                cylinder's parameter vector carries separate
                                spreads of r and L): size[k] is multiplied by
                                its own y_k ~ N(1, poly_sep[k]^2) kept where
                                positive (inverse CDF), y_0 from the word the
                                single draw uses, y_1 and y_2 from a fourth
                                Philox block.  All 0: none.  Otherwise
                                Monte Carlo mode only, poly = 0 and poly_kind
                                SANS_POLY_GAUSSIAN, for the sphere (k = 0),
                                cylinder (k <= 1), ellipsoid,
                                parallelepiped and elliptical cylinder
                                (k <= 2), whose volumes are products of
                                powers of the sizes (<V> = V prod <y_k^e_k>);
                                the batched launch refuses it              */
    double guide[9];         /* a straight neutron guide upstream of the
                                source aperture (the paper's KWS-1
                                instrument brings the beam to its apertures
                                through guides; Methods): length guide[0] (m;
                                0 = no guide), width guide[1] and height
                                guide[2] (m, centred on the beam axis), gap
                                guide[3] (m) from its exit to the source
                                aperture, supermirror m = guide[4] and the
                                reflectivity R0 = guide[5], Qc = guide[6]
                                (1/A), alpha = guide[7] (A), W = guide[8]
                                (1/A): R(Q) = R0 up to Qc, then R0/2 (1 -
                                tanh((Q - m Qc)/W)) (1 - alpha (Q - Qc)),
                                0 where negative.  The moderator fills the
                                guide's entrance; each traced neutron is
                                followed back from its source point along its
                                flight: its weight is 0 if it misses the
                                guide's exit, else R(Q_x)^n_x R(Q_y)^n_y for
                                its n_x and n_y reflections (Q = 4 pi
                                sin(grazing angle)/lambda).  Also weights the
                                transmitted beam.  Runs with a guide take
                                the tallies attenuated ones take; the
                                batched launch and the surrogate mode refuse
                                a guide                                     */
} sans_params;

typedef struct sans_model_s* sans_model_t;

/* Validates p, builds the inverse-CDF tables (FP64, staged in LDS by the
 * kernels: the sizes' Schulz or positive-Gaussian quantiles at M knots
 * equally spaced in t = -ln(2 min(u, 1 - u)) with step 32 ln 2 / (M/2 - 1),
 * knot j < M/2 at u = e^(-j dt)/2 and knot M/2 + j at u = 1 - e^(-j dt)/2,
 * so that both tails, which carry the high size moments the weight divides
 * by, are tabulated to the farthest probability a 32-bit uniform reaches;
 * the orientation's standard normal quantiles at u = (k + 1/2)/M)
 * and the model constants.  *out receives an opaque handle owning its device
 * buffers.  Errors: SANS_E_INVALID_ARG (null pointers, wrong abi_version, a
 * size <= 0, a cap radius below the cylinder radius, negative widths or
 * spreads, phi or sq_phi outside [0, 1) / [0, 0.6), nx*ny outside 1..2^26),
 * SANS_E_UNSUPPORTED (unknown kind/mode/orient, QUAD with Gaussian or
 * uniform-angle orientation, a capped body with poly > 0 and poly_mask != 7),
 * SANS_E_NOMEM, SANS_E_HIP. */
int sans_model_create(const sans_params* p, sans_model_t* out);

/* Frees the handle and its device buffers (after synchronising its streams'
 * pending use is the caller's duty).  NULL is accepted. */
int sans_model_destroy(sans_model_t m);

/* Traces neutrons 0 .. n_neutrons-1 of experiment 0 with the given seed and
 * overwrites detector_out (device, FP64 [ny][nx]).  params: NULL to use the
 * handle's parameters, otherwise new parameters that replace them for this and
 * later calls (validated as in sans_model_create; the kind may change).  This
 * is the paper's per-neutron Monte Carlo (Methods; Eq. (3)). */
int sans_trace(sans_model_t m, uint64_t n_neutrons, uint64_t seed, const sans_params* params,
               double* detector_out, void* stream);

/* As sans_trace for neutrons first .. first+n-1 of experiment exp_id.  flags:
 * SANS_ACCUMULATE adds to det (chunked or sharded runs).  SANS_TRANSMITTED
 * also tallies the transmitted (unscattered) beam: each neutron's straight
 * flight from its source point through its slit point (the same random
 * numbers as its scattered flight) meets the detector plane with weight
 * exp(-mu_att chord), the chord being its path inside the slab (1 when it
 * misses the slab): the direct beam that the instrument's sample removes
 * neutrons from (paper: Methods, the KWS-1 instrument and its sample
 * component), tallied by global atomics whatever the tally mode, one per
 * distinct pixel of each 64-neutron wave.  det_w2 (sum of w^2) and
 * det_count (hits, uint64) are optional device outputs (NULL = none) and
 * follow the same overwrite/accumulate rule; with SANS_TRANSMITTED they
 * include the transmitted events. */
int sans_trace_ex(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                  uint32_t flags, double* det, double* det_w2, uint64_t* det_count,
                  void* stream);

/* The same trace as sans_trace_ex without det_w2/det_count, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc,
 * hipFree or allocating library routine.  The handle must have been created
 * beforehand (sans_model_create allocates its tables).  The tally goes
 * through eight per-XCD FP64 replicas of the detector held in a fixed device
 * array inside the library (16 MiB on every GPU the library runs on, kept
 * until the process ends), cleared by each call and summed into det.
 *   det    device FP64 [ny][nx], caller-owned; overwritten, or added to with
 *          SANS_ACCUMULATE (the only flag)
 * Errors: SANS_E_INVALID_ARG for NULL pointers, unknown flags, an overflowing
 * neutron range or a detector of more than 262144 (512 x 512) pixels;
 * SANS_E_UNSUPPORTED in SANS_MODE_SURROGATE (its fallback queue is allocated).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams or threads) race and give wrong detectors; serialise
 * them.  n = 0 only clears det (unless accumulating). */
int sans_trace_noalloc(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed,
                       uint32_t exp_id, uint32_t flags, double* det, void* stream);

/* Per-neutron outputs for neutrons first .. first+n-1, computed by the same
 * device code as the tally kernels: pixel (device int32, -1 = not tallied),
 * w (device float, 0 when not tallied) and q = |Q| (device float, 0 when the
 * sample is missed).  Any output may be NULL. */
int sans_debug_trace(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed,
                     uint32_t exp_id, int32_t* pixel, float* w, float* q, void* stream);

/* Per-neutron transmitted events of neutrons first .. first+n-1 (n at most
 * 2^31), computed by the same device code as the SANS_TRANSMITTED tally:
 * pixel (device int32, -1 off the detector) and w (device double, 0 off the
 * detector). */
int sans_debug_transmitted(sans_model_t m, uint64_t first, uint64_t n, uint64_t seed, uint32_t exp_id,
                           int32_t* pixel, double* w, void* stream);

/* Raw Philox4x32-10 words (Salmon et al., SC'11) of the neutron streams:
 * out (device uint32 [n][n_blocks][4]) receives block b of neutron first+j,
 * counter (lo i, hi i, b, exp_id), key (lo seed, hi seed). */
int sans_debug_philox(uint64_t seed, uint64_t first, uint64_t n, uint32_t n_blocks,
                      uint32_t exp_id, uint32_t* out, void* stream);

/* Copies the handle's FP64 table knots to host memory: which = 0 standard
 * normal, 1 Schulz.  out (host double [n]) with n = table_size.
 * SANS_E_UNSUPPORTED if the handle has no such table. */
int sans_debug_table(sans_model_t m, int32_t which, double* out, int32_t n);

/* Host only (no device work, usable without a GPU): validates p as
 * sans_model_create does and returns the number-averaged particle volume
 * <V> (A^3; 1 for models whose weight is a cross-section or per unit volume
 * fraction; the binary mixture's total volume fraction over its total number
 * density) and the weight's scale per metre of path, 1e10 dOmega phi / <V>
 * (1e2 dOmega for the shape-independent models).  Either output may be NULL. */
int sans_debug_weight_scale(const sans_params* p, double* mean_volume, double* wscale);

/* Traces n_exp independent virtual experiments (the paper's high-throughput
 * use: many models, parameters and neutron counts; Introduction and
 * Conclusion) in one persistent launch.  Experiment e traces neutrons
 * 0 .. n_neutrons[e]-1 with seed seeds[e] and experiment id e -- the same
 * random streams and the same detector as sans_trace_ex(model(p[e]), 0,
 * n_neutrons[e], seeds[e], e, ...) up to FP64 summation order.
 *   p            host sans_params [n_exp]; Monte Carlo mode; all with the same
 *                nx, ny and table_size; nx*ny*8 (+ table_size*8 if any
 *                experiment is polydisperse) must fit in 160 KiB of LDS
 *   n_neutrons   host uint64 [n_exp];  seeds: host uint64 [n_exp]
 *   detectors_out device FP64 [n_exp][ny][nx], overwritten
 *   tune_cache   NULL, or a path to a JSON file of tuned tile sizes: read when
 *                it holds an entry for this batch shape, otherwise the tile
 *                size is tuned by timing the batch on the stream (the output
 *                is rewritten by the final run) and the entry is written.
 * Work is split into tiles (experiment, neutron range) popped from a device
 * queue; the sequence (clear, Schulz tables, queue reset, persistent kernel)
 * is captured once per batch shape as a HIP graph and replayed afterwards.
 * The library keeps the graph and its buffers until sans_batch_release(). */
int sans_trace_batch(int n_exp, const sans_params* p, const uint64_t* n_neutrons,
                     const uint64_t* seeds, double* detectors_out, const char* tune_cache,
                     void* stream);

/* Frees the batch path's cached buffers and graph. */
int sans_batch_release(void);

/* Evaluates, on the device, the weight factor F^2 that replaces the drawn
 * size and orientation in SANS_MODE_QUAD: the Schulz size average and, for
 * isotropic orientation, the orientation average of F^2 by Gauss-Legendre
 * quadrature at q (device float [n]) -> out (device float [n]).  Fixed
 * orientation takes qvec (device float [n][3], may be NULL for isotropic
 * models). */
int sans_pq_avg(sans_model_t m, const float* q, const float* qvec, int64_t n, float* out,
                void* stream);

/* Host-side constants of the handle, for tests: out[0] = <V>, out[1] = the
 * per-metre weight scale 1e10 * dOmega * phi / <V>, out[2] = 1 - cos alpha. */
int sans_model_constants(sans_model_t m, double* out3);

/* ---------------------------------------------------------------------------
 * Learned surrogate of the exact average (the orientation- and size-averaged
 * form factor that SANS_MODE_QUAD computes by quadrature).  Not in the paper:
 * the paper averages by Monte Carlo draws only; this network replaces the
 * quadrature inside the tracer.
 *
 * Network: 8 inputs -> 4 hidden layers of 256 SiLU units -> 1 output.
 * Parameters (199,937), flat, in the order W0[8][256] b0[256] W1[256][256]
 * b1[256] W2 b2 W3 b3 W4[256] b4[1], W_l stored [in][out].  "w_bf16" is that
 * vector in BF16 (device), "w32" in FP32.  All matrix products are BF16 MFMA
 * (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; operands are rounded to
 * BF16 (round to nearest even) when they are loaded, except the 8 inputs of
 * the first layer, which enter as two BF16 parts hi = bf16(x) and
 * lo = bf16(x - hi), both multiplied by W0 (16 bits of input precision), and
 * the last hidden activations, which enter the output layer in FP32.
 * ------------------------------------------------------------------------- */

/* Number of parameters (199,937). */
int64_t sans_mlp_param_count(void);

/* Device workspace (bytes) that forward/backward need for n samples. */
uint64_t sans_mlp_workspace_bytes(int64_t n);

/* y[n] = net(x[n][8]) (device FP32).  The pre-activations and activations
 * of every hidden layer are left in ws for a following sans_mlp_backward on
 * the same x.  n <= 2^24. */
int sans_mlp_forward(const void* w_bf16, const float* x, int64_t n, float* y, void* ws, void* stream);

/* dw (device FP32 [199,937], overwritten) = d(sum_i dy_i y_i)/dw for the
 * samples of the preceding sans_mlp_forward (same w, x, n, ws). */
int sans_mlp_backward(const void* w_bf16, const float* x, const float* dy, int64_t n, float* dw,
                      void* ws, void* stream);

/* One Adam step (Kingma & Ba, 2015) on w32 with gradient dw and moments m, v
 * (all device FP32 [n]); writes the BF16 copy w_bf16.  step >= 1. */
int sans_adam_step(float* w32, void* w_bf16, const float* dw, float* m, float* v, int64_t n,
                   float lr, float beta1, float beta2, float eps, int step, void* stream);

/* Mean squared error of y against t (device FP32 [n]): dy = 2 (y - t)/n and,
 * if loss is not NULL, loss[0] += sum (y - t)^2 / n. */
int sans_mse_grad(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream);

/* y[i] = BF16(x[i]) (round to nearest even), device arrays. */
int sans_f32_to_bf16(const float* x, void* y, int64_t n, void* stream);

/* Text of the last error of the surrogate entry points of this thread. */
const char* sans_mlp_last_error(void);

/* Attaches a trained network to a model in SANS_MODE_SURROGATE (an
 * ellipsoid of revolution, size[0] = size[1], or a parallelepiped, with
 * isotropic orientation).  w_bf16: device BF16 parameters (copied).
 * domain_lo/hi: host float[4], the training box of the physical inputs
 * x = (ln(q size[0]), ln(size[1]/size[0]), ln(size[2]/size[0]), poly); the
 * network sees u_k = (2 x_k - lo_k - hi_k)/(hi_k - lo_k) (0 where lo_k = hi_k).
 * Tracing then weights a neutron by <F^2>(0) P_ref(q) exp(net(u)) in place
 * of the quadrature average <F^2>(q) of SANS_MODE_QUAD, with the reference
 * curve P_ref = (1 + q^2 Rg^2/6)^-2, Rg^2 = (s0^2 + s1^2 + s2^2)/12 for the
 * parallelepiped and /5 for the ellipsoid (it has the Guinier and the q^-4
 * limits; the network learns the rest); neutrons whose q falls
 * outside the box are queued and traced again with the exact quadrature (no
 * divergent branch in the network kernel).  A model whose own shape lies
 * outside the box is traced with the exact quadrature throughout. */
int sans_model_attach_surrogate(sans_model_t m, const void* w_bf16, const float* domain_lo,
                                const float* domain_hi);

/* The exact quadrature as the network's in-domain judge (synchronous).  On
 * the model's own line of inputs (its size ratios and width fixed, ln(q
 * size[0]) over the box) the network's output is compared with the exact
 * average's training target (sans_pq_dataset) at the edges and midpoints of
 * nbins equal bins of ln(q size[0]); every bin where the two differ by more
 * than tol (in ln <F^2>) at any of its three points is flagged, and
 * in-domain neutrons whose ln(q size[0]) (FP64) falls in a flagged bin are
 * queued for the exact pass like out-of-domain ones.  Attaching a network
 * runs this judge with tol = 1e-3 and 2048 bins; calling it again replaces
 * the flags (tol = infinity: no neutron leaves the network).
 *   err    host float [2 nbins + 1] or NULL: |network - exact| at the points
 *   flags  host uint8 [nbins] or NULL: 1 = the bin takes the exact average
 * Errors: SANS_E_INVALID_ARG (nbins outside 1..65536, tol < 0 or NaN),
 * SANS_E_UNSUPPORTED (no network attached).  A model whose own shape lies
 * outside the box takes the exact average throughout and gets no flags. */
int sans_model_judge_surrogate(sans_model_t m, double tol, int32_t nbins, float* err, uint8_t* flags);

/* Training targets: out[i] = ln(<F^2>(q) / <F^2>(0)) - ln P_ref(q) (P_ref as
 * for sans_model_attach_surrogate) of an isotropically
 * oriented particle (kind SANS_ELLIPSOID: of revolution, 1D orientation
 * average; SANS_PARALLELEPIPED: 2D) for physical inputs x[i][8] =
 * (ln(q s0), ln(s1/s0), ln(s2/s0), poly, 0, 0, 0, 0) (device FP32), with
 * quad_n Gauss-Legendre nodes per dimension and the Schulz size average when
 * poly > 0 -- the same quadrature as SANS_MODE_QUAD.  Synchronous. */
int sans_pq_dataset(int32_t kind, const float* x, int64_t n, float* out, int32_t quad_n, void* stream);

/* sizeof(sans_params) as compiled into the library (binding layout check). */
uint32_t sans_abi_params_size(void);

/* Text of a status code, and of the last error of the calling thread. */
const char* sans_status_string(int status);
const char* sans_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SANS_H */
