"""The parity bars shared by the GPU tests (HIP path against the FP64 oracle
on the same seeded inputs and Philox streams):

  - per-neutron weight: |dw| <= 1e-5 * w_max + 1e-4 * |w| (w_max the largest
    |w| of the oracle over the compared neutrons);
  - total detected intensity: 1e-6 relative;
  - every hit pixel: 1e-4 relative, where pixels hold many neutrons; where
    they hold few (a pixel can be one neutron near a zero of the amplitude,
    which only the per-neutron bar governs), the per-neutron bar summed over
    the pixel's neutrons, 1e-4 |pixel| + 1e-5 w_max count;
  - the set of hit pixels: identical.
"""
import os

import numpy as np

import oracle

NTHREADS = max(1, min(16, os.cpu_count() or 1))


def check_weights(w_gpu, w_orc, where=""):
    w_gpu = np.asarray(w_gpu, dtype=np.float64)
    wmax = np.max(np.abs(w_orc)) if w_orc.size else 0.0
    tol = 1e-5 * wmax + 1e-4 * np.abs(w_orc)
    bad = np.abs(w_gpu - w_orc) > tol
    assert not bad.any(), (f"{where}: {bad.sum()} weights out of tolerance; worst "
                           f"{np.max(np.abs(w_gpu - w_orc) / np.maximum(tol, 1e-300)):.3g} x tol")


def check_detector(d_gpu, d_orc, where="", count=None, w_max=None):
    """Same hit pixels, total within 1e-6 and every hit pixel within 1e-4
    relative.  With count (the oracle's hits per pixel) and w_max (the
    largest single weight), a pixel may instead deviate by the sum of the
    per-neutron bar over its neutrons, 1e-4 |pixel| + 1e-5 w_max count: the
    bar for models whose amplitude has zeros inside the Q range (the capped
    bodies, the thin-walled prism), where a sparse pixel can be one neutron
    near a zero of F."""
    d_gpu = np.asarray(d_gpu)
    assert d_gpu.shape == d_orc.shape
    # same set of hit pixels
    assert np.array_equal(d_gpu != 0, d_orc != 0), f"{where}: hit patterns differ"
    tot_g, tot_o = d_gpu.sum(), d_orc.sum()
    assert abs(tot_g - tot_o) <= 1e-6 * abs(tot_o), f"{where}: total {tot_g} vs {tot_o}"
    nz = d_orc != 0
    err = np.abs(d_gpu[nz] - d_orc[nz])
    if count is None:
        rel = err / np.abs(d_orc[nz])
        assert rel.max() <= 1e-4 if rel.size else True, f"{where}: worst pixel rel {rel.max():.3g}"
    else:
        tol = 1e-4 * np.abs(d_orc[nz]) + 1e-5 * w_max * count[nz].astype(np.float64)
        assert (err <= tol).all(), f"{where}: worst pixel {np.max(err / tol):.3g} x the summed bar"


# models judged pixel by pixel with the summed per-neutron bar at any count
SUMMED_BAR = ("barbell", "capped_cylinder", "hollow_prism", "superball", "pringle")


def oracle_detector(p, n, seed, first=0):
    """The oracle's detector, plus (count, w_max) for the summed bar where the
    model needs it (w_max over the first 100003 of these neutrons)."""
    if p["kind"] not in SUMMED_BAR:
        return oracle.trace(p, n, seed, first=first, nthreads=NTHREADS), {}
    ref, _, cnt = oracle.trace(p, n, seed, first=first, nthreads=NTHREADS, with_count=True)
    _, w, _ = oracle.trace_debug(p, min(n, 100003), seed, first=first)
    return ref, dict(count=cnt, w_max=float(np.max(np.abs(w))))




def oracle_detector_sparse(p, n, seed, exp_id=0, per_pixel=100.0, first=0):
    """The oracle's detector and the bar for it: the summed per-neutron bar
    when the hit pixels hold fewer than per_pixel neutrons on average (or the
    model needs it at any count), else the plain 1e-4 pixel bar."""
    ref, _, cnt = oracle.trace(p, n, seed, first=first, exp_id=exp_id, nthreads=NTHREADS, with_count=True)
    nz = ref != 0
    if p["kind"] not in SUMMED_BAR and (not nz.any() or cnt[nz].mean() >= per_pixel):
        return ref, {}
    _, w, _ = oracle.trace_debug(p, min(n, 100003), seed, first=first, exp_id=exp_id)
    return ref, dict(count=cnt, w_max=float(np.max(np.abs(w))) if w.size else 0.0)
