"""Shared helpers of the test suite (comparison rules; no method arithmetic)."""
import numpy as np


def widen(a):
    """float32/float64 array -> float64 (exact)."""
    return np.asarray(a, dtype=np.float64)


def force_err(acc, acc_ref, amag, kappa_max=1e3):
    """Per-particle relative force error with a cancellation floor.

    err_i = |a_i - a_ref_i| / max(|a_ref_i|, A_i / kappa_max), A_i = sum_j |f_ij|
    the sum of the magnitudes of particle i's terms.  It is the plain relative
    error whenever the cancellation ratio A_i/|a_i| is at most kappa_max.  A
    particle with no terms at all (A_i = 0, e.g. alone in its cluster) must
    match exactly: its error is the absolute difference.
    """
    acc = widen(acc)
    acc_ref = widen(acc_ref)
    den = np.maximum(np.linalg.norm(acc_ref, axis=1), widen(amag) / kappa_max)
    den = np.where(den > 0, den, 1.0)
    return np.linalg.norm(acc - acc_ref, axis=1) / den


def floor_share(acc_ref, amag, kappa_max=1e3):
    """Share of particles whose error denominator is the cancellation floor A_i / kappa_max
    rather than |a_ref_i| (their force cancels by more than kappa_max)."""
    a = np.linalg.norm(widen(acc_ref), axis=1)
    if len(a) == 0:
        return 0.0
    return float(np.mean(widen(amag) / kappa_max > a))


def check_forces(acc, acc_ref, amag, tol, label="", max_floor_share=1e-3, log=print):
    """Assert the per-particle force errors (force_err) are within tol, reporting the worst error,
    the 99th percentile and the share of particles where the cancellation floor sets the
    denominator; that share must stay at most max_floor_share, so that the floor cannot hide a
    loose comparison.  Returns the errors."""
    e = force_err(acc, acc_ref, amag)
    share = floor_share(acc_ref, amag)
    kap = widen(amag) / np.maximum(np.linalg.norm(widen(acc_ref), axis=1), 1e-300)
    if len(e):
        log(f"  {label} max err {e.max():.3e}  p99 {np.quantile(e, 0.99):.3e}  floor share {share:.2e}  "
            f"max A/|a| {kap.max():.1f}")
        assert e.max() <= tol, f"{label}: max force error {e.max():.3e} > {tol:g}"
    assert share <= max_floor_share, f"{label}: cancellation floor used for {share:.2e} of the particles"
    return e


def walk_slots(pos64, mass64):
    """Position of every target (caller index) in the walk's default target order (the Hilbert
    order, from the oracle's own construction): target i belongs to walk group slots[i] // 64."""
    from oracle import hilbert
    order = hilbert.walk_order(pos64, mass64)
    slots = np.empty(len(order), np.int64)
    slots[order] = np.arange(len(order))
    return slots


def pot_err(pot, pot_ref):
    """Relative potential error (absolute where the reference is exactly 0)."""
    pot = widen(pot)
    pot_ref = widen(pot_ref)
    den = np.abs(pot_ref)
    return np.abs(pot - pot_ref) / np.where(den > 0, den, 1.0)


def tree_cases():
    """Small particle sets that exercise the tree build's corner cases."""
    rng = np.random.default_rng(5)
    cases = {}
    # (8192 and 12289: whole sort tiles of 4096 keys, and several tiles with a ragged tail)
    for n in (1, 2, 3, 5, 8, 13, 16, 100, 1000, 8192, 12289):
        cases[f"random{n}"] = rng.random((n, 3))
    p = rng.random((12, 3))
    p[5] = p[2]; p[9] = p[2]; p[7] = p[1]
    cases["duplicates"] = p
    cases["coincident"] = np.tile(rng.random((1, 3)), (6, 1))
    p = rng.random((10, 3))
    p[3] = p[4] + 1e-9
    cases["finest_cell_pair"] = p
    p = np.zeros((9, 3)); p[:, 0] = np.arange(9) * 2.0 ** -18
    cases["collinear_deep"] = p
    p = rng.random((777, 3)) * np.array([1.0, 1e-3, 1e-6])     # flat, anisotropic
    cases["flat"] = p
    return cases
