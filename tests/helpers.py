"""Shared test helpers: tolerance checks and problem upload (no method arithmetic)."""
from __future__ import annotations

import numpy as np

# Floating-point bar: |x - x*| <= REL * M elementwise, with M the oracle's sum
# of |terms| (the a-priori error bound of a sum scales with it).  FP32 sums
# of depth d satisfy |x - x*| <= gamma_d * M with gamma_d = d u / (1 - d u),
# u = 2^-24; every kernel here keeps d <= ~100, so gamma_d <= 6e-6 < 1e-5.
REL = 1e-5


def assert_within_mag(got, ref, mag, rel=REL, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    err = np.abs(got - ref)
    bound = rel * mag + 1e-37
    bad = err > bound
    if bad.any():
        i = np.flatnonzero(bad.ravel())[0]
        raise AssertionError(
            f"{what}: {bad.sum()} of {bad.size} elements exceed {rel}*M; first at {i}: "
            f"got {got.ravel()[i]!r} ref {ref.ravel()[i]!r} M {mag.ravel()[i]!r}")
    return float((err / np.maximum(mag, 1e-300)).max()) if err.size else 0.0


def error_report(got, ref, mag):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    err = np.abs(got - ref)
    big = np.abs(ref) > 1e-3 * np.abs(ref).max() if ref.size else np.zeros(0, bool)
    rel = err[big] / np.abs(ref[big]) if big.any() else np.zeros(1)
    return dict(max_err_over_M=float((err / np.maximum(mag, 1e-300)).max()) if err.size else 0.0,
                mean_err_over_M=float((err / np.maximum(mag, 1e-300)).mean()) if err.size else 0.0,
                normwise=float(np.linalg.norm(err) / max(np.linalg.norm(ref), 1e-300)),
                max_rel=float(rel.max()), mean_rel=float(rel.mean()))
