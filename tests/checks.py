"""Amplitude comparison of the GPU parity tests (both bounds are asserted).

For amplitudes ``a`` against FP64 reference values ``ref`` and a tolerance
``tol`` (1e-5 for the FP32 path, 1e-4 for the split-BF16 assembly):

* norm-wise:    ||a - ref||_2 <= tol * ||ref||_2;
* element-wise: max_i |a_i - ref_i| <= K_MAX * tol * rms(ref).

Why K_MAX = 8.  Every amplitude is a sum over copies of products of half
amplitudes, each carrying FP32 rounding from the gate passes and the
contraction; the error of one amplitude is a sum of many small independent
terms of random sign, so it is close to a complex Gaussian, and its spread
depends on sum_k |U_k[u] L_k[l]|^2, not on |a| itself, so it is about the same
for every amplitude.  The norm-wise bound caps that spread at tol * rms(ref).
The largest of m such errors is about sqrt(ln m) standard deviations:
sqrt(ln 2^28) = 4.4 for the largest sets here.  K_MAX = 8 leaves a factor of
about two over that.  An error confined to a few amplitudes (one wrong copy
column, one wrong index bit) passes a norm-wise bound of 1e-5 over 2^20 values
at up to 1e-2 of rms(ref); the element-wise bound catches it above 8e-5.
"""

from __future__ import annotations

import numpy as np

K_MAX = 8.0


def errors(a, ref) -> dict:
    """norm: ||a - ref|| / ||ref||; max_abs: max |a - ref|; max_over_rms:
    max |a - ref| / rms(ref); median_rel: median of |a_i - ref_i| / |ref_i|
    over the nonzero ref_i (reported only: ill-conditioned near the zeros of
    a Porter-Thomas distribution)."""
    a = np.asarray(a).astype(np.complex128).ravel()
    ref = np.asarray(ref).astype(np.complex128).ravel()
    d = np.abs(a - ref)
    nref = float(np.linalg.norm(ref))
    rms = nref / np.sqrt(max(1, ref.size))
    nz = np.abs(ref) > 0
    return {
        "norm": float(np.linalg.norm(a - ref) / nref) if nref > 0 else float(np.linalg.norm(a - ref)),
        "max_abs": float(d.max()) if d.size else 0.0,
        "max_over_rms": float(d.max() / rms) if (d.size and rms > 0) else 0.0,
        "median_rel": float(np.median(d[nz] / np.abs(ref[nz]))) if nz.any() else 0.0,
    }


def assert_close(a, ref, tol: float, what: str = "") -> dict:
    """Both bounds of the module docstring; returns the errors."""
    e = errors(a, ref)
    tag = f"{what}: " if what else ""
    assert e["norm"] < tol, f"{tag}norm-wise error {e['norm']:.3e} >= {tol:.1e} ({e})"
    assert e["max_over_rms"] <= K_MAX * tol, (
        f"{tag}max |a - ref| / rms(ref) = {e['max_over_rms']:.3e} > {K_MAX * tol:.1e} ({e})")
    return e
