"""Error gates shared by the GPU parity tests (readings of "relative error" where the reference
vanishes at band edges and gaps)."""
import numpy as np


def dos_err(got, ref):
    """max |D - D_ref| / max |D_ref| (the DOS gate)."""
    scale = np.abs(ref).max()
    return np.abs(got - ref).max() / scale if scale > 0 else np.abs(got).max()


def gate(got, ref, rel=1e-3, floor=1e-6):
    """Per-element gradient gate: |g - g_ref| <= rel |g_ref| where |g_ref| >= 1e-3 max|g_ref|, else
    <= floor max|g_ref|. Returns (passed, worst relative error on the large entries, normwise error)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    assert scale > 0, "the reference gradient is identically zero: the case pins nothing"
    big = np.abs(ref) >= 1e-3 * scale
    err = np.abs(got - ref)
    ok = np.where(big, err <= rel * np.abs(ref), err <= floor * scale)
    worst_big = float((err[big] / np.abs(ref[big])).max()) if big.any() else 0.0
    return bool(ok.all()), worst_big, float(err.max() / scale)
