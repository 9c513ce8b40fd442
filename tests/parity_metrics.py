"""Error measures of a device result against the FP64 oracle.

Two numbers are reported and bounded for every compared cube: the relative
Frobenius error ||X - X_ref||_F / ||X_ref||_F, and the largest element error
relative to the largest oracle magnitude, max |X - X_ref| / max |X_ref|.  The
second catches a single wrong band, tile seam or tail block that the norm of
a large cube would hide.  Both use the same tolerance: 1e-10 for FP64 cubes,
1e-5 for FP32 and 1e-3 for the mixed-precision path.
"""
import numpy as np

TOL = {"float64": 1e-10, "float32": 1e-5, "mixed": 1e-3}


def errors(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    fro = float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))
    mx = float(np.abs(d).max() / max(np.abs(ref).max(), 1e-300)) if d.size else 0.0
    return fro, mx


def assert_close(got, ref, tol, what=""):
    fro, mx = errors(got, ref)
    assert fro <= tol, ("relative Frobenius error", what, fro, tol)
    assert mx <= tol, ("max element error / max |ref|", what, mx, tol)
    return fro, mx
