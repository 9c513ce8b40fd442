"""Error measures of a device result against the FP64 oracle.

Two numbers are reported and bounded for every compared cube:

* the relative Frobenius error ||X - X_ref||_F / ||X_ref||_F, bounded by the
  precision's tolerance: 1e-10 for FP64 cubes, 1e-5 for FP32, 1e-3 for the
  mixed-precision path;
* the largest element error relative to the largest oracle magnitude,
  max |X - X_ref| / max |X_ref|, bounded by ten times that tolerance.

Why the element bound is looser than the norm bound.  Rounding in the Gram
perturbs C by about eps ||C||; an eigenvector inside the noise bulk (the
components beyond the signal rank, whose eigenvalues differ by a few parts in
a thousand) turns by about eps ||C|| / gap, far more than the others.  Those
components are soft-thresholded near the universal threshold, so the few
coefficients that survive, and with them the error of the turned vector, sit on
a few pixels: the peak of the error is 10-30 times its root mean square while
the peak of X is about twice its root mean square.  An FP32 solve of rank 12
on a 100-band cube measured 1.4e-6 by the norm and 3.7e-5 by the element
measure.  The element bound still catches what the norm of a large cube hides:
a wrong or missing band, a tile seam with a slipped blend weight, a wrong tail
block, all of which are errors of 1e-3 of max |X| or more.
"""
import numpy as np

TOL = {"float64": 1e-10, "float32": 1e-5, "mixed": 1e-3}
ELEMENT_FACTOR = 10.0


def errors(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    fro = float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))
    mx = float(np.abs(d).max() / max(np.abs(ref).max(), 1e-300)) if d.size else 0.0
    return fro, mx


def assert_close(got, ref, tol, what=""):
    """tol bounds the relative Frobenius error; ELEMENT_FACTOR * tol the element error."""
    fro, mx = errors(got, ref)
    assert fro <= tol, ("relative Frobenius error", what, fro, tol)
    assert mx <= ELEMENT_FACTOR * tol, ("max element error / max |ref|", what, mx, ELEMENT_FACTOR * tol)
    return fro, mx
