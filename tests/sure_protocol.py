"""How a device threshold is judged against the oracle's SURE curve.

The device's threshold is one of its own coefficient magnitudes, which differ
from the oracle's by the rounding of the device computation (relative eps:
about 1e-12 for FP64 cubes, 1e-6 for FP32, 1e-4 for mixed).  Near the minimum
the SURE curve is flat up to steps of 2 (one coefficient changing sides), so
those rounding differences can move the argmin to another near-optimal
candidate.  A device threshold is accepted when the oracle's SURE, taken at
the best point within the rounding window around it, exceeds the oracle's
minimum by no more than what the rounding explains: the change of
sum min(b^2, t^2) under relative perturbations eps (2 eps sum_{|b| <= t} b^2,
twice for the two curves), 2 per coefficient inside the window, and 2 for the
candidate itself.
"""
import numpy as np

from oracle import hyres_oracle as O

EPS = {"float64": 1e-12, "float32": 1e-6, "mixed": 1e-4}


def window_sure(b, t, eps):
    a = np.abs(np.asarray(b, dtype=np.float64))
    lo, hi = t * (1 - 4 * eps), t * (1 + 4 * eps)
    cands = np.concatenate([[t, lo, hi], a[(a >= lo) & (a <= hi)]])
    return min(O.sure_at(b, float(c)) for c in cands)


def slack(b, t, eps):
    a = np.abs(np.asarray(b, dtype=np.float64))
    t_hi = t * (1 + 4 * eps)
    inside = np.count_nonzero((a >= t * (1 - 4 * eps)) & (a <= t_hi))
    return 2.0 + 4.0 * eps * float(np.sum(a[a <= t_hi] ** 2)) + 2.0 * inside


def accept(b, t_dev, t_ref, s_ref, eps):
    """(ok, gap, allowed) for a device threshold t_dev against the oracle's (t_ref, s_ref)."""
    gap = window_sure(b, t_dev, eps) - s_ref
    allowed = slack(b, t_dev, eps)
    return gap <= allowed, gap, allowed
