"""Error measures used to compare reconstructions (FP64)."""
from __future__ import annotations

import numpy as np

from . import fd as _fd


def rel_l1(p, ref):
    """sum |p - ref| / sum |ref|."""
    p = np.asarray(p, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sum(np.abs(p - ref)) / np.sum(np.abs(ref)))


def rel_l2(g, ref):
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((g - ref) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(g * g)))


def chi2(a, b):
    """Eq. 16: sum_i (a_i - b_i)^2 / (a_i + b_i), over terms with a_i + b_i > 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = a + b
    live = s > 0
    return float(np.sum((a[live] - b[live]) ** 2 / s[live]))


def kappa(entries, cut, p_abs_sum):
    """Cancellation factor: (2^-K sum_l prod_c sum_{x_c} |E_c[row_c(l), x_c]|) / sum_x |p_x|.

    The numerator bounds sum_x sum_l |term(l, x)|; kappa times the unit
    roundoff bounds the relative L1 error of any summation order of the terms.
    """
    K = cut.n_cuts
    absrow = [np.sum(np.abs(np.asarray(E, dtype=np.float64)), axis=1) for E in entries]
    tot = 0.0
    for l in range(4 ** K):
        d = _fd.label_digits(l, K)
        t = 1.0
        for c in range(cut.n_sub):
            t *= absrow[c][_fd.row_of(cut, c, d)]
        tot += t
    return tot * (2.0 ** -K) / p_abs_sum
