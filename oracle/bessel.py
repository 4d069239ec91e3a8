"""Integer-order Bessel J_m and Hankel H_m^(1) values (paper sec. 4.2: the diagonal
matrices J, J', H, H' at k a_p and the separation symbols H_{m-n}(k b_pq)).

Oracle module (test infrastructure only).  Values come from SciPy (AMOS) at
non-negative orders; negative orders use the exact reflection
J_{-n} = (-1)^n J_n, H_{-n} = (-1)^n H_n so that identities of the truncated
system hold to rounding.  Derivatives use J'_n = (J_{n-1} - J_{n+1}) / 2 and
the same for H.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _reflect(fun, m, x):
    m = np.asarray(m, dtype=np.int64)
    x = np.asarray(x, dtype=np.float64)
    am = np.abs(m)
    v = fun(am.astype(np.float64), x)
    sign = np.where((m < 0) & (am % 2 == 1), -1.0, 1.0)
    return sign * v


def besselj(m, x):
    """J_m(x), integer m of any sign, real x (float64)."""
    return _reflect(special.jv, m, x)


def hankel1(m, x):
    """H_m^(1)(x) = J_m(x) + i Y_m(x), integer m of any sign, real x > 0."""
    return _reflect(special.hankel1, m, x)


def besselj_d(m, x):
    """J'_m(x) = (J_{m-1}(x) - J_{m+1}(x)) / 2."""
    m = np.asarray(m, dtype=np.int64)
    return 0.5 * (besselj(m - 1, x) - besselj(m + 1, x))


def hankel1_d(m, x):
    """H'_m(x) = (H_{m-1}(x) - H_{m+1}(x)) / 2."""
    m = np.asarray(m, dtype=np.int64)
    return 0.5 * (hankel1(m - 1, x) - hankel1(m + 1, x))
