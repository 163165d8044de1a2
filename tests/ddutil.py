"""Test helpers for comparing double-double pairs at high precision (mpmath).

Used only by the tests; independent of both the oracle and the device library."""
import mpmath
import numpy as np

mpmath.mp.prec = 256


def mpc(hi, lo=0j):
    hi = complex(hi)
    lo = complex(lo)
    return mpmath.mpc(hi.real, hi.imag) + mpmath.mpc(lo.real, lo.imag)


def mpr(hi, lo=0.0):
    return mpmath.mpf(float(hi)) + mpmath.mpf(float(lo))


def dd_abs_diff(a_hi, a_lo, b_hi, b_lo):
    """max |(a_hi + a_lo) - (b_hi + b_lo)| elementwise, evaluated at 256 bits."""
    a_hi = np.atleast_1d(a_hi); a_lo = np.atleast_1d(a_lo)
    b_hi = np.atleast_1d(b_hi); b_lo = np.atleast_1d(b_lo)
    m = mpmath.mpf(0)
    for i in range(a_hi.size):
        d = abs(mpc(a_hi.flat[i], a_lo.flat[i]) - mpc(b_hi.flat[i], b_lo.flat[i]))
        if d > m:
            m = d
    return float(m)


def dd_to_mpmatrix(hi, lo):
    r, c = hi.shape
    return mpmath.matrix([[mpc(hi[i, j], lo[i, j]) for j in range(c)] for i in range(r)])
