"""Host pins of the device double-double arithmetic (csrc/dd.h, compiled with g++)
against 256-bit mpmath: each operation's result hi + lo must be within a small
multiple of 2^-104 (relative) of the exact value, on random and adversarial
inputs (cancellation, huge exponent gaps, values next to powers of two)."""
import ctypes as C
import os

import mpmath
import numpy as np
import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1111_3124_amd", "libdd_host.so")
mpmath.mp.prec = 256

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdd_host.so not built")


def lib():
    L = C.CDLL(LIB)
    dp = C.POINTER(C.c_double)
    L.dd_host_op.argtypes = [C.c_int, C.c_long, dp, dp, dp]
    L.dd_host_cdot.argtypes = [C.c_long, dp, dp, dp]
    return L


def normalised_pairs(rng, n, scale_spread=20):
    """Random valid double-double values: hi random, lo within half an ulp of hi."""
    hi = rng.standard_normal(n) * np.exp2(rng.integers(-scale_spread, scale_spread, n))
    lo = hi * rng.uniform(-1, 1, n) * 2.0 ** -53
    s = hi + lo
    lo = (hi - s) + lo  # two_sum-normalise in numpy (exact for these magnitudes)
    return np.stack([s, lo], axis=1).ravel()


def mpv(a, i):
    return mpmath.mpf(float(a[2 * i])) + mpmath.mpf(float(a[2 * i + 1]))


def adversarial(rng):
    a = [1.0, 1.0 + 2 ** -52, 2 ** 60, 3.0, 1e-300 * 2 ** 50, -1.0, 0.5]
    b = [-1.0 + 2 ** -60, -1.0, 2 ** -60, 1.0 / 3.0, 7.0, 1.0 - 2 ** -53, -0.5 - 2 ** -80]
    out_a, out_b = [], []
    for x, y in zip(a, b):
        out_a += [x, 0.0]
        out_b += [y, 0.0]
    return np.array(out_a), np.array(out_b)


@pytest.mark.parametrize("op,name", [(0, "add"), (1, "sub"), (2, "mul"), (3, "div"), (4, "sqrt")])
def test_dd_ops(op, name):
    L = lib()
    rng = np.random.default_rng(op)
    n = 2000
    a = normalised_pairs(rng, n)
    b = normalised_pairs(rng, n)
    if op == 4:
        a = np.abs(a.reshape(-1, 2)) * np.sign(a.reshape(-1, 2)[:, :1])
        a = a.ravel()
    aa, bb = adversarial(rng)
    a = np.concatenate([a, np.abs(aa) if op == 4 else aa])
    b = np.concatenate([b, bb])
    m = a.size // 2
    out = np.zeros_like(a)
    L.dd_host_op(op, m, a.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)),
                 out.ctypes.data_as(C.POINTER(C.c_double)))
    worst = 0.0
    for i in range(m):
        x, y = mpv(a, i), mpv(b, i)
        exact = {0: x + y, 1: x - y, 2: x * y, 3: x / y, 4: mpmath.sqrt(x) if x >= 0 else 0}[op]
        got = mpv(out, i)
        if exact == 0:
            assert got == 0
            continue
        # add/sub: error relative to the operands (cancellation is exact up to lo parts)
        ref = max(abs(x), abs(y)) if op in (0, 1) else abs(exact)
        worst = max(worst, float(abs(got - exact) / ref))
        # hi must be the rounding of hi + lo (normalised pair)
        assert abs(out[2 * i + 1]) <= abs(out[2 * i]) * 2.0 ** -52 + 1e-300
    bound = {0: 4, 1: 4, 2: 8, 3: 16, 4: 16}[op] * 2.0 ** -104
    assert worst <= bound, (name, worst)


def test_error_free_transforms():
    """two_sum and two_prod are exact: hi + lo equals a + b (a * b) exactly."""
    L = lib()
    rng = np.random.default_rng(7)
    n = 1000
    a = np.stack([rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n)), np.zeros(n)], 1).ravel()
    b = np.stack([rng.standard_normal(n) * np.exp2(rng.integers(-40, 40, n)), np.zeros(n)], 1).ravel()
    for op, f in ((5, lambda x, y: x * y), (6, lambda x, y: x + y)):
        out = np.zeros_like(a)
        L.dd_host_op(op, n, a.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)),
                     out.ctypes.data_as(C.POINTER(C.c_double)))
        for i in range(n):
            assert mpv(out, i) == f(mpmath.mpf(float(a[2 * i])), mpmath.mpf(float(b[2 * i])))


def test_complex_dot_accumulation():
    """sum a_i b_i over 512 complex dd terms: error <= 2^-100 of sum |a_i||b_i|."""
    L = lib()
    rng = np.random.default_rng(11)
    n = 512
    a = np.stack([normalised_pairs(rng, n, 3).reshape(-1, 2), normalised_pairs(rng, n, 3).reshape(-1, 2)], 1).ravel()
    b = np.stack([normalised_pairs(rng, n, 3).reshape(-1, 2), normalised_pairs(rng, n, 3).reshape(-1, 2)], 1).ravel()
    out = np.zeros(4)
    L.dd_host_cdot(n, a.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double)),
                   out.ctypes.data_as(C.POINTER(C.c_double)))
    s = mpmath.mpc(0)
    mag = mpmath.mpf(0)
    for i in range(n):
        x = mpmath.mpc(mpmath.mpf(a[4 * i]) + mpmath.mpf(a[4 * i + 1]), mpmath.mpf(a[4 * i + 2]) + mpmath.mpf(a[4 * i + 3]))
        y = mpmath.mpc(mpmath.mpf(b[4 * i]) + mpmath.mpf(b[4 * i + 1]), mpmath.mpf(b[4 * i + 2]) + mpmath.mpf(b[4 * i + 3]))
        s += x * y
        mag += abs(x) * abs(y)
    got = mpmath.mpc(mpmath.mpf(out[0]) + mpmath.mpf(out[1]), mpmath.mpf(out[2]) + mpmath.mpf(out[3]))
    assert abs(got - s) <= mag * 2.0 ** -100
