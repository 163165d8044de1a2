"""ctypes wrapper of ``libmps_oracle.so`` (test infrastructure only).

Values cross the boundary as double-double pairs (hi, lo): the oracle computes at
``prec`` bits (256 by default) and rounds every output to hi + lo.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libmps_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        from . import build as _b
        _b.build()
    L = C.CDLL(lib_path)
    dp = C.POINTER(C.c_double)
    L.omps_create.restype = C.c_void_p
    L.omps_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int]
    L.omps_destroy.argtypes = [C.c_void_p]
    L.omps_set_max_sweeps.argtypes = [C.c_int]
    L.omps_set_trunc.argtypes = [C.c_void_p, C.c_int, C.c_double]
    L.omps_apply.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, dp]
    L.omps_bond_dim.argtypes = [C.c_void_p, C.c_int]
    L.omps_schmidt.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_int]
    L.omps_amplitude.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte), dp]
    L.omps_last_stats.argtypes = [C.c_void_p, dp]
    L.omps_load.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(dp), C.POINTER(dp),
                            C.POINTER(dp), C.POINTER(dp)]
    L.osvd.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, dp, dp, dp, dp, dp, dp]
    L.osv_create.restype = C.c_void_p
    L.osv_create.argtypes = [C.c_int, C.c_int]
    L.osv_destroy.argtypes = [C.c_void_p]
    L.osv_apply.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), dp, dp]
    L.osv_amplitudes.argtypes = [C.c_void_p, dp]
    L.omps_rdo.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), dp]
    L.oracle_threads.restype = C.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _cplx_pair(u_hi, u_lo):
    hi = np.ascontiguousarray(np.asarray(u_hi, dtype=np.complex128)).view(np.float64).copy()
    lo = None
    if u_lo is not None:
        lo = np.ascontiguousarray(np.asarray(u_lo, dtype=np.complex128)).view(np.float64).copy()
    return hi, lo


def oracle_threads() -> int:
    return int(_load().oracle_threads())


def set_max_sweeps(s: int) -> None:
    _load().omps_set_max_sweeps(int(s))


class OracleMPS:
    """MPS in Gamma-lambda form (the paper's Eq. (1)), initial state |0...0>."""

    def __init__(self, n: int, chi_max: int, eps: float = 0.0, prec: int = 256):
        L = _load()
        self.n, self.chi_max, self.eps, self.prec = n, chi_max, eps, prec
        self._h = L.omps_create(n, chi_max, float(eps), prec)
        if not self._h:
            raise ValueError("omps_create rejected its arguments")

    def close(self):
        if self._h:
            _load().omps_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_trunc(self, chi_max: int, eps: float) -> None:
        if _load().omps_set_trunc(self._h, int(chi_max), float(eps)) != 0:
            raise ValueError("bad truncation parameters")
        self.chi_max, self.eps = chi_max, eps

    def apply(self, first: int, k: int, u_hi, u_lo=None) -> None:
        hi, lo = _cplx_pair(u_hi, u_lo)
        assert hi.size == 2 * 4 ** k
        rc = _load().omps_apply(self._h, first, k, _dp(hi), _dp(lo))
        if rc == -5:
            raise RuntimeError("oracle Jacobi iteration did not converge")
        if rc != 0:
            raise ValueError(f"omps_apply failed ({rc})")

    def apply_gate(self, g) -> None:
        self.apply(g.first, g.k, g.u_hi, g.u_lo)

    def apply_gate2(self, q0: int, q1: int, u_hi, u_lo=None) -> None:
        """Two-qubit gate on qubits q0 != q1, U's first index bit on q0 (the paper's
        applyU(U, q0, q1), Section 3.2).  Adjacent: one U(4) on min(q0, q1) (for
        q0 > q1 the gate with its two qubits exchanged, S U S with S = SWAP).
        Otherwise, a = min, b = max: SWAPs on sites (b-1, b) down to (a+2, a+3) bring
        qubit b next but one to a, the U(8) (U on the window's outer sites) (x) the
        identity on the middle one acts on a..a+2, and SWAPs on (a+2, a+3) up to
        (b-1, b) take it back (the routing the paper leaves open, read as the one
        that needs the fewest swaps with three-qubit gates elementary)."""
        if q0 == q1 or not (0 <= q0 < self.n and 0 <= q1 < self.n):
            raise ValueError("qubits must be distinct and in range")
        S = np.zeros((4, 4), dtype=np.complex128)
        S[0, 0] = S[1, 2] = S[2, 1] = S[3, 3] = 1.0
        mats = [np.asarray(u_hi, dtype=np.complex128)]
        if u_lo is not None:
            mats.append(np.asarray(u_lo, dtype=np.complex128))
        a, b = min(q0, q1), max(q0, q1)
        if b == a + 1:
            g = [m if q0 < q1 else S @ m @ S for m in mats]  # permutations: exact
            self.apply(a, 2, g[0], g[1] if len(g) > 1 else None)
            return
        # U(8) index (x_a, x_mid, x_b): U acts on (x_q0, x_q1), the identity on x_mid
        eye = np.eye(2)
        g8 = []
        for m in mats:
            t = m.reshape(2, 2, 2, 2)  # [out q0, out q1, in q0, in q1]
            if q0 > q1:
                t = t.transpose(1, 0, 3, 2)  # -> [out a, out b, in a, in b]
            g8.append(np.einsum("ikIK,jJ->ijkIJK", t, eye).reshape(8, 8))
        for p in range(b - 1, a + 1, -1):
            self.apply(p, 2, S)
        self.apply(a, 3, g8[0], g8[1] if len(g8) > 1 else None)
        for p in range(a + 2, b):
            self.apply(p, 2, S)

    def bond_dim(self, bond: int) -> int:
        return int(_load().omps_bond_dim(self._h, bond))

    def bond_dims(self) -> list[int]:
        return [self.bond_dim(b) for b in range(self.n - 1)]

    def schmidt(self, bond: int):
        m = self.bond_dim(bond)
        hi = np.zeros(m)
        lo = np.zeros(m)
        _load().omps_schmidt(self._h, bond, _dp(hi), _dp(lo), m)
        return hi, lo

    def amplitude(self, bits):
        b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint8))
        assert b.size == self.n
        out = np.zeros(4)
        _load().omps_amplitude(self._h, b.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(out))
        return (complex(out[0], out[2]), complex(out[1], out[3]))

    def amplitudes(self, bits_2d):
        hi = np.zeros(len(bits_2d), dtype=np.complex128)
        lo = np.zeros(len(bits_2d), dtype=np.complex128)
        for i, b in enumerate(bits_2d):
            hi[i], lo[i] = self.amplitude(b)
        return hi, lo

    def rdo(self, qubits):
        """Reduced density operator of `qubits` (in the order given: the first is the
        most significant bit of the basis index), as (hi, lo) complex 2^L x 2^L arrays."""
        L = len(qubits)
        q = (C.c_int * L)(*[int(x) for x in qubits])
        out = np.zeros(4 << (2 * L))
        if _load().omps_rdo(self._h, L, q, _dp(out)) != 0:
            raise ValueError("bad qubit list")
        o = out.reshape(1 << L, 1 << L, 4)
        return o[..., 0] + 1j * o[..., 2], o[..., 1] + 1j * o[..., 3]

    def last_stats(self) -> list[dict]:
        out = np.zeros(18)
        ns = _load().omps_last_stats(self._h, _dp(out))
        keys = ["W", "W_lo", "w", "w_lo", "k", "sweeps", "gap", "epsdist", "rank"]
        return [dict(zip(keys, out[9 * i: 9 * i + 9].tolist())) for i in range(ns)]

    def load(self, B, lam, B_lo=None, lam_lo=None) -> None:
        """Replace the state by (B_s, lambda_s) with B_s = Gamma_s lambda_s."""
        n = self.n
        assert len(B) == n and len(lam) == n - 1
        dims = (C.c_int * max(1, n - 1))(*[len(l) for l in lam])
        keep = []

        def ptrs(arrs, cplx):
            if arrs is None:
                return None
            P = (C.POINTER(C.c_double) * len(arrs))()
            for i, a in enumerate(arrs):
                x = np.ascontiguousarray(np.asarray(a, dtype=np.complex128 if cplx else np.float64))
                x = x.view(np.float64).copy() if cplx else x.copy()
                keep.append(x)
                P[i] = _dp(x)
            return P

        bh = ptrs(B, True)
        bl = ptrs(B_lo, True)
        lh = ptrs(lam, False) if n > 1 else (C.POINTER(C.c_double) * 1)()
        ll = ptrs(lam_lo, False) if lam_lo is not None else None
        rc = _load().omps_load(self._h, dims, bh, bl, lh, ll)
        if rc != 0:
            raise ValueError("omps_load failed")


class OracleSV:
    """Dense state vector, qubit 0 = most significant bit of the basis index."""

    def __init__(self, n: int, prec: int = 256):
        self.n = n
        self._h = _load().osv_create(n, prec)
        if not self._h:
            raise ValueError("osv_create rejected its arguments")

    def close(self):
        if self._h:
            _load().osv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, qubits, u_hi, u_lo=None) -> None:
        hi, lo = _cplx_pair(u_hi, u_lo)
        q = (C.c_int * len(qubits))(*qubits)
        rc = _load().osv_apply(self._h, len(qubits), q, _dp(hi), _dp(lo))
        if rc != 0:
            raise ValueError("osv_apply failed")

    def apply_gate(self, g) -> None:
        self.apply(list(range(g.first, g.first + g.k)), g.u_hi, g.u_lo)

    def amplitudes(self):
        out = np.zeros(4 << self.n)
        _load().osv_amplitudes(self._h, _dp(out))
        out = out.reshape(-1, 4)
        return out[:, 0] + 1j * out[:, 2], out[:, 1] + 1j * out[:, 3]


def osvd(a_hi, a_lo=None, prec: int = 256):
    """Jacobi SVD of a complex matrix (given as a 2-D complex array).  Returns
    dict with sigma, V, W = A V as (hi, lo) pairs, columns sorted by sigma."""
    a_hi = np.asarray(a_hi, dtype=np.complex128)
    M, N = a_hi.shape
    ah = np.asfortranarray(a_hi).ravel(order="F").view(np.float64).copy()
    al = None
    if a_lo is not None:
        al = np.asfortranarray(np.asarray(a_lo, dtype=np.complex128)).ravel(order="F").view(np.float64).copy()
    sh, sl = np.zeros(N), np.zeros(N)
    vh, vl = np.zeros(2 * N * N), np.zeros(2 * N * N)
    wh, wl = np.zeros(2 * M * N), np.zeros(2 * M * N)
    rc = _load().osvd(M, N, _dp(ah), _dp(al), prec, _dp(sh), _dp(sl), _dp(vh), _dp(vl), _dp(wh), _dp(wl))
    if rc < 0:
        raise RuntimeError(f"osvd failed ({rc})")

    def cm(x, r, c):
        return x.view(np.complex128).reshape(c, r).T.copy()

    return dict(sweeps=rc, sigma=(sh, sl), V=(cm(vh, N, N), cm(vl, N, N)), W=(cm(wh, M, N), cm(wl, M, N)))
