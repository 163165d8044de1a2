"""Thin ctypes binding of the C ABI in include/mps.h (argument marshalling only).

Every function here has the name of the C entry point it wraps; ``MPS`` is a small
convenience class over them.  All arithmetic happens in the HIP kernels of
``libmps_hip.so``; importing this module raises if that library is missing, and
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmps_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"device library {LIB_PATH} is not built: run `python -m paper_1111_3124_amd.build`")

_lib = C.CDLL(LIB_PATH)

MPS_OK, MPS_EINVAL, MPS_ERANGE, MPS_ENOMEM, MPS_EDEVICE, MPS_ENOCONV, MPS_ENONFINITE, MPS_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
MPS_PREC_FP64, MPS_PREC_DD = 0, 1
MPS_OPT_MAX_SWEEPS, MPS_OPT_JACOBI_TOL, MPS_OPT_KERNEL_TIMING, MPS_OPT_RANK_FLOOR = 1, 2, 3, 4
MPS_OPT_BLOCK_WIDTH, MPS_OPT_MAX_INNER, MPS_OPT_MAX_SLOTS, MPS_OPT_WORKSPACE_MB = 5, 6, 7, 8
MPS_OPT_DD_REFINE, MPS_OPT_JACOBI_STREAMS, MPS_OPT_FUSE, MPS_OPT_QR, MPS_OPT_STEP_SPLIT = 9, 10, 11, 12, 13
MPS_OPT_DD_STREAM, MPS_OPT_MAX_INNER_FEW, MPS_OPT_TICK_SWEEPS, MPS_OPT_GRAPH = 14, 15, 16, 17
KERNEL_CLASSES = ["theta", "jacobi", "truncate", "split", "gate1", "amplitude", "dd_refine", "rdo"]
COUNTER_SWEEPS, COUNTER_SWEEPS_DD, COUNTER_NOCONV, COUNTER_GRAPHS = 8, 9, 10, 11

_STATUS = {0: "MPS_OK", -1: "MPS_EINVAL", -2: "MPS_ERANGE", -3: "MPS_ENOMEM", -4: "MPS_EDEVICE",
           -5: "MPS_ENOCONV", -6: "MPS_ENONFINITE", -7: "MPS_ESTATE"}


class MPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class mps_update_stats(C.Structure):
    _fields_ = [("W", C.c_double), ("w", C.c_double), ("gap", C.c_double), ("epsdist", C.c_double),
                ("k", C.c_int), ("rank", C.c_int), ("sweeps", C.c_int), ("splits", C.c_int),
                ("dd_sweeps", C.c_int), ("reserved", C.c_int)]


_dp = C.POINTER(C.c_double)
_h = C.c_void_p
_lib.mps_create.restype = _h
_lib.mps_create.argtypes = [C.c_int, C.c_int, C.c_double]
_lib.mps_create_ex.restype = _h
_lib.mps_create_ex.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p]
_lib.mps_destroy.argtypes = [_h]
_lib.mps_apply_gate.argtypes = [_h, C.c_int, C.c_int, _dp]
_lib.mps_apply_gate_dd.argtypes = [_h, C.c_int, C.c_int, _dp, _dp]
_lib.mps_apply_gates.argtypes = [_h, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _dp, _dp]
_lib.mps_apply_gate2.argtypes = [_h, C.c_int, C.c_int, _dp]
_lib.mps_apply_gate2_dd.argtypes = [_h, C.c_int, C.c_int, _dp, _dp]
_lib.mps_export.argtypes = [_h, C.c_void_p, C.c_long, C.POINTER(C.c_long)]
_lib.mps_import.restype = _h
_lib.mps_import.argtypes = [C.c_void_p, C.c_long, C.c_void_p]
_lib.mps_bond_dim.argtypes = [_h, C.c_int, C.POINTER(C.c_int)]
_lib.mps_schmidt.argtypes = [_h, C.c_int, _dp, C.c_int, C.POINTER(C.c_int)]
_lib.mps_schmidt_dd.argtypes = [_h, C.c_int, _dp, _dp, C.c_int, C.POINTER(C.c_int)]
_lib.mps_amplitude.argtypes = [_h, C.POINTER(C.c_ubyte), _dp]
_lib.mps_amplitude_dd.argtypes = [_h, C.POINTER(C.c_ubyte), _dp]
_lib.mps_amplitudes.argtypes = [_h, C.c_int, C.POINTER(C.c_ubyte), _dp]
_lib.mps_amplitudes_noalloc.argtypes = [_h, C.c_int, C.POINTER(C.c_ubyte), _dp]
_lib.mps_stats.argtypes = [_h, C.POINTER(mps_update_stats)]
_lib.mps_load.argtypes = [_h, C.POINTER(C.c_int), C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_dp), C.POINTER(_dp)]
_lib.mps_get_site.argtypes = [_h, C.c_int, _dp, _dp, C.c_long]
_lib.mps_set_option.argtypes = [_h, C.c_int, C.c_double]
_lib.mps_sync.argtypes = [_h]
_lib.mps_kernel_time.argtypes = [_h, C.c_int, _dp, C.POINTER(C.c_long), C.c_int]
_lib.mps_last_error.restype = C.c_char_p
_lib.mps_last_error.argtypes = [_h]
_lib.mps_version.restype = C.c_char_p
_lib.mps_tuning_key.restype = C.c_char_p
_lib.mps_tuning_key.argtypes = []
_lib.mps_rdo.argtypes = [_h, C.c_int, C.POINTER(C.c_int), _dp]
_lib.mps_rdo_dd.argtypes = [_h, C.c_int, C.POINTER(C.c_int), _dp, _dp]
_lib.mps_rdo_block.argtypes = [_h, C.c_int, C.c_int, _dp]
_b = C.c_void_p
_ip = C.POINTER(C.c_int)
_lib.mps_batch_create.restype = _b
_lib.mps_batch_create.argtypes = [C.c_int, _ip, _ip, _dp, C.c_int]
_lib.mps_batch_run.argtypes = [_b, C.c_long, _ip, _ip, _ip, _dp, _dp]
_lib.mps_batch_get.restype = _h
_lib.mps_batch_get.argtypes = [_b, C.c_int]
_lib.mps_batch_set_option.argtypes = [_b, C.c_int, C.c_double]
_lib.mps_batch_last_error.restype = C.c_char_p
_lib.mps_batch_last_error.argtypes = [_b]
_lib.mps_batch_destroy.argtypes = [_b]

EXPORTED = ["mps_create", "mps_create_ex", "mps_destroy", "mps_apply_gate", "mps_apply_gate_dd",
            "mps_apply_gates", "mps_apply_gate2", "mps_apply_gate2_dd", "mps_bond_dim", "mps_schmidt", "mps_schmidt_dd", "mps_amplitude",
            "mps_amplitude_dd", "mps_amplitudes", "mps_amplitudes_noalloc", "mps_stats", "mps_load", "mps_get_site",
            "mps_export", "mps_import",
            "mps_set_option", "mps_sync", "mps_kernel_time", "mps_last_error", "mps_version", "mps_tuning_key",
            "mps_rdo", "mps_rdo_dd", "mps_rdo_block", "mps_batch_create", "mps_batch_run", "mps_batch_get", "mps_batch_set_option",
            "mps_batch_last_error", "mps_batch_destroy"]


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _check(h, rc):
    if rc != MPS_OK:
        raise MPSError(rc, mps_last_error(h))
    return rc


def _gate_doubles(u, k):
    if u is None:
        return None
    a = np.ascontiguousarray(np.asarray(u, dtype=np.complex128).reshape(1 << k, 1 << k))
    return a.view(np.float64).ravel().copy()


# ---------------------------------------------------------------- C-ABI mirrors
def mps_version() -> str:
    return _lib.mps_version().decode()


def mps_tuning_key() -> str:
    return (_lib.mps_tuning_key() or b"").decode()


def mps_last_error(h=None) -> str:
    return (_lib.mps_last_error(h) or b"").decode()


def mps_create(n: int, chi_max: int, eps: float):
    h = _lib.mps_create(n, chi_max, float(eps))
    if not h:
        raise MPSError(MPS_EINVAL, mps_last_error(None))
    return h


def mps_create_ex(n: int, chi_max: int, eps: float, prec: int = MPS_PREC_FP64, hip_stream=None):
    h = _lib.mps_create_ex(n, chi_max, float(eps), prec, hip_stream)
    if not h:
        raise MPSError(MPS_EINVAL, mps_last_error(None))
    return h


def mps_destroy(h) -> int:
    return _lib.mps_destroy(h)


def mps_export(h) -> bytes:
    """The state as a checkpoint image (bytes)."""
    size = C.c_long(0)
    _check(h, _lib.mps_export(h, None, 0, C.byref(size)))
    buf = C.create_string_buffer(size.value)
    _check(h, _lib.mps_export(h, buf, size.value, C.byref(size)))
    return buf.raw[: size.value]


def mps_import(image: bytes, hip_stream=None):
    """A new handle from a checkpoint image written by mps_export."""
    buf = C.create_string_buffer(bytes(image), len(image))
    h = _lib.mps_import(buf, len(image), hip_stream)
    if not h:
        raise MPSError(MPS_EINVAL, mps_last_error(None))
    return h


def mps_apply_gate(h, first: int, k: int, U) -> int:
    u = _gate_doubles(U, k)
    return _check(h, _lib.mps_apply_gate(h, first, k, _ptr(u)))


def mps_apply_gate_dd(h, first: int, k: int, U_hi, U_lo) -> int:
    uh, ul = _gate_doubles(U_hi, k), _gate_doubles(U_lo, k)
    return _check(h, _lib.mps_apply_gate_dd(h, first, k, _ptr(uh), _ptr(ul)))


def mps_apply_gate2(h, q0: int, q1: int, U) -> int:
    """Two-qubit gate on any two distinct qubits (U's first index bit is q0)."""
    u = _gate_doubles(U, 2)
    return _check(h, _lib.mps_apply_gate2(h, q0, q1, _ptr(u)))


def mps_apply_gate2_dd(h, q0: int, q1: int, U_hi, U_lo) -> int:
    uh, ul = _gate_doubles(U_hi, 2), _gate_doubles(U_lo, 2)
    return _check(h, _lib.mps_apply_gate2_dd(h, q0, q1, _ptr(uh), _ptr(ul)))


def _pack(gates):
    first = (C.c_int * len(gates))(*[g.first for g in gates])
    ks = (C.c_int * len(gates))(*[g.k for g in gates])
    uh = np.concatenate([_gate_doubles(g.u_hi, g.k) for g in gates])
    ul = None
    if any(getattr(g, "u_lo", None) is not None for g in gates):
        ul = np.concatenate([_gate_doubles(g.u_lo, g.k) if getattr(g, "u_lo", None) is not None
                             else np.zeros(2 << (2 * g.k)) for g in gates])
    return first, ks, uh, ul


def mps_apply_gates(h, gates, allow_noconv: bool = False) -> int:
    """gates: sequence of objects with .first, .k, .u_hi and optional .u_lo."""
    if not gates:
        return MPS_OK
    first, ks, uh, ul = _pack(gates)
    rc = _lib.mps_apply_gates(h, len(gates), first, ks, _ptr(uh), _ptr(ul))
    if rc == MPS_ENOCONV and allow_noconv:
        return rc
    return _check(h, rc)


def mps_bond_dim(h, bond: int) -> int:
    m = C.c_int()
    _check(h, _lib.mps_bond_dim(h, bond, C.byref(m)))
    return m.value


def mps_schmidt(h, bond: int) -> np.ndarray:
    cap = mps_bond_dim(h, bond)
    lam = np.zeros(max(cap, 1))
    m = C.c_int()
    _check(h, _lib.mps_schmidt(h, bond, _ptr(lam), cap, C.byref(m)))
    return lam[: m.value]


def mps_schmidt_dd(h, bond: int):
    cap = mps_bond_dim(h, bond)
    hi, lo = np.zeros(max(cap, 1)), np.zeros(max(cap, 1))
    m = C.c_int()
    _check(h, _lib.mps_schmidt_dd(h, bond, _ptr(hi), _ptr(lo), cap, C.byref(m)))
    return hi[: m.value], lo[: m.value]


def _bits(b, n=None):
    a = np.ascontiguousarray(np.asarray(b, dtype=np.uint8))
    return a, a.ctypes.data_as(C.POINTER(C.c_ubyte))


def mps_amplitude(h, bits) -> complex:
    a, p = _bits(bits)
    out = np.zeros(2)
    _check(h, _lib.mps_amplitude(h, p, _ptr(out)))
    return complex(out[0], out[1])


def mps_amplitude_dd(h, bits):
    a, p = _bits(bits)
    out = np.zeros(4)
    _check(h, _lib.mps_amplitude_dd(h, p, _ptr(out)))
    return complex(out[0], out[2]), complex(out[1], out[3])


def mps_amplitudes(h, bits_2d, dd: bool = False, noalloc: bool = False):
    a, p = _bits(bits_2d)
    count = a.shape[0]
    out = np.zeros(count * (4 if dd else 2))
    fn = _lib.mps_amplitudes_noalloc if noalloc else _lib.mps_amplitudes
    _check(h, fn(h, count, p, _ptr(out)))
    if dd:
        o = out.reshape(count, 4)
        return o[:, 0] + 1j * o[:, 2], o[:, 1] + 1j * o[:, 3]
    o = out.reshape(count, 2)
    return o[:, 0] + 1j * o[:, 1]


def mps_amplitudes_noalloc(h, bits_2d, dd: bool = False):
    """mps_amplitudes through the entry point that allocates nothing."""
    return mps_amplitudes(h, bits_2d, dd, noalloc=True)


def mps_rdo(h, qubits):
    """Reduced density operator of `qubits` (the first is the most significant bit)."""
    L = len(qubits)
    q = (C.c_int * L)(*[int(x) for x in qubits])
    out = np.zeros(2 << (2 * L))
    _check(h, _lib.mps_rdo(h, L, q, _ptr(out)))
    return out.view(np.complex128).reshape(1 << L, 1 << L)


def mps_rdo_dd(h, qubits):
    L = len(qubits)
    q = (C.c_int * L)(*[int(x) for x in qubits])
    hi, lo = np.zeros(2 << (2 * L)), np.zeros(2 << (2 * L))
    _check(h, _lib.mps_rdo_dd(h, L, q, _ptr(hi), _ptr(lo)))
    return (hi.view(np.complex128).reshape(1 << L, 1 << L), lo.view(np.complex128).reshape(1 << L, 1 << L))


def mps_rdo_block(h, first: int, last: int):
    L = last - first + 1
    out = np.zeros(2 << (2 * max(L, 0)))
    _check(h, _lib.mps_rdo_block(h, first, last, _ptr(out)))
    return out.view(np.complex128).reshape(1 << L, 1 << L)


def mps_stats(h) -> dict:
    s = mps_update_stats()
    _check(h, _lib.mps_stats(h, C.byref(s)))
    return {f: getattr(s, f) for f, _ in s._fields_}


def mps_load(h, B, lam, B_lo=None, lam_lo=None) -> int:
    n = len(B)
    dims = (C.c_int * max(1, n - 1))(*[len(l) for l in lam])
    keep = []

    def ptrs(arrs, cplx):
        if arrs is None:
            return None
        P = (_dp * len(arrs))()
        for i, x in enumerate(arrs):
            y = np.ascontiguousarray(np.asarray(x, dtype=np.complex128 if cplx else np.float64))
            y = y.view(np.float64).copy() if cplx else y.copy()
            keep.append(y)
            P[i] = _ptr(y)
        return P

    lp = ptrs(lam, False) if n > 1 else (_dp * 1)()
    return _check(h, _lib.mps_load(h, dims, ptrs(B, True), ptrs(B_lo, True), lp, ptrs(lam_lo, False)))


def mps_get_site(h, s: int, dims, dd: bool = False):
    a, b = dims
    hi = np.zeros(a * 2 * b * 2)
    lo = np.zeros_like(hi) if dd else None
    _check(h, _lib.mps_get_site(h, s, _ptr(hi), _ptr(lo), hi.size))
    hi = hi.view(np.complex128).reshape(a, 2, b)
    return (hi, lo.view(np.complex128).reshape(a, 2, b)) if dd else hi


def mps_set_option(h, key: int, value: float) -> int:
    return _check(h, _lib.mps_set_option(h, key, float(value)))


def mps_sync(h) -> int:
    return _check(h, _lib.mps_sync(h))


def mps_kernel_time(h, cls: int, reset: bool = False):
    ms = C.c_double()
    cnt = C.c_long()
    _check(h, _lib.mps_kernel_time(h, cls, C.byref(ms), C.byref(cnt), int(reset)))
    return ms.value, cnt.value


def mps_batch_last_error(b=None) -> str:
    return (_lib.mps_batch_last_error(b) or b"").decode()


def _bcheck(b, rc):
    if rc != MPS_OK:
        raise MPSError(rc, mps_batch_last_error(b))
    return rc


def mps_batch_create(n, chi_max, eps, prec: int = MPS_PREC_FP64):
    count = len(n)
    ni = (C.c_int * count)(*[int(x) for x in n])
    ci = (C.c_int * count)(*[int(x) for x in chi_max])
    ep = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
    b = _lib.mps_batch_create(count, ni, ci, _ptr(ep), prec)
    if not b:
        raise MPSError(MPS_EINVAL, mps_batch_last_error(None))
    return b


def mps_batch_run(b, circuit, gates, allow_noconv: bool = False) -> int:
    """circuit[i]: the circuit gate i acts on; gates as for mps_apply_gates."""
    if not len(gates):
        return MPS_OK
    first, ks, uh, ul = _pack(gates)
    ci = (C.c_int * len(gates))(*[int(c) for c in circuit])
    rc = _lib.mps_batch_run(b, len(gates), ci, first, ks, _ptr(uh), _ptr(ul))
    if rc == MPS_ENOCONV and allow_noconv:
        return rc
    return _bcheck(b, rc)


def mps_batch_get(b, circuit: int):
    h = _lib.mps_batch_get(b, circuit)
    if not h:
        raise MPSError(MPS_EINVAL, f"no circuit {circuit} in the batch")
    return h


def mps_batch_set_option(b, key: int, value: float) -> int:
    return _bcheck(b, _lib.mps_batch_set_option(b, key, float(value)))


def mps_batch_destroy(b) -> int:
    return _lib.mps_batch_destroy(b)


# ---------------------------------------------------------------- convenience classes
class MPS:
    """An n-qubit state on the device (Section 3.1 of the paper)."""

    def __init__(self, n: int, chi_max: int, eps: float = 0.0, prec: int = MPS_PREC_FP64, _borrowed=None):
        self.n, self.chi_max, self.eps, self.prec = n, chi_max, eps, prec
        self._owned = _borrowed is None
        self.h = mps_create_ex(n, chi_max, eps, prec, None) if self._owned else _borrowed

    def close(self):
        if self.h and self._owned:
            mps_destroy(self.h)
        self.h = None

    def export(self) -> bytes:
        """Checkpoint image of the state (mps_export)."""
        return mps_export(self.h)

    @classmethod
    def from_image(cls, image: bytes) -> "MPS":
        """Resume from a checkpoint image (mps_import); n, chi_max, eps and the
        precision come from the image."""
        import struct
        _, n, chi, prec = struct.unpack_from("<4i", image, 8)
        (eps,) = struct.unpack_from("<d", image, 24)
        m = cls.__new__(cls)
        m.n, m.chi_max, m.eps, m.prec = n, chi, eps, prec
        m._owned = True
        m.h = mps_import(image)
        return m

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def dd(self) -> bool:
        return self.prec == MPS_PREC_DD

    def apply(self, first, k, u_hi, u_lo=None):
        if u_lo is not None:
            return mps_apply_gate_dd(self.h, first, k, u_hi, u_lo)
        return mps_apply_gate(self.h, first, k, u_hi)

    def apply_gate(self, g):
        return self.apply(g.first, g.k, g.u_hi, getattr(g, "u_lo", None))

    def apply_gate2(self, q0, q1, u_hi, u_lo=None):
        """U(4) on qubits q0 and q1, adjacent or not (SWAP routing in the library)."""
        if u_lo is not None:
            return mps_apply_gate2_dd(self.h, q0, q1, u_hi, u_lo)
        return mps_apply_gate2(self.h, q0, q1, u_hi)

    def apply_gates(self, gates, allow_noconv=False):
        return mps_apply_gates(self.h, gates, allow_noconv)

    def bond_dim(self, b):
        return mps_bond_dim(self.h, b)

    def bond_dims(self):
        return [mps_bond_dim(self.h, b) for b in range(self.n - 1)]

    def schmidt(self, b):
        return mps_schmidt(self.h, b)

    def schmidt_dd(self, b):
        return mps_schmidt_dd(self.h, b)

    def amplitude(self, bits):
        return mps_amplitude(self.h, bits)

    def amplitudes(self, bits_2d, dd=False, noalloc=False):
        return mps_amplitudes(self.h, bits_2d, dd, noalloc)

    def stats(self):
        return mps_stats(self.h)

    def rdo(self, qubits, dd=False):
        return mps_rdo_dd(self.h, qubits) if dd else mps_rdo(self.h, qubits)

    def rdo_block(self, first, last):
        return mps_rdo_block(self.h, first, last)

    def load(self, B, lam, B_lo=None, lam_lo=None):
        return mps_load(self.h, B, lam, B_lo, lam_lo)

    def site(self, s):
        dims = [1] + self.bond_dims() + [1]
        return mps_get_site(self.h, s, (dims[s], dims[s + 1]), self.dd)

    def set_option(self, key, value):
        return mps_set_option(self.h, key, value)

    def sync(self):
        return mps_sync(self.h)

    def kernel_time(self, cls, reset=False):
        return mps_kernel_time(self.h, cls, reset)


class Batch:
    """Independent circuits evolved together (one scheduler, shared launches)."""

    def __init__(self, n, chi_max, eps, prec: int = MPS_PREC_FP64):
        self.prec = prec
        self.b = mps_batch_create(n, chi_max, eps, prec)
        self.states = [MPS(int(n[i]), int(chi_max[i]), float(eps[i]), prec, _borrowed=mps_batch_get(self.b, i))
                       for i in range(len(n))]

    def __len__(self):
        return len(self.states)

    def __getitem__(self, i) -> MPS:
        return self.states[i]

    def run(self, circuit, gates, allow_noconv=False):
        return mps_batch_run(self.b, circuit, gates, allow_noconv)

    def set_option(self, key, value):
        return mps_batch_set_option(self.b, key, value)

    def close(self):
        if self.b:
            for s in self.states:
                s.h = None
            mps_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
