"""Seeded synthetic inputs shared by the device path, the oracle and the benchmark.

This module only *draws* inputs: gate matrices, circuit schedules, bitstrings and
random MPS tensors.  It holds none of the gate-update arithmetic (no contraction,
no decomposition, no truncation), so that the oracle and the device path stay
independent and meet only here.

Conventions (used by every caller):

* A k-site gate is a 2^k x 2^k complex matrix, row-major, ``U[r, c] = <r|U|c>``.
  The basis index of the gate is ``r = sum_t i_{first+t} * 2^(k-1-t)``: the first
  (leftmost) site is the most significant bit.  Qubit 0 is the leftmost qubit of
  the state |i_0 ... i_{n-1}> written in the paper's Section 3.1.
* Double-double inputs are pairs ``(hi, lo)`` of float64 arrays whose exact sum is
  the value; ``lo`` is zero for gates that are exact binary64 values.
* Seeds: ``numpy.random.Generator(PCG64(seed))``.  One generator per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng_for", "haar_unitary", "brickwork", "brickwork_layer", "random_triples",
    "bitstrings", "ghz_circuit", "paper_sample_circuit", "embed_gate",
    "product_state_prep", "qft_lnn_circuit", "random_mps_B", "batch_spec",
    "Gate", "hadamard", "cnot", "dd_split", "haar_unitary_dd", "brickwork_dd",
    "random_circuit_dd", "basis_prep", "batch_gates", "CircuitSpec",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Gate:
    """One gate of a circuit: ``k`` adjacent sites starting at ``first``."""
    first: int
    k: int
    u_hi: np.ndarray                     # complex128, (2^k, 2^k)
    u_lo: np.ndarray | None = field(default=None)  # complex128 or None (exact binary64)

    @property
    def u(self) -> np.ndarray:
        return self.u_hi


def haar_unitary(d: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed U(d): QR of a complex Ginibre matrix with the phases of
    diag(R) divided out (Mezzadri, Notices AMS 54, 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return np.ascontiguousarray(q * ph[None, :])


def haar_unitary_dd(d: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """A Haar U(d) drawn as in ``haar_unitary`` and then made unitary to ~1e-60 by two
    Newton-Schulz polar steps U <- U (3 I - U^H U) / 2 at 256 bits, rounded to
    double-double (hi, lo).  Used where a pin needs an exactly unitary gate."""
    import mpmath
    u0 = haar_unitary(d, rng)
    with mpmath.workprec(256):
        U = mpmath.matrix([[mpmath.mpc(complex(u0[r, c])) for c in range(d)] for r in range(d)])
        I3 = 3 * mpmath.eye(d)
        for _ in range(2):
            U = U * (I3 - U.H * U) / 2
        hi = np.zeros((d, d), dtype=np.complex128)
        lo = np.zeros((d, d), dtype=np.complex128)
        for r in range(d):
            for c in range(d):
                hi[r, c], lo[r, c] = _cdd(U[r, c])
    return hi, lo


def brickwork_dd(n: int, depth: int, seed: int) -> list[list[Gate]]:
    """Brickwork circuit with exactly unitary (double-double) Haar gates."""
    rng = rng_for(seed)
    out = []
    for t in range(depth):
        layer = []
        for j in range(t % 2, n - 1, 2):
            hi, lo = haar_unitary_dd(4, rng)
            layer.append(Gate(j, 2, hi, lo))
        out.append(layer)
    return out


def brickwork_layer(n: int, t: int, rng: np.random.Generator) -> list[Gate]:
    """Layer t of a brickwork circuit: U(4) gates on sites (j, j+1), j = t (mod 2)."""
    return [Gate(j, 2, haar_unitary(4, rng)) for j in range(t % 2, n - 1, 2)]


def brickwork(n: int, depth: int, seed: int) -> list[list[Gate]]:
    rng = rng_for(seed)
    return [brickwork_layer(n, t, rng) for t in range(depth)]


def random_triples(n: int, count: int, seed: int) -> list[Gate]:
    """``count`` Haar U(8) gates on contiguous triples, first site uniform in [0, n-3]."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        first = int(rng.integers(0, n - 2))
        out.append(Gate(first, 3, haar_unitary(8, rng)))
    return out


def random_circuit_dd(n: int, count: int, seed: int, ks=(1, 2, 3)) -> list[Gate]:
    """Random gates of mixed width k in ``ks`` on random contiguous windows, exactly
    unitary (double-double)."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        k = int(rng.choice([k for k in ks if k <= n]))
        first = int(rng.integers(0, n - k + 1))
        hi, lo = haar_unitary_dd(1 << k, rng)
        out.append(Gate(first, k, hi, lo))
    return out


def basis_prep(bits) -> list[Gate]:
    """Pauli-X gates preparing the basis state |bits> from |0...0>."""
    x = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    return [Gate(q, 1, x.copy()) for q, b in enumerate(bits) if b]


def bitstrings(n: int, count: int, seed: int) -> np.ndarray:
    return rng_for(seed).integers(0, 2, size=(count, n), dtype=np.uint8)


def hadamard() -> np.ndarray:
    s = 1.0 / math.sqrt(2.0)
    return np.array([[s, s], [s, -s]], dtype=np.complex128)


def cnot() -> np.ndarray:
    """Control = first (most significant) qubit of the gate index."""
    u = np.zeros((4, 4), dtype=np.complex128)
    u[0, 0] = u[1, 1] = u[2, 3] = u[3, 2] = 1.0
    return u


def embed_gate(u: np.ndarray, qubits: list[int], k: int) -> np.ndarray:
    """Embed a gate acting on positions ``qubits`` (within a k-site window, position
    0 = most significant) into a 2^k x 2^k matrix acting as identity elsewhere.
    Used to express a non-adjacent gate as one gate on a contiguous window."""
    m = len(qubits)
    d = 1 << k
    out = np.zeros((d, d), dtype=np.complex128)
    rest = [p for p in range(k) if p not in qubits]
    for r in range(d):
        rb = [(r >> (k - 1 - p)) & 1 for p in range(k)]
        for c in range(d):
            cb = [(c >> (k - 1 - p)) & 1 for p in range(k)]
            if any(rb[p] != cb[p] for p in rest):
                continue
            rr = sum(rb[q] << (m - 1 - t) for t, q in enumerate(qubits))
            cc = sum(cb[q] << (m - 1 - t) for t, q in enumerate(qubits))
            out[r, c] = u[rr, cc]
    return out


def paper_sample_circuit() -> list[Gate]:
    """The 3-qubit example of the paper (Section 3.2): |000>, H on qubit 0, then CNOT
    with control 0 and target 2, written as one U(8) on sites 0..2."""
    return [Gate(0, 1, hadamard()), Gate(0, 3, embed_gate(cnot(), [0, 2], 3))]


def ghz_circuit(n: int) -> list[Gate]:
    return [Gate(0, 1, hadamard())] + [Gate(s, 2, cnot()) for s in range(n - 1)]


def dd_split(x_mp) -> tuple[float, float]:
    """Round an mpmath number to a double-double pair (hi, lo)."""
    import mpmath
    hi = float(x_mp)
    lo = float(x_mp - mpmath.mpf(hi))
    return hi, lo


def _cdd(z_mp) -> tuple[complex, complex]:
    import mpmath
    rh, rl = dd_split(mpmath.re(z_mp))
    ih, il = dd_split(mpmath.im(z_mp))
    return complex(rh, ih), complex(rl, il)


def product_state_prep(n: int, seed: int) -> list[Gate]:
    """Single-qubit preparation gates [[a, -conj(b)], [b, conj(a)]] with
    a = cos(t/2), b = e^{i phi} sin(t/2), cos t ~ U[-1, 1], phi ~ U[0, 2 pi);
    evaluated at 256 bits and rounded to double-double."""
    import mpmath
    rng = rng_for(seed)
    out = []
    with mpmath.workprec(256):
        for q in range(n):
            ct = mpmath.mpf(float(rng.uniform(-1.0, 1.0)))
            phi = mpmath.mpf(float(rng.uniform(0.0, 2.0 * math.pi)))
            th = mpmath.acos(ct)
            a = mpmath.cos(th / 2)
            b = mpmath.expj(phi) * mpmath.sin(th / 2)
            ent = [[a, -mpmath.conj(b)], [b, mpmath.conj(a)]]
            hi = np.zeros((2, 2), dtype=np.complex128)
            lo = np.zeros((2, 2), dtype=np.complex128)
            for r in range(2):
                for c in range(2):
                    hi[r, c], lo[r, c] = _cdd(mpmath.mpc(ent[r][c]))
            out.append(Gate(q, 1, hi, lo))
    return out


def qft_lnn_circuit(n: int) -> list[Gate]:
    """Quantum Fourier transform as a nearest-neighbour network.

    For j = 0..n-1: a Hadamard at position 0 (which holds logical qubit j), then
    n-1-j fused gates walking right, each SWAP * diag(1, 1, 1, e^{2 pi i / 2^m}) with
    m = q - j + 1 where q is the logical qubit being crossed.  The network ends
    with the qubit order reversed, so position p holds output bit y_p and the
    amplitudes come out in standard order.  Phases are double-double."""
    import mpmath
    out: list[Gate] = []
    with mpmath.workprec(256):
        hs = mpmath.sqrt(mpmath.mpf(2)) / 2
        hh, hl = dd_split(hs)
        Hhi = np.array([[hh, hh], [hh, -hh]], dtype=np.complex128)
        Hlo = np.array([[hl, hl], [hl, -hl]], dtype=np.complex128)
        # order[p] = logical qubit at position p
        order = list(range(n))
        for j in range(n):
            assert order[0] == j
            out.append(Gate(0, 1, Hhi.copy(), Hlo.copy()))
            for p in range(0, n - 1 - j):
                q = order[p + 1]
                m = q - j + 1
                ph = mpmath.expj(2 * mpmath.pi / mpmath.mpf(2) ** m)
                phi, plo = _cdd(ph)
                hi = np.zeros((4, 4), dtype=np.complex128)
                lo = np.zeros((4, 4), dtype=np.complex128)
                # SWAP . diag(1,1,1,w):  |ab> -> w^{ab} |ba>
                hi[0, 0] = 1.0
                hi[2, 1] = 1.0
                hi[1, 2] = 1.0
                hi[3, 3] = phi
                lo[3, 3] = plo
                out.append(Gate(p, 2, hi, lo))
                order[p], order[p + 1] = order[p + 1], order[p]
    return out


def random_mps_B(dims: list[int], rng: np.random.Generator, spread: float = 0.0):
    """A random MPS in the (B, lambda) gauge for single-update tests.

    ``dims`` = [m_0, ..., m_{n-2}] bond dims.  Returns (B, lam): B[s] complex128 of
    shape (m_{s-1}, 2, m_s) with i.i.d. Gaussian entries scaled by 1/sqrt(2 m_s),
    lam[s] positive, sorted descending, with sum of squares 1 (values drawn as
    exp(-spread * u), u ~ U[0,1), then normalised).  The state is generally not in
    canonical form; the update is still a well-defined function of it."""
    n = len(dims) + 1
    full = [1] + list(dims) + [1]
    B, lam = [], []
    for s in range(n):
        a, b = full[s], full[s + 1]
        z = (rng.standard_normal((a, 2, b)) + 1j * rng.standard_normal((a, 2, b)))
        B.append(np.ascontiguousarray(z / math.sqrt(4.0 * b)))
    for s in range(n - 1):
        v = np.exp(-spread * rng.uniform(0.0, 1.0, size=dims[s]))
        v = np.sort(v)[::-1]
        v = v / math.sqrt(float(np.sum(v * v)))
        lam.append(np.ascontiguousarray(v))
    return B, lam


@dataclass
class CircuitSpec:
    n: int
    chi_max: int
    depth: int
    seed: int


def batch_spec(count: int, seed: int) -> list[CircuitSpec]:
    """Independent circuits: n ~ U{16..48}, chi_max ~ U{32, 64, 128, 256},
    depth ~ U{8..24}, each with its own spawned seed."""
    rng = rng_for(seed)
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(count)
    out = []
    for i in range(count):
        n = int(rng.integers(16, 49))
        chi = int(rng.choice([32, 64, 128, 256]))
        depth = int(rng.integers(8, 25))
        out.append(CircuitSpec(n, chi, depth, int(kids[i].generate_state(1)[0])))
    return out


def batch_gates(specs: list[CircuitSpec]) -> tuple[list[int], list[Gate]]:
    """The brickwork circuits of `specs` (Haar U(4), each from its own seed) as one
    gate list, layer-interleaved: layer t of every circuit, then layer t + 1.
    Returns (circuit index per gate, gates)."""
    layers = [brickwork(s.n, s.depth, s.seed) for s in specs]
    circ, gates = [], []
    for t in range(max((s.depth for s in specs), default=0)):
        for i, ls in enumerate(layers):
            if t < len(ls):
                circ += [i] * len(ls[t])
                gates += ls[t]
    return circ, gates


def _saturated_dims(n: int, chi: int) -> list[int]:
    return [min(chi, 2 ** (b + 1), 2 ** (n - 1 - b)) for b in range(n - 1)]


def update_chi256_inputs() -> dict:
    """One two-site update at a = b = c = 256: a 20-qubit random (B, V) state whose
    bonds 7..11 hold 256 values, a Haar U(4) on sites 9, 10 (theta 512 x 512),
    chi_max = 256 (binding), eps = 1e-12, 24 random bitstrings (seed 256)."""
    n, chi, eps, seed = 20, 256, 1e-12, 256
    dims = _saturated_dims(n, chi)
    rng = rng_for(seed)
    Bt, lam = random_mps_B(dims, rng, spread=4.0)
    U = haar_unitary(4, rng)
    bits = bitstrings(n, 24, seed + 1)
    return dict(n=n, chi=chi, eps=eps, seed=seed, dims=dims, B=Bt, lam=lam, U=U, first=9, bits=bits)


def update3_chi512_inputs() -> dict:
    """One three-site update at a = b = c = d = 512: a 22-qubit random (B, V) state
    whose bonds 8..12 hold 512 values, a Haar U(8) on sites 9, 10, 11 (first split
    theta 1024 x 2048, second 1024 x 1024), chi_max = 512 (binding), eps = 1e-14, 24
    random bitstrings (seed 512)."""
    n, chi, eps, seed = 22, 512, 1e-14, 512
    dims = _saturated_dims(n, chi)
    rng = rng_for(seed)
    Bt, lam = random_mps_B(dims, rng, spread=4.0)
    U = haar_unitary(8, rng)
    bits = bitstrings(n, 24, seed + 1)
    return dict(n=n, chi=chi, eps=eps, seed=seed, dims=dims, B=Bt, lam=lam, U=U, first=9, bits=bits)
