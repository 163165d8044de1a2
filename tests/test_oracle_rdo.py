"""Pins of the oracle's reduced density operators (paper, Section 3.2: RDO_block and
RDO(list)): rho = Tr over the other qubits of |Psi><Psi|, the first listed qubit being
the most significant bit of the basis index."""
import os

import mpmath
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
mpmath.mp.prec = 256


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def partial_trace(psi_flat, n, q):
    """Textbook partial trace of |psi><psi| keeping qubits q (in that order)."""
    psi = psi_flat.reshape([2] * n)
    rest = [x for x in range(n) if x not in q]
    t = np.transpose(psi, list(q) + rest).reshape(1 << len(q), -1)
    return t @ t.conj().T


def test_paper_sample_rdo_printed_values(oracle_mod):
    """The paper's printed output: RDO_block(0, 2) of |000> and, after H(0) and
    CNOT(0 -> 2) as one U(8), RDO of qubits {0, 2}."""
    rows = [l.split() for l in open(os.path.join(GOLD, "paper_sample.txt")) if l.strip() and not l.startswith("#")]
    m = oracle_mod.OracleMPS(3, 8, 0.0)
    for stage in ("initial", "final"):
        if stage == "final":
            for g in W.paper_sample_circuit():
                m.apply_gate(g)
        sel = [r for r in rows if r[0] == stage]
        q = [int(x) for x in sel[0][1].split(",")]
        want = np.zeros((1 << len(q), 1 << len(q)))
        for r in sel:
            want[int(r[2], 2), int(r[3], 2)] = float(r[4])
        h, l = m.rdo(q)
        assert np.max(np.abs((h - want) + l)) < 1e-30


@pytest.mark.parametrize("q", [[2], [0, 3], [5, 1], [2, 3, 4], [6, 0, 4], [0, 1, 2, 3, 4, 5, 6]])
def test_rdo_equals_partial_trace_of_amplitudes(oracle_mod, q):
    """Brickwork state (no truncation) on 7 qubits: the oracle's contraction against a
    numpy partial trace of its 128 amplitudes (themselves pinned to the state vector)."""
    n = 7
    om = oracle_mod.OracleMPS(n, 128, 0.0)
    for layer in W.brickwork(n, 5, 3):
        for g in layer:
            om.apply_gate(g)
    ah, al = om.amplitudes(all_bits(n))
    ref = partial_trace(ah + al, n, q)
    h, l = om.rdo(q)
    assert np.max(np.abs(h + l - ref)) < 1e-14


def test_rdo_ghz_closed_form(oracle_mod):
    """GHZ on 6 qubits: a proper subset sees (|0..0><0..0| + |1..1><1..1|)/2, the whole
    register the pure state with 1/2 in the four corners."""
    n = 6
    om = oracle_mod.OracleMPS(n, 4, 0.0)
    for g in W.ghz_circuit(n):
        om.apply_gate(g)
    for q in ([1, 4], [0, 2, 5], list(range(n))):
        d = 1 << len(q)
        want = np.zeros((d, d))
        want[0, 0] = want[-1, -1] = 0.5
        if len(q) == n:
            want[0, -1] = want[-1, 0] = 0.5
        h, l = om.rdo(q)
        assert np.max(np.abs((h - want) + l)) < 1e-30


def test_rdo_product_state_closed_form(oracle_mod):
    """A product state prepared by single-qubit gates: rho of one qubit is the pure
    state U|0> (the gate's first column), of two qubits the Kronecker product; checked
    at 256 bits against the dd gate entries."""
    n = 5
    prep = W.product_state_prep(n, 11)
    om = oracle_mod.OracleMPS(n, 4, 0.0)
    for g in prep:
        om.apply_gate(g)

    def col0(g):
        return [mpmath.mpc(complex(g.u_hi[r, 0])) + mpmath.mpc(complex(g.u_lo[r, 0])) for r in range(2)]

    for q in ([2], [1, 3], [4, 0]):
        vec = [mpmath.mpc(1)]
        for x in q:
            c = col0(prep[x])
            vec = [a * b for a in vec for b in c]
        h, l = om.rdo(q)
        worst = 0
        for r in range(len(vec)):
            for c in range(len(vec)):
                want = vec[r] * mpmath.conj(vec[c])
                got = mpmath.mpc(mpmath.mpf(h[r, c].real) + mpmath.mpf(l[r, c].real),
                                 mpmath.mpf(h[r, c].imag) + mpmath.mpf(l[r, c].imag))
                worst = max(worst, abs(got - want))
        assert worst < 1e-30


def test_rdo_trace_one_exact_unitaries(oracle_mod):
    """Exactly unitary (dd) gates, no truncation: Tr rho = <Psi|Psi> = 1 to 256-bit
    rounding, for any list."""
    n = 8
    om = oracle_mod.OracleMPS(n, 64, 0.0)
    for layer in W.brickwork_dd(n, 6, 6):
        for g in layer:
            om.apply_gate(g)
    for q in ([3, 7], [0], [6, 1, 2]):
        h, l = om.rdo(q)
        tr = mpmath.fsum(mpmath.mpf(h[i, i].real) + mpmath.mpf(l[i, i].real) for i in range(len(h)))
        assert abs(tr - 1) < 1e-30


def test_rdo_invariants_truncated_state(oracle_mod):
    """A truncated state: every RDO is Hermitian and positive semidefinite, its trace
    is 1 up to the truncations (canonical form is kept only approximately when values
    are cut), and tracing out one qubit of RDO({a, b}) gives RDO({a})."""
    n = 9
    om = oracle_mod.OracleMPS(n, 8, 1e-6)
    for layer in W.brickwork(n, 8, 6):
        for g in layer:
            om.apply_gate(g)
    for q in ([3, 7], [0, 8], [4, 5]):
        h, l = om.rdo(q)
        rho = h + l
        assert np.max(np.abs(rho - rho.conj().T)) < 1e-15
        assert min(np.linalg.eigvalsh(rho)) > -1e-14
        assert abs(np.trace(rho).real - 1) < 1e-12
        ha, la = om.rdo([q[0]])
        red = (rho.reshape(2, 2, 2, 2)).trace(axis1=1, axis2=3)
        assert np.max(np.abs(red - (ha + la))) < 1e-15


def test_rdo_loaded_state_not_canonical(oracle_mod):
    """A loaded random (B, lambda) state that is not in canonical form: the RDO is the
    partial trace of the (unnormalised) state, not a canonical-form shortcut."""
    rng = W.rng_for(21)
    dims = [2, 4, 3, 2, 2]
    Bt, lam = W.random_mps_B(dims, rng, spread=1.0)
    n = len(dims) + 1
    om = oracle_mod.OracleMPS(n, 8, 0.0)
    om.load(Bt, lam)
    ah, al = om.amplitudes(all_bits(n))
    psi = ah + al
    for q in ([1, 4], [3], [5, 0, 2]):
        ref = partial_trace(psi, n, q)
        h, l = om.rdo(q)
        assert np.max(np.abs(h + l - ref)) < 1e-14 * max(1.0, np.max(np.abs(ref)))
