"""Pins of the oracle's two-qubit gates on arbitrary qubits (OracleMPS.apply_gate2;
the paper's applyU(U, q0, q1), Section 3.2): against the dense state vector, whose
gate application takes any qubit list, and against the paper's printed RDOs."""
import os

import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


@pytest.mark.parametrize("pairs", [[(0, 2), (4, 1), (5, 0)], [(3, 4), (2, 1), (0, 5), (5, 2)]])
def test_gate2_equals_state_vector(oracle_mod, pairs):
    """6 qubits, a brickwork layer then Haar U(4) on the listed (q0, q1) pairs
    (adjacent and not, either order), no truncation: every amplitude equals the
    state vector's at 256 bits (SWAP routing is exact without truncation)."""
    n = 6
    rng = W.rng_for(11)
    om = oracle_mod.OracleMPS(n, 64, 0.0)
    sv = oracle_mod.OracleSV(n)
    # dd-exact unitaries, so that the MPS's renormalisation after each split changes
    # nothing at 256 bits
    for s in range(0, n - 1, 2):
        uh, ul = W.haar_unitary_dd(4, rng)
        om.apply(s, 2, uh, ul)
        sv.apply([s, s + 1], uh, ul)
    for q0, q1 in pairs:
        uh, ul = W.haar_unitary_dd(4, rng)
        om.apply_gate2(q0, q1, uh, ul)
        sv.apply([q0, q1], uh, ul)
    mh, ml = om.amplitudes(all_bits(n))
    sh, sl = sv.amplitudes()
    assert np.max(np.abs((mh - sh) + (ml - sl))) < 1e-28


def test_gate2_dd_gate_planes(oracle_mod):
    """A dd gate (hi + lo) on non-adjacent qubits: the lo plane reaches the state
    (the result differs from the hi-only gate by the lo part's first-order term)."""
    n = 5
    rng = W.rng_for(12)
    u_hi, u_lo = W.haar_unitary_dd(4, rng)
    layer = [W.haar_unitary_dd(4, rng) for _ in range(2)]
    res = []
    for lo in (None, u_lo):
        om = oracle_mod.OracleMPS(n, 32, 0.0)
        for i, (gh, gl) in enumerate(layer):
            om.apply(2 * i, 2, gh, gl)
        om.apply_gate2(3, 0, u_hi, lo)
        mh, ml = om.amplitudes(all_bits(n))
        res.append((mh, ml))
    sv = oracle_mod.OracleSV(n)
    for i, (gh, gl) in enumerate(layer):
        sv.apply([2 * i, 2 * i + 1], gh, gl)
    sv.apply([3, 0], u_hi, u_lo)
    sh, sl = sv.amplitudes()
    (ah, al), (bh, bl) = res
    assert np.max(np.abs((bh - sh) + (bl - sl))) < 1e-28
    # without the lo plane the gate is off by |u_lo| ~ 1e-17 (then renormalised)
    assert 1e-19 < np.max(np.abs((ah - bh) + (al - bl))) < 1e-15


def test_gate2_paper_example_printed_rdo(oracle_mod):
    """The paper's example with the CNOT applied as applyU(CNOT, 0, 2): RDO of qubits
    {0, 2} as printed."""
    rows = [l.split() for l in open(os.path.join(GOLD, "paper_sample.txt")) if l.strip() and not l.startswith("#")]
    sel = [r for r in rows if r[0] == "final"]
    want = np.zeros((4, 4))
    for r in sel:
        want[int(r[2], 2), int(r[3], 2)] = float(r[4])
    m = oracle_mod.OracleMPS(3, 8, 0.0)
    m.apply(0, 1, W.hadamard())
    m.apply_gate2(0, 2, W.cnot())
    h, l = m.rdo([0, 2])
    assert np.max(np.abs((h - want) + l)) < 1e-30


def test_gate2_argument_errors(oracle_mod):
    m = oracle_mod.OracleMPS(4, 8, 0.0)
    for q0, q1 in [(1, 1), (-1, 2), (0, 4)]:
        with pytest.raises(ValueError):
            m.apply_gate2(q0, q1, np.eye(4))
