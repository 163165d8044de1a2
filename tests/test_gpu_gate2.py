"""Two-qubit gates on any two qubits (mps_apply_gate2, the paper's applyU(U, q0, q1),
Section 3.2) through the C ABI against the oracle's own routing of the same gates:
FP64 within 1e-12 and dd within 1e-26 per amplitude, without and with truncation,
the paper's example with the CNOT on qubits 0 and 2, and argument errors."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL, TOL_DD = 1e-12, 1e-26
PAIRS = [(0, 2), (5, 1), (3, 4), (7, 0), (2, 1), (6, 3), (1, 7)]


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def flush(msg):
    print(msg, flush=True)


def circuit(n, seed, dd):
    """A layer of U(4) on bonds 0, 2, ... then Haar U(4) on PAIRS (adjacent and not,
    either order); dd: exactly unitary (hi, lo) gates."""
    rng = W.rng_for(seed)
    mk = (lambda: W.haar_unitary_dd(4, rng)) if dd else (lambda: (W.haar_unitary(4, rng), None))
    layer = [(s, *mk()) for s in range(0, n - 1, 2)]
    pairs = [(q0, q1, *mk()) for q0, q1 in PAIRS if max(q0, q1) < n]
    return layer, pairs


def run_both(B, oracle_mod, n, chi, eps, seed, dd):
    layer, pairs = circuit(n, seed, dd)
    om = oracle_mod.OracleMPS(n, chi, eps)
    dev = B.MPS(n, chi, eps, B.MPS_PREC_DD if dd else B.MPS_PREC_FP64)
    for s, uh, ul in layer:
        om.apply(s, 2, uh, ul)
        dev.apply(s, 2, uh, ul)
    for q0, q1, uh, ul in pairs:
        om.apply_gate2(q0, q1, uh, ul)
        dev.apply_gate2(q0, q1, uh, ul)
    return om, dev


@pytest.mark.parametrize("dd", [False, True])
def test_gate2_vs_oracle_untruncated(B, oracle_mod, dd):
    flush(f"gate2 untruncated: n=8 chi=64 seed=31 dd={dd}")
    n = 8
    om, dev = run_both(B, oracle_mod, n, 64, 0.0, 31, dd)
    assert dev.bond_dims() == om.bond_dims()
    bits = all_bits(n)
    oh, ol = om.amplitudes(bits)
    if dd:
        gh, gl = dev.amplitudes(bits, dd=True)
        assert np.max(np.abs((gh - oh) + (gl - ol))) <= TOL_DD
    else:
        assert np.max(np.abs(dev.amplitudes(bits) - (oh + ol))) <= TOL


@pytest.mark.parametrize("dd", [False, True])
def test_gate2_vs_oracle_truncated(B, oracle_mod, dd):
    """chi_max 6 and eps 1e-14 on 8 qubits: every SWAP and the U(8) truncate."""
    flush(f"gate2 truncated: n=8 chi=6 seed=32 dd={dd}")
    n = 8
    om, dev = run_both(B, oracle_mod, n, 6, 1e-14, 32, dd)
    assert dev.bond_dims() == om.bond_dims()
    assert max(om.bond_dims()) == 6
    bits = all_bits(n)
    oh, ol = om.amplitudes(bits)
    if dd:
        gh, gl = dev.amplitudes(bits, dd=True)
        assert np.max(np.abs((gh - oh) + (gl - ol))) <= TOL_DD
    else:
        assert np.max(np.abs(dev.amplitudes(bits) - (oh + ol))) <= TOL


def test_gate2_paper_example(B):
    """|000>, H(0), applyU(CNOT, 0, 2): the Bell pair on qubits 0 and 2 (the paper's
    printed RDO), and qubit 1 untouched."""
    flush("gate2 paper example")
    d = B.MPS(3, 8, 0.0)
    d.apply(0, 1, W.hadamard())
    d.apply_gate2(0, 2, W.cnot())
    s = 2 ** -0.5
    amps = d.amplitudes(all_bits(3))
    assert np.max(np.abs(amps - np.array([s, 0, 0, 0, 0, s, 0, 0]))) < 1e-15
    rho = d.rdo([0, 2])
    want = np.zeros((4, 4))
    want[0, 0] = want[0, 3] = want[3, 0] = want[3, 3] = 0.5
    assert np.max(np.abs(rho - want)) < 1e-15
    # the same gate with its qubits listed the other way round: CNOT with control 2
    d2 = B.MPS(3, 8, 0.0)
    d2.apply(2, 1, W.hadamard())
    d2.apply_gate2(2, 0, W.cnot())
    assert np.max(np.abs(d2.amplitudes(all_bits(3)) - np.array([s, 0, 0, 0, 0, s, 0, 0]))) < 1e-15


def test_gate2_errors(B):
    d = B.MPS(4, 8, 0.0)
    for q0, q1 in [(1, 1), (-1, 2), (0, 4)]:
        with pytest.raises(B.MPSError) as ei:
            d.apply_gate2(q0, q1, np.eye(4))
        assert ei.value.code == B.MPS_EINVAL
    bad = np.eye(4, dtype=np.complex128)
    bad[1, 2] = np.nan
    with pytest.raises(B.MPSError) as ei:
        d.apply_gate2(0, 3, bad)
    assert ei.value.code == B.MPS_ENONFINITE
    assert d.bond_dims() == [1, 1, 1]
