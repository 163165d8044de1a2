"""Gate fusion in mps_apply_gates / mps_batch_run (MPS_OPT_FUSE): single-site gates
are multiplied into the latest earlier gate touching their site, or into a later gate
on it.  The fused runs must match the oracle applying every gate separately (FP64
1e-12, dd 1e-26 per amplitude, also with truncation), take no single-site launches
when every U(2) can be absorbed, and batches must still equal standalone runs."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL, TOL_DD = 1e-12, 1e-26


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def flush(msg):
    print(msg, flush=True)


def fusable_circuit(n, seed, dd):
    """Layers of: U(2) on every qubit, U(4) on even bonds, the same U(4) pairs again,
    U(2) on the odd qubits, U(8) on sites 1..3 then a U(4) and a U(2) inside it."""
    rng = W.rng_for(seed)

    def u(d):
        if dd:
            return W.haar_unitary_dd(d, rng)
        return W.haar_unitary(d, rng), None

    gates = []
    for rep in range(2):
        for q in range(n):
            gates.append(W.Gate(q, 1, *u(2)))
        for s in range(0, n - 1, 2):
            gates.append(W.Gate(s, 2, *u(4)))
        for s in range(0, n - 1, 2):
            gates.append(W.Gate(s, 2, *u(4)))
        for q in range(1, n, 2):
            gates.append(W.Gate(q, 1, *u(2)))
        gates.append(W.Gate(1, 3, *u(8)))
        gates.append(W.Gate(2, 2, *u(4)))
        gates.append(W.Gate(3, 1, *u(2)))
        for s in range(1, n - 1, 2):
            gates.append(W.Gate(s, 2, *u(4)))
    return gates


@pytest.mark.parametrize("dd,chi", [(False, 64), (True, 64), (False, 6), (True, 6)])
def test_fused_vs_oracle(B, oracle_mod, dd, chi):
    flush(f"fusion: n=8 chi={chi} seed=51 dd={dd}")
    n = 8
    gates = fusable_circuit(n, 51, dd)
    om = oracle_mod.OracleMPS(n, chi, 0.0)
    for g in gates:
        om.apply_gate(g)
    bits = all_bits(n)
    oh, ol = om.amplitudes(bits)
    launches = {}
    for fuse in (1, 0):
        d = B.MPS(n, chi, 0.0, B.MPS_PREC_DD if dd else B.MPS_PREC_FP64)
        d.set_option(B.MPS_OPT_FUSE, fuse)
        d.set_option(B.MPS_OPT_KERNEL_TIMING, 1)
        d.apply_gates(gates)
        assert d.bond_dims() == om.bond_dims()
        if dd:
            gh, gl = d.amplitudes(bits, dd=True)
            assert np.max(np.abs((gh - oh) + (gl - ol))) <= TOL_DD
        else:
            assert np.max(np.abs(d.amplitudes(bits) - (oh + ol))) <= TOL
        launches[fuse] = d.kernel_time(4)[1]  # single-site gate launches
    assert launches[0] > 0 and launches[1] == 0


def test_fused_batch_equals_standalone(B):
    flush("fusion: batch of 3 vs standalone")
    specs = [(6, 16, 0.0, 52), (8, 8, 1e-14, 53), (7, 32, 0.0, 54)]
    circs = [fusable_circuit(n, seed, False) for n, _, _, seed in specs]
    bt = B.Batch([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs])
    order = [(i, g) for i, c in enumerate(circs) for g in c]
    bt.run([i for i, _ in order], [g for _, g in order])
    for i, (n, chi, eps, _) in enumerate(specs):
        alone = B.MPS(n, chi, eps)
        alone.apply_gates(circs[i])
        assert bt[i].bond_dims() == alone.bond_dims()
        assert np.array_equal(bt[i].amplitudes(all_bits(n)), alone.amplitudes(all_bits(n)))
        alone.close()
