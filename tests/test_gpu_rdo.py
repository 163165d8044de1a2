"""Reduced density operators on the device (mps_rdo, mps_rdo_dd, mps_rdo_block; the
paper's RDO(list) and RDO_block) against the 256-bit oracle, the paper's printed values
and invariants.  Bars as for amplitudes: 1e-12 (FP64), 1e-26 (dd), absolute per entry."""
import os
import time

import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def flush(msg):
    print(msg, flush=True)


def oracle_state(oracle_mod, n, chi, eps, gates):
    om = oracle_mod.OracleMPS(n, chi, eps)
    for g in gates:
        om.apply_gate(g)
    return om


def dd_err(gh, gl, oh, ol):
    return float(np.max(np.abs((gh - oh) + (gl - ol))))


@pytest.mark.parametrize("prec,tol", [(0, 1e-15), (1, 1e-30)])
def test_paper_sample_rdo(B, prec, tol):
    flush(f"rdo paper sample prec={prec}")
    rows = [l.split() for l in open(os.path.join(GOLD, "paper_sample.txt")) if l.strip() and not l.startswith("#")]
    d = B.MPS(3, 8, 0.0, prec)
    for stage in ("initial", "final"):
        if stage == "final":
            d.apply_gates(W.paper_sample_circuit())
        sel = [r for r in rows if r[0] == stage]
        q = [int(x) for x in sel[0][1].split(",")]
        want = np.zeros((1 << len(q), 1 << len(q)))
        for r in sel:
            want[int(r[2], 2), int(r[3], 2)] = float(r[4])
        h, l = d.rdo(q, dd=True)
        assert np.max(np.abs((h - want) + l)) < tol
    assert np.allclose(d.rdo_block(0, 2), np.outer([2 ** -0.5, 0, 0, 0, 0, 2 ** -0.5, 0, 0],
                                                  [2 ** -0.5, 0, 0, 0, 0, 2 ** -0.5, 0, 0]), atol=1e-15)


LISTS = [[3], [2, 7], [9, 0, 5], [4, 5, 6], [1, 8, 3, 6]]


def test_rdo_fp64_vs_oracle(B, oracle_mod):
    flush("rdo fp64: n=10 brickwork depth 8 chi=32")
    n = 10
    gates = [g for layer in W.brickwork(n, 8, 12) for g in layer]
    om = oracle_state(oracle_mod, n, 32, 0.0, gates)
    d = B.MPS(n, 32, 0.0)
    d.apply_gates(gates)
    for q in LISTS:
        oh, ol = om.rdo(q)
        assert np.max(np.abs(d.rdo(q) - (oh + ol))) <= 1e-12


def test_rdo_dd_vs_oracle(B, oracle_mod):
    flush("rdo dd: n=10 brickwork_dd depth 8 chi=32")
    n = 10
    gates = [g for layer in W.brickwork_dd(n, 8, 12) for g in layer]
    om = oracle_state(oracle_mod, n, 32, 0.0, gates)
    d = B.MPS(n, 32, 0.0, B.MPS_PREC_DD)
    d.apply_gates(gates)
    for q in LISTS:
        oh, ol = om.rdo(q)
        gh, gl = d.rdo(q, dd=True)
        assert dd_err(gh, gl, oh, ol) <= 1e-26


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-26)])
def test_rdo_truncated_and_three_site(B, oracle_mod, prec, tol):
    flush(f"rdo truncated / mixed widths: n=10 chi=8 eps=1e-8 prec={prec}")
    n = 10
    gates = W.random_circuit_dd(n, 40, 31)
    if prec == 0:
        gates = [W.Gate(g.first, g.k, g.u_hi) for g in gates]
    om = oracle_state(oracle_mod, n, 8, 1e-8, gates)
    gaps = []
    om2 = oracle_mod.OracleMPS(n, 8, 1e-8)
    for g in gates:
        om2.apply_gate(g)
        gaps += [st["gap"] for st in om2.last_stats()]
    assert min(gaps) > (1e-10 if prec == 0 else 1e-20)
    d = B.MPS(n, 8, 1e-8, prec)
    d.apply_gates(gates)
    assert d.bond_dims() == om.bond_dims()
    for q in ([0, 9], [4, 2], [5, 6, 7]):
        oh, ol = om.rdo(q)
        gh, gl = d.rdo(q, dd=True)
        assert dd_err(gh, gl, oh, ol) <= tol


def test_rdo_loaded_state(B, oracle_mod):
    """A loaded (B, V) state that is not canonical: the device contracts exactly."""
    flush("rdo loaded state")
    rng = W.rng_for(33)
    dims = [2, 4, 8, 11, 8, 4, 2]
    Bt, lam = W.random_mps_B(dims, rng, spread=1.0)
    n = len(dims) + 1
    om = oracle_mod.OracleMPS(n, 16, 0.0)
    om.load(Bt, lam)
    for prec, tol in ((0, 1e-12), (1, 1e-26)):
        d = B.MPS(n, 16, 0.0, prec)
        d.load(Bt, lam)
        for q in ([3], [0, 7], [6, 2, 4]):
            oh, ol = om.rdo(q)
            gh, gl = d.rdo(q, dd=True)
            scale = max(1.0, float(np.max(np.abs(oh))))
            assert dd_err(gh, gl, oh, ol) <= tol * scale


def test_rdo_full_size_invariants(B):
    """The benchmark's saturated state (40 qubits, chi = 256): RDOs in the middle of the
    chain are Hermitian and positive semidefinite, consistent under a further partial
    trace, and all have the same trace <Psi|Psi> (within 1e-5 of 1: with chi_max
    binding, each truncation keeps the canonical form, hence the norm, only
    approximately); timed."""
    flush("rdo full size: n=40 chi=256")
    rng = W.rng_for(2)
    d = B.MPS(40, 256, 1e-12)
    t = 0
    while t < 40:
        d.apply_gates(W.brickwork_layer(40, t, rng))
        t += 1
        if min(d.bond_dims()[7:32]) == 256:
            break
    assert min(d.bond_dims()[7:32]) == 256
    d.set_option(B.MPS_OPT_KERNEL_TIMING, 1)
    d.kernel_time(7, reset=True)
    t0 = time.perf_counter()
    rho = d.rdo([19, 20])
    dt = time.perf_counter() - t0
    ms, _ = d.kernel_time(7)
    flush(f"rdo of 2 qubits at chi=256: {1e3 * dt:.1f} ms wall, {ms:.1f} ms device")
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-13
    assert min(np.linalg.eigvalsh(rho)) > -1e-12
    norm2 = np.trace(rho).real
    assert abs(norm2 - 1) < 1e-5
    r19 = d.rdo([19])
    for q in ([0], [39], [5, 33]):
        assert abs(np.trace(d.rdo(q)).real - norm2) < 1e-12
    assert np.max(np.abs(rho.reshape(2, 2, 2, 2).trace(axis1=1, axis2=3) - r19)) < 1e-12
    r4 = d.rdo([10, 19, 20, 30])
    red = np.einsum("aibcajdc->ibjd", r4.reshape([2] * 8)).reshape(4, 4)  # trace out qubits 10 and 30
    assert np.max(np.abs(red - rho)) < 1e-12


def test_rdo_errors_and_batch(B):
    d = B.MPS(4, 4, 0.0)
    for q in ([], [0, 0], [4], list(range(4)) + [0, 1, 2, 3]):
        with pytest.raises((B.MPSError, ValueError)):
            d.rdo(q)
    bt = B.Batch([3, 5], [4, 4], [0.0, 0.0])
    bt.run([0, 0], W.paper_sample_circuit())
    assert np.allclose(bt[0].rdo([0, 2]), 0.5 * np.array([[1, 0, 0, 1], [0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 1]]),
                       atol=1e-15)
    assert np.allclose(bt[1].rdo([4]), np.diag([1.0, 0.0]))
    bt.close()
