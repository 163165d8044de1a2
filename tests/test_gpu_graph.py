"""Launch modes of the Jacobi sweeps: one or two sweeps a scheduler tick
(MPS_OPT_TICK_SWEEPS) and stream launches or replayed HIP graphs (MPS_OPT_GRAPH).
The convergence test stays on the device (an update whose last sweep rotated
nothing leaves every later sweep's blocks at once), so every mode must give the
same state bit for bit as the default one: standalone circuits with tall, square
and wide thetas, QR-preconditioned and split-step launches, FP64 and dd, and a
batch of independent circuits; the graph counter must show replays."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [(1, 0), (2, 0), (1, 1), (2, 1)]  # (sweeps per tick, graph)


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def snapshot(m, n, dd):
    bits = W.bitstrings(n, 48, 7)
    out = [np.array(m.bond_dims())]
    out += list(m.amplitudes(bits, dd=True)) if dd else [m.amplitudes(bits)]
    for b in range(n - 1):
        out += list(m.schmidt_dd(b)) if dd else [m.schmidt(b)]
    return out


def same(a, b):
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("dd", [False, True])
def test_modes_standalone_bit_identical(B, dd):
    # 14 qubits, chi_max 48: bonds grow to 48 (thetas up to 96 x 96, QR from N = 64),
    # wide thetas on the left half, 1..7 updates a tick (split step at <= 4)
    n, chi, depth, seed = 14, 48, 10, 61
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    gates = [g for layer in W.brickwork(n, depth, seed) for g in layer]
    ref = None
    for ts, gr in MODES:
        print(f"graph modes: n={n} chi={chi} depth={depth} seed={seed} dd={dd} tick_sweeps={ts} graph={gr}",
              flush=True)
        m = B.MPS(n, chi, 1e-13, prec)
        m.set_option(B.MPS_OPT_TICK_SWEEPS, ts)
        m.set_option(B.MPS_OPT_GRAPH, gr)
        m.kernel_time(B.COUNTER_GRAPHS, reset=True)
        m.apply_gates(gates)
        built, replays = m.kernel_time(B.COUNTER_GRAPHS)
        if gr:
            assert replays > 0 and 0 < built <= replays
        else:
            assert replays == 0
        snap = snapshot(m, n, dd)
        m.close()
        if ref is None:
            ref = snap
        else:
            assert same(ref, snap), (ts, gr)


@pytest.mark.parametrize("dd", [False, True])
def test_modes_three_site_bit_identical(B, dd):
    n, chi, seed = 10, 24, 62
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    gates = W.random_circuit_dd(n, 30, seed)
    if not dd:
        gates = [W.Gate(g.first, g.k, g.u_hi) for g in gates]
    ref = None
    for ts, gr in MODES:
        print(f"graph modes, mixed U(2)/U(4)/U(8): n={n} chi={chi} seed={seed} dd={dd} tick_sweeps={ts} graph={gr}",
              flush=True)
        m = B.MPS(n, chi, 1e-12, prec)
        m.set_option(B.MPS_OPT_TICK_SWEEPS, ts)
        m.set_option(B.MPS_OPT_GRAPH, gr)
        m.apply_gates(gates)
        snap = snapshot(m, n, dd)
        m.close()
        if ref is None:
            ref = snap
        else:
            assert same(ref, snap), (ts, gr)


def test_modes_batch_bit_identical(B):
    rng = W.rng_for(63)
    shapes = [(12, 32, 1e-12), (9, 16, 0.0), (16, 64, 1e-12), (7, 8, 0.0)]
    circs = [[g for layer in W.brickwork(n, 8, int(rng.integers(1 << 30))) for g in layer] for n, _, _ in shapes]
    circ, gates = [], []
    for j in range(max(len(c) for c in circs)):
        for i, c in enumerate(circs):
            if j < len(c):
                circ.append(i)
                gates.append(c[j])
    ref = None
    for ts, gr in MODES:
        print(f"graph modes, batch of 4 circuits: tick_sweeps={ts} graph={gr}", flush=True)
        bt = B.Batch([s[0] for s in shapes], [s[1] for s in shapes], [s[2] for s in shapes], B.MPS_PREC_FP64)
        bt.set_option(B.MPS_OPT_TICK_SWEEPS, ts)
        bt.set_option(B.MPS_OPT_GRAPH, gr)
        bt.run(circ, gates)
        snap = [x for i, (n, _, _) in enumerate(shapes) for x in snapshot(bt[i], n, False)]
        bt.close()
        if ref is None:
            ref = snap
        else:
            assert same(ref, snap), (ts, gr)


def test_option_values_checked(B):
    m = B.MPS(4, 4, 0.0)
    for key, bad in ((B.MPS_OPT_TICK_SWEEPS, 3), (B.MPS_OPT_TICK_SWEEPS, 0), (B.MPS_OPT_GRAPH, 2)):
        with pytest.raises(B.MPSError):
            m.set_option(key, bad)
    m.close()
