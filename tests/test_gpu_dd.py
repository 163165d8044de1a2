"""Parity of the double-double refined device path with the 256-bit oracle and with
closed forms.  Bar (the dd path's tolerance): |amplitude difference|
<= 1e-26 element by element; seeds whose truncation cut is degenerate at 1e-20
(relative gap) are excluded."""
import mpmath
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-26
mpmath.mp.prec = 256


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def flush(msg):
    print(msg, flush=True)


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def dd_diff(a_hi, a_lo, b_hi, b_lo):
    """max |(a_hi + a_lo) - (b_hi + b_lo)|; the hi difference of close values is exact."""
    return float(np.max(np.abs((a_hi - b_hi) + (a_lo - b_lo))))


def oracle_run(oracle_mod, n, chi, eps, gates):
    m = oracle_mod.OracleMPS(n, chi, eps)
    gaps = []
    for g in gates:
        m.apply_gate(g)
        gaps += [st["gap"] for st in m.last_stats()]
    return m, gaps


def dev_run(B, n, chi, eps, gates, batched=True):
    d = B.MPS(n, chi, eps, B.MPS_PREC_DD)
    if batched:
        d.apply_gates(gates)
    else:
        for g in gates:
            d.apply_gate(g)
    return d


def test_brickwork_dd_gates_vs_oracle(B, oracle_mod):
    """10 qubits, depth-10 brickwork of exactly unitary (dd) Haar gates, no truncation."""
    flush("dd brickwork: n=10 depth=10 chi=32 seed=1")
    n = 10
    gates = [g for layer in W.brickwork_dd(n, 10, 1) for g in layer]
    om, _ = oracle_run(oracle_mod, n, 32, 0.0, gates)
    d = dev_run(B, n, 32, 0.0, gates)
    assert d.bond_dims() == om.bond_dims()
    bits = all_bits(n)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL
    for b in range(n - 1):
        lh, ll = d.schmidt_dd(b)
        oh2, ol2 = om.schmidt(b)
        assert dd_diff(lh, ll, oh2, ol2) <= TOL


def test_dd_stream_bit_identical(B):
    """The dd work on its own stream (the default) or on the handle's stream: the same
    kernels on the same inputs, so the same state bit for bit (truncated brickwork)."""
    flush("dd stream on/off: n=12 depth=12 chi=16 eps=1e-10 seed=7")
    n = 12
    gates = [g for layer in W.brickwork_dd(n, 12, 7) for g in layer]
    out = []
    for on in (0, 1):
        d = B.MPS(n, 16, 1e-10, B.MPS_PREC_DD)
        d.set_option(B.MPS_OPT_DD_STREAM, on)
        d.apply_gates(gates)
        out.append((d.bond_dims(), d.amplitudes(all_bits(n), dd=True), [d.schmidt_dd(b) for b in range(n - 1)]))
        d.close()
    (d0, a0, s0), (d1, a1, s1) = out
    assert d0 == d1
    assert all(np.array_equal(x, y) for x, y in zip(a0, a1))
    assert all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) for x, y in zip(s0, s1))


def test_config1_fp64_gates_on_dd_path(B, oracle_mod):
    """Config-1 circuit (binary64 Haar gates taken as exact values) on the dd path."""
    flush("dd config1: n=10 depth=10 chi=32 seed=1 (binary64 gates)")
    n = 10
    gates = [g for layer in W.brickwork(n, 10, 1) for g in layer]
    om, _ = oracle_run(oracle_mod, n, 32, 0.0, gates)
    d = dev_run(B, n, 32, 0.0, gates, batched=False)
    bits = all_bits(n)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL


@pytest.mark.parametrize("n,x", [(6, 37), (9, 300)])
def test_qft_basis_state_closed_form(B, n, x):
    """QFT of a basis state: c(y) = 2^{-n/2} exp(2 pi i x y / 2^n), dd gates."""
    flush(f"dd qft basis: n={n} x={x}")
    bits = [(x >> (n - 1 - q)) & 1 for q in range(n)]
    d = dev_run(B, n, 1 << n, 1e-24, W.basis_prep(bits) + W.qft_lnn_circuit(n))
    assert d.bond_dims() == [1] * (n - 1)
    ys = all_bits(n)
    gh, gl = d.amplitudes(ys, dd=True)
    worst = 0.0
    for y in range(1 << n):
        want = mpmath.mpf(2) ** (-mpmath.mpf(n) / 2) * mpmath.expj(2 * mpmath.pi * x * y / mpmath.mpf(2 ** n))
        got = mpmath.mpc(mpmath.mpf(gh[y].real) + mpmath.mpf(gl[y].real), mpmath.mpf(gh[y].imag) + mpmath.mpf(gl[y].imag))
        worst = max(worst, float(abs(got - want)))
    assert worst <= TOL


def test_qft_product_state_closed_form(B):
    """QFT of a seeded random product state (no truncation): the product formula."""
    flush("dd qft product: n=8 seed=5")
    n = 8
    prep = W.product_state_prep(n, 5)
    d = dev_run(B, n, 1 << n, 0.0, prep + W.qft_lnn_circuit(n))
    ys = all_bits(n)
    gh, gl = d.amplitudes(ys, dd=True)
    worst = 0.0
    for y in range(1 << n):
        c = mpmath.mpf(2) ** (-mpmath.mpf(n) / 2)
        for q, g in enumerate(prep):
            a = mpmath.mpc(g.u_hi[0, 0]) + mpmath.mpc(g.u_lo[0, 0])
            b = mpmath.mpc(g.u_hi[1, 0]) + mpmath.mpc(g.u_lo[1, 0])
            mod = 1 << (q + 1)
            c *= a + b * mpmath.expj(2 * mpmath.pi * (y % mod) / mod)
        got = mpmath.mpc(mpmath.mpf(gh[y].real) + mpmath.mpf(gl[y].real), mpmath.mpf(gh[y].imag) + mpmath.mpf(gl[y].imag))
        worst = max(worst, float(abs(got - c)))
    assert worst <= TOL


@pytest.mark.parametrize("chi,eps", [(8, 0.0), (64, 1e-4)])
def test_truncation_dd_vs_oracle(B, oracle_mod, chi, eps):
    flush(f"dd truncation: n=12 depth=12 chi={chi} eps={eps} seed=5")
    n = 12
    gates = [g for layer in W.brickwork_dd(n, 12, 5) for g in layer]
    om, gaps = oracle_run(oracle_mod, n, chi, eps, gates)
    assert min(gaps) > 1e-20
    d = dev_run(B, n, chi, eps, gates)
    assert d.bond_dims() == om.bond_dims()
    bits = W.bitstrings(n, 400, 6)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL


def test_loaded_state_dd(B, oracle_mod):
    """A random (B, lambda) state (binary64 values) and one dd gate at a bond whose
    theta (74 x 74) spans several 32-wide dd tiles with a ragged tail."""
    flush("dd loaded: dims with 37, seed=8")
    rng = W.rng_for(8)
    dims = [2, 4, 8, 16, 32, 37, 37, 37, 32, 16, 8, 4, 2]
    Bt, lam = W.random_mps_B(dims, rng, spread=3.0)
    n = len(dims) + 1
    hi, lo = W.haar_unitary_dd(4, rng)
    om = oracle_mod.OracleMPS(n, 64, 0.0)
    om.load(Bt, lam)
    om.apply(6, 2, hi, lo)
    d = B.MPS(n, 64, 0.0, B.MPS_PREC_DD)
    d.load(Bt, lam)
    d.apply(6, 2, hi, lo)
    assert d.bond_dims() == om.bond_dims()
    bits = W.bitstrings(n, 300, 9)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    scale = max(1.0, float(np.max(np.abs(oh))))
    assert dd_diff(gh, gl, oh, ol) <= TOL * scale
    lh, ll = d.schmidt_dd(6)
    oh2, ol2 = om.schmidt(6)
    assert dd_diff(lh, ll, oh2, ol2) <= TOL


def test_mixed_widths_dd(B, oracle_mod):
    flush("dd mixed: n=9 gates=60 seed=7")
    n = 9
    gates = W.random_circuit_dd(n, 60, 7, ks=(1, 2))
    om, _ = oracle_run(oracle_mod, n, 64, 0.0, gates)
    d = dev_run(B, n, 64, 0.0, gates)
    bits = all_bits(n)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL


def test_ghz_dd(B):
    flush("dd ghz: n=16")
    n = 16
    d = dev_run(B, n, 4, 0.0, W.ghz_circuit(n))
    s = mpmath.mpf(1) / mpmath.sqrt(2)
    for bits in ([0] * n, [1] * n):
        h, l = B.mps_amplitude_dd(d.h, bits)
        assert abs(mpmath.mpf(h.real) + mpmath.mpf(l.real) - s) < 1e-30


def test_paper_sample_three_site_dd(B):
    flush("dd paper sample (k=3)")
    d = B.MPS(3, 8, 0.0, B.MPS_PREC_DD)
    d.apply_gates(W.paper_sample_circuit())
    gh, gl = d.amplitudes(all_bits(3), dd=True)
    s = mpmath.mpf(1) / mpmath.sqrt(2)
    for x in range(8):
        want = s if x in (0, 5) else 0
        got = mpmath.mpc(mpmath.mpf(gh[x].real) + mpmath.mpf(gl[x].real), mpmath.mpf(gh[x].imag) + mpmath.mpf(gl[x].imag))
        assert abs(got - want) < 1e-30


def test_three_site_dd_vs_oracle(B, oracle_mod):
    flush("dd mixed k<=3: n=7 gates=40 seed=21")
    n = 7
    gates = W.random_circuit_dd(n, 40, 21)
    om, _ = oracle_run(oracle_mod, n, 128, 0.0, gates)
    d = dev_run(B, n, 128, 0.0, gates)
    bits = all_bits(n)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL


def test_triples_truncated_dd_vs_oracle(B, oracle_mod):
    flush("dd triples: n=10 count=30 chi=16 eps=1e-14 seed=3")
    n = 10
    gates = W.random_triples(n, 30, 3)
    om, gaps = oracle_run(oracle_mod, n, 16, 1e-14, gates)
    assert min(gaps) > 1e-20
    d = dev_run(B, n, 16, 1e-14, gates)
    assert d.bond_dims() == om.bond_dims()
    bits = W.bitstrings(n, 300, 4)
    gh, gl = d.amplitudes(bits, dd=True)
    oh, ol = om.amplitudes(bits)
    assert dd_diff(gh, gl, oh, ol) <= TOL
