"""The double-double path's fallbacks against the 256-bit oracle (bar 1e-26 on every
amplitude and Schmidt value):

* refinement switched off (MPS_OPT_DD_REFINE = 0): every update goes from the FP64
  Jacobi straight to the pairwise dd Jacobi polish;
* exactly degenerate Schmidt spectra: a GHZ state (two equal Schmidt values on every
  bond) under layers of product gates u (x) v on every pair, which leave each bond's
  spectrum exactly degenerate.  The simultaneous first-order correction of the
  refinement divides by the gap of a pair, so such pairs void a pass and send the
  update to the polish; the passes queued after a void one must change nothing.
  Gates are exact in dd (entries rounded from 256-bit values)."""
import mpmath
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-26


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def dd_diff(a_hi, a_lo, b_hi, b_lo):
    return float(np.max(np.abs((a_hi - b_hi) + (a_lo - b_lo))))


def dd_gate(first, k, m):
    """Gate from a matrix of 256-bit complex entries, rounded to (hi, lo)."""
    d = 1 << k
    hi = np.zeros((d, d), dtype=np.complex128)
    lo = np.zeros((d, d), dtype=np.complex128)
    for r in range(d):
        for c in range(d):
            z = mpmath.mpc(m[r][c])
            rh, rl = W.dd_split(z.real)
            ih, il = W.dd_split(z.imag)
            hi[r, c], lo[r, c] = complex(rh, ih), complex(rl, il)
    return W.Gate(first, k, hi, lo)


def haar2_mp(rng):
    """A random U(2) at 256 bits: [[a, -conj(b)], [b, conj(a)]] times a phase."""
    t = mpmath.acos(mpmath.mpf(float(rng.uniform(-1.0, 1.0))))
    phi, chi = (mpmath.mpf(float(rng.uniform(0.0, 2.0 * np.pi))) for _ in range(2))
    a = mpmath.cos(t / 2)
    b = mpmath.expj(phi) * mpmath.sin(t / 2)
    g = mpmath.expj(chi)
    return [[g * a, -g * mpmath.conj(b)], [g * b, g * mpmath.conj(a)]]


def degenerate_circuit(n, layers, seed):
    with mpmath.workprec(256):
        s = 1 / mpmath.sqrt(2)
        gates = [dd_gate(0, 1, [[s, s], [s, -s]])]
        gates += [W.Gate(q, 2, W.cnot()) for q in range(n - 1)]
        rng = W.rng_for(seed)
        for t in range(layers):
            for q in range(t % 2, n - 1, 2):
                u, v = haar2_mp(rng), haar2_mp(rng)
                kron = [[u[r >> 1][c >> 1] * v[r & 1][c & 1] for c in range(4)] for r in range(4)]
                gates.append(dd_gate(q, 2, kron))
    return gates


def run_both(B, oracle_mod, n, chi, gates, refine):
    om = oracle_mod.OracleMPS(n, chi, 0.0)
    for g in gates:
        om.apply_gate(g)
    d = B.MPS(n, chi, 0.0, B.MPS_PREC_DD)
    d.set_option(B.MPS_OPT_DD_REFINE, refine)
    d.set_option(B.MPS_OPT_KERNEL_TIMING, 1)
    d.apply_gates(gates)
    dd_sweeps = d.kernel_time(B.COUNTER_SWEEPS_DD)[1]
    gh, gl = d.amplitudes(all_bits(n), dd=True)
    oh, ol = om.amplitudes(all_bits(n))
    err = dd_diff(gh, gl, oh, ol)
    # Schmidt values: the oracle keeps the values a rank-deficient theta leaves at
    # ~1e-33, below the device's rank floor (2^-96 relative); they compare as zeros
    serr = 0.0
    for b in range(n - 1):
        lh, ll = d.schmidt_dd(b)
        oh2, ol2 = om.schmidt(b)
        assert len(lh) <= len(oh2)
        pad = len(oh2) - len(lh)
        lh, ll = np.concatenate([lh, np.zeros(pad)]), np.concatenate([ll, np.zeros(pad)])
        serr = max(serr, dd_diff(lh, ll, oh2, ol2))
    d.close()
    return err, serr, dd_sweeps


def test_polish_only_vs_oracle(B, oracle_mod):
    print("dd polish only (refinement off): n=10 brickwork depth 6 chi=32 seed 3", flush=True)
    n = 10
    gates = [g for layer in W.brickwork_dd(n, 6, 3) for g in layer]
    err, serr, sw = run_both(B, oracle_mod, n, 32, gates, 0)
    print(f"  amplitude error {err:.3e}, Schmidt error {serr:.3e}, dd sweeps {sw:.0f}", flush=True)
    assert err <= TOL and serr <= TOL


@pytest.mark.parametrize("refine", [1, 0])
def test_degenerate_spectra_vs_oracle(B, oracle_mod, refine):
    print(f"dd degenerate spectra: GHZ n=10 + 6 layers of product gates, refine={refine}", flush=True)
    n = 10
    gates = degenerate_circuit(n, 6, 11)
    err, serr, sw = run_both(B, oracle_mod, n, 8, gates, refine)
    print(f"  amplitude error {err:.3e}, Schmidt error {serr:.3e}, dd passes + polish sweeps {sw:.0f}", flush=True)
    assert err <= TOL and serr <= TOL
