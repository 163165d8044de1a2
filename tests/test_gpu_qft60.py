"""Configuration 5 at full size: a 60-qubit random product state (single-qubit
preparation gates [[a, -conj(b)], [b, conj(a)]], seed 5, exact in dd) followed by the
quantum Fourier transform as a nearest-neighbour network (60 Hadamards and 1770 fused
SWAP-phase U(4) gates), on the dd path with chi_max = 1024.

The transform of a product state factorises over the bits, so every output amplitude
has a closed form, c(y) = 2^{-n/2} prod_q (a_q + b_q exp(2 pi i (y mod 2^{q+1}) / 2^{q+1})),
evaluated here at 256 bits for 64 sampled bitstrings:
* eps = 0: the state is exact up to rounding (the bond dims stay far below chi_max, and
  the rank floor drops only values below 2^-96 of the largest): amplitudes within 1e-26
  absolute, and within 1e-24 of the largest sampled amplitude (they are all ~2^-30);
* eps = 1e-24, the configuration's own truncation, gates applied one at a time: a
  renormalised truncation moves the state by at most sqrt(2 w) in norm (w its relative
  discarded weight, reported per split), the gates preserve distances, so every
  amplitude lies within the sum of sqrt(2 w_i) of the closed form; and, against the
  256-bit oracle run of the same gates with the same truncation rule
  (tests/golden/qft60_eps.json, written by tests/golden/make_golden.py qft60_eps), the
  same bond dims everywhere and the 64 amplitudes within 1e-26.  The oracle run's
  smallest relative gap at a cut (2.4e-13) and smallest relative distance of an eps
  decision from its boundary (0.23) keep every cut far from the ambiguous cases, so
  both sides keep the same subspaces."""
import json
import math
import os

import mpmath
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

N, CHI, SEED = 60, 1024, 5
TOL = 1e-26
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "qft60_eps.json")


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


@pytest.fixture(scope="module")
def case():
    prep = W.product_state_prep(N, SEED)
    circ = prep + W.qft_lnn_circuit(N)
    bits = np.random.default_rng(55).integers(0, 2, (64, N)).astype(np.uint8)
    want = []
    with mpmath.workprec(256):
        for row in bits:
            y = int("".join(str(int(b)) for b in row), 2)  # qubit 0 most significant
            c = mpmath.mpf(2) ** (-mpmath.mpf(N) / 2)
            for q, g in enumerate(prep):
                a = mpmath.mpc(g.u_hi[0, 0]) + mpmath.mpc(g.u_lo[0, 0])
                b = mpmath.mpc(g.u_hi[1, 0]) + mpmath.mpc(g.u_lo[1, 0])
                mod = 1 << (q + 1)
                c *= a + b * mpmath.expj(2 * mpmath.pi * (y % mod) / mod)
            want.append(c)
    return circ, bits, want


def worst_error(d, bits, want):
    gh, gl = d.amplitudes(bits, dd=True)
    worst = 0.0
    with mpmath.workprec(256):
        for i, c in enumerate(want):
            got = mpmath.mpc(mpmath.mpf(gh[i].real) + mpmath.mpf(gl[i].real),
                             mpmath.mpf(gh[i].imag) + mpmath.mpf(gl[i].imag))
            worst = max(worst, float(abs(got - c)))
    return worst


def test_qft60_exact(B, case):
    circ, bits, want = case
    print(f"config 5: n={N} chi={CHI} eps=0 seed={SEED}, {len(circ)} gates", flush=True)
    d = B.MPS(N, CHI, 0.0, B.MPS_PREC_DD)
    d.apply_gates(circ)
    assert max(d.bond_dims()) < CHI
    worst = worst_error(d, bits, want)
    scale = max(float(abs(c)) for c in want)
    print(f"  max bond dim {max(d.bond_dims())}, worst |amplitude - closed form| {worst:.3e}", flush=True)
    assert worst <= TOL
    assert worst <= 1e-24 * scale
    d.close()


def test_qft60_truncated_vs_oracle_and_bound(B, case):
    circ, bits, want = case
    print(f"config 5: n={N} chi={CHI} eps=1e-24 seed={SEED}, gate by gate", flush=True)
    d = B.MPS(N, CHI, 1e-24, B.MPS_PREC_DD)
    bound = 0.0
    for g in circ:
        d.apply(g.first, g.k, g.u_hi, g.u_lo)
        st = d.stats()
        if st["splits"] > 0:
            assert 0.0 <= st["w"] <= 1e-24 * (1 + 1e-12)
            bound += math.sqrt(2.0 * st["w"])
    worst = worst_error(d, bits, want)
    print(f"  max bond dim {max(d.bond_dims())}, worst {worst:.3e}, bound {bound:.3e}", flush=True)
    assert worst <= bound + TOL
    # the oracle's run of the same gates with the same truncation
    g = json.load(open(GOLDEN))
    assert g["n"] == N and g["chi"] == CHI and g["eps"] == 1e-24 and g["gates"] == len(circ)
    assert d.bond_dims() == g["dims_after"]
    gh, gl = d.amplitudes(bits, dd=True)
    oh = np.array(g["amp_re_hi"]) + 1j * np.array(g["amp_im_hi"])
    ol = np.array(g["amp_re_lo"]) + 1j * np.array(g["amp_im_lo"])
    err = float(np.max(np.abs((gh - oh) + (gl - ol))))
    print(f"  vs the 256-bit oracle (same truncation): worst |amplitude error| {err:.3e}", flush=True)
    assert err <= TOL
    d.close()
