"""QR preconditioning of two-site updates (MPS_OPT_QR): one update of a loaded random
state with theta square (80 x 80), tall (80 x 64), rank-deficient (80 x 80 of rank at
most 40) and wide rank-deficient (64 x 80 of rank at most 40, which never takes QR:
the transposed path), with the option on and off, against the oracle: FP64 within
1e-12 and dd within 1e-26 per amplitude (scaled by the largest amplitude), Schmidt
values likewise.  dd takes QR only for square thetas, so its tall case checks the
fallback to the plain Jacobi with the option on.  In the rank-deficient cases the
null space's singular values are rounding noise (about 1.5e-13 of the largest after
the plain FP64 Jacobi, 3e-29 after the dd refinement).  Where Z is formed from W's
columns (QR, wide thetas) the columns the Jacobi treated as zero are dropped; the
plain path may keep some noise columns, harmless there since Z = V is unitary.  So
the extra Schmidt values are checked to be noise (below the tolerance relative to the
largest) and the first ones compared as usual; amplitudes are compared in full."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def flush(msg):
    print(msg, flush=True)


CASES = {
    # bond dims of a 14-qubit state; the gate acts on sites 6, 7: a = dims[5], b = dims[6], c = dims[7]
    "square": [2, 4, 8, 16, 32, 40, 40, 40, 32, 16, 8, 4, 2],
    "tall": [2, 4, 8, 16, 32, 40, 40, 32, 32, 16, 8, 4, 2],
    "rank_deficient": [2, 4, 8, 16, 32, 40, 10, 40, 32, 16, 8, 4, 2],
    "wide_rank_deficient": [2, 4, 8, 16, 32, 32, 10, 40, 32, 16, 8, 4, 2],
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [0, 1])
def test_qr_update_vs_oracle(B, oracle_mod, case, prec):
    flush(f"qr update: case={case} prec={prec} seed=61")
    dims = CASES[case]
    rng = W.rng_for(61)
    Bt, lam = W.random_mps_B(dims, rng, spread=2.0)
    n = len(dims) + 1
    hi, lo = W.haar_unitary_dd(4, rng)
    om = oracle_mod.OracleMPS(n, 128, 0.0)
    om.load(Bt, lam)
    om.apply(6, 2, hi, lo if prec else None)
    bits = W.bitstrings(n, 200, 62)
    oh, ol = om.amplitudes(bits)
    sh, sl = om.schmidt(6)
    tol = 1e-26 if prec else 1e-12
    scale = max(1.0, float(np.max(np.abs(oh))))
    for qr in (1, 0):
        d = B.MPS(n, 128, 0.0, prec)
        d.set_option(B.MPS_OPT_QR, qr)
        d.load(Bt, lam)
        if prec:
            d.apply(6, 2, hi, lo)
        else:
            d.apply(6, 2, hi)
        dims_d, dims_o = d.bond_dims(), om.bond_dims()
        m = dims_o[6]
        if case.endswith("rank_deficient"):
            assert dims_d[:6] == dims_o[:6] and dims_d[7:] == dims_o[7:] and dims_d[6] >= m
            s_all = sum(d.schmidt_dd(6)) if prec else d.schmidt(6)
            assert float(np.max(s_all[m:], initial=0.0)) < tol * s_all[0]
        else:
            assert dims_d == dims_o
        if prec:
            gh, gl = d.amplitudes(bits, dd=True)
            assert float(np.max(np.abs((gh - oh) + (gl - ol)))) <= tol * scale
            lh, ll = d.schmidt_dd(6)
            assert float(np.max(np.abs((lh[:m] - sh) + (ll[:m] - sl)))) <= tol
        else:
            assert float(np.max(np.abs(d.amplitudes(bits) - (oh + ol)))) <= tol * scale
            assert float(np.max(np.abs(d.schmidt(6)[:m] - (sh + sl)))) <= tol
        d.close()
