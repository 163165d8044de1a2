"""Pins of the oracle's one-sided Jacobi SVD against textbook facts, checked at 256
bits outside the oracle (mpmath), and against LAPACK through numpy."""
import mpmath
import numpy as np
import pytest

from tests.ddutil import dd_to_mpmatrix, mpr


def _rand(rng, M, N, rank=None):
    if rank is None:
        return rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    # small Gaussian integers: the product is exact in binary64, so the rank is exact
    a = rng.integers(-3, 4, (M, rank)) + 1j * rng.integers(-3, 4, (M, rank))
    b = rng.integers(-3, 4, (rank, N)) + 1j * rng.integers(-3, 4, (rank, N))
    return a @ b


def _check_identities(A, out, tol=1e-29):
    M, N = A.shape
    Amp = mpmath.matrix([[mpmath.mpc(complex(A[i, j])) for j in range(N)] for i in range(M)])
    V = dd_to_mpmatrix(*out["V"])
    Wm = dd_to_mpmatrix(*out["W"])
    scale = mpmath.sqrt(sum(abs(Amp[i, j]) ** 2 for i in range(M) for j in range(N)))
    # W = A V
    D = Amp * V - Wm
    assert max(abs(D[i, j]) for i in range(M) for j in range(N)) < tol * scale
    # V unitary
    E = V.H * V - mpmath.eye(N)
    assert max(abs(E[i, j]) for i in range(N) for j in range(N)) < tol
    # W columns orthogonal; sigma = column norms, descending
    sig = [mpr(h, l) for h, l in zip(*out["sigma"])]
    G = Wm.H * Wm
    for p in range(N):
        assert abs(mpmath.sqrt(abs(G[p, p])) - sig[p]) < tol * scale
        for q in range(p + 1, N):
            assert abs(G[p, q]) < tol * scale * scale
    assert all(sig[j] >= sig[j + 1] for j in range(N - 1))
    return sig


@pytest.mark.parametrize("M,N,rank", [(6, 6, None), (9, 5, None), (4, 9, 2), (7, 7, 3)])
def test_svd_identities(oracle_mod, M, N, rank):
    rng = np.random.default_rng(M * 100 + N)
    A = _rand(rng, M, N, rank)
    out = oracle_mod.osvd(A)
    sig = _check_identities(A, out)
    ref = np.linalg.svd(A, compute_uv=False)
    r = min(M, N)
    for j in range(r):
        assert abs(float(sig[j]) - ref[j]) <= 1e-13 * ref[0]
    for j in range(r, N):
        assert float(sig[j]) < 1e-60 * ref[0]
    if rank is not None:
        for j in range(rank, N):
            assert float(sig[j]) < 1e-60 * ref[0]


def test_svd_two_by_two_closed_form(oracle_mod):
    """sigma^2 of a 2x2 matrix are the roots of x^2 - ||A||_F^2 x + |det A|^2."""
    rng = np.random.default_rng(7)
    for _ in range(4):
        A = _rand(rng, 2, 2)
        out = oracle_mod.osvd(A)
        a = [[mpmath.mpc(complex(A[i, j])) for j in range(2)] for i in range(2)]
        f2 = sum(abs(a[i][j]) ** 2 for i in range(2) for j in range(2))
        det2 = abs(a[0][0] * a[1][1] - a[0][1] * a[1][0]) ** 2
        disc = mpmath.sqrt(f2 ** 2 - 4 * det2)
        want = [mpmath.sqrt((f2 + disc) / 2), mpmath.sqrt((f2 - disc) / 2)]
        for j in range(2):
            assert abs(mpr(out["sigma"][0][j], out["sigma"][1][j]) - want[j]) < 1e-29 * want[0]


def test_svd_special_matrices(oracle_mod):
    """Diagonal input: sigma = |d| sorted; unitary input: all sigma = 1."""
    d = np.array([0.5, -3.0, 2.0j, 1e-3, 0.0])
    out = oracle_mod.osvd(np.diag(d))
    sig = [mpr(h, l) for h, l in zip(*out["sigma"])]
    for s, w in zip(sig, sorted(np.abs(d), reverse=True)):
        assert abs(s - mpmath.mpf(float(w))) < 1e-40
    from paper_1111_3124_amd.workloads import haar_unitary_dd, rng_for
    hi, lo = haar_unitary_dd(8, rng_for(3))
    out = oracle_mod.osvd(hi, lo)
    for h, l in zip(*out["sigma"]):
        assert abs(mpr(h, l) - 1) < 1e-30


def test_svd_repeated_singular_values(oracle_mod):
    """A = Q1 diag(2, 2, 1, 1) Q2^H: the repeated values come out repeated."""
    from paper_1111_3124_amd.workloads import haar_unitary, rng_for
    rng = rng_for(5)
    q1, q2 = haar_unitary(4, rng), haar_unitary(4, rng)
    A = q1 @ np.diag([2.0, 2.0, 1.0, 1.0]) @ q2.conj().T
    out = oracle_mod.osvd(A)
    sig = [float(mpr(h, l)) for h, l in zip(*out["sigma"])]
    assert np.allclose(sig, [2, 2, 1, 1], atol=1e-14)
    _check_identities(A, out)


def test_load_roundtrip(oracle_mod):
    """A state loaded in the (B, lambda) gauge gives the amplitudes of the plain
    product B_0[b0] B_1[b1] ... (B_s = Gamma_s lambda_s), evaluated in numpy."""
    from paper_1111_3124_amd.workloads import random_mps_B, rng_for
    rng = rng_for(9)
    dims = [2, 3, 5, 3, 2]
    B, lam = random_mps_B(dims, rng, spread=2.0)
    m = oracle_mod.OracleMPS(6, 8, 0.0)
    m.load(B, lam)
    assert m.bond_dims() == dims
    for x in range(0, 64, 5):
        bits = [(x >> (5 - q)) & 1 for q in range(6)]
        v = np.ones((1,), dtype=np.complex128)
        for s in range(6):
            v = v @ B[s][:, bits[s], :]
        hi, lo = m.amplitude(bits)
        assert abs(hi - v[0]) < 1e-14
    for b in range(5):
        hi, _ = m.schmidt(b)
        assert np.allclose(hi, lam[b], rtol=0, atol=1e-16)
