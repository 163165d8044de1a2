"""Checkpoint and resume (mps_export / mps_import) through the C ABI: an imported
state equals the exported one bit for bit, and so do both after the same further
gates (FP64 and dd); corrupt or truncated images are rejected."""
import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


def all_bits(n):
    x = np.arange(1 << n)
    return ((x[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.uint8)


def flush(msg):
    print(msg, flush=True)


def snapshot(d, dd):
    n = d.n
    out = [np.array(d.bond_dims())]
    for b in range(n - 1):
        out += list(d.schmidt_dd(b)) if dd else [d.schmidt(b)]
    out += list(d.amplitudes(all_bits(n), dd=True)) if dd else [d.amplitudes(all_bits(n))]
    return out


@pytest.mark.parametrize("dd", [False, True])
def test_export_import_resume_bit_identical(B, dd):
    flush(f"checkpoint: n=10 chi=12 eps=1e-12 seed=41 dd={dd}")
    n, chi, eps = 10, 12, 1e-12
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    layers = W.brickwork_dd(n, 12, 41) if dd else W.brickwork(n, 12, 41)
    first, rest = [g for l in layers[:6] for g in l], [g for l in layers[6:] for g in l]
    a = B.MPS(n, chi, eps, prec)
    a.apply_gates(first)
    img = a.export()
    b = B.MPS.from_image(img)
    assert (b.n, b.chi_max, b.eps, b.prec) == (n, chi, eps, prec)
    for x, y in zip(snapshot(a, dd), snapshot(b, dd)):
        assert np.array_equal(x, y)
    assert b.export() == img  # the image of the imported state is the same image
    a.apply_gates(rest)
    b.apply_gates(rest)
    for x, y in zip(snapshot(a, dd), snapshot(b, dd)):
        assert np.array_equal(x, y)


def test_import_rejects_bad_images(B):
    flush("checkpoint: bad images")
    a = B.MPS(6, 8, 0.0)
    a.apply_gates([g for l in W.brickwork(6, 3, 42) for g in l])
    img = a.export()
    bad = [img[:-1], b"XXXXXXXX" + img[8:], img[:40] + bytes([img[40] ^ 1]) + img[41:], b""]
    for x in bad:
        with pytest.raises(B.MPSError):
            B.mps_import(x)
    assert "mps_import" in B.mps_last_error(None)


@pytest.mark.parametrize("dd", [False, True])
def test_resume_matches_oracle_uninterrupted(B, oracle_mod, dd):
    """Export half-way through a truncated circuit, resume from the image in a new
    handle, finish the circuit there, and compare with the oracle running the whole
    circuit without interruption: bond dims, every Schmidt vector and all 1024
    amplitudes, FP64 within 1e-12 and dd within 1e-26."""
    flush(f"checkpoint vs oracle: n=10 chi=12 eps=1e-12 seed=43 dd={dd}")
    n, chi, eps = 10, 12, 1e-12
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    tol = 1e-26 if dd else 1e-12
    layers = W.brickwork_dd(n, 12, 43) if dd else W.brickwork(n, 12, 43)
    gates = [g for l in layers for g in l]
    first, rest = [g for l in layers[:6] for g in l], [g for l in layers[6:] for g in l]
    om = oracle_mod.OracleMPS(n, chi, eps)
    for g in gates:
        om.apply_gate(g)
        for st in om.last_stats():
            assert st["gap"] > (1e-20 if dd else 1e-10)
    a = B.MPS(n, chi, eps, prec)
    a.apply_gates(first)
    img = a.export()
    a.close()
    b = B.MPS.from_image(img)
    b.apply_gates(rest)
    assert b.bond_dims() == om.bond_dims()
    assert max(om.bond_dims()) == chi  # the truncation binds
    for bond in range(n - 1):
        oh, ol = om.schmidt(bond)
        if dd:
            lh, ll = b.schmidt_dd(bond)
            err = float(np.max(np.abs((lh - oh) + (ll - ol))))
        else:
            err = float(np.max(np.abs(b.schmidt(bond) - (oh + ol))))
        assert err <= tol, (bond, err)
    bits = all_bits(n)
    ah, al = om.amplitudes(bits)
    if dd:
        gh, gl = b.amplitudes(bits, dd=True)
        err = float(np.max(np.abs((gh - ah) + (gl - al))))
    else:
        err = float(np.max(np.abs(b.amplitudes(bits) - (ah + al))))
    flush(f"max |amplitude error| = {err:.3e}")
    assert err <= tol
