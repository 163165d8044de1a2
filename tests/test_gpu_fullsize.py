"""Parity at the benchmark's size: one two-site update with a = b = c = 256 (theta
512 x 512, truncation to chi_max = 256 binding) in the benchmark's launch path,
against stored 256-bit oracle values (tests/golden/update_chi256.json, written by
tests/golden/make_golden.py from the oracle only).  Checked: new bond dims, the 256
Schmidt values of the updated bond, and 24 amplitudes."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "update_chi256.json")


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


@pytest.fixture(scope="module")
def fixture():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_golden
    return json.load(open(GOLD)), make_golden.update_chi256_inputs()


@pytest.mark.parametrize("bw", [None, 16, 4])
@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-26)])
def test_update_chi256(B, fixture, prec, tol, bw):
    """bw None: the tuned step configuration; 16 and 4: that block width forced (32-
    and 8-column pairs: 31 or 127 steps a sweep instead of 63)."""
    g, inp = fixture
    print(f"full-size update: prec={prec} bw={bw} n={inp['n']} site={inp['first']}", flush=True)
    assert g["split"]["gap"] > (1e-10 if prec == 0 else 1e-20)
    d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
    if bw is not None:
        d.set_option(B.MPS_OPT_BLOCK_WIDTH, bw)
    d.load(inp["B"], inp["lam"])
    d.apply(inp["first"], 2, inp["U"])
    assert d.bond_dims() == g["dims_after"]
    oh = np.array(g["schmidt_hi"]); ol = np.array(g["schmidt_lo"])
    if prec:
        lh, ll = d.schmidt_dd(inp["first"])
        assert float(np.max(np.abs((lh - oh) + (ll - ol)))) <= tol
    else:
        assert float(np.max(np.abs(d.schmidt(inp["first"]) - (oh + ol)))) <= tol
    ah = np.array(g["amp_re_hi"]) + 1j * np.array(g["amp_im_hi"])
    al = np.array(g["amp_re_lo"]) + 1j * np.array(g["amp_im_lo"])
    scale = max(1.0, float(np.max(np.abs(ah))))
    if prec:
        gh, gl = d.amplitudes(inp["bits"], dd=True)
        err = float(np.max(np.abs((gh - ah) + (gl - al))))
    else:
        err = float(np.max(np.abs(d.amplitudes(inp["bits"]) - (ah + al))))
    print(f"max |amplitude error| = {err:.3e} (scale {scale:.3e})", flush=True)
    assert err <= tol * scale


@pytest.mark.parametrize("prec,qr", [(0, 1), (1, 1), (0, 0)])
def test_update_chi256_split_step_bit_identical(B, fixture, prec, qr):
    """The Jacobi step as one fused launch or as the two-launch split form (used for
    launches of few updates) forms the same Gram in the same order and every row of W
    and V by the same instructions; the fused form applies V's rotation one step late
    (extra blocks of the next launch, then a flush), the split form at once.  The
    update's Schmidt values and amplitudes agree bit for bit.  V is accumulated by dd
    updates and by FP64 ones without QR preconditioning."""
    _, inp = fixture
    print(f"split vs fused step: prec={prec} qr={qr} n={inp['n']} site={inp['first']}", flush=True)
    out = []
    for limit in (0, 4):
        d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
        d.set_option(B.MPS_OPT_STEP_SPLIT, limit)
        if not qr:
            d.set_option(B.MPS_OPT_QR, 0)
        d.load(inp["B"], inp["lam"])
        d.apply(inp["first"], 2, inp["U"])
        lam = d.schmidt_dd(inp["first"]) if prec else (d.schmidt(inp["first"]),)
        amp = d.amplitudes(inp["bits"], dd=True) if prec else (d.amplitudes(inp["bits"]),)
        out.append((d.bond_dims(), lam, amp, d.stats()["sweeps"]))
        d.close()
    (dims0, lam0, amp0, sw0), (dims1, lam1, amp1, sw1) = out
    assert dims0 == dims1 and sw0 == sw1
    for a, b in zip(lam0 + amp0, lam1 + amp1):
        assert np.array_equal(a, b)



@pytest.mark.parametrize("prec", [0, 1])
def test_update_chi256_fused_launch_modes_bit_identical(B, fixture, prec):
    """The one-launch step (V's rotations applied one step late by extra blocks of the
    next launch, the last step's by a flush after each tick's sweeps) under every
    launch mode: one or two sweeps a tick, launched one by one or replayed from a
    captured graph.  The same state bit for bit; FP64 without QR preconditioning, so
    that V is accumulated there too."""
    _, inp = fixture
    out = []
    for ts, gr in ((2, 0), (1, 0), (2, 1), (1, 1)):
        print(f"fused-step launch modes: prec={prec} tick_sweeps={ts} graph={gr}", flush=True)
        d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
        d.set_option(B.MPS_OPT_STEP_SPLIT, 0)
        d.set_option(B.MPS_OPT_TICK_SWEEPS, ts)
        d.set_option(B.MPS_OPT_GRAPH, gr)
        if not prec:
            d.set_option(B.MPS_OPT_QR, 0)
        d.load(inp["B"], inp["lam"])
        d.apply(inp["first"], 2, inp["U"])
        lam = d.schmidt_dd(inp["first"]) if prec else (d.schmidt(inp["first"]),)
        amp = d.amplitudes(inp["bits"], dd=True) if prec else (d.amplitudes(inp["bits"]),)
        out.append((d.bond_dims(), lam, amp))
        d.close()
    for dims, lam, amp in out[1:]:
        assert dims == out[0][0]
        for a, b in zip(lam + amp, out[0][1] + out[0][2]):
            assert np.array_equal(a, b)
