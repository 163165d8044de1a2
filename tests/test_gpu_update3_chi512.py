"""Configuration 3's update at its real size: one Haar U(8) on sites 9, 10, 11 of a
22-qubit random (B, V) state whose bonds 8..12 hold chi_max = 512 values
(a = b = c = d = 512), eps = 1e-14, against stored 256-bit oracle values
(tests/golden/update3_chi512.json, written by tests/golden/make_golden.py
update3_chi512 from the oracle only).  The first split's theta is 1024 x 2048 (wide:
the Jacobi runs on theta_w^H, 2048 x 1024), truncated to 512 by chi_max; the second
split's theta is 1024 x 1024 (QR-preconditioned), truncated to 512.  This runs the
three-site kernels over many tiles, the N = 1024 Jacobi and, in FP64, the 64-panel
QR.  Checked, FP64 within 1e-12 and dd within 1e-26: the new bond dims, the Schmidt
values of both updated bonds and 24 amplitudes."""
import json
import os

import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "update3_chi512.json")


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


@pytest.fixture(scope="module")
def case():
    return json.load(open(GOLD)), W.update3_chi512_inputs()


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-26)])
def test_update3_chi512(B, case, prec, tol):
    g, inp = case
    print(f"config 3 update at full size: prec={prec} n={inp['n']} sites {inp['first']}..{inp['first'] + 2}",
          flush=True)
    # the cuts are not near-degenerate at either precision's noise level
    for sp in g["splits"]:
        assert sp["gap"] > (1e-10 if prec == 0 else 1e-20)
    d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
    d.load(inp["B"], inp["lam"])
    d.apply(inp["first"], 3, inp["U"])
    assert d.bond_dims() == g["dims_after"]
    for j, bond in enumerate((inp["first"], inp["first"] + 1)):
        oh, ol = np.array(g[f"schmidt{j}_hi"]), np.array(g[f"schmidt{j}_lo"])
        if prec:
            lh, ll = d.schmidt_dd(bond)
            err = float(np.max(np.abs((lh - oh) + (ll - ol))))
        else:
            err = float(np.max(np.abs(d.schmidt(bond) - (oh + ol))))
        print(f"  bond {bond}: max |Schmidt value error| {err:.3e}", flush=True)
        assert err <= tol
    ah = np.array(g["amp_re_hi"]) + 1j * np.array(g["amp_im_hi"])
    al = np.array(g["amp_re_lo"]) + 1j * np.array(g["amp_im_lo"])
    scale = max(1.0, float(np.max(np.abs(ah))))
    if prec:
        gh, gl = d.amplitudes(inp["bits"], dd=True)
        err = float(np.max(np.abs((gh - ah) + (gl - al))))
    else:
        err = float(np.max(np.abs(d.amplitudes(inp["bits"]) - (ah + al))))
    print(f"  max |amplitude error| {err:.3e} (scale {scale:.3e})", flush=True)
    assert err <= tol * scale
    d.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_update3_chi512_fused_vs_split_bit_identical(B, case, prec):
    """The same update with every Jacobi step as one launch (V's rotations applied one
    step late by extra blocks, then a flush: the wide first split accumulates V at
    N = 1024 in dd) and as the two-launch split form (V updated at once): the same
    bond dims, Schmidt values and amplitudes bit for bit."""
    _, inp = case
    out = []
    for limit in (0, 1 << 20):
        print(f"config 3 update, fused vs split step: prec={prec} split limit={limit}", flush=True)
        d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
        d.set_option(B.MPS_OPT_STEP_SPLIT, limit)
        d.load(inp["B"], inp["lam"])
        d.apply(inp["first"], 3, inp["U"])
        lam = []
        for bond in (inp["first"], inp["first"] + 1):
            lam += list(d.schmidt_dd(bond)) if prec else [d.schmidt(bond)]
        amp = list(d.amplitudes(inp["bits"], dd=True)) if prec else [d.amplitudes(inp["bits"])]
        out.append((d.bond_dims(), lam + amp))
        d.close()
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
