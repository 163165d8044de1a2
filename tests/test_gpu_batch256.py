"""Configuration 4 at full size: 256 independent brickwork circuits of Haar U(4)
gates (seed 4: n ~ U{16..48}, chi_max ~ U{32, 64, 128, 256}, depth ~ U{8..24},
eps = 1e-12; 66 308 gates), all handed to one batch in a single call, FP64 and dd.

* Three circuits (indices 125, 222, 199) against stored 256-bit oracle runs of the
  same gates (tests/golden/batch256_subset.json, written by
  tests/golden/make_golden.py batch256_subset): same bond dims, 32 amplitudes each
  within 1e-12 (FP64) and 1e-26 (dd).  The oracle's smallest relative gap at a cut
  (2.4e-5) and smallest relative distance of an eps decision from its boundary
  (4.2e-3) keep both sides on the same subspaces.
* Those three and two larger circuits (chi_max = 256) run alone on standalone
  handles: bit for bit the batch's states (the launch shapes differ, the per-update
  arithmetic does not)."""
import json
import os

import numpy as np
import pytest

from paper_1111_3124_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch256_subset.json")


@pytest.fixture(scope="module")
def B():
    from paper_1111_3124_amd import binding
    return binding


@pytest.fixture(scope="module")
def workload():
    specs = W.batch_spec(256, 4)
    circ, gates = W.batch_gates(specs)
    return specs, circ, gates


@pytest.mark.parametrize("dd", [False, True])
def test_batch256_vs_oracle_and_standalone(B, workload, dd):
    specs, circ, gates = workload
    prec = B.MPS_PREC_DD if dd else B.MPS_PREC_FP64
    print(f"config 4: 256 circuits, {len(gates)} gates, dd={dd}", flush=True)
    bt = B.Batch([s.n for s in specs], [s.chi_max for s in specs], [1e-12] * len(specs), prec)
    bt.run(circ, gates)
    g = json.load(open(GOLDEN))
    tol = 1e-26 if dd else 1e-12
    for c in g["circuits"]:
        i = c["index"]
        sp = specs[i]
        assert (sp.n, sp.chi_max, sp.depth) == (c["n"], c["chi_max"], c["depth"])
        assert bt[i].bond_dims() == c["dims_after"], i
        bits = W.bitstrings(sp.n, 32, 4000 + i)
        oh = np.array(c["amp_re_hi"]) + 1j * np.array(c["amp_im_hi"])
        ol = np.array(c["amp_re_lo"]) + 1j * np.array(c["amp_im_lo"])
        if dd:
            gh, gl = bt[i].amplitudes(bits, dd=True)
            err = float(np.max(np.abs((gh - oh) + (gl - ol))))
        else:
            err = float(np.max(np.abs(bt[i].amplitudes(bits) - (oh + ol))))
        print(f"  circuit {i} (n={sp.n}, chi_max={sp.chi_max}, depth={sp.depth}) vs oracle: {err:.3e}", flush=True)
        assert err <= tol
    big = [i for i, s in enumerate(specs) if s.chi_max == 256][:2]
    for i in [c["index"] for c in g["circuits"]] + big:
        sp = specs[i]
        print(f"  circuit {i} alone (n={sp.n}, chi_max={sp.chi_max}, depth={sp.depth})", flush=True)
        alone = B.MPS(sp.n, sp.chi_max, 1e-12, prec)
        alone.apply_gates([gg for layer in W.brickwork(sp.n, sp.depth, sp.seed) for gg in layer])
        assert alone.bond_dims() == bt[i].bond_dims()
        bits = W.bitstrings(sp.n, 32, 5000 + i)
        if dd:
            ah, al = alone.amplitudes(bits, dd=True)
            gh, gl = bt[i].amplitudes(bits, dd=True)
            assert np.array_equal(ah, gh) and np.array_equal(al, gl)
        else:
            assert np.array_equal(alone.amplitudes(bits), bt[i].amplitudes(bits))
        for b in range(sp.n - 1):
            assert np.array_equal(alone.schmidt(b), bt[i].schmidt(b))
        alone.close()
    bt.close()
