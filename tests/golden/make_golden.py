"""Write the stored expected values used by the full-size parity tests.

Only the oracle (oracle/) and the seeded input generators are called here; the
device library is never imported.  Run from the repository root:

    python tests/golden/make_golden.py update_chi256

update_chi256: a 20-qubit random (B, V) state with bond dims at capacity for
chi_max = 256 (bonds 7..11 hold 256), one Haar U(4) on sites 9, 10 (theta 512 x 512,
truncation by chi_max binding), eps = 1e-12.  Stores the new bond dims, the 256
Schmidt values of bond 9 and 24 amplitudes as double-double pairs, plus the
oracle's diagnostics of the split (gap at the cut, discarded weight).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1111_3124_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def update_chi256_inputs():
    n, chi, eps, seed = 20, 256, 1e-12, 256
    dims = [min(chi, 2 ** (b + 1), 2 ** (n - 1 - b)) for b in range(n - 1)]
    rng = W.rng_for(seed)
    Bt, lam = W.random_mps_B(dims, rng, spread=4.0)
    U = W.haar_unitary(4, rng)
    bits = W.bitstrings(n, 24, seed + 1)
    return dict(n=n, chi=chi, eps=eps, seed=seed, dims=dims, B=Bt, lam=lam, U=U, first=9, bits=bits)


def make_update_chi256():
    inp = update_chi256_inputs()
    t0 = time.time()
    om = oracle.OracleMPS(inp["n"], inp["chi"], inp["eps"])
    om.load(inp["B"], inp["lam"])
    om.apply(inp["first"], 2, inp["U"])
    st = om.last_stats()[0]
    sh, sl = om.schmidt(inp["first"])
    ah, al = om.amplitudes(inp["bits"])
    out = dict(
        recipe="tests/golden/make_golden.py update_chi256 (oracle at 256 bits)",
        n=inp["n"], chi=inp["chi"], eps=inp["eps"], seed=inp["seed"], first=inp["first"],
        dims_after=om.bond_dims(),
        schmidt_hi=sh.tolist(), schmidt_lo=sl.tolist(),
        amp_re_hi=ah.real.tolist(), amp_re_lo=al.real.tolist(),
        amp_im_hi=ah.imag.tolist(), amp_im_lo=al.imag.tolist(),
        split=dict(gap=st["gap"], w=st["w"], k=st["k"], rank=st["rank"], sweeps=st["sweeps"]),
        oracle_seconds=time.time() - t0, oracle_threads=oracle.oracle_threads(),
    )
    with open(os.path.join(HERE, "update_chi256.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote update_chi256.json", out["split"], f"{out['oracle_seconds']:.0f} s")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "update_chi256"
    {"update_chi256": make_update_chi256}[what]()
