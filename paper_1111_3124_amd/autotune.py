"""Autotuner of the Jacobi step configuration, per precision and problem size.

    python -m paper_1111_3124_amd.autotune [--out PATH] [--classes 16,32,...] [--reps 2]

For each size class chi (Jacobi problems of N = 2 chi columns: square thetas of
updates with a = b = c = chi, the truncation binding at chi) and each precision, a
batch of independent circuits is loaded with random saturated states and one layer
of Haar gates on disjoint windows is timed through the library with every candidate
configuration:
  * block width 4, 8 or 16 (column blocks of the one-sided block Jacobi),
  * inner sweeps per block pair for problems with fewer than 16 blocks (FP64: 1, 2
    or 4; dd keeps 12, the margin its refinement needs on rank-deficient thetas),
  * QR preconditioning on or off (N >= 64).
A candidate whose layer leaves an update unconverged is rejected.  The best one
(least wall time over `reps` runs, each on a freshly loaded batch) is written to the
tuning table under this device's key (mps_tuning_key: architecture and HIP runtime
version); the library reads it when a handle or batch is created.  The concurrency
of each class is timed twice, with many two-site updates in flight (a batch of
circuits) and with three U(8) updates (one circuit of three-site gates), and
candidates are ranked by the geometric mean of the two rates (see CONCURRENCY).

The tuning table is plain text, one section per key:
    key <arch> <hip runtime version>
    <fp64|dd> <nmax> <block width> <inner sweeps> <qr>
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_1111_3124_amd import binding as B  # noqa: E402
from paper_1111_3124_amd import workloads as W  # noqa: E402

# Each size class is timed on two workloads: many two-site updates in flight (a batch
# of circuits; CONCURRENCY updates a layer) and FEW three-site updates (one circuit of
# U(8) gates: tall Jacobi problems, few in flight).  The best block width depends on
# how many blocks a step launch holds and on the problem's shape (wide blocks pay off
# when many updates fill the GPU), but an update's configuration may depend only on
# its own size and precision, so that batches and standalone runs agree bit for bit:
# each candidate is scored by the geometric mean of its two rates.
CONCURRENCY = {8: 512, 16: 256, 32: 128, 64: 64, 128: 32, 256: 12, 512: 6}
FEW = 3


def layer_case(chi: int, seed: int, total: int | None = None, k: int = 2):
    """C circuits of n qubits whose bonds hold chi values around the gated sites;
    g Haar U(2^k) gates per circuit on disjoint windows of k sites whose bonds all
    hold chi (k = 2: theta 2 chi x 2 chi; k = 3: first split 2 chi x 4 chi, run on
    its conjugate transpose, then 2 chi x 2 chi), `total` (default CONCURRENCY[chi])
    gates in all, rounded up to whole circuits."""
    L = int(round(math.log2(chi)))
    total = total or CONCURRENCY[chi]
    g = min(total, 12)
    C = (total + g - 1) // g
    n = 2 * L + k + k * g
    dims = W._saturated_dims(n, chi)
    rng = W.rng_for(seed)
    states = [W.random_mps_B(dims, rng, spread=4.0) for _ in range(C)]
    gates = []
    for c in range(C):
        for j in range(g):
            s = L + k * j
            hi, lo = W.haar_unitary_dd(1 << k, rng)
            gates.append((c, W.Gate(s, k, hi, lo)))
    return n, C, states, gates


def candidates(prec: int, N: int):
    out = []
    for bw in (4, 8, 16):
        few = N < 16 * bw  # fewer than 16 blocks: the inner-sweep limit applies
        inners = ((12,) if prec == B.MPS_PREC_DD else ((1, 2, 4) if few else (1,)))
        for inner in inners:
            for qr in ((0, 1) if N >= 64 else (0,)):
                out.append((bw, inner, qr))
    return out


def time_candidate(chi, prec, cand, case, reps):
    n, C, states, gates = case
    bw, inner, qr = cand
    best = math.inf
    for _ in range(reps):
        bt = B.Batch([n] * C, [chi] * C, [1e-12] * C, prec)
        try:
            for key, v in ((B.MPS_OPT_BLOCK_WIDTH, bw), (B.MPS_OPT_MAX_INNER_FEW, inner), (B.MPS_OPT_QR, qr)):
                bt.set_option(key, v)
            for c in range(C):
                Bt, lam = states[c]
                bt[c].load(Bt, lam)
            circ = [c for c, _ in gates]
            gl = [gg if prec == B.MPS_PREC_DD else W.Gate(gg.first, gg.k, gg.u_hi) for _, gg in gates]
            bt[0].sync()
            t0 = time.perf_counter()
            try:
                bt.run(circ, gl)
            except B.MPSError as e:
                if e.code == B.MPS_ENOCONV:
                    return None
                raise
            bt[0].sync()
            best = min(best, time.perf_counter() - t0)
        finally:
            bt.close()
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    ap.add_argument("--classes", default="16,32,64,128,256,512")
    ap.add_argument("--precisions", default="fp64,dd")
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    key = B.mps_tuning_key()
    if not key:
        sys.exit("autotune: no device")
    rows, notes = [], []
    for pname in args.precisions.split(","):
        prec = B.MPS_PREC_DD if pname == "dd" else B.MPS_PREC_FP64
        for chi in (int(x) for x in args.classes.split(",")):
            N = 2 * chi
            cases = [layer_case(chi, 1000 + chi), layer_case(chi, 2000 + chi, FEW, 3)]
            nupd = [len(c[3]) for c in cases]
            rates = {}
            for cand in candidates(prec, N):
                ts = [time_candidate(chi, prec, cand, c, args.reps) for c in cases]
                if any(t is None for t in ts):
                    print(f"# {pname} chi={chi} N={N} bw={cand[0]} inner={cand[1]} qr={cand[2]}: unconverged",
                          flush=True)
                    continue
                rates[cand] = [u / t for u, t in zip(nupd, ts)]
                print(f"# {pname} chi={chi} N={N} bw={cand[0]} inner={cand[1]} qr={cand[2]}: "
                      + " / ".join(f"{r:.1f}" for r in rates[cand]) + " updates/s", flush=True)
            if not rates:
                continue
            score = {c: math.sqrt(r[0] * r[1]) for c, r in rates.items()}
            best = max(score, key=score.get)
            dflt = (8, 12 if prec == B.MPS_PREC_DD else 1, 1 if N >= 64 else 0)
            rows.append(f"{pname} {N} {best[0]} {best[1]} {best[2]}")
            fmt = lambda c: " / ".join(f"{r:.1f}" for r in rates[c]) if c in rates else "n/a"
            notes.append(f"# {pname} N<={N}: {nupd[0]} / {nupd[1]} updates a layer; best {fmt(best)} updates/s "
                         f"(bw {best[0]}, inner {best[1]}, qr {best[2]}); defaults (bw 8) {fmt(dflt)}")
    text = ["# Jacobi step configurations measured by python -m paper_1111_3124_amd.autotune",
            f"# {time.strftime('%Y-%m-%d')}, per size class one layer of Haar U(4) updates (many in flight) and of "
            f"{FEW} U(8) updates (bond dims chi around every gate)"]
    text += notes
    text += [f"key {key}"] + rows
    # keep the sections of other keys
    old = []
    if os.path.exists(args.out):
        keep = False
        for line in open(args.out):
            w = line.split()
            if w and w[0] == "key":
                keep = " ".join(w[1:3]) != key
            if keep:
                old.append(line.rstrip("\n"))
    with open(args.out, "w") as f:
        f.write("\n".join(text + old) + "\n")
    print(f"wrote {args.out} ({len(rows)} rows for key {key})", flush=True)


if __name__ == "__main__":
    main()
