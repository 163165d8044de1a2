"""Benchmark: MPS gate updates per second at chi = 256 on one MI355X.

Workload (seeded, synthetic): a 40-qubit MPS, chi_max = 256, eps = 1e-12, driven by
a brickwork circuit of Haar-random U(4) gates (seed 2).  Untimed setup applies
brickwork layers until every bond that can hold 256 Schmidt values does (bonds
7..31).  One step then applies the next brickwork layer's gates on bonds 8..30,
where a = b = c = 256 (theta is 512 x 512): 12 or 11 gate updates (theta GEMM,
Jacobi SVD, truncation, split; for the dd variant also the double-double
refinement).  The K timed layers are handed to the library in one call; its
scheduler runs every update whose sites are free, so updates of consecutive
layers overlap.  ms_per_step = timed seconds / K.

Output: one JSON line.  `value` is the headline variant's gate updates per second
(dd-refined when available, else FP64); the other variant is reported beside it.
`roofline` is for the dominant kernel (the Jacobi step); `cpu_baseline` times the
256-bit oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPS gate updates/s at χ=256: FP64 vs dd-refined, error vs 256-bit oracle"
N_QUBITS, CHI, EPS, SEED = 40, 256, 1e-12, 2
PEAK_FP64 = 78.6e12  # MI355X FP64 vector (and matrix) peak, FLOP/s
PEAK_HBM = 8.0e12    # MI355X HBM3E bandwidth, B/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobi_step_chi256_traffic.md")
FP64_OPS_FILE = os.path.join(ROOT, "profiles", "jacobi_step_chi256_fp64_ops.md")
S_REF = 10  # reference sweep count of the algorithmic work unit
KERNEL_SRC = os.path.join(ROOT, "paper_1111_3124_amd", "csrc", "kernels.hip")


def jacobi_flops(M: int, N: int) -> float:
    """Scalar one-sided Jacobi work per sweep, J(M, N) = N(N-1)/2 (28 M + 20 N)."""
    return N * (N - 1) / 2.0 * (28.0 * M + 20.0 * N)


def update_flops(a: int, b: int, c: int, k: int, sweeps: float) -> float:
    """Algorithmic FP64 flops of one 2-site update: theta GEMM + gate mix,
    `sweeps` Jacobi sweeps on the 2a x 2c theta, and the split GEMM."""
    return 32.0 * a * b * c + 128.0 * a * c + sweeps * jacobi_flops(2 * a, 2 * c) + 32.0 * a * c * k


def saturate(m, B, W, rng, max_layers=40):
    sat_bonds = [b for b in range(N_QUBITS - 1) if min(CHI, 2 ** (b + 1), 2 ** (N_QUBITS - 1 - b)) == CHI]
    t = 0
    while t < max_layers:
        m.apply_gates(W.brickwork_layer(N_QUBITS, t, rng))
        t += 1
        dims = m.bond_dims()
        if all(dims[b] == CHI for b in sat_bonds):
            break
    return t


def step_gates(W, rng, t):
    layer = W.brickwork_layer(N_QUBITS, t, rng)
    return [g for g in layer if 8 <= g.first <= 30]


def run_variant(B, W, prec: int, steps: int, warmup: int):
    rng = W.rng_for(SEED)
    m = B.MPS(N_QUBITS, CHI, EPS, prec)
    t = saturate(m, B, W, rng)
    dims = m.bond_dims()
    # the layers of the timed region (and the warmup) are drawn up front; each call
    # hands the runtime a whole list of layers, which it schedules with overlap
    warm = [g for i in range(warmup) for g in step_gates(W, rng, t + i)]
    t += warmup
    timed = [g for i in range(steps) for g in step_gates(W, rng, t + i)]
    if warm:
        m.apply_gates(warm, allow_noconv=True)
    m.sync()
    dims = m.bond_dims()
    for g in timed:
        assert dims[g.first - 1] == dims[g.first] == dims[g.first + 1] == CHI
    m.set_option(B.MPS_OPT_KERNEL_TIMING, 1)
    for c in list(range(len(B.KERNEL_CLASSES))) + [B.COUNTER_SWEEPS, B.COUNTER_SWEEPS_DD]:
        m.kernel_time(c, reset=True)
    m.sync()
    t0 = time.perf_counter()
    rc = m.apply_gates(timed, allow_noconv=True)
    m.sync()
    dt = time.perf_counter() - t0
    ktimes = {name: m.kernel_time(c) for c, name in enumerate(B.KERNEL_CLASSES)}
    slot_sweeps = m.kernel_time(B.COUNTER_SWEEPS)[1]
    slot_sweeps_dd = m.kernel_time(B.COUNTER_SWEEPS_DD)[1]
    dims = m.bond_dims()
    assert all(dims[g.first] == CHI for g in timed)
    lam_ok = all(abs(float((m.schmidt(b) ** 2).sum()) - 1.0) < 1e-12 for b in range(N_QUBITS - 1))
    m.close()
    return dict(rate=len(timed) / dt, ms_per_step=1e3 * dt / steps, gates=len(timed), seconds=dt,
                mean_sweeps=slot_sweeps / len(timed), mean_dd_sweeps=slot_sweeps_dd / len(timed),
                slot_sweeps=slot_sweeps, ktimes=ktimes, lam_ok=lam_ok, noconv=rc != 0, steps=steps)


def step_bytes(M: int, N: int, jvec: int = 1) -> float:
    """Memory traffic of one step of one update: every column of W (M x N) and, when
    V is accumulated (jvec), of V (N x N) is read once and written once (complex128)."""
    return 2.0 * 16.0 * (M * N + jvec * N * N)


def step_flops(M: int, N: int, jvec: int = 1) -> float:
    """Scalar one-sided Jacobi work of one step of one update: J(M, N) / (N/8 - 1), with
    the V rotations (the 20 N term) only when V is accumulated."""
    return N * (N - 1) / 2.0 * (28.0 * M + jvec * 20.0 * N) / (N // 8 - 1)


def measured(path, key):
    """A per-update-step figure of the Jacobi step kernel (N = 512) from a committed
    rocprofv3 counter summary, or None if there is none or kernels.hip changed since
    the counters were taken."""
    try:
        import hashlib
        text = open(path).read()
        kv = dict(l.split(":", 1) for l in text.splitlines() if l.startswith((key + ":", "kernels_hip_sha256:")))
        digest = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if kv["kernels_hip_sha256"].strip() != digest:
            return None
        return float(kv[key].strip())
    except (OSError, KeyError, ValueError):
        return None


def roofline(res, jvec: int):
    """Dominant kernel: the FP64 Jacobi step (k_jacobi_step<8>).  A step serves each
    iterating update with one of the nsteps = N/8 - 1 steps of its sweep:
    step_flops(M, N) and step_bytes(M, N) of algorithmic work (jvec: V accumulated,
    as in the dd variant; the FP64 variant's QR-preconditioned updates accumulate no
    V).  The updates of a step are split into two halves whose launches run
    concurrently on two streams, so a launch lasts about as long as the step.  Totals
    over the timed region: update-sweeps executed x nsteps x those; achieved = total /
    the steps' HIP-event time.  The primary bound is the one the kernel is closer to.
    The counter-based figures (memory-fabric traffic, executed FP64 flops: VALU adds,
    multiplies, 2 x FMAs, and MFMA operations) were taken on the dd variant."""
    ms, launches = res["ktimes"]["jacobi"]
    if launches == 0:
        return None
    M = N = 2 * CHI
    nsteps = N // 8 - 1
    sec = ms * 1e-3
    usteps = res["slot_sweeps"] * nsteps  # update-steps in the timed region
    flops = usteps * step_flops(M, N, jvec)
    nbytes = usteps * step_bytes(M, N, jvec)
    f_alu = flops / sec / PEAK_FP64
    f_hbm = nbytes / sec / PEAK_HBM
    per_step = measured(TRAFFIC_FILE, "bytes_per_update_step") if jvec else None
    traffic = per_step * usteps / launches if per_step else None
    hbm = {"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": f_hbm,
           "traffic": traffic, "bytes_per_launch": nbytes / launches}
    alu = {"bound": "alu", "achieved": flops / sec / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": f_alu,
           "traffic": traffic, "flops_per_launch": flops / launches}
    ops = measured(FP64_OPS_FILE, "fp64_flops_per_update_step") if jvec else None
    alu["executed"] = None if ops is None else {
        "flops_per_launch": ops * usteps / launches, "achieved": ops * usteps / sec / 1e12,
        "frac": ops * usteps / sec / PEAK_FP64}
    main, other = (hbm, alu) if f_hbm >= f_alu else (alu, hbm)
    main = dict(main)
    main.update({"kernel": "k_jacobi_step<8>", "avg_launch_us": 1e3 * ms / launches, "launches": launches,
                 "concurrent_launches": 2, "other_bound": other})
    return main


def work_at_s_ref(rate: float) -> dict:
    """The algorithmic FP64 work of one update at the reference sweep count (theta
    GEMM and gate mix, S_REF one-sided Jacobi sweeps with V, split GEMM) times the
    update rate, against the FP64 peak: a sweep saved shows as speed, not as a lower
    fraction."""
    f = update_flops(CHI, CHI, CHI, CHI, S_REF)
    return {"flops_per_update": f, "sweeps": S_REF, "achieved": rate * f / 1e12, "unit": "TFLOP/s",
            "frac": rate * f / PEAK_FP64}


def calibrate_copy(mib: int = 256, reps: int = 10):
    """A plain device-to-device copy of known size (the calibration kernel for the
    FETCH_SIZE / WRITE_SIZE counters): reads and writes `mib` MiB per dispatch."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_dispatch": mib << 20,
                      "bytes_written_per_dispatch": mib << 20, "dispatches": reps}), flush=True)


def cpu_baseline():
    """The 256-bit oracle on the host cores: one two-site update at a = b = c = 128
    (theta 256 x 256) of a seeded 40-qubit state, scaled to a = b = c = 256 by the
    paper's O(m^3) cost of one U(4) update (x 8)."""
    import oracle
    from paper_1111_3124_amd import workloads as W
    n, chi = N_QUBITS, 128
    dims = [min(chi, 2 ** (b + 1), 2 ** (n - 1 - b)) for b in range(n - 1)]
    rng = W.rng_for(1000)
    Bt, lam = W.random_mps_B(dims, rng, spread=2.0)
    om = oracle.OracleMPS(n, chi, EPS)
    om.load(Bt, lam)
    U = W.haar_unitary(4, rng)
    t0 = time.perf_counter()
    om.apply(19, 2, U)
    dt = time.perf_counter() - t0
    scale = (CHI / chi) ** 3
    return {"value": 1.0 / (dt * scale), "unit": "gate updates/s", "cores": oracle.oracle_threads(),
            "kind": "oracle",
            "sample": f"1 two-site update at a=b=c={chi} (theta {2*chi}x{2*chi}), 256-bit MPFR, "
                      f"{dt:.1f} s measured; scaled x{scale:.0f} to a=b=c={CHI} by the O(m^3) per-gate cost",
            "measured_s": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variants", default="auto", help="fp64, dd, both or auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    from paper_1111_3124_amd import binding as B
    from paper_1111_3124_amd import workloads as W

    want = args.variants
    dd_ok = True
    try:
        B.MPS(2, 2, 0.0, B.MPS_PREC_DD).close()
    except B.MPSError:
        dd_ok = False
    if want == "auto":
        want = "both" if dd_ok else "fp64"
    results = {}
    if want in ("fp64", "both"):
        results["fp64"] = run_variant(B, W, B.MPS_PREC_FP64, args.steps, args.warmup)
        print(f"# fp64: {results['fp64']['rate']:.1f} updates/s, mean sweeps {results['fp64']['mean_sweeps']:.1f}",
              file=sys.stderr, flush=True)
    if want in ("dd", "both"):
        results["dd"] = run_variant(B, W, B.MPS_PREC_DD, args.steps, args.warmup)
        print(f"# dd: {results['dd']['rate']:.1f} updates/s, mean sweeps {results['dd']['mean_sweeps']:.1f} "
              f"+ dd {results['dd']['mean_dd_sweeps']:.1f}",
              file=sys.stderr, flush=True)
    head = "dd" if "dd" in results else "fp64"
    r = results[head]
    line = {
        "metric": METRIC,
        "value": r["rate"],
        "unit": "gate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "dd" if head == "dd" else "f64",
        "data": "synthetic",
        "config": {"workload": "40-qubit MPS, brickwork Haar U(4) layers on bonds 8..30 with "
                               "a=b=c=256 (theta 512x512), chi_max=256, eps=1e-12, seed 2",
                   "updates_per_step": r["gates"] / args.steps, "variant": head,
                   "schedule": "all timed layers submitted in one call; updates overlap across layers"},
        "variants": {k: {"value": v["rate"], "ms_per_step": v["ms_per_step"],
                         "mean_sweeps": v["mean_sweeps"], "mean_dd_sweeps": v["mean_dd_sweeps"],
                         "kernel_ms": {n: t[0] for n, t in v["ktimes"].items()},
                         "schmidt_normalised": v["lam_ok"],
                         "roofline": roofline(v, 1 if k == "dd" else 0),
                         "work_at_s_ref": work_at_s_ref(v["rate"])} for k, v in results.items()},
        "roofline": roofline(r, 1 if head == "dd" else 0),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
