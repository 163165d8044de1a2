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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobi_step_chi256_{}_traffic.md")
FP64_OPS_FILE = os.path.join(ROOT, "profiles", "jacobi_step_chi256_{}_fp64_ops.md")
S_REF = 10  # reference sweep count of the algorithmic work unit
KERNEL_SRC = os.path.join(ROOT, "paper_1111_3124_amd", "csrc", "kernels.hip")
GOLDEN = os.path.join(ROOT, "tests", "golden", "update_chi256.json")


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


def run_variant(B, W, prec: int, steps: int, warmup: int, launch=None):
    rng = W.rng_for(SEED)
    m = B.MPS(N_QUBITS, CHI, EPS, prec)
    for key, value in (launch or {}).items():
        m.set_option(key, value)
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
    for c in list(range(len(B.KERNEL_CLASSES))) + [B.COUNTER_SWEEPS, B.COUNTER_SWEEPS_DD, B.COUNTER_NOCONV,
                                                   B.COUNTER_GRAPHS]:
        m.kernel_time(c, reset=True)
    m.sync()
    t0 = time.perf_counter()
    rc = m.apply_gates(timed, allow_noconv=True)
    m.sync()
    dt = time.perf_counter() - t0
    ktimes = {name: m.kernel_time(c) for c, name in enumerate(B.KERNEL_CLASSES)}
    slot_sweeps = m.kernel_time(B.COUNTER_SWEEPS)[1]
    slot_sweeps_dd = m.kernel_time(B.COUNTER_SWEEPS_DD)[1]
    noconv = m.kernel_time(B.COUNTER_NOCONV)[1]
    graphs = m.kernel_time(B.COUNTER_GRAPHS)
    dims = m.bond_dims()
    assert all(dims[g.first] == CHI for g in timed)
    lam_ok = all(abs(float((m.schmidt(b) ** 2).sum()) - 1.0) < 1e-12 for b in range(N_QUBITS - 1))
    m.close()
    return dict(rate=len(timed) / dt, ms_per_step=1e3 * dt / steps, gates=len(timed), seconds=dt,
                mean_sweeps=slot_sweeps / len(timed), mean_dd_sweeps=slot_sweeps_dd / len(timed),
                slot_sweeps=slot_sweeps, ktimes=ktimes, lam_ok=lam_ok, noconv=noconv, noconv_rc=rc != 0,
                steps=steps, graphs_built=int(graphs[0]), graph_replays=graphs[1])


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


def update_bytes(chi: int, dd: bool) -> float:
    """Algorithmic HBM bytes of one two-site update at a = b = c = k = chi: the site
    tensors read and written and the Schmidt values, 16 (2ab + 2bc + 2ak + 2kc) + 8a
    + 256 bytes (x2 for double-double)."""
    a = b = c = k = chi
    return (16.0 * (2 * a * b + 2 * b * c + 2 * a * k + 2 * k * c) + 8.0 * a + 256.0) * (2 if dd else 1)


def roofline(res, jvec: int, dd: bool):
    """Dominant kernel: the Jacobi step (k_jacobi_step<8>), an FP64 contraction (the
    pair Grams on the matrix cores, the rotations on the vector units; MI355X's FP64
    matrix and vector peaks are both 78.6 TFLOP/s).  A step serves each iterating
    update with one of the nsteps = N/8 - 1 steps of its sweep, and is credited with
    the scalar method's work for it, J(M, N) / nsteps (step_flops; jvec: V
    accumulated, as in the dd variant; the FP64 variant's QR-preconditioned updates
    accumulate no V).  The updates of a step are split into two halves whose launches
    run concurrently on two streams, so a launch lasts about as long as the step.
    Totals over the timed region: update-sweeps executed x nsteps x step_flops;
    achieved = total / the steps' HIP-event time.
    `traffic`: memory-fabric bytes per launch from the committed FETCH_SIZE and
    WRITE_SIZE counter summary of this variant (null once kernels.hip has changed);
    `traffic_per_update` compares them, summed over an update's steps, with the
    update's algorithmic bytes (update_bytes), and `hbm_algorithmic` gives those bytes
    at the measured update rate against the HBM peak."""
    ms, launches = res["ktimes"]["jacobi"]
    if launches == 0:
        return None
    M = N = 2 * CHI
    nsteps = N // 8 - 1
    sec = ms * 1e-3
    usteps = res["slot_sweeps"] * nsteps  # update-steps in the timed region
    flops = usteps * step_flops(M, N, jvec)
    tag = "dd" if dd else "fp64"
    per_step = measured(TRAFFIC_FILE.format(tag), "bytes_per_update_step")
    traffic = per_step * usteps / launches if per_step else None
    ub = update_bytes(CHI, dd)
    out = {"bound": "mfma", "achieved": flops / sec / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
           "frac": flops / sec / PEAK_FP64, "traffic": traffic,
           "kernel": "k_jacobi_step<8>", "dtype": "f64", "flops_per_launch": flops / launches,
           "avg_launch_us": 1e3 * ms / launches, "launches": launches, "concurrent_launches": 2,
           "update_steps_per_launch": usteps / launches}
    if per_step:
        steps_per_update = res["mean_sweeps"] * nsteps
        out["traffic_per_update"] = {"bytes": per_step * steps_per_update, "algorithmic_bytes": ub,
                                     "ratio": per_step * steps_per_update / ub}
    out["hbm_algorithmic"] = {"bytes_per_update": ub, "achieved_GBps": res["rate"] * ub / 1e9,
                              "frac": res["rate"] * ub / PEAK_HBM}
    ops = measured(FP64_OPS_FILE.format(tag), "fp64_flops_per_update_step")
    out["executed"] = None if ops is None else {
        "flops_per_launch": ops * usteps / launches, "achieved": ops * usteps / sec / 1e12,
        "frac": ops * usteps / sec / PEAK_FP64}
    return out


def golden_error(B, W, prec: int) -> dict:
    """Untimed accuracy check in the same process: the chi = 256 update of the stored
    256-bit oracle result (tests/golden/update_chi256.json: a 20-qubit random state,
    one Haar U(4) on sites 9, 10, theta 512 x 512, chi_max binding) run through the
    library at this precision; worst absolute error of its 24 amplitudes and of the
    256 Schmidt values of the updated bond against the oracle's."""
    import numpy as np
    g = json.load(open(GOLDEN))
    inp = W.update_chi256_inputs()
    d = B.MPS(inp["n"], inp["chi"], inp["eps"], prec)
    d.load(inp["B"], inp["lam"])
    rc = d.apply_gates([W.Gate(inp["first"], 2, inp["U"])], allow_noconv=True)
    oh, ol = np.array(g["schmidt_hi"]), np.array(g["schmidt_lo"])
    ah = np.array(g["amp_re_hi"]) + 1j * np.array(g["amp_im_hi"])
    al = np.array(g["amp_re_lo"]) + 1j * np.array(g["amp_im_lo"])
    dims_ok = d.bond_dims() == g["dims_after"]
    if prec:
        lh, ll = d.schmidt_dd(inp["first"])
        lam_err = float(np.max(np.abs((lh - oh) + (ll - ol)))) if dims_ok else float("inf")
        gh, gl = d.amplitudes(inp["bits"], dd=True)
        amp_err = float(np.max(np.abs((gh - ah) + (gl - al))))
    else:
        lam_err = float(np.max(np.abs(d.schmidt(inp["first"]) - (oh + ol)))) if dims_ok else float("inf")
        amp_err = float(np.max(np.abs(d.amplitudes(inp["bits"]) - (ah + al))))
    d.close()
    bound = 1e-26 if prec else 1e-12
    return {"max_abs_amplitude_error": amp_err, "max_abs_schmidt_error": lam_err, "bound": bound,
            "within_bound": bool(dims_ok and rc == 0 and amp_err <= bound and lam_err <= bound),
            "reference": "256-bit oracle, one chi=256 update (theta 512x512), 24 amplitudes"}


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
    """The 256-bit oracle as it stands, on all host threads (OpenMP), on a bounded
    sample of the workload:
      * the chi = 256 update of tests/golden/update_chi256.json (a = b = c = 256,
        theta 512 x 512, the bench's shape), run twice with the oracle's sweep limit
        at 1 and at 2: t1 = theta + one Jacobi sweep + truncation and split, t2 - t1 =
        one sweep.  The update's time is t1 + (S - 1)(t2 - t1) with S the oracle's own
        sweep count for that update (stored with the golden values);
      * configuration 1 in full (10 qubits, brickwork depth 10, chi_max = 32), timed
        end to end."""
    import oracle
    from paper_1111_3124_amd import workloads as W
    g = json.load(open(GOLDEN))
    S = int(g["split"]["sweeps"])
    inp = W.update_chi256_inputs()
    t = []
    try:
        for limit in (1, 2):
            om = oracle.OracleMPS(inp["n"], inp["chi"], inp["eps"])
            om.load(inp["B"], inp["lam"])
            oracle.set_max_sweeps(limit)
            t0 = time.perf_counter()
            try:
                om.apply(inp["first"], 2, inp["U"])
            except RuntimeError:  # stopped at the sweep limit, as intended
                pass
            t.append(time.perf_counter() - t0)
            om.close()
    finally:
        oracle.set_max_sweeps(80)
    sweep = t[1] - t[0]
    est = t[0] + (S - 1) * sweep
    gates = [gg for layer in W.brickwork(10, 10, 1) for gg in layer]
    om = oracle.OracleMPS(10, 32, 0.0)
    t0 = time.perf_counter()
    for gg in gates:
        om.apply_gate(gg)
    t_c1 = time.perf_counter() - t0
    om.close()
    return {"value": 1.0 / est, "unit": "gate updates/s", "cores": oracle.oracle_threads(), "kind": "oracle",
            "sample": f"one chi=256 update (a=b=c=256, theta 512x512) at 256 bits: theta+1 sweep+split "
                      f"{t[0]:.1f} s, one more sweep {sweep:.1f} s measured; x{S} sweeps (the oracle's own "
                      f"count for this update) = {est:.0f} s per update",
            "measured_s": t[0] + t[1],
            "config1": {"updates": len(gates), "seconds": t_c1, "updates_per_s": len(gates) / t_c1,
                        "workload": "10 qubits, brickwork depth 10, chi_max=32, eps=0, all 45 gates"}}


def batch_workload(B, W, prec: int, launch=None) -> dict:
    """Configuration 4: 256 independent brickwork circuits of Haar U(4) gates (seed 4:
    n ~ U{16..48}, chi_max ~ U{32, 64, 128, 256}, depth ~ U{8..24}, eps = 1e-12), all
    gates handed to one batch in a single call (layer-interleaved across circuits).
    Timed from the call to its return; states created and zeroed beforehand."""
    specs = W.batch_spec(256, 4)
    circ, gates = W.batch_gates(specs)
    bt = B.Batch([s.n for s in specs], [s.chi_max for s in specs], [1e-12] * len(specs), prec)
    for key, value in (launch or {}).items():
        bt.set_option(key, value)
    bt[0].set_option(B.MPS_OPT_KERNEL_TIMING, 1)
    bt[0].sync()
    t0 = time.perf_counter()
    rc = bt.run(circ, gates, allow_noconv=True)
    bt[0].sync()
    dt = time.perf_counter() - t0
    noconv = bt[0].kernel_time(B.COUNTER_NOCONV)[1]
    sweeps = bt[0].kernel_time(B.COUNTER_SWEEPS)[1]
    ktimes = {name: bt[0].kernel_time(c)[0] for c, name in enumerate(B.KERNEL_CLASSES)}
    multi = sum(1 for g in gates if g.k > 1)
    bt.close()
    return {"updates": multi, "seconds": dt, "rate": multi / dt, "noconv": noconv, "noconv_rc": rc != 0,
            "update_sweeps": sweeps, "kernel_ms": ktimes}


def triples_workload(B, W, prec: int, launch=None) -> dict:
    """Configuration 3: 30 qubits, 200 Haar U(8) gates on random contiguous triples
    (seed 3), chi_max = 512, eps = 1e-14, from |0...0>, all gates in one call."""
    gates = W.random_triples(30, 200, 3)
    m = B.MPS(30, 512, 1e-14, prec)
    for key, value in (launch or {}).items():
        m.set_option(key, value)
    m.set_option(B.MPS_OPT_KERNEL_TIMING, 1)
    m.sync()
    t0 = time.perf_counter()
    rc = m.apply_gates(gates, allow_noconv=True)
    m.sync()
    dt = time.perf_counter() - t0
    noconv = m.kernel_time(B.COUNTER_NOCONV)[1]
    ktimes = {name: m.kernel_time(c)[0] for c, name in enumerate(B.KERNEL_CLASSES)}
    dims = m.bond_dims()
    lam_ok = all(abs(float((m.schmidt(b) ** 2).sum()) - 1.0) < 1e-12 for b in range(29))
    m.close()
    return {"gates": len(gates), "seconds": dt, "rate": len(gates) / dt, "noconv": noconv, "noconv_rc": rc != 0,
            "max_bond_dim": max(dims), "saturated_bonds": sum(d == 512 for d in dims), "schmidt_normalised": lam_ok,
            "kernel_ms": ktimes}


def other_workload(B, W, name: str, want: str, launch) -> None:
    """One JSON line for configuration 4 (batch256) or 3 (triples), FP64 and dd."""
    fn, metric, unit = {
        "batch256": (batch_workload, "batched MPS gate updates/s (256 independent circuits)", "gate updates/s"),
        "triples": (triples_workload, "U(8) gate updates/s at chi_max=512", "U(8) gates/s")}[name]
    res = {}
    for k in (("fp64", "dd") if want in ("both", "auto") else (want,)):
        res[k] = fn(B, W, B.MPS_PREC_DD if k == "dd" else B.MPS_PREC_FP64, launch)
        print(f"# {name} {k}: {res[k]['rate']:.1f} {unit}", file=sys.stderr, flush=True)
    head = "dd" if "dd" in res else "fp64"
    line = {"metric": metric, "value": res[head]["rate"], "unit": unit, "n_gpus": 1, "higher_is_better": True,
            "dtype": "dd" if head == "dd" else "f64", "data": "synthetic",
            "config": {"workload": name}, "variants": res}
    print(json.dumps(line), flush=True)
    if any(v["noconv"] or v["noconv_rc"] for v in res.values()):
        print(f"bench.py: {name}: unconverged updates", file=sys.stderr, flush=True)
        sys.exit(3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variants", default="auto", help="fp64, dd, both or auto")
    ap.add_argument("--workload", default="chi256", choices=["chi256", "batch256", "triples"],
                    help="chi256: the headline line (chi = 256 updates); batch256: configuration 4 "
                         "(256 independent circuits); triples: configuration 3 (U(8) gates, chi_max 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tick-sweeps", type=int, default=None,
                    help="Jacobi sweeps per scheduler tick (1 or 2; default: the library's)")
    ap.add_argument("--graph", type=int, default=None,
                    help="1: replay the Jacobi sweeps from captured HIP graphs, 0: stream launches "
                         "(default: the library's)")
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
    launch = {}
    if args.tick_sweeps is not None:
        launch[B.MPS_OPT_TICK_SWEEPS] = args.tick_sweeps
    if args.graph is not None:
        launch[B.MPS_OPT_GRAPH] = args.graph
    dd_ok = True
    try:
        B.MPS(2, 2, 0.0, B.MPS_PREC_DD).close()
    except B.MPSError:
        dd_ok = False
    if want == "auto":
        want = "both" if dd_ok else "fp64"
    if args.workload != "chi256":
        other_workload(B, W, args.workload, want, launch)
        return
    results = {}
    if want in ("fp64", "both"):
        results["fp64"] = run_variant(B, W, B.MPS_PREC_FP64, args.steps, args.warmup, launch)
        results["fp64"]["error"] = golden_error(B, W, B.MPS_PREC_FP64)
        print(f"# fp64: {results['fp64']['rate']:.1f} updates/s, mean sweeps {results['fp64']['mean_sweeps']:.1f}",
              file=sys.stderr, flush=True)
    if want in ("dd", "both"):
        results["dd"] = run_variant(B, W, B.MPS_PREC_DD, args.steps, args.warmup, launch)
        results["dd"]["error"] = golden_error(B, W, B.MPS_PREC_DD)
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
                         "error_vs_oracle": v["error"], "noconv_updates": v["noconv"],
                         "mean_sweeps": v["mean_sweeps"], "mean_dd_sweeps": v["mean_dd_sweeps"],
                         "graphs": {"built": v["graphs_built"], "replays": v["graph_replays"]},
                         "kernel_ms": {n: t[0] for n, t in v["ktimes"].items()},
                         "schmidt_normalised": v["lam_ok"],
                         "roofline": roofline(v, 1 if k == "dd" else 0, k == "dd"),
                         "work_at_s_ref": work_at_s_ref(v["rate"])} for k, v in results.items()},
        "error_vs_oracle": r["error"],
        "noconv_updates": sum(v["noconv"] for v in results.values()),
        "roofline": roofline(r, 1 if head == "dd" else 0, head == "dd"),
    }
    bad = [k for k, v in results.items() if v["noconv"] or v["noconv_rc"] or not v["error"]["within_bound"]
           or not v["lam_ok"]]
    if bad:
        # an update that stopped at its sweep limit, or a result outside its error
        # bound, makes the measurement invalid: no line is reported
        print("bench.py: invalid run (" + ", ".join(
            f"{k}: noconv {results[k]['noconv']}, error {results[k]['error']}" for k in bad) + ")",
            file=sys.stderr, flush=True)
        sys.exit(3)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
