#!/usr/bin/env python3
"""Throughput of the dense FP64 triangular solve with many right-hand sides.

Workload: op(A) X = B with A lower-triangular n x n, no transpose, non-unit
diagonal, alpha = 1, n = nrhs = 8192, column-major, FP64; A's strict lower
part i.i.d. U(-1, 1) with diagonal 1 + sum |row|, B i.i.d. N(0, 1), seeded.
One step = restore B from a pristine device copy, then one full solve through
the C-ABI (redsea_trsm).  Flops are counted as n^2 * nrhs per solve.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (the MFMA product update, timed live with HIP events through the
library's trace API), the CPU oracle timed on a bounded sample of the
same workload (a subset of right-hand-side columns) on the host cores, and
the metric's mixed-precision leg: n = 16384, nrhs = 4096 at kappa_1 ~ 1e4,
plain FP64 against FP32 and BF16 inner solves with FP64 refinement to a
backward error of 1e-12 (wall time, refinement statistics, oracle-sampled
backward error).  `value` is the FP64 throughput of the n = 8192 workload.
A last key times the Cholesky factorisation built on the solve
(redsea_potrf, FP64 lower, n = 8192) with the oracle's componentwise
backward error on sampled entries.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK = 78.6  # TFLOP/s, MI355X dense FP64 matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2305_19917_amd", "csrc", "k_gemm.hip")


def measured_traffic(n, nrhs, variant, nb):
    """HBM bytes per product launch from the committed rocprofv3 counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None when
    they were taken on another workload or the product kernel's source
    changed since."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    if (rec.get("n"), rec.get("nrhs"), rec.get("variant"), rec.get("nb")) != (n, nrhs, variant, nb):
        return None
    return rec.get("bytes_per_launch")


def leaf_rows(nb):
    """Rows of the leaf kernel for leaf size nb (the library splits larger
    leaves recursively down to 256 rows)."""
    return 256 if nb >= 256 else min(nb, 128)


def algorithmic_bytes(n, nrhs, nb):
    """8 (MK + KN + 2MN) summed over the product launches of the recursive
    schedule down to leaves of nb rows, per launch (the unit of `traffic`)."""
    nb = leaf_rows(nb)
    total, count = 0, 0
    def split(rows):
        nonlocal total, count
        if rows <= nb:
            return
        nblk = (rows + nb - 1) // nb
        top = ((nblk + 1) // 2) * nb
        bot = rows - top
        split(top)
        total += 8 * (bot * top + top * nrhs + 2 * bot * nrhs)
        count += 1
        split(bot)
    split(n)
    return total / max(1, count)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(L, B, n, budget_s, threads):
    """Time the plain CPU oracle on a subset of columns of the same system."""
    import numpy as np
    import oracle
    # pilot: one column per thread
    cols = threads
    t0 = time.perf_counter()
    oracle.trsm_plain(0, 0, 0, 0, 1.0, L, np.asfortranarray(B[:, :cols]), nthreads=threads)
    pilot = time.perf_counter() - t0
    reps = max(1, int(budget_s / max(pilot, 1e-3)))
    cols = min(B.shape[1], threads * reps)
    t0 = time.perf_counter()
    oracle.trsm_plain(0, 0, 0, 0, 1.0, L, np.asfortranarray(B[:, :cols]), nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(float(n) * n * cols / dt / 1e12, 6), "unit": "TFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": "plain FP64 substitution of the first %d of %d right-hand-side columns of "
                      "the same n=%d system (%.1f s)" % (cols, B.shape[1], n, dt)}


# Constant-diagonal factor c of the kappa family (L_ii = c (1 + max row sum of
# |strict part|)) that gives kappa_1(L) ~ 1e4 at n = 16384 for the matrix key
# (2, 0, 0); found by bisection with the oracle's Hager-Higham estimate
# (9.6e3), stored with the other orders in tests/golden/kappa_family.json.
MIXED_C_KAPPA_1E4 = 0.009821718891880384


def mixed_leg(n, nrhs, reps, log):
    """The precision pattern at n = 16384, nrhs = 4096, kappa_1 ~ 1e4: plain
    FP64 against FP32 and BF16 inner solves with FP64 refinement, wall time
    of whole calls (conversions, every refinement step and the certifying
    residual included), the library's refinement statistics, and the
    oracle's normwise backward error on sampled columns."""
    import numpy as np
    import torch

    import oracle
    import paper_2305_19917_amd as rs
    import synth

    log("mixed leg: generating n=%d nrhs=%d" % (n, nrhs))
    L = synth.kappa_lower(n, MIXED_C_KAPPA_1E4, (2, 0, 0))
    B = synth.rhs_normal(n, nrhs, (2, 0, 1))
    dL = rs.fortran_tensor(L)
    dB0 = rs.fortran_tensor(B)
    dB = dB0.clone()
    cols = [0, nrhs // 3, 2 * nrhs // 3, nrhs - 1]
    Bs = np.asfortranarray(B[:, cols])
    flops = float(n) * n * nrhs
    stream = torch.cuda.current_stream()

    def timed(call):
        times, st = [], None
        for r in range(reps + 1):
            dB.copy_(dB0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st = call()
            e1.record(stream)
            e1.synchronize()
            if r > 0:  # the first call warms up
                times.append(e0.elapsed_time(e1))
        times.sort()
        return times[len(times) // 2], st

    out = {"workload": "FP64 in/out TRSM left/lower/no-transpose/non-unit, n=%d, nrhs=%d, "
                       "constant-diagonal family at kappa_1 ~ 1e4 (c=%.6g), recursive schedule, "
                       "leaf nb=256; refinement to normwise backward error <= 1e-12"
                       % (n, nrhs, MIXED_C_KAPPA_1E4),
           "reps": reps, "sampled_columns": cols}
    legs = [("fp64", lambda: rs.trsm(dL, dB, variant="recursive", nb=256, stream=stream)),
            ("fp32_ir", lambda: rs.trsm_mixed(dL, dB, inner=1, stream=stream)),
            ("bf16_ir", lambda: rs.trsm_mixed(dL, dB, inner=2, stream=stream)),
            # labelled variants: the residual by exact integer emulation on the
            # INT8 matrix cores (Ozaki scheme II) instead of FP64 products
            ("fp32_ir_int8res", lambda: rs.trsm_mixed(dL, dB, inner=1 | rs.RESIDUAL_INT8,
                                                      stream=stream)),
            ("bf16_ir_int8res", lambda: rs.trsm_mixed(dL, dB, inner=2 | rs.RESIDUAL_INT8,
                                                      stream=stream))]
    for name, call in legs:
        log("mixed leg: %s" % name)
        ms, st = timed(call)
        Xs = dB[:, cols].cpu().numpy()
        rec = {"ms": round(ms, 3), "tflops_effective": round(flops / (ms * 1e-3) / 1e12, 3),
               "eta_oracle": oracle.backward_error(0, 0, 0, 0, 1.0, L, Bs, Xs)}
        if name != "fp64":
            rec.update(iterations=st.iterations, fell_back=st.fell_back, eta_library=st.eta)
        out[name] = rec
    for name in ("fp32_ir", "bf16_ir", "fp32_ir_int8res", "bf16_ir_int8res"):
        out[name]["speed_vs_fp64"] = round(out["fp64"]["ms"] / out[name]["ms"], 4)
    return out


def cholesky_leg(n, reps, log):
    """redsea_potrf, FP64 lower, n x n symmetric diagonally dominant matrix
    (off-diagonal U(-1, 1) mirrored, diagonal 1 + row sum of magnitudes):
    median time of `reps` factorisations after a warm-up (the matrix restored
    by a device copy outside the events), n^3/3 TFLOP/s, info, the time per
    kernel class of one traced factorisation, and the oracle's componentwise
    backward error max |A - L L^T| / (|L||L^T|) on sampled entries.  Any
    failure is reported in the record, never raised."""
    try:
        import numpy as np
        import torch

        import oracle
        import paper_2305_19917_amd as rs
        import synth

        log("cholesky leg: generating n=%d" % n)
        A = synth.spd_dominant(n, (140, n, 0))
        dA0 = rs.fortran_tensor(A)
        dA = dA0.clone()
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream()
        times = []
        for r in range(reps + 1):
            dA.copy_(dA0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rs.potrf(dA, info=info, stream=stream)
            e1.record(stream)
            e1.synchronize()
            if r > 0:
                times.append(e0.elapsed_time(e1))
        times.sort()
        ms = times[len(times) // 2]
        dA.copy_(dA0)
        rs.trace_begin()
        rs.potrf(dA, info=info, stream=stream)
        torch.cuda.synchronize()
        tr = rs.trace_end()
        F = np.tril(dA.cpu().numpy())
        g = synth.rng((140, n, 1))
        i = g.integers(0, n, size=1000)
        j = np.minimum((g.random(1000) * (i + 1)).astype(np.int64), i)
        pairs = np.concatenate([np.stack([i, j], axis=1), [[n - 1, n - 1], [n - 1, 0]]])
        return {"workload": "FP64 Cholesky (redsea_potrf) lower, n=%d, leaf order 128, "
                            "symmetric diagonally dominant" % n,
                "reps": reps, "ms": round(ms, 3),
                "tflops": round(n ** 3 / 3.0 / (ms * 1e-3) / 1e12, 3),
                "info": int(info.item()),
                "kernel_ms": {k: round(v[1], 3) for k, v in tr.items() if v[0]},
                "omega_sampled": oracle.chol_backward_error(0, A, F, pairs)}
    except Exception as e:  # the headline line must not depend on this leg
        return {"error": repr(e)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--nrhs", type=int, default=8192)
    ap.add_argument("--variant", default="recursive")
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--mixed-reps", type=int, default=3)
    ap.add_argument("--no-cholesky", action="store_true", help="skip the Cholesky leg")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the solve shards by right-hand-side columns "
              "across GPUs, but this build runs and reports a single MI355X (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2305_19917_amd as rs
    import synth

    if not os.path.exists(rs.LIB_PATH):
        from paper_2305_19917_amd import build as libbuild
        libbuild.build()
    rs.lib()
    n, nrhs = args.n, args.nrhs
    log("generating n=%d nrhs=%d" % (n, nrhs))
    L = synth.dominant_lower(n, (1, 0, 0))
    B = synth.rhs_normal(n, nrhs, (1, 0, 1))
    dev = torch.device("cuda:0")
    dA = rs.fortran_tensor(L, dev)
    dB0 = rs.fortran_tensor(B, dev)
    dB = rs.fortran_tensor(np.zeros((n, nrhs)), dev)
    stream = torch.cuda.current_stream()

    def step():
        dB.copy_(dB0)
        rs.trsm(dA, dB, variant=args.variant, nb=args.nb, stream=stream)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    log("timed %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    flops = float(n) * n * nrhs
    value = flops / (ms_per_step * 1e-3) / 1e12

    # solve-only time per step (events around the solve, restore excluded)
    solve_ms = []
    for _ in range(args.steps):
        dB.copy_(dB0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rs.trsm(dA, dB, variant=args.variant, nb=args.nb, stream=stream)
        e1.record(stream)
        e1.synchronize()
        solve_ms.append(e0.elapsed_time(e1))
    solve_ms.sort()
    solve_med = solve_ms[len(solve_ms) // 2]

    # dominant kernel: the product update, timed per launch with HIP events on
    # the library's stream over the same number of steps
    log("traced %d steps" % args.steps)
    rs.trace_begin()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tr = rs.trace_end()
    g_launch, g_ms, g_fl = tr["gemm"]
    achieved = g_fl / (g_ms * 1e-3) / 1e12 if g_ms > 0 else 0.0
    shares = {k: round(v[1] / args.steps, 4) for k, v in tr.items()}

    # sampled parity of the final result against the CPU oracle
    import oracle
    cols = [0, nrhs // 2, nrhs - 1]
    Xs = dB[:, cols].cpu().numpy()
    eta = oracle.backward_error(0, 0, 0, 0, 1.0, L, np.asfortranarray(B[:, cols]), Xs)

    mixed = None if args.no_mixed else mixed_leg(16384, 4096, args.mixed_reps, log)
    chol = None if args.no_cholesky else cholesky_leg(8192, 3, log)

    cpu = None
    if not args.no_cpu_baseline:
        # the host's CPU share for one GPU (OMP_NUM_THREADS on the GPU machines),
        # at most every core the host has
        threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
        log("cpu baseline, %d threads" % threads)
        cpu = cpu_baseline(L, B, n, args.cpu_seconds, threads)
        cpu["cpu_model"] = cpu_model()
        cpu["host_cores"] = os.cpu_count()

    out = {
        "metric": "TRSM TFLOP/s (n\u00b2\u00b7nrhs): FP64 vs BF16/FP32+refine at backward err \u22641e-12",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 TRSM left/lower/no-transpose/non-unit, n=%d, nrhs=%d, "
                               "alpha=1, column-major, %s schedule, leaf nb=%d"
                               % (n, nrhs, args.variant, args.nb),
                   "n": n, "nrhs": nrhs, "variant": args.variant, "nb": args.nb},
        "solve_ms_median": round(solve_med, 4),
        "solve_tflops": round(flops / (solve_med * 1e-3) / 1e12, 3),
        "frac_of_fp64_peak": round(value / FP64_MFMA_PEAK, 4),
        "kernel_ms_per_step": shares,
        "eta_sampled": eta,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK, 4),
                     "traffic": measured_traffic(n, nrhs, args.variant, args.nb),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": (round(algorithmic_bytes(n, nrhs, args.nb))
                                                      if args.variant == "recursive" else None),
                     "kernel": "gemm_dma_kernel (FP64 product update, all tiles)",
                     "launches_per_step": g_launch // max(1, args.steps)},
        "cpu_baseline": cpu,
        "mixed": mixed,
        "cholesky": chol,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
