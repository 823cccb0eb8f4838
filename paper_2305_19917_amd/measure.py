"""Measurements of the solver on the workloads it is specified for, one JSON
line per result (python -m paper_2305_19917_amd.measure [rows ...]).

Rows:
  peak     achievable FP64/FP32 MFMA rate (the library's MFMA-only probe),
           device-to-device copy bandwidth, and the vendor FP64 GEMM
           (torch.matmul) as an achievable-GEMM reference
  small    FP64 lower/N/non-unit, n = 512, nrhs = 64: microseconds per solve
  thin     FP64 n = 8192, nrhs = 1024: upper/transposed and lower/unit-diagonal
           (diagonal stored as NaN), plus lower/N for nrhs in {1, 8, 32}, with
           the HBM rate implied by the algorithmic bytes
  sides    FP64 n = nrhs = 8192: all side / uplo / trans combinations, and the
           triangular product (redsea_trmm) on the matrix cores and by INT8
           emulation
  mixed    FP64 in/out, n = 16384, nrhs = 4096, conditioning family with
           kappa_1 in {1e2, 1e4, 1e6}: plain FP64 against FP32 + FP64 refinement
           and BF16 + FP64 refinement (effective TFLOP/s of the whole call,
           iterations and the library's own final backward error)
  mixed1e4 the same at kappa_1 ~ 1e4 only, one timed repetition (for tracing)
  batched  2000 systems, n log-uniform in [32, 1024], nrhs in [1, 256], FP64
           and FP32: every task shape, the autotuner's pick, and one plan
           launch with that pick (eager and hipGraph replay)
  potrf    Cholesky factorisation (redsea_potrf), FP64 lower, n in {2048,
           4096, 8192, 16384} x leaf order {32, 64, 128}, then FP64 upper and
           FP32 lower at n = 8192: milliseconds, n^3/3 TFLOP/s and the time
           per kernel class from the library trace
  potrf8192  FP64 lower n = 8192 with the default leaf only (for profiling)
  blockedla  FP64 n = 8192, blocked model, nb 256, nrhs in {128, 512, 1024}:
           look-ahead off against on (REDSEA_LOOKAHEAD = 0 / 1)

Timing: hipEvents on the stream, B restored by a device copy outside the
events, median of the repetitions.  Inputs are the seeded synthetic systems of
the `synth` module.  Accuracy is checked by the tests, not here.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _emit(rec):
    print(json.dumps(rec), flush=True)


def _time(fn, restore, reps):
    import torch
    st = torch.cuda.current_stream()
    restore()
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        restore()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def row_peak():
    import torch
    import paper_2305_19917_amd as rs
    rec = {"row": "peak", "mfma_f64_tflops": round(rs.mfma_peak("f64"), 2),
           "mfma_f32_tflops": round(rs.mfma_peak("f32"), 2),
           "datasheet_f64_tflops": 78.6, "datasheet_f32_tflops": 157.3, "datasheet_hbm_tbs": 8.0}
    n = 1 << 27  # 1 GiB of doubles
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    ms = _time(lambda: b.copy_(a), lambda: None, 10)
    rec["copy_tbs"] = round(2 * 8 * n / (ms * 1e-3) / 1e12, 3)
    del a, b
    for m in (4096, 8192):
        x = torch.randn(m, m, dtype=torch.float64, device="cuda")
        y = torch.randn(m, m, dtype=torch.float64, device="cuda")
        ms = _time(lambda: torch.matmul(x, y), lambda: None, 5)
        rec["torch_dgemm_%d_tflops" % m] = round(2.0 * m ** 3 / (ms * 1e-3) / 1e12, 2)
        del x, y
    torch.cuda.empty_cache()
    _emit(rec)


def row_small():
    import torch
    import paper_2305_19917_amd as rs
    import synth
    n, nrhs = 512, 64
    L = synth.dominant_lower(n, (0, 0, 0))
    B = synth.rhs_normal(n, nrhs, (0, 0, 1))
    dL, dB0 = rs.fortran_tensor(L), rs.fortran_tensor(B)
    dB = dB0.t().clone().t()
    out = {"row": "small", "n": n, "nrhs": nrhs}
    for variant, nb in (("recursive", 64), ("recursive", 128), ("recursive", 256),
                        ("iterative", 128), ("iterative", 256), ("blocked", 64)):
        ms = _time(lambda: rs.trsm(dL, dB, variant=variant, nb=nb), lambda: dB.copy_(dB0), 200)
        out["%s_nb%d_us" % (variant, nb)] = round(ms * 1e3, 2)
    _emit(out)


def row_thin():
    import torch
    import paper_2305_19917_amd as rs
    import synth
    n = 8192
    L = synth.dominant_lower(n, (1, 0, 0))
    dL = rs.fortran_tensor(L)

    def report(tag, nrhs, A, side_args, reps):
        B = synth.rhs_normal(n, nrhs, (1, 0, 1))
        dB0 = rs.fortran_tensor(B)
        dB = dB0.t().clone().t()
        ms = _time(lambda: rs.trsm(A, dB, *side_args, variant="recursive", nb=256),
                   lambda: dB.copy_(dB0), reps)
        flops = float(n) * n * nrhs
        byts = 8.0 * (n * (n + 1) / 2 + 2.0 * n * nrhs)
        _emit({"row": "thin", "case": tag, "n": n, "nrhs": nrhs, "ms": round(ms, 4),
               "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
               "algorithmic_gbs": round(byts / (ms * 1e-3) / 1e9, 1),
               "roof_ms_fp64": round(flops / 78.6e12 * 1e3, 4), "roof_ms_hbm": round(byts / 8e12 * 1e3, 4)})

    U = np.asfortranarray(L.T)
    dU = rs.fortran_tensor(U)
    report("left upper T", 1024, dU, ("L", "U", "T", "N"), 10)
    del dU
    Lu = synth.unit_lower(n, (1, 0, 0))
    dLu = rs.fortran_tensor(Lu)
    report("left lower N unit", 1024, dLu, ("L", "L", "N", "U"), 10)
    del dLu
    for nrhs in (1, 8, 32, 1024):
        report("left lower N", nrhs, dL, ("L", "L", "N", "N"), 10)


def row_thincross():
    """The one-launch thin solve against the split recursive schedule (the
    REDSEA_THIN switch) and the best iterative leaf, over orders and
    right-hand-side counts up to the thin limit of 64."""
    import os
    import paper_2305_19917_amd as rs
    import synth
    for n in (512, 1024, 2048, 4096, 8192):
        L = synth.dominant_lower(n, (1, 0, 0))
        dL = rs.fortran_tensor(L)
        for nrhs in (1, 4, 16, 32, 64):
            B = synth.rhs_normal(n, nrhs, (1, 0, 1))
            dB0 = rs.fortran_tensor(B)
            dB = dB0.t().clone().t()
            out = {"row": "thincross", "n": n, "nrhs": nrhs}
            for tag, env, variant, nb in (("thin_ms", "1", "recursive", 256), ("split_ms", "0", "recursive", 256),
                                          ("iterative256_ms", "0", "iterative", 256)):
                os.environ["REDSEA_THIN"] = env
                out[tag] = round(_time(lambda: rs.trsm(dL, dB, variant=variant, nb=nb),
                                       lambda: dB.copy_(dB0), 10), 4)
            os.environ.pop("REDSEA_THIN", None)
            _emit(out)


def row_widecross():
    """The one-launch solve over column groups against the split recursive
    and the iterative schedules, from 64 right-hand sides up."""
    import os
    import paper_2305_19917_amd as rs
    import synth
    for n in (512, 2048, 4096, 8192):
        L = synth.dominant_lower(n, (1, 0, 0))
        dL = rs.fortran_tensor(L)
        for nrhs in (64, 96, 128, 192, 256, 512, 1024):
            B = synth.rhs_normal(n, nrhs, (1, 0, 1))
            dB0 = rs.fortran_tensor(B)
            dB = dB0.t().clone().t()
            out = {"row": "widecross", "n": n, "nrhs": nrhs}
            for tag, env, variant in (("thin_ms", "1", "recursive"), ("split_ms", "0", "recursive"),
                                      ("iterative256_ms", "0", "iterative")):
                os.environ["REDSEA_THIN"] = env
                out[tag] = round(_time(lambda: rs.trsm(dL, dB, variant=variant, nb=256),
                                       lambda: dB.copy_(dB0), 5), 4)
            os.environ.pop("REDSEA_THIN", None)
            out["thin_tflops"] = round(float(n) * n * nrhs / (out["thin_ms"] * 1e-3) / 1e12, 2)
            _emit(out)
            del dB, dB0


# Constant-diagonal factors c of the kappa family at n = 16384 (matrix key
# (2, 0, 0)) and the one-norm condition numbers they give, estimated with the
# Hager-Higham estimator when the table of the family was made.
KAPPA_FAMILY_16384 = ((1e2, 0.10366329284376985, 100.5), (1e4, 0.009821718891880384, 9608.0),
                      (1e6, 0.0032196784442513815, 959245.0))


def row_sides():
    """f2: every flag combination at n = 8192 with 8192 right-hand sides (the
    right side solves X op(A) = B with B of 8192 rows), and the triangular
    product (redsea_trmm) on both methods, TFLOP/s of n^2 nrhs."""
    import torch
    import paper_2305_19917_amd as rs
    import synth
    n = nrhs = 8192
    L = synth.dominant_lower(n, (1, 0, 0))
    B = synth.rhs_normal(n, nrhs, (1, 0, 1))
    dL = rs.fortran_tensor(L)
    dU = rs.fortran_tensor(np.asfortranarray(L.T))
    dB0 = rs.fortran_tensor(B)
    dB = dB0.t().clone().t()
    flops = float(n) * n * nrhs
    out = {"row": "sides", "n": n, "nrhs": nrhs}
    for side in ("L", "R"):
        for uplo, A in (("L", dL), ("U", dU)):
            for trans in ("N", "T"):
                ms = _time(lambda: rs.trsm(A, dB, side, uplo, trans, "N", variant="recursive", nb=256),
                           lambda: dB.copy_(dB0), 5)
                out["trsm_%s%s%s_tflops" % (side, uplo, trans)] = round(flops / (ms * 1e-3) / 1e12, 2)
    dC = dB0.t().clone().t()
    for method in ("mfma", "int8"):
        ms = _time(lambda: rs.trmm(dL, dB0, dC, alpha=-1.0, beta=1.0, method=method),
                   lambda: dC.copy_(dB0), 5)
        out["trmm_%s_ms" % method] = round(ms, 3)
        out["trmm_%s_tflops" % method] = round(flops / (ms * 1e-3) / 1e12, 2)
    _emit(out)


def row_mixed(targets=(1e2, 1e4, 1e6), reps=3):
    import torch
    import paper_2305_19917_amd as rs
    import synth
    n, nrhs = 16384, 4096
    for target, c, kappa1 in KAPPA_FAMILY_16384:
        if target not in targets:
            continue
        e = {"target": target, "kappa1": kappa1}
        L = synth.kappa_lower(n, c, (2, 0, 0))
        B = synth.rhs_normal(n, nrhs, (2, 0, 1))
        dL, dB0 = rs.fortran_tensor(L), rs.fortran_tensor(B)
        dB = dB0.t().clone().t()
        rec = {"row": "mixed", "n": n, "nrhs": nrhs, "kappa_target": e["target"], "kappa1": e["kappa1"]}
        for name, fn in (("fp64", lambda: rs.trsm(dL, dB, variant="recursive", nb=256)),
                         ("fp32_ir", lambda: rs.trsm_mixed(dL, dB, inner=1)),
                         ("bf16_ir", lambda: rs.trsm_mixed(dL, dB, inner=2)),
                         ("fp32_ir_int8res", lambda: rs.trsm_mixed(dL, dB, inner=1 | rs.RESIDUAL_INT8)),
                         ("bf16_ir_int8res", lambda: rs.trsm_mixed(dL, dB, inner=2 | rs.RESIDUAL_INT8))):
            ms = _time(fn, lambda: dB.copy_(dB0), reps)
            dB.copy_(dB0)
            st = fn()
            torch.cuda.synchronize()
            r = {"ms": round(ms, 3), "tflops_eff": round(float(n) * n * nrhs / (ms * 1e-3) / 1e12, 3)}
            if isinstance(st, rs.MixedStats):
                r.update({"iterations": st.iterations, "eta": st.eta, "fell_back": st.fell_back})
            rec[name] = r
        _emit(rec)
        del dL, dB0, dB
        torch.cuda.empty_cache()


def row_batched():
    import torch
    import paper_2305_19917_amd as rs
    import synth
    ns, ks = synth.batch_shapes(2000, (3, 0, 2))
    flops = float((ns.astype(float) ** 2 * ks).sum())
    for dt, es in ((np.float64, 8), (np.float32, 4)):
        byts = float(sum(es * (n * (n + 1) / 2 + 2.0 * n * k) for n, k in zip(ns, ks)))
        As = [rs.fortran_tensor(synth.dominant_lower(int(n), (3, i, 0)).astype(dt)) for i, n in enumerate(ns)]
        Bs = [rs.fortran_tensor(synth.rhs_normal(int(n), int(k), (3, i, 1)).astype(dt))
              for i, (n, k) in enumerate(zip(ns, ks))]
        info = torch.zeros(len(Bs), dtype=torch.int32, device="cuda")
        # every task shape on this batch, and the autotuner's pick (which it
        # makes on generated systems of the same shapes)
        per_tile = {}
        for tile in range(1, 13):
            p_t = rs.BatchPlan(As, Bs, tile=tile)
            per_tile[tile] = round(_time(lambda: p_t.run(info), lambda: None, 10), 4)
            p_t.close()
        best, tune_ms = rs.batched_tune(ns, ks, dtype="f64" if es == 8 else "f32", reps=3)
        plan = rs.BatchPlan(As, Bs, tile=best)
        ms = _time(lambda: plan.run(info), lambda: None, 20)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=s):
            plan.run(info, stream=s)
        torch.cuda.synchronize()
        gms = _time(lambda: g.replay(), lambda: None, 20)
        _emit({"row": "batched", "dtype": np.dtype(dt).name, "systems": len(Bs), "tile": best,
               "ms_per_tile": per_tile, "tuner_ms_per_tile": [round(x, 4) for x in tune_ms],
               "ms": round(ms, 4),
               "graph_ms": round(gms, 4), "systems_per_s": round(len(Bs) / (gms * 1e-3)),
               "tflops": round(flops / (gms * 1e-3) / 1e12, 3),
               "algorithmic_gbs": round(byts / (gms * 1e-3) / 1e9, 1),
               "info_nonzero": int((info != 0).sum().item())})
        plan.close()
        del As, Bs, g
        torch.cuda.empty_cache()


def row_batchedfp64(tile=1, runs=5):
    """The FP64 batch of the batched row at one task shape, plain launches
    only (no graph, no tuning): the command the counter runs profile."""
    import torch
    import paper_2305_19917_amd as rs
    import synth
    ns, ks = synth.batch_shapes(2000, (3, 0, 2))
    As = [rs.fortran_tensor(synth.dominant_lower(int(n), (3, i, 0))) for i, n in enumerate(ns)]
    Bs = [rs.fortran_tensor(synth.rhs_normal(int(n), int(k), (3, i, 1))) for i, (n, k) in enumerate(zip(ns, ks))]
    info = torch.zeros(len(Bs), dtype=torch.int32, device="cuda")
    plan = rs.BatchPlan(As, Bs, tile=tile)
    ms = _time(lambda: plan.run(info), lambda: None, runs)
    byts = float(sum(8 * (n * (n + 1) / 2 + 2.0 * n * k) for n, k in zip(ns, ks)))
    _emit({"row": "batchedfp64", "tile": tile, "runs": runs + 1, "ms": round(ms, 4),
           "algorithmic_bytes": byts, "info_nonzero": int((info != 0).sum().item())})
    plan.close()


def row_potrf(ns=(2048, 4096, 8192, 16384), nbs=(32, 64, 128), reps=3, extra=True):
    import torch
    import paper_2305_19917_amd as rs
    import synth
    cases = [(n, nb, "L", torch.float64) for n in ns for nb in nbs]
    if extra:
        cases += [(8192, 0, "U", torch.float64), (8192, 0, "L", torch.float32)]
    made = {}
    for n, nb, uplo, dt in cases:
        if (n, dt) not in made:
            made.clear()
            torch.cuda.empty_cache()
            A0 = rs.fortran_tensor(synth.spd_dominant(n, (140, n, 0))).to(dt)
            made[(n, dt)] = (A0, A0.clone())
        A0, A = made[(n, dt)]
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        ms = _time(lambda: rs.potrf(A, uplo=uplo, nb=nb, info=info), lambda: A.copy_(A0), reps)
        A.copy_(A0)
        rs.trace_begin()
        rs.potrf(A, uplo=uplo, nb=nb, info=info)
        torch.cuda.synchronize()
        tr = rs.trace_end()
        _emit({"row": "potrf", "n": n, "nb": nb or "default", "uplo": uplo,
               "dtype": "f64" if dt == torch.float64 else "f32", "ms": round(ms, 4),
               "tflops": round(n ** 3 / 3.0 / (ms * 1e9), 3), "info": int(info.item()),
               "kernel_ms": {k: round(v[1], 4) for k, v in tr.items() if v[0]},
               "launches": {k: v[0] for k, v in tr.items() if v[0]}})


def row_blockedla(n=8192, widths=(128, 512, 1024), nb=256, reps=5):
    import paper_2305_19917_amd as rs
    import synth
    dL = rs.fortran_tensor(synth.dominant_lower(n, (1, 0, 0)))
    for nrhs in widths:
        dB0 = rs.fortran_tensor(synth.rhs_normal(n, nrhs, (1, 0, 1)))
        dB = dB0.clone()
        rec = {"row": "blockedla", "n": n, "nrhs": nrhs, "nb": nb}
        for la in ("0", "1"):
            os.environ["REDSEA_LOOKAHEAD"] = la
            ms = _time(lambda: rs.trsm(dL, dB, variant="blocked", nb=nb), lambda: dB.copy_(dB0),
                       reps)
            rec["ms_lookahead_" + ("off" if la == "0" else "on")] = round(ms, 4)
        os.environ.pop("REDSEA_LOOKAHEAD", None)
        rec["tflops_on"] = round(float(n) * n * nrhs / (rec["ms_lookahead_on"] * 1e9), 3)
        _emit(rec)


ROWS = {"peak": row_peak, "small": row_small, "thin": row_thin, "thincross": row_thincross,
        "widecross": row_widecross,
        "sides": row_sides,
        "mixed": row_mixed,
        "mixed1e4": lambda: row_mixed((1e4,), reps=1), "batched": row_batched,
        "batchedfp64": row_batchedfp64, "potrf": row_potrf,
        "potrf8192": lambda: row_potrf((8192,), (0,), reps=3, extra=False),
        "blockedla": row_blockedla}


def main(argv):
    names = argv or list(ROWS)
    for name in names:
        t0 = time.perf_counter()
        print("# row %s" % name, file=sys.stderr, flush=True)
        ROWS[name]()
        print("# row %s done in %.1f s" % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
