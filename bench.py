#!/usr/bin/env python3
"""Benchmark of the emulated-FP64 (Ozaki scheme) GEMM and two-site H_eff.psi on
one MI355X, against the native FP64 MFMA GEMM on the same GPU.

Headline (one JSON line on stdout): emulated-FP64 TFLOP/s (2 n^3 / wall time of
one ozaki_dgemm call, exponents + slicing + pair GEMMs + recombination) for the
square n = 8192 GEMM with N(0,1) 2^u entries, u in [-10, 10], at the smallest
slice count whose error against the double-double reference is no larger than
that of the native FP64 MFMA GEMM ("equal error").  The last stdout line is a
compact record (a few KB): the headline, the roofline of the dominant kernel
(the int8 pair GEMM, timed with HIP events on its own stream), the CPU oracle
timed on a bounded sample, the FP64 rates and errors, and the H_eff.psi
applies/s and Davidson figures as scalars.  Every section's full tables go to
the file named by --full-json; progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sampled_rows(n, count, seed=1):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(count, n), replace=False))


def time_calls(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def phase_means(ctx, names):
    out = {}
    rec = ctx.phase_times()
    for nm in names:
        v = [t for (p, t) in rec if p == nm]
        out[nm] = (float(np.mean(v)) if v else None, len(v))
    return out


def gemm_section(args, ozaki, ctx, torch, oracle):
    from paper_2510_04795_amd import workloads as wl
    n = args.n
    log("[bench] generating n=%d GEMM operands" % n)
    A, B = wl.gemm_pair(n, U=10, seed=0)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    rows = sampled_rows(n, args.err_rows)
    log("[bench] double-double reference on %d sampled rows" % len(rows))
    t0 = time.perf_counter()
    hi, lo = oracle.dgemm_dd(A[rows], B)
    absAB = np.abs(A[rows]) @ np.abs(B)
    log("[bench]   dd reference %.1f s" % (time.perf_counter() - t0))
    flops = 2.0 * n * n * n
    idx = torch.from_numpy(rows).cuda()

    def errs(X):
        x = X[idx].cpu().numpy()
        return oracle.rel_frobenius(x, hi, lo), oracle.componentwise(x, hi, lo, absAB)

    results = []
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    # native FP64 MFMA
    ctx.dgemm(dA, dB, slices=0, C=C)
    err64, cw64 = errs(C)
    ctx.set_timing(True)
    t = time_calls(lambda: ctx.dgemm(dA, dB, slices=0, C=C), args.steps, args.warmup, torch)
    ph = phase_means(ctx, ["fp64"])
    fp64 = {"slices": 0, "ms": t * 1e3, "tflops": flops / t / 1e12, "rel_frobenius": err64,
            "componentwise": cw64, "kernel_ms": ph["fp64"][0], "frac_of_fp64_peak": flops / t / 1e12 / FP64_PEAK_TFLOPS}
    log("[bench] fp64 mfma: %.3f ms  %.2f TFLOP/s  relF %.2e" % (t * 1e3, fp64["tflops"], err64))

    # a plain device copy of known size (1 GiB read + 1 GiB written): the
    # reference that scales the HBM byte counters of rocprofv3 --pmc runs
    cal = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    cal2 = torch.empty_like(cal)
    cal2.copy_(cal)
    torch.cuda.synchronize()
    del cal, cal2
    # external reference: the vendor FP64 GEMM behind torch.mm (rocBLAS / hipBLASLt)
    Ct = torch.mm(dA, dB)
    err_t, cw_t = errs(Ct)
    t = time_calls(lambda: torch.mm(dA, dB, out=Ct), args.steps, args.warmup, torch)
    vendor = {"ms": t * 1e3, "tflops": flops / t / 1e12, "rel_frobenius": err_t, "componentwise": cw_t,
              "frac_of_fp64_peak": flops / t / 1e12 / FP64_PEAK_TFLOPS,
              "note": "torch.mm float64 (vendor BLAS), timed as an external reference"}
    log("[bench] vendor fp64 (torch.mm): %.3f ms  %.2f TFLOP/s  relF %.2e" % (t * 1e3, vendor["tflops"], err_t))
    del Ct

    if args.gemm_configs:
        configs = [tuple(int(v) for v in c.split(":")) for c in args.gemm_configs.split(",")]
    else:
        configs = [(S, G) for S in range(4, 9) for G in (S, S + 1)]
    ws = ctx.workspace(n, n, n, 8, 9)
    for (S, G) in configs:
        if args.variant >= 0:
            ctx.set_variant(S, G, args.variant)
            variant, tune_ms = args.variant, {}
        else:
            # pick the tile variant by timing them all on this GEMM (outside the timed region)
            variant, tune_ms = ctx.tune(dA, dB, slices=S, ndiag=G, C=C, workspace=ws)
        ctx.dgemm(dA, dB, slices=S, ndiag=G, C=C, workspace=ws)
        err, cw = errs(C)
        ctx.phase_times()
        t = time_calls(lambda: ctx.dgemm(dA, dB, slices=S, ndiag=G, C=C, workspace=ws),
                       args.steps, args.warmup, torch)
        ph = phase_means(ctx, ["slice", "pair"])
        P = ozaki.pair_count(S, G)
        pair_ms = ph["pair"][0]
        slice_ms = ph["slice"][0]
        r = {"slices": S, "ndiag": G, "pairs": P, "variant": variant,
             "tune_ms": {str(k): round(v, 4) for k, v in tune_ms.items()},
             "ms": t * 1e3, "tflops": flops / t / 1e12,
             "rel_frobenius": err, "componentwise": cw, "pair_kernel_ms": pair_ms, "slice_ms": slice_ms,
             "int8_tops": P * flops / (pair_ms * 1e-3) / 1e12 if pair_ms else None}
        r["int8_frac"] = r["int8_tops"] / INT8_PEAK_TOPS if r["int8_tops"] else None
        # slicing: read A and B (8 B per element, twice: exponent pass + slice pass),
        # write S bytes per element of each
        r["slice_gbs"] = (2 * n * n * (16 + S)) / (slice_ms * 1e-3) / 1e9 if slice_ms else None
        r["slice_hbm_frac"] = r["slice_gbs"] / HBM_PEAK_GBS if slice_ms else None
        results.append(r)
        log("[bench] S=%d G=%d P=%2d v%d: %.3f ms  %.2f TFLOP/s  relF %.2e comp %.2e  pair %.3f ms "
            "(%.1f%% int8 peak) slice %.3f ms" % (S, G, P, variant, t * 1e3, r["tflops"], err, cw, pair_ms or 0,
                                                  100 * (r["int8_frac"] or 0), slice_ms or 0))
    ctx.set_timing(False)
    S_a, G_a, st = ctx.choose_slices(dA, dB)
    auto = {"slices": S_a, "ndiag": G_a, "predicted_error": st["predicted"],
            "predicted_native_error": st["native"], "rho_a": st["rho_a"], "rho_b": st["rho_b"]}
    log("[bench] automatic width: S=%d G=%d (predicted relF %.2e, native %.2e)"
        % (S_a, G_a, st["predicted"], st["native"]))
    eq = [r for r in results if r["rel_frobenius"] <= err64]
    chosen = min(eq, key=lambda r: r["ms"]) if eq else min(results, key=lambda r: r["rel_frobenius"])
    tol = [r for r in results if r["rel_frobenius"] <= 1e-12]
    at_1e12 = min(tol, key=lambda r: r["ms"]) if tol else None
    return {"n": n, "fp64": fp64, "vendor_fp64": vendor, "emulated": results, "chosen": chosen,
            "at_1e-12": at_1e12, "rows_for_error": len(rows), "auto": auto}, (A, B)


def gemm_case(ozaki, ctx, torch, oracle, n, U, err_rows, steps, warmup, slices=range(4, 9)):
    """One square GEMM workload: native FP64 (own kernel and vendor) and the
    emulated GEMM for every (S, G) in {S, S+1}, each with its tuned tile
    variant, errors against the double-double reference on sampled rows."""
    from paper_2510_04795_amd import workloads as wl
    A, B = wl.gemm_pair(n, U=U, seed=0)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    rows = sampled_rows(n, err_rows)
    hi, lo = oracle.dgemm_dd(A[rows], B)
    absAB = np.abs(A[rows]) @ np.abs(B)
    idx = torch.from_numpy(rows).cuda()
    flops = 2.0 * n ** 3
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")

    def errs(X):
        x = X[idx].cpu().numpy()
        return oracle.rel_frobenius(x, hi, lo), oracle.componentwise(x, hi, lo, absAB)

    out = {"n": n, "U": U, "rows_for_error": len(rows)}
    ctx.dgemm(dA, dB, slices=0, C=C)
    rf, cw = errs(C)
    t = time_calls(lambda: ctx.dgemm(dA, dB, slices=0, C=C), steps, warmup, torch)
    out["fp64"] = {"ms": t * 1e3, "tflops": flops / t / 1e12, "rel_frobenius": rf, "componentwise": cw}
    if n <= 1024:
        # the plain FP64 definition on the CPU, all rows: same error class
        naive = oracle.dgemm_fp64(A, B)
        out["fp64"]["max_abs_diff_vs_cpu_naive_fp64"] = float(np.max(np.abs(C.cpu().numpy() - naive)))
    Ct = torch.mm(dA, dB)
    rf, cw = errs(Ct)
    t = time_calls(lambda: torch.mm(dA, dB, out=Ct), steps, warmup, torch)
    out["vendor_fp64"] = {"ms": t * 1e3, "tflops": flops / t / 1e12, "rel_frobenius": rf, "componentwise": cw}
    del Ct
    ws = ctx.workspace(n, n, n, 8, 9)
    res = []
    for S in slices:
        for G in (S, S + 1):
            v, _ = ctx.tune(dA, dB, slices=S, ndiag=G, C=C, workspace=ws)
            ctx.dgemm(dA, dB, slices=S, ndiag=G, C=C, workspace=ws)
            rf, cw = errs(C)
            t = time_calls(lambda: ctx.dgemm(dA, dB, slices=S, ndiag=G, C=C, workspace=ws), steps, warmup, torch)
            res.append({"slices": S, "ndiag": G, "variant": v, "ms": t * 1e3, "tflops": flops / t / 1e12,
                        "rel_frobenius": rf, "componentwise": cw})
    out["emulated"] = res
    # emulation modes: the automatic width and the performant path for this shape
    S_a, G_a, st = ctx.choose_slices(dA, dB)
    auto = {"slices": S_a, "ndiag": G_a, "rho_a": st["rho_a"], "rho_b": st["rho_b"],
            "predicted_error": st["predicted"], "predicted_native_error": st["native"]}
    hit = [r for r in res if (r["slices"], r["ndiag"]) == (S_a, G_a)]
    if hit:
        auto["rel_frobenius"] = hit[0]["rel_frobenius"]
        auto["ms"] = hit[0]["ms"]
    # performant dispatch at the 53-bit width (the automatic width re-reads the
    # operand statistics on every call, which would dominate small shapes)
    aw = ctx.auto_workspace(n, n, n)
    _, S_p, G_p = ctx.dgemm_auto(dA, dB, bits=53, performant=True, C=C, workspace=aw)
    t = time_calls(lambda: ctx.dgemm_auto(dA, dB, bits=53, performant=True, C=C, workspace=aw),
                   steps, warmup, torch)
    auto["performant"] = {"slices": S_p, "ndiag": G_p, "ms": t * 1e3, "tflops": flops / t / 1e12,
                          "path": "emulated" if S_p else "native fp64"}
    out["auto"] = auto
    eq = [r for r in res if r["rel_frobenius"] <= out["fp64"]["rel_frobenius"]]
    out["equal_error"] = min(eq, key=lambda r: r["ms"]) if eq else None
    log("[bench] n=%d U=%d: fp64 %.3f ms (relF %.2e), vendor %.3f ms; equal error: %s"
        % (n, U, out["fp64"]["ms"], out["fp64"]["rel_frobenius"], out["vendor_fp64"]["ms"],
           None if not eq else "S=%d G=%d %.3f ms %.1f TFLOP/s" % (out["equal_error"]["slices"],
                                                                   out["equal_error"]["ndiag"],
                                                                   out["equal_error"]["ms"],
                                                                   out["equal_error"]["tflops"])))
    log("[bench]   automatic width: S=%d G=%d (relF %s); performant at 53 bits: %s %.3f ms"
        % (S_a, G_a, "%.2e" % auto["rel_frobenius"] if "rel_frobenius" in auto else "-",
           auto["performant"]["path"], auto["performant"]["ms"]))
    for r in res:
        log("[bench]   S=%d G=%d v%d %.3f ms %.1f TFLOP/s relF %.2e comp %.2e"
            % (r["slices"], r["ndiag"], r["variant"], r["ms"], r["tflops"], r["rel_frobenius"], r["componentwise"]))
    return out


def sweep_section(args, ozaki, ctx, torch, oracle):
    cases = [(512, 10), (2048, 10), (4096, 10), (2048, 30), (4096, 30), (8192, 30)]
    return [gemm_case(ozaki, ctx, torch, oracle, n, U, min(args.err_rows, n), args.steps, args.warmup)
            for (n, U) in cases]


PAIR_SOURCES = ["internal.h", "asm_steps.h", "pairgemm_impl.h", "pairgemm.hip"] + ["pairgemm_s%d.hip" % s for s in range(2, 9)]
COUNTERS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                             "pair_gemm_n8192_hbm_counters.txt")


def pair_bytes(n, S):
    """Algorithmic HBM bytes of one pair-GEMM launch on square n: both packed
    operands read once (S bytes per element), exponents read, C written."""
    return 2 * S * n * n + 2 * 4 * n + 8 * n * n


def pair_source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2510_04795_amd", "csrc")
    for f in PAIR_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pair_traffic(n, S, G, variant):
    """HBM bytes per pair-GEMM launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the plain-copy calibration),
    or None when there is none for this case or the kernel sources changed
    since the counters were taken."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    meta, rows = {}, {}
    with open(COUNTERS_FILE) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "=" in line:
                k, v = line.split("=", 1)
                meta[k.strip()] = v.strip()
                continue
            f = line.split()
            if f[0].isdigit():
                rows[(int(f[0]), int(f[1]), int(f[2]), int(f[3]))] = (float(f[5]), float(f[6]))
    if meta.get("source_sha256") != pair_source_hash():
        return None
    got = rows.get((n, S, G, variant))
    if got is None:
        return None
    fetch_kib, write_kib = got
    return (fetch_kib * float(meta["fetch_factor"]) + write_kib * float(meta["write_factor"])) * 1024.0


def heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, S, G=0, diag=None):
    dL = torch.from_numpy(Lf).cuda()
    dR = torch.from_numpy(Rf).cuda()
    dd = torch.from_numpy(diag).cuda() if diag is not None else None
    t0 = time.perf_counter()
    plan = ozaki.HeffPlan(ctx, layout, dL, dR, triples, diag=dd, slices=S, ndiag=G)
    torch.cuda.synchronize()
    return plan, time.perf_counter() - t0, (dL, dR, dd)


def dense_dd_reference(oracle, L, R, psi, pairs, cols):
    """sigma[i, j, r] = sum_k L_k[i, :] psi[:, j, :] R_k[r, :]^T for the sampled
    (i, j) in pairs and r in cols, to double-double accuracy: u_k = L_k[i, :]
    psi_j by the oracle's double-double GEMM, then u_k R_k[cols, :]^T the same
    way (the low part of u_k in FP64), the 2 Kop partial sums added exactly.
    Returns (flat indices into sigma, values)."""
    from fractions import Fraction
    kop, D, _ = L.shape
    phys = psi.shape[1]
    idx, val = [], []
    for (i, j) in pairs:
        pj = np.ascontiguousarray(psi[:, j, :])
        acc = [Fraction(0)] * len(cols)
        for k in range(kop):
            uh, ul = oracle.dgemm_dd(L[k][i:i + 1], pj)
            Rt = np.ascontiguousarray(R[k][cols, :].T)
            h, l = oracle.dgemm_dd(uh, Rt)
            lo = ul @ Rt
            for c in range(len(cols)):
                acc[c] += Fraction(float(h[0, c])) + Fraction(float(l[0, c])) + Fraction(float(lo[0, c]))
        for c, r in enumerate(cols):
            idx.append((i * phys + j) * D + r)
            val.append(float(acc[c]))
    return np.array(idx), np.array(val)


def heff_section(args, ozaki, ctx, torch, name, layout, Lf, Rf, pf, triples, slices_list, dd_ref=None):
    """Warm applies/s (operator slices cached), error against the FP64 plan
    and, when dd_ref = (indices, values) is given, against double-double
    values of sampled outputs."""
    dpsi = torch.from_numpy(pf).cuda()
    out = {"workload": name, "n": int(pf.size)}

    def dd_err(sig):
        if dd_ref is None:
            return None
        got = sig[torch.from_numpy(dd_ref[0]).cuda()].cpu().numpy()
        return float(np.max(np.abs(got - dd_ref[1])) / np.max(np.abs(dd_ref[1])))

    sig64, nrm = None, None
    if not args.heff_no_fp64:
        plan, tplan, keep = heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, 0)
        sig64 = plan.apply(dpsi)
        t = time_calls(lambda: plan.apply(dpsi, sig64), args.heff_steps, 1, torch)
        out["flops_per_apply"] = plan.flops
        out["fp64"] = {"ms": t * 1e3, "applies_per_s": 1.0 / t, "tflops": plan.flops / t / 1e12,
                       "frac_of_fp64_peak": plan.flops / t / 1e12 / FP64_PEAK_TFLOPS, "plan_s": tplan,
                       "rel_err_vs_dd_sampled": dd_err(sig64)}
        log("[bench] %s fp64: %.3f ms/apply  %.2f TFLOP/s  vs dd %s" % (name, t * 1e3, plan.flops / t / 1e12,
                                                                        out["fp64"]["rel_err_vs_dd_sampled"]))
        nrm = torch.linalg.vector_norm(sig64).item()
        plan.close()
        del keep
    res = []
    for (S, G) in slices_list:
        plan, tplan, keep = heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, S, G)
        out["flops_per_apply"] = plan.flops
        sig = plan.apply(dpsi)
        err = None if sig64 is None else torch.linalg.vector_norm(sig - sig64).item() / nrm
        # warm applies replay the plan's captured graph
        t = time_calls(lambda: plan.apply(dpsi, sig), args.heff_steps, 1, torch)
        # phase split: the same launches issued directly, with events between phases
        ctx.set_timing(True)
        ctx.phase_times()
        napplies = 2
        for _ in range(napplies):
            plan.apply(dpsi, sig)
        torch.cuda.synchronize()
        ph = ctx.phase_times()
        ctx.set_timing(False)
        phs = {}
        for (nm, ms) in ph:
            phs.setdefault(nm, []).append(ms)
        phs = {k: float(np.sum(v)) / napplies for k, v in phs.items()}
        P = ozaki.pair_count(S, G)
        r = {"slices": S, "ndiag": G, "pairs": P, "ms": t * 1e3, "applies_per_s": 1.0 / t,
             "tflops": plan.flops / t / 1e12, "rel_frobenius_vs_fp64": err, "plan_s": tplan,
             "rel_err_vs_dd_sampled": dd_err(sig),
             "cold_ms": (t + tplan) * 1e3, "phase_ms": phs,
             "tile_variants": list(plan.variants), "streamed_launches": list(plan.launches),
             "chunks": plan.chunks, "plan_bytes": plan.bytes[0], "plan_T_bytes": plan.bytes[1],
             "phase_choice": {"L": list(plan.phase(0)), "R": list(plan.phase(1))},
             "int8_frac_pair_phases": (P * plan.flops / ((phs.get("heff_L", 0) + phs.get("heff_R", 0)) * 1e-3)
                                       / 1e12 / INT8_PEAK_TOPS) if phs else None}
        res.append(r)
        log("[bench] %s S=%d G=%d: %.3f ms/apply  %.2f TFLOP/s  err vs fp64 %s  vs dd %s  phases %s  "
            "choice L %s R %s (variant:order:launch)  chunks %d  plan %.2f GiB (T %.2f GiB)"
            % (name, S, G, t * 1e3, r["tflops"], err, r["rel_err_vs_dd_sampled"],
               {k: round(v, 3) for k, v in phs.items()}, ":".join(map(str, plan.phase(0))),
               ":".join(map(str, plan.phase(1))), plan.chunks, plan.bytes[0] / 2 ** 30, plan.bytes[1] / 2 ** 30))
        plan.close()
        del keep
    out["emulated"] = res
    return out


def heff_slices(args):
    return [(int(v), int(v)) for v in args.heff_slices.split(",")]


def davidson_section(args, ozaki, ctx, torch):
    from paper_2510_04795_amd import workloads as wl
    D = args.dav_d
    log("[bench] Davidson problem D=%d (n=%d), Kop=32" % (D, D * D))
    prob = wl.davidson_problem(D=D, kop=32)
    layout, Lf, Rf, _, triples = wl.flatten_dense(prob.L, prob.R, prob.x0[:, None, :])
    hd = torch.from_numpy(prob.hdiag.ravel().copy()).cuda()
    x0 = torch.from_numpy(prob.x0.ravel().copy()).cuda()
    out = {"D": D, "n": D * D, "kop": 32, "tol": 1e-8, "runs": []}
    e64 = None
    for S in (int(x) for x in args.dav_slices.split(",")):
        plan, tplan, keep = heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, S, 0,
                                           diag=prob.delta.ravel().copy())
        dav = ozaki.Davidson(ctx, plan, hd, x0, m_max=32, tol=1e-8, max_iter=300)
        torch.cuda.synchronize()
        # every step synchronises (theta and rho come back to the host); the
        # first two capture the step graphs, later steps replay them
        t0 = time.perf_counter()
        t2, nsteps = None, 0
        while True:
            info = dav.step()
            nsteps += 1
            if nsteps == 2:
                t2 = time.perf_counter()
            if info.status != ozaki.OZ_OK:
                break
        t = time.perf_counter() - t0
        steady = (time.perf_counter() - t2) / (nsteps - 2) * 1e3 if nsteps > 2 else None
        theta, status, its, res = info.theta, ozaki.STATUS[info.status], info.iter, info.resnorm
        if S == 0:
            e64 = theta
        r = {"slices": S, "energy": theta, "status": status, "iterations": its, "residual": res,
             "ms_per_iteration": t / max(its, 1) * 1e3, "ms_per_iteration_after_capture": steady,
             "matvec_flops": plan.flops, "energy_error_vs_fp64": None if S == 0 or e64 is None else abs(theta - e64)}
        out["runs"].append(r)
        log("[bench] Davidson S=%d: E=%.12f  %s in %d it  (%.2f ms/it, %s ms/it after the graph captures)  |dE|=%s"
            % (S, theta, status, its, r["ms_per_iteration"], "%.2f" % steady if steady else "-",
               r["energy_error_vs_fp64"]))
        dav.close()
        plan.close()
        del keep
    return out


def dispatch_section(args, ozaki, ctx, torch):
    """Emulated (S = 6) against native FP64 on the block-sparse batch by block
    size: the triples grouped by their largest sector, each group applied
    as a plan of its own, best of 3 x 20 applies per path.  Whether a
    per-block choice between the two paths could gain anything."""
    from paper_2510_04795_amd import workloads as wl
    prob = wl.heff_sparse()
    d = prob.dims
    out = []
    for lo, hi in [(1, 64), (65, 128), (129, 256), (257, 512), (513, 1 << 30)]:
        tr = [t for t in prob.triples if lo <= max(d[t[1]], d[t[2]], d[t[3]], d[t[4]]) <= hi]
        if not tr:
            continue
        sub = wl.HeffSparse(dims=prob.dims, psi_blocks=prob.psi_blocks, psi=prob.psi, L=prob.L, R=prob.R,
                            triples=tr)
        layout, Lf, Rf, pf, triples = wl.flatten_sparse(sub)
        psi = torch.from_numpy(pf).cuda()
        r = {"largest_sector": [lo, hi], "triples": len(tr)}
        for S in (6, 0):
            plan, _, keep = heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, S, 0)
            sig = plan.apply(psi)
            for _ in range(5):
                plan.apply(psi, sig)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(3):
                t0 = time.perf_counter()
                for _ in range(20):
                    plan.apply(psi, sig)
                torch.cuda.synchronize()
                best = min(best, (time.perf_counter() - t0) / 20 * 1e3)
            r["flops"] = plan.flops
            r["emulated_ms" if S else "fp64_ms"] = round(best, 4)
            plan.close()
            del keep
        r["fp64_over_emulated"] = round(r["fp64_ms"] / r["emulated_ms"], 3)
        log("[bench] dispatch by size: largest sector %d..%d, %d triples: emulated %.3f ms, FP64 %.3f ms (x%.2f)"
            % (lo, hi, len(tr), r["emulated_ms"], r["fp64_ms"], r["fp64_over_emulated"]))
        out.append(r)
    return out


def stability_section(args, ozaki, ctx, torch):
    """Low-slice stability of the two Krylov solvers (the paper's numerical
    stability study): for several independent H_eff problems (standing in
    for the successive steps of a sweep), Davidson and Lanczos at S = 2, 3, 4
    and residual thresholds 1e-2 .. 1e-8, against the FP64 ground energy E0
    of the same problem (FP64 Lanczos to 1e-10).  Reported per solver, S and
    threshold: iterations (mean over problems), statuses, the largest
    |E - E0| / |E0| and the number of non-variational energies (E below E0 by
    more than 1e-13 |E0|)."""
    from paper_2510_04795_amd import workloads as wl
    D, kop, nprob = args.stab_d, 8, args.stab_problems
    tols = [1e-2, 1e-3, 1e-4, 1e-5, 1e-8]
    log("[bench] stability study: %d problems D=%d (n=%d), Kop=%d" % (nprob, D, D * D, kop))
    acc = {}
    for seed in range(nprob):
        prob = wl.davidson_problem(D=D, kop=kop, seed=seed)
        layout, Lf, Rf, _, triples = wl.flatten_dense(prob.L, prob.R, prob.x0[:, None, :])
        hd = torch.from_numpy(prob.hdiag.ravel().copy()).cuda()
        x0 = torch.from_numpy(prob.x0.ravel().copy()).cuda()
        e0 = None
        for S in [0, 2, 3, 4]:
            plan, tplan, keep = heff_flat_plan(ozaki, ctx, torch, layout, Lf, Rf, triples, S, 0,
                                               diag=prob.delta.ravel().copy())
            if S == 0:
                lz = ozaki.Lanczos(ctx, plan, x0, m_max=32, tol=1e-10, max_iter=600)
                e0, st, _, _ = lz.run()
                lz.close()
                if st != "converged":
                    raise RuntimeError("FP64 reference Lanczos did not converge (%s)" % st)
            for tol in tols:
                for method in ("davidson", "lanczos"):
                    if method == "davidson":
                        sol = ozaki.Davidson(ctx, plan, hd, x0, m_max=32, tol=tol, max_iter=300)
                    else:
                        sol = ozaki.Lanczos(ctx, plan, x0, m_max=32, tol=tol, max_iter=300)
                    th, st, its, _ = sol.run()
                    sol.close()
                    r = acc.setdefault((method, S, tol), {"iterations": [], "status": {}, "rel_err": [],
                                                          "nonvariational": 0})
                    r["iterations"].append(its)
                    r["status"][st] = r["status"].get(st, 0) + 1
                    r["rel_err"].append((th - e0) / abs(e0))
                    if th < e0 - 1e-13 * abs(e0):
                        r["nonvariational"] += 1
            plan.close()
            del keep
    rows = []
    for (method, S, tol), r in sorted(acc.items()):
        rows.append({"solver": method, "slices": S, "tol": tol,
                     "mean_iterations": float(np.mean(r["iterations"])),
                     "status": r["status"], "max_abs_rel_err": float(np.max(np.abs(r["rel_err"]))),
                     "min_rel_err": float(np.min(r["rel_err"])), "nonvariational": r["nonvariational"]})
        log("[bench] stability %-8s S=%d tol=%.0e: it %.1f  %s  max|dE/E| %.2e  non-variational %d/%d"
            % (method, S, tol, rows[-1]["mean_iterations"], r["status"], rows[-1]["max_abs_rel_err"],
               r["nonvariational"], nprob))
    return {"D": D, "n": D * D, "kop": kop, "problems": nprob, "m_max": 32, "rows": rows}


def rdm_section(args, ozaki, ctx, torch):
    """Truncation and renormalisation (the site-update steps beside the H_eff
    diagonalisation) with their linear algebra emulated at S slices or in
    native FP64, as in the paper's numerical-stability discussion: rho =
    psi psi^T of a planted two-site tensor (Schmidt values known), its D
    dominant eigenpairs by the block-Jacobi solver, and U^T O U for Kop
    block operators.  Errors are against the planted spectrum and subspace
    (truncation) and against the FP64 renormalisation."""
    from paper_2510_04795_amd import workloads as wl
    n, D, kop = args.rdm_n, args.rdm_n // 4, args.rdm_kop
    log("[bench] RDM truncation: rho %d x %d, keep D=%d; renormalisation of %d operators" % (n, n, D, kop))
    t = wl.two_site_psi(n, seed=12)
    psi = torch.from_numpy(t.psi).cuda()
    s2 = t.schmidt ** 2
    dw_exact = float(s2[D:].sum())
    left = torch.from_numpy(np.ascontiguousarray(t.left[:, :D])).cuda()
    out = {"n": n, "D": D, "kop": kop, "spectrum": "s_i^2 ~ exp(-i / (n/64)), unit trace", "truncation": [],
           "renormalisation": []}
    U64 = None
    for S in [0, 2, 3, 4, 5, 6, 7, 8]:
        eig = ozaki.RdmEig(ctx, n, S)
        ozaki.truncate(ctx, psi, D, slices=S, eig=eig, max_sweeps=1)  # warm-up (allocations, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, w, dw, info = ozaki.truncate(ctx, psi, D, slices=S, eig=eig, max_sweeps=args.rdm_sweeps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        eig.close()
        wn = w.cpu().numpy()
        orth = float((U.T @ U - torch.eye(D, dtype=torch.float64, device=U.device)).abs().max().item())
        sv = torch.linalg.svdvals(left.T @ U)
        r = {"slices": S, "ms": ms, "sweeps": info.sweeps, "status": ozaki.STATUS[info.status],
             "eig_rel_err": float(np.max(np.abs(wn - s2[:D])) / s2[0]),
             "discarded_weight": dw, "discarded_weight_err": abs(dw - dw_exact),
             "orthogonality": orth, "subspace_err": float(1.0 - sv.min().item())}
        out["truncation"].append(r)
        log("[bench] truncation S=%d: %.1f ms, %d sweeps (%s), eig err %.1e, dw err %.1e, |U^T U - I| %.1e, "
            "subspace %.1e" % (S, ms, info.sweeps, r["status"], r["eig_rel_err"], r["discarded_weight_err"], orth,
                               r["subspace_err"]))
        if S == 0:
            U64 = U
    rho = ctx.dgemm(psi, psi, slices=0, transb="T")
    torch.linalg.eigh(rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    torch.linalg.eigh(rho)
    torch.cuda.synchronize()
    out["vendor_eigh_ms"] = (time.perf_counter() - t0) * 1e3
    log("[bench] vendor FP64 eigh (torch.linalg.eigh) of rho: %.1f ms" % out["vendor_eigh_ms"])
    ops = [torch.from_numpy(o).cuda() for o in wl.block_operators(n, kop, seed=13)]
    ref = None
    for S in [0, 3, 6, 7]:
        ws = torch.empty(ozaki._lib.ozaki_renormalize_workspace_bytes(n, D, S, 0), dtype=torch.uint8, device="cuda")
        res = ctx.renormalize(U64, ops, slices=S, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.renormalize(U64, ops, slices=S, workspace=ws, outs=res)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if S == 0:
            ref = [x.clone() for x in res]
        err = max(float(torch.linalg.norm(a - b).item() / torch.linalg.norm(b).item()) for a, b in zip(res, ref))
        flops = kop * (2.0 * n * n * D + 2.0 * D * D * n)
        out["renormalisation"].append({"slices": S, "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
                                       "rel_err_vs_fp64": err})
        log("[bench] renormalisation S=%d: %.2f ms for %d operators (%.1f TFLOP/s), rel err vs FP64 %.1e"
            % (S, ms, kop, flops / (ms * 1e-3) / 1e12, err))
    return out


def oracle_section(args, oracle):
    """The CPU oracle timed beside the H_eff and Davidson workloads, on the
    host's cores (bounded samples, each stated):
      dense   full emulated O4 (S = 6) of the dense recipe at D = 256, Kop = 64,
              phys 16, and one row alpha' of the D = 2048 benchmark shape;
      sparse  full emulated O4 (S = 6) and FP64 O4 of the 40-sector batch, or
              its first triples when the whole batch would exceed the budget;
      davidson  FP64 Davidson at D = 16 (to convergence) and one FP64 matvec
              of the D = 1024, Kop = 32 operator (the per-iteration cost)."""
    from paper_2510_04795_amd import workloads as wl
    out = {"cores": oracle.num_threads(), "cpu_model": cpu_model()}
    t0 = time.perf_counter()
    L, R, psi = wl.heff_dense(D=256, kop=64, phys=16)
    t1 = time.perf_counter()
    oracle.heff_dense(L, R, psi, S=6)
    t = time.perf_counter() - t1
    fl = 64.0 * 64 * 256 ** 3
    out["dense_d256_kop64_s6"] = {"s": t, "tflops": fl / t / 1e12, "flops": fl, "sample": "full O4, D=256 Kop=64 phys=16"}
    log("[bench] oracle dense D=256 Kop=64 S=6: %.1f s (%.4f TFLOP/s)" % (t, fl / t / 1e12))
    del L, R, psi
    L, R, psi = wl.heff_dense(D=args.heff_d, kop=args.heff_kop, phys=16)
    t1 = time.perf_counter()
    oracle.heff_dense_rows(L, R, psi, [args.heff_d // 2], S=6)
    t = time.perf_counter() - t1
    # one output row: per operator pair, the row of L_k times the D x 16D view
    # of psi, then that 16 x D row block times R_k^T
    fl_row = 2.0 * args.heff_kop * 16 * args.heff_d * (args.heff_d + args.heff_d)
    out["dense_benchmark_row_s6"] = {"s": t, "rows": 1, "flops": fl_row, "tflops": fl_row / t / 1e12,
                                     "full_apply_s_extrapolated": t * args.heff_d,
                                     "sample": "one row alpha' (all j, beta') of D=%d Kop=%d phys=16, incl. the "
                                               "column split of Psi" % (args.heff_d, args.heff_kop)}
    log("[bench] oracle dense D=%d one row S=6: %.1f s (x%d rows = %.0f s per apply)"
        % (args.heff_d, t, args.heff_d, t * args.heff_d))
    del L, R, psi
    prob = wl.heff_sparse()
    tri = list(prob.triples)
    for S in (6, 0):
        t1 = time.perf_counter()
        n_used = 0
        sub_t = []
        for k in range(0, len(tri), 100):
            sub = wl.HeffSparse(dims=prob.dims, psi_blocks=prob.psi_blocks, psi=prob.psi, L=prob.L, R=prob.R,
                                triples=tri[k:k + 100])
            oracle.heff_sparse(sub, S=S)
            n_used = k + 100
            if time.perf_counter() - t1 > args.oracle_seconds:
                break
        t = time.perf_counter() - t1
        frac = min(n_used, len(tri)) / len(tri)
        key = "sparse_s6" if S else "sparse_fp64"
        out[key] = {"s": t, "triples": min(n_used, len(tri)), "full_apply_s_extrapolated": t / frac,
                    "sample": "O4 over the first %d of %d triples (each 100-triple slice from zero sigma)"
                              % (min(n_used, len(tri)), len(tri))}
        log("[bench] oracle sparse %s: %d triples in %.1f s (full apply ~%.1f s)"
            % ("S=6" if S else "FP64", min(n_used, len(tri)), t, t / frac))
    prob16 = wl.davidson_problem(D=16, kop=32)
    t1 = time.perf_counter()
    th, _, st, its, _ = oracle.davidson(oracle.heff_matvec(prob16.L, prob16.R, prob16.delta), prob16.hdiag, prob16.x0)
    out["davidson_d16_fp64"] = {"s": time.perf_counter() - t1, "iterations": its, "status": st, "energy": th}
    prob = wl.davidson_problem(D=args.dav_d, kop=32)
    mv = oracle.heff_matvec(prob.L, prob.R, prob.delta)
    t1 = time.perf_counter()
    mv(prob.x0.ravel())
    t = time.perf_counter() - t1
    out["davidson_d1024_fp64_matvec"] = {"s": t, "sample": "one FP64 matvec of D=%d Kop=32 (one Davidson iteration's "
                                                           "dominant cost)" % args.dav_d}
    log("[bench] oracle Davidson D=16: %d iterations; FP64 matvec D=%d: %.2f s" % (its, args.dav_d, t))
    out["total_s"] = time.perf_counter() - t0
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def device_record(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "memory_gib": round(p.total_memory / 2 ** 30, 1)}


def cpu_baseline(oracle, A, B, S, G, seconds):
    """The oracle's emulated GEMM at the chosen (S, G) on a bounded sample of
    rows of A (all of B), sized from a probe so that the timed run takes about
    ``seconds`` (the per-call slicing of B and the per-row cost estimated from
    two probes); the rate is scaled as 2 * rows * n^2 / time."""
    n = A.shape[0]
    # two probes separate the per-call cost (slicing all of B) from the per-row cost
    tp = []
    for k in (8, 24):
        probe = sampled_rows(n, k, seed=2)
        t0 = time.perf_counter()
        oracle.ozaki_dgemm(A[probe], B, S, G)
        tp.append(time.perf_counter() - t0)
    per_row = max((tp[1] - tp[0]) / 16, tp[1] / 24 / 4, 1e-9)
    fixed = max(tp[0] - 8 * per_row, 0.0)
    count = int(min(max((seconds - fixed) / per_row, 8), n))
    rows = sampled_rows(n, count, seed=2)
    t0 = time.perf_counter()
    oracle.ozaki_dgemm(A[rows], B, S, G)
    t = time.perf_counter() - t0
    return {"value": 2.0 * len(rows) * n * n / t / 1e12, "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "emulated GEMM (S=%d, G=%d) of %d sampled rows of A (n=%d) times all of B, "
                      "%.1f s; rate scaled as 2*rows*n*n/time" % (S, G, len(rows), n, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--err-rows", type=int, default=256,
                    help="rows of the n = 8192 product checked against the double-double reference")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the timed CPU-oracle sample")
    ap.add_argument("--full-json", default="bench_full.json",
                    help="file for the full record (every section's tables); '' to skip")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-seconds", type=float, default=10.0,
                    help="budget of each bounded oracle sample in the oracle section")
    ap.add_argument("--sections", default="gemm,dense,sparse,davidson,dispatch,stability,rdm,sweep,oracle",
                    help="comma list of gemm, dense, sparse, davidson, dispatch, stability, rdm, sweep, oracle; without gemm "
                         "(profiling runs) the last line holds the sections' records, not the headline")
    ap.add_argument("--gemm-configs", default="",
                    help="comma list of S:G for the GEMM section (default: S = 4..8, G in {S, S+1})")
    ap.add_argument("--variant", type=int, default=-1,
                    help="fixed pair-GEMM tile variant for the GEMM section (default: tuned per S, G)")
    ap.add_argument("--heff-d", type=int, default=2048)
    ap.add_argument("--heff-kop", type=int, default=64)
    ap.add_argument("--heff-steps", type=int, default=3)
    ap.add_argument("--heff-slices", default="6,7,8", help="comma list of S (G = S) for the H_eff sections")
    ap.add_argument("--heff-no-fp64", action="store_true", help="skip the FP64 H_eff plans (profiling runs)")
    ap.add_argument("--heff-variant", type=int, default=-1,
                    help="fixed pair-GEMM tile variant for the H_eff plans, with plan timing off (profiling runs)")
    ap.add_argument("--heff-fix", default="",
                    help="fixed phase choices of the emulated H_eff plans, e.g. L=0:1:256,R=4:1:0 "
                         "(variant:order:launch per phase, as the bench log prints them); nothing is timed")
    ap.add_argument("--heff-launch", type=int, default=-1,
                    help="H_eff grouped launch: -1 timed choice, 0 one workgroup per tile, k > 0 streamed on k "
                         "CUs, -2 resident first phase, -3 paired-term second phase")
    ap.add_argument("--dd-samples", type=int, default=3,
                    help="(i, j) pairs of the dense sigma checked against double-double (4 columns each)")
    ap.add_argument("--dav-d", type=int, default=1024)
    ap.add_argument("--dav-slices", default="0,4,5,6,7,8",
                    help="comma list of S for the Davidson section (0 = native FP64, the reference of |dE|)")
    ap.add_argument("--rdm-n", type=int, default=2048)
    ap.add_argument("--rdm-kop", type=int, default=16)
    ap.add_argument("--rdm-sweeps", type=int, default=40)
    ap.add_argument("--stab-d", type=int, default=96)
    ap.add_argument("--stab-problems", type=int, default=6)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import oracle
    from paper_2510_04795_amd import ozaki
    torch.cuda.init()
    ctx = ozaki.Context(0)
    sections = set(args.sections.split(","))
    from paper_2510_04795_amd import workloads as wl
    ctx.set_heff_launch(args.heff_launch)
    for item in filter(None, args.heff_fix.split(",")):
        ph, spec = item.split("=")
        v, o, l = (int(x) for x in spec.split(":"))
        ctx.set_heff_phase({"L": 0, "R": 1}[ph], v, o, l)
    gemm = None
    if "gemm" in sections:
        gemm, (A, B) = gemm_section(args, ozaki, ctx, torch, oracle)
        chosen = gemm["chosen"]
        cpu = None
        if not args.no_cpu:
            log("[bench] CPU oracle sample")
            cpu = cpu_baseline(oracle, A, B, chosen["slices"], chosen["ndiag"], args.cpu_seconds)
        del A, B
    # the GEMM section fixed its tuned tile variant per (S, G) in the context;
    # the H_eff plans time their own per phase (unless one is forced here)
    for S in range(2, 9):
        for G in sorted({S, S + 1, 2 * S - 1}):
            ctx.set_variant(S, G, -1)
    if args.heff_variant >= 0:
        ctx.set_autotune(False)
        for S, _ in heff_slices(args):
            ctx.set_variant(S, S, args.heff_variant)
    extra = {}
    if "dense" in sections:
        log("[bench] generating dense two-site problem D=%d Kop=%d phys=16" % (args.heff_d, args.heff_kop))
        L, R, psi = wl.heff_dense(D=args.heff_d, kop=args.heff_kop, phys=16)
        layout, Lf, Rf, pf, triples = wl.flatten_dense(L, R, psi)
        dd_ref = None
        if args.dd_samples > 0:
            t0 = time.perf_counter()
            rng = np.random.default_rng(3)
            pairs = [(int(rng.integers(args.heff_d)), int(rng.integers(16))) for _ in range(args.dd_samples)]
            cols = sorted(int(c) for c in rng.choice(args.heff_d, 4, replace=False))
            dd_ref = dense_dd_reference(oracle, L, R, psi, pairs, cols)
            log("[bench] double-double reference of %d sigma entries: %.1f s" % (len(dd_ref[0]),
                                                                                time.perf_counter() - t0))
        del L, R, psi
        extra["heff_dense"] = heff_section(
            args, ozaki, ctx, torch, "dense D=%d Kop=%d phys=16" % (args.heff_d, args.heff_kop),
            layout, Lf, Rf, pf, triples, heff_slices(args), dd_ref=dd_ref)
        del Lf, Rf, pf
    if "sparse" in sections:
        log("[bench] generating block-sparse batch (40 sectors, 2000 triples)")
        prob = wl.heff_sparse()
        layout, Lf, Rf, pf, triples = wl.flatten_sparse(prob)
        extra["heff_sparse"] = heff_section(
            args, ozaki, ctx, torch, "block-sparse 40 sectors, %d triples" % len(triples),
            layout, Lf, Rf, pf, triples, heff_slices(args))
    if "davidson" in sections:
        extra["davidson"] = davidson_section(args, ozaki, ctx, torch)
    if "dispatch" in sections:
        extra["dispatch_by_size"] = dispatch_section(args, ozaki, ctx, torch)
    if "stability" in sections:
        extra["stability"] = stability_section(args, ozaki, ctx, torch)
    if "rdm" in sections:
        extra["rdm"] = rdm_section(args, ozaki, ctx, torch)
    if "sweep" in sections:
        extra["gemm_sweep"] = sweep_section(args, ozaki, ctx, torch, oracle)
    if "oracle" in sections and not args.no_cpu:
        extra["oracle_timings"] = oracle_section(args, oracle)
    if gemm is None:
        print(json.dumps({"sections": sorted(sections), "records": extra}), flush=True)
        return
    roofline = {"bound": "mfma", "achieved": chosen["int8_tops"], "peak": INT8_PEAK_TOPS,
                "unit": "TFLOP/s", "frac": chosen["int8_frac"],
                "traffic": pair_traffic(gemm["n"], chosen["slices"], chosen["ndiag"], chosen["variant"]),
                "kernel": "k_pair_single variant %d: pairs * 2n^3 int8 ops / mean kernel time "
                          "(HIP events on its stream)" % chosen["variant"],
                "algorithmic_bytes": pair_bytes(gemm["n"], chosen["slices"]),
                "kernel_ms": chosen["pair_kernel_ms"]}
    full = {
        "config": {"n": gemm["n"], "U": 10, "slices": chosen["slices"], "ndiag": chosen["ndiag"],
                   "variant": chosen["variant"], "rows_for_error": gemm["rows_for_error"]},
        "roofline": roofline,
        "fp64_mfma": gemm["fp64"],
        "vendor_fp64": gemm["vendor_fp64"],
        "emulated_per_slices": gemm["emulated"],
        "at_1e-12": gemm["at_1e-12"],
        "automatic_width": gemm["auto"],
        "cpu_baseline": cpu,
        "device": device_record(torch),
    }
    full.update(extra)
    if args.full_json:
        d = os.path.dirname(args.full_json)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.full_json, "w") as fh:
            json.dump(full, fh, indent=1)
        log("[bench] full record written to %s" % args.full_json)

    def heff_scalar(key):
        sec = extra.get(key)
        if not sec:
            return None
        s6 = [r for r in sec["emulated"] if r["slices"] == 6]
        if not s6:
            return None
        r = s6[0]
        return {"slices": 6, "applies_per_s": round(r["applies_per_s"], 3), "ms": round(r["ms"], 3),
                "tflops": round(r["tflops"], 2), "int8_frac_pair_phases": r["int8_frac_pair_phases"],
                "fp64_applies_per_s": round(sec["fp64"]["applies_per_s"], 3) if "fp64" in sec else None,
                "rel_err_vs_fp64": r["rel_frobenius_vs_fp64"]}

    dav = None
    if "davidson" in extra:
        runs = extra["davidson"]["runs"]
        r6 = [r for r in runs if r["slices"] == 6]
        r0 = [r for r in runs if r["slices"] == 0]
        if r6 and r0:
            dav = {"D": extra["davidson"]["D"], "slices": 6, "ms_per_iteration": round(r6[0]["ms_per_iteration"], 3),
                   "ms_per_iteration_after_capture": (round(r6[0]["ms_per_iteration_after_capture"], 3)
                                                      if r6[0]["ms_per_iteration_after_capture"] else None),
                   "iterations": r6[0]["iterations"], "energy_error_vs_fp64": r6[0]["energy_error_vs_fp64"],
                   "fp64_ms_per_iteration": round(r0[0]["ms_per_iteration"], 3)}
    line = {
        "metric": "Emulated-FP64 TFLOP/s vs native FP64 MFMA at equal error; H_eff.psi applies/s",
        "value": chosen["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64-emulated (int8 slices, int32 accumulation, fp64 recombination)",
        "data": "synthetic",
        "config": {"workload": "emulated DGEMM n=%d, entries N(0,1)*2^u, u in [-10,10], seed 0; S=%d G=%d, "
                               "the fastest width at equal error with FP64 MFMA (%d sampled rows vs "
                               "double-double)" % (gemm["n"], chosen["slices"], chosen["ndiag"],
                                                   gemm["rows_for_error"]),
                   "n": gemm["n"], "slices": chosen["slices"], "ndiag": chosen["ndiag"],
                   "variant": chosen["variant"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error": {"emulated_rel_frobenius": chosen["rel_frobenius"], "emulated_componentwise": chosen["componentwise"],
                  "fp64_rel_frobenius": gemm["fp64"]["rel_frobenius"],
                  "fp64_componentwise": gemm["fp64"]["componentwise"],
                  "vendor_rel_frobenius": gemm["vendor_fp64"]["rel_frobenius"]},
        "fp64_mfma_tflops": gemm["fp64"]["tflops"],
        "vendor_fp64_tflops": gemm["vendor_fp64"]["tflops"],
        "speedup_vs_fp64": gemm["fp64"]["ms"] / chosen["ms"],
        "speedup_vs_vendor_fp64": gemm["vendor_fp64"]["ms"] / chosen["ms"],
        "at_1e-12": None if gemm["at_1e-12"] is None else
        {"slices": gemm["at_1e-12"]["slices"], "ndiag": gemm["at_1e-12"]["ndiag"],
         "tflops": gemm["at_1e-12"]["tflops"], "rel_frobenius": gemm["at_1e-12"]["rel_frobenius"]},
        "heff_dense": heff_scalar("heff_dense"),
        "heff_sparse": heff_scalar("heff_sparse"),
        "davidson": dav,
        "full_record": args.full_json or None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
