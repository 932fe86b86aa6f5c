#!/usr/bin/env python3
"""Benchmark: ILS solves per second on one MI355X.

Workload: dense FP64 ILS with A1 18000 x 1000 and A2 2000 x 1000 (i.i.d.
Gaussian, A2 scaled to ||A2||_2 = 0.5 sigma_min(A1)), b = A x* + 1e-8 noise,
x0 = 0, solved by the SP method (Algorithm 1) in FP64 until
||x - x*|| / ||x*|| < 1e-6.  One "step" is one whole solve with A and b
already resident in HBM: column pass, both Gram products, block Gauss-Jordan
for B and c, and the outer iterations with their stop tests.

Printed as one JSON line.  Besides the headline FP64 SP number it reports
the other forms on the same problem, the dominant kernel (the MFMA Gram
A1^T A1) against the FP64 matrix peak, and the CPU oracle timed on this
host's cores on the same workload (all cores and one thread).
"""
import argparse
import gc
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P_ROWS, Q_ROWS, N_COLS = 18000, 2000, 1000
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector = matrix)
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gram_fp64_20000x1000_traffic.json")
GRAM_SAMPLE = 8  # timed solves per HIP-event sample of the Gram launch
TUNE_FILE = os.path.join(ROOT, "paper_2203_15340_amd", "tune", "gram_mi355x.json")
GRAM_SRC = os.path.join(ROOT, "paper_2203_15340_amd", "csrc", "k_gram.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash():
    with open(GRAM_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def tuned_entry(path, precision, n, K):
    """The entry of a saved Gram launch table for (precision, n, K)."""
    def bucket(x):
        b = 0
        while (1 << b) < x:
            b += 1
        return b
    with open(path) as f:
        for e in json.load(f)["entries"]:
            if (e["kernel"] == "gram" and e["precision"] == precision and e["n_bucket"] == bucket(n)
                    and e["k_bucket"] == bucket(K)):
                return {"kernel": "gram", "precision": precision, "n": n, "K": K, "tile": e["tile"],
                        "workgroups": e["workgroups"], "kind": e.get("kind", 0), "source": "file"}
    return None


def batched_launch_entry(form, precision, nmax, count):
    """The committed table's batched-solver entry for this batch, or the
    built-in default (stage rows 32, 2 workgroups per CU, largest first)."""
    def bucket(x):
        b = 0
        while (1 << b) < x:
            b += 1
        return b
    try:
        with open(TUNE_FILE) as f:
            for e in json.load(f)["entries"]:
                if (e["kernel"] == "batched" and e["precision"] == precision and e["form"] == form
                        and e["n_bucket"] == bucket(nmax) and e["k_bucket"] == bucket(count)):
                    return {"stage_rows": e["tile"], "workgroups_per_cu": e["workgroups"],
                            "order": "as given" if e["kind"] == 1 else "largest first", "source": "file"}
    except (OSError, ValueError, KeyError):
        pass
    return {"stage_rows": 32, "workgroups_per_cu": 2, "order": "largest first", "source": "default"}


def gram_kernel_name(tuned):
    what = "A1^T A1, A2^T A2 and border columns b1, b2 in one launch, FP64 MFMA"
    if tuned is not None and tuned.get("kind", 0) == 1:
        return f"k_gram_pers ({what}; resident grid, operands loaded straight into LDS)"
    return f"k_gram<double, 64> ({what}; split-K grid)"


def measured_traffic(tuned):
    """HBM bytes per Gram launch from the committed rocprofv3 counter runs,
    or None when the kernel source or its launch configuration changed since
    they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    cfg = t.get("config")
    if tuned is not None and (cfg is None or cfg.get("tile") != tuned["tile"]
                              or cfg.get("workgroups") != tuned["workgroups"]
                              or cfg.get("kind", 0) != tuned.get("kind", 0)):
        return None
    return t.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, reps=3, one_thread_budget_s=12.0):
    """The oracle's FP64 SP on the host cores, same problem and stop rule as
    the GPU line: both of its variants (explicit iteration matrix of the
    update (Sec23), and triangular solves with the Cholesky factor) on all
    cores, median of `reps` runs each; then the faster variant on one thread
    (median of `reps` runs, or a single run when one takes longer than
    `one_thread_budget_s`, which keeps the whole baseline near 30 s)."""
    import numpy as np

    import oracle as O
    allc = len(os.sched_getaffinity(0))

    def timed(variant, threads, count):
        O.set_threads(threads)
        ts = []
        for _ in range(count):
            t0 = time.perf_counter()
            _, info = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-6,
                                 variant=variant)
            ts.append(time.perf_counter() - t0)
            assert info.status == O.OK, info
            if threads == 1 and ts[0] > one_thread_budget_s:
                break
        med = float(np.median(ts))
        return {"threads": threads, "runs": len(ts), "median_s": med, "solves_per_s": 1.0 / med,
                "times_s": [round(t, 4) for t in ts], "outer": int(info.outer_iters)}

    runs = {"explicit_all_cores": timed(O.SP_EXPLICIT, allc, reps),
            "cholesky_all_cores": timed(O.SP_CHOLESKY, allc, reps)}
    fast = min(("explicit", "cholesky"), key=lambda v: runs[v + "_all_cores"]["median_s"])
    runs[fast + "_1_thread"] = timed(O.SP_EXPLICIT if fast == "explicit" else O.SP_CHOLESKY, 1, reps)
    O.set_threads(allc)
    best = runs[fast + "_all_cores"]
    return {"value": best["solves_per_s"], "unit": "solves/s", "cores": allc, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"FP64 SP solves of the same {P.p}+{P.q} x {P.n} problem to rel.err 1e-6 "
                      f"({best['outer']} outer iterations); value = the faster oracle variant "
                      f"({fast}) on {allc} threads, median of {best['runs']} runs; every run in 'runs'",
            "runs": runs}


def time_rk_multi(ils, W, np, torch, P, A, x, nrhs=16):
    """SP-RK-RGS (correction form) for nrhs right-hand sides sharing the
    headline A and one index stream: the headline b and nrhs - 1 more with
    planted solutions (same noise level), to rel.err 1e-6 per column."""
    rng = np.random.default_rng(77)
    Xs = np.empty((P.n, nrhs))
    Xs[:, 0] = P.x_star
    Xs[:, 1:] = rng.standard_normal((P.n, nrhs - 1))
    B = P.A @ Xs
    B[:, 0] = P.b
    B[:, 1:] += 1e-8 * rng.standard_normal((P.A.shape[0], nrhs - 1))
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda().t()
    xr = torch.from_numpy(np.ascontiguousarray(Xs.T)).cuda().t()
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-6, form=ils.FORM_CORRECTION)
    torch.cuda.synchronize()
    t = time.perf_counter()
    X, inf, iters = ils.rk_solve_multi(A, Bd, P.p, x_ref=xr, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    log(f"multi-RHS SP-RK-RGS: {nrhs} right-hand sides in {el * 1e3:.1f} ms")
    return {"solves_per_s": nrhs / el, "ms_per_call": el * 1e3, "nrhs": nrhs, "max_outer": int(max(iters)),
            "inner": inf.inner_iters, "max_rel_err": inf.rel_err, "status": inf.status}


def bench_ratio09(ils, W, np, torch):
    """The headline problem with A2 scaled to ||A2|| = 0.9 sigma_min(A1) (the
    same A1 and x*, slower outer convergence): the SP forms, FP64 and mixed."""
    log("ratio 0.9 variant")
    P = W.large(ratio=0.9, seed=1)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b = torch.from_numpy(P.b).cuda()
    xs = torch.from_numpy(P.x_star).cuda()
    x = torch.empty(P.n, dtype=torch.float64, device="cuda")
    kw = dict(stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6)
    out = {"workload": "dense ILS, A1 18000x1000 + A2 2000x1000 Gaussian, ||A2|| = 0.9 sigma_min(A1), "
                       "b = A x* + 1e-8 noise, to ||x-x*||/||x*|| < 1e-6"}
    for name, reps, extra in (("sp_fp64_paper", 20, {}),
                              ("sp_fp64_correction", 5, dict(form=ils.FORM_CORRECTION)),
                              ("sp_mixed_correction", 5, dict(form=ils.FORM_CORRECTION, precision=ils.PREC_MIXED))):
        ils.sp_solve(A, b, P.p, out=x, **kw, **extra)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, inf = ils.sp_solve(A, b, P.p, out=x, **kw, **extra)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / reps
        out[name] = {"solves_per_s": 1.0 / el, "ms": el * 1e3, "outer": inf.outer_iters,
                     "rel_err": inf.rel_err, "status": inf.status}
    log(f"ratio 0.9: {out}")
    return out


def bench_batched(ils, W, np, torch, count=4096, single_sample=256):
    """4096 independent problems, n ~ U{32..256}, p = 4n, q = n/2, solved to
    rel.err 1e-6 in one persistent launch (graph replay) vs one ils_sp_solve
    call per problem (FP64 SP) on the first `single_sample` problems."""
    log(f"batched workload: {count} problems")
    B = W.batched(count, seed=3, threads=len(os.sched_getaffinity(0)))
    dv = [(torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t(), torch.from_numpy(P.b).cuda(), P.p)
          for P in B]
    xr = [torch.from_numpy(P.x_star).cuda() for P in B]
    plan = ils.BatchPlan(dv, x_refs=xr)
    out = {"problems": count, "n_range": [min(P.n for P in B), max(P.n for P in B)],
           "total_flop_gram_a1": int(sum(P.p * P.n * (P.n + 1) for P in B))}
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-6)
    for name, extra, reps in (("fp64_paper", dict(form=ils.FORM_PAPER), 5),
                              ("mixed_correction", dict(form=ils.FORM_CORRECTION,
                                                        precision=ils.PREC_MIXED), 3)):
        rc = plan.solve(**kw, **extra)  # captures the launch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rc = plan.solve(**kw, **extra)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        res = plan.results()
        out[name] = {"solves_per_s": count / el, "ms_per_batch": el * 1e3, "status": rc,
                     "max_rel_err": max(r.rel_err for r in res),
                     "max_outer": max(r.outer_iters for r in res),
                     "device_ms": res[0].device_ms,
                     "launch": batched_launch_entry(extra.get("form", ils.FORM_PAPER),
                                                    extra.get("precision", ils.PREC_FP64),
                                                    max(P.n for P in B), count)}
        log(f"batched {name}: {count / el:.0f} solves/s ({el * 1e3:.2f} ms per batch)")
    xs = torch.empty(max(P.n for P in B), dtype=torch.float64, device="cuda")
    ils.sp_solve(*dv[0][:2], dv[0][2], out=xs[:B[0].n], x_ref=xr[0], **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for i in range(single_sample):
        _, inf = ils.sp_solve(dv[i][0], dv[i][1], dv[i][2], out=xs[:B[i].n], x_ref=xr[i], **kw)
        worst = max(worst, inf.rel_err)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / single_sample
    out["fp64_sp_one_call_each"] = {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3,
                                    "sample": f"first {single_sample} of the {count} problems",
                                    "max_rel_err": worst}
    log(f"one ils_sp_solve per problem: {1.0 / el:.0f} solves/s")
    return out


def bench_warm_start(ils, W, np, torch, n_train=50000, n_test=2000, single_sample=20):
    """Learned warm start on a family sharing A (18000 + 2000 x 1000, ratio
    0.5): x = U theta + 1e-3 eps with U a random 1000 x 32 orthonormal basis,
    b = A x.  Training pairs (b, x_SP) come from the multi-right-hand-side SP
    solve at RR < 1e-20 (relative residual 1e-10); the network sees every
    10th row of b and trains in 8 stages of 10 epochs with the step size
    halved each stage.  Test: n_test fresh right-hand sides solved to rel.err
    1e-6 on the prepared A (Gram products and elimination done once), from
    the zero start and from the network's x0 (inference timed)."""
    log("warm start: generating the family")
    P, U = W.ws_problem(seed=4)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    rows = W.ws_in_rows(P.m)

    def rhs(X):
        # b = A x for every column (input construction on the device)
        Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t()
        Bd = torch.empty((X.shape[1], P.m), dtype=torch.float64, device="cuda").t()
        torch.matmul(A, Xd, out=Bd)
        return Xd, Bd

    Xtr, Btr = rhs(W.ws_solutions(U, n_train, seed=(4, 2)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xsp, inf, _ = ils.sp_solve_multi(A, Btr, P.p, stop_rule=ils.STOP_RR, tol=1e-20, max_outer=200)
    torch.cuda.synchronize()
    t_sp = time.perf_counter() - t0
    assert inf.status == ils.OK, inf
    sp_err = float(((Xsp - Xtr).norm(dim=0) / Xtr.norm(dim=0)).max())
    log(f"training targets: {n_train} SP solves in {t_sp:.2f} s, max outer {inf.outer_iters}, "
        f"max rel.err vs planted {sp_err:.1e}")
    del Xtr
    hidden = 1024
    schedule = [(10, 1e-3 * 0.5 ** i) for i in range(8)]
    ws = ils.WarmStart(P.m, P.n, rows, hidden=hidden, seed=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep, lr in schedule:
        loss = ws.train(Btr, Xsp, epochs=ep, batch=256, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    epochs = sum(e for e, _ in schedule)
    log(f"training: {epochs} epochs in {t_train:.2f} s, final loss {loss:.3e}")
    del Btr, Xsp
    torch.cuda.empty_cache()

    Xte, Bte = rhs(W.ws_solutions(U, n_test, seed=(4, 3)))
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-6, x_ref=Xte)
    out = {"family": "A 18000+2000 x 1000 ratio 0.5 (seed 4); x = U theta + 1e-3 eps, U 1000 x 32",
           "train_pairs": n_train, "test_rhs": n_test, "hidden": hidden, "epochs": epochs,
           "schedule": "8 stages of 10 epochs, step 1e-3 halved per stage, batch 256",
           "final_loss": loss, "train_s": t_train,
           "train_targets": {"sp_solves_per_s": n_train / t_sp, "max_outer": inf.outer_iters,
                             "rr_tol": 1e-20, "max_rel_err_vs_planted": sp_err}}
    X0 = ws.infer(Bte)
    e0 = ((X0 - Xte).norm(dim=0) / Xte.norm(dim=0)).cpu().numpy()
    out["warm_start_initial_rel_err"] = {"median": float(np.median(e0)), "max": float(e0.max())}

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prep = ils.SPPrepared(A, P.p)
    torch.cuda.synchronize()
    out["prepare_ms"] = (time.perf_counter() - t0) * 1e3
    reps = 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, r

    # per-batch work without outer steps: A^T J B, c = P A^T J B, copies
    el0, _ = timed(lambda: prep.solve_multi(Bte, stop_rule=ils.STOP_FIXED, max_outer=0))
    out["per_batch_setup_ms"] = el0 * 1e3
    el_inf, _ = timed(lambda: ws.infer(Bte))
    out["inference_ms_per_batch"] = el_inf * 1e3
    for name in ("zero_start", "warm_start"):
        def run(warm=(name == "warm_start")):
            x0 = ws.infer(Bte) if warm else None
            return prep.solve_multi(Bte, X0=x0, **kw)
        el, (X, inf2, it) = timed(run)
        steps_ms = el * 1e3 - el0 * 1e3 - (el_inf * 1e3 if name == "warm_start" else 0.0)
        out[name] = {"solves_per_s": n_test / el, "ms_per_batch": el * 1e3, "status": inf2.status,
                     "mean_outer": float(it.mean()), "max_outer": int(it.max()),
                     "outer_steps_ms": steps_ms, "max_rel_err": inf2.rel_err}
        log(f"{name} (prepared A): {n_test / el:.0f} solves/s, mean outer {it.mean():.2f}, "
            f"max {int(it.max())}, outer steps {steps_ms:.2f} ms")
    z, w = out["zero_start"], out["warm_start"]
    out["ratios"] = {"max_outer_warm_over_zero": w["max_outer"] / max(z["max_outer"], 1),
                     "outer_steps_ms_warm_over_zero": w["outer_steps_ms"] / max(z["outer_steps_ms"], 1e-9),
                     "solves_per_s_warm_over_zero": w["solves_per_s"] / z["solves_per_s"]}
    prep.close()
    # the unprepared multi-right-hand-side solve (Grams and elimination per call), for context
    el, (X, inf3, it) = timed(lambda: ils.sp_solve_multi(A, Bte, P.p, **kw))
    out["unprepared_zero_start"] = {"solves_per_s": n_test / el, "ms_per_batch": el * 1e3,
                                    "mean_outer": float(it.mean())}
    x = torch.empty(P.n, dtype=torch.float64, device="cuda")
    ils.sp_solve(A, Bte[:, 0], P.p, out=x, stop_rule=ils.STOP_XREF, tol=1e-6, x_ref=Xte[:, 0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(single_sample):
        ils.sp_solve(A, Bte[:, j], P.p, out=x, stop_rule=ils.STOP_XREF, tol=1e-6,
                     x_ref=Xte[:, j].contiguous())
    torch.cuda.synchronize()
    out["fp64_sp_one_call_each"] = {"solves_per_s": single_sample / (time.perf_counter() - t0),
                                    "sample": f"first {single_sample} test right-hand sides"}
    ws.close()
    return out


def bench_sparse(ils, W, np, torch, reps=3, rk_steps=20000):
    """Sparse ILS: p = 180000, q = 20000, n = 4000, i.i.d. Bernoulli(0.005)
    pattern with N(0,1) values, A1[i, i] += 1, A2 scaled to ratio 0.7;
    b = A x*.  SP and SP-SCD to rel.err 1e-6; SP-RK-RGS timed per inner step
    on a fixed schedule (a full solve needs ~47 n inner steps per outer step)."""
    log("sparse workload: generating")
    P = W.sparse_large(seed=2)
    t0 = time.perf_counter()
    S = ils.SparseA.from_scipy(P.A, P.p)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    b = torch.from_numpy(P.b).cuda()
    xs = torch.from_numpy(P.x_star).cuda()
    kw = dict(stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6)
    out = {"workload": "sparse A 180000+20000 x 4000, density 0.005, ratio 0.7", "nnz": int(P.A.nnz),
           "csr_upload_and_csc_build_s": t_build}
    ils.set_profiling(True)
    S.sp_solve(b, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phases = []
    for _ in range(reps):
        _, inf = S.sp_solve(b, **kw)
        phases.append(ils.phase_times())
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    ph = {k: statistics.mean(q[k] for q in phases) for k in ils.PHASES}
    out["sp_fp64_paper"] = {"solves_per_s": 1.0 / el, "ms": el * 1e3, "outer": inf.outer_iters,
                            "rel_err": inf.rel_err, "status": inf.status, "phases_ms": ph}
    log(f"sparse SP: {1.0 / el:.2f} solves/s, outer {inf.outer_iters}, phases {ph}")
    for name, extra in (("sp_fp64_correction", dict(form=ils.FORM_CORRECTION)),):
        t0 = time.perf_counter()
        _, inf = S.sp_solve(b, **kw, **extra)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"solves_per_s": 1.0 / el, "outer": inf.outer_iters, "rel_err": inf.rel_err,
                     "status": inf.status}
    t0 = time.perf_counter()
    _, inf = S.rgs_solve(b, form=ils.FORM_CORRECTION, seed=1, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["sp_scd_correction"] = {"solves_per_s": 1.0 / el, "outer": inf.outer_iters,
                                "inner": inf.inner_iters, "rel_err": inf.rel_err, "status": inf.status}
    log(f"sparse SP-SCD: {1.0 / el:.3f} solves/s, outer {inf.outer_iters}, inner {inf.inner_iters}")
    S.rk_solve(b, stop_rule=ils.STOP_FIXED, max_outer=1, max_inner=1000, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, inf = S.rk_solve(b, stop_rule=ils.STOP_FIXED, max_outer=1, max_inner=rk_steps, seed=1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["sp_rk_rgs_inner_step_us"] = el / rk_steps * 1e6
    log(f"sparse SP-RK-RGS: {el / rk_steps * 1e6:.2f} us per inner step")
    # residual sweep A^T J (b - A x): CSR + CSC bytes against HBM
    x = torch.zeros(P.n, dtype=torch.float64, device="cuda")
    S.residual(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        S.residual(b, x)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 20
    nbytes = 2 * 12 * P.A.nnz + 8 * (P.m + 1) + 8 * (P.n + 1) + 8 * 3 * P.m + 8 * 2 * P.n
    out["residual"] = {"ms": el * 1e3, "algorithmic_bytes": nbytes, "GB_per_s": nbytes / el / 1e9,
                       "note": "host-timed call incl. launch and sync"}
    S.close()
    return out


# The paper's Tables 2-5 (Sec. 5): MATLAB CPU seconds on an i7-9700, quoted as context only.
PAPER_TABLES = [
    ("q=n", 30000, 13000, 13000, {"sp": 559.3, "sp_rk_rgs": 514.6313, "sp_scd": 227.7141}),
    ("q=n", 30000, 14000, 14000, {"sp": 619.1, "sp_rk_rgs": 592.2625, "sp_scd": 286.9359}),
    ("q=n", 30000, 15000, 15000, {"sp": 830.2, "sp_rk_rgs": 803.0406, "sp_scd": 324.5609}),
    ("q=1", 50000, 1, 13000, {"sp": 566.9453}),
    ("q=1", 50000, 1, 14000, {"sp": 731.0016}),
    ("q=1", 50000, 1, 15000, {"sp": 881.0750}),
]


def bench_paper_tables(ils, W, np, torch):
    """The paper's own family at the paper's sizes: A1 = U[0,1) p x n, A2 =
    7 eye(q, n), b = U[0,1), x0 = 0, RR < 1e-6 (Sec. 5).  SP (Algorithm 1)
    and SP-RK-RGS (Algorithm 2, paper form) on the GPU; the paper's CPU
    times are context, not a target (different machine and precision of
    measurement)."""
    out = []
    for tag, p, q, n, paper_cpu in PAPER_TABLES:
        log(f"paper family {tag}: {p + q} x {n}")
        P = W.paper_family(p, q, n, seed=0)
        A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
        del P.A
        b = torch.from_numpy(P.b).cuda()
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        row = {"family": tag, "m": p + q, "n": n, "paper_cpu_s": paper_cpu}
        for name, fn, kw in (("sp", ils.sp_solve, {}),
                             ("sp_rk_rgs", ils.rk_solve, {"seed": 1, "max_inner": 200000, "max_outer": 3})):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = fn(A, b, p, out=x, stop_rule=ils.STOP_RR, tol=1e-6, **kw)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            row[name] = {"s": el, "it": inf.outer_iters, "it_inner": inf.inner_iters, "rr": inf.rr,
                         "status": inf.status}
            log(f"  {name}: {el:.3f} s, IT {inf.outer_iters}, inner {inf.inner_iters}, RR {inf.rr:.2e}")
        out.append(row)
        del A, b
        torch.cuda.empty_cache()
    return out


def probe_peaks(torch):
    """What this box achieves with vendor kernels, next to the published
    peaks: a 1 GiB device-to-device copy (HBM read + write) and an FP64
    8192^3 matrix product (the platform BLAS).  Context for the roofline
    fractions; the solver does not use either."""
    out = {}
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["hbm_copy_GB_per_s"] = 2 * src.numel() * 8 / (ms * 1e-3) / 1e9
    del src, dst
    a = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
    b = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
    c = a @ b
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        c = a @ b
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 3
    out["fp64_gemm_TFLOP_per_s"] = 2 * 8192 ** 3 / (ms * 1e-3) / 1e12
    out["note"] = "torch copy_ and FP64 matmul (platform BLAS) on the same GPU"
    del a, b, c
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the non-headline forms")
    ap.add_argument("--forms", default="",
                    help="comma-separated subset of the non-headline forms to time (default: all)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 4096-problem batch")
    ap.add_argument("--no-warm-start", action="store_true", help="skip the learned warm start")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparse workload")
    ap.add_argument("--no-tune", action="store_true", help="keep the default Gram configuration")
    ap.add_argument("--tune", choices=("file", "live", "none"), default="file",
                    help="Gram launch table: the committed MI355X table (file), a fresh sweep "
                         "(live) or the built-in defaults (none)")
    ap.add_argument("--paper-tables", action="store_true",
                    help="also run the paper's own family at the paper's sizes (several GB, minutes)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and FP64 GEMM peak probes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this solver runs each problem on a single "
              "MI355X (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2203_15340_amd as ils
    # no cyclic garbage collection while timing (as timeit does): a full
    # pass over the interpreter's heap with torch loaded takes tens of ms
    gc.collect()
    gc.disable()
    import workloads as W

    log("generating workload")
    P = W.large(ratio=0.5, seed=1)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b = torch.from_numpy(P.b).cuda()
    xs = torch.from_numpy(P.x_star).cuda()
    x = torch.empty(P.n, dtype=torch.float64, device="cuda")
    kw = dict(stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6)

    if args.calibrate_copy:
        src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 256 MiB read + 256 MiB written")
        del src, dst
    tuned = None
    mode = "none" if args.no_tune else args.tune
    if mode == "live":
        tuned = ils.tune_gram(A, 0, P.p, precision=ils.PREC_FP64, reps=5)
        ils.tune_gram(A, 0, P.p, precision=ils.PREC_MIXED, reps=5)
        ils.tune_gram(A, P.p, P.m, precision=ils.PREC_FP64, reps=5)  # A2^T A2
        tuned["source"] = "live"
        log(f"autotuned A1 Gram: {tuned}")
    elif mode == "file":
        ils.tune_load(TUNE_FILE)
        tuned = tuned_entry(TUNE_FILE, ils.PREC_FP64, P.n, P.p)
        log(f"Gram launch table {TUNE_FILE}: A1 {tuned}")
    # every GRAM_SAMPLE-th timed solve carries the two HIP events around the
    # Gram launch (each event costs device time and its read-back host time);
    # the full phase breakdown comes from extra solves after the timed region
    ils.set_profiling(ils.PROFILE_OFF)
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        _, info = ils.sp_solve(A, b, P.p, out=x, **kw)
        assert info.status == ils.OK, info
    torch.cuda.synchronize()
    log(f"timing {args.steps} solves")
    gram_ms, infos = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        sample = i % GRAM_SAMPLE == 0
        if sample:
            ils.set_profiling(ils.PROFILE_GRAM)
        _, info = ils.sp_solve(A, b, P.p, out=x, **kw)
        infos.append(info)
        if sample:
            gram_ms.append(ils.phase_times()["gram"])
            ils.set_profiling(ils.PROFILE_OFF)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(i.status == ils.OK for i in infos)
    ms = dt / args.steps * 1e3
    value = args.steps / dt
    ils.set_profiling(ils.PROFILE_PHASES)
    phases = []
    for _ in range(max(3, min(args.steps, 10))):
        ils.sp_solve(A, b, P.p, out=x, **kw)
        phases.append(ils.phase_times())
    ils.set_profiling(ils.PROFILE_OFF)
    ph = {k: statistics.mean(p[k] for p in phases) for k in ils.PHASES}
    # one launch: lower triangles of A1^T A1 and A2^T A2 plus A1^T b1 and
    # A2^T b2 (the border columns), 2 flops per multiply-add
    gram_flops = P.m * P.n * (P.n + 3)
    gram_avg = statistics.mean(gram_ms)
    achieved = gram_flops / (gram_avg * 1e-3) / 1e12
    traffic = measured_traffic(tuned)
    log(f"SP FP64: {value:.1f} solves/s, {ms:.3f} ms, phases {ph}")

    forms = {}
    if not args.no_forms:
        def time_form(fn, reps, **k):
            fn(A, b, P.p, out=x, **k)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                _, inf = fn(A, b, P.p, out=x, **k)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t) / reps
            return {"solves_per_s": 1.0 / el, "ms": el * 1e3, "outer": inf.outer_iters,
                    "inner": inf.inner_iters, "rel_err": inf.rel_err, "status": inf.status}
        log("other forms")
        forms["sp_fp64_paper"] = {"solves_per_s": value, "ms": ms, "outer": infos[-1].outer_iters,
                                  "rel_err": infos[-1].rel_err}
        table = {
            "sp_fp64_correction": (ils.sp_solve, 5, dict(form=ils.FORM_CORRECTION)),
            "sp_mixed_correction": (ils.sp_solve, 5, dict(form=ils.FORM_CORRECTION, precision=ils.PREC_MIXED)),
            "sp_scd_correction": (ils.rgs_solve, 1, dict(form=ils.FORM_CORRECTION)),
            "sp_rk_rgs_correction": (ils.rk_solve, 1, dict(form=ils.FORM_CORRECTION)),
            "sp_rk_rgs_mixed_correction": (ils.rk_solve, 1, dict(form=ils.FORM_CORRECTION,
                                                                 precision=ils.PREC_MIXED)),
        }
        multi = "sp_rk_rgs_multi16_correction"
        pick = [f for f in args.forms.split(",") if f] or list(table) + [multi]
        for name in pick:
            if name == multi:
                forms[name] = time_rk_multi(ils, W, np, torch, P, A, x, nrhs=16)
                continue
            fn, reps, extra = table[name]
            forms[name] = time_form(fn, reps, **extra, **kw)
        ils.set_profiling(True)

    ratio09 = None if args.no_forms else bench_ratio09(ils, W, np, torch)

    batched = None
    if not args.no_batched:
        batched = bench_batched(ils, W, np, torch)
    warm = None
    if not args.no_warm_start:
        warm = bench_warm_start(ils, W, np, torch)
    sparse = None
    if not args.no_sparse:
        sparse = bench_sparse(ils, W, np, torch)
    paper_tables = bench_paper_tables(ils, W, np, torch) if args.paper_tables else None
    peaks = None
    if not args.no_peaks:
        log("peak probes")
        peaks = probe_peaks(torch)
        peaks["gram_frac_of_fp64_gemm"] = achieved / peaks["fp64_gemm_TFLOP_per_s"]
        log(f"peaks: {peaks}")

    line = {
        "metric": "ILS solves/s to rel.err 1e-6, plain FP64 SP vs chosen form; % HBM/MFMA peak",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense ILS, A1 18000x1000 + A2 2000x1000 Gaussian, "
                               "||A2|| = 0.5 sigma_min(A1), b = A x* + 1e-8 noise, FP64 SP to "
                               "||x-x*||/||x*|| < 1e-6",
                   "p": P.p, "q": P.q, "n": P.n, "ratio": 0.5,
                   "outer_iters": infos[-1].outer_iters, "rel_err": infos[-1].rel_err},
        "autotune": tuned,
        "roofline": {"bound": "mfma",
                     "kernel": gram_kernel_name(tuned),
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_launch": gram_flops, "avg_launch_ms": gram_avg,
                     "launch_samples": len(gram_ms)},
        "phases_ms": ph,
        "forms": forms,
        "ratio_0_9": ratio09,
        "batched": batched,
        "warm_start": warm,
        "sparse": sparse,
        "paper_tables": paper_tables,
        "peaks_measured": peaks,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(P)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
