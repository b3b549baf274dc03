#!/usr/bin/env python3
"""Benchmark of the BM-Global matrix-completion hot path on one MI355X.

Headline workload: the Yahoo! Music-shaped synthetic problem (624,961 x
1,000,990, |Omega| = 2.5e8, power-law (1.1) row and column degrees, rank-30
truth + noise variance 0.5, lambda = 50, k0 = 32), FP64: the largest of the
benchmark configurations.  One step = one call of bmg_solve limited to one
outer iteration: HMT + Nystrom initialisation, 3 BM epochs, one inexact PG
step (subspace iteration + exact SVD + soft-threshold) and the objective,
every sparse pass in the library's HIP kernels.  Every step starts from the
same state, so every step does identical work.  --workload netflix runs the
Netflix-shaped problem (17,770 x 480,189, |Omega| = 1e8, lambda = 20, k0 = 16)
instead; with extras on, its step runs beside the headline anyway.

value = algorithmic bytes of all sparse passes of the timed steps / wall time.
roofline = the kernel class with the largest time, its algorithmic bytes per
launch / its launch time, both from HIP events on the problem's stream.
cpu_baseline = the CPU oracle's residual + product pair on the same data.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload yahoo|netflix]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# the benchmark workloads (synth generators): the Yahoo! Music-shaped one is the
# largest of the configurations and carries the headline line
WORKLOADS = {
    "yahoo": dict(gen="yahoo_shape", name="yahoo_shape", k0=32, lam=50.0, k_cap=80,
                  desc="power-law (1.1) degrees, rank-30 truth + noise var 0.5"),
    "netflix": dict(gen="netflix_shape", name="netflix_shape", k0=16, lam=20.0, k_cap=64,
                    desc="capped Zipf(1.2) degrees, rank-20 truth + noise var 0.25 clipped to [1, 5]"),
}
KERNEL_NAMES = ["k_grad (fused sampled residual + sparse product)",
                "k_sddmm (sampled residual / curvature)",
                "k_spmm (sparse x dense of the subspace iteration)"]
KERNEL_SYMBOLS = ["k_grad", "k_sddmm", "k_spmm"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_for(kernel_symbol, workload, precision="fp64"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    suffix = "" if precision == "fp64" else "_" + precision
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s%s.json" % (kernel_symbol, workload, suffix))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    from paper_2204_14067_amd.build import kernel_sources_sha256
    if rec.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(p, k):
    """Oracle R = P_Omega(W H^T - A) then G = R H over the whole workload at the
    workload's k0, FP64, on the host cores; bytes counted with the same formula
    as the GPU pass."""
    import numpy as np
    from oracle import core
    rng = np.random.default_rng(0)
    W = 0.3 * rng.standard_normal((p.m, k))
    H = 0.3 * rng.standard_normal((p.n, k))
    reps, t_tot = 0, 0.0
    while reps < 2 or (t_tot < 10.0 and reps < 200):
        t0 = time.perf_counter()
        R = core.sddmm(p, W, H)
        G = core.spmm(p, R, H)
        t_tot += time.perf_counter() - t0
        reps += 1
        del R, G
    nbytes = p.nnz * (4 + 8) + (p.m + p.n) * k * 8 + p.m * k * 8 + 8 * (p.m + 1)
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    return {"value": round(nbytes * reps / t_tot / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": "%d x (residual pass + row-oriented sparse product) over the full workload "
                      "%s, k=%d, FP64, %.1f s" % (reps, p.name, k, t_tot)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--bm-solver", default=None, choices=["psd", "polymf"],
                    help="BM solver (psd: preconditioned gradient steps; polymf: polyMF-SS).  Default: psd for "
                         "the benchmark step (whole-Omega passes, the dense-row panel), the library default "
                         "(polymf) for --small-solve-only")
    ap.add_argument("--workload", default="yahoo", choices=sorted(WORKLOADS),
                    help="yahoo: 624,961 x 1,000,990, |Omega| = 2.5e8 (the headline); netflix: 17,770 x "
                         "480,189, |Omega| = 1e8")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (tests only)")
    ap.add_argument("--dense-rows", type=float, default=0.25,
                    help="rows of Omega at least this dense go to the dense panel (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB (3 times), to scale HBM counters")
    ap.add_argument("--qsdp-only", action="store_true",
                    help="only run one kernel-estimation QSDP solve (20,000 objects, tol 1e-4)")
    ap.add_argument("--verbose", action="store_true", help="per-iteration log of the solver (stderr)")
    ap.add_argument("--qsdp-tol", type=float, default=1e-4, help="stop residual of --qsdp-only")
    ap.add_argument("--small-solve-only", action="store_true",
                    help="only run one FP64 solve of the 1000 x 1500 workload to tol 1e-6 (seed 11)")
    ap.add_argument("--only", default=None,
                    choices=["bf16_mode", "serve", "serve_literal", "time_to_tol", "time_to_tol_gpu_bound",
                             "rke_qsdp", "paper_tables"],
                    help="run one extra measurement alone and print its JSON")
    ap.add_argument("--serve-count", type=int, default=256,
                    help="requests replayed by the serving measurement (256 in the full stream)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (--gpus %d requested): the path is not sharded over "
              "several GPUs." % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2204_14067_amd as bmg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    if args.qsdp_only:
        q = synth.rke(20_000, 40, lam=10.0, seed=7)
        dq = bmg.Problem.from_host(q.row_ptr, q.col, q.val, q.m, q.n, k_cap=RKE_K_CAP, device=dev,
                                   lmsvd_p=RKE_LMSVD_P)
        t0 = time.perf_counter()
        _, k, r = dq.bmg_rke_solve(lam=10.0, k_init=8, tol=args.qsdp_tol, seed=1, max_iter=3000,
                                   bm_epochs=10, lmsvd_p=RKE_LMSVD_P, verbose=args.verbose)
        print(json.dumps({"qsdp_objects": q.n, "pairs": q.nnz // 2, "seconds": time.perf_counter() - t0,
                          "iters": r["iters"], "ssi_iters": r["ssi_iters"],
                          "ssi_per_pg_step": r["ssi_iters"] / (r["iters"] + 1), "rank": k, "F": r["F"],
                          "status": r["status"]}))
        return
    if args.small_solve_only:
        p = synth.small_uniform()
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=256, precision="fp64",
                                     device=dev)
        t0 = time.perf_counter()
        bs = args.bm_solver or "polymf"
        _, _, k, r = prob.bmg_solve(lam=p.lam, k_init=p.k0, tol=1e-6, seed=11, max_iter=1000, bm_solver=bs)
        print(json.dumps({"workload": "small_uniform 1000x1500 nnz=50000 lambda=0.5", "bm_solver": bs,
                          "seconds": time.perf_counter() - t0, "iters": r["iters"], "rank": k,
                          "F": r["F"], "status": r["status"], "ssi_iters": r["ssi_iters"],
                          "host_la_seconds": r["host_la_seconds"],
                          "host_wait_seconds": r["host_wait_seconds"], "host_syncs": r["host_syncs"],
                          "sparse_passes": r["sparse_passes"]}))
        return
    if args.only:
        fn = {"bf16_mode": lambda: bf16_mode(bmg, synth, dev), "serve": lambda: serving(bmg, synth, dev, args.serve_count),
              "time_to_tol": lambda: time_to_tol(bmg, synth, dev),
              "time_to_tol_gpu_bound": lambda: time_to_tol_gpu_bound(bmg, synth, dev),
              "rke_qsdp": lambda: rke_qsdp(bmg, synth, dev),
              "serve_literal": lambda: serving_literal(bmg, synth, dev),
              "paper_tables": lambda: paper_tables(bmg, synth, dev)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8,
                          "copies": 3}))
        return
    t0 = time.time()
    p = getattr(synth, WORKLOADS[args.workload]["gen"])(scale=args.scale)
    log("workload %s generated in %.1fs" % (p.name, time.time() - t0))
    wl = WORKLOADS[args.workload]
    # the workspace also holds two LmSVD history blocks (the history comparison)
    line, prob, W, H, recs, sec = step_line(bmg, p, args.workload, args.scale, args.precision, args.steps,
                                            args.warmup, args.bm_solver or "psd", dev,
                                            hist=0 if args.no_extras or args.workload != "netflix" else 2,
                                            dense_rows=args.dense_rows)
    out = {
        "metric": "SDDMM+SpMM GB/s (% HBM peak); time-to-tol vs plain; serve p50/p99 latency",
        "value": line["value"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": line["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": line["dtype"], "data": "synthetic",
        "config": line["config"], "roofline": line["roofline"], "kernels": line["kernels"],
    }
    if not args.no_extras:
        if args.workload == "yahoo":
            # the same step in FP32 on this workload, and the Netflix-shaped
            # workload's step (FP64 and the lower precisions, and the variants)
            out["yahoo_shape_fp32"] = step_line(bmg, p, "yahoo", args.scale, "fp32", 3, 1, "psd", dev,
                                                dense_rows=args.dense_rows)[0]
            del prob, W, H
            import torch
            torch.cuda.empty_cache()
            q = synth.netflix_shape(scale=args.scale)
            nline, prob, W, H, recs, sec = step_line(bmg, q, "netflix", args.scale, "fp64", 5, 1, "psd", dev,
                                                      hist=2, dense_rows=args.dense_rows)
            out["netflix_shape_fp64"] = nline
        else:
            q = p
        kq, lq = WORKLOADS["netflix"]["k0"], WORKLOADS["netflix"]["lam"]
        out["lmsvd_history"] = lmsvd_history(bmg, synth, dev, prob, W, H, kq, lq, recs, sec)
        out["precision_modes"] = precision_steps(bmg, q, dev, kq, lq, recs[-1]["F"])
        out["time_to_tol"] = time_to_tol(bmg, synth, dev)
        out["paper_tables"] = paper_tables(bmg, synth, dev)
        out["time_to_tol_gpu_bound"] = time_to_tol_gpu_bound(bmg, synth, dev)
        out["bf16_mode"] = bf16_mode(bmg, synth, dev)
        out["sparsa_step"] = sparsa_step(bmg, synth, dev, out["time_to_tol"]["fp64"],
                                         out["time_to_tol_gpu_bound"]["lambda_100"]["fp64"])
        out["polymf_bm"] = polymf_bm(bmg, synth, dev, prob, q, out["time_to_tol"]["fp64"],
                                     out["time_to_tol_gpu_bound"]["lambda_100"]["fp64"])
        del prob
        out["rke_qsdp"] = rke_qsdp(bmg, synth, dev)
        out["serve"] = serving(bmg, synth, dev, args.serve_count)
        out["serve_literal_lambda"] = serving_literal(bmg, synth, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(p, wl["k0"])
    print(json.dumps(out), flush=True)


def step_line(bmg, p, workload, scale, precision, steps, warmup, bm_solver, dev, hist=0, dense_rows=0.0):
    """Times `steps` benchmark steps (after `warmup`) on problem p: one step is
    bmg_solve limited to one outer iteration (initialisation, 3 BM epochs, one
    PG step, objective), every step from the same state.  Returns the line's
    fields, the problem, its factor buffers, the step records and seconds per
    step."""
    import torch
    wl = WORKLOADS[workload]
    k0, lam, k_cap = wl["k0"], wl["lam"], wl["k_cap"]
    prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=k_cap, precision=precision,
                                 device=dev, lmsvd_p=hist, dense_rows=dense_rows if bm_solver == "psd" else 0.0)
    W, H = prob.zeros_factors()
    log("%s %s resident on %s (%.2f GB workspace)" % (p.name, precision, dev, prob.ws.numel() / 1e9))

    def step():
        return prob.bmg_solve(W, H, lam=lam, k_init=k0, max_iter=1, tol=0.0, seed=1003, timing=1,
                              bm_solver=bm_solver)[3]

    for i in range(warmup):
        r = step()
        log("warmup %d: k=%d F=%.6g passes=%d" % (i, r["k"], r["F"], r["sparse_passes"]))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    recs = []
    for i in range(steps):
        recs.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log("%s %s: timed %d steps in %.3fs" % (workload, precision, steps, elapsed))
    nbytes = sum(r["sparse_bytes"] for r in recs)
    value = nbytes / elapsed / 1e9
    kms = [sum(r["kernel_ms"][c] for r in recs) for c in range(3)]
    kby = [sum(r["kernel_bytes"][c] for r in recs) for c in range(3)]
    kla = [sum(r["kernel_launches"][c] for r in recs) for c in range(3)]
    dom = max(range(3), key=lambda c: kms[c])
    achieved = kby[dom] / (kms[dom] / 1e3) / 1e9 if kms[dom] > 0 else 0.0
    name = wl["name"] if scale == 1.0 else "%s_x%g" % (wl["name"], scale)
    traffic = traffic_for(KERNEL_SYMBOLS[dom], name, precision)
    line = {
        "value": round(value, 3), "ms_per_step": round(elapsed / steps * 1e3, 3),
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[precision],
        "config": {"workload": "%s: %dx%d, nnz=%d, %s, lambda=%g, k0=%d" % (
                       name, p.m, p.n, p.nnz, wl["desc"], lam, k0),
                   "step": "init (HMT+Nystrom) + 3 BM epochs + 1 inexact PG step + objective",
                   "precision": precision, "bm_solver": bm_solver, "k_cap": k_cap,
                   "dense_rows": dense_rows if bm_solver == "psd" else 0.0,
                   "rank_after_step": recs[-1]["k"],
                   "ssi_iters_per_step": recs[-1]["ssi_iters"],
                   "sparse_passes_per_step": recs[-1]["sparse_passes"],
                   "frac_of_hbm_peak_whole_step": round(value / PEAK_HBM_GBS, 4)},
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom],
                     "achieved": round(achieved, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(kby[dom] / max(kla[dom], 1)),
                     "avg_launch_us": round(kms[dom] / max(kla[dom], 1) * 1e3, 2)},
        "kernels": {KERNEL_SYMBOLS[c]: {"launches": kla[c], "ms": round(kms[c], 3),
                                        "GB/s": round(kby[c] / (kms[c] / 1e3) / 1e9, 2) if kms[c] else None}
                    for c in range(3)},
        "F_after_step": recs[-1]["F"],
    }
    return line, prob, W, H, recs, elapsed / steps


def lmsvd_history(bmg, synth, dev, prob, W, H, k0, lam, recs0, sec0, steps=3):
    """Algorithm 2 with p_t = 1, 2 history blocks against p_t = 0, in FP64:
    the benchmark step itself, the 1000 x 1500 solve to residual 1e-6 (three
    seeds, objective against the certified optimum) and the quarter-scale
    Netflix-shaped solve at lambda 100 to 1e-4 (three seeds).  Reports wall
    time, summed subspace iterations and sparse passes."""
    import numpy as np
    import torch
    out = {"step": {"p0": {"ms_per_step": round(sec0 * 1e3, 3), "ssi_iters": recs0[-1]["ssi_iters"],
                           "sparse_passes": recs0[-1]["sparse_passes"]}}}
    for hp in (1, 2):
        run = lambda: prob.bmg_solve(W, H, lam=lam, k_init=k0, max_iter=1, tol=0.0, seed=1003,  # noqa: E731
                                     lmsvd_p=hp, bm_solver="psd")[3]
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rr = [run() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out["step"]["p%d" % hp] = {"ms_per_step": round(dt * 1e3, 3), "ssi_iters": rr[-1]["ssi_iters"],
                                   "sparse_passes": rr[-1]["sparse_passes"],
                                   "rel_F_vs_p0": abs(rr[-1]["F"] - recs0[-1]["F"]) / abs(recs0[-1]["F"])}
        log("step with lmsvd_p=%d: %.1f ms, %d subspace iterations" % (hp, dt * 1e3, rr[-1]["ssi_iters"]))
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "small_uniform.json")))
    cases = [("small_uniform tol 1e-6", synth.small_uniform(), 0.5, 8, 1e-6, (11, 12, 13), 256,
              golden["F"], (0, 1, 2)),
             ("netflix_shape x0.25 lambda 100 tol 1e-4", synth.netflix_shape(scale=0.25), 100.0, 16,
              1e-4, (3, 4, 5), 128, None, (0, 1))]
    for name, p, lm, kk, tol, seeds, kc, Fref, hps in cases:
        prob2 = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=kc, precision="fp64",
                                      device=dev, lmsvd_p=max(hps))
        rec = {}
        for hp in hps:
            prob2.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=seeds[0], max_iter=2, lmsvd_p=hp)
            secs, ssi, passes, Fs = [], [], [], []
            for sd in seeds:
                t0 = time.perf_counter()
                W2, H2, k2, r = prob2.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=sd, max_iter=1000,
                                                lmsvd_p=hp)
                secs.append(time.perf_counter() - t0)
                ssi.append(r["ssi_iters"]); passes.append(r["sparse_passes"]); Fs.append(r["F"])
            rec["p%d" % hp] = {"seconds_median": round(float(np.median(secs)), 4), "ssi_iters": ssi,
                               "sparse_passes": passes}
            if Fref is not None:
                rec["p%d" % hp]["max_rel_err_vs_oracle_optimum"] = max(abs(F - Fref) / Fref for F in Fs)
            else:
                rec["p%d" % hp]["F"] = Fs
            log("%s lmsvd_p=%d: median %.3fs, subspace iterations %s" % (name, hp, np.median(secs), ssi))
        out[name] = rec
        del prob2
    return out


def sparsa_step(bmg, synth, dev, fixed_small, fixed_quarter):
    """The SpaRSA step rule (BB step + backtracking on eq. back) against the
    fixed step alpha = 1.99, FP64: the 1000 x 1500 solve to 1e-6 (five seeds,
    objective against the certified optimum) and the quarter-scale
    Netflix-shaped solve at lambda 100 to 1e-4 (three seeds).  Fixed-step
    figures are those of the time-to-tolerance runs above."""
    import numpy as np
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "small_uniform.json")))
    out = {}
    cases = [("small_uniform tol 1e-6", synth.small_uniform(), 0.5, 8, 1e-6, (11, 12, 13, 14, 15), 256,
              fixed_small),
             ("netflix_shape x0.25 lambda 100 tol 1e-4", synth.netflix_shape(scale=0.25), 100.0, 16, 1e-4,
              (3, 4, 5), 128, fixed_quarter)]
    for name, p, lm, kk, tol, seeds, kc, fixed in cases:
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=kc, precision="fp64",
                                     device=dev, sparsa=True)
        prob.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=seeds[0], max_iter=2, step_rule="sparsa")
        secs, iters, trials, ssi, Fs = [], [], [], [], []
        for sd in seeds:
            t0 = time.perf_counter()
            W, H, k, r = prob.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=sd, max_iter=1000,
                                        step_rule="sparsa")
            secs.append(time.perf_counter() - t0)
            iters.append(r["iters"]); trials.append(r["pg_trials"]); ssi.append(r["ssi_iters"])
            Fs.append(r["F"])
        rec = {"seconds_median": round(float(np.median(secs)), 4), "iters": iters, "prox_computations": trials,
               "ssi_iters": ssi, "fixed_step_seconds_median": fixed["seconds_median"],
               "fixed_step_iters": fixed["iters"]}
        if name.startswith("small"):
            rec["max_rel_err_vs_oracle_optimum"] = max(abs(F - golden["F"]) / golden["F"] for F in Fs)
        else:
            rec["F"] = Fs
        out[name] = rec
        log("sparsa %s: median %.3fs (fixed %.3fs), iters %s (fixed %s), prox computations %s" % (
            name, rec["seconds_median"], fixed["seconds_median"], iters, fixed["iters"], trials))
        del prob
    return out


def polymf_bm(bmg, synth, dev, prob, p, fixed_small, fixed_quarter):
    """The polyMF-SS BM solver (the library default, as in the paper) against
    the preconditioned steepest descent, FP64: three epochs of each from the
    same factors on the Netflix-shaped workload (rank 16, lambda 20; BM
    objective after each epoch and time per epoch), then the 1000 x 1500 solve
    to 1e-6 (five seeds) and the quarter-scale Netflix-shaped solve at lambda
    100 to 1e-4 (three seeds) with steepest descent in the BM phase.  The
    polyMF-SS figures of the solves are those of the time-to-tolerance runs
    above."""
    import numpy as np
    import torch
    k, lam = 16, 20.0
    rng = np.random.default_rng(7)
    W0 = np.zeros((p.m, 64)); H0 = np.zeros((p.n, 64))
    W0[:, :k] = 0.3 * rng.standard_normal((p.m, k))
    H0[:, :k] = 0.3 * rng.standard_normal((p.n, k))
    out = {"epochs_netflix_shape_k16": {}}
    for name, fn in (("psd", prob.bmg_bm_epochs), ("polymf", prob.bmg_polymf_epochs)):
        W = torch.as_tensor(W0, device=dev); H = torch.as_tensor(H0, device=dev)
        Fs, ts = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Fs.append(fn(W, H, k, lam, epochs=1))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out["epochs_netflix_shape_k16"][name] = {"F_bm_after_epoch": Fs,
                                                 "ms_per_epoch": [round(x * 1e3, 2) for x in ts]}
        log("BM %s: F after epochs %s, ms %s" % (name, ["%.6g" % f for f in Fs], ["%.1f" % (x * 1e3) for x in ts]))
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "small_uniform.json")))
    cases = [("small_uniform tol 1e-6", synth.small_uniform(), 0.5, 8, 1e-6, (11, 12, 13, 14, 15), 256,
              fixed_small),
             ("netflix_shape x0.25 lambda 100 tol 1e-4", synth.netflix_shape(scale=0.25), 100.0, 16, 1e-4,
              (3, 4, 5), 128, fixed_quarter)]
    for name, q, lm, kk, tol, seeds, kc, fixed in cases:
        pq = bmg.Problem.from_host(q.row_ptr, q.col, q.val, q.m, q.n, k_cap=kc, precision="fp64", device=dev)
        pq.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=seeds[0], max_iter=2, bm_solver="psd")
        secs, iters, Fs = [], [], []
        for sd in seeds:
            t0 = time.perf_counter()
            W, H, k2, r = pq.bmg_solve(lam=lm, k_init=kk, tol=tol, seed=sd, max_iter=1000, bm_solver="psd")
            secs.append(time.perf_counter() - t0)
            iters.append(r["iters"]); Fs.append(r["F"])
        rec = {"psd_seconds_median": round(float(np.median(secs)), 4), "psd_iters": iters,
               "polymf_seconds_median": fixed["seconds_median"], "polymf_iters": fixed["iters"],
               "polymf_speedup": round(float(np.median(secs)) / fixed["seconds_median"], 3)}
        if name.startswith("small"):
            rec["max_rel_err_vs_oracle_optimum"] = max(abs(F - golden["F"]) / golden["F"] for F in Fs)
        else:
            rec["F"] = Fs
        out[name] = rec
        log("psd BM %s: median %.3fs (polymf %.3fs), iters %s (polymf %s)" % (
            name, rec["psd_seconds_median"], fixed["seconds_median"], iters, fixed["iters"]))
        del pq
    return out


RKE_K_CAP, RKE_LMSVD_P = 160, 1   # kernel-estimation runs: rank cap and LmSVD history


def rke_qsdp(bmg, synth, dev):
    """BM-Global on the kernel-estimation QSDP (bmg_rke_solve, FP64) to relative
    prox-gradient residual 1e-4: synthetic objects in R^3 with about 40 random
    partners each and noisy squared distances (stored symmetrically), two
    sizes, two algorithm seeds each."""
    out = {}
    for n, lam in ((20_000, 10.0), (100_000, 20.0)):
        p = synth.rke(n, 40, lam=lam, seed=7)
        dp = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=RKE_K_CAP, device=dev,
                                   lmsvd_p=RKE_LMSVD_P)
        dp.bmg_rke_solve(lam=lam, k_init=8, tol=1e-4, seed=1, max_iter=2, bm_epochs=10,
                         lmsvd_p=RKE_LMSVD_P)
        secs, iters, ranks, Fs, ssi = [], [], [], [], []
        for sd in (1, 2):
            t0 = time.perf_counter()
            W, k, r = dp.bmg_rke_solve(lam=lam, k_init=8, tol=1e-4, seed=sd, max_iter=3000, bm_epochs=10,
                                       lmsvd_p=RKE_LMSVD_P)
            secs.append(time.perf_counter() - t0)
            iters.append(r["iters"]); ranks.append(k); Fs.append(r["F"])
            ssi.append(round(r["ssi_iters"] / (r["iters"] + 1), 2))
            assert r["status"] == 0
        out["n%d_pairs%d" % (n, p.nnz // 2)] = {"lambda": lam, "seconds": [round(x, 3) for x in secs],
                                                 "iters": iters, "rank": ranks, "F": Fs,
                                                 "ssi_per_pg_step": ssi, "lmsvd_p": RKE_LMSVD_P,
                                                 "rel_F_spread": (max(Fs) - min(Fs)) / abs(max(Fs))}
        log("rke n=%d (%d pairs): %s s, iters %s, rank %s" % (n, p.nnz // 2, ["%.2f" % x for x in secs],
                                                              iters, ranks))
        del dp
    return out


def precision_steps(bmg, p, dev, k0, lam, F64, steps=2):
    """The same step (one outer iteration from the same start) in the lower
    precision modes on the same workload; rel_F_vs_fp64 compares the objective
    each mode reports after the step (FP64 evaluation of its factors) with the
    FP64 mode's."""
    import torch
    out = {}
    for prec in ("fp32", "bf16"):
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=64, precision=prec,
                                     device=dev)
        W, H = prob.zeros_factors()
        run = lambda: prob.bmg_solve(W, H, lam=lam, k_init=k0, max_iter=1, tol=0.0, seed=1003,  # noqa: E731
                                     timing=1, refresh_every=1000, bm_solver="psd")[3]
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = [run() for _ in range(steps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        kms = [sum(r["kernel_ms"][c] for r in recs) / steps for c in range(3)]
        out[prec] = {"ms_per_step": round(dt * 1e3, 3),
                     "GB/s": round(sum(r["sparse_bytes"] for r in recs) / steps / dt / 1e9, 2),
                     "bf16_pass_fraction": round(recs[-1]["bf16_passes"] / max(recs[-1]["sparse_passes"], 1), 4),
                     "rank_after_step": recs[-1]["k"],
                     "rel_F_vs_fp64": abs(recs[-1]["F"] - F64) / abs(F64),
                     "kernel_ms_per_step": {KERNEL_SYMBOLS[c]: round(kms[c], 3) for c in range(3)}}
        log("step %s: %.1f ms" % (prec, dt * 1e3))
        del prob
    return out


def bf16_mode(bmg, synth, dev, seeds=(3, 4, 5)):
    """The BF16 mode (BF16 gathers, FP32 accumulation and masters, FP64 refresh
    every 5 outer iterations) on the Netflix-shaped generator at scale 0.25,
    lambda = 300, where tests/golden holds the oracle's certified optimum F*:
    the objective error against F* after each refresh and the fraction of
    sparse passes that gathered BF16; then time to tolerance against the FP64
    solver at the same tolerance (1e-3, which the BF16 phase reaches itself, and
    1e-5), with the final objective errors, the speed-up at equal accuracy.
    Steepest descent in the BM phase throughout: its whole-Omega passes gather
    BF16 (polyMF-SS's column passes gather FP32)."""
    import numpy as np
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "netflix_quarter_lam300.json")))
    p = synth.netflix_shape(scale=0.25)
    lam, k0, Fs = g["lam"], g["k0"], g["F"]
    evaluator = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=64, precision="fp64",
                                      device=dev)
    probs = {pr: bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=64, precision=pr, device=dev)
             for pr in ("fp64", "bf16")}
    out = {"workload": "netflix_shape x0.25: %dx%d nnz=%d, lambda=%g, k0=%d; F* = %.10g (oracle, duality gap "
                       "%.2g)" % (p.m, p.n, p.nnz, lam, k0, Fs, g["dual_gap"]),
           "per_refresh": []}
    for it in (5, 10, 15, 20, 25, 30):
        W, H, k, r = probs["bf16"].bmg_solve(lam=lam, k_init=k0, tol=0.0, max_iter=it, seed=seeds[0],
                                             refresh_every=5, bm_solver="psd")
        F = evaluator.bmg_objective(W, H, k, lam)
        out["per_refresh"].append({"iters": it, "rel_F_err_vs_oracle": (F - Fs) / Fs, "residual": r["residual"],
                                   "rank": k, "bf16_pass_fraction": round(r["bf16_passes"] / r["sparse_passes"], 4)})
    for tol in (1e-3, 1e-5):
        rec = {}
        for pr in ("fp64", "bf16"):
            probs[pr].bmg_solve(lam=lam, k_init=k0, tol=tol, seed=seeds[0], max_iter=2, bm_solver="psd")
            secs, errs, fr, iters = [], [], [], []
            for sd in seeds:
                t0 = time.perf_counter()
                W, H, k, r = probs[pr].bmg_solve(lam=lam, k_init=k0, tol=tol, seed=sd, max_iter=400,
                                                 bm_solver="psd")
                secs.append(time.perf_counter() - t0)
                F = evaluator.bmg_objective(W, H, k, lam)
                errs.append(abs(F - Fs) / Fs)
                fr.append(r["bf16_passes"] / max(r["sparse_passes"], 1))
                iters.append(r["iters"])
            rec[pr] = {"seconds_median": round(float(np.median(secs)), 4), "iters": iters,
                       "max_rel_F_err_vs_oracle": max(errs), "bf16_pass_fraction": round(float(np.mean(fr)), 4)}
        rec["bf16_speedup_vs_fp64"] = round(rec["fp64"]["seconds_median"] / rec["bf16"]["seconds_median"], 3)
        out["tol_%g" % tol] = rec
        log("bf16 mode tol %g: fp64 %.3fs (err %.1e) bf16 %.3fs (err %.1e, %.0f%% bf16 passes)" % (
            tol, rec["fp64"]["seconds_median"], rec["fp64"]["max_rel_F_err_vs_oracle"],
            rec["bf16"]["seconds_median"], rec["bf16"]["max_rel_F_err_vs_oracle"],
            100 * rec["bf16"]["bf16_pass_fraction"]))
    del probs, evaluator
    return out


def time_to_tol_gpu_bound(bmg, synth, dev, lams=(300.0, 100.0), seeds=(3, 4, 5)):
    """Time to relative residual 1e-4 on the quarter-scale Netflix-shaped
    problem (4,442 x 120,047, |Omega| = 6.25e6, same generator), where the
    sparse passes dominate, in FP64, FP32 and BF16: median over algorithm
    seeds; each solution's objective is evaluated in FP64 by the library and
    compared with the FP64 solution of the same seed."""
    import numpy as np
    p = synth.netflix_shape(scale=0.25)
    evaluator = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=128, precision="fp64",
                                  device=dev)
    out = {"workload": "netflix_shape x0.25: %dx%d nnz=%d, k0=16, tol 1e-4" % (p.m, p.n, p.nnz)}
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "netflix_quarter_lam300.json")))
    for lam in lams:
        rec = {}
        ref = {}
        for prec in ("fp64", "fp32", "bf16"):
            prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=128,
                                         precision=prec, device=dev)
            prob.bmg_solve(lam=lam, k_init=16, tol=1e-4, seed=seeds[0], max_iter=2)
            secs, errs, iters, ranks, Fs_all = [], [], [], [], []
            for sd in seeds:
                t0 = time.perf_counter()
                W, H, k, r = prob.bmg_solve(lam=lam, k_init=16, tol=1e-4, seed=sd, max_iter=400)
                secs.append(time.perf_counter() - t0)
                F = evaluator.bmg_objective(W, H, k, lam)
                Fs_all.append(F)
                if prec == "fp64":
                    ref[sd] = F
                errs.append(abs(F - ref[sd]) / abs(ref[sd]))
                iters.append(r["iters"]); ranks.append(k)
            rec[prec] = {"seconds_median": round(float(np.median(secs)), 4), "iters": iters,
                         "rank": ranks, "max_rel_F_vs_fp64": max(errs)}
            if lam == golden["lam"]:
                rec[prec]["max_rel_F_err_vs_oracle_optimum"] = max(abs(F - golden["F"]) / golden["F"]
                                                                   for F in Fs_all)
            del prob
        for prec in ("fp32", "bf16"):
            rec[prec]["speedup_vs_fp64"] = round(rec["fp64"]["seconds_median"] / rec[prec]["seconds_median"], 3)
        out["lambda_%g" % lam] = rec
        log("time-to-tol (x0.25, lambda %g): fp64 %.3fs fp32 %.3fs bf16 %.3fs" % (
            lam, rec["fp64"]["seconds_median"], rec["fp32"]["seconds_median"], rec["bf16"]["seconds_median"]))
    return out


def serving(bmg, synth, dev, count):
    """Serving stream: requests arrive (Poisson, 20/s) with m ~ U[500, 20000],
    n ~ U[1000, 50000], density ~ U[0.5%, 2%], rank 3..15, noise variance 0.05,
    lambda midway between the sampling-noise level of P_Omega(A) and the
    weakest truth direction; FP32 solves to residual 1e-5 (steepest-descent BM
    solver, 1.6x the throughput of polyMF-SS on these requests) through the server
    (admission by footprint in an 8 GiB arena, 8 slots, sparse passes of the
    running problems sharing launches).  Latency = completion - arrival.  Also
    the same requests all submitted at once (capacity).  Baseline: the same
    problems one after another with the plain FP64 solver to the same residual.
    Per truth-rank class: how many results have the truth's rank, and p50/p99."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    reqs = synth.serving_stream(count=count)
    t0 = time.time()
    # the generator runs in C without the GIL: build the requests in parallel
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        probs = list(ex.map(synth.request_problem, reqs))
    log("serving: %d requests generated in %.1fs (nnz %.1fM..%.1fM)" % (
        count, time.time() - t0, min(p.nnz for p in probs) / 1e6, max(p.nnz for p in probs) / 1e6))
    # steepest descent in the BM phase: on these small low-rank requests its
    # whole-Omega passes take fewer launches than polyMF-SS's column passes
    opts = dict(tol=1e-5, k_init=8, max_iter=3000, seed=7, bm_solver="psd")

    def run(paced):
        srv = bmg.Server(8 << 30, max_slots=8, device=dev)
        tickets = []
        start = time.perf_counter()
        for r, p in zip(reqs, probs):
            if paced:
                delay = r.arrival - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
            tickets.append(srv.submit(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=128,
                                      precision="fp32", lam=r.lam, **opts))
        srv.drain()
        makespan = time.perf_counter() - start
        infos = [srv.poll(t)[0] for t in tickets]
        st = srv.stats()
        srv.close()
        lat = np.array([i["total_s"] for i in infos])
        return infos, {"p50_s": round(float(np.percentile(lat, 50)), 4),
                       "p99_s": round(float(np.percentile(lat, 99)), 4),
                       "throughput_per_s": round(count / makespan, 3),
                       "makespan_s": round(makespan, 3), "peak_running": st["peak_running"],
                       "peak_arena_GB": round(st["peak_bytes"] / 1e9, 3),
                       "shared_launches": st["shared_launches"],
                       "batched_passes": st["batched_passes"]}

    infos, paced = run(True)
    binfos, burst = run(False)
    ok = sum(1 for i in infos if i["state"] == 2 and i["status"] == 0)
    # plain FP64 solver, one problem at a time, same tolerance
    t1 = time.perf_counter()
    plain = []
    for r, p in zip(reqs, probs):
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=128, precision="fp64",
                                     device=dev)
        tt = time.perf_counter()
        try:
            _, _, k, res = prob.bmg_solve(lam=r.lam, **opts)
            plain.append((time.perf_counter() - tt, res["F"]))
        except bmg.BmgError as e:
            log("plain fp64 solve failed: %s" % e)
            plain.append((time.perf_counter() - tt, float("nan")))
        del prob
    plain_total = time.perf_counter() - t1
    rel = [abs(i["result"]["F"] - f) / abs(f) for i, (_, f) in zip(infos, plain)
           if i["state"] == 2 and f == f and f != 0]
    same = all(a["result"]["F"] == b["result"]["F"] for a, b in zip(infos, binfos))
    out = {"requests": count, "converged": ok, "arrival_span_s": round(reqs[-1].arrival, 3),
           "poisson_20_per_s": paced, "all_at_once": burst,
           "plain_fp64_sequential": {"total_s": round(plain_total, 3),
                                     "p50_solve_s": round(float(np.median([p[0] for p in plain])), 4),
                                     "throughput_per_s": round(count / plain_total, 3)},
           "capacity_vs_plain_fp64": round(burst["throughput_per_s"] * plain_total / count, 3),
           "max_rel_F_diff_vs_fp64": float(max(rel)) if rel else None,
           "F_identical_paced_vs_burst": same,
           "ranks": sorted({i["k"] for i in infos}),
           "rank0_results": sum(1 for i in infos if i["k"] == 0),
           "truth_rank_recovered": sum(1 for i, r in zip(infos, reqs) if i["k"] == r.rank),
           "truth_above_noise": sum(1 for r in reqs if r.dsig_r > r.L)}
    classes = {}
    for i, r in zip(infos, reqs):
        c = classes.setdefault(r.rank, {"requests": 0, "rank_equal": 0, "ranks": [], "lat": []})
        c["requests"] += 1
        c["rank_equal"] += int(i["k"] == r.rank)
        c["ranks"].append(i["k"])
        c["lat"].append(i["total_s"])
    out["by_truth_rank"] = {str(rk): {"requests": c["requests"], "rank_equal": c["rank_equal"],
                                      "rank_min": min(c["ranks"]), "rank_max": max(c["ranks"]),
                                      "p50_s": round(float(np.percentile(c["lat"], 50)), 4),
                                      "p99_s": round(float(np.percentile(c["lat"], 99)), 4)}
                            for rk, c in sorted(classes.items())}
    log("serving: p50 %.3fs p99 %.3fs at 20/s; all at once %.2f req/s vs plain fp64 sequential %.2f req/s" % (
        paced["p50_s"], paced["p99_s"], burst["throughput_per_s"], out["plain_fp64_sequential"]["throughput_per_s"]))
    return out


PAPER_CPU_S = {"100k": {"1e-04": 0.44, "1e-08": 1.7, "1e-12": 3.3},
               "toy": {"1e-04": 1.2, "1e-08": 4.9, "1e-12": 8.0}}


def paper_tables(bmg, synth, dev, seed=3):
    """Time to relative objective error eps = (F - F*) / F* <= 1e-4, 1e-8, 1e-12,
    the measure of the paper's timing tables, on rating-shaped stand-ins of
    its two tabled problems (synth.movielens_shape: the MovieLens-100k shape
    at lambda 15 and the toy example's shape at lambda 36), FP64, the default
    options (polyMF-SS, 3 BM epochs per PG step, alpha 1.99).  F* is the
    oracle's, certified by its duality gap (tests/golden).  The solve runs to
    relative residuals 1e-3 ... 1e-12; the time to eps is that of the fastest
    run whose objective (FP64, by the library) is within eps.  The paper's
    CPU times (8-core Xeon, real data of the same shape) are quoted beside,
    as context only."""
    import numpy as np
    out = {}
    for which, fname in (("100k", "movielens100k_shape_lam15.json"), ("toy", "toy_shape_lam36.json")):
        path = os.path.join(ROOT, "tests", "golden", fname)
        if not os.path.exists(path):
            continue
        g = json.load(open(path))
        p = synth.movielens_shape(which)
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=192, precision="fp64", device=dev)
        prob.bmg_solve(lam=p.lam, k_init=p.k0, tol=1e-3, seed=seed, max_iter=2)
        runs = []
        for e in range(3, 13):
            tol = 10.0 ** -e
            t0 = time.perf_counter()
            W, H, k, r = prob.bmg_solve(lam=p.lam, k_init=p.k0, tol=tol, seed=seed, max_iter=5000)
            sec = time.perf_counter() - t0
            F = prob.bmg_objective(W, H, k, p.lam)
            runs.append({"tol": tol, "seconds": round(sec, 4), "iters": r["iters"], "rank": k,
                         "rel_F_err": (F - g["F"]) / g["F"], "status": r["status"]})
        tte = {}
        for eps in (1e-4, 1e-8, 1e-12):
            ok = [x["seconds"] for x in runs if x["rel_F_err"] <= eps]
            tte["%.0e" % eps] = min(ok) if ok else None
        out[p.name] = {"lambda": p.lam, "F_star": g["F"], "rank_star": g["rank"],
                       "dual_gap_rel": g["dual_gap"] / g["F"], "time_to_eps_s": tte,
                       "paper_cpu_s_same_shape": PAPER_CPU_S[which], "runs": runs}
        log("paper table %s: time to 1e-4 / 1e-8 / 1e-12: %s (paper, CPU: %s)" % (
            p.name, tte, PAPER_CPU_S[which]))
        del prob
    return out


def serving_literal(bmg, synth, dev, count=64):
    """The serving stream with the configuration's literal lambda ~ U[0.1, 5]
    (lam_rule "uniform"), which lies below the sampling-noise level of nearly
    every request: the solutions fit the noise at ranks far above the truth's.
    The first `count` requests of the stream, FP32 solves to 1e-5 with k_cap
    512 through a 32 GiB arena, 8 slots, Poisson 20/s.  Reports p50/p99
    latency, throughput, the rank distribution, how many results end at rank 0
    or below their truth rank, and the requests whose rank outgrew k_cap."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    reqs = synth.serving_stream(count=count, lam_rule="uniform")
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        probs = list(ex.map(synth.request_problem, reqs))
    opts = dict(tol=1e-5, k_init=8, max_iter=3000, seed=7, bm_solver="psd")
    srv = bmg.Server(32 << 30, max_slots=8, device=dev)
    tickets, start = [], time.perf_counter()
    for r, p in zip(reqs, probs):
        delay = r.arrival - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=512, precision="fp32",
                                  lam=r.lam, **opts))
    srv.drain()
    makespan = time.perf_counter() - start
    infos = [srv.poll(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    done = [(i, r) for i, r in zip(infos, reqs) if i["state"] == 2]
    lat = np.array([i["total_s"] for i, _ in done]) if done else np.zeros(1)
    ranks = [i["k"] for i, _ in done]
    out = {"requests": count, "lambda_rule": "uniform [0.1, 5]", "completed": len(done),
           "failed": sum(1 for i in infos if i["state"] == 3),
           "p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
           "throughput_per_s": round(count / makespan, 3), "peak_running": st["peak_running"],
           "rank_min": min(ranks) if ranks else None, "rank_median": float(np.median(ranks)) if ranks else None,
           "rank_max": max(ranks) if ranks else None,
           "rank0_results": sum(1 for k in ranks if k == 0),
           "below_truth_rank": sum(1 for i, r in done if i["k"] < r.rank),
           "above_truth_rank": sum(1 for i, r in done if i["k"] > r.rank)}
    log("serving (literal lambda): %d/%d done, p50 %.3fs p99 %.3fs, ranks %s..%s" % (
        len(done), count, out["p50_s"], out["p99_s"], out["rank_min"], out["rank_max"]))
    return out


def time_to_tol(bmg, synth, dev, seeds=(11, 12, 13, 14, 15)):
    """Full solves of the 1000 x 1500 workload (|Omega| = 50,000, lambda = 0.5,
    k0 = 8) to relative optimality residual 1e-6 in FP64, FP32 and BF16 (BF16:
    FP64 refresh every 5 outer iterations, whose PG steps gather FP32), one per
    algorithm seed; median and interquartile range of the wall time.  Each
    solution's objective is evaluated in FP64 by the library (bmg_objective on
    an FP64 instance of the problem) and compared with the certified optimum
    stored in tests/golden/small_uniform.json."""
    import numpy as np
    p = synth.small_uniform()
    out = {"workload": "small_uniform 1000x1500 nnz=50000 lambda=0.5 k0=8", "tol": 1e-6,
           "seeds": list(seeds)}
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "small_uniform.json")))
    evaluator = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=256, precision="fp64",
                                  device=dev)
    for prec in ("fp64", "fp32", "bf16"):
        # intermediate prox outputs can reach rank ~130 on the way to the rank-91 optimum
        prob = bmg.Problem.from_host(p.row_ptr, p.col, p.val, p.m, p.n, k_cap=256, precision=prec,
                                     device=dev)
        prob.bmg_solve(lam=p.lam, k_init=p.k0, tol=1e-6, seed=seeds[0], max_iter=2)   # warm caches
        secs, errs, iters, ranks, conv, fr = [], [], [], [], [], []
        for sd in seeds:
            t0 = time.perf_counter()
            W, H, k, r = prob.bmg_solve(lam=p.lam, k_init=p.k0, tol=1e-6, seed=sd, max_iter=1000)
            secs.append(time.perf_counter() - t0)
            F64 = evaluator.bmg_objective(W, H, k, p.lam)
            errs.append((F64 - golden["F"]) / golden["F"])
            iters.append(r["iters"]); ranks.append(k); conv.append(r["status"] == 0)
            fr.append(r["bf16_passes"] / max(r["sparse_passes"], 1))
        q1, med, q3 = (float(v) for v in np.percentile(secs, [25, 50, 75]))
        out[prec] = {"seconds_median": round(med, 4), "seconds_iqr": [round(q1, 4), round(q3, 4)],
                     "iters": iters, "rank": ranks, "converged": all(conv),
                     "max_rel_err_vs_oracle_optimum": max(abs(x) for x in errs)}
        if prec == "bf16":
            out[prec]["bf16_pass_fraction"] = round(float(np.mean(fr)), 4)
        log("time-to-tol %s: median %.3fs over %d seeds, iters %s" % (prec, med, len(seeds), iters))
    for prec in ("fp32", "bf16"):
        out[prec]["speedup_vs_fp64"] = round(out["fp64"]["seconds_median"] / out[prec]["seconds_median"], 3)
    return out


if __name__ == "__main__":
    main()
