#!/usr/bin/env python3
"""Benchmark of the MI355X interior-point hot path on the sparse-SOCP workload.

One step = one complete solve to the 1e-8 tests from the initial point
(every row of the hot path: residuals, cone scalings, KKT factorisation,
refinement solves, directions, step lengths, update), with the problem
already resident in HBM.  `value` = IPM iterations per second over the timed
solves; ms_per_step = milliseconds per solve.

Prints one JSON line.  Flags: --steps K --warmup W (solves), --gpus N (only
N = 1 exists: there is one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_nt_f64_sparse_socp_traffic.json")

METRIC = "time per IPM iteration & solve-to-1e-8 gap; batched solves/s + p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


_T0 = time.perf_counter()


def progress(msg):
    """One line per step on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def workload_desc(p):
    return (f"sparse_socp: n={p.n} (x 20,000 + 20 factor vars), m={p.m} (zero 10,020 incl. 20 dense lift rows, "
            f"nonneg 30,000, 40,000 SOC-3), A 6 nnz/row N(0,1), P = diag(U(0.01,1)) + rank-20 factor, seed 0")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the reference copy kernel), or
    None when there is none or the kernel source changed since it was taken."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if rec.get("kernel") != kernel or hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def calibrate_copy(nbytes=1 << 30, reps=3):
    """Runs the reference copy kernel (known traffic: nbytes read, nbytes
    written per launch) so that a counter run can scale byte counters."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        HC.test_copy(src, dst)
    torch.cuda.synchronize()
    assert bool((dst == 1).all())
    print(f"reference copy: {reps} launches of {nbytes} bytes", file=sys.stderr)


HBM_PEAK_GBS = 8000.0


def cone_roofline(info):
    """Cone layer (scalings, M blocks, H applications, d_s, recovery, step
    lengths) from one profiled solve: summed device time of its launches (HIP
    events on the solver's stream) against their algorithmic bytes."""
    ms, b = info["cone_kernel_ms"], info["cone_bytes"]
    achieved = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=None, device_ms_per_iteration=ms / max(1, info["iterations"]),
                algorithmic_bytes_per_iteration=b / max(1, info["iterations"]),
                launches_per_iteration=info["cone_launches"] / max(1, info["iterations"]))


def run_gpu(prob, precision, steps, warmup):
    """Timed solves (no profiling events), then one profiled solve with the
    look-ahead's trailing updates on the main stream (settings.profile = 2) so
    that no timed MFMA update overlaps another kernel: the roofline comes from
    that solve, the throughput from the timed ones."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    progress(f"{prob.name} {precision}: set-up, {warmup} warm-up and {steps} timed solves")
    solver = HC.Solver(prob, precision=precision, profile=0)
    for _ in range(warmup):
        solver.solve()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(solver.solve())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = sum(i["iterations"] for i in infos)
    last = infos[-1]
    solver.close()
    progress(f"{prob.name} {precision}: profiled solve (settings.profile = 2)")
    prof = HC.Solver(prob, precision=precision, profile=2)
    t1 = time.perf_counter()
    pi = prof.solve()
    torch.cuda.synchronize()
    prof_ms = 1e3 * (time.perf_counter() - t1)
    prof.close()
    gemm_ms, gemm_flops, launches = pi["gemm_ms"], pi["gemm_flops"], pi["gemm_launches"]
    peak = FP64_PEAK_TFLOPS if precision == "fp64" else FP32_PEAK_TFLOPS
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms > 0 else 0.0
    kernel = "k_gemm_nt_dma" if precision == "fp64" else "k_gemm_nt_dma32"
    return dict(
        wall=wall, iters=iters, infos=infos, status=last["status_name"], objective=last["obj_primal"],
        res_primal=last["res_primal"], res_dual=last["res_dual"], gap=last["gap"],
        iterations_per_solve=iters / steps, ms_per_solve=1e3 * wall / steps, ms_per_iteration=1e3 * wall / iters,
        factor_ms_per_iteration=sum(i["factor_ms"] for i in infos) / iters,
        kkt_ms_per_iteration=sum(i["solve_kkt_ms"] for i in infos) / iters,
        ir_solves_per_iteration=sum(i["ir_solves"] for i in infos) / iters,
        fp64_fallbacks_per_solve=sum(i["fp64_fallbacks"] for i in infos) / steps,
        roofline=dict(bound="mfma", kernel=kernel,
                      achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
                      traffic=measured_traffic(kernel), traffic_unit="HBM bytes per launch",
                      launches=launches, avg_launch_us=1e3 * gemm_ms / max(1, launches),
                      algorithmic_flops_per_launch=gemm_flops / max(1, launches),
                      measured_in="one solve with settings.profile = 2 (trailing updates on the main stream, "
                                  "no overlap)",
                      gemm_ms_per_solve=gemm_ms, profiled_solve_ms=prof_ms),
        cone_roofline=cone_roofline(pi),
    )


def run_seeds(precision, seeds=(1, 2, 3, 4)):
    """The same configuration at other seeds: one solve each after a warm-up
    (problem resident); time per solve and per iteration."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    out = {}
    for sd in seeds:
        prob = W.sparse_socp(sd)
        progress(f"seed {sd} {precision}")
        s = HC.Solver(prob, precision=precision, profile=0)
        s.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        out[str(sd)] = dict(status=info["status_name"], iterations=info["iterations"], ms_per_solve=1e3 * wall,
                            ms_per_iteration=1e3 * wall / max(1, info["iterations"]), objective=info["obj_primal"])
    return out


def spread(vals):
    v = sorted(vals)
    return dict(median=v[len(v) // 2], min=v[0], max=v[-1])


OTHER_WORKLOADS = ("logreg_exp", "psd_pow", "entropy_max", "portfolio_qp", "multistage_portfolio", "psd_sides_to_32")
MIXED_TOO = ("logreg_exp",)   # also solved in mixed precision (the logistic regression's stated precision)


def run_other_workloads(steps=1, only=None):
    """The other full-size configurations, one FP64 solve each after a warm-up
    solve: status, iterations and time per iteration (problem resident)."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    makers = {"logreg_exp": lambda: W.logreg_exp(0), "psd_pow": lambda: W.psd_pow(0),
              "entropy_max": lambda: W.entropy_max(0, n=10000), "portfolio_qp": lambda: W.portfolio_qp(0, n=25000),
              "multistage_portfolio": lambda: W.multistage_portfolio(0, n=5000, k=50, T=5),
              "psd_sides_to_32": lambda: W.psd_mixed(0, n=2000, sides=(8, 20, 32), per_side=30)}
    out = {}
    for name in OTHER_WORKLOADS:
        if only and name != only:
            continue
        prob = makers[name]()
        progress(f"{name}: set-up, warm-up, {steps} timed and one profiled solve")
        s = HC.Solver(prob)
        s.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [s.solve() for _ in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        it = sum(i["iterations"] for i in infos)
        last = infos[-1]
        s.close()
        sp = HC.Solver(prob, profile=2)
        pinfo = sp.solve()
        sp.close()
        out[name] = dict(problem=prob.name, n=prob.n, m=prob.m, status=last["status_name"],
                         iterations=last["iterations"], objective=last["obj_primal"],
                         ms_per_iteration=1e3 * wall / max(1, it), ms_per_solve=1e3 * wall / steps,
                         factor_ms_per_iteration=last["factor_ms"] / max(1, last["iterations"]),
                         setup_ms=last["setup_ms"],
                         dense_tail=last["n_ordered"], leaf_blocks=last["n_leaves"],
                         cone_roofline=cone_roofline(pinfo))
        if name in MIXED_TOO:   # the configuration's stated precision: FP32 factor, FP64 refinement
            progress(f"{name}: mixed precision, warm-up and {steps} timed solves")
            sm = HC.Solver(prob, precision="mixed")
            sm.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            minfos = [sm.solve() for _ in range(steps)]
            torch.cuda.synchronize()
            mwall = time.perf_counter() - t0
            sm.close()
            mit = sum(i["iterations"] for i in minfos)
            ml = minfos[-1]
            out[name]["mixed"] = dict(
                status=ml["status_name"], iterations=ml["iterations"], objective=ml["obj_primal"],
                objective_rel_diff_vs_fp64=abs(ml["obj_primal"] - last["obj_primal"]) / max(1.0, abs(last["obj_primal"])),
                ms_per_iteration=1e3 * mwall / max(1, mit), ms_per_solve=1e3 * mwall / steps,
                ms_per_solve_vs_fp64=(mwall / steps) / (wall / steps),
                factor_ms_per_iteration=ml["factor_ms"] / max(1, ml["iterations"]),
                ir_solves_per_iteration=sum(i["ir_solves"] for i in minfos) / max(1, mit),
                fp64_fallbacks_per_solve=sum(i["fp64_fallbacks"] for i in minfos) / steps)
    return out


def run_served(count, precision="fp64", rate=2000.0, workers=4, slots=32, budget=64 << 30, seed=0, batched=True,
               feeders=4):
    """The served form on a stream of MPC requests: problems are generated
    beforehand, submitted at their Poisson arrival times by `feeders` threads
    (request i by thread i mod feeders; submit is thread-safe and runs the
    host analysis), and every ticket is waited for; throughput and latency
    come from the server."""
    import threading
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    progress(f"served stream: {count} requests, {precision}, {'batched' if batched else 'per-slot'}")
    probs = [W.mpc_socp(seed, i) for i in range(count)]
    arrivals = W.mpc_arrivals(seed, count, rate)
    srv = HC.Server(hbm_budget_bytes=budget, max_slots=slots, workers=workers, batched=batched,
                    precision=precision)
    tickets = [None] * count
    t0 = time.perf_counter()

    def feed(k):
        for i in range(k, count, feeders):
            dt = arrivals[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(probs[i], tag=i)

    ths = [threading.Thread(target=feed, args=(k,)) for k in range(feeders)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    res = [srv.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    statuses = {}
    for r in res:
        statuses[r["status_name"]] = statuses.get(r["status_name"], 0) + 1
    return dict(
        workload=f"MPC SOCP stream: {count} requests, Poisson {rate:g}/s, T in [10,100], nx in [4,12], "
                 f"nu in [2,6] (n in [64,1812]), seed {seed}",
        precision=precision, engine="batched (one wavefront per problem, one graph launch per tick)" if batched
        else "per-slot workers",
        requests=count, wall_s=wall, solves_per_s=st["solves_per_s"], p50_latency_ms=st["p50_latency_ms"],
        p99_latency_ms=st["p99_latency_ms"], mean_latency_ms=st["mean_latency_ms"],
        mean_iterations=st["iterations"] / max(1, st["completed"]), statuses=statuses,
        hbm_peak_bytes=st["hbm_peak"], workers=workers, max_slots=slots, hbm_budget_bytes=budget,
        feeder_threads=feeders)


def run_batch(count, precision="fp64", seed=0):
    """The first `count` requests of the served stream solved together by one
    hc_solve_batch call (one wave per problem, plain kernel launches, no
    server): problems set up beforehand; solves/s of the call."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    probs = [W.mpc_socp(seed, i) for i in range(count)]
    HC.solve_batch(probs[:8], precision=precision)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = HC.solve_batch(probs, precision=precision)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    statuses = {}
    for r in res:
        statuses[r["status_name"]] = statuses.get(r["status_name"], 0) + 1
    return dict(workload=f"first {count} requests of the MPC stream (seed {seed}) in one hc_solve_batch call",
                precision=precision, requests=count, wall_s=wall, solves_per_s=count / wall,
                mean_iterations=sum(r["iterations"] for r in res) / count, statuses=statuses,
                note="includes the call's host set-up of the batch (plans, uploads)")


def run_sequential(count, seed=0):
    """The same MPC requests solved one after another by a plain FP64 solver
    (set-up, solve, results, release per request): the baseline the served
    form is compared with."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    probs = [W.mpc_socp(seed, i) for i in range(count)]
    s = HC.Solver(probs[0])   # warm-up (first-call costs)
    s.solve()
    s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solved = 0
    for p in probs:
        s = HC.Solver(p)
        info = s.solve()
        s.solution()
        s.close()
        solved += info["status_name"] == "solved"
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(requests=count, solves_per_s=count / wall, mean_latency_ms=1e3 * wall / count, solved=solved)


def run_parametric(count=50, T=100, nx=12, nu=6):
    """Parametric re-solves (hc_update_data) against fresh set-ups, on MPC
    problems of one structure (the largest request shape of the stream):
    re-solves per second both ways and the host time of a data update
    against that of a set-up."""
    import torch
    from paper_2412_19027_amd import hipcone as HC
    from paper_2412_19027_amd import workloads as W
    probs = [W.mpc_socp(seed, 0, T=T, nx=nx, nu=nu) for seed in range(count + 1)]
    s = HC.Solver(probs[0])
    s.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upd_ms, solved_u = 0.0, 0
    for p in probs[1:]:
        t1 = time.perf_counter()
        s.update_data(P_val=p.P.tocsr().data, q=p.q, A_val=p.A.tocsr().data, b=p.b)
        upd_ms += 1e3 * (time.perf_counter() - t1)
        solved_u += s.solve()["status_name"] == "solved"
        s.solution()
    torch.cuda.synchronize()
    wall_u = time.perf_counter() - t0
    s.close()
    t0 = time.perf_counter()
    setup_ms, solved_f = 0.0, 0
    for p in probs[1:]:
        f = HC.Solver(p)
        info = f.solve()
        f.solution()
        setup_ms += info["setup_ms"]
        solved_f += info["status_name"] == "solved"
        f.close()
    torch.cuda.synchronize()
    wall_f = time.perf_counter() - t0
    return dict(workload=f"MPC SOCP T={T}, nx={nx}, nu={nu} (n={probs[0].n}, m={probs[0].m}), {count} data sets",
                update_solves_per_s=count / wall_u, fresh_solves_per_s=count / wall_f,
                update_host_ms=upd_ms / count, setup_host_ms=setup_ms / count, solved_update=solved_u,
                solved_fresh=solved_f)


def _oracle_mpc(args):
    """One MPC request solved by the oracle (worker process of the served
    CPU baseline)."""
    seed, i = args
    from oracle import ipm
    from paper_2412_19027_amd import workloads as W
    r = ipm.solve(W.mpc_socp(seed, i))
    return r.status == ipm.SOLVED


def cpu_served_baseline(count=400, workers=16, rate=2000.0, seed=0):
    """The oracle on the served stream: a pool of single-threaded worker
    processes takes the first `count` MPC requests first come first served at
    their Poisson arrival times; solves/s and latency from arrival to result."""
    import concurrent.futures as cf
    import multiprocessing as mp
    from paper_2412_19027_amd import workloads as W
    arrivals = W.mpc_arrivals(seed, count, rate)
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
            list(pool.map(_oracle_mpc, [(seed, i) for i in range(workers)]))   # start-up and imports
            done_at = [0.0] * count
            futs = []
            t0 = time.perf_counter()
            for i in range(count):
                dt = arrivals[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                f = pool.submit(_oracle_mpc, (seed, i))
                f.add_done_callback(lambda f, i=i: done_at.__setitem__(i, time.perf_counter() - t0))
                futs.append(f)
            solved = sum(f.result() for f in futs)
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    lat = sorted(1e3 * (done_at[i] - arrivals[i]) for i in range(count))
    return dict(value=count / wall, unit="solves/s", cores=workers, kind="oracle",
                sample=f"the first {count} requests of the served MPC stream (seed {seed}, Poisson {rate:.0f}/s), "
                       f"{workers} single-threaded oracle processes, first come first served",
                p50_latency_ms=float(lat[count // 2]), p99_latency_ms=float(lat[min(count - 1, int(0.99 * count))]),
                solved=solved)


def cpu_baseline(prob):
    """The oracle as it stands, on one IPM iteration of the same problem
    (its setup and initial point are not timed)."""
    from oracle import ipm
    s = ipm.Solver(prob)
    t0 = time.perf_counter()
    s.iterate()
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=1.0 / dt, unit="IPM iterations/s", cores=cores, kind="oracle",
                sample="one IPM iteration of the same sparse-SOCP problem (oracle setup, equilibration and "
                       "initial point excluded); numpy/scipy FP64 with a LAPACK Cholesky of the 20,020 Schur "
                       f"complement; {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (tests only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--served", type=int, default=10000,
                    help="requests in the served-form measurement (MPC stream at 2000/s); 0 = skip")
    ap.add_argument("--no-seeds", action="store_true", help="skip the seeds 1-4 solves")
    ap.add_argument("--served-only", action="store_true",
                    help="run only the served-form measurement (FP64 and mixed) and print its JSON")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other full-size configurations")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run the reference copy kernel (for byte-counter scaling)")
    ap.add_argument("--sequential", type=int, default=200,
                    help="requests of the same stream solved one by one (plain FP64 baseline of the served form); "
                         "0 = skip")
    ap.add_argument("--batch-only", type=int, default=0,
                    help="solve the first N requests of the MPC stream in one batched call (FP64) and print its JSON")
    ap.add_argument("--workload-only", choices=OTHER_WORKLOADS,
                    help="run only this other configuration (one warm-up and one timed solve) and print its line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    sys.path.insert(0, ROOT)
    from paper_2412_19027_amd import workloads as W
    if args.workload_only:
        print(json.dumps(run_other_workloads(only=args.workload_only)))
        if args.calibrate_copy:
            calibrate_copy()
        return
    if args.batch_only > 0:
        print(json.dumps(run_batch(args.batch_only)))
        return
    if args.served_only:
        sv = run_served(args.served, "fp64")
        sv["mixed"] = run_served(args.served, "mixed")
        print(json.dumps(sv))
        return
    sc = args.scale
    prob = W.sparse_socp(0, nx=int(20000 * sc), n_zero=int(10000 * sc), n_nonneg=int(30000 * sc),
                         n_soc=int(40000 * sc))
    progress("start")
    main_run = run_gpu(prob, args.precision, args.steps, args.warmup)
    other = None
    if not args.no_mixed:
        alt = "mixed" if args.precision == "fp64" else "fp64"
        r = run_gpu(prob, alt, args.steps, args.warmup)
        other = {k: r[k] for k in ("status", "objective", "res_primal", "res_dual", "gap", "iterations_per_solve",
                                   "ms_per_solve", "ms_per_iteration", "factor_ms_per_iteration",
                                   "kkt_ms_per_iteration", "ir_solves_per_iteration", "fp64_fallbacks_per_solve")}
        other["precision"] = alt
        other["roofline"] = r["roofline"]
        other["cone_roofline"] = r["cone_roofline"]
        other["ms_per_solve_vs_main"] = r["ms_per_solve"] / main_run["ms_per_solve"]
        other["objective_rel_diff_vs_main"] = abs(r["objective"] - main_run["objective"]) / max(
            1.0, abs(main_run["objective"]))
    seeds = None
    if not args.no_seeds and sc == 1.0:
        per = run_seeds(args.precision)
        per["0"] = dict(status=main_run["status"], iterations=main_run["iterations_per_solve"],
                        ms_per_solve=main_run["ms_per_solve"], ms_per_iteration=main_run["ms_per_iteration"],
                        objective=main_run["objective"])
        seeds = dict(per_seed=per, ms_per_solve=spread([v["ms_per_solve"] for v in per.values()]),
                     ms_per_iteration=spread([v["ms_per_iteration"] for v in per.values()]),
                     iterations=spread([v["iterations"] for v in per.values()]))
    served = None
    if args.served > 0:
        served = run_served(args.served, "fp64")
        served["mixed"] = run_served(args.served, "mixed")
        served["per_slot_fp64_1000"] = run_served(min(1000, args.served), "fp64", budget=16 << 30, batched=False)
        if args.sequential > 0:
            progress(f"sequential FP64 solves of {args.sequential} requests")
            served["plain_fp64_sequential"] = run_sequential(args.sequential)
    if args.served > 0:
        progress("parametric re-solves")
    parametric = run_parametric() if args.served > 0 else None
    others = None if args.no_workloads else run_other_workloads()
    if args.calibrate_copy:
        calibrate_copy()
    if not args.no_cpu_baseline:
        progress("oracle: one IPM iteration on the host")
    cpu = None if args.no_cpu_baseline else cpu_baseline(prob)
    if cpu is not None and args.served > 0:
        progress("oracle pool on the served stream")
        cpu["served"] = cpu_served_baseline()
    out = {
        "metric": METRIC,
        "value": main_run["iters"] / main_run["wall"],
        "unit": "IPM iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-factor/f64",
        "data": "synthetic",
        "config": {"workload": workload_desc(prob), "precision": args.precision, "eps": 1e-8,
                   "step": "one full solve from the initial point"},
        "status": main_run["status"],
        "objective": main_run["objective"],
        "res_primal": main_run["res_primal"],
        "res_dual": main_run["res_dual"],
        "iterations_per_solve": main_run["iterations_per_solve"],
        "ms_per_iteration": main_run["ms_per_iteration"],
        "factor_ms_per_iteration": main_run["factor_ms_per_iteration"],
        "kkt_ms_per_iteration": main_run["kkt_ms_per_iteration"],
        "ir_solves_per_iteration": main_run["ir_solves_per_iteration"],
        "roofline": main_run["roofline"],
        "cone_roofline": main_run["cone_roofline"],
        "seeds": seeds,
        "alt_precision": other,
        "served": served,
        "parametric": parametric,
        "workloads": others,
        "cpu_baseline": cpu,
    }
    progress("done")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
