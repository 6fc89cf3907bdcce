#!/usr/bin/env python3
"""Benchmark: batched Faddeev-Merkuriev linear solves on one MI355X.

Workload (default): the energy scan of the H^- system, masses (1, 1, 1836),
charges (-1, -1, +1), L = 0, quintic Hermite splines 64 x 64 x 24 with x, y in
[0, 40] graded quadratically toward 0, 32 energies uniform in [-0.6, -0.1],
one seeded N(0, 1) right-hand side per energy.  All 32 solves share the
problem's device-resident factors and run as one batch.

One step = one fm_solve call on all 32 requests, each to a true FP64 relative
residual of 1e-10 (inputs already resident in HBM).  value = solves per second
of the FP64 path, timed with nothing but the solves in the timed region.

Also reported, each timed the same way: the batch with the preconditioner's
products in FP32 and BF16x3 MFMA (error against the FP64 GPU solution); the
other single-GPU workloads (the small cubic case beside the oracle's dense LU
timings, the quintic 127 x 127 x 32 request at three precisions, the L = 2
request with both preconditioner variants, a bounded sample of the serving
stream at a sustained arrival rate).  Kernel shares, the roofline of the class
with the largest share and the MFMA fraction of the x-y products come from a
second pass of the same steps with the library's per-launch HIP events on the
solve's stream (algorithmic bytes/flops from the problem sizes and step
counts).  The CPU oracle is timed on this host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6         # MI355X FP64 vector and matrix

ROOT = os.path.dirname(os.path.abspath(__file__))

WORKLOAD_TEXT = {
    "hminus_scan": "H- energy scan, L=0, quintic 64x64x24, x,y in [0,40] quadratic, 32 energies in [-0.6,-0.1], "
                   "seeded N(0,1) RHS",
    "ps_q127": "Ps- like (1,1,1)/(+1,-1,-1), L=0, quintic x,y 127 on [0,20] x cubic z 32, E=-0.25, seeded RHS",
    "ps_l2_q97": "Ps- like, L=2 tau=+1 (3 M' blocks), quintic x,y 97 on [0,20] x cubic z 32, E=-0.2, seeded RHS",
}
sys.path.insert(0, ROOT)


def cpu_baseline(seconds_cap=30.0):
    """The oracle (explicit assembly + LU) on this host's cores, on a bounded
    sample: the same H^- energy scan on a reduced quintic grid 22 x 22 x 9
    (N = 13068), energies taken from the scan until the time cap."""
    import numpy as np
    from oracle.assemble import Problem as OracleProblem
    from oracle.solve import lu_solve
    from paper_2005_05398_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    c = W.hminus_scan()
    d = W.make_desc(*W.H_MINUS, 22, 9, deg_xy=5, deg_z=5, R=40.0, xy_map="quadratic")
    O = OracleProblem(d)
    n_done = 0
    t0 = time.perf_counter()
    for E, seed in zip(c["E"], c["seeds"]):
        b = W.rhs(seed, O.N)
        A = O.assemble(E)
        x = lu_solve(A, b)
        assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
        n_done += 1
        if time.perf_counter() - t0 > seconds_cap:
            break
    dt = time.perf_counter() - t0
    # the oracle at the scan's full size: its row assembly, timed on chunks of
    # rows for about 10 s and extrapolated to one whole matrix (an LU of it,
    # N = 294,912 with ~620 nonzeros per row, does not fit a host's memory)
    Of = OracleProblem(c["desc"])
    nrows, nnz = 0, 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < 10.0 and nrows < Of.N:
        rows = np.arange(nrows, min(Of.N, nrows + 4096))
        nnz += Of.rows(c["E"][0], rows).nnz
        nrows += rows.size
    rate = nrows / (time.perf_counter() - t1)
    return {"value": n_done / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle assembly + dense LU of the same H^- scan on a reduced quintic 22x22x9 grid "
                      f"(N={O.N}), {n_done} of the 32 energies, {dt:.1f} s",
            "full_size_assembly": {"N": Of.N, "rows_timed": nrows, "rows_per_s": rate,
                                   "nonzeros_per_row": nnz / max(1, nrows),
                                   "seconds_per_matrix_extrapolated": Of.N / rate}}


def eigs_bench(args):
    """Helium 2 1P and 3 1P (with 2 3P and 3 3P, which the unsymmetrised
    system also holds) by shift-invert Arnoldi on the grids of Table 1 (Sec. 4, the comparison with Pardiso)."""
    import torch
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    torch.zeros(1, device="cuda:0")          # torch's device context before the library's
    stream = torch.cuda.current_stream()
    rows = []
    t_all = time.perf_counter()
    for g1, g3, printed in W.HE_TABLE1:
        desc = dict(W.helium_desc(g1, g3), precond="coupled")
        t0 = time.perf_counter()
        P = fm.Problem(desc)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        st, E, res, info = P.eigs(-2.095, nev=4, ncv=24, tol=1e-10, max_restarts=40, restart=100, rtol=1e-11,
                                  max_iters=4000, raise_on_error=False, stream=stream)
        t_eig = time.perf_counter() - t0
        Es = sorted(e.real for e in E)
        singlet = [min(Es, key=lambda e: abs(e - b)) for b in W.HE_1P_BENCHMARK]
        rows.append({"grid": {"1": g1, "3": g3}, "N": P.N, "status": fm.STATUS_NAMES.get(st), "energies": Es,
                     "E_2_1P": singlet[0], "E_3_1P": singlet[1], "paper_printed": printed,
                     "diff_vs_printed": [s - q for s, q in zip(singlet, printed)],
                     "diff_vs_benchmark": [s - b for s, b in zip(singlet, W.HE_1P_BENCHMARK)],
                     "setup_s": t_setup, "eigs_s": t_eig, "info": info,
                     "max_ritz_residual": max(res)})
        print(f"eigs: grid {g1}/{g3} N={P.N}: {['%.8f' % e for e in Es]} in {t_eig:.2f} s "
              f"({info['solves']} solves)", file=sys.stderr, flush=True)
        del P
    line = {"metric": "helium 1P energies by shift-invert Arnoldi (grids of the paper's Table 1, Sec. 4)",
            "value": sum(r["eigs_s"] for r in rows), "unit": "s (all five grids)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "He (nucleus 1e15 a.u.), J=1, tau=+1, quintic, map-pow x/y, sin z, "
                                   "domains (1: 36, 36; 3: 9, 6), x0=1, nu=2.01, sigma=-2.095, nev=4, ncv=24, "
                                   "inner FGMRES(100) to 1e-11, coupled preconditioner",
                       "benchmark_1P": W.HE_1P_BENCHMARK},
            "rows": rows, "wall_s": time.perf_counter() - t_all}
    print(json.dumps(line))


def calibration_copy():
    """One plain device copy of COPY_BYTES and one pure read of the same bytes,
    the reference dispatches for scaling the HBM counters of a counter run."""
    import torch
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    total = float(src.sum())
    torch.cuda.synchronize()
    assert total == float(src.numel())
    del src, dst


PAPER_TABLE3_IRAM_MIN = (6.3, 33.0, 60.0, 280.0)     # the paper's IRAM wall time per basis set, minutes


def j10_runs(runs, stream, echo=True):
    """fm_eigs on helium J = 10 for each (basis 1, basis 3, printed energies,
    preconditioner, exchange) of runs; one result row each."""
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    rows = []
    for g1, g3, printed, pc, ex in runs:
        desc = dict(W.helium_desc(g1, g3, dom1=W.HE_TABLE3_DOMAINS[0], dom3=W.HE_TABLE3_DOMAINS[1], J=10, tau=1),
                    precond=pc, exchange=ex)
        t0 = time.perf_counter()
        P = fm.Problem(desc)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        st, E, res, info = P.eigs(-2.0045, nev=6, ncv=24, tol=1e-9, max_restarts=40, restart=200, rtol=1e-10,
                                  max_iters=4000, raise_on_error=False, stream=stream)
        t_eig = time.perf_counter() - t0
        Es = sorted(e.real for e in E)
        got = [min(Es, key=lambda e: abs(e - q)) for q in printed]
        rows.append({"grid": {"1": g1, "3": g3}, "precond": pc, "exchange": ex, "N": P.N,
                     "N_exchange_reduced": 11 * (g1[0] * g1[1] * g1[2] + g3[0] * g3[1] * g3[2]),
                     "status": fm.STATUS_NAMES.get(st), "energies": Es, "E_ground": got[0], "E_first_excited": got[1],
                     "paper_printed": printed, "diff_vs_printed": [a - b for a, b in zip(got, printed)],
                     "setup_s": t_setup, "eigs_s": t_eig, "info": info, "max_ritz_residual": max(res)})
        if echo:
            print(f"eigs-j10: grid {g1}/{g3} {pc} exchange {ex} N={P.N}: {['%.6f' % e for e in Es]} in {t_eig:.1f} s "
                  f"({info['solves']} solves, {info['inner_iters']} inner steps)", file=sys.stderr, flush=True)
        P.close()
    return rows


def j10_table3_entry():
    """The default bench's sub-object: the four basis sets of the paper's
    Table 3 (p = +1, coupled preconditioner), each energy pair against the
    printed one and the eigs time beside the paper's IRAM wall time."""
    import torch
    from paper_2005_05398_amd import workloads as W
    rows = j10_runs([(g1, g3, pr, "coupled", 1) for g1, g3, pr in W.HE_TABLE3_J10], torch.cuda.current_stream(),
                    echo=False)
    out = {"config": "helium J=10 tau=+1 p=+1 (the paper's Table 3 systems, Sec. 4), shift-invert Arnoldi at "
                     "sigma=-2.0045, nev=6, ncv=24, coupled preconditioner, inner FGMRES(200) to 1e-10",
           "rows": [{"basis": f"{r['grid']['1']}/{r['grid']['3']}", "N": r["N"], "status": r["status"],
                     "E": [r["E_ground"], r["E_first_excited"]], "printed": list(r["paper_printed"]),
                     "max_abs_diff": max(abs(d) for d in r["diff_vs_printed"]), "eigs_s": r["eigs_s"],
                     "paper_iram_min": PAPER_TABLE3_IRAM_MIN[i], "inner_steps": r["info"]["inner_iters"]}
                    for i, r in enumerate(rows)],
           "eigs_s_total": sum(r["eigs_s"] for r in rows)}
    print(f"bench: helium J=10 Table 3: {out['eigs_s_total']:.2f} s for the four basis sets", file=sys.stderr,
          flush=True)
    return out


def eigs_j10_bench(args):
    """Helium at J = 10 (tau = +1, eleven M' blocks) by shift-invert Arnoldi on
    the basis sets of the paper's Table 3 (Sec. 4, the high-J runs; domains
    (1: 280, 280; 3: 2, 2)), electron-exchange parity p = +1 (the paper's
    printed system sizes), coupled preconditioner; the same with the
    block-Jacobi one, and the first basis set unreduced (each level then
    appears for both parities)."""
    import torch
    from paper_2005_05398_amd import workloads as W
    torch.zeros(1, device="cuda:0")
    t_all = time.perf_counter()
    # the paper's systems: electron-exchange parity p = +1 (its printed sizes),
    # coupled preconditioner; then the block-Jacobi one, and the first basis
    # set unreduced (both parities)
    runs = [(g1, g3, printed, "coupled", 1) for g1, g3, printed in W.HE_TABLE3_J10]
    runs += [(g1, g3, printed, "block_jacobi", 1) for g1, g3, printed in W.HE_TABLE3_J10]
    runs += [(*W.HE_TABLE3_J10[0], "coupled", 0)]
    if args.j10_runs:
        runs = [runs[int(i)] for i in args.j10_runs.split(",")]
    rows = j10_runs(runs, torch.cuda.current_stream())
    line = {"metric": "helium J=10 energies by shift-invert Arnoldi (basis sets of the paper's Table 3, Sec. 4)",
            "value": sum(r["eigs_s"] for r in rows if r["precond"] == "coupled" and r["exchange"] == 1),
            "unit": "s (the basis sets run, coupled preconditioner, p = +1)", "n_gpus": 1,
            "higher_is_better": False,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "He (nucleus 1e15 a.u.), J=10, tau=+1, eleven M' blocks, quintic, map-pow x/y, "
                                   "sin z, domains (1: 280, 280; 3: 2, 2), x0=1, nu=2.01, sigma=-2.0045, nev=6, "
                                   "ncv=24, Ritz tol 1e-9, inner FGMRES(200) to 1e-10, electron-exchange "
                                   "parity p=+1 (an unreduced run: both parities)"},
            "rows": rows, "wall_s": time.perf_counter() - t_all}
    print(json.dumps(line))


def eigs_3d_bench(args):
    """Helium 3 1D (J = 2, tau = +1) by shift-invert Arnoldi with the set-up of
    the paper's Fig. 4 (domains (1: 45, 45; 3: 11, 6) a.u.), on basis sets
    growing to its final one (1: 238, 238, 24; 3: 52, 40, 27); the caption's
    benchmark value is quoted."""
    import torch
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    bench_3d = -2.05562073285224648939
    torch.zeros(1, device="cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    # the last row is the paper's own system: the final basis with the electron
    # symmetry (p = +1), N = 4,246,848, the largest it reports
    for g1, g3, ex in (((100, 100, 12), (40, 31, 18), 0), ((160, 160, 18), (46, 37, 24), 0),
                       ((238, 238, 24), (52, 40, 27), 0), ((238, 238, 24), (52, 40, 27), 1)):
        t0 = time.perf_counter()
        P = fm.Problem(dict(W.helium_desc(g1, g3, dom1=(45.0, 45.0), dom3=(11.0, 6.0), J=2, tau=1),
                            precond="coupled", exchange=ex))
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        st, E, res, info = P.eigs(-2.06, nev=4 if ex == 0 else 2, ncv=24, tol=1e-11, max_restarts=40, restart=150,
                                  rtol=1e-10, max_iters=4000, raise_on_error=False, stream=stream)
        t_eig = time.perf_counter() - t0
        Es = sorted(e.real for e in E)
        e3d = min(Es, key=lambda e: abs(e - bench_3d))
        rows.append({"grid": {"1": g1, "3": g3}, "exchange": ex, "N": P.N, "status": fm.STATUS_NAMES.get(st),
                     "energies": Es, "E_3_1D": e3d, "rel_err_vs_benchmark": (e3d - bench_3d) / abs(bench_3d),
                     "setup_s": t_setup, "eigs_s": t_eig, "info": info, "max_ritz_residual": max(res)})
        print(f"eigs-3d: grid {g1}/{g3} exchange {ex} N={P.N}: 3 1D {e3d:.10f} "
              f"(rel. err {rows[-1]['rel_err_vs_benchmark']:+.2e}) "
              f"in {t_eig:.1f} s", file=sys.stderr, flush=True)
        del P
        torch.cuda.empty_cache()
    line = {"metric": "helium 3 1D energy by shift-invert Arnoldi (the paper's Fig. 4 set-up)",
            "value": rows[-1]["rel_err_vs_benchmark"], "unit": "relative error vs benchmark", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "He (nucleus 1e15 a.u.), J=2, tau=+1, quintic, map-pow x/y, sin z, domains "
                                   "(1: 45, 45; 3: 11, 6) a.u. (unscaled Jacobi lengths), x0=1, nu=2.01, sigma=-2.06, "
                                   "nev=4 (2 with the exchange symmetry), ncv=24, inner FGMRES(150) to 1e-10 (at most 4000 steps), "
                                   "coupled preconditioner",
                       "benchmark_3_1D": bench_3d},
            "rows": rows}
    print(json.dumps(line))


def serve_phase(srv, reqs, rhs, indices, arrivals, label, args):
    """Submit requests `indices` at the given arrival times (s from the start)
    and wait for all of them.  Returns (results by tag, wall time, samples of
    the number of requests outstanding (submitted, not finished) over time)."""
    import numpy as np
    done = {}
    xs = {}
    qlen = []
    t0 = time.perf_counter()
    t_report = t0
    t_sample = t0
    k = 0
    while len(done) < len(indices):
        now = time.perf_counter() - t0
        while k < len(indices) and arrivals[k] <= now:
            i = indices[k]
            r = reqs[i]
            xs[i] = np.zeros(rhs[i].size)
            srv.submit(r["desc"], r["E"], rhs[i], xs[i], i, restart=args.serve_restart, rtol=1e-10,
                       max_iters=args.serve_max_iters, prec=args.serve_prec)
            k += 1
        block = k >= len(indices)
        for o in srv.poll(block=block):
            done[o["tag"]] = o
        t = time.perf_counter()
        if t - t_sample > 0.25:
            t_sample = t
            qlen.append((t - t0, k - len(done)))
        if t - t_report > 20:
            t_report = t
            print(f"serve {label}: {len(done)}/{len(indices)} done, {k} submitted, {t - t0:.0f} s", file=sys.stderr,
                  flush=True)
        if not block:
            time.sleep(0.001)
    return done, time.perf_counter() - t0, qlen


def serve_summary(done, wall, qlen):
    """Latency percentiles, status counts and the queue-length trend of one phase."""
    import numpy as np
    lat = np.array([o["t_done"] - o["t_submit"] for o in done.values()])
    wait = np.array([o["t_start"] - o["t_submit"] for o in done.values() if o["t_start"] > 0])
    status = {}
    for o in done.values():
        status[o["status"]] = status.get(o["status"], 0) + 1
    ok = [o for o in done.values() if o["status"] == "FM_OK"]
    q = np.array([n for _, n in qlen]) if qlen else np.zeros(1)
    h = max(1, q.size // 2)
    return {
        "solves_per_s": len(ok) / wall, "wall_s": wall,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean()), "max": float(lat.max())},
        "queue_wait_s": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))}
        if wait.size else None,
        # requests outstanding (submitted, not yet finished), sampled every 0.25 s: a sustained
        # rate keeps it flat (second-half mean close to the first-half mean)
        "outstanding": {"mean_first_half": float(q[:h].mean()), "mean_second_half": float(q[h:].mean())
                        if q.size > h else float(q.mean()), "max": int(q.max())},
        "status_counts": status,
        "not_converged_tags": sorted(o["tag"] for o in done.values() if o["status"] == "FM_E_NOT_CONVERGED"),
        "iters_mean": float(np.mean([o["iters"] for o in ok])) if ok else None,
        "max_rel_residual_ok": max(o["rel_residual"] for o in ok) if ok else None,
    }


def serve_run(args, nreq, rates):
    """The seeded request stream against one server: a saturation phase (the
    requests submitted all at once, cold: every problem is built as its first
    request arrives) measures the saturated rate; then one Poisson phase per
    entry of `rates` (a fraction of the saturated rate) on the same requests,
    with the problems already built, as a running service has them."""
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    import numpy as np

    reqs = [W.serving_request(i) for i in range(nreq)]
    for r in reqs:                      # the preconditioner variant of the L > 0 requests
        if r["desc"]["J"] > 0:
            r["desc"] = dict(r["desc"], precond=args.serve_precond)
    rhs = [W.rhs(r["seed"], W.n_unknowns(r["desc"])) for r in reqs]
    srv = fm.Server(hbm_budget_bytes=int(args.budget_gb * (1 << 30)), max_batch=args.max_batch)
    idx = list(range(nreq))
    sat, sat_wall, _ = serve_phase(srv, reqs, rhs, idx, np.zeros(nreq), "saturation", args)
    sat_rate = nreq / sat_wall
    print(f"serve saturation: {nreq} requests in {sat_wall:.1f} s ({sat_rate:.2f} solves/s)", file=sys.stderr,
          flush=True)
    phases = {}
    for frac in rates:
        rate = frac * sat_rate
        done, wall, qlen = serve_phase(srv, reqs, rhs, idx, W.serving_arrivals(nreq, rate), f"poisson{frac}", args)
        phases[f"{frac:g}x_saturated"] = dict(serve_summary(done, wall, qlen), arrival_rate_per_s=rate)
    stats = srv.stats()
    srv.close()
    return {
        "config": {"workload": "seeded stream: quintic x,y nominal {32,64,96,128} taken as {31,64,97,127} "
                               "(3K+1 sizes), cubic z {8,16,32}, L in {0,1,2} (tau=+1), E in [-0.6,-0.05], "
                               "masses (1,1,1) or (1,1,1836), seeded N(0,1) RHS",
                   "requests": nreq, "max_batch": args.max_batch, "restart": args.serve_restart,
                   "max_iters": args.serve_max_iters, "budget_gb": args.budget_gb,
                   "precond_L_gt_0": args.serve_precond, "products": args.serve_prec},
        "saturation": {"requests": nreq, "solves_per_s": sat_rate, "wall_s": sat_wall,
                       "ok": sum(1 for o in sat.values() if o["status"] == "FM_OK"),
                       "not_converged_tags": sorted(o["tag"] for o in sat.values()
                                                    if o["status"] == "FM_E_NOT_CONVERGED")},
        "poisson": phases,
        "server_end": stats,
    }


def serve_bench(args):
    """Serving: the whole seeded stream; Poisson arrivals at a rate the server
    sustains, at 0.8 x and at 1.0 x the saturated rate, each reported on its
    own."""
    out = serve_run(args, args.requests, (args.serve_rate, 0.8, 1.0))
    sus = out["poisson"][f"{args.serve_rate:g}x_saturated"]
    line = {
        "metric": "serving: solves/s at rel. residual 1e-10 and p50/p99 latency (Poisson arrivals)",
        "value": sus["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64" if args.serve_prec == "fp64" else f"f64+{args.serve_prec}", "data": "synthetic",
        **out,
    }
    print(json.dumps(line))


COPY_BYTES = 512 << 20
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic.json")
KERNEL_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2005_05398_amd", "csrc",
                             "kernels.hip")


def traffic_variant(args):
    """The configuration a counter record belongs to: the workload, plus every
    option that changes what the timed kernels do (the committed records are
    for the defaults, whose name is the workload's alone)."""
    v = args.workload
    if args.exchange:
        v += f"-exchange{args.exchange:+d}"
    if args.precond != "block_jacobi":
        v += f"-{args.precond}"
    if args.prec != "fp64":
        v += f"-{args.prec}"
    if args.restart != (300 if args.workload == "hminus_scan" else 60):
        v += f"-restart{args.restart}"
    return v


def measured_traffic(workload, kclass):
    """HBM bytes per launch of the dominant kernel class from the committed
    counter runs (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy factor),
    or None when there is none for this configuration (`traffic_variant`) and
    class or the kernel source changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    e = rec.get("entries", {}).get(f"{workload}:{kclass}")
    if not e or e.get("kernels_hip_sha256") != sha:
        return None
    return e["hbm_bytes_per_launch"]


FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 (vector and dense matrix)
BF16_PEAK_TFLOPS = 2500.0       # MI355X dense BF16 matrix
MFMA_PEAK = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_PEAK_TFLOPS,
             # BF16x3: three BF16 products per product of the definition
             "bf16x3": BF16_PEAK_TFLOPS / 3.0}


def kernel_table(prof):
    """Per kernel class: summed HIP-event time, launches, average launch and
    algorithmic GB/s and TFLOP/s."""
    kernels = {}
    for k, v in prof.items():
        if v["launches"] == 0:
            continue
        s = v["ms"] * 1e-3
        kernels[k] = {"ms": round(v["ms"], 3), "launches": v["launches"],
                      "avg_launch_ms": v["ms"] / v["launches"],
                      "GB/s": v["bytes"] / s / 1e9 if s > 0 else None,
                      "TFLOP/s": v["flops"] / s / 1e12 if s > 0 else None}
    return kernels


def roofline_of(kernels, prec, traffic_key=None):
    """Roofline of the kernel class with the largest time share: the x-y
    products against the MFMA peak of their arithmetic, the operator classes
    against the FP64 peak (ALU-bound), everything else against HBM."""
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    d = kernels[dom]
    if dom == "xy":
        roof = {"bound": "mfma", "achieved": d["TFLOP/s"], "peak": MFMA_PEAK[prec], "unit": "TFLOP/s"}
    elif dom in ("matvec", "coupling"):
        roof = {"bound": "alu", "achieved": d["TFLOP/s"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": d["GB/s"], "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update({"kernel": dom, "avg_launch_ms": d["avg_launch_ms"], "launches": d["launches"],
                 "traffic": measured_traffic(traffic_key, dom) if traffic_key else None})
    return roof


def measure(P, Es, B, X, restart, prec, steps, warmup, stream, profile=True, traffic_key=None, graphs=True):
    """Solves/s of `steps` fm_solve calls on the whole batch with nothing but
    the solves in the timed region; then (profile=True) the same number of
    calls again with the library's per-launch HIP events on the solve's
    stream, for the kernel shares and the roofline."""
    import numpy as np
    import torch
    from paper_2005_05398_amd import fm

    def step():
        st, res = P.solve(Es, B, X, restart=restart, rtol=1e-10, max_iters=20000, prec=prec, stream=stream,
                          graphs=graphs)
        if st != fm.FM_OK:
            raise RuntimeError(f"solve failed: {fm.STATUS_NAMES.get(st)} {res}")
        return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nreq = len(Es)
    iters = [r["iters"] for r in res]
    out = {"solves_per_s": nreq * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps, "graphs": bool(graphs),
           "iters": {"min": min(iters), "mean": float(np.mean(iters)), "max": max(iters)},
           "max_rel_residual": max(r["rel_residual"] for r in res)}
    if profile:
        P.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el_p = time.perf_counter() - t0
        prof = P.profile_read()
        P.profile(False)
        kernels = kernel_table(prof)
        total = sum(v["ms"] for v in prof.values())
        out["profiled_ms_per_step"] = 1e3 * el_p / steps
        out["kernel_ms_share"] = {k: round(v["ms"] / total, 4) for k, v in prof.items() if v["launches"]}
        out["kernels"] = kernels
        out["roofline"] = roofline_of(kernels, prec, traffic_key)
        if "xy" in kernels:
            out["mfma"] = {"kernel": "xy", "achieved_TFLOP/s": kernels["xy"]["TFLOP/s"],
                           "peak_TFLOP/s": MFMA_PEAK[prec],
                           "frac": kernels["xy"]["TFLOP/s"] / MFMA_PEAK[prec]}
    return out


def workload_entry(name, args, precs, precond="block_jacobi", restart=None, profile=True, traffic=False,
                   compare_eager=False):
    """One workload at several precisions of the preconditioner products; the
    error of each solution against the FP64 GPU solution of the same batch."""
    import torch
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    c = W.WORKLOADS[name]()
    restart = restart or (300 if name == "hminus_scan" else 30 if name == "ps_cubic16" else 60)
    t0 = time.perf_counter()
    P = fm.Problem(dict(c["desc"], precond=precond))
    setup_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    B = torch.as_tensor(W.rhs_batch(c["seeds"], P.N), device=dev)
    X = torch.zeros_like(B)
    stream = torch.cuda.current_stream()
    out = {"N_per_request": P.N, "requests_per_step": len(c["E"]), "restart": restart, "precond": precond,
           "setup_s": setup_s}
    X64 = None
    for prec in precs:
        key = None
        if traffic:
            key = traffic_variant(argparse.Namespace(workload=name, exchange=0, precond=precond, prec=prec,
                                                     restart=restart))
        e = measure(P, c["E"], B, X, restart, prec, args.steps, args.warmup, stream, profile=profile,
                    traffic_key=key, graphs=bool(args.graphs))
        if compare_eager:
            # the same solves launched one kernel at a time (no captured graphs)
            ee = measure(P, c["E"], B, X, restart, prec, args.steps, args.warmup, stream, profile=False,
                         graphs=False)
            e["eager_solves_per_s"] = ee["solves_per_s"]
            e["eager_ms_per_step"] = ee["ms_per_step"]
        if prec == "fp64":
            X64 = X.clone()
        elif X64 is not None:
            e["max_rel_error_vs_fp64_gpu"] = (torch.linalg.norm(X - X64, dim=1) /
                                              torch.linalg.norm(X64, dim=1)).max().item()
        out[prec] = e
        print(f"bench: {name} {precond} {prec}: {e['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    P.close()
    return out


def complex_entry(args):
    """The energy scan at complex energies E_k + 0.01 i with complex seeded
    right-hand sides (two real rows per request), FP64, timed like the others."""
    import numpy as np
    import torch
    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W
    c = W.hminus_scan()
    P = fm.Problem(c["desc"])
    Es = [complex(e, 0.01) for e in c["E"]]
    B = torch.as_tensor(np.stack([np.concatenate([W.rhs(s, P.N), W.rhs(s + 500, P.N)]) for s in c["seeds"]]),
                        device=torch.device("cuda:0"))
    X = torch.zeros_like(B)
    stream = torch.cuda.current_stream()

    def step():
        st, res = P.solve_complex(Es, B, X, restart=300, rtol=1e-10, max_iters=20000, stream=stream,
                                  graphs=bool(args.graphs))
        if st != fm.FM_OK:
            raise RuntimeError(f"complex solve failed: {fm.STATUS_NAMES.get(st)} {res}")
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = [r["iters"] for r in res]
    P.close()
    out = {"config": "H- scan, 32 energies E_k + 0.01 i, complex seeded RHS (re: seed 2001+k, im: 2501+k), FP64, "
                     "restart 300",
           "solves_per_s": len(Es) * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
           "iters": {"min": min(iters), "mean": float(np.mean(iters)), "max": max(iters)},
           "max_rel_residual": max(r["rel_residual"] for r in res)}
    print(f"bench: hminus_scan complex: {out['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    return out


def oracle_lu_timing():
    """The oracle on the small workload (cubic 16 x 16 x 8, N = 6144): assembly,
    dense LU factorisation and the solve, timed separately on this host."""
    import numpy as np
    from oracle.assemble import Problem as OracleProblem
    from oracle.solve import rel_residual
    import scipy.linalg as sla
    from paper_2005_05398_amd import workloads as W
    c = W.ps_cubic16()
    t0 = time.perf_counter()
    O = OracleProblem(c["desc"])
    A = O.assemble(c["E"][0])
    t1 = time.perf_counter()
    lu = sla.lu_factor(A.toarray())
    t2 = time.perf_counter()
    b = W.rhs(c["seeds"][0], O.N)
    x = sla.lu_solve(lu, b)
    t3 = time.perf_counter()
    return {"N": O.N, "assembly_s": t1 - t0, "lu_factor_s": t2 - t1, "lu_solve_s": t3 - t2,
            "rel_residual": rel_residual(A, x, b), "threads": blas_threads()}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--restart", type=int, default=None, help="default: 300 (hminus_scan), 60 (ps_q127, ps_l2_q97)")
    ap.add_argument("--workload", default="hminus_scan", choices=["hminus_scan", "ps_q127", "ps_l2_q97"])
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--exchange", type=int, default=0, choices=[-1, 0, 1],
                    help="solve only the part of parity p under exchange of particles 1 and 2 (H- scan: the "
                         "two electrons); 0: the full three-component system")
    ap.add_argument("--precond", default="block_jacobi", choices=["block_jacobi", "coupled"],
                    help="preconditioner variant (coupled: the approximate matrix with its M'+-1 blocks, L > 0)")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="1: Arnoldi steps replayed from captured HIP graphs; 0: one launch at a time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the reduced-precision comparison runs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-GPU workloads (small cubic, ps_q127, ps_l2_q97, serving sample)")
    ap.add_argument("--serve", action="store_true", help="run the serving benchmark instead")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--serve-sample", type=int, default=96,
                    help="requests of the serving sample in the default run (0: none)")
    ap.add_argument("--serve-rate", type=float, default=0.5,
                    help="Poisson arrival rate as a fraction of the saturated rate (the sustained phase)")
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--serve-restart", type=int, default=200)
    ap.add_argument("--serve-max-iters", type=int, default=6000)
    ap.add_argument("--serve-prec", default="fp32", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the preconditioner products in the serving stream")
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-precond", default="coupled", choices=["block_jacobi", "coupled"],
                    help="preconditioner of the L > 0 requests in the serving stream")
    ap.add_argument("--eigs", action="store_true",
                    help="helium 1P levels by shift-invert Arnoldi on the grids of the paper's Table 1 (Sec. 4)")
    ap.add_argument("--eigs-3d", action="store_true",
                    help="helium 3 1D level (L=2) on growing basis sets up to the paper's Fig. 4 one (N ~ 8.3M)")
    ap.add_argument("--eigs-j10", action="store_true",
                    help="helium J = 10 levels on the basis sets of the paper's Table 3 (Sec. 4)")
    ap.add_argument("--j10-runs", default="",
                    help="with --eigs-j10: comma list of runs (0-3: the four basis sets, coupled, p = +1; "
                         "4-7: the same with block-Jacobi; 8: the first unreduced); default all")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 512 MiB device copy first (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on exactly one GPU (there is no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.calibrate_copy:
        calibration_copy()
    if args.eigs:
        eigs_bench(args)
        return
    if args.eigs_3d:
        eigs_3d_bench(args)
        return
    if args.eigs_j10:
        eigs_j10_bench(args)
        return

    import numpy as np
    import torch

    from paper_2005_05398_amd import fm
    from paper_2005_05398_amd import workloads as W

    dev = torch.device("cuda:0")
    c = W.WORKLOADS[args.workload]()
    desc, Es, seeds = c["desc"], c["E"], c["seeds"]
    if args.restart is None:
        args.restart = 300 if args.workload == "hminus_scan" else 60
    t_setup = time.perf_counter()
    if args.exchange:
        desc = dict(desc, exchange=args.exchange)
    P = fm.Problem(dict(desc, precond=args.precond))
    t_setup = time.perf_counter() - t_setup
    nreq = len(Es)
    B = torch.as_tensor(W.rhs_batch(seeds, P.N), device=dev)
    X = torch.zeros_like(B)
    stream = torch.cuda.current_stream()

    head = measure(P, Es, B, X, args.restart, args.prec, args.steps, args.warmup, stream,
                   traffic_key=traffic_variant(args), graphs=bool(args.graphs))
    if args.graphs:
        ee = measure(P, Es, B, X, args.restart, args.prec, args.steps, args.warmup, stream, profile=False,
                     graphs=False)
        head["eager_solves_per_s"] = ee["solves_per_s"]
    print(f"bench: {args.workload} {args.prec}: {head['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
    line = {
        "metric": ("solves/s to rel. residual 1e-10 (FP64, batched energy scan)" if args.workload == "hminus_scan"
                   else f"solves/s to rel. residual 1e-10 ({args.workload})"),
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else f"f64+{args.prec}",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "N_per_request": P.N, "requests_per_step": nreq, "restart": args.restart,
                   "precond": args.precond, "precond_products": args.prec, "rtol": 1e-10,
                   "exchange": args.exchange, "graphs": bool(args.graphs)},
        "eager_solves_per_s": head.get("eager_solves_per_s"),
        "iters": head["iters"],
        "max_rel_residual": head["max_rel_residual"],
        "setup_s": t_setup,
        "profiled_ms_per_step": head.get("profiled_ms_per_step"),
        "kernel_ms_share": head.get("kernel_ms_share"),
        "kernels": head.get("kernels"),
        "roofline": head.get("roofline"),
        "mfma": head.get("mfma"),
    }
    if not args.no_mixed:
        # the same batch with the preconditioner's products in FP32 / BF16x3 MFMA (FP64 Arnoldi,
        # residual and divide), timed exactly as the FP64 run; error against the FP64 GPU solution
        X64 = X.clone()
        mixed = {}
        for prec in ("fp32", "bf16x3"):
            if prec == args.prec:
                continue
            key = traffic_variant(argparse.Namespace(**dict(vars(args), prec=prec)))
            e = measure(P, Es, B, X, args.restart, prec, args.steps, args.warmup, stream, traffic_key=key,
                        graphs=bool(args.graphs))
            e["max_rel_error_vs_fp64_gpu"] = (torch.linalg.norm(X - X64, dim=1) /
                                              torch.linalg.norm(X64, dim=1)).max().item()
            e["speedup_vs_fp64"] = e["solves_per_s"] / head["solves_per_s"]
            mixed[prec] = e
            print(f"bench: {args.workload} {prec}: {e['solves_per_s']:.2f} solves/s", file=sys.stderr, flush=True)
        line["mixed_precision"] = mixed
    P.close()
    del B, X
    if not args.no_configs and args.workload == "hminus_scan":
        torch.cuda.empty_cache()
        cfgs = {}
        small = workload_entry("ps_cubic16", args, ("fp64",), restart=30, compare_eager=True)
        small["config"] = "cubic 16x16x8 on [0,20]^2, Ps- like (1,1,1)/(+1,-1,-1), L=0, E=-0.25, GMRES(30), N=6144"
        if not args.no_cpu_baseline:
            small["oracle_dense_lu"] = oracle_lu_timing()
        cfgs["ps_cubic16"] = small
        q = workload_entry("ps_q127", args, ("fp64", "fp32", "bf16x3"), traffic=True)
        q["config"] = ("quintic x,y 127 (the nominal 128 taken as 3K+1 = 127) x cubic z 32 on [0,20]^2, "
                       "Ps- like, L=0, E=-0.25, FGMRES(60)")
        cfgs["ps_q127"] = q
        l2 = {"config": "L=2 tau=+1 (3 M' blocks), quintic x,y 97 (the nominal 96 taken as 3K+1 = 97) x cubic z 32 "
                        "on [0,20]^2, Ps- like, E=-0.2, FGMRES(60); FP32 products (FP64 for reference)"}
        for pc in ("block_jacobi", "coupled"):
            l2[pc] = workload_entry("ps_l2_q97", args, ("fp64", "fp32"), precond=pc, traffic=True)
        cfgs["ps_l2_q97"] = l2
        cfgs["hminus_scan_complex"] = complex_entry(args)
        torch.cuda.empty_cache()
        cfgs["helium_j10_table3"] = j10_table3_entry()
        torch.cuda.empty_cache()
        if args.serve_sample > 0:
            sv = serve_run(args, args.serve_sample, (args.serve_rate,))
            cfgs["serving_sample"] = sv
        line["configs"] = cfgs
    if not args.no_cpu_baseline and args.workload == "hminus_scan":
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
