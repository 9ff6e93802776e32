#!/usr/bin/env python
"""Benchmark: backward-Euler time steps per second on the 256^3 workload.

Workload: 256^3 cells (16.8 M unknowns) on a 64 cm cube, seeded log-normal
K_s (sigma_lnK 2.5, correlation 16/16/4 cells), upstream interface mean,
dt = 10 s, initial head -61.5 cm, top face held at -20.7 cm, Newton
tolerance 1e-8, GMRES(30) with eta 1e-6, AMG V(1,1) with l1-Jacobi.
The mixed-precision run (AMG hierarchy stored and applied in FP32, all
else FP64) is the headline; the all-FP64 run of the same steps is reported
beside it.  One "step" is one full backward-Euler step: Newton iterations,
residuals, Jacobian rebuilds and every AMG-preconditioned GMRES solve.

The first `--warmup` steps (which include the one-time AMG set-up on the
first Jacobian) are untimed; the next `--steps` steps are timed.  Inputs are
resident on the GPU before timing starts.  Kernel times inside the timed
region come from HIP events recorded by the library on its own stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-steps/s at 256^3 (FP64 vs mixed AMG); SpMV HBM GB/s; p50/p99 step ms"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(rec, precision, warmup, steps, ks_dev, p0_dev, profile):
    import copy

    import torch

    import paper_2112_05051_amd as rich
    opts = copy.deepcopy(rec.options)
    opts.precision = precision
    s = rich.Solver(rec.problem, opts, ks_dev)
    s.set_state(p0_dev)
    torch.cuda.synchronize()
    log(f"[bench] warm-up ({warmup} steps, includes the AMG set-up)")
    t0 = time.perf_counter()
    warm = s.step(warmup, raise_on_error=False) if warmup > 0 else []
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    log(f"[bench] precision={'mixed' if precision else 'fp64'} warmup {warmup} steps {t_warm:.2f}s "
        f"(AMG set-up and refreshes {sum(w['t_setup'] for w in warm):.2f}s, "
        f"GMRES {sum(w['gmres_its'] for w in warm)} its)")
    if profile:
        s.profile(True)
    p_prev = None
    per_step = []
    stats = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        if k == steps - 1:
            p_prev = s.get_state()
        ts = time.perf_counter()
        st = s.step(1, raise_on_error=False)[0]
        torch.cuda.synchronize()
        per_step.append(time.perf_counter() - ts)
        stats.append(st)
        log(f"[bench]   step {k}: {per_step[-1] * 1e3:.1f} ms newton {st['newton_its']} gmres {st['gmres_its']} "
            f"jac {st['jac_builds']} status {st['status']}")
    torch.cuda.synchronize()
    t_timed = time.perf_counter() - t1
    prof = s.profile_read() if profile else None
    if profile:
        s.profile(False)
    p_final = s.get_state()
    levels = [list(s.level_size(l)) for l in range(s.levels())]
    return dict(solver=s, t_warm=t_warm, t_timed=t_timed, per_step=per_step, stats=stats, warm=warm,
                prof=prof, p_final=p_final, p_prev=p_prev, levels=levels)


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else float("nan")


def cpu_baseline(n_sample=64, nsteps=2):
    """The oracle, single-threaded, on the first nsteps steps of the same recipe
    at n_sample^3 (field statistics in cells unchanged), the rate scaled by the
    cell count to 256^3 (an optimistic figure for the CPU: iteration counts
    grow with the grid)."""
    import synth
    from oracle import oracle as orc
    rec = synth.recipe("c3", n=n_sample)
    ks, p = rec.ks(), rec.p0()
    S = orc.Solver(rec.problem, rec.options, ks)
    t0 = time.perf_counter()
    sts = [S.step(p) for _ in range(nsteps)]
    dt = time.perf_counter() - t0
    scale = (n_sample ** 3) / (256 ** 3)
    return {"value": nsteps * scale / dt, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {nsteps} backward-Euler steps of the 256^3 recipe's statistics on a {n_sample}^3 "
                      f"grid ({dt:.1f} s, {sum(s['newton_its'] for s in sts)} Newton, "
                      f"{sum(s['gmres_its'] for s in sts)} GMRES its, statuses {[s['status'] for s in sts]}), "
                      f"rate scaled by the cell ratio {n_sample}^3/256^3"}


# Kernel families of the per-kernel table: the library's timer name, the
# rocprofv3 kernel-name prefix and the source file that defines the kernel.
FAMILIES = {
    "update": ("k_update_norm<", "la.hip"),
    "multidot": ("k_multidot<", "la.hip"),
    "spmv_J": ("k_spmv_J<float>", "fine.hip"),
    "vc0_pre": ("k_st25<double, float, 0>", "fine.hip"),
    "residual": ("k_residual", "fine.hip"),
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_c3_256cube_mixed.md")


def algorithmic_bytes(name, n, mixed=True):
    """Algorithmic HBM bytes (read, written) of one launch of a fine-grid
    kernel at n unknowns (the per-cell figures of the kernel table of the
    design notes); None when the launch size is not fixed by n alone."""
    import re
    t = 4 if mixed else 8
    m = re.search(r"k_(multidot|update_norm)<(\d+)>", name)
    if m:
        k = int(m.group(2))
        return (8 * n * (k + 1), 0) if m.group(1) == "multidot" else (8 * n * (k + 1), 8 * n)
    if "k_spmv_J<float>" in name:
        return (60 * n, 8 * n)
    if "k_st25<double, float, 0>" in name or "k_st_pre<double, float>" in name:
        return (8 * n + 5 * t * n, t * n)
    if "k_residual" in name:
        return (24 * n, 8 * n)
    return None


def source_digest(fname):
    import hashlib
    path = os.path.join(ROOT, "paper_2112_05051_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def source_digests():
    return {f: source_digest(f) for f in sorted({src for _, src in FAMILIES.values()})}


def pmc_summary(fetch_csv, write_csv, n, digests=None):
    """Per-kernel HBM traffic from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs,
    calibrated by the 1 GiB device copy of --calibrate-copy.  The trailing
    'family' lines (measured bytes over algorithmic bytes, summed over the
    family's launches, with the digest of the kernel's source file) are what
    the benchmark reads back to report measured traffic.  `digests` are the
    source digests the profiled run printed (its "source_digests")."""
    digests = digests or source_digests()
    import collections
    import csv
    vals = {}
    for path, cname in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == cname:
                d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
        vals[cname] = d
    gib = float(1 << 30)
    cal = {}
    for cname in vals:
        copies = [v for k, lst in vals[cname].items() if "copyBuffer" in k for v in lst]
        cal[cname] = gib / max(copies) if copies else 1.0
    lines = [f"calibration (1 GiB copy): FETCH_SIZE x{cal['FETCH_SIZE']:.4f}, WRITE_SIZE x{cal['WRITE_SIZE']:.4f}",
             "",
             f"{'kernel':58s} {'launches':>8s} {'fetch MB':>10s} {'write MB':>10s} {'alg MB':>10s} {'traffic/alg':>11s}"]
    rows = []
    for k, lst in vals["FETCH_SIZE"].items():
        w = vals["WRITE_SIZE"].get(k, [0.0])
        f_b = cal["FETCH_SIZE"] * sum(lst) / len(lst)
        w_b = cal["WRITE_SIZE"] * sum(w) / len(w)
        alg = algorithmic_bytes(k, n)
        rows.append((k, len(lst), f_b, w_b, alg))
    rows.sort(key=lambda r: -(r[2] + r[3]) * r[1])
    for k, cnt, f_b, w_b, alg in rows[:40]:
        short = k.replace("rich::(anonymous namespace)::", "").replace("void ", "")[:58]
        a = (alg[0] + alg[1]) if alg else None
        lines.append(f"{short:58s} {cnt:8d} {f_b / 1e6:10.2f} {w_b / 1e6:10.2f} "
                     f"{(a / 1e6 if a else float('nan')):10.2f} {((f_b + w_b) / a if a else float('nan')):11.3f}")
    lines += ["", "family      launches  traffic/alg  source digest"]
    for fam, (prefix, src) in FAMILIES.items():
        sel = [r for r in rows if prefix in r[0] and r[4]]
        if not sel:
            continue
        meas = sum((r[2] + r[3]) * r[1] for r in sel)
        alg = sum((r[4][0] + r[4][1]) * r[1] for r in sel)
        lines.append(f"family {fam} {sum(r[1] for r in sel)} {meas / alg:.4f} {src} {digests[src]}")
    return "\n".join(lines)


def traffic_ratio(family):
    """Measured/algorithmic HBM bytes of a kernel family from the committed
    counter summary, or None if there is none or the kernel's source has
    changed since the counters were taken."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    for line in text.splitlines():
        f = line.split()
        if len(f) == 6 and f[0] == "family" and f[1] == family:
            return float(f[3]) if f[5] == source_digest(f[4]) else None
    return None


def stats_summary(stats_csv):
    """Kernel time by kernel family from a rocprofv3 --stats kernel_stats.csv."""
    import collections
    import csv
    import re
    fam = collections.defaultdict(lambda: [0, 0.0])
    rows = list(csv.DictReader(open(stats_csv)))
    for r in rows:
        name = r["Name"].replace("void ", "").replace("rich::(anonymous namespace)::", "")
        key = re.sub(r"<.*", "", name.split("(")[0])
        fam[key][0] += int(r["Calls"])
        fam[key][1] += float(r["TotalDurationNs"])
    tot = sum(v[1] for v in fam.values())
    lines = [f"total kernel time {tot / 1e9:.3f} s", f"{'kernel family':28s} {'calls':>8s} {'total ms':>10s} {'avg us':>9s} {'share':>6s}"]
    for k, (c, t) in sorted(fam.items(), key=lambda kv: -kv[1][1])[:25]:
        lines.append(f"{k:28s} {c:8d} {t / 1e6:10.1f} {t / c / 1e3:9.1f} {100 * t / tot:5.1f}%")
    lines.append("")
    lines.append(f"{'kernel (instance)':70s} {'calls':>8s} {'avg us':>9s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:20]:
        name = r["Name"].replace("void ", "").replace("rich::(anonymous namespace)::", "")[:70]
        lines.append(f"{name:70s} {int(r['Calls']):8d} {float(r['AverageNs']) / 1e3:9.1f}")
    return "\n".join(lines)


def run_serving(args):
    """Ensemble serving: the seeded Poisson request stream (cubic grids of
    32..96 cells, their own log-normal K_s, random interface mean, mixed
    precision) submitted at its arrival times to a rich_server; reports
    aggregate steps/s, p50/p99 per-step latency and admission waits."""
    import numpy as np

    import paper_2112_05051_amd as rich
    import synth
    sizes = tuple(int(v) for v in args.serve_sizes.split(","))
    reqs = synth.serving_stream(count=args.serve_count, rate=args.serve_rate, nsteps=args.serve_steps, sizes=sizes)
    if args.serve_mean:
        for _, rec in reqs:
            rec.problem.mean = synth.MEAN_NAMES[args.serve_mean]
    log(f"[serve] generating {len(reqs)} request fields")
    inputs = [(t, rec, rec.ks(), rec.p0()) for t, rec in reqs]
    srv = rich.Server(int(args.serve_budget_gb * (1 << 30)), args.serve_active, fused=args.serve_fused)
    ids = []
    t0 = time.perf_counter()
    for t_arr, rec, ks, p0 in inputs:
        now = time.perf_counter() - t0
        if t_arr > now:
            time.sleep(t_arr - now)
        ids.append(srv.submit(rec.problem, rec.options, ks, p0, rec.nsteps))
    log(f"[serve] all {len(ids)} submitted after {time.perf_counter() - t0:.1f}s")
    done = {}
    while len(done) < len(ids):
        for i in ids:
            if i not in done:
                r = srv.poll(i)
                if r is not None:
                    done[i] = r
                    log(f"[serve] request {i} done: status {r['status']} steps {len(r['step_ms'])} "
                        f"wait {r['wait_s']:.2f}s run {r['run_s']:.2f}s ({len(done)}/{len(ids)})")
        time.sleep(0.05)
    makespan = time.perf_counter() - t0
    flushes, products = srv.batch_stats()
    srv.close()
    step_ms = np.concatenate([d["step_ms"] for d in done.values()])
    waits = np.array([d["wait_s"] for d in done.values()])
    total_steps = int(sum(len(d["step_ms"]) for d in done.values()))
    by_mean = {}
    for (t_arr, rec, _, _), i in zip(inputs, ids):
        m = ["arith", "upstream", "harmonic"][rec.problem.mean]
        by_mean.setdefault(m, []).append(done[i]["status"])
    return {
        "metric": "ensemble serving: aggregate time-steps/s, p50/p99 per-step ms",
        "value": total_steps / makespan, "unit": "time-steps/s", "n_gpus": 1,
        "requests": len(ids), "steps_per_request": args.serve_steps, "arrival_rate_per_s": args.serve_rate,
        "max_active": args.serve_active, "budget_gb": args.serve_budget_gb, "makespan_s": makespan,
        "fused": args.serve_fused, "batched_flushes": flushes,
        "batched_products": products, "mean_batch": products / flushes if flushes else None,
        "total_steps": total_steps, "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)), "admission_wait_p50_s": float(np.percentile(waits, 50)),
        "admission_wait_p99_s": float(np.percentile(waits, 99)),
        "status_by_mean": {k: {str(s): v.count(s) for s in sorted(set(v))} for k, v in by_mean.items()},
        "dtype": "f64 (Newton, GMRES) + f32 (AMG V-cycle)", "data": "synthetic",
        "config": {"workload": "c4_ensemble_poisson", "sizes": list(sizes), "mean": args.serve_mean or "random"},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="cube size (256 = the benchmark workload)")
    ap.add_argument("--workload", choices=["c3", "c5", "paper3d"], default="c3",
                    help="c3: the 256^3 benchmark; c5: the 512^3 harmonic-mean instance; paper3d: the paper's "
                         "own 3-D infiltration test (798 x 798 x 38 unknowns; run it with --warmup 0 --steps 9 "
                         "for the whole simulation)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-profile", action="store_true", help="no per-kernel event timing")
    ap.add_argument("--full-newton", action="store_true",
                    help="also time the same steps with a fresh Jacobian every Newton iteration (msbset=1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM traffic counters)")
    ap.add_argument("--mean", choices=["arith", "upstream", "harmonic", "geometric", "integral"],
                    help="override the workload's interface mean (experiments)")
    ap.add_argument("--set", action="append", default=[], metavar="OPT=VALUE",
                    help="override a solver option (experiments; the headline uses the defaults)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="print the calibrated per-kernel traffic table of two rocprofv3 --pmc runs "
                         "(BENCH_JSON: the JSON line the profiled run printed) and exit")
    ap.add_argument("--serving", action="store_true", help="run the ensemble serving benchmark instead")
    ap.add_argument("--serve-count", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-active", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-fused", action="store_true",
                    help="fuse the preconditioned products of same-size simulations into batched launches")
    ap.add_argument("--serve-sizes", default="32,48,64,80,96", help="cube sizes the requests draw from")
    ap.add_argument("--serve-mean", choices=["arith", "upstream", "harmonic"],
                    help="one interface mean for every request (default: drawn per request)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="print kernel time by family from a rocprofv3 --stats run and exit")
    args = ap.parse_args()
    if args.stats_summary:
        print(stats_summary(args.stats_summary))
        return
    if args.pmc_summary:
        digests = json.load(open(args.pmc_summary[2]))["source_digests"]
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.n ** 3, digests))
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              f"(how the path would shard is a design note, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2112_05051_amd as rich
    import synth
    from oracle import oracle as orc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rich.load()
    if args.serving:
        print(json.dumps(run_serving(args)), flush=True)
        return
    rec = (synth.recipe("c3", n=args.n) if args.workload == "c3" else
           synth.recipe("c5") if args.workload == "c5" else synth.recipe("paper3d"))
    if args.mean:
        rec.problem.mean = synth.MEAN_NAMES[args.mean]
    for kv in args.set:
        k, v = kv.split("=")
        setattr(rec.options, k, type(getattr(rec.options, k))(float(v)))
    t = time.perf_counter()
    ks = rec.ks()
    p0 = rec.p0()
    log(f"[bench] K_s field {rec.problem.nx}^3 generated in {time.perf_counter() - t:.1f}s")
    ks_dev = torch.from_numpy(ks).cuda()
    p0_dev = torch.from_numpy(p0).cuda()
    torch.cuda.synchronize()
    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del a, b

    mixed = run_gpu(rec, rich.PREC_MIXED, args.warmup, args.steps, ks_dev, p0_dev, not args.no_profile)
    mixed["solver"].close()
    fp64 = None
    if not args.no_fp64:
        fp64 = run_gpu(rec, rich.PREC_FP64, args.warmup, args.steps, ks_dev, p0_dev, False)
        fp64["solver"].close()

    full = None
    if args.full_newton:
        import copy
        rec_full = copy.deepcopy(rec)
        rec_full.options.msbset = 1
        full = {}
        for name, prec in (("mixed", rich.PREC_MIXED), ("fp64", rich.PREC_FP64)):
            r = run_gpu(rec_full, prec, args.warmup, args.steps, ks_dev, p0_dev, False)
            r["solver"].close()
            full[name] = {"value": args.steps / r["t_timed"], "ms_per_step": 1e3 * r["t_timed"] / max(args.steps, 1),
                          "p50_step_ms": 1e3 * percentile(r["per_step"], 50),
                          "p99_step_ms": 1e3 * percentile(r["per_step"], 99),
                          "newton_its": sum(x["newton_its"] for x in r["stats"]),
                          "gmres_its": sum(x["gmres_its"] for x in r["stats"]),
                          "jac_builds": sum(x["jac_builds"] for x in r["stats"])}
        full["mixed_over_fp64"] = full["mixed"]["value"] / full["fp64"]["value"]

    steps = args.steps
    value = steps / mixed["t_timed"] if steps else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mixed["t_timed"] / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (Newton, GMRES) + f32 (AMG V-cycle)",
        "data": "synthetic",
        "config": {"workload": rec.name, "cells": rec.problem.n,
                   "grid": [rec.problem.nx, rec.problem.ny, rec.problem.nz],
                   "mean": ["arith", "upstream", "harmonic", "geometric", "integral"][rec.problem.mean],
                   "dt_s": rec.problem.dt, "ks_sigma_ln": rec.ks_sigma,
                   "ks_corr_cells": list(rec.ks_ell), "newton_tol": rec.options.fnormtol,
                   "gmres": f"GMRES({rec.options.gmres_restart}) eta {rec.options.eta}",
                   "amg": "matching aggregation (<=8), V(1,1) l1-Jacobi, dense coarsest"},
        "p50_step_ms": 1e3 * percentile(mixed["per_step"], 50),
        "p99_step_ms": 1e3 * percentile(mixed["per_step"], 99),
        "run_incl_warmup_s": mixed["t_warm"] + mixed["t_timed"],
        "newton_its": sum(s["newton_its"] for s in mixed["stats"]),
        "gmres_its": sum(s["gmres_its"] for s in mixed["stats"]),
        "jac_builds": sum(s["jac_builds"] for s in mixed["stats"]),
        "levels": mixed["stats"][-1]["levels"] if mixed["stats"] else None,
        "opc": mixed["stats"][-1]["opc"] if mixed["stats"] else None,
        "statuses": sorted({s["status"] for s in mixed["stats"]}),
        "linsolve_fails": sum(s["linsolve_fails"] for s in mixed["stats"]),
        "ls_backtracks": sum(s["ls_backtracks"] for s in mixed["stats"]),
        "hierarchy_n_nnz": mixed["levels"],
        "options": {k: getattr(rec.options, k) for k in vars(rec.options)},
        "source_digests": source_digests(),
    }
    if fp64 is not None:
        out["fp64"] = {"value": steps / fp64["t_timed"], "ms_per_step": 1e3 * fp64["t_timed"] / max(steps, 1),
                       "p50_step_ms": 1e3 * percentile(fp64["per_step"], 50),
                       "p99_step_ms": 1e3 * percentile(fp64["per_step"], 99),
                       "newton_its": sum(s["newton_its"] for s in fp64["stats"]),
                       "gmres_its": sum(s["gmres_its"] for s in fp64["stats"])}
        out["mixed_over_fp64"] = out["value"] / out["fp64"]["value"]
        a, b = mixed["p_final"].cpu().numpy(), fp64["p_final"].cpu().numpy()
        out["mixed_vs_fp64_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))

    if full is not None:
        out["full_newton_msbset1"] = full

    # Property that holds at any size: the oracle's residual at the GPU's final
    # state (with the GPU's previous state as theta_old) is below the tolerance.
    if mixed["p_prev"] is not None:
        pp = mixed["p_prev"].cpu().numpy()
        pf = mixed["p_final"].cpu().numpy()
        F = orc.residual(rec.problem, ks, pf, orc.theta(rec.problem, pp))
        out["oracle_residual_inf_at_gpu_state"] = float(np.max(np.abs(F)))

    prof = mixed["prof"]
    if prof:
        kern = {}
        for name, (n, ms, by) in prof.items():
            if n:
                kern[name] = {"launches": n, "avg_us": 1e3 * ms / n, "total_ms": ms,
                              "gbs": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                              "bytes_per_launch": by / n}
        out["kernels"] = kern
        dom = max(kern, key=lambda k: kern[k]["total_ms"])
        d = kern[dom]
        ratio = traffic_ratio(dom) if (args.n == 256 and args.workload == "c3") else None
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": d["gbs"] / HBM_PEAK_GBS,
                           "traffic": ratio * d["bytes_per_launch"] if ratio is not None else None,
                           "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                           "avg_us": d["avg_us"], "bytes_per_launch": d["bytes_per_launch"]}
        if "spmv_J" in kern:
            out["spmv_hbm_gbs"] = kern["spmv_J"]["gbs"]
    if not args.no_cpu:
        log("[bench] oracle CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
