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
        f"(AMG set-up and refreshes {sum(w['t_setup'] + w['t_aux'] for w in warm):.2f}s, "
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


def host_cpu():
    """Core count and model of this host (the oracle runs on one of its cores)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0)), "model": model}


def oracle_unit_times(rec, ks, gmres_sample=5):
    """Per-unit oracle times on the recipe's initial state at its full grid:
    one residual evaluation, one assembly of J and the auxiliary matrix, the
    AMG set-up, one numeric refresh of the hierarchy and the mean of the first
    `gmres_sample` iterations of a GMRES solve."""
    from oracle import oracle as orc
    P = rec.problem
    p0 = rec.p0()
    t = {}
    th = orc.theta(P, p0)
    t1 = time.perf_counter()
    F = orc.residual(P, ks, p0, th)
    t["residual"] = time.perf_counter() - t1
    t0 = time.perf_counter()
    J = orc.jacobian(P, ks, p0)
    M = orc.auxiliary(P, ks, p0)
    t["assembly"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    amg = orc.AMG(rec.options, M)
    t["amg_setup"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    amg.update_fine(M)
    t["refresh"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.gmres(J, -F, amg, rec.options.gmres_restart, rec.options.eta, gmres_sample)
    t["gmres_iteration"] = (time.perf_counter() - t0) / gmres_sample
    return t


def oracle_omp_unit_times(rec, ks, threads, gmres_sample=5):
    """The same per-unit times with the OpenMP build of the oracle (its
    per-row loops on `threads` cores; reductions serial, results identical),
    in a child process that loads that build."""
    import pickle
    import subprocess
    import tempfile

    import numpy as np
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "ks.npy"), ks)
        with open(os.path.join(d, "recipe.pkl"), "wb") as f:
            pickle.dump({"recipe": rec, "gmres_sample": gmres_sample}, f)
        env = dict(os.environ, RICH_ORACLE_OMP="1", OMP_NUM_THREADS=str(threads))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-units", d], env=env,
                           capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"oracle OpenMP leg failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(rec, ks, timed_stats, gmres_sample=5):
    """The oracle (plain C, one thread) timed on a bounded sample of the
    benchmark's own workload: per-unit times (oracle_unit_times) weighted by
    the counts of the GPU's timed steps (residual evaluations, rebuilds, GMRES
    iterations; the GPU's counts equal the oracle's in the parity tests) give
    the oracle's time per step.  Optimistic for the CPU: the sampled GMRES
    iterations have the shortest Gram-Schmidt of a cycle, and set-up, norms
    and line-search vector work are not counted.  The same figure for the
    OpenMP build of the oracle on the host's cores is reported beside it."""
    N = rec.problem.n
    P = rec.problem
    t = oracle_unit_times(rec, ks, gmres_sample)
    steps = max(len(timed_stats), 1)
    n_res = sum(s["bytes_feval"] for s in timed_stats) / (32.0 * N)
    n_build = sum(s["jac_builds"] for s in timed_stats)
    n_gmres = sum(s["gmres_its"] for s in timed_stats)

    def per_step(u):
        return (n_res * u["residual"] + n_build * (u["assembly"] + u["refresh"]) +
                n_gmres * u["gmres_iteration"]) / steps

    ps = per_step(t)
    out = {"value": 1.0 / ps, "unit": "time-steps/s", "cores": 1, "kind": "oracle",
           "host": host_cpu(),
           "sample": (f"per-unit oracle times on the {P.nx}x{P.ny}x{P.nz} recipe at its initial state "
                      f"(residual {t['residual']:.1f} s, J+M assembly {t['assembly']:.1f} s, AMG set-up "
                      f"{t['amg_setup']:.1f} s (not counted: once per run), refresh {t['refresh']:.1f} s, "
                      f"GMRES iteration {t['gmres_iteration']:.2f} s over the first {gmres_sample}) weighted by "
                      f"the GPU's timed steps: {n_res / steps:.1f} residuals, {n_build / steps:.2f} rebuilds, "
                      f"{n_gmres / steps:.0f} GMRES iterations per step"),
           "unit_seconds": t, "per_step_s": ps}
    threads = int(os.environ.get("OMP_NUM_THREADS", 0) or len(os.sched_getaffinity(0)))
    try:
        u = oracle_omp_unit_times(rec, ks, threads, gmres_sample)
        out["openmp"] = {"value": 1.0 / per_step(u), "unit": "time-steps/s", "cores": threads,
                         "sample": "the same units with the OpenMP build of the oracle (per-row loops on all "
                                   "cores; dot products, restriction and Galerkin sums serial)",
                         "unit_seconds": u, "per_step_s": per_step(u)}
    except Exception as e:  # the single-thread figure stands on its own
        out["openmp"] = {"error": repr(e)[:500]}
    return out


# Kernel families of the per-kernel table: the library's timer name, the
# rocprofv3 kernel-name prefixes and the source file that defines the kernels.
FAMILIES = {
    "update": ("k_update_norm<", "la.hip"),
    "multidot": ("k_multidot<", "la.hip"),
    "block_dot": (("k_block_dot<", "k_block_dot_wide<", "k_block_dot_wide_small<"), "la.hip"),
    "block_update": ("k_block_update<", "la.hip"),
    "spmv_J": ("k_spmv_J<float>", "fine.hip"),
    "vc0_pre": ("k_st25<double, float, 0>", "fine.hip"),
    "vc0_post": ("k_st25<double, float, 1>", "fine.hip"),
    "restrict": ("k_restrict<float>", "amg.hip"),
    "csr_pre": ("k_csr_stream<2, float, float, false>", "amg.hip"),
    "csr_post": ("k_csr_stream<2, float, float, true>", "amg.hip"),
    "residual": ("k_faces_tiled<false", "fine.hip"),
    "assembly": ("k_faces_tiled<true", "fine.hip"),
}
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_c3_256cube_mixed.md")


def _ceil(a, b):
    return (a + b - 1) // b


def _xcd(blocks):
    return _ceil(blocks, 8) * 8


def algorithmic_bytes(name, n, blocks=None, levels=None, mixed=True, shifted=True):
    """Algorithmic HBM bytes of one launch (the per-row figures of the kernel
    table of the design notes): fine-grid kernels from n alone; the coarse
    kernels of level l from that level's rows and entries, the level found by
    the launch's block count (CSR-stream: one block per 1536 entries, the
    restriction: one block per 256 coarse rows, both padded to a multiple of
    8).  shifted: the J products of GMRES form the s-step power basis (they
    also read the shift vector).  None when the launch cannot be placed (the
    block Gram-Schmidt kernels: their basis length is not in the launch)."""
    import re
    t = 4 if mixed else 8
    m = re.search(r"k_(multidot|update_norm)<(\d+)>", name)
    if m:
        k = int(m.group(2))
        return 8 * n * (k + 1) + (8 * n if m.group(1) == "update_norm" else 0)
    if "k_spmv_J<float>" in name:
        return (76 if shifted else 68) * n
    if "k_st25<double, float, 0>" in name or "k_st_pre<double, float>" in name:
        return 8 * n + 6 * t * n
    if "k_faces_tiled<false" in name or "k_residual" in name:
        return 32 * n
    if "k_faces_tiled<true" in name:
        return n * (16 + 56 + 32 + 8 + (20 if mixed else 0))
    if not levels or blocks is None:
        return None
    if "k_st25<double, float, 1>" in name:
        return 8 * n + 6 * t * n + 4 * n + t * levels[1][0]
    if "k_restrict<" in name:
        for l in range(len(levels) - 1):
            nl, nc = levels[l][0], levels[l + 1][0]
            if _xcd(_ceil(nc, 256)) == blocks:
                x0 = l + 1 < len(levels) - 1  # the coarse pre-smoothed iterate is stored below the coarsest
                return nl * (t + 4) + nc * (8 + t + (2 * t if x0 else 0))
        return None
    m = re.search(r"k_csr_stream<\d+, float, float, (true|false)>", name)
    if m:
        for l in range(1, len(levels) - 1):
            nl, nnz = levels[l]
            if _xcd(_ceil(nnz, 1536)) == blocks:
                if m.group(1) == "false":
                    return nnz * (4 + t) + nl * (8 + 3 * t)
                return nnz * (4 + t) + nl * (12 + 7 * t) + levels[l + 1][0] * t
        return None
    return None


def source_digest(fname):
    import hashlib
    path = os.path.join(ROOT, "paper_2112_05051_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def source_digests():
    return {f: source_digest(f) for f in sorted({src for _, src in FAMILIES.values()})}


def pmc_summary(fetch_csv, write_csv, n, digests=None, levels=None, info=None):
    """Per-kernel HBM traffic from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs,
    calibrated by the 1 GiB device copy of --calibrate-copy, per kernel and
    launch size.  The trailing 'family' lines (measured bytes over algorithmic
    bytes, summed over the family's launches, with the digest of the kernel's
    source file) are what the benchmark reads back to report measured traffic.
    `digests` are the source digests the profiled run printed, `levels` its
    hierarchy ([rows, entries] per level), `info` its JSON line: its options
    say whether the J products were shifted, and its per-kernel event timings
    give the block Gram-Schmidt kernels' algorithmic bytes (the library's own
    count over the same launches)."""
    digests = digests or source_digests()
    info = info or {}
    shifted = info.get("options", {}).get("gmres_block", 1) > 1
    import collections
    import csv
    vals = {}
    for path, cname in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        d = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == cname:
                grid = int(r["Grid_Size"]) if r.get("Grid_Size") else 0
                d[(r["Kernel_Name"], grid)].append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
        vals[cname] = d
    gib = float(1 << 30)
    cal = {}
    for cname in vals:
        copies = [v for (k, _), lst in vals[cname].items() if "copyBuffer" in k for v in lst]
        cal[cname] = gib / max(copies) if copies else 1.0
    lines = [f"calibration (1 GiB copy): FETCH_SIZE x{cal['FETCH_SIZE']:.4f}, WRITE_SIZE x{cal['WRITE_SIZE']:.4f}",
             "",
             f"{'kernel':52s} {'blocks':>7s} {'launches':>8s} {'fetch MB':>9s} {'write MB':>9s} {'alg MB':>9s} "
             f"{'traffic/alg':>11s}"]
    rows = []
    for (k, grid), lst in vals["FETCH_SIZE"].items():
        w = vals["WRITE_SIZE"].get((k, grid), [0.0])
        f_b = cal["FETCH_SIZE"] * sum(lst) / len(lst)
        w_b = cal["WRITE_SIZE"] * sum(w) / len(w)
        blocks = grid // 256 if grid else None
        alg = algorithmic_bytes(k, n, blocks, levels, shifted=shifted)
        rows.append((k, blocks, len(lst), f_b, w_b, alg))
    rows.sort(key=lambda r: -(r[3] + r[4]) * r[2])
    for k, blocks, cnt, f_b, w_b, alg in rows[:45]:
        short = k.replace("rich::(anonymous namespace)::", "").replace("void ", "")[:52]
        lines.append(f"{short:52s} {blocks if blocks else 0:7d} {cnt:8d} {f_b / 1e6:9.2f} {w_b / 1e6:9.2f} "
                     f"{(alg / 1e6 if alg else float('nan')):9.2f} {((f_b + w_b) / alg if alg else float('nan')):11.3f}")
    lines += ["", "family      launches  traffic/alg  source digest"]
    kern = info.get("kernels", {})
    for fam, (prefix, src) in FAMILIES.items():
        prefixes = prefix if isinstance(prefix, tuple) else (prefix,)
        named = [r for r in rows if any(p in r[0] for p in prefixes)]
        if fam in ("block_dot", "block_update"):
            # per-launch bytes vary with the basis length: the library's total over the run
            sel = named
            k = kern.get(fam)
            if not sel or not k or k["launches"] != sum(r[2] for r in sel):
                continue
            meas = sum((r[3] + r[4]) * r[2] for r in sel)
            alg = k["bytes_per_launch"] * k["launches"]
        else:
            sel = [r for r in named if r[5]]
            if not sel:
                continue
            meas = sum((r[3] + r[4]) * r[2] for r in sel)
            alg = sum(r[5] * r[2] for r in sel)
        lines.append(f"family {fam} {sum(r[2] for r in sel)} {meas / alg:.4f} {src} {digests[src]}")
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


def trace_gaps(trace_csv):
    """GPU idle time between kernels from a rocprofv3 --kernel-trace
    kernel_trace.csv: the span from the first kernel's start to the last one's
    end, the time no kernel ran, and that idle time by the pair of kernel
    families it fell between."""
    import collections
    import csv
    import re

    def fam(k):
        k = k.replace("void ", "").replace("rich::(anonymous namespace)::", "").replace("rich::", "")
        return re.sub(r"<.*", "", k.split("(")[0])[:28]
    ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), fam(r["Kernel_Name"]))
                for r in csv.DictReader(open(trace_csv)))
    t0, t1 = ks[0][0], max(e for _, e, _ in ks)
    busy, last, prev = 0, t0, "start"
    cnt, tot = collections.Counter(), collections.Counter()
    for s, e, k in ks:
        if s > last:
            cnt[(prev, k)] += 1
            tot[(prev, k)] += s - last
        busy += max(0, e - max(s, last))
        last, prev = max(last, e), k
    span = t1 - t0
    lines = [f"kernels {len(ks)}, span {span / 1e9:.3f} s, busy {busy / 1e9:.3f} s, "
             f"idle {(span - busy) / 1e9:.3f} s ({100 * (span - busy) / span:.1f}%)",
             f"{'idle between':62s} {'ms':>8s} {'gaps':>7s} {'avg us':>7s}"]
    for (a, b), v in tot.most_common(20):
        lines.append(f"{a + ' -> ' + b:62s} {v / 1e6:8.1f} {cnt[(a, b)]:7d} {v / cnt[(a, b)] / 1e3:7.1f}")
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
    srv = rich.Server(int(args.serve_budget_gb * (1 << 30)), args.serve_active,
                      fused=args.serve_fused or args.serve_persistent, persistent=args.serve_persistent)
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
    ok_ms = [d["step_ms"] for d in done.values() if d["status"] >= 0]
    ok_ms = np.concatenate(ok_ms) if ok_ms else np.zeros(0)
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
        "fused": args.serve_fused or args.serve_persistent, "persistent": args.serve_persistent,
        "batched_flushes": flushes,
        "batched_products": products, "mean_batch": products / flushes if flushes else None,
        "total_steps": total_steps, "p50_step_ms": float(np.percentile(step_ms, 50)),
        "p99_step_ms": float(np.percentile(step_ms, 99)),
        "converged_requests": sum(1 for d in done.values() if d["status"] >= 0),
        "converged_steps": int(ok_ms.size),
        "converged_steps_per_s": ok_ms.size / makespan,
        "p50_step_ms_converged": float(np.percentile(ok_ms, 50)) if ok_ms.size else None,
        "p99_step_ms_converged": float(np.percentile(ok_ms, 99)) if ok_ms.size else None,
        "admission_wait_p50_s": float(np.percentile(waits, 50)),
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
    ap.add_argument("--max-newton", type=int,
                    help="Newton iteration limit per step (default: the recipe's; c5 with its harmonic mean: 3, "
                         "enough to show that its steps do not converge)")
    ap.add_argument("--set", action="append", default=[], metavar="OPT=VALUE",
                    help="override a solver option (experiments; the headline uses the defaults)")
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"),
                    help="print the calibrated per-kernel traffic table of two rocprofv3 --pmc runs "
                         "(BENCH_JSON: the JSON line the profiled run printed) and exit")
    ap.add_argument("--serving", action="store_true", help="run the ensemble serving benchmark instead")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the C4 serving run that the default line carries beside the 256^3 figures")
    ap.add_argument("--serve-count", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-active", type=int, default=8, help="resident simulations (server workers)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-fused", action="store_true",
                    help="fuse the preconditioned products of same-size simulations into batched launches")
    ap.add_argument("--serve-persistent", action="store_true",
                    help="fused batched launches as persistent grids taking work from a device-side queue")
    ap.add_argument("--serve-sizes", default="32,48,64,80,96", help="cube sizes the requests draw from")
    ap.add_argument("--serve-mean", choices=["arith", "upstream", "harmonic"],
                    help="one interface mean for every request (default: drawn per request)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="print kernel time by family from a rocprofv3 --stats run and exit")
    ap.add_argument("--oracle-units", metavar="DIR", help=argparse.SUPPRESS)
    ap.add_argument("--trace-gaps", metavar="KERNEL_TRACE_CSV",
                    help="print the GPU idle time between kernels of a rocprofv3 --kernel-trace run and exit")
    args = ap.parse_args()
    if args.stats_summary:
        print(stats_summary(args.stats_summary))
        return
    if args.trace_gaps:
        print(trace_gaps(args.trace_gaps))
        return
    if args.oracle_units:
        # child of the CPU baseline's OpenMP leg (the oracle build is chosen by the environment)
        import pickle

        import numpy as np
        with open(os.path.join(args.oracle_units, "recipe.pkl"), "rb") as f:
            job = pickle.load(f)
        ks = np.load(os.path.join(args.oracle_units, "ks.npy"))
        print(json.dumps(oracle_unit_times(job["recipe"], ks, job["gmres_sample"])), flush=True)
        return
    if args.pmc_summary:
        info = json.loads(open(args.pmc_summary[2]).read().strip().splitlines()[-1])
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.n ** 3, info["source_digests"],
                          info.get("hierarchy_n_nnz"), info))
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
    if args.max_newton:
        rec.options.max_newton = args.max_newton
    elif args.workload == "c5" and rec.problem.mean == synth.HARMONIC:
        # With the harmonic mean at this spacing and dt the Jacobian is indefinite along the
        # infiltration mode and Newton from the previous level cannot converge (the CPU tests
        # show the mechanism); a few iterations show it without spending minutes per step.
        rec.options.max_newton = 3
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
    converged = all(s["status"] >= 0 for s in mixed["stats"])
    value = steps / mixed["t_timed"] if steps and converged else 0.0
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
        # s-step block rounds, and those finished vector by vector
        "gmres_rounds": sum(s["gmres_rounds"] for s in mixed["stats"]),
        "gmres_redone": sum(s["gmres_redone"] for s in mixed["stats"]),
        "jac_builds": sum(s["jac_builds"] for s in mixed["stats"]),
        "levels": mixed["stats"][-1]["levels"] if mixed["stats"] else None,
        "opc": mixed["stats"][-1]["opc"] if mixed["stats"] else None,
        "statuses": sorted({s["status"] for s in mixed["stats"]}),
        "converged": converged,
        "max_newton": rec.options.max_newton,
        "linsolve_fails": sum(s["linsolve_fails"] for s in mixed["stats"]),
        # discrete mass balance at each accepted state: dt * sum_c Phi_c (the
        # storage change minus the boundary inflow), and the Newton residual there
        "max_abs_mass_residual": max((abs(s["mass_residual"]) for s in mixed["stats"]), default=None),
        "max_fnorm_inf": max((s["fnorm_inf"] for s in mixed["stats"]), default=None),
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
    if not args.no_cpu and mixed["stats"]:
        log("[bench] oracle CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline(rec, ks, mixed["stats"])
    if not args.no_serving and args.workload == "c3" and args.n == 256:
        # the C4 request stream as specified (64 requests x 20 steps, Poisson rate 4/s)
        log("[bench] C4 serving stream ...")
        del ks_dev, p0_dev
        torch.cuda.empty_cache()
        try:
            sv = run_serving(args)
        except Exception as e:  # the headline above stands on its own
            sv = None
            out["serving_c4"] = {"error": repr(e)}
        keep = ("value", "unit", "requests", "steps_per_request", "arrival_rate_per_s", "max_active", "makespan_s",
                "total_steps", "p50_step_ms", "p99_step_ms", "converged_requests", "converged_steps_per_s",
                "p50_step_ms_converged", "p99_step_ms_converged", "admission_wait_p50_s", "admission_wait_p99_s",
                "status_by_mean")
        if sv is not None:
            out["serving_c4"] = {k: sv[k] for k in keep}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
