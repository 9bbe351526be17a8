"""Benchmark: SpTRSV solves/s and HBM GB/s, rewritten vs plain level-set.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4]

Workload (default, the largest single-GPU configuration): the lower factor of
the 200^3 3D 7-point stencil (pattern only, diagonally dominant random values)
followed by a 5,000-row near-serial tail; n = 8,005,000, nnz = 31,900,000,
32 right-hand sides stored by rows (n x 32 row-major, read and written through
the level order by sptrsv_solve_rows), FP64, each solve a replay of a hipGraph;
the same variants with column-major right-hand sides are timed beside it.
Variants on the same matrix and right-hand sides, each autotuned first:
  plain    level-set solve of L
  naive    L' after the naive rewrite (levels with < 32 rows, fill cap 4x)
  learned  L' after the rewrite with per-level actions chosen by the trained
           policy, or the naive rule's L' when that autotunes faster on this
           matrix (a measured per-matrix fallback; config.chosen says which)
A step is one solve of the headline variant (learned if a trained policy is
available, else naive). Every variant is checked against the CPU oracle
(relative error <= 1e-10) before it is timed; rewriting and tuning are
preprocessing and are reported separately. value / ms_per_step come from the
median of the per-step device times; graph workloads also report five
repetitions of 100 replays. --config 1 is the 2D stencil + 20,000-row chain
(one right-hand side, stream launches), --config 2 the 4M-row power law.

Prints ONE JSON line. Inputs are resident in HBM when the timed region starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SpTRSV solves/s & HBM GB/s: learned-rewrite vs plain level-set, relerr<=1e-10"
HBM_PEAK_GBS = 8000.0
TOL = 1e-10

WORKLOADS = {
    0: "window-64 random lower CSR, n=2,000, up to 5 off-diagonals/row, nrhs=1",
    1: "2D 1000x1000 5-point lower factor + 20,000-row chain, n=1,020,000, nnz=3,078,000, nrhs=1",
    2: "power-law (Zipf 1.2 in-degree) lower CSR, n=4,000,000, nnz=36,016,553 (8.0 distinct off-diagonals/row), "
       "3,969 levels, nrhs=1",
    3: "512 window-64 random lower CSR matrices, n_i uniform in [1000, 50000], ~6 nnz/row, nrhs=16 each",
    4: "3D 200^3 7-point lower factor + 5,000-row tail, n=8,005,000, nnz=31,900,000, nrhs=32",
    5: "preconditioner application z = L^-T L^-1 r (incomplete-Cholesky style) with the 3D 200^3 7-point lower "
       "factor + 5,000-row tail, n=8,005,000, nnz=31,900,000, nrhs=32",
}
GRAPH_DEFAULT = {4}  # workloads timed as hipGraph replays of the solve
ROWS_DEFAULT = {4}  # workloads whose right-hand sides are stored by rows by default


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(n, nnz, nlev, nrhs, nnz_t=0, rewritten=False):
    """Compulsory traffic of one solve: 12 B per nonzero (value + column),
    8 B per row (row pointer + level row map), 4 B per level pointer, 16 B per
    row and right-hand side (read b, write x); a rewritten solve adds T's
    nonzeros and its row pointers."""
    if not rewritten:
        return 12.0 * nnz + 8.0 * n + 4.0 * (nlev + 1) + 16.0 * n * nrhs
    return 12.0 * (nnz + nnz_t) + 12.0 * n + 4.0 * (nlev + 1) + 16.0 * n * nrhs


# Sources whose text decides what a kernel reads and writes (thin runs read
# the window images k_image.hip builds).
KERNEL_SOURCE = {"k_thin_run": ("k_thin.hip", "k_image.hip", "sync.h"),
                 "k_batch_run": ("k_thin.hip", "k_image.hip", "sync.h"),
                 "k_wide_level": ("k_wide.hip", "sync.h"), "k_wide_run": ("k_wide.hip", "sync.h"),
                 "k_flow_run": ("k_flow.hip",), "k_gather": ("k_vec.hip",), "k_scatter": ("k_vec.hip",),
                 "k_sf_solve": ("k_syncfree.hip",)}


def source_hash(kernel):
    """Hash of the source files of a kernel together with the shared header."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCE[kernel] + ("common.h",):
        with open(os.path.join(ROOT, "paper_2206_05843_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload_key):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(f"{kernel}:{workload_key}")
    if not e or e.get("source_hash") != source_hash(kernel):
        return None
    return e.get("bytes_per_launch")


def bench_batch(args, np, torch, gen, oracle, sp):
    """The batched workload: every matrix and right-hand side in one persistent
    launch (captured in a hipGraph and replayed) against the loop of
    per-matrix solves it replaces. A step solves all matrices."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    mats, nrhs = gen.config_matrix(3)
    ns = [m.n for m in mats]
    rp = torch.from_numpy(np.concatenate([m.row_ptr for m in mats]).astype(np.int32)).to(dev)
    ci = torch.from_numpy(np.concatenate([m.col for m in mats])).to(dev)
    va = torch.from_numpy(np.concatenate([m.val for m in mats])).to(dev)
    b_np = [gen.rhs(m, nrhs) for m in mats]
    b = torch.from_numpy(np.concatenate([x.reshape(-1) for x in b_np])).to(dev)
    n_tot, nnz_tot = sum(ns), sum(m.nnz for m in mats)
    log(f"[bench] generated {len(mats)} matrices, n={n_tot} nnz={nnz_tot} nrhs={nrhs} "
        f"in {time.perf_counter() - t0:.1f}s")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    h = sp.Handle()
    t = time.perf_counter()
    h.batch_analyze(ns, rp, ci, va)
    torch.cuda.synchronize()
    pre = time.perf_counter() - t
    t = time.perf_counter()
    h.autotune(sp.BATCH, nrhs)
    tune_s = time.perf_counter() - t
    sched = h.get_schedule(sp.BATCH, nrhs)
    log(f"[bench] batch schedule {sched} (tuned in {tune_s:.2f}s)")
    nlev = [int(h.batch_levels(i)[0].numel()) - 1 for i in range(len(mats))]
    x = torch.zeros_like(b)
    h.batch_solve(b, x, nrhs)
    h.check()
    xs = x.cpu().numpy()
    off, worst = 0, 0.0
    t = time.perf_counter()
    for m, bm in zip(mats, b_np):
        xm = xs[off * nrhs:(off + m.n) * nrhs].reshape(nrhs, m.n)
        worst = max(worst, oracle.relerr(xm, oracle.solve(m, bm)))
        off += m.n
    t_oracle_all = time.perf_counter() - t
    if not worst <= TOL:
        raise SystemExit(f"[bench] batched solve failed parity: relerr={worst:.3e}")
    x2 = torch.zeros_like(b)
    h.batch_solve(b, x2, nrhs, looped=True)
    h.check()
    if not torch.equal(x, x2):
        raise SystemExit("[bench] looped and batched solutions differ")
    log(f"[bench] parity ok: max relerr {worst:.2e} over {len(mats)} matrices; oracle {t_oracle_all:.1f}s")

    def run_steps(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        h.batch_solve(b, x, nrhs)
    ms = run_steps(g.replay, args.steps, args.warmup)
    h.check()
    ms_eager = run_steps(lambda: h.batch_solve(b, x, nrhs), max(5, args.steps // 2), args.warmup)
    ms_loop = run_steps(lambda: h.batch_solve(b, x2, nrhs, looped=True), max(5, args.steps // 2), args.warmup)
    h.check()
    # live event timing of the persistent kernel on the solve stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record(stream)
        h.batch_solve(b, x, nrhs)
        e1.record(stream)
    torch.cuda.synchronize()
    ms_ev = sum(e0.elapsed_time(e1) for e0, e1 in ev) / len(ev)
    alg = sum(12.0 * m.nnz + 8.0 * m.n + 4.0 * (nl + 1) + 16.0 * m.n * nrhs for m, nl in zip(mats, nlev))
    achieved = alg / (ms_ev * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu:
        reps = max(1, int(12.0 / max(t_oracle_all, 1e-6)))
        t = time.perf_counter()
        for _ in range(reps):
            for m, bm in zip(mats, b_np):
                oracle.solve(m, bm)
        el_c = time.perf_counter() - t
        cpu = {"value": round(reps / el_c, 4), "unit": "batch solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} passes over all {len(mats)} matrices x {nrhs} RHS by the serial FP64 oracle "
                         f"({el_c:.1f}s); host nproc={os.cpu_count()}"}
    res = {
        "metric": METRIC, "value": round(1e3 / ms, 3), "unit": "batch solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator of the workload's structure; no dataset)",
        "config": {"workload": WORKLOADS[3], "variant": "batched persistent launch, hipGraph replays",
                   "nmat": len(mats), "n": n_tot, "nnz": nnz_tot, "nrhs": nrhs, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": None, "kernel": "k_batch_run",
                     "avg_step_ms_events": round(ms_ev, 5), "alg_bytes_per_step": alg},
        "cpu_baseline": cpu,
        "variants": {"batched_graph": {"ms": round(ms, 5)}, "batched_eager": {"ms": round(ms_eager, 5)},
                     "looped_per_matrix": {"ms": round(ms_loop, 5)}},
        "speedup_vs_looped": round(ms_loop / ms, 4),
        "matrix_solves_per_s": round(len(mats) * 1e3 / ms, 1),
        "preprocess_s": round(pre, 3), "autotune_s": round(tune_s, 3), "schedule": sched, "max_relerr": worst,
        "levels": {"min": min(nlev), "max": max(nlev), "total": sum(nlev)},
    }
    print(json.dumps(res), flush=True)


def bench_precond(args, np, torch, gen, oracle, sp):
    """One step = z = L^-T (L^-1 r): a forward solve with L and a transposed
    solve with the same factor (sptrsv_analyze_form, LOWER_TRANS), each
    rewritten by the naive rule and autotuned, replayed as hipGraphs. r, the
    intermediate y and z are stored by rows (n x nrhs) unless --layout cols."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    m, nrhs = gen.config_matrix(4)
    r_np = gen.rhs(m, nrhs)
    t0 = time.perf_counter()
    z_ref = oracle.solve_form(m, oracle.solve(m, r_np), oracle.LOWER_TRANS)
    t_oracle = time.perf_counter() - t0
    log(f"[bench] oracle application {t_oracle:.1f}s")
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (m.row_ptr, m.col, m.val))
    rows = (args.layout or "rows") == "rows"
    r = torch.from_numpy(r_np).to(dev)
    if rows:
        r = r.t().contiguous()  # (n, nrhs): a row's right-hand sides together

    def solve(h, which, b, x):
        return h.solve_rows(b, which, x) if rows else h.solve(b, which, x)

    def graph(h, which, b, x):
        return h.graph_create_rows(b, x, which) if rows else h.graph_create(b, x, which)

    out_var = {}
    best = None
    for name, rewrite in (("plain", False), ("naive", True)):
        hs, info = [], {}
        y = torch.empty_like(r)
        z = torch.empty_like(r)
        for form in (sp.LOWER, sp.LOWER_TRANS):
            h = sp.Handle()
            nlev = h.analyze(rp, ci, va, form=form)
            which = sp.ORIGINAL
            key = "L" if form == sp.LOWER else "LT"
            info[f"nlev_{key}"] = nlev
            if rewrite:
                st = h.rewrite(sp.THIN_ROWS, 32, 4.0, 0)
                which = sp.REWRITTEN
                info[f"nlev_{key}"] = st["nlev_after"]
                info[f"nnz_T_{key}"] = st["nnz_T"]
            h.autotune(which, nrhs, rows=rows)
            info[f"schedule_{key}"] = h.get_schedule(which, nrhs)
            hs.append((h, which))
        solve(hs[0][0], hs[0][1], r, y)
        solve(hs[1][0], hs[1][1], y, z)
        for h, _ in hs:
            h.check()
        info["relerr"] = oracle.relerr((z.t() if rows else z).cpu().numpy(), z_ref)
        if not info["relerr"] <= TOL:
            raise SystemExit(f"[bench] {name} application failed parity: relerr={info['relerr']:.3e}")
        g0 = graph(hs[0][0], hs[0][1], r, y)
        g1 = graph(hs[1][0], hs[1][1], y, z)
        for _ in range(args.warmup):
            hs[0][0].graph_launch(g0)
            hs[1][0].graph_launch(g1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            hs[0][0].graph_launch(g0)
            hs[1][0].graph_launch(g1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        # per-kernel-class profile of as many eager applications
        for h, _ in hs:
            h.profile_start()
        for _ in range(args.steps):
            solve(hs[0][0], hs[0][1], r, y)
            solve(hs[1][0], hs[1][1], y, z)
        torch.cuda.synchronize()
        prof = {}
        for h, _ in hs:
            for k, v in h.profile_stop().items():
                if k == "in_timed_region":
                    continue
                acc = prof.setdefault(k, {"launches": 0, "ms": 0.0, "bytes": 0.0})
                for f in ("launches", "ms", "bytes"):
                    acc[f] += v[f]
        for h, _ in hs:
            h.check()
        info["ms"] = ms
        info["profile"] = prof
        out_var[name] = info
        log(f"[bench] {name}: {ms:.3f} ms per application, relerr {info['relerr']:.2e}")
        if best is None or ms < out_var[best]["ms"]:
            best = name
    head = out_var[best]
    prof = head["profile"]
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dp = prof[dom]
    per_launch_ms = dp["ms"] / max(1, dp["launches"])
    bpl = dp["bytes"] / max(1, dp["launches"])
    achieved = bpl / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    kname = {"thin_run": "k_thin_run", "wide_level": "k_wide_level", "gather": "k_gather", "scatter": "k_scatter"}[dom]
    hsched = head["schedule_L"]
    if dom == "wide_level" and hsched["mode"] == 3:
        kname = "k_sf_solve"
    elif dom == "wide_level" and hsched["mode"] == 4:
        kname = "k_flow_run"
    elif dom == "wide_level" and hsched["wide_grid"] > 0:
        kname = "k_wide_run"
    cpu = None
    if not args.no_cpu:
        cpu = {"value": round(1.0 / t_oracle, 5), "unit": "applications/s", "cores": 1, "kind": "oracle",
               "sample": f"one application (forward and transposed substitution, {nrhs} right-hand sides) by the "
                         f"serial FP64 oracle ({t_oracle:.1f}s, includes its transpose of L)"}
    res = {
        "metric": "preconditioner applications/s (z = L^-T L^-1 r), relerr<=1e-10",
        "value": round(1e3 / head["ms"], 3), "unit": "applications/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["ms"], 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded generator of the workload's structure; no dataset)",
        "config": {"workload": WORKLOADS[5], "variant": best, "nrhs": nrhs, "n": m.n, "nnz": m.nnz,
                   "layout": ("r, y and z by rows (n x nrhs row-major)" if rows
                              else "r, y and z by columns (column-major, leading dimension n)"),
                   "parallelism": "single GPU", "timing": "hipGraph replays (one graph per solve)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": load_traffic(kname, "config5_" + best),
                     "kernel": kname, "launches": dp["launches"], "avg_launch_ms": round(per_launch_ms, 5),
                     "alg_bytes_per_launch": bpl, "events": "eager applications after the timed region"},
        "cpu_baseline": cpu,
        "variants": {k: {kk: (round(vv, 5) if isinstance(vv, float) and kk != "relerr" else vv)
                         for kk, vv in v.items() if kk != "profile"} for k, v in out_var.items()},
    }
    print(json.dumps(res), flush=True)


def bench_analysis(args, np, torch, gen, oracle, sp):
    """Preprocessing only: wall time of each step (synchronised) on the
    workload, with the oracle's serial level pass beside it."""
    dev = torch.device("cuda:0")
    m, nrhs = gen.config_matrix(args.config)
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (m.row_ptr, m.col, m.val))
    t = time.perf_counter()
    lv = oracle.levels(m)
    t_oracle = time.perf_counter() - t
    out = {"workload": WORKLOADS[args.config], "oracle_levels_s": round(t_oracle, 4), "nlev": lv.nlev, "runs": []}
    from paper_2206_05843_amd import policy
    pol = policy.load_default()
    for rep in range(3):
        r = {}
        torch.cuda.synchronize()
        h = sp.Handle()
        t = time.perf_counter()
        nlev = h.analyze(rp, ci, va)
        torch.cuda.synchronize()
        r["analyze_s"] = time.perf_counter() - t
        assert nlev == lv.nlev
        t = time.perf_counter()
        h.level_features()
        torch.cuda.synchronize()
        r["features_s"] = time.perf_counter() - t
        t = time.perf_counter()
        h.rewrite(sp.THIN_ROWS, 32, 4.0, 0)
        torch.cuda.synchronize()
        r["rewrite_naive_s"] = time.perf_counter() - t
        if pol is not None:
            t = time.perf_counter()
            policy.rewrite_learned(h, pol)
            torch.cuda.synchronize()
            r["rewrite_learned_s"] = time.perf_counter() - t
        out["runs"].append({k: round(v, 4) for k, v in r.items()})
        log(f"[bench] analysis rep {rep}: {out['runs'][-1]}")
    print(json.dumps(out), flush=True)


def calibrate_copy(torch, mib):
    """Ten device-to-device copies of a buffer of known size: the FETCH_SIZE and
    WRITE_SIZE counters of these launches scale the counters of the solve
    kernels to bytes."""
    n = mib * (1 << 20) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n * 8, "launches": 10}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-fallback", action="store_true",
                    help="learned variant without the measured per-matrix fallback to the naive rewrite")
    ap.add_argument("--variants", default="plain,naive,learned",
                    help="comma-separated subset of plain,naive,learned to set up and time")
    ap.add_argument("--schedules", default=None,
                    help="JSON object variant -> schedule (mode, thin_rows, wg_threads, wide_threads, "
                         "lanes_per_row); those variants skip the autotuner (for profiled runs)")
    ap.add_argument("--layout", default=None, choices=("cols", "rows"),
                    help="how the right-hand sides are stored: cols (column-major, a column per right-hand side) "
                         "or rows (n x nrhs row-major, solved with sptrsv_solve_rows); default rows for the 3D "
                         "stencil workloads (the solve, whose other layout is timed too and reported beside it, "
                         "and the preconditioner application)")
    ap.add_argument("--graph", type=int, default=None, choices=(0, 1),
                    help="time hipGraph replays of the solve (default: on for the 3D stencil workload)")
    ap.add_argument("--analysis-only", action="store_true",
                    help="only time the preprocessing of the workload (analysis, level features with the "
                         "longest-path heights, naive and learned rewrites), no solves")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 10 device copies of MIB MiB (the reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the solve of one matrix is not sharded "
                                   "across GPUs (a level-set solve would need a device-wide exchange per level)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy(torch, args.calibrate_copy)
        return

    import gen
    import oracle
    import paper_2206_05843_amd as sp

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.config == 3:
        bench_batch(args, np, torch, gen, oracle, sp)
        return
    if args.config == 5:
        bench_precond(args, np, torch, gen, oracle, sp)
        return
    if args.analysis_only:
        bench_analysis(args, np, torch, gen, oracle, sp)
        return
    use_graph = (args.config in GRAPH_DEFAULT) if args.graph is None else bool(args.graph)
    layout = args.layout or ("rows" if args.config in ROWS_DEFAULT else "cols")
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream
    torch.cuda.set_stream(stream)
    t0 = time.perf_counter()
    m, nrhs = gen.config_matrix(args.config)
    b_np = gen.rhs(m, nrhs)
    log(f"[bench] generated n={m.n} nnz={m.nnz} nrhs={nrhs} in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    x_ref = oracle.solve(m, b_np)
    t_oracle_one = time.perf_counter() - t0
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (m.row_ptr, m.col, m.val))
    b = torch.from_numpy(b_np).to(dev)
    if nrhs == 1:
        b = b.view(-1)
        layout = "cols"  # one right-hand side: both layouts are the same vector
    b_rows = b.t().contiguous() if layout == "rows" else None  # (n, nrhs): a row's right-hand sides together

    variants = {}
    probe = sp.Handle()
    costs = probe.measure_level_costs()
    log(f"[bench] empty-level costs (ns): { {k: round(v, 1) for k, v in costs.items()} }")

    def setup(name, rewrite_fn=None, rewrite=True):
        h = sp.Handle()
        t = time.perf_counter()
        nlev = h.analyze(rp, ci, va)
        which = sp.ORIGINAL
        info = dict(nlev=nlev, nnz=m.nnz, nnz_t=0)
        if rewrite:
            st = rewrite_fn(h) if rewrite_fn else h.rewrite(sp.THIN_ROWS, 32, 4.0, 0)
            if isinstance(st, tuple):
                st, info["chosen"] = st
            which = sp.REWRITTEN
            info.update(nlev=st["nlev_after"], nnz=st["nnz_Lp"], nnz_t=st["nnz_T"], rows_rewritten=st["rows_rewritten"],
                        nlev_before=st["nlev_before"], max_distance=st["max_distance"])
        torch.cuda.synchronize()
        info["preprocess_s"] = time.perf_counter() - t
        t = time.perf_counter()
        if name in fixed_sched:
            h.set_schedule(which, **fixed_sched[name])
            info["tuned_ms"] = None
        else:
            info["tuned_ms"] = h.autotune(which, nrhs, rows=layout == "rows")
            info["tune"] = h.tune_info()
        info["schedule"] = h.get_schedule(which, nrhs)
        info["autotune_s"] = time.perf_counter() - t
        x = h.solve(b, which)
        h.check()
        info["relerr"] = oracle.relerr(x.view(nrhs, -1).cpu().numpy(), x_ref)
        if layout == "rows":
            xr = h.solve_rows(b_rows, which)
            h.check()
            info["relerr_cols"] = info["relerr"]
            info["relerr"] = oracle.relerr(xr.t().cpu().numpy(), x_ref)
        if not max(info["relerr"], info.get("relerr_cols", 0.0)) <= TOL:
            raise SystemExit(f"[bench] variant {name} failed parity: relerr={info['relerr']:.3e}")
        info["bytes"] = alg_bytes(m.n, info["nnz"], info["nlev"], nrhs, info["nnz_t"], rewrite)
        info["level_floor_us"] = h.level_floor(costs, which, nrhs, graph=use_graph, rows=layout == "rows")
        variants[name] = (h, which, info)
        log(f"[bench] {name}: nlev={info['nlev']} relerr={info['relerr']:.2e} pre={info['preprocess_s']:.2f}s "
            f"schedule={info['schedule']} level floor {info['level_floor_us']:.1f} us")

    want = set(v.strip() for v in args.variants.split(",") if v.strip())
    fixed_sched = json.loads(args.schedules) if args.schedules else {}
    if "plain" in want:
        setup("plain", rewrite=False)
    if "naive" in want:
        try:
            setup("naive")
        except sp.SptrsvError as e:
            log(f"[bench] naive rewrite unavailable: {e}")
    if "learned" in want and not args.no_learned:
        try:
            from paper_2206_05843_amd import policy
            pol = policy.load_default()
            if pol is not None:
                if args.no_fallback:
                    setup("learned", rewrite_fn=lambda h: policy.rewrite_learned(h, pol))
                else:
                    setup("learned", rewrite_fn=lambda h: policy.rewrite_learned_checked(h, pol, nrhs,
                                                                                         csr=(rp, ci, va)))
        except (ImportError, sp.SptrsvError, FileNotFoundError) as e:
            log(f"[bench] learned policy unavailable: {e}")

    def timed(name, steps, warmup, rows):
        """Per-step device times (HIP events on the solve stream around every
        step: a graph replay, or an eager solve) and the wall time of all
        steps; plus, for graph replays, the protocol of five repetitions of
        100 replays (mean per solve of each, median of the five)."""
        h, which, _ = variants[name]
        bb = b_rows if rows else b
        x = torch.empty_like(bb)
        if use_graph:
            gid = h.graph_create_rows(bb, x, which) if rows else h.graph_create(bb, x, which)
            run = lambda: h.graph_launch(gid)  # noqa: E731
        elif rows:
            run = lambda: h.solve_rows(bb, which, x)  # noqa: E731
        else:
            run = lambda: h.solve(bb, which, x)  # noqa: E731
        for _ in range(warmup):
            run()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            run()
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        reps = None
        if use_graph:
            reps = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(100):
                    run()
                e1.record(stream)
                torch.cuda.synchronize()
                reps.append(e0.elapsed_time(e1) / 100)
        h.check()
        return per, wall, reps

    def kernel_profile(name, steps):
        """Per-kernel-class HIP-event profile of eager solves on the solve
        stream (after the timed region: no events inside a graph)."""
        h, which, _ = variants[name]
        bb = b_rows if layout == "rows" else b
        solve = h.solve_rows if layout == "rows" else h.solve
        x = torch.empty_like(bb)
        solve(bb, which, x)
        h.profile_start()
        for _ in range(steps):
            solve(bb, which, x)
        torch.cuda.synchronize()
        prof = h.profile_stop()
        h.check()
        return prof

    def median(v):
        v = sorted(v)
        k = len(v)
        return v[k // 2] if k % 2 else 0.5 * (v[k // 2 - 1] + v[k // 2])

    headline = "learned" if "learned" in variants else ("naive" if "naive" in variants else "plain")
    for name in variants:
        steps = args.steps if name == headline else max(20, args.steps // 2)
        per, wall, reps = timed(name, steps, args.warmup, layout == "rows")
        info = variants[name][2]
        if layout == "rows":  # the same variant with column-major right-hand sides, for comparison
            per_c, _, reps_c = timed(name, max(20, args.steps // 2), args.warmup, False)
            info["ms_cols"] = median(per_c)
            if reps_c is not None:
                info["graph_reps_median_ms_cols"] = median(reps_c)
        info["ms"] = median(per)
        info["ms_wall_mean"] = wall * 1e3 / steps
        info["steps"] = steps
        if reps is not None:
            info["graph_reps_ms"] = reps
            info["graph_reps_median_ms"] = median(reps)
    ms = variants[headline][2]["ms"]
    prof = kernel_profile(headline, max(5, min(args.steps, 20)))

    # roofline of the dominant kernel class, from the live profile
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dp = prof[dom]
    per_launch_ms = dp["ms"] / max(1, dp["launches"])
    bytes_per_launch = dp["bytes"] / max(1, dp["launches"])
    achieved = bytes_per_launch / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    kname = {"thin_run": "k_thin_run", "wide_level": "k_wide_level", "gather": "k_gather",
             "scatter": "k_scatter"}[dom]
    hsched = variants[headline][2]["schedule"]
    if dom == "wide_level" and hsched["mode"] == 3:
        kname = "k_sf_solve"  # the synchronisation-free launch is profiled with the device-wide class
    elif dom == "wide_level" and hsched["mode"] == 4:
        kname = "k_flow_run"  # dataflow runs of the wide levels
    elif dom == "wide_level" and hsched["wide_grid"] > 0:
        kname = "k_wide_run"  # persistent runs of consecutive wide levels
    traffic = load_traffic(kname, f"config{args.config}_{headline}")
    total_prof_ms = sum(v["ms"] for v in prof.values())
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic, "kernel": kname,
                "launches_per_solve": round(dp["launches"] / max(5, min(args.steps, 20)), 3),
                "avg_launch_ms": round(per_launch_ms, 6), "alg_bytes_per_launch": bytes_per_launch,
                "events": "HIP events on the solve stream around every launch of eager solves after the timed region",
                "kernel_share_of_step": round(dp["ms"] / total_prof_ms, 4) if total_prof_ms > 0 else None}
    hinfo = variants[headline][2]
    path = {"alg_bytes_per_solve": hinfo["bytes"], "achieved": round(hinfo["bytes"] / (ms * 1e-3) / 1e9, 3),
            "unit": "GB/s", "frac": round(hinfo["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 6),
            "level_floor_us": round(hinfo["level_floor_us"], 2),
            "ms_over_level_floor": round(ms * 1e3 / hinfo["level_floor_us"], 3) if hinfo["level_floor_us"] > 0 else None}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(oracle, m, b_np, t_oracle_one)

    out_var = {}
    for name, (_, _, info) in variants.items():
        gbs = info["bytes"] / (info["ms"] * 1e-3) / 1e9
        out_var[name] = {"solves_per_s": round(1e3 / info["ms"], 3), "ms": round(info["ms"], 5),
                         "ms_wall_mean": round(info["ms_wall_mean"], 5), "steps": info["steps"],
                         "alg_GBps": round(gbs, 3), "hbm_frac": round(gbs / HBM_PEAK_GBS, 6), "nlev": info["nlev"],
                         "nnz": info["nnz"], "nnz_T": info["nnz_t"], "relerr": info["relerr"],
                         "level_floor_us": round(info["level_floor_us"], 2),
                         "preprocess_s": round(info["preprocess_s"], 3), "autotune_s": round(info["autotune_s"], 3),
                         "schedule": info["schedule"], "tune": info.get("tune"),
                         "us_per_level": round(info["ms"] * 1e3 / max(1, info["nlev"]), 4)}
        if "graph_reps_ms" in info:
            out_var[name]["graph_reps_ms"] = [round(v, 5) for v in info["graph_reps_ms"]]
            out_var[name]["graph_reps_median_ms"] = round(info["graph_reps_median_ms"], 5)
        for k in ("rows_rewritten", "max_distance", "chosen", "relerr_cols"):
            if k in info:
                out_var[name][k] = info[k]
        for k in ("ms_cols", "graph_reps_median_ms_cols"):
            if k in info:
                out_var[name][k] = round(info[k], 5)
    res = {
        "metric": METRIC,
        "value": round(1e3 / ms, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": variants[headline][2]["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator of the workload's structure; no dataset)",
        "config": {"workload": WORKLOADS[args.config], "variant": headline,
                   "chosen": variants[headline][2].get("chosen", headline), "nrhs": nrhs, "n": m.n, "nnz": m.nnz,
                   "layout": ("right-hand sides by rows (n x nrhs row-major)" if layout == "rows"
                              else "right-hand sides by columns (column-major, leading dimension n)"),
                   "parallelism": "single GPU", "timing": ("hipGraph replays" if use_graph else "stream launches")
                   + "; value and ms_per_step from the median of the per-step HIP-event times"},
        "roofline": roofline,
        "path": path,
        "cpu_baseline": cpu,
        "variants": out_var,
        "speedup_vs_plain": round(out_var["plain"]["ms"] / ms, 4) if "plain" in out_var else None,
        "level_costs_ns": {k: round(v, 2) for k, v in costs.items()},
        "kernel_profile": prof,
    }
    print(json.dumps(res), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(oracle, m, b_np, t_one):
    """The serial FP64 oracle on one host core (the calling thread pinned to
    the first core it may run on; restored afterwards): one warm-up solve,
    then the median of five (more, up to about 12 s, when a solve is short)."""
    import statistics
    keep = os.sched_getaffinity(0)
    core = min(keep)
    os.sched_setaffinity(0, {core})
    try:
        oracle.solve(m, b_np)
        reps = max(5, min(201, int(12.0 / max(t_one, 1e-6))))
        if reps % 2 == 0:
            reps += 1
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            oracle.solve(m, b_np)
            times.append(time.perf_counter() - t)
    finally:
        os.sched_setaffinity(0, keep)
    med = statistics.median(times)
    return {"value": round(1.0 / med, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole solve of the same matrix and right-hand side(s) by the serial FP64 oracle, pinned "
                      f"to host core {core}: 1 warm-up, median of {reps} ({med * 1e3:.2f} ms each); host "
                      f"nproc={os.cpu_count()}, CPU {cpu_model()}"}


if __name__ == "__main__":
    main()
