"""Benchmark: LABPSD solves on one MI355X, eigenpairs/s to relative residual 1e-8.

A step is one complete solve (every step of the hot path, iterated to convergence)
of the synthetic PUFE-shaped 64^3-element / 128-atom cell (n = 296,540 dofs,
nev = 512, m0 = 52) from the seeded cold start, with H, S and the global factor
already resident in HBM.  The FP64 solve is the headline value; the
mixed-precision solve (FP32 preconditioner apply and MINRES) is timed the same way
beside it, with its speedup and its per-eigenpair error against the FP64 run and
against the stored ARPACK shift-invert eigenvalues.  A short SCF-like serving
stream follows (p50/p99 request latency), then the CPU oracle's bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload c5|c3|c2] [--no-cpu-baseline]
                    [--no-serving] [--no-mixed]
    python bench.py --serving            # only the SCF-like request stream
    python bench.py --copy-calibration   # plain device copies of known size (counter scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "eigenpairs/s to rel. residual 1e-8, mixed vs FP64; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_MFMA_PEAK_TFS = 78.6      # MI355X dense FP64 matrix, TFLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="serve the SCF-like request stream instead of single solves")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave the short serving stream out of the single-solve line")
    ap.add_argument("--systems", type=int, default=25)
    ap.add_argument("--chain", type=int, default=8)
    ap.add_argument("--rate", type=float, default=4.0, help="system arrivals per second (Poisson)")
    ap.add_argument("--rates", help="comma-separated arrival rates for a sweep (with --serving)")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--ablation", action="store_true",
                    help="global-only / local-only / hybrid preconditioning over SCF-like sequences")
    ap.add_argument("--abl-workload", default="c2nl")
    ap.add_argument("--abl-steps", type=int, default=10)
    ap.add_argument("--no-measured-peaks", action="store_true",
                    help="skip the device copy and DGEMM that measure this GPU's peaks")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 8 plain device copies of 512 MiB (the scale for the HBM byte counters)")
    ap.add_argument("--next-rows", action="store_true",
                    help="eigenpairs/s of the variants on the 15,977-dof cell: plain, one-step refinement, "
                         "FP32 factorisation, nonlocal term, k-point pencil")
    ap.add_argument("--apply-levels", action="store_true",
                    help="time the global apply on --workload with the single-launch sweep and level by level "
                         "(one launch per elimination-tree level and phase)")
    ap.add_argument("--apply-cols", type=int, default=512)
    ap.add_argument("--apply-reps", type=int, default=3)
    ap.add_argument("--summarize-apply-levels", metavar="DIR",
                    help="write the per-level table of a rocprofv3 --kernel-trace run of --apply-levels (to --out)")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="write the kernel table of a rocprofv3 --kernel-trace --stats run (to --out)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "CAL_FETCH", "CAL_WRITE"),
                    help="write HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of the "
                         "workload and of --copy-calibration (to --out)")
    ap.add_argument("--out", help="summary file to write")
    ap.add_argument("--command", default="", help="the profiling command, recorded in the summary")
    return ap.parse_args()


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else float("nan")


def rr_flops(k, nwant):
    """Algorithmic flops of the reduced dense GHEP for its lowest nwant pairs (the LAPACK
    route): Cholesky k^3/3, reduction to standard form k^3, tridiagonalisation 4k^3/3,
    back-transformation of the vectors 2k^2 nwant, triangular solve k^2 nwant."""
    return (8.0 / 3.0) * k ** 3 + 3.0 * k * k * nwant


def spmm_bytes(P, w):
    """Algorithmic bytes of one fused H/S product on w columns: the pattern (int32 columns,
    int64 row offsets) and both FP64 value arrays once, X read once, Y_H and Y_S written."""
    return 4 * P.nnz + 16 * P.nnz + 8 * (P.n + 1) + 8 * P.n * w + 16 * P.n * w


def rr_orders(res_hist, b, tol):
    """Orders k of the Rayleigh-Ritz problems of one solve: the start block (k = b), then
    b + |U| for every iteration that found unconverged pairs."""
    ks = [b]
    for row in res_hist:
        p = int(np.count_nonzero(row > tol))
        if p:
            ks.append(b + p)
    return ks


PROFILE_DIR = os.path.join(ROOT, "profiles")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary
    (profiles/hbm_traffic_<workload>.txt), or None when there is none or the kernel's
    source has changed since the counters were taken."""
    path = os.path.join(PROFILE_DIR, "hbm_traffic_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        if f.get("kernel") != kernel:
            continue
        src = os.path.join(ROOT, f["source"])
        if not os.path.exists(src):
            return None
        if source_digest(src) != f["sha256"]:
            return None
        return float(f["bytes_per_launch"])
    return None


def source_digest(src):
    """sha256 of a kernel's source file followed by the header every kernel source includes
    (the shared device helpers, e.g. the sliced-ELL slot loop, live there)."""
    h = hashlib.sha256(open(src, "rb").read())
    h.update(open(os.path.join(os.path.dirname(src), "common.h"), "rb").read())
    return h.hexdigest()


def measured_peaks():
    """Peaks measured on this GPU beside the published ones: a 1 GiB device copy (bytes
    read + written per second) and an FP64 8192^3 matrix product (the vendor library's
    DGEMM on the matrix cores).  Outside every timed region."""
    import torch
    out = {}
    n = 2 ** 30 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["hbm_copy_GBps"] = 10 * 2 * 8 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    m = 8192
    a = torch.rand((m, m), dtype=torch.float64, device="cuda")
    b = torch.rand((m, m), dtype=torch.float64, device="cuda")
    c = a @ b
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    out["fp64_dgemm_TFLOPs"] = 3 * 2.0 * m ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    out["note"] = ("torch device copy of 1 GiB (read + write) and torch FP64 matmul 8192^3 on this GPU; "
                   "'frac' uses the published peaks, 'frac_of_measured' these")
    del a, b, c
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ rocprofv3 summaries

KERNEL_SOURCES = {"k_block_update": "dense.hip", "k_gram": "dense.hip", "k_residual": "dense.hip",
                  "k_spmm_hs": "spmm.hip", "k_sn_sweep": "precond.hip", "k_minres_spmv": "minres.hip"}


def short_kernel_name(full):
    """'void labpsd::(anonymous namespace)::k_gram<64, 32>(long, ...)' -> 'k_gram<64,32>'."""
    s = full.strip().strip('"')
    if s.startswith("void "):
        s = s[5:]
    s = s.replace("labpsd::(anonymous namespace)::", "").replace("labpsd::", "")
    return s.split("(")[0].replace(" ", "")


def kernel_source(name):
    base = name.split("<")[0]
    for k, f in KERNEL_SOURCES.items():
        if base.startswith(k):
            return "paper_1308_2445_amd/csrc/" + f
    return None


def _csvs(d, suffix):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def summarize_stats(d, out, command):
    import csv
    rows = []
    for path in _csvs(d, "_kernel_stats.csv"):
        for r in csv.DictReader(open(path)):
            rows.append((short_kernel_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                         float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda r: -r[2])
    total = sum(r[2] for r in rows)
    with open(out, "w") as f:
        f.write("# rocprofv3 kernel statistics; durations in microseconds, pct of the total kernel time\n")
        f.write("# command: %s\n#\n" % command)
        f.write("%-44s %8s %14s %12s %7s\n" % ("kernel", "calls", "total_us", "avg_us", "pct"))
        for r in rows[:40]:
            name = r[0] if len(r[0]) <= 44 else r[0][:41] + "..."
            f.write("%-44s %8d %14.1f %12.1f %7.2f\n" % ((name,) + r[1:]))
        f.write("\ntotal kernel time %.1f ms\n" % (total / 1e3))


def _counter_means(d, counter):
    """Mean counter value per dispatch (KiB) of every kernel in a --pmc run."""
    import csv
    acc = {}
    for path in _csvs(d, "_counter_collection.csv"):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            k = short_kernel_name(r["Kernel_Name"])
            v = acc.setdefault(k, [0.0, 0])
            v[0] += float(r["Counter_Value"])
            v[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def summarize_traffic(dirs, out, command):
    fetch, write = _counter_means(dirs[0], "FETCH_SIZE"), _counter_means(dirs[1], "WRITE_SIZE")
    cf, cw = _counter_means(dirs[2], "FETCH_SIZE"), _counter_means(dirs[3], "WRITE_SIZE")
    copy_kib = 512 * 1024   # --copy-calibration: 512 MiB read and written per dispatch
    ff = cf["__amd_rocclr_copyBuffer"][0] / copy_kib
    wf = cw["__amd_rocclr_copyBuffer"][0] / copy_kib
    with open(out, "w") as f:
        f.write("# HBM traffic per launch from rocprofv3 counters, one counter per run\n")
        f.write("# commands: %s\n" % command)
        f.write("# copy calibration: FETCH_SIZE %.1f KiB per 512 MiB copy -> factor %.4f; WRITE_SIZE %.1f KiB -> "
                "factor %.4f\n" % (ff * copy_kib, ff, wf * copy_kib, wf))
        f.write("# bytes_per_launch = (FETCH_SIZE / fetch factor + WRITE_SIZE / write factor) * 1024, mean over the\n"
                "# kernel's dispatches; sha256 is that of the kernel's source file followed by csrc/common.h when\n"
                "# the counters were taken (bench.py reports the figure only while both are unchanged).  FETCH_SIZE\n"
                "# counts L2 fills from the fabric, hits in the MALL included, so it bounds HBM reads from above.\n#\n")
        for k in sorted(set(fetch) & set(write)):
            src = kernel_source(k)
            if src is None:
                continue
            sha = source_digest(os.path.join(ROOT, src))
            by = (fetch[k][0] / ff + write[k][0] / wf) * 1024
            f.write("kernel=%s source=%s sha256=%s dispatches=%d fetch_kib_per_dispatch=%.1f "
                    "write_kib_per_dispatch=%.1f fetch_factor=%.4f write_factor=%.4f bytes_per_launch=%.0f\n"
                    % (k, src, sha, fetch[k][1], fetch[k][0], write[k][0], ff, wf, by))


def next_rows(args):
    """Each variant solved on its 15,977-dof cell (nev 32, m0 4, tol 1e-8, the library's seeded
    start), one warm-up and three timed solves per precision (each solve synchronises;
    wall clock around the call)."""
    import paper_1308_2445_amd as lp
    import pufe
    ctx = lp.Context(0)
    cases = [("plain", "c2", {}), ("one-step refinement", "c2", {"refine": lp.REFINE_ONESTEP}),
             ("FP32 factorisation", "c2", {"panels": lp.FACTOR_FP32}), ("nonlocal term", "c2nl", {}),
             ("k-point", "c2k", {})]
    out = []
    for label, wl, opt in cases:
        P = pufe.workload(wl, 0)
        nev = pufe.WORKLOADS[wl]["nev"]
        m0 = pufe.guard_vectors(nev)
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P), panels=opt.get("panels", 0))
        if "refine" in opt:
            pr.set_refine_method(opt["refine"])
        for prec, pname in ((lp.FP64, "fp64"), (lp.MIXED, "mixed")):
            pr.solve(nev, m0, None, tol=args.tol, sigma0=P.sigma0, precision=prec, seed=1)
            ts, o = [], None
            for _ in range(3):
                t0 = time.perf_counter()
                o = pr.solve(nev, m0, None, tol=args.tol, sigma0=P.sigma0, precision=prec, seed=1)
                ts.append(time.perf_counter() - t0)
            assert o.converged, (label, pname)
            r = {"case": label, "workload": wl, "n": P.n, "precision": pname, "eigenpairs_per_s": nev / np.mean(ts),
                 "ms_per_solve": 1e3 * np.mean(ts), "outer_iters": o.stats["outer_iters"], "la": o.stats["la"]}
            out.append(r)
            print("[next] %-22s %-5s n=%6d: %7.1f eigenpairs/s, %6.1f ms per solve, %d iterations, La %.2f"
                  % (label, pname, P.n, r["eigenpairs_per_s"], r["ms_per_solve"], r["outer_iters"], r["la"]),
                  flush=True)
        pr.close()
    ctx.close()
    print(json.dumps({"next_rows": out}), flush=True)


def apply_levels(args):
    """The global apply of the workload's factor on apply_cols random right-hand sides, in
    both precisions, with the single-launch sweep and with one launch per level and phase
    (HIP events on the current stream, apply_reps applies each after a warm-up)."""
    import torch

    import paper_1308_2445_amd as lp
    import pufe
    P = pufe.workload(args.workload, 0)
    ctx = lp.Context(0)
    coords = pufe.dof_coordinates(P)
    routes = {}
    for name, extra in (("sweep", 0), ("levels", lp.APPLY_LEVELS)):
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, coords, panels=lp.PANELS_FP64 | lp.PANELS_FP32 | extra)
        routes[name] = pr
    fi = routes["sweep"].factor_info()
    rng = np.random.default_rng(5)
    R = torch.from_numpy(rng.standard_normal((args.apply_cols, P.n))).cuda()
    out = {"workload": args.workload, "n": P.n, "cols": args.apply_cols, "levels": fi["n_levels"],
           "supernodes": fi["n_supernodes"], "nnz_factor": fi["nnz_factor"], "ms": {}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for prec, pname in ((lp.FP64, "fp64"), (lp.MIXED, "fp32")):
        for name, pr in routes.items():
            Pd = torch.empty_like(R)
            lp.labpsd_precond_apply(pr, prec, R, Pd)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.apply_reps):
                lp.labpsd_precond_apply(pr, prec, R, Pd)
            e1.record()
            torch.cuda.synchronize()
            out["ms"]["%s_%s" % (pname, name)] = e0.elapsed_time(e1) / args.apply_reps
            print("[apply] %s %s: %.2f ms per apply of %d columns" % (pname, name, out["ms"]["%s_%s" % (pname, name)],
                                                                   args.apply_cols), flush=True)
    for pr in routes.values():
        pr.close()
    ctx.close()
    print(json.dumps({"apply_levels": out}), flush=True)


def summarize_apply_levels(d, out, command):
    """Per-level table of the level-by-level applies in a kernel trace: the k_sn_product
    dispatches of one apply run forward (leaves first), diagonal, backward (root first)."""
    import csv
    rows = []
    for path in _csvs(d, "_kernel_trace.csv"):
        for r in csv.DictReader(open(path)):
            nm = short_kernel_name(r["Kernel_Name"])
            if nm.startswith("k_sn_product") or nm.startswith("k_sn_sweep"):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), nm, int(r["Grid_Size_X"]),
                             int(r["Grid_Size_Y"])))
    rows.sort()
    # split into applies: a forward product after a backward one (or a sweep) starts a new apply
    applies, cur, last = [], [], None
    for r in rows:
        kind = r[2]
        if cur and (kind.startswith("k_sn_sweep") or (kind.endswith(",2>") and last is not None
                                                      and last.endswith(",3>"))):
            applies.append(cur)
            cur = []
        cur.append(r)
        last = kind
        if kind.startswith("k_sn_sweep"):
            applies.append(cur)
            cur, last = [], None
    if cur:
        applies.append(cur)
    with open(out, "w") as f:
        f.write("# global apply per elimination-tree level (one launch per level and phase), rocprofv3 kernel trace\n")
        f.write("# command: %s\n#\n" % command)
        seen = set()
        for ap in applies:
            kinds = {r[2] for r in ap}
            key = tuple(sorted(kinds))
            if key in seen:
                continue   # the first apply of each route and precision (the warm-up)
            seen.add(key)
            tot = sum(r[1] - r[0] for r in ap) / 1e3
            span = (ap[-1][1] - ap[0][0]) / 1e3
            typ = ap[0][2].split("<")[1].split(",")[0]
            if ap[0][2].startswith("k_sn_sweep"):
                f.write("%s single-launch sweep: %.1f us (%d work-groups)\n\n" % (typ, tot, ap[0][3] // 256))
                continue
            f.write("%s level by level: %d launches, %.1f us of kernels, %.1f us first start to last end\n"
                    % (typ, len(ap), tot, span))
            f.write("%-10s %6s %10s %12s %8s\n" % ("phase", "step", "tasks", "us", "pct"))
            fi = bi = 0
            for r in ap:
                op = r[2].rstrip(">").split(",")[-1]
                phase = {"2": "forward", "0": "diagonal", "3": "backward"}[op]
                if op == "2":
                    step, fi = fi, fi + 1
                elif op == "3":
                    step, bi = bi, bi + 1
                else:
                    step = 0
                us = (r[1] - r[0]) / 1e3
                f.write("%-10s %6d %10d %12.1f %8.2f\n" % (phase, step, r[3] // 256, us, 100 * us / tot))
            f.write("(forward steps count up from the leaves, backward steps down from the root; tasks = work-groups "
                    "per right-hand-side group)\n\n")


def block_update_ct(b):
    """MFMA tiles per wavefront of the wide block update for b output columns: the width
    16 CT (CT in 9, 8, 6) that pads b the least, then the fewest column groups (the
    library's own choice, repeated here to name the kernel)."""
    best, cost = 8, None
    for ct in (9, 8, 6):
        g = (b + 16 * ct - 1) // (16 * ct)
        c = (g * 16 * ct - b) * 4 + g
        if cost is None or c < cost:
            best, cost = ct, c
    return best


def copy_calibration():
    """Plain device-to-device copies of a known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = 512 * 2 ** 20 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(8):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_dispatch": 8 * n, "bytes_written_per_dispatch": 8 * n,
                                           "dispatches": 8}}), flush=True)


def serving(args, ctx=None):
    """SCF-like stream: systems arrive as a Poisson process; each is a chain of GHEPs
    whose potential drifts by up to 1% per step, every step warm-started from the last.
    Returns the stream's figures (eigenpairs/s over the makespan, request latency)."""
    import torch

    import paper_1308_2445_amd as lp
    import pufe
    rng = np.random.default_rng(2024)
    t0 = time.perf_counter()
    pencils = []
    for i in range(args.systems):
        ne = int(rng.choice([12, 16, 24, 32]))
        na = int(rng.integers(1, 17))
        nev = int(rng.choice([8, 16, 32, 64]))
        P = pufe.generate(ne / 2.0, ne, na, 100 + i)
        scales = np.cumprod(1.0 + rng.uniform(-0.01, 0.01, args.chain))
        pencils.append((P, nev, scales))
    t_gen = time.perf_counter() - t0
    own_ctx = ctx is None
    if own_ctx:
        ctx = lp.Context(0)
    systems = []
    t0 = time.perf_counter()
    for P, nev, _ in pencils:
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P), panels=lp.PANELS_FP32)
        systems.append(pr)
    t_setup = time.perf_counter() - t0
    print("[serve] %d systems generated in %.1fs, factorised in %.1fs" % (len(systems), t_gen, t_setup),
          flush=True)
    rates = [float(r) for r in args.rates.split(",")] if getattr(args, "rates", None) else [args.rate]
    gaps = rng.exponential(1.0, args.systems)   # unit-rate gaps; each rate scales the same draws
    results = []
    for rate in rates:
        arrivals = np.cumsum(gaps / rate)
        results.append(_serve_stream(args, lp, pufe, torch, ctx, pencils, systems, arrivals, rate))
    for pr in systems:
        pr.close()
    if own_ctx:
        ctx.close()
    if len(results) == 1:
        return results[0]
    out = dict(results[0])
    out["sweep"] = results
    return out


def _serve_stream(args, lp, pufe, torch, ctx, pencils, systems, arrivals, rate):
    """One Poisson stream over the resident systems: every system's chain of SCF-like steps,
    each step submitted when the previous one completes."""
    srv = lp.Server(ctx, int(args.budget_gb * 2 ** 30), args.slots)
    torch.cuda.synchronize()
    start = time.perf_counter()
    outstanding = {}            # request id -> (system index, step)
    nxt = 0
    done = []
    while len(done) < args.systems * args.chain:
        now = time.perf_counter() - start
        while nxt < args.systems and arrivals[nxt] <= now:
            P, nev, sc = pencils[nxt]
            m0 = pufe.guard_vectors(nev)
            rid = srv.submit(systems[nxt], nev, m0, X0=pufe.start_block(P.n, nev + m0, nxt),
                             h_val=P.h_scaled(sc[0]), tol=args.tol, sigma0=P.sigma0, precision=lp.MIXED)
            outstanding[rid] = (nxt, 0)
            nxt += 1
        for rid in list(outstanding):
            r = srv.poll(rid)
            if r is None:
                continue
            i, j = outstanding.pop(rid)
            assert r.converged, "a served solve did not converge"
            done.append((i, j, r))
            if j + 1 < args.chain:
                P, nev, sc = pencils[i]
                m0 = pufe.guard_vectors(nev)
                rid2 = srv.submit(systems[i], nev, m0, h_val=P.h_scaled(sc[j + 1]), tol=args.tol,
                                  sigma0=P.sigma0, precision=lp.MIXED)
                outstanding[rid2] = (i, j + 1)
        time.sleep(0.0005)
    makespan = time.perf_counter() - start
    torch.cuda.synchronize()
    mem = srv.memory()
    srv.close()
    lat = [r.latency for _, _, r in done]
    pairs = sum(pencils[i][1] for i, _, _ in done)
    print("[serve] rate %.1f/s: %.1f eigenpairs/s, p50 %.1f ms, p99 %.1f ms" % (
        rate, pairs / makespan, 1e3 * percentile(lat, 50), 1e3 * percentile(lat, 99)), flush=True)
    return {"value": pairs / makespan, "unit": "eigenpairs/s", "requests": len(done),
            "makespan_s": makespan, "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
            "memory_bytes": {"budget": int(args.budget_gb * 2 ** 30), "held_at_end": mem["held"],
                             "peak": mem["peak"]},
            "workload": "%d systems x %d SCF-like steps, meshes 12-32^3 at h=0.5, 1-16 atoms, nev 8-64, "
                        "Poisson arrivals %.1f/s, mixed precision, %d slots"
                        % (args.systems, args.chain, rate, args.slots),
            "iterations_cold_warm": [float(np.mean([r.stats["outer_iters"] for _, j, r in done if j == 0])),
                                     float(np.mean([r.stats["outer_iters"] for _, j, r in done if j > 0]))]}


def serving_line(args):
    sv = serving(args)
    line = {"metric": METRIC, "value": sv["value"], "unit": "eigenpairs/s", "n_gpus": 1,
            "steps": sv["requests"], "warmup": 0, "ms_per_step": 1e3 * sv["makespan_s"] / sv["requests"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
            "data": "synthetic", "config": {"workload": "serving: " + sv["workload"]},
            "latency_ms": {"p50": sv["p50_ms"], "p99": sv["p99_ms"]},
            "iterations_cold_warm": sv["iterations_cold_warm"], "makespan_s": sv["makespan_s"]}
    print(json.dumps(line), flush=True)


def ablation(args):
    """Section 5.4's comparison on synthetic SCF-like sequences: the same chain of GHEPs
    (potential amplitudes drifting by up to 1% per step, every step warm-started from the
    previous one's resident block and Ritz values) solved with the global preconditioner
    only (step 6(a); outer cap 200), the local one only (localised pairs refined by MINRES
    from zero; outer cap 100, MINRES cap 500; the first, cold step global only, as the
    paper's footnote does until pairs localise) and the hybrid scheme (caps 200 / 20); and
    the hybrid scheme again with a global factor computed in single precision (the
    conclusions' suggestion).  Reports Hp, La, stalled steps and the chain's time."""
    import torch

    import paper_1308_2445_amd as lp
    import pufe
    P = pufe.workload(args.abl_workload, 0)
    nev = pufe.WORKLOADS[args.abl_workload]["nev"]
    m0 = pufe.guard_vectors(nev)
    rng = np.random.default_rng(77)
    scales = np.cumprod(1.0 + rng.uniform(-0.01, 0.01, args.abl_steps))
    ctx = lp.Context(0)
    # eps_bar: the default reading (V_min - 0.1, far below the wanted pairs); "global_near"
    # repeats global-only with eps_bar just below lambda_1 (from the hybrid run's first step)
    configs = [("hybrid", lp.HYBRID, 200, 20, 0, None), ("global", lp.GLOBAL_ONLY, 200, 20, 0, None),
               ("global_near", lp.GLOBAL_ONLY, 200, 20, 0, "near"), ("local", lp.LOCAL_ONLY, 100, 500, 0, None),
               ("hybrid_fp32_factor", lp.HYBRID, 200, 20, lp.FACTOR_FP32, None)]
    out = {"workload": "%s: n=%d, nev=%d, m0=%d, %s, %d SCF-like steps (amplitude drift <= 1%%/step), tol %g, "
                       "mixed precision" % (args.abl_workload, P.n, nev, m0,
                                            "k=%d projectors" % P.F.shape[1] if P.F is not None else "local V only",
                                            args.abl_steps, args.tol), "modes": {}}
    ref_lam = None
    lam1 = None
    for name, mode, cap_outer, cap_inner, fmask, shift in configs:
        pr = lp.Problem.from_pencil(ctx, P)
        t0 = time.perf_counter()
        eps_bar = P.eps_bar if shift is None else lam1 - 0.1
        pr.set_global_precond(eps_bar, pufe.dof_coordinates(P), panels=lp.PANELS_FP32 | fmask)
        t_fac = time.perf_counter() - t0
        srv = lp.Server(ctx, 1 << 40, 1)
        steps = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(args.abl_steps):
            # the cold step of the local-only run uses the global preconditioner (paper's footnote)
            pr.set_local_precond(mode=lp.GLOBAL_ONLY if (mode == lp.LOCAL_ONLY and j == 0) else mode,
                                 max_inner=cap_inner)
            rid = srv.submit(pr, nev, m0, X0=pufe.start_block(P.n, nev + m0, 0) if j == 0 else None,
                             h_val=P.h_scaled(scales[j]), tol=args.tol, max_outer=cap_outer, sigma0=P.sigma0,
                             precision=lp.MIXED)
            r = srv.wait(rid)
            steps.append(dict(outer=r.stats["outer_iters"], minres=r.stats["minres_iters"],
                              converged=bool(r.converged), seconds=r.finished - r.started, lam=r.lam))
        t_chain = time.perf_counter() - t0
        srv.close()
        pr.close()
        outer = sum(st["outer"] for st in steps)
        minres = sum(st["minres"] for st in steps)
        lam_last = steps[-1]["lam"]
        if name == "hybrid":
            ref_lam = lam_last
            lam1 = float(steps[0]["lam"][0])
        rec = {"Hp": outer / len(steps), "La": minres / max(1, outer * nev), "outer_per_step": [st["outer"] for st in steps],
               "minres_per_step": [st["minres"] for st in steps],
               "stalled_steps": sum(1 for st in steps if not st["converged"]), "chain_s": t_chain,
               "factor_s": t_fac, "warm_Hp": float(np.mean([st["outer"] for st in steps[1:]])) if len(steps) > 1 else None,
               "eps_bar": eps_bar}
        if name != "hybrid" and steps[-1]["converged"]:
            rec["last_step_max_rel_diff_vs_hybrid"] = float(np.max(np.abs(lam_last - ref_lam) / np.abs(ref_lam - P.sigma0)))
        out["modes"][name] = rec
        print("[ablation] %s: Hp %.2f (warm %.2f) La %.2f stalled %d chain %.2fs factor %.1fs" % (
            name, rec["Hp"], rec["warm_Hp"] or 0, rec["La"], rec["stalled_steps"], t_chain, t_fac), flush=True)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"ablation": out}), flush=True)


def golden_lam(name):
    """Stored eigenvalues of an independent CPU route for this workload (ARPACK shift-invert
    Lanczos, written by tests/golden/make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "%s_eigs.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    lam = g.get("lam_eigsh", g.get("lam"))
    return None if lam is None else (np.asarray(lam), g)


def err_stats(lam, ref, sigma0):
    d = np.abs(np.asarray(lam) - np.asarray(ref)) / np.abs(np.asarray(ref) - sigma0)
    return {"max": float(d.max()), "median": float(np.median(d))}


def rooflines(P, agg, b, hbm_peak, fp64_peak):
    """Per-launch rooflines of the single-kernel steps, from the step events recorded on
    the solver's stream over the instrumented solve.  Algorithmic work per launch:
      block update   6 n k b flops (Psi, Psi_H, Psi_S = [.] W, k the search-space width)
      Gram           2 n k (k + 1) flops (upper triangles of H_R and S_R)
      H/S products   20 nnz + 8 (n + 1) + 24 n w bytes (pattern and both value arrays once,
                     X read once, Y_H and Y_S written; w columns)
    k, w: the summed column counts of each step over its launches."""
    out = {}
    t, nl, cols = agg["t"], agg["n_launch"], agg["cols"]
    n = P.n
    if nl["block_update"]:
        fl = 6.0 * n * b * cols["block_update"]
        out["block_update"] = dict(kernel="k_block_update_wide<%d>" % block_update_ct(b) if b >= 96
                                   else "k_block_update",
                                   bound="mfma", unit="TFLOP/s", peak=fp64_peak, launches=int(nl["block_update"]),
                                   avg_launch_us=1e6 * t["block_update"] / nl["block_update"],
                                   algorithmic_flops_per_launch=fl / nl["block_update"],
                                   achieved=fl / t["block_update"] / 1e12)
    if nl["gram"]:
        # k(k+1) summed over launches needs the individual widths: the refreshes use b, the
        # iterations b + p; the mean width reproduces sum k within rounding of sum k^2
        kk = agg["gram_kk"]
        fl = 2.0 * n * kk
        out["gram"] = dict(kernel=("k_gram<64,32>" if b >= 192 else "k_gram<32,64>") + " (+ k_gram_reduce)",
                           bound="mfma", unit="TFLOP/s", peak=fp64_peak,
                           launches=int(nl["gram"]), avg_launch_us=1e6 * t["gram"] / nl["gram"],
                           algorithmic_flops_per_launch=fl / nl["gram"], achieved=fl / t["gram"] / 1e12)
    nl_pp = nl["products_p"] + nl["products_psi"]
    if nl_pp:
        tp = t["products_p"] + t["products_psi"]
        by = nl_pp * (20.0 * P.nnz + 8.0 * (n + 1)) + 24.0 * n * (cols["products_p"] + cols["products_psi"])
        out["spmm"] = dict(kernel="k_spmm_hs<4>", bound="hbm", unit="GB/s", peak=hbm_peak, launches=int(nl_pp),
                           avg_launch_us=1e6 * tp / nl_pp, algorithmic_bytes_per_launch=by / nl_pp,
                           achieved=by / tp / 1e9)
    for r in out.values():
        r["frac"] = r["achieved"] / r["peak"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); %d GPUs were requested" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving_line(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.apply_levels:
        apply_levels(args)
        return
    if args.next_rows:
        next_rows(args)
        return
    if args.summarize_apply_levels:
        summarize_apply_levels(args.summarize_apply_levels, args.out, args.command)
        return
    if args.summarize_stats:
        summarize_stats(args.summarize_stats, args.out, args.command)
        return
    if args.summarize_traffic:
        summarize_traffic(args.summarize_traffic, args.out, args.command)
        return
    if args.ablation:
        ablation(args)
        return
    import torch

    import paper_1308_2445_amd as lp
    import pufe

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = pufe.WORKLOADS[args.workload]
    nev = w["nev"]
    m0 = pufe.guard_vectors(nev)
    b = nev + m0
    t0 = time.perf_counter()
    P = pufe.workload(args.workload, 0)
    t_gen = time.perf_counter() - t0
    print("[bench] workload %s n=%d nnz=%d nev=%d m0=%d (generated in %.1fs)" % (args.workload, P.n, P.nnz,
                                                                              nev, m0, t_gen), flush=True)
    ctx = lp.Context(0)
    pr = lp.Problem.from_pencil(ctx, P)
    t0 = time.perf_counter()
    pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
    t_setup = time.perf_counter() - t0
    fi = pr.factor_info()
    print("[bench] global factor: %d supernodes, %d levels, nnz(L)=%.3e, order %.2fs factor %.2fs upload %.2fs"
          % (fi["n_supernodes"], fi["n_levels"], fi["nnz_factor"], fi["t_order_s"], fi["t_factor_s"],
             fi["t_upload_s"]), flush=True)
    X0 = torch.from_numpy(np.ascontiguousarray(pufe.start_block(P.n, b, 0).T)).cuda()

    def run(precision, steps, timing):
        lat, outs = [], []
        agg = None
        for _ in range(steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = pr.solve(nev, m0, X0, tol=args.tol, sigma0=P.sigma0, precision=precision, timing=timing,
                           device_out=True)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t)
            outs.append(out)
            st = out.stats
            # Gram widths: the start block (b), every iteration's b + p, every refresh (b)
            ks = rr_orders(out.res_hist.cpu().numpy(), b, args.tol)
            kk = sum(k * (k + 1) for k in ks) + (st["n_launch"]["gram"] - len(ks)) * b * (b + 1)
            if agg is None:
                agg = {"t": dict(st["t_step_s"]), "n_launch": dict(st["n_launch"]),
                       "cols": dict(st["cols"]), "gram_kk": 0.0}
            else:
                for k in agg["t"]:
                    agg["t"][k] += st["t_step_s"][k]
                    agg["n_launch"][k] += st["n_launch"][k]
                    agg["cols"][k] += st["cols"][k]
            agg["gram_kk"] += kk
        return lat, outs, agg

    modes = [("fp64", lp.FP64)] + ([] if args.no_mixed else [("mixed", lp.MIXED)])
    results = {}
    for name, prec in modes:
        for _ in range(args.warmup):
            run(prec, 1, False)
        lat, outs, _ = run(prec, args.steps, False)
        assert all(o.converged for o in outs), "a timed solve did not converge"
        # the per-step device times (HIP events around every step, whose recording and
        # read-back cost host time on small cells) come from one more solve after the timed ones
        _, touts, agg = run(prec, 1, True)
        assert touts[0].converged
        tot = sum(lat)
        results[name] = dict(lat=lat, outs=outs, agg=agg, agg_solves=1, value=args.steps * nev / tot,
                             ms=1e3 * tot / args.steps, stats0=outs[0].stats)
        print("[bench] %s: %.1f eigenpairs/s, %.2f ms/solve, iterations %d, La %.2f" % (
            name, results[name]["value"], results[name]["ms"], outs[0].stats["outer_iters"],
            outs[0].stats["la"]), flush=True)

    f = results["fp64"]
    agg = f["agg"]
    steps_ms = {k: 1e3 * v / f["agg_solves"] for k, v in agg["t"].items()}
    rl = rooflines(P, agg, b, HBM_PEAK_GBS, FP64_MFMA_PEAK_TFS)
    # the roofline of the kernel with the largest share of the solve: the MFMA-bound block
    # update or Gram (one launch per step, timed per launch by the step events)
    dom = max(("block_update", "gram"), key=lambda k: agg["t"][k] if k in rl else -1.0)
    roofline = dict(rl[dom])
    for r in rl.values():
        r["traffic"] = measured_traffic(r["kernel"].split(" ")[0], args.workload)
    roofline["traffic"] = rl[dom]["traffic"]
    roofline["share_of_fp64_solve"] = agg["t"][dom] / (f["ms"] * 1e-3 * f["agg_solves"])
    lam64 = f["outs"][0].lam.cpu().numpy()
    gold = golden_lam(args.workload)
    line = {
        "metric": METRIC, "value": f["value"], "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "PUFE-shaped periodic cell L=%g bohr, %d^3 trilinear elements, %d atoms, "
                               "n=%d, nnz=%d; nev=%d, m0=%d, tol=%g, FP64, cold start seed 0"
                               % (P.L, P.ne, len(P.atoms), P.n, P.nnz, nev, m0, args.tol),
                   "n": P.n, "nnz": P.nnz, "nev": nev, "m0": m0, "tol": args.tol, "precision": "fp64"},
        "latency_ms": {"p50": 1e3 * percentile(f["lat"], 50), "p99": 1e3 * percentile(f["lat"], 99)},
        "iterations": f["outs"][0].stats["outer_iters"], "la": f["outs"][0].stats["la"],
        "rank_dropped": f["outs"][0].stats["rank_dropped"],
        "device": {"name": torch.cuda.get_device_name(0)},
        "steps_ms_per_solve": steps_ms,
        "setup_s": {"generate": t_gen, "factor_total": t_setup, "order": fi["t_order_s"],
                    "factor": fi["t_factor_s"], "upload": fi["t_upload_s"], "nnz_factor": fi["nnz_factor"]},
        "roofline": roofline,
        "rooflines": rl,
    }
    if gold is not None:
        line["fp64_error_vs_cpu_route"] = err_stats(lam64, gold[0], P.sigma0)
        line["fp64_error_vs_cpu_route"]["route"] = gold[1].get("eigsh_route", gold[1].get("route"))
    if "mixed" in results:
        mx = results["mixed"]
        lam32 = mx["outs"][0].lam.cpu().numpy()
        line["mixed"] = {"value": mx["value"], "ms_per_step": mx["ms"],
                         "p50_ms": 1e3 * percentile(mx["lat"], 50), "p99_ms": 1e3 * percentile(mx["lat"], 99),
                         "speedup_vs_fp64": mx["value"] / f["value"],
                         "iterations": mx["outs"][0].stats["outer_iters"],
                         "steps_ms_per_solve": {k: 1e3 * v / mx["agg_solves"] for k, v in mx["agg"]["t"].items()},
                         "per_eigenpair_error_vs_fp64": err_stats(lam32, lam64, P.sigma0)}
        if gold is not None:
            line["mixed"]["per_eigenpair_error_vs_cpu_route"] = err_stats(lam32, gold[0], P.sigma0)
    # release every library resource before the process tears down the runtime
    for r in results.values():
        r["outs"].clear()
    del X0
    torch.cuda.synchronize()
    pr.close()
    if not args.no_measured_peaks:
        try:
            mp = measured_peaks()
            line["measured_peaks"] = mp
            line["roofline"]["frac_of_measured"] = roofline["achieved"] / mp["fp64_dgemm_TFLOPs"]
        except Exception as exc:   # the peaks are context; the line is printed regardless
            line["measured_peaks"] = {"error": str(exc)}
    if not args.no_serving:
        sv = serving(args, ctx)
        line["serving"] = sv
        line["serving_p50_ms"] = sv["p50_ms"]
        line["serving_p99_ms"] = sv["p99_ms"]
    torch.cuda.synchronize()
    ctx.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, nev, m0, args.tol, f["stats0"])
    print(json.dumps(line), flush=True)


def cpu_baseline(P, nev, m0, tol, gpu_stats):
    """The oracle, as it stands, on the host cores, on a bounded sample of this workload,
    extrapolated to one solve.

    Small cells (n <= 20000): one full cold-start oracle solve (its SuperLU factorisation
    timed apart and excluded, as the GPU's host factorisation is).  Larger cells: the
    oracle's own step functions on the full pencil, one of each at the first iteration's
    width -- residual, Gram, Rayleigh-Ritz, block update -- plus the H/S products of a
    64-column sample and MINRES iterations on one column, scaled to the widths and MINRES
    counts of the GPU FP64 run, times its outer iteration count.  The global apply is NOT
    in that sample: the oracle's SuperLU factorisation of a pencil this size takes more than
    five minutes on its single thread, so the extrapolated value is an upper bound of the
    oracle's throughput."""
    from oracle import labpsd as olab
    from oracle import precond as oprec
    from oracle import rr as orr
    import pufe
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    H, S = P.H(), P.S()
    b = nev + m0
    if P.n <= 20000:
        t0 = time.perf_counter()
        K = oprec.GlobalPreconditioner(H, S, P.eps_bar)
        t_fac = time.perf_counter() - t0
        prm = olab.Params(nev=nev, m0=m0, tol=tol, sigma0=P.sigma0, eps_bar=P.eps_bar)
        res = olab.solve(H, S, prm, pufe.start_block(P.n, b, 0), precond=K)
        return {"value": nev / res.t_solve, "unit": "eigenpairs/s", "cores": int(cores), "kind": "oracle",
                "sample": "one full oracle solve of the same workload (%d outer iterations, %.1fs); "
                          "its sparse factorisation (%.1fs, single-threaded SuperLU) excluded"
                          % (res.outer_iters, res.t_solve, t_fac)}
    hp = max(1, int(gpu_stats["outer_iters"]))
    p = nev                                   # the first iterations precondition every wanted column
    k = b + p
    minres_its = float(gpu_stats["minres_iters"])
    rng = np.random.default_rng(5)
    t = {}
    X0 = pufe.start_block(P.n, b, 0)
    t0 = time.perf_counter()
    E, Psi, PsiH, PsiS = olab.initial_rr(H, S, X0, b)
    t["initial_rr"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    R, res = olab.residual_block(PsiH, PsiS, E, nev, P.sigma0)
    t["residual"] = time.perf_counter() - t0
    ws = 64
    Pw = rng.standard_normal((P.n, ws))
    t0 = time.perf_counter()
    PH, PS = H @ Pw, S @ Pw
    t["products"] = (time.perf_counter() - t0) * p / ws
    Pfull = np.asfortranarray(np.tile(Pw, (1, p // ws + 1))[:, :p])
    Z = np.hstack([Psi, Pfull])
    ZH = np.hstack([PsiH, np.tile(PH, (1, p // ws + 1))[:, :p]])
    ZS = np.hstack([PsiS, np.tile(PS, (1, p // ws + 1))[:, :p]])
    del Pfull
    t0 = time.perf_counter()
    HR, SR = orr.gram(Z, ZH, ZS)
    t["gram"] = time.perf_counter() - t0
    # a full-rank reduced pencil of the same order for the timing of the dense solve
    G = rng.standard_normal((k, k))
    SRt = G @ G.T + k * np.eye(k)
    t0 = time.perf_counter()
    gam, W, _ = orr.rayleigh_ritz(0.5 * (HR + HR.T), SRt, b)
    t["rayleigh_ritz"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = (Z @ W, ZH @ W, ZS @ W)
    t["update"] = time.perf_counter() - t0
    del Z, ZH, ZS, _
    t0 = time.perf_counter()
    inner = 3
    _, its = olab.local_refine(H, S, np.zeros(P.n), R[:, 0], float(E[0]), 1e-300, inner)
    t_m = (time.perf_counter() - t0) / max(1, its)
    t["minres_per_inner_iteration"] = t_m
    per_iter = t["residual"] + t["products"] + t["gram"] + t["rayleigh_ritz"] + t["update"]
    total = t["initial_rr"] + hp * per_iter + minres_its * t_m
    return {"value": nev / total, "unit": "eigenpairs/s", "cores": int(cores), "kind": "oracle",
            "extrapolated": True, "upper_bound": True,
            "step_seconds": t,
            "sample": ("extrapolated: the oracle's step functions on the full %d-dof pencil, one each at the "
                       "first iteration's width k = %d (residual, Gram, Rayleigh-Ritz, block update), H/S "
                       "products of a %d-column sample scaled to %d columns, one column's MINRES iterations "
                       "scaled to the GPU FP64 run's %d; times its %d outer iterations, plus the initial "
                       "Rayleigh-Ritz step. The global apply is not sampled (the oracle's SuperLU "
                       "factorisation of this pencil runs more than 5 minutes single-threaded), so the value "
                       "is an upper bound of the oracle's rate. Sampled CPU work %.1f s."
                       % (P.n, k, ws, p, int(minres_its), hp, sum(v for kk, v in t.items()
                                                                     if kk != "minres_per_inner_iteration")))}


if __name__ == "__main__":
    main()
