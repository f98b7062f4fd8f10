"""Benchmark: LABPSD solves on one MI355X, eigenpairs/s to relative residual 1e-8.

A step is one complete solve (every step of the hot path, iterated to convergence)
of the synthetic PUFE-shaped 24^3-element / 8-atom cell (n = 15,977 dofs, nev = 32,
m0 = 4) from the seeded cold start, with H, S and the global factor already resident
in HBM.  The FP64 solve is the headline value; the mixed-precision solve (FP32
preconditioner) is timed the same way beside it.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--no-cpu-baseline]
    python bench.py --serving            # SCF-like request stream
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
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="serve the SCF-like request stream instead of single solves")
    ap.add_argument("--systems", type=int, default=25)
    ap.add_argument("--chain", type=int, default=8)
    ap.add_argument("--rate", type=float, default=4.0, help="system arrivals per second (Poisson)")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 8 plain device copies of 512 MiB (the scale for the HBM byte counters)")
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


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when
    there is none or the kernel's source has changed since the counters were taken."""
    path = os.path.join(PROFILE_DIR, "hbm_traffic_c2.txt")
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
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
            return None
        return float(f["bytes_per_launch"])
    return None


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


def serving(args):
    """SCF-like stream: systems arrive as a Poisson process; each is a chain of GHEPs
    whose potential drifts by up to 1% per step, every step warm-started from the last."""
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
    ctx = lp.Context(0)
    systems = []
    t0 = time.perf_counter()
    for P, nev, _ in pencils:
        pr = lp.Problem.from_pencil(ctx, P)
        pr.set_global_precond(P.eps_bar, pufe.dof_coordinates(P))
        systems.append(pr)
    t_setup = time.perf_counter() - t0
    print("[serve] %d systems generated in %.1fs, factorised in %.1fs" % (len(systems), t_gen, t_setup),
          flush=True)
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, args.systems))
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
    srv.close()
    lat = [r.latency for _, _, r in done]
    pairs = sum(pencils[i][1] for i, _, _ in done)
    line = {"metric": METRIC, "value": pairs / makespan, "unit": "eigenpairs/s", "n_gpus": 1,
            "steps": len(done), "warmup": 0, "ms_per_step": 1e3 * makespan / len(done), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "serving: %d systems x %d SCF-like steps, meshes 12-32^3 at h=0.5, 1-16 "
                                   "atoms, nev 8-64, Poisson arrivals %.1f/s, mixed precision, %d slots"
                                   % (args.systems, args.chain, args.rate, args.slots)},
            "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99)},
            "iterations_cold_warm": [float(np.mean([r.stats["outer_iters"] for _, j, r in done if j == 0])),
                                     float(np.mean([r.stats["outer_iters"] for _, j, r in done if j > 0]))],
            "makespan_s": makespan}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); %d GPUs were requested" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
        return
    if args.copy_calibration:
        copy_calibration()
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
            ks = rr_orders(out.res_hist.cpu().numpy(), b, args.tol)
            nrr, krr = st["n_launch"]["rayleigh_ritz"], st["cols"]["rayleigh_ritz"]
            if len(ks) != nrr or sum(ks) != krr:
                # the history does not resolve the orders: use their mean
                print("[bench] Rayleigh-Ritz orders from the history disagree with the counters; "
                      "using the mean order", file=sys.stderr, flush=True)
                ks = [krr / max(1, nrr)] * nrr
            if agg is None:
                agg = {"t": dict(st["t_step_s"]), "n_launch": dict(st["n_launch"]),
                       "cols": dict(st["cols"]), "applies": st["outer_iters"], "rr_flops": 0.0}
            else:
                for k in agg["t"]:
                    agg["t"][k] += st["t_step_s"][k]
                    agg["n_launch"][k] += st["n_launch"][k]
                    agg["cols"][k] += st["cols"][k]
                agg["applies"] += st["outer_iters"]
            agg["rr_flops"] += sum(rr_flops(k, b) for k in ks)
        return lat, outs, agg

    modes = [("fp64", lp.FP64)] + ([] if args.no_mixed else [("mixed", lp.MIXED)])
    results = {}
    for name, prec in modes:
        for _ in range(args.warmup):
            run(prec, 1, True)
        lat, outs, agg = run(prec, args.steps, True)
        assert all(o.converged for o in outs), "a timed solve did not converge"
        tot = sum(lat)
        results[name] = dict(lat=lat, outs=outs, agg=agg, value=args.steps * nev / tot,
                             ms=1e3 * tot / args.steps)
        print("[bench] %s: %.1f eigenpairs/s, %.2f ms/solve, iterations %d, La %.2f" % (
            name, results[name]["value"], results[name]["ms"], outs[0].stats["outer_iters"],
            outs[0].stats["la"]), flush=True)

    f = results["fp64"]
    agg = f["agg"]
    steps_ms = {k: 1e3 * v / args.steps for k, v in agg["t"].items()}
    # Roofline of the dominant kernel.  Steps that are one kernel launch each are timed
    # per launch by the step events on the solver's stream: k_rayleigh_ritz (one per
    # Rayleigh-Ritz step) dominates them; k_spmm_hs (the P and Psi products) is the
    # dominant HBM-bound one.
    nl_rr = max(1, agg["n_launch"]["rayleigh_ritz"])
    t_rr = agg["t"]["rayleigh_ritz"] / nl_rr
    rr_achieved = agg["rr_flops"] / nl_rr / t_rr / 1e12
    roofline = {"bound": "mfma", "kernel": "k_rayleigh_ritz", "achieved": rr_achieved,
                "peak": FP64_MFMA_PEAK_TFS, "unit": "TFLOP/s", "frac": rr_achieved / FP64_MFMA_PEAK_TFS,
                "traffic": measured_traffic("k_rayleigh_ritz"),
                "launches": int(nl_rr), "avg_launch_us": 1e6 * t_rr,
                "algorithmic_flops_per_launch": agg["rr_flops"] / nl_rr,
                "note": ("one work-group solving the reduced pencil of order k <= %d: latency-bound "
                         "(dependent steps and barriers), not throughput-bound" % (b + nev)) if b + nev <= 128 else
                        ("reduced pencil of order k <= %d: orders above 128 run as a sequence of "
                         "many-work-group kernels (blocked Cholesky and substitutions on MFMA, cooperative "
                         "tridiagonalisation with two grid barriers per reflector): latency-bound" % (b + nev))}
    nl_pp = agg["n_launch"]["products_p"] + agg["n_launch"]["products_psi"]
    t_pp = (agg["t"]["products_p"] + agg["t"]["products_psi"]) / max(1, nl_pp)
    bytes_pp = (agg["n_launch"]["products_p"] * spmm_bytes(P, 0) + agg["n_launch"]["products_psi"]
                * spmm_bytes(P, 0) + 24 * P.n * (agg["cols"]["products_p"] + agg["cols"]["products_psi"]))
    pp_achieved = bytes_pp / max(1, nl_pp) / t_pp / 1e9
    roofline_hbm = {"bound": "hbm", "kernel": "k_spmm_hs", "achieved": pp_achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": pp_achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_spmm_hs"),
                    "launches": int(nl_pp), "avg_launch_us": 1e6 * t_pp,
                    "algorithmic_bytes_per_launch": bytes_pp / max(1, nl_pp)}
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
        "device": {"name": torch.cuda.get_device_name(0),
                   "lds_per_block": getattr(torch.cuda.get_device_properties(0), "shared_memory_per_block", None)},
        "steps_ms_per_solve": steps_ms,
        "setup_s": {"generate": t_gen, "factor_total": t_setup, "order": fi["t_order_s"],
                    "factor": fi["t_factor_s"], "upload": fi["t_upload_s"], "nnz_factor": fi["nnz_factor"]},
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
    }
    if "mixed" in results:
        mx = results["mixed"]
        lam64 = f["outs"][0].lam.cpu().numpy()
        lam32 = mx["outs"][0].lam.cpu().numpy()
        line["mixed"] = {"value": mx["value"], "ms_per_step": mx["ms"],
                         "p50_ms": 1e3 * percentile(mx["lat"], 50), "p99_ms": 1e3 * percentile(mx["lat"], 99),
                         "speedup_vs_fp64": mx["value"] / f["value"],
                         "iterations": mx["outs"][0].stats["outer_iters"],
                         "max_rel_eig_diff_vs_fp64": float(np.max(np.abs(lam32 - lam64) /
                                                                  np.abs(lam64 - P.sigma0)))}
    try:
        mp = measured_peaks()
        line["measured_peaks"] = mp
        line["roofline"]["frac_of_measured"] = rr_achieved / mp["fp64_dgemm_TFLOPs"]
        line["roofline_hbm"]["frac_of_measured"] = pp_achieved / mp["hbm_copy_GBps"]
    except Exception as exc:   # the peaks are context; the line is printed regardless
        line["measured_peaks"] = {"error": str(exc)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, nev, m0, args.tol)
    print(json.dumps(line), flush=True)


def cpu_baseline(P, nev, m0, tol):
    """The oracle, as it stands, on the host cores: one full cold-start solve of the
    same workload (global factorisation timed apart and excluded, as on the GPU)."""
    from oracle import labpsd as olab
    from oracle import precond as oprec
    import pufe
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    K = oprec.GlobalPreconditioner(P.H(), P.S(), P.eps_bar)
    t_fac = time.perf_counter() - t0
    prm = olab.Params(nev=nev, m0=m0, tol=tol, sigma0=P.sigma0, eps_bar=P.eps_bar)
    res = olab.solve(P.H(), P.S(), prm, pufe.start_block(P.n, nev + m0, 0), precond=K)
    return {"value": nev / res.t_solve, "unit": "eigenpairs/s", "cores": int(cores), "kind": "oracle",
            "sample": "one full oracle solve of the same workload (%d outer iterations, %.1fs); "
                      "its sparse factorisation (%.1fs, single-threaded SuperLU) excluded"
                      % (res.outer_iters, res.t_solve, t_fac)}


if __name__ == "__main__":
    main()
