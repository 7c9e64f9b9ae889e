"""Benchmark: time to solution of the coupled SaP solver on one MI355X.

One step = sap_factor + sap_solve (factorization, spike tips, reduced
systems and BiCGStab(2) to a 1e-10 true relative residual) on the resident
N=200000, K=50, P=64, d=1 system.  The FP64 run is the headline value; the
same steps with FP32 factors/tips/sweeps (FP64 Krylov) are timed beside it.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: this build runs on one
GPU only.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve ms & HBM GB/s, N=200k K=50; FP32-factor vs FP64 SaP at 1e-10 resid"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP64_VEC_TFLOPS = 78.6          # MI355X vector FP64 (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
FP32_VEC_TFLOPS = 157.3         # MI355X published vector FP32
PROFILE_DIR = os.path.join(ROOT, "profiles")


def sweep_bytes(n, k, sf, coupled):
    """Algorithmic bytes of one sweep launch: the K+1 coefficients of every
    row plus input and output vectors, averaged over the sweeps of one
    preconditioner application (SaP-C: in/out = (8,s) (s,s) (8,s) (s,8);
    SaP-D: (8,s) (s,8))."""
    io = (24 + 5 * sf) / 4.0 if coupled else 8.0 + sf
    return n * (k + 1) * sf + n * io


def spmv_bytes(n, k):
    return 8.0 * (2 * k + 1) * n + 16.0 * n


def lu_bytes(n, k, sf, coupled):
    dirs = 2 if coupled else 1
    return dirs * 8.0 * (2 * k + 1) * n + 2.0 * n * (k + 1) * sf


def lu_flops(n, k, coupled):
    """Block LU (and UL for SaP-C): per pivot K divisions and K^2 FMAs."""
    return (2 if coupled else 1) * (2.0 * n * k * k + n * k)


def tips_flops(n, k, p):
    """Per interface: four K x K triangular solves with K right-hand sides
    (4 * K^3 flops), Rbar = I - W V (2 K^3), LU of Rbar (2/3 K^3) and its
    inverse (2 K^3)."""
    return (p - 1) * (4.0 + 2.0 + 2.0 / 3.0 + 2.0) * k ** 3


def kernel_source_hash(name: str) -> str:
    path = os.path.join(ROOT, "paper_1509_07919_amd", "csrc", name)
    if not name or not os.path.exists(path):
        return ""
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profiles(tag: str):
    """HBM bytes per unit (a launch; a whole sweep for the sweeps) measured with
    rocprofv3 counters, from a committed summary that records the hash of the
    kernel source it was taken on; None if absent or if the kernel changed."""
    path = os.path.join(PROFILE_DIR, "traffic_%s.json" % tag.split("_", 2)[2])
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(tag)
    if not ent or ent.get("source_sha256_16") != kernel_source_hash(ent.get("source", "")):
        return None
    return ent.get("bytes_per_unit")


# kernel name -> (class, source file of that kernel)
KERNEL_CLASSES = (
    ("k_lu_wide", "lu", "k_lu_wide.hip"), ("k_lu_mfma", "lu", "k_lu_mfma.hip"),
    ("k_banded_lu", "lu", "k_factor.hip"), ("k_block_norm", "norm", "k_factor.hip"),
    ("k_sweep_xfer", "xfer", "k_sweep.hip"), ("k_sweep", "sweep", "k_sweep.hip"),
    ("k_tips", "tips", "k_tips.hip"), ("k_spmv", "spmv", "k_vec.hip"),
    ("k_correction", "corr", "k_vec.hip"), ("k_dots", "krylov", "k_vec.hip"),
    ("k_update", "krylov", "k_vec.hip"),
)


def summarize_counters(fetch_dir, write_dir, workload, prec):
    """Per-class HBM bytes from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) of `bench.py --steps 1 --warmup 0 --no-cpu
    --race-d 0 --no-cold --batch-rhs 0 --precs <prec> --copy-calibration`,
    each scaled by what the counter reads for the run's 1 GiB device copy.
    Units: a launch, a factorization for the tips, a whole sweep for the
    sweeps.  Merges into profiles/traffic_<workload>.json and prints a
    markdown table."""
    import csv
    import glob

    def load(d, counter):
        per = {}
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                for row in csv.DictReader(f):
                    if row.get("Counter_Name") != counter:
                        continue
                    key = (row["Kernel_Name"], row.get("Dispatch_Id") or row.get("Correlation_Id"))
                    per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
        by_kernel = {}
        for (name, _), v in per.items():
            by_kernel.setdefault(name, []).append(v)
        return by_kernel

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")

    def bench_line(d):
        for path in glob.glob(os.path.join(d, "**", "stdout.txt"), recursive=True):
            for line in open(path):
                if line.startswith("{"):
                    return json.loads(line)
        raise RuntimeError("no bench JSON line under " + d)

    line = bench_line(fetch_dir)
    copy_f = [v for nm, vs in fetch.items() if "copyBuffer" in nm for v in vs]
    copy_w = [v for nm, vs in write.items() if "copyBuffer" in nm for v in vs]
    cal = line["copy_calibration_bytes"]
    fcal = cal["read"] / (max(copy_f) * 1024.0)
    wcal = cal["write"] / (max(copy_w) * 1024.0)
    cfg = sapgen_workload(workload)
    coupled = cfg["mode"] == "coupled"
    st = line["runs"][prec]
    steps = 2                                   # the timed step and the profiled one
    sweeps = steps * (int(round(st["iters"] * 4)) + 1) * (4 if coupled else 2)
    classes = {}
    for name in sorted(set(fetch) | set(write)):
        hit = next(((c, src) for pat, c, src in KERNEL_CLASSES if pat in name), None)
        if not hit:
            continue
        c, src = hit
        ent = classes.setdefault(c, {"dispatches": 0, "read": 0.0, "write": 0.0, "source": src,
                                     "kernels": []})
        fr, wr = fetch.get(name, []), write.get(name, [])
        ent["dispatches"] += max(len(fr), len(wr))
        ent["read"] += sum(fr) * 1024.0 * fcal
        ent["write"] += sum(wr) * 1024.0 * wcal
        ent["kernels"].append((name, max(len(fr), len(wr)), sum(fr) / max(len(fr), 1),
                               sum(wr) / max(len(wr), 1)))
    nfac = classes.get("lu", {}).get("dispatches", steps)
    path = os.path.join(PROFILE_DIR, "traffic_%s.json" % workload)
    data = json.load(open(path)) if os.path.exists(path) else {}
    rows = []
    for c, ent in sorted(classes.items()):
        units = sweeps if c == "sweep" else (nfac if c == "tips" else ent["dispatches"])
        tag = "%s_%s_%s" % (c, prec, workload)
        data[tag] = {"dispatches": ent["dispatches"], "source": ent["source"],
                     "source_sha256_16": kernel_source_hash(ent["source"]), "units": units,
                     "bytes_per_unit": (ent["read"] + ent["write"]) / units,
                     "read_bytes_per_unit": ent["read"] / units,
                     "write_bytes_per_unit": ent["write"] / units}
        rows.append("| %s | %s | %d | %.1f | %.1f |" % (c, prec, units, ent["read"] / units / 1e6,
                                                      ent["write"] / units / 1e6))
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("calibration: read x %.3f, write x %.3f (1 GiB copy)" % (fcal, wcal))
    print("| kernel | dispatches | FETCH_SIZE KiB (avg) | WRITE_SIZE KiB (avg) |")
    print("|---|---|---|---|")
    for c, ent in sorted(classes.items()):
        for name, nd, fa, wa in ent["kernels"]:
            print("| `%s` | %d | %.0f | %.0f |" % (name[:90], nd, fa, wa))
    print()
    print("| class | precision | units | read MB per unit | write MB per unit |")
    print("|---|---|---|---|---|")
    print("\n".join(rows))


def sapgen_workload(name):
    import sapgen
    return dict(sapgen.WORKLOADS.get(name) or sapgen.SPD_WORKLOADS[name])


def outer_solve(args, s, b, x):
    """One solve with the outer method of the run: BiCGStab(2) or, for the
    symmetric positive definite workloads, CG."""
    cfg = args.cfg
    if getattr(args, "solver", "bicgstab2") == "cg":
        return s.solve_cg(b, x, tol=cfg["tol"], maxit=args.maxit)
    return s.solve(b, x, tol=cfg["tol"], maxit=args.maxit)


def applications(args, st):
    """Preconditioner applications of one solve (BiCGStab(2) applies it
    once more than its counted operator applications, to b)."""
    return st.n_apply + (0 if getattr(args, "solver", "bicgstab2") == "cg" else 1)


def run_cold(args, prec, a, b):
    """The same steps with the 256 MB last-level cache flushed before each
    one (a 1 GiB buffer is written, untimed): every step starts with A, the
    factors and the vectors in HBM only.  Returns (ms per step from events
    around each step, per-kernel times of the flushed steps)."""
    import torch
    from paper_1509_07919_amd import SapSolver

    cfg = args.cfg
    s = SapSolver(cfg["n"], cfg["k"], cfg["p"], mode=cfg["mode"], factor_prec=prec)
    x = torch.empty_like(b)
    flush = torch.empty(1 << 27, dtype=torch.float64, device=a.device)
    for _ in range(args.warmup):
        s.factor(a)
        outer_solve(args, s, b, x)
    st_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    en_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        flush.fill_(float(i))
        st_ev[i].record()
        s.factor(a)
        outer_solve(args, s, b, x)
        en_ev[i].record()
    torch.cuda.synchronize()
    ms = sum(st_ev[i].elapsed_time(en_ev[i]) for i in range(args.steps)) / args.steps
    s.profile(True)
    for i in range(args.steps):
        flush.fill_(float(i))
        s.factor(a)
        outer_solve(args, s, b, x)
    torch.cuda.synchronize()
    kt = s.kernel_times()
    s.profile(False)
    s.close()
    del flush
    return ms, kt


def run_gpu(args, prec, pb, a, b):
    import torch
    from paper_1509_07919_amd import SapSolver

    cfg = args.cfg
    s = SapSolver(cfg["n"], cfg["k"], cfg["p"], mode=cfg["mode"], factor_prec=prec)
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        s.factor(a)
        outer_solve(args, s, b, x)
    # the timed steps run without per-launch events; the per-kernel device
    # times come from as many steps again with events around every launch
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.factor(a)
        _, st = outer_solve(args, s, b, x)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.profile(True)
    for _ in range(args.steps):
        s.factor(a)
        outer_solve(args, s, b, x)
    torch.cuda.synchronize()
    kt = s.kernel_times()
    s.profile(False)
    kt["phases"] = s.tips_phase_times()
    xs = x.cpu().numpy()
    s.close()
    return (t1 - t0) * 1e3 / args.steps, stats, kt, xs


def run_backward(args, prec, pb, a, b):
    """The differentiation step: factor and forward solve, then the backward
    pass of L = 0.5 ||x - x_target||^2 (x_target ~ N(0, 1)): the adjoint solve
    A^T lambda = x - x_target on the same factors (dL/db = lambda) and the band
    gradient dL/dA = band(-lambda x^T).  Events on the launch stream time the
    forward part and the backward part of each step, and the band gradient
    alone; a second round with per-launch timing gives the backward pass's
    kernels."""
    import torch

    import sapgen
    from paper_1509_07919_amd import SapSolver

    cfg = args.cfg
    n, k = cfg["n"], cfg["k"]
    s = SapSolver(n, k, cfg["p"], mode=cfg["mode"], factor_prec=prec, adjoint=True)
    xt = torch.from_numpy(sapgen.normal_draws(args.seed, sapgen.STREAM_XTARGET, n)).to(a.device)
    x, g, lam = torch.empty_like(b), torch.empty_like(b), torch.empty_like(b)
    gband = torch.empty((2 * k + 1) * n, dtype=torch.float64, device=a.device)

    def one(ev=None):
        if ev:
            ev[0].record()
        s.factor(a)
        _, st = s.solve(b, x, tol=cfg["tol"], maxit=args.maxit)
        if ev:
            ev[1].record()
        torch.sub(x, xt, out=g)
        _, sta = s.solve_adjoint(g, lam, tol=cfg["tol"], maxit=args.maxit)
        if ev:
            ev[2].record()
        s.band_grad(lam, x, gband)
        if ev:
            ev[3].record()
        return st, sta

    for _ in range(args.warmup):
        one()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    stats = [one(ev) for ev in evs]
    torch.cuda.synchronize()
    fwd = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    bwd = sum(e[1].elapsed_time(e[3]) for e in evs) / args.steps
    # the band gradient alone: 10 launches queued behind a spin on the GPU, so
    # that they run back to back (one launch is shorter than the host's
    # launch latency that follows the adjoint solve's final synchronization)
    reps = 10
    ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(5_000_000)
    ga.record()
    for _ in range(reps):
        s.band_grad(lam, x, gband)
    gb.record()
    torch.cuda.synchronize()
    grad = ga.elapsed_time(gb) / reps
    s.profile(True)
    for _ in range(args.steps):
        torch.sub(x, xt, out=g)
        s.solve_adjoint(g, lam, tol=cfg["tol"], maxit=args.maxit)
    torch.cuda.synchronize()
    kt = s.kernel_times()
    s.profile(False)
    s.close()
    st, sta = stats[-1]
    grad_bytes = 8.0 * (2 * k + 1) * n + 16.0 * n          # writes the band, reads lambda and x
    return {
        "forward_ms": round(fwd, 4), "backward_ms": round(bwd, 4),
        "adjoint_iters": sta.iters, "adjoint_restarts": sta.restarts,
        "adjoint_rel_resid_true": sta.rel_resid_true, "adjoint_converged": bool(sta.converged),
        "forward_iters": st.iters,
        "band_grad": {"avg_us": round(grad * 1e3, 2), "bytes_per_unit": grad_bytes,
                      "algorithmic_GBps": grad_bytes / (grad * 1e-3) / 1e9,
                      "frac_of_hbm_peak": grad_bytes / (grad * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "adjoint_kernels": {c: {"ms_per_step": ms_ / args.steps, "launches_per_step": cnt / args.steps}
                            for c, (ms_, cnt) in kt.items() if cnt},
    }


def run_sparse(args):
    """The sparse front end on a synthetic sparse system (sapgen's hidden band
    of half-bandwidth K0, scattered by random permutations): the host analysis
    split into the time buckets T_DB (matching and scaling), T_CM
    (Cuthill-McKee) and T_Drop (reordered structure and drop-off), then per
    step on the GPU T_Asmbl (values and band of A_hat), sap_factor and
    sap_solve_sparse, timed with events.  Prints one JSON line."""
    import numpy as np
    import torch

    import sapgen
    from paper_1509_07919_amd import SapSolver, SapSparse

    n, k0, dens = (float(v) for v in args.sparse.split(","))
    n, k0 = int(n), int(k0)
    sp = sapgen.make_sparse_problem(n, k0, density=dens, seed=args.seed)
    t0 = time.perf_counter()
    plan = SapSparse(n, sp.rowptr, sp.colidx, sp.vals, db=True, cm=True,
                     drop_frac=args.sparse_drop)
    t_create = (time.perf_counter() - t0) * 1e3
    info, times = plan.info(), plan.times()
    k = info["k"]
    dev = torch.device("cuda:0")
    vals = torch.from_numpy(sp.vals).to(dev)
    b = torch.from_numpy(sp.b).to(dev)
    x = torch.empty_like(b)
    band = plan.assemble(vals)
    line = {"sparse": {"n": n, "k0": k0, "density": dens, "nnz": int(sp.rowptr[-1]),
                       "drop_frac": args.sparse_drop, "k": k, "k_full": info["k_full"],
                       "p": args.sparse_p, "mode": "coupled", "tol": 1e-10, "seed": args.seed},
            "analysis_ms": {"total": round(t_create, 2),
                            **{kk: round(v, 2) for kk, v in times.items()}},
            "runs": {}}
    for prec in args.precs.split(","):
        s = SapSolver(n, k, args.sparse_p, mode="coupled", factor_prec=prec)
        for _ in range(args.warmup):
            plan.assemble(vals, band)
            s.factor(band)
            s.solve_sparse(plan, b, x, tol=1e-10, maxit=args.maxit)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        sts = []
        for ev in evs:
            ev[0].record()
            plan.assemble(vals, band)
            ev[1].record()
            s.factor(band)
            _, st = s.solve_sparse(plan, b, x, tol=1e-10, maxit=args.maxit)
            ev[2].record()
            sts.append(st)
        torch.cuda.synchronize()
        st = sts[-1]
        xs = x.cpu().numpy()
        line["runs"][prec] = {
            "ms": round(sum(e[0].elapsed_time(e[2]) for e in evs) / args.steps, 4),
            "t_asmbl_ms": round(sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps, 4),
            "t_factor_ms": round(st.t_factor_ms, 4), "t_solve_ms": round(st.t_solve_ms, 4),
            "iters": st.iters, "restarts": st.restarts, "converged": bool(st.converged),
            "rel_err_vs_xtrue": float(np.linalg.norm(xs - sp.x_true) / np.linalg.norm(sp.x_true))}
        s.close()
    plan.close()
    print(json.dumps(line), flush=True)


# The paper's dense banded studies (Sec. 4.1.1-4.1.3), on synthetic matrices
# generated as for the benchmark (sapgen): time to solution of SaP-C and SaP-D
# with an FP32 preconditioner and FP64 BiCGStab(2), as the paper runs them.
#   psweep: N = 200000, K = 200, d = 1, P varied (Sec. 4.1.1)
#   dsweep: N = 200000, K = 200, P = 50, d in [0.06, 1.2] (Sec. 4.1.2)
#   grid:   P = 50, d = 1, N x K (Table t:denseBandedSweep; K <= 255 here)
EXPERIMENTS = {
    "psweep": [dict(n=200000, k=200, p=p_, d=1.0) for p_ in (10, 20, 30, 40, 50, 64, 80, 100)],
    "dsweep": [dict(n=200000, k=200, p=50, d=d_) for d_ in (0.06, 0.08, 0.1, 0.2, 0.4, 0.6, 0.8, 1.0, 1.2)],
    "grid": [dict(n=n_, k=k_, p=50, d=1.0) for n_ in (10000, 50000, 200000, 1000000)
             for k_ in (10, 20, 50, 100, 200)],
}


def run_experiment(args, configs=None):
    """Runs the configurations of one study (or `configs`), prints one JSON
    line per configuration and mode, and returns those records."""
    import numpy as np
    import torch

    import sapgen
    dev = torch.device("cuda:0")
    lines = []
    for c in (EXPERIMENTS[args.experiment] if configs is None else configs):
        pb = sapgen.make_problem(c["n"], c["k"], d=c["d"], seed=args.seed)
        a = torch.from_numpy(pb.band).to(dev)
        b = torch.from_numpy(pb.b).to(dev)
        for mode in ("coupled", "decoupled"):
            args.cfg = {"n": c["n"], "k": c["k"], "p": c["p"], "mode": mode, "tol": 1e-10}
            line = {"experiment": args.experiment, "n": c["n"], "k": c["k"], "p": c["p"],
                    "d": c["d"], "mode": "SaP-C" if mode == "coupled" else "SaP-D",
                    "factor_prec": "fp32", "steps": args.steps}
            try:
                ms, stats, _, xs = run_gpu(args, "fp32", pb, a, b)
                st = stats[-1]
                line.update({"ms": round(ms, 3), "iters": st.iters, "restarts": st.restarts,
                             "converged": bool(st.converged),
                             "rel_resid_true": st.rel_resid_true,
                             "t_factor_ms": round(st.t_factor_ms, 3),
                             "t_solve_ms": round(st.t_solve_ms, 3),
                             "rel_err_vs_xtrue": float(np.linalg.norm(xs - pb.x_true)
                                                       / np.linalg.norm(pb.x_true))})
            except Exception as e:      # e.g. not converged within maxit, or K unsupported
                line["error"] = str(e)[:200]
            print(json.dumps(line), flush=True)
            lines.append(line)
        del a, b
    return lines


def run_batch(args, prec, pb, a, m):
    """Factor once and solve m right-hand sides with sap_solve_batch; the
    same m columns one sap_solve at a time beside it (same factorization)."""
    import numpy as np
    import torch

    import oracle
    import sapgen
    from paper_1509_07919_amd import SapSolver

    cfg = args.cfg
    n, k = cfg["n"], cfg["k"]
    xs = np.stack([sapgen.splitmix64_uniform(300 + c, sapgen.STREAM_XTRUE, np.arange(n))
                   for c in range(m)])
    B = torch.from_numpy(np.stack([oracle.bandmv(pb.band, n, k, xs[c]) for c in range(m)])).to(a.device)
    s = SapSolver(n, k, cfg["p"], mode=cfg["mode"], factor_prec=prec, nrhs=m)
    X = torch.empty_like(B)
    s.factor(a)
    for _ in range(args.warmup):
        s.solve_batch(B, X, tol=cfg["tol"], maxit=args.maxit)
        for c in range(m):
            s.solve(B[c], X[c], tol=cfg["tol"], maxit=args.maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, sts = s.solve_batch(B, X, tol=cfg["tol"], maxit=args.maxit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    err = float(max(np.abs(X[c].cpu().numpy() - xs[c]).max() for c in range(m)))
    for _ in range(args.steps):
        for c in range(m):
            s.solve(B[c], X[c], tol=cfg["tol"], maxit=args.maxit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.close()
    batch_ms = (t1 - t0) * 1e3 / args.steps
    single_ms = (t2 - t1) * 1e3 / args.steps
    return {"m": m, "factor_prec": prec, "batch_solve_ms": round(batch_ms, 4),
            "batch_ms_per_rhs": round(batch_ms / m, 4),
            "single_solves_ms": round(single_ms, 4),
            "speedup_vs_single": round(single_ms / batch_ms, 3),
            "iters": [st.iters for st in sts], "converged": all(st.converged for st in sts),
            "max_abs_err_vs_xtrue": err}


def cpu_model() -> str:
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, pb, reps, solver="bicgstab2"):
    """The CPU oracle (plain FP64 SaP + BiCGStab(2), or CG for the SPD
    workloads) on the same workload, single thread, median of `reps` full
    solves."""
    from threadpoolctl import threadpool_limits

    import oracle
    times, x = [], None
    with threadpool_limits(1):
        for _ in range(reps):
            t0 = time.perf_counter()
            fn = oracle.sap_solve_cg if solver == "cg" else oracle.sap_solve
            x, res, _ = fn(pb.band, cfg["n"], cfg["k"], pb.b, cfg["p"],
                           cfg["mode"] == "coupled", tol=cfg["tol"])
            times.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(times), x, res


def cpu_lapack_context(cfg, pb, reps):
    """Context only: LAPACK's banded LU with partial pivoting (dgbsv through
    scipy.linalg.solve_banded) on the same system, with the host BLAS's own
    thread count; median of `reps` solves and the relative error against
    x_true.  The band layout is LAPACK's band storage with kl = ku = K
    (entry a(i, j) at row K + i - j of column j), so the array is passed as is."""
    import numpy as np
    import scipy.linalg as sla
    from threadpoolctl import threadpool_info
    n, k = cfg["n"], cfg["k"]
    ab = pb.band.reshape(2 * k + 1, n)
    times, x = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        x = sla.solve_banded((k, k), ab, pb.b, check_finite=False)
        times.append((time.perf_counter() - t0) * 1e3)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    err = float(np.linalg.norm(x - pb.x_true) / np.linalg.norm(pb.x_true))
    return statistics.median(times), threads, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sapc_n200k_k50")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--maxit", type=int, default=100)
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precs", default="fp64,fp32")
    ap.add_argument("--race-d", default="0.12,0.11",
                    help="also race FP32 against FP64 factors on the same N, K, P at these "
                         "diagonal dominances (comma list; 0 or empty: skip)")
    ap.add_argument("--race-steps", type=int, default=5)
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the steps timed with the last-level cache flushed first")
    ap.add_argument("--batch-rhs", type=int, default=8,
                    help="also time sap_solve_batch with this many right-hand sides on the "
                         "same factorization (0: skip)")
    ap.add_argument("--solver", choices=("auto", "bicgstab2", "cg"), default="auto",
                    help="outer Krylov method; auto: CG for the symmetric positive definite "
                         "workloads, BiCGStab(2) otherwise")
    ap.add_argument("--backward", choices=("auto", "on", "off"), default="auto",
                    help="also time the backward pass (adjoint solve and band gradient); "
                         "auto: for the workloads whose configuration includes it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="build profiles/traffic_<workload>.json from two rocprofv3 --pmc "
                         "runs (FETCH_SIZE, WRITE_SIZE) of this script with --precs <one>")
    ap.add_argument("--sparse", metavar="N,K0,DENSITY",
                    help="instead of the benchmark line, time the sparse front end on a "
                         "synthetic sparse system (e.g. 200000,50,0.2)")
    ap.add_argument("--sparse-drop", type=float, default=0.0,
                    help="drop-off fraction for --sparse")
    ap.add_argument("--sparse-p", type=int, default=64, help="partitions for --sparse")
    ap.add_argument("--experiment", choices=sorted(EXPERIMENTS),
                    help="instead of the benchmark line, run one of the paper's dense "
                         "sensitivity studies and print one JSON line per configuration")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.experiment:
        run_experiment(args)
        return
    if args.sparse:
        run_sparse(args)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.workload,
                           args.precs.split(",")[0])
        return

    import numpy as np
    import torch

    import sapgen
    cfg = sapgen_workload(args.workload)
    args.cfg = cfg
    spd = args.workload in sapgen.SPD_WORKLOADS
    if args.solver == "auto":
        args.solver = "cg" if spd else "bicgstab2"
    n, k = cfg["n"], cfg["k"]
    pb = sapgen.make_problem(n, k, d=cfg["d"], seed=args.seed,
                             row_scale_decades=cfg["row_scale_decades"],
                             symmetric=cfg.get("symmetric", False))
    dev = torch.device("cuda:0")
    a = torch.from_numpy(pb.band).to(dev)
    b = torch.from_numpy(pb.b).to(dev)
    coupled = cfg["mode"] == "coupled"

    runs = {}
    for prec in args.precs.split(","):
        ms, stats, kt, xs = run_gpu(args, prec, pb, a, b)
        runs[prec] = dict(ms=ms, stats=stats, kt=kt, x=xs)

    head = "fp64" if "fp64" in runs else next(iter(runs))
    sf = 8 if head == "fp64" else 4
    r = runs[head]
    steps = args.steps
    per_launch = {
        "sweep": sweep_bytes(n, k, sf, coupled),
        "spmv": spmv_bytes(n, k),
        "lu": lu_bytes(n, k, sf, coupled),
    }
    # a sweep (one triangular solve over all blocks) is one or two launches
    # (chunked form: zero-state pass, then the pass from the chained states);
    # its unit is the whole sweep.  Sweeps per step: 2 (SaP-D) or 4 (SaP-C)
    # per preconditioner application, n_apply + 1 applications per solve.
    sweeps = sum(applications(args, st) * (4 if coupled else 2) for st in r["stats"])
    units = {"sweep": sweeps}
    kernels = {}
    for name, val in r["kt"].items():
        if name == "phases":
            continue
        tms, cnt = val
        if cnt == 0:
            continue
        nu = units.get(name, cnt)
        ent = {"ms_per_step": tms / steps, "launches_per_step": cnt / steps,
               "units_per_step": nu / steps, "avg_us": 1e3 * tms / nu}
        if name in per_launch:
            ent["bytes_per_unit"] = per_launch[name]
            ent["algorithmic_GBps"] = per_launch[name] / (1e-3 * tms / nu) / 1e9
        kernels[name] = ent
    flops_per_launch = {"lu": lu_flops(n, k, coupled), "tips": tips_flops(n, k, cfg["p"])}
    for name, fl in flops_per_launch.items():
        if name in kernels:
            kernels[name]["flops_per_unit"] = fl
            kernels[name]["algorithmic_TFLOPs"] = fl / (1e-6 * kernels[name]["avg_us"]) / 1e12
    dom = max(kernels, key=lambda q: kernels[q]["ms_per_step"])
    avg_s = 1e-6 * kernels[dom]["avg_us"]
    traffic = traffic_from_profiles("%s_%s_%s" % (dom, head, args.workload))
    if dom in per_launch and dom not in flops_per_launch:
        ach = per_launch[dom] / avg_s / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_us": round(avg_s * 1e6, 2),
                "bytes_per_unit": per_launch[dom]}
    elif dom in flops_per_launch:
        peak = FP64_VEC_TFLOPS if head == "fp64" else FP32_VEC_TFLOPS
        ach = flops_per_launch[dom] / avg_s / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 4), "peak": peak,
                "unit": "TFLOP/s", "frac": round(ach / peak, 5), "traffic": traffic,
                "avg_us": round(avg_s * 1e6, 2), "flops_per_unit": flops_per_launch[dom],
                "bytes_per_unit": per_launch.get(dom)}
    else:
        roof = {"kernel": dom, "bound": None, "note": "no work model for this kernel class"}

    def summary(prec):
        q = runs[prec]
        st = q["stats"][-1]
        err_true = float(np.linalg.norm(q["x"] - pb.x_true) / np.linalg.norm(pb.x_true))
        return {"ms": round(q["ms"], 4), "iters": st.iters, "restarts": st.restarts,
                "rel_resid_true": st.rel_resid_true, "converged": bool(st.converged),
                "t_factor_ms": round(st.t_factor_ms, 4), "t_lu_ms": round(st.t_lu_ms, 4),
                "t_tips_ms": round(st.t_tips_ms, 4), "t_solve_ms": round(st.t_solve_ms, 4),
                "tips_phases_ms": {kk: round(v, 4) for kk, v in q["kt"]["phases"].items()},
                "rel_err_vs_xtrue": err_true}

    out = {
        "metric": METRIC, "value": round(r["ms"], 4), "unit": "ms", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32-factor/f64-krylov", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "k": k, "p": cfg["p"],
                   "mode": cfg["mode"], "d": cfg["d"], "tol": cfg["tol"], "seed": args.seed,
                   "factor_prec": head, "solver": args.solver},
        "roofline": roof,
        "runs": {p_: summary(p_) for p_ in runs},
        "kernels": kernels,
        "paper_context": {"sap_c_ms": 186.756, "sap_d_ms": 187.717, "mkl_ms": 367.638,
                          "hardware": "Tesla K20X (paper Table t:denseBandedSweep, P=50)"},
    }
    if "fp64" in runs and "fp32" in runs:
        out["race"] = {"fp64_ms": round(runs["fp64"]["ms"], 4),
                       "fp32_factor_ms": round(runs["fp32"]["ms"], 4),
                       "fp32_speedup": round(runs["fp64"]["ms"] / runs["fp32"]["ms"], 3)}
    race_ds = [float(v) for v in str(args.race_d).split(",") if v.strip() and float(v) > 0]
    if spd or args.solver == "cg":
        race_ds = []                # the weak-dominance race is a BiCGStab(2) study
    if race_ds and "fp64" in runs and "fp32" in runs:
        # the same race where the FP64 preconditioner is no longer exact after
        # one application, so both precisions iterate
        out["race_weak_dominance"] = []
        for dw in race_ds:
            pbw = sapgen.make_problem(n, k, d=dw, seed=args.seed,
                                      row_scale_decades=cfg["row_scale_decades"])
            aw = torch.from_numpy(pbw.band).to(dev)
            bw = torch.from_numpy(pbw.b).to(dev)
            wargs = argparse.Namespace(**vars(args))
            wargs.steps, wargs.warmup = args.race_steps, 1
            rw = {}
            for prec in ("fp64", "fp32"):
                ms, stats, _, xs = run_gpu(wargs, prec, pbw, aw, bw)
                st = stats[-1]
                rw[prec] = {"ms": round(ms, 4), "iters": st.iters, "restarts": st.restarts,
                            "converged": bool(st.converged), "rel_resid_true": st.rel_resid_true,
                            "t_factor_ms": round(st.t_factor_ms, 4),
                            "t_solve_ms": round(st.t_solve_ms, 4),
                            "rel_err_vs_xtrue": float(np.linalg.norm(xs - pbw.x_true)
                                                      / np.linalg.norm(pbw.x_true))}
            out["race_weak_dominance"].append({
                "config": {"n": n, "k": k, "p": cfg["p"], "mode": cfg["mode"], "d": dw,
                           "tol": cfg["tol"], "seed": args.seed},
                "steps": args.race_steps, "fp64": rw["fp64"], "fp32": rw["fp32"],
                "fp32_speedup": round(rw["fp64"]["ms"] / rw["fp32"]["ms"], 3)})
            del aw, bw
    if not args.no_cold:
        # flushed-cache (cold) figures: the step, and per kernel the sweeps
        # and SpMV rates, whose operands otherwise partly stay in the 256 MB
        # last-level cache between launches (A alone is 161.6 MB here)
        out["cold"] = {}
        for p_ in runs:
            cms, ckt = run_cold(args, p_, a, b)
            sfp = 8 if p_ == "fp64" else 4
            ent = {"ms_per_step": round(cms, 4)}
            nsw = sum(applications(args, st) * (4 if coupled else 2) for st in runs[p_]["stats"])
            for name, nunits, bpu in (("sweep", nsw, sweep_bytes(n, k, sfp, coupled)),
                                      ("spmv", None, spmv_bytes(n, k))):
                tms, cnt = ckt[name]
                if cnt:
                    nu = nunits if nunits else cnt
                    ent[name] = {"avg_us": round(1e3 * tms / nu, 2),
                                 "algorithmic_GBps": round(bpu / (1e-3 * tms / nu) / 1e9, 1)}
            out["cold"][p_] = ent
    if args.batch_rhs > 0 and args.solver != "cg":
        out["multi_rhs"] = [run_batch(args, p_, pb, a, args.batch_rhs) for p_ in runs]
    backward = args.backward == "on" or (args.backward == "auto" and args.workload in
                                         ("sapc_n100k_k32_adjoint", "sapc_n200k_k100_weak"))
    if backward:
        out["backward"] = {p_: run_backward(args, p_, pb, a, b) for p_ in runs}
    if args.copy_calibration:
        src_t = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src_t.numel() * 8, "write": dst_t.numel() * 8}
        del src_t, dst_t
    if not args.no_cpu:
        cms, xo, res = cpu_baseline(cfg, pb, args.cpu_reps, args.solver)
        out["cpu_baseline"] = {
            "value": round(cms, 2), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": "full workload, median of %d oracle solves (FP64 SaP-%s, P=%d, "
                      "%s to %g), 1 thread" % (args.cpu_reps, "C" if coupled else "D", cfg["p"],
                                               "CG" if args.solver == "cg" else "BiCGStab(2)",
                                               cfg["tol"]),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
        for p_ in runs:
            out["runs"][p_]["rel_err_vs_oracle"] = float(
                np.linalg.norm(runs[p_]["x"] - xo) / np.linalg.norm(xo))
        lms, lthr, lerr = cpu_lapack_context(cfg, pb, args.cpu_reps)
        out["cpu_context"] = {
            "value": round(lms, 2), "unit": "ms", "kind": "lapack_dgbsv",
            "threads": lthr, "rel_err_vs_xtrue": lerr,
            "sample": "full workload, median of %d scipy.linalg.solve_banded solves "
                      "(banded LU with partial pivoting)" % args.cpu_reps}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
