"""Benchmark: solved right-hand sides per second on one MI355X.

Workload: 3D convection-diffusion -Lap u + beta . grad u, 7-point stencil on a
128^3 grid (n = 2,097,152, nnz = 14,581,760), beta = (30, 20, 10), h = 1/129,
s = 16 Gaussian right-hand sides, FP64 CSR, relative residual 1e-8.  One step
solves the 16 right-hand sides once with each of Bl-BiCG-rQ, eGl-QMR and
Bl-BiCGStab-rQ (48 solved right-hand sides per step).  A, B and X are resident
in device memory before the timed region.  The three solves are independent and
by default run at the same time, each on its own context, stream and host
thread (--concurrent 0 runs them one after another); per_method then gives each
solve's own wall time, which overlaps the others'.

Also reported: the roofline position of the sparse x block product (the kernel
every iteration runs; algorithmic bytes A_b + 2 n s 8 per launch, timed with HIP
events on the stream it runs on) and the CPU oracle's throughput on a bounded
sample (set-up plus 20 timed iterations over the three methods, scaled by the
oracle's own converged iteration counts).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METHODS = ("bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading
    for a plain device copy of known size).  Reported only while the source the
    counters were taken on is unchanged (its SHA-256 is recorded beside them);
    otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "spmm_csr_convdiff3d128_s16_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    rec = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            rec[k.strip("` ")] = v.strip("` ")
    src = os.path.join(ROOT, "paper_1504_04395_amd", "csrc", "spmm.hpp")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernel") != kernel or rec.get("spmm.hpp sha256") != sha:
        return None
    try:
        return int(rec["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def spmm_roofline(pkg, ctx, A, n, nnz, s, stream, reps=50, X=None, kernel="k_spmm_csr8<double,EpiNone>",
                  adjoint=False):
    """Average duration of the sparse x block kernel (same launch configuration
    as inside the solver) from HIP events on its stream, against the
    algorithmic bytes nnz (b + 4) + 4 (n + 1) + 2 n s b (b = 8 real, 16
    complex FP64)."""
    import torch
    if X is None:
        X = torch.randn(n, s, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    b = 16 if X.dtype == torch.complex128 else 8
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for _ in range(5):
            pkg.spmm(ctx, A, X, Y, adjoint=adjoint, sync=False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            pkg.spmm(ctx, A, X, Y, adjoint=adjoint, sync=False)
        e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_alg = nnz * (b + 4) + 4 * (n + 1) + 2 * n * s * b
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": counter_traffic(kernel),
            "kernel": kernel, "avg_us": round(ms * 1e3, 2), "bytes_per_launch": bytes_alg}


def spmm_only_config(pkg, inputs, k, fmt, stream, reps=20):
    """The product with A of workload k (full size) alone, for kernel traces
    and hardware counters: `reps` timed launches after 5 warm-ups, then 20
    plain device copies of one n x s block (the counters' calibration)."""
    import numpy as np
    import torch
    prob = inputs.config(k, "full")
    ctx = pkg.Context(0, stream=stream.cuda_stream)
    kw = dict(fmt="sell", sell_C=16, sell_sigma=256) if fmt == "sell" else {}
    A = pkg.Matrix.from_csr(ctx, prob.A, **kw)
    X = torch.from_numpy(np.ascontiguousarray(prob.B)).cuda()
    n, s = X.shape
    roof = spmm_roofline(pkg, ctx, A, n, prob.A.nnz, s, stream, reps=reps, X=X, kernel=f"config {k} {fmt}")
    roof["traffic"] = None
    C = torch.empty_like(X)
    for _ in range(20):
        C.copy_(X)
    torch.cuda.synchronize()
    out = {"workload": prob.name, "format": fmt, "n": n, "nnz": prob.A.nnz, "s": s,
           "dtype": str(X.dtype).replace("torch.", ""), "spmm": roof,
           "copy_bytes_per_launch": 2 * X.numel() * X.element_size()}
    A.close()
    ctx.close()
    return out


# iterations timed per method by the CPU baseline (20 in all), beyond one
# untimed-per-iteration run that captures the set-up
CPU_SAMPLE_ITERS = {"bl_bicg_rq": 4, "egl_qmr": 10, "bl_bicgstab_rq": 6}


def oracle_counts(grid, path=None):
    """The oracle's own converged iteration counts on the unperturbed workload
    (seed 0), from the file the oracle-only script tests/golden/
    make_fullsize_counts.py writes; {} when the grid has no entry."""
    path = path or os.path.join(ROOT, "tests", "golden", "fullsize_iterations.txt")
    out = {}
    try:
        for line in open(path):
            f = line.split()
            if not f or f[0].startswith("#") or len(f) < 6:
                continue
            if int(f[0]) == grid and int(f[2]) == 0 and int(f[3]) == 0:
                out[f[1]] = int(f[4])
    except OSError:
        pass
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(prob, gpu_iters, solved, grid, sample_iters=None):
    """The oracle, untuned, on a bounded sample of the workload: per method one
    run of 1 iteration and one of 1 + k iterations on the full problem.  Their
    difference gives the time per iteration without the set-up (QR of the
    right-hand sides, shadow initialisation, final residual), the first run the
    set-up; a full solve is set-up + per-iteration time x the oracle's own
    converged iteration count (the GPU's count is used only where the oracle's
    is not on file, and the sample then says so).  The numerator is the same
    number of solved right-hand sides as the GPU step's."""
    import oracle
    sample_iters = sample_iters or CPU_SAMPLE_ITERS
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    counts = oracle_counts(grid)
    total = 0.0
    used = {}
    for m in METHODS:
        k = sample_iters[m]
        t = time.perf_counter()
        oracle.solve(prob.A, prob.B, m, tol=0.0, maxit=1)
        t1 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.solve(prob.A, prob.B, m, tol=0.0, maxit=1 + k)
        tk = time.perf_counter() - t
        per_it = max(tk - t1, 0.0) / k
        setup = max(t1 - per_it, 0.0)
        count = counts.get(m)
        used[m] = {"oracle_iterations": count if count is not None else None,
                   "scaled_by": count if count is not None else gpu_iters[m],
                   "s_per_iteration": round(per_it, 3), "setup_s": round(setup, 3)}
        total += setup + per_it * used[m]["scaled_by"]
        log(f"cpu oracle {m}: set-up {setup:.2f} s, {per_it:.2f} s per iteration ({k} timed), "
            f"x {used[m]['scaled_by']} iterations")
    value = solved / total
    src = "the oracle's own converged counts" if all(u["oracle_iterations"] for u in used.values()) else \
        "the oracle's counts where on file, else the GPU's"
    return {"value": round(value, 6), "unit": "RHS/s", "cores": cores, "kind": "oracle",
            "cpu_model": host_cpu_model(), "per_method": used,
            "sample": f"1 and 1+k iterations of each method on the full {grid}^3 problem "
                      f"(k = {dict(sample_iters)}, {sum(sample_iters.values())} timed iterations in all); "
                      f"set-up + per-iteration time x {src}; numpy/scipy FP64, BLAS threads={cores}, "
                      f"scipy sparse products single-threaded"}


# Table 2 of the paper (no preconditioning; Matlab on a CPU, its own
# discretisation): iterations and final relative block residual ("div." = above 1)
PAPER_TABLE2 = {
    "bl_bicg":        {1: (500, "div."), 2: (500, "div."), 3: (500, "0.28")},
    "bl_bicg_rq":     {1: (500, "1e-8"), 2: (500, "div."), 3: (156, "2e-10")},
    "bl_bicgstab":    {1: (500, "0.093"), 2: (500, "div."), 3: (111, "2e-10")},
    "bl_bicgstab_rq": {1: (355, "1e-10"), 2: (500, "div."), 3: (101, "2e-10")},
}
# the same table's rows with right no-fill ILU preconditioning
PAPER_TABLE2_ILU = {
    "bl_bicg":        {1: (500, "0.04"), 2: (28, "2e-10"), 3: (50, "3e-10")},
    "bl_bicg_rq":     {1: (163, "1e-10"), 2: (28, "8e-11"), 3: (50, "3e-10")},
    "bl_bicgstab":    {1: (113, "3e-10"), 2: (16, "4e-11"), 3: (33, "6e-11")},
    "bl_bicgstab_rq": {1: (115, "3e-11"), 2: (16, "3e-11"), 3: (33, "5e-11")},
}
ALL_METHODS = ("li_bicg", "li_qmr", "li_bicgstab", "gl_bicg", "egl_bicg", "gl_qmr", "egl_qmr", "gl_bicgstab",
               "bl_bicg", "bl_bicg_rq", "bl_bicgstab", "bl_bicgstab_rq")


def paper_table2(pkg, ctx, inputs, reps=3, examples=(1, 2, 3), preconds=(None, "ilu0"), methods=None):
    """Examples 1-3 of Section 5.1 at full size, every method, without and with
    right no-fill ILU preconditioning, stopping at a 1e-10 reduction of the
    block residual or 500 iterations (Section 5.2).  Reports iterations, final
    true relative residual and GPU seconds per solve (the best of ``reps``;
    the ILU set-up is timed once and reported apart), with Table 2's entries
    beside the block methods."""
    import numpy as np
    import torch
    rows = []
    for k in examples:
        prob = inputs.paper_example(k, "full")
        A = pkg.Matrix.from_csr(ctx, prob.A)
        B = torch.from_numpy(prob.B).cuda()
        X = torch.zeros_like(B)
        for pc in preconds:
            setup = None
            if pc:
                t = time.perf_counter()
                A.ilu0()
                setup = time.perf_counter() - t
                log(f"ex{k} ILU(0) set-up {setup * 1e3:.1f} ms")
            table = PAPER_TABLE2_ILU if pc else PAPER_TABLE2
            for m in methods or ALL_METHODS:
                best = None
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    _, info = pkg.solve(ctx, A, B, m, X=X, x0_zero=True, tol=1e-10, maxit=500, precond=pc)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t
                    best = dt if best is None else min(best, dt)
                res = info.rel_res_true
                row = {"example": k, "n": prob.A.n, "s": prob.B.shape[1], "method": m,
                       "precond": pc or "none", "iterations": info.iterations, "status": info.status_name,
                       "rel_res_true": ("div." if not np.isfinite(res) or res > 1 else float(f"{res:.1e}")),
                       "seconds": round(best, 4)}
                if setup is not None:
                    row["ilu_setup_seconds"] = round(setup, 4)
                if m in table:
                    it, r = table[m][k]
                    row["paper"] = {"iterations": it, "rel_res": r}
                rows.append(row)
                log(f"ex{k} {pc or 'none'} {m}: it={info.iterations} {info.status_name} res={res:.1e} "
                    f"{best * 1e3:.1f} ms")
        A.close()
    return rows


def config_solves(pkg, ctx, inputs, k, methods, precision, fmt, reps, inner_tol=1e-4, max_outer=20, precond=None):
    """Solve workload k of inputs.config (full size) with each method to 1e-8
    (at most 3000 iterations); the best of `reps` timed solves per method.  With
    FP32 inner solves, `inner_tol` and `max_outer` set the refinement, and the
    record carries the true relative residual before each outer step and
    after the last.  precond='ilu0': right ILU(0) (FP64), with its set-up time
    (host factorisation and level schedules) in the record."""
    import numpy as np
    import torch
    prob = inputs.config(k, "full")
    log(f"{prob.name}: n={prob.A.n} nnz={prob.A.nnz} s={prob.B.shape[1]}")
    A = pkg.Matrix.from_csr(ctx, prob.A, fmt=fmt, make_fp32=precision != "fp64")
    B = torch.from_numpy(np.ascontiguousarray(prob.B)).cuda()
    X = torch.zeros_like(B)
    kw = {} if precision == "fp64" else dict(precision=precision, inner_tol=inner_tol, max_outer=max_outer)
    setup_s = None
    if precond:
        torch.cuda.synchronize()
        t = time.perf_counter()
        A.ilu0()
        torch.cuda.synchronize()
        setup_s = round(time.perf_counter() - t, 4)
        log(f"ILU(0) set-up {setup_s * 1e3:.1f} ms")
        kw["precond"] = precond
    rows = []
    for m in methods or prob.methods:
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = pkg.solve(ctx, A, B, m, X=X, x0_zero=True, tol=1e-8, maxit=3000, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        row = {"workload": prob.name, "format": fmt, "precision": precision, "method": m,
               "status": info.status_name, "iterations": info.iterations,
               "outer": info.outer_iterations, "rel_res_true": info.rel_res_true, "seconds": round(best, 4)}
        if precond:
            row.update(precond=precond, precond_setup_s=setup_s)
        if precision != "fp64":
            row.update(inner_tol=inner_tol, max_outer=max_outer, outer_redone_in_fp64=info.fp64_outer_iterations,
                       outer_history=[float(f"{h:.3e}") for h in info.history])
        rows.append(row)
        log(f"{m}: {info.status_name} it={info.iterations} {best * 1e3:.1f} ms")
    A.close()
    return rows


def perturbed_counts(pkg, inputs, grid, seeds, maxit):
    """The benchmark's three solves on B and on B perturbed by 1e-15 relative
    noise (numpy default_rng(seed), the recipe of the oracle's count file):
    the GPU's own iteration-count spread under rounding-level changes."""
    import numpy as np
    import torch
    A_csr = inputs.convdiff3d(grid, (30.0, 20.0, 10.0))
    B0 = inputs.gaussian_block(A_csr.n, 16, seed=0)
    ctx = pkg.Context(0)
    A = pkg.Matrix.from_csr(ctx, A_csr)
    out = {m: {} for m in METHODS}
    for seed in [0] + list(seeds):
        Bs = B0 if seed == 0 else B0 * (1 + 1e-15 * np.random.default_rng(seed).standard_normal(B0.shape))
        B = torch.from_numpy(np.ascontiguousarray(Bs)).cuda()
        for m in METHODS:
            _, info = pkg.solve(ctx, A, B, m, tol=1e-8, maxit=maxit)
            out[m][seed] = {"iterations": info.iterations, "status": info.status_name}
        log(f"seed {seed}: " + ", ".join(f"{m} {out[m][seed]['iterations']}" for m in METHODS))
    A.close()
    ctx.close()
    return {"workload": f"convdiff3d-{grid}^3-s16", "tol": 1e-8, "maxit": maxit, "counts": out}


def config1_latency(pkg, inputs, reps=7):
    """The small 2D workload (32 x 32 grid, n = 1024, s = 4, FP64): Gl-BiCG and
    eGl-BiCG (and Gl-BiCGStab) to 1e-8 on the single-workgroup path (every iteration in one
    launch, the default for this size) and on the general schedule with the
    iteration captured in a hipGraph and launched eagerly; the median solve
    time of `reps`, microseconds per iteration, and the oracle's full solve in
    seconds (untuned, on the host)."""
    import numpy as np
    import torch
    import oracle
    prob = inputs.config(1)
    ctx = pkg.Context(0)
    A = pkg.Matrix.from_csr(ctx, prob.A)
    B = torch.from_numpy(prob.B).cuda()
    X = torch.zeros_like(B)
    rows = {}
    for m in ("gl_bicg", "egl_bicg", "gl_bicgstab"):   # the workload's two methods, and the third fused one
        r = {}
        for mode, fused, graph in (("fused", True, True), ("graph", False, True), ("eager", False, False)):
            ts = []
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, info = pkg.solve(ctx, A, B, m, X=X, x0_zero=True, tol=1e-8, use_graph=graph, fused_small=fused)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            med = float(np.median(ts[1:]))      # the first solve also builds the graph
            r[mode] = {"ms_per_solve": round(med * 1e3, 3),
                                                "us_per_iteration": round(med * 1e6 / info.iterations, 2),
                                                "iterations": info.iterations, "status": info.status_name}
        t = time.perf_counter()
        ref = oracle.solve(prob.A, prob.B, m, tol=1e-8)
        r["oracle"] = {"s_per_solve": round(time.perf_counter() - t, 4), "iterations": ref.iterations}
        rows[m] = r
        log(f"config 1 {m}: fused {r['fused']['us_per_iteration']} us/it ({r['fused']['ms_per_solve']} ms), "
            f"graph {r['graph']['us_per_iteration']} us/it, eager {r['eager']['us_per_iteration']} us/it, "
            f"oracle {r['oracle']['s_per_solve']} s")
    A.close()
    ctx.close()
    return {"workload": prob.name, "n": prob.A.n, "s": int(prob.B.shape[1]), "tol": 1e-8, "methods": rows}


def accel_ratio(pkg, inputs, configs=(2, 3, 4, 5), reps=20):
    """Table 1's blocking gain a, measured as the paper does: the time of s
    products with single vectors over the time of one product with the n x s
    block (same matrix, CSR, FP64 or complex FP64), with HIP events on the
    context's stream; both products with A and with A^H."""
    import numpy as np
    import torch
    stream = torch.cuda.Stream()
    ctx = pkg.Context(0, stream=stream.cuda_stream)
    out = []
    for k in configs:
        prob = inputs.config(k, "full")
        A = pkg.Matrix.from_csr(ctx, prob.A)
        Bk = np.ascontiguousarray(prob.B)
        s = Bk.shape[1]
        X = torch.from_numpy(Bk).cuda()
        Y = torch.empty_like(X)
        cols = [torch.from_numpy(np.ascontiguousarray(Bk[:, j:j + 1])).cuda() for j in range(s)]
        ycols = [torch.empty_like(c) for c in cols]
        torch.cuda.synchronize()
        row = {"workload": prob.name, "n": prob.A.n, "nnz": prob.A.nnz, "s": s}
        for adj in (False, True):
            def timed(fn):
                with torch.cuda.stream(stream):
                    for _ in range(3):
                        fn()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        fn()
                    e1.record(stream)
                e1.synchronize()
                return e0.elapsed_time(e1) * 1e3 / reps

            t_blk = timed(lambda: pkg.spmm(ctx, A, X, Y, adjoint=adj, sync=False))

            def singles():
                for c, y in zip(cols, ycols):
                    pkg.spmm(ctx, A, c, y, adjoint=adj, sync=False)
            t_vec = timed(singles)
            key = "AH" if adj else "A"
            row[key] = {"spmm_us": round(t_blk, 1), "s_spmv_us": round(t_vec, 1), "a": round(t_vec / t_blk, 2)}
            log(f"{prob.name} {key}: one block product {t_blk:.1f} us, {s} vector products {t_vec:.1f} us, "
                f"a = {t_vec / t_blk:.2f}")
        out.append(row)
        A.close()
        del X, Y, cols, ycols
        torch.cuda.empty_cache()
    ctx.close()
    return out


def sell_sweep(pkg, ctx, inputs, stream, reps=20):
    """Sparse x block product on the power-law workload (complex, s = 32, 2^20
    rows with lengths 4..400): CSR, and SELL-C-sigma for C in {16, 32, 64} and
    sigma in {C, 256, 1024, 8192}, each with its padding ratio (stored slots /
    nnz) and the average kernel time from HIP events on the context's stream."""
    import numpy as np
    import torch
    prob = inputs.config(4, "full")
    log(f"{prob.name}: n={prob.A.n} nnz={prob.A.nnz} s={prob.B.shape[1]}")
    X = torch.from_numpy(np.ascontiguousarray(prob.B)).cuda()
    Y = torch.empty_like(X)
    torch.cuda.synchronize()

    def timed(A):
        with torch.cuda.stream(stream):
            for _ in range(3):
                pkg.spmm(ctx, A, X, Y, sync=False)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                pkg.spmm(ctx, A, X, Y, sync=False)
            e1.record(stream)
        e1.synchronize()
        return round(e0.elapsed_time(e1) * 1e3 / reps, 1)

    rows = []
    A = pkg.Matrix.from_csr(ctx, prob.A)
    rows.append({"format": "csr", "padding": 1.0, "us": timed(A)})
    A.close()
    log(f"csr: {rows[-1]['us']} us")
    for C in (16, 32, 64):
        for sigma in sorted({C, 256, 1024, 8192}):
            A = pkg.Matrix.from_csr(ctx, prob.A, fmt="sell", sell_C=C, sell_sigma=sigma)
            rows.append({"format": "sell", "C": C, "sigma": sigma, "padding": round(A.sell_padding, 4),
                         "us": timed(A)})
            A.close()
            log(f"sell C={C} sigma={sigma}: padding {rows[-1]['padding']} {rows[-1]['us']} us")
    return {"workload": prob.name, "n": prob.A.n, "nnz": prob.A.nnz, "s": int(prob.B.shape[1]), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed-steps", type=int, default=1)
    ap.add_argument("--maxit", type=int, default=1200,
                    help="iteration cap per solve: the paper's largest cap (Section 5.2); the "
                         "converging methods need 250-450 iterations here")
    ap.add_argument("--spmm-only", action="store_true",
                    help="only the sparse x block kernel and a plain device copy of one block "
                         "(the workload of the hardware-counter runs); with --config K, workload K "
                         "(--format csr or sell: SELL-16-256)")
    ap.add_argument("--concurrent", type=int, default=1,
                    help="1 (default): the step's three solves run at the same time, each on its own "
                         "context, stream and host thread (same kernels and arithmetic, bit-identical "
                         "results; their latency-bound phases overlap); 0: one after another")
    ap.add_argument("--paper-table2", action="store_true",
                    help="instead of the benchmark: Examples 1-3 of Section 5.1 at full size with "
                         "every method (tol 1e-10, 500 iterations), beside the paper's Table 2")
    ap.add_argument("--examples", default="1,2,3", help="with --paper-table2: which examples")
    ap.add_argument("--precond", default="none,ilu0",
                    help="with --paper-table2: none, ilu0 or both; with --config: ilu0 preconditions the solves")
    ap.add_argument("--methods", default="", help="with --paper-table2 or --config: comma-separated subset")
    ap.add_argument("--reps", type=int, default=3, help="with --paper-table2 or --config: solves per entry "
                                                          "(best is kept)")
    ap.add_argument("--config", type=int, default=0,
                    help="instead of the benchmark: solve workload K of inputs.config at full size with "
                         "--methods (default: the workload's own list)")
    ap.add_argument("--precision", default="fp64", help="with --config: fp64 or fp32_refine")
    ap.add_argument("--inner-tol", type=float, default=1e-4, help="with --config and fp32_refine: inner tolerance")
    ap.add_argument("--max-outer", type=int, default=20, help="with --config and fp32_refine: outer step cap")
    ap.add_argument("--format", default="csr", help="with --config: csr or sell")
    ap.add_argument("--accel-ratio", action="store_true",
                    help="instead of the benchmark: Table 1's blocking gain a (s vector products over one "
                         "block product) on workloads 2-5 at full size")
    ap.add_argument("--no-config1", action="store_true", help="skip the small-workload latency figures")
    ap.add_argument("--config1-only", action="store_true",
                    help="instead of the benchmark: only the small-workload latency figures")
    ap.add_argument("--perturbed-counts", type=int, default=0,
                    help="instead of the benchmark: iteration counts of the three solves on B and on K copies "
                         "perturbed by 1e-15 (seeds 1..K)")
    ap.add_argument("--sell-sweep", action="store_true",
                    help="instead of the benchmark: the sparse x block product on the power-law workload "
                         "in CSR and SELL-C-sigma (C in 16, 32, 64; sigma in C, 256, 1024, 8192)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "described but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_1504_04395_amd as pkg

    if args.config1_only:
        print(json.dumps({"config1_latency": config1_latency(pkg, inputs)}), flush=True)
        return

    if args.config and not args.spmm_only:
        ctx = pkg.Context(0)
        rows = config_solves(pkg, ctx, inputs, args.config, tuple(m for m in args.methods.split(",") if m),
                             args.precision, args.format, args.reps, args.inner_tol, args.max_outer,
                             "ilu0" if args.precond == "ilu0" else None)
        print(json.dumps({"config_solves": rows}), flush=True)
        ctx.close()
        return

    if args.accel_ratio:
        print(json.dumps({"accel_ratio": accel_ratio(pkg, inputs)}), flush=True)
        return

    if args.perturbed_counts:
        print(json.dumps({"perturbed_counts": perturbed_counts(pkg, inputs, args.grid,
                                                               range(1, args.perturbed_counts + 1), args.maxit)}),
              flush=True)
        return

    if args.spmm_only and args.config:
        stream = torch.cuda.Stream()
        print(json.dumps(spmm_only_config(pkg, inputs, args.config, args.format, stream)), flush=True)
        return

    if args.sell_sweep:
        stream = torch.cuda.Stream()
        ctx = pkg.Context(0, stream=stream.cuda_stream)
        print(json.dumps({"sell_sweep": sell_sweep(pkg, ctx, inputs, stream)}), flush=True)
        ctx.close()
        return

    if args.paper_table2:
        ctx = pkg.Context(0)
        rows = paper_table2(pkg, ctx, inputs, reps=args.reps,
                            examples=tuple(int(k) for k in args.examples.split(",")),
                            preconds=tuple(None if p == "none" else p for p in args.precond.split(",")),
                            methods=tuple(m for m in args.methods.split(",") if m) or None)
        print(json.dumps({"paper_examples": rows}), flush=True)
        ctx.close()
        return

    t0 = time.perf_counter()
    A_csr = inputs.convdiff3d(args.grid, (30.0, 20.0, 10.0))
    B_np = inputs.gaussian_block(A_csr.n, 16, seed=0)
    n, nnz, s = A_csr.n, A_csr.nnz, 16
    log(f"generated n={n} nnz={nnz} in {time.perf_counter() - t0:.1f} s")

    stream = torch.cuda.Stream()
    ctx = pkg.Context(0, stream=stream.cuda_stream)
    A = pkg.Matrix.from_csr(ctx, A_csr)
    B = torch.from_numpy(B_np).cuda()
    if args.spmm_only:
        roof = spmm_roofline(pkg, ctx, A, n, nnz, s, stream, reps=20)
        C = torch.empty_like(B)
        for _ in range(20):     # plain copy of one n x s block: calibration of the traffic counters
            C.copy_(B)
        torch.cuda.synchronize()
        print(json.dumps({"spmm": roof, "copy_bytes_per_launch": 2 * B.numel() * 8}), flush=True)
        return
    Xs = {m: torch.zeros_like(B) for m in METHODS}
    torch.cuda.synchronize()

    infos = {}
    lanes = {}
    if args.concurrent:
        # one context (own stream, own arena) and one matrix handle per method
        import threading
        for m in METHODS:
            st_m = torch.cuda.Stream()
            c_m = pkg.Context(0, stream=st_m.cuda_stream)
            lanes[m] = (c_m, pkg.Matrix.from_csr(c_m, A_csr), st_m)

    mixed_kw = dict(precision="fp32_refine", inner_tol=1e-4, max_outer=20)

    def solve_one(m, per_method, mixed, out):
        c_m, A_m = (lanes[m][0], lanes[m][1]) if lanes else (ctx, A)
        tm = time.perf_counter()
        X, info = pkg.solve(c_m, A_m, B, m, X=Xs[m], x0_zero=True, tol=args.tol, maxit=args.maxit,
                            **(mixed_kw if mixed else {}))
        if per_method is not None:
            if lanes:
                lanes[m][2].synchronize()
            else:
                torch.cuda.synchronize()
            per_method[m] += time.perf_counter() - tm
        out[m] = (X, info)

    def solve_all(per_method=None, mixed=False, out=infos):
        if not lanes:
            for m in METHODS:
                solve_one(m, per_method, mixed, out)
            return
        errors = {}

        def run(m):
            try:
                solve_one(m, per_method, mixed, out)
            except Exception as ex:   # re-raised below, after every thread has ended
                errors[m] = ex

        ths = [threading.Thread(target=run, args=(m,)) for m in METHODS]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        if errors:
            raise RuntimeError(f"concurrent solves failed: {errors}")

    for _ in range(args.warmup):
        solve_all()
        log("warmup step done: " + ", ".join(f"{m} it={infos[m][1].iterations} st={infos[m][1].status_name}"
                                             for m in METHODS))
    torch.cuda.synchronize()
    times = []
    per_method = {m: 0.0 for m in METHODS}
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        solve_all(per_method)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {k}: {times[-1]:.3f} s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ms_per_step = 1e3 * total / args.steps
    # only right-hand sides that reached the tolerance count as solved; the time
    # of a solve that did not converge within maxit still counts
    solved = sum(s for m in METHODS if infos[m][1].status == 0)
    value = solved / (total / args.steps)

    # the same step with FP32 inner solves inside FP64 iterative refinement, in
    # the same execution mode as the FP64 step (concurrent or one after another)
    mixed = {}
    t_mixed = 0.0
    if args.mixed_steps > 0:
        minfo = {}
        mper = {m: 0.0 for m in METHODS}
        solve_all(mixed=True, out=minfo)          # warm-up: FP32 value copies, graphs
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        for k in range(args.mixed_steps):
            solve_all(mper, mixed=True, out=minfo)
            torch.cuda.synchronize()
        t_mixed = time.perf_counter() - tm0
        for m in METHODS:
            info = minfo[m][1]
            dt = mper[m] / args.mixed_steps
            mixed[m] = {"status": info.status_name, "outer": info.outer_iterations,
                        "outer_redone_in_fp64": info.fp64_outer_iterations,
                        "inner_iterations": info.iterations, "rel_res_true": info.rel_res_true,
                        "s_per_solve": round(dt, 4), "rhs_per_s": round(s / dt, 3)}
        log("mixed step: " + ", ".join(f"{m} {mixed[m]['status']} outer={mixed[m]['outer']}" for m in METHODS))

    roof = spmm_roofline(pkg, ctx, A, n, nnz, s, stream)
    gpu_iters = {m: infos[m][1].iterations for m in METHODS}
    out = {
        "metric": "solved RHS/s at 1e-8 rel. residual (FP64 vs mixed); SpMM HBM GB/s vs peak",
        "value": round(value, 4), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"convdiff3d-{args.grid}^3-s16", "n": n, "nnz": nnz, "s": s,
                   "methods": list(METHODS), "tol": args.tol, "maxit": args.maxit, "format": "csr",
                   "precision": "fp64", "concurrent_solves": bool(args.concurrent),
                   "rhs_per_step": len(METHODS) * s, "rhs_solved_per_step": solved},
        "per_method": {m: {"iterations": infos[m][1].iterations, "status": infos[m][1].status_name,
                           "rel_res_true": infos[m][1].rel_res_true,
                           "s_per_solve": round(per_method[m] / args.steps, 4),
                           "rhs_per_s": round(s / (per_method[m] / args.steps), 3)} for m in METHODS},
        "roofline": roof,
    }
    if args.mixed_steps > 0:
        ok = sum(s for m in METHODS if mixed[m]["status"] == "ok")
        out["mixed_fp32_refine"] = {"value": round(ok / (t_mixed / args.mixed_steps), 4), "unit": "RHS/s",
                                    "steps": args.mixed_steps, "concurrent_solves": bool(args.concurrent),
                                    "per_method": mixed}
    if not args.no_config1:
        out["config1_latency"] = config1_latency(pkg, inputs)
    if not args.no_cpu:
        prob = inputs.Problem("convdiff3d", A_csr, B_np, METHODS, {})
        out["cpu_baseline"] = cpu_baseline(prob, gpu_iters, solved, args.grid)
    print(json.dumps(out), flush=True)
    for c_m, A_m, _ in lanes.values():
        A_m.close()
        c_m.close()
    A.close()
    ctx.close()


if __name__ == "__main__":
    main()
