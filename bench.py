#!/usr/bin/env python3
"""LS-AMG-DD solve throughput on one MI355X.

Metric: solve DOF/s to a 1e-8 relative residual (PCG from x0 = 0, one V-cycle
per iteration) plus setup seconds, FP32 cycle inside FP64 PCG versus the plain
FP64 method, on the grad-div workload in H(div): RTCF_3 on a 128 x 128 quad
mesh of the unit square (295,680 DOFs), kappa_T ~ lognormal(0, 1) on the div
term, 1e-4 mass weight, two standard-aggregation passes on level 0, threshold
tau_cut = 0.75 max mult, at most 3 levels.  Inputs are seeded synthetic data
(numpy default_rng(0)) already resident in HBM when timing starts.

A step = one complete PCG solve on the resident hierarchy (V-cycles with the
colour-parallel Schwarz smoother, transfers, coarsest solve, PCG vector work).
Setup (element Gram factors, aggregation, local spectral problems, Galerkin
products, subdomain and coarsest inverses) is timed separately and reported
as setup_s.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 128] [--no-cpu-baseline]

Other workloads (not the default line): --workload batch (64 uneven Q1 elasticity
instances, 8 right-hand sides each, one batched hierarchy) and --workload q2grad
(Q2 hexahedral elasticity on 24^3 with per-element coefficients: solve, adjoint
gradient of the compliance and central differences on 32 elements), --workload h2
(bicubic Hermite hyperdiffusion on 256 x 256) and --workload closure_table (the
closure comparison of Sec. 5.3: standalone V-cycles from a random start to a 1e-10
residual reduction on CG1 triangles, 1,089 ... 1,050,625 DOFs, A-closure against
G-row closure).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve DOF/s to 1e-8 rel residual + setup s; FP32-cycle vs FP64, 1 MI355X"
HBM_PEAK_GBS = 8000.0
SMOOTHERS = {"ms": 0, "ras": 1, "bj": 2}
SMOOTHER = 0          # set from --smoother

# HBM bytes per launch of the dominant solve kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs of this bench (FP64 cycle, 128 x 128; average over the 220 launches of one traced solve)
# scaled by a 1 GiB device-copy calibration (read factor 2.0, write factor 1.0).  Valid only for
# the kernel source these counters were taken on: the hash covers the text of the k_sub_symv
# template in kernels.hip and the partial-sum layout header symv.hpp.
TRAFFIC = {("sub_symv", "graddiv_rtcf3_128x128", "f64"): ("2df36fed9990df39", 2.501e8)}


def _kernels_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_2607_07485_amd", "csrc")
    src = open(os.path.join(csrc, "kernels.hip")).read()
    i = src.index("__global__ void __launch_bounds__(WG) k_sub_symv(")
    text = src[src.rindex("template", 0, i):src.index("\n}\n", i) + 3]
    return hashlib.sha256((text + open(os.path.join(csrc, "symv.hpp")).read()).encode()).hexdigest()[:16]


def _params(P, **kw):
    base = dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1, precision=1, rtol=1e-8,
                smoother=SMOOTHER)
    base.update(kw)
    return P.Params.default(**base)


def _timed_solves(torch, h, b, steps, warmup):
    for _ in range(warmup):
        x, inf = h.solve(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for _ in range(steps):
        x, inf = h.solve(b)
        its.append(inf[0].iters)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return x, dt, its, inf[0]


def _anorm_err(h, x, x_ref):
    e = x - x_ref
    Ae = h.apply(e)
    Ax = h.apply(x_ref)
    return float(np.sqrt(abs(float((e * Ae).sum())) / float((x_ref * Ax).sum())))


def _anorm_err_max(h, X, X_ref, seg_off):
    """Largest relative A-norm error over the (instance, right-hand side) pairs: A is
    block diagonal over the instances, so each segment's error is measured alone."""
    worst = 0.0
    Xs = X if X.dim() == 2 else X[None]
    Rs = X_ref if X_ref.dim() == 2 else X_ref[None]
    for x, xr in zip(Xs, Rs):
        e = (x - xr).contiguous()
        Ae, Ar = h.apply(e), h.apply(xr.contiguous())
        for a, b in zip(seg_off[:-1], seg_off[1:]):
            num = float((e[a:b] * Ae[a:b]).sum())
            den = float((xr[a:b] * Ar[a:b]).sum())
            worst = max(worst, float(np.sqrt(abs(num) / den)) if den > 0 else 0.0)
    return worst


def _reference_solution(h, b):
    """FP64-cycle PCG to 1e-12 on the same hierarchy (the reference of the A-norm errors)."""
    h.set_cycle_precision(0)
    h.set_solve_params(1e-12, 3000)
    x_ref, _ = h.solve(b, allow_noconv=True)
    h.set_solve_params(1e-8, 1000)
    return x_ref


def _extended_reference(h, b_np):
    """Solution of A_0 x = b accurate beyond FP64: sparse LU of the library's assembled A_0
    in FP64 plus iterative refinement with residuals and iterate in extended precision
    (numpy longdouble, 64-bit mantissa): each step contracts by about eps_64 cond(A), the
    result is within about eps_ld cond(A) of the exact solution.  FP64 solvers themselves
    stop near eps_64 cond(A) from it on ill-conditioned operators.  Returns (x, A)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    ex = h.export_level(0)
    n = len(ex["rowptr"]) - 1
    A = sp.csr_matrix((ex["val"], ex["col"], ex["rowptr"]), shape=(n, n))
    A.sort_indices()
    lu = spla.splu(A.tocsc())
    ld = np.longdouble
    x = lu.solve(b_np).astype(ld)
    for _ in range(6):
        r = b_np.astype(ld) - np.add.reduceat(A.data.astype(ld) * x[A.indices], A.indptr[:-1])
        x = x + lu.solve(np.asarray(r, dtype=np.float64)).astype(ld)
    return np.asarray(x, dtype=np.float64), A


def _anorm_rel(A, x, x_ref):
    d = x - x_ref
    return float(np.sqrt(d @ (A @ d)) / np.sqrt(x_ref @ (A @ x_ref)))


def cpu_baseline(N_sample: int):
    """The oracle, as it stands, on the same workload at a bounded size."""
    import fegen
    import oracle
    prob, b = fegen.graddiv_hdiv(N=N_sample)
    t0 = time.perf_counter()
    h = oracle.setup(prob, oracle.Params(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1))
    t1 = time.perf_counter()
    x, info = oracle.pcg(h, b)
    t2 = time.perf_counter()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": prob.n / (t2 - t1), "unit": "DOF/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"same workload at {N_sample}x{N_sample} ({prob.n} DOFs): oracle setup {t1 - t0:.2f} s, "
                      f"PCG {info.iters} its in {t2 - t1:.2f} s",
            "setup_s": t1 - t0}


def _practical_read_gbs(torch):
    """Measured read ceiling of this GPU: the fastest of five full reductions of a 2 GiB
    FP64 tensor (torch's own sum, timed with events), in GB/s.  Context for the
    roofline fractions, which stay against the published 8 TB/s."""
    x = torch.ones(1 << 28, dtype=torch.float64, device="cuda:0")
    best = float("inf")
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x.sum()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    n = x.numel() * 8
    del x
    torch.cuda.empty_cache()
    return n / best / 1e9


def _trace_dominant(h, torch, run):
    """Per-kernel HIP-event timing of one more run; returns (kernels dict, dominant (name, rec))."""
    h.trace(True)
    run()
    h.trace(False)
    tr = h.trace_read()
    dom = max(tr.items(), key=lambda kv: kv[1]["ms"])
    kernels = {k: dict(launches=v["launches"], ms=round(v["ms"], 4),
                       gbs=round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)) for k, v in tr.items()}
    return kernels, dom


def run_batch(a, torch, P, fegen, dev):
    """64 uneven Q1 elasticity instances (N_i ~ U{48..256}, nu_i ~ U(0.3, 0.49)), 8 RHS each, one
    batched hierarchy (vertex-patch cover on level 0, threshold modes, paper stopping tests per
    instance); FP64 and FP32 cycles in FP64 PCG, one recurrence per (instance, RHS)."""
    batch = fegen.elasticity_batch(64, 48, 256, seed=0, nrhs=8)
    probs = [p for p, _ in batch]
    B_np = np.ascontiguousarray(np.concatenate([bb for _, bb in batch], axis=1))
    n_tot, nrhs = B_np.shape[1], B_np.shape[0]
    B = torch.from_numpy(B_np).to(dev)
    # both cycles at the residual that meets the 1e-8 A-norm gate on every pair
    prm = _params(P, max_levels=a.max_levels or 3, rtol=2.5e-9)
    P.Hierarchy.setup_batched([fegen.elasticity_q1(4)], prm).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_batched(probs, prm)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] batch setup {setup_s:.2f} s, levels {info['n']}", file=sys.stderr, flush=True)
    res, sols = {}, {}
    for prec in (0, 1):
        h.set_cycle_precision(prec)
        h.set_graph(False)
        tuning = h.autotune(block=True)
        h.set_graph(True)
        X, infs = h.solve(B, allow_noconv=True)
        if not all(f.converged for f in infs):
            # a smoother other than the default may not give a convergent cycle on every instance
            bad = sum(1 for f in infs if not f.converged)
            res["fp32" if prec else "fp64"] = {"converged": False, "not_converged_pairs": bad}
            print(f"[bench] batch prec {prec}: {bad} (instance, rhs) pairs did not converge", file=sys.stderr,
                  flush=True)
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            X, infs = h.solve(B)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        its = [f.iters for f in infs]
        sols["fp32" if prec else "fp64"] = X.clone()
        res["fp32" if prec else "fp64"] = {"value": n_tot * nrhs / dt, "ms_per_step": dt * 1e3,
                                          "iters_min": min(its), "iters_max": max(its),
                                          "converged": all(f.converged for f in infs), "tuning": tuning}
        print(f"[bench] batch prec {prec}: {dt * 1e3:.1f} ms, its {min(its)}..{max(its)}", file=sys.stderr,
              flush=True)
    h.set_graph(False)
    ok = [k for k in ("fp64", "fp32") if res[k].get("converged")]
    if ok:
        X_ref = _reference_solution(h, B)
        seg = h.segments()[1]
        for k_ in ok:
            res[k_]["anorm_err_max"] = _anorm_err_max(h, sols[k_], X_ref, seg)
    if not ok:
        h.close()
        print(json.dumps({"metric": METRIC, "value": None, "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
                          "config": {"workload": f"elasticity_q1_batch64_{nrhs}rhs", "n_dofs": n_tot,
                                     "smoother": a.smoother},
                          "setup_s": setup_s, **res, "roofline": None, "cpu_baseline": None}))
        return
    h.set_cycle_precision(1 if "fp32" in ok else 0)
    kernels, (dname, d) = _trace_dominant(h, torch, lambda: h.solve(B, allow_noconv=True))
    if ok and not a.no_galerkin32:
        res["fp32_galerkin32"] = _batch_galerkin32(a, torch, P, probs, B, X_ref, h.segments()[1], n_tot * nrhs)
    h.close()
    best = max(ok, key=lambda k: res[k]["value"])
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out = {"metric": METRIC, "value": res[best]["value"], "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
           "warmup": 1, "ms_per_step": res[best]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if best == "fp32" else "f64", "data": "synthetic",
           "config": {"workload": f"elasticity_q1_batch64_{nrhs}rhs", "n_dofs": n_tot, "nrhs": nrhs,
                      "levels": info["n"], "oc": round(info["oc"], 3)},
           "setup_s": setup_s, **res,
           "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1)},
           "kernels": kernels, "cpu_baseline": None}
    print(json.dumps(out))


def _batch_galerkin32(a, torch, P, probs, B, X_ref, seg, n_work):
    """The batch again with its Galerkin products on the FP32 matrix cores (operands rounded
    to FP32, FP32 accumulation) and the FP32 cycle: setup time, solve rate, iterations and
    the A-norm error against the FP64 hierarchy's reference solution (same A_0)."""
    prm = _params(P, max_levels=a.max_levels or 3, rtol=2.5e-9, galerkin_precision=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        g = P.Hierarchy.setup_batched(probs, prm)
    except P.LsddError as ex:
        return {"setup_error": str(ex)}
    torch.cuda.synchronize()
    out = {"setup_s": time.perf_counter() - t0}
    g.set_cycle_precision(1)
    g.set_graph(False)
    g.autotune(block=True)
    g.set_graph(True)
    X, infs = g.solve(B, allow_noconv=True)
    if all(f.converged for f in infs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            X, infs = g.solve(B)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        its = [f.iters for f in infs]
        g.set_graph(False)
        out.update(value=n_work / dt, ms_per_step=dt * 1e3, iters_min=min(its), iters_max=max(its), converged=True,
                   anorm_err_max=_anorm_err_max(g, X, X_ref, seg))
    else:
        out.update(converged=False, not_converged_pairs=sum(1 for f in infs if not f.converged))
    g.close()
    print(f"[bench] batch with FP32 Galerkin products: {out}", file=sys.stderr, flush=True)
    return out


def run_h2(a, torch, P, fegen, dev):
    """Bicubic Hermite anisotropic hyperdiffusion on 256 x 256 (264,196 DOFs), eps = 1e-4 rotated
    30 degrees, Nitsche clamp; threshold modes with tau_cut = max mult, at most 4 levels."""
    N = a.N if a.N != 128 else 256
    prob, b_np = fegen.hyperdiffusion_h2(N=N)
    b = torch.from_numpy(b_np).to(dev)
    prm = _params(P, max_levels=4, tau_const=1.0)
    P.Hierarchy.setup_problem(fegen.hyperdiffusion_h2(N=8)[0], prm).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_problem(prob, prm)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] h2 setup {setup_s:.2f} s, levels {info['n']}", file=sys.stderr, flush=True)
    h.set_cycle_precision(0)
    tuning = h.autotune(block=False)
    h.set_graph(True)
    res, sols = {}, {}
    for prec in (0, 1):
        h.set_cycle_precision(prec)
        try:
            x, inf = h.solve(b, allow_noconv=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.steps):
                x, inf = h.solve(b, allow_noconv=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / a.steps
            sols["fp32" if prec else "fp64"] = x.clone()
            res["fp32" if prec else "fp64"] = {"value": prob.n / dt, "ms_per_step": dt * 1e3, "iters": inf[0].iters,
                                              "converged": bool(inf[0].converged)}
        except P.LsddError as ex:
            res["fp32" if prec else "fp64"] = {"converged": False, "error": str(ex)}
        print(f"[bench] h2 prec {prec}: {res['fp32' if prec else 'fp64']}", file=sys.stderr, flush=True)
    h.set_cycle_precision(0)
    h.set_graph(False)
    x_ref = _reference_solution(h, b)
    for k_ in ("fp64", "fp32"):
        if res[k_].get("converged"):
            res[k_]["anorm_err"] = _anorm_err(h, sols[k_], x_ref)
    kernels, (dname, d) = _trace_dominant(h, torch, lambda: h.solve(b))
    h.close()
    ok = [k for k in ("fp64", "fp32") if res[k].get("converged")]
    best = max(ok, key=lambda k: res[k]["value"])
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out = {"metric": METRIC, "value": res[best]["value"], "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
           "warmup": 1, "ms_per_step": res[best]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if best == "fp32" else "f64", "data": "synthetic",
           "config": {"workload": f"hyperdiffusion_bfs_{N}x{N}", "n_dofs": prob.n, "levels": info["n"],
                      "oc": round(info["oc"], 3)},
           "setup_s": setup_s, "tuning": tuning, **res,
           "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1)},
           "kernels": kernels, "cpu_baseline": None}
    print(json.dumps(out))


def run_closure_table(a, torch, P, fegen, dev):
    """Sec. 5.3 closure comparison: -div((1 + x + y) grad u) = 0 on CG1 triangles of the
    uniformly refined unit square, u = 0 by Nitsche, standalone V-cycles from a N(0, 1)
    start until the residual falls by 1e-10; tau_cut = max mult, two aggregation passes,
    at most 3 levels; A-closure (closure = 1) against G-row closure (closure = 0)."""
    sizes = [32, 64, 128, 256, 512, 1024]
    P.Hierarchy.setup_problem(fegen.closure_comparison(8)[0], _params(P, tau_const=1.0)).close()
    rows = []
    for N in sizes:
        prob, b_np, x0_np = fegen.closure_comparison(N)
        b = torch.from_numpy(b_np).to(dev)
        for cl in (1, 0):
            prm = _params(P, tau_const=1.0, closure=cl, rtol=1e-10, max_iter=3000, precision=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = P.Hierarchy.setup_problem(prob, prm)
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            info = h.info()
            x = torch.from_numpy(x0_np).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, inf = h.solve_stationary(b, x, allow_noconv=True)
            torch.cuda.synchronize()
            solve_s = time.perf_counter() - t0
            h.close()
            row = {"n": prob.n, "closure": "A" if cl else "G", "cycles": inf[0].iters,
                   "converged": bool(inf[0].converged), "rel_res": inf[0].rel_res, "levels": info["n"],
                   "oc": round(info["oc"], 3), "setup_s": round(setup_s, 3), "solve_s": round(solve_s, 4),
                   "ms_per_cycle": round(solve_s * 1e3 / max(inf[0].iters, 1), 3)}
            rows.append(row)
            print(f"[bench] closure table {row}", file=sys.stderr, flush=True)
    big = [r for r in rows if r["n"] == max(r2["n"] for r2 in rows) and r["closure"] == "G"][0]
    out = {"metric": "standalone_cycle_solve_dofs_per_s", "value": big["n"] / big["solve_s"], "unit": "DOF/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": big["solve_s"] * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "closure_comparison_cg1_triangles", "sizes": [(n + 1) ** 2 for n in sizes],
                      "reduction": 1e-10, "tau_const": 1.0},
           "table": rows,
           "paper_cycles": {"A": [10, 12, 13, 28, 72, 158], "G": [10, 10, 11, 11, 11, 11]},
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def run_setup_only(a, torch, P, fegen, dev):
    """One hierarchy build of the grad-div or Q2-hex workload (after a small warm-up build
    that loads the code objects), for profiling the setup kernels."""
    if a.workload == "q2grad":
        N = a.N if a.N != 128 else 24
        theta = np.exp(0.5 * np.random.default_rng(0).standard_normal(N ** 3))
        prob = fegen.elasticity_q2hex(N, nu=0.3, theta=theta)
        prm = _params(P, max_levels=3, agg_passes=1, agg_passes_coarse=1)
        warm = fegen.elasticity_q2hex(2, nu=0.3)
        name = f"elasticity_q2hex_{N}cubed"
    elif a.workload == "graddiv":
        prob, _ = fegen.graddiv_hdiv(N=a.N)
        prm = _params(P)
        warm = fegen.graddiv_hdiv(N=4)[0]
        name = f"graddiv_rtcf3_{a.N}x{a.N}"
    else:
        raise SystemExit("--setup-only supports --workload graddiv and q2grad")
    P.Hierarchy.setup_problem(warm, prm).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_problem(prob, prm)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    h.close()
    print(json.dumps({"metric": "setup_s", "value": setup_s, "unit": "s", "higher_is_better": False,
                      "config": {"workload": name, "n_dofs": prob.n, "levels": info["n"]}}))


def run_q2grad(a, torch, P, fegen, dev):
    """Q2 hex elasticity on N^3 (default 24^3), theta ~ lognormal(0, 0.5); compliance J = b^T u and its
    gradient through the autograd Function (adjoint solve on the same hierarchy), checked by central
    differences on 32 elements with the hierarchy kept as the preconditioner."""
    from paper_2607_07485_amd import autograd as AG
    N = a.N if a.N != 128 else 24
    rng = np.random.default_rng(0)
    theta = np.exp(0.5 * rng.standard_normal(N ** 3))
    prob = fegen.elasticity_q2hex(N, nu=0.3)
    b_np = rng.standard_normal(prob.n)
    prm = _params(P, max_levels=3, agg_passes=1, agg_passes_coarse=1)
    system = AG.ElementSystem(prob, prm)
    th = torch.tensor(theta, device=dev, requires_grad=True)
    b = torch.tensor(b_np, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = AG.solve(th, b, system)
    J = torch.dot(b, u)
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    g = th.grad.cpu().numpy()
    homog = abs(float(theta @ g) + J.item()) / J.item()
    print(f"[bench] q2grad forward+backward {t_grad:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    h = system.hierarchy(torch.tensor(theta, device=dev))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    res, sols, tunings = {}, {}, {}
    for prec in (0, 1):                    # launch shapes (and full-product form) per cycle precision
        h.set_cycle_precision(prec)
        tunings["fp32" if prec else "fp64"] = h.autotune(block=False)
    h.set_graph(True)
    for prec in (0, 1):
        h.set_cycle_precision(prec)
        h.set_tuning(tunings["fp32" if prec else "fp64"])
        x, inf = h.solve(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            x, inf = h.solve(b)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        sols["fp32" if prec else "fp64"] = x.clone()
        res["fp32" if prec else "fp64"] = {"value": prob.n / dt, "ms_per_step": dt * 1e3, "iters": inf[0].iters}
    h.set_graph(False)
    setup_lib_s = inf[0].setup_s          # the library's own clock around the hierarchy build
    x_ref = _reference_solution(h, b)
    for k_ in ("fp64", "fp32"):
        res[k_]["anorm_err"] = _anorm_err(h, sols[k_], x_ref)
    h.set_cycle_precision(0)
    h.set_solve_params(1e-11, 1000)
    errs = []
    for e in rng.choice(len(theta), size=32, replace=False):
        step = 1e-4 * theta[e]
        Js = []
        for sgn in (1.0, -1.0):
            tp = theta.copy()
            tp[e] += sgn * step
            h.update_theta(torch.tensor(tp, device=dev))
            x, _ = h.solve(b)
            Js.append(torch.dot(b, x).item())
        errs.append(abs((Js[0] - Js[1]) / (2 * step) - g[e]) / abs(g[e]))
    h.update_theta(torch.tensor(theta, device=dev))
    h.set_solve_params(1e-8, 1000)
    best = max(("fp64", "fp32"), key=lambda k: res[k]["value"])
    h.set_cycle_precision(1 if best == "fp32" else 0)
    h.set_tuning(tunings[best])
    kernels, (dname, d) = _trace_dominant(h, torch, lambda: h.solve(b))
    h.close()
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    out = {"metric": METRIC, "value": res[best]["value"], "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
           "warmup": 1, "ms_per_step": res[best]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64" if best == "fp32" else "f64", "data": "synthetic",
           "config": {"workload": f"elasticity_q2hex_{N}cubed_grad", "n_dofs": prob.n, "levels": info["n"]},
           "setup_s": setup_s, "setup_lib_s": setup_lib_s, **res, "tuning": tunings, "graphs": True,
           "gradient": {"forward_backward_s": t_grad, "homogeneity_rel": homog,
                        "fd_max_rel_err": max(errs), "fd_median_rel_err": float(np.median(errs)),
                        "fd_elements": 32},
           "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                        "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1)},
           "kernels": kernels, "cpu_baseline": None}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--max-levels", type=int, default=None,
                    help="hierarchy depth cap (default 3)")
    ap.add_argument("--cpu-sample", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-leg", action="store_true",
                    help="skip the FP32/FP64 legs on the 64-instance Q1 batch in the default line")
    ap.add_argument("--no-galerkin32", action="store_true",
                    help="skip the hierarchies with FP32 matrix-core Galerkin products")
    ap.add_argument("--workload", choices=["graddiv", "batch", "q2grad", "h2", "closure_table"], default="graddiv")
    ap.add_argument("--smoother", choices=list(SMOOTHERS), default="ms",
                    help="block Schwarz smoother: multiplicative (default), restricted additive, block Jacobi")
    ap.add_argument("--setup-only", action="store_true",
                    help="only build the hierarchy of the workload (graddiv or q2grad) once and report setup_s "
                         "(for profiling the setup kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB five times (HBM counter calibration for profiling)")
    a = ap.parse_args()
    global SMOOTHER
    SMOOTHER = SMOOTHERS[a.smoother]
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (the hot path has no multi-GPU leg); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if a.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")      # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": src.numel() * 8, "copies": 5}))
        return

    import fegen
    import paper_2607_07485_amd as P

    dev = torch.device("cuda:0")
    print(f"[bench] device {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    # a stream of our own (default priority), so the PCG iteration can run as captured HIP graphs
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if a.setup_only:
            return run_setup_only(a, torch, P, fegen, dev)
        if a.workload == "batch":
            return run_batch(a, torch, P, fegen, dev)
        if a.workload == "q2grad":
            return run_q2grad(a, torch, P, fegen, dev)
        if a.workload == "h2":
            return run_h2(a, torch, P, fegen, dev)
        if a.workload == "closure_table":
            return run_closure_table(a, torch, P, fegen, dev)
        return run_graddiv(a, torch, P, fegen, dev)


def _batch_legs(a, torch, P, fegen, dev):
    """FP64 and FP32 cycles on the 64-instance Q1 batch (8 right-hand sides), both at the
    residual that meets the 1e-8 A-norm gate on every (instance, right-hand side) pair."""
    batch = fegen.elasticity_batch(64, 48, 256, seed=0, nrhs=8)
    probs = [p for p, _ in batch]
    B_np = np.ascontiguousarray(np.concatenate([bb for _, bb in batch], axis=1))
    n_tot, nrhs = B_np.shape[1], B_np.shape[0]
    B = torch.from_numpy(B_np).to(dev)
    rtol = 2.5e-9
    P.Hierarchy.setup_batched([fegen.elasticity_q1(4)], _params(P, max_levels=3, rtol=rtol)).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_batched(probs, _params(P, max_levels=3, rtol=rtol))
    torch.cuda.synchronize()
    out = {"workload": f"elasticity_q1_batch64_{nrhs}rhs", "n_dofs": n_tot, "rtol": rtol,
           "setup_s": time.perf_counter() - t0}
    sols = {}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        h.set_cycle_precision(prec)
        h.set_graph(False)
        h.autotune(block=True)
        h.set_graph(True)
        X, infs = h.solve(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            X, infs = h.solve(B)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        its = [f.iters for f in infs]
        sols[name] = X.clone()
        out[name] = {"value": n_tot * nrhs / dt, "ms_per_step": dt * 1e3, "iters_min": min(its),
                     "iters_max": max(its)}
    h.set_graph(False)
    X_ref = _reference_solution(h, B)
    seg = h.segments()[1]
    for name in ("fp64", "fp32"):
        out[name]["anorm_err_max"] = _anorm_err_max(h, sols[name], X_ref, seg)
    out["fp32_vs_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    if not a.no_galerkin32:
        out["fp32_galerkin32"] = _batch_galerkin32(a, torch, P, probs, B, X_ref, seg, n_tot * nrhs)
    h.close()
    return out


def run_graddiv(a, torch, P, fegen, dev):
    # load code objects once on a tiny instance so setup timing excludes module loading
    pw, bw = fegen.graddiv_hdiv(N=4)
    P.Hierarchy.setup_problem(pw, _params(P, max_levels=a.max_levels or 3, precision=2)).close()

    prob, b_np = fegen.graddiv_hdiv(N=a.N)
    b = torch.from_numpy(b_np).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_problem(prob, _params(P, max_levels=a.max_levels or 3, precision=2))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] setup {setup_s:.2f} s, levels {info['n']}, oc {info['oc']:.2f}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    x_true, A0 = _extended_reference(h, b_np)
    print(f"[bench] extended-precision reference solution {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)

    # three cycles inside FP64 PCG, each with launch shapes picked by the autotuner for it:
    # the plain FP64 method; the FP32 cycle (FP32 operator entries and explicit subdomain
    # inverses); the mixed cycle (FP32 factor-form subdomain solves and transfers, FP64
    # operator entries)
    legs, tunings, times = {}, {}, {}
    autotune_s = 0.0
    for name, prec in (("fp64", 0), ("fp32", 1), ("mixed", 2)):
        if a.smoother != "ms" and prec == 2:
            continue
        h.set_cycle_precision(prec)
        h.set_graph(False)
        t0 = time.perf_counter()
        tunings[name] = h.autotune(block=False)
        torch.cuda.synchronize()
        autotune_s += time.perf_counter() - t0
        h.set_graph(True)
        try:
            _, probe = h.solve(b, allow_noconv=True)
            leg = {"converged": bool(probe[0].converged), "iters": probe[0].iters, "rel_res": probe[0].rel_res}
        except P.LsddError as ex:          # PCG breakdown
            leg = {"converged": False, "error": str(ex)}
        if leg["converged"]:
            x, dt, its, _ = _timed_solves(torch, h, b, a.steps, a.warmup)
            leg.update(value=prob.n / dt, ms_per_step=dt * 1e3, iters=its[-1],
                       anorm_err=_anorm_rel(A0, x.cpu().numpy(), x_true))
            times[name] = dt
            print(f"[bench] {name} cycle: {dt * 1e3:.2f} ms/solve, its {its}, A-norm error {leg['anorm_err']:.2e}",
                  file=sys.stderr, flush=True)
        else:
            print(f"[bench] {name} cycle did not converge: {leg}", file=sys.stderr, flush=True)
        legs[name] = leg
    if "fp64" not in times:
        print(json.dumps({"metric": METRIC, "value": None, "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
                          "warmup": a.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": f"graddiv_rtcf3_{a.N}x{a.N}", "n_dofs": prob.n,
                                     "levels": info["n"], "smoother": a.smoother},
                          "setup_s": setup_s, **legs, "roofline": None, "cpu_baseline": None}))
        h.close()
        return
    # accuracy gate: the 1e-8 A-norm bound, or -- where FP64 itself cannot reach it (the
    # grad-div operator: eps cond(A) ~ 2e-6) -- the plain FP64 method's own accuracy (x 1.5)
    gate = max(1e-8, 1.5 * legs["fp64"]["anorm_err"])
    equal = None
    if "mixed" in times:
        equal = {"rtol": 1e-8, "mixed_ms": legs["mixed"]["ms_per_step"], "fp64_ms": legs["fp64"]["ms_per_step"],
                 "mixed_anorm_err": legs["mixed"]["anorm_err"], "fp64_anorm_err": legs["fp64"]["anorm_err"],
                 "equal_accuracy": legs["mixed"]["anorm_err"] <= gate,
                 "speedup_mixed_over_fp64": legs["fp64"]["ms_per_step"] / legs["mixed"]["ms_per_step"]}
        print(f"[bench] mixed vs fp64: {json.dumps(equal)}", file=sys.stderr, flush=True)
    # the reported variant: the fastest one that meets the accuracy gate
    ok = [k for k in times if legs[k]["anorm_err"] <= gate]
    best = min(ok, key=lambda k: times[k])
    prec = {"fp64": 0, "fp32": 1, "mixed": 2}[best]
    dt = times[best]
    h.set_cycle_precision(prec)

    # per-kernel timing of one more solve of each other converged leg (HIP events), for the record
    for name in times:
        if name == best:
            continue
        h.set_cycle_precision({"fp64": 0, "fp32": 1, "mixed": 2}[name])
        h.set_tuning(tunings[name])          # the launch shapes this leg was timed with
        h.trace(True)
        h.solve(b)
        h.trace(False)
        trl = h.trace_read()
        legs[name]["kernels"] = {k: dict(launches=v["launches"], ms=round(v["ms"], 4),
                                         gbs=round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)) for k, v in trl.items()}
        lb = sum(v["bytes"] for v in trl.values())
        legs[name]["cycle_roofline"] = {"achieved": lb / times[name] / 1e9, "frac": lb / times[name] / 1e9 / HBM_PEAK_GBS,
                                        "bytes_per_solve": lb}
        print(f"[bench] {name} kernels {json.dumps(legs[name]['kernels'])}", file=sys.stderr, flush=True)
    h.set_cycle_precision(prec)
    h.set_tuning(tunings[best])
    # live per-kernel timing of one more solve of the reported variant (HIP events on the solve stream)
    h.trace(True)
    h.solve(b)
    h.trace(False)
    tr = h.trace_read()
    dom = max(tr.items(), key=lambda kv: kv[1]["ms"])
    dname, d = dom
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    kernels = {k: dict(launches=v["launches"], ms=round(v["ms"], 4),
                       gbs=round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)) for k, v in tr.items()}
    print(f"[bench] kernels {json.dumps(kernels)}", file=sys.stderr, flush=True)
    # the whole solve against the same roof: every traced launch's algorithmic bytes over
    # the untraced (graph-replayed) solve time
    solve_bytes = sum(v["bytes"] for v in tr.values())
    cycle_gbs = solve_bytes / dt / 1e9
    h.close()

    g32 = None
    if not a.no_galerkin32:
        # the same hierarchy with its Galerkin products on the FP32 matrix cores: the coarse
        # operators lose the mass term (about 1e-8 of the div term) to FP32 cancellation
        try:
            t0 = time.perf_counter()
            g = P.Hierarchy.setup_problem(prob, _params(P, max_levels=a.max_levels or 3, precision=2,
                                                        galerkin_precision=1))
            g32 = {"setup_s": time.perf_counter() - t0}
            g.set_cycle_precision(0)
            x, inf = g.solve(b, allow_noconv=True)
            g32.update(converged=bool(inf[0].converged), iters=inf[0].iters,
                       anorm_err=_anorm_rel(A0, x.cpu().numpy(), x_true))
            g.close()
        except P.LsddError as ex:
            g32 = {"setup_error": str(ex)}
        print(f"[bench] FP32 Galerkin products: {g32}", file=sys.stderr, flush=True)

    batch = None
    if not a.no_batch_leg:
        batch = _batch_legs(a, torch, P, fegen, dev)
        print(f"[bench] batch legs {json.dumps(batch)}", file=sys.stderr, flush=True)

    cb = None
    if not a.no_cpu_baseline:
        cb = cpu_baseline(a.cpu_sample)
        print(f"[bench] cpu baseline {cb['sample']}", file=sys.stderr, flush=True)

    practical = _practical_read_gbs(torch)
    workload = f"graddiv_rtcf3_{a.N}x{a.N}"
    vdt = "f64" if best == "fp64" else "f32+f64"
    rec = TRAFFIC.get((dname, workload, vdt))
    traffic = rec[1] if rec is not None and rec[0] == _kernels_hash() else None
    res = {
        "metric": METRIC, "value": prob.n / dt, "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": vdt, "data": "synthetic",
        "config": {"workload": workload, "n_dofs": prob.n, "levels": info["n"],
                   "oc": round(info["oc"], 3), "gc": round(info["gc"], 3), "rtol": 1e-8,
                   "cycle": {"fp64": "FP64 V-cycle in FP64 PCG", "fp32": "FP32 V-cycle in FP64 PCG",
                             "mixed": "mixed V-cycle (FP32 factor-form local solves, FP64 operator) in FP64 PCG"}[best],
                   "smoother": a.smoother},
        "setup_s": setup_s,
        "autotune_s": autotune_s, "tuning": tunings, "graphs": True,
        **legs,
        "mixed_vs_fp64": equal,
        "anorm_ref": "sparse LU of A_0 with extended-precision iterative refinement (accurate beyond FP64)",
        "accuracy_gate": gate,
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": d["bytes"] / max(d["launches"], 1),
                     "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1),
                     "practical_read_gbs": practical, "frac_of_practical": achieved / practical},
        "cycle_roofline": {"bound": "hbm", "achieved": cycle_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": cycle_gbs / HBM_PEAK_GBS, "bytes_per_solve": solve_bytes,
                           "practical_read_gbs": practical, "frac_of_practical": cycle_gbs / practical,
                           "what": "sum of the algorithmic bytes of every launch of one solve / solve time"},
        "kernels": kernels,
        "galerkin32": g32,
        "batch": batch,
        "cpu_baseline": None if cb is None else {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
