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

# HBM bytes per launch of the dominant solve kernel, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs of this bench (FP64 cycle, 128 x 128) scaled by a 1 GiB device-copy calibration (read
# factor 2.0, write factor 1.0).  Valid only for the kernel source these counters were taken on.
TRAFFIC = {("sub_symv", "graddiv_rtcf3_128x128", "f64"): ("7380094f6174f17c", 2.599e8)}


def _kernels_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_2607_07485_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _params(P, **kw):
    base = dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1, precision=1, rtol=1e-8)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB five times (HBM counter calibration for profiling)")
    a = ap.parse_args()
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
    # load code objects once on a tiny instance so setup timing excludes module loading
    pw, bw = fegen.graddiv_hdiv(N=4)
    P.Hierarchy.setup_problem(pw, _params(P)).close()

    prob, b_np = fegen.graddiv_hdiv(N=a.N)
    b = torch.from_numpy(b_np).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = P.Hierarchy.setup_problem(prob, _params(P))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] setup {setup_s:.2f} s, levels {info['n']}, oc {info['oc']:.2f}", file=sys.stderr, flush=True)

    # plain FP64 method: FP64 V-cycle inside FP64 PCG
    h.set_cycle_precision(0)
    x64, dt64, its64, inf64 = _timed_solves(torch, h, b, a.steps, a.warmup)
    print(f"[bench] fp64 cycle: {dt64 * 1e3:.2f} ms/solve, its {its64}", file=sys.stderr, flush=True)
    h.set_solve_params(1e-12, 2000)
    x_ref, inf_ref = h.solve(b, allow_noconv=True)
    h.set_solve_params(1e-8, 1000)
    err64 = _anorm_err(h, x64, x_ref)

    # FP32 V-cycle inside FP64 (flexible) PCG, at the same 1e-8 stopping rule
    h.set_cycle_precision(1)
    h.set_solve_params(1e-8, 200)
    try:
        _, probe = h.solve(b, allow_noconv=True)
        fp32 = {"converged": bool(probe[0].converged), "iters": probe[0].iters, "rel_res": probe[0].rel_res}
    except P.LsddError as ex:          # PCG breakdown of the FP32 cycle
        fp32 = {"converged": False, "error": str(ex)}
    dt32 = None
    if fp32["converged"]:
        x32, dt32, its32, inf32 = _timed_solves(torch, h, b, a.steps, a.warmup)
        fp32.update(value=prob.n / dt32, ms_per_step=dt32 * 1e3, anorm_err=_anorm_err(h, x32, x_ref))
        print(f"[bench] fp32 cycle: {dt32 * 1e3:.2f} ms/solve, its {its32}", file=sys.stderr, flush=True)
    else:
        print(f"[bench] fp32 cycle did not converge: {fp32}", file=sys.stderr, flush=True)
    h.set_solve_params(1e-8, 1000)
    use32 = dt32 is not None and dt32 < dt64
    h.set_cycle_precision(1 if use32 else 0)
    dt = dt32 if use32 else dt64

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
    out = {"fp64": {"value": prob.n / dt64, "ms_per_step": dt64 * 1e3, "iters": its64[-1], "anorm_err": err64},
           "fp32": fp32, "anorm_ref": f"FP64-cycle PCG to 1e-12 on the same hierarchy ({inf_ref[0].iters} its)"}
    h.close()

    cb = None
    if not a.no_cpu_baseline:
        cb = cpu_baseline(a.cpu_sample)
        print(f"[bench] cpu baseline {cb['sample']}", file=sys.stderr, flush=True)

    workload = f"graddiv_rtcf3_{a.N}x{a.N}"
    rec = TRAFFIC.get((dname, workload, "f32" if use32 else "f64"))
    traffic = rec[1] if rec is not None and rec[0] == _kernels_hash() else None
    res = {
        "metric": METRIC, "value": prob.n / dt, "unit": "DOF/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if use32 else "f64", "data": "synthetic",
        "config": {"workload": workload, "n_dofs": prob.n, "levels": info["n"],
                   "oc": round(info["oc"], 3), "gc": round(info["gc"], 3), "rtol": 1e-8,
                   "cycle": "FP32 V-cycle in FP64 PCG" if use32 else "FP64 V-cycle in FP64 PCG"},
        "setup_s": setup_s,
        **out,
        "roofline": {"bound": "hbm", "kernel": dname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": d["bytes"] / max(d["launches"], 1),
                     "avg_launch_us": d["ms"] * 1e3 / max(d["launches"], 1)},
        "kernels": kernels,
        "cpu_baseline": None if cb is None else {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")},
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
