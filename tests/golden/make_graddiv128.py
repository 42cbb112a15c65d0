"""Write the oracle's values for the grad-div workload at its benchmark size.

RTCF_3 on 128 x 128 (295,680 DOFs), kappa_T ~ lognormal(0, 1) on the div term,
beta = 1e-4 mass, seed 0; threshold modes with tau_cut = 0.75 max mult, two
standard-aggregation passes on level 0 and one above, at most 4 levels, PCG to
a 1e-8 relative residual (and to 1e-12 for the reference solution).

Only the oracle runs here (about half an hour on one host); the output
``graddiv128_oracle.npz`` holds the level sizes, the aggregates of the coarse
levels, the retained-mode counts and the eigenvalues on either side of each
aggregate's cut, the PCG iteration count, the reference solution (PCG to 1e-12)
and the A-norm error of the 1e-8 solution against it.

    python tests/golden/make_graddiv128.py [out.npz]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fegen  # noqa: E402
import oracle  # noqa: E402

KW = dict(max_levels=4, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                             "graddiv128_oracle.npz")
    prob, b = fegen.graddiv_hdiv(N=128)
    t0 = time.time()
    h = oracle.setup(prob, oracle.Params(**KW))
    t_setup = time.time() - t0
    print(f"setup {t_setup:.0f} s: n = {[lv.n for lv in h.levels]}", flush=True)
    d = dict(n=np.array([lv.n for lv in h.levels], np.int64), nnz=np.array([lv.nnz for lv in h.levels], np.int64),
             setup_s=t_setup)
    for l, lv in enumerate(h.levels[:-1]):
        k = np.asarray(lv.k, np.int32)
        nw = np.array([len(a) for a in lv.aggs], np.int32)
        m = np.array([len(o) for o in lv.omegas], np.int32)
        last = np.array([mu[ki - 1] if ki > 0 else -1.0 for mu, ki in zip(lv.mu, k)])
        first = np.array([mu[ki] if ki < len(mu) else 2.0 for mu, ki in zip(lv.mu, k)])
        d[f"k{l}"], d[f"nw{l}"], d[f"m{l}"] = k, nw, m
        d[f"mu_kept{l}"], d[f"mu_drop{l}"] = last, first
        d[f"tau_cut{l}"] = lv.tau_cut
        d[f"agg{l}"] = np.asarray(lv.agg_of_dof, np.int32)
    t0 = time.time()
    x, info = oracle.pcg(h, b)
    t_pcg = time.time() - t0
    print(f"pcg 1e-8: {info.iters} iterations, {t_pcg:.0f} s", flush=True)
    xr, ir = oracle.pcg(h, b, rtol=1e-12)
    print(f"pcg 1e-12: {ir.iters} iterations", flush=True)
    A = h.levels[0].A
    e = x - xr
    d.update(iters=info.iters, hist=np.array(info.history), iters_ref=ir.iters, x_ref=xr, pcg_s=t_pcg,
             anorm_err=float(np.sqrt(e @ (A @ e)) / np.sqrt(xr @ (A @ xr))))
    np.savez_compressed(out, **d)
    print(f"A-norm error of the 1e-8 solution: {d['anorm_err']:.3e}; wrote {out}", flush=True)


if __name__ == "__main__":
    main()
