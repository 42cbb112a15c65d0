"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

The oracle cannot build these hierarchies whole in a test's time, so it checks
what it can compute one piece at a time, from the problem data alone:

* grad-div RTCF_3 on 128 x 128 (295,680 DOFs), FP64 cycle, autotuned launch
  shapes, captured PCG iterations: the assembled operator (all entries, 1e-13),
  sampled element Gram factors (ranks bit-exact, G_T^T G_T to 1e-10), the
  level-0 aggregates and overlap sizes (bit-exact), and the local problems of
  sampled aggregates (eq. gep_reduced).  At this size A_ww reaches condition
  numbers near 1e10, and two correct FP64 routes through the same pencil (the
  Cholesky reduction, LAPACK's generalized solver) already differ by up to
  1e-5 in mu; the spectra are held to ten times that spread of the oracle's
  own (never below 1e-10), the mode counts are bit-exact unless the modes in
  between lie within that tolerance of the cut or of the cluster gap, and the
  projectors Z Z^T onto the leading modes below a gap wider than 1e3 times that
  tolerance to ten times the two routes' own spread.  Properties that hold at any size: A_1 = P^T A_0 P
  for the exported P within the rounding bound of the double sum, the symmetry
  and positivity of the V-cycle, and the normwise backward error of the PCG
  result against the oracle's A.
* the four-level grad-div hierarchy against the values of the oracle's own run at
  this size (tests/golden/): aggregates, retained-mode counts, level sizes, PCG
  iterations and the A-norm error against the oracle's reference solution.
* the 64-instance Q1 batch with 8 right-hand sides, FP32 cycle in FP64 PCG
  (blocks, autotuned shapes, captured iterations): on sampled instances the true
  residuals against the oracle's A and the A-norm errors against a sparse
  direct solve of that A, beside those of the FP64 cycle, both at the 1e-8 gate.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import fegen
import oracle
from refsol import anorm_rel, extended_reference
from oracle import lsdd as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BENCH_KW = dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)


def _lsdd():
    import paper_2607_07485_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch.device("cuda:0")


def _csr(ex):
    n = len(ex["rowptr"]) - 1
    return sp.csr_matrix((ex["val"], ex["col"], ex["rowptr"]), shape=(n, n))


def _elem_lists(prob):
    nE = prob.n_elem
    dofs = [np.asarray(prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]], np.int64) for e in range(nE)]
    offs = prob.block_offsets()
    blocks = [np.asarray(prob.blocks[offs[e]:offs[e + 1]]).reshape(len(dofs[e]), -1) for e in range(nE)]
    return dofs, blocks


MU_TOL = 1e-10          # floor of the local-spectra tolerance (mu in [0, max multiplicity])


@pytest.fixture(scope="module")
def graddiv(dev):
    """The benchmark's grad-div hierarchy and solve (FP64 cycle, tuned shapes, graphs)."""
    P = _lsdd()
    prob, b = fegen.graddiv_hdiv(N=128)
    b = b.ravel()
    prm = P.Params.default(**BENCH_KW, precision=1, rtol=1e-8)
    h = P.Hierarchy.setup_problem(prob, prm)
    h.set_cycle_precision(0)
    h.autotune(block=False)
    h.set_graph(True)
    x, infs = h.solve(torch.from_numpy(b).to(dev))
    x, infs = h.solve(torch.from_numpy(b).to(dev))     # the replayed (captured) iterations
    out = dict(prob=prob, b=b, x=x.cpu().numpy(), info=infs[0], l0=h.export_level(0), l1=h.export_level(1),
               gram=h.export_gram(prob.elem_ptr), levels=h.info(), h=h)
    yield out
    h.close()


def test_graddiv_operator_and_element_factors(graddiv):
    prob = graddiv["prob"]
    assert prob.n == 295680
    dofs, blocks = _elem_lists(prob)
    A = O.assemble(prob.n, dofs, blocks)
    A_gpu = _csr(graddiv["l0"])
    assert np.abs(A_gpu - A).max() <= 1e-13 * np.abs(A).max()
    ranks, G = graddiv["gram"]
    offs = prob.block_offsets()
    rng = np.random.default_rng(11)
    for e in rng.choice(prob.n_elem, 64, replace=False):
        ne = len(dofs[e])
        G_or = O.element_gram_factor(blocks[e])
        assert ranks[e] == G_or.shape[0]
        Ge = G[offs[e]:offs[e + 1]].reshape(ne, ne)[:ranks[e]]
        scale = np.abs(blocks[e]).max()
        assert np.abs(Ge.T @ Ge - G_or.T @ G_or).max() <= 1e-10 * scale


def test_graddiv_aggregates_and_sampled_local_problems(graddiv):
    prob, l0 = graddiv["prob"], graddiv["l0"]
    dofs, blocks = _elem_lists(prob)
    node = np.asarray(prob.node_of_dof, np.int64)
    adj = O.supernode_graph(int(node.max()) + 1, node, dofs)
    agg_of_dof = O.aggregate_supernodes(adj, BENCH_KW["agg_passes"])[node]
    assert np.array_equal(l0["agg_of_dof"], agg_of_dof)
    n_agg = int(agg_of_dof.max()) + 1
    aggs, omegas, cl, mult = O.closures(n_agg, agg_of_dof, dofs)
    assert np.array_equal(l0["omega_sizes"], [len(o) for o in omegas])
    prm = oracle.Params(**BENCH_KW)
    tau_cut = prm.tau_const * float(mult.max())
    A = _csr(l0)
    nw = np.array([len(a) for a in aggs])
    mu_off = np.concatenate([[0], np.cumsum(nw)])
    z_off = np.concatenate([[0], np.cumsum(nw * l0["k"])])
    rng = np.random.default_rng(12)
    sample = list(rng.choice(n_agg, 24, replace=False)) + [int(np.argmax([len(o) for o in omegas]))]
    for i in sample:
        At = O.local_splitting(omegas[i], cl[i], dofs, blocks, mult)
        S = O.schur_pinv(At, nw[i])
        Aww = A[aggs[i]][:, aggs[i]].toarray()
        mu, V, L = O.local_spectral(S, Aww)
        k = O.select_modes(mu, prm, tau_cut)
        # the oracle's own rounding spread on this pencil: the Cholesky reduction
        # against LAPACK's generalized eigensolver, and the pseudo-inverse Schur
        # complement against its projector form on the weighted Gram rows, all FP64.
        # On the finest grad-div level A_ww has condition numbers near 1e10, so two
        # correct FP64 routes differ by far more than 1e-10; the tolerance is ten
        # times the larger spread, never below 1e-10
        mu2, Z2 = sla.eigh(S, Aww)
        H = O.local_gram_rows(omegas[i], cl[i], dofs, {e: O.element_gram_factor(blocks[e]) for e in cl[i]}, mult)
        mu3, _, _ = O.local_spectral(O.schur_projector(H, nw[i]), Aww)
        spread = max(float(np.abs(np.maximum(mu2, 0.0) - mu).max()), float(np.abs(mu3 - mu).max()))
        mu_tol = max(MU_TOL, 10 * spread)
        k_g = int(l0["k"][i])
        mu_g = l0["mu"][mu_off[i]:mu_off[i + 1]]
        assert np.abs(mu_g - mu).max() <= mu_tol, (i, np.abs(mu_g - mu).max(), mu_tol)
        if k_g != k:
            # the count is an integer decided by floating point: it may differ only
            # where every mode in between sits within mu_tol of the cut or of the
            # cluster-completion gap (then both counts are correct)
            thr = 1.0 / tau_cut + prm.band_tol
            for j in range(min(k, k_g), max(k, k_g)):
                near_cut = abs(mu[j] - thr) <= 2 * mu_tol
                near_gap = j > 0 and abs((mu[j] - mu[j - 1]) - prm.cluster_tol) <= 2 * mu_tol
                assert near_cut or near_gap, (i, j, k, k_g, mu[j] - thr, mu_g[j] - thr)
        # retained modes: with spectra known to mu_tol only the span of the modes
        # below a gap much wider than mu_tol is determined, so the A_ww-weighted
        # projectors onto the leading kc modes are compared (basis-free), kc the
        # last such gap within both counts
        kc = 0
        for j in range(min(k, k_g), 0, -1):
            if mu[j] - mu[j - 1] >= 1e3 * mu_tol:
                kc = j
                break
        if kc == 0:
            continue
        Z_or = sla.solve_triangular(L.T, V[:, :kc], lower=False)
        Z_g = l0["Z"][z_off[i]:z_off[i + 1]].reshape(nw[i], k_g)[:, :kc]
        Pi_o, Pi_2, Pi_g = Z_or @ Z_or.T, Z2[:, :kc] @ Z2[:, :kc].T, Z_g @ Z_g.T
        ps = np.abs(Pi_o).max()
        p_tol = max(1e-10, 10 * float(np.abs(Pi_2 - Pi_o).max()) / ps)
        assert np.abs(Pi_g - Pi_o).max() <= p_tol * ps, (i, kc, np.abs(Pi_g - Pi_o).max() / ps, p_tol)


def test_graddiv_galerkin_cycle_and_solution_properties(graddiv, dev):
    prob, l0, l1 = graddiv["prob"], graddiv["l0"], graddiv["l1"]
    assert graddiv["levels"]["n"][:2] == [295680, int(l0["k"].sum())]
    # A_1 = P^T A_0 P for the exported interpolation (aggregate-major coarse DOFs)
    agg = l0["agg_of_dof"]
    k = l0["k"]
    order = np.argsort(agg, kind="stable")
    nw = np.bincount(agg, minlength=len(k))
    a_off = np.concatenate([[0], np.cumsum(nw)])
    c_off = np.concatenate([[0], np.cumsum(k)])
    z_off = np.concatenate([[0], np.cumsum(nw * k)])
    rows, cols, vals = [], [], []
    for i in range(len(k)):
        if k[i] == 0:
            continue
        rows.append(np.repeat(order[a_off[i]:a_off[i + 1]], k[i]))
        cols.append(np.tile(np.arange(c_off[i], c_off[i + 1]), nw[i]))
        vals.append(l0["Z"][z_off[i]:z_off[i + 1]])
    Pm = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(len(agg), int(c_off[-1])))
    A0, A1 = _csr(l0), _csr(l1)
    Ac = (Pm.T @ A0 @ Pm).tocsr()
    # two FP64 evaluations of the same double sum (coarse elements here, the
    # assembled product there): each entry has at most m = (row length of A_0) x
    # (aggregate size) terms, so they differ by at most 2 gamma_m (|P|^T |A_0| |P|)
    # entrywise, gamma_m = m eps / (1 - m eps)
    m = int(np.diff(A0.indptr).max()) * int(nw.max())
    gam = m * np.finfo(float).eps / (1 - m * np.finfo(float).eps)
    Pa = abs(Pm)
    M = (Pa.T @ abs(A0) @ Pa).tocsr()
    D = (A1 - Ac).tocsr()
    bound = 2 * gam * M
    viol = abs(D) - bound
    assert viol.max() <= 0.0, (abs(D).max(), gam)
    # ... and the coarse operator carries the A_ww-orthonormality of the modes
    assert np.abs(A1.diagonal() - 1.0).max() <= 1e-4
    # the V-cycle is a symmetric positive definite map
    h = graddiv["h"]
    rng = np.random.default_rng(13)
    r1, r2 = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    v1 = h.vcycle(torch.from_numpy(r1).to(dev)).cpu().numpy()
    v2 = h.vcycle(torch.from_numpy(r2).to(dev)).cpu().numpy()
    # FP64 rounding through local inverses of condition up to ~1e12 leaves a
    # defect near 1e-9 |V| |r1| |r2| here (measured 8e-10 against a power-iteration
    # estimate of |V|); a smoother applied in the same order before and after the
    # coarse correction would leave one of order 1e-1.  |V| is bounded below by
    # |V r| / |r|, which makes the check stricter
    n1, n2 = np.linalg.norm(r1), np.linalg.norm(r2)
    vn = max(np.linalg.norm(v1) / n1, np.linalg.norm(v2) / n2)
    assert abs(v1 @ r2 - r1 @ v2) <= 2e-8 * vn * n1 * n2
    assert v1 @ r1 > 0 and v2 @ r2 > 0
    # the PCG result meets the residual criterion against the oracle's operator
    dofs, blocks = _elem_lists(prob)
    A = O.assemble(prob.n, dofs, blocks)
    b, x = graddiv["b"], graddiv["x"]
    assert graddiv["info"].converged
    # the normwise backward error: with condition numbers near 1e11 the product
    # A x alone carries rounding near eps |A| |x|, far above 1e-8 |b|, so the
    # residual is measured against the scale that computing it can resolve
    r = b - A @ x
    eta = np.abs(r).max() / (spla.norm(A, np.inf) * np.abs(x).max() + np.abs(b).max())
    assert eta <= 1e-8, eta


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "graddiv128_oracle.npz")
GOLDEN_KW = dict(max_levels=4, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)
# local spectra at this size: two correct FP64 routes through the same pencil differ
# by up to 1e-6 in mu (the Cholesky reduction against LAPACK's generalized solver,
# measured on sampled aggregates); ten times that
GOLDEN_MU_TOL = 1e-5


def test_graddiv_four_levels_against_the_oracle_run(dev):
    """The whole four-level grad-div hierarchy at 128 x 128 against the oracle's own run
    (tests/golden/make_graddiv128.py, the oracle only): level-0 aggregates bit-exact;
    retained-mode counts per level-0 aggregate bit-exact except where every mode in
    between lies within GOLDEN_MU_TOL of the cut 1/tau_cut or of a cluster-completion
    gap; the level-1 size equal to the sum of the counts; the coarser sizes within 1 %
    (their aggregates follow the level-1 numbering); PCG iterations +-1; and the A-norm
    error of the GPU solution against a reference accurate beyond FP64 within twice
    that of the oracle's own FP64 solution (PCG to 1e-12).

    The cut 1/tau_cut = 1/(0.75 * 4) = 1/3 falls on the eigenvalue 1/mult of modes
    that live inside elements touching three aggregates, a cluster that every
    aggregate's spectrum holds; the oracle's own rounding puts members of it up to
    1e-8 on either side of the cut (its first dropped mode lies within 1e-8 of the cut
    on 237 of 493 aggregates), so the counts there are decided by rounding."""
    P = _lsdd()
    g = dict(np.load(GOLDEN))
    prob, b = fegen.graddiv_hdiv(N=128)
    with P.Hierarchy.setup_problem(prob, P.Params.default(**GOLDEN_KW, rtol=1e-8)) as h:
        n = h.info()["n"]
        assert len(n) == 4 and n[0] == int(g["n"][0])
        l0 = h.export_level(0)
        assert np.array_equal(l0["agg_of_dof"], g["agg0"])
        k_g, k_o = np.asarray(l0["k"]), g["k0"]
        thr = 1.0 / float(g["tau_cut0"])
        nw = g["nw0"]
        mu_off = np.concatenate([[0], np.cumsum(nw)])
        prm = oracle.Params(**GOLDEN_KW)
        differ = np.flatnonzero(k_g != k_o)
        for i in differ:
            mu = l0["mu"][mu_off[i]:mu_off[i + 1]]
            for j in range(min(k_g[i], k_o[i]), max(k_g[i], k_o[i])):
                near_cut = abs(mu[j] - thr) <= GOLDEN_MU_TOL
                near_gap = j > 0 and abs((mu[j] - mu[j - 1]) - prm.cluster_tol) <= 2 * GOLDEN_MU_TOL
                assert near_cut or near_gap, (i, j, k_g[i], k_o[i], mu[j] - thr)
        assert n[1] == int(k_g.sum())
        for l in (2, 3):
            assert abs(n[l] - int(g["n"][l])) <= 0.01 * int(g["n"][l]), (n, g["n"])
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert infos[0].converged == 1 and abs(infos[0].iters - int(g["iters"])) <= 1
        dofs, blocks = _elem_lists(prob)
        A = O.assemble(prob.n, dofs, blocks)
        # both solutions against one accurate beyond FP64 (LU + extended-precision
        # refinement): FP64 itself stops near eps cond(A) ~ 2e-6 from it here, so the
        # GPU solution is held to the accuracy of the oracle's own FP64 solution
        x_true = extended_reference(A, b)
        err = anorm_rel(A, x.cpu().numpy(), x_true)
        err_or = anorm_rel(A, g["x_ref"], x_true)
        assert err <= 2.0 * err_or + 1e-9, (err, err_or)
        print(f"four-level grad-div: GPU levels {n}, oracle {g['n'].tolist()}, "
              f"{len(differ)} aggregates with other counts ({int(k_g.sum()) - int(k_o.sum()):+d} modes), "
              f"its {infos[0].iters} / {int(g['iters'])}, A-norm error {err:.2e} (oracle {err_or:.2e})")


def test_q1_batch_sampled_instances(dev):
    P = _lsdd()
    batch = fegen.elasticity_batch(64, 48, 256, seed=0, nrhs=8)
    probs = [p for p, _ in batch]
    B_np = np.ascontiguousarray(np.concatenate([bb for _, bb in batch], axis=1))
    # the stiffest instances (nu near 0.49) stop at an A-norm error near 2e-8 with a
    # 1e-8 residual for either cycle: both are tightened by the same factor (to 2.5e-9)
    # so that every sampled (instance, right-hand side) pair meets the 1e-8 gate
    prm = P.Params.default(**BENCH_KW, precision=1, rtol=2.5e-9)
    h = P.Hierarchy.setup_batched(probs, prm)
    try:
        seg = h.segments()[1]
        assert seg[-1] == B_np.shape[1] == sum(p.n for p in probs)
        sols = {}
        for prec in (0, 1):
            h.set_cycle_precision(prec)
            h.set_graph(False)
            h.autotune(block=True)
            h.set_graph(True)
            X, infs = h.solve(torch.from_numpy(B_np).to(dev))
            assert all(f.converged for f in infs)
            sols[prec] = X.cpu().numpy()
        rng = np.random.default_rng(14)
        sizes = np.array([p.n for p in probs])
        picks = {int(np.argmin(sizes)), int(np.argmax(sizes))} | set(int(i) for i in rng.choice(64, 4, replace=False))
        for i in sorted(picks):
            dofs, blocks = _elem_lists(probs[i])
            A = O.assemble(probs[i].n, dofs, blocks).tocsc()
            lu = spla.splu(A)
            a, e = seg[i], seg[i + 1]
            for q in range(B_np.shape[0]):
                bq = B_np[q, a:e]
                xs = lu.solve(bq)
                nA = np.sqrt(xs @ (A @ xs))
                err = {}
                for prec in (0, 1):
                    xq = sols[prec][q, a:e]
                    assert np.linalg.norm(bq - A @ xq) <= 1.5 * 2.5e-9 * np.linalg.norm(bq), (i, q, prec)
                    d = xq - xs
                    err[prec] = np.sqrt(d @ (A @ d)) / nA
                # the FP32 cycle reaches the accuracy of the FP64 cycle at the same stopping
                # test, and both meet the 1e-8 A-norm gate
                assert err[1] <= 1.1 * err[0] + 1e-10, (i, q, err)
                assert err[0] <= 1e-8 and err[1] <= 1e-8, (i, q, err)
    finally:
        h.close()
