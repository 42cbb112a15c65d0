"""Galerkin products on the FP32 matrix cores (params.galerkin_precision = 1).

Level-0 Gram factors and retained modes are FP64 and identical with either
setting, so the FP32 coarse operator differs from the FP64 one only by the
rounding of Y_e = G_e P_e and A_g = Y^T Y in FP32.  Standard bounds for sums of
products: |fl(Y) - Y| <= gamma_p |G_e| |P_e| and |fl(Y^T Y) - Y^T Y| <=
gamma_q |Y|^T |Y| with gamma_k = k u / (1 - k u), u = 2^-24, p the inner length
of G_e P_e (the element size, plus 2 for rounding the operands to FP32) and q
the rows stacked per group.  The test holds the coarse operator to that bound,
and the solve to the FP64 hierarchy's iteration count and A-norm error.  On
grad-div with beta = 1e-4 the mass term (about 1e-8 of the div term) sits below
FP32 resolution in these products and the coarse operators are no longer
positive definite: the library reports that instead of building a hierarchy.
"""
import numpy as np
import pytest

import fegen
from canon import _csr, _gpu_Z_blocks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch.device("cuda:0")


def _gamma(k):
    return k * U32 / (1.0 - k * U32)


def test_fp32_galerkin_coarse_operator_within_the_fp32_bound(dev):
    import paper_2607_07485_amd as P
    prob, _ = fegen.elasticity_small(N=32)
    kw = dict(max_levels=2, modes_fixed=4)
    with P.Hierarchy.setup_problem(prob, P.Params.default(**kw)) as h64, \
            P.Hierarchy.setup_problem(prob, P.Params.default(galerkin_precision=1, **kw)) as h32:
        l0, l0b = h64.export_level(0), h32.export_level(0)
        assert np.array_equal(l0["Z"], l0b["Z"]) and np.array_equal(l0["k"], l0b["k"])
        A64, A32 = _csr(h64.export_level(1)).toarray(), _csr(h32.export_level(1)).toarray()
        # |Y| |P| products on the host from the FP64 operands the GPU multiplied
        ranks, G = h64.export_gram(prob.elem_ptr)
        agg = l0["agg_of_dof"]
        nw = np.bincount(agg)
        Z = _gpu_Z_blocks(l0, nw)
        coff = np.concatenate([[0], np.cumsum(l0["k"])])
        pos = np.zeros(prob.n, np.int64)                  # row of each DOF inside its aggregate
        for i in range(len(nw)):
            pos[np.flatnonzero(agg == i)] = np.arange(nw[i])
        nc = int(coff[-1])
        absY = np.zeros((int(ranks.sum()), nc))           # |G| |P| rows, all elements stacked
        r0 = 0
        offs = prob.block_offsets()
        for e in range(prob.n_elem):
            S = prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]]
            ne = len(S)
            Ge = np.abs(G[offs[e]:offs[e + 1]].reshape(ne, ne)[:ranks[e]])
            Pe = np.zeros((ne, nc))
            for a, d in enumerate(S):
                i = agg[d]
                Pe[a, coff[i]:coff[i + 1]] = np.abs(Z[i][pos[d]])
            absY[r0:r0 + ranks[e]] = Ge @ Pe
            r0 += ranks[e]
        # inner length of A_g = Y^T Y: the rows stacked for a group (elements touching the
        # same set of aggregates)
        rows_of = {}
        for e in range(prob.n_elem):
            key = tuple(np.unique(agg[prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]]]))
            rows_of[key] = rows_of.get(key, 0) + int(ranks[e])
        q = max(rows_of.values())
        Ybnd = _gamma(8 + 2) * absY                       # 8 = element size, 2 = operand rounding
        # |fl(Y)^T fl(Y) - Y^T Y| <= 2 |Y|^T dY + dY^T dY + gamma_q (|Y| + dY)^T (|Y| + dY)
        bound = 2 * absY.T @ Ybnd + Ybnd.T @ Ybnd + _gamma(q) * (absY + Ybnd).T @ (absY + Ybnd)
        diff = np.abs(A32 - A64)
        assert (diff <= bound + 1e-300).all(), float((diff / np.maximum(bound, 1e-300)).max())
        assert diff.max() > 0.0          # the FP32 path is really taken


def test_fp32_galerkin_solve_matches_the_fp64_hierarchy(dev):
    """Elasticity 32 x 32 and 128 x 128 (three levels): PCG to 1e-8 needs the same
    iterations (+-1) and reaches the FP64 hierarchy's A-norm error (within 1.5x)
    against a reference accurate beyond FP64."""
    import paper_2607_07485_amd as P
    from refsol import anorm_rel, extended_reference
    for N, kw in ((32, dict(max_levels=2, modes_fixed=4)), (128, dict(max_levels=3, modes_fixed=4))):
        prob, b = fegen.elasticity_small(N=N)
        with P.Hierarchy.setup_problem(prob, P.Params.default(**kw)) as h64, \
                P.Hierarchy.setup_problem(prob, P.Params.default(galerkin_precision=1, **kw)) as h32:
            A0 = _csr(h64.export_level(0))
            A0.sort_indices()
            x_true = extended_reference(A0, b)
            bd = torch.from_numpy(b).to(dev)
            x64, i64 = h64.solve(bd)
            x32, i32 = h32.solve(bd)
            assert i64[0].converged == 1 and i32[0].converged == 1
            assert abs(i32[0].iters - i64[0].iters) <= 1
            e64, e32 = anorm_rel(A0, x64.cpu().numpy(), x_true), anorm_rel(A0, x32.cpu().numpy(), x_true)
            assert e32 <= 1.5 * e64 + 1e-12, (N, e64, e32)


def test_fp32_galerkin_batched_instances(dev):
    """Four uneven Q1 instances with 8 right-hand sides, FP32 Galerkin products and
    the FP32 cycle: every (instance, right-hand side) pair converges to 1e-8 within
    one iteration of the FP64-Galerkin hierarchy."""
    import paper_2607_07485_amd as P
    batch = fegen.elasticity_batch(4, 24, 64, seed=3, nrhs=8)
    probs = [p for p, _ in batch]
    B = torch.from_numpy(np.ascontiguousarray(np.concatenate([bb for _, bb in batch], axis=1))).to(dev)
    its = {}
    for g in (0, 1):
        with P.Hierarchy.setup_batched(probs, P.Params.default(max_levels=3, precision=1,
                                                                galerkin_precision=g)) as h:
            h.set_cycle_precision(1)
            _, infs = h.solve(B)
            assert all(f.converged for f in infs)
            its[g] = np.array([f.iters for f in infs])
    assert np.abs(its[1] - its[0]).max() <= 1


def test_fp32_galerkin_is_refused_where_fp32_cannot_carry_the_coarse_operator(dev):
    import paper_2607_07485_amd as P
    prob, _ = fegen.graddiv_hdiv(N=16)
    kw = dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_problem(prob, P.Params.default(galerkin_precision=1, **kw))
    assert ei.value.code == 8                                 # LSDD_E_NUMERIC


def test_galerkin_precision_argument_check(dev):
    import paper_2607_07485_amd as P
    prob, _ = fegen.elasticity_small(N=8)
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_problem(prob, P.Params.default(max_levels=2, modes_fixed=4, galerkin_precision=2))
    assert ei.value.code == 1
