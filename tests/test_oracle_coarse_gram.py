"""Pins of the oracle's coarse Gram rows (Sec. 5.1, the remark that sums of
element Gram blocks are Gram blocks of the coarser scale; factorisation of
Sec. 5.2).

The literal coarse factor G P keeps one row per level-0 Gram row on every level.
Re-factoring each grouped coarse element block A_g gives rank(A_g) rows instead,
and the coarse operator stays the Galerkin product P^T A P up to the rounding of
that product and the truncation of each factorisation.  The pins check that
against P^T A P formed here from the finer level, with the standard bound of a
sum of products (eps times the same sum of absolute values) plus the truncation
tolerance n_g eps max diag(A_g) of every group that holds the entry, and the
counting facts that hold exactly: n_l <= sum_g rank(A_g) (A_l is SPD) and the
re-factored rows are fewer than the inherited ones.
"""
import numpy as np
import pytest

import fegen
import oracle

EPS = np.finfo(np.float64).eps
GAMMA = 64.0     # accumulation-length factor of the rounding bound (sums of at most a few hundred terms)

CASES = {
    "elasticity": (lambda: fegen.elasticity_small(N=16)[0], dict(max_levels=3, modes_fixed=4)),
    "graddiv_beta1": (lambda: fegen.graddiv_hdiv(N=12, beta=1.0)[0],
                      dict(max_levels=3, tau_const=0.75, agg_passes=1, agg_passes_coarse=1)),
    "graddiv_beta1e-4": (lambda: fegen.graddiv_hdiv(N=8)[0],
                         dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)),
}


@pytest.fixture(scope="module", params=list(CASES))
def hierarchy(request):
    make, kw = CASES[request.param]
    return oracle.setup(make(), oracle.Params(**kw))


def _dense(n, elem_dofs, mats):
    A = np.zeros((n, n))
    for S, M in zip(elem_dofs, mats):
        A[np.ix_(S, S)] += M
    return A


def _excess(lv, fv, Gs):
    """Largest ratio |sum_g G_g^T G_g - P^T A P| / bound over the entries, with the
    bound: rounding of the Galerkin sums, eps |P|^T (sum_e |B_e|) |P|, plus the
    truncation n_g eps max diag(A_g) of every group holding the entry."""
    Ad = _dense(lv.n, lv.elem_dofs, [G.T @ G for G in Gs])
    Ac = (fv.P.T @ fv.A @ fv.P).toarray()
    absA = oracle.assemble(fv.n, fv.elem_dofs, [np.abs(B) for B in fv.blocks])
    aP = abs(fv.P)
    bound = EPS * (aP.T @ absA @ aP).toarray()
    bound += _dense(lv.n, lv.elem_dofs, [np.full(B.shape, len(B) * EPS * B.diagonal().max()) for B in lv.blocks])
    diff = np.abs(Ad - Ac)
    if (diff[bound == 0] != 0).any():
        return np.inf
    return float((diff[bound > 0] / bound[bound > 0]).max())


def test_coarse_gram_rows_reproduce_the_galerkin_operator(hierarchy):
    h = hierarchy
    assert len(h.levels) >= 2
    for l in range(1, len(h.levels)):
        lv, fv = h.levels[l], h.levels[l - 1]
        Gs = oracle.coarse_gram_factors(lv)
        assert len(Gs) == len(lv.elem_dofs)
        assert _excess(lv, fv, Gs) <= GAMMA


def test_coarse_gram_rows_are_fewer_and_span_the_coarse_space(hierarchy):
    h = hierarchy
    m0 = sum(G.shape[0] for G in h.G0)          # rows of the literal G P on every level
    for l in range(1, len(h.levels)):
        lv = h.levels[l]
        Gs = oracle.coarse_gram_factors(lv)
        ranks = np.array([G.shape[0] for G in Gs])
        sizes = np.array([len(S) for S in lv.elem_dofs])
        assert (ranks <= sizes).all()
        assert all(G.shape[1] == n for G, n in zip(Gs, sizes))
        assert lv.n <= ranks.sum() < m0
        # each factor reproduces its own block to the pivoted-Cholesky truncation bound
        for B, G in zip(lv.blocks, Gs):
            assert np.abs(B - G.T @ G).max() <= 2.0 * len(B) * EPS * B.diagonal().max()


def test_a_planted_row_drop_is_caught(hierarchy):
    """Dropping the first row of the largest group's factor (an off-by-one in the
    row range) must break the reproduction pin.  (The last rows may sit at the
    truncation level, where dropping one is within the bound.)"""
    h = hierarchy
    lv, fv = h.levels[1], h.levels[0]
    Gs = oracle.coarse_gram_factors(lv)
    g = int(np.argmax([G.shape[0] for G in Gs]))
    Gs[g] = Gs[g][1:]
    assert _excess(lv, fv, Gs) > GAMMA
