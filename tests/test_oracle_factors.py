"""Oracle pins of the pivoted Cholesky element factor (Sec. 5.2), the alternative to
the eigendecomposition range factor."""
import numpy as np
import pytest

import fegen
import oracle
from oracle import lsdd as O


def _pivots(G):
    """Pivot order of a pivoted Cholesky factor: DOF p_k is zero in every later row."""
    r, n = G.shape
    piv = []
    for k in range(r):
        cand = [j for j in range(n) if j not in piv and G[k, j] != 0.0 and not np.any(G[k + 1:, j] != 0.0)]
        assert len(cand) == 1
        piv.append(cand[0])
    return piv


def test_spd_block_gives_the_cholesky_factor_of_the_permuted_block():
    """For an SPD block the factor is L^T of the symmetrically permuted block, the
    unique Cholesky factor (checked against LAPACK through numpy)."""
    prob, _ = fegen.graddiv_hdiv(N=4, beta=1.0)
    for e in (0, 7):
        _, Ae = prob.element(e)
        G = O.element_gram_factor_pchol(Ae)
        assert G.shape == Ae.shape
        piv = _pivots(G)
        assert piv[0] == int(np.argmax(np.diag(Ae)))
        L = np.linalg.cholesky(Ae[np.ix_(piv, piv)])
        assert np.abs(G[:, piv] - L.T).max() <= 1e-12 * np.abs(L).max()


def test_semidefinite_blocks_rank_and_reproduction():
    """Interior Q1 elasticity blocks have rank 5 (8 - 3 rigid modes) and Q2 hex blocks
    rank 75 (81 - 6); on every element the rank equals the eigendecomposition's and
    G^T G reproduces the block."""
    for prob, interior, rank in ((fegen.elasticity_q1(4, nu=0.3), 1, 5),
                                 (fegen.elasticity_q2hex(2, nu=0.3), 1, 75)):
        for e in range(prob.n_elem):
            _, Ae = prob.element(e)
            G = O.element_gram_factor_pchol(Ae)
            assert np.abs(G.T @ G - Ae).max() <= 1e-13 * np.abs(Ae).max()
            assert G.shape[0] == O.element_gram_factor(Ae).shape[0]
        _, Ai = prob.element(interior)
        assert O.element_gram_factor_pchol(Ai).shape[0] == rank


@pytest.mark.parametrize("A", [np.diag([1.0, -0.5, 2.0]),
                               np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]])])
def test_indefinite_blocks_are_rejected(A):
    with pytest.raises(O.NotSPSD):
        O.element_gram_factor_pchol(A)


def test_galerkin_identity_holds_for_both_factors():
    """A_c = P^T A P = sum_T (G_T P_T)^T (G_T P_T) with either factor (Sec. 2, Galerkin
    Gram recursion; Sec. 5.2 factors differ by an orthogonal transformation)."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    for f in ("eig", "chol"):
        h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4, elem_factor=f))
        lv = h.levels[0]
        Pd = lv.P.toarray()
        Ac = np.zeros((Pd.shape[1],) * 2)
        for e, S in enumerate(lv.elem_dofs):
            GP = h.G0[e] @ Pd[S]
            Ac += GP.T @ GP
        ref = h.levels[1].A.toarray()
        assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()
