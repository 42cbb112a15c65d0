"""Oracle pins of the block Schwarz smoothers other than multiplicative Schwarz
(Sec. 2: restricted additive Schwarz and aggregate block Jacobi, pre-smoother M^{-1},
post-smoother M^{-T})."""
import numpy as np
import pytest
import scipy.linalg as sla

import fegen
import oracle
from oracle import lsdd as O


def _small(smoother, **kw):
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4, smoother=smoother, **kw))
    return prob, h


def _smoother_matrix(lev, post):
    n = lev.n
    M = np.zeros((n, n))
    for j in range(n):
        x = np.zeros(n)
        e = np.zeros(n)
        e[j] = 1.0
        O.smooth_additive(lev, x, e, post)
        M[:, j] = x
    return M


def test_ras_post_smoother_is_the_transpose_and_partition_of_unity():
    """M^{-T} applied column by column is the transpose of M^{-1}; the corrections
    of M^{-1} come from the aggregates only (each row of M^{-1} is row p of
    A_Omega_i^{-1} for the one aggregate i holding p)."""
    prob, h = _small("ras")
    lev = h.levels[0]
    Mpre, Mpost = _smoother_matrix(lev, False), _smoother_matrix(lev, True)
    assert np.abs(Mpost - Mpre.T).max() <= 1e-14 * np.abs(Mpre).max()
    A = lev.A.toarray()
    for i, w in enumerate(lev.aggs):
        Om = lev.omegas[i]
        inv = np.linalg.inv(A[np.ix_(Om, Om)])
        for a, p in enumerate(w):
            row = np.zeros(lev.n)
            row[Om] = inv[a]
            assert np.abs(Mpre[p] - row).max() <= 1e-12 * np.abs(inv).max()
    # not symmetric once overlaps exist (the correction is restricted, the residual is not)
    assert np.abs(Mpre - Mpre.T).max() > 1e-6 * np.abs(Mpre).max()


def test_block_jacobi_smoother_is_the_block_inverse():
    prob, h = _small("bj")
    lev = h.levels[0]
    M = _smoother_matrix(lev, False)
    A = lev.A.toarray()
    ref = np.zeros_like(A)
    for w in lev.aggs:
        ref[np.ix_(w, w)] = np.linalg.inv(A[np.ix_(w, w)])
    assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(_smoother_matrix(lev, True), M)


@pytest.mark.parametrize("smoother", ["ras", "bj"])
def test_cycles_with_additive_smoothers_are_symmetric(smoother):
    prob, h = _small(smoother)
    rng = np.random.default_rng(1)
    r, s = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    a, b = oracle.vcycle(h, r) @ s, r @ oracle.vcycle(h, s)
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("smoother", ["ras", "bj"])
def test_single_aggregate_makes_the_smoother_exact(smoother):
    """One aggregate covering every DOF: Omega = omega, M^{-1} = A^{-1}, so one
    stand-alone cycle solves the problem."""
    prob = fegen.elasticity_q1(4, nu=0.3)
    prob.agg_of_dof = np.zeros(prob.n, dtype=np.int32)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4, smoother=smoother))
    b = np.random.default_rng(0).standard_normal(prob.n)
    x, info = oracle.stationary(h, b, np.zeros(prob.n), reduction=1e-10)
    assert info.iters == 1 and info.history[1] < 1e-12


@pytest.mark.parametrize("smoother", ["ms", "ras", "bj"])
def test_two_level_pcg_converges_with_each_smoother(smoother):
    prob, b = fegen.elasticity_small(N=16)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4, smoother=smoother))
    x, info = oracle.pcg(h, b)
    A = h.levels[0].A
    assert info.converged and info.iters < 60
    assert np.linalg.norm(b - A @ x) <= 1.01e-8 * np.linalg.norm(b)
