"""Pins of the oracle gradient of u = A(theta)^{-1} b against what the
mathematics fixes: central finite differences of the objective, the degree -1
homogeneity of the compliance (J(s theta) = J(theta) / s, so
sum_e theta_e dJ/dtheta_e = -J), and the symmetry of the adjoint pairing."""
import numpy as np
import pytest

import fegen
import oracle
from oracle.adjoint import solve


def _q1(N=6, seed=0):
    rng = np.random.default_rng(seed)
    prob = fegen.elasticity_q1(N, nu=0.35)
    theta = np.exp(0.5 * rng.standard_normal(N * N))
    return prob, theta, rng


def _q2(N=2, seed=1):
    rng = np.random.default_rng(seed)
    prob = fegen.elasticity_q2hex(N, nu=0.3)
    theta = np.exp(0.5 * rng.standard_normal(N ** 3))
    return prob, theta, rng


@pytest.mark.parametrize("make", [_q1, _q2])
def test_compliance_gradient_matches_central_differences(make):
    prob, theta, rng = make()
    b = rng.standard_normal(prob.n)
    J, g = oracle.compliance_gradient(prob, theta, b)
    for e in rng.choice(len(theta), size=6, replace=False):
        h = 1e-4 * theta[e]
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h
        tm[e] -= h
        fd = (b @ solve(prob, tp, b) - b @ solve(prob, tm, b)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * abs(g[e])


@pytest.mark.parametrize("make", [_q1, _q2])
def test_compliance_is_homogeneous_of_degree_minus_one(make):
    prob, theta, rng = make()
    b = rng.standard_normal(prob.n)
    J, g = oracle.compliance_gradient(prob, theta, b)
    assert J > 0
    assert abs(theta @ g + J) <= 1e-11 * J
    J2, _ = oracle.compliance_gradient(prob, 2.5 * theta, b)
    assert abs(J2 - J / 2.5) <= 1e-12 * J


def test_general_adjoint_matches_finite_differences_and_pairing():
    prob, theta, rng = _q1(N=5, seed=3)
    b = rng.standard_normal(prob.n)
    w = rng.standard_normal(prob.n)                  # L(u) = w^T u
    u, g, lam = oracle.adjoint_gradient(prob, theta, b, w)
    # dL/db = lambda: L is linear in b, so L(b + d) - L(b) = lambda^T d exactly
    d = rng.standard_normal(prob.n)
    assert abs(w @ solve(prob, theta, b + d) - w @ u - lam @ d) <= 1e-10 * abs(lam @ d)
    for e in rng.choice(len(theta), size=4, replace=False):
        h = 1e-4 * theta[e]
        tp, tm = theta.copy(), theta.copy()
        tp[e] += h
        tm[e] -= h
        fd = (w @ solve(prob, tp, b) - w @ solve(prob, tm, b)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * max(abs(g[e]), 1e-3 * np.abs(g).max())
    # pairing: with the loads swapped the same bilinear form appears (A symmetric)
    u2, g2, lam2 = oracle.adjoint_gradient(prob, theta, w, b)
    assert np.allclose(lam2, u, rtol=1e-10, atol=1e-12 * np.abs(u).max())
    assert np.allclose(g2, g, rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_planted_sign_error_is_caught():
    """A gradient with the wrong sign violates the homogeneity pin."""
    prob, theta, rng = _q1()
    b = rng.standard_normal(prob.n)
    J, g = oracle.compliance_gradient(prob, theta, b)
    assert abs(theta @ (-g) + J) > 1.0 * J
