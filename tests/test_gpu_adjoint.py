"""GPU parity of the differentiable solve u = A(theta)^{-1} b (autograd Function
over per-element coefficients) against the oracle's exact adjoint gradient, and
against central finite differences taken with lsdd_update_theta.

Tolerances: solutions 1e-10 relative (PCG to 1e-12), gradients 1e-7 relative to
the oracle (the requirement is 1e-5) and 1e-5 to finite differences.
"""
import numpy as np
import pytest

import fegen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lsdd():
    import paper_2607_07485_amd as P
    from paper_2607_07485_amd import autograd as AG
    return P, AG


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch.device("cuda:0")


CASES = {
    "q1": (lambda: fegen.elasticity_q1(8, nu=0.35), dict(max_levels=2, modes_fixed=4, rtol=1e-12)),
    "q2hex": (lambda: fegen.elasticity_q2hex(3, nu=0.3),
              dict(max_levels=3, agg_passes=1, agg_passes_coarse=1, tau_const=0.75, rtol=1e-12)),
}


def _case(name, seed=0):
    make, kw = CASES[name]
    prob = make()
    ne = len(prob.elem_ptr) - 1
    rng = np.random.default_rng(seed)
    theta = np.exp(0.5 * rng.standard_normal(ne))
    b = rng.standard_normal(prob.n)
    return prob, kw, theta, b, rng


@pytest.mark.parametrize("name", ["q1", "q2hex"])
def test_compliance_gradient_matches_oracle(dev, name):
    P, AG = _lsdd()
    prob, kw, theta, b, _ = _case(name)
    system = AG.ElementSystem(prob, P.Params.default(**kw))
    th = torch.tensor(theta, device=dev, requires_grad=True)
    bt = torch.tensor(b, device=dev, requires_grad=True)
    u = AG.solve(th, bt, system)
    J = torch.dot(torch.tensor(b, device=dev), u)
    J.backward()
    J_or, g_or = oracle.compliance_gradient(prob, theta, b)
    u_or = oracle.adjoint.solve(prob, theta, b)
    assert np.linalg.norm(u.detach().cpu().numpy() - u_or) <= 1e-10 * np.linalg.norm(u_or)
    assert abs(J.item() - J_or) <= 1e-10 * abs(J_or)
    g = th.grad.cpu().numpy()
    assert np.abs(g - g_or).max() <= 1e-7 * np.abs(g_or).max()
    # through the load: dJ/db (via the solve) = lambda = u
    assert np.linalg.norm(bt.grad.cpu().numpy() - u_or) <= 1e-9 * np.linalg.norm(u_or)


def test_general_objective_and_several_right_hand_sides(dev):
    """L = sum_k w_k^T u_k over a block of right-hand sides."""
    P, AG = _lsdd()
    prob, kw, theta, _, rng = _case("q1", seed=2)
    B = rng.standard_normal((3, prob.n))
    W = rng.standard_normal((3, prob.n))
    system = AG.ElementSystem(prob, P.Params.default(**kw))
    th = torch.tensor(theta, device=dev, requires_grad=True)
    bt = torch.tensor(B, device=dev, requires_grad=True)
    U = AG.solve(th, bt, system)
    (torch.tensor(W, device=dev) * U).sum().backward()
    g_or = np.zeros_like(theta)
    for k in range(3):
        _, gk, lam = oracle.adjoint_gradient(prob, theta, B[k], W[k])
        g_or += gk
        assert np.linalg.norm(bt.grad[k].cpu().numpy() - lam) <= 1e-9 * np.linalg.norm(lam)
    assert np.abs(th.grad.cpu().numpy() - g_or).max() <= 1e-7 * np.abs(g_or).max()


def test_gradient_matches_central_differences_with_update_theta(dev):
    """Finite differences J(theta +- h e_k) solved with the theta hierarchy as the
    preconditioner of A(theta +- h e_k) (lsdd_update_theta)."""
    P, AG = _lsdd()
    prob, kw, theta, b, rng = _case("q2hex", seed=4)
    system = AG.ElementSystem(prob, P.Params.default(**kw))
    th = torch.tensor(theta, device=dev, requires_grad=True)
    bt = torch.tensor(b, device=dev)
    u = AG.solve(th, bt, system)
    torch.dot(bt, u).backward()
    g = th.grad.cpu().numpy()
    h = system.hierarchy(torch.tensor(theta, device=dev))
    try:
        x0, _ = h.solve(bt)
        for e in rng.choice(len(theta), size=5, replace=False):
            step = 1e-4 * theta[e]
            Js = []
            for sgn in (1.0, -1.0):
                tp = theta.copy()
                tp[e] += sgn * step
                h.update_theta(torch.tensor(tp, device=dev))
                x, infos = h.solve(bt)
                assert infos[0].converged == 1
                Js.append(torch.dot(bt, x).item())
            fd = (Js[0] - Js[1]) / (2 * step)
            assert abs(fd - g[e]) <= 1e-5 * abs(g[e])
        h.update_theta(torch.tensor(theta, device=dev))      # restores the operator bit for bit
        x1, _ = h.solve(bt)
        assert torch.equal(x1, x0)
    finally:
        h.close()
