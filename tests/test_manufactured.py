"""Manufactured solutions: the generated discretisations, solved by the oracle's
PCG with the LS-AMG-DD V-cycle, converge at the finite-element rates.

* CG1 triangles, -div(kappa grad u) = f with kappa = 1 + x + y, u = sin(pi x) sin(pi y)
  (zero on the boundary, Nitsche terms with zero data): L2 error O(h^2), H1 O(h).
* Plane-strain Q1 elasticity, u = (sin(pi x) y^2, x^2 cos(pi y)) (zero on the clamped
  edge x = 0, Nitsche there), body force -div sigma(u) and the tractions sigma(u) n of
  u on the other three edges: L2 error O(h^2), energy error O(h).

Right-hand sides come from sympy derivatives of the exact fields, integrated with
Gauss rules of degree well above the elements'.  Observed rates must be within 0.15
of the expected ones between the two finest meshes.
"""
import numpy as np
import pytest

import fegen
import oracle

sympy = pytest.importorskip("sympy")


def _gauss(k):
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (x + 1.0), 0.5 * w


def _tri_rule(k=6):
    """Collapsed (Duffy) tensor Gauss rule on the reference triangle (0,0),(1,0),(0,1)."""
    g, w = _gauss(k)
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            pts.append((a, b * (1.0 - a)))
            wts.append(wa * wb * (1.0 - a))
    return np.array(pts), np.array(wts)


def _rates(err, hs):
    return [np.log(err[i] / err[i + 1]) / np.log(hs[i] / hs[i + 1]) for i in range(len(err) - 1)]


def _solve(prob, b, **kw):
    h = oracle.setup(prob, oracle.Params(**kw))
    x, info = oracle.pcg(h, b, rtol=1e-12, max_iter=500)
    assert info.converged
    return x


# ----------------------------------------------------------------------------- CG1 diffusion

def _p1_case():
    X, Y = sympy.symbols("x y")
    u = sympy.sin(sympy.pi * X) * sympy.sin(sympy.pi * Y)
    kap = 1 + X + Y
    f = -(sympy.diff(kap * sympy.diff(u, X), X) + sympy.diff(kap * sympy.diff(u, Y), Y))
    lam = lambda e: sympy.lambdify((X, Y), e, "numpy")
    return lam(u), lam(sympy.diff(u, X)), lam(sympy.diff(u, Y)), lam(f)


def _p1_errors(N, solve=None):
    """(L2, H1-seminorm) errors of the CG1 solution; `solve(prob, b)` defaults to the
    oracle's PCG."""
    uf, ux, uy, ff = _p1_case()
    prob = fegen.diffusion_p1_triangles(N)
    qp, qw = _tri_rule()
    nx = N + 1
    xy = np.stack(np.meshgrid(np.arange(nx) / N, np.arange(nx) / N, indexing="xy"), -1).reshape(-1, 2)
    tris = prob.elem_dofs.reshape(-1, 3)
    P = xy[tris]                                                  # T x 3 x 2
    J = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], -1)      # T x 2 x 2, columns = edges
    det = np.abs(np.linalg.det(J))
    lam = np.stack([1 - qp[:, 0] - qp[:, 1], qp[:, 0], qp[:, 1]], 1)   # Q x 3
    pts = P[:, :1, :] + np.einsum("qk,tdk->tqd", qp, J)          # T x Q x 2
    fv = ff(pts[..., 0], pts[..., 1])
    b = np.zeros(prob.n)
    np.add.at(b, tris, np.einsum("tq,q,qa->ta", fv, qw, lam) * det[:, None])
    x = _solve(prob, b, tau_const=1.0) if solve is None else solve(prob, b)
    Gi = np.linalg.inv(J)                                         # rows: grad lambda_1, grad lambda_2
    grads = np.stack([-(Gi[:, 0] + Gi[:, 1]), Gi[:, 0], Gi[:, 1]], 1)   # T x 3 x 2
    xe = x[tris]
    uh = xe @ lam.T                                               # T x Q
    gh = np.einsum("ta,tad->td", xe, grads)                       # T x 2
    wq = qw[None, :] * det[:, None]
    e0 = np.sum(wq * (uh - uf(pts[..., 0], pts[..., 1])) ** 2)
    e1 = np.sum(wq * ((gh[:, None, 0] - ux(pts[..., 0], pts[..., 1])) ** 2 +
                      (gh[:, None, 1] - uy(pts[..., 0], pts[..., 1])) ** 2))
    return np.sqrt(e0), np.sqrt(e1)


def test_cg1_diffusion_converges_at_the_p1_rates():
    Ns = [8, 16, 32]
    errs = [_p1_errors(N) for N in Ns]
    hs = [1.0 / N for N in Ns]
    r0 = _rates([e[0] for e in errs], hs)
    r1 = _rates([e[1] for e in errs], hs)
    assert abs(r0[-1] - 2.0) <= 0.15, (errs, r0)
    assert abs(r1[-1] - 1.0) <= 0.15, (errs, r1)


# ----------------------------------------------------------------------------- Q1 elasticity

def _q1_case(lam_, mu_):
    X, Y = sympy.symbols("x y")
    u = [sympy.sin(sympy.pi * X) * Y ** 2, X ** 2 * sympy.cos(sympy.pi * Y)]
    grad = [[sympy.diff(u[i], v) for v in (X, Y)] for i in range(2)]
    eps = [[(grad[i][j] + grad[j][i]) / 2 for j in range(2)] for i in range(2)]
    tr = eps[0][0] + eps[1][1]
    sig = [[2 * mu_ * eps[i][j] + (lam_ * tr if i == j else 0) for j in range(2)] for i in range(2)]
    f = [-(sympy.diff(sig[i][0], X) + sympy.diff(sig[i][1], Y)) for i in range(2)]
    L = lambda e: sympy.lambdify((X, Y), e, "numpy")
    return ([L(c) for c in u], [[L(grad[i][j]) for j in range(2)] for i in range(2)], [L(c) for c in f],
            [[L(sig[i][j]) for j in range(2)] for i in range(2)])


def _ev(fn, x, y):
    return np.broadcast_to(np.asarray(fn(x, y), dtype=np.float64), np.shape(x))


def _q1_errors(N):
    prob = fegen.elasticity_q1(N, nu=0.3, E=1.0)
    lam_, mu_ = prob.meta["lam"], prob.meta["mu"]
    uf, gf, ff, sf = _q1_case(lam_, mu_)
    h = 1.0 / N
    nx = N + 1
    g, w = _gauss(4)
    b = np.zeros(prob.n)
    e0 = en = 0.0
    D = np.array([[lam_ + 2 * mu_, lam_, 0.0], [lam_, lam_ + 2 * mu_, 0.0], [0.0, 0.0, mu_]])
    # body force
    for j in range(N):
        for i in range(N):
            nodes = [j * nx + i, j * nx + i + 1, (j + 1) * nx + i, (j + 1) * nx + i + 1]
            for xi, wx in zip(g, w):
                for eta, wy in zip(g, w):
                    Nn = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta])
                    X, Y = (i + xi) * h, (j + eta) * h
                    wt = wx * wy * h * h
                    for c in range(2):
                        b[2 * np.array(nodes) + c] += wt * Nn * float(_ev(ff[c], X, Y))
    # tractions on x = 1 (n = (1, 0)), y = 0 (n = (0, -1)), y = 1 (n = (0, 1))
    for k in range(N):
        for s, ws in zip(g, w):
            t = (k + s) * h
            for (X, Y, nrm, a, bnode) in ((1.0, t, (1.0, 0.0), k * nx + N, (k + 1) * nx + N),
                                          (t, 0.0, (0.0, -1.0), k, k + 1),
                                          (t, 1.0, (0.0, 1.0), N * nx + k, N * nx + k + 1)):
                phi = (1 - s, s)
                for c in range(2):
                    tc = float(_ev(sf[c][0], X, Y)) * nrm[0] + float(_ev(sf[c][1], X, Y)) * nrm[1]
                    b[2 * a + c] += ws * h * phi[0] * tc
                    b[2 * bnode + c] += ws * h * phi[1] * tc
    x = _solve(prob, b, max_levels=2, modes_fixed=4)
    for j in range(N):
        for i in range(N):
            nodes = np.array([j * nx + i, j * nx + i + 1, (j + 1) * nx + i, (j + 1) * nx + i + 1])
            ue = np.stack([x[2 * nodes], x[2 * nodes + 1]], 1)            # 4 x 2
            for xi, wx in zip(g, w):
                for eta, wy in zip(g, w):
                    Nn = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta])
                    dN = np.array([[-(1 - eta), -(1 - xi)], [1 - eta, -xi], [-eta, 1 - xi], [eta, xi]]) / h
                    X, Y = (i + xi) * h, (j + eta) * h
                    wt = wx * wy * h * h
                    uh = Nn @ ue
                    Gh = ue.T @ dN                                          # Gh[c, d] = d u_c / d x_d
                    du = uh - np.array([float(_ev(uf[0], X, Y)), float(_ev(uf[1], X, Y))])
                    dG = Gh - np.array([[float(_ev(gf[c][d], X, Y)) for d in range(2)] for c in range(2)])
                    e = np.array([dG[0, 0], dG[1, 1], dG[0, 1] + dG[1, 0]])
                    e0 += wt * du @ du
                    en += wt * e @ D @ e
    return np.sqrt(e0), np.sqrt(en)


@pytest.mark.slow
def test_q1_elasticity_converges_at_the_q1_rates():
    Ns = [8, 16, 32]
    errs = [_q1_errors(N) for N in Ns]
    hs = [1.0 / N for N in Ns]
    r0 = _rates([e[0] for e in errs], hs)
    r1 = _rates([e[1] for e in errs], hs)
    assert abs(r0[-1] - 2.0) <= 0.15, (errs, r0)
    assert abs(r1[-1] - 1.0) <= 0.15, (errs, r1)
