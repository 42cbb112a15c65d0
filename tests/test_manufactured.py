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


# ----------------------------------------------------------------------------- RTCF_3 grad-div

def _rtcf3_errors(N, beta=1.0):
    """L2 error of the RTCF_3 solution of -grad(div u) + beta u = f (kappa = 1) with the
    natural boundary condition div u = g of the form without boundary terms: the load
    is (f, v) + <g, v.n> with g = div u of the exact field."""
    from fegen.common import gauss_legendre_01, gll_nodes_01, lagrange_1d
    from fegen.hdiv import rtcf3_dofs
    X, Y = sympy.symbols("x y")
    u = [sympy.sin(sympy.pi * X) * sympy.cos(2 * Y) + X ** 2 * Y, sympy.exp(X) * sympy.sin(sympy.pi * Y)]
    div = sympy.diff(u[0], X) + sympy.diff(u[1], Y)
    f = [-sympy.diff(div, X) + beta * u[0], -sympy.diff(div, Y) + beta * u[1]]
    L = lambda e: sympy.lambdify((X, Y), e, "numpy")
    uf, ff, gf = [L(c) for c in u], [L(c) for c in f], L(div)
    prob = fegen.graddiv_rtcf3(N, beta=beta)
    dofs, _, _ = rtcf3_dofs(N)
    h = 1.0 / N
    phi = lagrange_1d(gll_nodes_01(4))[0]
    psi = lagrange_1d(gauss_legendre_01(3)[0])[0]
    qp, qw = gauss_legendre_01(6)
    P, S = phi(qp), psi(qp)                                     # [q, 4], [q, 3]
    # basis values on the reference cell, [qx, qy, comp, 24]
    V = np.zeros((len(qp), len(qp), 2, 24))
    for a in range(4):
        for b in range(3):
            V[:, :, 0, 3 * a + b] = np.outer(P[:, a], S[:, b])
            V[:, :, 1, 12 + 3 * a + b] = np.outer(S[:, b], P[:, a])
    W = np.outer(qw, qw) * h * h
    cells = np.arange(N * N)
    ci, cj = cells % N, cells // N
    xq = (ci[:, None, None] + qp[None, :, None]) * h + 0.0 * qp[None, None, :]
    yq = (cj[:, None, None] + qp[None, None, :]) * h + 0.0 * qp[None, :, None]
    fq = np.stack([np.broadcast_to(ff[c](xq, yq), xq.shape) for c in range(2)], -1)      # [T, qx, qy, 2]
    b = np.zeros(prob.n)
    np.add.at(b, dofs, np.einsum("tijc,ijck,ij->tk", fq, V, W))
    # <g, v.n>: the edge basis functions phi_0 (at 0) and phi_3 (at 1) times psi_b
    for side in ("left", "right", "bottom", "top"):
        sel = {"left": ci == 0, "right": ci == N - 1, "bottom": cj == 0, "top": cj == N - 1}[side]
        for t in np.flatnonzero(sel):
            s = (cj[t] if side in ("left", "right") else ci[t]) * h + qp * h
            xy = {"left": (0.0 * s, s), "right": (1.0 + 0.0 * s, s),
                  "bottom": (s, 0.0 * s), "top": (s, 1.0 + 0.0 * s)}[side]
            g = np.broadcast_to(gf(*xy), s.shape)
            sign = -1.0 if side in ("left", "bottom") else 1.0
            a = 0 if side in ("left", "bottom") else 3
            base = 0 if side in ("left", "right") else 12
            for bb in range(3):
                b[dofs[t, base + 3 * a + bb]] += sign * np.sum(qw * h * g * S[:, bb])
    x = _solve(prob, b, max_levels=3, tau_const=0.75, agg_passes=1)
    uh = np.einsum("tk,ijck->tijc", x[dofs], V)
    ue = np.stack([np.broadcast_to(uf[c](xq, yq), xq.shape) for c in range(2)], -1)
    return float(np.sqrt(np.sum(W[None, :, :, None] * (uh - ue) ** 2)))


def test_rtcf3_graddiv_converges_at_the_rt3_rate():
    """RTCF_3 (Q_{3,2} x Q_{2,3}) on the grad-div form: L2 error O(h^3)."""
    Ns = [4, 8, 16]
    errs = [_rtcf3_errors(N) for N in Ns]
    r = _rates(errs, [1.0 / N for N in Ns])
    assert abs(r[-1] - 3.0) <= 0.15, (errs, r)


# ----------------------------------------------------------------------------- BFS hyperdiffusion

def _bfs_errors(N, eps=0.25, theta=np.pi / 6):
    """L2 error of the clamped hyperdiffusion solution (q(q(u)) = f, q = div(D grad .),
    u = d_n u = 0 by the Nitsche terms) for u = sin^2(pi x) sin^2(pi y)."""
    from fegen.common import gauss_legendre_01
    from fegen.hermite import _derivs, diffusion_tensor
    X, Y = sympy.symbols("x y")
    D = diffusion_tensor(eps, theta)
    u = sympy.sin(sympy.pi * X) ** 2 * sympy.sin(sympy.pi * Y) ** 2
    q = lambda w: D[0, 0] * sympy.diff(w, X, 2) + 2 * D[0, 1] * sympy.diff(w, X, Y) + D[1, 1] * sympy.diff(w, Y, 2)
    uf, ff = sympy.lambdify((X, Y), u, "numpy"), sympy.lambdify((X, Y), q(q(u)), "numpy")
    prob = fegen.hyperdiffusion_h2(N, eps=eps, theta=theta)[0]
    h = 1.0 / N
    qp, qw = gauss_legendre_01(6)
    Bv = np.array([[_derivs(x, y, h)[(0, 0)] for y in qp] for x in qp])       # [qx, qy, 16]
    W = np.outer(qw, qw) * h * h
    nx = N + 1
    cells = np.arange(N * N)
    ci, cj = cells % N, cells // N
    verts = np.stack([cj * nx + ci, cj * nx + ci + 1, (cj + 1) * nx + ci, (cj + 1) * nx + ci + 1], 1)
    dofs = (4 * verts[:, :, None] + np.arange(4)[None, None, :]).reshape(N * N, 16)
    xq = (ci[:, None, None] + qp[None, :, None]) * h + 0.0 * qp[None, None, :]
    yq = (cj[:, None, None] + qp[None, None, :]) * h + 0.0 * qp[None, :, None]
    b = np.zeros(prob.n)
    np.add.at(b, dofs, np.einsum("tij,ijk,ij->tk", ff(xq, yq), Bv, W))
    x = _solve(prob, b, max_levels=3, tau_const=1.0, agg_passes=1)
    uh = np.einsum("tk,ijk->tij", x[dofs], Bv)
    return float(np.sqrt(np.sum(W[None] * (uh - uf(xq, yq)) ** 2)))


def test_bfs_hyperdiffusion_converges_at_the_bicubic_rate():
    """Bogner-Fox-Schmit bicubics, anisotropic D (eps = 0.25 at 30 degrees), clamped by
    the symmetric Nitsche terms: L2 error O(h^4)."""
    Ns = [4, 8, 16]
    errs = [_bfs_errors(N) for N in Ns]
    r = _rates(errs, [1.0 / N for N in Ns])
    assert abs(r[-1] - 4.0) <= 0.15, (errs, r)


# ----------------------------------------------------------------------------- Q2 hex elasticity

def _q2hex_errors(N, nu=0.3):
    """L2 and energy errors of the Q2 hexahedral elasticity solution: u vanishes on the
    clamped face x = 0 (Nitsche there), body force -div sigma(u) and the tractions
    sigma(u) n of u on the other five faces."""
    from fegen.common import gauss_legendre_01, lame_plane_strain
    from fegen.elasticity import _q2_1d
    lam_, mu_ = lame_plane_strain(1.0, nu)
    X, Y, Z = sympy.symbols("x y z")
    u = [X * sympy.sin(sympy.pi * Y) * (1 + Z), X ** 2 * sympy.cos(sympy.pi * Z), X * Y * Z ** 2]
    V = (X, Y, Z)
    grad = [[sympy.diff(u[i], v) for v in V] for i in range(3)]
    eps = [[(grad[i][j] + grad[j][i]) / 2 for j in range(3)] for i in range(3)]
    tr = eps[0][0] + eps[1][1] + eps[2][2]
    sig = [[2 * mu_ * eps[i][j] + (lam_ * tr if i == j else 0) for j in range(3)] for i in range(3)]
    f = [-sum(sympy.diff(sig[i][j], V[j]) for j in range(3)) for i in range(3)]
    L = lambda e: sympy.lambdify(V, e, "numpy")
    uf, ff = [L(c) for c in u], [L(c) for c in f]
    gf = [[L(grad[i][j]) for j in range(3)] for i in range(3)]
    sf = [[L(sig[i][j]) for j in range(3)] for i in range(3)]
    ev = lambda fn, *p: np.broadcast_to(np.asarray(fn(*p), dtype=np.float64), np.shape(p[0]))
    prob = fegen.elasticity_q2hex(N, nu=nu)
    h = 1.0 / N
    M = 2 * N + 1
    qp, qw = gauss_legendre_01(4)
    nq = len(qp)
    v1, d1 = _q2_1d(qp)                                          # [3, q]
    # reference basis on the q^3 points: values [q3, 27], gradients [q3, 27, 3] (physical)
    idx = [(a, b, c) for c in range(3) for b in range(3) for a in range(3)]
    pts = [(i, j, k) for k in range(nq) for j in range(nq) for i in range(nq)]
    Bv = np.array([[v1[a, i] * v1[b, j] * v1[c, k] for (a, b, c) in idx] for (i, j, k) in pts])
    Bg = np.array([[[d1[a, i] * v1[b, j] * v1[c, k], v1[a, i] * d1[b, j] * v1[c, k],
                     v1[a, i] * v1[b, j] * d1[c, k]] for (a, b, c) in idx] for (i, j, k) in pts]) / h
    W = np.array([qw[i] * qw[j] * qw[k] for (i, j, k) in pts]) * h ** 3
    e = np.arange(N ** 3)
    ex, ey, ez = e % N, (e // N) % N, e // (N * N)
    loc = np.array(idx)
    nodes = ((2 * ez[:, None] + loc[None, :, 2]) * M + (2 * ey[:, None] + loc[None, :, 1])) * M \
        + (2 * ex[:, None] + loc[None, :, 0])
    P = np.array(pts, dtype=np.float64)
    xq = (ex[:, None] + qp[P[:, 0].astype(int)][None]) * h
    yq = (ey[:, None] + qp[P[:, 1].astype(int)][None]) * h
    zq = (ez[:, None] + qp[P[:, 2].astype(int)][None]) * h
    b = np.zeros(prob.n)
    for c in range(3):
        np.add.at(b, 3 * nodes + c, np.einsum("eq,qa,q->ea", ev(ff[c], xq, yq, zq), Bv, W))
    # tractions on the faces x = 1, y = 0, y = 1, z = 0, z = 1 (face rule: q^2 points)
    g2 = [(i, j) for j in range(nq) for i in range(nq)]
    W2 = np.array([qw[i] * qw[j] for (i, j) in g2]) * h * h
    for axis, side, nrm in ((0, 1, 1.0), (1, 0, -1.0), (1, 1, 1.0), (2, 0, -1.0), (2, 1, 1.0)):
        ecoord = (ex, ey, ez)[axis]
        sel = np.flatnonzero(ecoord == (N - 1 if side else 0))
        t = 1.0 if side else 0.0
        other = [d for d in range(3) if d != axis]
        fv = np.zeros((len(g2), 27))
        for q, (i, j) in enumerate(g2):
            ref = [0.0, 0.0, 0.0]
            ref[axis] = t
            ref[other[0]], ref[other[1]] = qp[i], qp[j]
            vv = [_q2_1d(np.array([r]))[0][:, 0] for r in ref]
            fv[q] = [vv[0][a] * vv[1][b2] * vv[2][c] for (a, b2, c) in idx]
        for e_ in sel:
            o = np.array([ex[e_], ey[e_], ez[e_]], dtype=np.float64) * h
            cq = np.zeros((len(g2), 3))
            cq[:, axis] = t
            cq[:, other[0]] = o[other[0]] + qp[[i for (i, _) in g2]] * h
            cq[:, other[1]] = o[other[1]] + qp[[j for (_, j) in g2]] * h
            for c in range(3):
                tc = nrm * ev(sf[c][axis], cq[:, 0], cq[:, 1], cq[:, 2])
                b[3 * nodes[e_] + c] += fv.T @ (W2 * tc)
    x = _solve(prob, b, max_levels=2, tau_const=0.75, agg_passes=1)
    xe = x[3 * nodes[:, :, None] + np.arange(3)[None, None, :]]           # [E, 27, 3]
    uh = np.einsum("qa,eac->eqc", Bv, xe)
    gh = np.einsum("qad,eac->eqcd", Bg, xe)                               # du_c / dx_d
    ue = np.stack([ev(uf[c], xq, yq, zq) for c in range(3)], -1)
    ge = np.stack([np.stack([ev(gf[c][d], xq, yq, zq) for d in range(3)], -1) for c in range(3)], -2)
    e0 = np.sum(W[None, :, None] * (uh - ue) ** 2)
    dG = gh - ge
    de = 0.5 * (dG + np.swapaxes(dG, -1, -2))
    trd = np.trace(de, axis1=-2, axis2=-1)
    en = np.sum(W[None, :] * (2 * mu_ * np.sum(de * de, axis=(-2, -1)) + lam_ * trd ** 2))
    return float(np.sqrt(e0)), float(np.sqrt(en))


@pytest.mark.slow
def test_q2_hex_elasticity_converges_at_the_q2_rates():
    """27-node hexahedra: L2 error O(h^3), energy error O(h^2)."""
    Ns = [2, 4, 8]
    errs = [_q2hex_errors(N) for N in Ns]
    hs = [1.0 / N for N in Ns]
    r0 = _rates([e[0] for e in errs], hs)
    r1 = _rates([e[1] for e in errs], hs)
    assert abs(r0[-1] - 3.0) <= 0.15, (errs, r0)
    assert abs(r1[-1] - 2.0) <= 0.15, (errs, r1)
