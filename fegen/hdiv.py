"""H(div) grad-div inputs: RTCF_3 (Q_{3,2} x Q_{2,3}) on uniform quads of (0,1)^2.

Per cell T the energy is  kappa_T (div u, div v)_T + beta (u, v)_T.  The global
vector field is built from tensor-product pieces:
    u_x = phi_a(xi) psi_b(eta)   (a = 0..3 normal direction, b = 0..2 tangential)
    u_y = psi_a(xi) phi_b(eta)
phi is the cubic Lagrange basis on the 4 Gauss-Lobatto nodes (phi_0, phi_3 are
the only functions nonzero on the cell edges), psi the quadratic Lagrange basis
on the 3 Gauss points.  Normal continuity across edges holds because the edge
DOF (coefficient of u_x on a vertical edge, of u_y on a horizontal one) is
shared by the two cells.  Every cell block is SPD (beta > 0).
"""
from __future__ import annotations

import numpy as np

from .common import Problem, gauss_legendre_01, gll_nodes_01, lagrange_1d, uniform_problem


def rtcf3_reference(h: float):
    """(Div, Mass) 24x24 reference matrices of a square cell of size h.

    Local order: u_x pieces 3a + b (a = 0..3 phi index along x, b = 0..2 psi index
    along y), then u_y pieces 12 + 3a + b (a = 0..3 phi index along y, b = 0..2
    psi index along x).
    """
    phi, dphi, _, _ = lagrange_1d(gll_nodes_01(4))
    psi, dpsi, _, _ = lagrange_1d(gauss_legendre_01(3)[0])
    qp, qw = gauss_legendre_01(5)
    P, dP = phi(qp), dphi(qp)        # [q, 4]
    S = psi(qp)                      # [q, 3]
    nq = len(qp)
    vals = np.zeros((nq, nq, 2, 24))  # field value (2 comps) per basis
    divs = np.zeros((nq, nq, 24))
    for a in range(4):
        for b in range(3):
            k = 3 * a + b
            vals[:, :, 0, k] = np.outer(P[:, a], S[:, b])
            divs[:, :, k] = np.outer(dP[:, a], S[:, b]) / h
            k2 = 12 + 3 * a + b          # u_y: phi_a along y, psi_b along x
            vals[:, :, 1, k2] = np.outer(S[:, b], P[:, a])
            divs[:, :, k2] = np.outer(S[:, b], dP[:, a]) / h
    w = np.outer(qw, qw) * h * h
    Div = np.einsum("ij,iju,ijv->uv", w, divs, divs)
    Mass = np.einsum("ij,ijcu,ijcv->uv", w, vals, vals)
    return 0.5 * (Div + Div.T), 0.5 * (Mass + Mass.T)


def rtcf3_dofs(N: int):
    """(dofs[N*N, 24], node_of_dof, n) with edges first (3 DOFs each), then cells (12)."""
    nV = (N + 1) * N
    nH = N * (N + 1)
    nE = nV + nH
    cell = np.arange(N * N)
    i, j = cell % N, cell // N
    vid = lambda ii, jj: jj * (N + 1) + ii
    hid = lambda ii, jj: nV + jj * N + ii
    dofs = np.empty((N * N, 24), dtype=np.int64)
    base_int = 3 * nE + 12 * cell
    for a in range(4):
        for b in range(3):
            k = 3 * a + b
            if a == 0:
                dofs[:, k] = 3 * vid(i, j) + b
            elif a == 3:
                dofs[:, k] = 3 * vid(i + 1, j) + b
            else:
                dofs[:, k] = base_int + 3 * (a - 1) + b
            k2 = 12 + 3 * a + b        # u_y, a = index along y (phi), b = along x (psi)
            if a == 0:
                dofs[:, k2] = 3 * hid(i, j) + b
            elif a == 3:
                dofs[:, k2] = 3 * hid(i, j + 1) + b
            else:
                dofs[:, k2] = base_int + 6 + 3 * (a - 1) + b
    n = 3 * nE + 12 * N * N
    node = np.empty(n, dtype=np.int64)
    node[: 3 * nE] = np.arange(3 * nE) // 3
    node[3 * nE:] = nE + np.arange(12 * N * N) // 12
    return dofs, node, n


def graddiv_rtcf3(N: int, kappa=None, beta: float = 1e-4) -> Problem:
    """kappa_T (div u, div v) + beta (u, v) on RTCF_3, no boundary terms (mass keeps it SPD)."""
    h = 1.0 / N
    Div, Mass = rtcf3_reference(h)
    dofs, node, n = rtcf3_dofs(N)
    kap = np.ones(N * N) if kappa is None else np.asarray(kappa, dtype=np.float64)
    blocks = kap[:, None, None] * Div[None] + beta * Mass[None]
    return uniform_problem(n, dofs, blocks, node, None,
                           meta=dict(kind="graddiv_rtcf3", N=N, beta=beta))
