"""Scalar H^1 diffusion on linear (CG1) triangles: the closure comparison problem.

-div(kappa grad u) = 0 on (0,1)^2 with kappa(x, y) = 1 + x + y and u = 0 on the
whole boundary, imposed weakly by the symmetric Nitsche terms
    <gamma kappa u, v>_F - <kappa d_n u, v>_F - <kappa d_n v, u>_F,   gamma_F = 24 p^2 / h_F,
on every boundary facet F (p = 1), so every element block stays symmetric
positive semidefinite and no DOF is eliminated (Sec. 5.1, remark on weakly
imposed boundary conditions).  The mesh is the uniformly refined unit square:
N x N squares, each cut into two right triangles by the diagonal from its
lower-left to its upper-right corner, so all diagonals are parallel.  Vertex
(i, j) carries DOF j (N + 1) + i; N = 32, 64, ..., 1024 give 1,089 ... 1,050,625
DOFs.

Element blocks are exact: kappa is linear, so the cell integral is
kappa(centroid) |T| grad phi_a . grad phi_b, and the facet integrals (at most
cubic) use the 2-point Gauss rule.  On a right triangle the two vertices of the
hypotenuse have orthogonal gradients, so away from the boundary the assembled
entry of every diagonal edge cancels to exactly zero while both vertices still
share the two elements of that edge.
"""
from __future__ import annotations

import numpy as np

from .common import Problem, gauss_legendre_01, uniform_problem


def kappa_linear(x, y):
    return 1.0 + x + y


def _gradients(P: np.ndarray):
    """Area and barycentric gradients g[3, 2] of triangle P[3, 2]."""
    v0, v1, v2 = P
    J = np.array([v1 - v0, v2 - v0]).T                  # columns: edge vectors
    Ginv = np.linalg.inv(J)                             # rows: grad lambda_1, grad lambda_2
    return 0.5 * abs(np.linalg.det(J)), np.vstack([-(Ginv[0] + Ginv[1]), Ginv[0], Ginv[1]])


def _nitsche(P: np.ndarray, kappa, gamma_c: float) -> np.ndarray:
    """Nitsche terms of the facets of triangle P[3, 2] (counter-clockwise) on the boundary."""
    _, g = _gradients(P)
    K = np.zeros((3, 3))
    qp, qw = gauss_legendre_01(2)
    for a, b in ((0, 1), (1, 2), (2, 0)):
        pa, pb = P[a], P[b]
        if not any(pa[d] == v and pb[d] == v for d in (0, 1) for v in (0.0, 1.0)):
            continue
        t = pb - pa
        hF = float(np.hypot(t[0], t[1]))
        nrm = np.array([t[1], -t[0]]) / hF               # outward for a counter-clockwise triangle
        dn = g @ nrm                                     # normal derivative of each basis function
        gamma = gamma_c / hF
        for s, w in zip(qp, qw):
            x = pa + s * t
            phi = np.zeros(3)
            phi[a] = 1.0 - s
            phi[b] = s
            k = kappa(x[0], x[1])
            K += w * hF * k * (gamma * np.outer(phi, phi) - np.outer(phi, dn) - np.outer(dn, phi))
    return K


def diffusion_p1_triangles(N: int, kappa=kappa_linear, gamma_c: float = 24.0) -> Problem:
    """CG1 diffusion with Nitsche u = 0 on the N x N structured triangle mesh of (0,1)^2."""
    h = 1.0 / N
    nxn = N + 1
    jj, ii = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()                      # square s = j N + i
    ll, lr, ul, ur = jj * nxn + ii, jj * nxn + ii + 1, (jj + 1) * nxn + ii, (jj + 1) * nxn + ii + 1
    # triangle 2s: (ll, lr, ur); triangle 2s+1: (ll, ur, ul); both counter-clockwise
    dofs = np.empty((2 * N * N, 3), dtype=np.int64)
    dofs[0::2] = np.stack([ll, lr, ur], 1)
    dofs[1::2] = np.stack([ll, ur, ul], 1)
    ref = [np.array([[0.0, 0.0], [h, 0.0], [h, h]]), np.array([[0.0, 0.0], [h, h], [0.0, h]])]
    x0, y0 = ii * h, jj * h
    blocks = np.empty((2 * N * N, 3, 3))
    for t in (0, 1):
        area, g = _gradients(ref[t])
        cx, cy = ref[t].mean(axis=0)
        kc = kappa(x0 + cx, y0 + cy)
        blocks[t::2] = kc[:, None, None] * (area * (g @ g.T))[None]
    # Nitsche terms on the triangles with a boundary facet
    bd = np.flatnonzero((ii == 0) | (jj == 0) | (ii == N - 1) | (jj == N - 1))
    for s in bd:
        i, j = int(ii[s]), int(jj[s])
        for t in (0, 1):
            P = ref[t] + np.array([i * h, j * h])
            P[np.abs(P - 1.0) < 1e-14] = 1.0             # exact boundary coordinates
            blocks[2 * s + t] += _nitsche(P, kappa, gamma_c)
    blocks = 0.5 * (blocks + blocks.transpose(0, 2, 1))
    n = nxn * nxn
    return uniform_problem(n, dofs, blocks, np.arange(n),
                           meta=dict(kind="diffusion_p1", N=N, gamma_c=gamma_c))
