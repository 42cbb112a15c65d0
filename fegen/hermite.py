"""Bicubic Hermite (Bogner-Fox-Schmit) discretisation of anisotropic
hyperdiffusion in H^2 on the unit square (the paper's H^2 problem class).

Form: a(u, v) = (q(u), q(v)) with q(w) = div(D grad w) for a constant tensor
D = eps I + (1 - eps) b b^T, b = (cos theta, sin theta), plus the symmetric
Nitsche terms for the clamped data u = 0, d_n u = 0 on every side:
gamma_0 <u, v> + gamma_1 <d_n u, d_n v> - <q(u), (D grad v).n> - <q(v), (D grad u).n>
+ <(D grad q(u)).n, v> + <(D grad q(v)).n, u>, gamma_0 = 24 p^4 / h^3 |D n|^2,
gamma_1 = 24 p^2 / h |D n|^2, p = 3.

Element DOFs: at each vertex (u, u_x, u_y, u_xy); 16 per element, global DOF
4 v + c for vertex v = j (N + 1) + i.  Supernode = vertex.  Quadrature: 4 x 4
Gauss on the element, 4 Gauss points on a boundary facet (exact for these
polynomial degrees with constant D).
"""
from __future__ import annotations

import numpy as np

from .common import gauss_legendre_01, uniform_problem


def _herm(t):
    """1-D cubic Hermite basis on [0, 1] (value at 0, slope at 0, value at 1,
    slope at 1) and its first three derivatives, rows = derivative order."""
    return np.array([
        [1 - 3 * t ** 2 + 2 * t ** 3, t - 2 * t ** 2 + t ** 3, 3 * t ** 2 - 2 * t ** 3, -t ** 2 + t ** 3],
        [-6 * t + 6 * t ** 2, 1 - 4 * t + 3 * t ** 2, 6 * t - 6 * t ** 2, -2 * t + 3 * t ** 2],
        [-6 + 12 * t, -4 + 6 * t, 6 - 12 * t, -2 + 6 * t],
        [12.0, 6.0, -12.0, 6.0],
    ])


# local DOF k = 4 * vertex + c, vertex (i, j) in {(0,0), (1,0), (0,1), (1,1)},
# c: 0 = u, 1 = u_x, 2 = u_y, 3 = u_xy
_VERT = [(0, 0), (1, 0), (0, 1), (1, 1)]


def _basis_1d_index(end: int, slope: int) -> int:
    return (0 if end == 0 else 2) + slope


def _derivs(x, y, h):
    """dict (a, b) -> array[16] of d^a/dx^a d^b/dy^b of the 16 physical basis
    functions at reference point (x, y) for a + b <= 3."""
    Hx, Hy = _herm(x), _herm(y)
    out = {}
    for a in range(4):
        for b in range(4 - a):
            v = np.empty(16)
            for vi, (i, j) in enumerate(_VERT):
                for c in range(4):
                    sx, sy = c & 1, c >> 1
                    fx = Hx[a, _basis_1d_index(i, sx)] * (h if sx else 1.0) / h ** a
                    fy = Hy[b, _basis_1d_index(j, sy)] * (h if sy else 1.0) / h ** b
                    v[4 * vi + c] = fx * fy
            out[(a, b)] = v
    return out


def bfs_element_matrices(D: np.ndarray, h: float):
    """(K_interior, F_left, F_right, F_bottom, F_top) for one element of size h."""
    qp, qw = gauss_legendre_01(4)
    D11, D12, D22 = D[0, 0], D[0, 1], D[1, 1]
    K = np.zeros((16, 16))
    for x, wx in zip(qp, qw):
        for y, wy in zip(qp, qw):
            d = _derivs(x, y, h)
            q = D11 * d[(2, 0)] + 2 * D12 * d[(1, 1)] + D22 * d[(0, 2)]
            K += wx * wy * h * h * np.outer(q, q)
    p = 3
    faces = {"left": (lambda s: (0.0, s), np.array([-1.0, 0.0])),
             "right": (lambda s: (1.0, s), np.array([1.0, 0.0])),
             "bottom": (lambda s: (s, 0.0), np.array([0.0, -1.0])),
             "top": (lambda s: (s, 1.0), np.array([0.0, 1.0]))}
    F = {}
    for name, (pt, n) in faces.items():
        Dn = D @ n
        dn2 = float(Dn @ Dn)
        g0 = 24.0 * p ** 4 / h ** 3 * dn2
        g1 = 24.0 * p ** 2 / h * dn2
        M = np.zeros((16, 16))
        for s, ws in zip(qp, qw):
            d = _derivs(*pt(s), h)
            u = d[(0, 0)]
            gu = np.stack([d[(1, 0)], d[(0, 1)]])                       # grad phi
            q = D11 * d[(2, 0)] + 2 * D12 * d[(1, 1)] + D22 * d[(0, 2)]
            gq = np.stack([D11 * d[(3, 0)] + 2 * D12 * d[(2, 1)] + D22 * d[(1, 2)],
                           D11 * d[(2, 1)] + 2 * D12 * d[(1, 2)] + D22 * d[(0, 3)]])
            dn_u = n @ gu                                               # d_n phi
            dDn_u = Dn @ gu                                             # (D grad phi) . n
            dDn_q = Dn @ gq                                             # (D grad q(phi)) . n
            w = ws * h
            M += w * (g0 * np.outer(u, u) + g1 * np.outer(dn_u, dn_u)
                      - np.outer(q, dDn_u) - np.outer(dDn_u, q)
                      + np.outer(dDn_q, u) + np.outer(u, dDn_q))
        F[name] = 0.5 * (M + M.T)
    return 0.5 * (K + K.T), F["left"], F["right"], F["bottom"], F["top"]


def diffusion_tensor(eps: float, theta: float) -> np.ndarray:
    b = np.array([np.cos(theta), np.sin(theta)])
    return eps * np.eye(2) + (1.0 - eps) * np.outer(b, b)


def hyperdiffusion_bfs(N: int, eps: float = 1e-4, theta: float = np.pi / 6):
    """Clamped anisotropic hyperdiffusion on an N x N mesh, 4 (N + 1)^2 DOFs."""
    h = 1.0 / N
    D = diffusion_tensor(eps, theta)
    K, FL, FR, FB, FT = bfs_element_matrices(D, h)
    nx = N + 1
    ei, ej = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    ei = ei.ravel()
    ej = ej.ravel()
    verts = np.stack([ej * nx + ei, ej * nx + ei + 1, (ej + 1) * nx + ei, (ej + 1) * nx + ei + 1], 1)
    dofs = (4 * verts[:, :, None] + np.arange(4)[None, None, :]).reshape(N * N, 16)
    blocks = np.repeat(K[None], N * N, axis=0)
    blocks[ei == 0] += FL
    blocks[ei == N - 1] += FR
    blocks[ej == 0] += FB
    blocks[ej == N - 1] += FT
    n = 4 * nx * nx
    return uniform_problem(n, dofs, blocks, np.arange(n) // 4, None,
                           meta=dict(kind="hyperdiffusion_bfs", N=N, eps=eps, theta=theta))
