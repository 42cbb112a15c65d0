"""Vector linear elasticity inputs (plane strain Q1 quads, Q2 hexes).

Bilinear form (strain/stress of the elasticity section):
    a(u, v) = 2 mu (eps(u), eps(v)) + lambda (div u, div v)
plus, on clamped facets, the symmetric Nitsche terms
    <gamma u, v> - <sigma(u) n, v> - <sigma(v) n, u>,  gamma_F = 24 p^2 (lambda + 2 mu) / h_F,
so every element block stays symmetric positive semidefinite and no DOF is
eliminated.  Element blocks are exact (Gauss rules of sufficient order).
"""
from __future__ import annotations

import numpy as np

from .common import Problem, gauss_legendre_01, lame_plane_strain, uniform_problem

# --------------------------------------------------------------------------- 2D Q1


def _q1_shape(xi, eta):
    """Q1 shape values / reference gradients at one point; nodes lexicographic a = ax + 2 ay."""
    lx = np.array([1.0 - xi, xi])
    ly = np.array([1.0 - eta, eta])
    dl = np.array([-1.0, 1.0])
    N = np.array([lx[a % 2] * ly[a // 2] for a in range(4)])
    dN = np.array([[dl[a % 2] * ly[a // 2], lx[a % 2] * dl[a // 2]] for a in range(4)])
    return N, dN


def q1_element_matrix(lam: float, mu: float, h: float, left_nitsche: bool = False) -> np.ndarray:
    """8x8 element matrix of a square Q1 cell of size h; DOF 2a+c (node a, component c)."""
    D = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    qp, qw = gauss_legendre_01(2)
    K = np.zeros((8, 8))
    for xi, wx in zip(qp, qw):
        for eta, wy in zip(qp, qw):
            _, dN = _q1_shape(xi, eta)
            g = dN / h
            B = np.zeros((3, 8))
            B[0, 0::2] = g[:, 0]
            B[1, 1::2] = g[:, 1]
            B[2, 0::2] = g[:, 1]
            B[2, 1::2] = g[:, 0]
            K += wx * wy * h * h * B.T @ D @ B
    if left_nitsche:
        gamma = 24.0 * 1.0 ** 2 / h * (lam + 2 * mu)
        n = np.array([-1.0, 0.0])
        for eta, wy in zip(qp, qw):
            N, dN = _q1_shape(0.0, eta)
            g = dN / h
            V = np.zeros((2, 8))
            V[0, 0::2] = N
            V[1, 1::2] = N
            # sigma(u) n for unit-coefficient DOFs: rows = traction components
            sxx = np.zeros(8); syy = np.zeros(8); sxy = np.zeros(8)
            sxx[0::2] = (lam + 2 * mu) * g[:, 0]; sxx[1::2] = lam * g[:, 1]
            syy[0::2] = lam * g[:, 0];            syy[1::2] = (lam + 2 * mu) * g[:, 1]
            sxy[0::2] = mu * g[:, 1];             sxy[1::2] = mu * g[:, 0]
            T = np.vstack([sxx * n[0] + sxy * n[1], sxy * n[0] + syy * n[1]])
            K += wy * h * (gamma * V.T @ V - V.T @ T - T.T @ V)
    return 0.5 * (K + K.T)


def vertex_patch_aggregates(nx_nodes: int, ny_nodes: int, comps: int, width: int = 3) -> np.ndarray:
    """Aggregates of width x width vertex blocks (last block may be narrower).

    DOF numbering is node-major: dof = comps * (iy * nx_nodes + ix) + c.
    """
    nbx = -(-nx_nodes // width)
    ix = np.arange(nx_nodes)
    iy = np.arange(ny_nodes)
    agg_node = (iy[:, None] // width) * nbx + (ix[None, :] // width)
    return np.repeat(agg_node.ravel(), comps).astype(np.int32)


def elasticity_q1(N: int, nu: float = 0.3, E: float = 1.0, theta=None, clamp_left: bool = True,
                  vertex_patches: bool = True) -> Problem:
    """Plane-strain Q1 elasticity on an N x N mesh of (0,1)^2, left edge clamped by Nitsche.

    theta: optional per-element Young's modulus multipliers (blocks are linear in E).
    """
    lam, mu = lame_plane_strain(E, nu)
    h = 1.0 / N
    K_in = q1_element_matrix(lam, mu, h, False)
    K_bd = q1_element_matrix(lam, mu, h, True) if clamp_left else K_in
    nxn = N + 1
    ei, ej = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")   # ej row-major
    ei = ei.ravel(); ej = ej.ravel()
    corner = np.stack([ej * nxn + ei, ej * nxn + ei + 1, (ej + 1) * nxn + ei, (ej + 1) * nxn + ei + 1], 1)
    dofs = np.empty((N * N, 8), dtype=np.int64)
    dofs[:, 0::2] = 2 * corner
    dofs[:, 1::2] = 2 * corner + 1
    blocks = np.where((ei == 0)[:, None, None], K_bd[None], K_in[None]).astype(np.float64)
    if theta is not None:
        blocks = blocks * np.asarray(theta, dtype=np.float64)[:, None, None]
    n = 2 * nxn * nxn
    node_of_dof = np.arange(n) // 2
    agg = vertex_patch_aggregates(nxn, nxn, 2) if vertex_patches else None
    return uniform_problem(n, dofs, blocks, node_of_dof, agg,
                           meta=dict(kind="elasticity_q1", N=N, nu=nu, E=E, lam=lam, mu=mu))


# --------------------------------------------------------------------------- 3D Q2


def _q2_1d(t):
    """Quadratic Lagrange basis on nodes {0, 1/2, 1} and derivatives."""
    v = np.array([2 * (t - 0.5) * (t - 1.0), -4 * t * (t - 1.0), 2 * t * (t - 0.5)])
    d = np.array([4 * t - 3.0, -8 * t + 4.0, 4 * t - 1.0])
    return v, d


def q2hex_element_matrices(lam: float, mu: float, h: float):
    """(K_interior, F_face) for a cube Q2 element (81 DOFs, DOF 3a+c, a lexicographic 27 nodes).

    F_face is the symmetric Nitsche contribution of the x = 0 face.
    """
    qp, qw = gauss_legendre_01(3)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2 * mu
    C[3:, 3:] = np.eye(3) * mu
    K = np.zeros((81, 81))

    def grads(x, y, z):
        vx, dx = _q2_1d(x); vy, dy = _q2_1d(y); vz, dz = _q2_1d(z)
        Nv = np.zeros(27); G = np.zeros((27, 3))
        for c in range(3):
            for b in range(3):
                for a in range(3):
                    k = a + 3 * b + 9 * c
                    Nv[k] = vx[a] * vy[b] * vz[c]
                    G[k] = [dx[a] * vy[b] * vz[c], vx[a] * dy[b] * vz[c], vx[a] * vy[b] * dz[c]]
        return Nv, G / h

    def bmat(G):
        B = np.zeros((6, 81))
        B[0, 0::3] = G[:, 0]; B[1, 1::3] = G[:, 1]; B[2, 2::3] = G[:, 2]
        B[3, 1::3] = G[:, 2]; B[3, 2::3] = G[:, 1]          # gamma_yz
        B[4, 0::3] = G[:, 2]; B[4, 2::3] = G[:, 0]          # gamma_xz
        B[5, 0::3] = G[:, 1]; B[5, 1::3] = G[:, 0]          # gamma_xy
        return B

    for x, wx in zip(qp, qw):
        for y, wy in zip(qp, qw):
            for z, wz in zip(qp, qw):
                _, G = grads(x, y, z)
                B = bmat(G)
                K += wx * wy * wz * h ** 3 * B.T @ C @ B
    F = np.zeros((81, 81))
    gamma = 24.0 * 2 ** 2 / h * (lam + 2 * mu)
    n = np.array([-1.0, 0.0, 0.0])
    for y, wy in zip(qp, qw):
        for z, wz in zip(qp, qw):
            Nv, G = grads(0.0, y, z)
            V = np.zeros((3, 81))
            for c in range(3):
                V[c, c::3] = Nv
            S = C @ bmat(G)      # Voigt stress [xx, yy, zz, yz, xz, xy] per DOF
            sig = np.array([[S[0], S[5], S[4]], [S[5], S[1], S[3]], [S[4], S[3], S[2]]])
            T = np.einsum("ijk,j->ik", sig, n)
            F += wy * wz * h * h * (gamma * V.T @ V - V.T @ T - T.T @ V)
    return 0.5 * (K + K.T), 0.5 * (F + F.T)


def elasticity_q2hex(N: int, nu: float = 0.3, E: float = 1.0, theta=None) -> Problem:
    """Q2 hexahedral elasticity on an N^3 mesh of (0,1)^3, x = 0 face clamped by Nitsche."""
    lam, mu = lame_plane_strain(E, nu)
    h = 1.0 / N
    K, F = q2hex_element_matrices(lam, mu, h)
    M = 2 * N + 1
    e = np.arange(N ** 3)
    ex, ey, ez = e % N, (e // N) % N, e // (N * N)
    loc = np.array([[a, b, c] for c in range(3) for b in range(3) for a in range(3)])
    nodes = ((2 * ez[:, None] + loc[None, :, 2]) * M + (2 * ey[:, None] + loc[None, :, 1])) * M \
        + (2 * ex[:, None] + loc[None, :, 0])
    dofs = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(len(e), 81)
    blocks = np.where((ex == 0)[:, None, None], (K + F)[None], K[None])
    if theta is not None:
        blocks = blocks * np.asarray(theta, dtype=np.float64)[:, None, None]
    n = 3 * M ** 3
    return uniform_problem(n, dofs, blocks, np.arange(n) // 3, None,
                           meta=dict(kind="elasticity_q2hex", N=N, nu=nu, E=E, lam=lam, mu=mu))
