"""Shared helpers for the seeded finite-element input generators.

These modules produce *inputs* for the solver: element blocks A_T with their
DOF lists (the cover of the conforming assembly A = sum_T R_T^T A_T R_T), the
supernode map, optional level-0 aggregates and right-hand sides.  They contain
none of the solver's arithmetic and are shared by the oracle tests and the GPU
tests/bench alike.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """An element-assembled SPD problem.

    n            number of global DOFs
    elem_ptr     int64[n_elem+1]   CSR offsets into elem_dofs
    elem_dofs    int32[sum n_T]    global DOFs of each element (local order)
    blocks       float64[sum n_T^2] element blocks, row-major, concatenated
    node_of_dof  int32[n]          supernode id of every DOF (all components /
                                   Hermite DOFs of a vertex, one edge, one cell)
    agg_of_dof   int32[n] or None  caller-given level-0 aggregates
    meta         free-form description of the workload
    """

    n: int
    elem_ptr: np.ndarray
    elem_dofs: np.ndarray
    blocks: np.ndarray
    node_of_dof: np.ndarray
    agg_of_dof: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return len(self.elem_ptr) - 1

    def element(self, e: int):
        """(dofs, dense block) of element e."""
        a, b = int(self.elem_ptr[e]), int(self.elem_ptr[e + 1])
        ne = b - a
        off = self.block_offsets()[e]
        return self.elem_dofs[a:b], self.blocks[off:off + ne * ne].reshape(ne, ne)

    def block_offsets(self) -> np.ndarray:
        if "_boff" not in self.__dict__:
            sizes = np.diff(self.elem_ptr)
            self.__dict__["_boff"] = np.concatenate([[0], np.cumsum(sizes * sizes)]).astype(np.int64)
        return self.__dict__["_boff"]


def uniform_problem(n, dofs_2d, blocks_3d, node_of_dof, agg_of_dof=None, meta=None) -> Problem:
    """Pack a problem whose elements all have the same size n_T."""
    n_elem, ne = dofs_2d.shape
    assert blocks_3d.shape == (n_elem, ne, ne)
    return Problem(
        n=int(n),
        elem_ptr=np.arange(0, (n_elem + 1) * ne, ne, dtype=np.int64),
        elem_dofs=np.ascontiguousarray(dofs_2d, dtype=np.int32).ravel(),
        blocks=np.ascontiguousarray(blocks_3d, dtype=np.float64).ravel(),
        node_of_dof=np.ascontiguousarray(node_of_dof, dtype=np.int32),
        agg_of_dof=None if agg_of_dof is None else np.ascontiguousarray(agg_of_dof, dtype=np.int32),
        meta=dict(meta or {}),
    )


def gauss_legendre_01(k: int):
    """k-point Gauss-Legendre rule on [0, 1] (exact for degree 2k-1)."""
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(nodes):
    """Return (eval, deriv, deriv2, deriv3) callables for the Lagrange basis on `nodes`.

    Each callable maps points t[m] to an array [m, len(nodes)].
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    k = len(nodes)
    V = np.vander(nodes, k, increasing=True)          # V[i, p] = t_i^p
    C = np.linalg.inv(V)                              # basis j = sum_p C[p, j] t^p

    def make(d):
        def f(t):
            t = np.atleast_1d(np.asarray(t, dtype=np.float64))
            out = np.zeros((len(t), k))
            for p in range(d, k):
                coef = np.prod(np.arange(p - d + 1, p + 1)) if d else 1.0
                out += coef * np.outer(t ** (p - d), C[p, :])
            return out
        return f

    return make(0), make(1), make(2), make(3)


def gll_nodes_01(k: int) -> np.ndarray:
    """k Gauss-Lobatto-Legendre nodes on [0, 1] (endpoints included)."""
    if k == 2:
        x = np.array([-1.0, 1.0])
    else:
        # interior GLL nodes are the roots of P'_{k-1}
        c = np.zeros(k)
        c[-1] = 1.0
        inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
        x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    return 0.5 * (x + 1.0)


def rhs(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. N(0, 1) right-hand sides, shape [n] (nrhs == 1) or [nrhs, n]."""
    b = rng.standard_normal((nrhs, n))
    return b[0] if nrhs == 1 else b


def lame_plane_strain(E: float, nu: float):
    """Lame parameters (lambda, mu) from Young's modulus and Poisson ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return lam, mu
