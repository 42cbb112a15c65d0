"""FP64 CPU oracle of the gradient of u = A(theta)^{-1} b (test infrastructure only).

Like ``oracle.lsdd`` this module is the checker, not the product: only the test
suite, the smoke entry point and the benchmark's CPU-baseline leg may import it.

Setting.  The element blocks are linear in a per-element coefficient,
A_e(theta) = theta_e A_e^(1) (Young's modulus multiplies every term of the
elasticity forms, the Nitsche boundary terms included), so the assembled operator
of the paper's elementwise formulation (Sec. 5.1, Prop. "elementwise Gram
formulation") is A(theta) = sum_e theta_e R_e^T A_e^(1) R_e and dA/dtheta_e =
R_e^T A_e^(1) R_e.  The paper does not treat derivatives; the formulas below are
the plain definition of the derivative of the solution map:

* d u / d theta_e = -A^{-1} (dA/dtheta_e) u, hence for a scalar output L(u) with
  adjoint load ubar = dL/du, lambda = A^{-1} ubar (A is symmetric) and
  dL/dtheta_e = -lambda_e^T A_e^(1) u_e, dL/db = lambda.
* For the compliance J = b^T u the adjoint load is b itself, lambda = u and
  dJ/dtheta_e = -u_e^T A_e^(1) u_e.

Solves are direct (sparse LU), so the oracle gradient is the exact one up to
rounding; it does not use the multilevel hierarchy.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _elements(prob):
    """(list of DOF index arrays, list of unit blocks) of a problem object."""
    ptr = np.asarray(prob.elem_ptr)
    offs = np.concatenate([[0], np.cumsum(np.diff(ptr) ** 2)])
    dofs = [np.asarray(prob.elem_dofs[ptr[e]:ptr[e + 1]], dtype=np.int64) for e in range(len(ptr) - 1)]
    blocks = [np.asarray(prob.blocks[offs[e]:offs[e + 1]]).reshape(len(dofs[e]), -1) for e in range(len(dofs))]
    return dofs, blocks


def assemble_scaled(prob_unit, theta) -> sp.csc_matrix:
    """A(theta) = sum_e theta_e R_e^T A_e^(1) R_e."""
    dofs, blocks = _elements(prob_unit)
    rows, cols, vals = [], [], []
    for e, (d, B) in enumerate(zip(dofs, blocks)):
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(theta[e] * B.ravel())
    n = prob_unit.n
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def solve(prob_unit, theta, b) -> np.ndarray:
    """u = A(theta)^{-1} b by sparse LU (b may hold several right-hand sides as rows)."""
    lu = spla.splu(assemble_scaled(prob_unit, theta))
    b = np.asarray(b, dtype=np.float64)
    return lu.solve(b.T).T if b.ndim == 2 else lu.solve(b)


def element_bilinear(prob_unit, u, v) -> np.ndarray:
    """out_e = u_e^T A_e^(1) v_e for every element."""
    dofs, blocks = _elements(prob_unit)
    return np.array([u[d] @ B @ v[d] for d, B in zip(dofs, blocks)])


def adjoint_gradient(prob_unit, theta, b, ubar):
    """(u, dL/dtheta, dL/db) for a scalar L(u) with dL/du = ubar."""
    lu = spla.splu(assemble_scaled(prob_unit, theta))
    u = lu.solve(np.asarray(b, dtype=np.float64))
    lam = lu.solve(np.asarray(ubar, dtype=np.float64))
    return u, -element_bilinear(prob_unit, lam, u), lam


def compliance_gradient(prob_unit, theta, b):
    """(J, dJ/dtheta) for the compliance J = b^T u(theta)."""
    u = solve(prob_unit, theta, b)
    return float(b @ u), -element_bilinear(prob_unit, u, u)
