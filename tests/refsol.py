"""Reference solutions accurate beyond FP64 for ill-conditioned test operators.

A sparse LU factorization in FP64 followed by iterative refinement whose residuals
b - A x are formed in extended precision (numpy longdouble, a 64-bit mantissa on
x86) with x kept in extended precision (Wilkinson's mixed-precision refinement).
Each step contracts the error by about eps_64 cond(A), so the result is accurate to
about eps_ld cond(A) in the A-norm, where any FP64 computation of A x, and hence
any FP64 solver, stops at about eps_64 cond(A).
"""
import numpy as np
import scipy.sparse.linalg as spla

LD = np.longdouble


def residual_ld(A, x, b):
    """b - A x in extended precision (A CSR with sorted indices)."""
    prod = A.data.astype(LD) * np.asarray(x, dtype=LD)[A.indices]
    return np.asarray(b, dtype=LD) - np.add.reduceat(prod, A.indptr[:-1])


def extended_reference(A, b, steps=6):
    A = A.tocsr()
    A.sort_indices()
    lu = spla.splu(A.tocsc())
    x = lu.solve(np.asarray(b, dtype=np.float64)).astype(LD)
    for _ in range(steps):
        x = x + lu.solve(np.asarray(residual_ld(A, x, b), dtype=np.float64)).astype(LD)
    return np.asarray(x, dtype=np.float64)


def anorm_rel(A, x, x_ref):
    d = np.asarray(x) - x_ref
    return float(np.sqrt(d @ (A @ d)) / np.sqrt(x_ref @ (A @ x_ref)))
