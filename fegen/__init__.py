"""Seeded synthetic inputs shaped like the paper's workloads (see each module).

Workload presets (all seeds through numpy.random.default_rng, draws in the order
mesh sizes, material parameters, element coefficients, right-hand sides):

* ``elasticity_small``  plane-strain Q1 elasticity, 32x32, E = 1, nu = 0.3, left
  edge clamped, vertex-patch cover (3x3-node blocks), 2,178 DOFs.
* ``graddiv_hdiv``      RTCF_3 grad-div on 128x128, kappa_T ~ lognormal(0, 1) on the
  div term, beta = 1e-4 mass, 295,680 DOFs.
* ``elasticity_batch``  64 Q1 instances, N_i ~ U{48..256}, nu_i ~ U(0.3, 0.49), 8 RHS.
* ``elasticity_q2``     Q2 hexes on 24^3, theta_T ~ lognormal(0, 0.5), nu = 0.3.
* ``hyperdiffusion_h2`` bicubic Hermite (BFS) anisotropic hyperdiffusion on 256x256, D rotated
  30 degrees, anisotropy 1e-4, clamped by Nitsche, 264,196 DOFs.
* ``closure_comparison`` CG1 triangles, kappa = 1 + x + y, u = 0 by Nitsche, b = 0 and a
  N(0, 1) initial iterate; N = 32 ... 1024 give 1,089 ... 1,050,625 DOFs.
"""
from __future__ import annotations

import numpy as np

from .common import Problem, rhs  # noqa: F401
from .elasticity import elasticity_q1, elasticity_q2hex  # noqa: F401
from .hdiv import graddiv_rtcf3  # noqa: F401
from .p1 import diffusion_p1_triangles  # noqa: F401


def elasticity_small(N: int = 32, seed: int = 0, nrhs: int = 1):
    """Plain elasticity workload (default 32x32 -> 2,178 DOFs); returns (problem, b)."""
    rng = np.random.default_rng(seed)
    prob = elasticity_q1(N, nu=0.3, E=1.0)
    return prob, rhs(prob.n, nrhs, rng)


def graddiv_hdiv(N: int = 128, seed: int = 0, nrhs: int = 1, beta: float = 1e-4, sigma: float = 1.0):
    """Grad-div workload (default 128x128 RTCF_3 -> 295,680 DOFs); returns (problem, b)."""
    rng = np.random.default_rng(seed)
    kappa = np.exp(sigma * rng.standard_normal(N * N))
    prob = graddiv_rtcf3(N, kappa=kappa, beta=beta)
    return prob, rhs(prob.n, nrhs, rng)


def elasticity_batch(n_inst: int = 64, nmin: int = 48, nmax: int = 256, seed: int = 0, nrhs: int = 8):
    """Uneven batch of Q1 elasticity instances; returns [(problem, b[nrhs, n])]."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(nmin, nmax + 1, size=n_inst)
    nus = rng.uniform(0.3, 0.49, size=n_inst)
    out = []
    for N, nu in zip(Ns, nus):
        out.append(elasticity_q1(int(N), nu=float(nu), E=1.0))
    return [(p, np.atleast_2d(rhs(p.n, nrhs, rng))) for p in out]


def elasticity_q2(N: int = 24, seed: int = 0, nrhs: int = 1):
    """Q2 hex elasticity with lognormal per-element modulus; returns (problem, b, theta)."""
    rng = np.random.default_rng(seed)
    theta = np.exp(0.5 * rng.standard_normal(N ** 3))
    prob = elasticity_q2hex(N, nu=0.3, E=1.0, theta=theta)
    return prob, rhs(prob.n, nrhs, rng), theta


def hyperdiffusion_h2(N: int = 256, seed: int = 0, nrhs: int = 1, eps: float = 1e-4, theta: float = np.pi / 6):
    """Clamped anisotropic hyperdiffusion on BFS elements (default 256 x 256 -> 264,196 DOFs); (problem, b)."""
    from .hermite import hyperdiffusion_bfs
    rng = np.random.default_rng(seed)
    prob = hyperdiffusion_bfs(N, eps=eps, theta=theta)
    return prob, rhs(prob.n, nrhs, rng)


def closure_comparison(N: int = 32, seed: int = 0):
    """Scalar diffusion on CG1 triangles with zero data and a random start; (problem, b, x0)."""
    rng = np.random.default_rng(seed)
    prob = diffusion_p1_triangles(N)
    return prob, np.zeros(prob.n), rng.standard_normal(prob.n)
