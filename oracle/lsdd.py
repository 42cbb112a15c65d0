"""Plain FP64 CPU oracle of the LS-AMG-DD hot path (test infrastructure only).

This module is the checker, not the product: only the test suite, the smoke
entry point and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the HIP library and is deliberately slow and literal: dense LAPACK
per element / aggregate, scipy.sparse for the assembled operators, Python loops
over aggregates in the order the method defines them.

Paper sections followed (Krzysik, Southworth, Wimmer, "A black-box, multilevel
algebraic preconditioning framework for conforming finite elements"):

* Sec. 5.1 (Prop. "elementwise Gram formulation"): A = sum_T R_T^T A_T R_T and
  G = [G_T R_T] stacked, with A_T = G_T^T G_T.
* Sec. 5.2: local factor G_T = Lambda_+^{1/2} Q_+^T from an eigendecomposition.
* Sec. 2, eq. (agg_def): disjoint aggregates from standard aggregation.
* Sec. 2, eqs. (calR_def), (overlap_def), Def. "G-row closure": rows touching an
  aggregate and the overlap Omega_i = union of their supports, Gamma_i = Omega_i minus omega_i.
* Sec. 2, eqs. (row_multiplicity), (Wmatrix-def), (SPSD_splitting): multiplicity
  weights and the exact local SPSD splitting A~_Omega = H^T H.
* Sec. 2, eqs. (gep_local), (gep_reduced), (tau-cut): the reduced local
  generalized eigenproblem on the aggregate, its Schur complement with a
  Moore-Penrose pseudo-inverse, and the adaptive cutoff tau_cut = c max mult.
* Sec. 2 (interpolation and Galerkin recursion): P = [R_w^T Z_i], A_c = P^T A P,
  G_c = G P; direct solve on the coarsest level.
* Sec. 2 (two-level cycle) and Sec. 6 (solver settings): forward multiplicative
  Schwarz pre-smoothing on the overlaps, reverse-order post-smoothing, stop rule
  (fewer than 10 DOFs, density above 25 %, level cap); the other block Schwarz
  smoothers Sec. 2 names (restricted additive Schwarz, block Jacobi) with the
  post-smoother M^{-T}.
* Outer iteration: preconditioned CG (Hestenes-Stiefel) from x0 = 0 to a relative
  residual tolerance; the paper's own standalone-cycle mode is ``stationary``.

Readings taken where the paper is silent (each is listed in the design notes):
R1 structural support of element rows (every row of G_T spans all DOFs of T),
R2 rank tolerance n_T eps lambda_max, R3 aggregation phases/passes and the
supernode graph, R4 pseudo-inverse tolerance |Gamma| eps d_max (and the equivalent
projector form on the weighted Gram rows as a second route), R5 the reduced
problem solved as S~ u = mu A_ww u with mu = 1/lambda, R6 tau_cut uses the
level-wide maximum multiplicity, R7/R8 cluster completion and threshold band,
R9 A_ww-orthonormal Z, R11 colour-major sweep order, R12 coarse elements grouped
by the set of aggregates they touch, R14 the local matrix on an A-closure is the
principal submatrix of the G-row closure's local matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

EPS = np.finfo(np.float64).eps


class NotSPSD(ValueError):
    """An element block has an eigenvalue below -spsd_tol * lambda_max."""


@dataclass
class Params:
    max_levels: int = 3
    agg_passes: int = 2           # standard-aggregation passes on level 0
    agg_passes_coarse: int = 1    # passes on coarser levels (reading R3)
    modes_fixed: int = 0          # 0: threshold selection with tau_cut
    tau_const: float = 0.75
    min_coarse: int = 10
    max_density: float = 0.25
    cluster_tol: float = 1e-9
    band_tol: float = 1e-9
    rank_rtol: float = 0.0        # 0: n_T * eps
    spsd_tol: float = 1e-12
    rtol: float = 1e-8
    max_iter: int = 1000
    # route to the Schur complement of eq. (gep_reduced): "pinv" (the Moore-Penrose
    # pseudo-inverse of A~_GammaGamma by its eigendecomposition, reading R4; the method's
    # definition and the default) or "projector" (the same quantity in its equivalent
    # form H_w^T (I - Pi_range(H_Gamma)) H_w on the weighted Gram rows, with the R4 rule
    # applied to the squared singular values of H_Gamma; a second FP64 route whose
    # distance from "pinv" measures how far rounding alone moves the result)
    interface: str = "pinv"
    # overlaps: "G" = G-row closure (Def. "G-row closure", the method's choice) or
    # "A" = algebraic A-closure (Def. "algebraic A-closure", the comparison of Sec. 5.3);
    # with "A" an entry counts as nonzero when |A(p,q)| > closure_tol sqrt(A(p,p) A(q,q))
    closure: str = "G"
    closure_tol: float = 1e-12
    # block Schwarz smoother M^{-1} of the cycle (Sec. 2, two-level propagator with
    # pre-smoother M^{-1} and post-smoother M^{-T}): "ms" forward multiplicative Schwarz
    # on the overlaps (post: reverse order; Sec. 6), "ras" restricted additive Schwarz
    # (local solves on the overlaps, corrections kept on the aggregates), "bj" block
    # Jacobi on the aggregates
    smoother: str = "ms"
    # element Gram factor (Sec. 5.2): "eig" = Lambda_+^{1/2} Q_+^T, "chol" = pivoted Cholesky
    elem_factor: str = "eig"


# ----------------------------------------------------------------- element factors (Sec. 5.2)

def element_gram_factor(Ae: np.ndarray, rank_rtol: float = 0.0, spsd_tol: float = 1e-12) -> np.ndarray:
    """Range factor G_T = Lambda_+^{1/2} Q_+^T with A_T = Q Lambda Q^T (Sec. 5.2).

    Eigenvalues above n_T * eps * lambda_max (or rank_rtol * lambda_max) count as
    the positive spectrum; an eigenvalue below -spsd_tol * lambda_max means the
    block is not SPSD, which the construction requires (Sec. 5.1).
    """
    ne = Ae.shape[0]
    w, Q = np.linalg.eigh(Ae)
    lmax = max(float(w[-1]), 0.0)
    if w[0] < -spsd_tol * lmax:
        raise NotSPSD(f"lambda_min = {w[0]:.3e}, lambda_max = {lmax:.3e}")
    tol = (rank_rtol if rank_rtol > 0 else ne * EPS) * lmax
    keep = w > tol
    return np.sqrt(w[keep])[:, None] * Q[:, keep].T


def element_gram_factor_pchol(Ae: np.ndarray, rank_rtol: float = 0.0, spsd_tol: float = 1e-12) -> np.ndarray:
    """Pivoted Cholesky factor (Sec. 5.2): G_T with rows g_1 .. g_r, A_T = G_T^T G_T up to
    the truncated remainder.

    Step k takes the largest remaining diagonal entry of the Schur complement S
    (lowest index among equal ones) as pivot p, forms g_k = S[:, p] / sqrt(S[p, p])
    (zero on the DOFs already eliminated) and subtracts g_k g_k^T.  The
    factorisation stops when the largest remaining diagonal entry is at most
    tol = (rank_rtol or n_T eps) * max diag(A_T); the rank is the number of steps.
    For an SPSD block the remainder is then bounded by tol entrywise (|S_ij| <=
    sqrt(S_ii S_jj)); a remainder entry above 2 max(tol, spsd_tol max diag), or a
    diagonal entry below -spsd_tol max diag, means the block is not SPSD.  For an
    SPD block the rows are the transposed Cholesky factor of the block with rows
    and columns in pivot order, so G_T is a square factor L_T^T up to that
    symmetric permutation.
    """
    ne = Ae.shape[0]
    S = np.array(Ae, dtype=np.float64, copy=True)
    dmax0 = float(np.max(np.diag(S))) if ne else 0.0
    if ne == 0 or dmax0 <= 0.0:
        if ne and np.abs(S).max() > 0.0:
            raise NotSPSD("non-positive diagonal with nonzero entries")
        return np.zeros((0, ne))
    tol = (rank_rtol if rank_rtol > 0 else ne * EPS) * dmax0
    live = np.ones(ne, dtype=bool)
    rows = []
    for _ in range(ne):
        d = np.where(live, np.diag(S), -np.inf)
        p = int(np.argmax(d))                    # first index of the maximum
        if not d[p] > tol:
            break
        g = np.where(live, S[:, p], 0.0) / np.sqrt(d[p])
        rows.append(g)
        S -= np.outer(g, g)
        live[p] = False
    if live.any():
        R = S[np.ix_(live, live)]
        chk = max(tol, spsd_tol * dmax0)
        if np.diag(R).min() < -spsd_tol * dmax0 or np.abs(R).max() > 2.0 * chk:
            raise NotSPSD(f"pivoted Cholesky remainder {np.abs(R).max():.3e} above {chk:.3e}")
    return np.array(rows).reshape(len(rows), ne)


# ----------------------------------------------------------------- assembly (Sec. 4, Sec. 5.1)

def assemble(n: int, elem_dofs, blocks) -> sp.csr_matrix:
    """A = sum_T R_T^T A_T R_T with the structural pattern kept (no zero dropping)."""
    rows, cols, vals = [], [], []
    for S, Ae in zip(elem_dofs, blocks):
        k = len(S)
        rows.append(np.repeat(S, k))
        cols.append(np.tile(S, k))
        vals.append(np.asarray(Ae).ravel())
    if not rows:
        return sp.csr_matrix((n, n))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def structural_pattern(n: int, elem_dofs) -> sp.csr_matrix:
    """Boolean pattern of sum_T R_T^T 1 R_T."""
    return assemble(n, elem_dofs, [np.ones((len(S), len(S))) for S in elem_dofs])


# ----------------------------------------------------------------- aggregation (eq. agg_def)

def supernode_graph(n_super: int, node_of_dof: np.ndarray, elem_dofs) -> sp.csr_matrix:
    """Supernodes s ~ t iff some element holds DOFs of both (all connections strong)."""
    rows, cols = [], []
    for e, S in enumerate(elem_dofs):
        nodes = np.unique(node_of_dof[S])
        rows.append(np.full(len(nodes), e))
        cols.append(nodes)
    E = sp.csr_matrix((np.ones(sum(len(c) for c in cols)), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(len(elem_dofs), n_super))
    Adj = (E.T @ E).tocsr()
    Adj.setdiag(0)
    Adj.eliminate_zeros()
    Adj.sort_indices()
    return Adj


def standard_aggregation(adj: sp.csr_matrix) -> np.ndarray:
    """Standard aggregation (Vanek-Mandel-Brezina) on a graph with all edges strong.

    1. In ascending order, a node whose neighbourhood is entirely unaggregated
       becomes a root; the aggregate is the root plus its neighbours.
    2. Every node still unaggregated joins the phase-1 aggregate of its
       lowest-index phase-1-aggregated neighbour.
    3. Any node left (none, unless isolated) starts an aggregate with its free
       neighbours.
    Aggregates are numbered in creation order.
    """
    n = adj.shape[0]
    agg = np.full(n, -1, dtype=np.int64)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = adj.indices[adj.indptr[i]:adj.indptr[i + 1]]
        if np.all(agg[nb] < 0):
            agg[i] = na
            agg[nb] = na
            na += 1
    phase1 = agg.copy()
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = np.sort(adj.indices[adj.indptr[i]:adj.indptr[i + 1]])
        for j in nb:
            if phase1[j] >= 0:
                agg[i] = phase1[j]
                break
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = adj.indices[adj.indptr[i]:adj.indptr[i + 1]]
        agg[i] = na
        agg[nb[agg[nb] < 0]] = na
        na += 1
    return agg


def aggregate_supernodes(adj: sp.csr_matrix, passes: int) -> np.ndarray:
    """Apply standard aggregation `passes` times; pass k+1 aggregates the aggregates of pass k."""
    n = adj.shape[0]
    agg = np.arange(n)
    g = adj
    for _ in range(passes):
        a = standard_aggregation(g)
        agg = a[agg]
        na = int(a.max()) + 1
        T = sp.csr_matrix((np.ones(len(a)), (np.arange(len(a)), a)), shape=(len(a), na))
        g = (T.T @ g @ T).tocsr()
        g.setdiag(0)
        g.eliminate_zeros()
        g.sort_indices()
    return agg


# ----------------------------------------------------------------- level data

@dataclass
class Level:
    n: int
    level: int
    elem_dofs: list                     # global DOFs per element (level numbering)
    blocks: list                        # dense A_T (level numbering)
    node_of_dof: np.ndarray             # supernode per DOF
    A: sp.csr_matrix = None
    nnz: int = 0                        # structural nonzeros of A
    # coarsening data (absent on the coarsest level)
    agg_of_dof: np.ndarray = None
    aggs: list = field(default_factory=list)      # omega_i, ascending
    omegas: list = field(default_factory=list)    # Omega_i: omega_i then Gamma_i (ascending each)
    closure: list = field(default_factory=list)   # elements touching omega_i
    mult: np.ndarray = None             # aggregate-touching multiplicity per element
    tau_cut: float = 0.0
    mu: list = field(default_factory=list)        # sorted local spectra per aggregate
    k: np.ndarray = None                # retained modes per aggregate
    Z: list = field(default_factory=list)
    P: sp.csr_matrix = None
    coarse_off: np.ndarray = None
    colors: np.ndarray = None
    order: np.ndarray = None            # sweep order: (colour, index) ascending
    chol: list = field(default_factory=list)      # Cholesky factors of A_Omega_i (A_ww for "bj")
    smoother: str = "ms"
    coarsest_chol: tuple = None
    gram: list = None                   # element Gram factors (level 0; "projector" route)


@dataclass
class Hierarchy:
    levels: list
    params: Params
    G0: list = None                     # level-0 element Gram factors


# ----------------------------------------------------------------- closures (Sec. 2, Sec. 5.3)

def closures(n_agg: int, agg_of_dof: np.ndarray, elem_dofs):
    """Element closures cl(omega_i), overlaps Omega_i (omega first), multiplicities.

    Under reading R1 every row of G_T is supported on all DOFs of T, so the rows
    touching omega_i are the rows of the elements with a DOF in omega_i and the
    G-row closure (Def. "G-row closure") is the union of those elements' DOFs.
    mult(T) counts the aggregates T touches (eq. row_multiplicity).
    """
    touched = [np.unique(agg_of_dof[S]) for S in elem_dofs]
    mult = np.array([len(t) for t in touched], dtype=np.int64)
    cl = [[] for _ in range(n_agg)]
    for e, t in enumerate(touched):
        for i in t:
            cl[i].append(e)
    aggs = [np.flatnonzero(agg_of_dof == i) for i in range(n_agg)]
    omegas = []
    for i in range(n_agg):
        if cl[i]:
            U = np.unique(np.concatenate([elem_dofs[e] for e in cl[i]]))
        else:
            U = aggs[i]
        gamma = np.setdiff1d(U, aggs[i])
        omegas.append(np.concatenate([aggs[i], gamma]).astype(np.int64))
    return aggs, omegas, [np.array(c, dtype=np.int64) for c in cl], mult


def a_closure(A: sp.csr_matrix, omega: np.ndarray, tol: float) -> np.ndarray:
    """Algebraic A-closure (Def. "algebraic A-closure"): omega_i, then the DOFs p
    outside omega_i whose row block A(p, omega_i) holds an entry with
    |A(p,q)| > tol sqrt(A(p,p) A(q,q)) (ascending).  A is symmetric, so the rows
    of omega_i are scanned."""
    d = A.diagonal()
    R = A[omega].tocoo()
    q = omega[R.row]
    keep = np.abs(R.data) > tol * np.sqrt(np.abs(d[q] * d[R.col]))
    gamma = np.setdiff1d(np.unique(R.col[keep]), omega)
    return np.concatenate([omega, gamma]).astype(np.int64)


def local_splitting(omega_dofs: np.ndarray, cl_elems, elem_dofs, blocks, mult) -> np.ndarray:
    """A~_Omega = sum_{T in cl} mult(T)^{-1} E_T^T A_T E_T (eq. SPSD_splitting under R1)."""
    pos = {int(d): a for a, d in enumerate(omega_dofs)}
    m = len(omega_dofs)
    At = np.zeros((m, m))
    for e in cl_elems:
        idx = np.array([pos[int(d)] for d in elem_dofs[e]])
        At[np.ix_(idx, idx)] += blocks[e] / mult[e]
    return At


def schur_pinv(At: np.ndarray, nw: int) -> np.ndarray:
    """S~ = A~_ww - A~_wG (A~_GG)^+ A~_Gw (eq. gep_reduced).

    The pseudo-inverse comes from the eigendecomposition of A~_GG: eigenvalues
    above |Gamma| eps d_max form its range (reading R4).  With Gamma empty,
    S~ = A~_ww.
    """
    Aww = At[:nw, :nw]
    if At.shape[0] == nw:
        return 0.5 * (Aww + Aww.T)
    AwG = At[:nw, nw:]
    AGG = At[nw:, nw:]
    d, V = np.linalg.eigh(AGG)
    dmax = max(float(d[-1]), 0.0)
    keep = d > AGG.shape[0] * EPS * dmax if dmax > 0 else np.zeros(len(d), bool)
    Vk = V[:, keep]
    W = AwG @ Vk
    S = Aww - (W / d[keep]) @ W.T
    return 0.5 * (S + S.T)


def schur_projector(H: np.ndarray, nw: int) -> np.ndarray:
    """The same Schur complement from the weighted Gram rows H of the overlap
    (A~_Omega = H^T H, eq. SPSD_splitting): S~ = H_w^T (I - U_r U_r^T) H_w with U_r
    the left singular vectors of H_Gamma whose squared singular values exceed
    |Gamma| eps s_max^2 (the R4 rule on the eigenvalues of A~_GG = H_G^T H_G).
    For A~_GG = V D V^T this is the pseudo-inverse expression term by term,
    A~_wG V_r D_r^{-1} V_r^T A~_Gw = H_w^T U_r U_r^T H_w, without forming A~_GG."""
    Hw = H[:, :nw]
    if H.shape[1] == nw:
        S = Hw.T @ Hw
        return 0.5 * (S + S.T)
    HG = H[:, nw:]
    U, sv, _ = np.linalg.svd(HG, full_matrices=False)
    smax = float(sv[0]) if len(sv) else 0.0
    keep = sv ** 2 > HG.shape[1] * EPS * smax ** 2 if smax > 0 else np.zeros(len(sv), bool)
    Y = U[:, keep].T @ Hw
    S = Hw.T @ Hw - Y.T @ Y
    return 0.5 * (S + S.T)


def local_gram_rows(omega_dofs: np.ndarray, cl_elems, elem_dofs, factors, mult) -> np.ndarray:
    """H_Omega: the rows mult(T)^{-1/2} G_T of the closure elements embedded in
    Omega (eq. Wmatrix-def), so that H^T H = A~_Omega."""
    pos = {int(d): a for a, d in enumerate(omega_dofs)}
    rows = []
    for e in cl_elems:
        F = factors[e]
        R = np.zeros((F.shape[0], len(omega_dofs)))
        idx = np.array([pos.get(int(d), -1) for d in elem_dofs[e]])
        ok = idx >= 0
        R[:, idx[ok]] = F[:, ok] / np.sqrt(mult[e])
        rows.append(R)
    return np.vstack(rows) if rows else np.zeros((0, len(omega_dofs)))


def local_spectral(S: np.ndarray, Aww: np.ndarray):
    """Solve S~ u = mu A_ww u (reading R5 of eq. gep_reduced, mu = 1/lambda).

    Returns mu ascending (negative round-off clamped to 0), the eigenvectors V of
    C = L^{-1} S~ L^{-T} and the Cholesky factor L of A_ww.
    """
    L = np.linalg.cholesky(Aww)
    X = sla.solve_triangular(L, S, lower=True)
    C = sla.solve_triangular(L, X.T, lower=True).T
    C = 0.5 * (C + C.T)
    mu, V = np.linalg.eigh(C)
    return np.maximum(mu, 0.0), V, L


def select_modes(mu: np.ndarray, params: Params, tau_cut: float) -> int:
    """Number of retained modes (eq. tau-cut and the retained-mode rule of Sec. 2).

    Keep lambda = 1/mu above tau_cut (mu < 1/tau_cut, a mode within band_tol of the
    cut counts as kept) including the infinite ones (mu = 0); with modes_fixed the
    smallest modes_fixed mu are kept.  A cluster cut at its edge is completed
    (gap <= cluster_tol), readings R7/R8.
    """
    nw = len(mu)
    if params.modes_fixed > 0:
        k = min(params.modes_fixed, nw)
    else:
        k = int(np.count_nonzero(mu < 1.0 / tau_cut + params.band_tol))
    while 0 < k < nw and mu[k] - mu[k - 1] <= params.cluster_tol:
        k += 1
    return k


# ----------------------------------------------------------------- colouring (reading R11)

def coloring(omegas, elem_dofs, n: int) -> np.ndarray:
    """Greedy colouring; i and k conflict iff some element meets both Omega_i and Omega_k."""
    subs_of_dof = [[] for _ in range(n)]
    for i, O in enumerate(omegas):
        for d in O:
            subs_of_dof[d].append(i)
    nb = [set() for _ in omegas]
    for S in elem_dofs:
        s = set()
        for d in S:
            s.update(subs_of_dof[d])
        for i in s:
            nb[i].update(s)
    colors = np.full(len(omegas), -1, dtype=np.int64)
    for i in range(len(omegas)):
        used = {colors[k] for k in nb[i] if colors[k] >= 0 and k != i}
        c = 0
        while c in used:
            c += 1
        colors[i] = c
    return colors


# ----------------------------------------------------------------- setup

def setup(prob, params: Params | None = None) -> Hierarchy:
    """Build the LS-AMG-DD hierarchy from element blocks and their cover."""
    params = params or Params()
    nE = len(prob.elem_ptr) - 1
    elem_dofs = [np.asarray(prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]], dtype=np.int64)
                 for e in range(nE)]
    offs = np.concatenate([[0], np.cumsum(np.diff(prob.elem_ptr) ** 2)])
    blocks = [np.asarray(prob.blocks[offs[e]:offs[e + 1]]).reshape(len(elem_dofs[e]), -1) for e in range(nE)]
    if params.elem_factor not in ("eig", "chol"):
        raise ValueError("elem_factor must be 'eig' or 'chol'")
    factor = element_gram_factor if params.elem_factor == "eig" else element_gram_factor_pchol
    G0 = [factor(B, params.rank_rtol, params.spsd_tol) for B in blocks]
    lev = Level(n=prob.n, level=0, elem_dofs=elem_dofs, blocks=blocks, node_of_dof=np.asarray(prob.node_of_dof, np.int64),
                gram=G0)
    levels = []
    agg_given = None if prob.agg_of_dof is None else np.asarray(prob.agg_of_dof, np.int64)
    while True:
        lev.A = assemble(lev.n, lev.elem_dofs, lev.blocks) if not levels else lev.A
        lev.nnz = structural_pattern(lev.n, lev.elem_dofs).nnz
        density = lev.nnz / float(lev.n) ** 2
        last = (len(levels) + 1 >= params.max_levels or lev.n < params.min_coarse
                or density > params.max_density)
        if not last:
            coarse = coarsen(lev, params, agg_given if not levels else None)
            if coarse is None:
                last = True
        if last:
            lev.coarsest_chol = sla.cho_factor(lev.A.toarray(), lower=True)
            levels.append(lev)
            break
        levels.append(lev)
        lev = coarse
    return Hierarchy(levels=levels, params=params, G0=G0)


def coarsen(lev: Level, params: Params, agg_of_dof=None):
    """Aggregates, overlaps, local problems, P and the Galerkin coarse level."""
    n = lev.n
    if agg_of_dof is None:
        n_super = int(lev.node_of_dof.max()) + 1
        adj = supernode_graph(n_super, lev.node_of_dof, lev.elem_dofs)
        passes = params.agg_passes if lev.level == 0 else params.agg_passes_coarse
        agg_super = aggregate_supernodes(adj, passes)
        agg_of_dof = agg_super[lev.node_of_dof]
    n_agg = int(agg_of_dof.max()) + 1
    aggs, omegas, cl, mult = closures(n_agg, agg_of_dof, lev.elem_dofs)
    lev.agg_of_dof, lev.aggs, lev.omegas, lev.closure, lev.mult = agg_of_dof, aggs, omegas, cl, mult
    lev.tau_cut = params.tau_const * float(mult.max())
    if params.closure == "A":
        # A-closure overlaps (subsets of the G-row closures, since the pattern of A
        # is the union of the element supports); the local matrix of each is the
        # principal submatrix of the G-row closure's A~_Omega on them, i.e. the rows
        # touching omega_i cut down to the A-closure (reading R14)
        omegas_g = omegas
        omegas = [a_closure(lev.A, aggs[i], params.closure_tol) for i in range(n_agg)]
        assert all(np.isin(a, g).all() for a, g in zip(omegas, omegas_g))
        lev.omegas = omegas
    elif params.closure != "G":
        raise ValueError("closure must be 'G' or 'A'")
    factors = None
    if params.interface == "projector":
        # Gram rows per element: the level-0 factors, and above them range factors of
        # the grouped coarse blocks (SPSD up to the rounding of the Galerkin products)
        factors = lev.gram if lev.gram is not None else \
            [element_gram_factor(B, params.rank_rtol, np.inf) for B in lev.blocks]
    lev.mu, lev.Z, ks = [], [], []
    for i in range(n_agg):
        O = omegas[i]
        nw = len(aggs[i])
        if params.closure == "A":
            At = local_splitting(omegas_g[i], cl[i], lev.elem_dofs, lev.blocks, mult)
            keep = np.isin(omegas_g[i], O)
            At = At[np.ix_(keep, keep)]
        else:
            At = local_splitting(O, cl[i], lev.elem_dofs, lev.blocks, mult)
        if params.interface == "projector":
            H = local_gram_rows(omegas_g[i] if params.closure == "A" else O, cl[i], lev.elem_dofs, factors, mult)
            if params.closure == "A":
                H = H[:, np.isin(omegas_g[i], O)]
            S = schur_projector(H, nw)
        elif params.interface == "pinv":
            S = schur_pinv(At, nw)
        else:
            raise ValueError("interface must be 'pinv' or 'projector'")
        Aww = lev.A[aggs[i]][:, aggs[i]].toarray()
        mu, V, L = local_spectral(S, Aww)
        k = select_modes(mu, params, lev.tau_cut)
        lev.mu.append(mu)
        lev.Z.append(sla.solve_triangular(L.T, V[:, :k], lower=False))
        ks.append(k)
    lev.k = np.array(ks, dtype=np.int64)
    lev.coarse_off = np.concatenate([[0], np.cumsum(lev.k)])
    nc = int(lev.coarse_off[-1])
    if nc == 0:
        return None
    rows, cols, vals = [], [], []
    for i in range(n_agg):
        k = lev.k[i]
        if k == 0:
            continue
        rows.append(np.repeat(aggs[i], k))
        cols.append(np.tile(np.arange(lev.coarse_off[i], lev.coarse_off[i] + k), len(aggs[i])))
        vals.append(lev.Z[i].ravel())
    lev.P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, nc))
    # smoother data
    if params.smoother not in ("ms", "ras", "bj"):
        raise ValueError("smoother must be 'ms', 'ras' or 'bj'")
    if params.smoother == "bj":
        lev.colors = np.zeros(n_agg, dtype=np.int64)          # disjoint blocks: one class
        lev.chol = [sla.cho_factor(lev.A[w][:, w].toarray(), lower=True) for w in aggs]
    else:
        lev.colors = coloring(omegas, lev.elem_dofs, n)
        lev.chol = [sla.cho_factor(lev.A[O][:, O].toarray(), lower=True) for O in omegas]
    lev.order = np.lexsort((np.arange(n_agg), lev.colors))
    lev.smoother = params.smoother
    # coarse level (Sec. 2, Galerkin recursion; Remark "finer-scale Grams induce
    # coarser-scale Grams"): the rows of element T give G_T P_T with structural
    # support on the coarse DOFs of the aggregates T touches.  Elements touching
    # the same aggregate set share that support and that multiplicity, so their
    # coarse blocks are summed into one coarse element (reading R12: exact, the
    # splitting and A_c are unchanged).
    sup_of_agg = np.cumsum(lev.k > 0) - 1
    groups = {}
    Pd = lev.P.tocsc()
    for e, S in enumerate(lev.elem_dofs):
        t = np.unique(agg_of_dof[S])
        t = t[lev.k[t] > 0]
        if len(t) == 0:
            continue
        key = tuple(int(i) for i in t)
        Sc = np.concatenate([np.arange(lev.coarse_off[i], lev.coarse_off[i + 1]) for i in t])
        Pe = Pd[S][:, Sc].toarray()
        Ac = Pe.T @ lev.blocks[e] @ Pe
        if key in groups:
            groups[key][1] += Ac
        else:
            groups[key] = [Sc, Ac]
    c_elem_dofs = [g[0] for g in groups.values()]
    c_blocks = [0.5 * (g[1] + g[1].T) for g in groups.values()]
    node_c = np.repeat(sup_of_agg[lev.k > 0], lev.k[lev.k > 0])
    coarse = Level(n=nc, level=lev.level + 1, elem_dofs=c_elem_dofs, blocks=c_blocks, node_of_dof=node_c)
    coarse.A = (lev.P.T @ lev.A @ lev.P).tocsr()
    coarse.A.sort_indices()
    return coarse


# ----------------------------------------------------------------- coarse Gram rows (Remark "coarse_gram")

def coarse_gram_factors(lev: Level, rank_rtol: float = 0.0):
    """Gram factors of the grouped coarse element blocks of a coarse level: the
    rows G_g with G_g^T G_g = A_g for every coarse element g (elements of the finer
    level summed over the set of aggregates they touch, reading R12), from the
    pivoted Cholesky factorization of Sec. 5.2 truncated at n_g eps max diag.

    Remark "finer-scale Grams induce coarser-scale Grams" (Sec. 5.1): a sum of SPSD
    element blocks is SPSD and has a Gram factor, so the literal coarse factor
    G_c = G P (one row per fine row) may be replaced by these re-factored rows,
    which number rank(A_g) per group.  The coarse operator is unchanged up to the
    truncation, A_c = sum_g R_g^T G_g^T G_g R_g.  The blocks are SPSD only up to
    the rounding of the Galerkin products, so no SPSD test is applied."""
    return [element_gram_factor_pchol(B, rank_rtol, np.inf) for B in lev.blocks]


# ----------------------------------------------------------------- cycle and outer iteration

def smooth(lev: Level, x: np.ndarray, r: np.ndarray, order) -> None:
    """One multiplicative Schwarz sweep over the overlaps in `order` (exact local solves)."""
    for i in order:
        O = lev.omegas[i]
        res = r[O] - lev.A[O] @ x
        x[O] += sla.cho_solve(lev.chol[i], res)


def smooth_additive(lev: Level, x: np.ndarray, r: np.ndarray, post: bool) -> None:
    """One additive step x += M^{-1} (r - A x) (post: M^{-T}).

    Block Jacobi: M^{-1} = sum_i R_w^T A_ww^{-1} R_w (symmetric).  RAS:
    M^{-1} = sum_i R_Omega^T D_i A_Omega^{-1} R_Omega with D_i the 0/1 diagonal of
    omega_i inside Omega_i (corrections kept on the aggregate, a partition of
    unity); its transpose M^{-T} = sum_i R_Omega^T A_Omega^{-1} D_i R_Omega solves
    with the residual restricted to the aggregate and keeps the whole correction."""
    res = r - lev.A @ x
    dx = np.zeros_like(x)
    for i, w in enumerate(lev.aggs):
        if lev.smoother == "bj":
            dx[w] += sla.cho_solve(lev.chol[i], res[w])
            continue
        O = lev.omegas[i]
        nw = len(w)
        if not post:
            dx[O[:nw]] += sla.cho_solve(lev.chol[i], res[O])[:nw]
        else:
            rr = np.zeros(len(O))
            rr[:nw] = res[O[:nw]]
            dx[O] += sla.cho_solve(lev.chol[i], rr)
    x += dx


def vcycle(h: Hierarchy, r: np.ndarray, l: int = 0) -> np.ndarray:
    """Symmetric V-cycle: pre-smoother M^{-1}, coarse correction, post-smoother M^{-T}
    (Sec. 2); for multiplicative Schwarz the post-sweep runs the overlaps in reverse
    order (Sec. 6)."""
    lev = h.levels[l]
    if l == len(h.levels) - 1:
        return sla.cho_solve(lev.coarsest_chol, r)
    x = np.zeros_like(r)
    if lev.smoother == "ms":
        smooth(lev, x, r, lev.order)
    else:
        smooth_additive(lev, x, r, post=False)
    t = r - lev.A @ x
    e = vcycle(h, lev.P.T @ t, l + 1)
    x += lev.P @ e
    if lev.smoother == "ms":
        smooth(lev, x, r, lev.order[::-1])
    else:
        smooth_additive(lev, x, r, post=True)
    return x


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    rel_res: float
    history: list


def pcg(h: Hierarchy, b: np.ndarray, rtol: float | None = None, max_iter: int | None = None, x0=None):
    """Preconditioned CG (Hestenes-Stiefel) with the V-cycle; iterations = A-applies."""
    rtol = h.params.rtol if rtol is None else rtol
    max_iter = h.params.max_iter if max_iter is None else max_iter
    A = h.levels[0].A
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn if bn > 0 else 0.0]
    if bn == 0.0:
        return x, SolveInfo(0, True, 0.0, hist)
    z = vcycle(h, r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0:
            raise FloatingPointError("PCG breakdown: p^T A p <= 0")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        hist.append(rel)
        if rel <= rtol:
            return x, SolveInfo(it, True, rel, hist)
        z = vcycle(h, r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, SolveInfo(max_iter, False, hist[-1], hist)


def stationary(h: Hierarchy, b: np.ndarray, x0: np.ndarray, reduction: float = 1e-10, max_iter: int = 500):
    """Standalone V-cycle iteration x <- x + V(b - A x) (the paper's solver mode, Sec. 6)."""
    A = h.levels[0].A
    x = x0.copy()
    r = b - A @ x
    r0 = np.linalg.norm(r)
    hist = [1.0]
    for it in range(1, max_iter + 1):
        x += vcycle(h, r)
        r = b - A @ x
        hist.append(np.linalg.norm(r) / r0)
        if hist[-1] <= reduction:
            return x, SolveInfo(it, True, hist[-1], hist)
    return x, SolveInfo(max_iter, False, hist[-1], hist)


def hierarchy_stats(h: Hierarchy):
    """Level sizes, operator complexity sum nnz(A_l)/nnz(A_0), grid complexity sum n_l / n_0."""
    n = [lv.n for lv in h.levels]
    nnz = [lv.nnz for lv in h.levels]
    return dict(n=n, nnz=nnz, oc=sum(nnz) / nnz[0], gc=sum(n) / n[0])
