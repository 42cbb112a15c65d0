"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
formula: they use an independent route (brute force, a different factorisation,
a theorem's other side, a hand-derived count) so that a dropped term, a wrong
index or a transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import fegen
import oracle
from oracle import lsdd as O


def _elem_lists(prob):
    nE = prob.n_elem
    dofs = [prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]].astype(np.int64) for e in range(nE)]
    blocks = [prob.element(e)[1] for e in range(nE)]
    return dofs, blocks


def _dense_G(prob, G0):
    """Stack G_T R_T (Prop. elementwise Gram formulation) as a dense m x n matrix."""
    dofs, _ = _elem_lists(prob)
    rows = []
    for S, Ge in zip(dofs, G0):
        R = np.zeros((Ge.shape[0], prob.n))
        R[:, S] = Ge
        rows.append(R)
    return np.vstack(rows)


# ------------------------------------------------------------ Sec. 5.1 / 5.2: element Gram factors

def test_gram_factor_reproduces_blocks_and_ranks():
    prob = fegen.elasticity_q1(4, nu=0.3)
    for e in range(prob.n_elem):
        _, Ae = prob.element(e)
        Ge = oracle.element_gram_factor(Ae)
        assert np.abs(Ge.T @ Ge - Ae).max() <= 1e-13 * np.abs(Ae).max()
        # interior Q1 elasticity block: 8 DOFs minus 3 rigid-body modes (2D)
        expect = 8 if e % 4 == 0 else 5
        assert Ge.shape[0] == expect


def test_gram_factor_rejects_indefinite_block():
    A = np.diag([1.0, 2.0, -0.5])
    with pytest.raises(oracle.NotSPSD):
        oracle.element_gram_factor(A)


def test_global_gram_identity_and_energy():
    """A = G^T G and u^T A u = sum_T ||G_T R_T u||^2 (eq. conforming_global_gram)."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=1))
    G = _dense_G(prob, h.G0)
    A = h.levels[0].A.toarray()
    assert np.abs(G.T @ G - A).max() <= 1e-13 * np.abs(A).max()
    u = np.random.default_rng(1).standard_normal(prob.n)
    assert abs(u @ A @ u - np.sum((G @ u) ** 2)) <= 1e-12 * abs(u @ A @ u)
    # rows of the stacked G: 4 x 6 boundary elements of rank 8, the rest rank 5
    assert G.shape[0] == 6 * 8 + 30 * 5


def test_gram_invariance_under_orthogonal_mixing():
    """(U G_T)^T (U G_T) = A_T leaves P and A_c unchanged (Sec. 5.2)."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    dofs, blocks = _elem_lists(prob)
    rng = np.random.default_rng(3)
    mixed = []
    for B in blocks:
        Ge = oracle.element_gram_factor(B)
        U, _ = np.linalg.qr(rng.standard_normal((Ge.shape[0], Ge.shape[0])))
        Gm = U @ Ge
        mixed.append(Gm.T @ Gm)
    prob2 = fegen.common.Problem(prob.n, prob.elem_ptr, prob.elem_dofs,
                                 np.concatenate([m.ravel() for m in mixed]), prob.node_of_dof, prob.agg_of_dof)
    p = oracle.Params(max_levels=2, modes_fixed=4)
    h1, h2 = oracle.setup(prob, p), oracle.setup(prob2, p)
    P1, P2 = h1.levels[0].P.toarray(), h2.levels[0].P.toarray()
    A = h1.levels[0].A
    # the retained subspaces agree aggregate by aggregate: compare projectors
    for i, w in enumerate(h1.levels[0].aggs):
        Z1, Z2 = h1.levels[0].Z[i], h2.levels[0].Z[i]
        Aww = A[w][:, w].toarray()
        Pr1 = Z1 @ Z1.T @ Aww
        Pr2 = Z2 @ Z2.T @ Aww
        assert np.abs(Pr1 - Pr2).max() <= 1e-9
    assert P1.shape == P2.shape


# ------------------------------------------------------------ Sec. 2: aggregation, closures, splitting

def test_vertex_patch_structure_small_elasticity(small_elasticity):
    """Hand-derived counts for 3x3-node patches on the 33x33-node grid."""
    prob, _, h = small_elasticity
    lv = h.levels[0]
    assert prob.n == 2178 and len(lv.aggs) == 121
    assert all(len(a) == 18 for a in lv.aggs)
    sizes, counts = np.unique([len(o) for o in lv.omegas], return_counts=True)
    assert dict(zip(sizes.tolist(), counts.tolist())) == {32: 4, 40: 36, 50: 81}
    assert np.bincount(lv.mult).tolist() == [0, 484, 440, 0, 100]
    # conflict graph of the patches is the king graph of an 11x11 grid -> 4 colours
    assert lv.colors.max() + 1 == 4
    ij = np.array([(i % 11, i // 11) for i in range(121)])
    for a in range(121):
        for b in range(a + 1, 121):
            if np.abs(ij[a] - ij[b]).max() <= 1:
                assert lv.colors[a] != lv.colors[b]


def test_standard_aggregation_is_a_partition_of_connected_sets():
    prob = fegen.graddiv_rtcf3(6)
    dofs, _ = _elem_lists(prob)
    nsup = int(prob.node_of_dof.max()) + 1
    adj = O.supernode_graph(nsup, prob.node_of_dof.astype(np.int64), dofs)
    agg = O.standard_aggregation(adj)
    assert agg.min() == 0 and np.all(agg >= 0)
    na = agg.max() + 1
    for a in range(na):
        members = np.flatnonzero(agg == a)
        sub = adj[members][:, members]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1
    # every phase-1 root aggregate contains the root's whole neighbourhood: the
    # first node (index 0) is always a root
    nb0 = adj.indices[adj.indptr[0]:adj.indptr[1]]
    assert np.all(agg[nb0] == agg[0])


def test_g_row_closure_equals_element_closure_bruteforce():
    """Thm. elem_closure: with a full-support row per element the G-row closure
    (Def. G_row_closure, computed from the numerical support of a dense G) equals
    the element closure used by the oracle."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    G = _dense_G(prob, h.G0)
    lv = h.levels[0]
    for i, w in enumerate(lv.aggs):
        rows = np.flatnonzero(np.any(G[:, w] != 0, axis=1))
        closure = np.flatnonzero(np.any(G[rows] != 0, axis=0))
        assert set(closure.tolist()) == set(lv.omegas[i].tolist())
        assert list(lv.omegas[i][:len(w)]) == list(w)
    # multiplicity per row = number of aggregates the row touches (eq. row_multiplicity)
    agg = lv.agg_of_dof
    mult_rows = np.array([len(np.unique(agg[np.flatnonzero(g != 0)])) for g in G])
    assert mult_rows.max() == 4 and mult_rows.min() == 1


def _check_splitting(lv, A):
    acc = np.zeros(A.shape)
    for i, O_ in enumerate(lv.omegas):
        At = O.local_splitting(O_, lv.closure[i], lv.elem_dofs, lv.blocks, lv.mult)
        assert np.linalg.eigvalsh(At).min() >= -1e-12 * np.abs(At).max()
        acc[np.ix_(O_, O_)] += At
    Ad = A.toarray()
    return np.abs(acc - Ad).max() / np.abs(Ad).max()


def test_exact_spsd_splitting_levels_0_and_1():
    """sum_i R_Omega^T A~_Omega R_Omega = A (eq. SPSD_splitting), also on the Galerkin level."""
    prob = fegen.graddiv_rtcf3(6, kappa=np.exp(np.random.default_rng(0).standard_normal(36)), beta=1.0)
    h = oracle.setup(prob, oracle.Params(max_levels=3, agg_passes=1, max_density=1.0))
    assert len(h.levels) == 3
    assert _check_splitting(h.levels[0], h.levels[0].A) <= 1e-13
    assert _check_splitting(h.levels[1], h.levels[1].A) <= 1e-12


def test_splitting_pin_catches_a_planted_multiplicity_error(monkeypatch):
    """Plant a mistake (multiplicity weight dropped) in the oracle; the pin must fail."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    lv = h.levels[0]
    real = O.local_splitting
    monkeypatch.setattr(O, "local_splitting", lambda o, c, d, b, m: real(o, c, d, b, np.ones_like(m)))
    assert _check_splitting(lv, lv.A) > 1e-3


# ------------------------------------------------------------ Sec. 2: local spectral problems

def _schur_by_projection(lv, i, G0_rows):
    """S~ = H_w^T (I - Pi_range(H_G)) H_w with H = W^{1/2} G(R_w, Omega) (eq. Wmatrix-def)."""
    O_ = lv.omegas[i]
    nw = len(lv.aggs[i])
    H = []
    for e in lv.closure[i]:
        pos = {int(d): a for a, d in enumerate(O_)}
        Ge = G0_rows[e]
        Hr = np.zeros((Ge.shape[0], len(O_)))
        Hr[:, [pos[int(d)] for d in lv.elem_dofs[e]]] = Ge / np.sqrt(lv.mult[e])
        H.append(Hr)
    H = np.vstack(H)
    Hw, Hg = H[:, :nw], H[:, nw:]
    Q, R, _ = sla.qr(Hg, mode="economic", pivoting=True)
    rank = int(np.sum(np.abs(np.diag(R)) > 1e-12 * np.abs(R[0, 0])))
    Q = Q[:, :rank]
    Y = Hw - Q @ (Q.T @ Hw)
    return Y.T @ Y


def test_schur_complement_matches_projection_route():
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    lv = h.levels[0]
    for i in range(len(lv.aggs)):
        At = O.local_splitting(lv.omegas[i], lv.closure[i], lv.elem_dofs, lv.blocks, lv.mult)
        S = O.schur_pinv(At, len(lv.aggs[i]))
        S2 = _schur_by_projection(lv, i, h.G0)
        assert np.abs(S - S2).max() <= 1e-10 * np.abs(At).max()
        H = O.local_gram_rows(lv.omegas[i], lv.closure[i], lv.elem_dofs, h.G0, lv.mult)
        assert np.abs(H.T @ H - At).max() <= 1e-13 * np.abs(At).max()
        assert np.abs(O.schur_projector(H, len(lv.aggs[i])) - S2).max() <= 1e-10 * np.abs(At).max()


def test_schur_pinv_on_singular_interface_block():
    """Moore-Penrose branch: a rank-deficient A~_GG still gives the minimum-energy Schur complement."""
    rng = np.random.default_rng(5)
    H = rng.standard_normal((6, 7))
    H[:, 5] = H[:, 6]                      # two identical interface columns -> A~_GG singular
    At = H.T @ H
    S = O.schur_pinv(At, 3)
    Q, _ = np.linalg.qr(H[:, 3:][:, :3])   # range of H_G spanned by its first 3 columns (w.p. 1)
    Y = H[:, :3] - Q @ (Q.T @ H[:, :3])
    assert np.abs(S - Y.T @ Y).max() <= 1e-10 * np.abs(At).max()


def test_local_spectrum_bounds_and_rigid_modes(small_elasticity):
    """mu in [0,1] (S~ <= A~_ww <= A_ww) and 3 zero modes (rigid motions) on interior patches."""
    _, _, h = small_elasticity
    lv = h.levels[0]
    for i, mu in enumerate(lv.mu):
        assert mu.min() >= 0.0 and mu.max() <= 1.0 + 1e-12
        if len(lv.omegas[i]) == 50:          # interior patch
            assert np.sum(mu < 1e-12) == 3 and mu[3] > 1e-3


def test_single_aggregate_reduces_to_direct_solve():
    """One aggregate: Omega = omega, mult = 1, S~ = A, all mu = 1; keeping them makes P
    square and the two-level preconditioner exact, so PCG stops after one step."""
    prob = fegen.elasticity_q1(3, nu=0.3, vertex_patches=False)
    prob.agg_of_dof = np.zeros(prob.n, dtype=np.int32)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=10 ** 6, min_coarse=1, max_density=2.0))
    lv = h.levels[0]
    assert np.allclose(lv.mu[0], 1.0, atol=1e-12)
    assert lv.P.shape == (prob.n, prob.n)
    b = np.random.default_rng(0).standard_normal(prob.n)
    x, info = oracle.pcg(h, b, rtol=1e-12)
    assert info.iters == 1


def test_interpolation_normalisation_and_galerkin_identity(small_elasticity):
    """Z_i^T A_ww Z_i = I (reading R9) and P^T A P equals the assembled coarse element
    blocks sum_T (G_T P_T)^T (G_T P_T) (Galerkin Gram recursion, Sec. 2)."""
    _, _, h = small_elasticity
    l0, l1 = h.levels
    A = l0.A
    for i, w in enumerate(l0.aggs):
        Z = l0.Z[i]
        assert np.abs(Z.T @ A[w][:, w].toarray() @ Z - np.eye(Z.shape[1])).max() <= 1e-10
    # coarse blocks rebuilt from the Gram factors, summed per group of elements
    P = l0.P.toarray()
    Ac = np.zeros((l1.n, l1.n))
    dofs = l0.elem_dofs
    for e, Ge in enumerate(h.G0):
        GP = Ge @ P[dofs[e]]
        Ac += GP.T @ GP
    assert np.abs(Ac - l1.A.toarray()).max() <= 1e-12 * np.abs(Ac).max()
    Ag = O.assemble(l1.n, l1.elem_dofs, l1.blocks).toarray()
    assert np.abs(Ag - Ac).max() <= 1e-12 * np.abs(Ac).max()


# ------------------------------------------------------------ cycle, PCG, two-level theory

def _vcycle_matrix(h):
    n = h.levels[0].n
    return np.column_stack([oracle.vcycle(h, np.eye(n)[:, j]) for j in range(n)])


def test_vcycle_is_symmetric_positive_definite():
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    B = _vcycle_matrix(h)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


@pytest.mark.parametrize("N", [2, 4, 8])
def test_pcg_matches_dense_solve(N):
    prob = fegen.elasticity_q1(N, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4, min_coarse=1))
    b = np.random.default_rng(N).standard_normal(prob.n)
    x, info = oracle.pcg(h, b, rtol=1e-14)
    xd = np.linalg.solve(h.levels[0].A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


def _smoother_matrices(h):
    """Forward multiplicative Schwarz sweep as a matrix M^{-1} (x = S_f(r) from x0 = 0)."""
    lv = h.levels[0]
    n = lv.n
    Minv = np.zeros((n, n))
    for j in range(n):
        x = np.zeros(n)
        O.smooth(lv, x, np.eye(n)[:, j], lv.order)
        Minv[:, j] = x
    return Minv


def test_two_level_theory_identity_and_bound():
    """||E_TG||_A = 1 - 1/K_TG with K_TG measured in the symmetrised-smoother norm
    (sharp two-level theory), and K_TG <= lambda_max(M_wJ^{-1} M~) tau_max, with
    M_wJ the aggregate block Jacobi and tau_max the largest discarded lambda."""
    prob = fegen.elasticity_q1(6, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    lv = h.levels[0]
    A = lv.A.toarray()
    n = lv.n
    B = _vcycle_matrix(h)
    E = np.eye(n) - B @ A
    Ah = sla.sqrtm(A).real
    normE = np.linalg.norm(Ah @ E @ np.linalg.inv(Ah), 2)
    Minv = _smoother_matrices(h)
    # M~ = M^T (M^T + M - A)^{-1} M, i.e. I - M~^{-1} A = (I - M^{-1} A)(I - M^{-T} A)
    Mt_inv = Minv + Minv.T - Minv @ A @ Minv.T
    Mt = np.linalg.inv(Mt_inv)
    Mt = 0.5 * (Mt + Mt.T)
    P = lv.P.toarray()
    Pi = P @ np.linalg.solve(P.T @ Mt @ P, P.T @ Mt)
    X = np.eye(n) - Pi
    K = sla.eigh(X.T @ Mt @ X, A, eigvals_only=True).max()
    assert abs(normE - (1.0 - 1.0 / K)) <= 1e-8
    MwJ = np.zeros((n, n))
    for w in lv.aggs:
        MwJ[np.ix_(w, w)] = A[np.ix_(w, w)]
    lam_tr = sla.eigh(Mt, MwJ, eigvals_only=True).max()
    tau_max = max(1.0 / mu[k] for mu, k in zip(lv.mu, lv.k) if k < len(mu))
    assert K <= lam_tr * tau_max * (1 + 1e-10)
    assert normE < 1.0


def test_threshold_selection_and_cluster_rule():
    """Keep mu < 1/tau_cut (band_tol), complete a cluster cut at its edge (R7/R8)."""
    p = oracle.Params(tau_const=0.75)
    mu = np.array([0.0, 0.0, 0.1, 0.5, 0.5 + 5e-10, 0.9])
    assert O.select_modes(mu, p, tau_cut=5.0) == 3          # cut at 0.2
    assert O.select_modes(mu, p, tau_cut=2.0) == 5          # cut at 0.5: the band keeps both 0.5 modes
    mu2 = np.array([0.0, 0.5 + 0.5e-9, 0.5 + 1.2e-9, 0.9])
    assert O.select_modes(mu2, p, tau_cut=2.0) == 3         # 3rd mode joins its cluster
    pf = oracle.Params(modes_fixed=4)
    assert O.select_modes(mu, pf, tau_cut=1.0) == 5         # 4th and 5th form a cluster


def test_stationary_cycle_converges():
    prob = fegen.elasticity_q1(8, nu=0.3)
    h = oracle.setup(prob, oracle.Params(max_levels=2, modes_fixed=4))
    b = np.zeros(prob.n)
    x0 = np.random.default_rng(0).standard_normal(prob.n)
    x, info = oracle.stationary(h, b, x0, reduction=1e-10)
    assert info.converged and info.iters < 40


def test_interface_routes_agree_on_singular_blocks_with_a_gap():
    """The pseudo-inverse route (eigendecomposition of A~_GG, reading R4) and the projector
    route on the weighted Gram rows give the same Schur complement on a singular interface
    block, equal to the minimum energy over interface extensions; moving one interface
    column out of the range changes it (Sec. 2, eq. gep_reduced)."""
    rng = np.random.default_rng(5)
    nw, ng, r = 6, 9, 5
    H = rng.standard_normal((12, nw + ng))
    H[:, nw:] = rng.standard_normal((12, r)) @ rng.standard_normal((r, ng))   # rank-r interface columns
    At = H.T @ H
    S1 = oracle.schur_pinv(At, nw)
    S2 = oracle.lsdd.schur_projector(H, nw)
    assert np.abs(S1 - S2).max() <= 1e-10 * np.abs(S1).max()
    # minimum-energy characterisation: S~ = min over interface extensions of the energy
    for _ in range(3):
        v = rng.standard_normal(nw)
        ext = -np.linalg.lstsq(H[:, nw:], H[:, :nw] @ v, rcond=None)[0]
        full = np.concatenate([v, ext])
        assert abs(v @ S1 @ v - full @ At @ full) <= 1e-9 * abs(v @ S1 @ v)
    Hc = H.copy()
    Hc[:, nw] = rng.standard_normal(12)                  # an interface column leaving the range: different S~
    assert np.abs(oracle.lsdd.schur_projector(Hc, nw) - S2).max() > 1e-3 * np.abs(S2).max()


def test_schur_complement_does_not_depend_on_the_generalized_inverse():
    """For a PSD A~_Omega the coupling A~_Gw lies in the range of A~_GG, so every generalized
    inverse gives the Moore-Penrose Schur complement; here one from eliminating a maximal
    set of pivots with the largest remaining diagonal (a truncated pivoted Cholesky) on a
    block with a 3-dimensional null space."""
    rng = np.random.default_rng(11)
    nw, ng = 5, 10
    H = rng.standard_normal((14, nw + ng))
    H[:, nw + 7:] = H[:, nw:nw + 3] @ rng.standard_normal((3, 3))   # 3 dependent interface columns
    At = H.T @ H
    M = At[nw:, nw:].copy()
    tol = ng * np.finfo(float).eps * M.diagonal().max()
    live = np.ones(ng, bool)
    piv = []
    while live.any():
        idx = np.flatnonzero(live)
        j = idx[np.argmax(M[idx, idx])]
        if not M[j, j] > tol:
            break
        c = np.where(live, M[:, j], 0.0) / np.sqrt(M[j, j])
        M -= np.outer(c, c)
        live[j] = False
        piv.append(j)
    assert len(piv) == ng - 3
    P = nw + np.array(piv)
    S_elim = At[:nw, :nw] - At[:nw, P] @ np.linalg.solve(At[np.ix_(P, P)], At[P, :nw])
    assert np.abs(S_elim - oracle.schur_pinv(At, nw)).max() <= 1e-9 * np.abs(At).max()
