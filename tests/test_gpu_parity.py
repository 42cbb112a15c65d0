"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances: FP64 solutions and preconditioner outputs 1e-10 relative, the
assembled operators 1e-13, canonicalised coarse operators 1e-10, PCG iteration
counts +-1; integer outputs (aggregates, colours, retained-mode counts, ranks)
bit-exact.  The FP32 cycle is held to an A-norm error of 1e-8 against a
reference solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import fegen
import oracle
from canon import _canon, _csr, _gpu_Z_blocks
from route_spread import mu_tol, oracle_routes, rel, tol_from

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lsdd():
    import paper_2607_07485_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch.device("cuda:0")


def _setup_both(prob, params_kw):
    P = _lsdd()
    h_or = oracle.setup(prob, oracle.Params(**params_kw))
    h_gpu = P.Hierarchy.setup_problem(prob, P.Params.default(**params_kw))
    return h_or, h_gpu


ELAST_KW = dict(max_levels=2, modes_fixed=4)


def test_small_elasticity_setup_parity(dev):
    prob, _ = fegen.elasticity_small(N=32)
    h_or, h = _setup_both(prob, ELAST_KW)
    try:
        # element Gram factors: ranks bit-exact, G^T G = A_T
        ranks, G = h.export_gram(prob.elem_ptr)
        assert ranks.tolist() == [g.shape[0] for g in h_or.G0]
        offs = prob.block_offsets()
        for e in range(0, prob.n_elem, 37):
            ne = 8
            Ge = G[offs[e]:offs[e + 1]].reshape(ne, ne)[:ranks[e]]
            _, Ae = prob.element(e)
            assert np.abs(Ge.T @ Ge - Ae).max() <= 1e-13 * np.abs(Ae).max()
        info = h.info()
        assert info["levels"] == 2 and info["n"] == [2178, 484]
        l0 = h.export_level(0)
        lv = h_or.levels[0]
        A_or = lv.A
        A_gpu = _csr(l0)
        assert np.abs((A_gpu - A_or)).max() <= 1e-13 * np.abs(A_or).max()
        # integer structure: bit-exact
        assert np.array_equal(l0["agg_of_dof"], lv.agg_of_dof)
        assert np.array_equal(l0["colors"], lv.colors)
        assert np.array_equal(l0["k"], lv.k)
        assert np.array_equal(l0["omega_sizes"], [len(o) for o in lv.omegas])
        # local spectra
        mu_or = np.concatenate(lv.mu)
        assert np.abs(l0["mu"] - mu_or).max() <= 1e-10
        # canonicalised Z and coarse operator
        nw = [len(a) for a in lv.aggs]
        Zg = _gpu_Z_blocks(l0, nw)
        Qg, Qo = [], []
        for i in range(len(nw)):
            Qg.append(_canon(Zg[i], lv.mu[i], nw[i]))
            Qo.append(_canon(lv.Z[i], lv.mu[i], nw[i]))
            assert np.abs(Zg[i] @ Qg[i] - lv.Z[i] @ Qo[i]).max() <= 1e-10 * np.abs(lv.Z[i]).max()
        from scipy.linalg import block_diag
        Bg, Bo = block_diag(*Qg), block_diag(*Qo)
        l1 = h.export_level(1)
        Ac_g = Bg.T @ _csr(l1).toarray() @ Bg
        Ac_o = Bo.T @ h_or.levels[1].A.toarray() @ Bo
        assert np.abs(Ac_g - Ac_o).max() <= 1e-10 * np.abs(Ac_o).max()
        # A_ww-orthonormal retained modes: diagonal blocks of A_c are identities
        off = 0
        for k in l0["k"]:
            assert np.abs(Ac_g[off:off + k, off:off + k] - np.eye(k)).max() <= 1e-10
            off += k
    finally:
        h.close()


def test_small_elasticity_vcycle_and_pcg_parity(dev):
    prob, b = fegen.elasticity_small(N=32)
    h_or, h = _setup_both(prob, ELAST_KW)
    try:
        r = np.random.default_rng(7).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert np.linalg.norm(z - z_or) <= 1e-10 * np.linalg.norm(z_or)
        y = h.apply(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert np.linalg.norm(y - h_or.levels[0].A @ r) <= 1e-13 * np.linalg.norm(y)
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        x = x.cpu().numpy()
        assert infos[0].converged == 1
        assert abs(infos[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x - x_or) <= 1e-10 * np.linalg.norm(x_or)
        # the residual is checked with the oracle's assembled operator
        assert np.linalg.norm(b - h_or.levels[0].A @ x) <= 1.0001e-8 * np.linalg.norm(b)
    finally:
        h.close()


def test_small_elasticity_fp32_cycle_accuracy(dev):
    prob, b = fegen.elasticity_small(N=32)
    P = _lsdd()
    A = oracle.assemble(prob.n, *[[prob.element(e)[i] for e in range(prob.n_elem)] for i in (0, 1)])
    x_ref = spla.spsolve(A.tocsc(), b)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(precision=1, rtol=1e-10, **ELAST_KW))
    try:
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        x = x.cpu().numpy()
        e = x - x_ref
        anorm = np.sqrt(e @ (A @ e)) / np.sqrt(x_ref @ (A @ x_ref))
        assert infos[0].converged == 1 and anorm <= 1e-8
    finally:
        h.close()


@pytest.mark.parametrize("N", [2, 5])
def test_tiny_and_ragged_meshes(dev, N):
    """Tiny meshes (one patch, partial last patches) solve to 1e-12 like a dense solve."""
    prob = fegen.elasticity_q1(N, nu=0.3)
    b = np.random.default_rng(N).standard_normal(prob.n)
    P = _lsdd()
    kw = dict(max_levels=2, modes_fixed=4, min_coarse=1, rtol=1e-12)
    h_or = oracle.setup(prob, oracle.Params(**kw))
    h = P.Hierarchy.setup_problem(prob, P.Params.default(**kw))
    try:
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        x_or, inf_or = oracle.pcg(h_or, b, rtol=1e-12)
        assert abs(infos[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
    finally:
        h.close()


def test_graddiv_multilevel_parity(dev):
    """RTCF3 grad-div with standard aggregation and threshold modes, 3 levels."""
    rng = np.random.default_rng(0)
    N = 10
    prob = fegen.graddiv_rtcf3(N, kappa=np.exp(rng.standard_normal(N * N)), beta=1.0)
    b = rng.standard_normal(prob.n)
    kw = dict(max_levels=3, tau_const=0.75, max_density=1.0, agg_passes=1, agg_passes_coarse=1)
    h_or, h = _setup_both(prob, kw)
    try:
        info = h.info()
        assert info["n"] == [lv.n for lv in h_or.levels]
        for l in range(len(h_or.levels) - 1):
            ex = h.export_level(l)
            assert np.array_equal(ex["agg_of_dof"], h_or.levels[l].agg_of_dof)
            assert np.array_equal(ex["k"], h_or.levels[l].k)
        r = rng.standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert np.linalg.norm(z - z_or) <= 1e-10 * np.linalg.norm(z_or)
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert abs(infos[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
    finally:
        h.close()


def test_error_paths_on_device(dev):
    P = _lsdd()
    prob = fegen.elasticity_q1(3, nu=0.3)
    bad = prob.blocks.copy().reshape(-1, 8, 8)
    bad[4] = -bad[4]                               # an indefinite element block
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, bad.ravel(), prob.node_of_dof,
                                   prob.agg_of_dof, P.Params.default(**ELAST_KW))
    assert ei.value.code == 2 and "element 4" in str(ei.value)
    asym = prob.blocks.copy().reshape(-1, 8, 8)
    asym[2, 0, 1] += 1.0
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, asym.ravel(), prob.node_of_dof,
                                   prob.agg_of_dof, P.Params.default(**ELAST_KW))
    assert ei.value.code == 1
    h = P.Hierarchy.setup_problem(prob, P.Params.default(**ELAST_KW))
    try:
        b = torch.zeros(prob.n, dtype=torch.float64, device=dev)
        x, infos = h.solve(b)                      # zero right-hand side: x = 0, no iteration
        assert infos[0].iters == 0 and float(x.abs().max()) == 0.0
        b[3] = float("nan")
        with pytest.raises(P.LsddError) as ei:
            h.solve(b)
        assert ei.value.code == 1
    finally:
        h.close()


def test_size_limits_are_reported(dev):
    """A caller cover with one aggregate of 4,802 DOFs (above the 4,096 the local
    spectral problems take) is refused with LSDD_E_UNSUPPORTED and a message naming
    the limit, before any local problem runs; the same mesh with its vertex-patch
    cover builds."""
    P = _lsdd()
    prob = fegen.elasticity_q1(48, nu=0.3)
    one = np.zeros(prob.n, np.int32)
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, prob.blocks, prob.node_of_dof, one,
                                   P.Params.default(**ELAST_KW))
    assert ei.value.code == 7 and "4096" in str(ei.value)
    with P.Hierarchy.setup_problem(prob, P.Params.default(**ELAST_KW)) as h:
        assert h.info()["levels"] == 2


def test_setup_and_solve_are_bitwise_reproducible(dev):
    """Every reduction has a fixed order: two setups and solves give identical bits."""
    P = _lsdd()
    rng = np.random.default_rng(4)
    N = 10
    prob = fegen.graddiv_rtcf3(N, kappa=np.exp(rng.standard_normal(N * N)), beta=1e-4)
    b = torch.from_numpy(rng.standard_normal(prob.n)).to(dev)
    kw = dict(max_levels=3, tau_const=0.75, max_density=1.0, agg_passes=1, agg_passes_coarse=1)
    xs = []
    for _ in range(2):
        with P.Hierarchy.setup_problem(prob, P.Params.default(**kw)) as h:
            x, _ = h.solve(b)
            z1 = h.vcycle(b)
            z2 = h.vcycle(b)
            assert torch.equal(z1, z2)
            xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("N, passes, eps", [(24, 1, 1e-4), (32, 2, 1.0)])
def test_hyperdiffusion_bfs_parity(dev, N, passes, eps):
    """Bicubic Hermite hyperdiffusion (anisotropic eps = 1e-4 at 30 degrees, and isotropic for
    the two-pass case; Nitsche clamp), threshold modes with tau_cut = max mult: level
    structure bit-exact, V-cycle and PCG solution against the Moore-Penrose oracle within
    ten times the distance between the oracle's two routes to the Schur complement (never
    below 1e-10), iterations +-1.  The interface blocks here are ill-conditioned (condition
    numbers near 1e11 on level 0, singular ones on the coarse levels), and the two FP64
    routes already move the cycle by about 1e-8 (N = 24) and 2e-10 (N = 32)."""
    P = _lsdd()
    prob, b = fegen.hyperdiffusion_h2(N=N, eps=eps)
    kw = dict(max_levels=4, tau_const=1.0, agg_passes=passes, agg_passes_coarse=1)
    h_or, h_pr = oracle_routes(prob, **kw)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(**kw))
    try:
        info = h.info()
        assert info["n"] == [lv.n for lv in h_or.levels]
        for l in range(len(h_or.levels) - 1):
            ex = h.export_level(l)
            assert np.array_equal(ex["agg_of_dof"], h_or.levels[l].agg_of_dof)
            assert np.array_equal(ex["k"], h_or.levels[l].k)
        r = np.random.default_rng(N).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert rel(z, z_or) <= tol_from(z_or, oracle.vcycle(h_pr, r))
        x_or, inf_or = oracle.pcg(h_or, b)
        x_pr, _ = oracle.pcg(h_pr, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert infos[0].converged == 1 and abs(infos[0].iters - inf_or.iters) <= 1
        assert rel(x.cpu().numpy(), x_or) <= tol_from(x_or, x_pr)
    finally:
        h.close()


def test_graddiv_benchmark_regime_parity(dev):
    """Grad-div in the benchmark's regime (beta = 1e-4, kappa lognormal, two aggregation
    passes on level 0, tau_cut = 0.75 max mult) on 16 x 16: level structure bit-exact,
    V-cycle and PCG solution against the Moore-Penrose oracle within ten times the
    distance between the oracle's two Schur-complement routes (about 5e-8 here: A_ww
    and the interface blocks carry the 1e-8 ratio of mass to div term), iterations +-1."""
    P = _lsdd()
    prob, b = fegen.graddiv_hdiv(N=16)
    kw = dict(max_levels=4, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)
    h_or, h_pr = oracle_routes(prob, **kw)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(**kw))
    try:
        assert h.info()["n"] == [lv.n for lv in h_or.levels]
        for l in range(len(h_or.levels) - 1):
            ex = h.export_level(l)
            assert np.array_equal(ex["agg_of_dof"], h_or.levels[l].agg_of_dof)
            assert np.array_equal(ex["k"], h_or.levels[l].k)
            assert np.abs(ex["mu"] - np.concatenate(h_or.levels[l].mu)).max() <= mu_tol(h_or, h_pr)
        r = np.random.default_rng(16).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert rel(z, z_or) <= tol_from(z_or, oracle.vcycle(h_pr, r))
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert infos[0].converged == 1 and abs(infos[0].iters - inf_or.iters) <= 1
        assert rel(x.cpu().numpy(), x_or) <= tol_from(x_or, oracle.pcg(h_pr, b)[0])
    finally:
        h.close()


@pytest.mark.parametrize("name", ["q2hex3", "graddiv10"])
def test_blocked_tridiagonal_reduction_parity(dev, name):
    """Local spectral problems reduced by the blocked multi-workgroup path
    (every aggregate of at least 66 DOFs): local spectra 1e-10 against the
    oracle and 1e-12 against the single-workgroup reduction, retained modes
    bit-exact in number, mode blocks 1e-10 after cluster canonicalisation
    (against the single-workgroup path on every level, against the oracle on
    level 0, where both order aggregate DOFs ascending), V-cycle and PCG
    solution against the oracle; the oracle comparisons within ten times the
    distance between the oracle's two Schur-complement routes (at least 1e-10)."""
    P = _lsdd()
    rng = np.random.default_rng(3)
    if name == "q2hex3":
        prob = fegen.elasticity_q2hex(3, nu=0.3)
        kw = dict(max_levels=3, agg_passes=1, agg_passes_coarse=1, tau_const=0.75)
    else:
        N = 10
        prob = fegen.graddiv_rtcf3(N, kappa=np.exp(rng.standard_normal(N * N)), beta=1.0)
        kw = dict(max_levels=3, tau_const=0.75, max_density=1.0, agg_passes=1, agg_passes_coarse=1)
    # level-1 interface blocks of the grad-div case are singular to working precision:
    # tolerances from the spread of the oracle's two Schur-complement routes
    h_or, h_pr = oracle_routes(prob, **kw)
    m_tol = mu_tol(h_or, h_pr)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(blocked_eig_min=66, **kw))
    h1 = P.Hierarchy.setup_problem(prob, P.Params.default(blocked_eig_min=-1, **kw))
    try:
        assert h.info()["n"] == [lv.n for lv in h_or.levels]
        n_big = 0
        for l in range(len(h_or.levels) - 1):
            lv = h_or.levels[l]
            ex, ex1 = h.export_level(l), h1.export_level(l)
            nw = [len(a) for a in lv.aggs]
            n_big += sum(x >= 66 for x in nw)
            assert np.array_equal(ex["k"], lv.k)
            mu_or = np.concatenate(lv.mu)
            scale = max(1.0, np.abs(mu_or).max())
            assert np.abs(ex["mu"] - mu_or).max() <= m_tol * scale
            assert np.abs(ex["mu"] - ex1["mu"]).max() <= 1e-12 * scale
            Zg, Z1 = _gpu_Z_blocks(ex, nw), _gpu_Z_blocks(ex1, nw)
            for i in range(len(nw)):
                if lv.k[i] == 0 or nw[i] < 66:
                    continue
                # near-degenerate modes (relative gaps down to 1e-6 on grad-div) are
                # compared as clusters: their individual vectors move by eps / gap
                Qg = _canon(Zg[i], lv.mu[i], nw[i], tol=1e-5)
                Q1 = _canon(Z1[i], lv.mu[i], nw[i], tol=1e-5)
                zs = np.abs(Z1[i]).max()
                assert np.abs(Zg[i] @ Qg - Z1[i] @ Q1).max() <= 1e-10 * zs
                if l == 0:
                    Qo = _canon(lv.Z[i], lv.mu[i], nw[i], tol=1e-5)
                    Zp = h_pr.levels[0].Z[i]
                    Qp = _canon(Zp, h_pr.levels[0].mu[i], nw[i], tol=1e-5)
                    zo = np.abs(lv.Z[i]).max()
                    z_tol = max(1e-10, 10 * np.abs(Zp @ Qp - lv.Z[i] @ Qo).max() / zo)
                    assert np.abs(Zg[i] @ Qg - lv.Z[i] @ Qo).max() <= z_tol * zo
        assert n_big > 0
        r = rng.standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert rel(z, z_or) <= tol_from(z_or, oracle.vcycle(h_pr, r))
        b = rng.standard_normal(prob.n)
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert infos[0].converged == 1 and abs(infos[0].iters - inf_or.iters) <= 1
        assert rel(x.cpu().numpy(), x_or) <= tol_from(x_or, oracle.pcg(h_pr, b)[0])
    finally:
        h.close()
        h1.close()


def _replay_pivoted(A, G):
    """Replay a pivoted Cholesky against the factor rows G: at each step the pivot
    must be a largest remaining diagonal entry up to rounding (relative 1e-10) and
    the row must equal the replayed one to 1e-12; returns the pivot order."""
    S = np.array(A, dtype=np.float64)
    live = np.ones(len(A), dtype=bool)
    scale = np.abs(np.diag(A)).max()
    piv = []
    for k in range(G.shape[0]):
        d = np.where(live, np.diag(S), -np.inf)
        cands = np.flatnonzero(d >= d.max() - 1e-10 * scale)
        best, err, gb = None, np.inf, None
        for p in cands:
            g = np.where(live, S[:, p], 0.0) / np.sqrt(S[p, p])
            e = np.abs(G[k] - g).max()
            if e < err:
                best, err, gb = int(p), e, g
        assert err <= 1e-12 * np.sqrt(scale)
        piv.append(best)
        S -= np.outer(gb, gb)
        live[best] = False
    return piv


@pytest.mark.parametrize("name", ["q1", "rtcf3", "q2hex"])
def test_pivoted_cholesky_element_factors(dev, name):
    """elem_factor = 1 (Sec. 5.2 pivoted Cholesky): ranks bit-exact against the oracle's
    factor, G^T G = A_T to 1e-13, every row equal to a replay of the factorisation in
    the GPU's pivot order, each pivot a largest remaining diagonal entry up to rounding
    (blocks with equal diagonal entries have near-ties that rounding may order
    differently from the oracle), rows equal to the oracle's wherever both took the
    same pivots, and a hierarchy whose V-cycle and PCG solution match the oracle's (the
    hierarchy does not depend on the factor) within ten times the distance between the
    oracle's two Schur-complement routes, never below 1e-10."""
    P = _lsdd()
    from oracle import lsdd as O
    if name == "q1":
        prob, b = fegen.elasticity_small(N=16)
        kw = dict(max_levels=2, modes_fixed=4)
    elif name == "rtcf3":
        rng = np.random.default_rng(0)
        prob = fegen.graddiv_rtcf3(6, kappa=np.exp(rng.standard_normal(36)), beta=1.0)
        b = rng.standard_normal(prob.n)
        kw = dict(max_levels=3, tau_const=0.75, max_density=1.0, agg_passes=1, agg_passes_coarse=1)
    else:
        prob = fegen.elasticity_q2hex(3, nu=0.3)
        b = np.random.default_rng(1).standard_normal(prob.n)
        kw = dict(max_levels=2, tau_const=0.75, agg_passes=1)
    # tolerances of the cycle and the solution from the spread of the oracle's two
    # Schur-complement routes (at least 1e-10)
    h_or, h_pr = oracle_routes(prob, elem_factor="chol", **kw)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(elem_factor=1, **kw))
    try:
        ranks, G = h.export_gram(prob.elem_ptr)
        assert ranks.tolist() == [g.shape[0] for g in h_or.G0]
        offs = prob.block_offsets()
        same = 0
        for e in range(prob.n_elem):
            ne = int(prob.elem_ptr[e + 1] - prob.elem_ptr[e])
            Ge = G[offs[e]:offs[e + 1]].reshape(ne, ne)[:ranks[e]]
            _, Ae = prob.element(e)
            assert np.abs(Ge.T @ Ge - Ae).max() <= 1e-13 * np.abs(Ae).max()
            Go = h_or.G0[e]
            if _replay_pivoted(Ae, Ge) == _replay_pivoted(Ae, Go):
                same += 1
                assert np.abs(Ge - Go).max() <= 1e-12 * np.abs(Go).max()
        r = np.random.default_rng(7).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert rel(z, z_or) <= tol_from(z_or, oracle.vcycle(h_pr, r))
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert abs(infos[0].iters - inf_or.iters) <= 1
        assert rel(x.cpu().numpy(), x_or) <= tol_from(x_or, oracle.pcg(h_pr, b)[0])
    finally:
        h.close()


def test_eigen_element_factors_of_large_blocks(dev):
    """81 x 81 Q2 blocks (above the Jacobi size) go through the tridiagonal route
    (Householder reduction, bisection, inverse iteration, back-transformation):
    ranks bit-exact against the oracle's eigendecomposition, G^T G = A_T and
    G G^T = diag(positive eigenvalues, ascending) to 1e-12 of the block's scale (a few
    n eps for the backward-stable reduction and the inverse-iteration residuals), and
    the hierarchy's V-cycle as with the oracle's factor."""
    P = _lsdd()
    prob = fegen.elasticity_q2hex(3, nu=0.3)
    kw = dict(max_levels=2, tau_const=0.75, agg_passes=1)
    h_or, h_pr = oracle_routes(prob, **kw)
    h = P.Hierarchy.setup_problem(prob, P.Params.default(**kw))
    try:
        ranks, G = h.export_gram(prob.elem_ptr)
        assert ranks.tolist() == [g.shape[0] for g in h_or.G0]
        offs = prob.block_offsets()
        for e in range(prob.n_elem):
            ne = int(prob.elem_ptr[e + 1] - prob.elem_ptr[e])
            assert ne == 81
            Ge = G[offs[e]:offs[e + 1]].reshape(ne, ne)[:ranks[e]]
            _, Ae = prob.element(e)
            scale = np.abs(Ae).max()
            assert np.abs(Ge.T @ Ge - Ae).max() <= 1e-12 * scale
            lam = np.linalg.eigvalsh(Ae)[ne - ranks[e]:]
            assert np.abs(Ge @ Ge.T - np.diag(lam)).max() <= 1e-12 * scale
        r = np.random.default_rng(7).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert rel(z, z_or) <= tol_from(z_or, oracle.vcycle(h_pr, r))
    finally:
        h.close()


def test_pivoted_cholesky_rejects_an_indefinite_block(dev):
    P = _lsdd()
    prob = fegen.elasticity_q1(3, nu=0.3)
    bad = prob.blocks.copy().reshape(-1, 8, 8)
    bad[4] = -bad[4]
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, bad.ravel(), prob.node_of_dof,
                                   prob.agg_of_dof, P.Params.default(elem_factor=1, **ELAST_KW))
    assert ei.value.code == 2 and "element 4" in str(ei.value)


def _rows_problem(prob, G0):
    """The cover of a stacked Gram factor: one member per row of G, supported on its
    element's DOFs, with block g g^T."""
    from fegen.common import Problem
    dofs, blocks, ptr = [], [], [0]
    rp, cols, vals = [0], [], []
    for e in range(prob.n_elem):
        S, _ = prob.element(e)
        for g in G0[e]:
            dofs.append(np.asarray(S, dtype=np.int32))
            blocks.append(np.outer(g, g).ravel())
            ptr.append(ptr[-1] + len(S))
            cols.append(np.asarray(S, dtype=np.int32))
            vals.append(g)
            rp.append(rp[-1] + len(S))
    P = Problem(n=prob.n, elem_ptr=np.array(ptr, dtype=np.int64), elem_dofs=np.concatenate(dofs),
                blocks=np.concatenate(blocks), node_of_dof=prob.node_of_dof, agg_of_dof=prob.agg_of_dof)
    return P, np.array(rp, dtype=np.int64), np.concatenate(cols), np.concatenate(vals)


def test_black_box_csr_gram_factor_parity(dev):
    """lsdd_setup_gram_csr (Sec. 2: A = G^T G from a sparse G, every row its own cover
    member): the hierarchy built from the stacked element factors of the small elasticity
    problem matches the oracle run on the same row cover (aggregates, k_i bit-exact;
    spectra, V-cycle and PCG solution 1e-10, iterations +-1)."""
    P = _lsdd()
    prob, b = fegen.elasticity_small(N=16)
    G0 = oracle.setup(prob, oracle.Params(max_levels=1)).G0
    rows, rp, col, val = _rows_problem(prob, G0)
    kw = dict(max_levels=2, modes_fixed=4)
    h_or = oracle.setup(rows, oracle.Params(**kw))
    h = P.Hierarchy.setup_gram_csr(len(rp) - 1, prob.n, rp, col, val, prob.node_of_dof, prob.agg_of_dof,
                                   P.Params.default(**kw))
    try:
        assert h.info()["n"] == [lv.n for lv in h_or.levels]
        ex, lv = h.export_level(0), h_or.levels[0]
        assert np.array_equal(ex["agg_of_dof"], lv.agg_of_dof)
        assert np.array_equal(ex["k"], lv.k)
        assert np.array_equal(ex["omega_sizes"], [len(o) for o in lv.omegas])
        assert np.abs(ex["mu"] - np.concatenate(lv.mu)).max() <= 1e-10
        A_gpu = _csr(ex)
        assert abs(A_gpu - lv.A).max() <= 1e-13 * abs(lv.A).max()
        r = np.random.default_rng(11).standard_normal(prob.n)
        z_or = oracle.vcycle(h_or, r)
        z = h.vcycle(torch.from_numpy(r).to(dev)).cpu().numpy()
        assert np.linalg.norm(z - z_or) <= 1e-10 * np.linalg.norm(z_or)
        x_or, inf_or = oracle.pcg(h_or, b)
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        assert abs(infos[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
    finally:
        h.close()


def test_black_box_csr_gram_factor_device_input(dev):
    """The same CSR factor handed over as device arrays (mem_is_device = 1) builds the
    identical hierarchy: level-0 Gram rows, operators and solve bit-for-bit equal."""
    P = _lsdd()
    prob, b = fegen.elasticity_small(N=8)
    G0 = oracle.setup(prob, oracle.Params(max_levels=1)).G0
    _, rp, col, val = _rows_problem(prob, G0)
    kw = dict(max_levels=2, modes_fixed=4)
    args = (prob.node_of_dof, prob.agg_of_dof, P.Params.default(**kw))
    m = len(rp) - 1
    dv = [torch.from_numpy(a).to(dev) for a in (rp, col, val)]
    with P.Hierarchy.setup_gram_csr(m, prob.n, rp, col, val, *args) as hh, \
            P.Hierarchy.setup_gram_csr(m, prob.n, *dv, *args) as hd:
        assert hh.info()["n"] == hd.info()["n"]
        for l in range(len(hh.info()["n"])):
            eh, ed = hh.export_level(l), hd.export_level(l)
            for key in eh:
                assert np.array_equal(eh[key], ed[key]), (l, key)
        gh, gd = hh.export_gram_level(0), hd.export_gram_level(0)
        assert np.array_equal(gh["ranks"], gd["ranks"]) and np.array_equal(gh["G"], gd["G"])
        assert (gh["ranks"] == 1).all()
        bd = torch.from_numpy(b).to(dev)
        xh, ih = hh.solve(bd)
        xd, idd = hd.solve(bd)
        assert ih[0].iters == idd[0].iters and torch.equal(xh, xd)
    bad = dv[2].clone()
    bad[3] = float("nan")
    with pytest.raises(P.LsddError, match="non-finite"):
        P.Hierarchy.setup_gram_csr(m, prob.n, dv[0], dv[1], bad, *args)


@pytest.mark.parametrize("case", ["one_level", "no_modes"])
def test_single_level_hierarchies(dev, case):
    """Degenerate hierarchies: max_levels = 1, and a cut so strict that no aggregate
    keeps a mode (the level becomes the coarsest).  Either way the cycle is the dense
    direct solve: PCG converges in one iteration to the oracle's solution."""
    P = _lsdd()
    rng = np.random.default_rng(2)
    prob = fegen.graddiv_rtcf3(6, kappa=np.exp(rng.standard_normal(36)), beta=1.0)
    b = rng.standard_normal(prob.n)
    kw = dict(max_levels=1) if case == "one_level" else dict(max_levels=3, tau_const=1e12, agg_passes=1)
    h_or = oracle.setup(prob, oracle.Params(**kw))
    assert len(h_or.levels) == 1
    with P.Hierarchy.setup_problem(prob, P.Params.default(**kw)) as h:
        assert h.info()["levels"] == 1
        x, infos = h.solve(torch.from_numpy(b).to(dev))
        x_or, inf_or = oracle.pcg(h_or, b)
        assert infos[0].iters == inf_or.iters == 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
