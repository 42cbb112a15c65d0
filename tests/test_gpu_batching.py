"""GPU parity of the batched paths (blocks of right-hand sides, captured PCG
iterations) against the FP64 oracle.

Each (instance, right-hand side) pair runs its own CG recurrence, so every
column is held to the single-solve bar: 1e-10 relative to the oracle's PCG
iterate, iterations +-1; zero columns give x = 0 after no iteration.  HIP-graph
replays must reproduce the eagerly launched solve bit for bit.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import fegen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ELAST_KW = dict(max_levels=2, modes_fixed=4)
GD_KW = dict(max_levels=3, tau_const=0.75, max_density=1.0, agg_passes=1, agg_passes_coarse=1)


def _lsdd():
    import paper_2607_07485_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return torch.device("cuda:0")


def _graddiv(N=10, seed=0):
    rng = np.random.default_rng(seed)
    return fegen.graddiv_rtcf3(N, kappa=np.exp(rng.standard_normal(N * N)), beta=1.0), rng


@pytest.mark.parametrize("nrhs", [3, 9])
def test_block_rhs_match_oracle(dev, nrhs):
    """nrhs = 9 runs one full block of 8 and a ragged block of 1."""
    P = _lsdd()
    prob, rng = _graddiv()
    B = rng.standard_normal((nrhs, prob.n))
    B[1] = 0.0
    h_or = oracle.setup(prob, oracle.Params(**GD_KW))
    with P.Hierarchy.setup_problem(prob, P.Params.default(**GD_KW)) as h:
        X, infos = h.solve(torch.from_numpy(B).to(dev))
        X = X.cpu().numpy()
        assert len(infos) == nrhs
        for k in range(nrhs):
            if k == 1:
                assert infos[k].iters == 0 and infos[k].converged == 1 and np.all(X[k] == 0.0)
                continue
            x_or, inf_or = oracle.pcg(h_or, B[k])
            assert infos[k].converged == 1
            assert abs(infos[k].iters - inf_or.iters) <= 1
            assert np.linalg.norm(X[k] - x_or) <= 1e-10 * np.linalg.norm(x_or)
            x1, inf1 = h.solve(torch.from_numpy(B[k]).to(dev))     # the same column alone
            assert inf1[0].iters == infos[k].iters
            assert np.linalg.norm(X[k] - x1.cpu().numpy()) <= 1e-10 * np.linalg.norm(x_or)


def test_block_fp32_cycle_anorm(dev):
    """FP32 block cycle inside FP64 PCG (flexible beta): A-norm error <= 1e-8 per column."""
    P = _lsdd()
    prob, _ = fegen.elasticity_small(N=16)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((3, prob.n))
    A = oracle.assemble(prob.n, *[[prob.element(e)[i] for e in range(prob.n_elem)] for i in (0, 1)]).tocsc()
    with P.Hierarchy.setup_problem(prob, P.Params.default(precision=1, rtol=1e-10, **ELAST_KW)) as h:
        X, infos = h.solve(torch.from_numpy(B).to(dev))
        X = X.cpu().numpy()
        for k in range(3):
            x_ref = spla.spsolve(A, B[k])
            e = X[k] - x_ref
            anorm = np.sqrt(e @ (A @ e)) / np.sqrt(x_ref @ (A @ x_ref))
            assert infos[k].converged == 1 and anorm <= 1e-8


def test_graph_replays_match_eager(dev):
    """Captured PCG halves replayed over several solves, with eager work in
    between, give the eager result bit for bit (single vectors and blocks)."""
    P = _lsdd()
    prob, rng = _graddiv(seed=5)
    b1 = torch.from_numpy(rng.standard_normal(prob.n)).to(dev)
    B3 = torch.from_numpy(rng.standard_normal((3, prob.n))).to(dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s), P.Hierarchy.setup_problem(prob, P.Params.default(**GD_KW)) as h:
        x_e, inf_e = h.solve(b1)
        X_e, infs_e = h.solve(B3)
        h.set_graph(True)
        for rep in range(3):
            junk = torch.randn(4096, device=dev, dtype=torch.float64)
            junk.mul_(2.0).sum().item()                 # eager work between replays
            x_g, inf_g = h.solve(b1)
            X_g, infs_g = h.solve(B3)
            torch.cuda.synchronize()
            assert torch.equal(x_g, x_e), f"replay {rep}"
            assert torch.equal(X_g, X_e), f"replay {rep}"
            assert inf_g[0].iters == inf_e[0].iters
            assert [i.iters for i in infs_g] == [i.iters for i in infs_e]
        h.set_graph(False)
        x_2, _ = h.solve(b1)
        assert torch.equal(x_2, x_e)


BATCH_KW = dict(max_levels=3, tau_const=0.75, max_density=1.0, min_coarse=1, agg_passes=2, agg_passes_coarse=1)


def _batch():
    """Uneven Q1 elasticity instances (vertex-patch cover, threshold modes)."""
    return [fegen.elasticity_q1(N, nu=nu) for N, nu in ((6, 0.3), (11, 0.45), (8, 0.38))]


def _check_batch_against_oracle(dev, probs, kw, nrhs_list=(1, 3), seed=21):
    """Per instance: level count and sizes, aggregates and retained modes on every
    level where the instance is coarsened, and every (instance, right-hand side)
    solve, against the instance's own oracle hierarchy."""
    P = _lsdd()
    h_ors = [oracle.setup(p, oracle.Params(**kw)) for p in probs]
    n_tot = sum(p.n for p in probs)
    B = np.random.default_rng(seed).standard_normal((max(nrhs_list), n_tot))
    with P.Hierarchy.setup_batched(probs, P.Params.default(**kw)) as h:
        nseg, off = h.segments()
        assert nseg == len(probs) and off == list(np.cumsum([0] + [p.n for p in probs]))
        info = h.info()
        depth = [len(ho.levels) for ho in h_ors]
        assert info["levels"] == max(depth)
        for l in range(info["levels"]):
            loff, term = h.level_segments(l)
            for i, ho in enumerate(h_ors):
                n_il = ho.levels[l].n if l < depth[i] else 0
                assert loff[i + 1] - loff[i] == n_il
                assert term[i] == (1 if l == depth[i] - 1 else 0)
            if l == info["levels"] - 1:
                continue
            ex = h.export_level(l)
            a0 = 0
            for i, ho in enumerate(h_ors):
                if l >= depth[i]:
                    continue
                agg = ex["agg_of_dof"][loff[i]:loff[i + 1]]
                if l == depth[i] - 1:
                    assert np.all(agg == -1)
                    continue
                lv = ho.levels[l]
                n_agg = len(lv.k)
                assert np.array_equal(agg - a0, lv.agg_of_dof)
                assert np.array_equal(ex["k"][a0:a0 + n_agg], lv.k)
                a0 += n_agg
        for nrhs in nrhs_list:
            X, infos = h.solve(torch.from_numpy(B[:nrhs].copy()).to(dev))
            X = X.cpu().numpy().reshape(nrhs, n_tot)
            for k in range(nrhs):
                for i, ho in enumerate(h_ors):
                    x_or, inf_or = oracle.pcg(ho, B[k, off[i]:off[i + 1]])
                    f = infos[k * nseg + i]
                    assert f.converged == 1 and abs(f.iters - inf_or.iters) <= 1
                    xi = X[k, off[i]:off[i + 1]]
                    assert np.linalg.norm(xi - x_or) <= 1e-10 * np.linalg.norm(x_or)


def test_batched_instances_match_per_instance_oracle(dev):
    """One union hierarchy over uneven instances of the same depth."""
    _check_batch_against_oracle(dev, _batch(), BATCH_KW)


def test_batched_instances_with_their_own_depths(dev):
    """Paper stopping tests per instance: the instances end their hierarchies on
    different levels (1, 2 and 3 levels) and are solved there directly."""
    probs = [fegen.elasticity_q1(N, nu=nu) for N, nu in ((2, 0.3), (20, 0.42), (9, 0.35))]
    kw = dict(max_levels=3, tau_const=0.75, agg_passes=2, agg_passes_coarse=1)
    depths = [len(oracle.setup(p, oracle.Params(**kw)).levels) for p in probs]
    assert depths == [1, 3, 2]
    _check_batch_against_oracle(dev, probs, kw)


def test_autotuned_shapes_keep_parity(dev):
    """The autotuner only changes launch shapes (and summation orders): solves
    still match the oracle for single vectors and blocks."""
    P = _lsdd()
    prob, rng = _graddiv(seed=8)
    h_or = oracle.setup(prob, oracle.Params(**GD_KW))
    b = rng.standard_normal(prob.n)
    B = rng.standard_normal((3, prob.n))
    with P.Hierarchy.setup_problem(prob, P.Params.default(**GD_KW)) as h:
        t1 = h.autotune(block=False)
        t8 = h.autotune(block=True)
        for t in t1 + t8:
            assert t["lanes"] in (8, 16, 32, 64) and t["lanes_block"] in (4, 8, 16, 32, 64)
            assert t["tiles_per_item"] in (2, 4, 8) and t["finalize_threads"] in (8, 32)
            assert t["elem_apply"] in (0, 1) and t["shared_cols"] in range(5) and t["fact_stash"] in (0, 1)
        x, inf = h.solve(torch.from_numpy(b).to(dev))
        x_or, inf_or = oracle.pcg(h_or, b)
        assert abs(inf[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
        X, infs = h.solve(torch.from_numpy(B).to(dev))
        X = X.cpu().numpy()
        for k in range(3):
            x_or, inf_or = oracle.pcg(h_or, B[k])
            assert abs(infs[k].iters - inf_or.iters) <= 1
            assert np.linalg.norm(X[k] - x_or) <= 1e-10 * np.linalg.norm(x_or)


def test_set_level_tuning_round_trip_and_checks(dev):
    """lsdd_set_level_tuning applies any candidate shape (read back by lsdd_level_tuning),
    the solve then matches the oracle as with the autotuner's shapes, and values outside
    the candidates are refused without changing anything."""
    P = _lsdd()
    prob, rng = _graddiv(seed=9)
    h_or = oracle.setup(prob, oracle.Params(**GD_KW))
    b = rng.standard_normal(prob.n)
    x_or, inf_or = oracle.pcg(h_or, b)
    with P.Hierarchy.setup_problem(prob, P.Params.default(**GD_KW)) as h:
        tuned = h.autotune(block=False)
        other = [dict(lanes=8 if t["lanes"] != 8 else 32, lanes_block=4, tiles_per_item=2 if t["tiles_per_item"] != 2 else 8,
                      finalize_threads=32 if t["finalize_threads"] == 8 else 8,
                      elem_apply=(1 - t["elem_apply"]) if l == 0 else 0) for l, t in enumerate(tuned)]
        h.set_tuning(other)
        levels = len(tuned)
        for l in range(levels):
            got = h.level_tuning(l)
            assert got["lanes"] == other[l]["lanes"] and got["finalize_threads"] == other[l]["finalize_threads"]
            assert got["elem_apply"] == other[l]["elem_apply"]
            if l < levels - 1:
                assert got["tiles_per_item"] == other[l]["tiles_per_item"]
        x, inf = h.solve(torch.from_numpy(b).to(dev))
        assert abs(inf[0].iters - inf_or.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
        before = h.level_tuning(0)
        for bad in (dict(before, lanes=12), dict(before, tiles_per_item=3), dict(before, finalize_threads=16),
                    dict(before, elem_apply=2), dict(before, shared_cols=5), dict(before, fact_stash=2)):
            with pytest.raises(P.LsddError) as ei:
                h.set_level_tuning(0, bad)
            assert ei.value.code == 1
        assert h.level_tuning(0) == before
        with pytest.raises(P.LsddError) as ei:                # element products exist on level 0 only
            h.set_level_tuning(1, dict(h.level_tuning(1), elem_apply=1))
        assert ei.value.code == 7
        h.set_tuning(tuned)
        x2, _ = h.solve(torch.from_numpy(b).to(dev))
        assert np.linalg.norm(x2.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)


@pytest.mark.parametrize("case", ["graddiv", "elasticity_q2hex"])
def test_element_triangle_products_match_the_csr_products(dev, case):
    """Full products of level 0 from the packed element triangles (elem_apply = 1):
    A x agrees with the CSR product to the rounding bound of the two summation orders
    (both sum the same products: 2 k u sum |A||x| per entry, k the longest CSR row plus
    the largest element), also after lsdd_update_theta; the FP64 PCG solve matches the
    oracle (1e-10, iterations +-1), and the FP32 and mixed cycles reach the tolerance
    in the CSR path's iteration count +-1."""
    P = _lsdd()
    rng = np.random.default_rng(17)
    if case == "graddiv":
        prob, _ = _graddiv(seed=9)
        kw = GD_KW
    else:
        prob = fegen.elasticity_q2hex(3, nu=0.3)
        kw = dict(max_levels=3, agg_passes=1, agg_passes_coarse=1, tau_const=0.75)
    theta = np.ones(prob.n_elem)
    with P.Hierarchy.setup_elements_scaled(prob.n, prob.elem_ptr, prob.elem_dofs, prob.blocks, theta,
                                           prob.node_of_dof, prob.agg_of_dof,
                                           P.Params.default(precision=2, **kw)) as h:
        t0 = h.level_tuning(0)
        x = torch.from_numpy(rng.standard_normal(prob.n)).to(dev)
        offs = prob.block_offsets()
        dofs = [prob.elem_dofs[prob.elem_ptr[e]:prob.elem_ptr[e + 1]] for e in range(prob.n_elem)]
        absA = oracle.assemble(prob.n, dofs, [np.abs(prob.blocks[offs[e]:offs[e + 1]]).reshape(len(S), len(S))
                                              for e, S in enumerate(dofs)])
        k = int(np.diff(absA.indptr).max()) + max(len(S) for S in dofs)

        def products(th):
            ys = []
            for ea in (0, 1):
                h.set_level_tuning(0, dict(t0, elem_apply=ea))
                ys.append(h.apply(x, level=0).cpu().numpy())
            bound = 2 * k * np.finfo(float).eps * (absA @ np.abs(x.cpu().numpy())) * th.max()
            assert (np.abs(ys[0] - ys[1]) <= bound).all()
            assert np.abs(ys[0] - ys[1]).max() > 0                 # the element path is taken

        products(theta)
        theta2 = np.exp(0.3 * rng.standard_normal(prob.n_elem))
        h.update_theta(torch.from_numpy(theta2).to(dev))
        products(theta2)
        h.update_theta(torch.from_numpy(theta).to(dev))
        b = rng.standard_normal(prob.n)
        h_or = oracle.setup(prob, oracle.Params(**kw))
        x_or, inf_or = oracle.pcg(h_or, b)
        bd = torch.from_numpy(b).to(dev)
        its = {}
        for ea in (0, 1):
            h.set_level_tuning(0, dict(t0, elem_apply=ea))
            for prec in (0, 1, 2):
                h.set_cycle_precision(prec)
                xs, inf = h.solve(bd)
                assert inf[0].converged == 1
                its[ea, prec] = inf[0].iters
                if prec == 0:
                    assert abs(inf[0].iters - inf_or.iters) <= 1
                    assert np.linalg.norm(xs.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
        for prec in (0, 1, 2):
            assert abs(its[1, prec] - its[0, prec]) <= 1, its


def test_shared_column_lists_match_per_entry_columns_bit_for_bit(dev):
    """On supernode-blocked levels the CSR kernels may read one column list per
    supernode instead of a column index per entry: V-cycles and PCG solves (FP64, FP32
    and mixed cycles, single vectors and blocks of 8 right-hand sides) equal the
    per-entry reads bit for bit; the coarse levels always offer the lists."""
    P = _lsdd()
    prob, rng = _graddiv(seed=9)
    r = torch.from_numpy(rng.standard_normal(prob.n)).to(dev)
    with P.Hierarchy.setup_problem(prob, P.Params.default(precision=2, **GD_KW)) as h:
        levels = h.info()["levels"]
        base = [h.level_tuning(l) for l in range(levels)]
        avail = []
        for l in range(levels):
            try:
                h.set_level_tuning(l, dict(base[l], shared_cols=1))
                avail.append(l)
            except P.LsddError as ex:
                assert ex.code == 7
        assert 1 in avail
        r1 = torch.from_numpy(rng.standard_normal(h.info()["n"][1])).to(dev)

        def run(sc):
            h.set_tuning([dict(t, shared_cols=sc if l in avail else 0) for l, t in enumerate(base)])
            out = []
            for prec in (0, 1, 2):
                h.set_cycle_precision(prec)
                x, inf = h.solve(r)
                assert inf[0].converged == 1
                out += [h.vcycle(r), x, h.apply(r1, level=1)]
            return out

        for a, b in zip(run(0), run(1)):
            assert torch.equal(a, b)
        # blocks of 8 right-hand sides (the block CSR kernels) read the same lists
        R = torch.from_numpy(rng.standard_normal((9, prob.n))).to(dev)
        h.set_cycle_precision(0)
        outs = []
        for sc in (0, 1):
            h.set_tuning([dict(t, shared_cols=sc if l in avail else 0) for l, t in enumerate(base)])
            outs.append(h.solve(R)[0])
        assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("sc", [2, 3, 4])
def test_supernode_row_blocks_match_the_oracle(dev, sc):
    """Sweep residuals by supernode row blocks (1, 2 or 4 waves per run of up to 8
    sweep rows of one supernode; the supernodes of this level are not multiples of 8,
    so full and ragged runs): the FP64 V-cycle and PCG solve match the oracle and the
    per-row kernels to 1e-10 (only the order of the cross-lane sums differs, a
    rounding-level change that the cycle's coarse solves amplify); with the FP32 and
    mixed cycles the distance from the FP64 cycle stays that of the per-row kernels
    (within 4x) and the solves converge in the same iteration counts +-1.  Levels
    without row blocks reject the option."""
    P = _lsdd()
    prob, rng = _graddiv(seed=11)
    h_or = oracle.setup(prob, oracle.Params(**GD_KW))
    r = rng.standard_normal(prob.n)
    rt = torch.from_numpy(r).to(dev)
    with P.Hierarchy.setup_problem(prob, P.Params.default(precision=2, **GD_KW)) as h:
        levels = h.info()["levels"]
        base = [h.level_tuning(l) for l in range(levels)]
        avail = []
        for l in range(levels):
            try:
                h.set_level_tuning(l, dict(base[l], shared_cols=sc))
                assert h.level_tuning(l)["shared_cols"] == sc
                avail.append(l)
            except P.LsddError as ex:
                assert ex.code == 7
        assert 1 in avail and levels - 1 not in avail

        def run(c):
            h.set_tuning([dict(t, shared_cols=c if l in avail else 0) for l, t in enumerate(base)])
            out = {}
            for prec in (0, 1, 2):
                h.set_cycle_precision(prec)
                x, inf = h.solve(rt)
                assert inf[0].converged == 1
                out[prec] = (h.vcycle(rt).cpu().numpy(), x.cpu().numpy(), inf[0].iters)
            return out

        rows, blocks = run(1), run(sc)
        z, x, it = blocks[0]
        z_or = oracle.vcycle(h_or, r)
        x_or, inf_or = oracle.pcg(h_or, r)
        assert np.linalg.norm(z - z_or) <= 1e-10 * np.linalg.norm(z_or)
        assert np.linalg.norm(x - x_or) <= 1e-10 * np.linalg.norm(x_or)
        assert abs(it - inf_or.iters) <= 1
        assert np.linalg.norm(z - rows[0][0]) <= 1e-10 * np.linalg.norm(z)
        for prec in (1, 2):
            # FP32 vectors: each order of the sums is its own FP32 rounding of the FP64
            # cycle; the row blocks' distance from it stays that of the per-row sums
            za, zb = rows[prec][0], blocks[prec][0]
            da, db = np.linalg.norm(za - z), np.linalg.norm(zb - z)
            print(f"cycle precision {prec}: |z32 - z64| / |z64| per-row {da / np.linalg.norm(z):.3e}, "
                  f"row blocks {db / np.linalg.norm(z):.3e}")
            assert db <= 4.0 * da
            assert abs(blocks[prec][2] - rows[prec][2]) <= 1
        # a repeated solve is bit-reproducible (fixed order of the cross-wave sums)
        h.set_cycle_precision(0)
        assert torch.equal(h.solve(rt)[0], h.solve(rt)[0])


@pytest.mark.parametrize("lanes_block", [4, 8, 16])
def test_supernode_row_blocks_for_blocks_of_rhs_are_bit_identical(dev, lanes_block):
    """Blocks of right-hand sides (9 = a full block of 8 and a ragged one): the sweep
    residuals by supernode row blocks (up to 4 rows of one supernode per x gather) use
    the per-row sums of the same lane count, so the solves equal the per-row kernels'
    bit for bit, and match the oracle per column."""
    P = _lsdd()
    prob, rng = _graddiv(seed=13)
    h_or = oracle.setup(prob, oracle.Params(**GD_KW))
    B = rng.standard_normal((9, prob.n))
    with P.Hierarchy.setup_problem(prob, P.Params.default(**GD_KW)) as h:
        levels = h.info()["levels"]
        base = [h.level_tuning(l) for l in range(levels)]
        avail = []
        for l in range(levels):
            try:
                h.set_level_tuning(l, dict(base[l], shared_cols=2, lanes_block=lanes_block))
                avail.append(l)
            except P.LsddError as ex:
                assert ex.code == 7
        assert 1 in avail
        outs = []
        for sc in (1, 2):
            h.set_tuning([dict(t, shared_cols=sc if l in avail else 0, lanes_block=lanes_block)
                          for l, t in enumerate(base)])
            X, infos = h.solve(torch.from_numpy(B).to(dev))
            outs.append((X, [f.iters for f in infos]))
        assert torch.equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
        X = outs[1][0].cpu().numpy()
        for k in (0, 8):
            x_or, inf_or = oracle.pcg(h_or, B[k])
            assert abs(outs[1][1][k] - inf_or.iters) <= 1
            assert np.linalg.norm(X[k] - x_or) <= 1e-10 * np.linalg.norm(x_or)


def test_solve_batched_over_separate_hierarchies(dev):
    """lsdd_solve_batched on three separately built hierarchies (two elasticity meshes and
    a grad-div one, two right-hand sides each): every instance's result equals its own
    lsdd_solve bit for bit, and the reports come back in instance order."""
    P = _lsdd()
    probs = [fegen.elasticity_small(N=8)[0], fegen.elasticity_small(N=12)[0], _graddiv(6)[0]]
    kws = [ELAST_KW, ELAST_KW, GD_KW]
    rng = np.random.default_rng(31)
    hs = [P.Hierarchy.setup_problem(p, P.Params.default(**kw)) for p, kw in zip(probs, kws)]
    try:
        bs = [torch.from_numpy(rng.standard_normal((2, p.n))).to(dev) for p in probs]
        xs, infos = P.solve_batched(hs, bs)
        assert len(infos) == 3
        for h, b, x, inf in zip(hs, bs, xs, infos):
            x1, inf1 = h.solve(b)
            assert torch.equal(x, x1)
            assert [f.iters for f in inf] == [f.iters for f in inf1] and all(f.converged for f in inf)
    finally:
        for h in hs:
            h.close()
