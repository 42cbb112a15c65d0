"""Checks of the seeded input generators (shapes, symmetry, semidefiniteness, DOF counts)."""
import numpy as np
import pytest

import fegen


def _check_blocks(prob, tol=1e-12):
    for e in range(0, prob.n_elem, max(1, prob.n_elem // 50)):
        _, B = prob.element(e)
        assert np.abs(B - B.T).max() <= 1e-14 * np.abs(B).max()
        w = np.linalg.eigvalsh(B)
        assert w[0] >= -tol * w[-1]


def test_elasticity_q1_counts_and_blocks():
    prob, b = fegen.elasticity_small()
    assert prob.n == 2178 and prob.n_elem == 1024 and b.shape == (2178,)
    assert prob.meta["lam"] == pytest.approx(0.576923076923) and prob.meta["mu"] == pytest.approx(0.384615384615)
    _check_blocks(prob)
    assert prob.agg_of_dof.max() + 1 == 121
    # every DOF is covered by at least one element
    assert np.unique(prob.elem_dofs).size == prob.n


def test_rtcf3_counts_and_blocks():
    for N in (2, 5, 128):
        dofs, node, n = fegen.hdiv.rtcf3_dofs(N)
        assert n == 6 * N * (N + 1) + 12 * N * N
    assert fegen.hdiv.rtcf3_dofs(128)[2] == 295680
    prob, _ = fegen.graddiv_hdiv(N=6)
    _check_blocks(prob)
    # normal continuity: an edge DOF is shared by exactly the two cells of an interior edge
    counts = np.bincount(prob.elem_dofs, minlength=prob.n)
    assert set(np.unique(counts)) == {1, 2}


def test_rtcf3_divergence_of_a_constant_field_vanishes():
    """u = (1, 0) lies in RTCF_3; its element coefficients make the div-div block vanish."""
    Div, Mass = fegen.hdiv.rtcf3_reference(0.25)
    c = np.zeros(24)
    c[:12] = 1.0            # Lagrange bases sum to one in each direction
    assert abs(c @ Div @ c) <= 1e-12
    assert c @ Mass @ c == pytest.approx(0.25 ** 2)


def test_q2hex_blocks():
    prob = fegen.elasticity_q2hex(2, nu=0.3)
    assert prob.n == 3 * 5 ** 3 and prob.n_elem == 8
    _check_blocks(prob, tol=1e-11)
    # interior-type block: 81 DOFs minus 6 rigid modes
    w = np.linalg.eigvalsh(prob.element(1)[1])
    assert np.sum(w < 1e-10 * w[-1]) == 6


def test_batch_preset_is_seeded():
    a = fegen.elasticity_batch(n_inst=3, nmin=4, nmax=8, nrhs=2)
    b = fegen.elasticity_batch(n_inst=3, nmin=4, nmax=8, nrhs=2)
    for (pa, ba), (pb, bb) in zip(a, b):
        assert pa.n == pb.n and np.array_equal(ba, bb) and ba.shape == (2, pa.n)


def test_bfs_hyperdiffusion_blocks():
    """BFS elements: symmetric SPSD blocks, the DOF count 4 (N+1)^2, and the interior energy of
    polynomials represented exactly by bicubic Hermite interpolation equals the analytic
    integral of q(u)^2 with q(u) = D11 u_xx + 2 D12 u_xy + D22 u_yy."""
    from fegen.hermite import bfs_element_matrices, diffusion_tensor, hyperdiffusion_bfs
    prob = hyperdiffusion_bfs(4)
    assert prob.n == 4 * 25 and len(prob.elem_ptr) - 1 == 16
    B = prob.blocks.reshape(-1, 16, 16)
    for Be in B:
        assert np.abs(Be - Be.T).max() <= 1e-12 * np.abs(Be).max()
        ev = np.linalg.eigvalsh(Be)
        assert ev[0] >= -1e-12 * ev[-1]
    D = diffusion_tensor(1e-4, np.pi / 6)
    h = 0.25
    K = bfs_element_matrices(D, h)[0]
    x0, y0 = 0.25, 0.5                                  # element corner; vertices in local order
    verts = [(x0, y0), (x0 + h, y0), (x0, y0 + h), (x0 + h, y0 + h)]
    # u, u_x, u_y, u_xy of test polynomials and their constant / affine q(u)
    polys = {
        "x2": (lambda x, y: (x * x, 2 * x, 0.0, 0.0), lambda x, y: 2 * D[0, 0]),
        "xy": (lambda x, y: (x * y, y, x, 1.0), lambda x, y: 2 * D[0, 1]),
        "y2": (lambda x, y: (y * y, 0.0, 2 * y, 0.0), lambda x, y: 2 * D[1, 1]),
        "x2y": (lambda x, y: (x * x * y, 2 * x * y, x * x, 2 * x), lambda x, y: 2 * D[0, 0] * y + 4 * D[0, 1] * x),
    }
    for name, (f, q) in polys.items():
        u = np.array([v for (x, y) in verts for v in f(x, y)])
        # q is at most affine: the midpoint/vertex Simpson-type rule below is exact for q^2 (degree 2)
        gx, gw = np.polynomial.legendre.leggauss(3)
        exact = sum(wa * wb * q(x0 + h * (a + 1) / 2, y0 + h * (b + 1) / 2) ** 2
                    for a, wa in zip(gx, gw) for b, wb in zip(gx, gw)) * h * h / 4
        assert abs(u @ K @ u - exact) <= 1e-10 * abs(exact), name


def _assembled(prob):
    import scipy.sparse as sp
    ne = np.diff(prob.elem_ptr)
    rows, cols, vals = [], [], []
    for e in range(prob.n_elem):
        d, B = prob.element(e)
        rows.append(np.repeat(d, len(d)))
        cols.append(np.tile(d, len(d)))
        vals.append(B.ravel())
    assert ne.min() == ne.max() == 3
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(prob.n, prob.n))


def test_p1_triangles_counts_and_five_point_stencil():
    """With kappa = 1, CG1 on right isosceles triangles is the 5-point Laplacian away
    from the boundary (4 on the diagonal, -1 to the axis neighbours, exactly 0 to the
    diagonal neighbour that shares two triangles)."""
    for N, n in ((32, 1089), (64, 4225)):
        assert (N + 1) ** 2 == n
    N = 8
    prob = fegen.diffusion_p1_triangles(N, kappa=lambda x, y: np.ones_like(np.asarray(x, dtype=float)))
    assert prob.n == 81 and prob.n_elem == 128
    _check_blocks(prob)
    A = _assembled(prob).toarray()
    nx = N + 1
    for j in range(2, N - 1):
        for i in range(2, N - 1):
            p = j * nx + i
            assert A[p, p] == pytest.approx(4.0, abs=1e-13)
            for q in (p - 1, p + 1, p - nx, p + nx):
                assert A[p, q] == pytest.approx(-1.0, abs=1e-13)
            assert A[p, p + nx + 1] == 0.0 and A[p, p - nx - 1] == 0.0
            assert np.count_nonzero(np.abs(A[p]) > 1e-14) == 5


def test_p1_nitsche_form_closed_values():
    """a_h(1, 1) = 24/h int_{bd} kappa ds = 192 N and a_h(x, x) = 96 N - 3 for
    kappa = 1 + x + y (cell term int kappa = 2, penalty 24/h * 4, and the two
    consistency terms -2 int_{x=1} kappa = -5); both functions lie in CG1."""
    for N in (4, 16):
        prob = fegen.diffusion_p1_triangles(N)
        A = _assembled(prob)
        one = np.ones(prob.n)
        x = np.tile(np.arange(N + 1) / N, N + 1)
        assert one @ (A @ one) == pytest.approx(192.0 * N, rel=1e-13)
        assert x @ (A @ x) == pytest.approx(96.0 * N - 3.0, rel=1e-13)
        _check_blocks(prob)


def test_p1_interior_diagonal_entries_cancel_with_variable_kappa():
    """Each triangle contributes exactly 0 to its hypotenuse pair, so the assembled
    entry vanishes away from the boundary although two elements hold both DOFs."""
    N = 16
    prob = fegen.diffusion_p1_triangles(N)
    A = _assembled(prob)
    nx = N + 1
    zero = [A[j * nx + i, (j + 1) * nx + i + 1] for j in range(1, N - 1) for i in range(1, N - 1)]
    assert max(abs(z) for z in zero) == 0.0
    # rows of interior DOFs sum to zero (constants are in the kernel of the cell term)
    rs = np.asarray(A.sum(axis=1)).ravel().reshape(nx, nx)[2:-2, 2:-2]
    assert np.abs(rs).max() <= 1e-12
