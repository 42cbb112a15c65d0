"""The allocation-free element contraction lsdd_elem_bilinear_noalloc against
lsdd_elem_bilinear, both called through the C-ABI: identical kernels, staging in a
static device array instead of per-call device allocations.  Two calls in a row
(the second on a smaller input, so stale staging from the first would show), and
the size limit rejected on the host."""
import ctypes as C

import numpy as np
import pytest

import fegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(name, prob, U, V, scale):
    import paper_2607_07485_amd as P
    L = P.lib()
    f = getattr(L, name)
    f.restype = C.c_int
    f.argtypes = [C.c_int64, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                  C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
    dev = U.device
    ptr = np.ascontiguousarray(prob.elem_ptr, dtype=np.int64)
    dofs = torch.from_numpy(np.ascontiguousarray(prob.elem_dofs, dtype=np.int32)).to(dev)
    blocks = torch.from_numpy(np.ascontiguousarray(prob.blocks, dtype=np.float64)).to(dev)
    out = torch.full((prob.n_elem,), float("nan"), dtype=torch.float64, device=dev)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = f(prob.n_elem, ptr.ctypes.data_as(C.POINTER(C.c_int64)), C.c_void_p(dofs.data_ptr()),
           C.c_void_p(blocks.data_ptr()), C.c_void_p(U.data_ptr()), C.c_void_p(V.data_ptr()), U.shape[0], U.shape[1],
           scale, C.c_void_p(out.data_ptr()), st)
    return rc, out.cpu().numpy()


def test_noalloc_contraction_matches_the_allocating_one():
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(21)
    cases = [(fegen.elasticity_q2hex(3, nu=0.3), 3, -1.0),      # 27 elements of 81 DOFs, 3 vector pairs
             (fegen.elasticity_q1(6, nu=0.3), 1, 1.0)]          # then a smaller input, one pair
    for prob, nrhs, scale in cases:
        U = torch.from_numpy(rng.standard_normal((nrhs, prob.n))).to(dev)
        V = torch.from_numpy(rng.standard_normal((nrhs, prob.n))).to(dev)
        rc0, ref = _call("lsdd_elem_bilinear", prob, U, V, scale)
        rc1, got = _call("lsdd_elem_bilinear_noalloc", prob, U, V, scale)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(got, ref)
        # and the value itself: the element forms summed over the pairs
        Un, Vn = U.cpu().numpy(), V.cpu().numpy()
        e = prob.n_elem // 2
        d, B = prob.element(e)
        want = scale * sum(Un[k, d] @ B @ Vn[k, d] for k in range(nrhs))
        assert abs(got[e] - want) <= 1e-12 * max(1.0, abs(want))


def test_noalloc_contraction_rejects_more_elements_than_its_scratch_holds():
    import paper_2607_07485_amd as P
    L = P.lib()
    f = L.lsdd_elem_bilinear_noalloc
    f.restype = C.c_int
    n_elem = (1 << 20) + 1
    ptr = np.arange(n_elem + 1, dtype=np.int64)             # host-only check, no device access
    dummy = C.c_void_p(8)
    rc = f(n_elem, ptr.ctypes.data_as(C.POINTER(C.c_int64)), dummy, dummy, dummy, dummy, 1, 1, 1.0, dummy,
           C.c_void_p(None))
    assert rc == 7 and b"1048576" in L.lsdd_last_error()
