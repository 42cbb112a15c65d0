"""ctypes binding of liblsdd.so (argument marshalling only).

The names follow the C-ABI in include/lsdd.h.  Device arrays are torch CUDA
(HIP) tensors; host arrays are numpy arrays.  The library must be built
(python -m paper_2607_07485_amd.build); importing this module fails loudly
when it is missing, and no operation has a CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_PKG, "liblsdd.so")

LSDD_STATUS = {0: "LSDD_OK", 1: "LSDD_E_INVAL", 2: "LSDD_E_NOT_SPSD", 3: "LSDD_E_NOMEM", 4: "LSDD_E_HIP",
               5: "LSDD_E_NOCONV", 6: "LSDD_E_BREAKDOWN", 7: "LSDD_E_UNSUPPORTED", 8: "LSDD_E_NUMERIC"}


class LsddError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{LSDD_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("max_levels", C.c_int32), ("agg_passes", C.c_int32), ("agg_passes_coarse", C.c_int32),
                ("modes_fixed", C.c_int32), ("min_coarse", C.c_int32), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("blocked_eig_min", C.c_int32),
                ("closure", C.c_int32), ("smoother", C.c_int32),
                ("elem_factor", C.c_int32), ("galerkin_precision", C.c_int32),
                ("tau_const", C.c_double), ("max_density", C.c_double), ("rtol", C.c_double),
                ("cluster_tol", C.c_double), ("band_tol", C.c_double), ("rank_rtol", C.c_double),
                ("spsd_tol", C.c_double), ("closure_tol", C.c_double)]

    @classmethod
    def default(cls, **kw) -> "Params":
        p = cls()
        lib().lsdd_params_default(C.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise AttributeError(k)
            setattr(p, k, v)
        return p


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("setup_s", C.c_double), ("solve_s", C.c_double)]


_LIB = None
_P = C.c_void_p


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is not built; run `python -m paper_2607_07485_amd.build`")
        L = C.CDLL(lib_path)
        i32p, i64p, f64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
        L.lsdd_params_default.argtypes = [C.POINTER(Params)]
        L.lsdd_params_default.restype = None
        L.lsdd_last_error.restype = C.c_char_p
        L.lsdd_setup_elements.argtypes = [C.c_int64, C.c_int64, i64p, i32p, _P, i32p, i32p, C.c_int,
                                          C.POINTER(Params), _P, C.POINTER(_P)]
        L.lsdd_setup_gram_csr.argtypes = [C.c_int64, C.c_int64, _P, _P, _P, i32p, i32p, C.c_int,
                                          C.POINTER(Params), _P, C.POINTER(_P)]
        L.lsdd_solve.argtypes = [_P, _P, _P, C.c_int32, _P, C.POINTER(Info)]
        L.lsdd_solve_stationary.argtypes = [_P, _P, _P, C.c_int32, _P, C.POINTER(Info)]
        L.lsdd_vcycle.argtypes = [_P, _P, _P, _P]
        L.lsdd_apply.argtypes = [_P, C.c_int32, _P, _P, _P]
        L.lsdd_hierarchy_info.argtypes = [_P, i32p, i64p, i64p, f64p, f64p]
        L.lsdd_level_sizes.argtypes = [_P, C.c_int32, i64p]
        L.lsdd_export_level.argtypes = [_P, C.c_int32, i32p, i32p, f64p, f64p, i32p, i64p, i32p, f64p, i32p]
        L.lsdd_export_gram.argtypes = [_P, i32p, f64p]
        L.lsdd_export_gram_level.argtypes = [_P, C.c_int32, i64p, i32p, i32p, f64p]
        L.lsdd_destroy.argtypes = [_P]
        L.lsdd_set_cycle_precision.argtypes = [_P, C.c_int32]
        L.lsdd_trace.argtypes = [_P, C.c_int32]
        L.lsdd_set_solve_params.argtypes = [_P, C.c_double, C.c_int32]
        L.lsdd_trace_get.argtypes = [_P, C.c_int32, C.c_char_p, C.c_int32, i64p, f64p, f64p]
        L.lsdd_set_allocator.argtypes = [_P, _P, _P]
        L.lsdd_set_graph.argtypes = [_P, C.c_int32]
        L.lsdd_setup_batched.argtypes = [C.c_int32, i64p, i64p, i64p, i32p, _P, i32p, i32p, C.c_int,
                                         C.POINTER(Params), _P, C.POINTER(_P)]
        L.lsdd_segments.argtypes = [_P, i32p, i64p]
        L.lsdd_level_segments.argtypes = [_P, C.c_int32, i64p, i32p]
        L.lsdd_autotune.argtypes = [_P, C.c_int32, _P]
        L.lsdd_setup_elements_scaled.argtypes = [C.c_int64, C.c_int64, i64p, i32p, _P, _P, i32p, i32p, C.c_int,
                                                 C.POINTER(Params), _P, C.POINTER(_P)]
        L.lsdd_update_theta.argtypes = [_P, _P, _P]
        L.lsdd_elem_bilinear.argtypes = [C.c_int64, i64p, _P, _P, _P, _P, C.c_int32, C.c_int64, C.c_double, _P,
                                         _P]
        L.lsdd_elem_bilinear_noalloc.argtypes = [C.c_int64, i64p, _P, _P, _P, _P, C.c_int32, C.c_int64,
                                                 C.c_double, _P, _P]
        L.lsdd_solve_batched.argtypes = [C.c_int32, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.c_int32, _P,
                                         C.POINTER(Info)]
        L.lsdd_level_tuning.argtypes = [_P, C.c_int32, i32p]
        L.lsdd_set_level_tuning.argtypes = [_P, C.c_int32, i32p]
        L.lsdd_set_allocator.restype = None
        for name in ("lsdd_setup_elements", "lsdd_setup_gram_csr", "lsdd_solve", "lsdd_solve_stationary",
                     "lsdd_vcycle", "lsdd_apply",
                     "lsdd_hierarchy_info", "lsdd_level_sizes", "lsdd_export_level", "lsdd_export_gram",
                     "lsdd_destroy", "lsdd_set_cycle_precision", "lsdd_trace", "lsdd_trace_get",
                     "lsdd_set_solve_params", "lsdd_set_graph", "lsdd_segments", "lsdd_setup_batched",
                     "lsdd_level_segments", "lsdd_autotune", "lsdd_level_tuning", "lsdd_setup_elements_scaled",
                     "lsdd_update_theta", "lsdd_elem_bilinear", "lsdd_elem_bilinear_noalloc",
                     "lsdd_solve_batched", "lsdd_export_gram_level", "lsdd_set_level_tuning"):
            getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def _check(code: int, allow=()):
    if code != 0 and code not in allow:
        raise LsddError(code, lib().lsdd_last_error().decode())
    return code


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def _stream():
    import torch
    if not torch.cuda.is_available():
        return C.c_void_p(None)        # host-side validation still runs; device calls then fail
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def elem_bilinear(elem_ptr, elem_dofs, blocks, u, v, scale=1.0, out=None):
    """lsdd_elem_bilinear: out[e] = scale * sum_k u_{k,e}^T B_e v_{k,e}.  elem_ptr host
    int64 array; elem_dofs a device int32 tensor; blocks float64 device tensor; u, v
    float64 device tensors [n] or [nrhs, n] of the same shape."""
    import torch
    elem_ptr = np.ascontiguousarray(elem_ptr, dtype=np.int64)
    if not (isinstance(elem_dofs, torch.Tensor) and elem_dofs.is_cuda and elem_dofs.dtype == torch.int32
            and elem_dofs.is_contiguous()):
        raise TypeError("elem_dofs: expected a contiguous int32 device tensor")
    if u.shape != v.shape or u.dim() not in (1, 2):
        raise ValueError("u and v: tensors of equal shape [n] or [nrhs, n]")
    u2, v2 = u.reshape(-1, u.shape[-1]).contiguous(), v.reshape(-1, v.shape[-1]).contiguous()
    ne = len(elem_ptr) - 1
    out = torch.empty(ne, dtype=torch.float64, device=u.device) if out is None else out
    _check(lib().lsdd_elem_bilinear(ne, _ptr(elem_ptr, C.c_int64), C.c_void_p(elem_dofs.data_ptr()), _dev_ptr(blocks),
                                    _dev_ptr(u2), _dev_ptr(v2), u2.shape[0], u2.shape[1], float(scale),
                                    _dev_ptr(out), _stream()))
    return out


def solve_batched(hs, bs, xs=None, allow_noconv=False):
    """lsdd_solve_batched: hs[i] x_i = b_i for separately built hierarchies (every b_i of
    shape [n_i] or [nrhs, n_i] with the same nrhs); returns (xs, [[Info] per instance])."""
    import torch
    n_inst = len(hs)
    if n_inst < 1 or len(bs) != n_inst:
        raise ValueError("one right-hand side tensor per hierarchy")
    nrhs = 1 if bs[0].dim() == 1 else bs[0].shape[0]
    xs = [torch.empty_like(b) for b in bs] if xs is None else xs
    nseg = [h.segments()[0] for h in hs]
    infos = (Info * (nrhs * sum(nseg)))()
    H = (C.c_void_p * n_inst)(*[h._h.value for h in hs])
    B = (C.c_void_p * n_inst)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * n_inst)(*[x.data_ptr() for x in xs])
    _check(lib().lsdd_solve_batched(n_inst, H, B, X, nrhs, _stream(), infos), allow=(5,) if allow_noconv else ())
    out, off = [], 0
    for k in nseg:
        out.append([infos[off + i] for i in range(nrhs * k)])
        off += nrhs * k
    return xs, out


class Hierarchy:
    """An LS-AMG-DD hierarchy owned by the library (lsdd_hierarchy*)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    # ---------------------------------------------------------------- setup
    @classmethod
    def setup_elements(cls, n, elem_ptr, elem_dofs, blocks, node_of_dof=None, agg_of_dof=None, params=None):
        """lsdd_setup_elements; `blocks` is a host numpy array or a float64 device tensor."""
        import torch
        elem_ptr = np.ascontiguousarray(elem_ptr, dtype=np.int64)
        elem_dofs = np.ascontiguousarray(elem_dofs, dtype=np.int32)
        nod = None if node_of_dof is None else np.ascontiguousarray(node_of_dof, dtype=np.int32)
        agg = None if agg_of_dof is None else np.ascontiguousarray(agg_of_dof, dtype=np.int32)
        if isinstance(blocks, torch.Tensor):
            bptr, on_dev = _dev_ptr(blocks), 1
        else:
            blocks = np.ascontiguousarray(blocks, dtype=np.float64)
            bptr, on_dev = C.c_void_p(blocks.ctypes.data), 0
        params = params or Params.default()
        h = C.c_void_p()
        _check(lib().lsdd_setup_elements(int(n), len(elem_ptr) - 1, _ptr(elem_ptr, C.c_int64),
                                         _ptr(elem_dofs, C.c_int32), bptr, _ptr(nod, C.c_int32),
                                         _ptr(agg, C.c_int32), on_dev, C.byref(params), _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def setup_elements_scaled(cls, n, elem_ptr, elem_dofs, blocks, theta, node_of_dof=None, agg_of_dof=None,
                              params=None):
        """lsdd_setup_elements_scaled: blocks (unit blocks) and theta both host numpy arrays or
        both float64 device tensors."""
        import torch
        elem_ptr = np.ascontiguousarray(elem_ptr, dtype=np.int64)
        elem_dofs = np.ascontiguousarray(elem_dofs, dtype=np.int32)
        nod = None if node_of_dof is None else np.ascontiguousarray(node_of_dof, dtype=np.int32)
        agg = None if agg_of_dof is None else np.ascontiguousarray(agg_of_dof, dtype=np.int32)
        if isinstance(blocks, torch.Tensor):
            bptr, tptr, on_dev = _dev_ptr(blocks), _dev_ptr(theta), 1
        else:
            blocks = np.ascontiguousarray(blocks, dtype=np.float64)
            theta = np.ascontiguousarray(theta, dtype=np.float64)
            bptr, tptr, on_dev = C.c_void_p(blocks.ctypes.data), C.c_void_p(theta.ctypes.data), 0
        params = params or Params.default()
        h = C.c_void_p()
        _check(lib().lsdd_setup_elements_scaled(int(n), len(elem_ptr) - 1, _ptr(elem_ptr, C.c_int64),
                                                _ptr(elem_dofs, C.c_int32), bptr, tptr, _ptr(nod, C.c_int32),
                                                _ptr(agg, C.c_int32), on_dev, C.byref(params), _stream(),
                                                C.byref(h)))
        return cls(h)

    def update_theta(self, theta):
        """lsdd_update_theta (theta: float64 device tensor)."""
        _check(lib().lsdd_update_theta(self._h, _dev_ptr(theta), _stream()))

    @classmethod
    def setup_problem(cls, prob, params=None, blocks_on_device=False):
        """Convenience: setup from an object with n/elem_ptr/elem_dofs/blocks/node_of_dof/agg_of_dof."""
        blocks = prob.blocks
        if blocks_on_device:
            import torch
            blocks = torch.from_numpy(np.ascontiguousarray(blocks)).cuda()
        return cls.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, blocks, prob.node_of_dof,
                                  prob.agg_of_dof, params)

    @classmethod
    def setup_batched(cls, problems, params=None):
        """lsdd_setup_batched over a list of problem objects (instance-local numbering);
        the union's DOFs are the instances' DOFs in list order."""
        probs = list(problems)
        inst_n = np.array([p.n for p in probs], dtype=np.int64)
        inst_ne = np.array([len(p.elem_ptr) - 1 for p in probs], dtype=np.int64)
        sizes = np.concatenate([np.diff(np.asarray(p.elem_ptr, dtype=np.int64)) for p in probs])
        elem_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        elem_dofs = np.ascontiguousarray(np.concatenate([np.asarray(p.elem_dofs) for p in probs]), dtype=np.int32)
        blocks = np.ascontiguousarray(np.concatenate([np.asarray(p.blocks) for p in probs]), dtype=np.float64)
        nod = None
        if all(p.node_of_dof is not None for p in probs):
            nod = np.ascontiguousarray(np.concatenate([p.node_of_dof for p in probs]), dtype=np.int32)
        agg = None
        if all(p.agg_of_dof is not None for p in probs):
            agg = np.ascontiguousarray(np.concatenate([p.agg_of_dof for p in probs]), dtype=np.int32)
        params = params or Params.default()
        h = C.c_void_p()
        _check(lib().lsdd_setup_batched(len(probs), _ptr(inst_n, C.c_int64), _ptr(inst_ne, C.c_int64),
                                        _ptr(elem_ptr, C.c_int64), _ptr(elem_dofs, C.c_int32),
                                        C.c_void_p(blocks.ctypes.data), _ptr(nod, C.c_int32), _ptr(agg, C.c_int32),
                                        0, C.byref(params), _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def setup_gram_csr(cls, m, n, rowptr, col, val, node_of_dof=None, agg_of_dof=None, params=None):
        """lsdd_setup_gram_csr.  rowptr/col/val are either host arrays or contiguous
        device tensors (int64, int32, float64), all three on the same side."""
        import torch
        dev = [isinstance(a, torch.Tensor) and a.is_cuda for a in (rowptr, col, val)]
        if any(dev) and not all(dev):
            raise TypeError("rowptr, col and val must all be host arrays or all device tensors")
        keep = []
        if all(dev):
            for a, dt in ((rowptr, torch.int64), (col, torch.int32), (val, torch.float64)):
                if a.dtype != dt or not a.is_contiguous():
                    raise TypeError("device CSR arrays: contiguous int64 rowptr, int32 col, float64 val")
            ptrs = [C.c_void_p(a.data_ptr()) for a in (rowptr, col, val)]
        else:
            keep = [np.ascontiguousarray(rowptr, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32),
                    np.ascontiguousarray(val, dtype=np.float64)]
            ptrs = [C.c_void_p(a.ctypes.data) for a in keep]
        nod = None if node_of_dof is None else np.ascontiguousarray(node_of_dof, dtype=np.int32)
        agg = None if agg_of_dof is None else np.ascontiguousarray(agg_of_dof, dtype=np.int32)
        params = params or Params.default()
        h = C.c_void_p()
        _check(lib().lsdd_setup_gram_csr(int(m), int(n), *ptrs, _ptr(nod, C.c_int32), _ptr(agg, C.c_int32),
                                         int(all(dev)), C.byref(params), _stream(), C.byref(h)))
        return cls(h)

    # ---------------------------------------------------------------- solve
    def solve(self, b, x=None, allow_noconv=False):
        """lsdd_solve for b of shape [n] or [nrhs, n]; returns (x, [Info]) with one
        Info per (right-hand side, segment), right-hand side major."""
        import torch
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if x is None:
            x = torch.empty_like(b)
        nseg = self.segments()[0]
        infos = (Info * (nrhs * nseg))()
        _check(lib().lsdd_solve(self._h, _dev_ptr(b), _dev_ptr(x), nrhs, _stream(), infos),
               allow=(5,) if allow_noconv else ())
        return x, [infos[i] for i in range(nrhs * nseg)]

    def solve_stationary(self, b, x0, allow_noconv=False):
        """lsdd_solve_stationary: x <- x + V(b - A x) from x0 (shape [n] or [nrhs, n],
        overwritten with the last iterates); returns (x, [Info]) per right-hand side."""
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        infos = (Info * nrhs)()
        _check(lib().lsdd_solve_stationary(self._h, _dev_ptr(b), _dev_ptr(x0), nrhs, _stream(), infos),
               allow=(5,) if allow_noconv else ())
        return x0, [infos[i] for i in range(nrhs)]

    def set_graph(self, on: bool):
        _check(lib().lsdd_set_graph(self._h, 1 if on else 0))

    def level_segments(self, level: int):
        """(inst_off list, terminal flags list) of one level."""
        ns = self.segments()[0]
        off = np.zeros(ns + 1, dtype=np.int64)
        term = np.zeros(ns, dtype=np.int32)
        _check(lib().lsdd_level_segments(self._h, int(level), off.ctypes.data_as(C.POINTER(C.c_int64)),
                                         term.ctypes.data_as(C.POINTER(C.c_int32))))
        return off.tolist(), term.tolist()

    def autotune(self, block: bool = False):
        """lsdd_autotune; returns the chosen shapes per level (lsdd_level_tuning)."""
        _check(lib().lsdd_autotune(self._h, 1 if block else 0, _stream()))
        return [self.level_tuning(l) for l in range(self.info()["levels"])]

    def level_tuning(self, level: int):
        out = np.zeros(7, dtype=np.int32)
        _check(lib().lsdd_level_tuning(self._h, int(level), out.ctypes.data_as(C.POINTER(C.c_int32))))
        return dict(lanes=int(out[0]), lanes_block=int(out[1]), tiles_per_item=int(out[2]), finalize_threads=int(out[3]),
                    elem_apply=int(out[4]), shared_cols=int(out[5]), fact_stash=int(out[6]))

    def set_level_tuning(self, level: int, t: dict):
        """lsdd_set_level_tuning with a dict as returned by level_tuning."""
        a = np.array([t["lanes"], t["lanes_block"], t["tiles_per_item"], t["finalize_threads"],
                      t.get("elem_apply", 0), t.get("shared_cols", 0), t.get("fact_stash", 1)], dtype=np.int32)
        _check(lib().lsdd_set_level_tuning(self._h, int(level), a.ctypes.data_as(C.POINTER(C.c_int32))))

    def set_tuning(self, tuning):
        """Apply a list of per-level shapes (the return value of autotune)."""
        for l, t in enumerate(tuning):
            self.set_level_tuning(l, t)

    def segments(self):
        """(n_seg, seg_off as a list)."""
        ns = C.c_int32()
        _check(lib().lsdd_segments(self._h, C.byref(ns), None))
        off = np.zeros(ns.value + 1, dtype=np.int64)
        _check(lib().lsdd_segments(self._h, None, off.ctypes.data_as(C.POINTER(C.c_int64))))
        return ns.value, off.tolist()

    def vcycle(self, r, z=None):
        import torch
        z = torch.empty_like(r) if z is None else z
        _check(lib().lsdd_vcycle(self._h, _dev_ptr(r), _dev_ptr(z), _stream()))
        return z

    def apply(self, x, level=0, y=None):
        import torch
        y = torch.empty_like(x) if y is None else y
        _check(lib().lsdd_apply(self._h, int(level), _dev_ptr(x), _dev_ptr(y), _stream()))
        return y

    def set_cycle_precision(self, precision: int):
        _check(lib().lsdd_set_cycle_precision(self._h, int(precision)))

    def set_solve_params(self, rtol: float, max_iter: int = 1000):
        _check(lib().lsdd_set_solve_params(self._h, float(rtol), int(max_iter)))

    def trace(self, on: bool):
        _check(lib().lsdd_trace(self._h, 1 if on else 0))

    def trace_read(self):
        out = {}
        i = 0
        while True:
            name = C.create_string_buffer(64)
            n, ms, by = C.c_int64(), C.c_double(), C.c_double()
            code = lib().lsdd_trace_get(self._h, i, name, 64, C.byref(n), C.byref(ms), C.byref(by))
            if code != 0:
                break
            out[name.value.decode()] = dict(launches=n.value, ms=ms.value, bytes=by.value)
            i += 1
        return out

    # ---------------------------------------------------------------- inspection
    def info(self):
        L = C.c_int32()
        n = np.zeros(16, np.int64)
        nnz = np.zeros(16, np.int64)
        oc, gc = C.c_double(), C.c_double()
        _check(lib().lsdd_hierarchy_info(self._h, C.byref(L), _ptr(n, C.c_int64), _ptr(nnz, C.c_int64),
                                         C.byref(oc), C.byref(gc)))
        return dict(levels=L.value, n=n[:L.value].tolist(), nnz=nnz[:L.value].tolist(), oc=oc.value, gc=gc.value)

    def level_sizes(self, level):
        s = np.zeros(8, np.int64)
        _check(lib().lsdd_level_sizes(self._h, int(level), _ptr(s, C.c_int64)))
        keys = ("n", "nnz", "n_agg", "z_len", "sub_len", "n_colors", "n_next", "n_elem")
        return dict(zip(keys, s.tolist()))

    def export_level(self, level):
        s = self.level_sizes(level)
        out = dict(sizes=s)
        rowptr = np.zeros(s["n"] + 1, np.int64)
        col = np.zeros(s["nnz"], np.int32)
        val = np.zeros(s["nnz"], np.float64)
        if s["n_agg"]:
            agg = np.zeros(s["n"], np.int32)
            k = np.zeros(s["n_agg"], np.int32)
            Z = np.zeros(max(s["z_len"], 1), np.float64)
            mu = np.zeros(s["n"], np.float64)
            colors = np.zeros(s["n_agg"], np.int32)
            osz = np.zeros(s["n_agg"], np.int32)
        else:
            agg = k = Z = mu = colors = osz = None
        _check(lib().lsdd_export_level(self._h, int(level), _ptr(agg, C.c_int32), _ptr(k, C.c_int32),
                                       _ptr(Z, C.c_double), _ptr(mu, C.c_double), _ptr(colors, C.c_int32),
                                       _ptr(rowptr, C.c_int64), _ptr(col, C.c_int32), _ptr(val, C.c_double),
                                       _ptr(osz, C.c_int32)))
        out.update(rowptr=rowptr, col=col, val=val, agg_of_dof=agg, k=k, Z=Z, mu=mu, colors=colors,
                   omega_sizes=osz)
        return out

    def export_gram(self, elem_ptr):
        sizes = np.diff(np.asarray(elem_ptr, np.int64))
        ranks = np.zeros(len(sizes), np.int32)
        G = np.zeros(int(np.sum(sizes * sizes)), np.float64)
        _check(lib().lsdd_export_gram(self._h, _ptr(ranks, C.c_int32), _ptr(G, C.c_double)))
        return ranks, G

    def export_gram_level(self, level, rows=True):
        """Element Gram factors of a level (level 0: as export_gram; coarse levels:
        re-factored rows of the grouped element blocks).  Returns a dict with
        elem_ptr, elem_dofs, ranks and G (each G_g row-major n_g x n_g, first
        ranks[g] rows the factor; None with rows=False)."""
        s = np.zeros(8, np.int64)
        _check(lib().lsdd_level_sizes(self._h, int(level), _ptr(s, C.c_int64)))
        ptr = np.zeros(int(s[7]) + 1, np.int64)
        _check(lib().lsdd_export_gram_level(self._h, int(level), _ptr(ptr, C.c_int64), None, None, None))
        sizes = np.diff(ptr)
        dofs = np.zeros(int(ptr[-1]), np.int32)
        ranks = np.zeros(len(sizes), np.int32)
        G = np.zeros(int(np.sum(sizes * sizes)), np.float64) if rows else None
        _check(lib().lsdd_export_gram_level(self._h, int(level), None, _ptr(dofs, C.c_int32),
                                            _ptr(ranks, C.c_int32), _ptr(G, C.c_double)))
        return dict(elem_ptr=ptr, elem_dofs=dofs, ranks=ranks, G=G)

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().lsdd_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


_ALLOC_CB = None


def set_torch_allocator(enable: bool = True):
    """Route the library's device allocations through torch's caching allocator."""
    global _ALLOC_CB
    import torch
    if not enable:
        lib().lsdd_set_allocator(None, None, None)
        _ALLOC_CB = None
        return
    AF = C.CFUNCTYPE(C.c_void_p, C.c_uint64, C.c_void_p)
    FF = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    _ALLOC_CB = (AF(_alloc), FF(_free))
    lib().lsdd_set_allocator(C.cast(_ALLOC_CB[0], C.c_void_p), C.cast(_ALLOC_CB[1], C.c_void_p), None)
