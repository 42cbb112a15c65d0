"""CPU-side checks of the C-ABI library: it loads, exports every declared entry
point, and rejects bad inputs during host validation (before any device call)."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lsdd.h")).read()
    return sorted(set(re.findall(r"\b(lsdd_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2607_07485_amd as P
    out = subprocess.run(["nm", "-D", "--defined-only", P.lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(lsdd_\w+)", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    assert len(_declared()) >= 13


def test_params_defaults_match_the_paper_settings():
    import paper_2607_07485_amd as P
    p = P.Params.default()
    assert (p.max_levels, p.agg_passes, p.min_coarse) == (3, 2, 10)
    assert p.max_density == 0.25 and p.tau_const == 0.75 and p.rtol == 1e-8


def _elems():
    import fegen
    return fegen.elasticity_q1(3, nu=0.3)


@pytest.mark.parametrize("mutate, msg", [
    (lambda p: p.elem_dofs.__setitem__(5, 10 ** 6), "out of range"),
    (lambda p: p.elem_dofs.__setitem__(1, p.elem_dofs[0]), "repeated DOF"),
])
def test_setup_rejects_bad_indices_before_any_device_call(mutate, msg):
    import paper_2607_07485_amd as P
    prob = _elems()
    prob.elem_dofs = prob.elem_dofs.copy()
    mutate(prob)
    with pytest.raises(P.LsddError) as ei:
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, prob.blocks, prob.node_of_dof,
                                   prob.agg_of_dof)
    assert ei.value.code == 1 and msg in str(ei.value)


def test_setup_rejects_uncovered_dof_and_bad_aggregates():
    import paper_2607_07485_amd as P
    prob = _elems()
    with pytest.raises(P.LsddError, match="belongs to no element"):
        P.Hierarchy.setup_elements(prob.n + 1, prob.elem_ptr, prob.elem_dofs, prob.blocks)
    agg = prob.agg_of_dof.copy()
    agg[agg == 0] = 7 + agg.max()           # leaves id 0 unused
    with pytest.raises(P.LsddError, match="aggregate ids"):
        P.Hierarchy.setup_elements(prob.n, prob.elem_ptr, prob.elem_dofs, prob.blocks, prob.node_of_dof, agg)


def test_batched_setup_validates_instance_local_indices():
    """A DOF index valid in the union but outside its own instance is rejected."""
    import copy

    import paper_2607_07485_amd as P
    a, b = _elems(), _elems()
    bad = copy.copy(b)
    bad.elem_dofs = b.elem_dofs.copy()
    bad.elem_dofs[3] = b.n + 2                   # would land in the next instance's range
    with pytest.raises(P.LsddError, match="instance's range"):
        P.Hierarchy.setup_batched([a, bad, _elems()])
    agg = b.agg_of_dof.copy()
    agg[agg == 0] = 5 + agg.max()
    bad2 = copy.copy(b)
    bad2.agg_of_dof = agg
    with pytest.raises(P.LsddError, match="aggregate ids of an instance"):
        P.Hierarchy.setup_batched([a, bad2])


def test_gram_csr_setup_validates_the_pattern_on_the_host():
    """Black-box CSR G: rowptr not starting at 0, a column index out of range, an
    empty column (A singular) and a row above 128 entries are refused before any
    device call."""
    import paper_2607_07485_amd as P
    n = 4
    rp = np.array([0, 2, 4], np.int64)
    col = np.array([0, 1, 2, 3], np.int32)
    val = np.ones(4)
    with pytest.raises(P.LsddError, match="start at 0"):
        P.Hierarchy.setup_gram_csr(2, n, rp + 1, col, np.ones(5))
    with pytest.raises(P.LsddError, match="out of range"):
        P.Hierarchy.setup_gram_csr(2, n, rp, np.array([0, 1, 2, 9], np.int32), val)
    with pytest.raises(P.LsddError, match="column 3 of G is empty") as ei:
        P.Hierarchy.setup_gram_csr(2, n, np.array([0, 2, 3], np.int64), col[:3], val[:3])
    assert ei.value.code == 1
    with pytest.raises(P.LsddError, match="more than 128") as ei:
        P.Hierarchy.setup_gram_csr(1, 129, np.array([0, 129], np.int64), np.arange(129, dtype=np.int32),
                                   np.ones(129))
    assert ei.value.code == 7


def test_params_struct_layout_matches_the_header(tmp_path):
    """The binding's Params mirrors lsdd_params field by field (offsets and size)."""
    import ctypes

    import paper_2607_07485_amd as P
    fields = [f for f, _ in P.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lsdd.h"\nint main(void) {\n'
                   + "".join(f'printf("%zu\\n", offsetof(lsdd_params, {f}));\n' for f in fields)
                   + 'printf("%zu\\n", sizeof(lsdd_params));\nreturn 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [getattr(P.Params, f).offset for f in fields] + [ctypes.sizeof(P.Params)]
    assert got == want
