"""Tolerances taken from the oracle's own rounding spread.

The Schur complement of eq. (gep_reduced) has two FP64 routes in the oracle: the
Moore-Penrose pseudo-inverse of A~_GammaGamma by its eigendecomposition (the
default, reading R4) and the equivalent projector form on the weighted Gram rows
(the same rank rule on the squared singular values).  They are equal in exact
arithmetic, so their distance in a computed quantity is what rounding alone does
to that quantity on the problem at hand.  Where interface blocks are singular or
ill-conditioned this distance exceeds 1e-10, and a GPU result is then held to ten
times it (never less than 1e-10), as for the local spectra at the benchmark sizes.
"""
import numpy as np

import oracle

FLOOR = 1e-10
FACTOR = 10.0


def oracle_routes(prob, **kw):
    """Hierarchies of both routes; asserts that they agree in every integer decision
    (level sizes, aggregates, retained-mode counts), so their outputs are comparable."""
    h = oracle.setup(prob, oracle.Params(**kw))
    h2 = oracle.setup(prob, oracle.Params(interface="projector", **kw))
    assert [lv.n for lv in h.levels] == [lv.n for lv in h2.levels]
    for a, b in zip(h.levels[:-1], h2.levels[:-1]):
        assert np.array_equal(a.agg_of_dof, b.agg_of_dof) and np.array_equal(a.k, b.k)
    return h, h2


def rel(a, b):
    """Relative 2-norm distance of a from the reference b."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def tol_from(q_ref, q_other, floor=FLOOR, factor=FACTOR):
    """Relative tolerance for a quantity whose two oracle routes give q_ref and q_other."""
    return max(floor, factor * rel(q_other, q_ref))


def mu_tol(h, h2, floor=FLOOR, factor=FACTOR):
    """Absolute tolerance for the local spectra (mu in [0, 1]) on every coarsened level."""
    d = max((float(np.abs(np.concatenate(a.mu) - np.concatenate(b.mu)).max())
             for a, b in zip(h.levels[:-1], h2.levels[:-1])), default=0.0)
    return max(floor, factor * d)
