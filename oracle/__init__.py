"""FP64 CPU oracle for the LS-AMG-DD hot path.

Test infrastructure only: imported by the tests, by the smoke entry point and by
the benchmark's CPU-baseline leg, never by the library or its Python binding.
"""
from .lsdd import (  # noqa: F401
    EPS, Hierarchy, Level, NotSPSD, Params, SolveInfo, assemble, closures, coarse_gram_factors, coloring,
    element_gram_factor, hierarchy_stats, local_spectral, local_splitting, pcg,
    schur_pinv, select_modes, setup, standard_aggregation, stationary, structural_pattern,
    supernode_graph, vcycle,
)
from .adjoint import (  # noqa: F401,E402
    adjoint_gradient, assemble_scaled, compliance_gradient, element_bilinear,
)
