"""MI355X-native LS-AMG-DD hot path: C-ABI library liblsdd.so plus a thin binding.

Every numerical step of setup and solve runs in the library's HIP kernels; this
package only marshals arguments (PyTorch supplies device memory and streams).
"""
from .lsdd import (  # noqa: F401
    LSDD_STATUS, Hierarchy, LsddError, Params, elem_bilinear, lib, lib_path, set_torch_allocator, solve_batched,
)
