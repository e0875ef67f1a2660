"""MI355X-native batched safety filter of Swarm-Gen (arXiv 2501.19042).

The solver runs in the HIP kernels of libswarmsf.so (C ABI in include/swarmsf.h);
this package marshals PyTorch device buffers and streams into that ABI.
"""
from .sf import (Batch, ProjectResult, SafetyFilter, factor_table, project_differentiable,  # noqa: F401
                 qp_equality, qp_equality_differentiable)
from . import _native  # noqa: F401
