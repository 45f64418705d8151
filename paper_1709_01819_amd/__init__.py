"""MI355X (gfx950) implicit DUGKS (arXiv:1709.01819): HIP kernels behind a C ABI.

``Solver`` wraps ``libidugks.so`` (built by ``paper_1709_01819_amd.build.build()``);
PyTorch only provides the device workspace and the HIP stream.
"""
from .abi import (  # noqa: F401
    BC_WALL, BC_FARFIELD, BC_PERIODIC, GAUSS_HERMITE, NEWTON_COTES, BGK, SHAKHOV, FP64,
    FP32_MIXED, EXPLICIT, IMPLICIT, IdugksError, load_library, library_path,
)
from .solver import Solver  # noqa: F401
