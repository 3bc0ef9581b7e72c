"""MI355X-native matrix-free finite element operator decomposition with
quadrature-point forward-mode AD (regularised p-Laplacian, hexahedral Q_k).

All computation runs in the HIP library ``_lib/libfeod.so`` behind the C ABI
``include/feod.h``; this package only marshals arguments.
"""
from .feod import (FeodError, HostSetup, Problem, adjoint_gradient, default_opts,  # noqa: F401
                   header_functions, jacobian_apply, lib, newton_solve, residual, setup_mesh)
from .design import DesignSolve  # noqa: F401
