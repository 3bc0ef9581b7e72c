"""ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU implementation of the matrix-free finite element
operator decomposition (paper, Fig. 1, Eq. (1)-(3)) for the regularised
p-Laplacian on hexahedral Q_k meshes, with a hand-derived analytic
linearisation, direct-solve Newton and adjoint design gradient.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything under ``oracle/``; the
product path never does.  It shares no code with the HIP path.
"""
from .rules import gauss_legendre, gll_nodes, lagrange  # noqa: F401
from .fem import Discretisation  # noqa: F401
from .solve import adjoint, newton, poisson_solution  # noqa: F401
