"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module draws random numbers and lays out plain lattices; it holds none of
the finite element method's arithmetic (no basis, quadrature, geometry or
operator code), so that the oracle and the HIP path can both consume the same
arrays without sharing any code of the method.

Workloads (the p-Laplacian problems the design study is run on):

=====  =========  ===  ====  =====  =====  =========================================
name   mesh       k    nq    p      eps    extras
=====  =========  ===  ====  =====  =====  =========================================
c1     4^3        2    3     3      1e-2   residual+JVP, Newton-CG
c2     32^3       3    5     4      1e-3   100 residual + 100 JVP, Newton-CG
c3     64^3       4    6     2.5    1e-2   JVP throughput FP64 vs mixed
c4     48^3       2    3     3      1e-2   per-element rho ~ U(0.1, 1), adjoint design
c5     16^3       7    9     3      1e-2   interior vertices perturbed by U(-0.1h, 0.1h)
=====  =========  ===  ====  =====  =====  =========================================

Draw order from ``numpy.random.default_rng(seed)`` (PCG64): vertex
perturbation (interior vertices, x fastest, 3 coordinates each), rho, u, v,
then the finite-difference element sample.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    k: int
    nq: int
    p: float
    eps: float
    seed: int
    perturb: bool = False      # perturb interior vertices by U(-0.1h, 0.1h)
    rho: bool = False          # per-element coefficient ~ U(0.1, 1)
    n_fd: int = 0              # elements sampled for finite-difference checks
    note: str = ""

    @property
    def n_elems(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def lattice(self) -> tuple[int, int, int]:
        return (self.k * self.nx + 1, self.k * self.ny + 1, self.k * self.nz + 1)

    @property
    def n_dofs(self) -> int:
        lx, ly, lz = self.lattice
        return lx * ly * lz

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS: dict[str, Workload] = {
    "c1": Workload("c1", 4, 4, 4, 2, 3, 3.0, 1e-2, 1,
                   note="p=3 eps=1e-2, 4^3 hex, Q2, 3^3 Gauss points, FP64"),
    "c2": Workload("c2", 32, 32, 32, 3, 5, 4.0, 1e-3, 2,
                   note="p=4 eps=1e-3, 32^3 hex, Q3, 5^3 Gauss points"),
    "c3": Workload("c3", 64, 64, 64, 4, 6, 2.5, 1e-2, 3,
                   note="p=2.5 eps=1e-2, 64^3 hex, Q4, 6^3 Gauss points"),
    "c4": Workload("c4", 48, 48, 48, 2, 3, 3.0, 1e-2, 4, rho=True, n_fd=20,
                   note="p=3 eps=1e-2, 48^3 hex, Q2, rho~U(0.1,1), compliance"),
    "c5": Workload("c5", 16, 16, 16, 7, 9, 3.0, 1e-2, 5, perturb=True,
                   note="p=3 eps=1e-2, 16^3 curved hex, Q7, 9^3 Gauss points"),
}


def lattice_vertices(nx: int, ny: int, nz: int) -> np.ndarray:
    """Vertices of the uniform nx*ny*nz lattice of the unit cube, x fastest,
    shape ((nx+1)(ny+1)(nz+1), 3)."""
    x = np.arange(nx + 1) / nx
    y = np.arange(ny + 1) / ny
    z = np.arange(nz + 1) / nz
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def make_inputs(w: Workload) -> dict:
    """All seeded arrays of a workload, drawn once in the documented order.

    Returns a dict with ``vertices`` (None for the uniform lattice), ``rho``
    (None when the coefficient is 1), ``u`` and ``v`` (length n_dofs, U(-1,1))
    and ``fd_elems`` (sorted element indices, possibly empty).
    """
    rng = np.random.default_rng(w.seed)
    out: dict = {"vertices": None, "rho": None}
    if w.perturb:
        verts = lattice_vertices(w.nx, w.ny, w.nz)
        hx = np.array([1.0 / w.nx, 1.0 / w.ny, 1.0 / w.nz])
        ni = (w.nx - 1) * (w.ny - 1) * (w.nz - 1)
        d = rng.uniform(-0.1, 0.1, size=(ni, 3)) * hx
        iz, iy, ix = np.meshgrid(np.arange(1, w.nz), np.arange(1, w.ny),
                                 np.arange(1, w.nx), indexing="ij")
        idx = (ix + (w.nx + 1) * (iy + (w.ny + 1) * iz)).ravel()
        verts[idx] += d
        out["vertices"] = verts
    if w.rho:
        out["rho"] = rng.uniform(0.1, 1.0, size=w.n_elems)
    out["u"] = rng.uniform(-1.0, 1.0, size=w.n_dofs)
    out["v"] = rng.uniform(-1.0, 1.0, size=w.n_dofs)
    if w.n_fd:
        out["fd_elems"] = np.sort(rng.choice(w.n_elems, w.n_fd, replace=False))
    else:
        out["fd_elems"] = np.zeros(0, dtype=np.int64)
    return out
