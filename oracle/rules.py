"""ORACLE (test infrastructure only) -- one-dimensional rules on [0, 1].

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything under ``oracle/``.  It shares no code with the
HIP path.

Hexahedral Q_k elements use a nodal (Lagrange) basis on the k+1 Gauss-Lobatto
(GLL) points and tensor-product Gauss-Legendre quadrature; the paper's operator
B (Section "Automatic differentiation in finite element analysis", Fig. 1) maps
element DOFs to values/gradients at those quadrature points.  The 1D pieces:

* GLL nodes: the two endpoints and the roots of P_k', mapped x -> (x+1)/2.
* Gauss-Legendre points/weights: numpy's ``leggauss``, mapped, weights halved.
* Lagrange values L[q, a] = prod_{b != a} (x_q - xi_b)/(xi_a - xi_b) and their
  derivatives by the product rule.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k: int) -> np.ndarray:
    """The k+1 Gauss-Lobatto-Legendre nodes on [0, 1], ascending."""
    if k < 1:
        raise ValueError("k >= 1 required")
    if k == 1:
        x = np.array([-1.0, 1.0])
    else:
        dPk = npleg.Legendre.basis(k).deriv()
        inner = np.sort(np.real(dPk.roots()))
        x = np.concatenate([[-1.0], inner, [1.0]])
    return (x + 1.0) / 2.0


def gauss_legendre(nq: int) -> tuple[np.ndarray, np.ndarray]:
    """nq-point Gauss-Legendre rule on [0, 1]: (points ascending, weights)."""
    x, w = npleg.leggauss(nq)
    order = np.argsort(x)
    return (x[order] + 1.0) / 2.0, w[order] / 2.0


def lagrange(nodes: np.ndarray, pts: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Lagrange basis on ``nodes`` evaluated at ``pts``.

    Returns (L, dL) with L[q, a] = l_a(pts[q]) and dL[q, a] = l_a'(pts[q]).
    Written as the product formula and its product-rule derivative.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    n = len(nodes)
    L = np.ones((len(pts), n))
    dL = np.zeros((len(pts), n))
    for a in range(n):
        others = [b for b in range(n) if b != a]
        for b in others:
            L[:, a] *= (pts - nodes[b]) / (nodes[a] - nodes[b])
        for m in others:
            term = np.full(len(pts), 1.0 / (nodes[a] - nodes[m]))
            for b in others:
                if b != m:
                    term *= (pts - nodes[b]) / (nodes[a] - nodes[b])
            dL[:, a] += term
    return L, dL
