"""ORACLE (test infrastructure only) -- Newton and adjoint solves with direct
sparse linear algebra.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything under ``oracle/``.

* Newton on R(u) = 0 (paper, Eq. (1)-(2)): the Jacobian of Eq. (3) is
  assembled and solved exactly (``spsolve``) on the interior rows; the step is
  damped by Armijo backtracking on the energy E(u) (c = 1e-4, halving, at most
  30 halvings).  When the predicted decrease is below the rounding level of E
  the full step is taken.  The iteration starts from the p = 2 (Poisson)
  solution u2 scaled by the alpha > 0 that minimises the energy E(alpha u2)
  along its ray (a reading: the paper gives no starting point), and stops
  when ||R(u)||_2 <= tol ||M b||_2.
* Adjoint (the design paragraph after Eq. (3)): J(u) lambda = M dPhi/du on the
  interior (J is symmetric), then the per-element gradient
  dPhi/drho = -lambda^T dR/drho.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import Discretisation


def _interior_solve(disc: Discretisation, K, rhs):
    inner = disc.mask > 0
    x = np.zeros(disc.N)
    x[inner] = spla.spsolve(K[inner][:, inner].tocsc(), rhs[inner])
    return x


def poisson_solution(disc: Discretisation):
    """Solve the p = 2 problem K u = M b (the Newton starting point)."""
    lin = disc.with_(p=2.0)
    return _interior_solve(lin, lin.jacobian(np.zeros(disc.N)), disc.mask * disc.b)


def scaled_start(disc: Discretisation, u2, max_steps=8):
    """alpha u2 with alpha > 0 minimising phi(alpha) = E(alpha u2).  phi is
    convex with phi'(alpha) = u2 . R(alpha u2) (R is the gradient of E) and
    phi''(alpha) = u2 . J(alpha u2) u2; Newton steps on phi' = 0 until the
    change is below 1e-3 alpha (halving instead of leaving alpha > 0)."""
    if disc.p == 2.0:
        return u2
    alpha = 1.0
    for _ in range(max_steps):
        g = float(np.dot(u2, disc.residual(alpha * u2)))
        h = float(np.dot(u2, disc.jvp(alpha * u2, u2)))
        if not (h > 0) or not np.isfinite(g):
            break
        nxt = alpha - g / h
        if not nxt > 0:
            nxt = 0.5 * alpha
        done = abs(nxt - alpha) <= 1e-3 * alpha
        alpha = nxt
        if done:
            break
    return alpha * u2


def newton(disc: Discretisation, u0=None, tol=1e-10, max_newton=60, c_armijo=1e-4,
           max_halvings=30):
    """Damped Newton with exact linear solves.  Returns (u, info)."""
    u = scaled_start(disc, poisson_solution(disc)) if u0 is None else disc.mask * np.asarray(u0, float)
    ref = np.linalg.norm(disc.mask * disc.b)
    history = []
    for it in range(max_newton + 1):
        R = disc.residual(u)
        nr = np.linalg.norm(R)
        history.append(nr)
        if nr <= tol * ref:
            return u, {"iters": it, "res": nr, "ref": ref, "history": history}
        if it == max_newton:
            break
        du = _interior_solve(disc, disc.jacobian(u), -R)
        E0 = disc.energy(u)
        slope = float(np.dot(R, du))
        t = 1.0
        if abs(slope) > 1e-13 * max(abs(E0), 1e-300):
            for _ in range(max_halvings):
                if disc.energy(u + t * du) <= E0 + c_armijo * t * slope:
                    break
                t *= 0.5
        u = u + t * du
    raise RuntimeError(f"oracle Newton did not converge: {history}")


def adjoint(disc: Discretisation, u, g_u):
    """lambda with J(u) lambda = M g_u, and dPhi/drho = -lambda^T dR/drho."""
    lam = _interior_solve(disc, disc.jacobian(u), disc.mask * np.asarray(g_u, float))
    return lam, disc.grad_rho(u, lam)
