"""Pins of the oracle's Newton and adjoint solves: manufactured solution
rates, cube symmetry, the Poisson series, the p = 2 compliance sensitivity and
finite differences of the design objective."""
import itertools

import numpy as np
import pytest

from oracle import Discretisation, adjoint, newton
from tests.oracle_helpers import relerr
from workloads import WORKLOADS, Workload, make_inputs


def _mms(p, eps):
    """u* = sin(pi x) sin(pi y) sin(pi z) and the load f* = -div(a*^r grad u*)."""
    r = (p - 2) / 2
    pi = np.pi

    def ustar(x, y, z):
        return np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)

    def fstar(x, y, z):
        sx, sy, sz = np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)
        cx, cy, cz = np.cos(pi * x), np.cos(pi * y), np.cos(pi * z)
        g = np.stack([pi * cx * sy * sz, pi * sx * cy * sz, pi * sx * sy * cz], -1)
        H = np.empty(x.shape + (3, 3))
        H[..., 0, 0] = H[..., 1, 1] = H[..., 2, 2] = -pi * pi * sx * sy * sz
        H[..., 0, 1] = H[..., 1, 0] = pi * pi * cx * cy * sz
        H[..., 0, 2] = H[..., 2, 0] = pi * pi * cx * sy * cz
        H[..., 1, 2] = H[..., 2, 1] = pi * pi * sx * cy * cz
        a = eps ** 2 + np.sum(g * g, -1)
        lap = np.trace(H, axis1=-2, axis2=-1)
        gHg = np.einsum("...i,...ij,...j->...", g, H, g)
        return -(a ** r * lap + (p - 2) * a ** (r - 1) * gHg)

    return ustar, fstar


def _l2_error(d, u, ustar, nq_hi=8):
    hi = Discretisation(d.nx, d.ny, d.nz, d.k, nq_hi, d.p, d.eps, vertices=d.vertices,
                        load=np.zeros(d.N))
    elems = np.arange(d.E)
    _, detJ, _, xq = hi.geometry(elems)
    uq = hi.gather(u, elems) @ hi.Bval.T
    us = ustar(xq[..., 0], xq[..., 1], xq[..., 2])
    return np.sqrt(np.sum(hi.w * detJ * (uq - us) ** 2))


@pytest.mark.parametrize("k,nq,expect", [(1, 2, 2.0), (2, 3, 3.0)])
def test_manufactured_solution_rates(k, nq, expect):
    p, eps = 3.0, 1e-2
    ustar, fstar = _mms(p, eps)
    errs = []
    ns = [2, 4, 8]
    for n in ns:
        d = Discretisation(n, n, n, k, nq, p, eps, f=fstar)
        u, _ = newton(d, tol=1e-11)
        errs.append(_l2_error(d, u, ustar))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > expect - 0.3, (errs, rates)
    assert rates[-1] < expect + 0.6, (errs, rates)


@pytest.mark.slow
def test_manufactured_solution_rate_curved_q2():
    p, eps = 2.5, 1e-2
    ustar, fstar = _mms(p, eps)
    errs = []
    for n in [2, 4, 8]:
        w = Workload("m", n, n, n, 2, 3, p, eps, 9, perturb=True)
        d = Discretisation(n, n, n, 2, 3, p, eps, vertices=make_inputs(w)["vertices"], f=fstar)
        u, _ = newton(d, tol=1e-11)
        errs.append(_l2_error(d, u, ustar))
    rate = np.log2(errs[1] / errs[2])
    assert 2.6 < rate < 3.6, errs


def test_newton_c1_cube_symmetry():
    w = WORKLOADS["c1"]
    d = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps)
    u, info = newton(d)
    assert info["res"] <= 1e-10 * info["ref"]
    assert np.linalg.norm(d.residual(u)) <= 1e-10 * np.linalg.norm(d.mask * d.b)
    U = u.reshape(d.Lz, d.Ly, d.Lx)
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product([False, True], repeat=3):
            V = np.transpose(U, perm)
            for ax, f in enumerate(flips):
                if f:
                    V = np.flip(V, axis=ax)
            assert np.abs(V - U).max() <= 1e-12 * np.abs(U).max()


def test_p2_one_newton_step_and_poisson_series():
    n = 8
    d = Discretisation(n, n, n, 2, 3, 2.0, 1e-2)
    u, info = newton(d, u0=np.zeros(d.N), tol=1e-12)
    assert info["iters"] == 1
    # centre value of -lap u = 1 on the unit cube, Fourier series
    m = np.arange(1, 400, 2)
    L, M_, N_ = np.meshgrid(m, m, m, indexing="ij", sparse=True)
    sgn = (-1.0) ** ((L - 1) // 2 + (M_ - 1) // 2 + (N_ - 1) // 2)
    series = np.sum(64 * sgn / (np.pi ** 5 * L * M_ * N_ * (L ** 2 + M_ ** 2 + N_ ** 2)))
    centre = u[(d.Lx // 2) + d.Lx * ((d.Ly // 2) + d.Ly * (d.Lz // 2))]
    assert abs(series - 0.0562) < 1e-3
    assert abs(centre - series) < 2e-4 * series


def test_p2_adjoint_is_compliance_sensitivity():
    w = Workload("a", 3, 2, 3, 2, 3, 2.0, 1e-2, 4, rho=True, perturb=True)
    inp = make_inputs(w)
    d = Discretisation(3, 2, 3, 2, 3, 2.0, 1e-2, vertices=inp["vertices"], rho=inp["rho"])
    u, _ = newton(d, tol=1e-13)
    lam, grad = adjoint(d, u, d.b)
    assert relerr(lam, u) < 1e-12
    # -int_e |grad u|^2, evaluated here from nodal gradients of u
    elems = np.arange(d.E)
    _, detJ, Jinv, _ = d.geometry(elems)
    gref = np.stack([d.gather(u, elems) @ d.Bgrad[i].T for i in range(3)], -1)
    gphys = np.linalg.solve(np.swapaxes(np.linalg.inv(Jinv), -1, -2), gref[..., None])[..., 0]
    expect = -np.sum(d.w * detJ * np.sum(gphys ** 2, -1), axis=1)
    assert relerr(grad, expect) < 1e-12


def test_adjoint_gradient_matches_central_differences():
    w = Workload("a", 3, 3, 2, 2, 3, 3.0, 1e-2, 4, rho=True, perturb=True)
    inp = make_inputs(w)
    d = Discretisation(3, 3, 2, 2, 3, 3.0, 1e-2, vertices=inp["vertices"], rho=inp["rho"])
    u, _ = newton(d, tol=1e-14)
    _, grad = adjoint(d, u, d.b)
    rng = np.random.default_rng(0)
    for e in rng.choice(d.E, 5, replace=False):
        h = 1e-3 * d.rho[e]
        phis = []
        for s in (+1, -1):
            rho = d.rho.copy()
            rho[e] += s * h
            dd = d.with_(rho=rho)
            us, _ = newton(dd, u0=u, tol=1e-14)
            phis.append(np.dot(d.b, us))
        fd = (phis[0] - phis[1]) / (2 * h)
        assert abs(fd - grad[e]) <= 1e-5 * abs(grad[e]), (e, fd, grad[e])
    # one random direction over all rho
    dr = rng.uniform(-1, 1, d.E) * d.rho
    h = 1e-4
    phis = []
    for s in (+1, -1):
        dd = d.with_(rho=d.rho + s * h * dr)
        us, _ = newton(dd, u0=u, tol=1e-14)
        phis.append(np.dot(d.b, us))
    fd = (phis[0] - phis[1]) / (2 * h)
    assert abs(fd - grad @ dr) <= 1e-7 * abs(grad @ dr)
