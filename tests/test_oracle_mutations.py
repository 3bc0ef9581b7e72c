"""Planted mistakes in the oracle (on the CPU) must each fail a pin.

Each case swaps one oracle function for a plausible wrong version and checks
that the pin designed to catch it now fails; this shows the pins constrain
every piece of the oracle, not only its overall shape.
"""
import numpy as np
import pytest

import oracle.fem as fem
from oracle import Discretisation, gll_nodes
from tests.oracle_helpers import kronecker_laplacian, relerr
from workloads import Workload, make_inputs


def _fd_jvp_error():
    w = Workload("t", 2, 2, 3, 2, 3, 3.0, 1e-2, 11, perturb=True, rho=True)
    inp = make_inputs(w)
    d = Discretisation(2, 2, 3, 2, 3, 3.0, 1e-2, vertices=inp["vertices"], rho=inp["rho"])
    u, v = 0.5 * inp["u"], inp["v"]
    h = 1e-6 * np.linalg.norm(u) / np.linalg.norm(v)
    fd = (d.residual(u + h * v) - d.residual(u - h * v)) / (2 * h)
    return relerr(d.jvp(u, v), fd)


def _fd_energy_error():
    w = Workload("t", 2, 2, 2, 2, 3, 2.5, 1e-2, 12, perturb=True)
    inp = make_inputs(w)
    d = Discretisation(2, 2, 2, 2, 3, 2.5, 1e-2, vertices=inp["vertices"])
    u = 0.3 * inp["u"]
    R = d.residual(u)
    fd = np.zeros(d.N)
    for i in np.nonzero(d.mask)[0]:
        e = np.zeros(d.N)
        e[i] = 1e-5
        fd[i] = (d.energy(u + e) - d.energy(u - e)) / 2e-5
    return relerr(fd, R)


def _fd_jvp_eps0_error():
    """Central differences of R at eps = 0, p = 3.5, with u zero on half of
    the mesh (zero gradient there: the a = 0 limit of the tangent is used;
    the formula itself gives 0^(-1/4) * 0)."""
    w = Workload("t", 4, 2, 2, 2, 3, 3.5, 0.0, 13, rho=True)
    inp = make_inputs(w)
    d = Discretisation(4, 2, 2, 2, 3, 3.5, 0.0, rho=inp["rho"])
    I = np.arange(d.N) % d.Lx
    u, v = np.where(I < d.Lx // 2, 0.0, 0.5 * inp["u"]), inp["v"]
    h = 1e-6 * np.linalg.norm(u) / np.linalg.norm(v)
    fd = (d.residual(u + h * v) - d.residual(u - h * v)) / (2 * h)
    return relerr(d.jvp(u, v), fd)


def _patch_error():
    w = Workload("t", 3, 2, 3, 2, 3, 3.0, 1e-2, 7, perturb=True)
    d = Discretisation(3, 2, 3, 2, 3, 3.0, 1e-2, vertices=make_inputs(w)["vertices"])
    x = d.node_coordinates()
    A = d.apply_full(0.7 * x[:, 0] - 1.3 * x[:, 1] + 0.4 * x[:, 2] + 2.0)
    scale = np.abs(d.apply_full(np.random.default_rng(1).uniform(-1, 1, d.N))).max()
    return np.abs(A[d.mask > 0]).max() / scale


def _kron_error():
    d = Discretisation(2, 3, 4, 2, 3, 2.0, 0.0)
    K, b = kronecker_laplacian(gll_nodes(2), 2, 3, 4)
    u = np.random.default_rng(3).uniform(-1, 1, d.N)
    return relerr(d.residual(u), d.mask * (K @ (d.mask * u) - b))


PINS = {"fd_jvp": (_fd_jvp_error, 1e-7), "fd_jvp_eps0": (_fd_jvp_eps0_error, 1e-7), "fd_energy": (_fd_energy_error, 1e-7),
        "patch": (_patch_error, 1e-13), "kron": (_kron_error, 1e-12)}


def _bad_tangent_no_p2(g, p, eps):
    a = eps * eps + np.sum(g * g, axis=-1)
    return (a ** ((p - 2) / 2))[..., None, None] * np.eye(3)


def _bad_tangent_sign(g, p, eps):
    r = (p - 2.0) / 2.0
    a = eps * eps + np.sum(g * g, axis=-1)
    T = a[..., None, None] * np.eye(3) - (p - 2.0) * g[..., :, None] * g[..., None, :]
    return (a ** (r - 1.0))[..., None, None] * T


def _bad_tangent_limit(g, p, eps):           # identity at a = 0 whatever p (the p = 2 limit)
    r = (p - 2.0) / 2.0
    a = eps * eps + np.sum(g * g, axis=-1)
    T = a[..., None, None] * np.eye(3) + (p - 2.0) * g[..., :, None] * g[..., None, :]
    out = (np.where(a == 0, 1.0, a) ** (r - 1.0))[..., None, None] * T
    out[a == 0] = np.eye(3)
    return out


def _bad_tangent_no_limit(g, p, eps):         # the formula as written: 0^(r-1) * 0 = nan at a = 0
    r = (p - 2.0) / 2.0
    a = eps * eps + np.sum(g * g, axis=-1)
    T = a[..., None, None] * np.eye(3) + (p - 2.0) * g[..., :, None] * g[..., None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        return (a ** (r - 1.0))[..., None, None] * T


def _bad_physical_gradient(Jinv, ghat):       # Jg^{-1} instead of Jg^{-T}
    return np.einsum("...ab,...b->...a", Jinv, ghat)


def _bad_pull_back(Jinv, F):                  # Jg^{-T} instead of Jg^{-1}
    return np.einsum("...ba,...b->...a", Jinv, F)


def _bad_flux_exponent(g, p, eps):
    a = eps * eps + np.sum(g * g, axis=-1)
    return (a ** (p / 2.0))[..., None] * g


def _bad_energy_density(g, p, eps):
    a = eps * eps + np.sum(g * g, axis=-1)
    return a ** (p / 2.0) / 2.0


MUTANTS = [
    ("tangent_matrix", _bad_tangent_no_p2, "fd_jvp"),
    ("tangent_matrix", _bad_tangent_sign, "fd_jvp"),
    ("tangent_matrix", _bad_tangent_limit, "fd_jvp_eps0"),
    ("tangent_matrix", _bad_tangent_no_limit, "fd_jvp_eps0"),
    ("physical_gradient", _bad_physical_gradient, "patch"),
    ("pull_back", _bad_pull_back, "patch"),
    ("flux", _bad_flux_exponent, "fd_energy"),
    ("energy_density", _bad_energy_density, "fd_energy"),
]


@pytest.mark.parametrize("name,bad,pin", MUTANTS, ids=[f"{m[0]}-{m[2]}-{i}" for i, m in enumerate(MUTANTS)])
def test_planted_mistake_fails_its_pin(monkeypatch, name, bad, pin):
    fn, tol = PINS[pin]
    assert fn() < tol                    # the true oracle passes
    monkeypatch.setattr(fem, name, bad)
    err = fn()
    assert not err <= 10 * tol           # the planted mistake fails (or gives nan)


def test_swapped_gradient_axes_fail_kronecker(monkeypatch):
    fn, tol = PINS["kron"]
    orig = Discretisation.__init__

    def init(self, *a, **kw):
        orig(self, *a, **kw)
        self.Bgrad = self.Bgrad[[1, 0, 2]]
    monkeypatch.setattr(Discretisation, "__init__", init)
    assert fn() > 10 * tol


def test_missing_detj_fails_kronecker(monkeypatch):
    fn, tol = PINS["kron"]
    orig = Discretisation.geometry

    def geometry(self, elems):
        Jg, detJ, Jinv, xq = orig(self, elems)
        return Jg, np.ones_like(detJ), Jinv, xq
    monkeypatch.setattr(Discretisation, "geometry", geometry)
    assert fn() > 10 * tol
