"""Pins of the oracle's operators against closed forms, invariants and finite
differences (nothing here re-types the oracle's own formulas)."""
import numpy as np
import pytest

from oracle import Discretisation, gll_nodes
from tests.oracle_helpers import kronecker_laplacian, relerr
from workloads import Workload, make_inputs


def _disc(nx, ny, nz, k, nq, p, eps, perturb=False, rho=False, seed=11, **kw):
    w = Workload("t", nx, ny, nz, k, nq, p, eps, seed, perturb=perturb, rho=rho)
    inp = make_inputs(w)
    return Discretisation(nx, ny, nz, k, nq, p, eps, vertices=inp["vertices"],
                          rho=inp["rho"], **kw), inp


# ---- p = 2 reduces to the Kronecker-sum Laplacian (textbook special case) --

@pytest.mark.parametrize("shape,k,nq", [((2, 3, 4), 1, 2), ((2, 3, 4), 2, 3),
                                        ((3, 2, 2), 3, 4), ((2, 2, 3), 3, 5),
                                        ((4, 4, 4), 2, 3)])
@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_p2_is_kronecker_laplacian(shape, k, nq, eps):
    d, inp = _disc(*shape, k, nq, 2.0, eps)
    K, b = kronecker_laplacian(gll_nodes(k), *shape)
    M = d.mask
    u, v = inp["u"], inp["v"]
    assert relerr(d.b, b) < 1e-12
    assert relerr(d.residual(u), M * (K @ (M * u) - b)) < 1e-12
    assert relerr(d.jvp(u, v), M * (K @ (M * v))) < 1e-12
    assert relerr(d.jacobian(u) @ v, M * (K @ (M * v))) < 1e-12


@pytest.mark.parametrize("p", [2.5, 3.0, 4.0])
def test_jvp_at_zero_and_residual_at_zero(p):
    eps = 0.05
    d, inp = _disc(2, 3, 2, 2, 3, p, eps)
    K, b = kronecker_laplacian(gll_nodes(2), 2, 3, 2)
    M = d.mask
    z = np.zeros(d.N)
    assert relerr(d.residual(z), -M * b) < 1e-15
    assert relerr(d.jvp(z, inp["v"]), eps ** (p - 2) * M * (K @ (M * inp["v"]))) < 1e-12


# ---- R = grad E, J = dR (finite differences) ---------------------------------

@pytest.mark.parametrize("case", ["c1", "curved"])
def test_residual_is_energy_gradient(case):
    if case == "c1":
        d, inp = _disc(4, 4, 4, 2, 3, 3.0, 1e-2, seed=1)
    else:
        d, inp = _disc(2, 3, 2, 2, 3, 2.5, 1e-2, perturb=True)
    u = 0.3 * inp["u"]
    R = d.residual(u)
    interior = np.nonzero(d.mask)[0]
    h = 1e-5
    fd = np.zeros(d.N)
    for i in interior:
        e = np.zeros(d.N)
        e[i] = h
        fd[i] = (d.energy(u + e) - d.energy(u - e)) / (2 * h)
    assert relerr(fd, R) < 1e-7


@pytest.mark.parametrize("p,eps,perturb", [(3.0, 1e-2, False), (4.0, 1e-3, False),
                                           (2.5, 1e-2, True), (1.5, 0.1, True)])
def test_jvp_matches_central_difference(p, eps, perturb):
    d, inp = _disc(2, 2, 3, 2, 3, p, eps, perturb=perturb, rho=True)
    u, v = 0.5 * inp["u"], inp["v"]
    h = 1e-6 * np.linalg.norm(u) / np.linalg.norm(v)
    fd = (d.residual(u + h * v) - d.residual(u - h * v)) / (2 * h)
    assert relerr(d.jvp(u, v), fd) < 1e-7


def test_jacobian_symmetric_and_consistent():
    d, inp = _disc(2, 3, 2, 3, 4, 3.0, 1e-2, perturb=True, rho=True)
    u, v = inp["u"], inp["v"]
    K = d.jacobian(u)
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    w = np.random.default_rng(5).uniform(-1, 1, d.N)
    lhs, rhs = w @ d.jvp(u, v), v @ d.jvp(u, w)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    assert relerr(K @ v, d.jvp(u, v)) < 1e-13


# ---- invariants ----------------------------------------------------------------

@pytest.mark.parametrize("perturb", [False, True])
@pytest.mark.parametrize("k,nq", [(1, 2), (2, 3), (3, 5)])
def test_patch_test_linear_solution(perturb, k, nq):
    d, _ = _disc(3, 2, 3, k, nq, 3.0, 1e-2, perturb=perturb, seed=7)
    x = d.node_coordinates()
    u = 0.7 * x[:, 0] - 1.3 * x[:, 1] + 0.4 * x[:, 2] + 2.0
    A = d.apply_full(u)
    inner = d.mask > 0
    scale = np.abs(d.apply_full(np.random.default_rng(1).uniform(-1, 1, d.N))).max()
    assert np.abs(A[inner]).max() < 1e-13 * scale


@pytest.mark.parametrize("perturb", [False, True])
def test_partition_of_unity(perturb):
    d, inp = _disc(2, 3, 2, 2, 3, 3.0, 1e-2, perturb=perturb)
    A = d.apply_full(inp["u"])
    assert abs(A.sum()) < 1e-12 * np.abs(A).sum()


def test_volume_and_load_moments_on_curved_mesh():
    d, _ = _disc(3, 3, 2, 3, 4, 3.0, 1e-2, perturb=True, seed=3)
    _, detJ, _, _ = d.geometry(np.arange(d.E))
    assert abs((detJ * d.w).sum() - 1.0) < 1e-14
    assert np.all(detJ > 0)
    assert abs(d.b.sum() - 1.0) < 1e-14
    bx = d.load_vector(lambda x, y, z: x)
    assert abs(bx.sum() - 0.5) < 1e-14
    bxyz = d.load_vector(lambda x, y, z: x * y * z)
    assert abs(bxyz.sum() - 0.125) < 1e-14


@pytest.mark.parametrize("p", [2.5, 3.0, 4.0])
def test_homogeneity_eps0(p):
    d, inp = _disc(2, 2, 2, 2, 3, p, 0.0, perturb=True)
    u = inp["u"]
    c = 1.7
    A1 = d.apply_unmasked(u)
    assert relerr(d.apply_unmasked(c * u), c ** (p - 1) * A1) < 1e-13
    assert relerr(d.jvp(u, u), (p - 1) * d.mask * A1) < 1e-13


def test_sampled_outputs_equal_full():
    d, inp = _disc(3, 4, 3, 2, 3, 3.0, 1e-2, perturb=True, rho=True)
    dofs = np.array([0, 17, 100, d.N // 2, d.N - 1])
    assert np.array_equal(d.residual_at(inp["u"], dofs)[[1, 2, 3]],
                          d.residual(inp["u"])[dofs][[1, 2, 3]]) or \
        relerr(d.residual_at(inp["u"], dofs), d.residual(inp["u"])[dofs]) < 1e-14
    assert relerr(d.jvp_at(inp["u"], inp["v"], dofs), d.jvp(inp["u"], inp["v"])[dofs]) < 1e-14


def test_element_tangents_assemble_to_jacobian_and_match_fd():
    d, inp = _disc(2, 2, 2, 2, 3, 3.0, 1e-2, perturb=True, rho=True)
    u = inp["u"]
    elems = np.arange(d.E)
    Ke = d.element_tangents(u, elems)
    # symmetric element matrices; K_e v_e equals the element Jacobian action
    assert np.abs(Ke - np.swapaxes(Ke, 1, 2)).max() <= 1e-13 * np.abs(Ke).max()
    v = inp["v"]
    ve = d.gather(v, elems)
    assert relerr(np.einsum("eab,eb->ea", Ke, ve), d.element_jvp(u, v, elems)) < 1e-13
    # central differences of the element residual in one local direction
    for e, j in [(0, 13), (0, 26), (5, 4)]:
        h = 1e-6
        assert d.mask[d.elem_dofs[e, j]] > 0
        du = np.zeros(d.N)
        du[d.elem_dofs[e, j]] = h
        fd = (d.element_residual(u + du, [e]) - d.element_residual(u - du, [e]))[0] / (2 * h)
        assert relerr(Ke[e][:, j], fd) < 1e-7


# ---- eps = 0 where the gradient vanishes (a = eps^2 + |g|^2 = 0) ----------------

def _vanishing_on_half(d, u):
    """u with every node of the lower half (x index below Lx/2) set to 0, so
    the elements there have a zero gradient at every quadrature point."""
    I = np.arange(d.N) % d.Lx
    return np.where(I < d.Lx // 2, 0.0, u)


@pytest.mark.parametrize("p", [2.0, 2.5, 3.0, 4.0])
def test_eps0_at_zero_is_the_limit_of_the_closed_form(p):
    """At eps = 0, R(0) = -M b and E(0) = 0; J(0) is the eps -> 0 limit of
    J(0) = eps^(p-2) K: the Kronecker Laplacian for p = 2, zero for p > 2."""
    d, inp = _disc(2, 3, 2, 2, 3, p, 0.0)
    K, b = kronecker_laplacian(gll_nodes(2), 2, 3, 2)
    M = d.mask
    z = np.zeros(d.N)
    assert relerr(d.residual(z), -M * b) < 1e-15
    assert d.energy(z) == 0.0
    jv = d.jvp(z, inp["v"])
    if p == 2.0:
        assert relerr(jv, M * (K @ (M * inp["v"]))) < 1e-12
    else:
        assert np.all(jv == 0.0)
    Ke = d.element_tangents(z, np.arange(d.E))
    assert np.all(np.isfinite(Ke))


@pytest.mark.parametrize("p", [4.0, 3.5, 3.0, 2.5])
@pytest.mark.parametrize("perturb", [False, True])
def test_eps0_jvp_matches_central_difference_where_gradient_vanishes(p, perturb):
    """J(u) v against central differences of R at eps = 0 with u zero on half
    the mesh.  At a zero-gradient point the difference quotient is
    |h grad v|^(p-2) grad v = O(h^(p-2)) against the limit 0 of the tangent.
    For p >= 3.5 that is below 1e-7 at h = 1e-6; for p = 3 and 2.5 it
    dominates, and the error must shrink at exactly that rate (a wrong finite
    limit at a = 0 would leave an error that does not shrink)."""
    d, inp = _disc(4, 2, 2, 2, 3, p, 0.0, perturb=perturb, rho=True)
    u, v = _vanishing_on_half(d, 0.5 * inp["u"]), inp["v"]
    jv = d.jvp(u, v)
    assert np.all(np.isfinite(jv))
    err = {}
    for hs in (1e-4, 1e-6):
        h = hs * np.linalg.norm(u) / np.linalg.norm(v)
        fd = (d.residual(u + h * v) - d.residual(u - h * v)) / (2 * h)
        err[hs] = relerr(jv, fd)
    if p >= 3.5:
        assert err[1e-6] < 1e-7
    else:
        rate = np.log10(err[1e-4] / err[1e-6]) / 2.0
        assert abs(rate - (p - 2.0)) < 0.05
        assert err[1e-6] < 1e-6 ** (p - 2.0)
    # the Euler identity J(u) u = (p-1) A(u) of the homogeneous flux holds there too
    assert relerr(d.jvp(u, u), (p - 1) * d.mask * d.apply_unmasked(u)) < 1e-13
