"""GPU (HIP) vs oracle parity of the operator applies, element by element.

Small meshes: whole vectors, relative L2 <= 1e-12 in FP64 (every mesh spans
several workgroup batches with a ragged last batch).  Full workload sizes:
whole-vector GPU applies checked at sampled DOFs the oracle computes one by
one, plus properties that hold at any size.
"""
import numpy as np
import pytest
import torch

import paper_2506_00746_amd as feod
from tests.gpu_helpers import announce, dev, host, relerr, setup
from workloads import WORKLOADS, Workload, make_inputs

pytestmark = pytest.mark.gpu

SMALL = [
    Workload("c1", 4, 4, 4, 2, 3, 3.0, 1e-2, 1),
    Workload("q2-ragged-rho", 5, 3, 7, 2, 3, 3.0, 1e-2, 21, rho=True),
    Workload("q2-curved", 3, 4, 2, 2, 3, 2.5, 1e-2, 22, perturb=True, rho=True),
    Workload("q3-p4", 3, 5, 2, 3, 5, 4.0, 1e-3, 23),
    Workload("q3-curved", 2, 3, 3, 3, 5, 4.0, 1e-3, 24, perturb=True),
    Workload("q4-p2.5", 3, 2, 3, 4, 6, 2.5, 1e-2, 25),
    Workload("q7-curved", 2, 2, 3, 7, 9, 3.0, 1e-2, 26, perturb=True),
    Workload("q1-curved", 5, 4, 3, 1, 2, 2.5, 1e-2, 27, perturb=True, rho=True),
    Workload("q2-nq4-generic-p", 3, 3, 4, 2, 4, 1.5, 0.1, 28, perturb=True),
    Workload("q2-p2", 4, 3, 2, 2, 3, 2.0, 1e-2, 29),
    Workload("q7-affine-rho-generic-p", 3, 3, 1, 7, 9, 1.7, 0.1, 30, rho=True),  # ragged last Q7 batch
]
IDS = [w.name for w in SMALL]


@pytest.mark.parametrize("w", SMALL, ids=IDS)
def test_residual_jvp_energy_fp64(w):
    announce("parity fp64", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    r = host(prob.residual(u))
    jv = host(prob.jacobian_apply(u, v))
    r2, jv2 = prob.residual_and_jvp(u, v)
    e = host(prob.energy(u))[0]
    r_o, jv_o = ora.residual(inp["u"]), ora.jvp(inp["u"], inp["v"])
    assert relerr(r, r_o) <= 1e-12
    assert relerr(jv, jv_o) <= 1e-12
    assert relerr(host(r2), r_o) <= 1e-12
    assert relerr(host(jv2), jv_o) <= 1e-12
    e_o = ora.energy(inp["u"])
    assert abs(e - e_o) <= 1e-12 * abs(e_o)
    inner = ora.mask > 0
    assert np.all(r[~inner] == 0) and np.all(jv[~inner] == 0)


@pytest.mark.parametrize("w", SMALL, ids=IDS)
def test_grad_rho_kernel_fp64(w):
    announce("grad kernel fp64", w)
    prob, ora, inp = setup(w)
    lam = np.random.default_rng(w.seed + 100).uniform(-1, 1, ora.N)
    g = host(prob.grad_rho(dev(inp["u"]), dev(lam)))
    assert relerr(g, ora.grad_rho(inp["u"], lam)) <= 1e-12


@pytest.mark.parametrize("w", SMALL, ids=IDS)
def test_mixed_precision_error_vs_fp64_oracle(w):
    announce("parity mixed", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    r = host(prob.residual(u, prec="mixed"))
    jv = host(prob.jacobian_apply(u, v, prec="mixed"))
    e_r = relerr(r, ora.residual(inp["u"]))
    e_j = relerr(jv, ora.jvp(inp["u"], inp["v"]))
    lam = np.random.default_rng(w.seed + 100).uniform(-1, 1, ora.N)
    e_g = relerr(host(prob.grad_rho(u, dev(lam), prec="mixed")), ora.grad_rho(inp["u"], lam))
    e_e = abs(host(prob.energy(u, prec="mixed"))[0] - ora.energy(inp["u"])) / abs(ora.energy(inp["u"]))
    print(f"mixed-precision rel. L2 error vs FP64 oracle [{w.name}]: residual {e_r:.2e} "
          f"jvp {e_j:.2e} grad {e_g:.2e} energy {e_e:.2e}")
    # FP32 B, D, B^T with FP32 accumulation: about 1e-7 measured at these sizes
    assert e_r <= 5e-6 and e_j <= 5e-6 and e_g <= 5e-6 and e_e <= 5e-6


@pytest.mark.parametrize("w", SMALL, ids=IDS)
def test_hand_coded_tangent_matches_dual_numbers(w):
    """The hand-coded J_D (Table 1's HND) gives the oracle's Jacobian action,
    and the dual-number one to rounding."""
    announce("hand-coded tangent", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    jv_dual = host(prob.jacobian_apply(u, v))
    prob.set_tangent_mode("hand")
    jv_hand = host(prob.jacobian_apply(u, v))
    prob.set_tangent_mode("dual")
    assert relerr(jv_hand, ora.jvp(inp["u"], inp["v"])) <= 1e-12
    assert relerr(jv_hand, jv_dual) <= 1e-13
    assert np.array_equal(host(prob.jacobian_apply(u, v)), jv_dual)


def test_bitwise_determinism_and_symmetry():
    w = SMALL[2]
    announce("determinism", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    wv = dev(np.random.default_rng(3).uniform(-1, 1, ora.N))
    a = host(prob.jacobian_apply(u, v))
    b = host(prob.jacobian_apply(u, v))
    assert np.array_equal(a, b)
    assert np.array_equal(host(prob.residual(u)), host(prob.residual(u)))
    lhs = float(host(wv) @ a)
    rhs = float(host(v) @ host(prob.jacobian_apply(u, wv)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_aliasing_and_bad_arguments_rejected():
    import paper_2506_00746_amd as feod
    w = SMALL[0]
    announce("errors", w)
    prob, _, inp = setup(w, oracle=False)
    u = dev(inp["u"])
    with pytest.raises(feod.FeodError, match="EINVAL"):
        prob.residual(u, out=u)
    with pytest.raises(feod.FeodError, match="EINVAL"):
        prob.jacobian_apply(u, u, out=u)
    with pytest.raises(ValueError):
        prob.residual(u[:-1])
    with pytest.raises(TypeError):
        prob.residual(u.float())


def _sample_dofs(ora, n=160, seed=0):
    rng = np.random.default_rng(seed)
    inner = np.nonzero(ora.mask)[0]
    pick = rng.choice(inner, n, replace=False)
    corners = [inner[0], inner[-1], inner[len(inner) // 2], 0, ora.N - 1]
    return np.unique(np.concatenate([pick, corners]))


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5"])
def test_full_size_sampled_parity(name):
    w = WORKLOADS[name]
    announce("full-size sampled parity", name)
    prob, ora, inp = setup(w, compute_load=False)
    u, v = dev(inp["u"]), dev(inp["v"])
    dofs = _sample_dofs(ora)
    r = host(prob.residual(u))
    jv = host(prob.jacobian_apply(u, v))
    assert relerr(r[dofs], ora.residual_at(inp["u"], dofs)) <= 1e-12
    assert relerr(jv[dofs], ora.jvp_at(inp["u"], inp["v"], dofs)) <= 1e-12
    # properties at full size: Dirichlet rows exactly zero, bitwise repeatable
    inner = ora.mask > 0
    assert np.all(r[~inner] == 0) and np.all(jv[~inner] == 0)
    assert np.array_equal(jv, host(prob.jacobian_apply(u, v)))
    rm = host(prob.jacobian_apply(u, v, prec="mixed"))
    print(f"[{name}] mixed JVP rel. error at sampled DOFs: "
          f"{relerr(rm[dofs], jv[dofs]):.2e}")
    # the hand-coded J_D at full size: the dual-number apply to rounding
    prob.set_tangent_mode("hand")
    assert relerr(host(prob.jacobian_apply(u, v)), jv) <= 1e-13
    prob.set_tangent_mode("dual")
    del prob
    torch.cuda.empty_cache()


@pytest.mark.parametrize("w", [SMALL[1], SMALL[4], SMALL[5], SMALL[6]], ids=["q2", "q3-curved", "q4", "q7-curved"])
def test_lattice_and_explicit_maps_bitwise_equal(w):
    """The computed map (tiled G^T for FP64 at k = 2, 4; lattice order
    otherwise) against the stored CSR map: bitwise equal applies and solves."""
    announce("map modes", w)
    prob, ora, inp = setup(w, oracle=False)
    u, v = dev(inp["u"]), dev(inp["v"])
    outs = {}
    for mode in ("lattice", "explicit"):
        prob.set_map_mode(mode)
        r, jv = prob.residual_and_jvp(u, v)
        rm = prob.residual(u, prec="mixed")
        rm2, jvm2 = prob.residual_and_jvp(u, v, prec="mixed")  # two FP32 E-vectors at once
        outs[mode] = [host(r), host(jv), host(rm), host(prob.jacobian_apply(u, v)), host(rm2), host(jvm2),
                      host(prob.jacobian_apply(u, v, prec="mixed"))]
    for a, b in zip(outs["lattice"], outs["explicit"]):
        assert np.array_equal(a, b)
    # the CG solves (fused G^T + p.q) give bitwise the same iterates too
    load = dev(feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq).load)
    sols = {}
    for mode in ("lattice", "explicit"):
        prob.set_map_mode(mode)
        un, rep = prob.newton_solve(rtol=1e-10)
        g, lam, arep = prob.adjoint_gradient(un, load, rtol=1e-10)
        gm, _, _ = prob.adjoint_gradient(un, load, rtol=1e-10, prec="mixed")
        sols[mode] = [host(un), host(g), host(lam), host(gm)]
    for a, b in zip(sols["lattice"], sols["explicit"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["c2", "c4", "c3"])
def test_full_size_lattice_and_explicit_maps_bitwise_equal(name):
    """At 32^3 Q3, 48^3 Q2 and 64^3 Q4 the computed G^T (FP64 tiles at k = 2
    and 4, lattice order at k = 3; FP32 element runs with wide stores at all
    three) spans several
    tiles of runs per lattice row and a ragged last one: its applies, and the
    adjoint CG solves through the fused G^T + p.q, must equal the stored CSR
    map's bit for bit, in FP64 and mixed precision."""
    w = WORKLOADS[name]
    announce("full-size map modes", name)
    prob, _, inp = setup(w, oracle=False)
    u, v = dev(inp["u"]), dev(inp["v"])
    g_u = dev(np.random.default_rng(71).standard_normal(w.n_dofs))
    outs = {}
    for mode in ("lattice", "explicit"):
        prob.set_map_mode(mode)
        res = []
        for prec in ("fp64", "mixed"):
            r, jv = prob.residual_and_jvp(u, v, prec=prec)
            res += [host(r), host(jv), host(prob.jacobian_apply(u, v, prec=prec))]
            g, lam, rep = prob.adjoint_gradient(u, g_u, rtol=1e-8, prec=prec)
            assert rep["status"] == 0, rep
            res += [host(g), host(lam)]
        outs[mode] = res
    for i, (a, b) in enumerate(zip(outs["lattice"], outs["explicit"])):
        assert np.array_equal(a, b), i
    prob.set_map_mode("lattice")
    del prob
    torch.cuda.empty_cache()


@pytest.mark.parametrize("w", [SMALL[0], SMALL[2], SMALL[3], SMALL[4], SMALL[5], SMALL[6], SMALL[8]],
                         ids=["c1", "q2-curved", "q3-p4", "q3-curved", "q4", "q7-curved", "q2-generic"])
def test_jacobian_diagonal_matches_assembled_oracle(w):
    announce("diagonal", w)
    prob, ora, inp = setup(w)
    d = host(prob.jacobian_diagonal(dev(inp["u"])))
    d_o = ora.jacobian(inp["u"]).diagonal()
    assert relerr(d, d_o) <= 1e-12
    dm = host(prob.jacobian_diagonal(dev(inp["u"]), prec="mixed"))
    print(f"[{w.name}] mixed diagonal rel. error vs FP64 oracle: {relerr(dm, d_o):.2e}")
    assert relerr(dm, d_o) <= 5e-6


@pytest.mark.parametrize("w", [SMALL[0], SMALL[1], SMALL[2], SMALL[3], SMALL[4], SMALL[5], SMALL[7], SMALL[8]],
                         ids=["c1", "q2-rho", "q2-curved", "q3-p4", "q3-curved", "q4", "q1-curved", "q2-generic"])
def test_element_tangents_match_oracle(w):
    announce("element tangents", w)
    prob, ora, inp = setup(w)
    Ke = host(prob.element_tangents(dev(inp["u"])))
    Ko = ora.element_tangents(inp["u"], np.arange(ora.E))
    assert relerr(Ke, Ko) <= 1e-12
    # a sub-range of elements gives the same matrices
    part = host(prob.element_tangents(dev(inp["u"]), first=1, count=ora.E - 2))
    assert np.array_equal(part, Ke[1:-1])
    # counts that leave a workgroup's element batch partly empty
    for cnt in (1, 3, 5):
        if 2 + cnt <= ora.E:
            part = host(prob.element_tangents(dev(inp["u"]), first=2, count=cnt))
            assert np.array_equal(part, Ke[2:2 + cnt])


@pytest.mark.parametrize("w", [SMALL[0], SMALL[1], SMALL[2], SMALL[3], SMALL[4], SMALL[5], SMALL[7], SMALL[8]],
                         ids=["c1", "q2-rho", "q2-curved", "q3-p4", "q3-curved", "q4", "q1-curved", "q2-generic"])
def test_element_level_ad_tangents_match_oracle(w):
    """The paper's ELM variant (forward AD through the whole element residual,
    one Jacobian action per local DOF) gives the same K_e as the oracle and as
    quadrature-point AD, on full meshes and on element sub-ranges."""
    announce("element-level AD tangents", w)
    prob, ora, inp = setup(w)
    u = dev(inp["u"])
    Kelm = host(prob.element_tangents(u, method="elm"))
    assert relerr(Kelm, ora.element_tangents(inp["u"], np.arange(ora.E))) <= 1e-12
    assert relerr(Kelm, host(prob.element_tangents(u))) <= 1e-13
    part = host(prob.element_tangents(u, first=1, count=ora.E - 2, method="elm"))
    assert np.array_equal(part, Kelm[1:-1])
    for cnt in (1, 3, 5):
        if 2 + cnt <= ora.E:
            part = host(prob.element_tangents(u, first=2, count=cnt, method="elm"))
            assert np.array_equal(part, Kelm[2:2 + cnt])


def test_element_tangents_sampled_on_design_mesh():
    w = WORKLOADS["c4"]
    announce("element tangents c4 sampled")
    prob, ora, inp = setup(w, compute_load=False)
    rng = np.random.default_rng(0)
    for first in rng.choice(ora.E - 16, 4, replace=False):
        Ke = host(prob.element_tangents(dev(inp["u"]), first=int(first), count=16))
        Ko = ora.element_tangents(inp["u"], np.arange(first, first + 16))
        assert relerr(Ke, Ko) <= 1e-12
        Kelm = host(prob.element_tangents(dev(inp["u"]), first=int(first), count=16, method="elm"))
        assert relerr(Kelm, Ko) <= 1e-12


def test_element_tangents_unsupported_order():
    import paper_2506_00746_amd as feod
    w = SMALL[6]  # Q7
    prob, _, inp = setup(w, oracle=False)
    with pytest.raises(feod.FeodError, match="UNSUPPORTED"):
        prob.element_tangents(dev(inp["u"]))
    with pytest.raises(feod.FeodError, match="UNSUPPORTED"):
        prob.element_tangents(dev(inp["u"]), method="elm")


@pytest.mark.parametrize("w", [SMALL[0], SMALL[2], SMALL[4], SMALL[6]], ids=["c1", "q2-curved", "q3-curved", "q7-curved"])
def test_partial_assembly_jvp_equals_fused(w):
    import paper_2506_00746_amd as feod
    announce("partial assembly", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    with pytest.raises(feod.FeodError, match="ESTATE"):
        prob.jacobian_apply_pa(v)
    for prec in ("fp64", "mixed"):
        prob.pa_setup(u, prec=prec)
        a = host(prob.jacobian_apply_pa(v, prec=prec))
        b = host(prob.jacobian_apply(u, v, prec=prec))
        assert np.array_equal(a, b), prec
    e_pa = relerr(host(prob.jacobian_apply_pa(v, prec="mixed")), ora.jvp(inp["u"], inp["v"]))
    print(f"[{w.name}] mixed partial-assembly JVP rel. error vs FP64 oracle: {e_pa:.2e}")
    assert e_pa <= 5e-6
    prob.pa_setup(u)
    assert relerr(host(prob.jacobian_apply_pa(v)), ora.jvp(inp["u"], inp["v"])) <= 1e-12


DEGENERATE = [
    Workload("one-elem-q3", 1, 1, 1, 3, 5, 4.0, 1e-3, 40, perturb=True, rho=True),  # one (curved-path) element
    Workload("slab-q4", 1, 6, 2, 4, 6, 2.5, 1e-2, 41, rho=True),                     # one element thick
    Workload("eps0-q2-curved", 3, 2, 4, 2, 3, 3.0, 0.0, 42, perturb=True),           # eps = 0 (p >= 2)
]


@pytest.mark.parametrize("w", DEGENERATE, ids=[w.name for w in DEGENERATE])
def test_degenerate_meshes_match_oracle(w):
    """Single element, single-element-thick slab and eps = 0: every operator
    against the oracle, partial assembly bitwise equal to the fused apply."""
    announce("degenerate", w)
    prob, ora, inp = setup(w)
    u, v = dev(inp["u"]), dev(inp["v"])
    r_o, jv_o = ora.residual(inp["u"]), ora.jvp(inp["u"], inp["v"])
    assert relerr(host(prob.residual(u)), r_o) <= 1e-12
    jv = prob.jacobian_apply(u, v)
    assert relerr(host(jv), jv_o) <= 1e-12
    r2, jv2 = prob.residual_and_jvp(u, v)
    assert relerr(host(r2), r_o) <= 1e-12 and relerr(host(jv2), jv_o) <= 1e-12
    e_o = ora.energy(inp["u"])
    assert abs(host(prob.energy(u))[0] - e_o) <= 1e-12 * abs(e_o)
    lam = np.random.default_rng(w.seed + 100).uniform(-1, 1, ora.N)
    assert relerr(host(prob.grad_rho(u, dev(lam))), ora.grad_rho(inp["u"], lam)) <= 1e-12
    e_m = relerr(host(prob.jacobian_apply(u, v, prec="mixed")), jv_o)
    print(f"[{w.name}] mixed JVP rel. error vs FP64 oracle: {e_m:.2e}")
    assert e_m <= 5e-6
    prob.pa_setup(u)
    assert torch.equal(prob.jacobian_apply_pa(v), jv)


def test_all_dirichlet_mesh_gives_exact_zeros():
    """One Q1 element: every node is a Dirichlet node, so the masked residual,
    Jacobian action and design gradient are exactly zero, and both solvers
    stop before their first step."""
    w = Workload("all-dirichlet-q1", 1, 1, 1, 1, 2, 3.0, 1e-2, 43)
    announce("all-dirichlet", w)
    prob, ora, inp = setup(w)
    assert ora.mask.sum() == 0
    u, v = dev(inp["u"]), dev(inp["v"])
    assert not host(prob.residual(u)).any()
    assert not host(prob.jacobian_apply(u, v)).any()
    e_o = ora.energy(inp["u"])
    assert abs(host(prob.energy(u))[0] - e_o) <= 1e-12 * abs(e_o)
    us, rep = prob.newton_solve(rtol=1e-10)
    assert rep["status"] == 0 and rep["newton_iters"] == 0 and rep["cg_iters_total"] == 0
    assert not host(us).any()
    grad, lam, rep = prob.adjoint_gradient(us, dev(ora.b))
    assert rep["status"] == 0 and rep["cg_iters_total"] == 0
    assert not host(lam).any() and not host(grad).any()


EPS0 = [
    Workload("eps0-p3-affine", 4, 3, 2, 2, 3, 3.0, 0.0, 44),
    Workload("eps0-p3-curved", 3, 2, 3, 2, 3, 3.0, 0.0, 45, perturb=True, rho=True),
    Workload("eps0-p2.5-affine", 3, 3, 2, 3, 5, 2.5, 0.0, 46, rho=True),
    Workload("eps0-p2.5-curved", 2, 3, 2, 3, 5, 2.5, 0.0, 47, perturb=True, rho=True),
    Workload("eps0-p2.5-q7-curved", 2, 2, 2, 7, 9, 2.5, 0.0, 48, perturb=True),
]


def _vanishing_on_half(w, u):
    """u with every node of the lower x half set to 0: the elements there have
    a zero gradient (a = eps^2 + |g|^2 = 0 at eps = 0) at every point."""
    Lx = w.k * w.nx + 1
    return np.where(np.arange(u.size) % Lx < Lx // 2, 0.0, u)


@pytest.mark.parametrize("w", EPS0, ids=[w.name for w in EPS0])
def test_eps0_zero_gradient(w):
    """eps = 0 where the gradient vanishes (the limit of Eq. (2)'s J_D there
    is 0 for p > 2): R(0) = -M b, E(0) = 0 and J(0) v = 0 exactly, in both
    precisions; and with u zero on half the mesh every operator matches the
    oracle element by element."""
    announce("eps = 0 zero gradient", w)
    prob, ora, inp = setup(w)
    N = ora.N
    bm = ora.mask * feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq, vertices=inp["vertices"]).load
    z = dev(np.zeros(N))
    v = dev(inp["v"])
    for prec in ("fp64", "mixed"):
        r0 = host(prob.residual(z, prec=prec))
        assert np.array_equal(r0, -bm), prec
        assert relerr(r0, -ora.mask * ora.b) <= 1e-12
        assert not host(prob.jacobian_apply(z, v, prec=prec)).any(), prec
        r2, jv2 = prob.residual_and_jvp(z, v, prec=prec)
        assert np.array_equal(host(r2), -bm) and not host(jv2).any(), prec
        assert not host(prob.jacobian_diagonal(z, prec=prec)).any(), prec
        assert not host(prob.grad_rho(z, v, prec=prec)).any(), prec
        assert host(prob.energy(z, prec=prec))[0] == 0.0, prec
    if w.k <= 4:
        assert not host(prob.element_tangents(z)).any()
        assert not host(prob.element_tangents(z, method="elm")).any()
    assert not ora.jvp(np.zeros(N), inp["v"]).any()
    # half the mesh at zero gradient, the other half random: every operator
    uh = _vanishing_on_half(w, inp["u"])
    u = dev(uh)
    r_o, jv_o = ora.residual(uh), ora.jvp(uh, inp["v"])
    assert relerr(host(prob.residual(u)), r_o) <= 1e-12
    jv = prob.jacobian_apply(u, v)
    assert relerr(host(jv), jv_o) <= 1e-12
    r2, jv2 = prob.residual_and_jvp(u, v)
    assert relerr(host(r2), r_o) <= 1e-12 and relerr(host(jv2), jv_o) <= 1e-12
    e_o = ora.energy(uh)
    assert abs(host(prob.energy(u))[0] - e_o) <= 1e-12 * abs(e_o)
    lam = np.random.default_rng(w.seed + 100).uniform(-1, 1, N)
    assert relerr(host(prob.grad_rho(u, dev(lam))), ora.grad_rho(uh, lam)) <= 1e-12
    assert relerr(host(prob.jacobian_diagonal(u)), ora.jacobian(uh).diagonal()) <= 1e-12
    if w.k <= 4:
        Ko = ora.element_tangents(uh, np.arange(ora.E))
        assert relerr(host(prob.element_tangents(u)), Ko) <= 1e-12
        assert relerr(host(prob.element_tangents(u, method="elm")), Ko) <= 1e-12
    prob.set_tangent_mode("hand")
    assert relerr(host(prob.jacobian_apply(u, v)), jv_o) <= 1e-12
    prob.set_tangent_mode("dual")
    prob.pa_setup(u)
    assert torch.equal(prob.jacobian_apply_pa(v), jv)
    e_m = relerr(host(prob.jacobian_apply(u, v, prec="mixed")), jv_o)
    print(f"[{w.name}] mixed JVP rel. error vs FP64 oracle at eps = 0: {e_m:.2e}")
    assert e_m <= 5e-6
