"""GPU Newton-CG and adjoint solves vs the oracle's direct-solve versions,
and the autograd design gradient vs central finite differences."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2506_00746_amd as feod
from oracle import Discretisation, adjoint, newton
from tests.gpu_helpers import announce, dev, host, relerr, setup
from workloads import WORKLOADS, Workload, make_inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_c1_matches_oracle(prec):
    w = WORKLOADS["c1"]
    announce("newton c1", prec)
    prob, ora, _ = setup(w)
    u, rep = prob.newton_solve(rtol=1e-12, prec=prec)
    u_o, info = newton(ora, tol=1e-13)
    print("GPU report", rep, "oracle iters", info["iters"])
    assert rep["status"] == 0
    assert rep["res_final"] <= 1e-12 * rep["ref_norm"]
    assert relerr(host(u), u_o) <= 1e-10
    # certified by the oracle residual at the GPU solution
    assert np.linalg.norm(ora.residual(host(u))) <= 1e-10 * np.linalg.norm(ora.mask * ora.b)


def test_newton_curved_q3_matches_oracle():
    w = Workload("nc", 3, 2, 3, 3, 5, 3.0, 1e-2, 31, perturb=True, rho=True)
    announce("newton curved", w)
    prob, ora, _ = setup(w)
    u, rep = prob.newton_solve(rtol=1e-12)
    u_o, _ = newton(ora, tol=1e-13)
    assert relerr(host(u), u_o) <= 1e-10


def test_adjoint_matches_oracle():
    w = Workload("adj", 4, 3, 3, 2, 3, 3.0, 1e-2, 32, perturb=True, rho=True)
    announce("adjoint", w)
    prob, ora, inp = setup(w)
    u, _ = prob.newton_solve(rtol=1e-13)
    b = dev(ora.b)
    for prec in ("fp64", "mixed"):
        grad, lam, rep = prob.adjoint_gradient(u, b, rtol=1e-13, prec=prec)
        lam_o, grad_o = adjoint(ora, host(u), ora.b)
        print(prec, rep, relerr(host(grad), grad_o))
        assert relerr(host(lam), lam_o) <= 1e-10
        assert relerr(host(grad), grad_o) <= 1e-10
        # mixed: the reported residual is the FP64 true residual M g_u - J lambda,
        # reached through reliable updates (FP64 CG reports its recursive one)
        jl = prob.jacobian_apply(u, lam)
        true_res = np.linalg.norm(ora.mask * ora.b - host(jl))
        ref = np.linalg.norm(ora.mask * ora.b)
        if prec == "mixed":
            assert rep["refine_iters"] >= 1
            assert true_res <= 1e-13 * ref * (1 + 1e-6)
            assert abs(true_res - rep["res_final"]) <= 1e-6 * rep["res_final"]
        else:
            assert true_res <= 1e-12 * ref


def test_design_solve_autograd_vs_finite_differences_c4():
    w = WORKLOADS["c4"]
    announce("design autograd c4")
    inp = make_inputs(w)
    prob = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, rho=inp["rho"], device="cuda:0")
    b = torch.as_tensor(feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq).load, device="cuda:0")
    rho = torch.as_tensor(inp["rho"], device="cuda:0").requires_grad_(True)
    opts = {"rtol": 1e-13}
    u = feod.DesignSolve.apply(rho, prob, opts)
    phi = torch.dot(b, u)
    phi.backward()
    grad = rho.grad.detach().cpu().numpy()
    u0 = u.detach()

    def phi_at(r):
        prob.set_rho(r)
        us, _ = prob.newton_solve(u0, init_poisson=0, rtol=1e-13)
        return float(torch.dot(b, us))

    rho0 = torch.as_tensor(inp["rho"], device="cuda:0")
    worst = 0.0
    for e in inp["fd_elems"]:
        h = 1e-3 * float(rho0[e])
        rp, rm = rho0.clone(), rho0.clone()
        rp[e] += h
        rm[e] -= h
        fd = (phi_at(rp) - phi_at(rm)) / (2 * h)
        worst = max(worst, abs(fd - grad[e]) / abs(grad[e]))
    print("worst relative FD mismatch over 20 elements:", worst)
    assert worst <= 1e-5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_jacobi_preconditioned_newton_and_adjoint(prec):
    w = Workload("pcg", 6, 5, 4, 3, 5, 4.0, 1e-3, 33, perturb=True, rho=True)
    announce("jacobi pcg", w, prec)
    prob, ora, _ = setup(w)
    u1, rep1 = prob.newton_solve(rtol=1e-12, prec=prec, jacobi=0)
    u2, rep2 = prob.newton_solve(rtol=1e-12, prec=prec, jacobi=1)
    print("CG iterations plain", rep1["cg_iters_total"], "jacobi", rep2["cg_iters_total"])
    assert rep2["status"] == 0 and rep2["res_final"] <= 1e-12 * rep2["ref_norm"]
    assert relerr(host(u2), host(u1)) <= 1e-10
    u_o, _ = newton(ora, tol=1e-13)
    assert relerr(host(u2), u_o) <= 1e-10
    b = dev(ora.b)
    g1, _, r1 = prob.adjoint_gradient(u2, b, rtol=1e-12, prec=prec, jacobi=0)
    g2, _, r2 = prob.adjoint_gradient(u2, b, rtol=1e-12, prec=prec, jacobi=1)
    assert relerr(host(g2), host(g1)) <= 1e-9


def test_partial_assembly_solves_match_fused():
    w = Workload("pa", 5, 4, 3, 3, 5, 3.0, 1e-2, 34, perturb=True, rho=True)
    announce("partial assembly solves", w)
    prob, ora, _ = setup(w)
    u0, r0 = prob.newton_solve(rtol=1e-12, partial_assembly=0)
    u1, r1 = prob.newton_solve(rtol=1e-12, partial_assembly=1)
    assert relerr(host(u1), host(u0)) <= 1e-10
    b = dev(ora.b)
    g0, _, _ = prob.adjoint_gradient(u1, b, rtol=1e-12, partial_assembly=0)
    g1, _, _ = prob.adjoint_gradient(u1, b, rtol=1e-12, partial_assembly=1)
    assert relerr(host(g1), host(g0)) <= 1e-10


def test_binding_argument_handling():
    """A u0 given without init_poisson is the Newton start (a converged one
    takes zero steps); a float32 design variable gets a float32 gradient equal
    to the FP64 one; a host output tensor is rejected before any launch."""
    w = Workload("bind", 3, 3, 2, 2, 3, 3.0, 1e-2, 34, perturb=True, rho=True)
    announce("binding arguments", w)
    prob, ora, inp = setup(w)
    u, rep = prob.newton_solve(rtol=1e-12)
    u2, rep2 = prob.newton(u, rtol=1e-12)
    assert rep2["newton_iters"] == 0 and rep2["cg_iters_total"] == 0
    assert torch.equal(u, u2)
    v = dev(inp["v"])
    assert torch.equal(prob.jvp(u, v), prob.jacobian_apply(u, v))
    # float32 rho: the gradient comes back in rho's dtype and device
    b = dev(ora.b)
    rho64 = torch.as_tensor(inp["rho"], device="cuda:0").requires_grad_(True)
    torch.dot(b, feod.DesignSolve.apply(rho64, prob, {"rtol": 1e-13})).backward()
    rho32 = torch.as_tensor(inp["rho"], device="cuda:0").float().requires_grad_(True)
    torch.dot(b, feod.DesignSolve.apply(rho32, prob, {"rtol": 1e-13})).backward()
    assert rho32.grad.dtype == torch.float32 and rho32.grad.device == rho32.device
    # rho32 rounds rho, so the two gradients agree to FP32 input precision
    assert relerr(rho32.grad.double().cpu().numpy(), rho64.grad.cpu().numpy()) <= 1e-5
    ne = (w.k + 1) ** 3
    with pytest.raises(TypeError):
        prob.element_tangents(u, 0, 1, out=torch.empty((1, ne, ne), dtype=torch.float64))
    with pytest.raises(ValueError):
        prob.element_tangents(u, 0, 2, out=torch.empty((1, ne, ne), dtype=torch.float64, device="cuda:0"))
    # an empty element range is a no-op for both tangent variants
    for method in ("res", "elm"):
        assert prob.element_tangents(u, first=3, count=0, method=method).shape == (0, ne, ne)


def test_design_solve_backward_uses_its_own_rho():
    """Two DesignSolve applies with different rho on one Problem before either
    backward: each gradient is the one taken at its own rho (the adjoint
    paragraph after Eq. (3)), equal to a single apply's gradient."""
    w = Workload("two-rho", 4, 3, 3, 2, 3, 3.0, 1e-2, 35, perturb=True, rho=True)
    announce("design solve two applies", w)
    prob, ora, inp = setup(w)
    b = dev(ora.b)
    rho_a = torch.as_tensor(inp["rho"], device="cuda:0")
    rho_b = torch.as_tensor(np.random.default_rng(36).uniform(0.1, 1.0, ora.E), device="cuda:0")
    opts = {"rtol": 1e-13}

    def single(r):
        x = r.clone().requires_grad_(True)
        torch.dot(b, feod.DesignSolve.apply(x, prob, opts)).backward()
        return x.grad.clone()

    ga, gb = single(rho_a), single(rho_b)
    assert relerr(host(ga), host(gb)) > 1e-3  # the two coefficients give different gradients
    xa = rho_a.clone().requires_grad_(True)
    xb = rho_b.clone().requires_grad_(True)
    phi_a = torch.dot(b, feod.DesignSolve.apply(xa, prob, opts))
    phi_b = torch.dot(b, feod.DesignSolve.apply(xb, prob, opts))
    phi_a.backward()
    phi_b.backward()
    assert relerr(host(xa.grad), host(ga)) <= 1e-10
    assert relerr(host(xb.grad), host(gb)) <= 1e-10
    # against the oracle's adjoint gradient at rho_a
    ora_a = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                           rho=inp["rho"])
    u_o, _ = newton(ora_a, tol=1e-13)
    _, g_o = adjoint(ora_a, u_o, ora_a.b)
    assert relerr(host(xa.grad), g_o) <= 1e-9


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_full_size_newton_certified_by_oracle_residual(name):
    """The 32^3 Q3 (p = 4, eps = 1e-3) and 48^3 Q2 design (p = 3, rho) Newton
    solutions in FP64 and mixed precision, certified by the oracle's own
    residual: ||R_oracle(u_gpu)||_2 <= 1e-10 ||M b||_2 (Eq. (1)), and the two
    precisions within 1e-9 of each other."""
    w = WORKLOADS[name]
    announce("full-size Newton certification", name)
    prob, ora, inp = setup(w)
    ref = np.linalg.norm(ora.mask * ora.b)
    sols = {}
    for prec in ("fp64", "mixed"):
        u, rep = prob.newton_solve(rtol=1e-10, prec=prec)
        assert rep["status"] == 0, rep
        uh = host(u)
        cert = np.linalg.norm(ora.residual(uh)) / ref
        print(f"[{name}] {prec}: Newton {rep['newton_iters']} steps, {rep['cg_iters_total']} CG iterations, "
              f"GPU rel. residual {rep['res_final'] / rep['ref_norm']:.2e}, oracle rel. residual {cert:.2e}")
        assert cert <= 1e-10
        sols[prec] = uh
    assert relerr(sols["mixed"], sols["fp64"]) <= 1e-9
    del prob
    torch.cuda.empty_cache()


def test_curved_q7_adjoint_gradient_c5():
    """16^3 Q7 curved workload: the adjoint design gradient at rho = 1 in FP64
    and mixed precision (the adjoint paragraph after Eq. (3)) against central
    finite differences of Phi = b^T u on seeded elements, and the gradient
    kernel against the oracle on those elements for the same u and lambda."""
    w = WORKLOADS["c5"]
    announce("adjoint c5")
    prob, ora, inp = setup(w, compute_load=False)
    b = dev(feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq, vertices=inp["vertices"]).load)
    # the FP64 residual of this workload has a floor near 2.6e-13 relative (one
    # ulp of u moves it by that much), so the solves stop at 1e-12
    u, rep = prob.newton_solve(rtol=1e-12)
    assert rep["status"] == 0, rep
    grads = {}
    for prec in ("fp64", "mixed"):
        g, lam, arep = prob.adjoint_gradient(u, b, rtol=1e-12, prec=prec)
        assert arep["status"] == 0, arep
        grads[prec] = (host(g), host(lam))
        print(f"[c5] adjoint {prec}: {arep['cg_iters_total']} CG iterations, "
              f"{arep['refine_iters']} reliable updates, rel. residual {arep['res_final'] / arep['ref_norm']:.2e}")
    g64, lam64 = grads["fp64"]
    e_mixed = relerr(grads["mixed"][0], g64)
    print(f"[c5] mixed vs FP64 adjoint gradient: {e_mixed:.2e}")
    assert e_mixed <= 1e-9
    elems = np.sort(np.random.default_rng(505).choice(w.n_elems, 6, replace=False))
    # gradient kernel vs the oracle at the same u, lambda (sampled elements)
    g_o = ora.grad_rho(host(u), lam64, elems)[elems]
    assert relerr(g64[elems], g_o) <= 1e-12
    gk32 = host(prob.grad_rho(u, dev(lam64), prec="mixed"))
    print(f"[c5] FP32 gradient kernel rel. error on sampled elements: {relerr(gk32[elems], g_o):.2e}")
    assert relerr(gk32[elems], g_o) <= 5e-6
    # central differences of Phi(rho) = b^T u(rho), rho_e = 1 -+ 1e-3
    u0 = u.clone()
    worst = 0.0
    for e in elems:
        phis = []
        for s in (1.0, -1.0):
            r = torch.ones(w.n_elems, dtype=torch.float64, device="cuda:0")
            r[int(e)] += s * 1e-3
            prob.set_rho(r)
            us, rp = prob.newton_solve(u0, init_poisson=0, rtol=1e-12)
            assert rp["status"] == 0, rp
            phis.append(float(torch.dot(b, us)))
        fd = (phis[0] - phis[1]) / 2e-3
        worst = max(worst, abs(fd - g64[e]) / abs(g64[e]))
    print(f"[c5] worst relative FD mismatch over {len(elems)} elements: {worst:.2e}")
    assert worst <= 1e-5
    del prob
    torch.cuda.empty_cache()


def _pcg_iterate(K, b, dinv, m):
    """x after m iterations of Jacobi-preconditioned CG on K x = b from x = 0,
    in the textbook recurrence (Hestenes and Stiefel, 1952), FP64."""
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    for _ in range(m):
        q = K @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


@pytest.mark.parametrize("max_cg,check_every", [(3, 10), (5, 2), (8, 1)])
def test_one_newton_step_with_capped_cg(max_cg, check_every):
    """One Newton step (max_newton = 1, called through the C ABI, which then
    reports the Newton cap) from u0 = M u*/2: the step u1 - u0 must be
    t du with t a power of two (the energy line search halves) and du the
    Jacobi-preconditioned CG iterate of J(u0) du = -R(u0) (Eq. (2)) after
    the reported number of iterations.  That number is max_cg, or a multiple
    of check_every at which the residual fell below the forcing term 0.1
    |R(u0)|: every CG step's alpha p must reach x, whether CG stops at the cap
    or at a residual check."""
    w = Workload("cap", 4, 3, 3, 3, 5, 3.0, 1e-2, 37, perturb=True, rho=True)
    announce("capped CG Newton step", w, max_cg, check_every)
    prob, ora, _ = setup(w)
    u_star, _ = newton(ora, tol=1e-13)
    u0 = ora.mask * (0.5 * u_star)
    u = dev(u0)
    o = feod.default_opts(max_newton=1, max_cg=max_cg, check_every=check_every, init_poisson=0)
    rep = feod.feod.SolverReport()
    L = feod.lib()
    prob._sync_stream()
    st = L.feod_newton_solve(prob._ctx, u.data_ptr(), ctypes.byref(o), ctypes.byref(rep))
    assert st == feod.feod.FEOD_ENOCONV, L.feod_last_error(prob._ctx).decode()
    rep = rep.as_dict()
    iters = rep["cg_iters_total"]
    print("CG iterations", iters, "report", rep)
    assert rep["newton_iters"] == 1 and 1 <= iters <= max_cg
    assert iters == max_cg or iters % check_every == 0
    R = ora.residual(u0)
    K = ora.jacobian(u0)
    d = K.diagonal()
    dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    du = _pcg_iterate(K, -R, dinv, iters)
    if iters < max_cg:
        assert np.linalg.norm(K @ du + R) <= 0.1 * np.linalg.norm(R) * (1 + 1e-9)
    step = host(u) - u0
    t_est = float(step @ du) / float(du @ du)
    t = 2.0 ** round(np.log2(t_est))
    assert abs(t_est - t) <= 1e-9 * t
    assert relerr(step, t * du) <= 1e-9


def test_cg_check_interval_and_cap_match_oracle():
    """The Newton solution (Eq. (1)) and the adjoint gradient (the paragraph
    after Eq. (3)) do not depend on how often CG reads its residual back or
    on a cap on the CG iterations of the inexact Newton steps, in FP64 and
    mixed precision; a capped adjoint CG that cannot converge is an error."""
    w = Workload("cgopt", 4, 3, 3, 3, 5, 3.0, 1e-2, 37, perturb=True, rho=True)
    announce("CG options", w)
    prob, ora, _ = setup(w)
    u_o, _ = newton(ora, tol=1e-13)
    b = dev(ora.b)
    lam_o, grad_o = adjoint(ora, u_o, ora.b)
    for prec in ("fp64", "mixed"):
        _, rep_d = prob.newton_solve(rtol=1e-12, prec=prec)
        for kw in ({"check_every": 1}, {"check_every": 7}, {"max_cg": 6}):
            u, rep = prob.newton_solve(rtol=1e-12, prec=prec, **kw)
            print(prec, kw, "Newton", rep["newton_iters"], "CG", rep["cg_iters_total"])
            assert rep["status"] == 0 and rep["res_final"] <= 1e-12 * rep["ref_norm"]
            assert relerr(host(u), u_o) <= 1e-10
            if "max_cg" in kw:
                assert rep["cg_iters_total"] <= 6 * (rep["newton_iters"] + 1)
                assert rep["newton_iters"] > rep_d["newton_iters"]
        u = dev(u_o)
        for ce in (1, 3):
            grad, lam, rep = prob.adjoint_gradient(u, b, rtol=1e-13, prec=prec, check_every=ce)
            print(prec, "adjoint check_every", ce, rep)
            assert relerr(host(lam), lam_o) <= 1e-10
            assert relerr(host(grad), grad_o) <= 1e-10
            if prec == "mixed":
                assert rep["refine_iters"] >= 1
        with pytest.raises(feod.FeodError) as err:
            prob.adjoint_gradient(u, b, rtol=1e-13, prec=prec, max_cg=2)
        assert err.value.status == feod.feod.FEOD_ENOCONV


def test_side_stream_results_equal_default_stream():
    """Every call enqueues on torch's current stream: the residual, the
    Jacobian action in both precisions, the Newton solve and the adjoint
    gradient issued under a second stream (default priority) equal the
    default stream's results bit for bit."""
    w = Workload("stream", 5, 4, 3, 2, 3, 3.0, 1e-2, 38, perturb=True, rho=True)
    announce("side stream", w)
    prob, ora, inp = setup(w)
    u, v, b = dev(inp["u"]), dev(inp["v"]), dev(ora.b)

    def run():
        r = prob.residual(u)
        jv = prob.jacobian_apply(u, v)
        jv32 = prob.jacobian_apply(u, v, prec="mixed")
        us, _ = prob.newton_solve(rtol=1e-12)
        g, lam, _ = prob.adjoint_gradient(us, b, rtol=1e-12)
        return r, jv, jv32, us, g, lam

    ref = run()
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device="cuda:0")
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for name, a, c in zip(("residual", "jvp", "jvp mixed", "newton u", "grad", "lambda"), ref, got):
        assert torch.equal(a, c), name
    assert relerr(host(got[0]), ora.residual(inp["u"])) <= 1e-12
