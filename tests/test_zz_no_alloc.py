"""The Jacobian action that allocates nothing (feod_jacobian_apply_noalloc,
for callers that cannot allocate): called through the C ABI, its output must
equal feod_jacobian_apply's bit for bit (same kernels, same summation order)
on two calls in a row, the second on a smaller mesh, in FP64 and mixed
precision; the oracle checks the FP64 result too."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2506_00746_amd as feod
from gpu_helpers import announce, dev, host, relerr, setup
from workloads import Workload

pytestmark = pytest.mark.gpu

# a larger then a smaller input: 12^3 Q3 (7.1 MB FP64 E-vector), then 5x4x3 Q2 curved
CASES = [Workload("noalloc-12c-q3", 12, 12, 12, 3, 5, 4.0, 1e-3, 61, rho=True),
         Workload("noalloc-5x4x3-q2-curved", 5, 4, 3, 2, 3, 3.0, 1e-2, 62, perturb=True, rho=True)]


def _noalloc(prob, u, v, out, prec):
    L = feod.lib()
    prob._sync_stream()
    st = L.feod_jacobian_apply_noalloc(prob._ctx, u.data_ptr(), v.data_ptr(), out.data_ptr(),
                                       feod.feod.PREC[prec])
    assert st == 0, L.feod_last_error(prob._ctx).decode()
    return out


def test_noalloc_jacobian_apply_matches_workspace_variant():
    for w in CASES:
        announce("noalloc Jacobian apply", w)
        prob, ora, inp = setup(w)
        u, v = dev(inp["u"]), dev(inp["v"])
        for prec in ("fp64", "mixed"):
            ref = prob.jacobian_apply(u, v, prec=prec)
            out = torch.full_like(u, float("nan"))
            _noalloc(prob, u, v, out, prec)
            assert torch.equal(out, ref), (w.name, prec)
            if prec == "fp64":
                assert relerr(host(out), ora.jvp(inp["u"], inp["v"])) <= 1e-12
        # the scratch keeps the last call's contents: a second call with a
        # different direction must not see the first one's E-vector
        v2 = dev(-0.5 * inp["v"])
        out2 = torch.empty_like(u)
        _noalloc(prob, u, v2, out2, "fp64")
        assert torch.equal(out2, prob.jacobian_apply(u, v2)), w.name
        del prob
        torch.cuda.synchronize()


def test_noalloc_rejects_large_mesh_and_bad_args():
    w = CASES[1]
    prob, _, inp = setup(w, oracle=False)
    u = dev(inp["u"])
    L = feod.lib()
    out = torch.empty_like(u)
    assert L.feod_jacobian_apply_noalloc(prob._ctx, u.data_ptr(), u.data_ptr(), u.data_ptr(), 0) == \
        feod.feod.FEOD_EINVAL  # output aliases the inputs
    assert L.feod_jacobian_apply_noalloc(prob._ctx, u.data_ptr(), None, out.data_ptr(), 0) == feod.feod.FEOD_EINVAL
    assert L.feod_jacobian_apply_noalloc(prob._ctx, u.data_ptr(), u.data_ptr(), out.data_ptr(), 7) == \
        feod.feod.FEOD_EINVAL


def test_noalloc_jacobian_apply_in_a_captured_graph():
    """The allocation-free Jacobian action captured once in a HIP graph and
    replayed with the direction v rewritten between replays (eager work and a
    synchronisation between them): every replay equals the eager
    feod_jacobian_apply of the same v bit for bit, FP64 and mixed."""
    w = CASES[1]
    announce("noalloc Jacobian apply in a graph", w)
    prob, _, inp = setup(w, oracle=False)
    u, v = dev(inp["u"]), dev(inp["v"])
    rng = np.random.default_rng(63)
    for prec in ("fp64", "mixed"):
        out = torch.zeros_like(u)
        side = torch.cuda.Stream(device="cuda:0")
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):  # an eager call before capture
            _noalloc(prob, u, v, out, prec)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            _noalloc(prob, u, v, out, prec)
        torch.cuda.synchronize()
        for rep in range(3):
            v.copy_(dev(rng.standard_normal(u.numel())))
            ref = prob.jacobian_apply(u, v, prec=prec)
            torch.cuda.synchronize()
            out.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (prec, rep)
        del g
        torch.cuda.synchronize()
