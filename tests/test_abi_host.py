"""C ABI checks that need no GPU: the library loads, exports every declared
symbol, and its host-side setup (1D tables, maps, load vector, validation)
agrees with the independent oracle."""
import ctypes

import numpy as np
import pytest

import paper_2506_00746_amd as feod
from oracle import Discretisation
from workloads import Workload, make_inputs


def test_library_exports_every_declared_symbol():
    L = feod.lib()
    names = feod.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    for n in ("feod_setup_mesh", "feod_residual", "feod_jacobian_apply", "feod_newton_solve",
              "feod_adjoint_gradient"):
        assert n in names


@pytest.mark.parametrize("k,nq", [(1, 2), (2, 3), (2, 4), (3, 5), (4, 6), (7, 9)])
def test_tables_match_oracle(k, nq):
    h = feod.HostSetup(1, 1, 1, k, nq)
    d = Discretisation(1, 1, 1, k, nq, 3.0, 1e-2)
    assert np.abs(h.nodes - d.nodes1d).max() < 1e-15
    assert np.abs(h.qpts - d.qp1d).max() < 1e-15
    assert np.abs(h.qwts - d.qw1d).max() < 1e-15
    assert np.abs(h.B - d.L1).max() < 1e-14
    assert np.abs(h.D - d.dL1).max() < 1e-12 * max(1, np.abs(d.dL1).max())


@pytest.mark.parametrize("shape,k,nq", [((2, 3, 4), 2, 3), ((3, 2, 2), 3, 5), ((1, 1, 1), 1, 2),
                                        ((4, 4, 4), 2, 3)])
def test_maps_match_oracle(shape, k, nq):
    h = feod.HostSetup(*shape, k, nq)
    d = Discretisation(*shape, k, nq, 3.0, 1e-2)
    expect = np.where(d.mask[d.elem_dofs] > 0, d.elem_dofs, -1)
    assert np.array_equal(h.emap, expect)
    # transposed map: row i lists the E-vector positions (e * Ne + local) of
    # DOF i by ascending element
    flat = expect.ravel()
    for i in range(d.N):
        row = h.tidx[h.toff[i]:h.toff[i + 1]]
        assert np.array_equal(row, np.nonzero(flat == i)[0])


@pytest.mark.parametrize("perturb", [False, True])
def test_load_matches_oracle(perturb):
    w = Workload("t", 3, 2, 4, 2, 3, 3.0, 1e-2, 5, perturb=perturb)
    inp = make_inputs(w)
    h = feod.HostSetup(3, 2, 4, 2, 3, vertices=inp["vertices"])
    d = Discretisation(3, 2, 4, 2, 3, 3.0, 1e-2, vertices=inp["vertices"])
    assert np.abs(h.load - d.b).max() < 1e-15 * 100


def test_setup_rejects_bad_input():
    def setup(**kw):
        args = dict(nx=2, ny=2, nz=2, order_k=2, nq=3, p=3.0, eps=1e-2, vertices=None,
                    rho=None, load=None, stream=None)
        args.update(kw)
        d = feod.feod.MeshDesc(*[args[f] for f, _ in feod.feod.MeshDesc._fields_])
        ctx = ctypes.c_void_p()
        st = feod.lib().feod_setup_mesh(ctypes.byref(d), ctypes.byref(ctx))
        if st == 0:
            feod.lib().feod_destroy(ctx)
        return st, feod.lib().feod_last_error(None).decode()
    assert setup()[0] == 0
    assert setup(nx=0)[0] == feod.feod.FEOD_EINVAL
    assert setup(p=1.0)[0] == feod.feod.FEOD_EINVAL
    assert setup(p=float("nan"))[0] == feod.feod.FEOD_EINVAL
    assert setup(eps=-1.0)[0] == feod.feod.FEOD_EINVAL
    assert setup(eps=0.0, p=1.5)[0] == feod.feod.FEOD_EINVAL
    st, msg = setup(order_k=6, nq=2)
    assert st == feod.feod.FEOD_EUNSUPPORTED and "k=6" in msg
    # the largest meshes the 32-bit DOF and E-vector indices take, checked
    # before anything is allocated: N = 1601^3 > 2^31, then E Ne = 162^3 512 > 2^31
    # with N = 1135^3 < 2^31
    for big in (dict(nx=400, ny=400, nz=400, order_k=4, nq=6), dict(nx=162, ny=162, nz=162, order_k=7, nq=9)):
        st, msg = setup(**big)
        assert st == feod.feod.FEOD_EUNSUPPORTED and "too large" in msg, (big, msg)
    # inverted element
    w = Workload("t", 2, 2, 2, 2, 3, 3.0, 1e-2, 5, perturb=True)
    v = make_inputs(w)["vertices"].copy()
    v[13] = [0.9, 0.9, 0.9]  # centre vertex pulled across its neighbours
    st, msg = setup(vertices=v.ctypes.data)
    assert st == feod.feod.FEOD_EINVAL and "detJ" in msg


def test_unbound_context_and_null_args():
    L = feod.lib()
    d = feod.feod.MeshDesc(2, 2, 2, 2, 3, 3.0, 1e-2, None, None, None, None)
    ctx = ctypes.c_void_p()
    assert L.feod_setup_mesh(ctypes.byref(d), ctypes.byref(ctx)) == 0
    try:
        assert L.feod_residual(ctx, 8, 16, 0) == feod.feod.FEOD_ESTATE
        nb = ctypes.c_size_t()
        assert L.feod_workspace_bytes(ctx, ctypes.byref(nb)) == 0 and nb.value > 0
        assert L.feod_bind_workspace(ctx, None, nb.value) == feod.feod.FEOD_EINVAL
        assert L.feod_bind_workspace(ctx, 256, 16) == feod.feod.FEOD_EINVAL  # too small
        b = ctypes.c_double()
        f = ctypes.c_double()
        assert L.feod_kernel_cost(ctx, 1, 0, ctypes.byref(b), ctypes.byref(f)) == 0
        assert b.value > 0 and f.value > 0
    finally:
        L.feod_destroy(ctx)
    assert L.feod_destroy(None) == 0


def test_profile_summary_parser_and_source_hash(tmp_path):
    from paper_2506_00746_amd import profiling
    sha = profiling.kernel_source_sha256()
    assert len(sha) == 64
    p = tmp_path / "x.md"
    p.write_text(f"# x\n\ntraffic_bytes_per_launch: 3.2e+07\nkernel_source_sha256: {sha}\n")
    assert profiling.read_traffic(str(p)) == (3.2e7, sha)
    assert profiling.read_traffic(str(tmp_path / "missing.md")) == (None, None)


def test_cost_model_matches_its_formula():
    """The roofline's algorithmic counts: FLOPs = E (passes S + nq^3 f_D) with
    S = 4 nq D1^3 + 6 nq^2 D1^2 + 6 nq^3 D1 per sum-factorised pass, f_D the
    per-point count of the pointwise operator; bytes = unique L-vector reads
    + E-vector writes (+ rho, vertices, stored gradients where used)."""
    from workloads import WORKLOADS, make_inputs
    cases = {"c2": ("jvp", 2 + 17 + 9 + 0 + 4),          # affine, r = 1
             "c4": ("jvp", 2 + 17 + 9 + 12 + 4),         # affine, r = 1/2
             "c5": ("jvp", 2 + 17 + 9 + 12 + 99)}        # curved, r = 1/2
    for name, (op, f_d) in cases.items():
        w = WORKLOADS[name]
        inp = make_inputs(w)
        hs = feod.HostSetup(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"], rho=inp["rho"])
        d1, nq, e, n = w.k + 1, w.nq, w.n_elems, w.n_dofs
        s = 4 * nq * d1 ** 3 + 6 * nq ** 2 * d1 ** 2 + 6 * nq ** 3 * d1
        flops = e * (3 * s + nq ** 3 * f_d)
        nbytes = 2 * 8.0 * n + 8.0 * e * d1 ** 3
        if inp["rho"] is not None:
            nbytes += 8.0 * e
        if inp["vertices"] is not None:
            nbytes += 24.0 * (w.nx + 1) * (w.ny + 1) * (w.nz + 1)
        b, f = hs.cost[(op, "fp64")]
        assert f == pytest.approx(flops, rel=1e-14), name
        assert b == pytest.approx(nbytes, rel=1e-14), name
        b32, f32 = hs.cost[(op, "mixed")]
        assert f32 == f and b32 == pytest.approx(nbytes - 4.0 * e * d1 ** 3, rel=1e-14)
        # element-level AD tangents: one Jacobian action per local DOF, u read
        # once, K_e written
        be, fe = hs.cost[("elm", "fp64")]
        assert fe == pytest.approx(d1 ** 3 * flops, rel=1e-14), name
        assert be == pytest.approx(nbytes - 8.0 * n - 8.0 * e * d1 ** 3 + 8.0 * e * d1 ** 6, rel=1e-14), name


def test_noalloc_apply_rejects_meshes_beyond_its_scratch():
    """feod_jacobian_apply_noalloc holds the E-vector in a 32 MiB static
    array: a 90^3 Q1 mesh (46.7 MB FP64 E-vector) is refused with
    FEOD_EINVAL before any GPU work, while its FP32 E-vector (23.3 MB) fits
    and the unbound context is then the error."""
    L = feod.lib()
    d = feod.feod.MeshDesc(90, 90, 90, 1, 2, 3.0, 1e-2, None, None, None, None)
    ctx = ctypes.c_void_p()
    assert L.feod_setup_mesh(ctypes.byref(d), ctypes.byref(ctx)) == 0
    try:
        assert L.feod_jacobian_apply_noalloc(ctx, 256, 512, 768, 0) == feod.feod.FEOD_EINVAL
        msg = L.feod_last_error(ctx).decode()
        assert "46656000" in msg and str(32 << 20) in msg
        assert L.feod_jacobian_apply_noalloc(ctx, 256, 512, 768, 1) == feod.feod.FEOD_ESTATE
        assert L.feod_jacobian_apply_noalloc(ctx, 256, 512, 768, 5) == feod.feod.FEOD_EINVAL
    finally:
        L.feod_destroy(ctx)
    assert L.feod_jacobian_apply_noalloc(None, 256, 512, 768, 0) == feod.feod.FEOD_EINVAL
