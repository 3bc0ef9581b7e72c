"""ctypes binding of ``libfeod.so`` (C ABI in ``include/feod.h``).

Argument marshalling only: every step of the operator runs in the library's
HIP kernels.  PyTorch provides device memory (vectors and the library
workspace) and the stream.  The library must be built in-tree
(``paper_2506_00746_amd/build.py``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfeod.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "feod.h")

FEOD_OK, FEOD_EINVAL, FEOD_EUNSUPPORTED, FEOD_EHIP, FEOD_ENOCONV, FEOD_ENONFINITE, \
    FEOD_EBREAKDOWN, FEOD_ESTATE = range(8)
STATUS_NAMES = {0: "FEOD_OK", 1: "FEOD_EINVAL", 2: "FEOD_EUNSUPPORTED", 3: "FEOD_EHIP",
                4: "FEOD_ENOCONV", 5: "FEOD_ENONFINITE", 6: "FEOD_EBREAKDOWN", 7: "FEOD_ESTATE"}
PREC = {"fp64": 0, "mixed": 1}
OPS = {"residual": 0, "jvp": 1, "resjvp": 2, "energy": 3, "grad": 4, "diag": 5, "pa_setup": 6, "jvp_pa": 7,
       "elm": 8, "jvp_hand": 9}


class FeodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("order_k", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("p", ctypes.c_double), ("eps", ctypes.c_double),
                ("vertices", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("load", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("cg_rtol_floor", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("max_cg", ctypes.c_int32),
                ("max_ls", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("init_poisson", ctypes.c_int32),
                ("jacobi", ctypes.c_int32), ("partial_assembly", ctypes.c_int32)]


class SolverReport(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("cg_iters_total", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("ls_halvings_total", ctypes.c_int32),
                ("res0", ctypes.c_double), ("res_final", ctypes.c_double),
                ("ref_norm", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_SIGS = {
    "feod_default_opts": (None, [_P]),
    "feod_setup_mesh": (ctypes.c_int, [_P, _P]),
    "feod_workspace_bytes": (ctypes.c_int, [_P, _P]),
    "feod_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "feod_sizes": (ctypes.c_int, [_P, _P, _P]),
    "feod_set_stream": (ctypes.c_int, [_P, _P]),
    "feod_set_map_mode": (ctypes.c_int, [_P, ctypes.c_int32]),
    "feod_set_tangent_mode": (ctypes.c_int, [_P, ctypes.c_int32]),
    "feod_residual": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "feod_jacobian_apply": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int]),
    "feod_jacobian_apply_noalloc": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    "feod_energy": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "feod_pa_setup": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "feod_jacobian_apply_pa": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "feod_element_tangents": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int64, _P]),
    "feod_element_tangents_elm": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_int64, _P]),
    "feod_element_vectors": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int]),
    "feod_jacobian_diagonal": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "feod_newton_solve": (ctypes.c_int, [_P, _P, _P, _P]),
    "feod_adjoint_gradient": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "feod_grad_rho": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    "feod_set_rho": (ctypes.c_int, [_P, _P]),
    "feod_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "feod_profile_read": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    "feod_kernel_cost": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int, _P, _P]),
    "feod_host_tables": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "feod_host_maps": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "feod_host_load": (ctypes.c_int, [_P, _P]),
    "feod_destroy": (ctypes.c_int, [_P]),
    "feod_last_error": (ctypes.c_char_p, [_P]),
}


def header_functions() -> list[str]:
    """Names of every function declared in include/feod.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(feod_[a-z_0-9]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    """Load the in-tree library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2506_00746_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, ctx=None):
    if status != FEOD_OK:
        msg = lib().feod_last_error(ctx)
        raise FeodError(status, msg.decode() if msg else "")


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    lib().feod_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k}")
        setattr(o, k, v)
    return o


def _dptr(t: torch.Tensor, n: int, name: str, device: torch.device | None = None) -> int:
    """Device address of a contiguous float64 GPU tensor of n entries (on
    ``device`` when given: the library's kernels run on its context's GPU)."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the problem on {device}")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} entries")
    return t.data_ptr()


def _host_array(x, n: int, name: str):
    import numpy as np
    if x is None:
        return None, None
    if isinstance(x, torch.Tensor):
        x = x.detach().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"{name} must have {n} entries, got {a.size}")
    return a, a.ctypes.data


class Problem:
    """One p-Laplacian discretisation bound to a GPU (C ABI context)."""

    def __init__(self, nx, ny, nz, order_k, nq, p, eps, vertices=None, rho=None, load=None,
                 device="cuda", stream=None):
        L = lib()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nx, self.ny, self.nz, self.k, self.nq = nx, ny, nz, order_k, nq
        self.p, self.eps = float(p), float(eps)
        n_dofs = (order_k * nx + 1) * (order_k * ny + 1) * (order_k * nz + 1)
        n_el = nx * ny * nz
        keep = []
        v_arr, v_ptr = _host_array(vertices, (nx + 1) * (ny + 1) * (nz + 1) * 3, "vertices")
        r_arr, r_ptr = _host_array(rho, n_el, "rho")
        l_arr, l_ptr = _host_array(load, n_dofs, "load")
        keep += [v_arr, r_arr, l_arr]
        d = MeshDesc(nx, ny, nz, order_k, nq, self.p, self.eps, v_ptr, r_ptr, l_ptr,
                     self.stream.cuda_stream)
        ctx = ctypes.c_void_p()
        _check(L.feod_setup_mesh(ctypes.byref(d), ctypes.byref(ctx)), None)
        self._ctx = ctx
        n = ctypes.c_int64()
        e = ctypes.c_int64()
        _check(L.feod_sizes(ctx, ctypes.byref(n), ctypes.byref(e)), ctx)
        self.n_dofs, self.n_elems = n.value, e.value
        nb = ctypes.c_size_t()
        _check(L.feod_workspace_bytes(ctx, ctypes.byref(nb)), ctx)
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            off = (-base) % 256
            _check(L.feod_bind_workspace(ctx, base + off, nb.value), ctx)

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            lib().feod_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, out=None):
        if out is None:
            return torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        self._ptr(out, self.n_dofs, "out")
        return out

    def _ptr(self, t, n, name):
        return _dptr(t, n, name, self.device)

    def _sync_stream(self):
        lib().feod_set_stream(self._ctx, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def set_map_mode(self, mode: str):
        """'lattice' (computed G/G^T, default) or 'explicit' (stored maps)."""
        _check(lib().feod_set_map_mode(self._ctx, {"lattice": 0, "explicit": 1}[mode]), self._ctx)

    def set_tangent_mode(self, mode: str):
        """'dual' (forward-mode dual numbers at the points, default) or 'hand'
        (the hand-coded J_D, for comparison) for the FP64 Jacobian actions."""
        _check(lib().feod_set_tangent_mode(self._ctx, {"dual": 0, "hand": 1}[mode]), self._ctx)

    # -- operators (Eq. (1), Eq. (2)) -------------------------------------
    def residual(self, u, out=None, prec="fp64"):
        out = self._vec(out)
        self._sync_stream()
        _check(lib().feod_residual(self._ctx, self._ptr(u, self.n_dofs, "u"), out.data_ptr(), PREC[prec]),
               self._ctx)
        return out

    def jacobian_apply(self, u, v, out=None, residual_out=None, prec="fp64"):
        out = self._vec(out)
        rp = None
        if residual_out is not None:
            rp = self._ptr(residual_out, self.n_dofs, "residual_out")
        self._sync_stream()
        _check(lib().feod_jacobian_apply(self._ctx, self._ptr(u, self.n_dofs, "u"),
                                         self._ptr(v, self.n_dofs, "v"), out.data_ptr(), rp, PREC[prec]),
               self._ctx)
        return out

    def jacobian_apply_noalloc(self, u, v, out, prec="fp64"):
        """J(u) v with the E-vector in the library's static scratch (no
        allocation by the library; ``out`` must be given)."""
        self._ptr(out, self.n_dofs, "out")
        self._sync_stream()
        _check(lib().feod_jacobian_apply_noalloc(self._ctx, self._ptr(u, self.n_dofs, "u"),
                                                 self._ptr(v, self.n_dofs, "v"), out.data_ptr(), PREC[prec]),
               self._ctx)
        return out

    def jvp(self, u, v, out=None, prec="fp64"):
        """J(u) v (the same call as ``jacobian_apply``)."""
        return self.jacobian_apply(u, v, out=out, prec=prec)

    def residual_and_jvp(self, u, v, prec="fp64"):
        r = self._vec()
        jv = self.jacobian_apply(u, v, residual_out=r, prec=prec)
        return r, jv

    def element_vectors(self, op: str, u, v=None, prec="fp64"):
        """Run only the element kernel (G, B, D, B^T) into the internal E-vector."""
        self._sync_stream()
        vp = None if v is None else self._ptr(v, self.n_dofs, "v")
        _check(lib().feod_element_vectors(self._ctx, {"residual": 0, "jvp": 1, "resjvp": 2}[op],
                                          self._ptr(u, self.n_dofs, "u"), vp, PREC[prec]), self._ctx)

    def element_tangents(self, u, first=0, count=None, out=None, method="res"):
        """K_e (Eq. 3) for elements first..first+count-1: (count, Ne, Ne) FP64.
        method "res": AD at the quadrature points, B^T J_D B contracted once;
        "elm": element-level forward AD, one Jacobian action per local DOF
        (the paper's ELM variant, for comparison)."""
        count = self.n_elems - first if count is None else count
        ne = (self.k + 1) ** 3
        if out is None:
            out = torch.empty((count, ne, ne), dtype=torch.float64, device=self.device)
        op = self._ptr(out, count * ne * ne, "out")
        fn = {"res": lib().feod_element_tangents, "elm": lib().feod_element_tangents_elm}[method]
        self._sync_stream()
        _check(fn(self._ctx, self._ptr(u, self.n_dofs, "u"), first, count, op), self._ctx)
        return out

    def pa_setup(self, u, prec="fp64"):
        """Partial assembly: store the reference gradients of M u at all points."""
        self._sync_stream()
        _check(lib().feod_pa_setup(self._ctx, self._ptr(u, self.n_dofs, "u"), PREC[prec]), self._ctx)

    def jacobian_apply_pa(self, v, out=None, prec="fp64"):
        """J(u) v at the u of the last pa_setup (same precision)."""
        out = self._vec(out)
        self._sync_stream()
        _check(lib().feod_jacobian_apply_pa(self._ctx, self._ptr(v, self.n_dofs, "v"), out.data_ptr(), PREC[prec]),
               self._ctx)
        return out

    def energy(self, u, prec="fp64"):
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        self._sync_stream()
        _check(lib().feod_energy(self._ctx, self._ptr(u, self.n_dofs, "u"), e.data_ptr(), PREC[prec]), self._ctx)
        return e

    def jacobian_diagonal(self, u, out=None, prec="fp64"):
        out = self._vec(out)
        self._sync_stream()
        _check(lib().feod_jacobian_diagonal(self._ctx, self._ptr(u, self.n_dofs, "u"), out.data_ptr(),
                                            PREC[prec]), self._ctx)
        return out

    def grad_rho(self, u, lam, out=None, prec="fp64"):
        if out is None:
            out = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        self._ptr(out, self.n_elems, "out")
        self._sync_stream()
        _check(lib().feod_grad_rho(self._ctx, self._ptr(u, self.n_dofs, "u"), self._ptr(lam, self.n_dofs, "lambda"),
                                   out.data_ptr(), PREC[prec]), self._ctx)
        return out

    def set_rho(self, rho):
        rho = rho.detach().to(device=self.device, dtype=torch.float64).contiguous()
        self._sync_stream()
        _check(lib().feod_set_rho(self._ctx, self._ptr(rho, self.n_elems, "rho")), self._ctx)
        self._rho_keep = rho  # stream-ordered copy; keep alive until it ran

    # -- solvers -----------------------------------------------------------
    def newton_solve(self, u0=None, **opts):
        """Newton-CG from the p = 2 solution (u0 None) or from u0 (then the
        Poisson start is off unless init_poisson=1 is passed, which discards u0)."""
        o = default_opts(**opts)
        u = torch.zeros(self.n_dofs, dtype=torch.float64, device=self.device) if u0 is None \
            else u0.detach().to(device=self.device, dtype=torch.float64).clone()
        if "init_poisson" not in opts:
            o.init_poisson = 1 if u0 is None else 0
        rep = SolverReport()
        self._sync_stream()
        st = lib().feod_newton_solve(self._ctx, self._ptr(u, self.n_dofs, "u"), ctypes.byref(o), ctypes.byref(rep))
        _check(st, self._ctx)
        return u, rep.as_dict()

    def newton(self, u0=None, **opts):
        """The Newton-CG solve (the same call as ``newton_solve``)."""
        return self.newton_solve(u0, **opts)

    def adjoint_gradient(self, u, g_u, **opts):
        o = default_opts(**opts)
        lam = self._vec()
        grad = torch.empty(self.n_elems, dtype=torch.float64, device=self.device)
        rep = SolverReport()
        self._sync_stream()
        st = lib().feod_adjoint_gradient(self._ctx, self._ptr(u, self.n_dofs, "u"), self._ptr(g_u, self.n_dofs, "g_u"),
                                         lam.data_ptr(), grad.data_ptr(), ctypes.byref(o), ctypes.byref(rep))
        _check(st, self._ctx)
        return grad, lam, rep.as_dict()

    # -- instrumentation ---------------------------------------------------
    def profile(self, enable: bool):
        _check(lib().feod_profile(self._ctx, int(bool(enable))), self._ctx)

    def profile_read(self) -> dict:
        stats = (KernelStat * 64)()
        n = ctypes.c_int32()
        _check(lib().feod_profile_read(self._ctx, stats, 64, ctypes.byref(n)), self._ctx)
        return {stats[i].name.decode(): (stats[i].launches, stats[i].total_ms) for i in range(n.value)}

    def kernel_cost(self, op: str, prec="fp64"):
        b = ctypes.c_double()
        f = ctypes.c_double()
        _check(lib().feod_kernel_cost(self._ctx, OPS[op], PREC[prec], ctypes.byref(b), ctypes.byref(f)),
               self._ctx)
        return b.value, f.value


class HostSetup:
    """Host-only view of a context (no GPU needed): tables, maps and load."""

    def __init__(self, nx, ny, nz, order_k, nq, p=3.0, eps=1e-2, vertices=None, rho=None, load=None):
        import numpy as np
        L = lib()
        n_dofs = (order_k * nx + 1) * (order_k * ny + 1) * (order_k * nz + 1)
        v_arr, v_ptr = _host_array(vertices, (nx + 1) * (ny + 1) * (nz + 1) * 3, "vertices")
        r_arr, r_ptr = _host_array(rho, nx * ny * nz, "rho")
        l_arr, l_ptr = _host_array(load, n_dofs, "load")
        d = MeshDesc(nx, ny, nz, order_k, nq, float(p), float(eps), v_ptr, r_ptr, l_ptr, None)
        ctx = ctypes.c_void_p()
        _check(L.feod_setup_mesh(ctypes.byref(d), ctypes.byref(ctx)), None)
        try:
            D1 = order_k + 1
            E = nx * ny * nz
            f64 = lambda n: np.zeros(n, dtype=np.float64)  # noqa: E731
            self.nodes, self.qpts, self.qwts = f64(D1), f64(nq), f64(nq)
            self.B, self.D = f64(nq * D1), f64(nq * D1)
            _check(L.feod_host_tables(ctx, self.nodes.ctypes.data, self.qpts.ctypes.data,
                                      self.qwts.ctypes.data, self.B.ctypes.data, self.D.ctypes.data), ctx)
            self.B = self.B.reshape(nq, D1)
            self.D = self.D.reshape(nq, D1)
            nt = ctypes.c_int64()
            _check(L.feod_host_maps(ctx, None, None, None, ctypes.byref(nt)), ctx)
            self.emap = np.zeros(E * D1 ** 3, dtype=np.int32)
            self.toff = np.zeros(n_dofs + 1, dtype=np.int32)
            self.tidx = np.zeros(nt.value, dtype=np.int32)
            _check(L.feod_host_maps(ctx, self.emap.ctypes.data, self.toff.ctypes.data,
                                    self.tidx.ctypes.data, None), ctx)
            self.emap = self.emap.reshape(E, D1 ** 3)
            self.load = f64(n_dofs)
            _check(L.feod_host_load(ctx, self.load.ctypes.data), ctx)
            # the library's cost model: (algorithmic bytes, FLOPs) per launch
            self.cost = {}
            for op, code in OPS.items():
                if op == "diag":
                    continue
                for prec, pc in PREC.items():
                    b, f = ctypes.c_double(), ctypes.c_double()
                    _check(L.feod_kernel_cost(ctx, code, pc, ctypes.byref(b), ctypes.byref(f)), ctx)
                    self.cost[(op, prec)] = (b.value, f.value)
        finally:
            L.feod_destroy(ctx)


# The C ABI names, as module-level functions.
def setup_mesh(nx, ny, nz, order_k, nq, p, eps, **kw) -> Problem:
    return Problem(nx, ny, nz, order_k, nq, p, eps, **kw)


def residual(problem: Problem, u, out=None, prec="fp64"):
    return problem.residual(u, out=out, prec=prec)


def jacobian_apply(problem: Problem, u, v, out=None, residual_out=None, prec="fp64"):
    return problem.jacobian_apply(u, v, out=out, residual_out=residual_out, prec=prec)


def newton_solve(problem: Problem, u0=None, **opts):
    return problem.newton_solve(u0, **opts)


def adjoint_gradient(problem: Problem, u, g_u, **opts):
    return problem.adjoint_gradient(u, g_u, **opts)
