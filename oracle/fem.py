"""ORACLE (test infrastructure only) -- plain FP64 finite element operator
decomposition for the regularised p-Laplacian on hexahedral Q_k meshes.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything under ``oracle/``.  Nothing here is shared
with, imported by, or imports the HIP path.

What is computed (paper, Fig. 1 and Eq. (1)-(3)):

* The operator factorises as A = P^T G^T B^T D B G P.  On one subdomain P is
  the identity.  G restricts an L-vector to element DOFs (fancy indexing
  through the element-to-DOF table), G^T sums element contributions back
  (``np.bincount`` with weights), B evaluates reference gradients at the
  quadrature points with *dense* per-element Kronecker matrices, and D is the
  pointwise flux.
* Eq. (1): R(u) = M (G^T B^T D(B G M u) - b), the masked nonlinear action
  (homogeneous Dirichlet rows are zero; M is the 0/1 interior mask).
* Eq. (2): J(u) v = M G^T B^T J_D(u_q) B G M v with J_D the *hand-derived*
  tangent dF/dg = a^(r-1) (a I + (p-2) g g^T), a = eps^2 + |g|^2,
  r = (p-2)/2 -- an analytic linearisation, not automatic differentiation.
* Eq. (3): element tangent K_e = B^T J_D B, assembled into a sparse matrix for
  small meshes.
* The model problem is the p-Laplacian -div((eps^2+|grad u|^2)^((p-2)/2)
  grad u) = f on the unit cube (the paper's numerical experiment); its energy
  E(u) = sum_e rho_e int (1/p) a^(p/2) - b^T M u has R = grad E exactly at the
  discrete level.
* The design sensitivity of a functional Phi(u) under R(u; rho) = 0 (the
  adjoint paragraph after Eq. (3)): J lambda = M dPhi/du, then
  dPhi/drho_e = -lambda^T dR/drho_e = -int_e a^r grad u . grad lambda.

Geometry is the trilinear map of each hexahedron's 8 vertices; reference
element [0,1]^3; node order x fastest.  rho multiplies the flux and the energy
density of its element (not the load).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .rules import gauss_legendre, gll_nodes, lagrange


# --------------------------------------------------------------------------
# Pointwise operator D (quadrature-point level).  Module-level functions so
# that tests can plant mistakes in them and see the pins fail.
# --------------------------------------------------------------------------

def physical_gradient(Jinv: np.ndarray, ghat: np.ndarray) -> np.ndarray:
    """grad_x u = Jg^{-T} grad_xi u.  Jinv[..., i, j] = (Jg^{-1})_{ij}."""
    return np.einsum("...ba,...b->...a", Jinv, ghat)


def pull_back(Jinv: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Reference-space flux Jg^{-1} F, so that F . grad_x phi = (Jg^{-1}F) . grad_xi phi."""
    return np.einsum("...ab,...b->...a", Jinv, F)


def flux(g: np.ndarray, p: float, eps: float) -> np.ndarray:
    """F(g) = (eps^2 + |g|^2)^((p-2)/2) g."""
    a = eps * eps + np.sum(g * g, axis=-1)
    return (a ** ((p - 2.0) / 2.0))[..., None] * g


def tangent_matrix(g: np.ndarray, p: float, eps: float) -> np.ndarray:
    """dF/dg = a^(r-1) (a I + (p-2) g g^T), hand-derived from F(g).

    a = 0 only when eps = 0 and g = 0 (allowed for p >= 2).  There the
    formula reads 0^(r-1) * 0; its limit as g -> 0 is taken instead: the
    matrix has eigenvalues a^r and (p-1) a^r (with eps = 0, |g|^2 = a), so it
    tends to 0 for p > 2 and equals I for p = 2."""
    r = (p - 2.0) / 2.0
    a = eps * eps + np.sum(g * g, axis=-1)
    eye = np.eye(3)
    T = a[..., None, None] * eye + (p - 2.0) * g[..., :, None] * g[..., None, :]
    zero = a == 0.0
    out = (np.where(zero, 1.0, a) ** (r - 1.0))[..., None, None] * T
    if np.any(zero):
        out[zero] = eye if p == 2.0 else 0.0
    return out


def flux_tangent(g: np.ndarray, dg: np.ndarray, p: float, eps: float) -> np.ndarray:
    """dF = (dF/dg) dg."""
    return np.einsum("...ab,...b->...a", tangent_matrix(g, p, eps), dg)


def energy_density(g: np.ndarray, p: float, eps: float) -> np.ndarray:
    """W(g) = (1/p) (eps^2 + |g|^2)^(p/2); dW/dg = F(g)."""
    a = eps * eps + np.sum(g * g, axis=-1)
    return a ** (p / 2.0) / p


def flux_coefficient(g: np.ndarray, p: float, eps: float) -> np.ndarray:
    """a^r, the scalar multiplying g in F(g) (dR/drho integrand)."""
    a = eps * eps + np.sum(g * g, axis=-1)
    return a ** ((p - 2.0) / 2.0)


# --------------------------------------------------------------------------
# Trilinear geometry
# --------------------------------------------------------------------------

def trilinear_tables(pts1d: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Q1 shape values N[q, v] and reference derivatives dN[q, v, d] at the
    tensor quadrature points (q = qx + nq (qy + nq qz)); vertex v = i + 2j + 4l."""
    n = [lambda t: 1.0 - t, lambda t: t]
    dn = [lambda t: -np.ones_like(t), lambda t: np.ones_like(t)]
    qz, qy, qx = np.meshgrid(pts1d, pts1d, pts1d, indexing="ij")
    X, Y, Z = qx.ravel(), qy.ravel(), qz.ravel()
    NQ = X.size
    N = np.zeros((NQ, 8))
    dN = np.zeros((NQ, 8, 3))
    for l in range(2):
        for j in range(2):
            for i in range(2):
                v = i + 2 * j + 4 * l
                N[:, v] = n[i](X) * n[j](Y) * n[l](Z)
                dN[:, v, 0] = dn[i](X) * n[j](Y) * n[l](Z)
                dN[:, v, 1] = n[i](X) * dn[j](Y) * n[l](Z)
                dN[:, v, 2] = n[i](X) * n[j](Y) * dn[l](Z)
    return N, dN


class Discretisation:
    """One p-Laplacian discretisation: mesh, tables, operators."""

    def __init__(self, nx, ny, nz, k, nq, p, eps, vertices=None, rho=None,
                 f=None, load=None, chunk=4096, compute_load=True):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.k, self.nq = int(k), int(nq)
        self.p, self.eps = float(p), float(eps)
        self.chunk = int(chunk)
        self.D1 = self.k + 1
        self.Ne = self.D1 ** 3
        self.NQ = self.nq ** 3
        self.Lx = self.k * self.nx + 1
        self.Ly = self.k * self.ny + 1
        self.Lz = self.k * self.nz + 1
        self.N = self.Lx * self.Ly * self.Lz
        self.E = self.nx * self.ny * self.nz

        # 1D rules and dense element matrices (x fastest: kron(z, kron(y, x)))
        self.nodes1d = gll_nodes(self.k)
        self.qp1d, self.qw1d = gauss_legendre(self.nq)
        L, dL = lagrange(self.nodes1d, self.qp1d)
        self.L1, self.dL1 = L, dL
        self.Bval = np.kron(L, np.kron(L, L))
        self.Bgrad = np.stack([np.kron(L, np.kron(L, dL)),
                               np.kron(L, np.kron(dL, L)),
                               np.kron(dL, np.kron(L, L))])
        self.w = np.kron(self.qw1d, np.kron(self.qw1d, self.qw1d))

        # element-to-DOF table and interior mask
        ez, ey, ex = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                                 np.arange(self.nx), indexing="ij")
        c, b, a = np.meshgrid(np.arange(self.D1), np.arange(self.D1),
                              np.arange(self.D1), indexing="ij")
        I = self.k * ex.ravel()[:, None] + a.ravel()[None, :]
        J = self.k * ey.ravel()[:, None] + b.ravel()[None, :]
        K = self.k * ez.ravel()[:, None] + c.ravel()[None, :]
        self.elem_dofs = (I + self.Lx * (J + self.Ly * K)).astype(np.int64)
        Kz, Jy, Ix = np.meshgrid(np.arange(self.Lz), np.arange(self.Ly),
                                 np.arange(self.Lx), indexing="ij")
        inner = ((Ix > 0) & (Ix < self.Lx - 1) & (Jy > 0) & (Jy < self.Ly - 1)
                 & (Kz > 0) & (Kz < self.Lz - 1))
        self.mask = inner.ravel().astype(np.float64)

        # vertices and each element's 8 corners
        if vertices is None:
            xs = np.arange(self.nx + 1) / self.nx
            ys = np.arange(self.ny + 1) / self.ny
            zs = np.arange(self.nz + 1) / self.nz
            vz, vy, vx = np.meshgrid(zs, ys, xs, indexing="ij")
            vertices = np.stack([vx.ravel(), vy.ravel(), vz.ravel()], axis=1)
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        corners = []
        for l in range(2):
            for j in range(2):
                for i in range(2):
                    corners.append((ex.ravel() + i) + (self.nx + 1) * (
                        (ey.ravel() + j) + (self.ny + 1) * (ez.ravel() + l)))
        self.elem_verts = np.stack(corners, axis=1)
        self.N8, self.dN8 = trilinear_tables(self.qp1d)

        self.rho = (np.ones(self.E) if rho is None
                    else np.asarray(rho, dtype=np.float64).copy())
        self.f = f
        if load is not None:
            self.b = np.asarray(load, dtype=np.float64).copy()
        elif compute_load:
            self.b = self.load_vector(f)
        else:
            self.b = None   # large meshes: load entries computed where sampled

    # ------------------------------------------------------------------
    def with_(self, **kw) -> "Discretisation":
        args = dict(nx=self.nx, ny=self.ny, nz=self.nz, k=self.k, nq=self.nq,
                    p=self.p, eps=self.eps, vertices=self.vertices,
                    rho=self.rho, load=self.b, chunk=self.chunk)
        args.update(kw)
        if "f" in kw:
            args.pop("load")
        return Discretisation(**args)

    def _chunks(self, elems):
        for s in range(0, len(elems), self.chunk):
            yield elems[s:s + self.chunk]

    def geometry(self, elems):
        """Per element and quadrature point: Jg, detJ, Jg^{-1}, x_q."""
        X = self.vertices[self.elem_verts[elems]]              # (ne, 8, 3)
        Jg = np.einsum("eva,qvb->eqab", X, self.dN8)           # d x_a / d xi_b
        detJ = np.linalg.det(Jg)
        Jinv = np.linalg.inv(Jg)
        xq = np.einsum("eva,qv->eqa", X, self.N8)
        return Jg, detJ, Jinv, xq

    # --- G and G^T ------------------------------------------------------
    def gather(self, u, elems, masked=True):
        """E-vector of M u (or of u when ``masked`` is False), shape (ne, Ne)."""
        src = self.mask * u if masked else np.asarray(u, dtype=np.float64)
        return src[self.elem_dofs[elems]]

    def assemble(self, Y, elems):
        """G^T: sum element vectors into an L-vector (unmasked)."""
        return np.bincount(self.elem_dofs[elems].ravel(), weights=Y.ravel(),
                           minlength=self.N)

    # --- B and B^T ------------------------------------------------------
    def ref_gradient(self, U):
        """B: reference gradients at quadrature points, shape (ne, NQ, 3)."""
        return np.stack([U @ self.Bgrad[d].T for d in range(3)], axis=-1)

    def ref_gradient_T(self, Fhat):
        """B^T: sum_d Bgrad_d^T Fhat_d, shape (ne, Ne)."""
        return sum(Fhat[..., d] @ self.Bgrad[d] for d in range(3))

    # --- element level --------------------------------------------------
    def _all(self, elems):
        return np.arange(self.E) if elems is None else np.asarray(elems)

    def element_residual(self, u, elems, masked=True):
        _, detJ, Jinv, _ = self.geometry(elems)
        g = physical_gradient(Jinv, self.ref_gradient(self.gather(u, elems, masked)))
        F = flux(g, self.p, self.eps)
        scale = self.rho[elems][:, None] * self.w[None, :] * detJ
        return self.ref_gradient_T(scale[..., None] * pull_back(Jinv, F))

    def element_jvp(self, u, v, elems):
        _, detJ, Jinv, _ = self.geometry(elems)
        g = physical_gradient(Jinv, self.ref_gradient(self.gather(u, elems)))
        dg = physical_gradient(Jinv, self.ref_gradient(self.gather(v, elems)))
        dF = flux_tangent(g, dg, self.p, self.eps)
        scale = self.rho[elems][:, None] * self.w[None, :] * detJ
        return self.ref_gradient_T(scale[..., None] * pull_back(Jinv, dF))

    # --- global operators -----------------------------------------------
    def apply_unmasked(self, u, elems=None):
        """A(M u) = G^T B^T D(B G M u) without the load or output mask."""
        elems = self._all(elems)
        out = np.zeros(self.N)
        for ch in self._chunks(elems):
            out += self.assemble(self.element_residual(u, ch), ch)
        return out

    def apply_full(self, u):
        """G^T B^T D(B G u) with no Dirichlet mask at all (input or output)."""
        out = np.zeros(self.N)
        for ch in self._chunks(np.arange(self.E)):
            out += self.assemble(self.element_residual(u, ch, masked=False), ch)
        return out

    def node_coordinates(self):
        """Physical position of every L-vector node (trilinear image of the
        reference GLL lattice of each element)."""
        xi = self.nodes1d
        cz, cy, cx = np.meshgrid(xi, xi, xi, indexing="ij")
        X, Y, Z = cx.ravel(), cy.ravel(), cz.ravel()
        N8 = np.zeros((self.Ne, 8))
        for l in range(2):
            for j in range(2):
                for i in range(2):
                    N8[:, i + 2 * j + 4 * l] = ((X if i else 1 - X) * (Y if j else 1 - Y)
                                                * (Z if l else 1 - Z))
        xyz = np.einsum("eva,nv->ena", self.vertices[self.elem_verts], N8)
        out = np.zeros((self.N, 3))
        out[self.elem_dofs.ravel()] = xyz.reshape(-1, 3)
        return out

    def residual(self, u, elems=None):
        """Eq. (1) with Dirichlet mask: R(u) = M (A(M u) - b)."""
        return self.mask * (self.apply_unmasked(u, elems) - self.b)

    def jvp(self, u, v, elems=None):
        """Eq. (2) applied matrix-free: J(u) v = M J_A(M u) M v."""
        elems = self._all(elems)
        out = np.zeros(self.N)
        for ch in self._chunks(elems):
            out += self.assemble(self.element_jvp(u, v, ch), ch)
        return self.mask * out

    def energy(self, u):
        """E(u) = sum_e rho_e sum_q w detJ W(grad u) - b^T M u."""
        total = 0.0
        for ch in self._chunks(np.arange(self.E)):
            _, detJ, Jinv, _ = self.geometry(ch)
            g = physical_gradient(Jinv, self.ref_gradient(self.gather(u, ch)))
            total += np.sum(self.rho[ch][:, None] * self.w[None, :] * detJ
                            * energy_density(g, self.p, self.eps))
        return total - np.dot(self.b, self.mask * u)

    def load_vector(self, f=None, elems=None):
        """b_i = sum_e sum_q w detJ f(x_q) phi_i(x_q); f = 1 by default."""
        out = np.zeros(self.N)
        for ch in self._chunks(self._all(elems)):
            _, detJ, _, xq = self.geometry(ch)
            fq = np.ones_like(detJ) if f is None else f(xq[..., 0], xq[..., 1], xq[..., 2])
            out += self.assemble((self.w[None, :] * detJ * fq) @ self.Bval, ch)
        return out

    def element_tangents(self, u, elems):
        """Eq. (3): K_e = B^T J_D B = sum_q Bgrad^T (rho w detJ Jinv (dF/dg) Jinv^T) Bgrad
        at the element values of M u, shape (ne, Ne, Ne), local numbering."""
        _, detJ, Jinv, _ = self.geometry(elems)
        g = physical_gradient(Jinv, self.ref_gradient(self.gather(u, elems)))
        T = tangent_matrix(g, self.p, self.eps)
        C = np.einsum("eqij,eqjk,eqlk->eqil", Jinv, T, Jinv)
        C *= (self.rho[elems][:, None] * self.w[None, :] * detJ)[..., None, None]
        return np.einsum("iqa,eqij,jqb->eab", self.Bgrad, C, self.Bgrad)

    def jacobian(self, u):
        """Eq. (3) per element, assembled: M J_A(M u) M as a CSR matrix."""
        rows, cols, vals = [], [], []
        for ch in self._chunks(np.arange(self.E)):
            Ke = self.element_tangents(u, ch)
            d = self.elem_dofs[ch]
            rows.append(np.repeat(d, self.Ne, axis=1).ravel())
            cols.append(np.tile(d, (1, self.Ne)).ravel())
            vals.append(Ke.ravel())
        K = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                            np.concatenate(cols))), shape=(self.N, self.N)).tocsr()
        Md = sps.diags(self.mask)
        return (Md @ K @ Md).tocsr()

    def grad_rho(self, u, lam, elems=None):
        """dPhi/drho_e = -sum_q w detJ a^r grad(Mu) . grad(M lam), per element
        (all elements, or only the listed ones: entries of the others are 0)."""
        out = np.zeros(self.E)
        for ch in self._chunks(self._all(elems)):
            _, detJ, Jinv, _ = self.geometry(ch)
            g = physical_gradient(Jinv, self.ref_gradient(self.gather(u, ch)))
            gl = physical_gradient(Jinv, self.ref_gradient(self.gather(lam, ch)))
            integrand = flux_coefficient(g, self.p, self.eps) * np.sum(g * gl, axis=-1)
            out[ch] = -np.sum(self.w[None, :] * detJ * integrand, axis=1)
        return out

    # --- sampled outputs for meshes too large to apply whole ---------------
    def elements_touching(self, dofs):
        sel = np.zeros(self.N, dtype=bool)
        sel[np.asarray(dofs)] = True
        return np.nonzero(sel[self.elem_dofs].any(axis=1))[0]

    def residual_at(self, u, dofs):
        """R(u) at the listed DOFs only (same arithmetic as ``residual``)."""
        dofs = np.asarray(dofs)
        elems = self.elements_touching(dofs)
        b = self.b if self.b is not None else self.load_vector(self.f, elems)
        return (self.mask * (self.apply_unmasked(u, elems) - b))[dofs]

    def jvp_at(self, u, v, dofs):
        return self.jvp(u, v, self.elements_touching(dofs))[np.asarray(dofs)]
