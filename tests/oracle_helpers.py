"""Independent closed forms used to pin the oracle.

Exact 1D finite element matrices by polynomial arithmetic (no quadrature), and
their Kronecker combinations for the p = 2 special case on affine lattices.
"""
import numpy as np
from numpy.polynomial import Polynomial


def lagrange_polys(nodes):
    """Lagrange basis polynomials through ``nodes`` built by fitting, not by
    the product formula."""
    n = len(nodes)
    V = np.vander(nodes, n, increasing=True)
    coef = np.linalg.solve(V, np.eye(n))           # column a = coefficients of l_a
    return [Polynomial(coef[:, a]) for a in range(n)]


def exact_1d_matrices(nodes, n_el, h):
    """Global 1D stiffness K1, mass M1 (exact integrals) and load m = M1 @ 1
    for n_el uniform elements of size h with Q_k nodes ``nodes`` on [0,1]."""
    polys = lagrange_polys(nodes)
    d = len(nodes)
    Kh = np.zeros((d, d))
    Mh = np.zeros((d, d))
    for a in range(d):
        for b in range(d):
            pk = (polys[a].deriv() * polys[b].deriv()).integ()
            pm = (polys[a] * polys[b]).integ()
            Kh[a, b] = pk(1.0) - pk(0.0)
            Mh[a, b] = pm(1.0) - pm(0.0)
    k = d - 1
    L = k * n_el + 1
    K1 = np.zeros((L, L))
    M1 = np.zeros((L, L))
    for e in range(n_el):
        sl = slice(k * e, k * e + d)
        K1[sl, sl] += Kh / h
        M1[sl, sl] += Mh * h
    return K1, M1, M1 @ np.ones(L)


def kronecker_laplacian(nodes, nx, ny, nz):
    """K = Mz(x)My(x)Kx + Mz(x)Ky(x)Mx + Kz(x)My(x)Mx and b = mz(x)my(x)mx
    (x fastest numbering) for the uniform nx*ny*nz lattice of the unit cube."""
    Kx, Mx, mx = exact_1d_matrices(nodes, nx, 1.0 / nx)
    Ky, My, my = exact_1d_matrices(nodes, ny, 1.0 / ny)
    Kz, Mz, mz = exact_1d_matrices(nodes, nz, 1.0 / nz)
    K = (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx))
         + np.kron(Kz, np.kron(My, Mx)))
    b = np.kron(mz, np.kron(my, mx))
    return K, b


def relerr(x, ref):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(ref)) / np.linalg.norm(ref))
