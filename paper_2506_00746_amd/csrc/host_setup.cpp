// Host-side setup: rules, tables, lattice maps and the load vector.
#include "host_setup.hpp"
#include "kernel_api.hpp"

#include <algorithm>
#include <cmath>

namespace feod {

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
static void legendre(int n, double x, double* pn, double* pnm1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *pn = 1.0;
    *pnm1 = 0.0;
    return;
  }
  for (int m = 1; m < n; ++m) {
    const double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pnm1 = p0;
}

// Interior Lobatto nodes are the roots of g(x) = P_{k-1}(x) - x P_k(x)
// (= (1-x^2) P_k'(x) / k), whose derivative is -(k+1) P_k(x).
static std::vector<double> lobatto_nodes(int k) {
  std::vector<double> x(k + 1);
  for (int j = 0; j <= k; ++j) {
    double t = -std::cos(M_PI * j / k);
    if (j > 0 && j < k) {
      for (int it = 0; it < 100; ++it) {
        double pk, pkm1;
        legendre(k, t, &pk, &pkm1);
        const double dt = (pkm1 - t * pk) / ((k + 1.0) * pk);
        t += dt;
        if (std::fabs(dt) < 1e-17) break;
      }
    }
    x[j] = t;
  }
  x[0] = -1.0;
  x[k] = 1.0;
  for (auto& v : x) v = 0.5 * (v + 1.0);
  std::sort(x.begin(), x.end());
  return x;
}

// Gauss-Legendre: Newton on P_n with P_n' = n (x P_n - P_{n-1}) / (x^2 - 1);
// weights 2 / ((1 - x^2) P_n'(x)^2), mapped to [0,1].
static void gauss_rule(int n, std::vector<double>* pts, std::vector<double>* wts) {
  pts->assign(n, 0.0);
  wts->assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      legendre(n, x, &pn, &pnm1);
      dp = n * (x * pn - pnm1) / (x * x - 1.0);
      const double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double pn, pnm1;
    legendre(n, x, &pn, &pnm1);
    dp = n * (x * pn - pnm1) / (x * x - 1.0);
    (*pts)[i] = 0.5 * (x + 1.0);
    (*wts)[i] = 1.0 / ((1.0 - x * x) * dp * dp);  // 2/(...) halved for [0,1]
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return (*pts)[a] < (*pts)[b]; });
  std::vector<double> p2(n), w2(n);
  for (int i = 0; i < n; ++i) {
    p2[i] = (*pts)[order[i]];
    w2[i] = (*wts)[order[i]];
  }
  *pts = p2;
  *wts = w2;
}

Tables1D make_tables(int k, int nq) {
  Tables1D T;
  T.k = k;
  T.nq = nq;
  T.nodes = lobatto_nodes(k);
  gauss_rule(nq, &T.qpts, &T.qwts);
  const int n = k + 1;
  // barycentric weights lambda_a = 1 / prod_{b != a} (xi_a - xi_b)
  std::vector<double> lam(n, 1.0);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (b != a) lam[a] /= (T.nodes[a] - T.nodes[b]);
  // nodal differentiation matrix Dn[b][a] = l_a'(xi_b)
  std::vector<double> Dn(n * n, 0.0);
  for (int b = 0; b < n; ++b) {
    double diag = 0.0;
    for (int a = 0; a < n; ++a) {
      if (a == b) continue;
      const double v = (lam[a] / lam[b]) / (T.nodes[b] - T.nodes[a]);
      Dn[b * n + a] = v;
      diag -= v;
    }
    Dn[b * n + b] = diag;
  }
  T.B.assign(nq * n, 0.0);
  T.D.assign(nq * n, 0.0);
  for (int q = 0; q < nq; ++q) {
    const double x = T.qpts[q];
    int hit = -1;
    for (int a = 0; a < n; ++a)
      if (x == T.nodes[a]) hit = a;
    if (hit >= 0) {
      T.B[q * n + hit] = 1.0;
    } else {
      double den = 0.0;
      for (int a = 0; a < n; ++a) den += lam[a] / (x - T.nodes[a]);
      for (int a = 0; a < n; ++a) T.B[q * n + a] = (lam[a] / (x - T.nodes[a])) / den;
    }
    // l_a' has degree k-1, so it equals its interpolant on the nodes
    for (int a = 0; a < n; ++a) {
      double s = 0.0;
      for (int b = 0; b < n; ++b) s += T.B[q * n + b] * Dn[b * n + a];
      T.D[q * n + a] = s;
    }
  }
  return T;
}

bool make_lattice(int nx, int ny, int nz, int k, Lattice* L, std::string* msg) {
  L->nx = nx;
  L->ny = ny;
  L->nz = nz;
  L->k = k;
  L->Lx = (int64_t)k * nx + 1;
  L->Ly = (int64_t)k * ny + 1;
  L->Lz = (int64_t)k * nz + 1;
  L->N = L->Lx * L->Ly * L->Lz;
  L->E = (int64_t)nx * ny * nz;
  const int D1 = k + 1;
  L->Ne = D1 * D1 * D1;
  if (L->N >= INT32_MAX || L->E * L->Ne >= INT32_MAX) {
    *msg = "mesh too large for 32-bit DOF / E-vector indices";
    return false;
  }
  L->interior.assign(L->N, 0);
  for (int64_t K = 1; K + 1 < L->Lz; ++K)
    for (int64_t J = 1; J + 1 < L->Ly; ++J)
      for (int64_t I = 1; I + 1 < L->Lx; ++I) L->interior[I + L->Lx * (J + L->Ly * K)] = 1;
  L->emap.assign(L->E * L->Ne, -1);
  std::vector<int32_t> count(L->N + 1, 0);
  for (int64_t e = 0; e < L->E; ++e) {
    const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
    for (int c = 0; c < D1; ++c)
      for (int b = 0; b < D1; ++b)
        for (int a = 0; a < D1; ++a) {
          const int64_t g = (k * ex + a) + L->Lx * ((k * ey + b) + L->Ly * (k * ez + c));
          const int64_t j = e * L->Ne + a + D1 * (b + D1 * c);
          if (L->interior[g]) {
            L->emap[j] = (int32_t)g;
            count[g + 1]++;
          }
        }
  }
  L->toff.assign(L->N + 1, 0);
  for (int64_t i = 0; i < L->N; ++i) L->toff[i + 1] = L->toff[i] + count[i + 1];
  L->tidx.assign(L->toff[L->N], 0);
  std::vector<int32_t> fill(L->toff.begin(), L->toff.end() - 1);
  for (int64_t j = 0; j < L->E * L->Ne; ++j) {  // ascending element => ascending within rows
    const int32_t g = L->emap[j];
    if (g >= 0) L->tidx[fill[g]++] = (int32_t)j;  // E-vector position e * Ne + local node
  }
  return true;
}

// Trilinear Jacobian determinant at reference point (xi, et, ze) of the
// element with corner coordinates X[v*3+al], v = i + 2j + 4l.
static double trilinear_det(const double* X, double xi, double et, double ze) {
  const double mx = 1 - xi, me = 1 - et, mz = 1 - ze;
  double J[3][3];
  for (int al = 0; al < 3; ++al) {
    auto x = [&](int v) { return X[v * 3 + al]; };
    J[al][0] = me * mz * (x(1) - x(0)) + et * mz * (x(3) - x(2)) + me * ze * (x(5) - x(4)) + et * ze * (x(7) - x(6));
    J[al][1] = mx * mz * (x(2) - x(0)) + xi * mz * (x(3) - x(1)) + mx * ze * (x(6) - x(4)) + xi * ze * (x(7) - x(5));
    J[al][2] = mx * me * (x(4) - x(0)) + xi * me * (x(5) - x(1)) + mx * et * (x(6) - x(2)) + xi * et * (x(7) - x(3));
  }
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

bool make_load(const Lattice& L, const Tables1D& T, const double* verts, std::vector<double>* b,
               std::string* msg) {
  const int D1 = T.k + 1, nq = T.nq, k = T.k;
  b->assign(L.N, 0.0);
  std::vector<double> mhat(D1, 0.0);  // int_0^1 l_a = sum_q w_q B[q][a]
  for (int a = 0; a < D1; ++a)
    for (int q = 0; q < nq; ++q) mhat[a] += T.qwts[q] * T.B[q * D1 + a];
  std::vector<double> W(nq * nq * nq), t1(D1 * nq * nq), t2(D1 * D1 * nq), be(L.Ne);
  double X[24];
  for (int64_t e = 0; e < L.E; ++e) {
    const int64_t ex = e % L.nx, ey = (e / L.nx) % L.ny, ez = e / ((int64_t)L.nx * L.ny);
    if (verts == nullptr) {
      const double vol = 1.0 / ((double)L.nx * L.ny * L.nz);
      for (int c = 0; c < D1; ++c)
        for (int bb = 0; bb < D1; ++bb)
          for (int a = 0; a < D1; ++a) be[a + D1 * (bb + D1 * c)] = vol * mhat[a] * mhat[bb] * mhat[c];
    } else {
      for (int v = 0; v < 8; ++v) {
        const int64_t gi = (ex + (v & 1)) + (L.nx + 1) * ((ey + ((v >> 1) & 1)) + (int64_t)(L.ny + 1) * (ez + (v >> 2)));
        for (int al = 0; al < 3; ++al) X[v * 3 + al] = verts[gi * 3 + al];
      }
      for (int qz = 0; qz < nq; ++qz)
        for (int qy = 0; qy < nq; ++qy)
          for (int qx = 0; qx < nq; ++qx) {
            const double det = trilinear_det(X, T.qpts[qx], T.qpts[qy], T.qpts[qz]);
            if (!(det > 0.0)) {
              *msg = "element " + std::to_string(e) + " has detJ <= 0 at a quadrature point";
              return false;
            }
            W[qx + nq * (qy + nq * qz)] = T.qwts[qx] * T.qwts[qy] * T.qwts[qz] * det;
          }
      // be = (B^T (x) B^T (x) B^T) W, contracting z, then y, then x
      for (int c = 0; c < D1; ++c)
        for (int qy = 0; qy < nq; ++qy)
          for (int qx = 0; qx < nq; ++qx) {
            double s = 0;
            for (int qz = 0; qz < nq; ++qz) s += T.B[qz * D1 + c] * W[qx + nq * (qy + nq * qz)];
            t1[qx + nq * (qy + nq * c)] = s;
          }
      for (int c = 0; c < D1; ++c)
        for (int bb = 0; bb < D1; ++bb)
          for (int qx = 0; qx < nq; ++qx) {
            double s = 0;
            for (int qy = 0; qy < nq; ++qy) s += T.B[qy * D1 + bb] * t1[qx + nq * (qy + nq * c)];
            t2[qx + nq * (bb + D1 * c)] = s;
          }
      for (int c = 0; c < D1; ++c)
        for (int bb = 0; bb < D1; ++bb)
          for (int a = 0; a < D1; ++a) {
            double s = 0;
            for (int qx = 0; qx < nq; ++qx) s += T.B[qx * D1 + a] * t2[qx + nq * (bb + D1 * c)];
            be[a + D1 * (bb + D1 * c)] = s;
          }
    }
    for (int c = 0; c < D1; ++c)
      for (int bb = 0; bb < D1; ++bb)
        for (int a = 0; a < D1; ++a) {
          const int64_t g = (k * ex + a) + L.Lx * ((k * ey + bb) + L.Ly * (k * ez + c));
          (*b)[g] += be[a + D1 * (bb + D1 * c)];
        }
  }
  return true;
}

}  // namespace feod
