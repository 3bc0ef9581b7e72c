// Host-side setup of one discretisation: 1D rules and basis tables, the
// structured hexahedral lattice, the element-to-DOF map G, its transpose for
// the gather-based G^T, and the load vector b.  Runs once; no GPU calls.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace feod {

struct Tables1D {
  int k = 0, nq = 0;
  std::vector<double> nodes;  // k+1 Gauss-Lobatto nodes on [0,1]
  std::vector<double> qpts;   // nq Gauss-Legendre points on [0,1]
  std::vector<double> qwts;   // their weights (sum 1)
  std::vector<double> B;      // B[q*(k+1)+a] = l_a(x_q)
  std::vector<double> D;      // D[q*(k+1)+a] = l_a'(x_q)
};

// Newton iterations on Legendre recurrences; barycentric Lagrange tables.
Tables1D make_tables(int k, int nq);

struct Lattice {
  int nx = 0, ny = 0, nz = 0, k = 0;
  int64_t Lx = 0, Ly = 0, Lz = 0, N = 0, E = 0;
  int Ne = 0;
  std::vector<int32_t> emap;  // E*Ne, global DOF or -1 on Dirichlet DOFs
  std::vector<int32_t> toff;  // N+1 row offsets of the transposed map
  std::vector<int32_t> tidx;  // E-vector positions of each DOF's entries, by ascending element
  std::vector<uint8_t> interior;
};

// Returns false (with msg) when a size would overflow 32-bit indices.
bool make_lattice(int nx, int ny, int nz, int k, Lattice* L, std::string* msg);

// Load vector b_i = sum_e sum_q w_q detJ f phi_i with f = 1, sum-factorised.
// verts == nullptr means the uniform unit-cube lattice.  Returns false with
// msg if some quadrature point has detJ <= 0 (inverted element).
bool make_load(const Lattice& L, const Tables1D& T, const double* verts, std::vector<double>* b,
               std::string* msg);

}  // namespace feod
