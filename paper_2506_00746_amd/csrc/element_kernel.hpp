// Fused element kernel of the finite element operator decomposition
// A = G^T B^T D B G (paper, Fig. 1, Eq. (1)-(2)).  One workgroup processes a
// batch of EB elements in four phases separated by barriers.  In every phase
// a thread owns whole 1D lines, so each value it loads feeds D1 or NQ
// multiply-adds; table operands that are uniform across the wavefront come
// from the kernel arguments (scalar registers):
//
//   A  G + x-pass     line (c,b): gather the D1 DOFs of an x-line of M u (and
//                     M v) through the element-to-DOF map straight from HBM,
//                     contract with B and D in x -> LDS.
//   C  y-pass, z-pass, D, z-back     line (qx,qy): contract the x-pass output
//                     in y for this column, finish the reference gradients at
//                     the NQ points of the z-column in registers, apply the
//                     pointwise operator D there (dual numbers for the Jacobian
//                     action; trilinear geometry recomputed per point on curved
//                     meshes) and contract the fluxes back over z -> LDS.
//                     Quadrature-point data never leaves registers.
//   D  y-back         line (c,qx) -> LDS.
//   E  x-back         line (c,b): D1 element residual entries written
//                     contiguously to the output E-vector, laid out
//                     [e][c][b][a] (each element's entries contiguous; G^T is
//                     the separate deterministic gather).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_api.hpp"
#include "pointwise.hpp"

namespace feod {

// 1D tables by value in the kernel arguments: B[q*D1+a] = l_a(x_q), the
// derivative table of each direction Dx, Dy, Dz[q*D1+a] = l_a'(x_q) / h_dir,
// Gauss weights w and points xi on [0,1].  On affine meshes the 1/h factor of
// each direction rides in its derivative table, so the passes produce
// physical gradients and take back physical fluxes with no per-point scaling;
// on curved meshes (and for the tangent kernel) the three are the reference
// table l_a'(x_q).  Each phase contracts along one direction and reads only
// that direction's table.
// Even-odd form of a 1D table.  The Gauss-Lobatto nodes and the Gauss points
// are symmetric about 1/2, so the value table is symmetric under the
// reflection (q, a) -> (NQ-1-q, D1-1-a) and a derivative table antisymmetric.
// Splitting a contraction's input into even and odd parts under the
// reflection roughly halves its multiply-adds.  Stored for the first
// QP = ceil(NQ/2) rows: P[q][a] = (M[q][a] + M[q][D1-1-a]) / 2 and
// N[q][a] = (M[q][a] - M[q][D1-1-a]) / 2 for a < D1/2, and the middle
// column P[q][D1/2] = M[q][D1/2] when D1 is odd.
template <int D1, int NQ>
struct EO {
  static constexpr int AH = D1 / 2, AP = (D1 + 1) / 2, QH = NQ / 2, QP = (NQ + 1) / 2;
};

template <int D1, int NQ, class T>
struct Tab {
  using E = EO<D1, NQ>;
  T B[NQ * D1];
  T Dx[NQ * D1];
  T Dy[NQ * D1];
  T Dz[NQ * D1];
  T w[NQ];
  T xi[NQ];
  // even-odd forms of B, Dx, Dy, Dz (the contractions of phases A, C, D, E)
  T Pb[E::QP * E::AP], Nb[E::QP * E::AH];
  T Px[E::QP * E::AP], Nx[E::QP * E::AH];
  T Py[E::QP * E::AP], Ny[E::QP * E::AH];
  T Pz[E::QP * E::AP], Nz[E::QP * E::AH];
};

// Even and odd parts of a line of D1 values (e[AH] = middle value, D1 odd).
template <int D1, int NQ, class T>
__device__ __forceinline__ void eo_split(const T (&x)[D1], T (&e)[EO<D1, NQ>::AP], T (&o)[EO<D1, NQ>::AH]) {
  constexpr int AH = EO<D1, NQ>::AH;
#pragma unroll
  for (int a = 0; a < AH; ++a) {
    e[a] = x[a] + x[D1 - 1 - a];
    o[a] = x[a] - x[D1 - 1 - a];
  }
  if constexpr (D1 % 2) e[AH] = x[AH];
}

// y = M x (D1 values -> NQ points) from the even / odd parts of x; SYM: M is
// a value table (symmetric), else a derivative table (antisymmetric).
template <int D1, int NQ, bool SYM, class T>
__device__ __forceinline__ void eo_forward(const T* P, const T* N, const T (&e)[EO<D1, NQ>::AP],
                                           const T (&o)[EO<D1, NQ>::AH], T (&y)[NQ]) {
  using E = EO<D1, NQ>;
#pragma unroll
  for (int q = 0; q < E::QH; ++q) {
    T s = P[q * E::AP] * e[0];
#pragma unroll
    for (int a = 1; a < E::AP; ++a) s += P[q * E::AP + a] * e[a];
    T d = N[q * E::AH] * o[0];
#pragma unroll
    for (int a = 1; a < E::AH; ++a) d += N[q * E::AH + a] * o[a];
    y[q] = s + d;
    y[NQ - 1 - q] = SYM ? s - d : d - s;
  }
  if constexpr (NQ % 2) {
    constexpr int q = E::QH;
    if constexpr (SYM) {
      T s = P[q * E::AP] * e[0];
#pragma unroll
      for (int a = 1; a < E::AP; ++a) s += P[q * E::AP + a] * e[a];
      y[q] = s;
    } else {
      T d = N[q * E::AH] * o[0];
#pragma unroll
      for (int a = 1; a < E::AH; ++a) d += N[q * E::AH + a] * o[a];
      y[q] = d;
    }
  }
}

// Backward (transposed) contraction y[a] = sum_q M[q][a] x[q] (NQ points ->
// D1 values), accumulated in even-odd form: x is given by its pair sums
// xe[q] = x[q] + x[NQ-1-q], differences xo[q] = x[q] - x[NQ-1-q] (q < NQ/2)
// and middle value xm (NQ odd); the results add into sp (a < AP) and sm
// (a < AH), from which eo_backward_finish forms y.  Several contractions
// (different tables and inputs) can add into the same sp, sm.
template <int D1, int NQ, bool SYM, class T>
__device__ __forceinline__ void eo_backward_add(const T* P, const T* N, const T (&xe)[EO<D1, NQ>::QH + 1],
                                                const T (&xo)[EO<D1, NQ>::QH + 1], T xm, T (&sp)[EO<D1, NQ>::AP],
                                                T (&sm)[EO<D1, NQ>::AH]) {
  using E = EO<D1, NQ>;
#pragma unroll
  for (int a = 0; a < E::AP; ++a) {
#pragma unroll
    for (int q = 0; q < E::QH; ++q) sp[a] += P[q * E::AP + a] * (SYM ? xe[q] : xo[q]);
    if constexpr (SYM && NQ % 2) sp[a] += P[E::QH * E::AP + a] * xm;
  }
#pragma unroll
  for (int a = 0; a < E::AH; ++a) {
#pragma unroll
    for (int q = 0; q < E::QH; ++q) sm[a] += N[q * E::AH + a] * (SYM ? xo[q] : xe[q]);
    if constexpr (!SYM && NQ % 2) sm[a] += N[E::QH * E::AH + a] * xm;
  }
}

template <int D1, int NQ, class T>
__device__ __forceinline__ void eo_pairs(const T (&x)[NQ], T (&xe)[EO<D1, NQ>::QH + 1], T (&xo)[EO<D1, NQ>::QH + 1],
                                         T& xm) {
  constexpr int QH = EO<D1, NQ>::QH;
#pragma unroll
  for (int q = 0; q < QH; ++q) {
    xe[q] = x[q] + x[NQ - 1 - q];
    xo[q] = x[q] - x[NQ - 1 - q];
  }
  xe[QH] = xo[QH] = T(0);
  xm = NQ % 2 ? x[QH] : T(0);
}

template <int D1, int NQ, class T>
__device__ __forceinline__ void eo_backward_finish(const T (&sp)[EO<D1, NQ>::AP], const T (&sm)[EO<D1, NQ>::AH],
                                                   T (&y)[D1]) {
  constexpr int AH = EO<D1, NQ>::AH;
#pragma unroll
  for (int a = 0; a < AH; ++a) {
    y[a] = sp[a] + sm[a];
    y[D1 - 1 - a] = sp[a] - sm[a];
  }
  if constexpr (D1 % 2) y[AH] = sp[AH];
}

// Launch shape per (D1, NQ, precision): NT threads per workgroup and EB
// elements per batch, so that phase C (NQ^2 lines per element, most of the
// work) fills the wavefronts and the LDS footprint leaves room for several
// workgroups per CU.
template <int D1, int NQ, class T>
struct Config {
  // One wavefront per workgroup at NQ <= 3 (7 Q2 elements, 63 columns): its
  // barriers cost next to nothing, and 48^3 Q2 runs 3% faster than with two
  // wavefronts (FP64 24.1 against 24.8 us, FP32 16.5 against 17.0).
  static constexpr int NT = NQ * NQ <= 9 ? 64 : (NQ * NQ <= 25 ? 128 : 256);
  static constexpr int EB0 = NT / (NQ * NQ);
  static constexpr int EB = EB0 < 1 ? 1 : EB0;
  // SEQ: the two input fields of a Jacobian action pass through the x-pass
  // buffer one after the other (halves it); needs one phase-C line per thread.
  static constexpr bool SEQ = false;
  // ALIAS2: two-field operations share one LDS region between the phases
  // (see Lds); one-field operations always do.
  static constexpr bool ALIAS2 = true;
  // WPE: minimum waves per SIMD asked of the register allocator, for affine
  // meshes with a specialised exponent (curved and generic-exponent kernels
  // need more registers and spill under it).  Q4 / nq 6 in FP32: 6 fits the
  // Jacobian kernel in 67 VGPRs (7 waves), 15% faster.  Q3 / nq 5 in FP64: 5
  // fits it in 95 VGPRs without spills (5 waves instead of 4).
  static constexpr int WPE = (D1 == 5 && NQ == 6 && sizeof(T) == 4) ? 6 : ((D1 == 4 && NQ == 5 && sizeof(T) == 8) ? 5 : 1);
  // RU: unroll factor of the runtime loops of high-order kernels
  static constexpr int RU = 1;
};
template <class T> struct Config<8, 9, T> {  // 81 lines: 3 elements on 4 wavefronts
  // The runtime loops of phases C and D (the forward z-pass over node rows,
  // the z-back and y-back over output node pairs, even-odd) are unrolled by
  // 2: each iteration waits for its table slice (scalar loads) and LDS
  // reads, and two in flight hide that wait at the two waves per SIMD these
  // kernels run at.  Fully unrolled they spill; the x-pass and x-back,
  // outside the register peak, are fully unrolled even-odd at every order.
  static constexpr int RU = 2;
  static constexpr int NT = 256;
  static constexpr int EB = 3;
  static constexpr bool SEQ = true;
  // The two-field kernels hold two fields' gradients at 9 points per thread
  // (over 168 VGPRs in FP64): registers, not LDS, bound their occupancy, so a
  // shared region would only add barriers (measured slower).
  static constexpr bool ALIAS2 = false;
  static constexpr int WPE = 1;
};

// Loops over a table index are fully unrolled for small D1/NQ (table entries
// become scalar operands); for large ones they run at runtime so that only one
// slice of the table is live in scalar registers.
template <int N>
struct Unroll {
  static constexpr bool full = N <= 6;
};

// LDS layout.  The x-pass buffer is [c][qx][b]; when D1 is a multiple of 8
// its qx stride is padded by one scalar, otherwise the NQ distinct qx columns
// phase C reads at once would fall on only two LDS banks.
//
// The x-pass outputs (read in phase C), the z-back outputs (written in C, read
// in D) and the y-back outputs (written in D, read in E) share one region per
// element: phases C and D first read what they need into registers, pass a
// barrier, then write.  This roughly halves the LDS per element, and LDS is
// what limits the number of resident workgroups.
template <int D1, int NQ, int XB, int HF, bool SHARE>
struct Lds {
  static constexpr int XQ = D1 % 8 ? D1 : D1 + 1;  // qx stride
  static constexpr int XC = NQ * XQ;              // c stride
  static constexpr int XS = D1 * XC;              // one x-pass output block [c][qx][b]
  static constexpr int X = XB * XS;               // XB blocks: x-pass outputs, later y-back outputs
  static constexpr int H = HF * D1 * NQ * NQ;     // HF z-back fields [h][c][qy][qx]
  static constexpr bool ALIAS = SHARE;
  static constexpr int XSTR = ALIAS ? (X > H ? X : H) : X;  // per-element stride of the x / y-back blocks
  static constexpr int HSTR = ALIAS ? XSTR : H;             // per-element stride of the z-back block
  static constexpr int HOFF = ALIAS ? 0 : X;                // z-back region offset, in units of EB
  static constexpr int region = ALIAS ? XSTR : X + H;       // per element, without the vertices
};

// Deterministic sum of n LDS values by one wavefront (fixed order).
template <class T>
__device__ __forceinline__ double wave_sum(const T* vals, int n, int lane) {
  double s = 0;
  for (int i = lane; i < n; i += 64) s += (double)vals[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

// G for one phase-A line (c, b) of element e (global index): the D1 DOFs of
// the x-line (k ex + a, k ey + b, k ez + c) of each of the NG fields, read
// straight from HBM through the stored map or the same map computed from the
// lattice; Dirichlet DOFs (on the cube's boundary) read as 0, and so does an
// element past the end of the mesh (valid false).
template <int D1, int NG, class T>
__device__ __forceinline__ void gather_line(const ElemParams& P, const double* const (&src)[NG], int e, bool valid,
                                            int cb, T (&in)[NG][D1]) {
  constexpr int Ne = D1 * D1 * D1;
  if (valid && P.emap != nullptr) {
    const int32_t* m = P.emap + (int64_t)e * Ne + cb * D1;
#pragma unroll
    for (int a = 0; a < D1; ++a) {
      const int idx = m[a];
#pragma unroll
      for (int f = 0; f < NG; ++f) in[f][a] = idx >= 0 ? (T)src[f][idx] : T(0);
    }
  } else if (valid) {
    const uint32_t t = fastdiv((uint32_t)e, P.div_nx), z = fastdiv(t, P.div_ny);
    const int ex = (int)((uint32_t)e - t * (uint32_t)P.nx), ey = (int)(t - z * (uint32_t)P.ny), ez = (int)z;
    const int c = cb / D1, b = cb - c * D1;
    const int I0 = P.k * ex, J = P.k * ey + b, K = P.k * ez + c;
    const bool row = J > 0 && J < P.Ly - 1 && K > 0 && K < P.Lz - 1;
    const int64_t base = I0 + (int64_t)P.Lx * (J + (int64_t)P.Ly * K);
    // every node of a valid element lies in the lattice: load unconditionally
    // (no branch per load) and zero the Dirichlet ones.  FP64 kernels read
    // the line's D1 contiguous DOFs with wide loads (48^3 Q2 element kernel
    // -2%, 16^3 Q7 -1.3%, 64^3 Q4 -0.4%); FP32 ones one DOF per load (wide
    // loads cost 64^3 Q4 +3% there).
    if constexpr (sizeof(T) == 8) {
      double raw[NG][D1];
#pragma unroll
      for (int f = 0; f < NG; ++f) __builtin_memcpy(raw[f], src[f] + base, sizeof raw[f]);
#pragma unroll
      for (int a = 0; a < D1; ++a) {
        const bool ok = row && I0 + a > 0 && I0 + a < P.Lx - 1;
#pragma unroll
        for (int f = 0; f < NG; ++f) in[f][a] = ok ? (T)raw[f][a] : T(0);
      }
    } else {
#pragma unroll
      for (int a = 0; a < D1; ++a) {
        const bool ok = row && I0 + a > 0 && I0 + a < P.Lx - 1;
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          const double val = src[f][base + a];
          in[f][a] = ok ? (T)val : T(0);
        }
      }
    }
  } else {
#pragma unroll
    for (int f = 0; f < NG; ++f)
#pragma unroll
      for (int a = 0; a < D1; ++a) in[f][a] = 0;
  }
}

// Phase A's contraction in x of one line: values (B) and x-derivatives (Dx)
// at the NQ points, into the x-pass buffer at x (the line's slot, [s][qx]
// with stride XQ, s = 0 values, s = 1 derivatives).
template <int D1, int NQ, int XQ, class T, class TB>
__device__ __forceinline__ void xpass_line(const TB& tb, const T (&in)[D1], T* x) {
  constexpr int XS = D1 * NQ * XQ;
  // even-odd form at every order: its tables are read once per line, and at
  // Q7 it runs the 16^3 Jacobian kernel (with the x-back below) in 54.9
  // against 57.4 us with runtime loops over the full tables (FP32 33.5 against
  // 35.8), registers unchanged
  T e[EO<D1, NQ>::AP], o[EO<D1, NQ>::AH], y0[NQ], y1[NQ];
  eo_split<D1, NQ>(in, e, o);
  eo_forward<D1, NQ, true>(tb.Pb, tb.Nb, e, o, y0);
  eo_forward<D1, NQ, false>(tb.Px, tb.Nx, e, o, y1);
#pragma unroll
  for (int qx = 0; qx < NQ; ++qx) {
    x[qx * XQ] = y0[qx];
    x[XS + qx * XQ] = y1[qx];
  }
}

// Phase C forward for one field: y-pass of column (qx,qy) from x-pass slot
// xs, then z-pass into gf[3][NQ] (reference gradient x, y, z at each qz).
// The z-pass takes the nodes c and D1-1-c together (even-odd form).
template <int D1, int NQ, int XQ, class T, class TB>
__device__ __forceinline__ void column_forward(const TB& tb, const T* xs, const T (&By)[D1],
                                               const T (&Dy)[D1], int qx, T (&gf)[3][NQ]) {
  constexpr int XS = D1 * NQ * XQ;
  using E = EO<D1, NQ>;
  // y-pass for this column at node row c: Y0 = D_y X0 (d/dy), Y1 = B_y X0
  // (d/dz), Y2 = B_y X1 (d/dx)
  auto ypass = [&](int c, T (&y)[3]) {
    const T* x0 = xs + (c * NQ + qx) * XQ;
    const T* x1 = x0 + XS;
    y[0] = Dy[0] * x0[0];
    y[1] = By[0] * x0[0];
    y[2] = By[0] * x1[0];
#pragma unroll
    for (int b = 1; b < D1; ++b) {
      y[0] += Dy[b] * x0[b];
      y[1] += By[b] * x0[b];
      y[2] += By[b] * x1[b];
    }
  };
  if constexpr (!Unroll<D1>::full) {
    // high order: full tables, runtime loop over the node rows (bounded
    // register use); gx += B_z Y2, gy += B_z Y0, gz += D_z Y1
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) gf[0][qz] = gf[1][qz] = gf[2][qz] = T(0);
#pragma unroll(Config<D1, NQ, T>::RU)
    for (int c = 0; c < D1; ++c) {
      T y[3];
      ypass(c, y);
#pragma unroll
      for (int qz = 0; qz < NQ; ++qz) {
        gf[0][qz] += tb.B[qz * D1 + c] * y[2];
        gf[1][qz] += tb.B[qz * D1 + c] * y[0];
        gf[2][qz] += tb.Dz[qz * D1 + c] * y[1];
      }
    }
    return;
  }
  // z-pass: gx = B_z Y2, gy = B_z Y0 (symmetric table), gz = D_z Y1
  // (antisymmetric); s: even parts, d: odd parts, per output pair
  T s[3][E::QP], d[3][E::QP];
#pragma unroll
  for (int q = 0; q < E::QP; ++q) s[0][q] = s[1][q] = s[2][q] = d[0][q] = d[1][q] = d[2][q] = T(0);
#pragma unroll
  for (int cp = 0; cp < E::AP; ++cp) {
    T ya[3], ee[3], oo[3];
    ypass(cp, ya);
    if (cp < E::AH) {
      T yb[3];
      ypass(D1 - 1 - cp, yb);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ee[k] = ya[k] + yb[k];
        oo[k] = ya[k] - yb[k];
      }
    } else {  // middle node row (D1 odd)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ee[k] = ya[k];
        oo[k] = T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < E::QP; ++q) {
      const T pb = tb.Pb[q * E::AP + cp];
      s[0][q] += pb * ee[2];
      s[1][q] += pb * ee[0];
      if (q < E::QH) s[2][q] += tb.Pz[q * E::AP + cp] * ee[1];
      if (cp < E::AH) {
        if (q < E::QH) {
          const T nb = tb.Nb[q * E::AH + cp];
          d[0][q] += nb * oo[2];
          d[1][q] += nb * oo[0];
        }
        d[2][q] += tb.Nz[q * E::AH + cp] * oo[1];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < E::QH; ++q) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      gf[k][q] = s[k][q] + d[k][q];
      gf[k][NQ - 1 - q] = s[k][q] - d[k][q];
    }
    gf[2][q] = s[2][q] + d[2][q];
    gf[2][NQ - 1 - q] = d[2][q] - s[2][q];
  }
  if constexpr (NQ % 2) {
    gf[0][E::QH] = s[0][E::QH];
    gf[1][E::QH] = s[1][E::QH];
    gf[2][E::QH] = d[2][E::QH];
  }
}

template <int D1, int NQ, class T, int OP, bool CURVED, int PK>
__global__ __launch_bounds__((Config<D1, NQ, T>::NT), ((CURVED || PK == POW_GENERIC) ? 1 : Config<D1, NQ, T>::WPE))
void element_kernel(ElemParams P, Tab<D1, NQ, T> tb) {
  using C = Config<D1, NQ, T>;
  constexpr int NT = C::NT;
  constexpr int EB = C::EB;
  constexpr int Ne = D1 * D1 * D1;
  constexpr int NQ2 = NQ * NQ;
  constexpr bool PA = OP == OP_JVP_PA, QSTORE = OP == OP_QSTORE;
  // element-level forward AD: one tangent column of K_e per blockIdx.y, the
  // direction being the unit vector of that local node (no gather)
  constexpr bool ELM = OP == OP_ELM;
  constexpr bool HND = OP == OP_JVP_HND;  // Jacobian action, hand-coded J_D
  constexpr int F = (OP == OP_JVP || OP == OP_RESJVP || OP == OP_GRAD || PA || ELM || HND) ? 2 : 1;  // register fields
  constexpr int O = (OP == OP_RESJVP) ? 2 : 1;                                    // output fields
  constexpr bool REDUCE = (OP == OP_ENERGY || OP == OP_GRAD);
  constexpr bool SEQ = C::SEQ && F == 2 && !PA;
  static_assert(!SEQ || EB * NQ2 <= NT, "sequential fields need one phase-C line per thread");
  constexpr int FX = (SEQ || PA) ? 1 : F;  // fields resident in the x-pass buffer at once
  constexpr bool DIAG = OP == OP_DIAG;
  // z-back fields: 3 per output (x, y, z flux components); the diagonal has 6
  // (the symmetric tensor terms); y-back blocks: 2 per output, 3 for the diagonal
  constexpr int HF = DIAG ? 6 : 3 * O;
  constexpr int KB = DIAG ? 3 : 2 * O;
  using L = Lds<D1, NQ, (2 * FX > KB ? 2 * FX : KB), HF, (F == 1 || C::ALIAS2)>;
  static_assert(EB * NQ2 <= NT && EB * D1 * NQ <= NT, "phases C and D take one line per thread");
  constexpr int VTX = CURVED ? 24 : 0;  // vertex coordinates per element (curved meshes only)
  __shared__ T smem[EB * (L::region + VTX)];
  __shared__ T sB[NQ * L::XQ], sD[NQ * L::XQ];  // table rows, same padded stride
  __shared__ T sW[NQ], sXi[NQ];                  // weights and points, read with per-thread indices
  T* Xs = smem;                     // [el][f][s][c][qx][b], later K [el][o][s][c][qx][b]
  T* Hs = smem + EB * L::HOFF;      // [el][o][d][c][qy][qx]; per-line sums for reductions
  T* Vs = smem + EB * L::region;    // [el][24] vertex coordinates

  const int tid = threadIdx.x;
  const int e0 = xcd_remap(blockIdx.x, gridDim.x) * EB;  // batch start, relative to eoff
  const int eoff = ELM ? P.e_first : 0;                   // global index of element 0
  const int n_valid = min(EB, P.E - e0);

  // ---- global loads first: G (this thread's phase-A line of the gathered
  // fields) and the batch's coefficients, so that their HBM latency overlaps
  // the set-up below instead of stalling the phases that use them
  constexpr int NG = (F == 2 && !PA && !ELM) ? 2 : 1;  // fields gathered from L-vectors
  static_assert(EB * D1 * D1 <= NT, "phase A takes one line per thread");
  const bool aline = tid < EB * D1 * D1;
  const int ael = aline ? tid / (D1 * D1) : 0, acb = aline ? tid - ael * (D1 * D1) : 0;
  T gin[NG][D1];
  {
    const double* const src1[1] = {PA ? P.v : P.u};
    const double* const src2[2] = {P.u, P.v};
    if constexpr (NG == 2)
      gather_line<D1, 2, T>(P, src2, eoff + e0 + ael, aline && ael < n_valid, acb, gin);
    else
      gather_line<D1, 1, T>(P, src1, eoff + e0 + ael, aline && ael < n_valid, acb, gin);
  }
  __shared__ T sRho[EB];  // coefficients of the batch's elements
  if (tid < EB) sRho[tid] = (P.rho != nullptr && tid < n_valid) ? (T)P.rho[eoff + e0 + tid] : T(1);

  for (int i = tid; i < NQ * D1; i += NT) {
    const int q = i / D1, a = i - q * D1;
    sB[q * L::XQ + a] = tb.B[i];
    sD[q * L::XQ + a] = tb.Dy[i];
  }
  for (int i = tid; i < NQ; i += NT) {
    sW[i] = tb.w[i];
    sXi[i] = tb.xi[i];
  }
  if (CURVED) {
    for (int i = tid; i < EB * 24; i += NT) {
      const int el = i / 24, r = i - el * 24, vtx = r / 3, al = r - vtx * 3;
      T val = 0;
      if (el < n_valid) {
        const uint32_t e = (uint32_t)(eoff + e0 + el), t = fastdiv(e, P.div_nx), z = fastdiv(t, P.div_ny);
        const int ex = (int)(e - t * (uint32_t)P.nx), ey = (int)(t - z * (uint32_t)P.ny), ez = (int)z;
        const int gi = (ex + (vtx & 1)) + (P.nx + 1) * ((ey + ((vtx >> 1) & 1)) + (P.ny + 1) * (ez + (vtx >> 2)));
        val = (T)P.verts[(int64_t)gi * 3 + al];
      }
      Vs[i] = val;
    }
  }

  __syncthreads();  // tables, coefficients and vertices visible to every thread

  // ---- A: x-pass of the gathered lines --------------------------------------
  if (aline) {
    T* x = Xs + ael * L::XSTR + (acb / D1) * NQ * L::XQ + (acb % D1);
    xpass_line<D1, NQ, L::XQ, T>(tb, gin[0], x);
    if constexpr (ELM) {  // the second field is the unit direction of local node blockIdx.y
      T unit[D1];
#pragma unroll
      for (int a = 0; a < D1; ++a) unit[a] = acb * D1 + a == (int)blockIdx.y ? T(1) : T(0);
      xpass_line<D1, NQ, L::XQ, T>(tb, unit, x + 2 * L::XS);
    } else if constexpr (NG == 2 && !SEQ) {
      xpass_line<D1, NQ, L::XQ, T>(tb, gin[1], x + 2 * L::XS);
    }
  }
  __syncthreads();

  // ---- C: y-pass + z-pass -> D -> z-back, one (qx,qy) column per line ---------
  const T eps2 = (T)P.eps2, r = (T)P.r, inv_p = (T)P.inv_p;
  T g[F][3][NQ];
  if constexpr (SEQ) {
    // field u: columns into registers, then the x-pass buffer takes field v
    const int l = tid;
    if (l < EB * NQ2) {
      const int el = l / NQ2, qxy = l - el * NQ2;
      const int qy = qxy / NQ, qx = qxy - qy * NQ;
      T By[D1], Dy[D1];
#pragma unroll
      for (int b = 0; b < D1; ++b) {
        By[b] = sB[qy * L::XQ + b];
        Dy[b] = sD[qy * L::XQ + b];
      }
      column_forward<D1, NQ, L::XQ, T>(tb, Xs + el * L::XSTR, By, Dy, qx, g[0]);
    }
    __syncthreads();
    if constexpr (NG == 2) {
      if (aline) xpass_line<D1, NQ, L::XQ, T>(tb, gin[1], Xs + ael * L::XSTR + (acb / D1) * NQ * L::XQ + (acb % D1));
    }
    __syncthreads();
  }
  const int l = tid;  // one column per thread
  const bool active = l < EB * NQ2;
  const int el = active ? l / NQ2 : 0, qxy = active ? l - el * NQ2 : 0;
  const int qy = qxy / NQ, qx = qxy - qy * NQ;
  if (active) {
    T By[D1], Dy[D1];
#pragma unroll
    for (int b = 0; b < D1; ++b) {
      By[b] = sB[qy * L::XQ + b];
      Dy[b] = sD[qy * L::XQ + b];
    }
    if constexpr (QSTORE) {
      column_forward<D1, NQ, L::XQ, T>(tb, Xs + el * L::XSTR, By, Dy, qx, g[0]);
      if (el < n_valid) {
        T* qd = static_cast<T*>(P.qdata) + (int64_t)(e0 + el) * 3 * NQ * NQ2 + qxy;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int qz = 0; qz < NQ; ++qz) qd[(d * NQ + qz) * NQ2] = g[0][d][qz];
      }
    } else if constexpr (PA) {
      // v from the x-pass buffer; u's reference gradients from the stored data
      column_forward<D1, NQ, L::XQ, T>(tb, Xs + el * L::XSTR, By, Dy, qx, g[1]);
      const T* qd = static_cast<const T*>(P.qdata) + (int64_t)(e0 + (el < n_valid ? el : 0)) * 3 * NQ * NQ2 + qxy;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int qz = 0; qz < NQ; ++qz) g[0][d][qz] = qd[(d * NQ + qz) * NQ2];
    } else if constexpr (SEQ) {
      column_forward<D1, NQ, L::XQ, T>(tb, Xs + el * L::XSTR, By, Dy, qx, g[1]);
    } else {
#pragma unroll
      for (int f = 0; f < F; ++f) column_forward<D1, NQ, L::XQ, T>(tb, Xs + el * L::XSTR + f * 2 * L::XS, By, Dy, qx, g[f]);
    }
  }
  if (L::ALIAS) __syncthreads();  // x-pass buffer consumed: the z-back may overwrite it
  if (active && !QSTORE) {
    const T rho = sRho[el];
    const T wxy = sW[qx] * sW[qy];
    // geometry: affine -> constant diagonal; curved -> Jg = J0 + xi_z J1 (column 2 constant)
    T J0[3][3], J1[3][2];
    // curved, Q7: the adjugate of Jg and det Jg as polynomials in xi_z along
    // the column (rows 0 and 1 of adj linear, row 2 and det quadratic, since
    // one column of Jg is constant), aL[i][j] = c0 + c1 z and aQ[j] = c0 + c1 z
    // + c2 z^2, so a point evaluates them (14 FMAs) instead of forming Jg, adj
    // and det (27).  16^3 Q7 Jacobian kernel 52.9 -> 52.4 us (FP64), 32.0 ->
    // 30.6 (FP32).  Below Q7 the 24 coefficients cost occupancy, so those
    // orders form Jg at every point.
    constexpr bool POLY = D1 >= 8;
    T aL[2][3][2], aQ[3][3], dQ[3];
    if (CURVED) {
      const T* X = Vs + el * 24;
      const T xi = sXi[qx], et = sXi[qy], mx = T(1) - xi, me = T(1) - et;
#pragma unroll
      for (int al = 0; al < 3; ++al) {
        const T* x = X + al;  // x[3v] = coordinate al of vertex v = i + 2j + 4l
        const T a0 = me * (x[3] - x[0]) + et * (x[9] - x[6]);
        const T a1 = me * (x[15] - x[12]) + et * (x[21] - x[18]);
        const T b0 = mx * (x[6] - x[0]) + xi * (x[9] - x[3]);
        const T b1 = mx * (x[18] - x[12]) + xi * (x[21] - x[15]);
        J0[al][0] = a0;
        J1[al][0] = a1 - a0;
        J0[al][1] = b0;
        J1[al][1] = b1 - b0;
        J0[al][2] = (mx * me) * (x[12] - x[0]) + (xi * me) * (x[15] - x[3]) + (mx * et) * (x[18] - x[6]) +
                    (xi * et) * (x[21] - x[9]);
      }
      if constexpr (POLY) {
        // linear entries L(a,b) = J0[a][b] + z J1[a][b] (b < 2), constants C(a) = J0[a][2]
        auto lc = [&](int a, int b, T c, T (&o)[2]) {  // L(a,b) * c
          o[0] = J0[a][b] * c;
          o[1] = J1[a][b] * c;
        };
        auto lsub = [&](const T (&u)[2], const T (&v)[2], T (&o)[2]) {
          o[0] = u[0] - v[0];
          o[1] = u[1] - v[1];
        };
        auto ll = [&](int a, int b, int c, int d, T (&o)[3]) {  // L(a,b) * L(c,d)
          o[0] = J0[a][b] * J0[c][d];
          o[1] = J0[a][b] * J1[c][d] + J1[a][b] * J0[c][d];
          o[2] = J1[a][b] * J1[c][d];
        };
        T u[2], v[2], q0[3], q1[3];
        lc(1, 1, J0[2][2], u); lc(2, 1, J0[1][2], v); lsub(u, v, aL[0][0]);  // J11 J22 - J12 J21
        lc(2, 1, J0[0][2], u); lc(0, 1, J0[2][2], v); lsub(u, v, aL[0][1]);  // J02 J21 - J01 J22
        lc(0, 1, J0[1][2], u); lc(1, 1, J0[0][2], v); lsub(u, v, aL[0][2]);  // J01 J12 - J02 J11
        lc(2, 0, J0[1][2], u); lc(1, 0, J0[2][2], v); lsub(u, v, aL[1][0]);  // J12 J20 - J10 J22
        lc(0, 0, J0[2][2], u); lc(2, 0, J0[0][2], v); lsub(u, v, aL[1][1]);  // J00 J22 - J02 J20
        lc(1, 0, J0[0][2], u); lc(0, 0, J0[1][2], v); lsub(u, v, aL[1][2]);  // J02 J10 - J00 J12
        ll(1, 0, 2, 1, q0); ll(1, 1, 2, 0, q1);                               // J10 J21 - J11 J20
        for (int k = 0; k < 3; ++k) aQ[0][k] = q0[k] - q1[k];
        ll(0, 1, 2, 0, q0); ll(0, 0, 2, 1, q1);                               // J01 J20 - J00 J21
        for (int k = 0; k < 3; ++k) aQ[1][k] = q0[k] - q1[k];
        ll(0, 0, 1, 1, q0); ll(0, 1, 1, 0, q1);                               // J00 J11 - J01 J10
        for (int k = 0; k < 3; ++k) aQ[2][k] = q0[k] - q1[k];
        // det = J00 adj00 + J01 adj10 + J02 adj20
        dQ[0] = J0[0][0] * aL[0][0][0] + J0[0][1] * aL[1][0][0] + J0[0][2] * aQ[0][0];
        dQ[1] = J0[0][0] * aL[0][0][1] + J1[0][0] * aL[0][0][0] + J0[0][1] * aL[1][0][1] + J1[0][1] * aL[1][0][0] +
                J0[0][2] * aQ[0][1];
        dQ[2] = J1[0][0] * aL[0][0][1] + J1[0][1] * aL[1][0][1] + J0[0][2] * aQ[0][2];
      }
    }
    double part = 0;  // energy / gradient partial over the column
    T cd[DIAG ? 6 : 1][NQ];  // diagonal: the six symmetric tensor terms per point
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      const T w3 = wxy * tb.w[qz];
      T gu[3], gv[3];
      T adj[3][3], det;
      if (CURVED) {
        const T ze = tb.xi[qz];
        if constexpr (POLY) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) adj[i][j] = aL[i][j][0] + ze * aL[i][j][1];
#pragma unroll
          for (int j = 0; j < 3; ++j) adj[2][j] = aQ[j][0] + ze * (aQ[j][1] + ze * aQ[j][2]);
          det = dQ[0] + ze * (dQ[1] + ze * dQ[2]);
        } else {
          T J[3][3];
#pragma unroll
          for (int al = 0; al < 3; ++al) {
            J[al][0] = J0[al][0] + ze * J1[al][0];
            J[al][1] = J0[al][1] + ze * J1[al][1];
            J[al][2] = J0[al][2];
          }
          adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
          adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
          adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
          adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
          adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
          adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
          adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
          adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
          adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
        }
        const T inv_det = fe_rcp(det);
        // physical gradient g = Jg^{-T} ghat = adj^T ghat / det
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gu[a] = (adj[0][a] * g[0][0][qz] + adj[1][a] * g[0][1][qz] + adj[2][a] * g[0][2][qz]) * inv_det;
          if constexpr (F == 2)
            gv[a] = (adj[0][a] * g[1][0][qz] + adj[1][a] * g[1][1][qz] + adj[2][a] * g[1][2][qz]) * inv_det;
        }
      } else {
        det = (T)P.det;  // the derivative tables carry 1/h: g is already physical
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gu[a] = g[0][a][qz];
          if constexpr (F == 2) gv[a] = g[1][a][qz];
        }
      }
      T Fo[O][3];
      if constexpr (DIAG) {
        // J_D by forward mode along each physical direction: Tm[a][d] = dF_a/dg_d
        T Tm[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          dual<T> gd[3], Fd[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) gd[a] = {gu[a], a == d ? T(1) : T(0)};
          flux<PK, dual<T>, T>(gd, eps2, r, Fd);
#pragma unroll
          for (int a = 0; a < 3; ++a) Tm[a][d] = Fd[a].d;
        }
        // reference-space tensor Chat = rho w det Jg^{-1} Tm Jg^{-T}
        T Ch[3][3];
        const T s = rho * w3;
        if (CURVED) {
          const T sd = s * fe_rcp(det);
          T AT[3][3];  // adj Tm
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) AT[i][j] = adj[i][0] * Tm[0][j] + adj[i][1] * Tm[1][j] + adj[i][2] * Tm[2][j];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ch[i][j] = sd * (AT[i][0] * adj[j][0] + AT[i][1] * adj[j][1] + AT[i][2] * adj[j][2]);
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ch[i][j] = (s * det) * Tm[i][j];  // 1/h in the tables
        }
        cd[0][qz] = Ch[0][0];
        cd[1][qz] = Ch[1][1];
        cd[2][qz] = Ch[2][2];
        cd[3][qz] = Ch[0][1] + Ch[1][0];
        cd[4][qz] = Ch[0][2] + Ch[2][0];
        cd[5][qz] = Ch[1][2] + Ch[2][1];
      } else if constexpr (OP == OP_RESIDUAL) {
        flux<PK, T, T>(gu, eps2, r, Fo[0]);
      } else if constexpr (HND) {
        flux_tangent_hand<PK, T>(gu, gv, eps2, r, Fo[0]);
      } else if constexpr (OP == OP_JVP || OP == OP_RESJVP || PA || ELM) {
        dual<T> gd[3], Fd[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gd[a] = {gu[a], gv[a]};
        flux<PK, dual<T>, T>(gd, eps2, r, Fd);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Fo[0][a] = Fd[a].d;                        // Jacobian action
          if constexpr (O == 2) Fo[1][a] = Fd[a].v;  // residual of residual + JVP
        }
      } else if constexpr (OP == OP_ENERGY) {
        T W, cf;
        density<PK, T>(gu, eps2, r, inv_p, &W, &cf);
        part += (double)(rho * w3 * det * W);
      } else if constexpr (OP == OP_GRAD) {
        T W, cf;
        density<PK, T>(gu, eps2, r, inv_p, &W, &cf);
        part -= (double)(w3 * det * cf * (gu[0] * gv[0] + gu[1] * gv[1] + gu[2] * gv[2]));
      }
      if constexpr (!REDUCE && !DIAG) {
        // reference flux Fhat = rho w det Jg^{-1} F = rho w adj F (stored over g);
        // affine: rho w det F, the 1/h of Jg^{-1} being in the tables
        const T s = rho * w3;
        const T sd = s * det;
#pragma unroll
        for (int o = 0; o < O; ++o) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if (CURVED)
              g[o][a][qz] = s * (adj[a][0] * Fo[o][0] + adj[a][1] * Fo[o][1] + adj[a][2] * Fo[o][2]);
            else
              g[o][a][qz] = sd * Fo[o][a];
          }
        }
      }
    }
    if constexpr (REDUCE) {
      Hs[l] = (T)part;
    } else if constexpr (DIAG) {
      // z factors of the six terms: B^2 (00, 11, 01), D^2 (22), B D (02, 12)
      T* h = Hs + el * L::HSTR + qxy;
#pragma unroll(Unroll<D1>::full ? D1 : 1)
      for (int c = 0; c < D1; ++c) {
        T s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int qz = 0; qz < NQ; ++qz) {
          const T bz = tb.B[qz * D1 + c], dz = tb.Dz[qz * D1 + c];
          const T bb = bz * bz, dd = dz * dz, bd = bz * dz;
          s[0] += bb * cd[0][qz];
          s[1] += bb * cd[1][qz];
          s[2] += dd * cd[2][qz];
          s[3] += bb * cd[3][qz];
          s[4] += bd * cd[4][qz];
          s[5] += bd * cd[5][qz];
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) h[(t * D1 + c) * NQ2] = s[t];
      }
    } else {
      // z-back: H0[c] = sum_qz B Fx, H1 = sum_qz B Fy, H2 = sum_qz D Fz
      using E = EO<D1, NQ>;
#pragma unroll
      for (int o = 0; o < O; ++o) {
        T* h = Hs + el * L::HSTR + o * 3 * D1 * NQ2 + qxy;
        if constexpr (!Unroll<D1>::full) {  // high order: even-odd, runtime loop over output pairs
          static_assert(D1 % 2 == 0, "the runtime even-odd loops take node pairs");
          T xe0[E::QH + 1], xo0[E::QH + 1], xm0, xe1[E::QH + 1], xo1[E::QH + 1], xm1, xe2[E::QH + 1],
              xo2[E::QH + 1], xm2;
          eo_pairs<D1, NQ>(g[o][0], xe0, xo0, xm0);
          eo_pairs<D1, NQ>(g[o][1], xe1, xo1, xm1);
          eo_pairs<D1, NQ>(g[o][2], xe2, xo2, xm2);
#pragma unroll(Config<D1, NQ, T>::RU)
          for (int a = 0; a < E::AH; ++a) {
            T sp0 = tb.Pb[a] * xe0[0], sm0 = tb.Nb[a] * xo0[0];
            T sp1 = tb.Pb[a] * xe1[0], sm1 = tb.Nb[a] * xo1[0];
            T sp2 = tb.Pz[a] * xo2[0], sm2 = tb.Nz[a] * xe2[0];
#pragma unroll
            for (int q = 1; q < E::QH; ++q) {
              const T pb = tb.Pb[q * E::AP + a], nb = tb.Nb[q * E::AH + a];
              sp0 += pb * xe0[q];
              sm0 += nb * xo0[q];
              sp1 += pb * xe1[q];
              sm1 += nb * xo1[q];
              sp2 += tb.Pz[q * E::AP + a] * xo2[q];
              sm2 += tb.Nz[q * E::AH + a] * xe2[q];
            }
            if constexpr (NQ % 2) {  // the middle point
              const T pm = tb.Pb[E::QH * E::AP + a];
              sp0 += pm * xm0;
              sp1 += pm * xm1;
              sm2 += tb.Nz[E::QH * E::AH + a] * xm2;
            }
            h[a * NQ2] = sp0 + sm0;
            h[(D1 - 1 - a) * NQ2] = sp0 - sm0;
            h[(D1 + a) * NQ2] = sp1 + sm1;
            h[(2 * D1 - 1 - a) * NQ2] = sp1 - sm1;
            h[(2 * D1 + a) * NQ2] = sp2 + sm2;
            h[(3 * D1 - 1 - a) * NQ2] = sp2 - sm2;
          }
          continue;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          T xe[E::QH + 1], xo[E::QH + 1], xm, sp[E::AP], sm[E::AH], y[D1];
#pragma unroll
          for (int a = 0; a < E::AP; ++a) sp[a] = T(0);
#pragma unroll
          for (int a = 0; a < E::AH; ++a) sm[a] = T(0);
          eo_pairs<D1, NQ>(g[o][k], xe, xo, xm);
          if (k < 2)
            eo_backward_add<D1, NQ, true>(tb.Pb, tb.Nb, xe, xo, xm, sp, sm);
          else
            eo_backward_add<D1, NQ, false>(tb.Pz, tb.Nz, xe, xo, xm, sp, sm);
          eo_backward_finish<D1, NQ>(sp, sm, y);
#pragma unroll
          for (int c = 0; c < D1; ++c) h[(k * D1 + c) * NQ2] = y[c];
        }
      }
    }
  }
  __syncthreads();

  if constexpr (QSTORE) return;
  if constexpr (REDUCE) {
    const int lane = tid & 63, wv = tid >> 6;
    double* outd = static_cast<double*>(P.out0);
    for (int el = wv; el < n_valid; el += NT / 64) {
      const double s = wave_sum<T>(Hs + el * NQ2, NQ2, lane);
      if (lane == 0) outd[e0 + el] = s;
    }
    return;
  }

  // ---- D: y-back: K0[b] = sum_qy B H0 ; K1[b] = sum_qy (D H1 + B H2) -> K ------
  {
    const int l = tid;  // one line (c, qx) per thread
    const bool active = l < EB * D1 * NQ;
    const int el = active ? l / (D1 * NQ) : 0, rem = active ? l - el * (D1 * NQ) : 0;
    const int c = rem / NQ, qx = rem - c * NQ;
    constexpr int NH = DIAG ? 6 : 3 * O;  // z-back fields read by this line
    T hv[NH][NQ];
    if (active) {
      const T* h = Hs + el * L::HSTR + c * NQ2 + qx;
#pragma unroll
      for (int t = 0; t < NH; ++t)
#pragma unroll
        for (int qy = 0; qy < NQ; ++qy) hv[t][qy] = h[t * D1 * NQ2 + qy * NQ];
    }
    if (L::ALIAS) __syncthreads();  // z-back buffer consumed: the y-back may overwrite it
    if (active) {
      if constexpr (DIAG) {
        // group by x factor: K_D2 (term 00), K_B2 (11, 22, 12), K_DB (01, 02)
        T* k = Xs + el * L::XSTR + (c * NQ + qx) * L::XQ;
#pragma unroll(Unroll<D1>::full ? D1 : 1)
        for (int b = 0; b < D1; ++b) {
          T kd2 = 0, kb2 = 0, kdb = 0;
#pragma unroll
          for (int qy = 0; qy < NQ; ++qy) {
            const T by = tb.B[qy * D1 + b], dy = tb.Dy[qy * D1 + b];
            const T bb = by * by, dd = dy * dy, bd = by * dy;
            kd2 += bb * hv[0][qy];
            kb2 += dd * hv[1][qy];
            kb2 += bb * hv[2][qy];
            kb2 += bd * hv[5][qy];
            kdb += bd * hv[3][qy];
            kdb += bb * hv[4][qy];
          }
          k[b] = kd2;
          k[L::XS + b] = kb2;
          k[2 * L::XS + b] = kdb;
        }
      } else {
        using E = EO<D1, NQ>;
#pragma unroll
        for (int o = 0; o < O; ++o) {
          T* k = Xs + el * L::XSTR + o * 2 * L::XS + (c * NQ + qx) * L::XQ;
          if constexpr (!Unroll<D1>::full) {  // high order: even-odd, runtime loop over output pairs
            static_assert(D1 % 2 == 0, "the runtime even-odd loops take node pairs");
            T xe0[E::QH + 1], xo0[E::QH + 1], xm0, xe1[E::QH + 1], xo1[E::QH + 1], xm1, xe2[E::QH + 1],
                xo2[E::QH + 1], xm2;
            eo_pairs<D1, NQ>(hv[3 * o], xe0, xo0, xm0);
            eo_pairs<D1, NQ>(hv[3 * o + 1], xe1, xo1, xm1);
            eo_pairs<D1, NQ>(hv[3 * o + 2], xe2, xo2, xm2);
#pragma unroll(Config<D1, NQ, T>::RU)
            for (int a = 0; a < E::AH; ++a) {
              T sp0 = tb.Pb[a] * xe0[0], sm0 = tb.Nb[a] * xo0[0];
              T sp1 = tb.Py[a] * xo1[0], sm1 = tb.Ny[a] * xe1[0];
              sp1 += tb.Pb[a] * xe2[0];
              sm1 += tb.Nb[a] * xo2[0];
#pragma unroll
              for (int q = 1; q < E::QH; ++q) {
                const T pb = tb.Pb[q * E::AP + a], nb = tb.Nb[q * E::AH + a];
                sp0 += pb * xe0[q];
                sm0 += nb * xo0[q];
                sp1 += tb.Py[q * E::AP + a] * xo1[q];
                sm1 += tb.Ny[q * E::AH + a] * xe1[q];
                sp1 += pb * xe2[q];
                sm1 += nb * xo2[q];
              }
              if constexpr (NQ % 2) {  // the middle point
                sp0 += tb.Pb[E::QH * E::AP + a] * xm0;
                sm1 += tb.Ny[E::QH * E::AH + a] * xm1;
                sp1 += tb.Pb[E::QH * E::AP + a] * xm2;
              }
              k[a] = sp0 + sm0;
              k[D1 - 1 - a] = sp0 - sm0;
              k[L::XS + a] = sp1 + sm1;
              k[L::XS + D1 - 1 - a] = sp1 - sm1;
            }
            continue;
          }
          // K0 = B^T H0; K1 = Dy^T H1 + B^T H2 (even-odd form, one sum for both)
          T xe[E::QH + 1], xo[E::QH + 1], xm, sp0[E::AP], sm0[E::AH], sp1[E::AP], sm1[E::AH], k0[D1], k1[D1];
#pragma unroll
          for (int a = 0; a < E::AP; ++a) sp0[a] = sp1[a] = T(0);
#pragma unroll
          for (int a = 0; a < E::AH; ++a) sm0[a] = sm1[a] = T(0);
          eo_pairs<D1, NQ>(hv[3 * o], xe, xo, xm);
          eo_backward_add<D1, NQ, true>(tb.Pb, tb.Nb, xe, xo, xm, sp0, sm0);
          eo_pairs<D1, NQ>(hv[3 * o + 1], xe, xo, xm);
          eo_backward_add<D1, NQ, false>(tb.Py, tb.Ny, xe, xo, xm, sp1, sm1);
          eo_pairs<D1, NQ>(hv[3 * o + 2], xe, xo, xm);
          eo_backward_add<D1, NQ, true>(tb.Pb, tb.Nb, xe, xo, xm, sp1, sm1);
          eo_backward_finish<D1, NQ>(sp0, sm0, k0);
          eo_backward_finish<D1, NQ>(sp1, sm1, k1);
#pragma unroll
          for (int b = 0; b < D1; ++b) {
            k[b] = k0[b];
            k[L::XS + b] = k1[b];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- E: x-back: out[a] = sum_qx D K0 + B K1 -> E-vector --------------------
  for (int l = tid; l < EB * D1 * D1; l += NT) {
    const int el = l / (D1 * D1), cb = l - el * (D1 * D1);
    const int c = cb / D1, b = cb - c * D1;
    if (el >= n_valid) continue;
    const int64_t pos = ELM ? ((int64_t)(e0 + el) * Ne + cb * D1) * Ne + blockIdx.y  // column of K_e
                            : (int64_t)(e0 + el) * Ne + cb * D1;
    constexpr int OSTR = ELM ? Ne : 1;  // output stride along a (a K_e column for ELM)
    if constexpr (DIAG) {
      const T* k = Xs + el * L::XSTR + c * L::XC + b;
      T kd2[NQ], kb2[NQ], kdb[NQ];
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) {
        kd2[qx] = k[qx * L::XQ];
        kb2[qx] = k[L::XS + qx * L::XQ];
        kdb[qx] = k[2 * L::XS + qx * L::XQ];
      }
      T* out = static_cast<T*>(P.out0) + pos;
#pragma unroll(Unroll<D1>::full ? D1 : 1)
      for (int a = 0; a < D1; ++a) {
        T sacc = 0;
#pragma unroll
        for (int qx = 0; qx < NQ; ++qx) {
          const T bx = tb.B[qx * D1 + a], dx = tb.Dx[qx * D1 + a];
          sacc += dx * dx * kd2[qx];
          sacc += bx * bx * kb2[qx];
          sacc += bx * dx * kdb[qx];
        }
        out[a] = sacc;
      }
      continue;
    }
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const T* k = Xs + el * L::XSTR + o * 2 * L::XS + c * L::XC + b;
      T k0[NQ], k1[NQ];
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) {
        k0[qx] = k[qx * L::XQ];
        k1[qx] = k[L::XS + qx * L::XQ];
      }
      // output 0 is the JVP (or residual); output 1 the residual of residual + JVP
      T* out = static_cast<T*>(o == 0 ? (OP == OP_RESJVP ? P.out1 : P.out0) : P.out0) + pos;
      // out = Dx^T K0 + B^T K1 (even-odd form at every order, one sum for both)
      using E = EO<D1, NQ>;
      T xe[E::QH + 1], xo[E::QH + 1], xm, sp[E::AP], sm[E::AH], y[D1];
#pragma unroll
      for (int a = 0; a < E::AP; ++a) sp[a] = T(0);
#pragma unroll
      for (int a = 0; a < E::AH; ++a) sm[a] = T(0);
      eo_pairs<D1, NQ>(k0, xe, xo, xm);
      eo_backward_add<D1, NQ, false>(tb.Px, tb.Nx, xe, xo, xm, sp, sm);
      eo_pairs<D1, NQ>(k1, xe, xo, xm);
      eo_backward_add<D1, NQ, true>(tb.Pb, tb.Nb, xe, xo, xm, sp, sm);
      eo_backward_finish<D1, NQ>(sp, sm, y);
#pragma unroll
      for (int a = 0; a < D1; ++a) out[a * OSTR] = y[a];
    }
  }
}

// hs: the 1/h factor of each direction folded into its derivative table
// (affine meshes), or nullptr for the reference tables.
template <int D1, int NQ, class T>
Tab<D1, NQ, T> make_tab(const double* h, const double* hs = nullptr) {
  Tab<D1, NQ, T> t;
  for (int i = 0; i < NQ * D1; ++i) {
    const double d = h[NQ * D1 + i];
    t.B[i] = (T)h[i];
    t.Dx[i] = (T)(hs ? d * hs[0] : d);
    t.Dy[i] = (T)(hs ? d * hs[1] : d);
    t.Dz[i] = (T)(hs ? d * hs[2] : d);
  }
  for (int i = 0; i < NQ; ++i) {
    t.w[i] = (T)h[2 * NQ * D1 + i];
    t.xi[i] = (T)h[2 * NQ * D1 + NQ + i];
  }
  // even-odd forms, computed in FP64 from the (scaled) FP64 tables
  using E = EO<D1, NQ>;
  auto eo = [&](const double* M, double scale, T* P, T* N) {
    for (int q = 0; q < E::QP; ++q) {
      for (int a = 0; a < E::AH; ++a) {
        const double m0 = M[q * D1 + a] * scale, m1 = M[q * D1 + D1 - 1 - a] * scale;
        P[q * E::AP + a] = (T)(0.5 * (m0 + m1));
        N[q * E::AH + a] = (T)(0.5 * (m0 - m1));
      }
      if (D1 % 2) P[q * E::AP + E::AH] = (T)(M[q * D1 + E::AH] * scale);
    }
  };
  eo(h, 1.0, t.Pb, t.Nb);
  eo(h + NQ * D1, hs ? hs[0] : 1.0, t.Px, t.Nx);
  eo(h + NQ * D1, hs ? hs[1] : 1.0, t.Py, t.Ny);
  eo(h + NQ * D1, hs ? hs[2] : 1.0, t.Pz, t.Nz);
  return t;
}

// Instantiate every operation, precision, geometry and exponent kind for one
// (D1, NQ) and register the launchers in the dispatch table.
inline void no_tangents(ElemLaunchers&) {}

#define FEOD_INSTANTIATE(DD, QQ, TANGENTS)                                                        \
  template <class T, int OP, bool CURVED, int PK>                                                 \
  static hipError_t launch_##DD##_##QQ(const ElemParams& P, hipStream_t s) {                      \
    constexpr int EB = Config<DD, QQ, T>::EB;                                                     \
    constexpr int NT = Config<DD, QQ, T>::NT;                                                     \
    const int blocks = (P.E + EB - 1) / EB;                                                       \
    if (blocks == 0) return hipSuccess;                                                           \
    const Tab<DD, QQ, T> tb = make_tab<DD, QQ, T>(P.htab, CURVED ? nullptr : P.hinv);             \
    const dim3 grid(blocks, OP == OP_ELM ? DD * DD * DD : 1);                                    \
    hipLaunchKernelGGL((element_kernel<DD, QQ, T, OP, CURVED, PK>), grid, dim3(NT), 0, s, P, tb);  \
    return hipGetLastError();                                                                     \
  }                                                                                               \
  template <class T, bool CURVED, int PK>                                                         \
  static void fill_pk_##DD##_##QQ(ElemLaunchers::PerPrec& t) {                                    \
    t.op[OP_RESIDUAL][CURVED][PK] = &launch_##DD##_##QQ<T, OP_RESIDUAL, CURVED, PK>;              \
    t.op[OP_JVP][CURVED][PK] = &launch_##DD##_##QQ<T, OP_JVP, CURVED, PK>;                        \
    t.op[OP_RESJVP][CURVED][PK] = &launch_##DD##_##QQ<T, OP_RESJVP, CURVED, PK>;                  \
    t.op[OP_ENERGY][CURVED][PK] = &launch_##DD##_##QQ<T, OP_ENERGY, CURVED, PK>;                  \
    t.op[OP_GRAD][CURVED][PK] = &launch_##DD##_##QQ<T, OP_GRAD, CURVED, PK>;                      \
    t.op[OP_DIAG][CURVED][PK] = &launch_##DD##_##QQ<T, OP_DIAG, CURVED, PK>;                      \
    t.op[OP_QSTORE][CURVED][PK] = &launch_##DD##_##QQ<T, OP_QSTORE, CURVED, PK>;                  \
    t.op[OP_JVP_PA][CURVED][PK] = &launch_##DD##_##QQ<T, OP_JVP_PA, CURVED, PK>;                  \
    if constexpr (sizeof(T) == 8 && DD <= 5)                                                      \
      t.op[OP_ELM][CURVED][PK] = &launch_##DD##_##QQ<T, OP_ELM, CURVED, PK>;                      \
    if constexpr (sizeof(T) == 8)                                                                 \
      t.op[OP_JVP_HND][CURVED][PK] = &launch_##DD##_##QQ<T, OP_JVP_HND, CURVED, PK>;              \
  }                                                                                               \
  template <class T, bool CURVED>                                                                 \
  static void fill_##DD##_##QQ(ElemLaunchers::PerPrec& t) {                                       \
    fill_pk_##DD##_##QQ<T, CURVED, POW_ZERO>(t);                                                  \
    fill_pk_##DD##_##QQ<T, CURVED, POW_QUARTER>(t);                                               \
    fill_pk_##DD##_##QQ<T, CURVED, POW_HALF>(t);                                                  \
    fill_pk_##DD##_##QQ<T, CURVED, POW_ONE>(t);                                                   \
    fill_pk_##DD##_##QQ<T, CURVED, POW_GENERIC>(t);                                               \
  }                                                                                               \
  ElemLaunchers make_launchers_##DD##_##QQ() {                                                    \
    ElemLaunchers L{};                                                                            \
    L.D1 = DD;                                                                                    \
    L.NQ = QQ;                                                                                    \
    fill_##DD##_##QQ<double, false>(L.prec[0]);                                                   \
    fill_##DD##_##QQ<double, true>(L.prec[0]);                                                    \
    fill_##DD##_##QQ<float, false>(L.prec[1]);                                                    \
    fill_##DD##_##QQ<float, true>(L.prec[1]);                                                     \
    L.eb[0] = Config<DD, QQ, double>::EB;                                                         \
    L.eb[1] = Config<DD, QQ, float>::EB;                                                          \
    TANGENTS(L);                                                                                  \
    return L;                                                                                     \
  }

}  // namespace feod
