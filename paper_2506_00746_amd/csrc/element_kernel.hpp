// Fused element kernel of the finite element operator decomposition
// A = G^T B^T D B G (paper, Fig. 1, Eq. (1)-(2)), one workgroup per batch of
// EB elements:
//
//   G    gather of M u (and M v) through the element-to-DOF map into LDS
//        (Dirichlet DOFs are encoded as -1 in the map and read as 0);
//   B    reference gradients at the nq^3 Gauss points by three sum-factorised
//        1D passes (x, y, z) through LDS;
//   D    the pointwise flux at every quadrature point, on dual numbers for the
//        Jacobian action (Eq. (2)), with the trilinear geometry recomputed per
//        point on curved meshes;
//   B^T  three transposed passes (z, y, x) back to element DOFs, written as
//        the output E-vector (G^T is a separate deterministic gather).
//
// Quadrature-point data lives only in LDS and registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_api.hpp"
#include "pointwise.hpp"

namespace feod {

constexpr int kThreads = 256;

template <int D1, int NQ>
struct Shape {
  static constexpr int Ne = D1 * D1 * D1;
  static constexpr int NQ3 = NQ * NQ * NQ;
  static constexpr int NX = D1 * D1 * NQ;   // one x-pass output field
  static constexpr int NY = D1 * NQ * NQ;   // one y-pass output field
  // per-element LDS footprint in scalars: two input fields, x/y scratch, two
  // gradient fields, 8 vertices
  static constexpr int per_elem = 2 * Ne + 2 * NX + 3 * NY + 6 * NQ3 + 24;
};

template <int D1, int NQ, class T>
struct Batch {
  static constexpr int lds_target = 48 * 1024;
  static constexpr int raw = lds_target / (Shape<D1, NQ>::per_elem * (int)sizeof(T));
  static constexpr int EB = raw < 1 ? 1 : (raw > 16 ? 16 : raw);
};

// ---------------------------------------------------------------------------
// B: in[el][c][b][a] (D1^3) -> G[el][d][qz][qy][qx] (3 fields of NQ^3),
// d = 0,1,2 the x,y,z reference derivative.
template <int D1, int NQ, int EB, class T>
__device__ __forceinline__ void grad_forward(const T* __restrict__ sB, const T* __restrict__ sD,
                                             const T* in, T* X, T* Y, T* G) {
  using S = Shape<D1, NQ>;
  const int tid = threadIdx.x;
  // x-pass: X0[c][b][qx] = sum_a B[qx][a] in[c][b][a], X1 with D
  for (int i = tid; i < EB * S::NX; i += kThreads) {
    const int el = i / S::NX, rem = i - el * S::NX;
    const int qx = rem % NQ, cb = rem / NQ;
    const T* src = in + el * S::Ne + cb * D1;
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int a = 0; a < D1; ++a) {
      const T x = src[a];
      s0 += sB[qx * D1 + a] * x;
      s1 += sD[qx * D1 + a] * x;
    }
    X[el * 2 * S::NX + rem] = s0;
    X[el * 2 * S::NX + S::NX + rem] = s1;
  }
  __syncthreads();
  // y-pass: Y0 = D_y X0 (-> d/dy), Y1 = B_y X0 (-> d/dz), Y2 = B_y X1 (-> d/dx)
  for (int i = tid; i < EB * S::NY; i += kThreads) {
    const int el = i / S::NY, rem = i - el * S::NY;
    const int qx = rem % NQ, qy = (rem / NQ) % NQ, c = rem / (NQ * NQ);
    const T* x0 = X + el * 2 * S::NX + c * D1 * NQ + qx;
    const T* x1 = x0 + S::NX;
    T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int b = 0; b < D1; ++b) {
      const T b0 = x0[b * NQ], b1 = x1[b * NQ];
      s0 += sD[qy * D1 + b] * b0;
      s1 += sB[qy * D1 + b] * b0;
      s2 += sB[qy * D1 + b] * b1;
    }
    T* y = Y + el * 3 * S::NY + rem;
    y[0] = s0;
    y[S::NY] = s1;
    y[2 * S::NY] = s2;
  }
  __syncthreads();
  // z-pass: Gx = B_z Y2, Gy = B_z Y0, Gz = D_z Y1
  for (int i = tid; i < EB * S::NQ3; i += kThreads) {
    const int el = i / S::NQ3, q = i - el * S::NQ3;
    const int qxy = q % (NQ * NQ), qz = q / (NQ * NQ);
    const T* y = Y + el * 3 * S::NY + qxy;
    T gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int c = 0; c < D1; ++c) {
      const T bz = sB[qz * D1 + c];
      gx += bz * y[2 * S::NY + c * NQ * NQ];
      gy += bz * y[c * NQ * NQ];
      gz += sD[qz * D1 + c] * y[S::NY + c * NQ * NQ];
    }
    T* g = G + el * 3 * S::NQ3 + q;
    g[0] = gx;
    g[S::NQ3] = gy;
    g[2 * S::NQ3] = gz;
  }
  __syncthreads();
}

// B^T: G[el][d][q] -> out (E-vector of the batch, T), out[el*Ne + (c*D1+b)*D1+a]
template <int D1, int NQ, int EB, class T>
__device__ __forceinline__ void grad_backward(const T* __restrict__ sB, const T* __restrict__ sD,
                                              const T* G, T* X, T* Y, T* __restrict__ out,
                                              int n_valid) {
  using S = Shape<D1, NQ>;
  const int tid = threadIdx.x;
  // z-back: Y0[c][qy][qx] = sum_qz B[qz][c] Gx, Y1 = B Gy, Y2 = D Gz
  for (int i = tid; i < EB * S::NY; i += kThreads) {
    const int el = i / S::NY, rem = i - el * S::NY;
    const int qxy = rem % (NQ * NQ), c = rem / (NQ * NQ);
    const T* g = G + el * 3 * S::NQ3 + qxy;
    T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      const T bz = sB[qz * D1 + c];
      s0 += bz * g[qz * NQ * NQ];
      s1 += bz * g[S::NQ3 + qz * NQ * NQ];
      s2 += sD[qz * D1 + c] * g[2 * S::NQ3 + qz * NQ * NQ];
    }
    T* y = Y + el * 3 * S::NY + rem;
    y[0] = s0;
    y[S::NY] = s1;
    y[2 * S::NY] = s2;
  }
  __syncthreads();
  // y-back: X0[c][b][qx] = sum_qy B[qy][b] Y0 ; X1 = sum_qy D[qy][b] Y1 + B[qy][b] Y2
  for (int i = tid; i < EB * S::NX; i += kThreads) {
    const int el = i / S::NX, rem = i - el * S::NX;
    const int qx = rem % NQ, b = (rem / NQ) % D1, c = rem / (NQ * D1);
    const T* y = Y + el * 3 * S::NY + c * NQ * NQ + qx;
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int qy = 0; qy < NQ; ++qy) {
      const T by = sB[qy * D1 + b];
      s0 += by * y[qy * NQ];
      s1 += sD[qy * D1 + b] * y[S::NY + qy * NQ] + by * y[2 * S::NY + qy * NQ];
    }
    X[el * 2 * S::NX + rem] = s0;
    X[el * 2 * S::NX + S::NX + rem] = s1;
  }
  __syncthreads();
  // x-back: out[c][b][a] = sum_qx D[qx][a] X0 + B[qx][a] X1
  for (int i = tid; i < n_valid * S::Ne; i += kThreads) {
    const int el = i / S::Ne, rem = i - el * S::Ne;
    const int a = rem % D1, cb = rem / D1;
    const T* x = X + el * 2 * S::NX + cb * NQ;
    T s = 0;
#pragma unroll
    for (int qx = 0; qx < NQ; ++qx) s += sD[qx * D1 + a] * x[qx] + sB[qx * D1 + a] * x[S::NX + qx];
    out[i] = s;
  }
}

// Geometry at one quadrature point: adjugate (transposed cofactor) of the
// Jacobian Jg = dx/dxi and its determinant.  Jg^{-1} = adj / det.
template <class T>
__device__ __forceinline__ void trilinear_adj(const T* X, T xi, T et, T ze, T adj[3][3], T* det) {
  const T mx = T(1) - xi, me = T(1) - et, mz = T(1) - ze;
  T J[3][3];
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    const T* x = X + al;  // X[v*3 + al], v = i + 2j + 4l
    J[al][0] = (me * mz) * (x[3] - x[0]) + (et * mz) * (x[9] - x[6]) + (me * ze) * (x[15] - x[12]) + (et * ze) * (x[21] - x[18]);
    J[al][1] = (mx * mz) * (x[6] - x[0]) + (xi * mz) * (x[9] - x[3]) + (mx * ze) * (x[18] - x[12]) + (xi * ze) * (x[21] - x[15]);
    J[al][2] = (mx * me) * (x[12] - x[0]) + (xi * me) * (x[15] - x[3]) + (mx * et) * (x[18] - x[6]) + (xi * et) * (x[21] - x[9]);
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
  *det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
}

// Deterministic sum of n LDS values by one wavefront (fixed order).
template <class T>
__device__ __forceinline__ double wave_sum(const T* vals, int n, int lane) {
  double s = 0;
  for (int i = lane; i < n; i += 64) s += (double)vals[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

template <int D1, int NQ, class T, int OP, bool CURVED>
__global__ __launch_bounds__(kThreads) void element_kernel(ElemParams P) {
  using S = Shape<D1, NQ>;
  constexpr int EB = Batch<D1, NQ, T>::EB;
  constexpr bool two_fields = (OP == OP_JVP || OP == OP_RESJVP || OP == OP_GRAD);
  __shared__ T sB[NQ * D1], sD[NQ * D1], sW[NQ], sQ[NQ];
  __shared__ T smem[EB * S::per_elem];
  T* sU = smem;                       // EB * Ne
  T* sV = sU + EB * S::Ne;            // EB * Ne
  T* X = sV + EB * S::Ne;             // EB * 2 * NX
  T* Y = X + EB * 2 * S::NX;          // EB * 3 * NY
  T* G1 = Y + EB * 3 * S::NY;         // EB * 3 * NQ3
  T* G2 = G1 + EB * 3 * S::NQ3;       // EB * 3 * NQ3
  T* sX = G2 + EB * 3 * S::NQ3;       // EB * 24

  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EB;
  const int n_valid = min(EB, P.E - e0);
  const T* tab = static_cast<const T*>(P.tab);
  for (int i = tid; i < NQ * D1; i += kThreads) {
    sB[i] = tab[i];
    sD[i] = tab[NQ * D1 + i];
  }
  for (int i = tid; i < NQ; i += kThreads) {
    sW[i] = tab[2 * NQ * D1 + i];
    sQ[i] = tab[2 * NQ * D1 + NQ + i];
  }
  // G: gather through the map (-1 = Dirichlet DOF, read as 0)
  for (int i = tid; i < EB * S::Ne; i += kThreads) {
    const int el = i / S::Ne;
    T xu = 0, xv = 0;
    if (el < n_valid) {
      const int m = P.emap[(int64_t)e0 * S::Ne + i];
      if (m >= 0) {
        xu = (T)P.u[m];
        if (two_fields) xv = (T)P.v[m];
      }
    }
    sU[i] = xu;
    if (two_fields) sV[i] = xv;
  }
  if (CURVED) {
    for (int i = tid; i < EB * 24; i += kThreads) {
      const int el = i / 24, r = i - el * 24, vtx = r / 3, al = r - vtx * 3;
      T val = 0;
      if (el < n_valid) {
        const int e = e0 + el;
        const int ex = e % P.nx, ey = (e / P.nx) % P.ny, ez = e / (P.nx * P.ny);
        const int gi = (ex + (vtx & 1)) + (P.nx + 1) * ((ey + ((vtx >> 1) & 1)) + (P.ny + 1) * (ez + (vtx >> 2)));
        val = (T)P.verts[(int64_t)gi * 3 + al];
      }
      sX[i] = val;
    }
  }
  __syncthreads();

  grad_forward<D1, NQ, EB, T>(sB, sD, sU, X, Y, G1);
  if (two_fields) grad_forward<D1, NQ, EB, T>(sB, sD, sV, X, Y, G2);

  // D at every quadrature point of the batch
  const T eps2 = (T)P.eps2, r = (T)P.r, inv_p = (T)P.inv_p;
  const int kind = P.powkind;
  for (int i = tid; i < EB * S::NQ3; i += kThreads) {
    const int el = i / S::NQ3, q = i - el * S::NQ3;
    const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
    const T w = sW[qx] * sW[qy] * sW[qz];
    T adj[3][3], det;
    if (CURVED) {
      trilinear_adj<T>(sX + el * 24, sQ[qx], sQ[qy], sQ[qz], adj, &det);
    } else {
      const T hx = (T)P.h[0], hy = (T)P.h[1], hz = (T)P.h[2];
      det = hx * hy * hz;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) adj[a][b] = 0;
      adj[0][0] = hy * hz;
      adj[1][1] = hx * hz;
      adj[2][2] = hx * hy;
    }
    const T inv_det = T(1) / det;
    T* g1 = G1 + el * 3 * S::NQ3 + q;
    T* g2 = G2 + el * 3 * S::NQ3 + q;
    const T rg[3] = {g1[0], g1[S::NQ3], g1[2 * S::NQ3]};
    // physical gradient g = Jg^{-T} ghat = adj^T ghat / det
    T gu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gu[a] = (adj[0][a] * rg[0] + adj[1][a] * rg[1] + adj[2][a] * rg[2]) * inv_det;
    const int e = e0 + el;
    const T rho = (P.rho != nullptr && el < n_valid) ? (T)P.rho[e] : T(1);
    if (OP == OP_RESIDUAL) {
      T F[3];
      flux<T, T>(gu, eps2, r, kind, F);
      const T s = rho * w;  // Fhat = rho w det Jg^{-1} F = rho w adj F
#pragma unroll
      for (int a = 0; a < 3; ++a) g1[a * S::NQ3] = s * (adj[a][0] * F[0] + adj[a][1] * F[1] + adj[a][2] * F[2]);
    } else if (OP == OP_JVP || OP == OP_RESJVP) {
      const T rv[3] = {g2[0], g2[S::NQ3], g2[2 * S::NQ3]};
      dual<T> g[3], F[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        g[a].v = gu[a];
        g[a].d = (adj[0][a] * rv[0] + adj[1][a] * rv[1] + adj[2][a] * rv[2]) * inv_det;
      }
      flux<dual<T>, T>(g, eps2, r, kind, F);
      const T s = rho * w;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T fd = s * (adj[a][0] * F[0].d + adj[a][1] * F[1].d + adj[a][2] * F[2].d);
        if (OP == OP_RESJVP) {
          g1[a * S::NQ3] = s * (adj[a][0] * F[0].v + adj[a][1] * F[1].v + adj[a][2] * F[2].v);
          g2[a * S::NQ3] = fd;
        } else {
          g1[a * S::NQ3] = fd;
        }
      }
    } else if (OP == OP_ENERGY) {
      T W, c;
      density<T>(gu, eps2, r, kind, inv_p, &W, &c);
      g1[0] = rho * w * det * W;
    } else if (OP == OP_GRAD) {
      const T rv[3] = {g2[0], g2[S::NQ3], g2[2 * S::NQ3]};
      T gl[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) gl[a] = (adj[0][a] * rv[0] + adj[1][a] * rv[1] + adj[2][a] * rv[2]) * inv_det;
      T W, c;
      density<T>(gu, eps2, r, kind, inv_p, &W, &c);
      g1[0] = -w * det * c * (gu[0] * gl[0] + gu[1] * gl[1] + gu[2] * gl[2]);
    }
  }
  __syncthreads();

  if (OP == OP_ENERGY || OP == OP_GRAD) {
    // per-element deterministic reduction over its quadrature points
    const int lane = tid & 63, wv = tid >> 6;
    double* outd = static_cast<double*>(P.out0);
    for (int el = wv; el < n_valid; el += kThreads / 64) {
      const double s = wave_sum<T>(G1 + el * 3 * S::NQ3, S::NQ3, lane);
      if (lane == 0) outd[e0 + el] = s;
    }
    return;
  }
  T* out0 = static_cast<T*>(P.out0) + (int64_t)e0 * S::Ne;
  grad_backward<D1, NQ, EB, T>(sB, sD, G1, X, Y, out0, n_valid);
  if (OP == OP_RESJVP) {
    __syncthreads();
    T* out1 = static_cast<T*>(P.out1) + (int64_t)e0 * S::Ne;
    grad_backward<D1, NQ, EB, T>(sB, sD, G2, X, Y, out1, n_valid);
  }
}

// Instantiate every operation, precision and geometry for one (D1, NQ) and
// register the launchers in the dispatch table.
#define FEOD_INSTANTIATE(DD, QQ)                                                              \
  template <class T, int OP, bool CURVED>                                                     \
  static hipError_t launch_##DD##_##QQ(const ElemParams& P, hipStream_t s) {                  \
    constexpr int EB = Batch<DD, QQ, T>::EB;                                                  \
    const int blocks = (P.E + EB - 1) / EB;                                                   \
    if (blocks == 0) return hipSuccess;                                                       \
    hipLaunchKernelGGL((element_kernel<DD, QQ, T, OP, CURVED>), dim3(blocks), dim3(kThreads), \
                       0, s, P);                                                              \
    return hipGetLastError();                                                                 \
  }                                                                                           \
  template <class T, bool CURVED>                                                             \
  static void fill_##DD##_##QQ(ElemLaunchers::PerPrec& t) {                                   \
    t.op[OP_RESIDUAL][CURVED] = &launch_##DD##_##QQ<T, OP_RESIDUAL, CURVED>;                  \
    t.op[OP_JVP][CURVED] = &launch_##DD##_##QQ<T, OP_JVP, CURVED>;                            \
    t.op[OP_RESJVP][CURVED] = &launch_##DD##_##QQ<T, OP_RESJVP, CURVED>;                      \
    t.op[OP_ENERGY][CURVED] = &launch_##DD##_##QQ<T, OP_ENERGY, CURVED>;                      \
    t.op[OP_GRAD][CURVED] = &launch_##DD##_##QQ<T, OP_GRAD, CURVED>;                          \
  }                                                                                           \
  ElemLaunchers make_launchers_##DD##_##QQ() {                                                \
    ElemLaunchers L{};                                                                        \
    L.D1 = DD;                                                                                \
    L.NQ = QQ;                                                                                \
    fill_##DD##_##QQ<double, false>(L.prec[0]);                                               \
    fill_##DD##_##QQ<double, true>(L.prec[0]);                                                \
    fill_##DD##_##QQ<float, false>(L.prec[1]);                                                \
    fill_##DD##_##QQ<float, true>(L.prec[1]);                                                 \
    L.eb[0] = Batch<DD, QQ, double>::EB;                                                      \
    L.eb[1] = Batch<DD, QQ, float>::EB;                                                       \
    return L;                                                                                 \
  }

}  // namespace feod
