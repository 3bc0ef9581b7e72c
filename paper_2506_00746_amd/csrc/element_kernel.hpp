// Fused element kernel of the finite element operator decomposition
// A = G^T B^T D B G (paper, Fig. 1, Eq. (1)-(2)).  One workgroup processes a
// batch of EB elements in five phases separated by barriers; in every phase a
// thread owns whole 1D lines, so each value it loads feeds D1 or NQ
// multiply-adds whose table operand is uniform across the wavefront (the 1D
// tables travel in the kernel arguments and are read as scalars):
//
//   A  G + x-pass   line (c,b): gather the D1 DOFs of an x-line of M u (and
//                   M v) through the element-to-DOF map straight from HBM,
//                   contract with B and D in x -> LDS.
//   B  y-pass       line (c,qx): contract in y -> LDS (three partial fields).
//   C  z-pass, D, z-back   line (qx,qy): finish the reference gradients at the
//                   NQ points of the z-column in registers, apply the pointwise
//                   operator D there (dual numbers for the Jacobian action,
//                   trilinear geometry recomputed per point on curved meshes),
//                   and contract the fluxes back over z -> LDS.  Quadrature
//                   data never leaves registers.
//   D  y-back       line (c,qx) -> LDS.
//   E  x-back       line (c,b): D1 element residual entries written
//                   contiguously to the output E-vector in HBM (G^T is the
//                   separate deterministic gather).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_api.hpp"
#include "pointwise.hpp"

namespace feod {

// 1D tables by value in the kernel arguments: B[q*D1+a] = l_a(x_q),
// D[q*D1+a] = l_a'(x_q), Gauss weights w and points xi on [0,1].
template <int D1, int NQ, class T>
struct Tab {
  T B[NQ * D1];
  T D[NQ * D1];
  T w[NQ];
  T xi[NQ];
};

// Launch shape per (D1, NQ, precision): threads per workgroup and elements
// per batch, chosen so that phase C (NQ^2 lines per element) fills the
// workgroup and the LDS footprint leaves room for several workgroups per CU.
template <int D1, int NQ, class T>
struct Config {
  static constexpr int lines_c = NQ * NQ;
  static constexpr int NT = lines_c <= 16 ? 64 : 128;
  static constexpr int EB0 = NT / lines_c;
  static constexpr int EB = EB0 < 1 ? 1 : EB0;
};

template <int D1, int NQ, int F>
struct Lds {
  static constexpr int X = 2 * NQ * D1 * D1;  // one field of x-pass output
  static constexpr int Y = 3 * NQ * NQ * D1;  // one field of y-pass output
  static constexpr int per_elem = F * X + 2 * Y + 24;
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

template <int D1, int NQ, class T, int OP, bool CURVED>
__global__ __launch_bounds__((Config<D1, NQ, T>::NT)) void element_kernel(ElemParams P, Tab<D1, NQ, T> tb) {
  constexpr int NT = Config<D1, NQ, T>::NT;
  constexpr int EB = Config<D1, NQ, T>::EB;
  constexpr int Ne = D1 * D1 * D1;
  constexpr int F = (OP == OP_JVP || OP == OP_RESJVP || OP == OP_GRAD) ? 2 : 1;  // input fields
  constexpr int O = (OP == OP_RESJVP) ? 2 : 1;                                    // output fields
  constexpr bool REDUCE = (OP == OP_ENERGY || OP == OP_GRAD);
  using L = Lds<D1, NQ, F>;
  __shared__ T smem[EB * L::per_elem];
  T* Xs = smem;                       // [el][f][2][c][b][qx]
  T* Ys = Xs + EB * F * L::X;         // [el][f][3][c][qy][qx], reused for H and K
  T* Vs = Ys + EB * 2 * L::Y;         // [el][24] vertex coordinates

  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EB;
  const int n_valid = min(EB, P.E - e0);

  if (CURVED) {
    for (int i = tid; i < EB * 24; i += NT) {
      const int el = i / 24, r = i - el * 24, vtx = r / 3, al = r - vtx * 3;
      T val = 0;
      if (el < n_valid) {
        const int e = e0 + el;
        const int ex = e % P.nx, ey = (e / P.nx) % P.ny, ez = e / (P.nx * P.ny);
        const int gi = (ex + (vtx & 1)) + (P.nx + 1) * ((ey + ((vtx >> 1) & 1)) + (P.ny + 1) * (ez + (vtx >> 2)));
        val = (T)P.verts[(int64_t)gi * 3 + al];
      }
      Vs[i] = val;
    }
  }

  // ---- A: gather + x-pass ---------------------------------------------------
  for (int l = tid; l < EB * D1 * D1; l += NT) {
    const int el = l / (D1 * D1), cb = l - el * (D1 * D1);
    T in[F][D1];
    if (el < n_valid) {
      const int32_t* m = P.emap + (int64_t)(e0 + el) * Ne + cb * D1;
#pragma unroll
      for (int a = 0; a < D1; ++a) {
        const int idx = m[a];
        in[0][a] = idx >= 0 ? (T)P.u[idx] : T(0);
        if (F == 2) in[F - 1][a] = idx >= 0 ? (T)P.v[idx] : T(0);
      }
    } else {
#pragma unroll
      for (int f = 0; f < F; ++f)
#pragma unroll
        for (int a = 0; a < D1; ++a) in[f][a] = 0;
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
      T* x = Xs + (el * F + f) * L::X + cb * NQ;
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int a = 0; a < D1; ++a) {
          s0 += tb.B[qx * D1 + a] * in[f][a];
          s1 += tb.D[qx * D1 + a] * in[f][a];
        }
        x[qx] = s0;
        x[NQ * D1 * D1 + qx] = s1;
      }
    }
  }
  __syncthreads();

  // ---- B: y-pass: Y0 = D_y X0 (d/dy), Y1 = B_y X0 (d/dz), Y2 = B_y X1 (d/dx) --
  for (int l = tid; l < EB * D1 * NQ; l += NT) {
    const int el = l / (D1 * NQ), rem = l - el * (D1 * NQ);
    const int c = rem / NQ, qx = rem - c * NQ;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const T* x = Xs + (el * F + f) * L::X + c * D1 * NQ + qx;
      T x0[D1], x1[D1];
#pragma unroll
      for (int b = 0; b < D1; ++b) {
        x0[b] = x[b * NQ];
        x1[b] = x[NQ * D1 * D1 + b * NQ];
      }
      T* y = Ys + (el * 2 + f) * L::Y + c * NQ * NQ + qx;
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int b = 0; b < D1; ++b) {
          s0 += tb.D[qy * D1 + b] * x0[b];
          s1 += tb.B[qy * D1 + b] * x0[b];
          s2 += tb.B[qy * D1 + b] * x1[b];
        }
        y[qy * NQ] = s0;
        y[NQ * NQ * D1 + qy * NQ] = s1;
        y[2 * NQ * NQ * D1 + qy * NQ] = s2;
      }
    }
  }
  __syncthreads();

  // ---- C: z-pass, pointwise D, z-back (registers) ---------------------------
  T* red = Xs;  // per-line partial sums for energy / gradient
  const T eps2 = (T)P.eps2, r = (T)P.r, inv_p = (T)P.inv_p;
  const int kind = P.powkind;
  for (int l = tid; l < EB * NQ * NQ; l += NT) {
    const int el = l / (NQ * NQ), qxy = l - el * (NQ * NQ);
    const int qy = qxy / NQ, qx = qxy - qy * NQ;
    T g[F][3][NQ];
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < NQ; ++q) g[f][d][q] = 0;
#pragma unroll
    for (int c = 0; c < D1; ++c) {
#pragma unroll
      for (int f = 0; f < F; ++f) {
        const T* y = Ys + (el * 2 + f) * L::Y + c * NQ * NQ + qxy;
        const T y0 = y[0], y1 = y[NQ * NQ * D1], y2 = y[2 * NQ * NQ * D1];
#pragma unroll
        for (int qz = 0; qz < NQ; ++qz) {
          g[f][0][qz] += tb.B[qz * D1 + c] * y2;
          g[f][1][qz] += tb.B[qz * D1 + c] * y0;
          g[f][2][qz] += tb.D[qz * D1 + c] * y1;
        }
      }
    }
    const bool valid = el < n_valid;
    const T rho = (P.rho != nullptr && valid) ? (T)P.rho[e0 + el] : T(1);
    const T wxy = tb.w[qx] * tb.w[qy] * rho;
    // geometry: affine -> constant diagonal; curved -> Jg = J0 + xi_z * J1
    T J0[3][3], J1[3][2];
    if (CURVED) {
      const T* X = Vs + el * 24;
      const T xi = tb.xi[qx], et = tb.xi[qy], mx = T(1) - xi, me = T(1) - et;
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
    }
    const T hinv[3] = {(T)P.hinv[0], (T)P.hinv[1], (T)P.hinv[2]};
    const T sdet[3] = {(T)P.sdet[0], (T)P.sdet[1], (T)P.sdet[2]};  // det * hinv (affine)
    const T det_aff = (T)P.det;
    double part = 0;  // energy / gradient partial over the column
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz) {
      const T wq = wxy * tb.w[qz];
      T gu[3], gv[3];
      T adj[3][3], inv_det = T(1), det = det_aff;
      if (CURVED) {
        const T ze = tb.xi[qz];
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
        inv_det = T(1) / det;
        // physical gradient g = Jg^{-T} ghat = adj^T ghat / det
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gu[a] = (adj[0][a] * g[0][0][qz] + adj[1][a] * g[0][1][qz] + adj[2][a] * g[0][2][qz]) * inv_det;
          if (F == 2) gv[a] = (adj[0][a] * g[F - 1][0][qz] + adj[1][a] * g[F - 1][1][qz] + adj[2][a] * g[F - 1][2][qz]) * inv_det;
        }
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gu[a] = g[0][a][qz] * hinv[a];
          if (F == 2) gv[a] = g[F - 1][a][qz] * hinv[a];
        }
      }
      // reference flux Fhat = rho w det Jg^{-1} F = rho w adj F
      T Fo[O][3];
      if (OP == OP_RESIDUAL) {
        flux<T, T>(gu, eps2, r, kind, Fo[0]);
      } else if (OP == OP_JVP || OP == OP_RESJVP) {
        dual<T> gd[3], Fd[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gd[a] = {gu[a], gv[a]};
        flux<dual<T>, T>(gd, eps2, r, kind, Fd);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Fo[0][a] = Fd[a].d;
          if (O == 2) Fo[O - 1][a] = Fd[a].v;  // residual part of residual + JVP
        }
      } else if (OP == OP_ENERGY) {
        T W, cf;
        density<T>(gu, eps2, r, kind, inv_p, &W, &cf);
        part += (double)(wq * det * W);
      } else if (OP == OP_GRAD) {
        T W, cf;
        density<T>(gu, eps2, r, kind, inv_p, &W, &cf);
        // no rho: dR/drho_e; wq carries rho, so divide it back out via wxy
        const T wnr = tb.w[qx] * tb.w[qy] * tb.w[qz];
        part -= (double)(wnr * det * cf * (gu[0] * gv[0] + gu[1] * gv[1] + gu[2] * gv[2]));
      }
      if (!REDUCE) {
#pragma unroll
        for (int o = 0; o < O; ++o) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            T fh;
            if (CURVED)
              fh = wq * (adj[a][0] * Fo[o][0] + adj[a][1] * Fo[o][1] + adj[a][2] * Fo[o][2]);
            else
              fh = wq * sdet[a] * Fo[o][a];
            g[o][a][qz] = fh;  // reuse the gradient registers for the fluxes
          }
        }
      }
    }
    if (REDUCE) {
      red[l] = (T)part;
    } else {
      // z-back: H0[c] = sum_qz B Fx, H1 = sum B Fy, H2 = sum D Fz -> in place over Y
#pragma unroll
      for (int o = 0; o < O; ++o) {
        T* h = Ys + (el * 2 + o) * L::Y + qxy;
#pragma unroll
        for (int c = 0; c < D1; ++c) {
          T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
          for (int qz = 0; qz < NQ; ++qz) {
            s0 += tb.B[qz * D1 + c] * g[o][0][qz];
            s1 += tb.B[qz * D1 + c] * g[o][1][qz];
            s2 += tb.D[qz * D1 + c] * g[o][2][qz];
          }
          h[c * NQ * NQ] = s0;
          h[NQ * NQ * D1 + c * NQ * NQ] = s1;
          h[2 * NQ * NQ * D1 + c * NQ * NQ] = s2;
        }
      }
    }
  }
  __syncthreads();

  if (REDUCE) {
    const int lane = tid & 63, wv = tid >> 6;
    double* outd = static_cast<double*>(P.out0);
    for (int el = wv; el < n_valid; el += NT / 64) {
      const double s = wave_sum<T>(red + el * NQ * NQ, NQ * NQ, lane);
      if (lane == 0) outd[e0 + el] = s;
    }
    return;
  }

  // ---- D: y-back: K0[b] = sum_qy B H0 ; K1[b] = sum_qy D H1 + B H2 -> X -------
  for (int l = tid; l < EB * D1 * NQ; l += NT) {
    const int el = l / (D1 * NQ), rem = l - el * (D1 * NQ);
    const int c = rem / NQ, qx = rem - c * NQ;
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const T* h = Ys + (el * 2 + o) * L::Y + c * NQ * NQ + qx;
      T h0[NQ], h1[NQ], h2[NQ];
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) {
        h0[qy] = h[qy * NQ];
        h1[qy] = h[NQ * NQ * D1 + qy * NQ];
        h2[qy] = h[2 * NQ * NQ * D1 + qy * NQ];
      }
      T* k = Xs + (el * F + o) * L::X + c * D1 * NQ + qx;
#pragma unroll
      for (int b = 0; b < D1; ++b) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int qy = 0; qy < NQ; ++qy) {
          s0 += tb.B[qy * D1 + b] * h0[qy];
          s1 += tb.D[qy * D1 + b] * h1[qy] + tb.B[qy * D1 + b] * h2[qy];
        }
        k[b * NQ] = s0;
        k[NQ * D1 * D1 + b * NQ] = s1;
      }
    }
  }
  __syncthreads();

  // ---- E: x-back: out[a] = sum_qx D K0 + B K1 -> E-vector --------------------
  for (int l = tid; l < n_valid * D1 * D1; l += NT) {
    const int el = l / (D1 * D1), cb = l - el * (D1 * D1);
#pragma unroll
    for (int o = 0; o < O; ++o) {
      const T* k = Xs + (el * F + o) * L::X + cb * NQ;
      T k0[NQ], k1[NQ];
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) {
        k0[qx] = k[qx];
        k1[qx] = k[NQ * D1 * D1 + qx];
      }
      // output 0 is the JVP (or residual), output 1 the residual of residual + JVP
      T* out = static_cast<T*>(o == 0 ? (OP == OP_RESJVP ? P.out1 : P.out0) : P.out0) +
               (int64_t)(e0 + el) * Ne + cb * D1;
#pragma unroll
      for (int a = 0; a < D1; ++a) {
        T s = 0;
#pragma unroll
        for (int qx = 0; qx < NQ; ++qx) s += tb.D[qx * D1 + a] * k0[qx] + tb.B[qx * D1 + a] * k1[qx];
        out[a] = s;
      }
    }
  }
}

template <int D1, int NQ, class T>
Tab<D1, NQ, T> make_tab(const double* h) {
  Tab<D1, NQ, T> t;
  for (int i = 0; i < NQ * D1; ++i) {
    t.B[i] = (T)h[i];
    t.D[i] = (T)h[NQ * D1 + i];
  }
  for (int i = 0; i < NQ; ++i) {
    t.w[i] = (T)h[2 * NQ * D1 + i];
    t.xi[i] = (T)h[2 * NQ * D1 + NQ + i];
  }
  return t;
}

// Instantiate every operation, precision and geometry for one (D1, NQ) and
// register the launchers in the dispatch table.
#define FEOD_INSTANTIATE(DD, QQ)                                                                \
  template <class T, int OP, bool CURVED>                                                       \
  static hipError_t launch_##DD##_##QQ(const ElemParams& P, hipStream_t s) {                    \
    constexpr int EB = Config<DD, QQ, T>::EB;                                                   \
    constexpr int NT = Config<DD, QQ, T>::NT;                                                   \
    const int blocks = (P.E + EB - 1) / EB;                                                     \
    if (blocks == 0) return hipSuccess;                                                         \
    const Tab<DD, QQ, T> tb = make_tab<DD, QQ, T>(P.htab);                                      \
    hipLaunchKernelGGL((element_kernel<DD, QQ, T, OP, CURVED>), dim3(blocks), dim3(NT), 0, s, P, \
                       tb);                                                                     \
    return hipGetLastError();                                                                   \
  }                                                                                             \
  template <class T, bool CURVED>                                                               \
  static void fill_##DD##_##QQ(ElemLaunchers::PerPrec& t) {                                     \
    t.op[OP_RESIDUAL][CURVED] = &launch_##DD##_##QQ<T, OP_RESIDUAL, CURVED>;                    \
    t.op[OP_JVP][CURVED] = &launch_##DD##_##QQ<T, OP_JVP, CURVED>;                              \
    t.op[OP_RESJVP][CURVED] = &launch_##DD##_##QQ<T, OP_RESJVP, CURVED>;                        \
    t.op[OP_ENERGY][CURVED] = &launch_##DD##_##QQ<T, OP_ENERGY, CURVED>;                        \
    t.op[OP_GRAD][CURVED] = &launch_##DD##_##QQ<T, OP_GRAD, CURVED>;                            \
  }                                                                                             \
  ElemLaunchers make_launchers_##DD##_##QQ() {                                                  \
    ElemLaunchers L{};                                                                          \
    L.D1 = DD;                                                                                  \
    L.NQ = QQ;                                                                                  \
    fill_##DD##_##QQ<double, false>(L.prec[0]);                                                 \
    fill_##DD##_##QQ<double, true>(L.prec[0]);                                                  \
    fill_##DD##_##QQ<float, false>(L.prec[1]);                                                  \
    fill_##DD##_##QQ<float, true>(L.prec[1]);                                                   \
    L.eb[0] = Config<DD, QQ, double>::EB;                                                       \
    L.eb[1] = Config<DD, QQ, float>::EB;                                                        \
    return L;                                                                                   \
  }

}  // namespace feod
