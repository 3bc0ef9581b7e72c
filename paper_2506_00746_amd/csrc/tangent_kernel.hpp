// Element tangent matrices K_e = d r_e / d u_e = B^T J_D(u_q) B (paper, Eq. 3),
// with J_D obtained at each quadrature point by forward-mode dual numbers
// (three directional evaluations of the flux) -- the quadrature-point ("RES")
// placement of AD the paper argues for, as opposed to differentiating through
// B at element level.
//
// One workgroup per element.  With Chat_q = rho w det Jg^{-1} J_D Jg^{-T}
// (3x3 per point) and psi_d the reference derivative of a basis function in
// direction d, K[i][j] = sum_q sum_{d,d'} psi_d(q,i) Chat_dd'(q) psi_d'(q,j).
// Each psi is a product of 1D factors, so every (d,d') term is contracted by
// sum factorisation in three stages (x, then y, then z) through LDS:
// O(nq^3 D1^2 + nq^2 D1^4) per term for the x and y stages, and the z stage
// O(nq D1^6) once per z-factor pair (four, not nine), instead of the dense
// O(nq^3 D1^6).  Supported for D1 <= 5 (the y-stage buffer nq D1^4 must fit).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "element_kernel.hpp"

namespace feod {

// One (d, d') tensor term: x stage (through LDS) into T1, then the y stage
// added into T2.  In the y stage a thread owns one (qz, a, a') and all
// (b, b') outputs: each T1 value is read once and the 1D factors are the
// same LDS word for every lane.
template <int D1, int NQ, int NT, int d, int d2, class T>
__device__ __forceinline__ void tangent_term(const T* sB, const T* sD, const T* Cdd, T* sT1, T* sT2, int tid) {
  constexpr int D2 = D1 * D1, D4 = D2 * D2;
  const T* Fx0 = d == 0 ? sD : sB;   // factor of psi_d in x
  const T* Fx1 = d2 == 0 ? sD : sB;  // factor of psi_d' in x
  // 1D factors in y: the same LDS word for every lane (broadcast reads)
  const T* Fy0 = d == 1 ? sD : sB;
  const T* Fy1 = d2 == 1 ? sD : sB;
  // x: T1[qz][qy][a][a'] = sum_qx Fx0[qx][a] Fx1[qx][a'] C(qx,qy,qz); a thread
  // owns (qy, qz, a) and all a', reading each C value once
  for (int t = tid; t < NQ * NQ * D1; t += NT) {
    const int qyz = t / D1, a = t - qyz * D1;
    T u[NQ];
#pragma unroll
    for (int qx = 0; qx < NQ; ++qx) u[qx] = Fx0[qx * D1 + a] * Cdd[qx + NQ * qyz];
#pragma unroll
    for (int a2 = 0; a2 < D1; ++a2) {
      T sacc = Fx1[a2] * u[0];
#pragma unroll
      for (int qx = 1; qx < NQ; ++qx) sacc += Fx1[qx * D1 + a2] * u[qx];
      sT1[qyz * D2 + a * D1 + a2] = sacc;
    }
  }
  __syncthreads();
  // y: T2[qz][b][b'][a][a'] += sum_qy Fy0[qy][b] Fy1[qy][b'] T1[qz][qy][a][a']
  for (int t = tid; t < NQ * D2; t += NT) {
    const int qz = t / D2, aa = t - qz * D2;
    T t1[NQ];
#pragma unroll
    for (int qy = 0; qy < NQ; ++qy) t1[qy] = sT1[(qz * NQ + qy) * D2 + aa];
#pragma unroll
    for (int b = 0; b < D1; ++b) {
      T u[NQ];
#pragma unroll
      for (int qy = 0; qy < NQ; ++qy) u[qy] = Fy0[qy * D1 + b] * t1[qy];
#pragma unroll
      for (int b2 = 0; b2 < D1; ++b2) {
        T sacc = Fy1[b2] * u[0];
#pragma unroll
        for (int qy = 1; qy < NQ; ++qy) sacc += Fy1[qy * D1 + b2] * u[qy];
        sT2[qz * D4 + (b * D1 + b2) * D2 + aa] += sacc;
      }
    }
  }
  __syncthreads();
}

// z stage of one z-factor group: K[c][c'][ab] += sum_qz Fz0[qz][c] Fz1[qz][c'] T2[qz][ab],
// a thread owning ab and all (c, c'): each T2 value is read once.
template <int D1, int NQ, int NT, bool zd0, bool zd1, class T>
__device__ __forceinline__ void tangent_zstage(const T* sB, const T* sD, const T* sT2, int tid,
                                               T (&acc)[(D1 * D1 * D1 * D1 + NT - 1) / NT][D1 * D1]) {
  constexpr int D4 = D1 * D1 * D1 * D1, SL = (D4 + NT - 1) / NT;
  const T* Fz0 = zd0 ? sD : sB;  // the same LDS word for every lane (broadcast)
  const T* Fz1 = zd1 ? sD : sB;
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int ab = tid + sl * NT;
    if (ab < D4) {
#pragma unroll
      for (int qz = 0; qz < NQ; ++qz) {
        const T t2 = sT2[qz * D4 + ab];
#pragma unroll
        for (int c = 0; c < D1; ++c) {
          const T u = Fz0[qz * D1 + c] * t2;
#pragma unroll
          for (int c2 = 0; c2 < D1; ++c2) acc[sl][c * D1 + c2] += Fz1[qz * D1 + c2] * u;
        }
      }
    }
  }
}

template <int D1, int NQ, class T, bool CURVED, int PK>
__global__ __launch_bounds__(256) void tangent_kernel(ElemParams P, Tab<D1, NQ, T> tb) {
  constexpr int NT = 256;
  constexpr int Ne = D1 * D1 * D1, NQ3 = NQ * NQ * NQ, NE2 = Ne * Ne;
  constexpr int D2 = D1 * D1, D4 = D2 * D2;
  __shared__ T sU[Ne];
  __shared__ T sG[3][NQ3];
  __shared__ T sC[9][NQ3];
  __shared__ T sT1[NQ * NQ * D2];  // [qz][qy][a][a']
  __shared__ T sT2[NQ * D4];       // [qz][b][b'][a][a']
  __shared__ T sX[24];
  __shared__ T sB[NQ * D1], sD[NQ * D1], sW[NQ], sQ[NQ];
  const int tid = threadIdx.x;
  for (int i = tid; i < NQ * D1; i += NT) {
    sB[i] = tb.B[i];
    sD[i] = tb.Dx[i];  // reference table (built without 1/h)
  }
  for (int i = tid; i < NQ; i += NT) {
    sW[i] = tb.w[i];
    sQ[i] = tb.xi[i];
  }
  const int e = P.e_first + blockIdx.x;
  const uint32_t et = fastdiv((uint32_t)e, P.div_nx), ez_ = fastdiv(et, P.div_ny);
  const int ex = (int)((uint32_t)e - et * (uint32_t)P.nx), ey = (int)(et - ez_ * (uint32_t)P.ny), ez = (int)ez_;

  // gather M u_e (lattice map; Dirichlet nodes read as 0) and the vertices
  for (int i = tid; i < Ne; i += NT) {
    const int a = i % D1, b = (i / D1) % D1, c = i / D2;
    const int I = P.k * ex + a, J = P.k * ey + b, K = P.k * ez + c;
    const bool in = I > 0 && I < P.Lx - 1 && J > 0 && J < P.Ly - 1 && K > 0 && K < P.Lz - 1;
    sU[i] = in ? (T)P.u[I + (int64_t)P.Lx * (J + (int64_t)P.Ly * K)] : T(0);
  }
  if (CURVED && tid < 24) {
    const int vtx = tid / 3, al = tid - vtx * 3;
    const int gi = (ex + (vtx & 1)) + (P.nx + 1) * ((ey + ((vtx >> 1) & 1)) + (P.ny + 1) * (ez + (vtx >> 2)));
    sX[tid] = (T)P.verts[(int64_t)gi * 3 + al];
  }
  __syncthreads();

  // reference gradients at every point (dense per point; small next to K)
  for (int q = tid; q < NQ3; q += NT) {
    const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
    T g0 = 0, g1 = 0, g2 = 0;
    for (int c = 0; c < D1; ++c)
      for (int b = 0; b < D1; ++b)
        for (int a = 0; a < D1; ++a) {
          const T u = sU[a + D1 * (b + D1 * c)];
          g0 += sD[qx * D1 + a] * sB[qy * D1 + b] * sB[qz * D1 + c] * u;
          g1 += sB[qx * D1 + a] * sD[qy * D1 + b] * sB[qz * D1 + c] * u;
          g2 += sB[qx * D1 + a] * sB[qy * D1 + b] * sD[qz * D1 + c] * u;
        }
    sG[0][q] = g0;
    sG[1][q] = g1;
    sG[2][q] = g2;
  }
  __syncthreads();

  // Chat at every point: J_D by three forward-mode evaluations of the flux
  const T rho = P.rho != nullptr ? (T)P.rho[e] : T(1);
  for (int q = tid; q < NQ3; q += NT) {
    const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
    const T w3 = sW[qx] * sW[qy] * sW[qz];
    T adj[3][3], det, gu[3];
    if (CURVED) {
      const T xi = sQ[qx], et = sQ[qy], ze = sQ[qz];
      const T mx = T(1) - xi, me = T(1) - et, mz = T(1) - ze;
      T Jm[3][3];
      for (int al = 0; al < 3; ++al) {
        const T* x = sX + al;
        Jm[al][0] = (me * mz) * (x[3] - x[0]) + (et * mz) * (x[9] - x[6]) + (me * ze) * (x[15] - x[12]) + (et * ze) * (x[21] - x[18]);
        Jm[al][1] = (mx * mz) * (x[6] - x[0]) + (xi * mz) * (x[9] - x[3]) + (mx * ze) * (x[18] - x[12]) + (xi * ze) * (x[21] - x[15]);
        Jm[al][2] = (mx * me) * (x[12] - x[0]) + (xi * me) * (x[15] - x[3]) + (mx * et) * (x[18] - x[6]) + (xi * et) * (x[21] - x[9]);
      }
      adj[0][0] = Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1];
      adj[0][1] = Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2];
      adj[0][2] = Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1];
      adj[1][0] = Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2];
      adj[1][1] = Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0];
      adj[1][2] = Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2];
      adj[2][0] = Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0];
      adj[2][1] = Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1];
      adj[2][2] = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
      det = Jm[0][0] * adj[0][0] + Jm[0][1] * adj[1][0] + Jm[0][2] * adj[2][0];
      for (int a = 0; a < 3; ++a) gu[a] = (adj[0][a] * sG[0][q] + adj[1][a] * sG[1][q] + adj[2][a] * sG[2][q]) / det;
    } else {
      det = (T)P.det;
      for (int a = 0; a < 3; ++a) gu[a] = sG[a][q] * (T)P.hinv[a];
    }
    T Tm[3][3];
    for (int d = 0; d < 3; ++d) {
      dual<T> gd[3], Fd[3];
      for (int a = 0; a < 3; ++a) gd[a] = {gu[a], a == d ? T(1) : T(0)};
      flux<PK, dual<T>, T>(gd, (T)P.eps2, (T)P.r, Fd);
      for (int a = 0; a < 3; ++a) Tm[a][d] = Fd[a].d;
    }
    const T s = rho * w3;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T cij;
        if (CURVED) {
          T acc = 0;
          for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) acc += adj[i][m] * Tm[m][n] * adj[j][n];
          cij = s * acc / det;
        } else {
          cij = s * det * (T)P.hinv[i] * (T)P.hinv[j] * Tm[i][j];
        }
        sC[i * 3 + j][q] = cij;
      }
  }
  __syncthreads();

  constexpr int SL = (D4 + NT - 1) / NT;
  T acc[SL][D2];
#pragma unroll
  for (int sl = 0; sl < SL; ++sl)
#pragma unroll
    for (int cc = 0; cc < D2; ++cc) acc[sl][cc] = 0;
  // The z factor of psi_d is D for d = 2 and B otherwise, so the nine (d,d')
  // terms fall into four groups by their z-factor pair; the z stage is linear,
  // so each group's y-stage outputs are summed first and contracted in z once.
  auto clear_t2 = [&] {
    for (int i = tid; i < NQ * D4; i += NT) sT2[i] = 0;
  };
  clear_t2();  // the first x stage's barrier orders this before the y stage
  tangent_term<D1, NQ, NT, 0, 0>(sB, sD, sC[0], sT1, sT2, tid);
  tangent_term<D1, NQ, NT, 0, 1>(sB, sD, sC[1], sT1, sT2, tid);
  tangent_term<D1, NQ, NT, 1, 0>(sB, sD, sC[3], sT1, sT2, tid);
  tangent_term<D1, NQ, NT, 1, 1>(sB, sD, sC[4], sT1, sT2, tid);
  tangent_zstage<D1, NQ, NT, false, false>(sB, sD, sT2, tid, acc);
  __syncthreads();
  clear_t2();
  tangent_term<D1, NQ, NT, 2, 0>(sB, sD, sC[6], sT1, sT2, tid);
  tangent_term<D1, NQ, NT, 2, 1>(sB, sD, sC[7], sT1, sT2, tid);
  tangent_zstage<D1, NQ, NT, true, false>(sB, sD, sT2, tid, acc);
  __syncthreads();
  clear_t2();
  tangent_term<D1, NQ, NT, 0, 2>(sB, sD, sC[2], sT1, sT2, tid);
  tangent_term<D1, NQ, NT, 1, 2>(sB, sD, sC[5], sT1, sT2, tid);
  tangent_zstage<D1, NQ, NT, false, true>(sB, sD, sT2, tid, acc);
  __syncthreads();
  clear_t2();
  tangent_term<D1, NQ, NT, 2, 2>(sB, sD, sC[8], sT1, sT2, tid);
  tangent_zstage<D1, NQ, NT, true, true>(sB, sD, sT2, tid, acc);
  // K_e row i = a + D1 (b + D1 c), column j = a' + D1 (b' + D1 c'), row-major;
  // ab = (b D1 + b') D2 + (a D1 + a'), cc = c D1 + c'
  T* Ke = static_cast<T*>(P.out0) + (int64_t)blockIdx.x * NE2;
#pragma unroll
  for (int sl = 0; sl < SL; ++sl) {
    const int ab = tid + sl * NT;
    if (ab < D4) {
      const int aa = ab % D2, bb = ab / D2, a = aa / D1, a2 = aa % D1, b = bb / D1, b2 = bb % D1;
#pragma unroll
      for (int cc = 0; cc < D2; ++cc) {
        const int c = cc / D1, c2 = cc % D1;
        Ke[(a + D1 * (b + D1 * c)) * Ne + (a2 + D1 * (b2 + D1 * c2))] = acc[sl][cc];
      }
    }
  }
}

#define FEOD_INSTANTIATE_TANGENT(DD, QQ)                                                            \
  template <bool CURVED, int PK>                                                                    \
  static hipError_t tangent_##DD##_##QQ(const ElemParams& P, hipStream_t s) {                       \
    if (P.E == 0) return hipSuccess;                                                                \
    const Tab<DD, QQ, double> tb = make_tab<DD, QQ, double>(P.htab);                                \
    hipLaunchKernelGGL((tangent_kernel<DD, QQ, double, CURVED, PK>), dim3(P.E), dim3(256), 0, s, P, tb); \
    return hipGetLastError();                                                                       \
  }                                                                                                 \
  template <bool CURVED>                                                                            \
  static void fill_tangent_##DD##_##QQ(ElemLaunch (&t)[2][5]) {                                     \
    t[CURVED][POW_ZERO] = &tangent_##DD##_##QQ<CURVED, POW_ZERO>;                                   \
    t[CURVED][POW_QUARTER] = &tangent_##DD##_##QQ<CURVED, POW_QUARTER>;                             \
    t[CURVED][POW_HALF] = &tangent_##DD##_##QQ<CURVED, POW_HALF>;                                   \
    t[CURVED][POW_ONE] = &tangent_##DD##_##QQ<CURVED, POW_ONE>;                                     \
    t[CURVED][POW_GENERIC] = &tangent_##DD##_##QQ<CURVED, POW_GENERIC>;                             \
  }                                                                                                 \
  void fill_tangents_##DD##_##QQ(ElemLaunchers& L) {                                                \
    fill_tangent_##DD##_##QQ<false>(L.tangent);                                                     \
    fill_tangent_##DD##_##QQ<true>(L.tangent);                                                      \
  }

}  // namespace feod
