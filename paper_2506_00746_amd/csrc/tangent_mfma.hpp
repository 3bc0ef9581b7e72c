// Element tangent matrices K_e = B^T J_D B (paper, Eq. 3) for Q2 elements on
// the FP64 matrix cores.  With three nodes per direction the contraction is
// small and dense:
//
//   K_e = G^T W_e,   W_e[(q,d)][j] = sum_d' Chat_dd'(q) G[(q,d')][j],
//
// where G[(q,d)][j] is the reference derivative of basis function j in
// direction d at quadrature point q (the same table for every element) and
// Chat(q) = rho w det Jg^{-1} J_D Jg^{-T} with J_D from three forward-mode
// dual evaluations of the flux, exactly as in the sum-factorised kernel.
// K_e (27 x 27) is 16 x 16 output tiles (rows and columns padded to 32)
// accumulated over 3 NQ^3 in steps of 4 by v_mfma_f64_16x16x4f64; K_e is
// symmetric (J_D is the Hessian of the energy density), so the lower-left
// tile is written as the transpose of the upper-right one; the
// B operand W is formed in registers for each step from Chat and G in LDS.
// G is built once per workgroup, whose wavefronts then loop over elements.
//
// Operand layout of the 16x16x4 FP64 instruction (checked on the device):
// lane l supplies A[l%16][l/16] and B[l/16][l%16], and its four results are
// D[4r + l/16][l%16], r = 0..3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "element_kernel.hpp"

namespace feod {

typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTangentMfmaBlocks = 2048;  // workgroups; each wave then loops over elements

template <int NQ>
struct TangentMfmaShape {
  static constexpr int WAVES = NQ <= 3 ? 4 : 2;  // elements per workgroup (LDS bound)
};

template <int NQ, bool CURVED, int PK>
__global__ __launch_bounds__(64 * TangentMfmaShape<NQ>::WAVES) void tangent_mfma_kernel(ElemParams P,
                                                                                      Tab<3, NQ, double> tb) {
  constexpr int D1 = 3, Ne = 27, NQ3 = NQ * NQ * NQ, KD = 3 * NQ3, KS = (KD + 3) / 4;
  constexpr int WAVES = TangentMfmaShape<NQ>::WAVES, NT = 64 * WAVES;
  constexpr int GS = Ne + 1;  // padded row stride of G
  __shared__ double sG[KD * GS];          // G[(q,d)][j]
  __shared__ double sC[WAVES][NQ3 * 9];   // Chat(q), row-major 3x3, per wave's element
  __shared__ double sU[WAVES][Ne];        // M u_e
  __shared__ double sg[WAVES][KD];        // reference gradient of u at the points
  __shared__ double sX[WAVES][24];        // vertices (curved meshes)
  __shared__ double sB[NQ * D1], sD[NQ * D1], sW[NQ], sQ[NQ];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  for (int i = tid; i < NQ * D1; i += NT) {
    sB[i] = tb.B[i];
    sD[i] = tb.Dx[i];  // reference table (built without 1/h)
  }
  for (int i = tid; i < NQ; i += NT) {
    sW[i] = tb.w[i];
    sQ[i] = tb.xi[i];
  }
  __syncthreads();
  // G[(q,d)][j] = psi_d(q, j): a product of three 1D factors
  for (int i = tid; i < KD * Ne; i += NT) {
    const int kd = i / Ne, j = i - kd * Ne;
    const int q = kd / 3, d = kd - 3 * q;
    const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
    const int a = j % D1, b = (j / D1) % D1, c = j / (D1 * D1);
    const double fx = d == 0 ? sD[qx * D1 + a] : sB[qx * D1 + a];
    const double fy = d == 1 ? sD[qy * D1 + b] : sB[qy * D1 + b];
    const double fz = d == 2 ? sD[qz * D1 + c] : sB[qz * D1 + c];
    sG[kd * GS + j] = fx * fy * fz;
  }

  // Each wave takes elements blockIdx * WAVES + wv + it * gridDim * WAVES;
  // every wave runs the same number of iterations (the last valid element
  // stands in past the end, without writing), so the barriers match.
  const int last = P.e_first + P.E - 1;
  const int stride = (int)gridDim.x * WAVES;
  const int iters = (P.E + stride - 1) / stride;
  for (int it = 0; it < iters; ++it) {
    __syncthreads();  // the previous element's LDS data is consumed
    const int e_raw = P.e_first + (int)blockIdx.x * WAVES + wv + it * stride;
    const bool valid = e_raw <= last;
    const uint32_t e = (uint32_t)(valid ? e_raw : last);
    const uint32_t et = fastdiv(e, P.div_nx), ezu = fastdiv(et, P.div_ny);
    const int ex = (int)(e - et * (uint32_t)P.nx), ey = (int)(et - ezu * (uint32_t)P.ny), ez = (int)ezu;
    if (lane < Ne) {
      const int a = lane % D1, b = (lane / D1) % D1, c = lane / (D1 * D1);
      const int I = P.k * ex + a, J = P.k * ey + b, K = P.k * ez + c;
      const bool in = I > 0 && I < P.Lx - 1 && J > 0 && J < P.Ly - 1 && K > 0 && K < P.Lz - 1;
      sU[wv][lane] = in ? P.u[I + (int64_t)P.Lx * (J + (int64_t)P.Ly * K)] : 0.0;
    }
    if (CURVED && lane < 24) {
      const int vtx = lane / 3, al = lane - vtx * 3;
      const int gi = (ex + (vtx & 1)) + (P.nx + 1) * ((ey + ((vtx >> 1) & 1)) + (P.ny + 1) * (ez + (vtx >> 2)));
      sX[wv][lane] = P.verts[(int64_t)gi * 3 + al];
    }
    __syncthreads();

    // reference gradient of u at every point
    for (int kd = lane; kd < KD; kd += 64) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < Ne; ++j) s += sG[kd * GS + j] * sU[wv][j];
      sg[wv][kd] = s;
    }
    __syncthreads();

    // Chat at every point: J_D by three forward-mode evaluations of the flux
    const double rho = (P.rho != nullptr) ? P.rho[e] : 1.0;
    for (int q = lane; q < NQ3; q += 64) {
      const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
      const double w3 = sW[qx] * sW[qy] * sW[qz];
      double adj[3][3], det, gu[3];
      if (CURVED) {
        const double xi = sQ[qx], et_ = sQ[qy], ze = sQ[qz];
        const double mx = 1.0 - xi, me = 1.0 - et_, mz = 1.0 - ze;
        double Jm[3][3];
        for (int al = 0; al < 3; ++al) {
          const double* x = sX[wv] + al;
          Jm[al][0] = (me * mz) * (x[3] - x[0]) + (et_ * mz) * (x[9] - x[6]) + (me * ze) * (x[15] - x[12]) +
                      (et_ * ze) * (x[21] - x[18]);
          Jm[al][1] = (mx * mz) * (x[6] - x[0]) + (xi * mz) * (x[9] - x[3]) + (mx * ze) * (x[18] - x[12]) +
                      (xi * ze) * (x[21] - x[15]);
          Jm[al][2] = (mx * me) * (x[12] - x[0]) + (xi * me) * (x[15] - x[3]) + (mx * et_) * (x[18] - x[6]) +
                      (xi * et_) * (x[21] - x[9]);
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
        for (int a = 0; a < 3; ++a)
          gu[a] = (adj[0][a] * sg[wv][3 * q] + adj[1][a] * sg[wv][3 * q + 1] + adj[2][a] * sg[wv][3 * q + 2]) / det;
      } else {
        det = P.det;
        for (int a = 0; a < 3; ++a) gu[a] = sg[wv][3 * q + a] * P.hinv[a];
      }
      double Tm[3][3];
      for (int d = 0; d < 3; ++d) {
        dual<double> gd[3], Fd[3];
        for (int a = 0; a < 3; ++a) gd[a] = {gu[a], a == d ? 1.0 : 0.0};
        flux<PK, dual<double>, double>(gd, P.eps2, P.r, Fd);
        for (int a = 0; a < 3; ++a) Tm[a][d] = Fd[a].d;
      }
      const double s = rho * w3;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double cij;
          if (CURVED) {
            double acc = 0;
            for (int m = 0; m < 3; ++m)
              for (int n = 0; n < 3; ++n) acc += adj[i][m] * Tm[m][n] * adj[j][n];
            cij = s * acc / det;
          } else {
            cij = s * det * P.hinv[i] * P.hinv[j] * Tm[i][j];
          }
          sC[wv][q * 9 + i * 3 + j] = cij;
        }
    }
    __syncthreads();

    // K_e = G^T W on the matrix cores: tiles (it, jt) of rows 16 it .. and
    // columns 16 jt .., k = (q, d) in steps of 4
    const int li = lane & 15, lk = lane >> 4;
    mfma_f64x4 acc00 = {0, 0, 0, 0}, acc01 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
    const bool c1 = 16 + li < Ne;  // second row / column tile holds 11 real entries
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk;
      double a0 = 0, a1 = 0, b0 = 0, b1 = 0;
      if (k < KD) {
        const int q = k / 3, d = k - 3 * q;
        const double* g = sG + 3 * q * GS;  // rows (q, 0..2)
        const double* C = sC[wv] + q * 9 + 3 * d;
        a0 = sG[k * GS + li];
        b0 = C[0] * g[li] + C[1] * g[GS + li] + C[2] * g[2 * GS + li];
        if (c1) {
          a1 = sG[k * GS + 16 + li];
          b1 = C[0] * g[16 + li] + C[1] * g[GS + 16 + li] + C[2] * g[2 * GS + 16 + li];
        }
      }
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
    }

    // K_e row-major, local node order a + 3 (b + 3 c)
    if (valid) {
      double* Ke = static_cast<double*>(P.out0) + (int64_t)(e_raw - P.e_first) * Ne * Ne;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i0 = 4 * r + lk, i1 = 16 + i0;
        Ke[i0 * Ne + li] = acc00[r];
        if (c1) Ke[i0 * Ne + 16 + li] = acc01[r];
        if (c1) Ke[(16 + li) * Ne + i0] = acc01[r];  // lower-left tile: K is symmetric
        if (i1 < Ne && c1) Ke[i1 * Ne + 16 + li] = acc11[r];
      }
    }
  }  // elements of this wave
}

#define FEOD_INSTANTIATE_TANGENT_MFMA(QQ)                                                            \
  template <bool CURVED, int PK>                                                                     \
  static hipError_t tangent_mfma_##QQ(const ElemParams& P, hipStream_t s) {                          \
    if (P.E == 0) return hipSuccess;                                                                 \
    constexpr int W = TangentMfmaShape<QQ>::WAVES;                                                   \
    const Tab<3, QQ, double> tb = make_tab<3, QQ, double>(P.htab);                                   \
    const int blocks = std::min((P.E + W - 1) / W, kTangentMfmaBlocks);                             \
    hipLaunchKernelGGL((tangent_mfma_kernel<QQ, CURVED, PK>), dim3(blocks), dim3(64 * W), 0, s, P, tb); \
    return hipGetLastError();                                                                        \
  }                                                                                                  \
  template <bool CURVED>                                                                             \
  static void fill_tangent_mfma_##QQ(ElemLaunch (&t)[2][5]) {                                        \
    t[CURVED][POW_ZERO] = &tangent_mfma_##QQ<CURVED, POW_ZERO>;                                      \
    t[CURVED][POW_QUARTER] = &tangent_mfma_##QQ<CURVED, POW_QUARTER>;                                \
    t[CURVED][POW_HALF] = &tangent_mfma_##QQ<CURVED, POW_HALF>;                                      \
    t[CURVED][POW_ONE] = &tangent_mfma_##QQ<CURVED, POW_ONE>;                                        \
    t[CURVED][POW_GENERIC] = &tangent_mfma_##QQ<CURVED, POW_GENERIC>;                                \
  }                                                                                                  \
  void fill_tangents_3_##QQ(ElemLaunchers& L) {                                                      \
    fill_tangent_mfma_##QQ<false>(L.tangent);                                                        \
    fill_tangent_mfma_##QQ<true>(L.tangent);                                                         \
  }

}  // namespace feod
