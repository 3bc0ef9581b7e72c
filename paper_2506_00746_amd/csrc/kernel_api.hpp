// Host-visible launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace feod {

// Exponent r = (p-2)/2 of the flux coefficient a^r, specialised by sqrt chains.
enum PowKind : int { POW_ZERO = 0, POW_QUARTER = 1, POW_HALF = 2, POW_ONE = 3, POW_GENERIC = 4 };

enum : int {
  OP_RESIDUAL = 0,  // E-vector of the residual
  OP_JVP = 1,       // E-vector of the Jacobian action
  OP_RESJVP = 2,    // both
  OP_ENERGY = 3,    // per-element energy
  OP_GRAD = 4,      // per-element dR/drho weighted by lambda
  OP_DIAG = 5,      // E-vector of diag(J)
  OP_QSTORE = 6,    // partial assembly: reference gradients of M u at every point -> qdata
  OP_JVP_PA = 7,    // Jacobian action with the stored gradients (v gathered only)
  OP_ELM = 8,       // element tangent column by element-level forward AD (FP64, D1 <= 5)
  OP_JVP_HND = 9,   // Jacobian action with the hand-coded J_D instead of dual numbers (FP64)
  OP_COUNT = 10
};

// Arguments of the fused element kernel (passed by value).
// Exact division by a runtime divisor d (1 <= d <= 2^31) of numerators
// n < 2^31 with one 32x32->64-bit multiply and a shift (the round-up
// multiplier method of Granlund and Montgomery, 1994): with l = ceil(log2 d),
// m = ceil(2^(31+l) / d) < 2^32 and s = 31 + l, floor(n/d) = (n m) >> s,
// since n m / 2^s = n/d + delta with 0 <= delta < 2^-l <= 1/d.
struct FastDiv {
  uint32_t m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  const uint64_t p = uint64_t(1) << (31 + l);
  return {(uint32_t)((p + d - 1) / d), 31 + l};
}
__host__ __device__ __forceinline__ uint32_t fastdiv(uint32_t n, FastDiv f) {
  return (uint32_t)(((uint64_t)n * f.m) >> f.s);
}

struct ElemParams {
  const double* u;        // L-vector (FP64)
  const double* v;        // second L-vector: JVP direction or adjoint lambda
  const int32_t* emap;    // E x Ne element-to-DOF map, -1 on Dirichlet DOFs; nullptr:
                          // computed from the lattice (same map, no memory traffic)
  const double* rho;      // E coefficients or nullptr (all ones)
  const double* verts;    // (nx+1)(ny+1)(nz+1) x 3, curved meshes only
  const void* tab;        // 1D tables in the kernel precision: B, D (nq x D1), w, xi (nq)
  void* out0;             // E-vector (kernel precision) or E doubles (energy, gradient)
  void* out1;             // second E-vector (residual + JVP)
  void* qdata;            // partial assembly: [e][d][qz][qy][qx] gradients of u (kernel precision;
                          // physical on affine meshes, reference on curved ones)
  const double* htab;     // host copy of the FP64 tables (B, D, w, xi); read by the launcher
  int32_t E, nx, ny, nz;
  int32_t e_first;        // first element (element-tangent kernels; E is then the count)
  int32_t k, Lx, Ly, Lz;  // order and node-lattice extents (k n + 1 per direction)
  double hinv[3];         // affine meshes: 1/h per direction
  double det;             // affine meshes: element volume h_x h_y h_z
  double p, eps2, r, inv_p;
  int32_t powkind;
  FastDiv div_nx, div_ny;  // element index -> (ex, ey, ez)
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that XCD j processes one contiguous range of the
// logical batches: neighbouring elements (and DOFs) then share an L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_remap(int w, int n) {
  const int q = n / kNumXcd, r = n % kNumXcd;
  const int j = w % kNumXcd, i = w / kNumXcd;
  return j * q + (j < r ? j : r) + i;
}

using ElemLaunch = hipError_t (*)(const ElemParams&, hipStream_t);

struct ElemLaunchers {
  int D1, NQ;
  struct PerPrec {
    ElemLaunch op[OP_COUNT][2][5];  // [op][curved][PowKind]
  } prec[2];                     // [0] FP64, [1] FP32
  ElemLaunch tangent[2][5];      // element tangent matrices, FP64: [curved][PowKind] (D1 <= 5)
  int eb[2];
};

// Registered (D1, NQ) instantiations; returns nullptr when not built.
const ElemLaunchers* find_launchers(int D1, int NQ);

// ---- L-vector kernels (vector_kernels.hip) ----------------------------------
constexpr int kRedBlocks = 1024;  // fixed grid of the two-stage reductions

// y[i] = sum_{j in row i} Y[idx[j]] - bm[i] (bm may be nullptr); optional
// second E-vector / output pair for residual + JVP.  TE = double or float.
hipError_t launch_gather_t(const int32_t* off, const int32_t* idx, const void* Y0, const void* Y1,
                           bool fp32, const double* bm, double* out0, double* out1, int64_t n,
                           hipStream_t s);

// Structured lattice of the element-to-DOF map, for the computed G^T.
struct LatticeDims {
  int32_t nx, ny, nz, k, Lx, Ly, Lz;
  FastDiv div_Lx, div_Ly, div_k;  // DOF index -> (I, J, K) -> element index
  // E-vector entries per element, (k+1)^3, and how far the lower candidate
  // element's entry of a DOF sits before the upper one's, per direction:
  // Ne - k, nx Ne - k (k+1), nx ny Ne - k (k+1)^2
  uint32_t ne, dlx, dly, dlz;
};
LatticeDims make_lattice_dims(int32_t nx, int32_t ny, int32_t nz, int32_t k);
// Same sums as launch_gather_t, in the same (ascending E-vector position)
// order, with each DOF's element list computed from the lattice.
hipError_t launch_gather_t_lattice(const LatticeDims& d, const void* Y0, const void* Y1, bool fp32,
                                   const double* bm, double* out0, double* out1, int64_t n,
                                   hipStream_t s);

// partial[b] = sum over block b's grid-stride share of x[i]*y[i] (y == nullptr: x[i]).
hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* partial,
                              hipStream_t s);
// out[0] = sum_b partial[b] * sign + (add ? add[0] : 0), fixed order, one block.
hipError_t launch_reduce_final(const double* partial, int nparts, double* out, double sign,
                               const double* add, hipStream_t s);

// ---- Fused CG iteration: kCgBlocks blocks, one partial sum per block -----
constexpr int kCgBlocks = 512;   // partial sums per CG inner product (two blocks per CU)
constexpr int kCgThreads = 512;  // threads per CG vector block
constexpr int kCgUnroll = 4;     // DOFs per thread per grid-stride pass
// q = G^T Y (the lattice map, or with csr the CSR map off/idx) and
// partial[b] = block b's share of p.q, for gather_dot_blocks(n) blocks of
// kGatherDotThreads (one DOF per thread up to kGatherDotMaxBlocks blocks);
// both maps take the DOFs in the same order, so their partials are bitwise
// equal.
constexpr int kGatherDotThreads = 1024;
constexpr int kGatherDotMaxBlocks = 4096;
inline int gather_dot_blocks(int64_t n) {
  const int64_t b = (n + kGatherDotThreads - 1) / kGatherDotThreads;
  return (int)(b < 1 ? 1 : (b > kGatherDotMaxBlocks ? kGatherDotMaxBlocks : b));
}
hipError_t launch_gather_t_dot(const LatticeDims& dims, bool csr, const int32_t* off, const int32_t* idx,
                               const void* Y, bool fp32, const double* p, double* q, int64_t n, double* partial,
                               hipStream_t s);
// x = 0, r = b, z = dinv r (z may alias r when dinv is null), p = z, partials of r.z and r.r
hipError_t launch_cg_init(double* x, double* r, double* z, double* p, const double* b, const double* dinv,
                          int64_t n, double* part_rz, double* part_rr, hipStream_t s);
// Reliable update: r = b - jx (the true residual of the current x), z = dinv r,
// partials of r.z and r.r; x and p are left as they are.
hipError_t launch_cg_true_residual(double* r, double* z, const double* b, const double* jx, const double* dinv,
                                   int64_t n, double* part_rz, double* part_rr, hipStream_t s);
// alpha = sum(part_rz)/sum(part_pq) (n_pq partials of p.q from the gather);
// r -= alpha q; z = dinv r; new partials of r.z (part_rz_new) and r.r
// (part_rr, when dinv); block 0 stores the two totals in sc[i_rz], sc[i_pq].
// x is left to launch_cg_direction or launch_cg_x_update.
hipError_t launch_cg_step(double* r, double* z, const double* q, const double* dinv, const double* part_rz,
                          const double* part_pq, int n_pq, int64_t n, double* part_rz_new, double* part_rr,
                          double* sc, int i_rz, int i_pq, hipStream_t s);
// beta = sum(part_new)/sum(part_old); x (unless null) += alpha p with the
// step's alpha = sum(part_old)/sum(part_pq); then p = z + beta p
hipError_t launch_cg_direction(double* p, const double* z, double* x, const double* part_new,
                               const double* part_old, const double* part_pq, int n_pq, int64_t n, hipStream_t s);
// x += alpha p, alpha = sum(part_rz)/sum(part_pq): the last step's update of x
hipError_t launch_cg_x_update(double* x, const double* p, const double* part_rz, const double* part_pq, int n_pq,
                              int64_t n, hipStream_t s);
// y = a*x + b*y with host scalars; x or y may alias out
hipError_t launch_axpby(double* out, double a, const double* x, double b, const double* y,
                        int64_t n, hipStream_t s);
// out = mask-free copy / fill
hipError_t launch_fill(double* out, double val, int64_t n, hipStream_t s);
// dinv[i] = d[i] > 0 ? 1/d[i] : 0
hipError_t launch_invert_diag(double* dinv, const double* d, int64_t n, hipStream_t s);
// out[i] = in[i] * (emask[i]) where mask derived from toff rows (interior iff row non-empty)
hipError_t launch_mask_copy(double* out, const double* in, const int32_t* toff, int64_t n,
                            hipStream_t s);
// dst[0..count) = src[0..count) on the device (count <= 64)
hipError_t launch_copy_scalar(double* dst, const double* src, int count, hipStream_t s);

}  // namespace feod
