// L-vector kernels: the deterministic transposed-map gather G^T, two-stage
// fixed-order FP64 reductions, and fused CG vector updates with the CG
// scalars kept on the device.
#include <hip/hip_runtime.h>

#include "kernel_api.hpp"

namespace feod {

constexpr int kVecThreads = 256;

static inline int vec_blocks(int64_t n) {
  int64_t b = (n + kVecThreads - 1) / kVecThreads;
  return (int)(b < 1 ? 1 : b);
}

// G^T: each DOF sums the E-vector entries listed in its row, in ascending
// E-vector order (no atomics: bitwise reproducible).  Dirichlet rows are
// empty and their load entry is 0, so the output row is exactly 0.
template <class TE, bool TWO>
__global__ __launch_bounds__(kVecThreads) void gather_t_kernel(const int32_t* __restrict__ off,
                                                               const int32_t* __restrict__ idx,
                                                               const TE* __restrict__ Y0,
                                                               const TE* __restrict__ Y1,
                                                               const double* __restrict__ bm,
                                                               double* __restrict__ out0,
                                                               double* __restrict__ out1, int64_t n) {
  const int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kVecThreads + threadIdx.x;
  if (i >= n) return;
  const int j0 = off[i], j1 = off[i + 1];
  double s0 = 0, s1 = 0;
  for (int j = j0; j < j1; ++j) {
    const int t = idx[j];
    s0 += (double)Y0[t];
    if (TWO) s1 += (double)Y1[t];
  }
  if (bm != nullptr) s0 -= bm[i];
  out0[i] = s0;
  if (TWO) out1[i] = s1;
}

hipError_t launch_gather_t(const int32_t* off, const int32_t* idx, const void* Y0, const void* Y1,
                           bool fp32, const double* bm, double* out0, double* out1, int64_t n,
                           hipStream_t s) {
  const int nb = vec_blocks(n);
  if (fp32) {
    if (Y1)
      hipLaunchKernelGGL((gather_t_kernel<float, true>), dim3(nb), dim3(kVecThreads), 0, s, off, idx,
                         (const float*)Y0, (const float*)Y1, bm, out0, out1, n);
    else
      hipLaunchKernelGGL((gather_t_kernel<float, false>), dim3(nb), dim3(kVecThreads), 0, s, off, idx,
                         (const float*)Y0, nullptr, bm, out0, nullptr, n);
  } else {
    if (Y1)
      hipLaunchKernelGGL((gather_t_kernel<double, true>), dim3(nb), dim3(kVecThreads), 0, s, off, idx,
                         (const double*)Y0, (const double*)Y1, bm, out0, out1, n);
    else
      hipLaunchKernelGGL((gather_t_kernel<double, false>), dim3(nb), dim3(kVecThreads), 0, s, off, idx,
                         (const double*)Y0, nullptr, bm, out0, nullptr, n);
  }
  return hipGetLastError();
}

LatticeDims make_lattice_dims(int32_t nx, int32_t ny, int32_t nz, int32_t k) {
  LatticeDims d{};
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.k = k;
  d.Lx = k * nx + 1;
  d.Ly = k * ny + 1;
  d.Lz = k * nz + 1;
  d.div_Lx = make_fastdiv((uint32_t)d.Lx);
  d.div_Ly = make_fastdiv((uint32_t)d.Ly);
  d.div_k = make_fastdiv((uint32_t)k);
  const uint32_t D1 = (uint32_t)k + 1, ne = D1 * D1 * D1;
  d.ne = ne;
  d.dlx = ne - (uint32_t)k;
  d.dly = (uint32_t)nx * ne - (uint32_t)k * D1;
  d.dlz = (uint32_t)nx * (uint32_t)ny * ne - (uint32_t)k * D1 * D1;
  return d;
}

// Computed transposed map: DOF (I,J,K) of the (k nx+1)(k ny+1)(k nz+1) node
// lattice lies in element ex = I/k (local a = I%k) and, when I is a multiple
// of k, also in ex-1 (local a = k); likewise in y and z.  The contributions are
// summed in ascending element order, which is the order of the explicit map.
// Dirichlet DOFs (on the lattice boundary) and indices past n get exactly 0.
//
// The gather is bound by memory latency (each wavefront's loads touch one
// short run per element), so a thread takes U DOFs and issues the candidate
// loads of all of them before it adds any.
template <class TE, bool TWO, int U>
__device__ __forceinline__ void lattice_rows_sum(const LatticeDims& d, const TE* __restrict__ Y0,
                                                 const TE* __restrict__ Y1, const int64_t (&i)[U], int64_t n,
                                                 double (&s0)[U], double (&s1)[U]) {
  TE v0[U][8], v1[U][8];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // n < 2^31 (checked at set-up): 32-bit unsigned index arithmetic
    const bool in = i[u] < n;
    const uint32_t iu = in ? (uint32_t)i[u] : 0u, t = fastdiv(iu, d.div_Lx);
    const int I = (int)(iu - t * (uint32_t)d.Lx), K = (int)fastdiv(t, d.div_Ly),
              J = (int)(t - (uint32_t)K * (uint32_t)d.Ly);
    const bool inner = in && I > 0 && I < d.Lx - 1 && J > 0 && J < d.Ly - 1 && K > 0 && K < d.Lz - 1;
    // The upper candidate (index/k, local index%k) always exists for an
    // interior DOF; the lower one in a direction (index/k - 1, local k)
    // exists when the index is a multiple of k, and its E-vector position is
    // the upper one's minus a constant of that direction.
    const uint32_t k = (uint32_t)d.k, D1 = k + 1;
    const uint32_t ix = fastdiv((uint32_t)I, d.div_k), iy = fastdiv((uint32_t)J, d.div_k),
                   iz = fastdiv((uint32_t)K, d.div_k);
    const uint32_t ai = (uint32_t)I - k * ix, bi = (uint32_t)J - k * iy, ci = (uint32_t)K - k * iz;
    const bool lx = ai == 0, ly = bi == 0, lz = ci == 0;
    const uint32_t j7 = (ix + (uint32_t)d.nx * (iy + (uint32_t)d.ny * iz)) * d.ne + ai + D1 * (bi + D1 * ci);
#pragma unroll
    for (int q = 0; q < 8; ++q) {  // q = tx + 2 ty + 4 tz, ascending element order
      const int tx = q & 1, ty = (q >> 1) & 1, tz = q >> 2;
      const bool use = inner && (tx || lx) && (ty || ly) && (tz || lz);
      const uint32_t j = j7 - (tx ? 0u : d.dlx) - (ty ? 0u : d.dly) - (tz ? 0u : d.dlz);
      v0[u][q] = use ? Y0[j] : TE(0);
      if (TWO) v1[u][q] = use ? Y1[j] : TE(0);
    }
  }
  // Adding +0 for absent candidates leaves the ordered sum unchanged.  The
  // sum starts from the first candidate rather than from 0, so that no
  // addition can be moved next to a load and make the thread wait for it
  // there; the final + 0 turns a -0 into +0, which makes the result bitwise
  // that of 0 + c_1 + c_2 + ... (the explicit map's sum): the two running
  // sums can differ only in the sign of a zero.
#pragma unroll
  for (int u = 0; u < U; ++u) {
    s0[u] = (double)v0[u][0];
    s1[u] = TWO ? (double)v1[u][0] : 0.0;
#pragma unroll
    for (int q = 1; q < 8; ++q) {
      s0[u] += (double)v0[u][q];
      if (TWO) s1[u] += (double)v1[u][q];
    }
    s0[u] += 0.0;
    if (TWO) s1[u] += 0.0;
  }
}

// DOFs (tiles) per thread of the plain lattice and tiled gathers.  One
// measured best with the current orders: the 64^3 Q4 FP64 tiled gather takes
// 94.8 us against 98.7 with two and 99.2 with four, 48^3 Q2 10.3 against
// 10.7 and 10.8, the 16^3 Q7 FP32 lattice gather 9.9 against 10.6 and 14.6
// (in lattice order alone two had been best: 64^3 Q4 120 against 124 us).
constexpr int kGatherUnroll = 1;

template <class TE, bool TWO>
__global__ __launch_bounds__(kVecThreads) void gather_t_lattice_kernel(LatticeDims d, const TE* __restrict__ Y0,
                                                                       const TE* __restrict__ Y1,
                                                                       const double* __restrict__ bm,
                                                                       double* __restrict__ out0,
                                                                       double* __restrict__ out1, int64_t n) {
  constexpr int U = kGatherUnroll;
  const int64_t i0 = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * (kVecThreads * U) + threadIdx.x;
  int64_t i[U];
  double bv[U], s0[U], s1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    i[u] = i0 + u * kVecThreads;
    bv[u] = (bm != nullptr && i[u] < n) ? bm[i[u]] : 0.0;
  }
  lattice_rows_sum<TE, TWO, U>(d, Y0, Y1, i, n, s0, s1);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (i[u] >= n) continue;
    if (bm != nullptr) s0[u] -= bv[u];  // bm is 0 on Dirichlet DOFs
    out0[i[u]] = s0[u];
    if (TWO) out1[i[u]] = s1[u];
  }
}

// The same gather with each wavefront on a tile of the node lattice: th = k
// rows (y) of tw = 64/k consecutive DOFs (x), the rows of one element layer.
// A wavefront's loads then read th adjacent x-lines of each element it
// touches (contiguous in the E-vector) instead of one line of 64 DOFs, which
// spans 64/k elements: at Q4, 4 spans of 160 bytes instead of 16 of 40.

struct GatherTiles {
  uint32_t th, tw, ntx, nty, ntiles;  // tile shape, tiles per row span and per plane, total
  FastDiv div_tw, div_ntx, div_nplane;
};

GatherTiles make_gather_tiles(const LatticeDims& d) {
  GatherTiles g{};
  g.th = (uint32_t)d.k;
  g.tw = 64 / g.th;
  g.ntx = ((uint32_t)d.Lx + g.tw - 1) / g.tw;
  g.nty = ((uint32_t)d.Ly + g.th - 1) / g.th;
  g.ntiles = g.ntx * g.nty * (uint32_t)d.Lz;
  g.div_tw = make_fastdiv(g.tw);
  g.div_ntx = make_fastdiv(g.ntx);
  g.div_nplane = make_fastdiv(g.ntx * g.nty);
  return g;
}

// Tiles where they measured faster: an FP64 E-vector with k = 2 or 4 (whole
// 64-lane tiles).  At 64^3 Q4 the plain gather takes 98.5 us against 117.5
// in lattice order, at 48^3 Q2 10.5 against 11.2; with k = 3 or 7 (63-lane
// tiles) and for FP32 E-vectors lattice order is 5-27% faster.
inline bool use_tiles(const LatticeDims& d, bool fp32) { return !fp32 && (d.k == 2 || d.k == 4); }

// DOF of the lane at (dx, dy) of tile t, or n when that lane falls outside
// the lattice (or t is past the last tile).
__device__ __forceinline__ int64_t tile_dof(const LatticeDims& d, const GatherTiles& g, uint32_t t, uint32_t dx,
                                            uint32_t dy, int64_t n) {
  const uint32_t kz = fastdiv(t, g.div_nplane), rem = t - kz * (g.ntx * g.nty);
  const uint32_t jt = fastdiv(rem, g.div_ntx), it = rem - jt * g.ntx;
  const uint32_t I = it * g.tw + dx, J = jt * g.th + dy;
  const bool ok = t < g.ntiles && dy < g.th && I < (uint32_t)d.Lx && J < (uint32_t)d.Ly;
  return ok ? (int64_t)I + (int64_t)d.Lx * ((int64_t)J + (int64_t)d.Ly * kz) : n;
}

template <class TE, bool TWO>
__global__ __launch_bounds__(kVecThreads) void gather_t_tiles_kernel(LatticeDims d, GatherTiles g,
                                                                     const TE* __restrict__ Y0,
                                                                     const TE* __restrict__ Y1,
                                                                     const double* __restrict__ bm,
                                                                     double* __restrict__ out0,
                                                                     double* __restrict__ out1, int64_t n) {
  constexpr int U = kGatherUnroll;
  const uint32_t lane = threadIdx.x & 63, w0 = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * (kVecThreads / 64) +
                                                   (threadIdx.x >> 6);
  const uint32_t dy = fastdiv(lane, g.div_tw), dx = lane - dy * g.tw;
  int64_t i[U];
  double bv[U], s0[U], s1[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    i[u] = tile_dof(d, g, w0 * U + u, dx, dy, n);  // this wavefront's u-th tile
    bv[u] = (bm != nullptr && i[u] < n) ? bm[i[u]] : 0.0;
  }
  lattice_rows_sum<TE, TWO, U>(d, Y0, Y1, i, n, s0, s1);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (i[u] >= n) continue;
    if (bm != nullptr) s0[u] -= bv[u];  // bm is 0 on Dirichlet DOFs
    out0[i[u]] = s0[u];
    if (TWO) out1[i[u]] = s1[u];
  }
}

// G^T by element runs.  A lane takes the k DOFs I = k r + a (a < k) of one
// lattice row (J, K): the nodes along x that element column r owns.  Each
// candidate element's x-line holding them is one contiguous run of k
// entries (wide loads); the DOF a = 0 also takes the entry a = k of element
// r - 1.  A wavefront covers th = k rows (one element layer) times 64/k runs,
// rows fastest, so the lanes of one run column read that element's adjacent
// x-lines (contiguous in the E-vector) and each row's stores are contiguous.
// Sums per DOF in ascending element order, absent candidates as +0 and a
// final + 0: bitwise the explicit map's 0 + c_1 + c_2 + ...
// Workgroup size of the run kernel per order: 512 threads at k = 4 (64^3
// Q4: 78.9-79.3 against 82.9-83.0 us with 256), 256 otherwise (32^3 Q3: 8.2
// against 8.5-8.6 us with 512; 48^3 Q2 the same either way).  The tile
// kernel keeps 256 (64^3 Q4 FP64: 95 against 99 us with 512).
template <int K>
constexpr int run_threads() {
  return K == 4 ? 512 : 256;
}

struct RunTiles {
  uint32_t th, tr, ngr, nplane, ntiles;  // rows and runs per tile, run groups per row group, tiles per plane, total
  FastDiv div_th, div_ngr, div_nplane;
};

// The sums (before the final + 0) of the k DOFs of run r of row (J, K = kz):
// candidates in ascending element order, absent ones as +0.
template <class TE, bool TWO, int K>
__device__ __forceinline__ void run_sums(const LatticeDims& d, const TE* __restrict__ Y0, const TE* __restrict__ Y1,
                                         uint32_t r, uint32_t J, uint32_t kz, double (&s0)[K], double (&s1)[K]) {
  constexpr uint32_t D1 = K + 1, NE = D1 * D1 * D1;
  const uint32_t nx = (uint32_t)d.nx;
#pragma unroll
  for (int a = 0; a < K; ++a) s0[a] = s1[a] = 0.0;
  if (J > 0 && J + 1 < (uint32_t)d.Ly && kz > 0 && kz + 1 < (uint32_t)d.Lz) {
    const uint32_t iy = J / K, iz = kz / K, bi = J - K * iy, ci = kz - K * iz;
    const bool ly = bi == 0, lz = ci == 0, up = r < nx, lo = r > 0 && r < nx;
    TE run0[4][K], run1[4][K], low0[4], low1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // q = ty + 2 tz: candidate element rows in ascending order
      const int ty = q & 1, tz = q >> 1;
      const bool use = (ty || ly) && (tz || lz);
      const uint32_t ey = iy - 1 + ty, ez = iz - 1 + tz;
      const uint32_t line = ((ey + (uint32_t)d.ny * ez) * nx + r) * NE + D1 * ((J - K * ey) + D1 * (kz - K * ez));
#pragma unroll
      for (int a = 0; a < K; ++a) run0[q][a] = run1[q][a] = TE(0);
      if (use && up) {
        __builtin_memcpy(run0[q], Y0 + line, K * sizeof(TE));
        if (TWO) __builtin_memcpy(run1[q], Y1 + line, K * sizeof(TE));
      }
      low0[q] = (use && lo) ? Y0[line - NE + K] : TE(0);  // element r - 1, entry a = k
      low1[q] = (TWO && use && lo) ? Y1[line - NE + K] : TE(0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s0[0] += (double)low0[q];
      if (TWO) s1[0] += (double)low1[q];
      if (lo) {  // a = 0 is interior in x only for 0 < r < nx
        s0[0] += (double)run0[q][0];
        if (TWO) s1[0] += (double)run1[q][0];
      }
#pragma unroll
      for (int a = 1; a < K; ++a) {
        s0[a] += (double)run0[q][a];
        if (TWO) s1[a] += (double)run1[q][a];
      }
    }
  }
}

template <class TE, bool TWO, int K>
__global__ __launch_bounds__(run_threads<K>()) void gather_t_runs_kernel(LatticeDims d, RunTiles g,
                                                                    const TE* __restrict__ Y0,
                                                                    const TE* __restrict__ Y1,
                                                                    const double* __restrict__ bm,
                                                                    double* __restrict__ out0,
                                                                    double* __restrict__ out1) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t t = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * (run_threads<K>() / 64) + (threadIdx.x >> 6);
  const uint32_t rr = fastdiv(lane, g.div_th), dy = lane - rr * g.th;
  const uint32_t kz = fastdiv(t, g.div_nplane), rem = t - kz * g.nplane;
  const uint32_t m = fastdiv(rem, g.div_ngr), gr = rem - m * g.ngr;
  const uint32_t nx = (uint32_t)d.nx, r = gr * g.tr + rr, J = m * g.th + dy;
  if (t >= g.ntiles || rr >= g.tr || r > nx || J >= (uint32_t)d.Ly) return;  // no barrier below
  const int64_t base = (int64_t)K * r + (int64_t)d.Lx * ((int64_t)J + (int64_t)d.Ly * kz);
  double s0[K], s1[K];
  run_sums<TE, TWO, K>(d, Y0, Y1, r, J, kz, s0, s1);
  // A full run is stored with wide stores (2 x 16 bytes per lane at k = 4):
  // per DOF stores left each instruction 8 of every 32 bytes of the lines it
  // touched, and cost 64^3 Q4 94 against 82 us.
  if (r < nx) {
    double v0[K], v1[K], b[K];
    if (bm != nullptr) __builtin_memcpy(b, bm + base, sizeof b);
#pragma unroll
    for (int a = 0; a < K; ++a) {
      v0[a] = s0[a] + 0.0;
      if (bm != nullptr) v0[a] -= b[a];  // bm is 0 on Dirichlet DOFs
      v1[a] = s1[a] + 0.0;
    }
    __builtin_memcpy(out0 + base, v0, sizeof v0);
    if (TWO) __builtin_memcpy(out1 + base, v1, sizeof v1);
  } else {  // the last run holds only the boundary DOF I = Lx - 1
    double v = s0[0] + 0.0;
    if (bm != nullptr) v -= bm[base];
    out0[base] = v;
    if (TWO) out1[base] = s1[0] + 0.0;
  }
}

static RunTiles make_run_tiles(const LatticeDims& d) {
  RunTiles g{};
  g.th = (uint32_t)d.k;
  g.tr = 64 / g.th;
  g.ngr = ((uint32_t)d.nx + 1 + g.tr - 1) / g.tr;
  g.nplane = g.ngr * (((uint32_t)d.Ly + g.th - 1) / g.th);
  g.ntiles = g.nplane * (uint32_t)d.Lz;
  g.div_th = make_fastdiv(g.th);
  g.div_ngr = make_fastdiv(g.ngr);
  g.div_nplane = make_fastdiv(g.nplane);
  return g;
}

template <class TE, bool TWO, int K>
static void launch_runs(const LatticeDims& d, const void* Y0, const void* Y1, const double* bm, double* out0,
                        double* out1, hipStream_t s) {
  const RunTiles g = make_run_tiles(d);
  constexpr int W = run_threads<K>() / 64;  // wavefronts per workgroup
  const int nb = (int)(((int64_t)g.ntiles + W - 1) / W);
  hipLaunchKernelGGL((gather_t_runs_kernel<TE, TWO, K>), dim3(nb), dim3(run_threads<K>()), 0, s, d, g, (const TE*)Y0,
                     (const TE*)Y1, bm, out0, out1);
}

template <class TE, bool TWO>
static bool launch_runs_k(const LatticeDims& d, const void* Y0, const void* Y1, const double* bm, double* out0,
                          double* out1, hipStream_t s) {
  switch (d.k) {
    case 2: launch_runs<TE, TWO, 2>(d, Y0, Y1, bm, out0, out1, s); return true;
    case 3: launch_runs<TE, TWO, 3>(d, Y0, Y1, bm, out0, out1, s); return true;
    case 4: launch_runs<TE, TWO, 4>(d, Y0, Y1, bm, out0, out1, s); return true;
    default: return false;
  }
}

hipError_t launch_gather_t_lattice(const LatticeDims& d, const void* Y0, const void* Y1, bool fp32,
                                   const double* bm, double* out0, double* out1, int64_t n, hipStream_t s) {
  // Per E-vector precision and order, the order measured fastest: runs for
  // an FP32 E-vector at k = 2, 3, 4 (64^3 Q4 76-79 against 113-115 us in
  // lattice order, 32^3 Q3 8.5 against 9.3-9.5, 48^3 Q2 10.1 against
  // 10.6-10.8), tiles for FP64 at k = 2, 4 (runs: 127 us at 64^3 Q4), and
  // lattice order for the rest (runs at 16^3 Q7: 12.6-12.7 against
  // 8.2-10.7 us; at 32^3 Q3 FP64 8.4 against 7.7-8.0).
  if (fp32) {
    if (Y1 ? launch_runs_k<float, true>(d, Y0, Y1, bm, out0, out1, s)
           : launch_runs_k<float, false>(d, Y0, nullptr, bm, out0, nullptr, s))
      return hipGetLastError();
  }
  if (use_tiles(d, fp32)) {
    const GatherTiles g = make_gather_tiles(d);
    const int64_t waves = ((int64_t)g.ntiles + kGatherUnroll - 1) / kGatherUnroll;
    const int nb = (int)((waves + kVecThreads / 64 - 1) / (kVecThreads / 64));
    if (fp32) {
      if (Y1)
        hipLaunchKernelGGL((gather_t_tiles_kernel<float, true>), dim3(nb), dim3(kVecThreads), 0, s, d, g,
                           (const float*)Y0, (const float*)Y1, bm, out0, out1, n);
      else
        hipLaunchKernelGGL((gather_t_tiles_kernel<float, false>), dim3(nb), dim3(kVecThreads), 0, s, d, g,
                           (const float*)Y0, nullptr, bm, out0, nullptr, n);
    } else {
      if (Y1)
        hipLaunchKernelGGL((gather_t_tiles_kernel<double, true>), dim3(nb), dim3(kVecThreads), 0, s, d, g,
                           (const double*)Y0, (const double*)Y1, bm, out0, out1, n);
      else
        hipLaunchKernelGGL((gather_t_tiles_kernel<double, false>), dim3(nb), dim3(kVecThreads), 0, s, d, g,
                           (const double*)Y0, nullptr, bm, out0, nullptr, n);
    }
    return hipGetLastError();
  }
  const int nb = vec_blocks((n + kGatherUnroll - 1) / kGatherUnroll);
  if (fp32) {
    if (Y1)
      hipLaunchKernelGGL((gather_t_lattice_kernel<float, true>), dim3(nb), dim3(kVecThreads), 0, s, d,
                         (const float*)Y0, (const float*)Y1, bm, out0, out1, n);
    else
      hipLaunchKernelGGL((gather_t_lattice_kernel<float, false>), dim3(nb), dim3(kVecThreads), 0, s, d,
                         (const float*)Y0, nullptr, bm, out0, nullptr, n);
  } else {
    if (Y1)
      hipLaunchKernelGGL((gather_t_lattice_kernel<double, true>), dim3(nb), dim3(kVecThreads), 0, s, d,
                         (const double*)Y0, (const double*)Y1, bm, out0, out1, n);
    else
      hipLaunchKernelGGL((gather_t_lattice_kernel<double, false>), dim3(nb), dim3(kVecThreads), 0, s, d,
                         (const double*)Y0, nullptr, bm, out0, nullptr, n);
  }
  return hipGetLastError();
}

// Fixed-shape block reduction: wavefront shuffles, then the 4 wave sums in order.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double ws[kVecThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kVecThreads / 64; ++i) s += ws[i];
  }
  return s;  // valid in thread 0
}

__global__ __launch_bounds__(kVecThreads) void dot_partial_kernel(const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  int64_t n, double* __restrict__ partial) {
  double s = 0;
  const int64_t stride = (int64_t)kRedBlocks * kVecThreads;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
    s += y ? x[i] * y[i] : x[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

hipError_t launch_dot_partial(const double* x, const double* y, int64_t n, double* partial,
                              hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kRedBlocks), dim3(kVecThreads), 0, s, x, y, n, partial);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecThreads) void reduce_final_kernel(const double* __restrict__ partial,
                                                                   int nparts, double* out, double sign,
                                                                   const double* add) {
  double s = 0;
  for (int i = threadIdx.x; i < nparts; i += kVecThreads) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = sign * s + (add ? add[0] : 0.0);
}

hipError_t launch_reduce_final(const double* partial, int nparts, double* out, double sign,
                               const double* add, hipStream_t s) {
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(kVecThreads), 0, s, partial, nparts, out, sign, add);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecThreads) void axpby_kernel(double* out, double a, const double* x, double b,
                                                            const double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (i >= n) return;
  out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

hipError_t launch_axpby(double* out, double a, const double* x, double b, const double* y, int64_t n,
                        hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, out, a, x, b, y, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecThreads) void fill_kernel(double* out, double val, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (i < n) out[i] = val;
}

hipError_t launch_fill(double* out, double val, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, out, val, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecThreads) void invert_diag_kernel(double* dinv, const double* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (i < n) dinv[i] = d[i] > 0.0 ? 1.0 / d[i] : 0.0;
}

hipError_t launch_invert_diag(double* dinv, const double* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(invert_diag_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, dinv, d, n);
  return hipGetLastError();
}

// interior iff the DOF's transposed-map row is non-empty
__global__ __launch_bounds__(kVecThreads) void mask_copy_kernel(double* out, const double* in,
                                                                const int32_t* toff, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (i < n) out[i] = (toff[i + 1] > toff[i]) ? in[i] : 0.0;
}

hipError_t launch_mask_copy(double* out, const double* in, const int32_t* toff, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(mask_copy_kernel, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, out, in, toff, n);
  return hipGetLastError();
}

__global__ void copy_scalar_kernel(double* dst, const double* src, int count) {
  if ((int)threadIdx.x < count) dst[threadIdx.x] = src[threadIdx.x];
}

hipError_t launch_copy_scalar(double* dst, const double* src, int count, hipStream_t s) {
  hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(64), 0, s, dst, src, count);
  return hipGetLastError();
}

// ---- Fused CG iteration --------------------------------------------------
// The CG vector kernels run kCgBlocks blocks of kCgThreads (one block per CU)
// over a grid-stride loop.  Every inner product leaves kCgBlocks partial sums;
// a kernel that needs the total sums the partials itself, each block in the
// same fixed order, so all blocks use the bitwise-same scalar and no separate
// single-block reduction launch (or cross-block fence) is needed.
static_assert(kCgThreads % 64 == 0, "CG blocks are whole wavefronts");

// Sum of v over the block, returned in every thread; fixed order.
__device__ __forceinline__ double cg_block_sum(double v, double* ws) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < kCgThreads / 64; ++i) s += ws[i];
  __syncthreads();  // ws may be reused
  return s;
}

__device__ __forceinline__ double cg_total(const double* __restrict__ part, double* ws, int count = kCgBlocks) {
  double v = 0;
  for (int i = threadIdx.x; i < count; i += kCgThreads) v += part[i];
  return cg_block_sum(v, ws);
}

// Block sum for the gather kernels (kGatherDotThreads threads), fixed order.
__device__ __forceinline__ double gather_block_sum(double v) {
  __shared__ double ws[kGatherDotThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < kGatherDotThreads / 64; ++i) s += ws[i];
  return s;  // the same in every thread
}

// The grid-stride kernels below take kCgUnroll DOFs per thread per pass (i,
// i + stride, ...) and issue all their loads before any store: indices past
// the end are clamped to n-1 for the loads and skipped for stores and sums.
// Each thread still adds its DOFs in ascending order.

// q = G^T Y and partial[b] = sum of p[i] q[i] over block b's share: a thread
// takes the DOFs i, i + S, i + 2S, ... (S = the grid's thread count) in that
// order, kGatherDotUnroll of them per pass with all their loads issued first.
// One per pass measured fastest: the grid already covers 4M DOFs per pass
// (at 64^3 Q4 the gather takes 143 us with one, 142-148 with two, 155 with
// four, whose registers cost occupancy).
constexpr int kGatherDotUnroll = 1;

template <class TE>
__global__ __launch_bounds__(kGatherDotThreads) void gather_t_lattice_dot_kernel(LatticeDims d,
                                                                                 const TE* __restrict__ Y,
                                                                                 const double* __restrict__ p,
                                                                                 double* __restrict__ q, int64_t n,
                                                                                 double* __restrict__ partial) {
  constexpr int U = kGatherDotUnroll;
  double acc = 0;
  const int64_t stride = (int64_t)gridDim.x * kGatherDotThreads;
  for (int64_t i0 = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kGatherDotThreads + threadIdx.x; i0 < n;
       i0 += U * stride) {
    int64_t i[U];
    double pv[U], s0[U], s1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      i[u] = i0 + u * stride;
      pv[u] = i[u] < n ? p[i[u]] : 0.0;
    }
    lattice_rows_sum<TE, false, U>(d, Y, nullptr, i, n, s0, s1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i[u] >= n) break;
      q[i[u]] = s0[u];
      acc += pv[u] * s0[u];
    }
  }
  acc = gather_block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <class TE>
__global__ __launch_bounds__(kGatherDotThreads) void gather_t_dot_kernel(const int32_t* __restrict__ off,
                                                                         const int32_t* __restrict__ idx,
                                                                         const TE* __restrict__ Y,
                                                                         const double* __restrict__ p,
                                                                         double* __restrict__ q, int64_t n,
                                                                         double* __restrict__ partial) {
  double acc = 0;
  const int64_t stride = (int64_t)gridDim.x * kGatherDotThreads;
  // same DOF-to-block assignment as the lattice kernel: bitwise-equal partials
  for (int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kGatherDotThreads + threadIdx.x; i < n;
       i += stride) {
    double s = 0;
    for (int j = off[i]; j < off[i + 1]; ++j) s += (double)Y[idx[j]];
    q[i] = s;
    acc += p[i] * s;
  }
  acc = gather_block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

hipError_t launch_gather_t_dot(const LatticeDims& dims, bool csr, const int32_t* off, const int32_t* idx,
                               const void* Y, bool fp32, const double* p, double* q, int64_t n, double* partial,
                               hipStream_t s) {
  // lattice order for both maps and precisions: the tiles of the plain FP64
  // gather measured no faster here (64^3 Q4 141.9 against 143.1 us, 48^3 Q2
  // 15.7 against 13.5), and its element runs for FP32 slower (64^3 Q4 190
  // against 145 us, 32^3 Q3 16.1 against 11.8, 48^3 Q2 16.6 against 13.3):
  // this kernel's fixed grid leaves 1-2 tiles per wavefront.
  const dim3 g(gather_dot_blocks(n)), b(kGatherDotThreads);
  const LatticeDims* d = csr ? nullptr : &dims;
  if (d) {
    if (fp32)
      hipLaunchKernelGGL((gather_t_lattice_dot_kernel<float>), g, b, 0, s, *d, (const float*)Y, p, q, n, partial);
    else
      hipLaunchKernelGGL((gather_t_lattice_dot_kernel<double>), g, b, 0, s, *d, (const double*)Y, p, q, n, partial);
  } else {
    if (fp32)
      hipLaunchKernelGGL((gather_t_dot_kernel<float>), g, b, 0, s, off, idx, (const float*)Y, p, q, n, partial);
    else
      hipLaunchKernelGGL((gather_t_dot_kernel<double>), g, b, 0, s, off, idx, (const double*)Y, p, q, n, partial);
  }
  return hipGetLastError();
}

// x = 0, r = b, z = dinv r (z aliases r when dinv is null), p = z;
// part_rz = partials of r.z, part_rr = partials of r.r (when dinv).
__global__ __launch_bounds__(kCgThreads) void cg_init_kernel(double* __restrict__ x, double* __restrict__ r,
                                                             double* __restrict__ z, double* __restrict__ p,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ dinv, int64_t n,
                                                             double* __restrict__ part_rz,
                                                             double* __restrict__ part_rr) {
  __shared__ double ws[kCgThreads / 64];
  double s0 = 0, s1 = 0;
  const int64_t stride = (int64_t)kCgBlocks * kCgThreads;
  for (int64_t i = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += stride) {
    const double ri = b[i];
    x[i] = 0.0;
    r[i] = ri;
    if (dinv) {
      const double zi = ri * dinv[i];
      z[i] = zi;
      p[i] = zi;
      s0 += ri * zi;
      s1 += ri * ri;
    } else {
      p[i] = ri;
      s0 += ri * ri;
    }
  }
  s0 = cg_block_sum(s0, ws);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = s0;
  if (dinv) {
    s1 = cg_block_sum(s1, ws);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s1;
  }
}

hipError_t launch_cg_init(double* x, double* r, double* z, double* p, const double* b, const double* dinv,
                          int64_t n, double* part_rz, double* part_rr, hipStream_t s) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(kCgBlocks), dim3(kCgThreads), 0, s, x, r, z, p, b, dinv, n, part_rz,
                     part_rr);
  return hipGetLastError();
}

// r = b - jx, z = dinv r; partials of r.z and r.r (x and p unchanged)
template <bool PREC>
__global__ __launch_bounds__(kCgThreads) void cg_true_residual_kernel(double* __restrict__ r, double* __restrict__ z,
                                                                      const double* __restrict__ b,
                                                                      const double* __restrict__ jx,
                                                                      const double* __restrict__ dinv, int64_t n,
                                                                      double* __restrict__ part_rz,
                                                                      double* __restrict__ part_rr) {
  __shared__ double ws[kCgThreads / 64];
  double s0 = 0, s1 = 0;
  const int64_t stride = (int64_t)kCgBlocks * kCgThreads;
  for (int64_t i = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += stride) {
    const double ri = b[i] - jx[i];
    r[i] = ri;
    if (PREC) {
      const double zi = ri * dinv[i];
      z[i] = zi;
      s0 += ri * zi;
      s1 += ri * ri;
    } else {
      s0 += ri * ri;
    }
  }
  s0 = cg_block_sum(s0, ws);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = s0;
  if (PREC) {
    s1 = cg_block_sum(s1, ws);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s1;
  }
}

hipError_t launch_cg_true_residual(double* r, double* z, const double* b, const double* jx, const double* dinv,
                                   int64_t n, double* part_rz, double* part_rr, hipStream_t s) {
  if (dinv)
    hipLaunchKernelGGL(cg_true_residual_kernel<true>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, r, z, b, jx, dinv, n,
                       part_rz, part_rr);
  else
    hipLaunchKernelGGL(cg_true_residual_kernel<false>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, r, r, b, jx,
                       nullptr, n, part_rz, nullptr);
  return hipGetLastError();
}

// alpha = (r.z) / (p.q) from the partials; r -= alpha q; z = dinv r; new
// partials of r.z and r.r.  x is not touched here: x += alpha p happens in
// the direction kernel (which reads p anyway) or, when CG stops or replaces
// its residual after this step, in cg_x_update.  Block 0 records r.z and p.q
// in sc[i_rz], sc[i_pq] for the host's convergence and breakdown checks.
template <bool PREC>
__global__ __launch_bounds__(kCgThreads) void cg_step_kernel(double* __restrict__ r, double* __restrict__ z,
                                                             const double* __restrict__ q,
                                                             const double* __restrict__ dinv,
                                                             const double* __restrict__ part_rz,
                                                             const double* __restrict__ part_pq, int n_pq, int64_t n,
                                                             double* __restrict__ part_rz_new,
                                                             double* __restrict__ part_rr, double* __restrict__ sc,
                                                             int i_rz, int i_pq) {
  __shared__ double ws[kCgThreads / 64];
  const int64_t stride = (int64_t)kCgBlocks * kCgThreads;
  const int64_t first = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  // the first pass's loads go out before the scalar sums, hiding their latency
  double rv[kCgUnroll], qv[kCgUnroll], dv[kCgUnroll];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < kCgUnroll; ++u) {
      const int64_t i = min(i0 + u * stride, n - 1);
      rv[u] = r[i];
      qv[u] = q[i];
      if (PREC) dv[u] = dinv[i];
    }
  };
  if (first < n) load(first);
  const double rz = cg_total(part_rz, ws), pq = cg_total(part_pq, ws, n_pq);
  const double alpha = rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[i_rz] = rz;
    sc[i_pq] = pq;
  }
  double s0 = 0, s1 = 0;
  for (int64_t i0 = first; i0 < n; i0 += kCgUnroll * stride) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < kCgUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
        const double ri = rv[u] - alpha * qv[u];
        r[i] = ri;
        if (PREC) {
          const double zi = ri * dv[u];
          z[i] = zi;
          s0 += ri * zi;
          s1 += ri * ri;
        } else {
          s0 += ri * ri;
        }
      }
    }
  }
  s0 = cg_block_sum(s0, ws);
  if (threadIdx.x == 0) part_rz_new[blockIdx.x] = s0;
  if (PREC) {
    s1 = cg_block_sum(s1, ws);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s1;
  }
}

hipError_t launch_cg_step(double* r, double* z, const double* q, const double* dinv, const double* part_rz,
                          const double* part_pq, int n_pq, int64_t n, double* part_rz_new, double* part_rr,
                          double* sc, int i_rz, int i_pq, hipStream_t s) {
  if (dinv)
    hipLaunchKernelGGL(cg_step_kernel<true>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, r, z, q, dinv, part_rz,
                       part_pq, n_pq, n, part_rz_new, part_rr, sc, i_rz, i_pq);
  else
    hipLaunchKernelGGL(cg_step_kernel<false>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, r, r, q, nullptr, part_rz,
                       part_pq, n_pq, n, part_rz_new, nullptr, sc, i_rz, i_pq);
  return hipGetLastError();
}

// beta = (r.z)_new / (r.z)_old from the partials; with x: x += alpha p (the
// step's alpha = (r.z)_old / (p.q), the same expression and partial sums as
// the step uses) before p = z + beta p.
template <bool XUPD>
__global__ __launch_bounds__(kCgThreads) void cg_direction_kernel(double* __restrict__ p,
                                                                  const double* __restrict__ z,
                                                                  double* __restrict__ x,
                                                                  const double* __restrict__ part_new,
                                                                  const double* __restrict__ part_old,
                                                                  const double* __restrict__ part_pq, int n_pq,
                                                                  int64_t n) {
  __shared__ double ws[kCgThreads / 64];
  const int64_t stride = (int64_t)kCgBlocks * kCgThreads;
  const int64_t first = (int64_t)blockIdx.x * kCgThreads + threadIdx.x;
  double zv[kCgUnroll], pv[kCgUnroll], xv[kCgUnroll];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < kCgUnroll; ++u) {
      const int64_t i = min(i0 + u * stride, n - 1);
      zv[u] = z[i];
      pv[u] = p[i];
      if (XUPD) xv[u] = x[i];
    }
  };
  if (first < n) load(first);
  const double rz_old = cg_total(part_old, ws);
  const double beta = cg_total(part_new, ws) / rz_old;
  const double alpha = XUPD ? rz_old / cg_total(part_pq, ws, n_pq) : 0.0;
  for (int64_t i0 = first; i0 < n; i0 += kCgUnroll * stride) {
    if (i0 != first) load(i0);
#pragma unroll
    for (int u = 0; u < kCgUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
        if (XUPD) x[i] = xv[u] + alpha * pv[u];
        p[i] = zv[u] + beta * pv[u];
      }
    }
  }
}

hipError_t launch_cg_direction(double* p, const double* z, double* x, const double* part_new,
                               const double* part_old, const double* part_pq, int n_pq, int64_t n, hipStream_t s) {
  if (x)
    hipLaunchKernelGGL(cg_direction_kernel<true>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, p, z, x, part_new,
                       part_old, part_pq, n_pq, n);
  else
    hipLaunchKernelGGL(cg_direction_kernel<false>, dim3(kCgBlocks), dim3(kCgThreads), 0, s, p, z, nullptr,
                       part_new, part_old, nullptr, 0, n);
  return hipGetLastError();
}

// x += alpha p with the last step's alpha = (r.z) / (p.q) from the partials:
// the update the direction kernel would have made, for a CG that stops (or
// replaces its residual) right after a step.
__global__ __launch_bounds__(kCgThreads) void cg_x_update_kernel(double* __restrict__ x,
                                                                 const double* __restrict__ p,
                                                                 const double* __restrict__ part_rz,
                                                                 const double* __restrict__ part_pq, int n_pq,
                                                                 int64_t n) {
  __shared__ double ws[kCgThreads / 64];
  const double rz = cg_total(part_rz, ws);
  const double alpha = rz / cg_total(part_pq, ws, n_pq);
  const int64_t stride = (int64_t)kCgBlocks * kCgThreads;
  for (int64_t i = (int64_t)blockIdx.x * kCgThreads + threadIdx.x; i < n; i += stride) x[i] = x[i] + alpha * p[i];
}

hipError_t launch_cg_x_update(double* x, const double* p, const double* part_rz, const double* part_pq, int n_pq,
                              int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cg_x_update_kernel, dim3(kCgBlocks), dim3(kCgThreads), 0, s, x, p, part_rz, part_pq, n_pq, n);
  return hipGetLastError();
}

}  // namespace feod
