// C ABI of the FEOD library: context, validation, workspace carving,
// operator dispatch, and the Newton-CG and adjoint drivers.
#include "feod.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "host_setup.hpp"
#include "kernel_api.hpp"
#include "noalloc.hpp"

using namespace feod;

namespace {

constexpr int kNumVec = 10;   // solver temporaries of length N
constexpr int kScalars = 64;  // device scalar slots
enum Vec { V_R = 0, V_DU, V_CR, V_CP, V_CQ, V_CZ, V_DINV, V_UT, V_AUX, V_AUX2 };
enum Scal { S_RZ = 0, S_PQ = 2, S_RR = 3, S_A = 4, S_B = 5, S_E = 6, S_T = 7 };
// CG partial-sum slots of kCgSlot doubles: p.q (up to kGatherDotMaxBlocks
// partials from the gather), r.z (two, alternating) and r.r (kCgBlocks each)
enum CgPart { C_PQ = 0, C_RZ0, C_RZ1, C_RR, kCgParts };
constexpr int kCgSlot = kGatherDotMaxBlocks > kCgBlocks ? kGatherDotMaxBlocks : kCgBlocks;

thread_local std::string g_setup_error;

struct ProfRec {
  int name;
  int ev;  // index into event pool (start = 2*ev, end = 2*ev+1)
};

}  // namespace

struct feod_ctx {
  // problem
  int nx = 0, ny = 0, nz = 0, k = 0, nq = 0, D1 = 0, Ne = 0, NQ3 = 0;
  double p = 2, eps = 0;
  bool curved = false;
  hipStream_t stream = nullptr;
  const ElemLaunchers* L = nullptr;
  Tables1D tab;
  Lattice lat;
  std::vector<double> load, rho, verts;
  std::vector<double> htab;  // B, D, w, xi concatenated (kernel argument source)
  bool has_rho = false;
  bool explicit_maps = false;  // G / G^T from stored maps (true) or computed from the lattice
  bool hand_tangent = false;   // FP64 Jacobian actions with the hand-coded J_D (comparison)
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  int device = -1;
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  int32_t *d_emap = nullptr, *d_toff = nullptr, *d_tidx = nullptr;
  double *d_bm = nullptr, *d_rho = nullptr, *d_verts = nullptr, *d_elem = nullptr;
  void *d_Y0 = nullptr, *d_Y1 = nullptr, *d_qdata = nullptr;
  int pa_prec = -1;  // precision of the stored partial-assembly data, -1: none
  double* d_vec[kNumVec] = {};
  double *d_part0 = nullptr, *d_part1 = nullptr, *d_cgpart = nullptr, *d_sc = nullptr;
  double* cg_part(int slot) const { return d_cgpart + (size_t)slot * kCgSlot; }
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> events;
  std::vector<ProfRec> recs;
  std::vector<std::string> names;
  std::map<std::string, std::pair<int64_t, double>> agg;
  std::string err;
};

namespace {

feod_status fail(feod_ctx* c, feod_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_setup_error = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail((ctx), FEOD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                        \
  do {                                   \
    feod_status s_ = (expr);             \
    if (s_ != FEOD_OK) return s_;        \
  } while (0)

int pow_kind(double p) {
  const double r = (p - 2.0) / 2.0;
  if (r == 0.0) return POW_ZERO;
  if (r == 0.25) return POW_QUARTER;
  if (r == 0.5) return POW_HALF;
  if (r == 1.0) return POW_ONE;
  return POW_GENERIC;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t tab64, tab32, emap, toff, tidx, bm, rho, verts, elem, Y0, Y1, qdata, vec, part0, part1, cgpart, sc, total;
};

Layout layout(const feod_ctx* c) {
  Layout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t ntab = 2 * (size_t)c->nq * c->D1 + 2 * (size_t)c->nq;
  const size_t E = (size_t)c->lat.E, N = (size_t)c->lat.N, Ene = E * c->Ne;
  l.tab64 = take(ntab * 8);
  l.tab32 = take(ntab * 4);
  l.emap = take(Ene * 4);
  l.toff = take((N + 1) * 4);
  l.tidx = take(c->lat.tidx.size() * 4 + 4);
  l.bm = take(N * 8);
  l.rho = take(E * 8);
  l.verts = take(c->curved ? c->verts.size() * 8 : 8);
  l.elem = take(E * 8);
  l.Y0 = take(Ene * 8);
  l.Y1 = take(Ene * 8);
  l.qdata = take(E * 3 * (size_t)c->NQ3 * 8);  // partial assembly: stored reference gradients
  l.vec = take(kNumVec * align_up(N * 8));
  l.part0 = take(kRedBlocks * 8);
  l.part1 = take(kRedBlocks * 8);
  l.cgpart = take(kCgParts * kCgSlot * 8);
  l.sc = take(kScalars * 8);
  l.total = off;
  return l;
}

feod_status need_bound(feod_ctx* c) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (!c->bound) return fail(c, FEOD_ESTATE, "feod_bind_workspace has not been called");
  return FEOD_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b) return false;
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

feod_status check_vec(feod_ctx* c, const void* ptr, const char* name) {
  if (!ptr) return fail(c, FEOD_EINVAL, std::string(name) + " is NULL");
  if (((uintptr_t)ptr) % 8) return fail(c, FEOD_EINVAL, std::string(name) + " is not 8-byte aligned");
  return FEOD_OK;
}

// ---- profiling -------------------------------------------------------------
int name_id(feod_ctx* c, const char* n) {
  for (size_t i = 0; i < c->names.size(); ++i)
    if (c->names[i] == n) return (int)i;
  c->names.push_back(n);
  return (int)c->names.size() - 1;
}

void harvest(feod_ctx* c) {
  if (c->recs.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (const auto& r : c->recs) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, c->events[2 * r.ev], c->events[2 * r.ev + 1]);
    auto& a = c->agg[c->names[r.name]];
    a.first += 1;
    a.second += ms;
  }
  c->recs.clear();
}

template <class F>
feod_status timed(feod_ctx* c, const char* name, F&& launch) {
  int ev = -1;
  if (c->prof) {
    if (c->recs.size() * 2 + 2 > c->events.size()) {
      if (c->events.size() >= 8192) {
        harvest(c);
      } else {
        for (int i = 0; i < 256; ++i) {
          hipEvent_t e;
          HIP_TRY(c, hipEventCreate(&e));
          c->events.push_back(e);
        }
      }
    }
    ev = (int)c->recs.size();
    HIP_TRY(c, hipEventRecord(c->events[2 * ev], c->stream));
  }
  hipError_t e = launch();
  if (e != hipSuccess) return fail(c, FEOD_EHIP, std::string(name) + ": " + hipGetErrorString(e));
  if (c->prof) {
    HIP_TRY(c, hipEventRecord(c->events[2 * ev + 1], c->stream));
    c->recs.push_back({name_id(c, name), ev});
  }
  return FEOD_OK;
}

// ---- operator pieces -------------------------------------------------------
ElemParams params(feod_ctx* c, const double* u, const double* v, void* out0, void* out1, int prec,
                  double p_override = 0.0) {
  ElemParams P{};
  P.u = u;
  P.v = v;
  P.emap = c->explicit_maps ? c->d_emap : nullptr;
  P.k = c->k;
  P.Lx = (int32_t)c->lat.Lx;
  P.Ly = (int32_t)c->lat.Ly;
  P.Lz = (int32_t)c->lat.Lz;
  P.rho = c->has_rho ? c->d_rho : nullptr;
  P.verts = c->curved ? c->d_verts : nullptr;
  P.tab = prec ? (const void*)c->d_tab32 : (const void*)c->d_tab64;
  P.out0 = out0;
  P.out1 = out1;
  P.qdata = c->d_qdata;
  P.E = (int32_t)c->lat.E;
  P.nx = c->nx;
  P.ny = c->ny;
  P.nz = c->nz;
  P.htab = c->htab.data();
  P.hinv[0] = c->nx;
  P.hinv[1] = c->ny;
  P.hinv[2] = c->nz;
  P.det = 1.0 / ((double)c->nx * c->ny * c->nz);
  const double p = p_override > 0 ? p_override : c->p;
  P.p = p;
  P.eps2 = c->eps * c->eps;
  P.r = (p - 2.0) / 2.0;
  P.inv_p = 1.0 / p;
  P.powkind = pow_kind(p);
  P.div_nx = make_fastdiv((uint32_t)c->nx);
  P.div_ny = make_fastdiv((uint32_t)c->ny);
  return P;
}

const char* op_name(int op, int prec) {
  static const char* n64[] = {"element_residual_f64", "element_jvp_f64", "element_resjvp_f64",
                              "element_energy_f64", "element_grad_f64", "element_diag_f64",
                              "element_qstore_f64", "element_jvp_pa_f64", "element_elm_f64",
                              "element_jvp_hand_f64"};
  static const char* n32[] = {"element_residual_f32", "element_jvp_f32", "element_resjvp_f32",
                              "element_energy_f32", "element_grad_f32", "element_diag_f32",
                              "element_qstore_f32", "element_jvp_pa_f32", "element_elm_f32",
                              "element_jvp_hand_f32"};
  return prec ? n32[op] : n64[op];
}

feod_status run_element(feod_ctx* c, int op, int prec, const ElemParams& P) {
  if (op == OP_JVP && prec == 0 && c->hand_tangent) op = OP_JVP_HND;
  ElemLaunch fn = c->L->prec[prec].op[op][c->curved ? 1 : 0][P.powkind];
  if (!fn) return fail(c, FEOD_EUNSUPPORTED, "operation not built for this (k, nq)");
  return timed(c, op_name(op, prec), [&] { return fn(P, c->stream); });
}

LatticeDims lattice_dims(const feod_ctx* c) { return make_lattice_dims(c->nx, c->ny, c->nz, c->k); }

// G^T of one or two E-vectors: y0 = G^T Y0 - bm (bm may be null), y1 = G^T Y1
hipError_t gather_t(feod_ctx* c, const void* Y0, const void* Y1, bool fp32, const double* bm, double* y0,
                    double* y1) {
  if (c->explicit_maps)
    return launch_gather_t(c->d_toff, c->d_tidx, Y0, Y1, fp32, bm, y0, y1, c->lat.N, c->stream);
  LatticeDims d = lattice_dims(c);
  return launch_gather_t_lattice(d, Y0, Y1, fp32, bm, y0, y1, c->lat.N, c->stream);
}

// r = M(A(Mu) - b) (bm != null) or M A(Mu)
feod_status apply_residual(feod_ctx* c, const double* u, double* r, int prec) {
  TRY(run_element(c, OP_RESIDUAL, prec, params(c, u, nullptr, c->d_Y0, nullptr, prec)));
  return timed(c, "gather_transpose", [&] { return gather_t(c, c->d_Y0, nullptr, prec == 1, c->d_bm, r, nullptr); });
}

feod_status apply_jvp(feod_ctx* c, const double* u, const double* v, double* jv, double* r, int prec,
                      double p_override = 0.0) {
  if (r) {
    TRY(run_element(c, OP_RESJVP, prec, params(c, u, v, c->d_Y0, c->d_Y1, prec, p_override)));
    return timed(c, "gather_transpose2", [&] { return gather_t(c, c->d_Y0, c->d_Y1, prec == 1, c->d_bm, r, jv); });
  }
  TRY(run_element(c, OP_JVP, prec, params(c, u, v, c->d_Y0, nullptr, prec, p_override)));
  return timed(c, "gather_transpose", [&] { return gather_t(c, c->d_Y0, nullptr, prec == 1, nullptr, jv, nullptr); });
}

// diag(J(u)) = M G^T (element diagonals), boundary rows 0
feod_status apply_diagonal(feod_ctx* c, const double* u, double* diag, int prec, double p_override = 0.0) {
  TRY(run_element(c, OP_DIAG, prec, params(c, u, nullptr, c->d_Y0, nullptr, prec, p_override)));
  return timed(c, "gather_transpose", [&] { return gather_t(c, c->d_Y0, nullptr, prec == 1, nullptr, diag, nullptr); });
}

// dinv = 1 / diag(J(u)) on interior DOFs, 0 on Dirichlet DOFs (Jacobi preconditioner)
feod_status jacobi(feod_ctx* c, const double* u, double* dinv, double* tmp, double p_override = 0.0) {
  TRY(apply_diagonal(c, u, tmp, 0, p_override));
  return timed(c, "invert_diag", [&] { return launch_invert_diag(dinv, tmp, c->lat.N, c->stream); });
}

// out_dev[0] = sum x*y (y may be null: sum x), deterministic
feod_status dot(feod_ctx* c, const double* x, const double* y, int64_t n, double* out_dev,
                double sign = 1.0, const double* add = nullptr) {
  TRY(timed(c, "dot_partial", [&] { return launch_dot_partial(x, y, n, c->d_part0, c->stream); }));
  return timed(c, "reduce_final",
               [&] { return launch_reduce_final(c->d_part0, kRedBlocks, out_dev, sign, add, c->stream); });
}

feod_status read_scalars(feod_ctx* c, int first, int count, double* host) {
  HIP_TRY(c, hipMemcpyAsync(host, c->d_sc + first, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FEOD_OK;
}

feod_status host_dot(feod_ctx* c, const double* x, const double* y, int64_t n, double* val) {
  TRY(dot(c, x, y, n, c->d_sc + S_T));
  return read_scalars(c, S_T, 1, val);
}

// E(u) = sum of the per-element energies (element kernel in precision prec,
// FP64 accumulation) - b . M u (FP64)
feod_status energy_dev(feod_ctx* c, const double* u, double* e_dev, int prec = 0) {
  TRY(run_element(c, OP_ENERGY, prec, params(c, u, nullptr, c->d_elem, nullptr, prec)));
  TRY(dot(c, c->d_elem, nullptr, c->lat.E, c->d_sc + S_A));
  return dot(c, c->d_bm, u, c->lat.N, e_dev, -1.0, c->d_sc + S_A);
}

feod_status host_energy(feod_ctx* c, const double* u, double* val) {
  TRY(energy_dev(c, u, c->d_sc + S_E));
  return read_scalars(c, S_E, 1, val);
}

// ---- CG on J(u) x = b (J symmetric, SPD on interior DOFs) ------------------
struct CgResult {
  int iters = 0, updates = 0;  // updates: reliable (true-residual) updates
  double res = 0, bnorm = 0;
  feod_status status = FEOD_OK;
};

// G^T of the E-vector Y0 into q, with the partial sums of p.q (CG slot C_PQ)
feod_status gather_t_dot(feod_ctx* c, bool fp32, const double* p, double* q) {
  return timed(c, "gather_transpose_dot", [&] {
    return launch_gather_t_dot(lattice_dims(c), c->explicit_maps, c->d_toff, c->d_tidx, c->d_Y0, fp32, p, q,
                               c->lat.N, c->cg_part(C_PQ), c->stream);
  });
}

// Preconditioned CG (Jacobi when dinv != null).  One iteration is four
// launches: the element kernel on p, G^T fused with the p.q partial sums, the
// step (alpha, r, z and the r.z / r.r partials) and the new direction (x +=
// alpha p, then beta and p; x and p are read once).  Inner products stay on the device as fixed-order partial sums;
// the host reads them every check_every iterations.  J applies use the fused
// kernel at u, or (pa) the stored partial-assembly data of u in precision prec
// (set up by the caller).
//
// reliable (with prec = FP32): the recursive residual of a CG whose Jacobian
// applies are FP32 drifts from the true one.  Whenever it has dropped by
// kReliableDrop since the last true residual (or below the tolerance), r is
// replaced by the FP64 true residual b - J64 x (x and p kept), and convergence
// is decided on that true residual only.
constexpr double kReliableDrop = 0.1;

feod_status cg(feod_ctx* c, const double* u, const double* b, double* x, double rtol, int max_it,
               int check_every, int prec, const double* dinv, CgResult* out, double p_override = 0.0,
               bool pa = false, bool reliable = false) {
  const int64_t N = c->lat.N;
  double* r = c->d_vec[V_CR];
  double* p = c->d_vec[V_CP];
  double* q = c->d_vec[V_CQ];
  double* z = dinv ? c->d_vec[V_CZ] : r;
  out->iters = 0;
  double bn2;
  TRY(host_dot(c, b, b, N, &bn2));
  out->bnorm = std::sqrt(bn2);
  if (!std::isfinite(bn2)) {
    out->status = FEOD_ENONFINITE;
    return fail(c, FEOD_ENONFINITE, "non-finite right-hand side in CG");
  }
  if (bn2 == 0.0) {
    out->res = 0;
    return timed(c, "fill", [&] { return launch_fill(x, 0.0, N, c->stream); });
  }
  int cur = C_RZ0, nxt = C_RZ1;
  TRY(timed(c, "cg_init", [&] {
    return launch_cg_init(x, r, z, p, b, dinv, N, c->cg_part(cur), c->cg_part(C_RR), c->stream);
  }));
  const double tol = rtol * out->bnorm;
  double last_true = out->bnorm;  // x = 0: r = b exactly
  // rr of the residual whose partials are in slot `slot` (r.r, or r.z = r.r without dinv)
  auto read_rr = [&](int slot, double* rr, double* pq) -> feod_status {
    TRY(timed(c, "reduce_final", [&] {
      return launch_reduce_final(c->cg_part(dinv ? C_RR : slot), kCgBlocks, c->d_sc + S_RR, 1.0, nullptr,
                                 c->stream);
    }));
    double sv[4];
    TRY(read_scalars(c, 0, 4, sv));
    *rr = sv[S_RR];
    *pq = sv[S_PQ];
    if (!std::isfinite(*rr) || !std::isfinite(*pq)) {
      out->status = FEOD_ENONFINITE;
      return fail(c, FEOD_ENONFINITE, "non-finite CG scalar");
    }
    return FEOD_OK;
  };
  for (int it = 0; it < max_it; ++it) {
    if (pa)
      TRY(run_element(c, OP_JVP_PA, prec, params(c, nullptr, p, c->d_Y0, nullptr, prec, p_override)));
    else
      TRY(run_element(c, OP_JVP, prec, params(c, u, p, c->d_Y0, nullptr, prec, p_override)));
    TRY(gather_t_dot(c, prec == 1, p, q));
    const int n_pq = gather_dot_blocks(N);
    TRY(timed(c, "cg_step", [&] {
      return launch_cg_step(r, z, q, dinv, c->cg_part(cur), c->cg_part(C_PQ), n_pq, N, c->cg_part(nxt),
                            c->cg_part(C_RR), c->d_sc, S_RZ, S_PQ, c->stream);
    }));
    // x += alpha p of this step, where the direction kernel cannot do it
    // (CG stops, or its residual is replaced from x, right after the step)
    bool x_done = false;
    auto update_x = [&]() -> feod_status {
      x_done = true;
      return timed(c, "cg_x_update", [&] {
        return launch_cg_x_update(x, p, c->cg_part(cur), c->cg_part(C_PQ), n_pq, N, c->stream);
      });
    };
    out->iters = it + 1;
    if ((it + 1) % check_every == 0 || it + 1 == max_it) {
      double rr, pq;
      TRY(read_rr(nxt, &rr, &pq));
      if (pq <= 0.0) {
        out->status = FEOD_EBREAKDOWN;
        return fail(c, FEOD_EBREAKDOWN, "CG breakdown: p^T J p <= 0");
      }
      out->res = std::sqrt(rr);
      if (reliable && (out->res <= tol || out->res <= kReliableDrop * last_true)) {
        // q is free here (consumed by the step): q = J64 x, then r = b - q
        TRY(update_x());
        TRY(apply_jvp(c, u, x, q, nullptr, 0, p_override));
        TRY(timed(c, "cg_true_residual", [&] {
          return launch_cg_true_residual(r, z, b, q, dinv, N, c->cg_part(nxt), c->cg_part(C_RR), c->stream);
        }));
        out->updates++;
        TRY(read_rr(nxt, &rr, &pq));
        out->res = last_true = std::sqrt(rr);
      }
      if (out->res <= tol) {
        if (!x_done) TRY(update_x());
        return FEOD_OK;
      }
    }
    TRY(timed(c, "cg_direction", [&] {
      return launch_cg_direction(p, z, x_done ? nullptr : x, c->cg_part(nxt), c->cg_part(cur), c->cg_part(C_PQ),
                                 n_pq, N, c->stream);
    }));
    std::swap(cur, nxt);
  }
  out->status = FEOD_ENOCONV;
  return FEOD_OK;  // caller decides; inexact Newton accepts a capped solve
}

feod_solver_opts defaults() {
  feod_solver_opts o;
  feod_default_opts(&o);
  return o;
}

feod_status validate_opts(feod_ctx* c, const feod_solver_opts& o) {
  if (!(o.rtol > 0) || !(o.cg_rtol_floor > 0) || o.max_newton < 0 || o.max_cg < 1 || o.max_ls < 0 ||
      o.check_every < 1 || (o.prec != FEOD_FP64 && o.prec != FEOD_MIXED))
    return fail(c, FEOD_EINVAL, "invalid solver options");
  return FEOD_OK;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ============================================================================
extern "C" {

void feod_default_opts(feod_solver_opts* o) {
  if (!o) return;
  o->rtol = 1e-10;
  o->cg_rtol_floor = 1e-12;
  o->max_newton = 50;
  o->max_cg = 20000;
  o->max_ls = 30;
  o->check_every = 10;
  o->prec = FEOD_FP64;
  o->init_poisson = 1;
  o->jacobi = 1;
  o->partial_assembly = 0;
}

feod_status feod_setup_mesh(const feod_mesh_desc* d, feod_ctx** out) {
  g_setup_error.clear();
  if (!d || !out) return fail(nullptr, FEOD_EINVAL, "null descriptor or output pointer");
  *out = nullptr;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(nullptr, FEOD_EINVAL, "nx, ny, nz must be >= 1");
  if (d->order_k < 1 || d->nq < 1) return fail(nullptr, FEOD_EINVAL, "order_k and nq must be >= 1");
  if (!std::isfinite(d->p) || !(d->p > 1.0)) return fail(nullptr, FEOD_EINVAL, "p must be finite and > 1");
  if (!std::isfinite(d->eps) || d->eps < 0) return fail(nullptr, FEOD_EINVAL, "eps must be finite and >= 0");
  if (d->eps == 0 && d->p < 2) return fail(nullptr, FEOD_EINVAL, "eps = 0 requires p >= 2");
  const ElemLaunchers* L = find_launchers(d->order_k + 1, d->nq);
  if (!L)
    return fail(nullptr, FEOD_EUNSUPPORTED,
                "no kernel built for k=" + std::to_string(d->order_k) + ", nq=" + std::to_string(d->nq));
  auto* c = new feod_ctx();
  c->nx = d->nx;
  c->ny = d->ny;
  c->nz = d->nz;
  c->k = d->order_k;
  c->nq = d->nq;
  c->D1 = c->k + 1;
  c->Ne = c->D1 * c->D1 * c->D1;
  c->NQ3 = c->nq * c->nq * c->nq;
  c->p = d->p;
  c->eps = d->eps;
  c->L = L;
  c->stream = (hipStream_t)d->stream;
  std::string msg;
  if (!make_lattice(c->nx, c->ny, c->nz, c->k, &c->lat, &msg)) {
    delete c;
    return fail(nullptr, FEOD_EUNSUPPORTED, msg);
  }
  c->tab = make_tables(c->k, c->nq);
  for (const auto* v : {&c->tab.B, &c->tab.D, &c->tab.qwts, &c->tab.qpts})
    c->htab.insert(c->htab.end(), v->begin(), v->end());
  const int64_t nv = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  if (d->vertices) {
    c->curved = true;
    c->verts.assign(d->vertices, d->vertices + nv * 3);
    for (double x : c->verts)
      if (!std::isfinite(x)) {
        delete c;
        return fail(nullptr, FEOD_EINVAL, "non-finite vertex coordinate");
      }
  }
  if (d->rho) {
    c->has_rho = true;
    c->rho.assign(d->rho, d->rho + c->lat.E);
    for (double x : c->rho)
      if (!(x > 0) || !std::isfinite(x)) {
        delete c;
        return fail(nullptr, FEOD_EINVAL, "rho must be finite and > 0");
      }
  } else {
    c->rho.assign(c->lat.E, 1.0);
  }
  if (d->load) {
    c->load.assign(d->load, d->load + c->lat.N);
  } else if (!make_load(c->lat, c->tab, c->curved ? c->verts.data() : nullptr, &c->load, &msg)) {
    delete c;
    return fail(nullptr, FEOD_EINVAL, msg);
  }
  if (c->curved && d->load) {  // still reject inverted elements
    std::vector<double> tmp;
    if (!make_load(c->lat, c->tab, c->verts.data(), &tmp, &msg)) {
      delete c;
      return fail(nullptr, FEOD_EINVAL, msg);
    }
  }
  *out = c;
  return FEOD_OK;
}

feod_status feod_workspace_bytes(const feod_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(nullptr, FEOD_EINVAL, "null argument");
  *bytes = layout(c).total;
  return FEOD_OK;
}

feod_status feod_bind_workspace(feod_ctx* c, void* dev, size_t bytes) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  const Layout l = layout(c);
  if (!dev) return fail(c, FEOD_EINVAL, "workspace pointer is NULL");
  if (((uintptr_t)dev) % 256) return fail(c, FEOD_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < l.total)
    return fail(c, FEOD_EINVAL, "workspace too small: need " + std::to_string(l.total) + " bytes");
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, noalloc_init(c->device));  // the static scratch of feod_jacobian_apply_noalloc on this device
  char* w = (char*)dev;
  c->ws = w;
  c->ws_bytes = bytes;
  c->d_tab64 = (double*)(w + l.tab64);
  c->d_tab32 = (float*)(w + l.tab32);
  c->d_emap = (int32_t*)(w + l.emap);
  c->d_toff = (int32_t*)(w + l.toff);
  c->d_tidx = (int32_t*)(w + l.tidx);
  c->d_bm = (double*)(w + l.bm);
  c->d_rho = (double*)(w + l.rho);
  c->d_verts = (double*)(w + l.verts);
  c->d_elem = (double*)(w + l.elem);
  c->d_Y0 = w + l.Y0;
  c->d_Y1 = w + l.Y1;
  c->d_qdata = w + l.qdata;
  c->pa_prec = -1;
  const size_t vstride = align_up((size_t)c->lat.N * 8);
  for (int i = 0; i < kNumVec; ++i) c->d_vec[i] = (double*)(w + l.vec + i * vstride);
  c->d_part0 = (double*)(w + l.part0);
  c->d_part1 = (double*)(w + l.part1);
  c->d_cgpart = (double*)(w + l.cgpart);
  c->d_sc = (double*)(w + l.sc);
  // tables: B, D, w, xi
  std::vector<double> t64;
  t64.insert(t64.end(), c->tab.B.begin(), c->tab.B.end());
  t64.insert(t64.end(), c->tab.D.begin(), c->tab.D.end());
  t64.insert(t64.end(), c->tab.qwts.begin(), c->tab.qwts.end());
  t64.insert(t64.end(), c->tab.qpts.begin(), c->tab.qpts.end());
  std::vector<float> t32(t64.begin(), t64.end());
  std::vector<double> bm(c->lat.N);
  for (int64_t i = 0; i < c->lat.N; ++i) bm[i] = c->lat.interior[i] ? c->load[i] : 0.0;
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpyAsync(c->d_tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_emap, c->lat.emap.data(), c->lat.emap.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_toff, c->lat.toff.data(), c->lat.toff.size() * 4, hipMemcpyHostToDevice, s));
  if (!c->lat.tidx.empty())
    HIP_TRY(c, hipMemcpyAsync(c->d_tidx, c->lat.tidx.data(), c->lat.tidx.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_bm, bm.data(), bm.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->d_rho, c->rho.data(), c->rho.size() * 8, hipMemcpyHostToDevice, s));
  if (c->curved)
    HIP_TRY(c, hipMemcpyAsync(c->d_verts, c->verts.data(), c->verts.size() * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->bound = true;
  return FEOD_OK;
}

feod_status feod_sizes(const feod_ctx* c, int64_t* n_dofs, int64_t* n_elems) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (n_dofs) *n_dofs = c->lat.N;
  if (n_elems) *n_elems = c->lat.E;
  return FEOD_OK;
}

feod_status feod_set_map_mode(feod_ctx* c, int32_t mode) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (mode != FEOD_MAPS_LATTICE && mode != FEOD_MAPS_EXPLICIT) return fail(c, FEOD_EINVAL, "invalid map mode");
  c->explicit_maps = mode == FEOD_MAPS_EXPLICIT;
  return FEOD_OK;
}

feod_status feod_set_tangent_mode(feod_ctx* c, int32_t mode) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (mode != FEOD_TANGENT_DUAL && mode != FEOD_TANGENT_HAND) return fail(c, FEOD_EINVAL, "invalid tangent mode");
  c->hand_tangent = mode == FEOD_TANGENT_HAND;
  return FEOD_OK;
}

feod_status feod_set_stream(feod_ctx* c, void* stream) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  c->stream = (hipStream_t)stream;
  return FEOD_OK;
}

static feod_status check_prec(feod_ctx* c, feod_prec prec) {
  if (prec != FEOD_FP64 && prec != FEOD_MIXED) return fail(c, FEOD_EINVAL, "invalid precision");
  return FEOD_OK;
}

feod_status feod_residual(feod_ctx* c, const double* u, double* r, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, r, "r"));
  const size_t nb = (size_t)c->lat.N * 8;
  if (overlap(u, nb, r, nb)) return fail(c, FEOD_EINVAL, "r overlaps u");
  return apply_residual(c, u, r, prec == FEOD_MIXED);
}

feod_status feod_jacobian_apply(feod_ctx* c, const double* u, const double* v, double* jv, double* r,
                                feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, v, "v"));
  TRY(check_vec(c, jv, "jv"));
  if (r) TRY(check_vec(c, r, "r"));
  const size_t nb = (size_t)c->lat.N * 8;
  if (overlap(u, nb, jv, nb) || overlap(v, nb, jv, nb)) return fail(c, FEOD_EINVAL, "jv overlaps an input");
  if (r && (overlap(u, nb, r, nb) || overlap(v, nb, r, nb) || overlap(jv, nb, r, nb)))
    return fail(c, FEOD_EINVAL, "r overlaps another argument");
  return apply_jvp(c, u, v, jv, r, prec == FEOD_MIXED);
}

feod_status feod_jacobian_apply_noalloc(feod_ctx* c, const double* u, const double* v, double* jv,
                                        feod_prec prec) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  TRY(check_prec(c, prec));
  const int pr = prec == FEOD_MIXED;
  const size_t need = (size_t)c->lat.E * c->Ne * (pr ? 4 : 8);
  if (need > kNoallocScratchBytes)
    return fail(c, FEOD_EINVAL,
                "the E-vector needs " + std::to_string(need) + " bytes, more than the " +
                    std::to_string(kNoallocScratchBytes) + "-byte static scratch: use feod_jacobian_apply");
  TRY(need_bound(c));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, v, "v"));
  TRY(check_vec(c, jv, "jv"));
  const size_t nb = (size_t)c->lat.N * 8;
  if (overlap(u, nb, jv, nb) || overlap(v, nb, jv, nb)) return fail(c, FEOD_EINVAL, "jv overlaps an input");
  void* Y = noalloc_scratch(c->device);
  if (!Y) return fail(c, FEOD_ESTATE, "static scratch not set up on the context's device");
  TRY(run_element(c, OP_JVP, pr, params(c, u, v, Y, nullptr, pr)));
  return timed(c, "gather_transpose", [&] { return gather_t(c, Y, nullptr, pr == 1, nullptr, jv, nullptr); });
}

feod_status feod_element_vectors(feod_ctx* c, int32_t op, const double* u, const double* v, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  if (op < 0 || op > 2) return fail(c, FEOD_EINVAL, "op must be 0, 1 or 2");
  if (op > 0) TRY(check_vec(c, v, "v"));
  const int pr = prec == FEOD_MIXED;
  const int kop = op == 0 ? OP_RESIDUAL : (op == 1 ? OP_JVP : OP_RESJVP);
  return run_element(c, kop, pr, params(c, u, op > 0 ? v : nullptr, c->d_Y0, c->d_Y1, pr));
}

feod_status feod_element_tangents(feod_ctx* c, const double* u, int64_t first, int64_t count, double* Ke) {
  TRY(need_bound(c));
  TRY(check_vec(c, u, "u"));
  if (first < 0 || count < 0 || first + count > c->lat.E)
    return fail(c, FEOD_EINVAL, "element range outside the mesh");
  if (count == 0) return FEOD_OK;  // nothing to write (Ke may be NULL)
  TRY(check_vec(c, Ke, "Ke"));
  if (count > INT32_MAX) return fail(c, FEOD_EINVAL, "too many elements in one call");
  ElemLaunch fn = c->L->tangent[c->curved ? 1 : 0][pow_kind(c->p)];
  if (!fn) return fail(c, FEOD_EUNSUPPORTED, "element tangents are built for k <= 4 only");
  if (overlap(u, (size_t)c->lat.N * 8, Ke, (size_t)count * c->Ne * c->Ne * 8))
    return fail(c, FEOD_EINVAL, "Ke overlaps u");
  ElemParams P = params(c, u, nullptr, Ke, nullptr, 0);
  P.e_first = (int32_t)first;
  P.E = (int32_t)count;
  return timed(c, "element_tangent_f64", [&] { return fn(P, c->stream); });
}

feod_status feod_element_tangents_elm(feod_ctx* c, const double* u, int64_t first, int64_t count, double* Ke) {
  TRY(need_bound(c));
  TRY(check_vec(c, u, "u"));
  if (first < 0 || count < 0 || first + count > c->lat.E)
    return fail(c, FEOD_EINVAL, "element range outside the mesh");
  if (count == 0) return FEOD_OK;  // nothing to write (Ke may be NULL)
  TRY(check_vec(c, Ke, "Ke"));
  if (count > INT32_MAX) return fail(c, FEOD_EINVAL, "too many elements in one call");
  ElemLaunch fn = c->L->prec[0].op[OP_ELM][c->curved ? 1 : 0][pow_kind(c->p)];
  if (!fn) return fail(c, FEOD_EUNSUPPORTED, "element-level tangents are built for k <= 4 only");
  if (overlap(u, (size_t)c->lat.N * 8, Ke, (size_t)count * c->Ne * c->Ne * 8))
    return fail(c, FEOD_EINVAL, "Ke overlaps u");
  ElemParams P = params(c, u, nullptr, Ke, nullptr, 0);
  P.e_first = (int32_t)first;
  P.E = (int32_t)count;
  return timed(c, "element_elm_f64", [&] { return fn(P, c->stream); });
}

feod_status feod_pa_setup(feod_ctx* c, const double* u, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  const int pr = prec == FEOD_MIXED;
  TRY(run_element(c, OP_QSTORE, pr, params(c, u, nullptr, nullptr, nullptr, pr)));
  c->pa_prec = pr;
  return FEOD_OK;
}

feod_status feod_jacobian_apply_pa(feod_ctx* c, const double* v, double* jv, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, v, "v"));
  TRY(check_vec(c, jv, "jv"));
  const int pr = prec == FEOD_MIXED;
  if (c->pa_prec != pr) return fail(c, FEOD_ESTATE, "feod_pa_setup has not been called for this precision");
  const size_t nb = (size_t)c->lat.N * 8;
  if (overlap(v, nb, jv, nb)) return fail(c, FEOD_EINVAL, "jv overlaps v");
  TRY(run_element(c, OP_JVP_PA, pr, params(c, nullptr, v, c->d_Y0, nullptr, pr)));
  return timed(c, "gather_transpose", [&] { return gather_t(c, c->d_Y0, nullptr, pr == 1, nullptr, jv, nullptr); });
}

feod_status feod_energy(feod_ctx* c, const double* u, double* e_dev, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, e_dev, "e_dev"));
  if (overlap(u, (size_t)c->lat.N * 8, e_dev, 8)) return fail(c, FEOD_EINVAL, "e_dev overlaps u");
  return energy_dev(c, u, e_dev, prec == FEOD_MIXED);
}

feod_status feod_jacobian_diagonal(feod_ctx* c, const double* u, double* diag, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, diag, "diag"));
  const size_t nb = (size_t)c->lat.N * 8;
  if (overlap(u, nb, diag, nb)) return fail(c, FEOD_EINVAL, "diag overlaps u");
  return apply_diagonal(c, u, diag, prec == FEOD_MIXED);
}

feod_status feod_grad_rho(feod_ctx* c, const double* u, const double* lam, double* grad, feod_prec prec) {
  TRY(need_bound(c));
  TRY(check_prec(c, prec));
  TRY(check_vec(c, u, "u"));
  TRY(check_vec(c, lam, "lambda"));
  TRY(check_vec(c, grad, "grad_rho"));
  const size_t nb = (size_t)c->lat.N * 8, ne = (size_t)c->lat.E * 8;
  if (overlap(u, nb, grad, ne) || overlap(lam, nb, grad, ne))
    return fail(c, FEOD_EINVAL, "grad_rho overlaps an input");
  const int pr = prec == FEOD_MIXED;
  return run_element(c, OP_GRAD, pr, params(c, u, lam, grad, nullptr, pr));
}

feod_status feod_set_rho(feod_ctx* c, const double* rho_dev) {
  TRY(need_bound(c));
  TRY(check_vec(c, rho_dev, "rho"));
  HIP_TRY(c, hipMemcpyAsync(c->d_rho, rho_dev, (size_t)c->lat.E * 8, hipMemcpyDeviceToDevice, c->stream));
  c->has_rho = true;
  return FEOD_OK;
}

// relative CG tolerance of the Poisson initial guess: only its shape is used
// (it is rescaled next), so a rough solve does
constexpr double kInitRtol = 1e-1;
constexpr int kScaleIters = 8;      // Newton steps of the 1D energy minimisation along the Poisson guess

feod_status feod_newton_solve(feod_ctx* c, double* u, const feod_solver_opts* opts_in,
                              feod_solver_report* rep_out) {
  const auto t0 = std::chrono::steady_clock::now();
  feod_solver_report rep{};
  rep.status = FEOD_OK;
  auto finish = [&](feod_status s) {
    rep.status = s;
    rep.seconds = seconds_since(t0);
    if (rep_out) *rep_out = rep;
    return s;
  };
  {
    feod_status s = need_bound(c);
    if (s != FEOD_OK) return finish(s);
  }
  const feod_solver_opts o = opts_in ? *opts_in : defaults();
  if (feod_status s = validate_opts(c, o); s != FEOD_OK) return finish(s);
  if (feod_status s = check_vec(c, u, "u"); s != FEOD_OK) return finish(s);
  const int64_t N = c->lat.N;
  const int prec = o.prec == FEOD_MIXED;
  double* R = c->d_vec[V_R];
  double* du = c->d_vec[V_DU];
  double* ut = c->d_vec[V_UT];
  double* rhs = c->d_vec[V_AUX];
  double ref2;
  if (feod_status s = host_dot(c, c->d_bm, c->d_bm, N, &ref2); s != FEOD_OK) return finish(s);
  rep.ref_norm = std::sqrt(ref2);
  CgResult cr;
  if (o.init_poisson) {
    // p = 2: J is the Laplacian, independent of u (linearised at u = 0)
    if (feod_status s = timed(c, "fill", [&] { return launch_fill(u, 0.0, N, c->stream); }); s != FEOD_OK)
      return finish(s);
    const double* dinv0 = nullptr;
    if (o.jacobi) {
      if (feod_status s = jacobi(c, u, c->d_vec[V_DINV], ut, 2.0); s != FEOD_OK) return finish(s);
      dinv0 = c->d_vec[V_DINV];
    }
    if (o.partial_assembly) {
      if (feod_status s = run_element(c, OP_QSTORE, prec, params(c, u, nullptr, nullptr, nullptr, prec)); s != FEOD_OK)
        return finish(s);
      c->pa_prec = prec;
    }
    // an initial guess only, whose shape matters (its size is set below):
    // the Poisson solve stops at 1e-1
    feod_status s = cg(c, u, c->d_bm, ut, kInitRtol, o.max_cg, o.check_every, prec, dinv0, &cr, 2.0,
                       o.partial_assembly);
    if (s != FEOD_OK) return finish(s);
    rep.cg_iters_total += cr.iters;
    // The p = 2 solution u2 has the right shape but, for p != 2, the wrong
    // size.  Scale it to the minimiser of the energy along its ray:
    // phi(alpha) = E(alpha u2) is convex, phi' = u2 . R(alpha u2) and
    // phi'' = u2 . J(alpha u2) u2, so a few Newton steps on phi' = 0 do.
    double alpha = 1.0;
    if (c->p != 2.0) {
      double* q = c->d_vec[V_DU];
      for (int k = 0; k < kScaleIters; ++k) {
        double g, h;
        if (feod_status s2 = timed(c, "axpby", [&] { return launch_axpby(u, alpha, ut, 0.0, nullptr, N, c->stream); });
            s2 != FEOD_OK)
          return finish(s2);
        if (feod_status s2 = apply_residual(c, u, R, 0); s2 != FEOD_OK) return finish(s2);
        if (feod_status s2 = host_dot(c, ut, R, N, &g); s2 != FEOD_OK) return finish(s2);
        if (feod_status s2 = apply_jvp(c, u, ut, q, nullptr, 0); s2 != FEOD_OK) return finish(s2);
        if (feod_status s2 = host_dot(c, ut, q, N, &h); s2 != FEOD_OK) return finish(s2);
        if (!(h > 0) || !std::isfinite(g)) break;  // flat or broken ray: keep what we have
        double next = alpha - g / h;
        if (!(next > 0)) next = 0.5 * alpha;  // stay on the positive ray
        const bool done = std::fabs(next - alpha) <= 1e-3 * alpha;
        alpha = next;
        if (done) break;
      }
    }
    if (feod_status s2 = timed(c, "axpby", [&] { return launch_axpby(u, alpha, ut, 0.0, nullptr, N, c->stream); });
        s2 != FEOD_OK)
      return finish(s2);
  } else {
    if (feod_status s = timed(c, "mask_copy", [&] { return launch_mask_copy(u, u, c->d_toff, N, c->stream); });
        s != FEOD_OK)
      return finish(s);
  }
  bool have_energy = false;  // energy_u holds E(u) for the current u
  double energy_u = 0.0;
  for (int it = 0;; ++it) {
    if (feod_status s = apply_residual(c, u, R, 0); s != FEOD_OK) return finish(s);
    double nr2;
    if (feod_status s = host_dot(c, R, R, N, &nr2); s != FEOD_OK) return finish(s);
    const double nr = std::sqrt(nr2);
    if (!std::isfinite(nr)) return finish(fail(c, FEOD_ENONFINITE, "non-finite residual"));
    if (it == 0) rep.res0 = nr;
    rep.res_final = nr;
    rep.newton_iters = it;
    if (nr <= o.rtol * rep.ref_norm) return finish(FEOD_OK);
    if (it >= o.max_newton) return finish(fail(c, FEOD_ENOCONV, "Newton iteration cap reached"));
    // forcing: eta = min(0.1, sqrt(|R_j| / |R_0|)), but never tighter than
    // the final tolerance needs (safeguard 0.5 tol |Mb| / |R_j|: a step that
    // reduces |R| by eta reaches the stopping test), floored at cg_rtol_floor
    double eta = std::min(0.1, std::sqrt(nr / rep.res0));
    eta = std::max(eta, 0.5 * o.rtol * rep.ref_norm / nr);
    eta = std::max(eta, o.cg_rtol_floor);
    if (feod_status s = timed(c, "axpby", [&] { return launch_axpby(rhs, -1.0, R, 0.0, nullptr, N, c->stream); });
        s != FEOD_OK)
      return finish(s);
    const double* dinv = nullptr;
    if (o.jacobi) {
      if (feod_status s = jacobi(c, u, c->d_vec[V_DINV], ut); s != FEOD_OK) return finish(s);
      dinv = c->d_vec[V_DINV];
    }
    if (o.partial_assembly) {
      if (feod_status s = run_element(c, OP_QSTORE, prec, params(c, u, nullptr, nullptr, nullptr, prec)); s != FEOD_OK)
        return finish(s);
      c->pa_prec = prec;
    }
    if (feod_status s = cg(c, u, rhs, du, eta, o.max_cg, o.check_every, prec, dinv, &cr, 0.0, o.partial_assembly);
        s != FEOD_OK)
      return finish(s);
    rep.cg_iters_total += cr.iters;
    // Armijo backtracking on the energy.  E(u) is known when the last step
    // came out of the line search: u was formed by the same axpby as the
    // accepted trial point, so the energy is bitwise the trial's.
    double E0, slope;
    if (have_energy)
      E0 = energy_u;
    else if (feod_status s = host_energy(c, u, &E0); s != FEOD_OK)
      return finish(s);
    if (feod_status s = host_dot(c, R, du, N, &slope); s != FEOD_OK) return finish(s);
    if (!std::isfinite(E0) || !std::isfinite(slope)) return finish(fail(c, FEOD_ENONFINITE, "non-finite energy"));
    double t = 1.0;
    have_energy = false;
    if (std::fabs(slope) > 1e-13 * std::fabs(E0)) {
      if (slope >= 0) return finish(fail(c, FEOD_EBREAKDOWN, "Newton direction is not a descent direction"));
      int h = 0;
      for (;; ++h) {
        if (feod_status s = timed(c, "axpby", [&] { return launch_axpby(ut, 1.0, u, t, du, N, c->stream); });
            s != FEOD_OK)
          return finish(s);
        double Et;
        if (feod_status s = host_energy(c, ut, &Et); s != FEOD_OK) return finish(s);
        if (std::isfinite(Et) && Et <= E0 + 1e-4 * t * slope) {
          energy_u = Et;  // the energy of the next u
          have_energy = true;
          break;
        }
        if (h >= o.max_ls) return finish(fail(c, FEOD_EBREAKDOWN, "line search failed"));
        t *= 0.5;
      }
      rep.ls_halvings_total += h;
    }
    if (feod_status s = timed(c, "axpby", [&] { return launch_axpby(u, 1.0, u, t, du, N, c->stream); });
        s != FEOD_OK)
      return finish(s);
  }
}

feod_status feod_adjoint_gradient(feod_ctx* c, const double* u, const double* g_u, double* lambda,
                                  double* grad, const feod_solver_opts* opts_in, feod_solver_report* rep_out) {
  const auto t0 = std::chrono::steady_clock::now();
  feod_solver_report rep{};
  auto finish = [&](feod_status s) {
    rep.status = s;
    rep.seconds = seconds_since(t0);
    if (rep_out) *rep_out = rep;
    return s;
  };
  if (feod_status s = need_bound(c); s != FEOD_OK) return finish(s);
  const feod_solver_opts o = opts_in ? *opts_in : defaults();
  if (feod_status s = validate_opts(c, o); s != FEOD_OK) return finish(s);
  for (auto pr : {std::make_pair((const void*)u, "u"), std::make_pair((const void*)g_u, "g_u"),
                  std::make_pair((const void*)grad, "grad_rho")})
    if (feod_status s = check_vec(c, pr.first, pr.second); s != FEOD_OK) return finish(s);
  const int64_t N = c->lat.N;
  const size_t nb = N * 8, ne = c->lat.E * 8;
  if (overlap(u, nb, grad, ne) || overlap(g_u, nb, grad, ne) ||
      (lambda && (overlap(u, nb, lambda, nb) || overlap(g_u, nb, lambda, nb) || overlap(grad, ne, lambda, nb))))
    return finish(fail(c, FEOD_EINVAL, "outputs overlap inputs"));
  double* rhs = c->d_vec[V_AUX];
  double* lam = lambda ? lambda : c->d_vec[V_DU];
  if (feod_status s = timed(c, "mask_copy", [&] { return launch_mask_copy(rhs, g_u, c->d_toff, N, c->stream); });
      s != FEOD_OK)
    return finish(s);
  CgResult cr;
  const double* dinv = nullptr;
  if (o.jacobi) {
    if (feod_status s = jacobi(c, u, c->d_vec[V_DINV], c->d_vec[V_AUX2]); s != FEOD_OK) return finish(s);
    dinv = c->d_vec[V_DINV];
  }
  if (o.partial_assembly) {
    const int pr = o.prec == FEOD_MIXED;
    if (feod_status s = run_element(c, OP_QSTORE, pr, params(c, u, nullptr, nullptr, nullptr, pr)); s != FEOD_OK)
      return finish(s);
    c->pa_prec = pr;
  }
  if (o.prec == FEOD_FP64) {
    if (feod_status s = cg(c, u, rhs, lam, o.rtol, o.max_cg, o.check_every, 0, dinv, &cr, 0.0, o.partial_assembly);
        s != FEOD_OK)
      return finish(s);
    rep.cg_iters_total = cr.iters;
    rep.ref_norm = cr.bnorm;
    rep.res0 = cr.bnorm;
    rep.res_final = cr.res;
    if (cr.status != FEOD_OK) return finish(fail(c, cr.status, "adjoint CG did not converge"));
  } else {
    // FP32 Jacobian applies inside one CG, FP64 vectors, reliable updates
    // with the FP64 true residual (convergence is decided on it)
    if (feod_status s = cg(c, u, rhs, lam, o.rtol, o.max_cg, o.check_every, 1, dinv, &cr, 0.0, o.partial_assembly,
                           /*reliable=*/true);
        s != FEOD_OK)
      return finish(s);
    rep.cg_iters_total = cr.iters;
    rep.refine_iters = cr.updates;
    rep.ref_norm = cr.bnorm;
    rep.res0 = cr.bnorm;
    rep.res_final = cr.res;
    if (cr.status != FEOD_OK) return finish(fail(c, cr.status, "adjoint CG did not converge"));
  }
  // The gradient kernel runs in FP64 in both modes: it is one pass, and the
  // refined lambda is FP64-accurate, so the result is too.
  if (feod_status s = run_element(c, OP_GRAD, 0, params(c, u, lam, grad, nullptr, 0)); s != FEOD_OK)
    return finish(s);
  if (hipError_t e = hipStreamSynchronize(c->stream); e != hipSuccess)
    return finish(fail(c, FEOD_EHIP, hipGetErrorString(e)));
  return finish(FEOD_OK);
}

feod_status feod_profile(feod_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (enable) {
    harvest(c);
    c->agg.clear();
    c->prof = true;
  } else {
    harvest(c);
    c->prof = false;
  }
  return FEOD_OK;
}

feod_status feod_profile_read(feod_ctx* c, feod_kernel_stat* stats, int32_t max, int32_t* n_out) {
  if (!c || !n_out || (max > 0 && !stats)) return fail(c, FEOD_EINVAL, "null argument");
  harvest(c);
  int n = 0;
  for (const auto& kv : c->agg) {
    if (n >= max) break;
    std::memset(stats[n].name, 0, sizeof(stats[n].name));
    std::strncpy(stats[n].name, kv.first.c_str(), sizeof(stats[n].name) - 1);
    stats[n].launches = kv.second.first;
    stats[n].total_ms = kv.second.second;
    ++n;
  }
  *n_out = n;
  return FEOD_OK;
}

// Floating-point operations of the pointwise operator D per quadrature point,
// counted from the kernel source (FMA = 2, mul/add = 1, reciprocal square
// root / division / pow = 1 each; a refined reciprocal square root is 1 + 8).
static double pointwise_flops(int op, int pk, bool curved) {
  // counted from the kernel source, FMA = 2, mul / add = 1, per point.
  // a^r: scalar and dual (value + tangent), by exponent kind
  const double apow_s[5] = {0, 20, 10, 0, 3};
  const double apow_d[5] = {0, 24, 12, 0, 6};
  // common to both geometries: weight w3 and s = rho w3 (2), a = eps^2 + |g|^2
  // (6 as a value, 17 as a dual), F = a^r g (3 as a value, 9 for the tangent)
  double f = 0;
  switch (op) {
    case OP_RESIDUAL: f = 2 + 6 + 3 + apow_s[pk]; break;
    case OP_JVP: f = 2 + 17 + 9 + apow_d[pk]; break;
    case OP_RESJVP: f = 2 + 17 + 12 + apow_d[pk]; break;  // tangent and value of F
    case OP_ENERGY: f = 1 + 6 + 2 + 4 + apow_s[pk]; break;  // W = a a^r / p, accumulate rho w det W
    case OP_GRAD: f = 1 + 6 + 5 + 4 + apow_s[pk]; break;    // a^r g_u . g_lambda, accumulate
    case OP_JVP_PA: f = 2 + 17 + 9 + apow_d[pk]; break;
    case OP_ELM: f = 2 + 17 + 9 + apow_d[pk]; break;  // one Jacobian action per direction
    case OP_JVP_HND: f = 2 + 17 + 9 + apow_d[pk]; break;  // the same count as the dual version
    default: f = 0;
  }
  // affine: the derivative tables carry 1/h; per point only sd = s det and
  // the output scaling sd F (per output field)
  const double affine[OP_COUNT] = {4, 4, 7, 0, 0, 0, 0, 4, 4, 4};
  // curved: Jg (12), adjugate (27), det (5), 1/det (1), physical gradient per
  // input field (18 each), reference flux s adj F per output field (18 each)
  const double geo[OP_COUNT] = {81, 99, 117, 63, 81, 0, 0, 99, 99, 99};
  return f + (curved ? geo[op] : affine[op]);
}

feod_status feod_kernel_cost(const feod_ctx* c, int32_t op, feod_prec prec, double* bytes, double* flops) {
  if (!c || !bytes || !flops || op < 0 || op >= OP_COUNT || op == OP_DIAG)
    return fail(nullptr, FEOD_EINVAL, "invalid argument");
  const double E = (double)c->lat.E, N = (double)c->lat.N, Ne = c->Ne, nq = c->nq, D1 = c->D1;
  const double NQ3 = (double)c->NQ3;
  const double ts = prec == FEOD_MIXED ? 4.0 : 8.0;
  // one sum-factorised gradient pass (B or B^T) per field, FMA = 2
  const double S = 4 * nq * D1 * D1 * D1 + 6 * nq * nq * D1 * D1 + 6 * nq * nq * nq * D1;
  const double passes[OP_COUNT] = {2, 3, 4, 1, 2, 0, 1, 2, 3, 3};
  const double fields[OP_COUNT] = {1, 2, 2, 1, 2, 1, 1, 1, 1, 2};
  const double outs[OP_COUNT] = {1, 1, 2, 0, 0, 1, 0, 1, 0, 1};
  // element-level AD (op 8): one Jacobian action per tangent direction, Ne of them
  const double dirs = op == OP_ELM ? Ne : 1.0;
  *flops = E * dirs * (passes[op] * S + NQ3 * pointwise_flops(op, pow_kind(c->p), c->curved));
  double b = fields[op] * 8.0 * N;  // unique L-vector reads
  if (c->explicit_maps) b += 4.0 * E * Ne;  // stored element-to-DOF map
  if (c->has_rho) b += 8.0 * E;
  if (c->curved) b += 24.0 * (c->nx + 1.0) * (c->ny + 1.0) * (c->nz + 1.0);
  b += outs[op] * ts * E * Ne;
  if (op == OP_ENERGY || op == OP_GRAD) b += 8.0 * E;
  if (op == OP_QSTORE || op == OP_JVP_PA) b += 3.0 * NQ3 * E * ts;  // stored gradients
  if (op == OP_ELM) b += 8.0 * E * Ne * Ne;                            // the K_e written
  *bytes = b;
  return FEOD_OK;
}

feod_status feod_host_tables(const feod_ctx* c, double* nodes, double* qpts, double* qwts, double* B, double* D) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (nodes) std::memcpy(nodes, c->tab.nodes.data(), c->tab.nodes.size() * 8);
  if (qpts) std::memcpy(qpts, c->tab.qpts.data(), c->tab.qpts.size() * 8);
  if (qwts) std::memcpy(qwts, c->tab.qwts.data(), c->tab.qwts.size() * 8);
  if (B) std::memcpy(B, c->tab.B.data(), c->tab.B.size() * 8);
  if (D) std::memcpy(D, c->tab.D.data(), c->tab.D.size() * 8);
  return FEOD_OK;
}

feod_status feod_host_maps(const feod_ctx* c, int32_t* emap, int32_t* toff, int32_t* tidx, int64_t* n_tidx) {
  if (!c) return fail(nullptr, FEOD_EINVAL, "null context");
  if (emap) std::memcpy(emap, c->lat.emap.data(), c->lat.emap.size() * 4);
  if (toff) std::memcpy(toff, c->lat.toff.data(), c->lat.toff.size() * 4);
  if (tidx) std::memcpy(tidx, c->lat.tidx.data(), c->lat.tidx.size() * 4);
  if (n_tidx) *n_tidx = (int64_t)c->lat.tidx.size();
  return FEOD_OK;
}

feod_status feod_host_load(const feod_ctx* c, double* load) {
  if (!c || !load) return fail(nullptr, FEOD_EINVAL, "null argument");
  std::memcpy(load, c->load.data(), c->load.size() * 8);
  return FEOD_OK;
}

feod_status feod_destroy(feod_ctx* c) {
  if (!c) return FEOD_OK;
  for (auto e : c->events) (void)hipEventDestroy(e);
  delete c;
  return FEOD_OK;
}

const char* feod_last_error(const feod_ctx* c) {
  return c ? c->err.c_str() : g_setup_error.c_str();
}

}  // extern "C"
