/*
 * feod.h -- C ABI of the MI355X (gfx950) matrix-free finite element operator
 * decomposition (FEOD) library for the regularised p-Laplacian.
 *
 * The operator factorises as A = P^T G^T B^T D B G P (paper, Fig. 1); on one
 * GPU the subdomain restriction P is the identity.  The library evaluates on
 * hexahedral tensor-product Q_k meshes of the unit cube (GLL nodal basis,
 * nq^3 Gauss-Legendre points, trilinear geometry):
 *
 *   residual  R(u)   = M ( G^T B^T D(B G M u) - b )                  Eq. (1)
 *   Jacobian  J(u) v = M G^T B^T J_D(u_q) B G M v                    Eq. (2)
 *
 * with D(g) = rho_e (eps^2 + |g|^2)^((p-2)/2) g at each quadrature point and
 * J_D obtained by forward-mode dual numbers at the quadrature points only
 * (the forward-mode remark after Eq. (2)).  M is the 0/1 mask of interior
 * (non-Dirichlet) DOFs and b the load vector of f.  Boundary rows of every
 * output are exactly 0 and boundary entries of every input are ignored.
 *
 * L-vectors have N = (k nx+1)(k ny+1)(k nz+1) entries ordered x fastest:
 * node (I,J,K) is I + (k nx+1)(J + (k ny+1) K).  Elements are ordered
 * ex + nx (ey + ny ez).
 *
 * Conventions for every entry point:
 *  - Vector arguments are caller-owned DEVICE pointers (float64, contiguous,
 *    8-byte aligned, length N for L-vectors and nx*ny*nz for element fields)
 *    on the device that was current at feod_bind_workspace.  The library never
 *    frees them.  Outputs must not overlap inputs (FEOD_EINVAL).
 *  - Host pointers are marked "host" and are copied before the call returns.
 *  - All device memory the library uses is the workspace the caller binds
 *    (feod_workspace_bytes / feod_bind_workspace); it allocates none itself.
 *  - Work is enqueued on the context's stream (a hipStream_t, may be NULL for
 *    the default stream).  Apply calls return without synchronising; solver
 *    calls synchronise and fill a report.
 *  - Errors are returned as feod_status; no exception or abort crosses the
 *    ABI.  feod_last_error(ctx) gives a message (ctx may be NULL for errors of
 *    feod_setup_mesh).  A context is not thread-safe.
 */
#ifndef FEOD_H
#define FEOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feod_ctx feod_ctx;

typedef enum {
  FEOD_OK = 0,
  FEOD_EINVAL = 1,        /* invalid argument, size, alignment or aliasing  */
  FEOD_EUNSUPPORTED = 2,  /* (k, nq) pair or size not built into this library */
  FEOD_EHIP = 3,          /* a HIP runtime call failed                       */
  FEOD_ENOCONV = 4,       /* solver hit its iteration cap                    */
  FEOD_ENONFINITE = 5,    /* NaN/Inf in a residual, energy or CG scalar      */
  FEOD_EBREAKDOWN = 6,    /* CG found p^T J p <= 0 or the line search failed */
  FEOD_ESTATE = 7         /* call made before feod_bind_workspace            */
} feod_status;

typedef enum { FEOD_FP64 = 0, FEOD_MIXED = 1 } feod_prec;

/* Problem description (paper: the p-Laplacian experiment; nonlinear action
 * Eq. (1)).  vertices: host, (nx+1)(ny+1)(nz+1) x 3 doubles, x fastest, or
 * NULL for the uniform lattice of the unit cube (affine elements).  rho: host,
 * nx*ny*nz per-element coefficients (> 0) or NULL for all ones.  load: host,
 * N doubles, the load vector b itself, or NULL for f = 1 computed internally.
 * stream: hipStream_t or NULL. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t order_k;   /* polynomial order k >= 1 (k+1 GLL nodes per direction) */
  int32_t nq;        /* Gauss-Legendre points per direction                   */
  double p;          /* exponent, p > 1                                       */
  double eps;        /* regularisation, eps >= 0 (eps > 0 required if p < 2)  */
  const double* vertices;
  const double* rho;
  const double* load;
  void* stream;
} feod_mesh_desc;

/* Newton-CG / adjoint options.  Newton stops when ||R(u)||_2 <= rtol ||M b||_2;
 * the adjoint solve when ||M g_u - J lambda||_2 <= rtol ||M g_u||_2.  CG inner
 * tolerance: eta_j = min(0.1, sqrt(||R_j||/||R_0||)), raised to at least
 * 0.5 rtol ||M b|| / ||R_j|| (no tighter than the stopping test needs) and
 * floored by cg_rtol_floor.  The p = 2 initial guess (init_poisson) is a CG
 * solve to 1e-1 relative, scaled (for p != 2) to the minimiser of the energy
 * along its ray by Newton steps on alpha -> u2 . R(alpha u2).
 * The line search is Armijo backtracking on the energy (c = 1e-4, halving,
 * at most max_ls halvings).  check_every: CG reads its residual norm back to
 * the host every this many iterations.  prec: FEOD_MIXED runs the Jacobian
 * applies inside CG in FP32 (residuals, CG vectors and dots stay FP64).  init_poisson: start Newton from the p = 2 solution
 * instead of the caller's u. */
typedef struct {
  double rtol;
  double cg_rtol_floor;
  int32_t max_newton;
  int32_t max_cg;
  int32_t max_ls;
  int32_t check_every;
  feod_prec prec;
  int32_t init_poisson;
  int32_t jacobi;    /* 1: precondition CG with diag J(u) (Jacobi), 0: none */
  int32_t partial_assembly; /* 1: CG applies J(u) from the stored gradients of u
                               (feod_pa_setup once per linearisation), 0: fused */
} feod_solver_opts;

typedef struct {
  int32_t newton_iters;
  int32_t cg_iters_total;
  int32_t refine_iters; /* adjoint, FEOD_MIXED: FP64 true-residual updates */
  int32_t ls_halvings_total;
  double res0;       /* initial residual norm                     */
  double res_final;  /* final residual norm                       */
  double ref_norm;   /* ||M b|| (Newton) or ||M g_u|| (adjoint)    */
  double seconds;    /* host wall time of the call                */
  feod_status status;
} feod_solver_report;

typedef struct {
  char name[40];
  int64_t launches;
  double total_ms;   /* sum of hipEvent-measured durations on the context stream */
} feod_kernel_stat;

/* Fill opts with defaults: rtol 1e-10, cg_rtol_floor 1e-12, max_newton 50,
 * max_cg 20000, max_ls 30, check_every 10, FP64, init_poisson 1, jacobi 1,
 * partial_assembly 0.  Jacobi preconditioning halves the CG iterations and
 * the Newton time on the 48^3 Q2 and 32^3 Q3 workloads.  Partial assembly
 * measured within 2.5% of the fused Jacobian action over whole Newton solves
 * on both (29.8 vs 30.5 ms and 38.8 vs 38.2 ms), so the default keeps the
 * fused action, whose quadrature data never leaves the registers.  At Q7 it
 * pays: the curved 16^3 Q7 Newton solve takes 95.4 instead of 104.8 ms and
 * its adjoint gradient 55.3 instead of 60.6 ms (FP64), so set it for Q6+. */
void feod_default_opts(feod_solver_opts* opts);

/* Build the mesh, element-to-DOF map G, transposed map for G^T, 1D tables and
 * load vector on the host (no GPU call).  *out receives a new context.
 * Returns FEOD_EINVAL for bad sizes/parameters or an inverted element, and
 * FEOD_EUNSUPPORTED for a (k, nq) pair without a compiled kernel or a mesh
 * whose DOF count or E-vector length (elements x (k+1)^3) reaches 2^31 - 1
 * (the kernels' 32-bit indices); nothing is allocated in that case. */
feod_status feod_setup_mesh(const feod_mesh_desc* desc, feod_ctx** out);

/* Bytes of device workspace the context needs (maps, tables, load, rho,
 * E-vectors, solver temporaries). */
feod_status feod_workspace_bytes(const feod_ctx* ctx, size_t* bytes);

/* Hand the context a caller-owned device buffer of at least
 * feod_workspace_bytes bytes, 256-byte aligned, on the current device; the
 * setup data is uploaded into it (synchronously).  The buffer must outlive
 * the context or the next bind. */
feod_status feod_bind_workspace(feod_ctx* ctx, void* dev_ptr, size_t bytes);

feod_status feod_sizes(const feod_ctx* ctx, int64_t* n_dofs, int64_t* n_elems);

/* How G and G^T find element DOFs (paper: G is "topological", independent
 * of the solution).  FEOD_MAPS_LATTICE (default): the element-to-DOF map and
 * its transpose are computed from the structured node lattice inside the
 * kernels; FEOD_MAPS_EXPLICIT: they are read from the stored map (E x (k+1)^3
 * int32) and transposed map (CSR).  Both give bitwise identical results: G^T
 * sums each DOF's element contributions in ascending E-vector order. */
enum { FEOD_MAPS_LATTICE = 0, FEOD_MAPS_EXPLICIT = 1 };
feod_status feod_set_map_mode(feod_ctx* ctx, int32_t mode);

/* How the FP64 Jacobian actions obtain J_D at the quadrature points (paper:
 * Table 1 compares AD with a hand-coded implementation, HND).
 * FEOD_TANGENT_DUAL (default): forward-mode dual numbers through the flux
 * (the remark after Eq. (2)).  FEOD_TANGENT_HAND: the same tangent written out
 * by hand, dF = a^r dg + (p-2) a^(r-1) (g . dg) g, for measuring the cost of
 * the dual numbers.  Affects the FP64 Jacobian action of feod_jacobian_apply
 * (without residual), feod_element_vectors op 1 and the fused applies of the
 * solvers; results agree to rounding. */
enum { FEOD_TANGENT_DUAL = 0, FEOD_TANGENT_HAND = 1 };
feod_status feod_set_tangent_mode(feod_ctx* ctx, int32_t mode);

/* Change the stream later calls enqueue on. */
feod_status feod_set_stream(feod_ctx* ctx, void* stream);

/* Eq. (1): r = M (A(M u) - b).  u, r: device, length N.  FEOD_MIXED evaluates
 * B, D and B^T in FP32 (G^T sums in FP64). */
feod_status feod_residual(feod_ctx* ctx, const double* u, double* r, feod_prec prec);

/* Eq. (2): jv = M J(M u) M v with J_D from dual numbers at quadrature points.
 * If r_or_null is not NULL the residual R(u) is produced by the same pass.
 * u, v, jv, r: device, length N. */
feod_status feod_jacobian_apply(feod_ctx* ctx, const double* u, const double* v,
                                double* jv, double* r_or_null, feod_prec prec);

/* For callers that cannot allocate device memory per call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * Jacobian action of feod_jacobian_apply (no residual) with the E-vector
 * between the element stage and G^T held in a library-owned static device
 * array of 32 MiB per GPU (looked up at feod_bind_workspace, kept until the
 * process ends) instead of the context's workspace.  Calls no allocating
 * routine.  Results are bitwise those of feod_jacobian_apply.  The
 * E-vector takes nx*ny*nz*(k+1)^3 * 8 bytes (FP64) or * 4 (FEOD_MIXED);
 * larger meshes return FEOD_EINVAL (use feod_jacobian_apply).  Every call on
 * one GPU, from any context, shares that GPU's array: calls that overlap in
 * time on one GPU (different streams or threads) race and must be ordered by
 * the caller.  The context's bound workspace still provides the mesh data
 * (coefficients, vertices, maps).  u, v, jv: device, length N. */
feod_status feod_jacobian_apply_noalloc(feod_ctx* ctx, const double* u, const double* v,
                                        double* jv, feod_prec prec);

/* The element stage alone, G -> B -> D -> B^T of Eq. (1)/(2), written into
 * the context's internal E-vector(s) (no G^T): op 0 residual, 1 Jacobian
 * action, 2 both.  For timing the element kernel on its own; u, v: device,
 * length N (v ignored for op 0). */
feod_status feod_element_vectors(feod_ctx* ctx, int32_t op, const double* u, const double* v,
                                 feod_prec prec);

/* Element tangent matrices (Eq. 3): K_e = d r_e / d u_e = B^T J_D(u_q) B for
 * elements first .. first+count-1, evaluated at the element values of M u,
 * with J_D from forward-mode dual numbers at each quadrature point and B^T J_D B
 * contracted by sum factorisation.  Ke: device, count * (k+1)^6 doubles, one
 * row-major (k+1)^3 x (k+1)^3 matrix per element in local node order
 * a + (k+1)(b + (k+1) c).  FP64; FEOD_EUNSUPPORTED for k > 4.  count = 0
 * writes nothing (Ke may then be NULL). */
feod_status feod_element_tangents(feod_ctx* ctx, const double* u, int64_t first, int64_t count,
                                  double* Ke);

/* The same matrices by element-level forward AD, the paper's ELM variant of
 * Table 1 (AD through the whole element residual r_e = B^T D(B u_e) of Eq. 3
 * instead of at the quadrature points): column j of K_e is one element
 * Jacobian action B^T J_D B e_j with the unit vector e_j of local node j as
 * the dual direction, so an element costs (k+1)^3 passes of B, D and B^T
 * where feod_element_tangents contracts B^T J_D B once.  Same arguments,
 * layout and errors as feod_element_tangents; for comparing the two. */
feod_status feod_element_tangents_elm(feod_ctx* ctx, const double* u, int64_t first, int64_t count,
                                      double* Ke);

/* Partial assembly (the pointwise data of Fig. 1's caption): store the
 * gradients of M u at every quadrature point (3 per point, in the precision
 * of prec; physical gradients on affine meshes, reference ones on curved
 * meshes) in the workspace, so that feod_jacobian_apply_pa can
 * apply J(u) without recomputing the gradient of u. */
feod_status feod_pa_setup(feod_ctx* ctx, const double* u, feod_prec prec);

/* jv = M J(u) M v at the u of the last feod_pa_setup with the same prec
 * (FEOD_ESTATE otherwise).  v, jv: device, length N. */
feod_status feod_jacobian_apply_pa(feod_ctx* ctx, const double* v, double* jv, feod_prec prec);

/* Energy E(u) = sum_e rho_e int_e (1/p)(eps^2+|grad Mu|^2)^(p/2) - b^T M u of
 * the p-Laplacian model problem, the functional whose gradient is the
 * residual of Eq. (1) (R = dE/du, quadrature included); the Newton line
 * search uses it as its merit function.  e_dev: device, 1 double.  prec:
 * FEOD_MIXED evaluates the element energies in FP32 (their sum and b^T M u in
 * FP64); the Newton driver always uses FP64, since its line search compares
 * energies that differ in their last digits. */
feod_status feod_energy(feod_ctx* ctx, const double* u, double* e_dev, feod_prec prec);

/* diag(J(u)): the diagonal of the masked Jacobian of Eq. (2) (boundary rows
 * 0), by sum-factorised quadrature of grad phi_i^T J_D grad phi_i followed by
 * G^T.  u, diag: device, length N. */
feod_status feod_jacobian_diagonal(feod_ctx* ctx, const double* u, double* diag,
                                   feod_prec prec);

/* Damped inexact Newton-CG on R(u) = 0 of Eq. (1), each step solving
 * J(u) du = -R(u) by CG with the matrix-free Jacobian action of Eq. (2) (J is
 * symmetric, positive definite on the interior DOFs), the step damped by the
 * line search on feod_energy.  u: device, length N; in: initial guess (used
 * unless opts->init_poisson), out: solution with boundary entries 0.  opts may
 * be NULL (defaults).  report may be NULL.  Synchronises the stream.  With
 * FEOD_MIXED the Jacobian actions inside CG run in FP32; residuals, energies,
 * CG vectors and inner products stay FP64, so the stopping test is the same
 * FP64 one. */
feod_status feod_newton_solve(feod_ctx* ctx, double* u, const feod_solver_opts* opts,
                              feod_solver_report* report);

/* Adjoint design gradient (paragraph after Eq. (3)): solve J(u) lambda = M g_u
 * by CG with the same matrix-free Jacobian action (J is symmetric), then
 * grad_rho[e] = dPhi/drho_e = -lambda^T dR/drho_e
 *             = -sum_q w detJ (eps^2+|grad u|^2)^((p-2)/2) grad u . grad lambda
 * by one per-element kernel (no G^T).  u, g_u, lambda_or_null: device,
 * length N; grad_rho: device, nx*ny*nz.  With FEOD_MIXED the CG runs FP32
 * Jacobian applies and replaces its recursive residual by the FP64 true
 * residual M g_u - J lambda (reliable updates) whenever the former has dropped
 * 10x since the last replacement; it stops on the true residual.  The gradient
 * kernel runs in FP64.  Synchronises. */
feod_status feod_adjoint_gradient(feod_ctx* ctx, const double* u, const double* g_u,
                                  double* lambda_or_null, double* grad_rho,
                                  const feod_solver_opts* opts,
                                  feod_solver_report* report);

/* The per-element gradient kernel alone, for given u and lambda:
 * grad_rho[e] = -sum_q w detJ a^r grad(Mu) . grad(M lambda). */
feod_status feod_grad_rho(feod_ctx* ctx, const double* u, const double* lambda,
                          double* grad_rho, feod_prec prec);

/* Replace the per-element coefficient: rho_dev is a device array of
 * nx*ny*nz doubles, copied (stream-ordered) into the workspace. */
feod_status feod_set_rho(feod_ctx* ctx, const double* rho_dev);

/* Per-kernel timing with hipEvents recorded around every launch on the
 * context stream (enable = 1 clears and starts, 0 stops).  feod_profile_read
 * synchronises and returns up to max aggregated entries. */
feod_status feod_profile(feod_ctx* ctx, int32_t enable);
feod_status feod_profile_read(feod_ctx* ctx, feod_kernel_stat* stats, int32_t max,
                              int32_t* n_out);

/* Algorithmic cost of one launch of the fused element kernel for an
 * operation (0 residual, 1 Jacobian apply, 2 residual+Jacobian, 3 energy,
 * 4 gradient, 6 partial-assembly set-up, 7 partial-assembly Jacobian apply,
 * 8 element-level tangents (all (k+1)^3 directions, K_e written), 9 the
 * Jacobian apply with the hand-coded J_D (counted as op 1);
 * 5 (diagonal) is not modelled) at precision prec: bytes moved to/from HBM by the
 * design (unique reads of inputs and maps, E-vector writes) and floating
 * point operations (FMA = 2).  Host only. */
feod_status feod_kernel_cost(const feod_ctx* ctx, int32_t op, feod_prec prec,
                             double* bytes, double* flops);

/* Host copies of setup data, for inspection without a GPU.
 * Tables: nodes[k+1], qpts[nq], qwts[nq], Bhat[nq*(k+1)], Dhat[nq*(k+1)]
 * (row q, column a).  Maps: emap[E*(k+1)^3] (global DOF or -1 on Dirichlet
 * DOFs), toff[N+1] and tidx[toff[N]] (E-vector positions e*(k+1)^3 + local
 * node of the entries summed into each DOF, by ascending element); any
 * pointer of these two may be NULL.  load: b (N doubles, unmasked), not NULL
 * (FEOD_EINVAL). */
feod_status feod_host_tables(const feod_ctx* ctx, double* nodes, double* qpts,
                             double* qwts, double* Bhat, double* Dhat);
feod_status feod_host_maps(const feod_ctx* ctx, int32_t* emap, int32_t* toff,
                           int32_t* tidx, int64_t* n_tidx);
feod_status feod_host_load(const feod_ctx* ctx, double* load);

/* Release the context (not the caller's workspace). NULL is accepted. */
feod_status feod_destroy(feod_ctx* ctx);

/* Message of the last failure on ctx (or of feod_setup_mesh when ctx is
 * NULL); empty string if none.  Valid until the next call on ctx. */
const char* feod_last_error(const feod_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FEOD_H */
