/*
 * paro.h - C ABI of the MI355X (gfx950) parallel orbital-updating engine.
 *
 * The library computes the lowest N eigenpairs of the P1 finite-element
 * discretisation of  -1/2 Laplace u + V u = lambda u  on a box with
 * homogeneous Dirichlet data, by the parallel orbital-updating (ParO)
 * iteration of Dai, Gong, Zhou and Zhu (arXiv:1405.0260):
 *   Algorithm A.1 (appendix; linear eigenproblem, a(u,v) = int A grad u .
 *   grad v + c u v with A = I/2 and c = V), with the N + m buffer orbitals of
 *   Algorithm 3.2; Step 2 (mesh adaptation) is the identity inside
 *   paro_step, and is offered separately (estimate, mark, refine,
 *   transfer) on the uniform mesh and on general bisection meshes:
 *     Step 3: for every orbital i independently solve the source problem
 *             a(u_i^{n+1/2}, v) = lambda_i^n (u_i^n, v) for all v,
 *     Step 4: Rayleigh-Ritz on span{u_i^{n+1/2}} giving (lambda_i^{n+1},
 *             u_i^{n+1}) with (u_i, u_j) = delta_ij.
 *
 * Conventions for every entry point
 *   - Return value: PARO_OK (0) or a negative PARO_E* code; nothing aborts
 *     and no C++ exception crosses the ABI.  paro_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *     h_* are host pointers.  The caller owns every buffer it passes; inputs
 *     are only read during the call (asynchronously on `stream` for device
 *     inputs of asynchronous calls: keep them alive until the stream has
 *     reached the call).
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).
 *   - Dofs: the interior vertices (i, j, k), 1 <= i <= nx-1 (likewise j, k),
 *     numbered d = (i-1) + (nx-1)((j-1) + (ny-1)(k-1)) (x fastest).
 *   - Orbital blocks are row-major n_dof x Nt (orbital index fastest), FP64,
 *     where Nt = N + m.  lambda arrays hold Nt FP64 values, ascending.
 *   - The library never allocates device memory after paro_assemble: all
 *     device state lives in the caller's workspace.
 */
#ifndef PARO_H
#define PARO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PARO_OK = 0,
  PARO_EINVAL = -1,     /* bad argument: shape, null pointer, non-finite V  */
  PARO_ENOMEM = -2,     /* workspace smaller than paro_query reports        */
  PARO_ENOTSPD = -3,    /* CG breakdown p^T A p <= 0 (shift above lambda_1) */
  PARO_ESINGULAR = -4,  /* Gram matrix W^T M W not positive definite        */
  PARO_ENOCONV = -5,    /* iteration cap reached; outputs/report still set  */
  PARO_EDEVICE = -6     /* a HIP runtime call failed                        */
};

enum { PARO_FP64 = 0, PARO_FP32_INNER = 1 };
enum { PARO_NT_MAX = 64 };  /* largest N + m */

/* Uniform Kuhn mesh: [lo, hi] cut into nx * ny * nz cubes, each split into
 * the six tetrahedra sharing the main diagonal (0,0,0)-(1,1,1)
 * (Sec. 2: conforming shape-regular tetrahedral mesh, P1 space S^{h,1}_0). */
typedef struct paro_box {
  int32_t nx, ny, nz;     /* cells per axis, each >= 2 */
  double lo[3], hi[3];
} paro_box_t;

typedef struct paro_opts {
  int32_t N;              /* requested orbitals (Algorithm 3.1/A.1 N) >= 1  */
  int32_t m;              /* buffer orbitals (Algorithm 3.2 m) >= 0         */
  int32_t max_steps;      /* ParO iterations in paro_solve                  */
  int32_t pcg_maxit;      /* CG iteration cap per source problem per step   */
  int32_t precision;      /* PARO_FP64, or PARO_FP32_INNER: FP32 CG inside
                             FP64 iterative refinement of the source solve  */
  int32_t sigma_mode;     /* 0: sigma = min V - 1 if min V < 0 else 0;
                             1: use `sigma` below                           */
  double sigma;           /* shift s of (H - s M) w = (lambda - s) M u       */
  double lambda_tol;      /* stop: max_{i<N} |dlambda_i| / scale_i <= this  */
  double resid_tol;       /* and max_{i<N} ||H u - l M u|| / (scale ||M u||) */
  double pcg_rtol;        /* source solves: ||b - A w|| <= rtol ||b||        */
  double inner_rtol;      /* FP32 inner solves: residual reduction per pass
                             (a pass stops at 0.8 pcg_rtol ||b|| at the
                             lowest; the FP64 residual decides)          */
  double pcg_reduce;      /* source solves also stop once ||b - A w|| <=
                             pcg_reduce ||b - A x0||, x0 = u_i the warm
                             start (Algorithm A.1 Step 3 solved inexactly:
                             x0's residual is the pair's eigen-residual
                             H u_i - lambda_i M u_i, so the solve shrinks
                             it by a fixed factor); in [0, 1), 0 (the
                             default) leaves only pcg_rtol               */
} paro_opts_t;

typedef struct paro_report {
  int32_t status;         /* PARO_OK / PARO_ENOCONV / ...                   */
  int32_t steps;          /* ParO steps taken                                */
  int64_t pcg_iters;      /* CG iterations summed over steps (max over cols) */
  int64_t refinements;    /* FP64 refinement passes (FP32_INNER mode)        */
  int64_t n_dof, nnz;
  double max_dlambda;     /* last step, over the N requested pairs          */
  double max_resid;
  double sigma;
  double seconds;         /* wall time of the call                          */
  int64_t reorth;         /* projections redone after re-orthonormalising a
                             nearly dependent basis (see paro_init)         */
} paro_report_t;

typedef struct paro_problem paro_problem;   /* opaque, host memory only */

/* Fill `opts` with defaults: m = 0, max_steps = 200, pcg_maxit = 10000,
 * FP64, automatic shift, lambda_tol = 1e-12, resid_tol = 1e-8,
 * pcg_rtol = 1e-10, inner_rtol = 1e-5, pcg_reduce = 0 (source solves to
 * pcg_rtol).  N must still be set. */
void paro_default_opts(paro_opts_t* opts);

/* Sizes for a box and options, host only.  n_dof = (nx-1)(ny-1)(nz-1);
 * nnz = number of nonzeros of the 15-point Kuhn P1 pattern (the size of
 * the CSR copy paro_export_csr writes);
 * workspace_bytes = device memory paro_assemble needs (the whole resident
 * footprint of the problem: stencil-order matrices, a copy of the nodal
 * potential for the matrix-free SpMM, solver blocks, reductions; no CSR
 * copy).
 * Any output pointer may be NULL. */
int paro_query(const paro_box_t* box, const paro_opts_t* opts,
               int64_t* n_dof, int64_t* nnz, size_t* workspace_bytes);

/* Assemble the source-problem operator on the device (Sec. 2 finite
 * elements; eq. (eq-operator-A) with the potential fixed):
 *   A_s = K/2 + M_V - s M (FP64, and an FP32 copy in PARO_FP32_INNER
 *   mode), M (FP64), the inverse of the diagonal of A_s,
 * with K the P1 stiffness, M the consistent mass and M_V the mass weighted
 * by the nodal interpolant of V, integrated exactly.  Storage is stencil
 * order, not CSR: on the uniform Kuhn mesh every interior row couples to
 * the same 15 neighbour offsets (the row itself, the 6 axis neighbours,
 * the 6 face diagonals +-(1,1,0), +-(1,0,1), +-(0,1,1) and the 2 body
 * diagonals +-(1,1,1)), so a matrix is 15 arrays of n_dof coefficients
 * (coefficient s of row r at [s][r], 0 where the neighbour lies outside
 * the box) and needs no column indices or row pointers.  A CSR copy is
 * made only on request (paro_export_csr).  On the uniform mesh K and M
 * are the same in every row; a row of M_V is a fixed linear function of the
 * potential at the row's 15 stencil vertices (weights in units of vol/60,
 * derived from the exact integrals of products of three barycentric
 * coordinates), which is how the coefficients are evaluated.
 *   d_V: (nx+1)(ny+1)(nz+1) nodal potential values, x fastest, all vertices
 *        including the boundary (device pointer, FP64; read during the
 *        call and copied into the workspace).
 *   d_workspace/bytes: caller-owned device memory of at least
 *        paro_query's workspace_bytes, 256-byte aligned; it must outlive the
 *        problem.  The problem keeps pointers into it.
 * Synchronises `stream` once (to read the shift back).  *out receives a
 * host-side handle, freed by paro_destroy.
 * Errors: PARO_EINVAL (nx < 2, Nt > PARO_NT_MAX, Nt > n_dof, non-finite V),
 * PARO_ENOMEM, PARO_EDEVICE. */
int paro_assemble(const paro_box_t* box, const double* d_V,
                  const paro_opts_t* opts, void* d_workspace, size_t bytes,
                  void* stream, paro_problem** out);

/* Step 1 of Algorithm A.1: from arbitrary linearly independent orbitals
 * d_U0 (n_dof x Nt) form the Rayleigh-Ritz pairs of their span, which are
 * M-orthonormal, into d_lambda (Nt) and d_U (n_dof x Nt).  d_U0 may equal
 * d_U.  Asynchronous on `stream`, so it neither reads nor repairs a failed
 * projection: when the Cholesky factorisation of U0^T M U0 fails, d_U
 * holds U0 and the problem's device status flag is set.  paro_solve,
 * paro_batch_solve and the server run Step 1 synchronously instead: a
 * start block whose Gram matrix fails its factorisation is first
 * re-orthonormalised by one shifted Cholesky-QR pass (W <- W L^{-T},
 * L L^T = W^T M W + s I, s a rounding-level shift, Fukaya et al., SIAM
 * J. Sci. Comput. 2020) and projected again; PARO_ESINGULAR only if that
 * fails too (columns dependent to rounding level).
 * Errors: PARO_EINVAL. */
int paro_init(paro_problem* p, const double* d_U0, double* d_lambda,
              double* d_U, void* stream);

/* One ParO iteration, Steps 3 and 4 (eq. (alg-bvp), (alg-evp)), in place:
 * reads (lambda^n, U^n) from d_lambda / d_U and overwrites them with
 * (lambda^{n+1}, U^{n+1}).  The Nt source problems
 *   (H - s M) w_i = (lambda_i - s) M u_i,   w_i^0 = u_i
 * are solved by Jacobi-preconditioned CG (one pass over the stencil
 * coefficients per CG iteration serves all Nt columns; each column keeps
 * its own alpha, beta and stopping test) to ||r_i|| <= pcg_rtol ||b_i||,
 * then Rayleigh-Ritz on span W.  A pure function of (lambda, U) and the problem.
 * If `report` is NULL the call is asynchronous on `stream` except for the
 * CG loop's convergence polling (one 4-byte read every few iterations);
 * otherwise it synchronises and fills `report` for this step, and a
 * projection whose Gram matrix W^T M W fails its Cholesky factorisation
 * is retried once after the shifted Cholesky-QR re-orthonormalisation of
 * W described at paro_init (report->status PARO_ESINGULAR if the retry
 * fails as well). */
int paro_step(paro_problem* p, double* d_lambda, double* d_U, void* stream,
              paro_report_t* report);

/* Whole solve: paro_init from d_U0, then ParO steps until both tolerances
 * hold for the N requested pairs or opts.max_steps steps were taken.
 * d_lambda (Nt) and d_U (n_dof x Nt) receive the final Ritz pairs (the
 * first N are the answer).  Returns PARO_OK, or PARO_ENOCONV if max_steps
 * was reached first (outputs and report are still filled).  Synchronous.
 * Its steps are paro_step's, except that each takes M u and H u from the
 * previous step's rotation (which stores them in the workspace) instead
 * of applying the operators again, which a public paro_step cannot do
 * since the caller may change U between calls; the results agree up to
 * rounding.  paro_batch_solve and the server do the same. */
int paro_solve(paro_problem* p, const double* d_U0, double* d_lambda,
               double* d_U, void* stream, paro_report_t* report);

/* Release the host handle (the workspace stays the caller's). */
void paro_destroy(paro_problem* p);

/* ---------------------------------------------------------------------
 * Batches: many independent problems advanced by the same launches.
 * Every kernel of a batched call serves all `count` problems at once
 * (each problem owns a share of the grid proportional to its work), so
 * uneven problems (different meshes, N, m, potentials) fill the GPU
 * together.  Each problem's arithmetic, and so its result, is bitwise the
 * same as when it runs alone.  All problems of a call must use the same
 * precision.  The caller passes device memory for the launch table:
 * d_batch_ws of at least paro_batch_workspace_bytes(count) bytes,
 * 256-byte aligned (it may be reused by later calls on the same stream).
 * Arrays of pointers are host arrays of `count` device pointers.
 * --------------------------------------------------------------------- */
enum { PARO_BATCH_MAX = 1024 };

size_t paro_batch_workspace_bytes(int32_t count);

/* Step 1 for every problem (see paro_init). */
int paro_batch_init(paro_problem* const* probs, int32_t count,
                    const double* const* d_U0, double* const* d_lambda,
                    double* const* d_U, void* d_batch_ws, size_t bytes,
                    void* stream);

/* One ParO step (Steps 3 and 4, see paro_step) for every problem.
 * reports: host array of `count` reports (NULL: no per-problem report and
 * no synchronisation beyond the CG polls).  Returns PARO_OK unless a
 * launch failed; per-problem failures are in reports[i].status. */
int paro_batch_step(paro_problem* const* probs, int32_t count,
                    double* const* d_lambda, double* const* d_U,
                    void* d_batch_ws, size_t bytes, void* stream,
                    paro_report_t* reports);

/* Whole solves of every problem (see paro_solve): problems that meet
 * their tolerances leave the batch, the others keep stepping until their
 * own max_steps.  reports (count, required) receive each problem's
 * summary; the return value is PARO_OK if every problem converged, else
 * the first non-OK status. */
int paro_batch_solve(paro_problem* const* probs, int32_t count,
                     const double* const* d_U0, double* const* d_lambda,
                     double* const* d_U, void* d_batch_ws, size_t bytes,
                     void* stream, paro_report_t* reports);

/* ---------------------------------------------------------------------
 * Kohn-Sham outer iteration (Sec. 2, eqs. (eq-ks), (weak-ks),
 * (eq-operator-A); Algorithm 3.1).  The problem's potential becomes the
 * effective potential V_ext + V_H(rho) + v_x(rho) of the mixed density
 * rho = occupancy * sum_{i<=N} u_i^2 (interior vertices), V_H from the P1
 * Poisson problem -Lap V_H = 4 pi rho with V_H = 0 on the boundary, i.e.
 * K V_H = 4 pi M rho (solved directly by the 3-D discrete sine transform,
 * which diagonalises the P1 stiffness matrix of the uniform box grid, or
 * by the library's Jacobi-PCG when poisson_maxit > 0), v_x the Slater
 * exchange -(3 rho/pi)^(1/3).
 * Outer iteration n: density of U^(n); rho_in = that density at n = 0,
 * else (1 - mixing) rho_in + mixing * density (or, with kerker_q0 > 0,
 * rho_in + mixing * the Kerker-filtered residual); V_eff; values-only
 * re-assembly (shift recomputed unless sigma_mode = 1); one ParO step.
 * --------------------------------------------------------------------- */
typedef struct paro_ks_opts {
  int32_t max_iter;       /* outer iterations at most                    */
  int32_t poisson_maxit;  /* 0: direct Hartree solve (default); > 0: CG
                             of the Hartree solve, capped at this        */
  double mixing;          /* linear density mixing, (0, 1]               */
  double occupancy;       /* electrons per orbital (2: spin-unpolarised) */
  double scf_tol;         /* stop when ||rho_out - rho_in|| / ||rho_in||
                             <= scf_tol and the problem's lambda_tol and
                             resid_tol hold for the step                  */
  double poisson_rtol;    /* relative CG tolerance (CG Hartree only)     */
  double kerker_q0;       /* 0: linear mixing rho_in += mixing (rho_out -
                             rho_in); > 0: the residual is first filtered
                             by (K + q0^2 vol I)^-1 K (K the P1 stiffness,
                             vol the cell volume), Kerker's q^2 / (q^2 +
                             q0^2) on the grid, which damps long-wavelength
                             charge sloshing; applied in the sine basis     */
} paro_ks_opts_t;

typedef struct paro_ks_report {
  int32_t status;         /* PARO_OK, PARO_ENOCONV (max_iter), or error  */
  int32_t iterations;
  int64_t paro_pcg_iters; /* CG iterations of the ParO steps              */
  int64_t poisson_iters;  /* CG iterations of the Hartree solves (0 when
                             solved directly)                            */
  double residual;        /* last density residual                       */
  double max_dlambda, max_resid, sigma;  /* of the last ParO step         */
  double seconds;
} paro_ks_report_t;

void paro_ks_default_opts(paro_ks_opts_t* opts);

/* Device workspace of paro_ks_solve for a box (Poisson operator, densities,
 * potentials). */
int paro_ks_query(const paro_box_t* box, size_t* workspace_bytes);

/* Values-only re-assembly of a problem for a new nodal potential d_V (all
 * (nx+1)(ny+1)(nz+1) vertices); the shift is recomputed as at assembly
 * unless opts.sigma_mode = 1.  Synchronous (reads the potential's range). */
int paro_update_potential(paro_problem* p, const double* d_V, void* stream);

/* The problem's current shift. */
double paro_sigma(const paro_problem* p);

/* Self-consistent iteration from the start block d_U0 (n_dof x (N + m));
 * d_Vext: the external potential at all vertices.  Outputs as paro_solve;
 * d_rho (n_dof, nullable) receives the last input density; h_history
 * (host, max_iter values, nullable) the density residual of every outer
 * iteration (0 for the first, which has none).  Synchronous.
 * Returns PARO_OK when converged, PARO_ENOCONV at max_iter (outputs and
 * report filled). */
int paro_ks_solve(paro_problem* p, const double* d_Vext,
                  const paro_ks_opts_t* opts, void* d_ks_ws, size_t bytes,
                  const double* d_U0, double* d_lambda, double* d_U,
                  double* d_rho, double* h_history, void* stream,
                  paro_ks_report_t* report);

/* ---------------------------------------------------------------------
 * Serving: a request loop with continuous batching (not in the paper).
 * Requests (box, nodal potential, options, start orbitals, all on the
 * host) queue at submit; each tick admits queued requests in arrival
 * order while a slot is free and their HBM footprint (workspace, potential,
 * orbitals, eigenvalues) fits in the caller's device arena, assembles and
 * initialises them, advances every resident problem by one ParO step in
 * one batched launch sequence, and retires the problems that met their
 * tolerances (or failed, or reached max_steps), copying their eigenpairs
 * to the host buffers given at submit and returning the arena space.  A
 * problem's arithmetic is the same whatever else is resident, so each
 * result equals the one of paro_solve on the same inputs, bitwise.
 * --------------------------------------------------------------------- */
typedef struct paro_server paro_server;     /* opaque, host memory only */

typedef struct paro_server_stats {
  int32_t queued;           /* submitted, not yet stepping (waiting, or
                               being uploaded and assembled)            */
  int32_t active;           /* resident on the device                     */
  int64_t done;             /* retired so far                             */
  size_t arena_used;        /* bytes of the arena held by requests        */
  size_t arena_bytes;
  int64_t ticks;
} paro_server_stats_t;

/* d_arena: device memory the server sub-allocates (256-byte aligned; the
 * caller keeps it alive until paro_server_destroy).  max_active: most
 * problems resident at once (1..PARO_BATCH_MAX).  stream: the steps run
 * on it.  Admitted requests are uploaded and assembled by a worker thread
 * of the server on a stream of its own (default priority), while ticks
 * step the resident problems; a request's first step waits for its
 * admission through an event, so no tick waits for an assembly unless
 * nothing else is resident. */
int paro_server_create(void* d_arena, size_t arena_bytes, int32_t max_active,
                       void* stream, paro_server** out);

/* Queue a request.  h_V ((nx+1)(ny+1)(nz+1) values) and h_U0 (n_dof x
 * (N + m), row-major) are copied at once; h_lambda (N + m) and h_U (n_dof
 * x (N + m)) receive the result when the request retires and must stay
 * valid until then.  PARO_ENOMEM if the request could never fit in the
 * arena.  *id identifies the request. */
int paro_server_submit(paro_server* s, const paro_box_t* box,
                       const double* h_V, const paro_opts_t* opts,
                       const double* h_U0, double* h_lambda, double* h_U,
                       int64_t* id);

/* One scheduling round: hand queued requests (arrival order, while a
 * slot is free and their block fits) to the admission worker, take Step 1
 * of the requests it has assembled, one batched ParO step of every
 * resident problem, retire.  Writes up to max_done ids of retired, not yet
 * returned requests to done_ids and their number to *n_done (the rest are
 * returned by later ticks).  Synchronous.  Per-request failures
 * (including a request that cannot be assembled, or a start block that
 * stays dependent) do not fail the tick; they are in the request's report.
 * A device error of a batched call fails every resident request with that
 * code (they retire, release their arena space and are returned as done)
 * and is returned. */
int paro_server_tick(paro_server* s, int64_t* done_ids, int32_t max_done,
                     int32_t* n_done, paro_server_stats_t* stats);

/* Report of a retired request (status, steps, CG iterations, ...). */
int paro_server_report(paro_server* s, int64_t id, paro_report_t* report);

/* Release the server (resident problems are dropped; the arena stays the
 * caller's). */
void paro_server_destroy(paro_server* s);

/* Polls and step reports reach the host through a small pinned host
 * buffer per calling thread (64 KB, hipHostMalloc'd on first use and kept
 * until the process ends) that the device writes directly. */

/* ---------------------------------------------------------------------
 * Step 2 on the uniform Kuhn mesh (Sec. 2, adaptive finite element
 * approximation: Solve -> Estimate -> Mark -> Refine; Algorithm 3.1
 * Step 2).  Elements: cell c (x fastest over nx * ny * nz cells) holds six
 * Kuhn elements q = 0..5, one per permutation p of the axes in
 * lexicographic order, vertices c, c + e_p0, c + e_p0 + e_p1, c + (1,1,1);
 * element index q * (nx ny nz) + c.
 * --------------------------------------------------------------------- */
enum { PARO_MARK_DORFLER = 0, PARO_MARK_MAXIMUM = 1 };

/* Number of elements of the box's Kuhn mesh, 6 nx ny nz (0 if invalid). */
int64_t paro_elements(const paro_box_t* box);

/* Estimate: the residual a posteriori indicator of the first nreq columns
 * of d_U (n_dof x ncols row-major, FP64, device) with eigenvalues
 * d_lambda, for -1/2 Lap u + V u = lambda u (d_V: nodal potential at all
 * vertices):
 *   eta_T^2 = sum_i h_T^2 ||lambda_i u_i - V_h u_i||^2_T
 *           + 1/2 sum_{F interior face of T} h_F ||[1/2 grad u_i . n_F]||^2_F
 * (h_T, h_F longest edges; the element term integrated exactly), one
 * value per element into d_eta (paro_elements doubles).  The paper names
 * the loop but not the estimator; this is the usual residual indicator.
 * Asynchronous.  PARO_EINVAL on bad shapes (1 <= nreq <= ncols <= 64). */
int paro_estimate(const paro_box_t* box, const double* d_V,
                  const double* d_lambda, const double* d_U, int32_t ncols,
                  int32_t nreq, double* d_eta, void* stream);

/* Mark: d_marked[k] (uint8, count) = 1 for the marked elements.
 * PARO_MARK_DORFLER, eq. (dorfler-strategy): a smallest set whose sum of
 * eta^2 reaches theta times the total -- every element above a threshold
 * and, lowest indices first, as many equal to it as needed.
 * PARO_MARK_MAXIMUM, eq. (maximum-strategy): eta >= theta max eta.
 * 0 < theta <= 1.  d_ws: device scratch of paro_mark_workspace_bytes(),
 * 256-byte aligned.  Synchronous (the threshold search reads sums back);
 * *h_nmarked (nullable) receives the count. */
size_t paro_mark_workspace_bytes(void);
int paro_mark(const double* d_eta, int64_t count, double theta,
              int32_t strategy, uint8_t* d_marked, int64_t* h_nmarked,
              void* d_ws, size_t bytes, void* stream);

/* Refine every element and carry the orbitals over: d_Uc (n_dof x ncols
 * of the box's mesh) -> d_Uf (n_dof x ncols of the same box with 2 nx,
 * 2 ny, 2 nz cells, whose Kuhn elements refine the coarse ones) by P1
 * interpolation: every fine vertex is a coarse vertex or the midpoint of
 * a coarse edge (axis, face diagonal or main diagonal) and takes the mean
 * of its ends.  Asynchronous; 1 <= ncols <= 64. */
int paro_prolong(const paro_box_t* coarse, const double* d_Uc, double* d_Uf,
                 int32_t ncols, void* stream);

/* ---------------------------------------------------------------------
 * Step 2 with local refinement: general bisection meshes of a box (Sec. 2
 * adaptive loop; Algorithm 3.1 Step 2 builds T_{n+1} from T_n).  The
 * paper leaves the refinement to the literature; the library uses
 * Maubach's tagged bisection: an element is an ordered vertex list
 * (x0, x1, x2, x3) with a tag k in {1, 2, 3}; it is cut at the midpoint z
 * of its refinement edge (x0, xk) into (x0, .., x_{k-1}, z, x_{k+1}, ..,
 * x3) and (x1, .., xk, z, x_{k+1}, .., x3), both tagged k - 1 (3 after
 * 1).  Before an element is cut at an edge, every element around the edge
 * with another refinement edge is bisected first (recursively), and then
 * all elements around it are cut together, so the mesh stays conforming.
 * The uniform Kuhn mesh (elements c, c + e_p0, c + e_p0 + e_p1,
 * c + (1,1,1), tag 3, numbered as for paro_elements) is the usual start.
 * Vertices on the box boundary carry the Dirichlet data; the interior
 * vertices in vertex order are the dofs.  A mesh is a host object;
 * problems assembled on it are solved by paro_init / paro_step /
 * paro_solve and the batch and cluster calls like box problems, in
 * PARO_FP64 (the operator is stored in CSR: no stencil, no FP32 copy).
 * --------------------------------------------------------------------- */
typedef struct paro_mesh paro_mesh;  /* opaque, host memory only */

/* The uniform Kuhn mesh of the box as a bisection mesh.  PARO_EINVAL for
 * a bad box or one beyond 32-bit element indices. */
int paro_mesh_create(const paro_box_t* box, paro_mesh** out);

/* A mesh from host arrays: X (nv x 3 coordinates), tets (ne x 4 ordered
 * vertex lists), tags (ne, in 1..3), parents (nv x 2: the ends of the
 * edge a vertex halves, each older than the vertex, or -1, -1; NULL: all
 * -1).  box: lo and hi of the domain (its cell counts are not used).
 * The arrays are copied.  PARO_EINVAL for indices out of range, repeated
 * corners, tags outside 1..3 or non-finite coordinates. */
int paro_mesh_from_arrays(const paro_box_t* box, int64_t nv, const double* X,
                          int64_t ne, const int32_t* tets,
                          const int32_t* tags, const int32_t* parents,
                          paro_mesh** out);

/* Sizes (any pointer may be NULL). */
int paro_mesh_info(const paro_mesh* m, int64_t* nv, int64_t* ne,
                   int64_t* n_dof);

/* Copies of the mesh into host buffers of the sizes paro_mesh_info gives
 * (any pointer may be NULL): X (nv x 3), tets (ne x 4), tags (ne),
 * parents (nv x 2), dof (nv: the dof of a vertex, -1 on the boundary). */
int paro_mesh_arrays(const paro_mesh* m, double* X, int32_t* tets,
                     int32_t* tags, int32_t* parents, int32_t* dof);

/* Refine: bisect every element with marked[e] != 0 (host array of ne
 * bytes, e.g. paro_mark's output copied to the host) at least once, with
 * the conforming closure, into a new mesh *out (m is unchanged).  Old
 * vertices keep their indices; new vertices follow in creation order with
 * their parents; surviving elements keep their order, new ones follow.
 * Host only. */
int paro_mesh_refine(const paro_mesh* m, const uint8_t* marked,
                     paro_mesh** out);

void paro_mesh_destroy(paro_mesh* m);

/* Sizes of a problem on the mesh (as paro_query): n_dof, nnz of the CSR
 * operator, and the workspace of paro_mesh_assemble.  Host only; builds
 * the pattern, so it costs about as much as the host part of assembly.
 * PARO_EINVAL also for a precision other than PARO_FP64. */
int paro_mesh_query(const paro_mesh* m, const paro_opts_t* opts,
                    int64_t* n_dof, int64_t* nnz, size_t* workspace_bytes);

/* Assemble on the mesh (as paro_assemble): d_V is the nodal potential at
 * every vertex (nv doubles, device; copied), the operator A_s = K/2 + M_V
 * - s M and M go to CSR in the workspace (values gathered row by row over
 * the incident elements in a fixed order: no atomics), together with the
 * mesh tables that paro_mesh_estimate reads.  Synchronises `stream` once.
 * The problem serves paro_init / paro_step / paro_solve, the batch calls,
 * paro_set_clusters, paro_spmm, paro_gram, paro_pcg and paro_export_csr;
 * paro_update_potential and paro_set_nonlocal return PARO_EINVAL. */
int paro_mesh_assemble(const paro_mesh* m, const double* d_V,
                       const paro_opts_t* opts, void* d_workspace,
                       size_t bytes, void* stream, paro_problem** out);

/* Estimate on a mesh problem: the indicator of paro_estimate for every
 * element of the mesh it was assembled on (d_eta: ne doubles), from the
 * first nreq columns of d_U (n_dof x ncols) with eigenvalues d_lambda and
 * the problem's nodal potential.  Asynchronous.  Mark with paro_mark. */
int paro_mesh_estimate(const paro_problem* p, const double* d_lambda,
                       const double* d_U, int32_t ncols, int32_t nreq,
                       double* d_eta, void* stream);

/* Carry orbitals to a refined mesh by P1 interpolation (exact: the coarse
 * space lies in the fine one): fine must come from coarse by
 * paro_mesh_refine (one call or several: old vertices keep their indices)
 * -- checked on the coordinates.  d_Uc (coarse n_dof x ncols) -> d_Uf
 * (fine n_dof x ncols): old dofs keep their values, a new vertex takes the
 * mean of the two ends of the edge it halves (0 on the boundary),
 * generation by generation.  d_ws: device scratch of
 * paro_mesh_prolong_workspace_bytes(coarse, fine), 256-byte aligned.
 * Synchronises `stream` once (the host tables it uploads). */
size_t paro_mesh_prolong_workspace_bytes(const paro_mesh* coarse,
                                         const paro_mesh* fine);
int paro_mesh_prolong(const paro_mesh* coarse, const paro_mesh* fine,
                      const double* d_Uc, double* d_Uf, int32_t ncols,
                      void* d_ws, size_t bytes, void* stream);

/* Message for the last failing call on this thread (never NULL). */
const char* paro_last_error(void);
const char* paro_strerror(int status);

/* ---------------------------------------------------------------------
 * Component entry points (each runs one kernel stage of the step above;
 * used for kernel-level checking and measurement).  All asynchronous.
 * --------------------------------------------------------------------- */

/* Write the assembled A_s and M in CSR form (rowptr int32[n+1],
 * col int32[nnz] ascending within a row, values FP64[nnz]) into caller
 * device buffers, built from the stencil-order arrays by one kernel (the
 * workspace holds no CSR copy); any of the four may be NULL.  Also the
 * shift (h_sigma, nullable).  Asynchronous on `stream`. */
int paro_export_csr(paro_problem* p, int32_t* d_rowptr, int32_t* d_col,
                    double* d_valA, double* d_valM, double* h_sigma,
                    void* stream);

/* Y = A_s X (which = 0), Y = M X (which = 1) or Y = H X = A_s X + s M X
 * (which = 2) for an n_dof x ncols row-major FP64 block, 1 <= ncols <= 64. */
int paro_spmm(paro_problem* p, int which, const double* d_X, double* d_Y,
              int ncols, void* stream);

/* G = W^T Y (ncols x ncols, row-major) for n_dof x ncols blocks W, Y,
 * on FP64 matrix cores; result in device memory d_G. */
int paro_gram(paro_problem* p, const double* d_W, const double* d_Y,
              double* d_G, int ncols, void* stream);

/* Allocation-free Gram, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): G = W^T Y (ncols x ncols, row-major, device d_G) for
 * n x ncols row-major FP64 device blocks W and Y, on FP64 matrix cores,
 * with the same kernels, segments and summation order as paro_gram on a
 * problem of n dofs and N + m = ncols (so the same bits).  Needs no
 * problem and no workspace: its scratch (a launch descriptor and the
 * first-stage tile partials, 16 MiB + 1 KiB) is a static device array
 * that every device holds for the life of the process.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library call)
 * and is asynchronous on `stream`.  Every call on a device shares that
 * device's scratch: calls that overlap on one device (other streams,
 * other threads) race and must be ordered by the caller.  The scratch
 * keeps the last call's contents; each call overwrites all of it that it
 * reads, so nothing needs clearing.
 * Errors: PARO_EINVAL (NULL pointer, ncols outside 1..64, n outside
 * 1..2^31-1: the scratch is sized for 64 columns), PARO_EDEVICE. */
int paro_gram_noalloc(const double* d_W, const double* d_Y, double* d_G,
                      int64_t n, int ncols, void* stream);

/* Dense generalised symmetric eigenproblem A c = theta B c, B positive
 * definite, n <= 64, on one workgroup: Cholesky B = L L^T, cyclic Jacobi
 * on L^{-1} A L^{-T}, theta ascending, C = L^{-T} Y (C^T B C = I), each
 * column's largest-magnitude entry made positive.  Device pointers,
 * row-major.  d_info (int32) receives 0, or k+1 if the k-th pivot of B
 * was not positive. */
int paro_small_geneig(const double* d_A, const double* d_B, int n,
                      double* d_theta, double* d_C, int32_t* d_info,
                      void* stream);

/* Solve (H - s M) X = B column by column with the step's block Jacobi-PCG
 * (FP64 or the FP32-inner refinement per opts.precision) from the start
 * X (in/out).  h_iters (ncols int32, may be NULL) receives each column's
 * CG iteration count.  Synchronous. */
int paro_pcg(paro_problem* p, const double* d_B, double* d_X, int ncols,
             int32_t* h_iters, void* stream);

/* ---------------------------------------------------------------------
 * Measurement.  With timing on, every kernel launch of the problem gets a
 * pair of HIP events stamped by the dispatch itself (kernel execution
 * only, no launch gaps) and its duration is added to the stage it belongs
 * to; off by default (no events are created).
 * --------------------------------------------------------------------- */
enum {
  PARO_ST_CG_SPMM = 0,   /* CG: Q = A P with p.q partials              */
  PARO_ST_CG_RUPD = 1,   /* CG: alpha; r -= alpha q, z, r.z, r.r       */
  PARO_ST_CG_PUPD = 2,   /* CG: beta, stop test; x += alpha p,
                            p = z + beta p                             */
  PARO_ST_START = 3,     /* source-problem start (b, r0, p0)           */
  PARO_ST_REFINE = 4,    /* FP64 residual + correction update          */
  PARO_ST_RR_SPMM = 5,   /* Rayleigh-Ritz: H W and M W                 */
  PARO_ST_GRAM = 6,      /* W^T H W, W^T M W on matrix cores           */
  PARO_ST_SMALL = 7,     /* small generalised eigensolve (one block)   */
  PARO_ST_ROTATE = 8,    /* U = W C with residual norms                */
  PARO_ST_CG_FINAL = 9,  /* unused: alpha and beta are formed inside
                            the update kernels                         */
  PARO_ST_NUM = 10
};

typedef struct paro_timing {
  int64_t launches[PARO_ST_NUM];
  double ms[PARO_ST_NUM];         /* summed kernel durations            */
  int64_t cg_iters;               /* CG iterations executed on device   */
  int64_t cg_col_iters;           /* sum over CG iterations of the
                                     number of active columns           */
} paro_timing_t;

/* CG iterations of single-problem calls run as captured HIP graphs
 * (instantiated once per launch shape and replayed) when on, or kernel by
 * kernel (the default).  Process-wide.  Timing mode always launches
 * kernel by kernel. */
void paro_set_graphs(int on);

/* Persistent CG (off by default): every CG iteration of a call's problems
 * (one problem or a whole batch) runs in one cooperative launch whose
 * phases -- SpMM, alpha, r-update, beta, p-update -- are separated by
 * grid-wide barriers instead of kernel boundaries, and which exits by
 * itself once every column has converged.  Results are bitwise those of
 * the kernel-by-kernel path.  When the grid cannot be co-resident (more
 * than 96 problems, or a device with fewer CUs) the call falls back to
 * kernel-by-kernel launches.  Process-wide. */
void paro_set_persistent(int on);

/* Matrix-free CG SpMM on uniform box problems (on by default): the
 * z-marching SpMM forms each row's 15 stencil coefficients from the nodal
 * potential at its stencil vertices (Sec. 2: the potential part of the P1
 * operator on a uniform Kuhn mesh is linear in those values, the rest is
 * the same for every row) instead of reading the 15 stored ones, with the
 * function the assembly stores them with (FP32 inner solves: rounded from
 * FP64, as the stored FP32 stencil is): results are bitwise those of the
 * stored-coefficient form, which off (0) selects.  Box problems keep a
 * copy of the potential in their workspace for it (paro_query's size
 * includes it).  Process-wide. */
void paro_set_matrix_free(int on);

/* Cluster-wise projection, the eigenvalue-separation variant of Sec. 3
 * (remarks after Algorithm 3.1): the N + m columns form `count`
 * consecutive clusters of sizes[0..count) (each >= 1, summing to N + m),
 * and every following Rayleigh-Ritz step (paro_step, paro_solve, batch
 * steps) projects each cluster's updated orbitals on its own span: the
 * Gram blocks coupling different clusters are dropped, the small problem
 * separates into one problem per cluster, and Ritz pairs are ordered
 * within each cluster, which keeps its columns.  The paper assumes initial
 * data close to each cluster's eigenspace.  In floating point, components
 * along lower eigenvectors grow (inverse iteration amplifies them by
 * (lambda_i - s) / (lambda_j - s) per step), so clustered steps must be
 * interleaved with full ones; count = 0 restores the full projection.
 * Synchronises `stream`; EINVAL on bad sizes. */
int paro_set_clusters(paro_problem* p, const int32_t* sizes, int32_t count,
                      void* stream);

/* Nonlocal pseudopotential term (Sec. 2, the pseudopotential model):
 * V_nl u = sum_j (u, zeta_j) zeta_j with k projector functions zeta_j,
 * given by their values at the interior vertices, d_zeta n x k row-major
 * (device).  Its Galerkin matrix is Z Z^T with Z = M zeta, which the
 * library forms in the caller's workspace d_ws (size from
 * paro_nonlocal_query, 256-byte aligned, kept alive and unmodified while
 * the term is set); the Hamiltonian of every later source solve and
 * projection is H + Z Z^T (the Jacobi preconditioner keeps the local
 * diagonal; the shift stays valid since Z Z^T is positive semidefinite).
 * FP64 precision only (EINVAL otherwise); 1 <= k <= 32; k = 0 removes the
 * term.  Asynchronous on `stream`.  The component calls (paro_spmm,
 * paro_pcg) and the persistent CG apply the local operator only; with the
 * term set, CG runs kernel by kernel. */
int paro_nonlocal_query(const paro_problem* p, int32_t k, size_t* bytes);
int paro_set_nonlocal(paro_problem* p, const double* d_zeta, int32_t k,
                      void* d_ws, size_t bytes, void* stream);

/* CG SpMM forms.  Meshes up to 2048 tiles of 248 rows sweep the rows in
 * tile order.  Larger meshes whose planes span at most 256 tiles march
 * along z instead: a unit owns a tile of one plane, a range of planes and
 * a group of column chunks, keeps the neighbour lines of the previous
 * plane in registers and loads only the new ones, so each value of the
 * search direction is read from memory about once per iteration instead
 * of three times; p.q partials are kept per (plane range, tile).
 *
 * Autotuner (on by default): at assembly, the CG SpMM of each new problem
 * shape (grid, N + m, precision) is timed for every variant -- the
 * z-marching SpMM with 1, 2 or 4 chunks per unit (variants 0, 1, 2; the
 * matrix-free FP64 form groups its chunks itself and has one), the
 * row sweep with one (variant 0) -- each with the full and the halved
 * real block count, and the fastest is kept for the shape for the rest of
 * the process.  The choice never changes the arithmetic or the results
 * (the reductions run over partial sums fixed by the mesh).
 * paro_set_autotune(0) keeps the defaults; paro_tuned reports a problem's
 * variant (-1 untuned) and real block count. */
void paro_set_autotune(int on);
int paro_tuned(const paro_problem* p, int32_t* variant, int32_t* blocks);
/* Pin a problem's SpMM variant (-1 default, 0, or for a z-marching
 * problem also 1 or 2) and real block count (a multiple of 8, at most its
 * reduction segment count).  PARO_EINVAL otherwise. */
int paro_set_tuning(paro_problem* p, int32_t variant, int32_t blocks);

/* Turn per-launch event timing on (1) or off (0); clears the sums. */
int paro_set_timing(paro_problem* p, int on);
/* Synchronise the problem's last stream and return the sums so far. */
int paro_get_timing(paro_problem* p, paro_timing_t* out);

#ifdef __cplusplus
}
#endif
#endif /* PARO_H */
