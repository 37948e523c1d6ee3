// Internal declarations shared by the HIP translation units of libparo.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "paro.h"

namespace paro {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kNtMax = PARO_NT_MAX;  // largest number of columns
#ifndef PARO_GRID
#define PARO_GRID 1024
#endif
// Largest grid of the streaming kernels (= reduction segments).
constexpr int kGridMax = PARO_GRID;
constexpr int kStencil = 15;         // Kuhn P1 pattern: 15 neighbours per row
constexpr int kGridDefault = PARO_GRID;  // default grid (4 per CU)
constexpr int kGramGrid = 512;       // first-stage blocks of the Gram
// Grids a batch launch shares out among its problems (each problem gets
// at most its own single-problem grid).
constexpr int kBatchGrid = 4 * PARO_GRID;
constexpr int kBatchGramGrid = 4 * kGramGrid;
// Tile entries per Gram block for nt16 = ceil(ncols / 16): two symmetric
// results, tile pairs I <= J, 16 x 16 each.
constexpr int gram_tiles(int ncols) {
  return 2 * (((ncols + 15) / 16) * ((ncols + 15) / 16 + 1) / 2) * 256;
}

// Status bits raised by device code (ColState::status).
enum : int {
  kStNotSpd = 1,      // CG breakdown p^T A p <= 0
  kStNoConv = 2,      // CG iteration cap reached
  kStSingular = 4,    // Cholesky of W^T M W failed
  kStNonFinite = 8,   // NaN / Inf met in a reduction
  // Set by the host only, in reports it has read: the problem's basis was
  // re-orthonormalised and projected again this step.
  kStReorth = 16,
};

// Per-column scalars of the block CG, resident in device memory.  One
// problem owns one ColState; all reductions end in it.
struct ColState {
  double bb[kNtMax];      // ||b||^2 of the current (outer) system
  double rz[kNtMax];      // r . z of the current iterate (the latest)
  double alpha[kNtMax];
  double beta[kNtMax];
  double rr[kNtMax];      // ||r||^2 of the current iterate
  double tol2[kNtMax];    // stop when rr <= tol2 (inner/outer threshold)
  double rr64[kNtMax];    // FP64 residual^2 of the outer (refinement) loop
  double rzp[2][kNtMax];  // r . z entering the CG iteration of parity s
  int itp[2][kNtMax];     // iterations taken before that iteration
  int act[2][kNtMax];     // CG column active in iteration of parity s
  int oact[kNtMax];       // outer refinement still running for this column
  int iters[kNtMax];      // CG iterations taken in this step (latest)
  int n_active[2];        // number of active columns, per parity
  int n_outer;            // columns still refining
  int status;             // kSt* bits
  int maxit;              // CG cap per column (copied from opts)
  int pad[3];
  unsigned long long cg_iters;      // CG iterations that did work
  unsigned long long cg_col_iters;  // their active columns, summed
  unsigned long long cg_mark;       // cg_iters when the current solve began
};

// Step results (device), read back when a report is requested.
struct StepInfo {
  double lam_old[kNtMax];
  double dlam[kNtMax];
  double resid[kNtMax];
  double max_dlambda;     // over the N requested pairs
  double max_resid;
  int geneig_info;
  int pad[3];
};

// Reduction counters (device), one per reduction site, reset by the last
// block of each reduction.
enum { kCntSpmm = 0, kCntRupd, kCntStart, kCntGram, kCntRot, kCntRefine,
       kCntMin, kCntSpmmTest, kCntNum };

// One problem of a launch.  Every solver kernel takes a table of these
// (device memory) and serves the problem that owns its block: problem p
// owns blocks [b0, b0 + nb) of the streaming kernels and [g0, g0 + gnb) of
// the Gram's first stage (b0, nb, g0, gnb multiples of 8, so that a
// problem's blocks keep the XCD round-robin of the whole grid).
//
// Reductions are split into segments fixed by the problem alone: ns
// "virtual blocks" for the streaming kernels (ns = the problem's own grid)
// and gns for the Gram.  Real block lb of nb serves virtual blocks lb,
// lb + nb, ... (nb <= ns), so the summation order, and every result, is
// the same whatever share of the grid the problem gets in a batch.  The
// vector widths v64 / v32 (columns per thread, FP64 / FP32) are likewise
// the problem's own.
struct Desc {
  long long n, nnz;
  int ncols;              // N + m
  int nreq;               // N
  int b0, nb;
  int g0, gnb;
  int maxit;
  int have_old;           // Rayleigh-Ritz after a step (1) or at the start
  int ns, gns;            // reduction segments (virtual blocks)
  int v64, v32;           // columns per thread
  double sigma, rtol, inner_rtol;
  double reduce2;         // (pcg_reduce / rtol)^2: 0, or the floor of ||b||^2
  double s1;              // component SpMM: Y1 = A X + s1 M X
  const double* dinv;
  const float* dinv32;
  const double* diagA;    // stencil order: [kStencil][n], 0 outside the box
  const double* diagM;
  const float* diagA32;
  const double* Vb;       // uniform box: nodal potential (all vertices) and
  const double* kconst;   // stencil constants (kuhn.h layout), or null
  int mx, my, mz;         // interior vertices per axis (rows = mx my mz)
  int cg_var;             // reserved (one CG SpMM kernel): -1 or 0
  const double* U0;       // start of the source solves (x0), gathered
  const double* Bin;      // given right-hand sides, or null
  double* lam;            // Ritz values (in: previous, out: new), or null
  double* X;              // source solutions = Rayleigh-Ritz basis W
  double* Uout;           // rotated orbitals
  double* R;
  double* P;
  double* Q;
  double* B;              // stored right-hand sides (refinement), or null
  double* HU;             // H U and M U of the last rotation (row-major),
  double* MU;             // written by every rotation
  int use_hu;             // the start forms A_s U from them (U, H unchanged);
                          // 2: from them after launch_csr_dual mode 2;
                          // 3: the last rotation emitted the start state
                          // (the start kernel only resets the column state)
  int emit;               // the rotation also writes the next step's start
                          // state (x0, r0, p0 and its partials) instead of
                          // H U and M U
  int start_part;         // first partial quantity the start finaliser
                          // reads (0, or 2 after an emitting rotation)
  int start_ready;        // host only: the last rotation emitted the start
                          // state and nothing has overwritten it since
  int hu_valid;           // host only: HU, MU hold H U, M U of the last
                          // rotation
  double* Xc;             // FP64 CG iterate, chunk-major (FP64 mode only)
  double* Xm;             // mixed precision, z-marching meshes: the FP64
  int rcm;                // refinement iterate chunk-major (rcm = 1; B is
                          // then chunk-major too and X is written from Xm
                          // after the solves), or null / 0
  float* R32;             // FP32 CG vectors, chunk-major (see cm_index)
  float* P32;
  float* Q32;
  float* X32;
  int ntc;                // chunk-major tiles: ceil(n / kCmRows)
  int cgn;                // partials per column of r.z and r.r (CG)
  long long cgstride;     // ... the stride between the two quantities
  double* cgp;            // ... and where they are (part, or cpart)
  int pqn;                // partials per column of p.q (CG SpMM segments)
  int spt, spg;           // SpMM tiles, and tiles per p.q segment
  int zm;                 // z-marching CG SpMM: plane ranges (a multiple
                          // of 8), or 0 (row sweep)
  int zxy;                // ... and xy tiles of kSpmmRows rows per plane
  double* pqp;            // ... and where they are
  double* Y1;             // component SpMM / Gram operands
  double* Y2;
  double* part;
  double* gpart;
  double* Ah;
  double* Bh;
  double* C;
  double* theta;
  ColState* cs;
  StepInfo* si;
  int* geneig_info;
  const int* clus;        // cluster id per column (cluster-wise Step 4),
                          // or null (full projection)
  const double* Zp;       // nonlocal term: Z = M zeta (n x kz, row-major),
                          // or null
  int kz;                 // number of projectors (0: none)
  double* zy;             // kz x ncols: Z^T X of the current phase
  double* zpart;          // kz ncols x ntc partial sums of Z^T X
  // General (bisection) meshes: the operator as CSR over the dofs
  // (csr = 1; then diagA / diagM are unused and mx, my, mz are 0).
  int csr;
  const int32_t* rowptr;  // n + 1
  const int32_t* colidx;  // nnz, ascending within a row
  const double* valA;     // A_s = H - s M
  const double* valM;     // M
  int csr_rows;           // rows per p.q segment of the CSR CG SpMM
};

// Columns per thread of a problem with `ncols` columns: the widest vector
// that divides ncols (FP64: 2 or 1; FP32: 4, 2 or 1).
constexpr int vec64_of(int ncols) { return ncols % 2 == 0 ? 2 : 1; }
constexpr int vec32_of(int ncols) {
  return ncols % 4 == 0 ? 4 : (ncols % 2 == 0 ? 2 : 1);
}
// Rows per streaming tile.
constexpr int tile_rows(int ncols, int V) { return kBlock / (ncols / V); }

// Tiles of the CG SpMM: each wavefront computes kSpmmWaveRows rows (its
// first and last lanes hold the neighbouring rows), kSpmmRows per block.
constexpr int kSpmmWaveRows = 62;
constexpr int kSpmmRows = (kBlock / 64) * kSpmmWaveRows;
// The SpMM's p.q partials, one per (column, segment); the segments are a
// function of n alone, so a problem's sums do not depend on the launch.
// Up to kSpmmSegMax tiles a segment is one tile (pqn = spt).  Beyond, the
// tiles are cut into kSpmmSlabs contiguous slabs of C = ceil(spt /
// kSpmmSlabs) tiles (the slabs of the XCD-aware tile walk), and segment
// g = x kSpmmSlabSegs + l holds tiles x C + l, x C + l + kSpmmSlabSegs, ...
// of slab x: with one segment per block, an XCD's blocks then sweep their
// slab in one contiguous pass (their k-th tiles are neighbours), so a
// plane's stencil neighbours are still in that XCD's L2 when the next
// planes need them.  pqn <= kSpmmSegMax keeps the per-column reductions
// that read the partials at one round of loads.
constexpr int kSpmmSegMax = 2048;
constexpr int kSpmmSlabs = 8;
constexpr int kSpmmSlabSegs = 128;
__host__ __device__ constexpr long long spmm_tiles(long long n) {
  return (n + kSpmmRows - 1) / kSpmmRows;
}
// Plane ranges of the z-marching CG SpMM for an mx x my x mz grid: used
// where the row sweep would need slab segments (more than kSpmmSegMax
// tiles), with at least 384 segments (plane range, xy tile) so that one
// active chunk group still spreads over the GPU, at most kSpmmSegMax, and
// at least 3 planes per range; 0 where that is not possible (the row
// sweep serves the problem).
inline int zm_ranges(int mx, int my, int mz) {
  const long long plane = (long long)mx * my;
  const long long nxy = (plane + kSpmmRows - 1) / kSpmmRows;
  const long long tiles = (plane * mz + kSpmmRows - 1) / kSpmmRows;
  if (tiles <= kSpmmSegMax || nxy * 8 > kSpmmSegMax) return 0;
  long long nzr = 8 * ((384 + 8 * nxy - 1) / (8 * nxy));
  while (nzr * nxy > kSpmmSegMax) nzr -= 8;
  if (nzr > mz / 3) nzr = (mz / 3) / 8 * 8;
  return nzr < 8 ? 0 : (int)nzr;
}
__host__ __device__ constexpr int spmm_segments(long long n) {
  return spmm_tiles(n) <= kSpmmSegMax ? (int)spmm_tiles(n)
                                      : kSpmmSlabs * kSpmmSlabSegs;
}
// Most tiles in one segment.
__host__ __device__ constexpr int spmm_seg_tiles(long long n) {
  return spmm_tiles(n) <= kSpmmSegMax
             ? 1
             : (int)(((spmm_tiles(n) + kSpmmSlabs - 1) / kSpmmSlabs +
                      kSpmmSlabSegs - 1) /
                     kSpmmSlabSegs);
}
static_assert(kSpmmSlabs * kSpmmSlabSegs <= kSpmmSegMax, "segment count");

// Tiles of the chunk-major FP32 CG kernels: kCmRpt rows per thread.
// Element (row, c) of an FP32 CG vector with vector width V sits at
// ((c / V) n + row) V + c % V: V-column chunks, each an n x V array.
constexpr int kCmRpt = 4;
constexpr int kCmRows = kBlock * kCmRpt;
__host__ __device__ constexpr long long cm_tiles(long long n) {
  return (n + kCmRows - 1) / kCmRows;
}

// Shape of one batched launch.
struct Launch {
  Desc* d;                // device table
  int nprob;
  int blocks;             // streaming grid (sum of nb)
  int gblocks;            // Gram first-stage grid (sum of gnb)
  int maxcols;            // largest ncols
  int mincols;            // smallest ncols (largest tile)
  int nt16;               // ceil(maxcols / 16)
  int tr64, tr32;         // largest tile rows (FP64 / FP32 widths)
  int vmax64;             // widest FP64 vector of the table
  int v64u, v32u;         // common vector width of all problems, or 0
  int nt16_mixed;         // problems differ in ceil(ncols / 16)
  int maxkz;              // most nonlocal projectors of a problem (0: none)
  int seg;                // some row-sweep problem has SpMM segments of
                          // > 1 tile
  int ntile;              // some problem uses the row-sweep CG SpMM
  int zm;                 // some problem uses the z-marching CG SpMM
  int zmg;                // chunks per z-marching unit (1, 2 or 4)
  int zmf;                // the z-marching SpMM forms the coefficients
                          // from the potential (matrix-free)
  int csr;                // some problem is on a general (CSR) mesh
};

// Per-problem step summary for the host (one PollReport per problem).
struct PollReport {
  int status;
  int max_iters;
  int geneig_info;
  int pad;
  double max_dlambda;
  double max_resid;
};

struct Timing;      // host-side event timing state (api.hip)
struct GraphCache;  // captured CG launch graphs (api.hip)

struct Problem {
  paro_box_t box;
  paro_opts_t opts;
  int mx, my, mz;         // interior vertices per axis
  int64_t n, nnz;
  int Nt, N;
  double sigma;
  double h[3];
  int grid;               // persistent grid (workgroups) of the solvers
  // device memory, carved from the caller's workspace
  double* dinv;           // 1 / diag(A_s)
  float* dinv32;
  double* diagA;          // A_s, M (and FP32 A_s) in stencil order
  double* diagM;
  float* diagA32;
  double* Vb = nullptr;     // uniform box: the nodal potential at all
                            // (mx + 2)(my + 2)(mz + 2) vertices, x fastest
  double* kconst = nullptr; // ... and its stencil constants (kuhn.h):
                            // what the matrix-free SpMMs read
  double* X;              // n x Nt blocks (FP64)
  double* R;
  double* P;
  double* Q;
  double* B;              // right-hand sides (refinement mode)
  double *HU, *MU;        // H U, M U of the last rotation
  double* Xc;             // chunk-major FP64 CG iterate (FP64 mode)
  double* Xm = nullptr;   // chunk-major FP64 refinement iterate (mixed)
  float* R32;             // n x Nt blocks (FP32 inner solves, chunk-major)
  float* P32;
  float* Q32;
  float* X32;
  double* part;           // kGridMax * kNtMax * 5 reduction partials
  int* clus;              // kNtMax cluster ids (paro_set_clusters)
  bool clustered;
  const double* Zp;       // nonlocal projectors (caller's workspace)
  int kz;
  double* zy;
  double* zpart;
  double* cpart;          // FP32 CG partials: 2 Nt cm_tiles(n) (r.z, r.r),
                          // then Nt ceil(n / kBlock) (p.q)
  double* gpart;          // Gram partials: kGramGrid * gram_tiles(Nt)
  double* Ah;             // Nt x Nt
  double* Bh;
  double* C;              // Ritz coefficients, Nt x Nt
  double* theta;
  double* vmin;           // [0]: min of the nodal potential, [1]: max
  ColState* cs;
  StepInfo* si;
  unsigned* cnt;          // kCntNum reduction counters
  int* flag;              // scratch flags
  size_t ws_bytes;
  Timing* timing;         // null unless paro_set_timing(p, 1)
  GraphCache* graphs;     // CG chunk graphs of this problem (lazy)
  hipStream_t last_stream;
  int cg_predict[5];      // CG iterations of the last solve per pass slot
  Desc hd;                // host copy of the problem's descriptor
  Desc* dd;               // its device slot (workspace)
  // General meshes (csr): the operator and the mesh on the device.
  bool csr = false;
  int32_t* rowptr = nullptr;
  int32_t* colidx = nullptr;
  double* valA = nullptr;
  double* valM = nullptr;
  int32_t* inc_ptr = nullptr;  // n + 1: incident (element, corner) pairs
  int32_t* inc = nullptr;      // of each dof row, 2 ints each
  int32_t* tets = nullptr;     // ne x 4
  double* Xv = nullptr;        // nv x 3 vertex coordinates
  double* Vv = nullptr;        // nv nodal potential
  int32_t* dofmap = nullptr;   // nv: dof of a vertex, -1 on the boundary
  int32_t* nbr = nullptr;      // ne x 4: element across the face opposite
                               // corner a, -1 on the boundary
  int64_t nv = 0, ne = 0;
};

// Kernel timing (api.hip): a pair of events for one launch when timing is
// on (false otherwise), and the launch's duration added to a stage.
bool timing_pair(Timing* t, hipEvent_t* a, hipEvent_t* b);
void timing_add(Timing* t, int stage, hipEvent_t a, hipEvent_t b);

// Workspace layout: byte offsets of every region for a problem shape.
struct Layout {
  size_t rowptr, colidx, valA, valM, inc_ptr, inc, tets, Xv, Vv, dofmap,
      nbr;  // general meshes only (0 otherwise)
  size_t dinv, dinv32, diagA, diagM, diagA32, vbox, kconst;
  size_t X, R, P, Q, B, HU, MU, Xc, Xm, R32, P32, Q32, X32;
  size_t part, cpart, gpart, Ah, Bh, C, theta, vmin, cs, si, cnt,
      flag;
  size_t desc, clus;
  size_t total;
};

// Sizes of a general mesh's device arrays (make_layout's mesh regions).
struct MeshSizes {
  int64_t nv, ne, ninc;  // vertices, elements, incident (element, corner)
                         // pairs of the dof rows
};
// ms: null for the uniform stencil format, else the CSR operator and mesh
// arrays replace the stencil coefficients.
// nvbox: vertices of a uniform box problem (its potential is kept for the
// matrix-free CG SpMM), 0 for none.
Layout make_layout(int64_t n, int64_t nnz, int Nt, int precision,
                   const MeshSizes* ms = nullptr, int64_t nvbox = 0);

// A bisection mesh of a box (host): ordered elements (x0, x1, x2, x3)
// with Maubach tags, and for every vertex made by bisection the two ends
// of the edge it halves (-1, -1 for the others).  Vertices on the box
// boundary carry the Dirichlet data; the others, in vertex order, are the
// dofs.
struct MeshData {
  double lo[3], hi[3];
  std::vector<double> X;         // nv x 3
  std::vector<int32_t> tets;     // ne x 4
  std::vector<int32_t> tags;     // ne, in {1, 2, 3}
  std::vector<int32_t> parents;  // nv x 2
  int64_t nv() const { return (int64_t)X.size() / 3; }
  int64_t ne() const { return (int64_t)tags.size(); }
};
// Host-built tables of a mesh's operator: the dof of every vertex, the
// CSR pattern over the dofs, the (element, corner) pairs incident to each
// dof row (ascending element), and the face neighbours of every element.
struct MeshOps {
  std::vector<int32_t> dof;
  int64_t n = 0;
  std::vector<int32_t> rowptr, colidx, inc_ptr, inc, nbr;
};
int mesh_ops(const MeshData& m, MeshOps* out);
// Values of the CSR operator (A_s, M), 1 / diag(A_s) and the mesh tables
// already in the problem's workspace, from the nodal potential p.Vv.
hipError_t launch_mesh_assemble(Problem& p, hipStream_t s);
// CSR operator kernels of general meshes (csr.hip).
// CG SpMM of the CSR problems of the table (FP64, chunk-major P -> Q and
// the p.q partials).
hipError_t launch_csr_cg_spmm(Launch& L, int par, hipStream_t s, Timing* t);
// Row-major products of the CSR problems: mode 0 Y1 = A X + s1 M X and
// Y2 = M X (component form), mode 1 HU = H X, MU = M X (Rayleigh-Ritz),
// mode 2 HU = H U0, MU = M U0 (a start that cannot reuse a rotation's).
hipError_t launch_csr_dual(Launch& L, int mode, hipStream_t s, Timing* t);
// paro_batch_step; trust: U and lambda of every problem come unchanged
// from its last rotation under the same operator (the library's own
// loops), so the start reuses that rotation's H U and M U.
int batch_step_impl(paro_problem* const* probs, int32_t count,
                    double* const* d_lambda, double* const* d_U, void* d_ws,
                    size_t bytes, void* stream, paro_report_t* reports,
                    bool trust);
// paro_init; with `status`, synchronous: it receives the status bits
// after Step 1's projection, with the re-orthonormalisation retry done.
int init_impl(paro_problem* h, const double* d_U0, double* d_lambda,
              double* d_U, void* stream, int* status);
// paro_batch_init; with `status`, synchronous: it receives every
// problem's status bits after Step 1's projection, with the
// re-orthonormalisation retry of nearly dependent start blocks done.
int batch_init_impl(paro_problem* const* probs, int32_t count,
                    const double* const* d_U0, double* const* d_lambda,
                    double* const* d_U, void* d_ws, size_t bytes,
                    void* stream, std::vector<int>* status);
// Status bits of a problem (ColState::status) as a PARO_* code (the
// error message recorded as with any failure).
int status_code(int st);
// Record `msg` as this thread's last error (paro_last_error); returns code.
int set_error(int code, const char* msg);
int64_t kuhn_nnz(int mx, int my, int mz);

// ---- launchers (assemble.hip) --------------------------------------------
hipError_t launch_potential_range(const double* V, int64_t nv, double* out,
                                  unsigned* cnt, double* part, hipStream_t s);
hipError_t launch_assemble(Problem& p, const double* V, hipStream_t s);
// CSR copy of the problem's A_s and M into caller buffers (any may be
// null): rowptr int32[n + 1], col int32[nnz], valA, valM FP64[nnz].
hipError_t launch_csr_export(const Problem& p, int32_t* rowptr, int32_t* col,
                             double* valA, double* valM, hipStream_t s);

// ---- launchers (solver.hip) ----------------------------------------------
// All take a Launch over a descriptor table; a single problem is a table of
// one.  Every launch is asynchronous on `s`.
hipError_t launch_spmm(Launch& L, bool rr, hipStream_t s, Timing* t);
// Start of the source solves: b = (lam - s) M U0 (or Bin), X = U0,
// R = b - A_s U0, P = D^-1 R; per-column ||b||^2, r.z, ||r||^2 and the
// first active set.
hipError_t launch_pcg_start(Launch& L, hipStream_t s, Timing* t);
// One CG iteration of parity `par` (FP64 or FP32 vectors).
hipError_t launch_pcg_iter(Launch& L, bool fp32, int par, hipStream_t s,
                           Timing* t);
// FP32 inner solves inside FP64 refinement.
// FP64 residual of the refinement and the next FP32 pass (the first pass
// starts from launch_pcg_start's state): the search direction is kept and
// launch_redirect (after the poll) turns it with the replaced residual.
hipError_t launch_refine_residual(Launch& L, hipStream_t s, Timing* t);
hipError_t launch_redirect(Launch& L, hipStream_t s, Timing* t);
// Autotuner: the CG SpMM alone (parity 0), and a set-up making every
// column active.
hipError_t launch_cg_spmm(Launch& L, bool fp32, hipStream_t s);
// All CG iterations of the table in one cooperative (persistent) launch,
// at most `iters` (even) of them; *fits = false, and nothing launched, if
// the grid cannot be co-resident on the device.
hipError_t launch_cg_persistent(Launch& L, bool fp32, int iters,
                                hipStream_t s, Timing* t, bool* fits);
// Nonlocal term: Z = M zeta for one problem (zeta n x k, row-major).
hipError_t launch_nl_mass(const Desc& d, const double* zeta, double* Z,
                          int k, hipStream_t s);
// FP64 source solves: the orbitals X receive the chunk-major iterate Xc.
hipError_t launch_cm_unpack(Launch& L, hipStream_t s, Timing* t);
hipError_t launch_all_active(Launch& L, hipStream_t s);
hipError_t launch_refine_update(Launch& L, hipStream_t s, Timing* t);
// Poll of the table into host-visible memory: out[1] = active CG columns
// of parity `which` (0, 1) or refining columns (which = 2) summed over the
// problems, out[2] = most CG iterations any problem has executed in its
// current solve, out[3] = OR of the problems' status bits; then out[0] =
// seq (system-scope release, for a host spinning on it).
hipError_t launch_count_active(Launch& L, int which, int* out, int seq,
                               hipStream_t s);
// Per-problem reports into out[0 .. nprob), then *seqp = seq.
hipError_t launch_gather_reports(Launch& L, PollReport* out, int* seqp,
                                 int seq, hipStream_t s);
// Rayleigh-Ritz on W = X: H W, M W, the two Grams, the small eigensolve,
// U = W C with residual norms and the step's convergence measures.
hipError_t launch_rayleigh_ritz(Launch& L, hipStream_t s, Timing* t);
// Shifted Cholesky-QR pass over U = W of every problem of the table (the
// state a failed Rayleigh-Ritz leaves), before the projection is redone.
hipError_t launch_reorth(Launch& L, hipStream_t s);
// ... and after the projection that follows it: flags a problem singular
// when its new basis still has a column of rounding-level independence.
hipError_t launch_reorth_check(Launch& L, hipStream_t s);
// Component Gram G = X^T Y1 into Y2 (non-symmetric, all tiles).
hipError_t launch_gram_full(Launch& L, hipStream_t s, Timing* t);
hipError_t launch_small_geneig(const double* A, const double* B, int n,
                               double* theta, double* C, int* info,
                               hipStream_t s);

}  // namespace paro

struct paro_mesh {
  paro::MeshData m;
  // The operator tables of the mesh, built by the first query or assembly
  // and kept (a mesh never changes after it is made).
  mutable std::shared_ptr<const paro::MeshOps> ops;
  mutable std::mutex ops_mu;
};


// The opaque handle of the C ABI: host metadata of one assembled problem.
struct paro_problem {
  paro::Problem p;
};
