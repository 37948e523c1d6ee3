// Internal declarations shared by the HIP translation units of libparo.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "paro.h"

namespace paro {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kNtMax = PARO_NT_MAX;  // largest number of columns
constexpr int kGridMax = 2048;       // largest persistent grid of the solvers
constexpr int kStencil = 15;         // Kuhn P1 pattern: 15 neighbours per row
constexpr int kGridDefault = 2048;   // default persistent grid
constexpr int kGramGrid = 1024;      // first-stage blocks of the Gram
constexpr int kGramY = 16;           // second-stage split of those blocks
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
};

// Per-column scalars of the block CG, resident in device memory.  One
// problem owns one ColState; all reductions end in it.
struct ColState {
  double bb[kNtMax];      // ||b||^2 of the current (outer) system
  double rz[kNtMax];      // r . z of the current iterate
  double alpha[kNtMax];
  double beta[kNtMax];
  double rr[kNtMax];      // ||r||^2 of the current iterate
  double tol2[kNtMax];    // stop when rr <= tol2 (inner/outer threshold)
  double rr64[kNtMax];    // FP64 residual^2 of the outer (refinement) loop
  int act[2][kNtMax];     // CG column active in iteration of parity s
  int oact[kNtMax];       // outer refinement still running for this column
  int iters[kNtMax];      // CG iterations taken in this step
  int n_active[2];        // number of active columns, per parity
  int n_outer;            // columns still refining
  int status;             // kSt* bits
  int maxit;              // CG cap per column (copied from opts)
  int pad[3];
  unsigned long long cg_iters;      // CG iterations that did work
  unsigned long long cg_col_iters;  // their active columns, summed
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

struct Timing;  // host-side event timing state (api.hip)

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
  int32_t* rowptr;
  int32_t* col;
  double* valA;           // A_s = K/2 + M_V - s M
  double* valM;           // M
  float* valA32;          // FP32 copy of A_s
  double* dinv;           // 1 / diag(A_s)
  float* dinv32;
  double* X;              // n x Nt blocks (FP64)
  double* R;
  double* P;
  double* Q;
  double* B;              // right-hand sides (refinement mode)
  float* R32;             // n x Nt blocks (FP32 inner solves)
  float* P32;
  float* Q32;
  float* X32;
  double* part;           // kGridMax * kNtMax * 3 reduction partials
  double* gpart;          // Gram partials: kGramGrid * gram_tiles(Nt)
  double* gsum;           // kGramY * gram_tiles(Nt)
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
  hipStream_t last_stream;
  int cg_predict[5];      // CG iterations of the last solve per pass slot
};

// Event bracketing of one launch (no-ops unless timing is on).
int timing_begin(Problem& p, int stage, hipStream_t s);
void timing_end(Problem& p, int slot, hipStream_t s);
struct TimedLaunch {
  Problem& p;
  int slot;
  hipStream_t s;
  TimedLaunch(Problem& pp, int stage, hipStream_t ss)
      : p(pp), slot(timing_begin(pp, stage, ss)), s(ss) {}
  ~TimedLaunch() { timing_end(p, slot, s); }
};

// Workspace layout: byte offsets of every region for a problem shape.
struct Layout {
  size_t rowptr, col, valA, valM, valA32, dinv, dinv32;
  size_t X, R, P, Q, B, R32, P32, Q32, X32;
  size_t part, gpart, gsum, Ah, Bh, C, theta, vmin, cs, si, cnt, flag;
  size_t total;
};

Layout make_layout(int64_t n, int64_t nnz, int Nt, int precision);
int64_t kuhn_nnz(int mx, int my, int mz);

// ---- launchers (assemble.hip) --------------------------------------------
hipError_t launch_potential_range(const double* V, int64_t nv, double* out,
                                  unsigned* cnt, double* part, hipStream_t s);
hipError_t launch_assemble(Problem& p, const double* V, hipStream_t s);

// ---- launchers (solver.hip) ----------------------------------------------
// which: 0 = A_s, 1 = M, 2 = H = A_s + s M.
hipError_t launch_spmm(Problem& p, int which, const double* X,
                       double* Y, int ncols, hipStream_t s);
// Start of the FP64 source solves: B = (lam - s) M U, X = U,
// R = B - A_s U, P = D^-1 R; sets bb, rz, rr, act[0].
hipError_t launch_pcg_start(Problem& p, const double* lam, const double* U,
                            int ncols, bool store_b, hipStream_t s);
// Start of a solve with a given right-hand side block B (paro_pcg).
hipError_t launch_pcg_start_rhs(Problem& p, const double* Bin, int ncols,
                                bool store_b, hipStream_t s);
// One CG iteration of parity `par` (FP64): three kernels.
hipError_t launch_pcg_iter(Problem& p, int ncols, int par, hipStream_t s);
// FP32 inner solves inside FP64 refinement.
hipError_t launch_refine_residual(Problem& p, int ncols, bool first,
                                  hipStream_t s);
hipError_t launch_pcg32_iter(Problem& p, int ncols, int par, hipStream_t s);
hipError_t launch_refine_update(Problem& p, int ncols, hipStream_t s);
// Rayleigh-Ritz: R = H X, Q = M X, Ah = X^T R, Bh = X^T Q, eigensolve,
// U = X C with residual norms and the convergence measures in StepInfo.
hipError_t launch_rayleigh_ritz(Problem& p, const double* W, double* lam,
                                double* U, int ncols, bool have_old,
                                hipStream_t s);
hipError_t launch_gram(Problem& p, const double* W, const double* Y1,
                       const double* Y2, double* G1, double* G2, int ncols,
                       hipStream_t s);
hipError_t launch_gram_full(Problem& p, const double* W,
                            const double* Y, double* G, int ncols,
                            hipStream_t s);
hipError_t launch_small_geneig(const double* A, const double* B, int n,
                               double* theta, double* C, int* info,
                               hipStream_t s);

}  // namespace paro
