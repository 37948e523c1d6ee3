// Recovery of a Rayleigh-Ritz step whose basis W is nearly dependent in
// the M inner product (Step 4, eq. (alg-evp)): the Cholesky factorisation
// of B = W^T M W fails when a pivot falls to rounding level of its
// diagonal.  One shifted Cholesky-QR pass then replaces W by a basis of
// the same span that is far better conditioned,
//
//     L L^T = B + s I,   W <- W L^{-T},
//
// with the shift s = 11 (n k + k (k + 1)) u ||B|| (n rows, k columns,
// u = 2^-53, ||B|| bounded by its trace) of the shifted Cholesky QR of
// Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto (SIAM J. Sci. Comput.
// 42, 2020), which makes the factorisation succeed for any W whose Gram
// matrix is positive semidefinite up to that rounding.  The ordinary
// Rayleigh-Ritz projection then runs again on the new basis (operators
// applied afresh), and its own Cholesky factorisation is the second pass.
// Columns that are dependent to rounding level stay dependent (no change
// of basis can undo that): what the pass makes of such a column is the
// rounding error of forming W L^{-T}, a vector of M-norm about
// u / sqrt(2 s) after its projection on the other columns, while a column
// that differs from the span of the others by a relative distance d
// keeps about d / sqrt(2 s), and the well-determined columns have norm
// about 1.  So after the second projection the Gram matrix of the new
// basis is factorised once more with an absolute pivot test (every pivot
// above 1e-14 of the largest diagonal entry, i.e. 1e-7 in norm): that
// separates the two by a factor of at least 50 for any shift the rule
// above can give, and a block that fails it is reported singular.
//
// The failed projection leaves U = W exactly (its coefficient matrix is
// the identity), so the pass reads and rewrites the orbitals in place.
#include "paro_internal.h"

namespace paro {
namespace {

constexpr int kLdR = kNtMax + 1;     // padded LDS row
constexpr int kTile = 4096;          // doubles of W staged per tile

// One block per problem: the shifted factor of B (the problem's Gram
// result, cluster-wise like the projection: entries coupling different
// clusters are dropped, so the new basis keeps every column inside its
// cluster) and C = L^{-T} into d.C.  Also clears the singular status bit
// and restores lambda to the values before the failed projection, so the
// projection that follows reports against the right previous step.
__global__ void __launch_bounds__(kBlock) reorth_factor_kernel(
    const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  const int n = d.ncols;
  __shared__ double S[kNtMax][kLdR];   // B + s I, then L (lower)
  __shared__ double Li[kNtMax][kLdR];  // L^{-1} (lower)
  __shared__ double s_shift;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kBlock) {
    const int i = e / n, j = e % n;
    const bool keep = !d.clus || d.clus[i] == d.clus[j];
    S[i][j] = keep ? d.Bh[e] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(S[i][i]);
    const double u = 0x1.0p-53;
    const double rows = (double)d.n;
    s_shift = 11.0 * (rows * n + (double)n * (n + 1)) * u * tr;
    s_bad = !(tr > 0.0) || !isfinite(tr);
    atomicAnd(&d.cs->status, ~(int)kStSingular);
    *d.geneig_info = 0;
  }
  if (d.have_old && d.lam)
    for (int c = tid; c < n; c += kBlock) d.lam[c] = d.si->lam_old[c];
  __syncthreads();
  if (tid < n) S[tid][tid] += s_shift;
  __syncthreads();
  // Right-looking Cholesky: column k is scaled by 1/sqrt(pivot), then the
  // trailing lower triangle loses its outer product.
  for (int k = 0; k < n && !s_bad; ++k) {
    const double piv = S[k][k];
    if (!(piv > 0.0) || !isfinite(piv)) {
      __syncthreads();
      if (tid == 0) s_bad = 1;
      __syncthreads();
      break;
    }
    const double lkk = sqrt(piv);
    for (int i = k + 1 + tid; i < n; i += kBlock) S[i][k] /= lkk;
    __syncthreads();  // every thread has read the pivot
    if (tid == 0) S[k][k] = lkk;
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += kBlock) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) S[i][j] -= S[i][k] * S[j][k];
    }
    __syncthreads();
  }
  if (s_bad) {  // C = I: the basis stays, the projection reports failure
    for (int e = tid; e < n * n; e += kBlock)
      d.C[e] = (e / n == e % n) ? 1.0 : 0.0;
    return;
  }
  // Column j of L^{-1} by forward substitution (thread j).
  if (tid < n) {
    const int j = tid;
    for (int i = 0; i < j; ++i) Li[i][j] = 0.0;
    Li[j][j] = 1.0 / S[j][j];
    for (int i = j + 1; i < n; ++i) {
      double acc = 0.0;
      for (int k = j; k < i; ++k) acc = fma(S[i][k], Li[k][j], acc);
      Li[i][j] = -acc / S[i][i];
    }
  }
  __syncthreads();
  // C[k][j] = (L^{-T})[k][j] = Li[j][k], upper triangular.
  for (int e = tid; e < n * n; e += kBlock) {
    const int k = e / n, j = e % n;
    d.C[e] = k <= j ? Li[j][k] : 0.0;
  }
}

// U <- U C in place (row-major n x ncols, C upper triangular), over the
// problem's own blocks [b0, b0 + nb) of the launch: each tile of rows is
// staged whole in LDS before any of its rows is written.
__global__ void __launch_bounds__(kBlock) reorth_rotate_kernel(
    const Desc* __restrict__ D, int nprob) {
  __shared__ double sC[kNtMax * kNtMax];
  __shared__ double sW[kTile];
  int p = 0;
  while (p + 1 < nprob && (int)blockIdx.x >= D[p + 1].b0) ++p;
  const Desc& d = D[p];
  const int lb = (int)blockIdx.x - d.b0;
  if (lb < 0 || lb >= d.nb) return;
  const int nc = d.ncols;
  for (int e = threadIdx.x; e < nc * nc; e += kBlock) sC[e] = d.C[e];
  const int tr = kTile / nc;
  const long long ntiles = (d.n + tr - 1) / tr;
  double* U = d.Uout;
  for (long long t = lb; t < ntiles; t += d.nb) {
    const long long r0 = t * tr;
    const int cnt = (int)min((long long)tr, d.n - r0) * nc;
    double* row0 = U + r0 * nc;
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += kBlock) sW[e] = row0[e];
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += kBlock) {
      const int r = e / nc, j = e % nc;
      const double* w = sW + r * nc;
      double acc = 0.0;
      for (int k = 0; k <= j; ++k) acc = fma(w[k], sC[k * nc + j], acc);
      row0[e] = acc;
    }
  }
}

// After the projection of the re-orthonormalised basis: its Gram matrix
// (d.Bh, cluster-wise) must factorise with every pivot above 1e-14 of the
// largest diagonal entry, else the problem is flagged singular.
__global__ void __launch_bounds__(kBlock) reorth_check_kernel(
    const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  const int n = d.ncols;
  __shared__ double S[kNtMax][kLdR];
  __shared__ double s_floor;
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kBlock) {
    const int i = e / n, j = e % n;
    const bool keep = !d.clus || d.clus[i] == d.clus[j];
    S[i][j] = keep ? d.Bh[e] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = fmax(dmax, S[i][i]);
    s_floor = 1e-14 * dmax;
    s_bad = 0;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = S[k][k];
    if (!(piv > s_floor) || !isfinite(piv)) {
      if (tid == 0) s_bad = k + 1;
      break;  // every thread read the same pivot
    }
    const double lkk = sqrt(piv);
    for (int i = k + 1 + tid; i < n; i += kBlock) S[i][k] /= lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = tid; e < m * m; e += kBlock) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) S[i][j] -= S[i][k] * S[j][k];
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) {
    atomicOr(&d.cs->status, (int)kStSingular);
    if (*d.geneig_info == 0) *d.geneig_info = s_bad;
  }
}

}  // namespace

hipError_t launch_reorth_check(Launch& L, hipStream_t s) {
  hipLaunchKernelGGL(reorth_check_kernel, dim3(L.nprob), dim3(kBlock), 0, s,
                     (const Desc*)L.d);
  return hipGetLastError();
}

hipError_t launch_reorth(Launch& L, hipStream_t s) {
  hipLaunchKernelGGL(reorth_factor_kernel, dim3(L.nprob), dim3(kBlock), 0, s,
                     (const Desc*)L.d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reorth_rotate_kernel, dim3(L.blocks), dim3(kBlock), 0, s,
                     (const Desc*)L.d, L.nprob);
  return hipGetLastError();
}

}  // namespace paro
