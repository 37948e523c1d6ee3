// Kernels of one ParO step on gfx950: block Jacobi-PCG for the Nt source
// problems of Step 3 and the Rayleigh-Ritz projection of Step 4.
//
// Data layout.  Orbital blocks are row-major n x Nt (orbital fastest), so a
// CSR neighbour gathered by the SpMM is Nt contiguous values; a thread owns
// V consecutive columns of one row ("chunk"), a workgroup a tile of
// kBlock / (Nt / V) rows.  Persistent grids walk the tiles; workgroup b
// serves the tile slab (b mod 8) so that the eight XCDs each sweep one
// contiguous slab of rows and keep their halo in their own L2.
//
// Reductions (per-column dot products) are two-stage and deterministic:
// each workgroup writes its partial sums, the last workgroup to finish
// (atomic ticket, agent-scope fences) adds the partials in a fixed order
// and updates the per-column CG scalars in ColState.  No float atomics.
#include <cmath>

#include "paro_internal.h"

namespace paro {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;
constexpr size_t kPartStride = (size_t)kGridMax * kNtMax;

template <typename T, int V>
struct VecT;
template <>
struct VecT<double, 1> { typedef double type; };
template <>
struct VecT<double, 2> { typedef double2 type; };
template <>
struct VecT<float, 1> { typedef float type; };
template <>
struct VecT<float, 2> { typedef float2 type; };
template <>
struct VecT<float, 4> { typedef float4 type; };

template <typename T, int V>
__device__ __forceinline__ void ldv(const T* p, T (&o)[V]) {
  typedef typename VecT<T, V>::type W;
  const W w = *reinterpret_cast<const W*>(p);
  const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
  for (int v = 0; v < V; ++v) o[v] = e[v];
}

template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const T (&o)[V]) {
  typedef typename VecT<T, V>::type W;
  W w;
  T* e = reinterpret_cast<T*>(&w);
#pragma unroll
  for (int v = 0; v < V; ++v) e[v] = o[v];
  *reinterpret_cast<W*>(p) = w;
}

// Tiles of workgroup b in an XCD-sliced grid-stride walk.
struct TileWalk {
  long long t, end, step;
};
__device__ __forceinline__ TileWalk tile_walk(long long ntiles) {
  const int G = gridDim.x, b = blockIdx.x;
  const int x = b % kXcd, l = b / kXcd, gx = G / kXcd;
  const long long chunk = (ntiles + kXcd - 1) / kXcd;
  TileWalk w;
  w.t = (long long)x * chunk + l;
  w.end = min(ntiles, (long long)(x + 1) * chunk);
  w.step = gx;
  return w;
}

// Per-column workgroup reduction of per-thread partials acc[a][v]
// (thread = (lr, ch)), written column-major: part[a][c][block].  NA arrays.
template <int V, int NA>
__device__ void block_partials(const double (&acc)[NA][V], int ncols, int cpr,
                               int tr, double* __restrict__ part) {
  __shared__ double red[NA][kBlock * V];
  const int tid = threadIdx.x;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int v = 0; v < V; ++v) red[a][tid * V + v] = acc[a][v];
  __syncthreads();
  if (tid < ncols) {
    const int ch = tid / V, v = tid % V;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      double s = 0.0;
      for (int lr = 0; lr < tr; ++lr) s += red[a][(lr * cpr + ch) * V + v];
      part[a * kPartStride + (size_t)tid * gridDim.x + blockIdx.x] = s;
    }
  }
}

// In a finalize kernel with one workgroup per column c = blockIdx.x: the
// fixed-order sum of part[a][c][0..nb).  Every thread receives the sums.
template <int NA>
__device__ void column_sums(const double* __restrict__ part, int nb,
                            double (&out)[NA]) {
  __shared__ double red[NA][kBlock];
  const int c = blockIdx.x, t = threadIdx.x;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const double* src = part + a * kPartStride + (size_t)c * nb;
    double s = 0.0;
    for (int b = t; b < nb; b += kBlock) s += src[b];
    red[a][t] = s;
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int a = 0; a < NA; ++a) red[a][t] += red[a][t + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < NA; ++a) out[a] = red[a][0];
  __syncthreads();
}

// Max of non-negative doubles through their bit patterns (order-free).
__device__ __forceinline__ void atomic_max_nonneg(double* dst, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(dst),
            (unsigned long long)__double_as_longlong(v));
}

// LDS view of one CSR tile: row pointers (tile-relative), columns and up
// to two value arrays, each region 16-byte aligned.
template <typename TM>
struct CsrTile {
  int32_t* rp;
  int32_t* col;
  TM* a;
  TM* b;
};

__host__ __device__ constexpr size_t align16(size_t x) {
  return (x + 15) & ~size_t(15);
}

// LDS bytes for a tile of tr rows with nvals value arrays.
__host__ __device__ constexpr size_t csr_tile_bytes(int tr, size_t vsize,
                                                    int nvals) {
  return align16(sizeof(int32_t) * (tr + 1)) +
         align16(sizeof(int32_t) * tr * kStencil) +
         nvals * align16(vsize * tr * kStencil);
}

template <typename TM>
__device__ __forceinline__ CsrTile<TM> csr_tile(unsigned char* smem, int tr,
                                                int nvals) {
  CsrTile<TM> t;
  size_t o = 0;
  t.rp = reinterpret_cast<int32_t*>(smem + o);
  o += align16(sizeof(int32_t) * (tr + 1));
  t.col = reinterpret_cast<int32_t*>(smem + o);
  o += align16(sizeof(int32_t) * tr * kStencil);
  t.a = reinterpret_cast<TM*>(smem + o);
  o += align16(sizeof(TM) * tr * kStencil);
  t.b = nvals > 1 ? reinterpret_cast<TM*>(smem + o) : nullptr;
  return t;
}

// Stage rows [r0, r1) of the CSR into the tile with coalesced loads; row
// pointers become tile-relative.  All threads of the block must call it.
template <typename TM>
__device__ __forceinline__ void stage_csr(const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ col,
                                          const TM* __restrict__ va,
                                          const TM* __restrict__ vb,
                                          long long r0, long long r1,
                                          CsrTile<TM>& t) {
  const int rows = (int)(r1 - r0);
  __syncthreads();  // the previous tile is no longer read
  for (int i = threadIdx.x; i <= rows; i += blockDim.x) t.rp[i] = rowptr[r0 + i];
  __syncthreads();
  const int k0 = t.rp[0], cnt = t.rp[rows] - k0;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    t.col[e] = col[k0 + e];
    t.a[e] = va[k0 + e];
    if (vb) t.b[e] = vb[k0 + e];
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= rows; i += blockDim.x) t.rp[i] -= k0;
  __syncthreads();
}

__device__ __forceinline__ bool chunk_active(const int* act, int ch, int V,
                                             int ncols) {
  bool a = false;
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    if (c < ncols) a = a || act[c] != 0;
  }
  return a;
}

// ------------------------------------------------------------------------
// SpMM for CG: Q = A P on the active columns, with per-column p . q.
// The tile's CSR slice is staged in LDS with coalesced loads.
// ------------------------------------------------------------------------
template <typename T, typename TM, int V>
__global__ void __launch_bounds__(kBlock)
spmm_cg_kernel(const int32_t* __restrict__ rowptr,
               const int32_t* __restrict__ col, const TM* __restrict__ val,
               const T* __restrict__ P, T* __restrict__ Q, long long n,
               int ncols, ColState* __restrict__ cs, int par,
               double* __restrict__ part) {
  if (cs->n_active[par] == 0) return;
  extern __shared__ unsigned char smem[];
  const int cpr = ncols / V, tr = kBlock / cpr;
  CsrTile<TM> tl = csr_tile<TM>(smem, tr, 1);
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  const bool on = lr < tr && chunk_active(cs->act[par], ch, V, ncols);
  double acc[1][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = 0.0;
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * tr;
    const long long r1 = min(n, r0 + tr);
    stage_csr<TM>(rowptr, col, val, nullptr, r0, r1, tl);
    const long long row = r0 + lr;
    if (on && row < r1) {
      const int rs = tl.rp[lr], re = tl.rp[lr + 1];
      T q[V];
#pragma unroll
      for (int v = 0; v < V; ++v) q[v] = T(0);
      for (int e = rs; e < re; ++e) {
        const T a = (T)tl.a[e];
        T pv[V];
        ldv<T, V>(P + (size_t)tl.col[e] * ncols + ch * V, pv);
#pragma unroll
        for (int v = 0; v < V; ++v) q[v] = fma(a, pv[v], q[v]);
      }
      stv<T, V>(Q + (size_t)row * ncols + ch * V, q);
      T po[V];
      ldv<T, V>(P + (size_t)row * ncols + ch * V, po);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[0][v] += (double)po[v] * (double)q[v];
    }
  }
  block_partials<V, 1>(acc, ncols, cpr, tr, part);
}

// alpha_c = (r.z)_c / (p.q)_c for the active columns (one workgroup per
// column).  Also clears the next parity's active count for cg_beta_kernel.
__global__ void __launch_bounds__(kBlock)
cg_alpha_kernel(const double* __restrict__ part, int nb,
                ColState* __restrict__ cs, int par) {
  const int c = blockIdx.x;
  if (cs->n_active[par] == 0) {
    // Nothing ran in this iteration: keep the next parity idle too, so
    // that launches queued after convergence stay no-ops.
    if (c == 0 && threadIdx.x == 0) cs->n_active[par ^ 1] = 0;
    return;
  }
  if (c == 0 && threadIdx.x == 0) {
    cs->n_active[par ^ 1] = 0;
    cs->cg_iters += 1;
  }
  if (!cs->act[par][c]) return;
  double tot[1];
  column_sums<1>(part, nb, tot);
  if (threadIdx.x == 0) {
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
      atomicOr(&cs->status, isfinite(pq) ? (int)kStNotSpd : (int)kStNonFinite);
      cs->alpha[c] = 0.0;
    } else {
      cs->alpha[c] = cs->rz[c] / pq;
    }
  }
}

// r -= alpha q, z = D^-1 r, partial r.z and r.r; the last block forms
// beta, counts iterations and decides which columns stay active.
template <typename T, typename TD, int V>
__global__ void __launch_bounds__(kBlock)
rupd_kernel(const T* __restrict__ Qb, T* __restrict__ R,
            const TD* __restrict__ dinv, long long n, int ncols,
            ColState* __restrict__ cs, int par, double* __restrict__ part) {
  if (cs->n_active[par] == 0) return;
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  const bool on = lr < tr && chunk_active(cs->act[par], ch, V, ncols);
  T al[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    al[v] = (c < ncols && cs->act[par][c]) ? (T)cs->alpha[c] : T(0);
  }
  double acc[2][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.0;
  const long long ntiles = (n + tr - 1) / tr;
  if (on) {
    for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
      const long long row = w.t * tr + lr;
      if (row >= n) continue;
      const size_t o = (size_t)row * ncols + ch * V;
      T r[V], q[V];
      ldv<T, V>(R + o, r);
      ldv<T, V>(Qb + o, q);
      const T di = (T)dinv[row];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        r[v] = fma(-al[v], q[v], r[v]);
        acc[0][v] += (double)r[v] * (double)(di * r[v]);
        acc[1][v] += (double)r[v] * (double)r[v];
      }
      stv<T, V>(R + o, r);
    }
  }
  block_partials<V, 2>(acc, ncols, cpr, tr, part);
}

// beta_c, iteration count and the stopping test of every active column
// (one workgroup per column); counts the columns active next iteration.
__global__ void __launch_bounds__(kBlock)
cg_beta_kernel(const double* __restrict__ part, int nb,
               ColState* __restrict__ cs, int par) {
  const int c = blockIdx.x;
  if (cs->n_active[par] == 0) return;
  if (!cs->act[par][c]) {
    if (threadIdx.x == 0) cs->act[par ^ 1][c] = 0;
    return;
  }
  double tot[2];
  column_sums<2>(part, nb, tot);
  if (threadIdx.x != 0) return;
  int next = 0;
  const double rz = tot[0], rr = tot[1];
  if (!isfinite(rz) || !isfinite(rr)) {
    atomicOr(&cs->status, (int)kStNonFinite);
  } else {
    cs->beta[c] = rz / cs->rz[c];
    cs->rz[c] = rz;
    cs->rr[c] = rr;
    const int it = cs->iters[c] + 1;
    cs->iters[c] = it;
    const bool more = rr > cs->tol2[c];
    if (more && it >= cs->maxit) atomicOr(&cs->status, (int)kStNoConv);
    next = (more && it < cs->maxit && !(cs->status & kStNotSpd)) ? 1 : 0;
  }
  cs->act[par ^ 1][c] = next;
  if (next) atomicAdd(&cs->n_active[par ^ 1], 1);
  atomicAdd(&cs->cg_col_iters, 1LL);
}

// x += alpha p (columns active this iteration); p = D^-1 r + beta p
// (columns active next iteration).
template <typename T, typename TD, int V>
__global__ void __launch_bounds__(kBlock)
pupd_kernel(T* __restrict__ X, T* __restrict__ P, const T* __restrict__ R,
            const TD* __restrict__ dinv, long long n, int ncols,
            const ColState* __restrict__ cs, int par) {
  if (cs->n_active[par] == 0) return;
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  if (lr >= tr || !chunk_active(cs->act[par], ch, V, ncols)) return;
  T al[V], be[V];
  bool nx[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    const bool a = c < ncols && cs->act[par][c];
    nx[v] = c < ncols && cs->act[par ^ 1][c];
    al[v] = a ? (T)cs->alpha[c] : T(0);
    be[v] = nx[v] ? (T)cs->beta[c] : T(0);
  }
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long row = w.t * tr + lr;
    if (row >= n) continue;
    const size_t o = (size_t)row * ncols + ch * V;
    T x[V], p[V], r[V];
    ldv<T, V>(X + o, x);
    ldv<T, V>(P + o, p);
    ldv<T, V>(R + o, r);
    const T di = (T)dinv[row];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      x[v] = fma(al[v], p[v], x[v]);
      p[v] = nx[v] ? fma(be[v], p[v], di * r[v]) : p[v];
    }
    stv<T, V>(X + o, x);
    stv<T, V>(P + o, p);
  }
}

// ------------------------------------------------------------------------
// Start of the FP64 source solves (eq. (alg-bvp) with the shift):
//   b = (lam - s) M u  (or a given block B),  x0 = u,
//   r = b - A_s x0,  p = D^-1 r;  partials ||b||^2, r.z, ||r||^2.
// ------------------------------------------------------------------------
template <int V>
__global__ void __launch_bounds__(kBlock)
pcg_start_kernel(const int32_t* __restrict__ rowptr,
                 const int32_t* __restrict__ col,
                 const double* __restrict__ valA,
                 const double* __restrict__ valM,
                 const double* __restrict__ dinv, const double* __restrict__ U,
                 const double* __restrict__ lam, const double* __restrict__ Bin,
                 double sigma, double rtol, double* __restrict__ X,
                 double* __restrict__ R, double* __restrict__ P,
                 double* __restrict__ Bout, long long n, int ncols,
                 int maxit, ColState* __restrict__ cs,
                 double* __restrict__ part) {
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  if (blockIdx.x == 0 && tid == 0) {  // read only by the finalize kernel
    cs->n_active[0] = 0;
    cs->n_active[1] = 0;
    cs->n_outer = 0;
    cs->status = 0;
    cs->maxit = maxit;
  }
  double sh[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    sh[v] = (lam && c < ncols) ? lam[c] - sigma : 0.0;
  }
  extern __shared__ unsigned char smem[];
  CsrTile<double> tl = csr_tile<double>(smem, tr, 2);
  double acc[3][V];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[a][v] = 0.0;
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * tr;
    const long long r1 = min(n, r0 + tr);
    stage_csr<double>(rowptr, col, valA, valM, r0, r1, tl);
    const long long row = r0 + lr;
    if (lr >= tr || row >= r1) continue;
    double au[V], mu[V];
#pragma unroll
    for (int v = 0; v < V; ++v) au[v] = mu[v] = 0.0;
    const int rs = tl.rp[lr], re = tl.rp[lr + 1];
    for (int e = rs; e < re; ++e) {
      const double a = tl.a[e], m = tl.b[e];
      double u[V];
      ldv<double, V>(U + (size_t)tl.col[e] * ncols + ch * V, u);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        au[v] = fma(a, u[v], au[v]);
        mu[v] = fma(m, u[v], mu[v]);
      }
    }
    const size_t o = (size_t)row * ncols + ch * V;
    double b[V], r[V], p[V], u[V];
    ldv<double, V>(U + o, u);
    if (Bin) {
      ldv<double, V>(Bin + o, b);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) b[v] = sh[v] * mu[v];
    }
    const double di = dinv[row];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      r[v] = b[v] - au[v];
      p[v] = di * r[v];
      acc[0][v] += b[v] * b[v];
      acc[1][v] += r[v] * p[v];
      acc[2][v] += r[v] * r[v];
    }
    if (X != U) stv<double, V>(X + o, u);
    stv<double, V>(R + o, r);
    stv<double, V>(P + o, p);
    if (Bout) stv<double, V>(Bout + o, b);
  }
  block_partials<V, 3>(acc, ncols, cpr, tr, part);
}

// Per-column start state: ||b||^2, r.z, ||r||^2, the stopping threshold
// and the first active set (one workgroup per column).
__global__ void __launch_bounds__(kBlock)
pcg_start_final_kernel(const double* __restrict__ part, int nb, double rtol,
                       ColState* __restrict__ cs) {
  const int c = blockIdx.x;
  double tot[3];
  column_sums<3>(part, nb, tot);
  if (threadIdx.x != 0) return;
  const double bb = tot[0], rz = tot[1], rr = tot[2];
  cs->bb[c] = bb;
  cs->rz[c] = rz;
  cs->rr[c] = rr;
  cs->rr64[c] = rr;
  cs->tol2[c] = rtol * rtol * bb;
  cs->iters[c] = 0;
  int a = 0;
  if (!isfinite(bb) || !isfinite(rr)) {
    atomicOr(&cs->status, (int)kStNonFinite);
  } else {
    a = rr > rtol * rtol * bb ? 1 : 0;
  }
  cs->act[0][c] = a;
  cs->act[1][c] = 0;
  cs->oact[c] = a;
  if (a) {
    atomicAdd(&cs->n_active[0], 1);
    atomicAdd(&cs->n_outer, 1);
  }
}

// ------------------------------------------------------------------------
// Mixed precision: FP64 residual of the outer (refinement) iteration and
// the start of an FP32 inner CG solve for the correction.
//   r64 = B - A_s X;  converged columns (||r64|| <= rtol ||b||) retire;
//   the others restart CG on A d = r64 in FP32 from d = 0, to
//   ||r|| <= inner_rtol ||r64||.
// ------------------------------------------------------------------------
template <int V>
__global__ void __launch_bounds__(kBlock)
refine_residual_kernel(const int32_t* __restrict__ rowptr,
                       const int32_t* __restrict__ col,
                       const double* __restrict__ valA,
                       const double* __restrict__ dinv,
                       const double* __restrict__ X,
                       const double* __restrict__ Bb,
                       float* __restrict__ R32, float* __restrict__ P32,
                       float* __restrict__ X32, double rtol, double inner_rtol,
                       long long n, int ncols, ColState* __restrict__ cs,
                       double* __restrict__ part) {
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  const bool on = lr < tr && chunk_active(cs->oact, ch, V, ncols);
  if (blockIdx.x == 0 && tid == 0) {  // read only by the finalize kernel
    cs->n_active[0] = 0;
    cs->n_active[1] = 0;
    cs->n_outer = 0;
  }
  extern __shared__ unsigned char smem[];
  CsrTile<double> tl = csr_tile<double>(smem, tr, 1);
  double acc[2][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.0;
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * tr;
    const long long r1 = min(n, r0 + tr);
    stage_csr<double>(rowptr, col, valA, nullptr, r0, r1, tl);
    const long long row = r0 + lr;
    if (!on || row >= r1) continue;
    double ax[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ax[v] = 0.0;
    const int rs = tl.rp[lr], re = tl.rp[lr + 1];
    for (int e = rs; e < re; ++e) {
      const double a = tl.a[e];
      double x[V];
      ldv<double, V>(X + (size_t)tl.col[e] * ncols + ch * V, x);
#pragma unroll
      for (int v = 0; v < V; ++v) ax[v] = fma(a, x[v], ax[v]);
    }
    const size_t o = (size_t)row * ncols + ch * V;
    double b[V];
    ldv<double, V>(Bb + o, b);
    const double di = dinv[row];
    float r32[V], p32[V], z32[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double r = b[v] - ax[v];
      acc[0][v] += r * r;
      r32[v] = (float)r;
      p32[v] = (float)(di * r);
      z32[v] = 0.0f;
      acc[1][v] += (double)r32[v] * (double)p32[v];
    }
    stv<float, V>(R32 + o, r32);
    stv<float, V>(P32 + o, p32);
    stv<float, V>(X32 + o, z32);
  }
  block_partials<V, 2>(acc, ncols, cpr, tr, part);
}

// Outer (refinement) test per column and the inner threshold of the next
// FP32 solve (one workgroup per column).
__global__ void __launch_bounds__(kBlock)
refine_final_kernel(const double* __restrict__ part, int nb, double rtol,
                    double inner_rtol, ColState* __restrict__ cs) {
  const int c = blockIdx.x;
  if (!cs->oact[c]) {
    if (threadIdx.x == 0) {
      cs->act[0][c] = 0;
      cs->act[1][c] = 0;
    }
    return;
  }
  double tot[2];
  column_sums<2>(part, nb, tot);
  if (threadIdx.x != 0) return;
  int a = 0;
  const double rr = tot[0];
  if (!isfinite(rr)) {
    atomicOr(&cs->status, (int)kStNonFinite);
  } else {
    cs->rr64[c] = rr;
    const bool more = rr > rtol * rtol * cs->bb[c];
    a = (more && cs->iters[c] < cs->maxit) ? 1 : 0;
    if (more && !a) atomicOr(&cs->status, (int)kStNoConv);
    cs->tol2[c] = inner_rtol * inner_rtol * rr;
    cs->rz[c] = tot[1];
  }
  cs->oact[c] = a;
  cs->act[0][c] = a;
  cs->act[1][c] = 0;
  if (a) {
    atomicAdd(&cs->n_active[0], 1);
    atomicAdd(&cs->n_outer, 1);
  }
}

// X += d (FP32 correction) for columns that refined in this pass.
template <int V>
__global__ void __launch_bounds__(kBlock)
refine_update_kernel(double* __restrict__ X, const float* __restrict__ X32,
                     long long n, int ncols, const ColState* __restrict__ cs) {
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  if (lr >= tr || !chunk_active(cs->oact, ch, V, ncols)) return;
  bool a[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    a[v] = c < ncols && cs->oact[c];
  }
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long row = w.t * tr + lr;
    if (row >= n) continue;
    const size_t o = (size_t)row * ncols + ch * V;
    double x[V];
    float d[V];
    ldv<double, V>(X + o, x);
    ldv<float, V>(X32 + o, d);
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] += a[v] ? (double)d[v] : 0.0;
    stv<double, V>(X + o, x);
  }
}

// ------------------------------------------------------------------------
// Plain SpMM (FP64): Y1 = A_s X + s1 M X, Y2 = M X (either may be null).
// ------------------------------------------------------------------------
template <int V>
__global__ void __launch_bounds__(kBlock)
spmm_dual_kernel(const int32_t* __restrict__ rowptr,
                 const int32_t* __restrict__ col,
                 const double* __restrict__ valA,
                 const double* __restrict__ valM, const double* __restrict__ X,
                 double* __restrict__ Y1, double* __restrict__ Y2, double s1,
                 long long n, int ncols) {
  const int cpr = ncols / V, tr = kBlock / cpr;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  const bool needA = Y1 != nullptr;
  const bool needM = Y2 != nullptr || s1 != 0.0;
  extern __shared__ unsigned char smem[];
  CsrTile<double> tl = csr_tile<double>(smem, tr, 2);
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * tr;
    const long long r1 = min(n, r0 + tr);
    stage_csr<double>(rowptr, col, needA ? valA : valM,
                      (needA && needM) ? valM : nullptr, r0, r1, tl);
    const long long row = r0 + lr;
    if (lr >= tr || row >= r1) continue;
    double ax[V], mx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ax[v] = mx[v] = 0.0;
    const int rs = tl.rp[lr], re = tl.rp[lr + 1];
    for (int e = rs; e < re; ++e) {
      double x[V];
      ldv<double, V>(X + (size_t)tl.col[e] * ncols + ch * V, x);
      const double a = needA ? tl.a[e] : 0.0;
      const double m = needA ? (needM ? tl.b[e] : 0.0) : tl.a[e];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        ax[v] = fma(a, x[v], ax[v]);
        mx[v] = fma(m, x[v], mx[v]);
      }
    }
    const size_t o = (size_t)row * ncols + ch * V;
    if (Y1) {
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = fma(s1, mx[v], ax[v]);
      stv<double, V>(Y1 + o, y);
    }
    if (Y2) stv<double, V>(Y2 + o, mx);
  }
}

// ------------------------------------------------------------------------
// Gram contractions G1 = W^T Y1, G2 = W^T Y2 on FP64 matrix cores
// (v_mfma_f64_16x16x4_f64).  Each wavefront consumes 4 rows per MFMA:
// A = 16 columns of W over the 4 rows (lane l: row l/16, column l%16),
// B = 16 columns of Y over the same rows; D accumulates 16 x 16 tiles.
// Only tile pairs I <= J are formed; the last block symmetrises.
// ------------------------------------------------------------------------
template <int NT16>
__global__ void __launch_bounds__(kBlock)
gram_kernel(const double* __restrict__ W, const double* __restrict__ Y1,
            const double* __restrict__ Y2, long long n, int ncols,
            double* __restrict__ gpart) {
  constexpr int NP = NT16 * (NT16 + 1) / 2;  // tile pairs I <= J
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const bool two = Y2 != nullptr;
  v4d acc1[NP], acc2[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    acc1[p] = v4d{0.0, 0.0, 0.0, 0.0};
    acc2[p] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  const long long nsteps = (n + 3) / 4;
  const long long gw = (long long)blockIdx.x * 4 + wave;
  const long long nw = (long long)gridDim.x * 4;
  // Contiguous range of 4-row steps per wavefront.
  const long long per = (nsteps + nw - 1) / nw;
  const long long s0 = gw * per, s1 = min(nsteps, s0 + per);
  for (long long st = s0; st < s1; ++st) {
    const long long row = st * 4 + lk;
    double a[NT16], y1[NT16], y2[NT16];
#pragma unroll
    for (int I = 0; I < NT16; ++I) {
      const int c = I * 16 + li;
      const bool ok = row < n && c < ncols;
      const size_t o = (size_t)row * ncols + c;
      a[I] = ok ? W[o] : 0.0;
      y1[I] = ok ? Y1[o] : 0.0;
      y2[I] = (ok && two) ? Y2[o] : 0.0;
    }
    int p = 0;
#pragma unroll
    for (int I = 0; I < NT16; ++I)
#pragma unroll
      for (int J = I; J < NT16; ++J, ++p) {
        acc1[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], y1[J], acc1[p],
                                                       0, 0, 0);
        if (two)
          acc2[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[I], y2[J],
                                                         acc2[p], 0, 0, 0);
      }
  }
  // D layout (measured): lane l, element r holds row l/16 + 4r, column l%16.
  __shared__ double sg[2][NP][256];
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int idx = (lk + 4 * r) * 16 + li;
          if (w == 0) {
            sg[0][p][idx] = acc1[p][r];
            sg[1][p][idx] = acc2[p][r];
          } else {
            sg[0][p][idx] += acc1[p][r];
            sg[1][p][idx] += acc2[p][r];
          }
        }
    }
    __syncthreads();
  }
  const int per_blk = 2 * NP * 256;
  for (int e = threadIdx.x; e < per_blk; e += kBlock)
    gpart[(size_t)blockIdx.x * per_blk + e] = (&sg[0][0][0])[e];
}

// Second stage of the Gram contractions: entry e of the tile array is the
// fixed-order sum over the first-stage blocks (one thread per entry,
// coalesced); then one block scatters the tiles into the ncols x ncols
// results.  mode 0: symmetric pair (G1, G2) from tile pairs I <= J;
// mode 1: one full matrix from all tiles.
__global__ void __launch_bounds__(kBlock)
gram_reduce_kernel(const double* __restrict__ gpart, int nb, int per_blk,
                   double* __restrict__ gsum) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= per_blk) return;
  const int y = blockIdx.y, chunk = (nb + kGramY - 1) / kGramY;
  const int b0 = y * chunk, b1 = min(nb, b0 + chunk);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += gpart[(size_t)b * per_blk + e];
  gsum[(size_t)y * per_blk + e] = s;
}

__global__ void __launch_bounds__(kBlock)
gram_scatter_kernel(const double* __restrict__ gsum, int per_blk, int nt16,
                    int mode, int ncols, double* __restrict__ G1,
                    double* __restrict__ G2) {
  const int np = mode == 0 ? nt16 * (nt16 + 1) / 2 : nt16 * nt16;
  auto tile = [&](int idx) {
    double v = 0.0;
    for (int y = 0; y < kGramY; ++y) v += gsum[(size_t)y * per_blk + idx];
    return v;
  };
  for (int t = threadIdx.x; t < ncols * ncols; t += kBlock) {
    const int i = t / ncols, j = t % ncols;
    if (mode == 1) {
      G1[t] = tile(((i / 16) * nt16 + j / 16) * 256 + (i % 16) * 16 + j % 16);
      continue;
    }
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int I = lo / 16, J = hi / 16;
    const int p = I * nt16 - I * (I - 1) / 2 + (J - I);
    const int a = (lo % 16) * 16 + hi % 16, b = (hi % 16) * 16 + lo % 16;
    for (int g = 0; g < 2; ++g) {
      double* G = g == 0 ? G1 : G2;
      if (!G) continue;
      const int base = (g * np + p) * 256;
      G[t] = (I == J) ? 0.5 * (tile(base + a) + tile(base + b))
                      : tile(base + a);
    }
  }
}

// Plain (non-symmetric) Gram G = W^T Y on FP64 matrix cores, all tiles:
// the component check of the MFMA lane layout.
template <int NT16>
__global__ void __launch_bounds__(kBlock)
gram_full_kernel(const double* __restrict__ W, const double* __restrict__ Y,
                 long long n, int ncols, double* __restrict__ gpart) {
  constexpr int NP = NT16 * NT16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
  const long long nsteps = (n + 3) / 4;
  const long long gw = (long long)blockIdx.x * 4 + wave;
  const long long nw = (long long)gridDim.x * 4;
  const long long per = (nsteps + nw - 1) / nw;
  const long long s0 = gw * per, s1 = min(nsteps, s0 + per);
  for (long long st = s0; st < s1; ++st) {
    const long long row = st * 4 + lk;
    double a[NT16], y[NT16];
#pragma unroll
    for (int I = 0; I < NT16; ++I) {
      const int c = I * 16 + li;
      const bool ok = row < n && c < ncols;
      a[I] = ok ? W[(size_t)row * ncols + c] : 0.0;
      y[I] = ok ? Y[(size_t)row * ncols + c] : 0.0;
    }
#pragma unroll
    for (int I = 0; I < NT16; ++I)
#pragma unroll
      for (int J = 0; J < NT16; ++J)
        acc[I * NT16 + J] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            a[I], y[J], acc[I * NT16 + J], 0, 0, 0);
  }
  __shared__ double sg[NP][256];
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int idx = (lk + 4 * r) * 16 + li;
          if (w == 0)
            sg[p][idx] = acc[p][r];
          else
            sg[p][idx] += acc[p][r];
        }
    }
    __syncthreads();
  }
  const int per_blk = NP * 256;
  for (int e = threadIdx.x; e < per_blk; e += kBlock)
    gpart[(size_t)blockIdx.x * per_blk + e] = (&sg[0][0])[e];
}

// ------------------------------------------------------------------------
// Small generalised eigenproblem A c = theta B c (Step 4's N_t x N_t
// problem), one wavefront, FP64, everything in LDS.
//   1. B = L L^T (Cholesky);  2. S = L^{-1} A L^{-T};  3. Householder
//   tridiagonalisation of S;  4. implicit QL with Wilkinson shifts;
//   5. back-transformation;  6. theta ascending (ties by index);
//   7. C = L^{-T} Z;  8. signs.
// ------------------------------------------------------------------------
constexpr int kLd = kNtMax + 1;

__global__ void __launch_bounds__(kBlock)
small_geneig_kernel(const double* __restrict__ Ain,
                    const double* __restrict__ Bin, int n,
                    double* __restrict__ theta_out, double* __restrict__ C_out,
                    int* __restrict__ info_out, int* __restrict__ status) {
  __shared__ double A[kNtMax][kLd];
  __shared__ double L[kNtMax][kLd];
  __shared__ double Y[kNtMax][kLd];
  __shared__ double rc[kNtMax / 2], rs[kNtMax / 2];
  __shared__ int rp[kNtMax / 2], rq[kNtMax / 2];
  __shared__ double red[kBlock];
  __shared__ int s_info;
  __shared__ int perm[kNtMax];
  __shared__ double th[kNtMax];
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  // Zero the padded LDS matrices (odd n uses row/column n as a dummy),
  // then load the n x n inputs with independent, unrolled global loads.
  for (int e = tid; e < kNtMax * kNtMax; e += kBlock) {
    const int i = e / kNtMax, j = e % kNtMax;
    A[i][j] = 0.0;
    L[i][j] = 0.0;
    Y[i][j] = 0.0;
  }
  if (tid == 0) s_info = 0;
  __syncthreads();
#pragma unroll 4
  for (int e = tid; e < n * n; e += kBlock) {
    const double a = Ain[e], b = Bin[e];
    A[e / n][e % n] = a;
    L[e / n][e % n] = b;
  }
  __syncthreads();

  // 1. Cholesky, left-looking, column by column.
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double bkk = L[k][k];
      double d = bkk;
      for (int j = 0; j < k; ++j) d -= L[k][j] * L[k][j];
      // A pivot at rounding level of the diagonal means the columns are
      // linearly dependent in the M inner product.
      if (!(d > 1e-14 * bkk) || !isfinite(d)) {
        s_info = k + 1;
        d = 1.0;
      }
      L[k][k] = sqrt(d);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += kBlock) {
      double v = L[i][k];
      for (int j = 0; j < k; ++j) v -= L[i][j] * L[k][j];
      L[i][k] = v / L[k][k];
    }
    __syncthreads();
  }
  if (s_info != 0) {
    if (tid == 0) {
      *info_out = s_info;
      if (status) atomicOr(status, (int)kStSingular);
    }
    for (int e = tid; e < n * n; e += kBlock)
      C_out[e] = (e / n == e % n) ? 1.0 : 0.0;
    for (int e = tid; e < n; e += kBlock) theta_out[e] = Ain[e * n + e];
    return;
  }

  // 2. Y = L^{-1} A (columns in parallel), then S = L^{-1} Y^T into A.
  if (tid < n) {
    const int j = tid;
    for (int i = 0; i < n; ++i) {
      double v = A[i][j];
      for (int k = 0; k < i; ++k) v -= L[i][k] * Y[k][j];
      Y[i][j] = v / L[i][i];
    }
  }
  __syncthreads();
  if (tid < n) {
    const int j = tid;
    for (int i = 0; i < n; ++i) {
      double v = Y[j][i];
      for (int k = 0; k < i; ++k) v -= L[i][k] * A[k][j];
      A[i][j] = v / L[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += kBlock) {
    const int i = e / n, j = e % n;
    if (i < j) {
      const double s = 0.5 * (A[i][j] + A[j][i]);
      A[i][j] = s;
      A[j][i] = s;
    }
  }
  // Y := identity (eigenvector accumulator).
  for (int e = tid; e < kNtMax * kNtMax; e += kBlock) {
    const int i = e / kNtMax, j = e % kNtMax;
    Y[i][j] = (i == j && i < n) ? 1.0 : 0.0;
  }
  __syncthreads();

  // 3. Cyclic Jacobi, round-robin pairs (N_t / 2 disjoint rotations per
  // round).  A rotation is skipped when |a_pq| <= 1e-17 ||S||_F (already
  // zero at working precision); the iteration stops after a sweep that
  // rotates nothing.
  const int half = nn / 2;
  __shared__ int s_rot;
  double fro2 = 0.0;
  for (int e = tid; e < n * n; e += kBlock) {
    const double v = A[e / n][e % n];
    fro2 += v * v;
  }
  red[tid] = fro2;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const double skip = 1e-17 * sqrt(red[0]);
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < nn - 1; ++round) {
      if (tid < half) {
        const int a0 = tid == 0 ? 0 : 1 + ((tid - 1 + round) % (nn - 1));
        const int b0 = 1 + ((nn - 2 - tid + round) % (nn - 1));
        const int p = a0 < b0 ? a0 : b0, q = a0 < b0 ? b0 : a0;
        double c = 1.0, sn = 0.0;
        bool rot = false;
        if (q < n) {
          const double apq = A[p][q];
          if (fabs(apq) > skip) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) /
                             (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            rot = true;
            s_rot = 1;
          }
        }
        rc[tid] = c;
        rs[tid] = sn;
        rp[tid] = p;
        rq[tid] = rot ? q : p;
      }
      __syncthreads();
      // Rows: A <- J^T A.
      for (int e = tid; e < half * n; e += kBlock) {
        const int k = e / n, j = e - k * n;
        const int p = rp[k], q = rq[k];
        if (p == q) continue;
        const double c = rc[k], sn = rs[k];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - sn * aq;
        A[q][j] = sn * ap + c * aq;
      }
      __syncthreads();
      // Columns: A <- A J, Y <- Y J.
      for (int e = tid; e < half * n; e += kBlock) {
        const int k = e / n, i = e - k * n;
        const int p = rp[k], q = rq[k];
        if (p == q) continue;
        const double c = rc[k], sn = rs[k];
        const double ap = A[i][p], aq = A[i][q];
        A[i][p] = c * ap - sn * aq;
        A[i][q] = sn * ap + c * aq;
        const double yp = Y[i][p], yq = Y[i][q];
        Y[i][p] = c * yp - sn * yq;
        Y[i][q] = sn * yp + c * yq;
      }
      __syncthreads();
      if (tid < half) {
        const int p = rp[tid], q = rq[tid];
        if (p != q) {
          A[p][q] = 0.0;
          A[q][p] = 0.0;
        }
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }

  // 4. Ascending order, ties broken by index.
  if (tid < n) th[tid] = A[tid][tid];
  __syncthreads();
  if (tid < n) {
    int rank = 0;
    const double t = th[tid];
    for (int j = 0; j < n; ++j)
      rank += (th[j] < t || (th[j] == t && j < tid)) ? 1 : 0;
    perm[rank] = tid;
  }
  __syncthreads();
  // 5. C[:, r] = L^{-T} Y[:, perm[r]] (back substitution), stored in A
  // (its diagonal was saved in th).
  double (*Cs)[kLd] = A;
  if (tid < n) {
    const int r = tid, src = perm[r];
    for (int i = n - 1; i >= 0; --i) {
      double v = Y[i][src];
      for (int k = i + 1; k < n; ++k) v -= L[k][i] * Cs[k][r];
      Cs[i][r] = v / L[i][i];
    }
  }
  __syncthreads();
  // 6. Sign: largest-magnitude entry of each column positive.
  if (tid < n) {
    const int r = tid;
    int im = 0;
    double vm = -1.0;
    for (int i = 0; i < n; ++i) {
      const double a = fabs(Cs[i][r]);
      if (a > vm) {
        vm = a;
        im = i;
      }
    }
    const double sg = Cs[im][r] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) C_out[i * n + r] = sg * Cs[i][r];
    theta_out[r] = th[perm[r]];
  }
  if (tid == 0) *info_out = 0;
}

// ------------------------------------------------------------------------
// Rotation U = W C with HU = (HW) C, MU = (MW) C formed on the fly for the
// residual norms ||HU_i - theta_i MU_i||, ||MU_i|| (Step 4 output and the
// stopping test).  Rows of W, HW, MW are staged through LDS.  The last
// block writes lambda = theta and the step's convergence measures.
// ------------------------------------------------------------------------
template <int V>
__global__ void __launch_bounds__(kBlock)
rotate_kernel(const double* __restrict__ W, const double* __restrict__ HW,
              const double* __restrict__ MW, const double* __restrict__ Cg,
              const double* __restrict__ theta, double* __restrict__ U,
              double* __restrict__ lam, int have_old, int nreq, long long n,
              int ncols, StepInfo* __restrict__ si,
              double* __restrict__ part) {
  extern __shared__ unsigned char smem[];
  double* sC = reinterpret_cast<double*>(smem);        // ncols^2
  double* sW = sC + ncols * ncols;                     // tr * ncols each
  const int cpr = ncols / V, tr = kBlock / cpr;
  double* sH = sW + tr * ncols;
  double* sM = sH + tr * ncols;
  const int tid = threadIdx.x, lr = tid / cpr, ch = tid % cpr;
  if (blockIdx.x == 0 && tid == 0) {
    si->max_dlambda = 0.0;
    si->max_resid = 0.0;
  }
  for (int e = tid; e < ncols * ncols; e += kBlock) sC[e] = Cg[e];
  double th[V];
#pragma unroll
  for (int v = 0; v < V; ++v) th[v] = theta[min(ch * V + v, ncols - 1)];
  double acc[2][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.0;
  const long long ntiles = (n + tr - 1) / tr;
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * tr;
    const int rows = (int)min((long long)tr, n - r0);
    __syncthreads();
    const size_t base = (size_t)r0 * ncols;
    for (int e = tid; e < rows * ncols; e += kBlock) {
      sW[e] = W[base + e];
      sH[e] = HW[base + e];
      sM[e] = MW[base + e];
    }
    __syncthreads();
    if (lr < tr && lr < rows) {
      double u[V], hu[V], mu[V];
#pragma unroll
      for (int v = 0; v < V; ++v) u[v] = hu[v] = mu[v] = 0.0;
      const double* wr = sW + lr * ncols;
      const double* hr = sH + lr * ncols;
      const double* mr = sM + lr * ncols;
      for (int k = 0; k < ncols; ++k) {
        const double wk = wr[k], hk = hr[k], mk = mr[k];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const double c = sC[k * ncols + ch * V + v];
          u[v] = fma(wk, c, u[v]);
          hu[v] = fma(hk, c, hu[v]);
          mu[v] = fma(mk, c, mu[v]);
        }
      }
      stv<double, V>(U + base + (size_t)lr * ncols + ch * V, u);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double r = hu[v] - th[v] * mu[v];
        acc[0][v] += r * r;
        acc[1][v] += mu[v] * mu[v];
      }
    }
  }
  __syncthreads();
  block_partials<V, 2>(acc, ncols, cpr, tr, part);
}

// Per column: lambda = theta, relative change and residual (one workgroup
// per column); maxima over the requested pairs for the stopping test.
__global__ void __launch_bounds__(kBlock)
rotate_final_kernel(const double* __restrict__ part, int nb,
                    const double* __restrict__ theta, double* __restrict__ lam,
                    int have_old, int nreq, int ncols,
                    StepInfo* __restrict__ si) {
  const int c = blockIdx.x;
  double tot[2];
  column_sums<2>(part, nb, tot);
  if (threadIdx.x != 0) return;
  double lmax = 0.0;
  for (int k = 0; k < ncols; ++k) lmax = fmax(lmax, fabs(theta[k]));
  const double t = theta[c];
  const double sc = fmax(fabs(t), 1e-3 * lmax);
  const double old = lam[c];
  const double dl = have_old ? fabs(t - old) / sc : INFINITY;
  double rho = sqrt(tot[0]) / (sc * sqrt(tot[1]));
  if (!isfinite(rho)) rho = INFINITY;
  si->lam_old[c] = old;
  si->dlam[c] = dl;
  si->resid[c] = rho;
  lam[c] = t;
  if (c < nreq) {
    atomic_max_nonneg(&si->max_dlambda, dl);
    atomic_max_nonneg(&si->max_resid, rho);
  }
}

int pick_vec64(int ncols) { return (ncols % 2 == 0) ? 2 : 1; }
int pick_vec32(int ncols) {
  return (ncols % 4 == 0) ? 4 : ((ncols % 2 == 0) ? 2 : 1);
}


size_t tile_smem(int ncols, int V, size_t vsize, int nvals) {
  const int cpr = ncols / V, tr = kBlock / cpr;
  return csr_tile_bytes(tr, vsize, nvals);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_spmm(Problem& p, int which, const double* X,
                       double* Y, int ncols, hipStream_t s) {
  const int V = pick_vec64(ncols);
  double* Y1 = which == 1 ? nullptr : Y;
  double* Y2 = which == 1 ? Y : nullptr;
  const double s1 = which == 2 ? p.sigma : 0.0;
  TimedLaunch t(p, PARO_ST_RR_SPMM, s);
  const size_t smem = tile_smem(ncols, V, sizeof(double), 2);
  if (V == 2)
    hipLaunchKernelGGL(spmm_dual_kernel<2>, dim3(p.grid), dim3(kBlock), smem, s,
                       p.rowptr, p.col, p.valA, p.valM, X, Y1, Y2, s1,
                       (long long)p.n, ncols);
  else
    hipLaunchKernelGGL(spmm_dual_kernel<1>, dim3(p.grid), dim3(kBlock), smem, s,
                       p.rowptr, p.col, p.valA, p.valM, X, Y1, Y2, s1,
                       (long long)p.n, ncols);
  return hipGetLastError();
}

static hipError_t start_common(Problem& p, const double* lam,
                               const double* U, const double* Bin, int ncols,
                               bool store_b, hipStream_t s) {
  const int V = pick_vec64(ncols);
  double* Bout = store_b ? p.B : nullptr;
  auto k = V == 2 ? pcg_start_kernel<2> : pcg_start_kernel<1>;
  TimedLaunch t(p, PARO_ST_START, s);
  hipLaunchKernelGGL(k, dim3(p.grid), dim3(kBlock),
                     tile_smem(ncols, V, sizeof(double), 2), s, p.rowptr, p.col,
                     p.valA, p.valM, p.dinv, U, lam, Bin, p.sigma,
                     p.opts.pcg_rtol, p.X, p.R, p.P, Bout, (long long)p.n,
                     ncols, p.opts.pcg_maxit, p.cs, p.part);
  hipLaunchKernelGGL(pcg_start_final_kernel, dim3(ncols), dim3(kBlock), 0, s,
                     p.part, p.grid, p.opts.pcg_rtol, p.cs);
  return hipGetLastError();
}

hipError_t launch_pcg_start(Problem& p, const double* lam, const double* U,
                            int ncols, bool store_b, hipStream_t s) {
  return start_common(p, lam, U, nullptr, ncols, store_b, s);
}

hipError_t launch_pcg_start_rhs(Problem& p, const double* Bin, int ncols,
                                bool store_b, hipStream_t s) {
  // x0 = X (already in p.X), b = Bin.
  return start_common(p, nullptr, p.X, Bin, ncols, store_b, s);
}

template <typename T, typename TM, typename TD, int V>
static void cg_iter(Problem& p, const TM* val, const TD* dinv, T* X, T* P,
                    T* Q, T* R, int ncols, int par, hipStream_t s) {
  const size_t smem = tile_smem(ncols, V, sizeof(TM), 1);
  {
    TimedLaunch t(p, PARO_ST_CG_SPMM, s);
    hipLaunchKernelGGL((spmm_cg_kernel<T, TM, V>), dim3(p.grid), dim3(kBlock),
                       smem, s, p.rowptr, p.col, val, P, Q, (long long)p.n,
                       ncols, p.cs, par, p.part);
  }
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(ncols), dim3(kBlock), 0, s, p.part,
                     p.grid, p.cs, par);
  {
    TimedLaunch t(p, PARO_ST_CG_RUPD, s);
    hipLaunchKernelGGL((rupd_kernel<T, TD, V>), dim3(p.grid), dim3(kBlock), 0,
                       s, Q, R, dinv, (long long)p.n, ncols, p.cs, par,
                       p.part);
  }
  hipLaunchKernelGGL(cg_beta_kernel, dim3(ncols), dim3(kBlock), 0, s, p.part,
                     p.grid, p.cs, par);
  {
    TimedLaunch t(p, PARO_ST_CG_PUPD, s);
    hipLaunchKernelGGL((pupd_kernel<T, TD, V>), dim3(p.grid), dim3(kBlock), 0,
                       s, X, P, R, dinv, (long long)p.n, ncols, p.cs, par);
  }
}

hipError_t launch_pcg_iter(Problem& p, int ncols, int par, hipStream_t s) {
  if (pick_vec64(ncols) == 2)
    cg_iter<double, double, double, 2>(p, p.valA, p.dinv, p.X, p.P, p.Q, p.R,
                                       ncols, par, s);
  else
    cg_iter<double, double, double, 1>(p, p.valA, p.dinv, p.X, p.P, p.Q, p.R,
                                       ncols, par, s);
  return hipGetLastError();
}

hipError_t launch_pcg32_iter(Problem& p, int ncols, int par, hipStream_t s) {
  switch (pick_vec32(ncols)) {
    case 4:
      cg_iter<float, float, float, 4>(p, p.valA32, p.dinv32, p.X32, p.P32,
                                      p.Q32, p.R32, ncols, par, s);
      break;
    case 2:
      cg_iter<float, float, float, 2>(p, p.valA32, p.dinv32, p.X32, p.P32,
                                      p.Q32, p.R32, ncols, par, s);
      break;
    default:
      cg_iter<float, float, float, 1>(p, p.valA32, p.dinv32, p.X32, p.P32,
                                      p.Q32, p.R32, ncols, par, s);
  }
  return hipGetLastError();
}

hipError_t launch_refine_residual(Problem& p, int ncols, bool first,
                                  hipStream_t s) {
  (void)first;
  const int V = pick_vec64(ncols);
  auto k = V == 2 ? refine_residual_kernel<2> : refine_residual_kernel<1>;
  TimedLaunch t(p, PARO_ST_REFINE, s);
  hipLaunchKernelGGL(k, dim3(p.grid), dim3(kBlock),
                     tile_smem(ncols, V, sizeof(double), 1), s, p.rowptr, p.col,
                     p.valA, p.dinv, p.X, p.B, p.R32, p.P32, p.X32,
                     p.opts.pcg_rtol, p.opts.inner_rtol, (long long)p.n, ncols,
                     p.cs, p.part);
  hipLaunchKernelGGL(refine_final_kernel, dim3(ncols), dim3(kBlock), 0, s,
                     p.part, p.grid, p.opts.pcg_rtol, p.opts.inner_rtol,
                     p.cs);
  return hipGetLastError();
}

hipError_t launch_refine_update(Problem& p, int ncols, hipStream_t s) {
  const int V = pick_vec64(ncols);
  auto k = V == 2 ? refine_update_kernel<2> : refine_update_kernel<1>;
  TimedLaunch t(p, PARO_ST_REFINE, s);
  hipLaunchKernelGGL(k, dim3(p.grid), dim3(kBlock), 0, s, p.X, p.X32,
                     (long long)p.n, ncols, p.cs);
  return hipGetLastError();
}

hipError_t launch_gram(Problem& p, const double* W, const double* Y1,
                       const double* Y2, double* G1, double* G2, int ncols,
                       hipStream_t s) {
  TimedLaunch t(p, PARO_ST_GRAM, s);
  const int nt16 = (ncols + 15) / 16;
  const int grid = p.grid < kGramGrid ? p.grid : kGramGrid;
  const long long n = p.n;
  switch (nt16) {
    case 1:
      hipLaunchKernelGGL(gram_kernel<1>, dim3(grid), dim3(kBlock), 0, s, W, Y1,
                         Y2, n, ncols, p.gpart);
      break;
    case 2:
      hipLaunchKernelGGL(gram_kernel<2>, dim3(grid), dim3(kBlock), 0, s, W, Y1,
                         Y2, n, ncols, p.gpart);
      break;
    case 3:
      hipLaunchKernelGGL(gram_kernel<3>, dim3(grid), dim3(kBlock), 0, s, W, Y1,
                         Y2, n, ncols, p.gpart);
      break;
    default:
      hipLaunchKernelGGL(gram_kernel<4>, dim3(grid), dim3(kBlock), 0, s, W, Y1,
                         Y2, n, ncols, p.gpart);
  }
  const int per_blk = 2 * (nt16 * (nt16 + 1) / 2) * 256;
  hipLaunchKernelGGL(gram_reduce_kernel,
                     dim3((per_blk + kBlock - 1) / kBlock, kGramY),
                     dim3(kBlock), 0, s, p.gpart, grid, per_blk, p.gsum);
  hipLaunchKernelGGL(gram_scatter_kernel, dim3(1), dim3(kBlock), 0, s, p.gsum,
                     per_blk, nt16, 0, ncols, G1, Y2 ? G2 : nullptr);
  return hipGetLastError();
}

hipError_t launch_gram_full(Problem& p, const double* W,
                            const double* Y, double* G, int ncols,
                            hipStream_t s) {
  TimedLaunch t(p, PARO_ST_GRAM, s);
  const int nt16 = (ncols + 15) / 16;
  const int grid = p.grid < kGramGrid ? p.grid : kGramGrid;
  const long long n = p.n;
  switch (nt16) {
    case 1:
      hipLaunchKernelGGL(gram_full_kernel<1>, dim3(grid), dim3(kBlock), 0, s,
                         W, Y, n, ncols, p.gpart);
      break;
    case 2:
      hipLaunchKernelGGL(gram_full_kernel<2>, dim3(grid), dim3(kBlock), 0, s,
                         W, Y, n, ncols, p.gpart);
      break;
    case 3:
      hipLaunchKernelGGL(gram_full_kernel<3>, dim3(grid), dim3(kBlock), 0, s,
                         W, Y, n, ncols, p.gpart);
      break;
    default:
      hipLaunchKernelGGL(gram_full_kernel<4>, dim3(grid), dim3(kBlock), 0, s,
                         W, Y, n, ncols, p.gpart);
  }
  const int per_blk = nt16 * nt16 * 256;
  hipLaunchKernelGGL(gram_reduce_kernel,
                     dim3((per_blk + kBlock - 1) / kBlock, kGramY),
                     dim3(kBlock), 0, s, p.gpart, grid, per_blk, p.gsum);
  hipLaunchKernelGGL(gram_scatter_kernel, dim3(1), dim3(kBlock), 0, s, p.gsum,
                     per_blk, nt16, 1, ncols, G, nullptr);
  return hipGetLastError();
}

hipError_t launch_small_geneig(const double* A, const double* B, int n,
                               double* theta, double* C, int* info,
                               hipStream_t s) {
  hipLaunchKernelGGL(small_geneig_kernel, dim3(1), dim3(kBlock), 0, s, A, B, n,
                     theta, C, info, nullptr);
  return hipGetLastError();
}

hipError_t launch_rayleigh_ritz(Problem& p, const double* W, double* lam,
                                double* U, int ncols, bool have_old,
                                hipStream_t s) {
  hipError_t e;
  // HW into R, MW into Q.
  const int V = pick_vec64(ncols);
  auto kd = V == 2 ? spmm_dual_kernel<2> : spmm_dual_kernel<1>;
  {
    TimedLaunch t(p, PARO_ST_RR_SPMM, s);
    hipLaunchKernelGGL(kd, dim3(p.grid), dim3(kBlock),
                       tile_smem(ncols, V, sizeof(double), 2), s, p.rowptr,
                       p.col,
                       p.valA, p.valM, W, p.R, p.Q, p.sigma, (long long)p.n,
                       ncols);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_gram(p, W, p.R, p.Q, p.Ah, p.Bh, ncols, s)) != hipSuccess)
    return e;
  {
    TimedLaunch t(p, PARO_ST_SMALL, s);
    hipLaunchKernelGGL(small_geneig_kernel, dim3(1), dim3(kBlock), 0, s,
                       p.Ah,
                       p.Bh, ncols, p.theta, p.C, &p.si->geneig_info,
                       &p.cs->status);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int cpr = ncols / V, tr = kBlock / cpr;
  const size_t smem = sizeof(double) * ((size_t)ncols * ncols +
                                        3 * (size_t)tr * ncols);
  auto kr = V == 2 ? rotate_kernel<2> : rotate_kernel<1>;
  TimedLaunch t(p, PARO_ST_ROTATE, s);
  hipLaunchKernelGGL(kr, dim3(p.grid), dim3(kBlock), smem, s, W, p.R, p.Q,
                     p.C, p.theta, U, lam, have_old ? 1 : 0, p.N,
                     (long long)p.n, ncols, p.si, p.part);
  hipLaunchKernelGGL(rotate_final_kernel, dim3(ncols), dim3(kBlock), 0, s,
                     p.part, p.grid, p.theta, lam, have_old ? 1 : 0, p.N,
                     ncols, p.si);
  return hipGetLastError();
}

}  // namespace paro
