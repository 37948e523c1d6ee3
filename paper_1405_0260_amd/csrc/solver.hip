// Kernels of one ParO step on gfx950: block Jacobi-PCG for the Nt source
// problems of Step 3 and the Rayleigh-Ritz projection of Step 4.
//
// Batching.  Every kernel serves a table of problems (Desc): problem p owns
// a contiguous range of blocks, so one launch advances all problems of a
// batch; a single problem is a table of one.  Per-problem arithmetic and
// summation order do not depend on the other problems of the table.
//
// Data layout.  Orbital blocks are row-major n x Nt (orbital fastest), so a
// stencil neighbour gathered by the once-per-step kernels is Nt contiguous
// values; there a thread owns V consecutive columns of one row ("chunk"),
// a workgroup a tile of kBlock / (Nt / V) rows.  The CG vectors are
// chunk-major (see the CG section): a thread owns one row of one chunk.
// A problem's blocks walk its tiles in eight contiguous slabs, slab =
// block mod 8, so that each XCD sweeps one slab of rows and keeps its halo
// in its own L2.  The operators are stored in stencil order (15
// coefficients per row, implicit neighbours).
//
// Reductions (per-column dot products) are two-stage and deterministic:
// each workgroup writes its partial sums, then a finalize kernel with one
// workgroup per (problem, column) adds them in a fixed order.  No float
// atomics.
#include <hip/hip_cooperative_groups.h>

#include <cmath>

#include "kuhn.h"
#include "paro_internal.h"

namespace paro {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;
constexpr size_t kPartStride = (size_t)kGridMax * kNtMax;

// V consecutive values loaded or stored as one vector access.
template <typename T, int V>
struct VecT {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecT<T, 1> {
  typedef T type;
};

// Launch bounds of the streaming kernels: 256 threads; PARO_MIN_WAVES
// (waves per SIMD the register allocation must allow) is a tuning knob.
#ifdef PARO_MIN_WAVES
#define PARO_STREAM_BOUNDS __launch_bounds__(kBlock, PARO_MIN_WAVES)
#else
#define PARO_STREAM_BOUNDS __launch_bounds__(kBlock)
#endif

// Pointers read from a descriptor table are generic (flat) to the
// compiler; re-qualified as global memory they give global_load /
// global_store, which do not wait on LDS traffic.
#define PARO_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const PARO_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(PARO_GLOBAL T*)p = v;
}

template <typename T, int V>
__device__ __forceinline__ void ldv(const T* p, T (&o)[V]) {
  typedef typename VecT<T, V>::type W;
  const W w = *(const PARO_GLOBAL W*)p;
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
  *(PARO_GLOBAL W*)p = w;
}

// The problem that owns block `bid` (binary search on the first blocks).
__device__ __forceinline__ int owner(const Desc* D, int nprob, int bid,
                                     bool gram) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((gram ? D[mid].g0 : D[mid].b0) <= bid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Tiles of local block lb (of nb) in an XCD-sliced grid-stride walk.
struct TileWalk {
  long long t, end, step;
};
__device__ __forceinline__ TileWalk tile_walk(long long ntiles, int lb,
                                              int nb) {
  const int x = lb % kXcd, l = lb / kXcd, gx = nb / kXcd;
  const long long chunk = (ntiles + kXcd - 1) / kXcd;
  TileWalk w;
  w.t = (long long)x * chunk + l;
  w.end = min(ntiles, (long long)(x + 1) * chunk);
  w.step = gx;
  return w;
}

// Per-column workgroup reduction of per-thread partials acc[a][v]
// (thread = (lr, ch)), written column-major: part[a][c][vb] (ns segments).
// red: LDS of NA * kBlock * V doubles, owned by the calling kernel.  Ends
// with a barrier, so red may be reused at once.
template <int V, int NA>
__device__ void block_partials(const double (&acc)[NA][V], int ncols, int cpr,
                               int tr, int vb, int ns,
                               double* __restrict__ part,
                               double* __restrict__ red) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int v = 0; v < V; ++v) red[(a * kBlock + tid) * V + v] = acc[a][v];
  __syncthreads();
  if (tid < ncols) {
    const int ch = tid / V, v = tid % V;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const double* ra = red + a * kBlock * V;
      double s = 0.0;
      for (int lr = 0; lr < tr; ++lr) s += ra[(lr * cpr + ch) * V + v];
      stg(part + a * kPartStride + (size_t)tid * ns + vb, s);
    }
  }
  __syncthreads();
}

// block_partials for a thread that holds the values of tile row lr and
// chunk ch (slot lr cpr + ch, whatever its thread index; slot < 0: none):
// the same sums in the same order.
template <int NA, int V>
__device__ void block_partials_slot(const double (&acc)[NA][V], int slot,
                                    int ncols, int cpr, int tr, int vb,
                                    int ns, double* __restrict__ part,
                                    double* __restrict__ red) {
  const int tid = threadIdx.x;
  if (slot >= 0)
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int v = 0; v < V; ++v)
        red[(a * kBlock + slot) * V + v] = acc[a][v];
  __syncthreads();
  if (tid < ncols) {
    const int ch = tid / V, v = tid % V;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const double* ra = red + a * kBlock * V;
      double s = 0.0;
      for (int lr = 0; lr < tr; ++lr) s += ra[(lr * cpr + ch) * V + v];
      stg(part + a * kPartStride + (size_t)tid * ns + vb, s);
    }
  }
  __syncthreads();
}

// Finalisers run one wavefront per (column, problem).
constexpr int kFinal = 64;

// In a finalize kernel: the fixed-order sum of part[a][c][0..nb) (lane l
// adds segments l, l + 64, ... in ascending order, then a butterfly over
// the wavefront, whose lanes all end with the same bits).  The loads of 16
// segments per lane are issued together (clamped addresses, masked adds):
// the partials come from every XCD, so each round trip costs the full
// fabric latency.  Every lane receives the sums.  KU (loads per lane in
// flight) changes the register use, not the order of the additions.
template <int NA, int kU = 16>
__device__ __forceinline__ void column_sums(const double* __restrict__ part,
                                            size_t stride, int c, int nb,
                                            double (&out)[NA]) {
  const int t = threadIdx.x & (kFinal - 1);  // lane of the wavefront
  double v[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) v[a] = 0.0;
  for (int b0 = 0; b0 < nb; b0 += kU * kFinal) {
    double x[NA][kU];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const double* src = part + a * stride + (size_t)c * nb;
#pragma unroll
      for (int i = 0; i < kU; ++i)
        x[a][i] = ldg(src + min(b0 + t + i * kFinal, nb - 1));
    }
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int i = 0; i < kU; ++i)
        v[a] = (b0 + t + i * kFinal < nb) ? v[a] + x[a][i] : v[a];
  }
#pragma unroll
  for (int a = 0; a < NA; ++a) {
#pragma unroll
    for (int o = kFinal / 2; o > 0; o >>= 1)
      v[a] += __shfl_xor(v[a], o, kFinal);
    out[a] = v[a];
  }
}

// Max of non-negative doubles through their bit patterns (order-free).
__device__ __forceinline__ void atomic_max_nonneg(double* dst, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(dst),
            (unsigned long long)__double_as_longlong(v));
}

// Whether any of the V columns of chunk ch is set in act (loads issued
// together: out-of-range columns read the last column and are masked).
__device__ __forceinline__ bool chunk_active(const int* act, int ch, int V,
                                             int ncols) {
  int a = 0;
  for (int v = 0; v < V; ++v) {
    const int c = ch * V + v;
    const int x = ldg(act + min(c, ncols - 1));
    a |= c < ncols ? x : 0;
  }
  return a != 0;
}

// Active columns as a mask (lane c of each wavefront reads column c's
// flag; at most 64 columns): one load for every chunk of a block.
__device__ __forceinline__ unsigned long long active_mask(const int* act,
                                                         int ncols) {
  const int lane = threadIdx.x & 63;
  const int x = ldg(act + min(lane, ncols - 1));  // unconditional load
  return __ballot(lane < ncols && x != 0);
}
template <int V>
__device__ __forceinline__ bool chunk_in_mask(unsigned long long m, int ch) {
  return ((m >> (ch * V)) & ((1ull << V) - 1)) != 0;
}

// The 15-point Kuhn stencil: neighbour offsets (x, y, z) in ascending
// linear order (x fastest); offset 7 is the row itself.
__host__ __device__ constexpr int st_off(int s, int a) {
  constexpr int t[kStencil][3] = {
      {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
      {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
      {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};
  return t[s][a];
}
constexpr int kSelf = 7;


// Stencil product of one row (interior vertex (i, j, k) of an mx x my x mz
// grid): y1 += a_s X[row + off_s] (and y2 += b_s X[row + off_s] if TWO)
// over the 15 offsets in ascending order, the gathers issued in groups of
// G (more overlap against more registers).  wa, wb: the row's first
// coefficient, either in a staged LDS tile (STAGED, stride tr) or in the
// stencil-order matrix itself (stride n); a coefficient is 0 where the
// neighbour lies outside the box, whose slot then reads the row itself.
// self receives X[row].
template <typename T, typename TM, int V, bool TWO, int G, bool STAGED>
__device__ __forceinline__ void stencil_product(
    const TM* __restrict__ wa, const TM* __restrict__ wb, long long stride,
    int mx, int my, int mz, long long row, const T* X, int ncols, int off,
    T (&y1)[V], T (&y2)[V], T (&self)[V]) {
  const unsigned r = (unsigned)row;
  const unsigned q = r / (unsigned)mx;
  const int i = (int)(r - q * (unsigned)mx);
  const unsigned k = q / (unsigned)my;
  const int j = (int)(q - k * (unsigned)my);
  // Row base; neighbour steps are uniform offsets from it.
  const T* xr = X + (size_t)row * ncols + off;
#pragma unroll
  for (int s0 = 0; s0 < kStencil; s0 += G) {
    T x[G][V];
    TM a[G], b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int s = s0 + g;
      if (s >= kStencil) break;
      const int ox = st_off(s, 0), oy = st_off(s, 1), oz = st_off(s, 2);
      const bool ok = (unsigned)(i + ox) < (unsigned)mx &&
                      (unsigned)(j + oy) < (unsigned)my &&
                      (unsigned)((int)k + oz) < (unsigned)mz;
      const int step = (ox + mx * (oy + my * oz)) * ncols;
      ldv<T, V>(xr + (ok ? step : 0), x[g]);
      if (STAGED) {
        a[g] = wa[s * stride];
        if (TWO) b[g] = wb[s * stride];
      } else {
        a[g] = ldg(wa + (size_t)s * stride);
        if (TWO) b[g] = ldg(wb + (size_t)s * stride);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int s = s0 + g;
      if (s >= kStencil) break;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        y1[v] = fma((T)a[g], x[g][v], y1[v]);
        if (TWO) y2[v] = fma((T)b[g], x[g][v], y2[v]);
      }
      if (s == kSelf) {
#pragma unroll
        for (int v = 0; v < V; ++v) self[v] = x[g][v];
      }
    }
    // Keep the groups apart: the next group's loads are not hoisted above
    // this group's arithmetic (bounds the registers in flight).
    if (G < kStencil) __builtin_amdgcn_sched_barrier(0);
  }
}

// Stage the stencil-order coefficients of rows [r0, r0 + rows) into LDS,
// w[s * tr + (row - r0)], with coalesced loads.  All threads of the block
// call it; the first barrier protects the previous tile.
template <typename TM, bool TWO>
__device__ __forceinline__ void stage_weights(const TM* __restrict__ da,
                                              const TM* __restrict__ db,
                                              long long n, long long r0,
                                              int rows, int tr,
                                              TM* __restrict__ wa,
                                              TM* __restrict__ wb) {
  __syncthreads();
  for (int e = threadIdx.x; e < kStencil * rows; e += kBlock) {
    const int s = e / rows, lr = e - s * rows;
    wa[s * tr + lr] = ldg(da + (size_t)s * n + r0 + lr);
    if (TWO) wb[s * tr + lr] = ldg(db + (size_t)s * n + r0 + lr);
  }
  __syncthreads();
}

// LDS bytes of a staged coefficient tile (tr rows, nmat matrices).
constexpr size_t weights_bytes(int tr, size_t vsize, int nmat) {
  return (size_t)kStencil * tr * vsize * nmat;
}

// Thread geometry of virtual block vb of a problem's streaming kernel.
struct Geo {
  int lb, nb;             // virtual block and the problem's segment count
  int cpr, tr, lr, ch;    // chunks per row, rows per tile, local row, chunk
  long long ntiles;
};
template <int V>
__device__ __forceinline__ Geo geo_of(const Desc& d, int vb) {
  Geo g;
  g.lb = vb;
  g.nb = d.ns;
  g.cpr = d.ncols / V;
  g.tr = kBlock / g.cpr;
  g.lr = threadIdx.x / g.cpr;
  g.ch = threadIdx.x % g.cpr;
  g.ntiles = (d.n + g.tr - 1) / g.tr;
  return g;
}

// The virtual blocks of the real block that runs this code: its problem
// `d` (owner of blockIdx.x) and the segments vb = lb, lb + nb, ... < ns.
// BODY runs once per segment with VV (constexpr) the problem's FP64
// vector width (2 or 1); a barrier separates consecutive segments.
#define PARO_VB_CASE(W, BODY) \
  {                           \
    constexpr int VV = W;     \
    BODY;                     \
  }
#define PARO_VB_LOOP_(D, nprob, VWIDTH, DISPATCH)              \
  {                                                          \
    const int p_ = owner(D, nprob, blockIdx.x, false);       \
    const Desc& d = D[p_];                                   \
    const int vw_ = (VWIDTH);                                \
    for (int vb = blockIdx.x - d.b0; vb < d.ns; vb += d.nb) { \
      DISPATCH;                                              \
      __syncthreads();                                       \
    }                                                        \
  }
// VFIX != 0: every problem of the launch has that width (one code path);
// VFIX = 0: each block branches on its problem's width.
#define PARO_VB_LOOP64(D, nprob, VFIX, BODY)                           \
  PARO_VB_LOOP_(D, nprob, d.v64,                                       \
                if constexpr (VFIX != 0) PARO_VB_CASE(VFIX, BODY) else if \
                    (vw_ == 2) PARO_VB_CASE(2, BODY) else PARO_VB_CASE(1, BODY))

// alpha_c = (r.z)_c / (p.q)_c for one column of a problem (one
// wavefront; the persistent CG's alpha phase).  Also clears the next
// parity's active count for the beta phase.
__device__ __forceinline__ void alpha_pair(const Desc& d, int c, int par) {
  const int lane = threadIdx.x & (kFinal - 1);
  ColState* cs = d.cs;
  if (c >= d.ncols) return;
  if (cs->n_active[par] == 0) {
    // Nothing ran in this iteration: keep the next parity idle too, so
    // that launches queued after convergence stay no-ops.
    if (c == 0 && lane == 0) cs->n_active[par ^ 1] = 0;
    return;
  }
  if (c == 0 && lane == 0) {
    cs->n_active[par ^ 1] = 0;
    cs->cg_iters += 1;
  }
  if (!cs->act[par][c]) return;
  double tot[1];
  column_sums<1>(d.pqp, 0, c, d.pqn, tot);
  if (lane == 0) {
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
      atomicOr(&cs->status, isfinite(pq) ? (int)kStNotSpd : (int)kStNonFinite);
      cs->alpha[c] = 0.0;
    } else {
      cs->alpha[c] = cs->rzp[par][c] / pq;
    }
  }
}


// The end of a CG iteration for one active column from its new r.z and
// r.r: beta, the iteration count and whether the column goes on.  Reads
// only state of parity `par`, so every unit of a kernel may evaluate it
// while one of them commits (beta_commit writes parity par ^ 1 and the
// latest copies).
struct BetaStep {
  double beta;
  int it, next, bad;
};
// The parity-par state beta_step reads, loaded ahead of the partials.
struct BetaIn {
  double rzp, tol2;
  int itp, maxit, status;
};
__device__ __forceinline__ BetaIn beta_in(const ColState* cs, int c,
                                          int par) {
  BetaIn q;
  q.rzp = ldg(&cs->rzp[par][c]);
  q.tol2 = ldg(&cs->tol2[c]);
  q.itp = ldg(&cs->itp[par][c]);
  q.maxit = ldg(&cs->maxit);
  q.status = ldg(&cs->status);
  return q;
}
__device__ __forceinline__ BetaStep beta_step(const BetaIn& q, double rz,
                                              double rr) {
  BetaStep b;
  b.bad = !isfinite(rz) || !isfinite(rr);
  b.beta = b.bad ? 0.0 : rz / q.rzp;
  b.it = q.itp + 1;
  const bool more = rr > q.tol2;
  b.next = (!b.bad && more && b.it < q.maxit && !(q.status & kStNotSpd))
               ? 1 : 0;
  return b;
}
__device__ __forceinline__ void beta_commit(ColState* cs, int c, int par,
                                            const BetaStep& b, double rz,
                                            double rr) {
  if (b.bad) {
    atomicOr(&cs->status, (int)kStNonFinite);
  } else {
    cs->beta[c] = b.beta;
    cs->rz[c] = rz;
    cs->rzp[par ^ 1][c] = rz;
    cs->rr[c] = rr;
    cs->iters[c] = b.it;
    cs->itp[par ^ 1][c] = b.it;
    if (rr > cs->tol2[c] && b.it >= cs->maxit)
      atomicOr(&cs->status, (int)kStNoConv);
  }
  cs->act[par ^ 1][c] = b.next;
  if (b.next) atomicAdd(&cs->n_active[par ^ 1], 1);
  atomicAdd(&cs->cg_col_iters, 1ULL);
}

// beta_c, iteration count and the stopping test of every active column
// (one wavefront; the persistent CG's beta phase); counts the columns
// active next iteration.
__device__ __forceinline__ void beta_pair(const Desc& d, int c, int par) {
  const int lane = threadIdx.x & (kFinal - 1);
  ColState* cs = d.cs;
  if (c >= d.ncols || cs->n_active[par] == 0) return;
  if (!cs->act[par][c]) {
    if (lane == 0) cs->act[par ^ 1][c] = 0;
    return;
  }
  const BetaIn q = beta_in(cs, c, par);
  double tot[2];
  column_sums<2>(d.cgp, (size_t)d.cgstride, c, d.cgn, tot);
  if (lane != 0) return;
  const BetaStep b = beta_step(q, tot[0], tot[1]);
  beta_commit(cs, c, par, b, tot[0], tot[1]);
}


// ------------------------------------------------------------------------
// The CG of the source solves, in chunk-major layout.
//
// The CG vectors (FP64: R, P, Q and Xc, a copy of the iterate; FP32 inner
// solves: R32, P32, Q32, X32) are internal to the library and stored as
// Nt / V chunks of V columns (V values = 16 bytes at full width), each an
// n x V array (cm_index), so a chunk of a row range is contiguous and a
// neighbour gather of a wavefront reads one contiguous kilobyte.  The work
// unit of the updates is (tile of kCmRows rows, chunk): a
// thread owns kCmRpt rows of the tile (rows tid, tid + 256, ...) in one
// chunk, accumulates its per-column products over them, and the unit ends
// with one wavefront reduction.  Converged chunks are skipped whole.
// Per-column partial sums are kept per (column, tile): cm_tiles(n) of them
// per column whatever the grid, so no result depends on the block count or
// on the batch.
// ------------------------------------------------------------------------

__device__ __forceinline__ size_t cm_index(long long n, long long row, int c,
                                           int V) {
  return ((size_t)(c / V) * n + row) * V + (c % V);
}

// The nonlocal share of row `row`, columns c0 .. c0 + V: Z[row] Y[:, c].
template <int V>
__device__ __forceinline__ void nl_add(const Desc& d, long long row, int c0,
                                       double (&y)[V]) {
  for (int j = 0; j < d.kz; ++j) {
    const double z = ldg(d.Zp + (size_t)row * d.kz + j);
#pragma unroll
    for (int v = 0; v < V; ++v)
      y[v] = fma(z, ldg(d.zy + j * d.ncols + c0 + v), y[v]);
  }
}

// Sum K values per lane over the wavefront (K a power of two, K <= 64).
// The first log2 K steps halve the values each lane holds (a lane keeps
// one half and adds its partner's copy of it), the rest are a butterfly;
// lane l ends with the total of value l >> (6 - log2 K), with the same
// bits on every lane that holds it.
template <int K>
__device__ __forceinline__ double wave_reduce_scatter(const double (&x)[K]) {
  const int lane = threadIdx.x & 63;
  double cur[K];
#pragma unroll
  for (int i = 0; i < K; ++i) cur[i] = x[i];
#pragma unroll
  for (int step = 0; step < 6; ++step) {
    const int o = 32 >> step;
    const int m = K >> step;
    if (m > 1) {
      const bool hi = (lane & o) != 0;
      double keep[K / 2 > 0 ? K / 2 : 1], got[K / 2 > 0 ? K / 2 : 1];
#pragma unroll
      for (int i = 0; i < m / 2; ++i) {
        const double send = hi ? cur[i] : cur[m / 2 + i];
        keep[i] = hi ? cur[m / 2 + i] : cur[i];
        got[i] = __shfl_xor(send, o, 64);
      }
#pragma unroll
      for (int i = 0; i < m / 2; ++i) cur[i] = keep[i] + got[i];
    } else {
      cur[0] += __shfl_xor(cur[0], o, 64);
    }
  }
  return cur[0];
}

// Per (column, tile) partials of a unit: K = NA * V values per lane
// (quantity-major), reduced over the wavefront, then over the four
// wavefronts in a fixed order; ws holds 4 * K doubles.  Ends with a
// barrier, so ws may be reused at once.
template <int NA, int V>
__device__ __forceinline__ void cm_unit_partials(const double (&x)[NA * V],
                                                 const Desc& d, int ch,
                                                 long long t,
                                                 double* __restrict__ ws) {
  constexpr int K = NA * V;
  constexpr int kGroup = 64 / K;
  const double tot = wave_reduce_scatter<K>(x);
  const int lane = threadIdx.x & 63;
  if ((lane & (kGroup - 1)) == 0) ws[(threadIdx.x >> 6) * K + lane / kGroup] = tot;
  __syncthreads();
  const int k = threadIdx.x;
  if (k < K) {
    const double s = ((ws[k] + ws[K + k]) + ws[2 * K + k]) + ws[3 * K + k];
    const int a = k / V, c = ch * V + k % V;
    stg(d.cgp + a * d.cgstride + (size_t)c * d.cgn + t, s);
  }
  __syncthreads();
}

// The CG operands of a problem in value type T.
template <typename T>
struct CmVecs;
template <>
struct CmVecs<double> {
  const double* diag;
  const double* dinv;
  double *X, *R, *P, *Q;
  __device__ CmVecs(const Desc& d)
      : diag(d.diagA), dinv(d.dinv), X(d.Xc), R(d.R), P(d.P), Q(d.Q) {}
};
template <>
struct CmVecs<float> {
  const float* diag;
  const float* dinv;
  float *X, *R, *P, *Q;
  __device__ CmVecs(const Desc& d)
      : diag(d.diagA32), dinv(d.dinv32), X(d.X32), R(d.R32), P(d.P32),
        Q(d.Q32) {}
};
template <typename T>
__device__ __forceinline__ int cm_width(const Desc& d) {
  return sizeof(T) == 4 ? d.v32 : d.v64;
}

// Unit u of a problem: tile u / cpr, chunk u % cpr.
struct CmUnit {
  long long t;
  int ch;
};
__device__ __forceinline__ CmUnit cm_unit(long long u, int cpr) {
  CmUnit r;
  r.t = u / cpr;
  r.ch = (int)(u - r.t * cpr);
  return r;
}

// A wavefront-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The value of the adjacent lane of a wavefront: lane - 1 (NEXT false,
// DPP wave_shr:1) or lane + 1 (NEXT true, wave_shl:1); the lane without a
// source (0, resp. 63) keeps `old`.
template <bool NEXT>
__device__ __forceinline__ int lane_shift(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, NEXT ? 0x130 : 0x138, 0xf, 0xf,
                                     false);
}
template <bool NEXT>
__device__ __forceinline__ float lane_shift(float old, float v) {
  return __int_as_float(
      lane_shift<NEXT>(__float_as_int(old), __float_as_int(v)));
}
template <bool NEXT>
__device__ __forceinline__ double lane_shift(double old, double v) {
  const long long o = __double_as_longlong(old);
  const long long x = __double_as_longlong(v);
  const unsigned lo = (unsigned)lane_shift<NEXT>((int)o, (int)x);
  const unsigned hi =
      (unsigned)lane_shift<NEXT>((int)(o >> 32), (int)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The 15 neighbour values of a thread's row (Pr: the row's V values; off:
// per-offset element steps, 0 where the neighbour lies outside the box).
// The lanes of a wavefront hold consecutive rows, so the x - 1 and x + 1
// neighbours of a row are the x-centred neighbours of the adjacent lanes'
// rows: only the 7 x-centred values are loaded and the other 8 arrive by
// a wavefront shift (lanes 0 and 63, the wavefront's halo rows, receive
// no valid shifted values).  Where a shifted value belongs to another
// grid line (x = 0 or x = mx - 1) its coefficient is 0.
template <typename T, int V>
__device__ __forceinline__ void stencil_gather(const T* Pr,
                                               const int (&off)[kStencil],
                                               T (&x)[kStencil][V]) {
  // Stencil order: the x-centred offset of plane k is 2k + 1; planes
  // k < 4 have their x - 1 offset at 2k, planes k >= 3 their x + 1 one at
  // 2k + 2.
#pragma unroll
  for (int k = 0; k < 7; ++k) ldv<T, V>(Pr + off[2 * k + 1], x[2 * k + 1]);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int u = 0; u < V; ++u) {
      x[2 * k][u] = lane_shift<false>(T(0), x[2 * k + 1][u]);
      x[2 * k + 8][u] = lane_shift<true>(T(0), x[2 * k + 7][u]);
    }
}

// Q = A P on the active chunks of SpMM tile t (kSpmmRows rows: each
// wavefront computes 62 consecutive rows on lanes 1..62, its lanes 0 and
// 63 holding the rows just before and after, whose x-centred neighbours
// the computing lanes need); per (column, tile) p . q.  The row's 15
// coefficients stay in registers across the chunks; each chunk ends with
// one wavefront reduction of the thread's V products.
template <typename T, int V, bool SEG>
__device__ __forceinline__ void spmm_cm_tile(const Desc& d, long long t,
                                             unsigned long long amask,
                                             double* __restrict__ ws) {
  const CmVecs<T> vs(d);
  const int tid = threadIdx.x;
  const long long n = d.n;
  const int mx = d.mx, my = d.my, mz = d.mz, ncols = d.ncols;
  const int cpr = ncols / V;
  const int lane = tid & 63;
  const long long row =
      t * kSpmmRows + (long long)(tid >> 6) * kSpmmWaveRows + lane - 1;
  const bool valid = lane >= 1 && lane <= kSpmmWaveRows && row < n;
  const long long rr = row < 0 ? 0 : (row < n ? row : n - 1);
  const unsigned ur = (unsigned)rr;
  const unsigned uq = ur / (unsigned)mx;
  const int i = (int)(ur - uq * (unsigned)mx);
  const unsigned uk = uq / (unsigned)my;
  const int j = (int)(uq - uk * (unsigned)my);
  const int k = (int)uk;
  T a[kStencil];
  int off[kStencil];
#pragma unroll
  for (int s = 0; s < kStencil; ++s) {
    const int ox = st_off(s, 0), oy = st_off(s, 1), oz = st_off(s, 2);
    const bool ok = (unsigned)(i + ox) < (unsigned)mx &&
                    (unsigned)(j + oy) < (unsigned)my &&
                    (unsigned)(k + oz) < (unsigned)mz;
    off[s] = ok ? (ox + mx * (oy + my * oz)) * V : 0;
    a[s] = ldg(vs.diag + (size_t)s * n + rr);
  }
  for (int ch = 0; ch < cpr; ++ch) {
    if (!chunk_in_mask<V>(amask, ch)) continue;
    const T* Pr = vs.P + ((size_t)ch * n + rr) * V;
    T x[kStencil][V];
    stencil_gather<T, V>(Pr, off, x);
    T q[V], self[V];
#pragma unroll
    for (int u = 0; u < V; ++u) q[u] = T(0);
#pragma unroll
    for (int s = 0; s < kStencil; ++s)
#pragma unroll
      for (int u = 0; u < V; ++u) q[u] = fma(a[s], x[s][u], q[u]);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      self[u] = valid ? x[kSelf][u] : T(0);
      q[u] = valid ? q[u] : T(0);
    }
    if (valid) {
      if constexpr (sizeof(T) == 8)
        if (d.kz) nl_add<V>(d, row, ch * V, q);  // + Z (Z^T p)
      stv<T, V>(vs.Q + ((size_t)ch * n + row) * V, q);
    }
    double pq[V];
#pragma unroll
    for (int u = 0; u < V; ++u) pq[u] = (double)self[u] * (double)q[u];
    const double tot = wave_reduce_scatter<V>(pq);
    constexpr int kGroup = 64 / V;
    if ((lane & (kGroup - 1)) == 0)
      ws[(tid >> 6) * ncols + ch * V + lane / kGroup] = tot;
  }
  __syncthreads();
  // Thread c < ncols: column c's tile sum is the partial (one tile per
  // segment), or is added to its segment's (kept in ws[4 ncols + c], which
  // only that thread touches).
  if (tid < ncols) {
    const double sum = ((ws[tid] + ws[ncols + tid]) + ws[2 * ncols + tid]) +
                       ws[3 * ncols + tid];
    if constexpr (SEG)
      ws[4 * ncols + tid] += sum;
    else if ((amask >> tid) & 1)
      stg(d.pqp + (size_t)tid * d.pqn + t, sum);
  }
  __syncthreads();  // ws is reused by the next tile
}

// The SpMM over segment g of a problem (its tiles in ascending order; one
// tile, or every kSpmmSlabSegs-th tile of a slab, as spmm_segments
// defines them); one p.q partial per (active column, segment).
// SEG false: every problem of the launch has one tile per segment (a
// separate instantiation: the segment loop costs the single-tile kernel
// registers).  ws: 5 kNtMax doubles.
static_assert(kSpmmSlabs == kXcd, "SpMM slabs follow the XCD tile walk");
template <typename T, int V, bool SEG>
__device__ __forceinline__ void spmm_cm_segment(const Desc& d, long long g,
                                                unsigned long long amask,
                                                double* __restrict__ ws) {
  if constexpr (!SEG) {
    spmm_cm_tile<T, V, false>(d, g, amask, ws);
  } else {
    const int c = threadIdx.x, ncols = d.ncols;
    if (c < ncols) ws[4 * ncols + c] = 0.0;
    long long t = g, end = g + 1, step = 1;
    if (d.pqn < d.spt) {  // slab segments
      const long long slab = (d.spt + kSpmmSlabs - 1) / kSpmmSlabs;
      const long long x = g / kSpmmSlabSegs;
      t = x * slab + (g - x * kSpmmSlabSegs);
      end = min((long long)d.spt, (x + 1) * slab);
      step = kSpmmSlabSegs;
    }
    for (; t < end; t += step) spmm_cm_tile<T, V, true>(d, t, amask, ws);
    if (c < ncols && ((amask >> c) & 1))
      stg(d.pqp + (size_t)c * d.pqn + g, ws[4 * ncols + c]);
  }
}

// The CG updates of chunk ch of tile t (kCmRpt rows per thread) in two
// halves: the loads, issued as soon as the unit is known to be active
// (before its alpha / beta are formed, so the two latencies overlap; all
// rows of a thread are loaded before any is stored, or the compiler,
// unable to rule out aliasing, serialises the rows), then the arithmetic
// and the stores.  Rows past the end load row n - 1 (unconditional loads
// stay in flight together) and contribute nothing.
template <typename T, int V>
struct RupdRegs {
  T r[kCmRpt][V], q[kCmRpt][V], di[kCmRpt];
};

template <typename T, int V>
__device__ __forceinline__ void rupd_cm_load(const Desc& d, long long t,
                                             int ch, RupdRegs<T, V>& g) {
  const long long n = d.n;
  const CmVecs<T> vs(d);
  const long long row0 = t * kCmRows + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const long long row = min(row0 + k * kBlock, n - 1);
    const size_t o = ((size_t)ch * n + row) * V;
    ldv<T, V>(vs.R + o, g.r[k]);
    ldv<T, V>(vs.Q + o, g.q[k]);
    g.di[k] = ldg(vs.dinv + row);
  }
}

// r -= alpha q, z = D^-1 r; r . z and r . r partials of the unit.
template <typename T, int V>
__device__ __forceinline__ void rupd_cm_finish(const Desc& d, long long t,
                                               int ch, const T (&al)[V],
                                               RupdRegs<T, V>& g,
                                               double* __restrict__ ws) {
  const long long n = d.n;
  const CmVecs<T> vs(d);
  const long long row0 = t * kCmRows + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const bool ok = row0 + k * kBlock < n;
    g.di[k] = ok ? g.di[k] : T(0);
#pragma unroll
    for (int u = 0; u < V; ++u) {
      g.r[k][u] = ok ? g.r[k][u] : T(0);
      g.q[k][u] = ok ? g.q[k][u] : T(0);
    }
  }
  double x[2 * V];
#pragma unroll
  for (int u = 0; u < 2 * V; ++u) x[u] = 0.0;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k)
#pragma unroll
    for (int u = 0; u < V; ++u) {
      g.r[k][u] = fma(-al[u], g.q[k][u], g.r[k][u]);
      x[u] += (double)g.r[k][u] * (double)(g.di[k] * g.r[k][u]);
      x[V + u] += (double)g.r[k][u] * (double)g.r[k][u];
    }
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const long long row = row0 + k * kBlock;
    if (row < n) stv<T, V>(vs.R + ((size_t)ch * n + row) * V, g.r[k]);
  }
  cm_unit_partials<2, V>(x, d, ch, t, ws);
}

template <typename T, int V>
struct PupdRegs {
  T x[kCmRpt][V], p[kCmRpt][V], r[kCmRpt][V], di[kCmRpt];
};

template <typename T, int V>
__device__ __forceinline__ void pupd_cm_load(const Desc& d, long long t,
                                             int ch, PupdRegs<T, V>& g) {
  const long long n = d.n;
  const CmVecs<T> vs(d);
  const long long row0 = t * kCmRows + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const long long row = min(row0 + k * kBlock, n - 1);
    const size_t o = ((size_t)ch * n + row) * V;
    ldv<T, V>(vs.X + o, g.x[k]);
    ldv<T, V>(vs.P + o, g.p[k]);
    ldv<T, V>(vs.R + o, g.r[k]);
    g.di[k] = ldg(vs.dinv + row);
  }
}

// x += alpha p (columns active this iteration); p = D^-1 r + beta p
// (columns active next iteration).
template <typename T, int V>
__device__ __forceinline__ void pupd_cm_finish(const Desc& d, long long t,
                                               int ch, const T (&al)[V],
                                               const T (&be)[V],
                                               const bool (&nx)[V],
                                               PupdRegs<T, V>& g) {
  const long long n = d.n;
  const CmVecs<T> vs(d);
  const long long row0 = t * kCmRows + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const long long row = row0 + k * kBlock;
    if (row >= n) continue;
#pragma unroll
    for (int u = 0; u < V; ++u) {
      g.x[k][u] = fma(al[u], g.p[k][u], g.x[k][u]);
      g.p[k][u] =
          nx[u] ? fma(be[u], g.p[k][u], g.di[k] * g.r[k][u]) : g.p[k][u];
    }
    const size_t o = ((size_t)ch * n + row) * V;
    stv<T, V>(vs.X + o, g.x[k]);
    stv<T, V>(vs.P + o, g.p[k]);
  }
}

// Run BODY with VV (constexpr) the vector width vw: 4, 2, 1 (FP32) or
// 2, 1 (FP64), or VFIX when it is not 0.
#define PARO_CM_WIDTH(T, VFIX, vw, BODY)                                   \
  if constexpr (VFIX != 0) PARO_VB_CASE(VFIX, BODY)                        \
  else if constexpr (sizeof(T) == 4) {                                     \
    if (vw == 4) PARO_VB_CASE(4, BODY)                                     \
    else if (vw == 2) PARO_VB_CASE(2, BODY)                                \
    else PARO_VB_CASE(1, BODY)                                             \
  } else {                                                                 \
    if (vw == 2) PARO_VB_CASE(2, BODY)                                     \
    else PARO_VB_CASE(1, BODY)                                             \
  }

// Chunks (of vw columns) with an active column, as a mask over chunks.
__device__ __forceinline__ unsigned long long chunk_mask(
    unsigned long long amask, int cpr, int vw) {
  const unsigned long long low = (1ull << vw) - 1;
  unsigned long long m = 0;
  for (int ch = 0; ch < cpr; ++ch)
    if ((amask >> (ch * vw)) & low) m |= 1ull << ch;
  return m;
}
// Unit u of the active units: tile u / nac and the (u % nac)-th chunk set
// in cm (nac of them).
__device__ __forceinline__ CmUnit cm_unit_active(long long u, int nac,
                                                 unsigned long long cm) {
  CmUnit r;
  r.t = u / nac;
  int k = (int)(u - r.t * nac);
  for (; k > 0; --k) cm &= cm - 1;  // drop the k lowest chunks
  r.ch = __builtin_ctzll(cm);
  return r;
}

// The units of the real block that runs this code, in its problem `d`
// (owner of blockIdx.x), with VV (constexpr) the problem's FP32 width:
// (tile, chunk) pairs over the chunks with an active column only, so the
// blocks share the live work evenly.
// Launches queued after convergence (no active column) do nothing: the
// column flags may be stale then.
// `amask` (bit c: column c active at parity par) is loaded once, with the
// active count.
#define PARO_CM_LOOP(T, D, nprob, par, VFIX, BODY)                         \
  {                                                                        \
    const Desc& d = D[owner(D, nprob, blockIdx.x, false)];                 \
    const int nact_ = ldg(&d.cs->n_active[par]);                           \
    const unsigned long long amask = active_mask(d.cs->act[par], d.ncols); \
    (void)amask;                                                           \
    if (nact_ == 0) return;                                                \
    const int lb_ = blockIdx.x - d.b0;                                     \
    const int vw_ = VFIX ? VFIX : cm_width<T>(d);                          \
    const int cpr_ = d.ncols / vw_;                                        \
    const unsigned long long cm_ = chunk_mask(amask, cpr_, vw_);           \
    const int nac_ = __popcll(cm_);                                        \
    for (TileWalk w_ = tile_walk((long long)d.ntc * nac_, lb_, d.nb);      \
         w_.t < w_.end; w_.t += w_.step) {                                 \
      const CmUnit un = cm_unit_active(w_.t, nac_, cm_);                   \
      PARO_CM_WIDTH(T, VFIX, vw_, BODY)                                    \
    }                                                                      \
  }

// The per-column CG scalars of chunk ch (uniform loads).
template <typename T, int V>
__device__ __forceinline__ bool cm_alpha(const ColState* cs, int par, int ch,
                                         T (&al)[V]) {
  bool any = false;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int c = ch * V + u;
    const bool on = ldg(&cs->act[par][c]) != 0;
    al[u] = on ? (T)ldg(&cs->alpha[c]) : T(0);
    any = any || on;
  }
  return any;
}

template <typename T, int V>
__device__ __forceinline__ void pupd_cm_chunk(const Desc& d, CmUnit un,
                                              int par) {
  const ColState* cs = d.cs;
  T al[V], be[V];
  bool nx[V];
  if (!cm_alpha<T, V>(cs, par, un.ch, al)) return;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int c = un.ch * V + u;
    nx[u] = ldg(&cs->act[par ^ 1][c]) != 0;
    be[u] = nx[u] ? (T)ldg(&cs->beta[c]) : T(0);
  }
  PupdRegs<T, V> g;
  pupd_cm_load<T, V>(d, un.t, un.ch, g);
  pupd_cm_finish<T, V>(d, un.t, un.ch, al, be, nx, g);
}

template <typename T, int V>
__device__ __forceinline__ void rupd_cm_chunk(const Desc& d, CmUnit un,
                                              int par, double* ws) {
  T al[V];
  if (cm_alpha<T, V>(d.cs, par, un.ch, al)) {
    RupdRegs<T, V> g;
    rupd_cm_load<T, V>(d, un.t, un.ch, g);
    rupd_cm_finish<T, V>(d, un.t, un.ch, al, g, ws);
  }
}

// VFIX: the common vector width of the launch's problems, or 0 (each
// block branches on its problem's width: 4, 2, 1 FP32 or 2, 1 FP64).
template <typename T, int VFIX, bool SEG>
__global__ void PARO_STREAM_BOUNDS
spmm_cm_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double ws[5 * kNtMax];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (d.zm != 0 || d.csr) return;  // served by spmm_zm_kernel or CSR
  const int nact = ldg(&d.cs->n_active[par]);
  const unsigned long long amask = active_mask(d.cs->act[par], d.ncols);
  if (nact == 0) return;  // queued after convergence
  const int lb = blockIdx.x - d.b0;
  const int vw = cm_width<T>(d);
  for (TileWalk w = tile_walk(d.pqn, lb, d.nb); w.t < w.end; w.t += w.step) {
    PARO_CM_WIDTH(T, VFIX, vw,
                  (spmm_cm_segment<T, VV, SEG>(d, w.t, amask, ws)))
  }
}


// ---------------------------------------------------------------------------
// z-marching CG SpMM (problems with zm > 0).  The sweep over rows above
// reads every P value of a plane three times, as the z + 1 neighbour, the
// centre and the z - 1 neighbour of rows one plane apart; on large meshes
// the rows in flight on an XCD span several planes of every active chunk,
// more than its 4 MB L2 holds, so the three reads reach the fabric.  Here
// a unit owns an xy tile of kSpmmRows consecutive rows of a plane (the
// same lane layout: lanes 0 and 63 of a wavefront hold the neighbouring
// rows for the x-shifts), a range of planes and a group of G chunks, and
// walks the planes upward.  Per chunk a thread keeps four of the seven
// x-centred lines it gathers (plane z - 1 at y and y - 1, plane z at y and
// y + 1) in registers from one plane to the next and loads three: plane z
// at y - 1 and plane z + 1 at y and y + 1.  The 15 coefficients of a row
// are loaded once per plane for the whole group; the other groups of the
// same tile and planes run on the same XCD at the same time and find them
// in its L2.
//
// q is formed exactly as in spmm_cm_tile (same products, same order), so
// Q is bitwise the same.  p.q is summed per (column, segment), segment =
// (plane range, xy tile): each thread adds its rows' products over the
// planes in ascending order, then one wavefront reduction and the four
// wavefronts in a fixed order.  The segments depend on the mesh alone and
// G only chooses which columns a unit serves, so every choice of G and of
// the block count gives the same bits.
//
// Unit walk: XCD x (= local block mod 8) owns the plane ranges
// [x zm / 8, (x + 1) zm / 8); its units are ordered (range, tile, group)
// with the group fastest, so the blocks of an XCD work on the groups of a
// few neighbouring tiles of one range at a time.
// ---------------------------------------------------------------------------

// The x-centred line of the thread's row at plane z and y offset oy
// (element offset oyo, 0 where j + oy leaves the box), plane clamped to
// the box (a plane outside it has coefficient 0 and reads a valid row).
template <typename T, int V>
__device__ __forceinline__ void zm_line(const T* __restrict__ Pc, int z,
                                        int mz, long long plane, int pc,
                                        int oyo, T (&o)[V]) {
  const int zq = z < 0 ? 0 : (z >= mz ? mz - 1 : z);
  ldv<T, V>(Pc + ((size_t)zq * plane + pc + oyo) * V, o);
}

template <typename T, int V, int G>
__device__ __forceinline__ void spmm_zm_unit(const Desc& d, int tau, int zeta,
                                             int ch0, unsigned long long amask,
                                             double* __restrict__ ws) {
  const CmVecs<T> vs(d);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long n = d.n;
  const int mx = d.mx, my = d.my, mz = d.mz, ncols = d.ncols;
  const int cpr = ncols / V;
  const long long plane = (long long)mx * my;
  const long long p = (long long)tau * kSpmmRows +
                      (long long)wave * kSpmmWaveRows + lane - 1;
  const bool valid = lane >= 1 && lane <= kSpmmWaveRows && p < plane;
  const int pc = (int)(p < 0 ? 0 : (p < plane ? p : plane - 1));
  const int j = pc / mx;
  const int oym = j > 0 ? -mx : 0, oyp = j < my - 1 ? mx : 0;
  const int za = (int)((long long)zeta * mz / d.zm);
  const int zb = (int)((long long)(zeta + 1) * mz / d.zm);
  bool on[G];
  const T* Pc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int ch = ch0 + g;
    on[g] = ch < cpr && chunk_in_mask<V>(amask, ch);
    Pc[g] = vs.P + (size_t)(ch < cpr ? ch : 0) * n * V;
  }
  // Carried lines: plane z - 1 at y and y - 1, plane z at y and y + 1.
  T cm0[G][V], cmm[G][V], c00[G][V], c0p[G][V];
  double acc[G][V];
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int u = 0; u < V; ++u) acc[g][u] = 0.0;
    if (on[g]) {
      zm_line<T, V>(Pc[g], za - 1, mz, plane, pc, 0, cm0[g]);
      zm_line<T, V>(Pc[g], za - 1, mz, plane, pc, oym, cmm[g]);
      zm_line<T, V>(Pc[g], za, mz, plane, pc, 0, c00[g]);
      zm_line<T, V>(Pc[g], za, mz, plane, pc, oyp, c0p[g]);
    }
  }
  for (int z = za; z < zb; ++z) {
    const size_t row = (size_t)z * plane + pc;
    T a[kStencil];
#pragma unroll
    for (int s = 0; s < kStencil; ++s) a[s] = ldg(vs.diag + (size_t)s * n + row);
    T c0m[G][V], c10[G][V], c1p[G][V];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (on[g]) {
        zm_line<T, V>(Pc[g], z, mz, plane, pc, oym, c0m[g]);
        zm_line<T, V>(Pc[g], z + 1, mz, plane, pc, 0, c10[g]);
        zm_line<T, V>(Pc[g], z + 1, mz, plane, pc, oyp, c1p[g]);
      }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!on[g]) continue;
      T x[kStencil][V];
#pragma unroll
      for (int u = 0; u < V; ++u) {
        x[1][u] = cmm[g][u];
        x[3][u] = cm0[g][u];
        x[5][u] = c0m[g][u];
        x[7][u] = c00[g][u];
        x[9][u] = c0p[g][u];
        x[11][u] = c10[g][u];
        x[13][u] = c1p[g][u];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          x[2 * k][u] = lane_shift<false>(T(0), x[2 * k + 1][u]);
          x[2 * k + 8][u] = lane_shift<true>(T(0), x[2 * k + 7][u]);
        }
      T q[V];
#pragma unroll
      for (int u = 0; u < V; ++u) q[u] = T(0);
#pragma unroll
      for (int s = 0; s < kStencil; ++s)
#pragma unroll
        for (int u = 0; u < V; ++u) q[u] = fma(a[s], x[s][u], q[u]);
      if (valid) {
        if constexpr (sizeof(T) == 8)
          if (d.kz) nl_add<V>(d, (long long)row, (ch0 + g) * V, q);
        stv<T, V>(vs.Q + ((size_t)(ch0 + g) * n + row) * V, q);
#pragma unroll
        for (int u = 0; u < V; ++u)
          acc[g][u] += (double)x[kSelf][u] * (double)q[u];
      }
      // Next plane: z becomes z - 1, z + 1 becomes z.
#pragma unroll
      for (int u = 0; u < V; ++u) {
        cm0[g][u] = c00[g][u];
        cmm[g][u] = c0m[g][u];
        c00[g][u] = c10[g][u];
        c0p[g][u] = c1p[g][u];
      }
    }
  }
  // Per (column, segment) p.q: wavefront, then the four wavefronts.
  constexpr int kGroup = 64 / V;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (!on[g]) continue;  // uniform over the block
    const double tot = wave_reduce_scatter<V>(acc[g]);
    if ((lane & (kGroup - 1)) == 0)
      ws[wave * ncols + (ch0 + g) * V + lane / kGroup] = tot;
  }
  __syncthreads();
  // Thread tid < ncols stores column tid's partial if the column is
  // active (so its chunk is one of this unit's G).
  const int c = tid - ch0 * V;
  if (c >= 0 && c < G * V && tid < ncols && ((amask >> tid) & 1)) {
    const double sum = ((ws[tid] + ws[ncols + tid]) + ws[2 * ncols + tid]) +
                       ws[3 * ncols + tid];
    stg(d.pqp + (size_t)tid * d.pqn + ((size_t)zeta * d.zxy + tau), sum);
  }
  __syncthreads();  // ws is reused by the next unit
}

// The g-th set bit of m (g < popcount(m)).
__device__ __forceinline__ int nth_bit(unsigned long long m, int g) {
  for (; g > 0; --g) m &= m - 1;
  return __builtin_ctzll(m);
}

template <typename T, int VFIX, int G>
__global__ void PARO_STREAM_BOUNDS
spmm_zm_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double ws[4 * kNtMax];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (d.zm == 0) return;  // served by spmm_cm_kernel
  const int nact = ldg(&d.cs->n_active[par]);
  const unsigned long long amask = active_mask(d.cs->act[par], d.ncols);
  if (nact == 0) return;  // queued after convergence
  const int lb = blockIdx.x - d.b0;
  const int vw = cm_width<T>(d);
  const int cpr = d.ncols / vw;
  // Groups of G chunks with an active column.
  const unsigned long long cm = chunk_mask(amask, cpr, vw);
  unsigned long long gm = 0;
  for (int g = 0; g * G < cpr; ++g)
    if ((cm >> (g * G)) & ((1ull << G) - 1)) gm |= 1ull << g;
  const int nag = __popcll(gm);
  const int x = lb % kXcd, l = lb / kXcd, gx = d.nb / kXcd;
  const int zr = d.zm / kXcd;
  const long long units = (long long)zr * d.zxy * nag;
  for (long long k = l; k < units; k += gx) {
    const long long rest = k / nag;
    const int gi = (int)(k - rest * nag);
    const int tau = (int)(rest % d.zxy);
    const int zeta = x * zr + (int)(rest / d.zxy);
    const int ch0 = nth_bit(gm, gi) * G;
    PARO_CM_WIDTH(T, VFIX, vw,
                  (spmm_zm_unit<T, VV, G>(d, tau, zeta, ch0, amask, ws)))
  }
}


// ---------------------------------------------------------------------------
// Matrix-free z-marching CG SpMM (uniform box problems).  The stored
// stencil holds 15 coefficients per row, 120 bytes in FP64 (60 in FP32)
// against the 16 of a chunk's P value: with a few active chunks the
// coefficients are most of the traffic, and every chunk group reads them
// again.  On a uniform Kuhn mesh a row's coefficients are c0 + vol/60 W v
// with v the potential at its 15 stencil vertices (kuhn.h), so this form
// reads the potential (8 bytes per vertex) instead and forms the
// coefficients with kuhn_row, the function the assembly stored them with
// (FP32: rounded from FP64, as the stored FP32 stencil is): the operator,
// Q and the p.q partials are bitwise those of spmm_zm_kernel.
//
// The potential lines march along z like the P lines: per plane a thread
// loads 7 values (plane z at y - 1, x - 1 and x; plane z at y, x - 1;
// plane z + 1 at y and y + 1, x and x + 1) and carries 8.  Units are
// (plane range, xy tile, chunk group) as in spmm_zm_kernel, with the
// active chunks compacted and cut into the fewest groups of at most 4
// chunks (3 for FP32 chunks of 4 columns), of as equal sizes as possible,
// so every chunk of a unit is active and the coefficients of a row are
// formed once per group.
// ---------------------------------------------------------------------------
// The z-march of one unit over the chunk-major block `src` (chunks cl[0..G)
// of V columns of type T): per plane z of [za, zb) and chunk g it calls
//   f(g, row, valid, mask, a, x)
// with row the thread's row of plane z, valid false on the wavefront's halo
// lanes and past the plane, mask the offsets whose neighbour lies in the
// box, a the row's 15 FP64 coefficients of A_s (kuhn_row; MF false: read
// from the stored stencil, the same values) and x[s][u] the value of
// column u at neighbour s (0-weighted where the neighbour is outside).
template <typename T, int V, int G, bool MF = true, class F>
__device__ __forceinline__ void zmf_march(const Desc& d, int tau, int zeta,
                                          const int (&cl)[4],
                                          const T* __restrict__ src, F&& f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long n = d.n;
  const int mx = d.mx, my = d.my, mz = d.mz;
  const long long plane = (long long)mx * my;
  const long long p = (long long)tau * kSpmmRows +
                      (long long)wave * kSpmmWaveRows + lane - 1;
  const bool valid = lane >= 1 && lane <= kSpmmWaveRows && p < plane;
  const int pc = (int)(p < 0 ? 0 : (p < plane ? p : plane - 1));
  const int j = pc / mx, i = pc - j * mx;
  const int oym = j > 0 ? -mx : 0, oyp = j < my - 1 ? mx : 0;
  const int za = (int)((long long)zeta * mz / d.zm);
  const int zb = (int)((long long)(zeta + 1) * mz / d.zm);
  // Offsets whose neighbour lies in the box, x and y (z per plane).
  unsigned mxy = 0;
#pragma unroll
  for (int s = 0; s < kStencil; ++s) {
    const int ox = kKuhnOff[s][0], oy = kKuhnOff[s][1];
    const bool vx = ox < 0 ? i > 0 : (ox > 0 ? i < mx - 1 : true);
    const bool vy = oy < 0 ? j > 0 : (oy > 0 ? j < my - 1 : true);
    mxy |= (vx && vy ? 1u : 0u) << s;
  }
  // The stencil constants are uniform: held in scalar registers.
  double c0[kStencil];
#pragma unroll
  for (int s = 0; s < kStencil; ++s) c0[s] = uniform(ldg(d.kconst + s));
  const double vol60 = uniform(ldg(d.kconst + kKcVol60));
  // Potential of vertex (i + 1 + dx, j + 1 + dy, K + dz): Vr[K sz + ...].
  const long long sy = mx + 2, sz = (long long)(mx + 2) * (my + 2);
  const double* Vr = d.Vb + (i + 1) + sy * (j + 1);
  const T* Pc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) Pc[g] = src + (size_t)cl[g] * n * V;
  T cm0[G][V], cmm[G][V], c00[G][V], c0p[G][V];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    zm_line<T, V>(Pc[g], za - 1, mz, plane, pc, 0, cm0[g]);
    zm_line<T, V>(Pc[g], za - 1, mz, plane, pc, oym, cmm[g]);
    zm_line<T, V>(Pc[g], za, mz, plane, pc, 0, c00[g]);
    zm_line<T, V>(Pc[g], za, mz, plane, pc, oyp, c0p[g]);
  }
  // Carried potential (stencil slots 0-3, 7-10 of plane za; vertex plane
  // K = z + 1 holds dof plane z).
  double w0, w1, w2, w3, w7, w8, w9, w10;
  {
    const double* b = Vr + sz * za;  // vertex plane K - 1
    w0 = ldg(b - 1 - sy);
    w1 = ldg(b - sy);
    w2 = ldg(b - 1);
    w3 = ldg(b);
    w7 = ldg(b + sz);
    w8 = ldg(b + sz + 1);
    w9 = ldg(b + sz + sy);
    w10 = ldg(b + sz + sy + 1);
  }
  for (int z = za; z < zb; ++z) {
    const long long row = (long long)z * plane + pc;
    const double* b = Vr + sz * (z + 1);
    double v[kStencil];
    v[0] = w0; v[1] = w1; v[2] = w2; v[3] = w3;
    v[4] = ldg(b - 1 - sy);
    v[5] = ldg(b - sy);
    v[6] = ldg(b - 1);
    v[7] = w7; v[8] = w8; v[9] = w9; v[10] = w10;
    v[11] = ldg(b + sz);
    v[12] = ldg(b + sz + 1);
    v[13] = ldg(b + sz + sy);
    v[14] = ldg(b + sz + sy + 1);
    T c0m[G][V], c10[G][V], c1p[G][V];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      zm_line<T, V>(Pc[g], z, mz, plane, pc, oym, c0m[g]);
      zm_line<T, V>(Pc[g], z + 1, mz, plane, pc, 0, c10[g]);
      zm_line<T, V>(Pc[g], z + 1, mz, plane, pc, oyp, c1p[g]);
    }
    unsigned mask = mxy;
    if (z == 0) mask &= ~0xfu;                // dz = -1: slots 0-3
    if (z == mz - 1) mask &= ~(0xfu << 11);   // dz = +1: slots 11-14
    double a[kStencil];
    if constexpr (MF) {
      kuhn_row(v, c0, vol60, mask, a);
    } else {
#pragma unroll
      for (int s = 0; s < kStencil; ++s)
        a[s] = ldg(d.diagA + (size_t)s * n + row);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      T x[kStencil][V];
#pragma unroll
      for (int u = 0; u < V; ++u) {
        x[1][u] = cmm[g][u];
        x[3][u] = cm0[g][u];
        x[5][u] = c0m[g][u];
        x[7][u] = c00[g][u];
        x[9][u] = c0p[g][u];
        x[11][u] = c10[g][u];
        x[13][u] = c1p[g][u];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < V; ++u) {
          x[2 * k][u] = lane_shift<false>(T(0), x[2 * k + 1][u]);
          x[2 * k + 8][u] = lane_shift<true>(T(0), x[2 * k + 7][u]);
        }
      f(g, row, valid, mask, a, x);
#pragma unroll
      for (int u = 0; u < V; ++u) {
        cm0[g][u] = c00[g][u];
        cmm[g][u] = c0m[g][u];
        c00[g][u] = c10[g][u];
        c0p[g][u] = c1p[g][u];
      }
    }
    w0 = v[4]; w1 = v[5]; w2 = v[6]; w3 = v[7];
    w7 = v[11]; w8 = v[12]; w9 = v[13]; w10 = v[14];
  }
}

template <typename T, int V, int G>
__device__ __forceinline__ void spmm_zmf_unit(const Desc& d, int tau,
                                              int zeta, const int (&cl)[4],
                                              unsigned long long amask,
                                              double* __restrict__ ws) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long n = d.n;
  const int ncols = d.ncols;
  const CmVecs<T> vs(d);
  double acc[G][V];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int u = 0; u < V; ++u) acc[g][u] = 0.0;
  zmf_march<T, V, G>(
      d, tau, zeta, cl, vs.P,
      [&](int g, long long row, bool valid, unsigned,
          const double (&a)[kStencil], const T (&x)[kStencil][V]) {
        // q = sum_s a_s x_s, s ascending, as spmm_zm_unit (FP32: the
        // coefficients rounded as in the stored FP32 stencil).
        T q[V];
#pragma unroll
        for (int u = 0; u < V; ++u) q[u] = T(0);
#pragma unroll
        for (int s = 0; s < kStencil; ++s) {
          const T as = (T)a[s];
#pragma unroll
          for (int u = 0; u < V; ++u) q[u] = fma(as, x[s][u], q[u]);
        }
        if (valid) {
          if constexpr (sizeof(T) == 8)
            if (d.kz) nl_add<V>(d, row, cl[g] * V, q);
          stv<T, V>(vs.Q + ((size_t)cl[g] * n + row) * V, q);
#pragma unroll
          for (int u = 0; u < V; ++u)
            acc[g][u] += (double)x[kSelf][u] * (double)q[u];
        }
      });
  // Per (column, segment) p.q, reduced as in spmm_zm_unit.
  constexpr int kGroup = 64 / V;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const double tot = wave_reduce_scatter<V>(acc[g]);
    if ((lane & (kGroup - 1)) == 0)
      ws[wave * ncols + cl[g] * V + lane / kGroup] = tot;
  }
  __syncthreads();
  // Thread tid < ncols stores column tid's partial if the column is active
  // and its chunk is one of this unit's.
  bool mine = false;
#pragma unroll
  for (int g = 0; g < G; ++g) mine = mine || tid / V == cl[g];
  if (mine && tid < ncols && ((amask >> tid) & 1)) {
    const double sum = ((ws[tid] + ws[ncols + tid]) + ws[2 * ncols + tid]) +
                       ws[3 * ncols + tid];
    stg(d.pqp + (size_t)tid * d.pqn + ((size_t)zeta * d.zxy + tau), sum);
  }
  __syncthreads();  // ws is reused by the next unit
}

// Most chunks per unit: 4, or 3 for FP32 chunks of 4 columns (16 columns
// per unit would need more registers than two wavefronts per SIMD have).
__host__ __device__ constexpr int zmf_group_max(int bytes, int V) {
  return bytes == 4 && V == 4 ? 3 : 4;
}

template <typename T, int V>
__device__ __forceinline__ void spmm_zmf_group(const Desc& d, int tau,
                                               int zeta, int gs,
                                               const int (&cl)[4],
                                               unsigned long long amask,
                                               double* ws) {
  switch (gs) {
    case 4:
      if constexpr (zmf_group_max(sizeof(T), V) == 4)
        spmm_zmf_unit<T, V, 4>(d, tau, zeta, cl, amask, ws);
      break;
    case 3: spmm_zmf_unit<T, V, 3>(d, tau, zeta, cl, amask, ws); break;
    case 2: spmm_zmf_unit<T, V, 2>(d, tau, zeta, cl, amask, ws); break;
    default: spmm_zmf_unit<T, V, 1>(d, tau, zeta, cl, amask, ws); break;
  }
}

// VFIX: the common width of the launch's problems in T, or 0.
template <typename T, int VFIX>
__global__ void PARO_STREAM_BOUNDS
spmm_zmf_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double ws[4 * kNtMax];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (d.zm == 0) return;  // served by spmm_cm_kernel or CSR
  const int nact = ldg(&d.cs->n_active[par]);
  const unsigned long long amask = active_mask(d.cs->act[par], d.ncols);
  if (nact == 0) return;  // queued after convergence
  const int lb = blockIdx.x - d.b0;
  const int vw = VFIX ? VFIX : cm_width<T>(d);
  const unsigned long long cm = chunk_mask(amask, d.ncols / vw, vw);
  const int nac = __popcll(cm);
  const int gmax = zmf_group_max(sizeof(T), vw);
  const int nag = (nac + gmax - 1) / gmax;
  const int x = lb % kXcd, l = lb / kXcd, gx = d.nb / kXcd;
  const int zr = d.zm / kXcd;
  const long long units = (long long)zr * d.zxy * nag;
  for (long long k = l; k < units; k += gx) {
    const long long rest = k / nag;
    const int gi = (int)(k - rest * nag);
    const int tau = (int)(rest % d.zxy);
    const int zeta = x * zr + (int)(rest / d.zxy);
    // Group gi: active chunks [gi nac / nag, (gi + 1) nac / nag).
    const int r0 = gi * nac / nag, r1 = (gi + 1) * nac / nag;
    int cl[4];
    unsigned long long rem = cm;
    for (int r = 0; r < r0; ++r) rem &= rem - 1;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      cl[g] = rem ? __builtin_ctzll(rem) : 0;
      if (g < r1 - r0) rem &= rem - 1;
    }
    if (sizeof(T) == 4 && vw == 4)
      spmm_zmf_group<T, 4>(d, tau, zeta, r1 - r0, cl, amask, ws);
    else if (vw == 2)
      spmm_zmf_group<T, 2>(d, tau, zeta, r1 - r0, cl, amask, ws);
    else
      spmm_zmf_group<T, 1>(d, tau, zeta, r1 - r0, cl, amask, ws);
  }
}

// The r-update with alpha computed in place (the alpha finaliser folded
// into the kernel): wavefront w < V of a unit forms alpha of column
// ch V + w from the p.q partials in the finaliser's order (same bits), the
// unit of tile 0 stores it for the p-update and sets the status bits, and
// block 0 does the finaliser's per-iteration bookkeeping.
template <typename T, int V>
__device__ __forceinline__ void rupd_alpha_chunk(const Desc& d, CmUnit un,
                                                 int par,
                                                 unsigned long long amask,
                                                 double* ws, double* al_s) {
  ColState* cs = d.cs;
  if (!chunk_in_mask<V>(amask, un.ch)) return;
  RupdRegs<T, V> g;
  rupd_cm_load<T, V>(d, un.t, un.ch, g);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < V) {
    const int c = un.ch * V + wave;
    double a = 0.0;
    if ((amask >> c) & 1) {
      const double rz = ldg(&cs->rzp[par][c]);
      double tot[1];
      column_sums<1>(d.pqp, 0, c, d.pqn, tot);
      const double pq = tot[0];
      const bool bad = !(pq > 0.0) || !isfinite(pq);
      a = bad ? 0.0 : rz / pq;
      if (lane == 0 && un.t == 0) {
        if (bad)
          atomicOr(&cs->status,
                   isfinite(pq) ? (int)kStNotSpd : (int)kStNonFinite);
        cs->alpha[c] = a;
      }
    }
    if (lane == 0) al_s[wave] = a;
  }
  __syncthreads();
  T al[V];
#pragma unroll
  for (int u = 0; u < V; ++u) al[u] = (T)al_s[u];
  rupd_cm_finish<T, V>(d, un.t, un.ch, al, g, ws);  // ends with a barrier
}

template <typename T, int VFIX>
__global__ void PARO_STREAM_BOUNDS
rupd_alpha_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double ws[4 * 8];
  __shared__ double al_s[4];
  {
    const Desc& d0 = D[owner(D, nprob, blockIdx.x, false)];
    if (blockIdx.x == d0.b0 && threadIdx.x == 0) {
      // As the finaliser: the next parity starts idle; one more iteration
      // when this one runs.
      ColState* cs = d0.cs;
      if (ldg(&cs->n_active[par]) != 0) cs->cg_iters += 1;
      cs->n_active[par ^ 1] = 0;
    }
  }
  PARO_CM_LOOP(T, D, nprob, par, VFIX,
               (rupd_alpha_chunk<T, VV>(d, un, par, amask, ws, al_s)))
}


// The p-update with beta computed in place (the beta finaliser folded
// into the kernel): wavefront w < V of a unit forms r.z and r.r of column
// ch V + w from the r-update's partials in the finaliser's order, every
// unit evaluates beta_step from the parity-par state (same bits), and the
// unit of tile 0 commits it.  Block 0 marks the inactive columns idle in
// the next parity.
template <typename T, int V>
__device__ __forceinline__ void pupd_beta_chunk(const Desc& d, CmUnit un,
                                                int par,
                                                unsigned long long amask,
                                                double* b_s) {
  ColState* cs = d.cs;
  if (!chunk_in_mask<V>(amask, un.ch)) return;
  T al[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int c = un.ch * V + u;  // < ncols (ncols is a multiple of V)
    const T a = (T)ldg(&cs->alpha[c]);  // unconditional: loads together
    al[u] = ((amask >> c) & 1) ? a : T(0);
  }
  PupdRegs<T, V> g;
  pupd_cm_load<T, V>(d, un.t, un.ch, g);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < V) {
    const int c = un.ch * V + wave;
    double beta = 0.0;
    int next = 0;
    if ((amask >> c) & 1) {
      const BetaIn q = beta_in(cs, c, par);
      double tot[2];
      // 4 loads per lane: the unit's data are in registers meanwhile.
      column_sums<2, 4>(d.cgp, (size_t)d.cgstride, c, d.cgn, tot);
      const BetaStep b = beta_step(q, tot[0], tot[1]);
      beta = b.beta;
      next = b.next;
      if (lane == 0 && un.t == 0) beta_commit(cs, c, par, b, tot[0], tot[1]);
    }
    if (lane == 0) {
      b_s[wave] = beta;
      b_s[4 + wave] = next ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  T be[V];
  bool nx[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    nx[u] = b_s[4 + u] != 0.0;
    be[u] = nx[u] ? (T)b_s[u] : T(0);
  }
  pupd_cm_finish<T, V>(d, un.t, un.ch, al, be, nx, g);
  __syncthreads();  // b_s is rewritten by the next unit
}

template <typename T, int VFIX>
__global__ void PARO_STREAM_BOUNDS
pupd_beta_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double b_s[8];
  {
    const Desc& d0 = D[owner(D, nprob, blockIdx.x, false)];
    if (blockIdx.x == d0.b0 && ldg(&d0.cs->n_active[par]) != 0)
      for (int c = threadIdx.x; c < d0.ncols; c += kBlock)
        if (!ldg(&d0.cs->act[par][c])) d0.cs->act[par ^ 1][c] = 0;
  }
  PARO_CM_LOOP(T, D, nprob, par, VFIX,
               (pupd_beta_chunk<T, VV>(d, un, par, amask, b_s)))
}

// Continuing FP32 pass after residual replacement: p = D^-1 r + beta p on
// the columns that refine (parity 0 of the coming CG iterations).
template <int V>
__device__ __forceinline__ void redirect_cm_chunk(const Desc& d, CmUnit un) {
  const ColState* cs = d.cs;
  const long long n = d.n;
  float be[V];
  bool on[V];
  bool any = false;
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int c = un.ch * V + u;
    on[u] = ldg(&cs->act[0][c]) != 0;
    be[u] = on[u] ? (float)ldg(&cs->beta[c]) : 0.0f;
    any = any || on[u];
  }
  if (!any) return;
#pragma unroll
  for (int k = 0; k < kCmRpt; ++k) {
    const long long row = un.t * kCmRows + threadIdx.x + k * kBlock;
    if (row >= n) break;
    const size_t o = ((size_t)un.ch * n + row) * V;
    float p[V], r[V];
    ldv<float, V>(d.P32 + o, p);
    ldv<float, V>(d.R32 + o, r);
    const float di = ldg(d.dinv32 + row);
#pragma unroll
    for (int u = 0; u < V; ++u) p[u] = on[u] ? fmaf(be[u], p[u], di * r[u]) : p[u];
    stv<float, V>(d.P32 + o, p);
  }
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
redirect_cm_kernel(const Desc* __restrict__ D, int nprob) {
  PARO_CM_LOOP(float, D, nprob, 0, VFIX, (redirect_cm_chunk<VV>(d, un)))
}

// ------------------------------------------------------------------------
// Nonlocal pseudopotential term (Sec. 2): V_nl u = sum_j (u, zeta_j) zeta_j
// has the Galerkin matrix Z Z^T with Z = M zeta (n x k), so the operator of
// the source problems and of the projection becomes A + Z Z^T.  It is
// applied as a low-rank correction inside the stencil kernels: Y = Z^T X
// first (per-(tile, chunk) partials, then one wavefront per (projector,
// column) in a fixed order), then the kernel that forms A X adds Z Y row
// by row (the CG SpMM, so p.q includes the term; the start residual; HW).
// ------------------------------------------------------------------------

// Z[row][j] = sum_s M[row][row + off_s] zeta[row + off_s][j].
__global__ void __launch_bounds__(kBlock)
nl_mass_kernel(Desc d, const double* __restrict__ zeta,
               double* __restrict__ Z, int k) {
  const long long total = d.n * k;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (long long)gridDim.x * kBlock) {
    const long long row = e / k;
    const int j = (int)(e - row * k);
    const unsigned ur = (unsigned)row;
    const unsigned uq = ur / (unsigned)d.mx;
    const int i = (int)(ur - uq * (unsigned)d.mx);
    const unsigned uk = uq / (unsigned)d.my;
    const int jj = (int)(uq - uk * (unsigned)d.my);
    const int kk = (int)uk;
    double acc = 0.0;
#pragma unroll
    for (int st = 0; st < kStencil; ++st) {
      const int ox = st_off(st, 0), oy = st_off(st, 1), oz = st_off(st, 2);
      const bool ok = (unsigned)(i + ox) < (unsigned)d.mx &&
                      (unsigned)(jj + oy) < (unsigned)d.my &&
                      (unsigned)(kk + oz) < (unsigned)d.mz;
      const long long nb = ok ? row + ox + (long long)d.mx * (oy + (long long)d.my * oz) : row;
      acc = fma(ldg(d.diagM + (size_t)st * d.n + row), zeta[nb * k + j], acc);
    }
    Z[e] = acc;
  }
}

// Sources of Z^T X: the FP64 CG direction P (chunk-major), the start
// orbitals U0 or the basis X (row-major).
enum { kZtP = 0, kZtU0 = 1, kZtX = 2 };

// Partials of Y = Z^T X for unit (tile t of kCmRows rows, FP64 chunk ch):
// a thread accumulates its rows' products for KP (>= k, a power of two)
// projectors and the chunk's V columns, then one wavefront reduction and
// a fixed-order sum over the four wavefronts; partial slot
// zpart[(j ncols + c) ntc + t].
template <int KP, int V>
__device__ __forceinline__ void zt_unit(const Desc& d, int src, long long t,
                                        int ch, double* __restrict__ ws) {
  constexpr int K = KP * V;
  const int k = d.kz, nc = d.ncols;
  double acc[K];
#pragma unroll
  for (int e = 0; e < K; ++e) acc[e] = 0.0;
  const double* X = src == kZtU0 ? d.U0 : d.X;
#pragma unroll
  for (int rr = 0; rr < kCmRpt; ++rr) {
    const long long row = t * kCmRows + threadIdx.x + rr * kBlock;
    if (row >= d.n) break;
    double x[V];
    if (src == kZtP)
      ldv<double, V>(d.P + ((size_t)ch * d.n + row) * V, x);
    else
      ldv<double, V>(X + (size_t)row * nc + ch * V, x);
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const double z = j < k ? ldg(d.Zp + (size_t)row * k + j) : 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) acc[j * V + v] = fma(z, x[v], acc[j * V + v]);
    }
  }
  constexpr int kGroup = 64 / K;
  const double tot = wave_reduce_scatter<K>(acc);
  const int lane = threadIdx.x & 63;
  if ((lane & (kGroup - 1)) == 0) ws[(threadIdx.x >> 6) * K + lane / kGroup] = tot;
  __syncthreads();
  const int e = threadIdx.x;
  if (e < K && e / V < k) {
    const double sum = ((ws[e] + ws[K + e]) + ws[2 * K + e]) + ws[3 * K + e];
    const int j = e / V, c = ch * V + e % V;
    stg(d.zpart + ((size_t)j * nc + c) * d.ntc + t, sum);
  }
  __syncthreads();
}

// par: the CG parity (source P: chunks without an active column and
// launches queued after convergence are skipped; their Y is not read).
template <int KP>
__global__ void __launch_bounds__(kBlock)
zt_partial_kernel(const Desc* __restrict__ D, int nprob, int src, int par) {
  __shared__ double ws[4 * 64];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (d.kz == 0) return;
  if (src == kZtP && ldg(&d.cs->n_active[par]) == 0) return;
  const int lb = blockIdx.x - d.b0;
  const int V = d.v64, cpr = d.ncols / V;
  for (TileWalk w = tile_walk((long long)d.ntc * cpr, lb, d.nb); w.t < w.end;
       w.t += w.step) {
    const CmUnit un = cm_unit(w.t, cpr);
    if (src == kZtP && !chunk_active(d.cs->act[par], un.ch, V, d.ncols))
      continue;
    if (V == 2)
      zt_unit<KP, 2>(d, src, un.t, un.ch, ws);
    else
      zt_unit<KP, 1>(d, src, un.t, un.ch, ws);
  }
}

// Y[j][c] = sum over tiles (one wavefront per pair; grid: pair x problem).
__global__ void __launch_bounds__(kFinal)
zt_final_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.y];
  const int q = blockIdx.x;
  if (d.kz == 0 || q >= d.kz * d.ncols) return;
  double tot[1];
  column_sums<1>(d.zpart, 0, q, d.ntc, tot);
  if ((threadIdx.x & (kFinal - 1)) == 0) d.zy[q] = tot[0];
}


// ------------------------------------------------------------------------
// Persistent CG: every iteration of every problem of the table in one
// cooperative launch.  The phases of an iteration -- SpMM, alpha, r-update,
// beta, p-update -- are the same device functions as the per-kernel path
// (same partial slots, same summation order: identical results), separated
// by grid-wide barriers instead of kernel boundaries.  A block keeps its
// problem's block range; the per-column scalar phases spread the (problem,
// column) pairs over all wavefronts of the grid.  Every block takes the
// same exit decision: after the beta phase it reads the next-parity active
// counts of all problems (final at that barrier); `iters` (even) bounds the
// loop, so every wavefront reaches the end.
// ------------------------------------------------------------------------
// Registers capped for three workgroups per CU (768 co-resident blocks).
template <typename T, int VFIX>
__global__ void __launch_bounds__(kBlock, 3)
cg_persistent_kernel(const Desc* __restrict__ D, int nprob, int iters) {
  namespace cgr = cooperative_groups;
  cgr::grid_group grid = cgr::this_grid();
  __shared__ double ws[5 * kNtMax];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  const int lb = blockIdx.x - d.b0;
  const int vw = cm_width<T>(d);
  const int cpr = d.ncols / vw;
  const int wave = threadIdx.x >> 6;
  const int nwaves = gridDim.x * (kBlock / 64);
  const int npairs = nprob * kNtMax;
  int par = 0;
  bool done = false;
  for (int it = 0; it < iters; ++it) {
    const bool on = ldg(&d.cs->n_active[par]) != 0;
    const unsigned long long amask = active_mask(d.cs->act[par], d.ncols);
    if (on)
      for (TileWalk w = tile_walk(d.pqn, lb, d.nb); w.t < w.end;
           w.t += w.step) {
        PARO_CM_WIDTH(T, VFIX, vw,
                      (spmm_cm_segment<T, VV, true>(d, w.t, amask, ws)))
      }
    grid.sync();
    for (int q = blockIdx.x * (kBlock / 64) + wave; q < npairs; q += nwaves)
      alpha_pair(D[q / kNtMax], q % kNtMax, par);
    grid.sync();
    if (on)
      for (TileWalk w = tile_walk((long long)d.ntc * cpr, lb, d.nb);
           w.t < w.end; w.t += w.step) {
        const CmUnit un = cm_unit(w.t, cpr);
        PARO_CM_WIDTH(T, VFIX, vw, (rupd_cm_chunk<T, VV>(d, un, par, ws)))
      }
    grid.sync();
    for (int q = blockIdx.x * (kBlock / 64) + wave; q < npairs; q += nwaves)
      beta_pair(D[q / kNtMax], q % kNtMax, par);
    grid.sync();
    int more = 0;
    for (int p = threadIdx.x; p < nprob; p += kBlock)
      more |= ldg(&D[p].cs->n_active[par ^ 1]) != 0;
    more = __syncthreads_or(more);
    if (on)
      for (TileWalk w = tile_walk((long long)d.ntc * cpr, lb, d.nb);
           w.t < w.end; w.t += w.step) {
        const CmUnit un = cm_unit(w.t, cpr);
        PARO_CM_WIDTH(T, VFIX, vw, (pupd_cm_chunk<T, VV>(d, un, par)))
      }
    grid.sync();
    par ^= 1;
    if (!more) {
      done = true;
      break;
    }
  }
  // Converged: keep both parities idle, the state the per-kernel path
  // reaches through its queued no-op iterations.  At the cap (an even
  // count) `par` is back at 0 and the counts stay, for the host to see.
  if (done && blockIdx.x == 0)
    for (int p = threadIdx.x; p < nprob; p += kBlock)
      D[p].cs->n_active[par ^ 1] = 0;
}

// FP64 source solves: the orbitals (row-major) receive the chunk-major
// iterate Xc of the CG.
template <int V>
__device__ __forceinline__ void cm_unpack_body(const Desc& d, int vb,
                                               double* __restrict__ red) {
  // FP64: the CG iterate; mixed (rcm): the refinement iterate.
  const double* src = d.Xc ? d.Xc : (d.rcm ? d.Xm : nullptr);
  if (!src) return;
  const Geo g = geo_of<V>(d, vb);
  if (g.lr >= g.tr) return;
  for (TileWalk w = tile_walk(g.ntiles, g.lb, g.nb); w.t < w.end;
       w.t += w.step) {
    const long long row = w.t * g.tr + g.lr;
    if (row >= d.n) continue;
    double x[V];
    ldv<double, V>(src + cm_index(d.n, row, g.ch * V, V), x);
    stv<double, V>(d.X + (size_t)row * d.ncols + g.ch * V, x);
  }
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
cm_unpack_kernel(const Desc* __restrict__ D, int nprob) {
  __shared__ double red[1];
  PARO_VB_LOOP64(D, nprob, VFIX, (cm_unpack_body<VV>(d, vb, red)))
}

// Squared floor of an FP32 inner pass's target, as a fraction of the outer
// tolerance: the pass stops at 0.8 rtol ||b|| at the lowest.  The 20 %
// margin covers the drift between the FP32 recursive residual and the FP64
// one; with a smaller margin the last pass over-solves (0.3: 4684 CG
// iterations per 64^3 solve, 0.8: 4403, FP64 alone: 4330), while a pass
// that stops short only costs one more (short) pass.
constexpr double kInnerFloor2 = 0.64;

// ------------------------------------------------------------------------
// Start of the FP64 source solves (eq. (alg-bvp) with the shift):
//   b = (lam - s) M u0  (or the given Bin),  x0 = u0,
//   r = b - A_s x0,  p = D^-1 r;  partials ||b||^2, r.z, ||r||^2.
// ------------------------------------------------------------------------
// HU: A_s u and M u come from the last rotation (d.HU, d.MU: U, lambda
// and the operator unchanged since), no operator application.
template <int V, bool HU>
__device__ __forceinline__ void pcg_start_body(const Desc& d, int vb,
    double* __restrict__ red) {
  const Geo g = geo_of<V>(d, vb);
  const int ncols = d.ncols;
  if (g.lb == 0 && threadIdx.x == 0) {  // read only by the finalize kernel
    ColState* cs = d.cs;
    cs->n_active[0] = 0;
    cs->n_active[1] = 0;
    cs->n_outer = 0;
    cs->status = 0;
    cs->maxit = d.maxit;
    cs->cg_mark = cs->cg_iters;
  }
  if (d.use_hu == 3) return;  // the last rotation emitted the start state
  const double* U = d.U0;
  double sh[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = g.ch * V + v;
    sh[v] = (d.lam && c < ncols) ? d.lam[c] - d.sigma : 0.0;
  }
  double acc[3][V];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[a][v] = 0.0;
  // The start state of one row from A_s u (au), M u (mu) and u.
  auto emit = [&](long long row, const double (&u)[V], const double (&au)[V],
                  const double (&mu)[V], double di) {
    const size_t o = (size_t)row * ncols + g.ch * V;
    double b[V], r[V], p[V];
    if (d.Bin) {
      ldv<double, V>(d.Bin + o, b);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) b[v] = sh[v] * mu[v];
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      r[v] = b[v] - au[v];
      p[v] = di * r[v];
      acc[0][v] += b[v] * b[v];
      acc[2][v] += r[v] * r[v];
    }
    if (d.R32) {
      // Mixed precision: this residual is also the first refinement
      // pass's (x0 = u0), so the FP32 inner CG starts from it directly:
      // r, p = D^-1 r rounded to FP32, correction 0, r.z of the rounded
      // values.
      float r32[V], p32[V], z32[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        r32[v] = (float)r[v];
        p32[v] = (float)p[v];
        z32[v] = 0.0f;
        acc[1][v] += (double)r32[v] * (double)p32[v];
      }
      const size_t o32 = cm_index(d.n, row, g.ch * V, d.v32);
      stv<float, V>(d.R32 + o32, r32);
      stv<float, V>(d.P32 + o32, p32);
      stv<float, V>(d.X32 + o32, z32);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) acc[1][v] += r[v] * p[v];
    }
    if (d.rcm) {  // mixed, chunk-major refinement: x0 and b
      const size_t oc = cm_index(d.n, row, g.ch * V, V);
      stv<double, V>(d.Xm + oc, u);
      stv<double, V>(d.B + oc, b);
      return;
    }
    if (d.X != U) stv<double, V>(d.X + o, u);
    if (d.Xc) {  // FP64 CG: its chunk-major start state
      const size_t oc = cm_index(d.n, row, g.ch * V, V);
      stv<double, V>(d.Xc + oc, u);
      stv<double, V>(d.R + oc, r);
      stv<double, V>(d.P + oc, p);
    }
    if (d.B) stv<double, V>(d.B + o, b);
  };
  if constexpr (HU) {
    // kTU tiles per group, all their loads before any store (which the
    // compiler cannot move the next tile's loads past); rows past the
    // end load row n - 1.  Rows are emitted in the same order as one
    // tile at a time.
    constexpr int kTU = 4;
    for (TileWalk w = tile_walk(g.ntiles, g.lb, g.nb); w.t < w.end;
         w.t += kTU * w.step) {
      double u[kTU][V], hu[kTU][V], mu[kTU][V], di[kTU];
      bool ok[kTU];
      long long rowk[kTU];
#pragma unroll
      for (int k = 0; k < kTU; ++k) {
        const long long t = w.t + k * w.step;
        const long long r0 = t * g.tr;
        ok[k] = t < w.end && g.lr < min((long long)g.tr, d.n - r0);
        rowk[k] = ok[k] ? r0 + g.lr : d.n - 1;
        const size_t o = (size_t)rowk[k] * ncols + g.ch * V;
        ldv<double, V>(U + o, u[k]);
        ldv<double, V>(d.HU + o, hu[k]);
        ldv<double, V>(d.MU + o, mu[k]);
        di[k] = ldg(d.dinv + rowk[k]);
      }
#pragma unroll
      for (int k = 0; k < kTU; ++k) {
        if (!ok[k]) continue;
        double au[V];
#pragma unroll
        for (int v = 0; v < V; ++v) au[v] = fma(-d.sigma, mu[k][v], hu[k][v]);
        emit(rowk[k], u[k], au, mu[k], di[k]);
      }
    }
  } else {
    extern __shared__ unsigned char smem[];
    double* wa = reinterpret_cast<double*>(smem);
    double* wb = wa + kStencil * g.tr;
    for (TileWalk w = tile_walk(g.ntiles, g.lb, g.nb); w.t < w.end;
         w.t += w.step) {
      const long long r0 = w.t * g.tr;
      const int rows = (int)min((long long)g.tr, d.n - r0);
      stage_weights<double, true>(d.diagA, d.diagM, d.n, r0, rows, g.tr, wa,
                                  wb);
      if (g.lr >= rows) continue;
      const long long row = r0 + g.lr;
      double au[V], mu[V], u[V];
#pragma unroll
      for (int v = 0; v < V; ++v) au[v] = mu[v] = 0.0;
      stencil_product<double, double, V, true, 8, true>(
          wa + g.lr, wb + g.lr, g.tr, d.mx, d.my, d.mz, row, U, ncols,
          g.ch * V, au, mu, u);
      if (d.kz) nl_add<V>(d, row, g.ch * V, au);  // A u += Z (Z^T u)
      emit(row, u, au, mu, ldg(d.dinv + row));
    }
  }
  block_partials<V, 3>(acc, ncols, g.cpr, g.tr, g.lb, g.nb, d.part, red);
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
pcg_start_kernel(const Desc* __restrict__ D, int nprob) {
  __shared__ double red[3 * kBlock * (VFIX ? VFIX : 2)];
  PARO_VB_LOOP64(D, nprob, VFIX,
                 (d.use_hu ? pcg_start_body<VV, true>(d, vb, red)
                           : pcg_start_body<VV, false>(d, vb, red)))
}

// Per-column start state: ||b||^2, r.z, ||r||^2, the stopping threshold
// and the first active set (grid: column x problem).  Every stopping test
// of the solve (the CG's, and the refinement's in mixed precision) is
// rtol^2 bb; with pcg_reduce the stored bb is raised to at least
// (pcg_reduce / rtol)^2 ||r0||^2, so the threshold becomes
// max(rtol ||b||, pcg_reduce ||r0||) in all of them.
__global__ void __launch_bounds__(kFinal)
pcg_start_final_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ncols) return;
  ColState* cs = d.cs;
  double tot[3];
  column_sums<3>(d.part + (size_t)d.start_part * kPartStride, kPartStride, c,
                 d.ns, tot);
  if (threadIdx.x != 0) return;
  const double rz = tot[1], rr = tot[2];
  // (A comparison, not fmax: a NaN ||b||^2 must stay NaN for the check
  // below.)
  const double bfl = d.reduce2 * rr;
  const double bb = tot[0] < bfl ? bfl : tot[0];
  const double rtol = d.rtol;
  cs->bb[c] = bb;
  cs->rz[c] = rz;
  cs->rzp[0][c] = rz;
  cs->rr[c] = rr;
  cs->rr64[c] = rr;
  // Mixed precision: the first inner FP32 pass's target (as in every
  // refinement pass); FP64: the solve's own.
  cs->tol2[c] = d.R32 ? fmax(d.inner_rtol * d.inner_rtol * rr,
                             kInnerFloor2 * rtol * rtol * bb)
                      : rtol * rtol * bb;
  cs->iters[c] = 0;
  cs->itp[0][c] = 0;
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
// the next FP32 inner CG pass for the correction.
//   r64 = B - A_s X;  converged columns (||r64|| <= rtol ||b||) retire;
//   the others solve A d = r64 in FP32 from d = 0, to
//   ||r|| <= inner_rtol ||r64||.  The first pass of a solve starts CG
//   (p = D^-1 r) from the start kernel's residual; the passes here keep
//   the search direction p and only replace the recursively updated
//   residual by the FP64 one (residual replacement), so CG continues
//   instead of restarting.
// ------------------------------------------------------------------------
template <int V>
__device__ __forceinline__ void refine_residual_body(const Desc& d, int vb,
    double* __restrict__ red) {
  if (d.rcm) return;  // refine_residual_zm_kernel
  const Geo g = geo_of<V>(d, vb);
  ColState* cs = d.cs;
  const int ncols = d.ncols;
  const bool on = g.lr < g.tr && chunk_active(cs->oact, g.ch, V, ncols);
  if (g.lb == 0 && threadIdx.x == 0) {  // read only by the finalize kernel
    cs->n_active[0] = 0;
    cs->n_active[1] = 0;
    cs->n_outer = 0;
    cs->cg_mark = cs->cg_iters;
  }
  double acc[2][V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[0][v] = acc[1][v] = 0.0;
  extern __shared__ unsigned char smem[];
  double* wa = reinterpret_cast<double*>(smem);
  for (TileWalk w = tile_walk(g.ntiles, g.lb, g.nb); w.t < w.end;
       w.t += w.step) {
    const long long r0 = w.t * g.tr;
    const int rows = (int)min((long long)g.tr, d.n - r0);
    stage_weights<double, false>(d.diagA, nullptr, d.n, r0, rows, g.tr, wa,
                                 nullptr);
    if (!on || g.lr >= rows) continue;
    const long long row = r0 + g.lr;
    double ax[V], unused[V], self[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ax[v] = 0.0;
    stencil_product<double, double, V, false, kStencil, true>(
        wa + g.lr, nullptr, g.tr, d.mx, d.my, d.mz, row, d.X, ncols,
        g.ch * V, ax, unused, self);
    const size_t o = (size_t)row * ncols + g.ch * V;
    double b[V];
    ldv<double, V>(d.B + o, b);
    const double di = ldg(d.dinv + row);
    float r32[V], z32[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double r = b[v] - ax[v];
      acc[0][v] += r * r;
      r32[v] = (float)r;
      z32[v] = 0.0f;
      acc[1][v] += (double)r32[v] * (double)(float)(di * r);
    }
    // FP32 vectors are chunk-major; the V FP64 columns of this thread lie
    // in one FP32 chunk (the FP32 width is a multiple of the FP64 one).
    const size_t o32 = cm_index(d.n, row, g.ch * V, d.v32);
    stv<float, V>(d.R32 + o32, r32);
    stv<float, V>(d.X32 + o32, z32);
  }
  block_partials<V, 2>(acc, ncols, g.cpr, g.tr, g.lb, g.nb, d.part, red);
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
refine_residual_kernel(const Desc* __restrict__ D, int nprob) {
  __shared__ double red[2 * kBlock * (VFIX ? VFIX : 2)];
  PARO_VB_LOOP64(D, nprob, VFIX,
                 (refine_residual_body<VV>(d, vb, red)))
}

// The same residual on a z-marching mesh whose refinement iterate Xm and
// right-hand sides B are chunk-major (rcm): a z-march over the chunks
// with an outer-active column (compacted into balanced groups), the
// coefficients formed from the potential (mf) or read from the stored
// stencil (the same values), the products in spmm_dual_kernel's order, so
// r64 is bitwise that of the row sweep.  Groups hold at most 3 chunks
// (two sums per column: 4 would leave one wavefront per SIMD).  The
// partials ||r64||^2 and the
// FP32 r.z go per (column, plane range x tile) to the p.q partial region
// (dead between CG passes): quantity a of column c, segment g at
// pqp[a ncols pqn + c pqn + g].
template <int V, int G, bool MF>
__device__ __forceinline__ void refine_zm_unit(const Desc& d, int tau,
                                               int zeta, const int (&cl)[4],
                                               unsigned long long amask,
                                               double* __restrict__ ws) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long n = d.n;
  const int ncols = d.ncols;
  double acc[G][2][V];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int u = 0; u < V; ++u) acc[g][a][u] = 0.0;
  zmf_march<double, V, G, MF>(
      d, tau, zeta, cl, d.Xm,
      [&](int g, long long row, bool valid, unsigned,
          const double (&a)[kStencil], const double (&x)[kStencil][V]) {
        double ax[V];
#pragma unroll
        for (int u = 0; u < V; ++u) ax[u] = 0.0;
#pragma unroll
        for (int s = 0; s < kStencil; ++s)
#pragma unroll
          for (int u = 0; u < V; ++u) ax[u] = fma(a[s], x[s][u], ax[u]);
        if (!valid) return;
        double b[V];
        ldv<double, V>(d.B + ((size_t)cl[g] * n + row) * V, b);
        const double di = ldg(d.dinv + row);
        float r32[V], z32[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
          const double r = b[u] - ax[u];
          acc[g][0][u] += r * r;
          r32[u] = (float)r;
          z32[u] = 0.0f;
          acc[g][1][u] += (double)r32[u] * (double)(float)(di * r);
        }
        const size_t o32 = cm_index(n, row, cl[g] * V, d.v32);
        stv<float, V>(d.R32 + o32, r32);
        stv<float, V>(d.X32 + o32, z32);
      });
  // Per (column, segment): wavefront, then the four wavefronts in order.
  constexpr int kGroup = 64 / V;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double tot = wave_reduce_scatter<V>(acc[g][a]);
      if ((lane & (kGroup - 1)) == 0)
        ws[(a * 4 + wave) * ncols + cl[g] * V + lane / kGroup] = tot;
    }
  __syncthreads();
  bool mine = false;
#pragma unroll
  for (int g = 0; g < G; ++g) mine = mine || tid / V == cl[g];
  if (mine && tid < ncols && ((amask >> tid) & 1)) {
    const size_t seg = (size_t)zeta * d.zxy + tau;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double* w = ws + a * 4 * ncols;
      const double sum = ((w[tid] + w[ncols + tid]) + w[2 * ncols + tid]) +
                         w[3 * ncols + tid];
      stg(d.pqp + ((size_t)a * ncols + tid) * d.pqn + seg, sum);
    }
  }
  __syncthreads();  // ws is reused by the next unit
}

template <int V, bool MF>
__device__ __forceinline__ void refine_zm_group(const Desc& d, int tau,
                                                int zeta, int gs,
                                                const int (&cl)[4],
                                                unsigned long long amask,
                                                double* ws) {
  switch (gs) {
    case 3: refine_zm_unit<V, 3, MF>(d, tau, zeta, cl, amask, ws); break;
    case 2: refine_zm_unit<V, 2, MF>(d, tau, zeta, cl, amask, ws); break;
    default: refine_zm_unit<V, 1, MF>(d, tau, zeta, cl, amask, ws); break;
  }
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
refine_residual_zm_kernel(const Desc* __restrict__ D, int nprob, int mf) {
  __shared__ double ws[2 * 4 * kNtMax];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (!d.rcm) return;  // refine_residual_kernel
  ColState* cs = d.cs;
  const int lb = blockIdx.x - d.b0;
  if (lb == 0 && threadIdx.x == 0) {  // read only by the finalize kernel
    cs->n_active[0] = 0;
    cs->n_active[1] = 0;
    cs->n_outer = 0;
    cs->cg_mark = cs->cg_iters;
  }
  const unsigned long long amask = active_mask(cs->oact, d.ncols);
  const int vw = VFIX ? VFIX : d.v64;
  const unsigned long long cm = chunk_mask(amask, d.ncols / vw, vw);
  const int nac = __popcll(cm);
  if (nac == 0) return;
  const int nag = (nac + 2) / 3;
  const int x = lb % kXcd, l = lb / kXcd, gx = d.nb / kXcd;
  const int zr = d.zm / kXcd;
  const long long units = (long long)zr * d.zxy * nag;
  for (long long k = l; k < units; k += gx) {
    const long long rest = k / nag;
    const int gi = (int)(k - rest * nag);
    const int tau = (int)(rest % d.zxy);
    const int zeta = x * zr + (int)(rest / d.zxy);
    const int r0 = gi * nac / nag, r1 = (gi + 1) * nac / nag;
    int cl[4];
    unsigned long long rem = cm;
    for (int r = 0; r < r0; ++r) rem &= rem - 1;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      cl[g] = rem ? __builtin_ctzll(rem) : 0;
      if (g < r1 - r0) rem &= rem - 1;
    }
    if (vw == 2) {
      if (mf)
        refine_zm_group<2, true>(d, tau, zeta, r1 - r0, cl, amask, ws);
      else
        refine_zm_group<2, false>(d, tau, zeta, r1 - r0, cl, amask, ws);
    } else {
      if (mf)
        refine_zm_group<1, true>(d, tau, zeta, r1 - r0, cl, amask, ws);
      else
        refine_zm_group<1, false>(d, tau, zeta, r1 - r0, cl, amask, ws);
    }
  }
}

// Outer (refinement) test per column and the inner threshold of the next
// FP32 solve (grid: column x problem).
__global__ void __launch_bounds__(kFinal)
refine_final_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ncols) return;
  ColState* cs = d.cs;
  if (!cs->oact[c]) {
    if (threadIdx.x == 0) {
      cs->act[0][c] = 0;
      cs->act[1][c] = 0;
    }
    return;
  }
  double tot[2];
  if (d.rcm)
    column_sums<2>(d.pqp, (size_t)d.ncols * d.pqn, c, d.pqn, tot);
  else
    column_sums<2>(d.part, kPartStride, c, d.ns, tot);
  if (threadIdx.x != 0) return;
  int a = 0;
  const double rr = tot[0], rtol = d.rtol, irt = d.inner_rtol;
  if (!isfinite(rr)) {
    atomicOr(&cs->status, (int)kStNonFinite);
  } else {
    cs->rr64[c] = rr;
    const bool more = rr > rtol * rtol * cs->bb[c];
    a = (more && cs->iters[c] < cs->maxit) ? 1 : 0;
    if (more && !a) atomicOr(&cs->status, (int)kStNoConv);
    // Inner target: inner_rtol ||r64||, but no lower than what the outer
    // test needs, with a margin (kInnerFloor2).
    cs->tol2[c] = fmax(irt * irt * rr, kInnerFloor2 * rtol * rtol * cs->bb[c]);
    // The continuing pass takes the last step's beta with the replaced
    // residual: beta = (r.z)_new / (r.z) of the step before.
    if (a) cs->beta[c] = cs->beta[c] * (tot[1] / cs->rz[c]);
    cs->rz[c] = tot[1];
    cs->rzp[0][c] = tot[1];  // the next pass starts at parity 0
    cs->itp[0][c] = cs->iters[c];
  }
  cs->oact[c] = a;
  cs->act[0][c] = a;
  cs->act[1][c] = 0;
  if (a) {
    atomicAdd(&cs->n_active[0], 1);
    atomicAdd(&cs->n_outer, 1);
  }
}

// Xm += d for a chunk-major refinement iterate (rcm): chunk by chunk
// (those with a refining column; uniform), the problem's threads over the
// chunk's rows, four rows per thread loaded before any is stored.
template <int V>
__device__ __forceinline__ void refine_update_cm(const Desc& d, int vb) {
  const ColState* cs = d.cs;
  const int cpr = d.ncols / V;
  const long long n = d.n;
  const long long stride = (long long)d.ns * kBlock;
  constexpr int kTU = 4;
  for (int ch = 0; ch < cpr; ++ch) {
    bool a[V], any = false;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      a[v] = ldg(&cs->oact[ch * V + v]) != 0;
      any = any || a[v];
    }
    if (!any) continue;
    double* xm = d.Xm + (size_t)ch * n * V;
    for (long long r0 = (long long)vb * kBlock + threadIdx.x; r0 < n;
         r0 += kTU * stride) {
      double x[kTU][V];
      float dx[kTU][V];
#pragma unroll
      for (int k = 0; k < kTU; ++k) {
        const long long row = min(r0 + k * stride, n - 1);
        ldv<double, V>(xm + (size_t)row * V, x[k]);
        ldv<float, V>(d.X32 + cm_index(n, row, ch * V, d.v32), dx[k]);
      }
#pragma unroll
      for (int k = 0; k < kTU; ++k) {
        const long long row = r0 + k * stride;
        if (row >= n) continue;
#pragma unroll
        for (int v = 0; v < V; ++v) x[k][v] += a[v] ? (double)dx[k][v] : 0.0;
        stv<double, V>(xm + (size_t)row * V, x[k]);
      }
    }
  }
}

// X += d (FP32 correction) for columns that refined in this pass.
template <int V>
__device__ __forceinline__ void refine_update_body(const Desc& d, int vb,
    double* __restrict__ red) {
  if (d.rcm) {
    refine_update_cm<V>(d, vb);
    return;
  }
  const Geo g = geo_of<V>(d, vb);
  const ColState* cs = d.cs;
  const int ncols = d.ncols;
  if (g.lr >= g.tr || !chunk_active(cs->oact, g.ch, V, ncols)) return;
  bool a[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int c = g.ch * V + v;
    a[v] = c < ncols && cs->oact[c];
  }
  // kTU tiles per group: all their loads before any store (the stores
  // could alias the next loads for the compiler, which would otherwise
  // wait a round trip per tile); rows past the end load row n - 1.
  constexpr int kTU = 4;
  for (TileWalk w = tile_walk(g.ntiles, g.lb, g.nb); w.t < w.end;
       w.t += kTU * w.step) {
    double x[kTU][V];
    float dx[kTU][V];
#pragma unroll
    for (int k = 0; k < kTU; ++k) {
      const long long t = w.t + k * w.step;
      const long long row =
          t < w.end ? min(t * g.tr + g.lr, d.n - 1) : d.n - 1;
      ldv<double, V>(d.X + (size_t)row * ncols + g.ch * V, x[k]);
      ldv<float, V>(d.X32 + cm_index(d.n, row, g.ch * V, d.v32), dx[k]);
    }
#pragma unroll
    for (int k = 0; k < kTU; ++k) {
      const long long t = w.t + k * w.step;
      const long long row = t * g.tr + g.lr;
      if (t >= w.end || row >= d.n) continue;
#pragma unroll
      for (int v = 0; v < V; ++v) x[k][v] += a[v] ? (double)dx[k][v] : 0.0;
      stv<double, V>(d.X + (size_t)row * ncols + g.ch * V, x[k]);
    }
  }
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
refine_update_kernel(const Desc* __restrict__ D, int nprob) {
  __shared__ double red[1 * kBlock * (VFIX ? VFIX : 2)];
  PARO_VB_LOOP64(D, nprob, VFIX, (refine_update_body<VV>(d, vb, red)))
}

// Sum over the table of the active CG columns (which = 0 or 1: that
// parity) or of the refining columns (which = 2), for the host's poll (one
// block); out[4] is always the refining count.
__global__ void __launch_bounds__(kBlock)
count_active_kernel(const Desc* __restrict__ D, int nprob, int which,
                    int* __restrict__ out, int seq) {
  __shared__ int red[kBlock], mx[kBlock], st[kBlock], ot[kBlock];
  int s = 0, m = 0, f = 0, o = 0;
  for (int p = threadIdx.x; p < nprob; p += kBlock) {
    const ColState* cs = D[p].cs;
    s += which == 2 ? cs->n_outer : cs->n_active[which];
    o += cs->n_outer;
    m = max(m, (int)(cs->cg_iters - cs->cg_mark));
    f |= cs->status;
  }
  red[threadIdx.x] = s;
  mx[threadIdx.x] = m;
  st[threadIdx.x] = f;
  ot[threadIdx.x] = o;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      mx[threadIdx.x] = max(mx[threadIdx.x], mx[threadIdx.x + w]);
      st[threadIdx.x] |= st[threadIdx.x + w];
      ot[threadIdx.x] += ot[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[1] = red[0];
    out[2] = mx[0];
    out[3] = st[0];
    out[4] = ot[0];
    // out is host memory the caller spins on: the values, then the
    // sequence number with system-scope release.
    __hip_atomic_store(&out[0], seq, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Per-problem status and convergence measures of the last step (one
// block), then the sequence number *seqp = seq (system-scope release).
__global__ void __launch_bounds__(kBlock)
gather_reports_kernel(const Desc* __restrict__ D, int nprob,
                      PollReport* __restrict__ out, int* __restrict__ seqp,
                      int seq) {
  for (int p = threadIdx.x; p < nprob; p += kBlock) {
    const Desc& d = D[p];
    const ColState* cs = d.cs;
    int it = 0;
    for (int c = 0; c < d.ncols; ++c) it = max(it, cs->iters[c]);
    PollReport r;
    r.status = cs->status;
    r.max_iters = it;
    r.geneig_info = *d.geneig_info;
    r.pad = 0;
    r.max_dlambda = d.si->max_dlambda;
    r.max_resid = d.si->max_resid;
    out[p] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(seqp, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------------
// SpMM (FP64): Y1 = A_s X + s1 M X, Y2 = M X.  Rayleigh-Ritz form (rr):
// X -> R = H X (s1 = sigma), Q = M X.  Component form: Y1, Y2, s1 of the
// descriptor (either output may be null).
// ------------------------------------------------------------------------
template <int V, bool NL>
__device__ __forceinline__ void spmm_dual_body(const Desc& d, int vb, int rr,
    double* __restrict__ red) {
  if (d.csr) return;  // csr_dual_kernel
  const Geo g = geo_of<V>(d, vb);
  const int ncols = d.ncols;
  double* Y1 = rr ? d.HU : d.Y1;  // Rayleigh-Ritz: H W, M W over H U, M U
  double* Y2 = rr ? d.MU : d.Y2;
  const double s1 = rr ? d.sigma : d.s1;
  const double* X = d.X;
  const bool needA = Y1 != nullptr;
  const bool needM = Y2 != nullptr || s1 != 0.0;
  extern __shared__ unsigned char smem[];
  double* wa = reinterpret_cast<double*>(smem);
  double* wb = wa + kStencil * g.tr;
  const bool two = needA && needM;
  const double* da = needA ? d.diagA : d.diagM;
  const double* db = two ? d.diagM : nullptr;
  // A tile's coefficients fit one per thread (15 tr <= 256: 15 or more
  // chunks per row): the next tile's are loaded into registers before this
  // tile's products, so their latency overlaps the products' loads, and
  // stored to LDS at the top of the next iteration.
  const bool pf = kStencil * g.tr <= kBlock;
  double na = 0.0, nm = 0.0;
  auto prefetch = [&](long long t) {
    const long long r0 = t * g.tr;
    const int rows = (int)min((long long)g.tr, d.n - r0);
    const int e = threadIdx.x;
    if (e < kStencil * rows) {
      const int s = e / rows, lr = e - s * rows;
      na = ldg(da + (size_t)s * d.n + r0 + lr);
      if (two) nm = ldg(db + (size_t)s * d.n + r0 + lr);
    }
  };
  TileWalk w = tile_walk(g.ntiles, g.lb, g.nb);
  if (pf && w.t < w.end) prefetch(w.t);
  for (; w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * g.tr;
    const int rows = (int)min((long long)g.tr, d.n - r0);
    if (pf) {
      __syncthreads();  // the previous tile's products are done with LDS
      const int e = threadIdx.x;
      if (e < kStencil * rows) {
        const int s = e / rows, lr = e - s * rows;
        wa[s * g.tr + lr] = na;
        if (two) wb[s * g.tr + lr] = nm;
      }
      __syncthreads();
      if (w.t + w.step < w.end) prefetch(w.t + w.step);
    } else if (two) {
      stage_weights<double, true>(da, db, d.n, r0, rows, g.tr, wa, wb);
    } else {
      stage_weights<double, false>(da, nullptr, d.n, r0, rows, g.tr, wa,
                                   nullptr);
    }
    if (g.lr >= rows) continue;
    const long long row = r0 + g.lr;
    double ax[V], mx[V], self[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ax[v] = mx[v] = 0.0;
    if (two)
      stencil_product<double, double, V, true, 8, true>(
          wa + g.lr, wb + g.lr, g.tr, d.mx, d.my, d.mz, row, X, ncols,
          g.ch * V, ax, mx, self);
    else if (needA)
      stencil_product<double, double, V, false, 8, true>(
          wa + g.lr, nullptr, g.tr, d.mx, d.my, d.mz, row, X, ncols,
          g.ch * V, ax, mx, self);
    else
      stencil_product<double, double, V, false, 8, true>(
          wa + g.lr, nullptr, g.tr, d.mx, d.my, d.mz, row, X, ncols,
          g.ch * V, mx, ax, self);
    const size_t o = (size_t)row * ncols + g.ch * V;
    if (Y1) {
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = fma(s1, mx[v], ax[v]);
      if (NL && rr && d.kz) nl_add<V>(d, row, g.ch * V, y);  // + Z Z^T W
      stv<double, V>(Y1 + o, y);
    }
    if (Y2) stv<double, V>(Y2 + o, mx);
  }
}

// NL: some problem of the table has a nonlocal term.
template <int VFIX, bool NL>
__global__ void PARO_STREAM_BOUNDS
spmm_dual_kernel(const Desc* __restrict__ D, int nprob, int rr) {
  __shared__ double red[1 * kBlock * (VFIX ? VFIX : 2)];
  PARO_VB_LOOP64(D, nprob, VFIX, (spmm_dual_body<VV, NL>(d, vb, rr, red)))
}


// ------------------------------------------------------------------------
// Gram contractions G1 = W^T Y1, G2 = W^T Y2 on FP64 matrix cores
// (v_mfma_f64_16x16x4_f64).  Each wavefront consumes 4 rows per MFMA:
// A = 16 columns of W over the 4 rows (lane l: row l/16, column l%16),
// B = 16 columns of Y over the same rows; D accumulates 16 x 16 tiles.
// sym: only tile pairs I <= J of (Y1 = H W, Y2 = M W) in the
// Rayleigh-Ritz form; otherwise all tiles of G = W^T Y1 (component form).
// Partial tiles per block; the reduction and scatter follow.
// ------------------------------------------------------------------------
// Tiles of one problem's Gram: pairs I <= J (sym) or all I, J, 16 x 16.
__host__ __device__ constexpr int gram_ntiles(int nt16, bool sym) {
  return sym ? nt16 * (nt16 + 1) / 2 : nt16 * nt16;
}

// Virtual block vb (of gns) of a problem: its wavefronts take contiguous
// ranges of 4-row steps; the block's tiles go to gpart[vb] in the
// problem's own tile numbering.  sg: LDS of NG * NP * 256 doubles.
template <int NT16, bool SYM>
__device__ __forceinline__ void gram_body(const Desc& d, int vb,
                                          double* __restrict__ sg) {
  constexpr int NP = gram_ntiles(NT16, SYM);
  constexpr int NG = SYM ? 2 : 1;
  const int nb = d.gns;
  const double* W = d.X;
  const double* Y1 = SYM ? d.HU : d.Y1;
  const double* Y2 = SYM ? d.MU : nullptr;
  const long long n = d.n;
  const int ncols = d.ncols;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc[NG][NP];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[g][q] = v4d{0.0, 0.0, 0.0, 0.0};
  const long long nsteps = (n + 3) / 4;
  const long long gw = (long long)vb * 4 + wave;
  const long long nw = (long long)nb * 4;
  const long long per = (nsteps + nw - 1) / nw;
  const long long s0 = gw * per, s1 = min(nsteps, s0 + per);
  // GU steps per group: their loads (unconditional, clamped addresses;
  // masked values are 0) are in flight together before the MFMAs, which
  // run step by step in the same order as one step at a time.
  constexpr int GU = NT16 <= 1 ? 8 : (NT16 <= 3 ? 4 : 2);
  for (long long st0 = s0; st0 < s1; st0 += GU) {
    double a[GU][NT16], y1[GU][NT16], y2[GU][NT16];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const long long row = (st0 + u) * 4 + lk;
      const bool rok = st0 + u < s1 && row < n;
#pragma unroll
      for (int I = 0; I < NT16; ++I) {
        const int c = I * 16 + li;
        const bool ok = rok && c < ncols;
        const size_t o = ok ? (size_t)row * ncols + c : 0;
        const double va = ldg(W + o), vy1 = ldg(Y1 + o);
        a[u][I] = ok ? va : 0.0;
        y1[u][I] = ok ? vy1 : 0.0;
        if (SYM) {
          const double vy2 = ldg(Y2 + o);
          y2[u][I] = ok ? vy2 : 0.0;
        } else {
          y2[u][I] = 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      int q = 0;
#pragma unroll
      for (int I = 0; I < NT16; ++I)
#pragma unroll
        for (int J = SYM ? I : 0; J < NT16; ++J, ++q) {
          acc[0][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              a[u][I], y1[u][J], acc[0][q], 0, 0, 0);
          if (SYM)
            acc[NG - 1][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a[u][I], y2[u][J], acc[NG - 1][q], 0, 0, 0);
        }
    }
  }
  // D layout (measured): lane l, element r holds row l/16 + 4r, column
  // l%16.  The four wavefronts' tiles are added in wave order.
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int q = 0; q < NP; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int idx = ((g * NP + q) * 16 + lk + 4 * r) * 16 + li;
            if (w == 0)
              sg[idx] = acc[g][q][r];
            else
              sg[idx] += acc[g][q][r];
          }
    }
    __syncthreads();
  }
  const int per_blk = NG * NP * 256;
  for (int e = threadIdx.x; e < per_blk; e += kBlock)
    stg(d.gpart + (size_t)vb * per_blk + e, sg[e]);
  __syncthreads();
}

// First stage: block lb of the problem's gnb serves virtual blocks lb,
// lb + gnb, ... < gns, at the problem's own tile count (NT16MAX: the
// widest problem of the launch; !MIXED: all problems have NT16MAX).
template <int NT16MAX, bool SYM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
gram_kernel(const Desc* __restrict__ D, int nprob) {
  __shared__ double sg[(SYM ? 2 : 1) * gram_ntiles(NT16MAX, SYM) * 256];
  const Desc& d = D[owner(D, nprob, blockIdx.x, true)];
  const int nt16 = (d.ncols + 15) / 16;
  for (int vb = blockIdx.x - d.g0; vb < d.gns; vb += d.gnb) {
    if constexpr (!MIXED) {
      gram_body<NT16MAX, SYM>(d, vb, sg);  // every problem has NT16MAX
    } else if (nt16 == 1) {
      gram_body<1, SYM>(d, vb, sg);
    } else if (nt16 == 2) {
      if constexpr (NT16MAX >= 2) gram_body<2, SYM>(d, vb, sg);
    } else if (nt16 == 3) {
      if constexpr (NT16MAX >= 3) gram_body<3, SYM>(d, vb, sg);
    } else {
      if constexpr (NT16MAX >= 4) gram_body<4, SYM>(d, vb, sg);
    }
  }
}

__device__ __forceinline__ int gram_per_blk(int ncols, bool sym) {
  return (sym ? 2 : 1) * gram_ntiles((ncols + 15) / 16, sym) * 256;
}

// Second stage, one wavefront per result entry (grid: entries / 4 x
// problem): the entry's first-stage partials over the problem's gns
// segments are summed in a fixed order (lane l adds segments l, l + 64,
// ..., then a butterfly) and written to Ah = W^T H W, Bh = W^T M W
// (sym: entries i <= j, mirrored, diagonal tiles symmetrised) or to
// Y2 = W^T Y1 (component form).
__device__ __forceinline__ double gram_entry_sum(const Desc& d, int per_blk,
                                                 int e) {
  // Lane l adds partials l, l + 64, ... in ascending order; the loads of
  // kU of them are issued together (clamped addresses, masked adds), so
  // the kGramGrid partials cost one round trip.
  constexpr int kU = kGramGrid / 64;
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  for (int b0 = 0; b0 < d.gns; b0 += kU * 64) {
    double x[kU];
#pragma unroll
    for (int i = 0; i < kU; ++i)
      x[i] = ldg(d.gpart +
                 (size_t)min(b0 + lane + i * 64, d.gns - 1) * per_blk + e);
#pragma unroll
    for (int i = 0; i < kU; ++i)
      v = (b0 + lane + i * 64 < d.gns) ? v + x[i] : v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(kBlock)
gram_final_kernel(const Desc* __restrict__ D, int sym) {
  const Desc& d = D[blockIdx.y];
  const int ncols = d.ncols;
  const int o = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (o >= ncols * ncols) return;
  const int i = o / ncols, j = o % ncols;
  const int nt16 = (ncols + 15) / 16;
  const int per_blk = gram_per_blk(ncols, sym != 0);
  const bool lead = (threadIdx.x & 63) == 0;
  if (!sym) {
    const double v = gram_entry_sum(
        d, per_blk, ((i / 16) * nt16 + j / 16) * 256 + (i % 16) * 16 + j % 16);
    if (lead) d.Y2[o] = v;
    return;
  }
  if (i > j) return;
  const int I = i / 16, J = j / 16;
  const int q = I * nt16 - I * (I - 1) / 2 + (J - I);
  const int np = gram_ntiles(nt16, true);
  const int ea = (i % 16) * 16 + j % 16, eb = (j % 16) * 16 + i % 16;
  for (int g = 0; g < 2; ++g) {
    const int base = (g * np + q) * 256;
    double v = gram_entry_sum(d, per_blk, base + ea);
    if (I == J) v = 0.5 * (v + gram_entry_sum(d, per_blk, base + eb));
    if (lead) {
      double* G = g == 0 ? d.Ah : d.Bh;
      G[i * ncols + j] = v;
      G[j * ncols + i] = v;
    }
  }
}

// ------------------------------------------------------------------------
// Small generalised eigenproblem A c = theta B c (Step 4's N_t x N_t
// problem), one workgroup of kGeThreads, FP64, everything in LDS.
//   1. B = L L^T (Cholesky, right-looking, one barrier per column);
//   2. Li = L^{-1} (column j by thread j: a forward substitution each,
//      no barriers), S = Li A Li^T as two small products;
//   3. cyclic Jacobi on S with round-robin ordering: N_t/2 disjoint
//      rotations per round, formed once (one thread per pair) into LDS,
//      then applied as independent 2 x 2 blocks from one LDS copy of S
//      into the other (two copies alternate) and to Y: two barriers per
//      round;
//   4. theta ascending (ties by index);  5. C = Li^T Y;  6. signs.
// ------------------------------------------------------------------------
constexpr int kLd = kNtMax + 1;
constexpr int kGeThreads = 512;

// Maximum over a wavefront (every lane receives it).
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Round-robin pair `slot` of round `round` over nn (even) indices: slot 0
// pairs index 0 with the rotating ring's head; the ring 1 .. nn-1
// advances by one per round.  Every index is in exactly one pair.
__device__ __forceinline__ void rr_pair(int slot, int round, int nn, int& p,
                                        int& q) {
  int a0 = slot == 0 ? 0 : slot + round;
  a0 = a0 > nn - 1 ? a0 - (nn - 1) : a0;
  int b0 = nn - 1 - slot + round;
  b0 = b0 > nn - 1 ? b0 - (nn - 1) : b0;
  p = a0 < b0 ? a0 : b0;
  q = a0 < b0 ? b0 : a0;
}

// The Jacobi rotation (c, s) annihilating S[p][q] (identity when q is the
// dummy index of an odd n or |S[p][q]| <= skip): the smaller angle, tan t =
// sgn(d) h / (|d| + r) with d = S[q][q] - S[p][p], h = 2 S[p][q] and
// r = sqrt(d^2 + h^2).  With w = |d| + r, 1 + tan^2 t = 2 r w / w^2, so
// c = w / sqrt(2 r w) and s = sgn(d) h / sqrt(2 r w): two square roots and
// one division on the round's critical path, no cancellation.
__device__ __forceinline__ bool jacobi_cs(const double (*S)[kLd], int p,
                                          int q, int n, double skip,
                                          double& c, double& sn) {
  c = 1.0;
  sn = 0.0;
  if (q >= n) return false;
  const double apq = S[p][q];
  if (!(fabs(apq) > skip)) return false;
  const double d = S[q][q] - S[p][p], h = 2.0 * apq;
  const double r = sqrt(fma(d, d, h * h));
  const double w = fabs(d) + r;
  const double k = 1.0 / sqrt(2.0 * r * w);
  c = w * k;
  sn = (d >= 0.0 ? h : -h) * k;
  return true;
}

__device__ void geneig_body(const double* __restrict__ Ain,
                            const double* __restrict__ Bin, int n,
                            double* __restrict__ theta_out,
                            double* __restrict__ C_out,
                            int* __restrict__ info_out,
                            int* __restrict__ status,
                            const int* __restrict__ clus) {
  __shared__ double Sa[kNtMax][kLd];  // A, then S and Jacobi ping
  __shared__ double Sb[kNtMax][kLd];  // Li A, then Jacobi pong, then C
  __shared__ double L[kNtMax][kLd];   // B; L^T (strict upper); Li (lower)
  __shared__ double Y[kNtMax][kLd];   // eigenvectors of S
  __shared__ double red[kGeThreads / 64];
  __shared__ int s_info, s_rot;
  __shared__ int perm[kNtMax];
  __shared__ double th[kNtMax];
  __shared__ double ld[kNtMax];  // diagonal of L
  __shared__ double rc_c[kNtMax / 2], rc_s[kNtMax / 2];
  __shared__ int rc_r[kNtMax / 2];
  const int tid = threadIdx.x;
  const int nn = n + (n & 1);
  // Zero the padded LDS matrices (odd n uses row/column n as a dummy),
  // then load the n x n inputs.
  for (int e = tid; e < kNtMax * kNtMax; e += kGeThreads) {
    const int i = e / kNtMax, j = e % kNtMax;
    Sa[i][j] = 0.0;
    Sb[i][j] = 0.0;
    L[i][j] = 0.0;
    Y[i][j] = (i == j && i < n) ? 1.0 : 0.0;
  }
  if (tid == 0) s_info = 0;
  __syncthreads();
  // Cluster-wise projection: entries coupling different clusters are
  // dropped, so every step below works block by block (the factor, its
  // inverse, the products and the rotations of a block-diagonal pencil
  // never mix blocks).
#pragma unroll 4
  for (int e = tid; e < n * n; e += kGeThreads) {
    const int i = e / n, j = e % n;
    const bool keep = !clus || clus[i] == clus[j];
    Sa[i][j] = keep ? Ain[e] : 0.0;
    L[i][j] = keep ? Bin[e] : 0.0;
  }
  if (tid < n) th[tid] = Bin[tid * n + tid];  // diagonal of B (pivot test)
  __syncthreads();

  // 1. Cholesky, right-looking: at step k the pivot d = B_k[k][k] of the
  // running Schur complement is read, column k scaled by 1/sqrt(d) is
  // stored transposed in the strict upper triangle (row k, which no later
  // step touches), and the trailing lower triangle is updated with the
  // unscaled column (b_ik b_jk / d), all in one phase.
  for (int k = 0; k < n; ++k) {
    const double piv = L[k][k];
    // A pivot at rounding level of the diagonal means the columns are
    // linearly dependent in the M inner product.
    const bool bad = !(piv > 1e-14 * th[k]) || !isfinite(piv);
    const double d = bad ? 1.0 : piv;
    const double lkk = sqrt(d), rd = 1.0 / d, rl = 1.0 / lkk;
    const int m = n - k - 1;
    for (int e = tid; e < m * (m + 1); e += kGeThreads) {
      if (e < m * m) {
        const int i = k + 1 + e / m, j = k + 1 + e % m;
        if (j <= i) L[i][j] -= (L[i][k] * rd) * L[j][k];
      } else {
        const int i = k + 1 + (e - m * m);
        L[k][i] = L[i][k] * rl;
      }
    }
    if (tid == 0) {
      ld[k] = lkk;
      if (bad && s_info == 0) s_info = k + 1;
    }
    __syncthreads();
  }
  if (s_info != 0) {
    if (tid == 0) {
      *info_out = s_info;
      if (status) atomicOr(status, (int)kStSingular);
    }
    for (int e = tid; e < n * n; e += kGeThreads)
      C_out[e] = (e / n == e % n) ? 1.0 : 0.0;
    for (int e = tid; e < n; e += kGeThreads) theta_out[e] = Ain[e * n + e];
    return;
  }

  // 2. Li = L^{-1}: thread j solves L x = e_j by forward substitution
  // (x_i = -(sum_{j <= k < i} L[i][k] x_k) / L[i][i]) and keeps x in
  // column j of the lower triangle (L[i][k] is read from its transposed
  // copy L^T[k][i]; the lower triangle's old contents are dead).
  if (tid < n) {
    const int j = tid;
    L[j][j] = 1.0 / ld[j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[k][i] * L[k][j];
      L[i][j] = -s / ld[i];
    }
  }
  __syncthreads();
  // Sb = Li A (Li lower triangular: k <= i).
  for (int e = tid; e < n * n; e += kGeThreads) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int k = 0; k <= i; ++k) s += L[i][k] * Sa[k][j];
    Sb[i][j] = s;
  }
  __syncthreads();
  // S = (Li A) Li^T, symmetrised: S[i][j] = S[j][i] = the mean of the two
  // computed triangles.
  for (int e = tid; e < n * n; e += kGeThreads) {
    const int i = e / n, j = e % n;
    if (i > j) continue;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k <= j; ++k) s1 += Sb[i][k] * L[j][k];
    for (int k = 0; k <= i; ++k) s2 += Sb[j][k] * L[i][k];
    const double s = i == j ? s1 : 0.5 * (s1 + s2);
    Sa[i][j] = s;
    Sa[j][i] = s;
  }
  __syncthreads();

  // 3. Cyclic Jacobi, round-robin pairs.  A rotation is skipped when
  // |s_pq| <= 1e-17 ||S||_F (already zero at working precision); the
  // iteration stops before a sweep that would rotate nothing.
  const int half = nn / 2;
  const int nblk = half * half;
  const int nwave = kGeThreads / 64;
  double fro2 = 0.0;
  for (int e = tid; e < n * n; e += kGeThreads) {
    const double v = Sa[e / n][e % n];
    fro2 += v * v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fro2 += __shfl_xor(fro2, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = fro2;
  __syncthreads();
  double tot = 0.0;
  for (int w = 0; w < nwave; ++w) tot += red[w];
  const double skip = 1e-17 * sqrt(tot);
  double (*Sc)[kLd] = Sa;  // the current S
  double (*Sn)[kLd] = Sb;  // the next S
  for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
    double off = 0.0;
    for (int e = tid; e < n * n; e += kGeThreads) {
      const int i = e / n, j = e % n;
      if (i < j) off = fmax(off, fabs(Sc[i][j]));
    }
    off = wave_max(off);
    __syncthreads();  // red is rewritten
    if ((tid & 63) == 0) red[tid >> 6] = off;
    if (tid == 0) s_rot = 0;
    __syncthreads();
    double mx = 0.0;
    for (int w = 0; w < nwave; ++w) mx = fmax(mx, red[w]);
    if (mx <= skip) break;
    for (int round = 0; round < nn - 1; ++round) {
      // The round's rotations, formed once (thread k: pair k), then
      // applied as independent 2 x 2 blocks and to Y.
      if (tid < half) {
        int p, q;
        rr_pair(tid, round, nn, p, q);
        double c, sn;
        const bool rot = jacobi_cs(Sc, p, q, n, skip, c, sn);
        rc_c[tid] = c;
        rc_s[tid] = sn;
        rc_r[tid] = rot ? 1 : 0;
        if (rot) s_rot = 1;
      }
      __syncthreads();
      for (int e = tid; e < nblk + n * half; e += kGeThreads) {
        if (e < nblk) {
          const int k = e / half, l = e - k * half;
          int p, q, r, t;
          rr_pair(k, round, nn, p, q);
          rr_pair(l, round, nn, r, t);
          const double c1 = rc_c[k], s1 = rc_s[k];
          const double c2 = rc_c[l], s2 = rc_s[l];
          const bool rot = rc_r[k] != 0;
          const double apr = Sc[p][r], apt = Sc[p][t];
          const double aqr = Sc[q][r], aqt = Sc[q][t];
          const double bpr = c1 * apr - s1 * aqr, bpt = c1 * apt - s1 * aqt;
          const double bqr = s1 * apr + c1 * aqr, bqt = s1 * apt + c1 * aqt;
          double cpt = s2 * bpr + c2 * bpt, cqr = c2 * bqr - s2 * bqt;
          if (k == l && rot) cpt = cqr = 0.0;  // the annihilated pair
          Sn[p][r] = c2 * bpr - s2 * bpt;
          Sn[p][t] = cpt;
          Sn[q][r] = cqr;
          Sn[q][t] = s2 * bqr + c2 * bqt;
        } else {
          const int e2 = e - nblk, l = e2 / n, i = e2 - l * n;
          int p, q;
          rr_pair(l, round, nn, p, q);
          const double c = rc_c[l], sn = rc_s[l];
          const double yp = Y[i][p], yq = Y[i][q];
          Y[i][p] = c * yp - sn * yq;
          Y[i][q] = sn * yp + c * yq;
        }
      }
      __syncthreads();
      double (*sw)[kLd] = Sc;
      Sc = Sn;
      Sn = sw;
    }
    if (s_rot == 0) break;
  }

  // 4. Ascending order, ties broken by index (with clusters: within each
  // cluster, which keeps its columns).
  if (tid < n) th[tid] = Sc[tid][tid];
  __syncthreads();
  if (tid < n) {
    int rank = 0;
    const double t = th[tid];
    const int c = clus ? clus[tid] : 0;
    for (int j = 0; j < n; ++j) {
      const int cj = clus ? clus[j] : 0;
      if (cj < c)
        ++rank;
      else if (cj == c)
        rank += (th[j] < t || (th[j] == t && j < tid)) ? 1 : 0;
    }
    perm[rank] = tid;
  }
  __syncthreads();
  // 5. C[:, r] = Li^T Y[:, perm[r]] (Li lower triangular: k >= i), into
  // the free copy of S.
  double (*Cs)[kLd] = Sn;
  for (int e = tid; e < n * n; e += kGeThreads) {
    const int i = e / n, r = e % n, src = perm[r];
    double s = 0.0;
    for (int k = i; k < n; ++k) s += L[k][i] * Y[k][src];
    Cs[i][r] = s;
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


__global__ void __launch_bounds__(kGeThreads)
small_geneig_kernel(const double* __restrict__ A, const double* __restrict__ B,
                    int n, double* __restrict__ theta, double* __restrict__ C,
                    int* __restrict__ info) {
  geneig_body(A, B, n, theta, C, info, nullptr, nullptr);
}

// Step 4's small eigenproblem of every problem of the table (one block
// per problem).
__global__ void __launch_bounds__(kGeThreads)
geneig_batch_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  geneig_body(d.Ah, d.Bh, d.ncols, d.theta, d.C, d.geneig_info,
              &d.cs->status, d.clus);
}

// ------------------------------------------------------------------------
// Rotation U = W C with HU = (HW) C, MU = (MW) C, for the residual norms
// ||HU_i - theta_i MU_i||, ||MU_i|| (Step 4 output and the stopping test).
// H W and M W are read from the HU and MU buffers.  Rows of W, HW, MW are
// staged through LDS, so W may be the output itself and HU, MU are
// rewritten in place (each tile is read before it is written).
//
// Without emit, HU and MU are stored for the next step's start (its
// right-hand side and residual need M U and A_s U = HU - s MU).  With emit
// (the library's own step loops, where U, lambda and the operator reach
// the next step unchanged) the rotation writes that start state itself,
// from the same registers and with the same arithmetic and order as the
// start kernel: b = (theta - s) MU, r = b - (HU - s MU), p = D^-1 r, the
// CG iterate x0 = U (FP64: chunk-major Xc, R, P; mixed: the FP32 r, p, 0
// and the FP64 b), and the start's partials ||b||^2, r.z, ||r||^2 as
// quantities 2..4 (after the rotation's 0..1).  The next start then only
// resets the column state; HU and MU keep H W and M W.
// ------------------------------------------------------------------------
// The start state of one row (VR consecutive columns from col0) from the
// rotation's registers; acc[2..4] take ||b||^2, r.z, ||r||^2.  The CG
// vectors are chunk-major with the problem's widths (FP64 v64, FP32 v32).
template <int VR>
__device__ __forceinline__ void start_emit(const Desc& d, long long row,
                                           int col0, const double (&u)[VR],
                                           const double (&hu)[VR],
                                           const double (&mu)[VR],
                                           const double (&sh)[VR], double di,
                                           double (&acc)[5][VR]) {
  const size_t o = (size_t)row * d.ncols + col0;
  double b[VR], r[VR], p[VR];
#pragma unroll
  for (int v = 0; v < VR; ++v) {
    const double au = fma(-d.sigma, mu[v], hu[v]);
    b[v] = sh[v] * mu[v];
    r[v] = b[v] - au;
    p[v] = di * r[v];
    acc[2][v] += b[v] * b[v];
    acc[4][v] += r[v] * r[v];
  }
  constexpr int VS = VR < 2 ? VR : 2;  // store width (VR > 1: ncols even)
  if (d.R32) {
    float r32[VR], p32[VR];
#pragma unroll
    for (int v = 0; v < VR; ++v) {
      r32[v] = (float)r[v];
      p32[v] = (float)p[v];
      acc[3][v] += (double)r32[v] * (double)p32[v];
    }
#pragma unroll
    for (int j = 0; j < VR; j += VS) {
      const size_t o32 = cm_index(d.n, row, col0 + j, d.v32);
      float a[VS], c[VS], z[VS];
#pragma unroll
      for (int v = 0; v < VS; ++v) {
        a[v] = r32[j + v];
        c[v] = p32[j + v];
        z[v] = 0.0f;
      }
      stv<float, VS>(d.R32 + o32, a);
      stv<float, VS>(d.P32 + o32, c);
      stv<float, VS>(d.X32 + o32, z);
    }
  } else {
#pragma unroll
    for (int v = 0; v < VR; ++v) acc[3][v] += r[v] * p[v];
  }
  if (d.Xc) {
#pragma unroll
    for (int j = 0; j < VR; j += VS) {
      const size_t oc = cm_index(d.n, row, col0 + j, VS);
      double a[VS], c[VS], e[VS];
#pragma unroll
      for (int v = 0; v < VS; ++v) {
        a[v] = u[j + v];
        c[v] = r[j + v];
        e[v] = p[j + v];
      }
      stv<double, VS>(d.Xc + oc, a);
      stv<double, VS>(d.R + oc, c);
      stv<double, VS>(d.P + oc, e);
    }
  }
  if (d.rcm) {  // mixed, chunk-major refinement: x0 = U and b
#pragma unroll
    for (int j = 0; j < VR; j += VS) {
      const size_t oc = cm_index(d.n, row, col0 + j, VS);
      double a[VS], c[VS];
#pragma unroll
      for (int v = 0; v < VS; ++v) {
        a[v] = u[j + v];
        c[v] = b[j + v];
      }
      stv<double, VS>(d.Xm + oc, a);
      stv<double, VS>(d.B + oc, c);
    }
  } else if (d.B) {
    stv<double, VR>(d.B + o, b);
  }
}

// One virtual block of the rotation with VR columns per thread (4 where
// N_t allows: each LDS read of a row's W, HW, MW value then serves four
// columns).  red: LDS scratch for the partials (3 kBlock VR doubles).
template <int VR>
__device__ __forceinline__ void rotate_rows(const Desc& d, int vb) {
  const Geo g = geo_of<VR>(d, vb);
  const int ncols = d.ncols;
  // Thread (tile row lr, chunk ch) with the row fastest: a wavefront's
  // chunk-major stores of the emitted start run along contiguous rows
  // (the row-major U store is the one that scatters).
  const int lr = threadIdx.x % g.tr;
  const int ch = threadIdx.x / g.tr < g.cpr ? threadIdx.x / g.tr : g.cpr;
  const bool own = ch < g.cpr;
  const bool emit = d.emit != 0;
  const double* W = d.X;
  const double* HW = d.HU;
  const double* MW = d.MU;
  double* U = d.Uout;
  extern __shared__ unsigned char smem[];
  // Row stride ld = ncols | 1 (odd): the rows a wavefront reads at once
  // fall in different LDS banks.
  const int ld = ncols | 1;
  double* sC = reinterpret_cast<double*>(smem);        // ncols^2
  double* sW = sC + ncols * ncols;                     // tr * ld each
  double* sH = sW + g.tr * ld;
  double* sM = sH + g.tr * ld;
  double* red = sW;  // after the last tile
  const int tid = threadIdx.x;
  if (g.lb == 0 && tid == 0) {
    d.si->max_dlambda = 0.0;
    d.si->max_resid = 0.0;
  }
  for (int e = tid; e < ncols * ncols; e += kBlock) sC[e] = ldg(d.C + e);
  double th[VR], sh[VR];
#pragma unroll
  for (int v = 0; v < VR; ++v) {
    th[v] = d.theta[min(min(ch, g.cpr - 1) * VR + v, ncols - 1)];
    sh[v] = th[v] - d.sigma;
  }
  double acc[5][VR];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int v = 0; v < VR; ++v) acc[a][v] = 0.0;
  // A tile's rows of W, HW, MW are loaded into registers (KR values of
  // each per thread) one tile ahead: the loads of the next tile are in
  // flight while this one is computed (they precede this tile's stores,
  // which they never overlap, also when U is W).
  constexpr int KR = VR;  // tr * ncols <= kBlock * VR
  double rw[KR], rh[KR], rm[KR];
  auto fetch = [&](long long t) {
    const long long r0 = t * g.tr;
    const int cnt = (int)min((long long)g.tr, d.n - r0) * ncols;
    const size_t base = (size_t)r0 * ncols;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int e = tid + k * kBlock;
      const size_t o = base + (e < cnt ? e : 0);
      rw[k] = ldg(W + o);
      rh[k] = ldg(HW + o);
      rm[k] = ldg(MW + o);
    }
  };
  TileWalk w = tile_walk(g.ntiles, g.lb, g.nb);
  if (w.t < w.end) fetch(w.t);
  for (; w.t < w.end; w.t += w.step) {
    const long long r0 = w.t * g.tr;
    const int rows = (int)min((long long)g.tr, d.n - r0);
    __syncthreads();
    const size_t base = (size_t)r0 * ncols;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int e = tid + k * kBlock;
      if (e < rows * ncols) {
        const int o = e + (e / ncols) * (ld - ncols);
        sW[o] = rw[k];
        sH[o] = rh[k];
        sM[o] = rm[k];
      }
    }
    __syncthreads();
    if (w.t + w.step < w.end) fetch(w.t + w.step);
    if (own && lr < rows) {
      double u[VR], hu[VR], mu[VR];
#pragma unroll
      for (int v = 0; v < VR; ++v) u[v] = hu[v] = mu[v] = 0.0;
      const double* wr = sW + lr * ld;
      const double* hr = sH + lr * ld;
      const double* mr = sM + lr * ld;
      for (int k = 0; k < ncols; ++k) {
        const double wk = wr[k], hk = hr[k], mk = mr[k];
#pragma unroll
        for (int v = 0; v < VR; ++v) {
          const double c = sC[k * ncols + ch * VR + v];
          u[v] = fma(wk, c, u[v]);
          hu[v] = fma(hk, c, hu[v]);
          mu[v] = fma(mk, c, mu[v]);
        }
      }
      const long long row = r0 + lr;
      const size_t o = base + (size_t)lr * ncols + ch * VR;
      stv<double, VR>(U + o, u);
      if (emit) {
        start_emit<VR>(d, row, ch * VR, u, hu, mu, sh, ldg(d.dinv + row),
                       acc);
      } else {
        stv<double, VR>(d.HU + o, hu);  // for the next start
        stv<double, VR>(d.MU + o, mu);
      }
#pragma unroll
      for (int v = 0; v < VR; ++v) {
        const double r = hu[v] - th[v] * mu[v];
        acc[0][v] += r * r;
        acc[1][v] += mu[v] * mu[v];
      }
    }
  }
  __syncthreads();  // the tiles are consumed: red may reuse them
  double rot[2][VR], st[3][VR];
#pragma unroll
  for (int v = 0; v < VR; ++v) {
    rot[0][v] = acc[0][v];
    rot[1][v] = acc[1][v];
    st[0][v] = acc[2][v];
    st[1][v] = acc[3][v];
    st[2][v] = acc[4][v];
  }
  const int slot = own ? lr * g.cpr + ch : -1;
  block_partials_slot<2, VR>(rot, slot, ncols, g.cpr, g.tr, g.lb, g.nb,
                             d.part, red);
  if (emit)
    block_partials_slot<3, VR>(st, slot, ncols, g.cpr, g.tr, g.lb, g.nb,
                               d.part + 2 * kPartStride, red);
}

template <int V>
__device__ __forceinline__ void rotate_body(const Desc& d, int vb) {
  if constexpr (V == 2) {
    if (d.ncols % 4 == 0)
      rotate_rows<4>(d, vb);
    else
      rotate_rows<2>(d, vb);
  } else {
    rotate_rows<1>(d, vb);
  }
}

template <int VFIX>
__global__ void PARO_STREAM_BOUNDS
rotate_kernel(const Desc* __restrict__ D, int nprob) {
  PARO_VB_LOOP64(D, nprob, VFIX, (rotate_body<VV>(d, vb)))
}

// Per column: lambda = theta, relative change and residual; maxima over
// the requested pairs for the stopping test (grid: column x problem).
__global__ void __launch_bounds__(kFinal)
rotate_final_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.y];
  const int c = blockIdx.x;
  const int ncols = d.ncols;
  if (c >= ncols) return;
  double tot[2];
  column_sums<2>(d.part, kPartStride, c, d.ns, tot);
  if (threadIdx.x != 0) return;
  const double* theta = d.theta;
  double lmax = 0.0;
  for (int k = 0; k < ncols; ++k) lmax = fmax(lmax, fabs(theta[k]));
  const double t = theta[c];
  const double sc = fmax(fabs(t), 1e-3 * lmax);
  const double old = d.lam[c];
  const double dl = d.have_old ? fabs(t - old) / sc : INFINITY;
  double rho = sqrt(tot[0]) / (sc * sqrt(tot[1]));
  if (!isfinite(rho)) rho = INFINITY;
  StepInfo* si = d.si;
  si->lam_old[c] = old;
  si->dlam[c] = dl;
  si->resid[c] = rho;
  d.lam[c] = t;
  if (c < d.nreq) {
    atomic_max_nonneg(&si->max_dlambda, dl);
    atomic_max_nonneg(&si->max_resid, rho);
  }
}

// ------------------------------------------------------------------------
// General (bisection) meshes: the operator in CSR over the dofs, FP64.
// The vector kernels of the CG (r- and p-update) and of Rayleigh-Ritz are
// layout-free and serve these problems unchanged; only the products with
// A_s and M differ.
//
// CG SpMM: a unit is (segment of csr_rows consecutive rows, group of
// kCsrG consecutive chunks with an active column); thread tid takes rows
// r0 + tid, r0 + tid + kBlock, ... of the segment, reads each entry of its
// row once for the whole group, forms q = A_s p in column order for every
// live chunk of the group, stores q (chunk-major) and adds p_row q to its
// p.q partials; then one wavefront reduction and the four wavefronts in a
// fixed order give the (column, segment) partials, so the sums depend on
// the problem alone (not on the grouping, which only decides which
// columns a unit serves).
// ------------------------------------------------------------------------
constexpr int kCsrG = 4;

template <int V>
__device__ __forceinline__ void csr_cg_unit(const Desc& d, long long seg,
                                            int ch0, unsigned long long amask,
                                            double* __restrict__ ws) {
  const long long n = d.n;
  const long long r0 = seg * d.csr_rows;
  const long long r1 = min(n, r0 + d.csr_rows);
  const int cpr = d.ncols / V;
  const double* P = d.P;
  bool on[kCsrG];
  double acc[kCsrG][V];
#pragma unroll
  for (int g = 0; g < kCsrG; ++g) {
    on[g] = ch0 + g < cpr && chunk_in_mask<V>(amask, ch0 + g);
#pragma unroll
    for (int v = 0; v < V; ++v) acc[g][v] = 0.0;
  }
  for (long long r = r0 + threadIdx.x; r < r1; r += kBlock) {
    double q[kCsrG][V];
#pragma unroll
    for (int g = 0; g < kCsrG; ++g)
#pragma unroll
      for (int v = 0; v < V; ++v) q[g][v] = 0.0;
    const int j1 = ldg(d.rowptr + r + 1);
    for (int j = ldg(d.rowptr + r); j < j1; ++j) {
      const int c = ldg(d.colidx + j);
      const double a = ldg(d.valA + j);
#pragma unroll
      for (int g = 0; g < kCsrG; ++g) {
        if (!on[g]) continue;
        double x[V];
        ldv<double, V>(P + cm_index(n, c, (ch0 + g) * V, V), x);
#pragma unroll
        for (int v = 0; v < V; ++v) q[g][v] = fma(a, x[v], q[g][v]);
      }
    }
#pragma unroll
    for (int g = 0; g < kCsrG; ++g) {
      if (!on[g]) continue;
      const size_t o = cm_index(n, r, (ch0 + g) * V, V);
      double self[V];
      ldv<double, V>(P + o, self);
      stv<double, V>(d.Q + o, q[g]);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[g][v] += self[v] * q[g][v];
    }
  }
  constexpr int kGroup = 64 / V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < kCsrG; ++g) {
    if (!on[g]) continue;  // uniform over the block
    const double tot = wave_reduce_scatter<V>(acc[g]);
    if ((lane & (kGroup - 1)) == 0)
      ws[wave * kCsrG * V + g * V + lane / kGroup] = tot;
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k < kCsrG * V) {
    const int g = k / V, c = (ch0 + g) * V + k % V;
    if (on[g] && ((amask >> c) & 1)) {
      const int w = kCsrG * V;
      const double sum =
          ((ws[k] + ws[w + k]) + ws[2 * w + k]) + ws[3 * w + k];
      stg(d.pqp + (size_t)c * d.pqn + seg, sum);
    }
  }
  __syncthreads();  // ws is reused by the next unit
}

__global__ void PARO_STREAM_BOUNDS
csr_cg_spmm_kernel(const Desc* __restrict__ D, int nprob, int par) {
  __shared__ double ws[4 * kCsrG * 2];
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (!d.csr) return;
  const int nact = ldg(&d.cs->n_active[par]);
  const unsigned long long amask = active_mask(d.cs->act[par], d.ncols);
  if (nact == 0) return;  // queued after convergence
  const int lb = blockIdx.x - d.b0;
  const int V = d.v64;
  const int cpr = d.ncols / V;
  // Groups of kCsrG chunks with an active column.
  const unsigned long long cm = chunk_mask(amask, cpr, V);
  unsigned long long gm = 0;
  for (int g = 0; g * kCsrG < cpr; ++g)
    if ((cm >> (g * kCsrG)) & ((1ull << kCsrG) - 1)) gm |= 1ull << g;
  const int nag = __popcll(gm);
  for (TileWalk w = tile_walk((long long)d.pqn * nag, lb, d.nb); w.t < w.end;
       w.t += w.step) {
    const long long seg = w.t / nag;
    const int gi = (int)(w.t - seg * nag);
    unsigned long long m = gm;
    for (int k = 0; k < gi; ++k) m &= m - 1;
    const int ch0 = __builtin_ctzll(m) * kCsrG;
    if (V == 2)
      csr_cg_unit<2>(d, seg, ch0, amask, ws);
    else
      csr_cg_unit<1>(d, seg, ch0, amask, ws);
  }
}

// Row-major products of the CSR problems, one thread per (row, chunk of V
// columns): mode 0 Y1 = A X + s1 M X, Y2 = M X (component form; either
// output may be absent); mode 1 HU = H X, MU = M X (Rayleigh-Ritz: H =
// A_s + s M; over the last rotation's H U, M U); mode 2 HU = H U0,
// MU = M U0 for the problems whose start
// cannot take them from a rotation (use_hu = 2: formed here, then read by
// the start like a rotation's).
template <int V>
__device__ __forceinline__ void csr_dual_rows(const Desc& d, int mode,
                                              int lb) {
  const double* X = mode == 2 ? d.U0 : d.X;
  double* Y1 = mode == 0 ? d.Y1 : d.HU;
  double* Y2 = mode == 0 ? d.Y2 : d.MU;
  const double s1 = mode == 0 ? d.s1 : d.sigma;
  const bool needA = Y1 != nullptr;
  const int ncols = d.ncols, cpr = ncols / V;
  const long long total = d.n * cpr;
  for (long long t = (long long)lb * kBlock + threadIdx.x; t < total;
       t += (long long)d.nb * kBlock) {
    const long long r = t / cpr;
    const int ch = (int)(t - r * cpr);
    double ax[V], mx[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ax[v] = mx[v] = 0.0;
    const int j1 = ldg(d.rowptr + r + 1);
    for (int j = ldg(d.rowptr + r); j < j1; ++j) {
      const int c = ldg(d.colidx + j);
      const double a = needA ? ldg(d.valA + j) : 0.0;
      const double m = ldg(d.valM + j);
      double x[V];
      ldv<double, V>(X + (size_t)c * ncols + ch * V, x);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        ax[v] = fma(a, x[v], ax[v]);
        mx[v] = fma(m, x[v], mx[v]);
      }
    }
    const size_t o = (size_t)r * ncols + ch * V;
    if (Y1) {
      double y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = fma(s1, mx[v], ax[v]);
      stv<double, V>(Y1 + o, y);
    }
    if (Y2) stv<double, V>(Y2 + o, mx);
  }
}

__global__ void PARO_STREAM_BOUNDS
csr_dual_kernel(const Desc* __restrict__ D, int nprob, int mode) {
  const Desc& d = D[owner(D, nprob, blockIdx.x, false)];
  if (!d.csr) return;
  if (mode == 2 && d.use_hu != 2) return;  // its start needs no H U0, M U0
  const int lb = blockIdx.x - d.b0;
  if (d.v64 == 2)
    csr_dual_rows<2>(d, mode, lb);
  else
    csr_dual_rows<1>(d, mode, lb);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// Launch a kernel; with timing on, the start and stop events are taken by
// the dispatch itself (kernel execution only, no launch gaps) and the
// duration is added to `stage`.
template <typename F, typename... Args>
static void klaunch(Timing* t, int stage, F kernel, dim3 grid, dim3 block,
                    size_t smem, hipStream_t s, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (timing_pair(t, &a, &b)) {
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)smem, s, a, b,
                          0, args...);
    timing_add(t, stage, a, b);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, smem, s, args...);
  }
}

// Launch KERNEL<W> with W the launch's common FP64 vector width, or
// W = 0 (per-block branch) when the problems differ.
#define PARO_LAUNCH_W64(W, T, ST, KERNEL, ...)                         \
  switch (W) {                                                         \
    case 2:                                                            \
      klaunch(T, ST, KERNEL<2>, __VA_ARGS__);                          \
      break;                                                           \
    case 1:                                                            \
      klaunch(T, ST, KERNEL<1>, __VA_ARGS__);                          \
      break;                                                           \
    default:                                                           \
      klaunch(T, ST, KERNEL<0>, __VA_ARGS__);                          \
  }

template <int W>
static void spmm_dual_w(Launch& L, bool rr, hipStream_t s, Timing* t) {
  const size_t smem = weights_bytes(L.tr64, sizeof(double), 2);
  if (L.maxkz)
    klaunch(t, PARO_ST_RR_SPMM, spmm_dual_kernel<W, true>, dim3(L.blocks),
            dim3(kBlock), smem, s, (const Desc*)L.d, L.nprob, rr ? 1 : 0);
  else
    klaunch(t, PARO_ST_RR_SPMM, spmm_dual_kernel<W, false>, dim3(L.blocks),
            dim3(kBlock), smem, s, (const Desc*)L.d, L.nprob, rr ? 1 : 0);
}

hipError_t launch_spmm(Launch& L, bool rr, hipStream_t s, Timing* t) {
  switch (L.v64u) {
    case 2: spmm_dual_w<2>(L, rr, s, t); break;
    case 1: spmm_dual_w<1>(L, rr, s, t); break;
    default: spmm_dual_w<0>(L, rr, s, t);
  }
  if (L.csr) return launch_csr_dual(L, rr ? 1 : 0, s, t);
  return hipGetLastError();
}

hipError_t launch_csr_dual(Launch& L, int mode, hipStream_t s, Timing* t) {
  klaunch(t, mode == 2 ? PARO_ST_START : PARO_ST_RR_SPMM, csr_dual_kernel,
          dim3(L.blocks), dim3(kBlock), 0, s, (const Desc*)L.d, L.nprob,
          mode);
  return hipGetLastError();
}

hipError_t launch_csr_cg_spmm(Launch& L, int par, hipStream_t s, Timing* t) {
  klaunch(t, PARO_ST_CG_SPMM, csr_cg_spmm_kernel, dim3(L.blocks),
          dim3(kBlock), 0, s, (const Desc*)L.d, L.nprob, par);
  return hipGetLastError();
}

// Y = Z^T (source) for every problem with a nonlocal term.
static void zt_launch(Launch& L, int src, hipStream_t s, Timing* t, int st,
                      int par = 0) {
  const Desc* D = L.d;
  const dim3 g(L.blocks), b(kBlock);
  const int n = L.nprob;
  if (L.maxkz <= 1) klaunch(t, st, zt_partial_kernel<1>, g, b, 0, s, D, n, src, par);
  else if (L.maxkz <= 2) klaunch(t, st, zt_partial_kernel<2>, g, b, 0, s, D, n, src, par);
  else if (L.maxkz <= 4) klaunch(t, st, zt_partial_kernel<4>, g, b, 0, s, D, n, src, par);
  else if (L.maxkz <= 8) klaunch(t, st, zt_partial_kernel<8>, g, b, 0, s, D, n, src, par);
  else if (L.maxkz <= 16) klaunch(t, st, zt_partial_kernel<16>, g, b, 0, s, D, n, src, par);
  else klaunch(t, st, zt_partial_kernel<32>, g, b, 0, s, D, n, src, par);
  klaunch(t, st, zt_final_kernel, dim3(L.maxkz * L.maxcols, L.nprob),
          dim3(kFinal), 0, s, (const Desc*)L.d);
}

hipError_t launch_nl_mass(const Desc& d, const double* zeta, double* Z,
                          int k, hipStream_t s) {
  const long long total = d.n * k;
  const int grid = (int)std::min<long long>((total + kBlock - 1) / kBlock,
                                            4096);
  hipLaunchKernelGGL(nl_mass_kernel, dim3(grid), dim3(kBlock), 0, s, d, zeta,
                     Z, k);
  return hipGetLastError();
}

hipError_t launch_pcg_start(Launch& L, hipStream_t s, Timing* t) {
  if (L.maxkz) zt_launch(L, kZtU0, s, t, PARO_ST_START);
  PARO_LAUNCH_W64(L.v64u, t, PARO_ST_START, pcg_start_kernel, dim3(L.blocks),
                  dim3(kBlock), weights_bytes(L.tr64, sizeof(double), 2), s,
                  L.d, L.nprob);
  klaunch(t, PARO_ST_START, pcg_start_final_kernel, dim3(L.maxcols, L.nprob),
          dim3(kFinal), 0, s, L.d);
  return hipGetLastError();
}

// One CG iteration of every problem of the table (chunk-major kernels).
template <typename T, int W>
static void cg_spmm_launch(Launch& L, int par, hipStream_t s, Timing* t) {
  const Desc* D = L.d;
  if constexpr (sizeof(T) == 8)
    if (L.csr) (void)launch_csr_cg_spmm(L, par, s, t);
  if (L.ntile) {
    if (L.seg)
      klaunch(t, PARO_ST_CG_SPMM, spmm_cm_kernel<T, W, true>, dim3(L.blocks),
              dim3(kBlock), 0, s, D, L.nprob, par);
    else
      klaunch(t, PARO_ST_CG_SPMM, spmm_cm_kernel<T, W, false>,
              dim3(L.blocks), dim3(kBlock), 0, s, D, L.nprob, par);
  }
  if (L.zm && L.zmf) {
    klaunch(t, PARO_ST_CG_SPMM, spmm_zmf_kernel<T, W>, dim3(L.blocks),
            dim3(kBlock), 0, s, D, L.nprob, par);
    return;
  }
  if (L.zm) {
    switch (L.zmg) {
      case 1:
        klaunch(t, PARO_ST_CG_SPMM, spmm_zm_kernel<T, W, 1>, dim3(L.blocks),
                dim3(kBlock), 0, s, D, L.nprob, par);
        break;
      case 4:
        klaunch(t, PARO_ST_CG_SPMM, spmm_zm_kernel<T, W, 4>, dim3(L.blocks),
                dim3(kBlock), 0, s, D, L.nprob, par);
        break;
      default:
        klaunch(t, PARO_ST_CG_SPMM, spmm_zm_kernel<T, W, 2>, dim3(L.blocks),
                dim3(kBlock), 0, s, D, L.nprob, par);
    }
  }
}

template <typename T, int W>
static void cg_iter_w(Launch& L, int par, hipStream_t s, Timing* t) {
  const Desc* D = L.d;
  if constexpr (sizeof(T) == 8)
    if (L.maxkz) zt_launch(L, kZtP, s, t, PARO_ST_CG_SPMM, par);
  cg_spmm_launch<T, W>(L, par, s, t);
  klaunch(t, PARO_ST_CG_RUPD, rupd_alpha_kernel<T, W>, dim3(L.blocks),
          dim3(kBlock), 0, s, D, L.nprob, par);
  klaunch(t, PARO_ST_CG_PUPD, pupd_beta_kernel<T, W>, dim3(L.blocks),
          dim3(kBlock), 0, s, D, L.nprob, par);
}

hipError_t launch_pcg_iter(Launch& L, bool fp32, int par, hipStream_t s,
                           Timing* t) {
  if (fp32) {
    switch (L.v32u) {
      case 4: cg_iter_w<float, 4>(L, par, s, t); break;
      case 2: cg_iter_w<float, 2>(L, par, s, t); break;
      case 1: cg_iter_w<float, 1>(L, par, s, t); break;
      default: cg_iter_w<float, 0>(L, par, s, t);
    }
  } else {
    switch (L.v64u) {
      case 2: cg_iter_w<double, 2>(L, par, s, t); break;
      case 1: cg_iter_w<double, 1>(L, par, s, t); break;
      default: cg_iter_w<double, 0>(L, par, s, t);
    }
  }
  return hipGetLastError();
}

// The CG SpMM alone (autotuner timing).
hipError_t launch_cg_spmm(Launch& L, bool fp32, hipStream_t s) {
  if (fp32) {
    switch (L.v32u) {
      case 4: cg_spmm_launch<float, 4>(L, 0, s, nullptr); break;
      case 2: cg_spmm_launch<float, 2>(L, 0, s, nullptr); break;
      case 1: cg_spmm_launch<float, 1>(L, 0, s, nullptr); break;
      default: cg_spmm_launch<float, 0>(L, 0, s, nullptr);
    }
  } else {
    switch (L.v64u) {
      case 2: cg_spmm_launch<double, 2>(L, 0, s, nullptr); break;
      case 1: cg_spmm_launch<double, 1>(L, 0, s, nullptr); break;
      default: cg_spmm_launch<double, 0>(L, 0, s, nullptr);
    }
  }
  return hipGetLastError();
}

// Persistent CG launch; *fits = false (nothing launched) when the grid
// cannot be co-resident.
template <typename T, int W>
static hipError_t cg_persistent_w(Launch& L, int iters, hipStream_t s,
                                  Timing* t, bool* fits) {
  // Co-resident capacity of this kernel on the current device.
  int per_cu = 0, cus = 0, dev = 0;
  hipError_t e0 = hipGetDevice(&dev);
  if (e0 == hipSuccess)
    e0 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                               dev);
  if (e0 == hipSuccess)
    e0 = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(cg_persistent_kernel<T, W>),
        kBlock, 0);
  if (e0 != hipSuccess) return e0;
  *fits = (long long)per_cu * cus >= L.blocks;
  if (!*fits) return hipSuccess;
  const Desc* D = L.d;
  int nprob = L.nprob;
  void* args[] = {(void*)&D, (void*)&nprob, (void*)&iters};
  hipEvent_t a = nullptr, b = nullptr;
  const bool timed = timing_pair(t, &a, &b);
  if (timed) (void)hipEventRecord(a, s);
  const hipError_t e = hipLaunchCooperativeKernel(
      reinterpret_cast<const void*>(cg_persistent_kernel<T, W>),
      dim3(L.blocks), dim3(kBlock), args, 0, s);
  if (timed) {
    (void)hipEventRecord(b, s);
    timing_add(t, PARO_ST_CG_SPMM, a, b);
  }
  return e;
}

hipError_t launch_cg_persistent(Launch& L, bool fp32, int iters,
                                hipStream_t s, Timing* t, bool* fits) {
  if (fp32) {
    switch (L.v32u) {
      case 4: return cg_persistent_w<float, 4>(L, iters, s, t, fits);
      case 2: return cg_persistent_w<float, 2>(L, iters, s, t, fits);
      case 1: return cg_persistent_w<float, 1>(L, iters, s, t, fits);
      default: return cg_persistent_w<float, 0>(L, iters, s, t, fits);
    }
  }
  switch (L.v64u) {
    case 2: return cg_persistent_w<double, 2>(L, iters, s, t, fits);
    case 1: return cg_persistent_w<double, 1>(L, iters, s, t, fits);
    default: return cg_persistent_w<double, 0>(L, iters, s, t, fits);
  }
}

hipError_t launch_cm_unpack(Launch& L, hipStream_t s, Timing* t) {
  PARO_LAUNCH_W64(L.v64u, t, PARO_ST_REFINE, cm_unpack_kernel, dim3(L.blocks),
                  dim3(kBlock), 0, s, L.d, L.nprob);
  return hipGetLastError();
}

// Every column of every problem active in parity 0 (autotuner set-up; the
// next source-solve start resets the column state).
__global__ void __launch_bounds__(kFinal)
all_active_kernel(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  for (int c = threadIdx.x; c < d.ncols; c += kFinal) d.cs->act[0][c] = 1;
  if (threadIdx.x == 0) d.cs->n_active[0] = d.ncols;
}

hipError_t launch_all_active(Launch& L, hipStream_t s) {
  hipLaunchKernelGGL(all_active_kernel, dim3(L.nprob), dim3(kFinal), 0, s,
                     (const Desc*)L.d);
  return hipGetLastError();
}

hipError_t launch_refine_residual(Launch& L, hipStream_t s, Timing* t) {
  PARO_LAUNCH_W64(L.v64u, t, PARO_ST_REFINE, refine_residual_kernel,
                  dim3(L.blocks), dim3(kBlock),
                  weights_bytes(L.tr64, sizeof(double), 1), s, L.d, L.nprob);
  if (L.zm)  // problems with a chunk-major refinement iterate
    PARO_LAUNCH_W64(L.v64u, t, PARO_ST_REFINE, refine_residual_zm_kernel,
                    dim3(L.blocks), dim3(kBlock), 0, s, L.d, L.nprob, L.zmf);
  klaunch(t, PARO_ST_REFINE, refine_final_kernel, dim3(L.maxcols, L.nprob),
          dim3(kFinal), 0, s, L.d);
  return hipGetLastError();
}

hipError_t launch_redirect(Launch& L, hipStream_t s, Timing* t) {
  const Desc* D = L.d;
  switch (L.v32u) {
    case 4: klaunch(t, PARO_ST_REFINE, redirect_cm_kernel<4>, dim3(L.blocks), dim3(kBlock), 0, s, D, L.nprob); break;
    case 2: klaunch(t, PARO_ST_REFINE, redirect_cm_kernel<2>, dim3(L.blocks), dim3(kBlock), 0, s, D, L.nprob); break;
    case 1: klaunch(t, PARO_ST_REFINE, redirect_cm_kernel<1>, dim3(L.blocks), dim3(kBlock), 0, s, D, L.nprob); break;
    default: klaunch(t, PARO_ST_REFINE, redirect_cm_kernel<0>, dim3(L.blocks), dim3(kBlock), 0, s, D, L.nprob);
  }
  return hipGetLastError();
}

hipError_t launch_refine_update(Launch& L, hipStream_t s, Timing* t) {
  PARO_LAUNCH_W64(L.v64u, t, PARO_ST_REFINE, refine_update_kernel,
                  dim3(L.blocks), dim3(kBlock), 0, s, L.d, L.nprob);
  return hipGetLastError();
}

hipError_t launch_gather_reports(Launch& L, PollReport* out, int* seqp,
                                 int seq, hipStream_t s) {
  hipLaunchKernelGGL(gather_reports_kernel, dim3(1), dim3(kBlock), 0, s, L.d,
                     L.nprob, out, seqp, seq);
  return hipGetLastError();
}

hipError_t launch_count_active(Launch& L, int which, int* out, int seq,
                               hipStream_t s) {
  hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(kBlock), 0, s, L.d,
                     L.nprob, which, out, seq);
  return hipGetLastError();
}

template <bool SYM, bool MIXED>
static void gram_first_m(Launch& L, hipStream_t s, Timing* t) {
  const Desc* D = L.d;
  switch (L.nt16) {
    case 1:
      klaunch(t, PARO_ST_GRAM, gram_kernel<1, SYM, MIXED>, dim3(L.gblocks),
              dim3(kBlock), 0, s, D, L.nprob);
      break;
    case 2:
      klaunch(t, PARO_ST_GRAM, gram_kernel<2, SYM, MIXED>, dim3(L.gblocks),
              dim3(kBlock), 0, s, D, L.nprob);
      break;
    case 3:
      klaunch(t, PARO_ST_GRAM, gram_kernel<3, SYM, MIXED>, dim3(L.gblocks),
              dim3(kBlock), 0, s, D, L.nprob);
      break;
    default:
      klaunch(t, PARO_ST_GRAM, gram_kernel<4, SYM, MIXED>, dim3(L.gblocks),
              dim3(kBlock), 0, s, D, L.nprob);
  }
}

template <bool SYM>
static void gram_first(Launch& L, hipStream_t s, Timing* t) {
  if (L.nt16_mixed)
    gram_first_m<SYM, true>(L, s, t);
  else
    gram_first_m<SYM, false>(L, s, t);
}

static hipError_t gram(Launch& L, bool sym, hipStream_t s, Timing* t) {
  if (sym)
    gram_first<true>(L, s, t);
  else
    gram_first<false>(L, s, t);
  klaunch(t, PARO_ST_GRAM, gram_final_kernel,
          dim3((L.maxcols * L.maxcols + 3) / 4, L.nprob), dim3(kBlock), 0, s,
          (const Desc*)L.d, sym ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gram_full(Launch& L, hipStream_t s, Timing* t) {
  return gram(L, false, s, t);
}

hipError_t launch_small_geneig(const double* A, const double* B, int n,
                               double* theta, double* C, int* info,
                               hipStream_t s) {
  hipLaunchKernelGGL(small_geneig_kernel, dim3(1), dim3(kGeThreads), 0, s, A, B, n,
                     theta, C, info);
  return hipGetLastError();
}

hipError_t launch_rayleigh_ritz(Launch& L, hipStream_t s, Timing* t) {
  hipError_t e;
  if (L.maxkz) zt_launch(L, kZtX, s, t, PARO_ST_RR_SPMM);  // Z^T W
  if ((e = launch_spmm(L, true, s, t)) != hipSuccess) return e;
  if ((e = gram(L, true, s, t)) != hipSuccess) return e;
  klaunch(t, PARO_ST_SMALL, geneig_batch_kernel, dim3(L.nprob), dim3(kGeThreads),
          0, s, (const Desc*)L.d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // Rotation: C (ncols^2) plus three row tiles of tr rows at stride
  // ncols | 1, tr * ncols <= kBlock * 4 values and tr <= kBlock each (the
  // tiles also hold the partials' scratch of 3 kBlock 4 doubles).
  const size_t smem = sizeof(double) * ((size_t)L.maxcols * L.maxcols +
                                        3 * (size_t)kBlock * 5);
  PARO_LAUNCH_W64(L.v64u, t, PARO_ST_ROTATE, rotate_kernel, dim3(L.blocks),
                  dim3(kBlock), smem, s, L.d, L.nprob);
  klaunch(t, PARO_ST_ROTATE, rotate_final_kernel, dim3(L.maxcols, L.nprob),
          dim3(kFinal), 0, s, (const Desc*)L.d);
  return hipGetLastError();
}

}  // namespace paro
