// Step 2 of Algorithm 3.1 on the uniform Kuhn mesh (Sec. 2, adaptive
// finite element approximation): the residual a posteriori estimator of
// the requested orbitals per element, Doerfler and maximum marking (eqs.
// (dorfler-strategy), (maximum-strategy)), and the transfer of orbitals to
// the mesh refined everywhere (twice the cells per axis, which refines
// every Kuhn element into Kuhn elements of half the size).
//
// Elements: cell c = (ci, cj, ck) of the nx x ny x nz cells (x fastest)
// holds the six Kuhn elements q = 0..5, one per permutation p of the axes
// in lexicographic order, with vertices v0 = c, v1 = v0 + e_p0,
// v2 = v1 + e_p1, v3 = v0 + (1, 1, 1); element index q * ncells + c.  The
// element across the face opposite v_k is, in cell coordinates:
//   k = 0: cell c + e_p0, permutation (p1, p2, p0);
//   k = 1: cell c, (p1, p0, p2);   k = 2: cell c, (p0, p2, p1);
//   k = 3: cell c - e_p2, (p2, p0, p1);
// a face whose neighbour cell lies outside the box is on the boundary.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "paro_internal.h"

namespace paro {
namespace {

// Axis permutations in lexicographic order.
__constant__ int kPerm6[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                 {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

__device__ __forceinline__ int perm_index(int a, int b) {
  // The permutation starting (a, b).
  return 2 * a + ((b == (a == 0 ? 1 : 0)) ? 0 : 1);
}

struct Grid3 {
  int nx, ny, nz;       // cells
  double lo[3], h[3];
};

// Value of orbital column i at vertex (I, J, K): 0 on the box boundary,
// else the dof's row of the row-major n x ncols block U.
__device__ __forceinline__ double vertex_u(const double* __restrict__ U,
                                           const Grid3& g, int ncols, int i,
                                           int I, int J, int K) {
  if (I <= 0 || J <= 0 || K <= 0 || I >= g.nx || J >= g.ny || K >= g.nz)
    return 0.0;
  const long long d =
      (I - 1) + (long long)(g.nx - 1) * ((J - 1) + (long long)(g.ny - 1) * (K - 1));
  return U[(size_t)d * ncols + i];
}

__device__ __forceinline__ double vertex_v(const double* __restrict__ V,
                                           const Grid3& g, int I, int J,
                                           int K) {
  return V[(size_t)I + (size_t)(g.nx + 1) * (J + (size_t)(g.ny + 1) * K)];
}

// The four vertices (integer vertex coordinates) of Kuhn element (cell, q).
__device__ __forceinline__ void kuhn_vertices(int ci, int cj, int ck, int q,
                                              int (&v)[4][3]) {
  const int p0 = kPerm6[q][0], p1 = kPerm6[q][1];
  v[0][0] = ci;
  v[0][1] = cj;
  v[0][2] = ck;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    v[1][a] = v[0][a] + (a == p0);
    v[2][a] = v[1][a] + (a == p1);
    v[3][a] = v[0][a] + 1;
  }
}

// Gradient of the P1 interpolant of values u0..u3 at the vertices of the
// Kuhn element with permutation q: along axis p_k it is
// (u_{k+1} - u_k) / h_{p_k}.
__device__ __forceinline__ void kuhn_grad(const double (&u)[4], int q,
                                          const double (&h)[3],
                                          double (&g)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) g[kPerm6[q][k]] = (u[k + 1] - u[k]) / h[kPerm6[q][k]];
}

// int_T phi_a phi_b phi_c phi_d / |T| = 3! prod k! / 7!, as a function of
// the multiplicities of a, b, c, d.
__device__ __forceinline__ double quartic(int a, int b, int c, int d) {
  int k[4] = {0, 0, 0, 0};
  ++k[a];
  ++k[b];
  ++k[c];
  ++k[d];
  const int f[5] = {1, 1, 2, 6, 24};
  return 6.0 * f[k[0]] * f[k[1]] * f[k[2]] * f[k[3]] / 5040.0;
}

// eta_T^2 = sum_i h_T^2 ||lambda_i u_i - V_h u_i||^2_T
//           + 1/2 sum_{F interior} h_F ||[1/2 grad u_i . n_F]||^2_F,
// one thread per (element, orbital i < NP), NP a power of two >= nreq
// dividing 64; the NP lanes of an element add their orbitals' shares in
// a fixed butterfly.
__global__ void __launch_bounds__(kBlock)
estimate_kernel(Grid3 g, const double* __restrict__ V,
                const double* __restrict__ lam, const double* __restrict__ U,
                int ncols, int nreq, int NP, long long nelem,
                double* __restrict__ eta) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long e = t / NP;
  const int i = (int)(t % NP);
  double s = 0.0;
  if (e < nelem && i < nreq) {
    const long long ncell = (long long)g.nx * g.ny * g.nz;
    const int q = (int)(e / ncell);
    const long long c = e - q * ncell;
    const int ci = (int)(c % g.nx);
    const int cj = (int)((c / g.nx) % g.ny);
    const int ck = (int)(c / ((long long)g.nx * g.ny));
    int v[4][3];
    kuhn_vertices(ci, cj, ck, q, v);
    double u[4], vv[4], X[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      u[a] = vertex_u(U, g, ncols, i, v[a][0], v[a][1], v[a][2]);
      vv[a] = vertex_v(V, g, v[a][0], v[a][1], v[a][2]);
#pragma unroll
      for (int x = 0; x < 3; ++x) X[a][x] = g.lo[x] + g.h[x] * v[a][x];
    }
    const double h[3] = {g.h[0], g.h[1], g.h[2]};
    const double vol = h[0] * h[1] * h[2] / 6.0;
    double hT2 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a + 1; b < 4; ++b) {
        double l2 = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x)
          l2 += (X[a][x] - X[b][x]) * (X[a][x] - X[b][x]);
        hT2 = fmax(hT2, l2);
      }
    // Element residual as the quadratic form R_ab phi_a phi_b.
    const double l = lam[i];
    double R[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        R[a][b] = 0.5 * l * (u[a] + u[b]) - 0.5 * (vv[a] * u[b] + vv[b] * u[a]);
    double r2 = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int cc = 0; cc < 4; ++cc)
#pragma unroll
          for (int d = 0; d < 4; ++d)
            r2 += R[a][b] * R[cc][d] * quartic(a, b, cc, d);
    s = hT2 * vol * r2;
    // Face jumps.
    double gT[3];
    kuhn_grad(u, q, h, gT);
    const int p0 = kPerm6[q][0], p1 = kPerm6[q][1], p2 = kPerm6[q][2];
    for (int k = 0; k < 4; ++k) {
      int nc3[3] = {ci, cj, ck}, nq;
      if (k == 0) {
        nc3[p0] += 1;
        nq = perm_index(p1, p2);
      } else if (k == 1) {
        nq = perm_index(p1, p0);
      } else if (k == 2) {
        nq = perm_index(p0, p2);
      } else {
        nc3[p2] -= 1;
        nq = perm_index(p2, p0);
      }
      if (nc3[0] < 0 || nc3[1] < 0 || nc3[2] < 0 || nc3[0] >= g.nx ||
          nc3[1] >= g.ny || nc3[2] >= g.nz)
        continue;  // boundary face
      int w[4][3];
      kuhn_vertices(nc3[0], nc3[1], nc3[2], nq, w);
      double un[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        un[a] = vertex_u(U, g, ncols, i, w[a][0], w[a][1], w[a][2]);
      double gN[3];
      kuhn_grad(un, nq, h, gN);
      // The face: the three vertices other than v_k.
      double F[3][3];
      int m = 0;
      for (int a = 0; a < 4; ++a) {
        if (a == k) continue;
#pragma unroll
        for (int x = 0; x < 3; ++x) F[m][x] = X[a][x];
        ++m;
      }
      const double e1[3] = {F[1][0] - F[0][0], F[1][1] - F[0][1],
                            F[1][2] - F[0][2]};
      const double e2[3] = {F[2][0] - F[0][0], F[2][1] - F[0][1],
                            F[2][2] - F[0][2]};
      const double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                             e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
      const double nn = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] +
                             nrm[2] * nrm[2]);
      const double area = 0.5 * nn;
      double hF2 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
          double l2 = 0.0;
#pragma unroll
          for (int x = 0; x < 3; ++x)
            l2 += (F[a][x] - F[b][x]) * (F[a][x] - F[b][x]);
          hF2 = fmax(hF2, l2);
        }
      double j = 0.0;
#pragma unroll
      for (int x = 0; x < 3; ++x) j += (gT[x] - gN[x]) * nrm[x];
      j = 0.5 * j / nn;
      s += 0.5 * sqrt(hF2) * area * j * j;
    }
  }
  for (int o = NP / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, NP);
  if (e < nelem && i == 0) eta[e] = sqrt(s);
}

// ---- marking ------------------------------------------------------------
// Thresholds act on eta itself: for non-negative doubles the order of the
// values is the order of their bit patterns, so the Doerfler threshold is
// found by bisection over bit patterns and every comparison is exact.
constexpr int kMarkGrid = 512;

// Block b of the fixed grid owns elements [b chunk, (b + 1) chunk).
__device__ __forceinline__ void mark_range(long long n, long long& k0,
                                           long long& k1) {
  const long long chunk = (n + kMarkGrid - 1) / kMarkGrid;
  k0 = (long long)blockIdx.x * chunk;
  k1 = k0 + chunk < n ? k0 + chunk : n;
}

// Per block: sum of eta^2 over eta >= t (mode 0) or eta > t (mode 1), the
// number of such elements, and the largest eta.
__global__ void __launch_bounds__(kBlock)
mark_partial_kernel(const double* __restrict__ eta, long long n, double t,
                    int strict, double* __restrict__ psum,
                    double* __restrict__ pmax,
                    long long* __restrict__ pcnt) {
  __shared__ double ss[kBlock], sm[kBlock];
  __shared__ long long sc[kBlock];
  long long k0, k1;
  mark_range(n, k0, k1);
  double s = 0.0, mx = 0.0;
  long long c = 0;
  for (long long k = k0 + threadIdx.x; k < k1; k += kBlock) {
    const double e = eta[k];
    const bool in = strict ? e > t : e >= t;
    s += in ? e * e : 0.0;
    c += in ? 1 : 0;
    mx = fmax(mx, e);
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    psum[blockIdx.x] = ss[0];
    pmax[blockIdx.x] = sm[0];
    pcnt[blockIdx.x] = sc[0];
  }
}

// out[0] = sum (fixed order), out[1] = max, out[2] = count (as double).
__global__ void __launch_bounds__(kBlock)
mark_final_kernel(const double* __restrict__ psum,
                  const double* __restrict__ pmax,
                  const long long* __restrict__ pcnt,
                  double* __restrict__ out) {
  __shared__ double ss[kBlock], sm[kBlock];
  __shared__ long long sc[kBlock];
  double s = 0.0, mx = 0.0;
  long long c = 0;
  for (int k = threadIdx.x; k < kMarkGrid; k += kBlock) {
    s += psum[k];
    mx = fmax(mx, pmax[k]);
    c += pcnt[k];
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mx;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ss[0];
    out[1] = sm[0];
    out[2] = (double)sc[0];
  }
}

// Elements with eta == t in each block's range (for the tie ranks).
__global__ void __launch_bounds__(kBlock)
mark_ties_count_kernel(const double* __restrict__ eta, long long n, double t,
                       long long* __restrict__ pcnt) {
  __shared__ long long sc[kBlock];
  long long k0, k1;
  mark_range(n, k0, k1);
  long long c = 0;
  for (long long k = k0 + threadIdx.x; k < k1; k += kBlock)
    c += eta[k] == t ? 1 : 0;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sc[threadIdx.x] += sc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) pcnt[blockIdx.x] = sc[0];
}

// marked[k] = eta_k >= t (strict 0) or eta_k > t (strict 1); with
// ties > 0 also the elements with eta == t whose rank in index order is
// below `ties` (tie_base[b]: ties in the ranges of blocks before b).
__global__ void __launch_bounds__(kBlock)
mark_set_kernel(const double* __restrict__ eta, long long n, double t,
                int strict, long long ties,
                const long long* __restrict__ tie_base,
                unsigned char* __restrict__ marked) {
  __shared__ long long wsum[kBlock / 64 + 1];
  long long k0, k1;
  mark_range(n, k0, k1);
  long long base = ties > 0 ? tie_base[blockIdx.x] : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (long long c0 = k0; c0 < k1; c0 += kBlock) {
    const long long k = c0 + threadIdx.x;
    const bool ok = k < k1;
    const double e = ok ? eta[k] : 0.0;
    unsigned char m = ok && (strict ? e > t : e >= t) ? 1 : 0;
    if (ties > 0) {
      const bool tie = ok && e == t;
      const unsigned long long b = __ballot(tie);
      if (lane == 0) wsum[wave] = __popcll(b);
      __syncthreads();
      long long before = base;
      for (int w = 0; w < wave; ++w) before += wsum[w];
      before += __popcll(b & ((1ull << lane) - 1));
      if (tie && before < ties) m = 1;
      long long tot = 0;
      for (int w = 0; w < kBlock / 64; ++w) tot += wsum[w];
      __syncthreads();
      base += tot;
    }
    if (ok) marked[k] = m;
  }
}

// ---- transfer -----------------------------------------------------------
// Fine vertex (I, J, K) of the grid with twice the cells: the midpoint of
// the coarse edge from (I, J, K) / 2 (rounded down) along the parities
// (I, J, K) mod 2 -- an axis, face-diagonal or main-diagonal edge of the
// Kuhn mesh -- so its P1 value is the mean of that edge's end values.
__global__ void __launch_bounds__(kBlock)
prolong_kernel(Grid3 cg, const double* __restrict__ Uc,
               double* __restrict__ Uf, int ncols) {
  const int fx = 2 * cg.nx, fy = 2 * cg.ny, fz = 2 * cg.nz;
  const long long nf = (long long)(fx - 1) * (fy - 1) * (fz - 1);
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long d = t / ncols;
  const int c = (int)(t % ncols);
  if (d >= nf) return;
  const int I = (int)(d % (fx - 1)) + 1;
  const int J = (int)((d / (fx - 1)) % (fy - 1)) + 1;
  const int K = (int)(d / ((long long)(fx - 1) * (fy - 1))) + 1;
  const int a = I >> 1, b = J >> 1, e = K >> 1;
  const double u0 = vertex_u(Uc, cg, ncols, c, a, b, e);
  double v = u0;
  if ((I | J | K) & 1)
    v = 0.5 * (u0 + vertex_u(Uc, cg, ncols, c, a + (I & 1), b + (J & 1),
                             e + (K & 1)));
  Uf[(size_t)d * ncols + c] = v;
}

Grid3 grid_of(const paro_box_t* box) {
  Grid3 g;
  g.nx = box->nx;
  g.ny = box->ny;
  g.nz = box->nz;
  const int n[3] = {box->nx, box->ny, box->nz};
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = box->lo[a];
    g.h[a] = (box->hi[a] - box->lo[a]) / n[a];
  }
  return g;
}

bool box_ok(const paro_box_t* box) {
  if (!box || box->nx < 2 || box->ny < 2 || box->nz < 2) return false;
  for (int a = 0; a < 3; ++a)
    if (!(box->hi[a] > box->lo[a])) return false;
  return true;
}

#define AD_HIP(expr)                                                    \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      std::string m_ = std::string(#expr) + ": " + hipGetErrorString(e_); \
      return set_error(PARO_EDEVICE, m_.c_str());                       \
    }                                                                   \
  } while (0)

// ---- general (bisection) meshes --------------------------------------
// The same indicator on an element of a general mesh: corners from the
// element list, values through the dof map (0 on the boundary), the
// gradient from the element's edge vectors, the element across each face
// from the face-neighbour table.

// Coordinates and values of orbital column i at the corners of element e.
__device__ __forceinline__ void mesh_corners(
    const int32_t* __restrict__ tets, const double* __restrict__ Xv,
    const int32_t* __restrict__ dofmap, const double* __restrict__ U,
    int ncols, int i, long long e, double (&X)[4][3], double (&u)[4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int32_t v = tets[4 * e + a];
#pragma unroll
    for (int x = 0; x < 3; ++x) X[a][x] = Xv[3 * (size_t)v + x];
    const int32_t d = dofmap[v];
    u[a] = d >= 0 ? U[(size_t)d * ncols + i] : 0.0;
  }
}

// Gradient of the P1 interpolant of u on the element with corners X (the
// edge vectors' inverse by cofactors); returns |det| = 6 |T|.
__device__ __forceinline__ double mesh_grad(const double (&X)[4][3],
                                            const double (&u)[4],
                                            double (&g)[3]) {
  double E[3][3], du[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    du[a] = u[a + 1] - u[0];
#pragma unroll
    for (int x = 0; x < 3; ++x) E[a][x] = X[a + 1][x] - X[0][x];
  }
  double cof[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
      const int x1 = (x + 1) % 3, x2 = (x + 2) % 3;
      cof[a][x] = E[a1][x1] * E[a2][x2] - E[a1][x2] * E[a2][x1];
    }
  const double det = E[0][0] * cof[0][0] + E[0][1] * cof[0][1] +
                     E[0][2] * cof[0][2];
  // E g = du  =>  g = E^{-1} du, (E^{-1})[x][a] = cof[a][x] / det.
#pragma unroll
  for (int x = 0; x < 3; ++x)
    g[x] = (cof[0][x] * du[0] + cof[1][x] * du[1] + cof[2][x] * du[2]) / det;
  return fabs(det);
}

__global__ void __launch_bounds__(kBlock)
mesh_estimate_kernel(const int32_t* __restrict__ tets,
                     const int32_t* __restrict__ nbr,
                     const double* __restrict__ Xv,
                     const int32_t* __restrict__ dofmap,
                     const double* __restrict__ Vv,
                     const double* __restrict__ lam,
                     const double* __restrict__ U, int ncols, int nreq,
                     int NP, long long nelem, double* __restrict__ eta) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long e = t / NP;
  const int i = (int)(t % NP);
  double s = 0.0;
  if (e < nelem && i < nreq) {
    double X[4][3], u[4], vv[4];
    mesh_corners(tets, Xv, dofmap, U, ncols, i, e, X, u);
#pragma unroll
    for (int a = 0; a < 4; ++a) vv[a] = Vv[tets[4 * e + a]];
    double hT2 = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a + 1; b < 4; ++b) {
        double l2 = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x)
          l2 += (X[a][x] - X[b][x]) * (X[a][x] - X[b][x]);
        hT2 = fmax(hT2, l2);
      }
    double gT[3];
    const double vol = mesh_grad(X, u, gT) / 6.0;
    const double l = lam[i];
    double R[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        R[a][b] = 0.5 * l * (u[a] + u[b]) - 0.5 * (vv[a] * u[b] + vv[b] * u[a]);
    double r2 = 0.0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int cc = 0; cc < 4; ++cc)
#pragma unroll
          for (int d = 0; d < 4; ++d)
            r2 += R[a][b] * R[cc][d] * quartic(a, b, cc, d);
    s = hT2 * vol * r2;
    for (int k = 0; k < 4; ++k) {
      const int32_t f = nbr[4 * e + k];
      if (f < 0) continue;  // boundary face
      double Xn[4][3], un[4], gN[3];
      mesh_corners(tets, Xv, dofmap, U, ncols, i, f, Xn, un);
      (void)mesh_grad(Xn, un, gN);
      double F[3][3];
      int m = 0;
      for (int a = 0; a < 4; ++a) {
        if (a == k) continue;
#pragma unroll
        for (int x = 0; x < 3; ++x) F[m][x] = X[a][x];
        ++m;
      }
      const double e1[3] = {F[1][0] - F[0][0], F[1][1] - F[0][1],
                            F[1][2] - F[0][2]};
      const double e2[3] = {F[2][0] - F[0][0], F[2][1] - F[0][1],
                            F[2][2] - F[0][2]};
      const double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                             e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
      const double nn = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] +
                             nrm[2] * nrm[2]);
      double hF2 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
          double l2 = 0.0;
#pragma unroll
          for (int x = 0; x < 3; ++x)
            l2 += (F[a][x] - F[b][x]) * (F[a][x] - F[b][x]);
          hF2 = fmax(hF2, l2);
        }
      double j = 0.0;
#pragma unroll
      for (int x = 0; x < 3; ++x) j += (gT[x] - gN[x]) * nrm[x];
      j = 0.5 * j / nn;
      s += 0.5 * sqrt(hF2) * (0.5 * nn) * j * j;
    }
  }
  for (int o = NP / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, NP);
  if (e < nelem && i == 0) eta[e] = sqrt(s);
}

}  // namespace
}  // namespace paro

using namespace paro;

extern "C" {

int paro_mesh_estimate(const paro_problem* h, const double* d_lambda,
                       const double* d_U, int32_t ncols, int32_t nreq,
                       double* d_eta, void* stream) {
  if (!h || !d_lambda || !d_U || !d_eta)
    return set_error(PARO_EINVAL, "bad argument to paro_mesh_estimate");
  const Problem& p = h->p;
  if (!p.csr)
    return set_error(PARO_EINVAL,
                     "paro_mesh_estimate needs a problem assembled on a "
                     "mesh (paro_estimate serves box problems)");
  if (ncols < 1 || ncols > kNtMax || nreq < 1 || nreq > ncols)
    return set_error(PARO_EINVAL, "need 1 <= nreq <= ncols <= 64");
  int NP = 1;
  while (NP < nreq) NP <<= 1;
  const long long threads = (long long)p.ne * NP;
  const long long blocks = (threads + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL)
    return set_error(PARO_EINVAL, "mesh too large for paro_mesh_estimate");
  hipLaunchKernelGGL(mesh_estimate_kernel, dim3((unsigned)blocks),
                     dim3(kBlock), 0, (hipStream_t)stream, p.tets, p.nbr,
                     p.Xv, p.dofmap, p.Vv, d_lambda, d_U, ncols, nreq, NP,
                     (long long)p.ne, d_eta);
  AD_HIP(hipGetLastError());
  return PARO_OK;
}

int64_t paro_elements(const paro_box_t* box) {
  if (!box_ok(box)) return 0;
  return 6LL * box->nx * box->ny * box->nz;
}

int paro_estimate(const paro_box_t* box, const double* d_V,
                  const double* d_lambda, const double* d_U, int32_t ncols,
                  int32_t nreq, double* d_eta, void* stream) {
  if (!box_ok(box) || !d_V || !d_lambda || !d_U || !d_eta)
    return set_error(PARO_EINVAL, "bad argument to paro_estimate");
  if (ncols < 1 || ncols > kNtMax || nreq < 1 || nreq > ncols)
    return set_error(PARO_EINVAL, "need 1 <= nreq <= ncols <= 64");
  const Grid3 g = grid_of(box);
  int NP = 1;
  while (NP < nreq) NP <<= 1;
  const long long nelem = 6LL * box->nx * box->ny * box->nz;
  const long long threads = nelem * NP;
  const long long blocks = (threads + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL)
    return set_error(PARO_EINVAL, "mesh too large for paro_estimate");
  hipLaunchKernelGGL(estimate_kernel, dim3((unsigned)blocks), dim3(kBlock), 0,
                     (hipStream_t)stream, g, d_V, d_lambda, d_U, ncols, nreq,
                     NP, nelem, d_eta);
  AD_HIP(hipGetLastError());
  return PARO_OK;
}

size_t paro_mark_workspace_bytes(void) {
  // out, then per-block sums, maxima, counts and tie offsets.
  return 256 + (sizeof(double) * 2 + sizeof(long long) * 2) * kMarkGrid;
}

int paro_mark(const double* d_eta, int64_t count, double theta,
              int32_t strategy, uint8_t* d_marked, int64_t* h_nmarked,
              void* d_ws, size_t bytes, void* stream) {
  if (!d_eta || !d_marked || !d_ws || count < 1)
    return set_error(PARO_EINVAL, "bad argument to paro_mark");
  if (!(theta > 0.0) || !(theta <= 1.0))
    return set_error(PARO_EINVAL, "theta must lie in (0, 1]");
  if (strategy != PARO_MARK_DORFLER && strategy != PARO_MARK_MAXIMUM)
    return set_error(PARO_EINVAL, "unknown marking strategy");
  if (bytes < paro_mark_workspace_bytes() || ((uintptr_t)d_ws & 255))
    return set_error(PARO_ENOMEM, "marking workspace too small or unaligned");
  hipStream_t s = (hipStream_t)stream;
  double* out = (double*)d_ws;
  double* psum = (double*)((char*)d_ws + 256);
  double* pmax = psum + kMarkGrid;
  long long* pcnt = (long long*)(pmax + kMarkGrid);
  long long* tbase = pcnt + kMarkGrid;
  // One fixed-order pass: (sum of eta^2, max eta, count) over eta >= t
  // (strict: eta > t).
  auto pass = [&](double t, int strict, double* res) -> int {
    hipLaunchKernelGGL(mark_partial_kernel, dim3(kMarkGrid), dim3(kBlock), 0,
                       s, d_eta, (long long)count, t, strict, psum, pmax,
                       pcnt);
    hipLaunchKernelGGL(mark_final_kernel, dim3(1), dim3(kBlock), 0, s,
                       (const double*)psum, (const double*)pmax,
                       (const long long*)pcnt, out);
    AD_HIP(hipGetLastError());
    AD_HIP(hipMemcpyAsync(res, out, 3 * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    return PARO_OK;
  };
  double all[3];
  int rc = pass(0.0, 0, all);
  if (rc) return rc;
  const double total = all[0], emax = all[1];
  double t = 0.0;
  int strict = 0;
  long long ties = 0, nmark = 0;
  if (strategy == PARO_MARK_MAXIMUM) {
    t = theta * emax;  // eq. (maximum-strategy): eta >= theta max eta
    double r[3];
    rc = pass(t, 0, r);
    if (rc) return rc;
    nmark = (long long)r[2];
  } else {
    // Largest T with sum_{eta >= T} eta^2 >= theta total (bisection over
    // the bit patterns of non-negative doubles, which order like their
    // values); then every element above T and, lowest indices first, as
    // many equal to T as the sum still needs.
    const double want = theta * total;
    uint64_t lo = 0, hi;
    std::memcpy(&hi, &emax, sizeof hi);
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo + 1) / 2;
      double tm;
      std::memcpy(&tm, &mid, sizeof tm);
      double r[3];
      rc = pass(tm, 0, r);
      if (rc) return rc;
      if (r[0] >= want)
        lo = mid;
      else
        hi = mid - 1;
    }
    std::memcpy(&t, &lo, sizeof t);
    strict = 1;
    double above[3];
    rc = pass(t, 1, above);
    if (rc) return rc;
    double acc = above[0];
    while (acc < want) {
      acc += t * t;
      ++ties;
    }
    nmark = (long long)above[2] + ties;
    if (ties > 0) {
      hipLaunchKernelGGL(mark_ties_count_kernel, dim3(kMarkGrid),
                         dim3(kBlock), 0, s, d_eta, (long long)count, t,
                         pcnt);
      AD_HIP(hipGetLastError());
      std::vector<long long> c(kMarkGrid), b(kMarkGrid);
      AD_HIP(hipMemcpyAsync(c.data(), pcnt, sizeof(long long) * kMarkGrid,
                            hipMemcpyDeviceToHost, s));
      AD_HIP(hipStreamSynchronize(s));
      long long run = 0;
      for (int k = 0; k < kMarkGrid; ++k) {
        b[k] = run;
        run += c[k];
      }
      AD_HIP(hipMemcpyAsync(tbase, b.data(), sizeof(long long) * kMarkGrid,
                            hipMemcpyHostToDevice, s));
      AD_HIP(hipStreamSynchronize(s));  // b is a stack array
    }
  }
  hipLaunchKernelGGL(mark_set_kernel, dim3(kMarkGrid), dim3(kBlock), 0, s,
                     d_eta, (long long)count, t, strict, ties,
                     (const long long*)tbase, d_marked);
  AD_HIP(hipGetLastError());
  if (h_nmarked) *h_nmarked = nmark;
  return PARO_OK;
}

int paro_prolong(const paro_box_t* coarse, const double* d_Uc, double* d_Uf,
                 int32_t ncols, void* stream) {
  if (!box_ok(coarse) || !d_Uc || !d_Uf)
    return set_error(PARO_EINVAL, "bad argument to paro_prolong");
  if (ncols < 1 || ncols > kNtMax)
    return set_error(PARO_EINVAL, "ncols must be 1..64");
  const Grid3 g = grid_of(coarse);
  const long long nf =
      (long long)(2 * g.nx - 1) * (2 * g.ny - 1) * (2 * g.nz - 1);
  const long long blocks = (nf * ncols + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL)
    return set_error(PARO_EINVAL, "mesh too large for paro_prolong");
  hipLaunchKernelGGL(prolong_kernel, dim3((unsigned)blocks), dim3(kBlock), 0,
                     (hipStream_t)stream, g, d_Uc, d_Uf, ncols);
  AD_HIP(hipGetLastError());
  return PARO_OK;
}

}  // extern "C"
