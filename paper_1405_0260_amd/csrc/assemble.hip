// Assembly of the P1 source-problem operator on a uniform Kuhn mesh.
//
// Finite elements as in Sec. 2 of the paper (continuous piecewise-linear
// functions on a conforming tetrahedral mesh, zero on the boundary) and the
// form of eq. (eq-operator-A) with a fixed potential:
//   a(w, v) = 1/2 (grad w, grad v) + (V_h w, v),
// V_h the nodal interpolant of V, integrated exactly.  One thread owns one
// matrix row (one interior vertex) and sums the contributions of the 24
// tetrahedra around it in a fixed order: no atomics, bitwise reproducible.
//
// Besides CSR, every value is also written in stencil order: diag[s][d] is
// the coefficient of row d and neighbour offset s (0 when the neighbour is
// outside the box), the layout the solver kernels stream.
//
// Pattern: every edge of a Kuhn tetrahedron is a multiple-free difference
// of e_x, e_y, e_z, e_i + e_j or (1,1,1), so a row couples its vertex to at
// most 15 vertices (itself included), listed in ascending column order in
// kOff.  Because validity of an offset factorises over the axes, the row
// pointer has a closed form (no scan).
#include <cmath>
#include <cstdio>

#include "paro_internal.h"

namespace paro {

namespace {

// The 15 neighbour offsets in ascending linear order (x fastest).
__constant__ int kOff[kStencil][3] = {
    {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
    {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
    {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};

// Local vertices of the Kuhn tetrahedron of permutation q of the axes:
// (0,0,0), e_q0, e_q0 + e_q1, (1,1,1).
__constant__ int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

struct Incidence {
  // For stencil offset s: entries [first[s], first[s+1]) of the lists.
  int first[kStencil + 1];
  unsigned char corner[96];  // cube corner occupied by the row vertex (bits)
  unsigned char perm[96];
  unsigned char la[96];      // local index of the row vertex
  unsigned char lb[96];      // local index of the column vertex
};

void local_vertex(int q, int a, int out[3]) {
  static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                 {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  out[0] = out[1] = out[2] = 0;
  if (a >= 1) out[perm[q][0]] = 1;
  if (a >= 2) out[perm[q][1]] = 1;
  if (a == 3) out[0] = out[1] = out[2] = 1;
}

// Enumerate, for each offset, every (cube, tetrahedron, local pair) whose
// two local vertices are the row vertex and the row vertex + offset.
Incidence build_incidence() {
  static const int off[kStencil][3] = {
      {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
      {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
      {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};
  Incidence t{};
  int k = 0;
  for (int s = 0; s < kStencil; ++s) {
    t.first[s] = k;
    for (int c = 0; c < 8; ++c) {
      int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      for (int q = 0; q < 6; ++q) {
        int la = -1, lb = -1;
        for (int a = 0; a < 4; ++a) {
          int L[3];
          local_vertex(q, a, L);
          if (L[0] == cv[0] && L[1] == cv[1] && L[2] == cv[2]) la = a;
          if (L[0] == cv[0] + off[s][0] && L[1] == cv[1] + off[s][1] &&
              L[2] == cv[2] + off[s][2])
            lb = a;
        }
        if (la >= 0 && lb >= 0) {
          t.corner[k] = (unsigned char)c;
          t.perm[k] = (unsigned char)q;
          t.la[k] = (unsigned char)la;
          t.lb[k] = (unsigned char)lb;
          ++k;
        }
      }
    }
  }
  t.first[kStencil] = k;
  return t;
}

// Number of i in [0, i0) with 0 <= i + o < m, for o in {-1, 0, 1}.
__device__ __forceinline__ long long prefix_valid(int i0, int o, int m) {
  if (o == 0) return i0;
  if (o > 0) return i0 < m - 1 ? i0 : m - 1;
  return i0 > 1 ? i0 - 1 : 0;
}

__device__ __forceinline__ bool valid(int i, int o, int m) {
  return i + o >= 0 && i + o < m;
}

__global__ void __launch_bounds__(kBlock)
assemble_kernel(Incidence inc, const double* __restrict__ V, int mx, int my,
                int mz, double hx, double hy, double hz, double sigma,
                double* __restrict__ dinv, float* __restrict__ dinv32,
                double* __restrict__ diagA, double* __restrict__ diagM,
                float* __restrict__ diagA32) {
  const long long n = (long long)mx * my * mz;
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const int nvx = mx + 2, nvy = my + 2;
  const int i = (int)(d % mx);
  const int j = (int)((d / mx) % my);
  const int k = (int)(d / ((long long)mx * my));

  const double vol = hx * hy * hz / 6.0;
  const double hv[3] = {hx, hy, hz};
  const int I = i + 1, J = j + 1, K = k + 1;  // vertex indices

  for (int s = 0; s < kStencil; ++s) {
    const int ox = kOff[s][0], oy = kOff[s][1], oz = kOff[s][2];
    if (!valid(i, ox, mx) || !valid(j, oy, my) || !valid(k, oz, mz)) {
      // Stencil order: a neighbour outside the box has coefficient 0.
      diagA[(size_t)s * n + d] = 0.0;
      diagM[(size_t)s * n + d] = 0.0;
      if (diagA32) diagA32[(size_t)s * n + d] = 0.0f;
      continue;
    }
    double a_sum = 0.0, m_sum = 0.0;
    for (int e = inc.first[s]; e < inc.first[s + 1]; ++e) {
      const int c = inc.corner[e], q = inc.perm[e];
      const int la = inc.la[e], lb = inc.lb[e];
      const int bx = I - (c & 1), by = J - ((c >> 1) & 1),
                bz = K - ((c >> 2) & 1);
      // Local vertex offsets and their potential values.
      int L[4][3];
      double Vl[4];
      for (int a = 0; a < 4; ++a) {
        L[a][0] = L[a][1] = L[a][2] = 0;
        if (a >= 1) L[a][kPerm[q][0]] = 1;
        if (a >= 2) L[a][kPerm[q][1]] = 1;
        if (a == 3) L[a][0] = L[a][1] = L[a][2] = 1;
        const long long vid = (long long)(bx + L[a][0]) +
                              (long long)nvx * ((by + L[a][1]) +
                                                (long long)nvy * (bz + L[a][2]));
        Vl[a] = V[vid];
      }
      // Edge matrix E (rows x_a - x_0, a = 1..3) and its inverse; the
      // barycentric gradients are the columns of E^{-1}.
      double E[3][3];
      for (int a = 0; a < 3; ++a)
        for (int x = 0; x < 3; ++x) E[a][x] = hv[x] * L[a + 1][x];
      const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                         E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                         E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
      double Ei[3][3];
      Ei[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
      Ei[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
      Ei[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
      Ei[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
      Ei[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
      Ei[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
      Ei[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
      Ei[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
      Ei[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
      double ga[3], gb[3];
      for (int x = 0; x < 3; ++x) {
        // grad lambda_a (a >= 1) = column a-1 of E^{-1}: Ei[x][a-1].
        const double g1 = Ei[x][0], g2 = Ei[x][1], g3 = Ei[x][2];
        const double gl[4] = {-(g1 + g2 + g3), g1, g2, g3};
        ga[x] = gl[la];
        gb[x] = gl[lb];
      }
      const double kab = vol * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
      const double vsum = Vl[0] + Vl[1] + Vl[2] + Vl[3];
      double mab, mvab;
      if (la == lb) {
        mab = vol / 10.0;
        mvab = vol / 60.0 * (vsum + 2.0 * Vl[la]);
      } else {
        mab = vol / 20.0;
        mvab = vol / 120.0 * (vsum + Vl[la] + Vl[lb]);
      }
      a_sum += 0.5 * kab + mvab - sigma * mab;
      m_sum += mab;
    }
    diagA[(size_t)s * n + d] = a_sum;
    diagM[(size_t)s * n + d] = m_sum;
    if (diagA32) diagA32[(size_t)s * n + d] = (float)a_sum;
    if (ox == 0 && oy == 0 && oz == 0) {
      dinv[d] = 1.0 / a_sum;
      if (dinv32) dinv32[d] = (float)(1.0 / a_sum);
    }
  }
}

// CSR copy of the stencil-order matrices (row d = thread d, plus the
// closing row pointer): the entries of a row are its in-box neighbours in
// stencil order, which is ascending column order; the row's first slot
// comes from a closed-form count of the entries of the rows before it.
// Any output may be null.
__global__ void __launch_bounds__(kBlock)
csr_export_kernel(int mx, int my, int mz, const double* __restrict__ diagA,
                  const double* __restrict__ diagM,
                  int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
                  double* __restrict__ valA, double* __restrict__ valM) {
  const long long n = (long long)mx * my * mz;
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d > n) return;
  if (d == n) {  // closing row pointer
    long long tot = 0;
    for (int s = 0; s < kStencil; ++s)
      tot += prefix_valid(mx, kOff[s][0], mx) *
             prefix_valid(my, kOff[s][1], my) *
             prefix_valid(mz, kOff[s][2], mz);
    if (rowptr) rowptr[n] = (int32_t)tot;
    return;
  }
  const int i = (int)(d % mx);
  const int j = (int)((d / mx) % my);
  const int k = (int)(d / ((long long)mx * my));
  // Rows before (i, j, k) in x-fastest order, offset by offset.
  long long start = 0;
  for (int s = 0; s < kStencil; ++s) {
    const int ox = kOff[s][0], oy = kOff[s][1], oz = kOff[s][2];
    const long long tx = prefix_valid(mx, ox, mx);
    const long long ty = prefix_valid(my, oy, my);
    const long long fz = valid(k, oz, mz), fy = valid(j, oy, my);
    start += prefix_valid(k, oz, mz) * ty * tx +
             fz * prefix_valid(j, oy, my) * tx +
             fz * fy * prefix_valid(i, ox, mx);
  }
  if (rowptr) rowptr[d] = (int32_t)start;
  long long slot = start;
  for (int s = 0; s < kStencil; ++s) {
    const int ox = kOff[s][0], oy = kOff[s][1], oz = kOff[s][2];
    if (!valid(i, ox, mx) || !valid(j, oy, my) || !valid(k, oz, mz))
      continue;
    if (col)
      col[slot] =
          (int32_t)(d + ox + (long long)mx * (oy + (long long)my * oz));
    if (valA) valA[slot] = diagA[(size_t)s * n + d];
    if (valM) valM[slot] = diagM[(size_t)s * n + d];
    ++slot;
  }
}

// min, max and the count of non-finite values of the nodal potential.
__global__ void __launch_bounds__(kBlock)
potential_range_kernel(const double* __restrict__ V, long long nv,
                       double* __restrict__ out, unsigned* __restrict__ cnt,
                       double* __restrict__ part) {
  __shared__ double smin[kBlock], smax[kBlock], sbad[kBlock];
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nv;
       t += (long long)gridDim.x * blockDim.x) {
    const double v = V[t];
    if (!isfinite(v)) {
      bad += 1.0;
    } else {
      lo = fmin(lo, v);
      hi = fmax(hi, v);
    }
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      sbad[threadIdx.x] += sbad[threadIdx.x + w];
    }
    __syncthreads();
  }
  __shared__ bool last;
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = smin[0];
    part[3 * blockIdx.x + 1] = smax[0];
    part[3 * blockIdx.x + 2] = sbad[0];
    __threadfence();
    const unsigned t = atomicAdd(cnt, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    double a = INFINITY, b = -INFINITY, c = 0.0;
    for (unsigned g = 0; g < gridDim.x; ++g) {
      a = fmin(a, part[3 * g + 0]);
      b = fmax(b, part[3 * g + 1]);
      c += part[3 * g + 2];
    }
    out[0] = a;
    out[1] = b;
    out[2] = c;
    *cnt = 0u;
  }
}

}  // namespace

hipError_t launch_potential_range(const double* V, int64_t nv, double* out,
                                  unsigned* cnt, double* part, hipStream_t s) {
  int grid = (int)((nv + kBlock - 1) / kBlock);
  if (grid > 256) grid = 256;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(potential_range_kernel, dim3(grid), dim3(kBlock), 0, s, V,
                     (long long)nv, out, cnt, part);
  return hipGetLastError();
}

hipError_t launch_assemble(Problem& p, const double* V, hipStream_t s) {
  static const Incidence inc = build_incidence();
  const int grid = (int)((p.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(assemble_kernel, dim3(grid), dim3(kBlock), 0, s, inc, V,
                     p.mx, p.my, p.mz, p.h[0], p.h[1], p.h[2], p.sigma,
                     p.dinv, p.dinv32, p.diagA, p.diagM, p.diagA32);
  return hipGetLastError();
}

hipError_t launch_csr_export(const Problem& p, int32_t* rowptr, int32_t* col,
                             double* valA, double* valM, hipStream_t s) {
  const long long rows = p.n + 1;
  const int grid = (int)((rows + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(csr_export_kernel, dim3(grid), dim3(kBlock), 0, s, p.mx,
                     p.my, p.mz, (const double*)p.diagA,
                     (const double*)p.diagM, rowptr, col, valA, valM);
  return hipGetLastError();
}

int64_t kuhn_nnz(int mx, int my, int mz) {
  static const int off[kStencil][3] = {
      {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
      {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
      {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};
  auto cnt = [](int o, int m) -> int64_t {
    return o == 0 ? m : (m > 1 ? m - 1 : 0);
  };
  int64_t z = 0;
  for (int s = 0; s < kStencil; ++s)
    z += cnt(off[s][0], mx) * cnt(off[s][1], my) * cnt(off[s][2], mz);
  return z;
}

}  // namespace paro
