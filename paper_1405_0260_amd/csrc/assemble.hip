// Assembly of the P1 source-problem operator on a uniform Kuhn mesh.
//
// Finite elements as in Sec. 2 of the paper (continuous piecewise-linear
// functions on a conforming tetrahedral mesh, zero on the boundary) and the
// form of eq. (eq-operator-A) with a fixed potential:
//   a(w, v) = 1/2 (grad w, grad v) + (V_h w, v) - s (w, v),
// V_h the nodal interpolant of V, integrated exactly.  The stiffness and
// mass parts of a row are the same at every interior vertex of a uniform
// mesh: they are summed once on the host over the tetrahedra around each
// vertex pair.  The potential part is the closed form of kuhn.h, which one
// thread per row evaluates from the potential at its 15 stencil vertices:
// no atomics, bitwise reproducible, and bitwise the coefficients the
// matrix-free CG SpMM forms on the fly.
//
// The values are written in stencil order: diag[s][d] is the coefficient of
// row d and neighbour offset s (0 when the neighbour is outside the box),
// the layout the solver kernels stream.  CSR copies come from the stencil
// arrays.
//
// Pattern: every edge of a Kuhn tetrahedron is a multiple-free difference
// of e_x, e_y, e_z, e_i + e_j or (1,1,1), so a row couples its vertex to at
// most 15 vertices (itself included), listed in ascending column order in
// kOff.  Because validity of an offset factorises over the axes, the row
// pointer has a closed form (no scan).
#include <cmath>
#include <cstdio>

#include "kuhn.h"
#include "paro_internal.h"

namespace paro {

namespace {

// The 15 neighbour offsets in ascending linear order (x fastest).
__constant__ int kOff[kStencil][3] = {
    {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
    {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
    {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};

// The row-independent part of the operator: for each offset s the
// stiffness sum K_s = sum_e vol grad lambda_a . grad lambda_b and the mass
// sum M_s = sum_e (phi_a, phi_b)_e over the tetrahedra e around the pair
// (row vertex = local vertex a, neighbour = local vertex b).
struct KuhnConst {
  double k[kKcCount];   // c0_s = 1/2 K_s - s M_s, vol / 60, M by pair class
                        // (the layout of kuhn.h)
  double m[kStencil];   // M_s
};

KuhnConst kuhn_constants(const double h[3], double sigma) {
  KuhnConst kc{};
  const double vol = h[0] * h[1] * h[2] / 6.0;
  for (int s = 0; s < kStencil; ++s) {
    double ksum = 0.0, msum = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int cv[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
      for (int q = 0; q < 6; ++q) {
        int L[4][3] = {};
        int la = -1, lb = -1;
        for (int a = 0; a < 4; ++a) {
          kuhn_local(q, a, L[a]);
          if (L[a][0] == cv[0] && L[a][1] == cv[1] && L[a][2] == cv[2]) la = a;
          if (L[a][0] == cv[0] + kKuhnOff[s][0] &&
              L[a][1] == cv[1] + kKuhnOff[s][1] &&
              L[a][2] == cv[2] + kKuhnOff[s][2])
            lb = a;
        }
        if (la < 0 || lb < 0) continue;
        // Edge matrix E (rows x_a - x_0, a = 1..3) and its inverse; the
        // barycentric gradients are the columns of E^{-1}.
        double E[3][3];
        for (int a = 0; a < 3; ++a)
          for (int x = 0; x < 3; ++x) E[a][x] = h[x] * L[a + 1][x];
        const double det =
            E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
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
        ksum += vol * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
        msum += la == lb ? vol / 10.0 : vol / 20.0;
      }
    }
    kc.k[s] = 0.5 * ksum - sigma * msum;
    kc.m[s] = msum;
  }
  kc.k[kKcVol60] = vol / 60.0;
  // The sums of a pair class are the same additions in the same order.
  kc.k[kKcM4] = kc.m[1];
  kc.k[kKcM6] = kc.m[0];
  kc.k[kKcMDiag] = kc.m[7];
  return kc;
}

__device__ __forceinline__ bool valid(int i, int o, int m) {
  return i + o >= 0 && i + o < m;
}

// Number of i in [0, i0) with 0 <= i + o < m, for o in {-1, 0, 1}.
__device__ __forceinline__ long long prefix_valid(int i0, int o, int m) {
  if (o == 0) return i0;
  if (o > 0) return i0 < m - 1 ? i0 : m - 1;
  return i0 > 1 ? i0 - 1 : 0;
}

// Mass coefficient of offset S (its pair class).
template <int S>
__device__ __forceinline__ void mass_row_from(const double* k, unsigned mask,
                                              double (&m)[kStencil]) {
  m[S] = (mask >> S) & 1u ? k[kuhn_mass_slot(S)] : 0.0;
  if constexpr (S + 1 < kStencil) mass_row_from<S + 1>(k, mask, m);
}

// One thread per row.  V holds all (mx + 2)(my + 2)(mz + 2) vertices, x
// fastest; the row of dof (i, j, k) is vertex (i + 1, j + 1, k + 1).
// Threads d < kKcCount also publish the stencil constants to `kconst`
// (the matrix-free SpMMs read them there).
__global__ void __launch_bounds__(kBlock)
assemble_kernel(KuhnConst kc, const double* __restrict__ V, int mx, int my,
                int mz, double* __restrict__ dinv, float* __restrict__ dinv32,
                double* __restrict__ diagA, double* __restrict__ diagM,
                float* __restrict__ diagA32, double* __restrict__ kconst) {
  const long long n = (long long)mx * my * mz;
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (kconst && d < kKcCount) kconst[d] = kc.k[d];
  if (d >= n) return;
  const int i = (int)(d % mx);
  const int j = (int)((d / mx) % my);
  const int k = (int)(d / ((long long)mx * my));
  const long long sy = mx + 2, sz = (long long)(mx + 2) * (my + 2);
  const double* Vr = V + (i + 1) + sy * (j + 1) + sz * (k + 1);
  double v[kStencil];
  unsigned mask = 0;
#pragma unroll
  for (int s = 0; s < kStencil; ++s) {
    const int ox = kKuhnOff[s][0], oy = kKuhnOff[s][1], oz = kKuhnOff[s][2];
    v[s] = Vr[ox + sy * oy + sz * oz];
    if (valid(i, ox, mx) && valid(j, oy, my) && valid(k, oz, mz))
      mask |= 1u << s;
  }
  double a[kStencil], m[kStencil];
  kuhn_row(v, kc.k, kc.k[kKcVol60], mask, a);
  mass_row_from<0>(kc.k, mask, m);
#pragma unroll
  for (int s = 0; s < kStencil; ++s) {
    diagA[(size_t)s * n + d] = a[s];
    diagM[(size_t)s * n + d] = m[s];
    if (diagA32) diagA32[(size_t)s * n + d] = (float)a[s];
  }
  dinv[d] = 1.0 / a[7];
  if (dinv32) dinv32[d] = (float)(1.0 / a[7]);
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
  const KuhnConst kc = kuhn_constants(p.h, p.sigma);
  if (p.Vb) {
    // The matrix-free CG SpMM reads the potential during every solve.
    const size_t nv = (size_t)(p.mx + 2) * (p.my + 2) * (p.mz + 2);
    const hipError_t e = hipMemcpyAsync(p.Vb, V, sizeof(double) * nv,
                                        hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  const int grid = (int)((p.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(assemble_kernel, dim3(grid), dim3(kBlock), 0, s, kc, V,
                     p.mx, p.my, p.mz, p.dinv, p.dinv32, p.diagA, p.diagM,
                     p.diagA32, p.kconst);
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
