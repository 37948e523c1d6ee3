// Kohn-Sham outer iteration around ParO (Sec. 2, eqs. (eq-ks), (weak-ks),
// (eq-operator-A); Algorithm 3.1): each outer iteration forms the density
// of the current orbitals, mixes it into the input density (linearly, or
// with the residual filtered by Kerker's (K + q0^2 vol I)^-1 K, which
// damps its long-wavelength part), solves the
// Poisson equation -Lap V_H = 4 pi rho for the Hartree potential (P1, zero
// on the box boundary: K V_H = 4 pi M rho, solved directly with the 3-D
// discrete sine transform that diagonalises K on the uniform box grid, or
// optionally by the library's Jacobi-PCG on (1/2) K), adds the Slater
// exchange potential -(3 rho / pi)^(1/3), re-assembles the Hamiltonian with
// the effective potential and takes one ParO step with it.
//
// Densities live on the interior dofs (the orbitals vanish on the
// boundary); the effective potential is nodal on all vertices, as the
// assembly expects.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "paro_internal.h"

namespace paro {
namespace {

constexpr int kKsGrid = 256;  // blocks of the density reductions

// rho_out[d] = occupancy * sum_{i < N} U[d][i]^2.
__global__ void __launch_bounds__(kBlock)
ks_density_kernel(const double* __restrict__ U, long long n, int ncols, int N,
                  double occ, double* __restrict__ rho) {
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock) {
    const double* u = U + (size_t)d * ncols;
    double s = 0.0;
    for (int i = 0; i < N; ++i) s = fma(u[i], u[i], s);
    rho[d] = occ * s;
  }
}

// Density residual partials (||rho_out - rho_in||^2, ||rho_in||^2 per
// block, fixed grid) and the mixing rho_in <- (1 - beta) rho_in + beta
// rho_out (first: rho_in <- rho_out, no residual).
__global__ void __launch_bounds__(kBlock)
ks_mix_kernel(const double* __restrict__ rho_out, double* __restrict__ rho_in,
              long long n, double beta, int first,
              double* __restrict__ part) {
  __shared__ double r0[kBlock], r1[kBlock];
  double a = 0.0, b = 0.0;
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock) {
    const double o = rho_out[d];
    if (first) {
      rho_in[d] = o;
      continue;
    }
    const double i = rho_in[d], e = o - i;
    a = fma(e, e, a);
    b = fma(i, i, b);
    rho_in[d] = (1.0 - beta) * i + beta * o;
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r0[0];
    part[kKsGrid + blockIdx.x] = r1[0];
  }
}

// Kerker-preconditioned mixing, first half: the density residual
// e = rho_out - rho_in into `e` and its norm partials (as ks_mix_kernel).
__global__ void __launch_bounds__(kBlock)
ks_resid_vec_kernel(const double* __restrict__ rho_out,
                    const double* __restrict__ rho_in, long long n,
                    double* __restrict__ e_out, double* __restrict__ part) {
  __shared__ double r0[kBlock], r1[kBlock];
  double a = 0.0, b = 0.0;
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock) {
    const double i = rho_in[d], e = rho_out[d] - i;
    e_out[d] = e;
    a = fma(e, e, a);
    b = fma(i, i, b);
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r0[0];
    part[kKsGrid + blockIdx.x] = r1[0];
  }
}

// Second half: rho_in += beta * (filtered residual).
__global__ void __launch_bounds__(kBlock)
ks_axpy_kernel(double* __restrict__ rho_in, const double* __restrict__ e,
               long long n, double beta) {
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock)
    rho_in[d] = fma(beta, e[d], rho_in[d]);
}

// Fixed-order sum of the partials: out[0] = ||rho_out - rho_in||^2,
// out[1] = ||rho_in||^2 (one block).
__global__ void __launch_bounds__(kBlock)
ks_residual_kernel(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double r0[kBlock], r1[kBlock];
  r0[threadIdx.x] = threadIdx.x < kKsGrid ? part[threadIdx.x] : 0.0;
  r1[threadIdx.x] = threadIdx.x < kKsGrid ? part[kKsGrid + threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

__global__ void __launch_bounds__(kBlock)
ks_scale_kernel(double* __restrict__ x, long long n, double a) {
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock)
    x[d] *= a;
}

// V_eff at every vertex: V_ext + V_H + v_x(rho_in) inside, V_ext on the
// boundary (rho = V_H = 0 there).
__global__ void __launch_bounds__(kBlock)
ks_potential_kernel(const double* __restrict__ Vext,
                    const double* __restrict__ vh,
                    const double* __restrict__ rho, int nx, int ny, int nz,
                    double* __restrict__ Veff) {
  const long long nv = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < nv;
       v += (long long)gridDim.x * kBlock) {
    const int i = (int)(v % (nx + 1));
    const int j = (int)((v / (nx + 1)) % (ny + 1));
    const int k = (int)(v / ((long long)(nx + 1) * (ny + 1)));
    double out = Vext[v];
    if (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz) {
      const long long d = (i - 1) + (long long)(nx - 1) *
                                        ((j - 1) + (long long)(ny - 1) * (k - 1));
      const double r = fmax(rho[d], 0.0);
      out += vh[d] - cbrt(3.0 * r / M_PI);
    }
    Veff[v] = out;
  }
}

// ---- Direct Hartree solve by the discrete sine transform ---------------
// On a uniform box grid the Kuhn P1 stiffness matrix is exactly the 7-point
// operator K = sum_a c_a T_a (T_a = tridiag(-1, 2, -1) along axis a, c_x =
// hy hz / hx and cyclically), so K V = f is diagonal in the sine basis:
// with S_a[p][q] = sin(pi (p + 1)(q + 1) / (m_a + 1)), S_a S_a =
// (m_a + 1) / 2 I and K = S^-1 diag(lambda) S, lambda_pqr = sum_a c_a
// 2 (1 - cos(pi (p_a + 1) / (m_a + 1))).  The transform along each axis is
// a small dense product, done by dgemm_kernel.

// Sine matrices of the three axes and the 1-D eigenvalue parts.
__global__ void __launch_bounds__(kBlock)
dst_tables_kernel(int mx, int my, int mz, double cx, double cy, double cz,
                  double* __restrict__ Sx, double* __restrict__ Sy,
                  double* __restrict__ Sz, double* __restrict__ ev) {
  const int m[3] = {mx, my, mz};
  const double c[3] = {cx, cy, cz};
  double* S[3] = {Sx, Sy, Sz};
  int evo = 0;
  for (int a = 0; a < 3; ++a) {
    const int ma = m[a];
    const double w = M_PI / (ma + 1);
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < ma * ma;
         e += gridDim.x * kBlock) {
      const int p = e / ma, q = e % ma;
      // (p+1)(q+1) mod 2(m+1) keeps the sine argument small and exact.
      const long long k = ((long long)(p + 1) * (q + 1)) % (2 * (ma + 1));
      S[a][e] = sin(w * (double)k);
    }
    for (int p = blockIdx.x * kBlock + threadIdx.x; p < ma;
         p += gridDim.x * kBlock)
      ev[evo + p] = c[a] * 2.0 * (1.0 - cos(w * (p + 1)));
    evo += ma;
  }
}

// C_b = alpha A_b B_b for a batch of row-major FP64 matrices (M x K times
// K x N), 64 x 64 output tiles, K in steps of 16 through LDS; thread
// (ty, tx) owns rows ty + 16 i and columns tx + 16 j, i, j < 4.
__global__ void __launch_bounds__(kBlock)
dgemm_kernel(int M, int N, int K, const double* __restrict__ A,
             long long lda, long long sA, const double* __restrict__ B,
             long long ldb, long long sB, double* __restrict__ C,
             long long ldc, long long sC, double alpha) {
  __shared__ double As[16][64 + 1], Bs[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  A += blockIdx.z * sA;
  B += blockIdx.z * sB;
  C += blockIdx.z * sC;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += kBlock) {
      const int r = e / 16, k = e % 16;  // A: row r, column k
      const int gm = m0 + r, gk = k0 + k;
      As[k][r] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.0;
      const int kb = e / 64, c = e % 64;  // B: row kb, column c
      const int gkb = k0 + kb, gn = n0 + c;
      Bs[kb][c] = (gkb < K && gn < N) ? B[(size_t)gkb * ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn < N) C[(size_t)gm * ldc + gn] = alpha * acc[i][j];
    }
  }
}

// g[x, y, z] /= lambda_xyz (sine coefficients).
__global__ void __launch_bounds__(kBlock)
dst_divide_kernel(double* __restrict__ g, int mx, int my, int mz,
                  const double* __restrict__ ev) {
  const long long n = (long long)mx * my * mz;
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock) {
    const int x = (int)(d % mx);
    const int y = (int)((d / mx) % my);
    const int z = (int)(d / ((long long)mx * my));
    g[d] /= ev[x] + ev[mx + y] + ev[mx + my + z];
  }
}

// Kerker filter in the sine basis: g[x, y, z] *= lambda / (lambda + c),
// lambda_xyz the eigenvalue of the stiffness matrix K, c = q0^2 times the
// cell volume (the lumped mass), i.e. (K + c I)^-1 K.
__global__ void __launch_bounds__(kBlock)
dst_kerker_kernel(double* __restrict__ g, int mx, int my, int mz,
                  const double* __restrict__ ev, double c) {
  const long long n = (long long)mx * my * mz;
  for (long long d = (long long)blockIdx.x * kBlock + threadIdx.x; d < n;
       d += (long long)gridDim.x * kBlock) {
    const int x = (int)(d % mx);
    const int y = (int)((d / mx) % my);
    const int z = (int)(d / ((long long)mx * my));
    const double lam = ev[x] + ev[mx + y] + ev[mx + my + z];
    g[d] *= lam / (lam + c);
  }
}

hipError_t dgemm(hipStream_t s, int M, int N, int K, const double* A,
                 long long lda, long long sA, const double* B, long long ldb,
                 long long sB, double* C, long long ldc, long long sC,
                 int batch, double alpha) {
  hipLaunchKernelGGL(dgemm_kernel, dim3((N + 63) / 64, (M + 63) / 64, batch),
                     dim3(kBlock), 0, s, M, N, K, A, lda, sA, B, ldb, sB, C,
                     ldc, sC, alpha);
  return hipGetLastError();
}

// out = (S_x (x) S_y (x) S_z) in, scaled by alpha (in and out distinct;
// tmp a third n-vector).  x is the fastest index.
hipError_t dst3(hipStream_t s, int mx, int my, int mz, const double* Sx,
                const double* Sy, const double* Sz, const double* in,
                double* tmp, double* out, double alpha) {
  const long long P = (long long)mx * my;
  // along x: rows of length mx times S_x (symmetric)
  hipError_t e = dgemm(s, (int)(P / mx * mz), mx, mx, in, mx, 0, Sx, mx, 0,
                       out, mx, 0, 1, 1.0);
  if (e != hipSuccess) return e;
  // along y: for each z plane, S_y times the my x mx plane
  e = dgemm(s, my, mx, my, Sy, my, 0, out, mx, P, tmp, mx, P, mz, 1.0);
  if (e != hipSuccess) return e;
  // along z: S_z times the mz x P matrix
  return dgemm(s, mz, (int)P, mz, Sz, mz, 0, tmp, P, 0, out, P, 0, 1, alpha);
}

int grid_for(long long n) {
  long long g = (n + kBlock - 1) / kBlock;
  if (g > kKsGrid) g = kKsGrid;
  return (int)(g < 1 ? 1 : g);
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

struct KsLayout {
  size_t poisson, vzero, rho_in, rho_out, vh, b, t1, veff, part, res, sx, sy,
      sz, ev, total;
};

KsLayout ks_layout(const paro_box_t* box, size_t poisson_ws) {
  const size_t nv = (size_t)(box->nx + 1) * (box->ny + 1) * (box->nz + 1);
  const size_t n = (size_t)(box->nx - 1) * (box->ny - 1) * (box->nz - 1);
  KsLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += up256(bytes);
    return r;
  };
  L.poisson = take(poisson_ws);
  L.vzero = take(8 * nv);
  L.rho_in = take(8 * n);
  L.rho_out = take(8 * n);
  L.vh = take(8 * n);
  L.b = take(8 * n);
  L.t1 = take(8 * n);
  L.veff = take(8 * nv);
  L.part = take(8 * 2 * kKsGrid);
  L.res = take(8 * 4);
  const size_t mx = box->nx - 1, my = box->ny - 1, mz = box->nz - 1;
  L.sx = take(8 * mx * mx);
  L.sy = take(8 * my * my);
  L.sz = take(8 * mz * mz);
  L.ev = take(8 * (mx + my + mz));
  L.total = o;
  return L;
}

paro_opts_t poisson_opts(const paro_ks_opts_t* k) {
  paro_opts_t o;
  paro_default_opts(&o);
  o.N = 1;
  o.m = 0;
  o.precision = PARO_FP64;
  o.sigma_mode = 1;  // (1/2) K exactly: no shift
  o.sigma = 0.0;
  o.pcg_rtol = k->poisson_rtol;
  o.pcg_maxit = k->poisson_maxit > 0 ? k->poisson_maxit : 1;  // 0: direct
  return o;
}

#define KS_HIP(expr)                                                      \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      std::string m_ = std::string(#expr) + ": " + hipGetErrorString(e_);  \
      return set_error(PARO_EDEVICE, m_.c_str());                         \
    }                                                                     \
  } while (0)

}  // namespace
}  // namespace paro

using namespace paro;

extern "C" {

void paro_ks_default_opts(paro_ks_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_iter = 200;
  o->mixing = 0.3;
  o->occupancy = 2.0;
  o->scf_tol = 1e-8;
  o->poisson_rtol = 1e-12;
  o->poisson_maxit = 0;  // direct sine-transform solve
  o->kerker_q0 = 0.0;    // plain linear mixing
}

int paro_ks_query(const paro_box_t* box, size_t* workspace_bytes) {
  if (!box || !workspace_bytes) return set_error(PARO_EINVAL, "NULL argument");
  paro_ks_opts_t k;
  paro_ks_default_opts(&k);
  const paro_opts_t po = poisson_opts(&k);
  int64_t n = 0, z = 0;
  size_t ws = 0;
  const int rc = paro_query(box, &po, &n, &z, &ws);
  if (rc) return rc;
  *workspace_bytes = ks_layout(box, ws).total;
  return PARO_OK;
}

int paro_ks_solve(paro_problem* p, const double* d_Vext,
                  const paro_ks_opts_t* kopt, void* d_ws, size_t bytes,
                  const double* d_U0, double* d_lambda, double* d_U,
                  double* d_rho, double* h_history, void* stream,
                  paro_ks_report_t* report) {
  try {
    if (!p || !d_Vext || !kopt || !d_ws || !d_U0 || !d_lambda || !d_U)
      return set_error(PARO_EINVAL, "NULL argument to paro_ks_solve");
    if (((uintptr_t)d_ws & 255) != 0)
      return set_error(PARO_EINVAL, "workspace must be 256-byte aligned");
    if (!(kopt->mixing > 0.0) || kopt->mixing > 1.0 || kopt->max_iter < 1 ||
        !(kopt->occupancy > 0.0) || !(kopt->kerker_q0 >= 0.0) ||
        !std::isfinite(kopt->kerker_q0))
      return set_error(PARO_EINVAL, "bad Kohn-Sham options");
    const paro_box_t box = p->p.box;
    const paro_opts_t eig = p->p.opts;
    const int64_t n = p->p.n;
    const int Nt = p->p.Nt, N = p->p.N;
    const size_t nv = (size_t)(box.nx + 1) * (box.ny + 1) * (box.nz + 1);
    const paro_opts_t po = poisson_opts(kopt);
    int64_t pn = 0, pz = 0;
    size_t pws = 0;
    int rc = paro_query(&box, &po, &pn, &pz, &pws);
    if (rc) return rc;
    const KsLayout L = ks_layout(&box, pws);
    if (bytes < L.total)
      return set_error(PARO_ENOMEM, "Kohn-Sham workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)d_ws;
    double* vzero = (double*)(base + L.vzero);
    double* rho_in = (double*)(base + L.rho_in);
    double* rho_out = (double*)(base + L.rho_out);
    double* vh = (double*)(base + L.vh);
    double* b = (double*)(base + L.b);
    double* veff = (double*)(base + L.veff);
    double* part = (double*)(base + L.part);
    double* res = (double*)(base + L.res);
    double* t1 = (double*)(base + L.t1);
    double* Sx = (double*)(base + L.sx);
    double* Sy = (double*)(base + L.sy);
    double* Sz = (double*)(base + L.sz);
    double* ev = (double*)(base + L.ev);
    const int mx = box.nx - 1, my = box.ny - 1, mz = box.nz - 1;
    const bool direct = kopt->poisson_maxit <= 0;
    const bool kerker = kopt->kerker_q0 > 0.0;
    const double hx = (box.hi[0] - box.lo[0]) / box.nx;
    const double hy = (box.hi[1] - box.lo[1]) / box.ny;
    const double hz = (box.hi[2] - box.lo[2]) / box.nz;
    const double kerker_c = kopt->kerker_q0 * kopt->kerker_q0 * hx * hy * hz;
    const double dst_inv = 8.0 / ((double)(mx + 1) * (my + 1) * (mz + 1));
    if (direct || kerker) {
      hipLaunchKernelGGL(dst_tables_kernel, dim3(64), dim3(kBlock), 0, s, mx,
                         my, mz, hy * hz / hx, hz * hx / hy, hx * hy / hz, Sx,
                         Sy, Sz, ev);
      KS_HIP(hipGetLastError());
    }
    KS_HIP(hipMemsetAsync(vzero, 0, 8 * nv, s));
    KS_HIP(hipMemsetAsync(vh, 0, 8 * n, s));
    // The potential-free operator (1/2) K of the Poisson problem.
    paro_problem* pois = nullptr;
    rc = paro_assemble(&box, vzero, &po, base + L.poisson, pws, s, &pois);
    if (rc) return rc;
    struct Guard {
      paro_problem* q;
      ~Guard() { paro_destroy(q); }
    } guard{pois};
    // The caller's problem holds H(V_ext): Step 1 with the bare Hamiltonian.
    rc = paro_update_potential(p, d_Vext, s);
    if (rc) return rc;
    int st0 = 0;
    rc = paro::init_impl(p, d_U0, d_lambda, d_U, s, &st0);
    if (rc) return rc;
    if (st0 & ~paro::kStReorth)
      return paro::status_code(st0 & ~paro::kStReorth);
    paro_ks_report_t rep{};
    rep.status = PARO_ENOCONV;
    const auto t0 = std::chrono::steady_clock::now();
    const int gd = grid_for(n);
    const int gv = grid_for((long long)nv);
    if (h_history) h_history[0] = 0.0;
    for (int it = 0; it < kopt->max_iter; ++it) {
      // Density of the current orbitals, residual, mixing.
      hipLaunchKernelGGL(ks_density_kernel, dim3(gd), dim3(kBlock), 0, s,
                         (const double*)d_U, (long long)n, Nt, N,
                         kopt->occupancy, rho_out);
      if (kerker && it > 0) {
        // rho_in += mixing * (K + c I)^-1 K (rho_out - rho_in): the
        // residual to the sine basis (rho_out is free once e is formed),
        // the filter, and back.
        hipLaunchKernelGGL(ks_resid_vec_kernel, dim3(kKsGrid), dim3(kBlock),
                           0, s, (const double*)rho_out,
                           (const double*)rho_in, (long long)n, b, part);
        KS_HIP(hipGetLastError());
        KS_HIP(dst3(s, mx, my, mz, Sx, Sy, Sz, b, t1, rho_out, 1.0));
        hipLaunchKernelGGL(dst_kerker_kernel, dim3(gd), dim3(kBlock), 0, s,
                           rho_out, mx, my, mz, (const double*)ev, kerker_c);
        KS_HIP(hipGetLastError());
        KS_HIP(dst3(s, mx, my, mz, Sx, Sy, Sz, rho_out, t1, b, dst_inv));
        hipLaunchKernelGGL(ks_axpy_kernel, dim3(gd), dim3(kBlock), 0, s,
                           rho_in, (const double*)b, (long long)n,
                           kopt->mixing);
      } else {
        hipLaunchKernelGGL(ks_mix_kernel, dim3(kKsGrid), dim3(kBlock), 0, s,
                           (const double*)rho_out, rho_in, (long long)n,
                           kopt->mixing, it == 0 ? 1 : 0, part);
      }
      hipLaunchKernelGGL(ks_residual_kernel, dim3(1), dim3(kBlock), 0, s,
                         (const double*)part, res);
      KS_HIP(hipGetLastError());
      // Hartree: K V_H = 4 pi M rho_in.
      rc = paro_spmm(pois, 1, rho_in, b, 1, s);
      if (rc) return rc;
      if (direct) {
        // V_H = S^-1 diag(lambda)^-1 S (4 pi M rho), S^-1 = prod_a
        // 2 / (m_a + 1) S.
        KS_HIP(dst3(s, mx, my, mz, Sx, Sy, Sz, b, t1, vh, 4.0 * M_PI));
        hipLaunchKernelGGL(dst_divide_kernel, dim3(gd), dim3(kBlock), 0, s,
                           vh, mx, my, mz, (const double*)ev);
        KS_HIP(hipGetLastError());
        KS_HIP(dst3(s, mx, my, mz, Sx, Sy, Sz, vh, t1, b, dst_inv));
        KS_HIP(hipMemcpyAsync(vh, b, 8 * n, hipMemcpyDeviceToDevice, s));
      } else {
        // (1/2) K V_H = 2 pi M rho_in by PCG, warm-started from the last V_H.
        hipLaunchKernelGGL(ks_scale_kernel, dim3(gd), dim3(kBlock), 0, s, b,
                           (long long)n, 2.0 * M_PI);
        KS_HIP(hipGetLastError());
        int32_t pit = 0;
        rc = paro_pcg(pois, b, vh, 1, &pit, s);
        if (rc) return rc;
        rep.poisson_iters += pit;
      }
      // Effective potential and the values-only re-assembly.
      hipLaunchKernelGGL(ks_potential_kernel, dim3(gv), dim3(kBlock), 0, s,
                         d_Vext, (const double*)vh, (const double*)rho_in,
                         box.nx, box.ny, box.nz, veff);
      KS_HIP(hipGetLastError());
      rc = paro_update_potential(p, veff, s);
      if (rc) return rc;
      // One ParO step with H(V_eff) for Steps 3 and 4.
      paro_report_t r{};
      rc = paro_step(p, d_lambda, d_U, s, &r);
      if (rc != PARO_OK && rc != PARO_ENOCONV) return rc;
      double hres[2];
      KS_HIP(hipMemcpyAsync(hres, res, sizeof hres, hipMemcpyDeviceToHost, s));
      KS_HIP(hipStreamSynchronize(s));
      rep.iterations = it + 1;
      rep.paro_pcg_iters += r.pcg_iters;
      rep.max_dlambda = r.max_dlambda;
      rep.max_resid = r.max_resid;
      rep.sigma = r.sigma;
      if (it > 0) {
        rep.residual = hres[1] > 0.0 ? std::sqrt(hres[0] / hres[1]) : 0.0;
        if (h_history) h_history[it] = rep.residual;
        if (rep.residual <= kopt->scf_tol && r.max_dlambda <= eig.lambda_tol &&
            r.max_resid <= eig.resid_tol) {
          rep.status = PARO_OK;
          break;
        }
      }
    }
    if (d_rho)
      KS_HIP(hipMemcpyAsync(d_rho, rho_in, 8 * n, hipMemcpyDeviceToDevice, s));
    KS_HIP(hipStreamSynchronize(s));
    rep.seconds = std::chrono::duration<double>(
                      std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    if (rep.status != PARO_OK)
      set_error(PARO_ENOCONV, "Kohn-Sham iteration reached max_iter");
    return rep.status;
  } catch (...) {
    return set_error(PARO_EDEVICE, "unexpected exception in paro_ks_solve");
  }
}

}  // extern "C"
