// The P1 stencil of a uniform Kuhn mesh and the closed form of its
// coefficients in the nodal potential.
//
// Sec. 2: the source operator is a(w, v) = 1/2 (grad w, grad v) + (V_h w, v)
// - s (w, v) on continuous piecewise-linear functions, V_h the nodal
// interpolant of the potential.  On a uniform Kuhn mesh (every box cell cut
// into the six tetrahedra along its main diagonal) the stiffness and mass
// parts of a row are the same at every interior vertex; only the potential
// part varies, and it is linear in the potential values at the 15 vertices
// that share a tetrahedron with the row vertex.  With lambda_a the
// barycentric coordinates of a tetrahedron of volume vol, the integral of a
// product of three of them is vol/20 (all equal), vol/60 (two equal) or
// vol/120 (all different), so
//   (V_h phi_a, phi_b)_e = vol/120 (sum_k V_k + V_a + V_b)   (a != b)
//   (V_h phi_a, phi_a)_e = vol/60  (sum_k V_k + 2 V_a).
// Summed over the tetrahedra around the pair (row vertex, neighbour s),
// every weight is an integer multiple of vol/60; the table is derived here
// at compile time from the tetrahedra themselves.  A row's coefficient is
//   a_s = c0_s + vol/60 sum_k W[s][k] V_k,
// c0_s = 1/2 K_s - s M_s the constant stiffness and shifted mass part,
// and 0 where neighbour s lies outside the box (Dirichlet boundary).
//
// The assembly writes these values in stencil order and the matrix-free
// CG SpMM forms them again on the fly; both go through kuhn_row, so the
// two operators are bitwise the same.
#pragma once

#include <hip/hip_runtime.h>

namespace paro {

// Offsets (dx, dy, dz) of the 15 stencil vertices in ascending linear
// order (x fastest); offset 7 is the row vertex itself.
constexpr int kKuhnOff[15][3] = {
    {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
    {0, -1, 0},   {-1, 0, 0},  {0, 0, 0},   {1, 0, 0},  {0, 1, 0},
    {1, 1, 0},    {0, 0, 1},   {1, 0, 1},   {0, 1, 1},  {1, 1, 1}};

struct KuhnTable {
  int w[15][15];  // potential weights of pair s on vertex k, units vol/60
  int nel[15];    // tetrahedra containing the row vertex and neighbour s
};

// Local vertex a of the tetrahedron with axis order q of a unit cube:
// (0,0,0), e_q0, e_q0 + e_q1, (1,1,1).
constexpr void kuhn_local(int q, int a, int (&o)[3]) {
  constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                              {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  o[0] = o[1] = o[2] = 0;
  if (a >= 1) o[perm[q][0]] = 1;
  if (a >= 2) o[perm[q][1]] = 1;
  if (a == 3) o[0] = o[1] = o[2] = 1;
}

constexpr int kuhn_offset_index(int dx, int dy, int dz) {
  for (int s = 0; s < 15; ++s)
    if (kKuhnOff[s][0] == dx && kKuhnOff[s][1] == dy && kKuhnOff[s][2] == dz)
      return s;
  return -1;
}

// Every tetrahedron around the row vertex: the 8 cubes that have it as a
// corner times the 6 tetrahedra of a cube that contain that corner.
constexpr KuhnTable make_kuhn_table() {
  KuhnTable t{};
  int w120[15][15] = {};
  for (int s = 0; s < 15; ++s)
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
        ++t.nel[s];
        for (int a = 0; a < 4; ++a) {
          const int k = kuhn_offset_index(L[a][0] - cv[0], L[a][1] - cv[1],
                                          L[a][2] - cv[2]);
          // In units of vol/120: (1 + [a = la] + [a = lb]) off the
          // diagonal, 2 (1 + 2 [a = la]) on it.
          w120[s][k] += la == lb ? 2 * (1 + 2 * (a == la))
                                 : 1 + (a == la) + (a == lb);
        }
      }
    }
  for (int s = 0; s < 15; ++s)
    for (int k = 0; k < 15; ++k) t.w[s][k] = w120[s][k] / 2;
  return t;
}

constexpr bool kuhn_table_even() {
  // Checks of the derivation: the row vertex lies in all 24 tetrahedra
  // around it, and with V = 1 the weights of a pair add up to its mass
  // integral over each of its tetrahedra, (4 + 2) / 120 vol = 3 (vol/60)
  // off the diagonal and (4 + 2) / 60 vol = 6 (vol/60) on it; every
  // summed weight is even in units of vol/120 (the halving is exact).
  const KuhnTable t = make_kuhn_table();
  if (t.nel[7] != 24) return false;
  for (int s = 0; s < 15; ++s) {
    int sum = 0;
    for (int k = 0; k < 15; ++k) sum += t.w[s][k];
    if (sum != (s == 7 ? 6 : 3) * t.nel[s]) return false;
  }
  return true;
}
static_assert(kuhn_table_even(), "Kuhn potential weights");

inline constexpr KuhnTable kKuhn = make_kuhn_table();

// The constants of a problem's stencil as the device reads them (the
// workspace copy written by the assembly): c0[15], vol / 60, then the mass
// coefficients, which depend on the offset only through the number of
// tetrahedra around the pair (vol / 20 each, vol / 10 each on the
// diagonal): M of a 4-tetrahedron pair, of a 6-tetrahedron pair, of the
// diagonal.
constexpr int kKcVol60 = 15;
constexpr int kKcM4 = 16, kKcM6 = 17, kKcMDiag = 18;
constexpr int kKcCount = 19;
// Slot of the mass coefficient of offset s in that array.
constexpr int kuhn_mass_slot(int s) {
  return s == 7 ? kKcMDiag : (kKuhn.nel[s] == 4 ? kKcM4 : kKcM6);
}
static_assert(kKuhn.nel[0] == 6 && kKuhn.nel[1] == 4, "Kuhn pair classes");

// Coefficient S of a row from the potential v[k] at its stencil vertices:
// c0[S] + vol60 sum_k W[S][k] v[k] (ascending k), or 0 where bit S of
// `mask` (neighbour inside the box) is clear.
template <int S>
__host__ __device__ __forceinline__ double kuhn_coeff(const double (&v)[15],
                                                      const double* c0,
                                                      double vol60,
                                                      unsigned mask) {
  // No contraction: the products and sums stay as written, so every
  // caller forms the same bits.
#pragma clang fp contract(off)
  double t = 0.0;
  bool first = true;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    const int w = kKuhn.w[S][k];
    if (w == 0) continue;
    if (first)
      t = w == 1 ? v[k] : (double)w * v[k];
    else
      t = w == 1 ? t + v[k] : __builtin_fma((double)w, v[k], t);
    first = false;
  }
  const double c = __builtin_fma(vol60, t, c0[S]);
  return (mask >> S) & 1u ? c : 0.0;
}

template <int S>
__host__ __device__ __forceinline__ void kuhn_row_from(const double (&v)[15],
                                                       const double* c0,
                                                       double vol60,
                                                       unsigned mask,
                                                       double (&a)[15]) {
  a[S] = kuhn_coeff<S>(v, c0, vol60, mask);
  if constexpr (S + 1 < 15) kuhn_row_from<S + 1>(v, c0, vol60, mask, a);
}

// All 15 coefficients of a row.
__host__ __device__ __forceinline__ void kuhn_row(const double (&v)[15],
                                                  const double* c0,
                                                  double vol60, unsigned mask,
                                                  double (&a)[15]) {
  kuhn_row_from<0>(v, c0, vol60, mask, a);
}

}  // namespace paro
