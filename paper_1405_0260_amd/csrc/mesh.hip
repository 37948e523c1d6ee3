// General bisection meshes of a box: Step 2 of Algorithm 3.1 with local
// refinement (Sec. 2.1: Solve -> Estimate -> Mark -> Refine).
//
// Host side (graph work): the uniform Kuhn mesh as the first bisection
// mesh, Maubach's tagged bisection with a conforming closure, and the
// tables the device needs (dof numbering, CSR pattern, the incident
// elements of every row, face neighbours).  Device side: the operator's
// values by a row gather over the incident elements (one thread per row,
// elements in ascending order: no atomics, the same bits on every run) and
// the transfer of orbitals to a refined mesh.
//
// Bisection (the paper defers to the literature for it): an element is an
// ordered vertex list (x0, x1, x2, x3) with a tag k in {1, 2, 3}; its
// refinement edge is (x0, xk); it is cut at the midpoint z of that edge
// into (x0, .., x_{k-1}, z, x_{k+1}, .., x3) and (x1, .., xk, z,
// x_{k+1}, .., x3), both tagged k - 1 (3 after 1).  The Kuhn elements
// (v, v + e_p0, v + e_p0 + e_p1, v + (1,1,1)) start with tag 3, so three
// rounds of bisection of everything halve the grid.  Before an element is
// cut at an edge, every element around that edge whose refinement edge
// differs is bisected first (recursively); then all elements around the
// edge are cut at it, so no hanging vertex remains.  Surviving elements
// keep their order and the children follow in creation order; old
// vertices keep their indices and new ones follow in creation order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "paro_internal.h"

namespace paro {
namespace {

uint64_t edge_key(int32_t a, int32_t b) {
  const uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
  return ((uint64_t)lo << 32) | hi;
}

// Vertex of the uniform mesh at grid point (i, j, k).
int32_t grid_vertex(const paro_box_t& b, int i, int j, int k) {
  return i + (b.nx + 1) * (j + (b.ny + 1) * k);
}

MeshData kuhn(const paro_box_t& b) {
  MeshData m;
  for (int a = 0; a < 3; ++a) {
    m.lo[a] = b.lo[a];
    m.hi[a] = b.hi[a];
  }
  const int nc[3] = {b.nx, b.ny, b.nz};
  double h[3];
  for (int a = 0; a < 3; ++a) h[a] = (b.hi[a] - b.lo[a]) / nc[a];
  const int64_t nv = (int64_t)(b.nx + 1) * (b.ny + 1) * (b.nz + 1);
  m.X.resize(3 * nv);
  for (int k = 0; k <= b.nz; ++k)
    for (int j = 0; j <= b.ny; ++j)
      for (int i = 0; i <= b.nx; ++i) {
        double* x = &m.X[3 * (size_t)grid_vertex(b, i, j, k)];
        x[0] = b.lo[0] + h[0] * i;
        x[1] = b.lo[1] + h[1] * j;
        x[2] = b.lo[2] + h[2] * k;
      }
  // Six elements per cell, one per axis order (p0, p1, p2), the orders in
  // lexicographic sequence; element q of cell c is at q ncell + c.
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                           {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  const int64_t ncell = (int64_t)b.nx * b.ny * b.nz;
  m.tets.resize(4 * 6 * ncell);
  m.tags.assign(6 * ncell, 3);
  for (int q = 0; q < 6; ++q)
    for (int ck = 0; ck < b.nz; ++ck)
      for (int cj = 0; cj < b.ny; ++cj)
        for (int ci = 0; ci < b.nx; ++ci) {
          const int64_t c = ci + (int64_t)b.nx * (cj + (int64_t)b.ny * ck);
          int o[3] = {0, 0, 0};
          int32_t* t = &m.tets[4 * (size_t)(q * ncell + c)];
          t[0] = grid_vertex(b, ci, cj, ck);
          o[perms[q][0]] = 1;
          t[1] = grid_vertex(b, ci + o[0], cj + o[1], ck + o[2]);
          o[perms[q][1]] = 1;
          t[2] = grid_vertex(b, ci + o[0], cj + o[1], ck + o[2]);
          t[3] = grid_vertex(b, ci + 1, cj + 1, ck + 1);
        }
  m.parents.assign(2 * nv, -1);
  return m;
}

// Maubach bisection with the conforming closure (see the file notes).
// The elements around an edge (a, b) are found from the elements at
// vertex a (a per-vertex list kept up to date as elements are cut), by
// testing each for vertex b.
class Refiner {
 public:
  explicit Refiner(const MeshData& in) : m_(in) {
    const int64_t ne = in.ne(), nv = in.nv();
    el_.resize(ne);
    std::vector<int32_t> deg(nv, 0);
    for (int64_t e = 0; e < ne; ++e) {
      for (int a = 0; a < 4; ++a) {
        el_[e].v[a] = in.tets[4 * e + a];
        ++deg[el_[e].v[a]];
      }
      el_[e].tag = in.tags[e];
      el_[e].alive = true;
    }
    at_.resize(nv);
    for (int64_t v = 0; v < nv; ++v) at_[v].reserve(deg[v] + 4);
    for (int64_t e = 0; e < ne; ++e) link((int32_t)e);
  }

  void bisect(int32_t i) {
    const int32_t a = el_[i].v[0], b = el_[i].v[el_[i].tag];
    const uint64_t e = edge_key(a, b);
    for (;;) {
      around(a, b, &tmp_);
      int32_t bad = -1;
      for (int32_t j : tmp_)
        if (ref_edge(j) != e) {
          bad = j;
          break;
        }
      if (bad < 0) break;
      bisect(bad);
    }
    around(a, b, &tmp_);
    const std::vector<int32_t> all = tmp_;
    for (int32_t j : all) cut(j);
  }

  bool alive(int64_t i) const { return el_[i].alive; }

  MeshData result() const {
    MeshData out;
    std::memcpy(out.lo, m_.lo, sizeof out.lo);
    std::memcpy(out.hi, m_.hi, sizeof out.hi);
    out.X = m_.X;
    out.parents = m_.parents;
    for (const Elem& e : el_) {
      if (!e.alive) continue;
      out.tets.insert(out.tets.end(), e.v, e.v + 4);
      out.tags.push_back(e.tag);
    }
    return out;
  }

 private:
  struct Elem {
    int32_t v[4];
    int32_t tag;
    bool alive;
  };

  uint64_t ref_edge(int32_t i) const {
    return edge_key(el_[i].v[0], el_[i].v[el_[i].tag]);
  }

  // Live elements with both a and b among their corners.
  void around(int32_t a, int32_t b, std::vector<int32_t>* out) const {
    out->clear();
    for (int32_t j : at_[a]) {
      const int32_t* v = el_[j].v;
      if (v[0] == b || v[1] == b || v[2] == b || v[3] == b) out->push_back(j);
    }
  }

  void link(int32_t i) {
    for (int a = 0; a < 4; ++a) at_[el_[i].v[a]].push_back(i);
  }

  void unlink(int32_t i) {
    for (int a = 0; a < 4; ++a) {
      std::vector<int32_t>& l = at_[el_[i].v[a]];
      auto it = std::find(l.begin(), l.end(), i);
      if (it != l.end()) {
        *it = l.back();
        l.pop_back();
      }
    }
  }

  int32_t midpoint(int32_t a, int32_t b) {
    const uint64_t k = edge_key(a, b);
    auto it = mid_.find(k);
    if (it != mid_.end()) return it->second;
    const int32_t z = (int32_t)m_.nv();
    for (int c = 0; c < 3; ++c)
      m_.X.push_back(0.5 * (m_.X[3 * (size_t)a + c] + m_.X[3 * (size_t)b + c]));
    m_.parents.push_back(std::min(a, b));
    m_.parents.push_back(std::max(a, b));
    at_.emplace_back();
    mid_[k] = z;
    return z;
  }

  void cut(int32_t i) {
    const Elem t = el_[i];
    const int k = t.tag;
    const int32_t z = midpoint(t.v[0], t.v[k]);
    Elem c1, c2;
    int n1 = 0, n2 = 0;
    for (int a = 0; a < 4; ++a) {
      if (a != k) c1.v[n1++] = t.v[a];
      else c1.v[n1++] = z;
    }
    for (int a = 1; a <= k; ++a) c2.v[n2++] = t.v[a];
    c2.v[n2++] = z;
    for (int a = k + 1; a < 4; ++a) c2.v[n2++] = t.v[a];
    c1.tag = c2.tag = k > 1 ? k - 1 : 3;
    c1.alive = c2.alive = true;
    unlink(i);
    el_[i].alive = false;
    el_.push_back(c1);
    link((int32_t)el_.size() - 1);
    el_.push_back(c2);
    link((int32_t)el_.size() - 1);
  }

  MeshData m_;
  std::vector<Elem> el_;
  std::vector<std::vector<int32_t>> at_;  // live elements at each vertex
  std::unordered_map<uint64_t, int32_t> mid_;
  std::vector<int32_t> tmp_;
};

bool inside_box(const MeshData& m, const double* x) {
  for (int a = 0; a < 3; ++a) {
    const double w = 1e-12 * (m.hi[a] - m.lo[a]);
    if (!(x[a] > m.lo[a] + w && x[a] < m.hi[a] - w)) return false;
  }
  return true;
}

int check_mesh(const MeshData& m) {
  const int64_t nv = m.nv(), ne = m.ne();
  if (nv < 4 || ne < 1) return set_error(PARO_EINVAL, "mesh too small");
  if ((int64_t)m.tets.size() != 4 * ne || (int64_t)m.parents.size() != 2 * nv)
    return set_error(PARO_EINVAL, "mesh arrays of inconsistent sizes");
  if (nv >= ((int64_t)1 << 31) || 4 * ne >= ((int64_t)1 << 31))
    return set_error(PARO_EINVAL, "mesh exceeds 32-bit indices");
  for (double x : m.X)
    if (!std::isfinite(x)) return set_error(PARO_EINVAL, "non-finite vertex");
  for (int64_t e = 0; e < ne; ++e) {
    if (m.tags[e] < 1 || m.tags[e] > 3)
      return set_error(PARO_EINVAL, "element tag outside 1..3");
    for (int a = 0; a < 4; ++a) {
      const int32_t v = m.tets[4 * e + a];
      if (v < 0 || v >= nv)
        return set_error(PARO_EINVAL, "element vertex out of range");
      for (int b = a + 1; b < 4; ++b)
        if (m.tets[4 * e + b] == v)
          return set_error(PARO_EINVAL, "element with a repeated vertex");
    }
  }
  for (int64_t v = 0; v < nv; ++v) {
    const int32_t a = m.parents[2 * v], b = m.parents[2 * v + 1];
    if ((a < 0) != (b < 0) || a >= v || b >= v)
      return set_error(PARO_EINVAL,
                       "parents must be two older vertices, or -1, -1");
  }
  return PARO_OK;
}

// ------------------------------------------------------------------------
// Device: operator values by row gather.
// ------------------------------------------------------------------------

// Barycentric gradients (rows) and volume of an element.
__device__ void element_geometry(const double* __restrict__ X,
                                 const int32_t* v, double g[4][3],
                                 double* vol) {
  double e[3][3];  // rows: x_a - x_0
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c)
      e[a][c] = X[3 * (size_t)v[a + 1] + c] - X[3 * (size_t)v[0] + c];
  // Cofactors: (E^{-1})[c][a] = cof[a][c] / det, and grad lambda_{a+1} is
  // column a of E^{-1}.
  double cof[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      cof[a][c] = e[a1][c1] * e[a2][c2] - e[a1][c2] * e[a2][c1];
    }
  const double det = e[0][0] * cof[0][0] + e[0][1] * cof[0][1] +
                     e[0][2] * cof[0][2];
  *vol = fabs(det) / 6.0;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) g[a + 1][c] = cof[a][c] / det;
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
}

__global__ void __launch_bounds__(kBlock) mesh_assemble_kernel(
    long long n, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ colidx, const int32_t* __restrict__ inc_ptr,
    const int32_t* __restrict__ inc, const int32_t* __restrict__ tets,
    const double* __restrict__ X, const double* __restrict__ V,
    const int32_t* __restrict__ dof, double sigma, double* __restrict__ valA,
    double* __restrict__ valM, double* __restrict__ dinv) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r >= n) return;
  const int j0 = rowptr[r], j1 = rowptr[r + 1];
  for (int j = j0; j < j1; ++j) valA[j] = valM[j] = 0.0;
  for (int k = inc_ptr[r]; k < inc_ptr[r + 1]; ++k) {
    const int32_t e = inc[2 * k], a = inc[2 * k + 1];
    int32_t v[4];
    double Ve[4];
    for (int c = 0; c < 4; ++c) {
      v[c] = tets[4 * (size_t)e + c];
      Ve[c] = V[v[c]];
    }
    double g[4][3], vol;
    element_geometry(X, v, g, &vol);
    for (int b = 0; b < 4; ++b) {
      const int32_t col = dof[v[b]];
      if (col < 0) continue;
      const double K = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] +
                              g[a][2] * g[b][2]);
      const double M = vol * (a == b ? 2.0 : 1.0) / 20.0;
      // int_T lambda_a lambda_b lambda_c / |T| = prod(multiplicity!) / 120.
      double mv = 0.0;
      for (int c = 0; c < 4; ++c) {
        const int same = (a == b) + (a == c) + (b == c);
        const double w = same == 3 ? 6.0 : (same == 1 ? 2.0 : 1.0);
        mv += Ve[c] * w;
      }
      const double H = 0.5 * K + vol * mv / 120.0;
      int j = j0;
      while (j < j1 && colidx[j] != col) ++j;
      if (j == j1) continue;  // not reached: the pattern has every pair
      valA[j] += H - sigma * M;
      valM[j] += M;
    }
  }
  int jd = j0;
  while (jd < j1 && colidx[jd] != (int32_t)r) ++jd;
  dinv[r] = jd < j1 ? 1.0 / valA[jd] : 0.0;
}

// ------------------------------------------------------------------------
// Device: transfer to a refined mesh (P1 interpolation, exact: the coarse
// space lies in the fine one).  Old interior vertices keep their values; a
// new vertex takes the mean of the two ends of the edge it halves (0 at
// the boundary), generation by generation so that both ends are final.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) prolong_copy_kernel(
    long long nvc, const int32_t* __restrict__ dofc,
    const int32_t* __restrict__ doff, const double* __restrict__ Uc,
    double* __restrict__ Uf, int ncols) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long v = t / ncols;
  const int c = (int)(t - v * ncols);
  if (v >= nvc) return;
  const int32_t dc = dofc[v], df = doff[v];
  if (df >= 0) Uf[(size_t)df * ncols + c] = dc >= 0 ? Uc[(size_t)dc * ncols + c] : 0.0;
}

__global__ void __launch_bounds__(kBlock) prolong_level_kernel(
    int count, const int32_t* __restrict__ verts,
    const int32_t* __restrict__ parents, const int32_t* __restrict__ doff,
    double* __restrict__ Uf, int ncols) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long i = t / ncols;
  const int c = (int)(t - i * ncols);
  if (i >= count) return;
  const int32_t v = verts[i];
  const int32_t df = doff[v];
  if (df < 0) return;
  const int32_t a = parents[2 * (size_t)v], b = parents[2 * (size_t)v + 1];
  const double ua = doff[a] >= 0 ? Uf[(size_t)doff[a] * ncols + c] : 0.0;
  const double ub = doff[b] >= 0 ? Uf[(size_t)doff[b] * ncols + c] : 0.0;
  Uf[(size_t)df * ncols + c] = 0.5 * (ua + ub);
}

std::vector<int32_t> dof_of(const MeshData& m, int64_t* n) {
  std::vector<int32_t> d(m.nv(), -1);
  int32_t k = 0;
  for (int64_t v = 0; v < m.nv(); ++v)
    if (inside_box(m, &m.X[3 * v])) d[v] = k++;
  *n = k;
  return d;
}

// Prolongation workspace: dof maps of both meshes, the fine mesh's
// parents, and its new vertices ordered by generation.
struct ProlongLayout {
  size_t dofc, doff, parents, order, total;
};
ProlongLayout prolong_layout(int64_t nvc, int64_t nvf) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  ProlongLayout L;
  size_t o = 0;
  L.dofc = o;
  o += up(sizeof(int32_t) * nvc);
  L.doff = o;
  o += up(sizeof(int32_t) * nvf);
  L.parents = o;
  o += up(sizeof(int32_t) * 2 * nvf);
  L.order = o;
  o += up(sizeof(int32_t) * (nvf - nvc + 1));
  L.total = o;
  return L;
}

}  // namespace

int mesh_ops(const MeshData& m, MeshOps* out) {
  MeshOps& o = *out;
  o.dof = dof_of(m, &o.n);
  const int64_t ne = m.ne(), n = o.n;
  if (n < 1) return set_error(PARO_EINVAL, "mesh has no interior vertex");
  // Incident (element, corner) pairs of every dof row, elements ascending.
  o.inc_ptr.assign(n + 1, 0);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a) {
      const int32_t d = o.dof[m.tets[4 * e + a]];
      if (d >= 0) ++o.inc_ptr[d + 1];
    }
  for (int64_t r = 0; r < n; ++r) o.inc_ptr[r + 1] += o.inc_ptr[r];
  o.inc.assign(2 * (size_t)o.inc_ptr[n], 0);
  {
    std::vector<int32_t> fill(o.inc_ptr.begin(), o.inc_ptr.end() - 1);
    for (int64_t e = 0; e < ne; ++e)
      for (int a = 0; a < 4; ++a) {
        const int32_t d = o.dof[m.tets[4 * e + a]];
        if (d < 0) continue;
        const int32_t k = fill[d]++;
        o.inc[2 * (size_t)k] = (int32_t)e;
        o.inc[2 * (size_t)k + 1] = a;
      }
  }
  // CSR pattern: the dofs of the incident elements' corners.
  o.rowptr.assign(n + 1, 0);
  o.colidx.clear();
  std::vector<int32_t> cols;
  for (int64_t r = 0; r < n; ++r) {
    cols.clear();
    for (int32_t k = o.inc_ptr[r]; k < o.inc_ptr[r + 1]; ++k) {
      const int32_t e = o.inc[2 * (size_t)k];
      for (int b = 0; b < 4; ++b) {
        const int32_t d = o.dof[m.tets[4 * (size_t)e + b]];
        if (d >= 0) cols.push_back(d);
      }
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    o.colidx.insert(o.colidx.end(), cols.begin(), cols.end());
    if (o.colidx.size() >= ((size_t)1 << 31))
      return set_error(PARO_EINVAL, "nnz exceeds 32-bit indices");
    o.rowptr[r + 1] = (int32_t)o.colidx.size();
  }
  // Face neighbours: the face opposite corner a as a sorted triple.
  struct Face {
    int32_t v[3];
    int32_t owner;  // 4 e + a
  };
  std::vector<Face> faces(4 * (size_t)ne);
  for (int64_t e = 0; e < ne; ++e)
    for (int a = 0; a < 4; ++a) {
      Face& f = faces[4 * e + a];
      int k = 0;
      for (int b = 0; b < 4; ++b)
        if (b != a) f.v[k++] = m.tets[4 * e + b];
      std::sort(f.v, f.v + 3);
      f.owner = (int32_t)(4 * e + a);
    }
  std::sort(faces.begin(), faces.end(), [](const Face& x, const Face& y) {
    if (x.v[0] != y.v[0]) return x.v[0] < y.v[0];
    if (x.v[1] != y.v[1]) return x.v[1] < y.v[1];
    if (x.v[2] != y.v[2]) return x.v[2] < y.v[2];
    return x.owner < y.owner;
  });
  o.nbr.assign(4 * (size_t)ne, -1);
  for (size_t i = 0; i + 1 < faces.size(); ++i) {
    const Face &x = faces[i], &y = faces[i + 1];
    if (x.v[0] == y.v[0] && x.v[1] == y.v[1] && x.v[2] == y.v[2]) {
      o.nbr[x.owner] = y.owner / 4;
      o.nbr[y.owner] = x.owner / 4;
    }
  }
  return PARO_OK;
}

hipError_t launch_mesh_assemble(Problem& p, hipStream_t s) {
  const int grid = (int)((p.n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(mesh_assemble_kernel, dim3(grid), dim3(kBlock), 0, s,
                     (long long)p.n, p.rowptr, p.colidx, p.inc_ptr, p.inc,
                     p.tets, p.Xv, p.Vv, p.dofmap, p.sigma, p.valA, p.valM,
                     p.dinv);
  return hipGetLastError();
}

}  // namespace paro

using namespace paro;

extern "C" {

int paro_mesh_create(const paro_box_t* box, paro_mesh** out) {
  try {
    if (!box || !out) return set_error(PARO_EINVAL, "NULL argument");
    *out = nullptr;
    if (box->nx < 2 || box->ny < 2 || box->nz < 2)
      return set_error(PARO_EINVAL, "need at least 2 cells per axis");
    for (int a = 0; a < 3; ++a)
      if (!(box->hi[a] > box->lo[a]) || !std::isfinite(box->lo[a]) ||
          !std::isfinite(box->hi[a]))
        return set_error(PARO_EINVAL, "box: need finite lo < hi");
    const int64_t ne = 6 * (int64_t)box->nx * box->ny * box->nz;
    if (4 * ne >= ((int64_t)1 << 31))
      return set_error(PARO_EINVAL, "mesh exceeds 32-bit indices");
    paro_mesh* m = new (std::nothrow) paro_mesh();
    if (!m) return set_error(PARO_EDEVICE, "host allocation failed");
    m->m = kuhn(*box);
    *out = m;
    return PARO_OK;
  } catch (...) {
    return set_error(PARO_EDEVICE, "host allocation failed");
  }
}

int paro_mesh_from_arrays(const paro_box_t* box, int64_t nv, const double* X,
                          int64_t ne, const int32_t* tets,
                          const int32_t* tags, const int32_t* parents,
                          paro_mesh** out) {
  try {
    if (!box || !X || !tets || !tags || !out)
      return set_error(PARO_EINVAL, "NULL argument");
    *out = nullptr;
    if (nv < 4 || ne < 1) return set_error(PARO_EINVAL, "mesh too small");
    MeshData m;
    for (int a = 0; a < 3; ++a) {
      if (!(box->hi[a] > box->lo[a]))
        return set_error(PARO_EINVAL, "box: need lo < hi");
      m.lo[a] = box->lo[a];
      m.hi[a] = box->hi[a];
    }
    m.X.assign(X, X + 3 * nv);
    m.tets.assign(tets, tets + 4 * ne);
    m.tags.assign(tags, tags + ne);
    if (parents)
      m.parents.assign(parents, parents + 2 * nv);
    else
      m.parents.assign(2 * nv, -1);
    const int rc = check_mesh(m);
    if (rc) return rc;
    paro_mesh* h = new (std::nothrow) paro_mesh();
    if (!h) return set_error(PARO_EDEVICE, "host allocation failed");
    h->m = std::move(m);
    *out = h;
    return PARO_OK;
  } catch (...) {
    return set_error(PARO_EDEVICE, "host allocation failed");
  }
}

int paro_mesh_info(const paro_mesh* m, int64_t* nv, int64_t* ne,
                   int64_t* n_dof) {
  if (!m) return set_error(PARO_EINVAL, "NULL mesh");
  if (nv) *nv = m->m.nv();
  if (ne) *ne = m->m.ne();
  if (n_dof) {
    int64_t n = 0;
    (void)dof_of(m->m, &n);
    *n_dof = n;
  }
  return PARO_OK;
}

int paro_mesh_arrays(const paro_mesh* m, double* X, int32_t* tets,
                     int32_t* tags, int32_t* parents, int32_t* dof) {
  try {
    if (!m) return set_error(PARO_EINVAL, "NULL mesh");
    const MeshData& d = m->m;
    if (X) std::memcpy(X, d.X.data(), sizeof(double) * d.X.size());
    if (tets) std::memcpy(tets, d.tets.data(), sizeof(int32_t) * d.tets.size());
    if (tags) std::memcpy(tags, d.tags.data(), sizeof(int32_t) * d.tags.size());
    if (parents)
      std::memcpy(parents, d.parents.data(),
                  sizeof(int32_t) * d.parents.size());
    if (dof) {
      int64_t n = 0;
      const std::vector<int32_t> v = dof_of(d, &n);
      std::memcpy(dof, v.data(), sizeof(int32_t) * v.size());
    }
    return PARO_OK;
  } catch (...) {
    return set_error(PARO_EDEVICE, "host allocation failed");
  }
}

int paro_mesh_refine(const paro_mesh* m, const uint8_t* marked,
                     paro_mesh** out) {
  try {
    if (!m || !marked || !out) return set_error(PARO_EINVAL, "NULL argument");
    *out = nullptr;
    Refiner r(m->m);
    const int64_t ne = m->m.ne();
    for (int64_t e = 0; e < ne; ++e)
      if (marked[e] && r.alive(e)) r.bisect((int32_t)e);
    MeshData res = r.result();
    if (res.nv() >= ((int64_t)1 << 31) || 4 * res.ne() >= ((int64_t)1 << 31))
      return set_error(PARO_EINVAL, "refined mesh exceeds 32-bit indices");
    paro_mesh* h = new (std::nothrow) paro_mesh();
    if (!h) return set_error(PARO_EDEVICE, "host allocation failed");
    h->m = std::move(res);
    *out = h;
    return PARO_OK;
  } catch (...) {
    return set_error(PARO_EDEVICE, "host allocation failed");
  }
}

void paro_mesh_destroy(paro_mesh* m) { delete m; }

size_t paro_mesh_prolong_workspace_bytes(const paro_mesh* coarse,
                                         const paro_mesh* fine) {
  if (!coarse || !fine || fine->m.nv() < coarse->m.nv()) return 0;
  return prolong_layout(coarse->m.nv(), fine->m.nv()).total;
}

int paro_mesh_prolong(const paro_mesh* coarse, const paro_mesh* fine,
                      const double* d_Uc, double* d_Uf, int32_t ncols,
                      void* d_ws, size_t bytes, void* stream) {
  try {
    if (!coarse || !fine || !d_Uc || !d_Uf || !d_ws)
      return set_error(PARO_EINVAL, "NULL argument");
    if (ncols < 1) return set_error(PARO_EINVAL, "ncols must be >= 1");
    const MeshData &c = coarse->m, &f = fine->m;
    const int64_t nvc = c.nv(), nvf = f.nv();
    if (nvf < nvc)
      return set_error(PARO_EINVAL, "the fine mesh has fewer vertices");
    for (int64_t v = 0; v < 3 * nvc; ++v)
      if (c.X[v] != f.X[v])
        return set_error(PARO_EINVAL,
                         "the fine mesh does not refine the coarse one "
                         "(old vertices must keep their indices)");
    for (int64_t v = nvc; v < nvf; ++v)
      if (f.parents[2 * v] < 0)
        return set_error(PARO_EINVAL, "a new vertex of the fine mesh has no parents");
    const ProlongLayout L = prolong_layout(nvc, nvf);
    if (((uintptr_t)d_ws & 255) != 0)
      return set_error(PARO_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < L.total)
      return set_error(PARO_ENOMEM, "prolongation workspace too small");
    int64_t nc_ = 0, nf_ = 0;
    const std::vector<int32_t> dofc = dof_of(c, &nc_), doff = dof_of(f, &nf_);
    // Generations of the new vertices: 1 + the older of the parents'.
    std::vector<int32_t> gen(nvf, 0);
    int32_t maxg = 0;
    for (int64_t v = nvc; v < nvf; ++v) {
      const int32_t a = f.parents[2 * v], b = f.parents[2 * v + 1];
      gen[v] = 1 + std::max(gen[a], gen[b]);
      maxg = std::max(maxg, gen[v]);
    }
    std::vector<int32_t> start(maxg + 2, 0), order(nvf - nvc);
    for (int64_t v = nvc; v < nvf; ++v) ++start[gen[v] + 1];
    for (int g = 0; g <= maxg; ++g) start[g + 1] += start[g];
    {
      std::vector<int32_t> fill(start.begin(), start.end() - 1);
      for (int64_t v = nvc; v < nvf; ++v) order[fill[gen[v]]++] = (int32_t)v;
    }
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)d_ws;
    int32_t* d_dofc = (int32_t*)(base + L.dofc);
    int32_t* d_doff = (int32_t*)(base + L.doff);
    int32_t* d_par = (int32_t*)(base + L.parents);
    int32_t* d_ord = (int32_t*)(base + L.order);
    auto up = [&](void* dst, const void* src, size_t n) {
      return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
    };
    if (up(d_dofc, dofc.data(), sizeof(int32_t) * nvc) != hipSuccess ||
        up(d_doff, doff.data(), sizeof(int32_t) * nvf) != hipSuccess ||
        up(d_par, f.parents.data(), sizeof(int32_t) * 2 * nvf) !=
            hipSuccess ||
        (nvf > nvc &&
         up(d_ord, order.data(), sizeof(int32_t) * (nvf - nvc)) != hipSuccess))
      return set_error(PARO_EDEVICE, "prolongation upload failed");
    const long long total = (long long)nvc * ncols;
    hipLaunchKernelGGL(prolong_copy_kernel,
                       dim3((unsigned)((total + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, s, (long long)nvc, d_dofc, d_doff,
                       d_Uc, d_Uf, (int)ncols);
    for (int g = 1; g <= maxg; ++g) {
      const int cnt = start[g + 1] - start[g];
      if (cnt == 0) continue;
      const long long t = (long long)cnt * ncols;
      hipLaunchKernelGGL(prolong_level_kernel,
                         dim3((unsigned)((t + kBlock - 1) / kBlock)),
                         dim3(kBlock), 0, s, cnt, d_ord + start[g], d_par,
                         d_doff, d_Uf, (int)ncols);
    }
    // The host tables must live until the uploads have been read.
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return set_error(PARO_EDEVICE, "prolongation launch failed");
    return PARO_OK;
  } catch (...) {
    return set_error(PARO_EDEVICE, "host allocation failed");
  }
}

}  // extern "C"
