// C ABI of libparo: argument checking, workspace layout, launch tables and
// the host-side sequencing of ParO steps (Algorithm A.1, Steps 3 and 4),
// for one problem or a batch.  Every arithmetic step runs in the kernels of
// assemble.hip and solver.hip; the host only launches them and polls small
// flags.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "paro_internal.h"

namespace paro {

// Host-side event timing of kernel launches (measurement only).  The
// events of a launch are stamped by its dispatch (hipExtLaunchKernel), so
// a duration covers the kernel's execution and no launch gap.
struct Timing {
  bool on = false;
  struct Pend {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pend> pend;
  int64_t launches[PARO_ST_NUM] = {};
  double ms[PARO_ST_NUM] = {};
  unsigned long long iters0 = 0, cols0 = 0;  // device counters at reset

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void resolve() {
    for (const Pend& q : pend) {
      float t = 0.0f;
      if (hipEventSynchronize(q.b) == hipSuccess &&
          hipEventElapsedTime(&t, q.a, q.b) == hipSuccess) {
        ms[q.stage] += t;
        launches[q.stage] += 1;
      }
      pool.push_back(q.a);
      pool.push_back(q.b);
    }
    pend.clear();
  }
  ~Timing() {
    resolve();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

bool timing_pair(Timing* t, hipEvent_t* a, hipEvent_t* b) {
  if (!t || !t->on) return false;
  *a = t->get();
  *b = t->get();
  if (*a && *b) return true;
  if (*a) t->pool.push_back(*a);
  if (*b) t->pool.push_back(*b);
  return false;
}

void timing_add(Timing* t, int stage, hipEvent_t a, hipEvent_t b) {
  t->pend.push_back({stage, a, b});
  if (t->pend.size() > 4096) t->resolve();
}

// Instantiated launch graphs of CG chunks (hipGraph), keyed by the launch
// shape, the precision, the starting parity and the chunk length.  The
// kernels read their descriptors from device memory at run time, so a
// graph stays valid while the launch shape (table address, grid, vector
// widths, problem count, nonlocal projector count, SpMM segmentation) is
// unchanged.
typedef std::array<int64_t, 23> GraphKey;
struct GraphCache {
  std::map<GraphKey, hipGraphExec_t> m;
  ~GraphCache() {
    for (auto& kv : m) (void)hipGraphExecDestroy(kv.second);
  }
};

namespace {

thread_local std::string g_err = "no error";
// Off by default: measured no faster than kernel-by-kernel launches once
// polls go through the host mailbox (the GPU-side dispatch gap between
// dependent kernels is what remains, and graphs do not shorten it).
std::atomic<int> g_graphs_on{0};
std::atomic<int> g_persistent_on{0};
std::atomic<int> g_matfree_on{1};
// Co-resident workgroups of the persistent CG kernel (three per CU on 256
// CUs); the launcher checks the device's actual capacity.
constexpr int kPersistGrid = 768;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_OR_FAIL(expr)                                                   \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(PARO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
int round8(int64_t x) { return (int)(((x + 7) / 8) * 8); }

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int check_box(const paro_box_t* box) {
  if (!box) return fail(PARO_EINVAL, "box is NULL");
  if (box->nx < 2 || box->ny < 2 || box->nz < 2)
    return fail(PARO_EINVAL, "need at least 2 cells per axis (got %d %d %d)",
                box->nx, box->ny, box->nz);
  for (int a = 0; a < 3; ++a)
    if (!(box->hi[a] > box->lo[a]) || !std::isfinite(box->lo[a]) ||
        !std::isfinite(box->hi[a]))
      return fail(PARO_EINVAL, "box axis %d: need finite lo < hi", a);
  return PARO_OK;
}

// All vertices of a box's Kuhn mesh (where its potential is given).
int64_t box_vertices(const paro_box_t& b) {
  return (int64_t)(b.nx + 1) * (b.ny + 1) * (b.nz + 1);
}

int check_opts(const paro_opts_t* o, int64_t n) {
  if (!o) return fail(PARO_EINVAL, "opts is NULL");
  if (o->N < 1 || o->m < 0)
    return fail(PARO_EINVAL, "need N >= 1 and m >= 0 (got %d, %d)", o->N, o->m);
  const int Nt = o->N + o->m;
  if (Nt > kNtMax)
    return fail(PARO_EINVAL, "N + m = %d exceeds %d", Nt, kNtMax);
  if (n >= 0 && Nt > n)
    return fail(PARO_EINVAL, "N + m = %d exceeds the %lld dofs", Nt,
                (long long)n);
  if (o->precision != PARO_FP64 && o->precision != PARO_FP32_INNER)
    return fail(PARO_EINVAL, "unknown precision %d", o->precision);
  if (o->pcg_maxit < 1) return fail(PARO_EINVAL, "pcg_maxit must be >= 1");
  if (!(o->pcg_rtol > 0.0) || !(o->pcg_rtol < 1.0))
    return fail(PARO_EINVAL, "pcg_rtol must lie in (0, 1)");
  if (!(o->pcg_reduce >= 0.0) || !(o->pcg_reduce < 1.0))
    return fail(PARO_EINVAL, "pcg_reduce must lie in [0, 1)");
  if (o->precision == PARO_FP32_INNER &&
      (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0)))
    return fail(PARO_EINVAL, "inner_rtol must lie in (0, 1)");
  if (o->sigma_mode == 1 && !std::isfinite(o->sigma))
    return fail(PARO_EINVAL, "sigma must be finite");
  return PARO_OK;
}

void carve(Problem& p, char* base, const Layout& L) {
  auto at = [&](size_t off) { return (void*)(base + off); };
  p.dinv = (double*)at(L.dinv);
  p.dinv32 = L.dinv32 ? (float*)at(L.dinv32) : nullptr;
  p.diagA = L.diagA ? (double*)at(L.diagA) : nullptr;
  p.diagM = L.diagM ? (double*)at(L.diagM) : nullptr;
  p.diagA32 = L.diagA32 ? (float*)at(L.diagA32) : nullptr;
  p.Vb = L.vbox ? (double*)at(L.vbox) : nullptr;
  p.kconst = L.kconst ? (double*)at(L.kconst) : nullptr;
  p.X = (double*)at(L.X);
  p.R = (double*)at(L.R);
  p.P = (double*)at(L.P);
  p.Q = (double*)at(L.Q);
  p.B = L.B ? (double*)at(L.B) : nullptr;
  p.HU = (double*)at(L.HU);
  p.MU = (double*)at(L.MU);
  p.Xc = L.Xc ? (double*)at(L.Xc) : nullptr;
  p.Xm = L.Xm ? (double*)at(L.Xm) : nullptr;
  p.R32 = L.R32 ? (float*)at(L.R32) : nullptr;
  p.P32 = L.P32 ? (float*)at(L.P32) : nullptr;
  p.Q32 = L.Q32 ? (float*)at(L.Q32) : nullptr;
  p.X32 = L.X32 ? (float*)at(L.X32) : nullptr;
  p.part = (double*)at(L.part);
  p.cpart = (double*)at(L.cpart);
  p.gpart = (double*)at(L.gpart);
  p.Ah = (double*)at(L.Ah);
  p.Bh = (double*)at(L.Bh);
  p.C = (double*)at(L.C);
  p.theta = (double*)at(L.theta);
  p.vmin = (double*)at(L.vmin);
  p.cs = (ColState*)at(L.cs);
  p.si = (StepInfo*)at(L.si);
  p.cnt = (unsigned*)at(L.cnt);
  p.flag = (int*)at(L.flag);
  p.dd = (Desc*)at(L.desc);
  p.clus = (int*)at(L.clus);
  p.clustered = false;
  p.Zp = nullptr;
  p.kz = 0;
  p.zy = p.zpart = nullptr;
  p.csr = L.rowptr != 0;
  if (p.csr) {
    p.rowptr = (int32_t*)at(L.rowptr);
    p.colidx = (int32_t*)at(L.colidx);
    p.valA = (double*)at(L.valA);
    p.valM = (double*)at(L.valM);
    p.inc_ptr = (int32_t*)at(L.inc_ptr);
    p.inc = (int32_t*)at(L.inc);
    p.tets = (int32_t*)at(L.tets);
    p.Xv = (double*)at(L.Xv);
    p.Vv = (double*)at(L.Vv);
    p.dofmap = (int32_t*)at(L.dofmap);
    p.nbr = (int32_t*)at(L.nbr);
  }
}

int pick_grid(int64_t n, int Nt) {
  const int V = (Nt % 2 == 0) ? 2 : 1;
  const int cpr = Nt / V, tr = kBlock / cpr;
  const int64_t tiles = (n + tr - 1) / tr;
  int64_t g = tiles < kGridDefault ? tiles : kGridDefault;
  g = ((g + 7) / 8) * 8;
  return (int)(g < 8 ? 8 : g);
}

// The static part of a problem's descriptor (sizes, operator, workspace).
void desc_init(Problem& p) {
  Desc& d = p.hd;
  std::memset(&d, 0, sizeof d);
  d.n = p.n;
  d.nnz = p.nnz;
  d.ncols = p.Nt;
  d.nreq = p.N;
  d.b0 = 0;
  d.nb = d.ns = p.grid;
  d.g0 = 0;
  d.gnb = d.gns = std::min(p.grid, kGramGrid);
  d.v64 = vec64_of(p.Nt);
  d.v32 = vec32_of(p.Nt);
  d.cg_var = -1;
  d.maxit = p.opts.pcg_maxit;
  d.sigma = p.sigma;
  d.rtol = p.opts.pcg_rtol;
  d.inner_rtol = p.opts.inner_rtol;
  {
    const double q = p.opts.pcg_reduce / p.opts.pcg_rtol;
    d.reduce2 = q * q;
  }
  d.dinv = p.dinv;
  d.dinv32 = p.dinv32;
  d.diagA = p.diagA;
  d.diagM = p.diagM;
  d.diagA32 = p.diagA32;
  d.Vb = p.Vb;
  d.kconst = p.kconst;
  d.mx = p.mx;
  d.my = p.my;
  d.mz = p.mz;
  d.X = d.Uout = p.X;
  d.U0 = p.X;
  d.R = p.R;
  d.P = p.P;
  d.Q = p.Q;
  d.B = p.B;
  d.HU = p.HU;
  d.MU = p.MU;
  d.use_hu = 0;
  d.Xc = p.Xc;
  d.R32 = p.R32;
  d.P32 = p.P32;
  d.Q32 = p.Q32;
  d.X32 = p.X32;
  d.ntc = (int)cm_tiles(p.n);
  // The CG kernels write one partial per (column, tile).
  d.cgp = p.cpart;
  d.cgn = d.ntc;
  d.cgstride = (long long)p.Nt * d.ntc;
  d.pqp = p.cpart + 2 * d.cgstride;
  d.spt = (int)spmm_tiles(p.n);
  d.spg = spmm_seg_tiles(p.n);
  d.pqn = spmm_segments(p.n);
  d.zm = zm_ranges(p.mx, p.my, p.mz);
  d.zxy = (int)(((long long)p.mx * p.my + kSpmmRows - 1) / kSpmmRows);
  if (d.zm) {
    d.pqn = d.zm * d.zxy;
    d.spg = 1;
  }
  // Mixed precision on a z-marching mesh: the FP64 refinement iterate and
  // right-hand sides chunk-major, its residual by a z-march whose two
  // partials per (column, segment) fit the p.q partial region.
  d.Xm = p.Xm;
  d.rcm = p.Xm && d.zm && 2 * (long long)d.pqn <= d.spt ? 1 : 0;
  d.part = p.part;
  d.gpart = p.gpart;
  d.Ah = p.Ah;
  d.Bh = p.Bh;
  d.C = p.C;
  d.theta = p.theta;
  d.cs = p.cs;
  d.si = p.si;
  d.geneig_info = &p.si->geneig_info;
  d.clus = p.clustered ? p.clus : nullptr;
  d.Zp = p.Zp;
  d.kz = p.kz;
  d.zy = p.zy;
  d.zpart = p.zpart;
  d.csr = p.csr ? 1 : 0;
  if (p.csr) {
    d.rowptr = p.rowptr;
    d.colidx = p.colidx;
    d.valA = p.valA;
    d.valM = p.valM;
    d.mx = d.my = d.mz = 0;
    d.zm = 0;
    // p.q segments of the CSR CG SpMM: kBlock rows each, or a multiple
    // when that would exceed kSpmmSegMax segments.
    const long long per = (p.n + kSpmmSegMax * (long long)kBlock - 1) /
                          (kSpmmSegMax * (long long)kBlock);
    d.csr_rows = (int)(kBlock * (per < 1 ? 1 : per));
    d.pqn = (int)((p.n + d.csr_rows - 1) / d.csr_rows);
    d.spg = 1;
  }
}

// Column count of a descriptor (component calls use fewer than N + m).
void set_cols(Desc& d, int ncols) {
  d.ncols = ncols;
  d.v64 = vec64_of(ncols);
  d.v32 = vec32_of(ncols);
}

// A launch over `n` descriptors already laid out (b0/nb, g0/gnb) in `tab`.
Launch make_launch(Desc* dtab, const Desc* tab, int n) {
  Launch L{};
  L.d = dtab;
  L.nprob = n;
  L.maxcols = 0;
  L.mincols = kNtMax;
  L.vmax64 = 1;
  for (int i = 0; i < n; ++i) {
    const Desc& d = tab[i];
    L.blocks = std::max(L.blocks, d.b0 + d.nb);
    L.gblocks = std::max(L.gblocks, d.g0 + d.gnb);
    L.maxcols = std::max(L.maxcols, d.ncols);
    L.mincols = std::min(L.mincols, d.ncols);
    L.tr64 = std::max(L.tr64, tile_rows(d.ncols, d.v64));
    L.tr32 = std::max(L.tr32, tile_rows(d.ncols, d.v32));
    L.vmax64 = std::max(L.vmax64, d.v64);
  }
  L.nt16 = (L.maxcols + 15) / 16;
  for (int i = 0; i < n; ++i) L.maxkz = std::max(L.maxkz, tab[i].kz);
  L.zmg = 0;
  for (int i = 0; i < n; ++i) {
    const Desc& d = tab[i];
    if (d.csr) {
      L.csr = 1;
    } else if (d.zm) {
      L.zm = 1;
      // Chunks per unit: the first z-marching problem's tuned variant
      // (any choice gives the same results).
      if (L.zmg == 0) L.zmg = d.cg_var >= 0 ? 1 << d.cg_var : 2;
    } else {
      L.ntile = 1;
      L.seg |= d.spg > 1 ? 1 : 0;
    }
  }
  if (L.zmg == 0) L.zmg = 2;
  // The matrix-free z-marching SpMM needs every z-marching problem's
  // potential (box problems keep it in their workspace).
  L.zmf = L.zm && g_matfree_on.load();
  for (int i = 0; i < n; ++i)
    if (tab[i].zm && !tab[i].csr && !(tab[i].Vb && tab[i].kconst)) L.zmf = 0;
  L.v64u = n > 0 ? tab[0].v64 : 0;
  L.v32u = n > 0 ? tab[0].v32 : 0;
  for (int i = 1; i < n; ++i) {
    if (tab[i].v64 != L.v64u) L.v64u = 0;
    if (tab[i].v32 != L.v32u) L.v32u = 0;
    if ((tab[i].ncols + 15) / 16 != L.nt16) L.nt16_mixed = 1;
  }
  if (n > 0 && (tab[0].ncols + 15) / 16 != L.nt16) L.nt16_mixed = 1;
  return L;
}

// Shares of the grids for a batch, proportional to each problem's work
// (n * ncols), each a multiple of 8, at least 8 blocks and at most the
// problem's own segment counts (ns, gns).
void layout_batch(std::vector<Desc>& tab) {
  double total = 0.0;
  for (const Desc& d : tab) total += (double)d.n * d.ncols;
  int b = 0, g = 0;
  for (Desc& d : tab) {
    const double w = (double)d.n * d.ncols / total;
    // d.nb: the problem's (tuned) single-problem block count.
    const int nb = std::max(8, std::min(d.nb, round8((int64_t)(w * kBatchGrid))));
    const int gnb =
        std::max(8, std::min(d.gns, round8((int64_t)(w * kBatchGramGrid))));
    d.b0 = b;
    d.nb = nb;
    d.g0 = g;
    d.gnb = gnb;
    b += nb;
    g += gnb;
  }
}

int status_to_code(int st) {
  if (st & kStNonFinite)
    return fail(PARO_EINVAL, "non-finite value in the iteration");
  if (st & kStNotSpd)
    return fail(PARO_ENOTSPD,
                "CG breakdown: p^T (H - sM) p <= 0 (shift not below lambda_1)");
  if (st & kStSingular)
    return fail(PARO_ESINGULAR, "Gram matrix W^T M W is not positive definite");
  if (st & kStNoConv)
    return fail(PARO_ENOCONV, "CG reached pcg_maxit before pcg_rtol");
  return PARO_OK;
}

// Host side of one launch table: where its table, poll words and reports
// live on the device, and the host copies.
struct Ctx {
  Launch L;
  std::vector<Desc> tab;
  Timing* timing;
  int* predict;           // 5 prediction slots (problem or batch)
  int maxit;
  int precision;
  GraphCache* graphs;     // null: launch kernel by kernel
  int last_status = 0;    // status bits seen by the last poll
  int last_outer = -1;    // refining columns seen by the last poll
  std::vector<Desc> ptab; // table laid out for the persistent CG grid
  std::vector<Problem*> owners;  // the problem of each table entry
};

// After a Rayleigh-Ritz of the table: what the next start can reuse.
void note_rotation(Ctx& c) {
  for (size_t i = 0; i < c.tab.size() && i < c.owners.size(); ++i) {
    Desc& h = c.owners[i]->hd;
    h.start_ready = c.tab[i].emit;
    h.hu_valid = c.tab[i].emit ? 0 : 1;
  }
}
// Before anything that overwrites the CG state or H U, M U.
void forget_rotation(Ctx& c) {
  for (Problem* p : c.owners) p->hd.start_ready = p->hd.hu_valid = 0;
}

// The stream CG chunks are captured on (capture only records; the graphs
// run on the caller's stream, which may be the null stream).
hipStream_t capture_stream() {
  thread_local hipStream_t cs = nullptr;
  if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    cs = nullptr;
  return cs;
}

// Launch `k` CG iterations from parity `par` as one cached graph.
int cg_graph(Ctx& c, bool fp32, int par, int k, hipStream_t s) {
  const Launch& L = c.L;
  // Every Launch field that selects a kernel, an instantiation or a grid
  // of launch_pcg_iter is part of the key (the nonlocal term's projector
  // count and the segmented SpMM included), so a change of any of them
  // captures a new graph instead of replaying a stale one.
  const GraphKey key = {
      (int64_t)(uintptr_t)L.d, L.nprob, L.blocks, L.gblocks, L.maxcols,
      L.mincols, L.nt16, L.tr64, L.tr32, L.vmax64, L.v64u, L.v32u,
      L.nt16_mixed, L.maxkz, L.seg, L.ntile, L.zm, L.zmg, L.zmf, L.csr,
      fp32 ? 1 : 0, par, k};
  auto it = c.graphs->m.find(key);
  if (it == c.graphs->m.end()) {
    hipStream_t cs = capture_stream();
    if (!cs) return fail(PARO_EDEVICE, "no capture stream");
    HIP_OR_FAIL(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int q = par;
    for (int i = 0; i < k; ++i) {
      (void)launch_pcg_iter(c.L, fp32, q, cs, nullptr);
      q ^= 1;
    }
    hipGraph_t g = nullptr;
    HIP_OR_FAIL(hipStreamEndCapture(cs, &g));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
      return fail(PARO_EDEVICE, "hipGraphInstantiate: %s",
                  hipGetErrorString(e));
    it = c.graphs->m.emplace(key, exec).first;
  }
  HIP_OR_FAIL(hipGraphLaunch(it->second, s));
  return PARO_OK;
}

// k CG iterations from parity par: graphs of 1, 2, 4, ... iterations (the
// binary digits of k), or kernel by kernel when timing or no cache.
int cg_launches(Ctx& c, bool fp32, int par, int k, hipStream_t s) {
  if (c.graphs && !(c.timing && c.timing->on) && g_graphs_on.load()) {
    for (int b = 1 << 8; b > 0; b >>= 1) {
      while (k >= b) {
        const int rc = cg_graph(c, fp32, par, b, s);
        if (rc) return rc;
        if (b & 1) par ^= 1;
        k -= b;
      }
    }
    return PARO_OK;
  }
  for (int i = 0; i < k; ++i) {
    hipError_t e = launch_pcg_iter(c.L, fp32, par, s, c.timing);
    if (e != hipSuccess)
      return fail(PARO_EDEVICE, "CG launch: %s", hipGetErrorString(e));
    par ^= 1;
  }
  return PARO_OK;
}

int upload(Ctx& c, hipStream_t s) {
  HIP_OR_FAIL(hipMemcpyAsync(c.L.d, c.tab.data(), sizeof(Desc) * c.tab.size(),
                             hipMemcpyHostToDevice, s));
  c.L = make_launch(c.L.d, c.tab.data(), (int)c.tab.size());
  return PARO_OK;
}

// Host mailbox of the calling thread: pinned, coherent host memory that
// the poll and report kernels write directly, so that the host learns a
// result by spinning on a sequence word rather than through a
// device-to-host copy and a stream synchronisation (which leave the GPU
// idle for tens of microseconds per poll).  Allocated once per thread on
// first use and kept for the life of the process.
struct Mailbox {
  char* h = nullptr;  // host address
  char* d = nullptr;  // device address of the same memory
  int seq = 0;
};
constexpr size_t kMbPoll = 0;  // poll words: seq, count, iters, status, refining
constexpr size_t kMbRepSeq = 64;    // report sequence word
constexpr size_t kMbReports = 128;  // PollReport[PARO_BATCH_MAX]
constexpr size_t kMailboxBytes = kMbReports + 32 * PARO_BATCH_MAX;

Mailbox* mailbox() {
  static_assert(sizeof(PollReport) <= 32, "report slot");
  thread_local Mailbox mb;
  if (!mb.h) {
    void* h = nullptr;
    if (hipHostMalloc(&h, kMailboxBytes,
                      hipHostMallocCoherent | hipHostMallocMapped) !=
        hipSuccess)
      return nullptr;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
      (void)hipHostFree(h);
      return nullptr;
    }
    std::memset(h, 0, kMailboxBytes);
    mb.h = static_cast<char*>(h);
    mb.d = static_cast<char*>(d);
  }
  return &mb;
}

// Spin until the device has written `seq` to the host word w.  Every 1024
// spins the stream is queried, so that a failed or finished stream that
// never wrote the word ends the wait with an error.
int wait_word(const int* w, int seq, hipStream_t s) {
  for (uint64_t it = 1;; ++it) {
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return PARO_OK;
    if ((it & 1023) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return PARO_OK;
        return fail(PARO_EDEVICE, "poll word not written by the device");
      }
      if (e != hipErrorNotReady)
        return fail(PARO_EDEVICE, "stream failed while polling: %s",
                    hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}

int poll(Ctx& c, int which, int out[2], hipStream_t s) {
  Mailbox* mb = mailbox();
  if (!mb) return fail(PARO_EDEVICE, "pinned host mailbox unavailable");
  const int seq = ++mb->seq;
  int* hw = reinterpret_cast<int*>(mb->h + kMbPoll);
  HIP_OR_FAIL(launch_count_active(
      c.L, which, reinterpret_cast<int*>(mb->d + kMbPoll), seq, s));
  const int rc = wait_word(hw, seq, s);
  if (rc) return rc;
  out[0] = hw[1];
  out[1] = hw[2];
  c.last_status = hw[3];
  c.last_outer = hw[4];
  if (c.timing) c.timing->resolve();
  return PARO_OK;
}

// Run CG iterations (FP64 or FP32) until no column of any problem is
// active.  The first batch of launches is as long as the previous solve in
// the same slot took, so that a converging solve usually needs one poll;
// later batches are short top-ups.  Launches after convergence are no-ops
// on the device, so no poll precedes the first batch.
// Shares of a persistent grid of `grid` blocks, proportional to each
// problem's work, multiples of 8, at least 8 and at most the problem's
// own block count (work distribution only: results do not depend on it).
void layout_persistent(std::vector<Desc>& tab, int grid) {
  double total = 0.0;
  for (const Desc& d : tab) total += (double)d.n * d.ncols;
  int b = 0;
  for (Desc& d : tab) {
    const double w = (double)d.n * d.ncols / total;
    const int nb = std::max(8, std::min(d.nb, (int)(w * grid) / 8 * 8));
    d.b0 = b;
    d.nb = nb;
    b += nb;
  }
}

// All CG iterations of the table in one persistent launch.  Returns 1
// (nothing launched) when the grid cannot be co-resident.
int run_cg_persistent(Ctx& c, bool fp32, hipStream_t s, int slot) {
  c.ptab = c.tab;
  layout_persistent(c.ptab, kPersistGrid);
  HIP_OR_FAIL(hipMemcpyAsync(c.L.d, c.ptab.data(),
                             sizeof(Desc) * c.ptab.size(),
                             hipMemcpyHostToDevice, s));
  Launch PL = make_launch(c.L.d, c.ptab.data(), (int)c.ptab.size());
  const int iters = (int)std::min<int64_t>(((int64_t)c.maxit + 65) / 2 * 2,
                                           1 << 30);
  bool fits = false;
  const hipError_t e = launch_cg_persistent(PL, fp32, iters, s, c.timing,
                                            &fits);
  int rc = upload(c, s);  // the per-kernel layout again (stream-ordered)
  if (e != hipSuccess)
    return fail(PARO_EDEVICE, "persistent CG launch: %s",
                hipGetErrorString(e));
  if (rc) return rc;
  if (!fits) return 1;
  int pw[2] = {0, 0};
  rc = poll(c, 0, pw, s);
  if (rc) return rc;
  if (pw[0] != 0)
    return fail(PARO_EDEVICE, "persistent CG stopped at its iteration cap");
  c.predict[slot] = pw[1];
  return PARO_OK;
}

int run_cg(Ctx& c, bool fp32, hipStream_t s, int slot) {
  if (g_persistent_on.load() && c.L.maxkz == 0 && c.L.zm == 0 &&
      c.L.csr == 0) {
    const int rc = run_cg_persistent(c, fp32, s, slot);
    if (rc != 1) return rc;  // 1: does not fit, run kernel by kernel
  }
  int pw[2] = {0, 0};
  const int64_t cap = (int64_t)c.maxit + 64;
  const int pred = c.predict[slot];
  int chunk = pred < 2 ? 2 : (pred > 256 ? 256 : pred);
  int par = 0;
  int64_t launched = 0;
  while (true) {
    if (launched >= cap)
      return fail(PARO_EDEVICE, "CG loop did not terminate on the device");
    const int rc0 = cg_launches(c, fp32, par, chunk, s);
    if (rc0) return rc0;
    if (chunk & 1) par ^= 1;
    launched += chunk;
    const int rc = poll(c, par, pw, s);
    if (rc) return rc;
    if (pw[0] == 0) break;
    chunk = (pred + 3) / 4;
    chunk = chunk < 2 ? 2 : (chunk > 16 ? 16 : chunk);
  }
  c.predict[slot] = pw[1];
  return PARO_OK;
}

// Source solves of one step, from the state prepared by the start kernel.
int solve_sources(Ctx& c, hipStream_t s, int64_t* refinements) {
  if (c.precision == PARO_FP64) {
    const int rc = run_cg(c, false, s, 0);
    if (rc) return rc;
    HIP_OR_FAIL(launch_cm_unpack(c.L, s, c.timing));
    return PARO_OK;
  }
  // Pass 0's residual, FP32 start state and inner target come from the
  // start kernel (x0 = u0).  Pass 0 needs no poll of its own: the start
  // kernel makes a column CG-active exactly where it refines, so with no
  // refining column the CG launches are no-ops, and the CG loop's last
  // poll also returns the refining count.
  for (int pass = 0;; ++pass) {
    int rc;
    if (pass > 0) {
      HIP_OR_FAIL(launch_refine_residual(c.L, s, c.timing));
      int pw[2];
      rc = poll(c, 2, pw, s);
      if (rc) return rc;
      if (pw[0] == 0) break;
      if (pass > 200)
        return fail(PARO_EDEVICE, "refinement loop did not terminate");
      HIP_OR_FAIL(launch_redirect(c.L, s, c.timing));
    }
    c.last_outer = -1;
    rc = run_cg(c, true, s, 1 + (pass < 3 ? pass : 3));
    if (rc) return rc;
    if (pass == 0) {
      if (c.last_outer < 0) {  // a CG path that did not poll
        int pw[2];
        rc = poll(c, 2, pw, s);
        if (rc) return rc;
      }
      if (c.last_outer == 0) break;
    }
    HIP_OR_FAIL(launch_refine_update(c.L, s, c.timing));
    if (refinements) ++*refinements;
  }
  // Problems whose refinement iterate is chunk-major hand it to X.
  if (c.L.zm) HIP_OR_FAIL(launch_cm_unpack(c.L, s, c.timing));
  return PARO_OK;
}

int read_reports(Ctx& c, std::vector<PollReport>& out, hipStream_t s) {
  Mailbox* mb = mailbox();
  if (!mb) return fail(PARO_EDEVICE, "pinned host mailbox unavailable");
  out.resize(c.tab.size());
  const int seq = ++mb->seq;
  HIP_OR_FAIL(launch_gather_reports(
      c.L, reinterpret_cast<PollReport*>(mb->d + kMbReports),
      reinterpret_cast<int*>(mb->d + kMbRepSeq), seq, s));
  const int rc =
      wait_word(reinterpret_cast<const int*>(mb->h + kMbRepSeq), seq, s);
  if (rc) return rc;
  std::memcpy(out.data(), mb->h + kMbReports, sizeof(PollReport) * out.size());
  return PARO_OK;
}

// General meshes have no operator path in the start kernel: a start that
// cannot reuse a rotation's H U and M U (use_hu = 0) forms them from U0
// first (use_hu = 2, launch_csr_dual mode 2).  True if any problem does.
bool mark_csr_starts(Ctx& c) {
  bool any = false;
  for (Desc& d : c.tab)
    if (d.csr && d.use_hu == 0) {
      d.use_hu = 2;
      any = true;
    }
  return any;
}

// Problems whose Rayleigh-Ritz factorisation of W^T M W failed (status
// bit kStSingular in the reports just read) get one shifted Cholesky-QR
// re-orthonormalisation of W and the projection again, on a table of
// those problems alone (their own block counts, so their arithmetic is
// what it is in any launch).  `pr` is updated with the new reports, their
// status marked kStReorth; a problem whose basis is dependent to rounding
// level keeps the singular status.
int retry_singular(Ctx& c, std::vector<PollReport>& pr, hipStream_t s) {
  std::vector<int> idx;
  for (size_t i = 0; i < pr.size(); ++i)
    if (pr[i].status & kStSingular) idx.push_back((int)i);
  if (idx.empty()) return PARO_OK;
  Ctx r = c;
  r.tab.clear();
  int b = 0, g = 0;
  for (int i : idx) {
    Desc d = c.tab[i];
    d.X = d.Uout;  // the failed projection left U = W
    d.b0 = b;
    d.g0 = g;
    b += d.nb;
    g += d.gnb;
    r.tab.push_back(d);
  }
  int rc = upload(r, s);
  if (rc) return rc;
  HIP_OR_FAIL(launch_reorth(r.L, s));
  HIP_OR_FAIL(launch_rayleigh_ritz(r.L, s, r.timing));
  HIP_OR_FAIL(launch_reorth_check(r.L, s));
  std::vector<PollReport> again;
  rc = read_reports(r, again, s);
  if (rc) return rc;
  for (size_t k = 0; k < idx.size(); ++k) {
    pr[idx[k]] = again[k];
    pr[idx[k]].status |= kStReorth;
  }
  return idx.size() == c.tab.size() ? PARO_OK : upload(c, s);
}

// One ParO step (Steps 3 and 4) for every problem of the table; the
// descriptors' U0 = X = Uout (the orbitals, in place) and lam are set.
// Per-problem status goes into `reps` (if given).  `single`: a CG
// breakdown stops before the projection and is returned.
// trust: U (and lambda) of every problem are the outputs of its last
// rotation, with the operator unchanged since (the library's own step
// loops), so the start takes A_s U = HU - s MU and M U from that rotation
// instead of applying the operators again.
int step_tables(Ctx& c, hipStream_t s, paro_report_t* reps, bool single,
                bool trust) {
  const double t0 = now_s();
  // The start: from the state the last rotation emitted (trusted loops),
  // else from its H U, M U (trusted loops after a rotation that kept
  // them), else by applying the operators.  The rotation of this step
  // emits the next start's state when the caller is a library loop.
  for (Desc& d : c.tab) {
    d.use_hu = !trust ? 0 : (d.start_ready ? 3 : (d.hu_valid ? 1 : 0));
    d.start_part = d.use_hu == 3 ? 2 : 0;
    d.emit = trust ? 1 : 0;
  }
  forget_rotation(c);
  const bool csr_hu = mark_csr_starts(c);
  int rc = upload(c, s);
  if (rc) return rc;
  if (csr_hu) HIP_OR_FAIL(launch_csr_dual(c.L, 2, s, c.timing));
  HIP_OR_FAIL(launch_pcg_start(c.L, s, c.timing));
  int64_t refinements = 0;
  rc = solve_sources(c, s, &refinements);
  if (rc) return rc;
  std::vector<PollReport> pr;
  // The last poll of the source solves carries the status bits.
  if (single && (c.last_status & (kStNonFinite | kStNotSpd)))
    return status_to_code(c.last_status);
  HIP_OR_FAIL(launch_rayleigh_ritz(c.L, s, c.timing));
  note_rotation(c);
  if (!reps) return PARO_OK;
  rc = read_reports(c, pr, s);
  if (rc) return rc;
  rc = retry_singular(c, pr, s);
  if (rc) return rc;
  const double dt = now_s() - t0;
  int first = PARO_OK;
  for (size_t i = 0; i < c.tab.size(); ++i) {
    paro_report_t& r = reps[i];
    r.steps = 1;
    r.pcg_iters = pr[i].max_iters;
    r.refinements = refinements;
    r.n_dof = c.tab[i].n;
    r.nnz = c.tab[i].nnz;
    r.max_dlambda = pr[i].max_dlambda;
    r.max_resid = pr[i].max_resid;
    r.sigma = c.tab[i].sigma;
    r.seconds = dt;
    r.status = status_to_code(pr[i].status & ~kStReorth);
    r.reorth = (pr[i].status & kStReorth) ? 1 : 0;
    if (first == PARO_OK) first = r.status;
  }
  return single ? first : PARO_OK;
}

// Step 1 (Rayleigh-Ritz of the start block) for every problem.
// status: null (asynchronous), or it receives every problem's status
// bits after the projection, with the re-orthonormalisation retry done
// (kStReorth marks a retried problem).
int init_tables(Ctx& c, hipStream_t s, std::vector<int>* status) {
  // A synchronous Step 1 belongs to a library loop, whose first step
  // starts from the state this rotation emits.
  for (Desc& d : c.tab) {
    d.emit = status ? 1 : 0;
    d.use_hu = 0;
  }
  forget_rotation(c);
  int rc = upload(c, s);
  if (rc) return rc;
  HIP_OR_FAIL(launch_rayleigh_ritz(c.L, s, c.timing));
  note_rotation(c);
  if (!status) return PARO_OK;
  std::vector<PollReport> pr;
  rc = read_reports(c, pr, s);
  if (rc) return rc;
  rc = retry_singular(c, pr, s);
  if (rc) return rc;
  status->resize(pr.size());
  for (size_t i = 0; i < pr.size(); ++i) (*status)[i] = pr[i].status;
  return PARO_OK;
}

Ctx single_ctx(Problem& p) {
  Ctx c;
  c.tab.assign(1, p.hd);
  c.owners.assign(1, &p);
  c.L = make_launch(p.dd, c.tab.data(), 1);
  c.timing = p.timing;
  c.predict = p.cg_predict;
  c.maxit = p.opts.pcg_maxit;
  c.precision = p.opts.precision;
  if (!p.graphs) p.graphs = new (std::nothrow) GraphCache();
  c.graphs = p.graphs;
  return c;
}

// Batch workspace: the descriptor table.
struct BatchLayout {
  size_t tab, total;
};
BatchLayout batch_layout(int count) {
  BatchLayout b;
  b.tab = 0;
  b.total = align256(sizeof(Desc) * (size_t)count);
  return b;
}

int batch_ctx(Ctx& c, paro_problem* const* probs, int count, void* ws,
              size_t bytes, int* predict) {
  if (!probs || count < 1 || count > PARO_BATCH_MAX)
    return fail(PARO_EINVAL, "batch needs 1..%d problems", PARO_BATCH_MAX);
  if (!ws || ((uintptr_t)ws & 255))
    return fail(PARO_EINVAL, "batch workspace must be 256-byte aligned");
  const BatchLayout bl = batch_layout(count);
  if (bytes < bl.total)
    return fail(PARO_ENOMEM, "batch workspace %zu < %zu bytes", bytes,
                bl.total);
  c.tab.clear();
  int prec = -1, maxit = 0;
  for (int i = 0; i < count; ++i) {
    if (!probs[i]) return fail(PARO_EINVAL, "NULL problem %d", i);
    const Problem& p = probs[i]->p;
    if (prec >= 0 && p.opts.precision != prec)
      return fail(PARO_EINVAL, "batch mixes precisions");
    prec = p.opts.precision;
    maxit = std::max(maxit, p.opts.pcg_maxit);
    c.tab.push_back(p.hd);
    c.owners.push_back(&probs[i]->p);
  }
  layout_batch(c.tab);
  char* base = (char*)ws;
  c.L = make_launch((Desc*)(base + bl.tab), c.tab.data(), count);
  c.timing = nullptr;
  c.predict = predict;
  c.maxit = maxit;
  c.precision = prec;
  c.graphs = nullptr;
  return PARO_OK;
}

// Autotuner of the CG SpMM: for a problem shape (grid, columns,
// precision) time every kernel variant (the z-marching SpMM with 1, 2 or
// 4 chunks per unit; the row sweep has one) with the full and the halved
// real block count on the problem's own operator (all columns active,
// scratch vectors), keep the fastest, and cache it for the process.  No
// choice changes the arithmetic: a variant only decides which columns a
// unit serves, the block count which block serves a unit, and the
// reduction segments stay the problem's own.
std::atomic<int> g_autotune_on{1};
std::mutex g_tune_mu;
std::map<std::array<int, 5>, std::pair<int, int>> g_tune;

int autotune(Problem& p, hipStream_t s) {
  const std::array<int, 5> key = {p.mx, p.my, p.mz, p.Nt,
                                  p.opts.precision};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      p.hd.cg_var = it->second.first;
      p.hd.nb = it->second.second;
      return PARO_OK;
    }
  }
  const bool fp32 = p.opts.precision == PARO_FP32_INNER;
  // Timing runs on zero vectors (the next source-solve start overwrites
  // them).
  const size_t vbytes = (fp32 ? 4 : 8) * (size_t)p.n * p.Nt;
  HIP_OR_FAIL(hipMemsetAsync(fp32 ? (void*)p.P32 : (void*)p.P, 0, vbytes, s));
  Ctx c;
  c.tab.assign(1, p.hd);
  c.L = make_launch(p.dd, c.tab.data(), 1);
  int rc = upload(c, s);
  if (rc) return rc;
  HIP_OR_FAIL(launch_all_active(c.L, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OR_FAIL(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PARO_EDEVICE, "hipEventCreate failed");
  }
  const int ns = p.hd.ns;
  const int half = std::max(8, ns / 2 / 8 * 8);
  // Variants: the row-sweep SpMM has one (0); the z-marching one serves
  // 1, 2 or 4 chunks per unit (variant log2 of that), except in its
  // matrix-free form, which balances its own chunk groups.
  const int nvar = p.hd.zm && !c.L.zmf ? 3 : 1;
  float best = 1e30f;
  int best_var = 0, best_nb = ns;
  hipError_t err = hipSuccess;
  for (int var = 0; var < nvar && err == hipSuccess && rc == PARO_OK; ++var)
    for (int nb : {ns, half}) {
      if (nb == half && half == ns) continue;
      c.tab[0].nb = nb;
      c.tab[0].cg_var = var;
      if ((rc = upload(c, s)) != PARO_OK) break;
      if ((err = launch_cg_spmm(c.L, fp32, s)) != hipSuccess) break;
      if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
      for (int k = 0; k < 5 && err == hipSuccess; ++k)
        err = launch_cg_spmm(c.L, fp32, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      if (err != hipSuccess) break;
      if (ms < best) {
        best = ms;
        best_nb = nb;
        best_var = var;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (err != hipSuccess)
    return fail(PARO_EDEVICE, "autotune: %s", hipGetErrorString(err));
  p.hd.cg_var = best_var;
  p.hd.nb = best_nb;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = {best_var, best_nb};
  return PARO_OK;
}

}  // namespace

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int status_code(int st) { return status_to_code(st); }

Layout make_layout(int64_t n, int64_t nnz, int Nt, int precision,
                   const MeshSizes* ms, int64_t nvbox) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const bool f32 = precision == PARO_FP32_INNER;
  const size_t blk = (size_t)n * Nt;
  if (ms) {
    // General mesh: the CSR operator and the mesh tables come first (the
    // first region sits at offset 0, so a nonzero offset marks a mesh).
    L.Xv = take(sizeof(double) * 3 * ms->nv);
    L.rowptr = take(sizeof(int32_t) * (n + 1));
    L.colidx = take(sizeof(int32_t) * nnz);
    L.valA = take(sizeof(double) * nnz);
    L.valM = take(sizeof(double) * nnz);
    L.inc_ptr = take(sizeof(int32_t) * (n + 1));
    L.inc = take(sizeof(int32_t) * 2 * ms->ninc);
    L.tets = take(sizeof(int32_t) * 4 * ms->ne);
    L.Vv = take(sizeof(double) * ms->nv);
    L.dofmap = take(sizeof(int32_t) * ms->nv);
    L.nbr = take(sizeof(int32_t) * 4 * ms->ne);
  }
  L.dinv = take(sizeof(double) * n);
  L.dinv32 = f32 ? take(sizeof(float) * n) : 0;
  L.diagA = ms ? 0 : take(sizeof(double) * kStencil * n);
  L.diagM = ms ? 0 : take(sizeof(double) * kStencil * n);
  L.diagA32 = f32 && !ms ? take(sizeof(float) * kStencil * n) : 0;
  L.vbox = !ms && nvbox > 0 ? take(sizeof(double) * nvbox) : 0;
  L.kconst = L.vbox ? take(sizeof(double) * 32) : 0;
  L.X = take(sizeof(double) * blk);
  L.R = take(sizeof(double) * blk);
  L.P = take(sizeof(double) * blk);
  L.Q = take(sizeof(double) * blk);
  L.B = f32 ? take(sizeof(double) * blk) : 0;
  L.HU = take(sizeof(double) * blk);
  L.MU = take(sizeof(double) * blk);
  L.Xc = f32 ? 0 : take(sizeof(double) * blk);
  // Mixed precision on a box: the chunk-major refinement iterate (used on
  // meshes with the z-marching SpMM).
  L.Xm = f32 && !ms && nvbox > 0 ? take(sizeof(double) * blk) : 0;
  L.R32 = f32 ? take(sizeof(float) * blk) : 0;
  L.P32 = f32 ? take(sizeof(float) * blk) : 0;
  L.Q32 = f32 ? take(sizeof(float) * blk) : 0;
  L.X32 = f32 ? take(sizeof(float) * blk) : 0;
  // Partials of 5 quantities: a rotation's 2 and the start state it may
  // emit (3), or a start's 3.
  L.part = take(sizeof(double) * 5 * (size_t)kGridMax * kNtMax);
  L.cpart = take(sizeof(double) * (size_t)Nt *
                 (2 * cm_tiles(n) + spmm_tiles(n)));
  L.gpart = take(sizeof(double) * (size_t)kGramGrid * gram_tiles(Nt));
  L.Ah = take(sizeof(double) * kNtMax * kNtMax);
  L.Bh = take(sizeof(double) * kNtMax * kNtMax);
  L.C = take(sizeof(double) * kNtMax * kNtMax);
  L.theta = take(sizeof(double) * kNtMax);
  L.vmin = take(sizeof(double) * 4);
  L.cs = take(sizeof(ColState));
  L.si = take(sizeof(StepInfo));
  L.cnt = take(sizeof(unsigned) * kCntNum);
  L.flag = take(sizeof(int) * 16);
  L.desc = take(sizeof(Desc));
  L.clus = take(sizeof(int) * kNtMax);
  L.total = off;
  return L;
}

// ---------------------------------------------------------------------------
// Allocation-free Gram (paro_gram_noalloc): its scratch -- one launch
// descriptor and the first-stage tile partials -- is this file-scope
// device array, of which every device holds its own copy for the life of
// the process.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocDescBytes = 1024;
constexpr size_t kNoAllocPartBytes =
    sizeof(double) * (size_t)kGramGrid * 16 * 256;  // 64 columns, 512 segments
constexpr size_t kNoAllocBytes = kNoAllocDescBytes + kNoAllocPartBytes;
static_assert(sizeof(Desc) <= kNoAllocDescBytes, "descriptor slot");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved on the
// first call per device).
int scratch_address(void** out) {
  int dev = 0;
  HIP_OR_FAIL(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(PARO_EDEVICE, "device %d beyond the supported %d", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PARO_EDEVICE, "hipGetSymbolAddress(scratch): %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PARO_OK;
}

// Writes a descriptor passed by value into device memory (no copy from
// host memory, nothing to allocate or pin).
__global__ void store_desc_kernel(Desc d, Desc* dst) {
  if (threadIdx.x == 0) *dst = d;
}

}  // namespace

}  // namespace paro

using namespace paro;

extern "C" {

void paro_default_opts(paro_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->N = 1;
  o->m = 0;
  o->max_steps = 200;
  o->pcg_maxit = 10000;
  o->precision = PARO_FP64;
  o->sigma_mode = 0;
  o->sigma = 0.0;
  o->lambda_tol = 1e-12;
  o->resid_tol = 1e-8;
  o->pcg_rtol = 1e-10;
  o->inner_rtol = 1e-5;
}

const char* paro_last_error(void) { return g_err.c_str(); }

const char* paro_strerror(int st) {
  switch (st) {
    case PARO_OK: return "ok";
    case PARO_EINVAL: return "invalid argument";
    case PARO_ENOMEM: return "workspace too small";
    case PARO_ENOTSPD: return "source-problem matrix not positive definite";
    case PARO_ESINGULAR: return "Gram matrix singular";
    case PARO_ENOCONV: return "iteration cap reached";
    case PARO_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

int paro_query(const paro_box_t* box, const paro_opts_t* opts,
               int64_t* n_dof, int64_t* nnz, size_t* workspace_bytes) {
  int rc = check_box(box);
  if (rc) return rc;
  const int64_t n = (int64_t)(box->nx - 1) * (box->ny - 1) * (box->nz - 1);
  rc = check_opts(opts, n);
  if (rc) return rc;
  const int64_t z = kuhn_nnz(box->nx - 1, box->ny - 1, box->nz - 1);
  if (z >= ((int64_t)1 << 31))
    return fail(PARO_EINVAL, "nnz %lld exceeds 32-bit indices", (long long)z);
  if (n_dof) *n_dof = n;
  if (nnz) *nnz = z;
  if (workspace_bytes)
    *workspace_bytes =
        make_layout(n, z, opts->N + opts->m, opts->precision, nullptr,
                    box_vertices(*box))
            .total;
  return PARO_OK;
}

int paro_assemble(const paro_box_t* box, const double* d_V,
                  const paro_opts_t* opts, void* d_ws, size_t bytes,
                  void* stream, paro_problem** out) {
  try {
    if (!out) return fail(PARO_EINVAL, "out is NULL");
    *out = nullptr;
    int64_t n = 0, z = 0;
    size_t need = 0;
    int rc = paro_query(box, opts, &n, &z, &need);
    if (rc) return rc;
    if (!d_V || !d_ws) return fail(PARO_EINVAL, "NULL device pointer");
    if (((uintptr_t)d_ws & 255) != 0)
      return fail(PARO_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need)
      return fail(PARO_ENOMEM, "workspace %zu bytes < %zu required", bytes,
                  need);
    hipStream_t s = (hipStream_t)stream;
    paro_problem* h = new (std::nothrow) paro_problem();
    if (!h) return fail(PARO_EDEVICE, "host allocation failed");
    Problem& p = h->p;
    p.box = *box;
    p.opts = *opts;
    p.mx = box->nx - 1;
    p.my = box->ny - 1;
    p.mz = box->nz - 1;
    p.n = n;
    p.nnz = z;
    p.N = opts->N;
    p.Nt = opts->N + opts->m;
    p.h[0] = (box->hi[0] - box->lo[0]) / box->nx;
    p.h[1] = (box->hi[1] - box->lo[1]) / box->ny;
    p.h[2] = (box->hi[2] - box->lo[2]) / box->nz;
    p.grid = pick_grid(n, p.Nt);
    p.ws_bytes = bytes;
    p.last_stream = s;
    const Layout L =
        make_layout(n, z, p.Nt, opts->precision, nullptr, box_vertices(*box));
    carve(p, (char*)d_ws, L);
    auto bail = [&](int code) {
      delete h;
      return code;
    };
    // Zero the small state (counters, column state, step info).
    hipError_t he =
        hipMemsetAsync((char*)d_ws + L.vmin, 0, L.total - L.vmin, s);
    if (he != hipSuccess)
      return bail(fail(PARO_EDEVICE, "hipMemsetAsync: %s",
                       hipGetErrorString(he)));
    const int64_t nv = (int64_t)(box->nx + 1) * (box->ny + 1) * (box->nz + 1);
    if (launch_potential_range(d_V, nv, p.vmin, p.cnt + kCntMin, p.part, s) !=
        hipSuccess)
      return bail(fail(PARO_EDEVICE, "potential range launch failed"));
    double rng[3];
    he = hipMemcpyAsync(rng, p.vmin, sizeof rng, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess)
      return bail(fail(PARO_EDEVICE, "reading the potential range: %s",
                       hipGetErrorString(he)));
    if (rng[2] != 0.0)
      return bail(fail(PARO_EINVAL, "potential has %.0f non-finite values",
                       rng[2]));
    if (opts->sigma_mode == 1)
      p.sigma = opts->sigma;
    else
      p.sigma = rng[0] >= 0.0 ? 0.0 : rng[0] - 1.0;
    if (launch_assemble(p, d_V, s) != hipSuccess)
      return bail(fail(PARO_EDEVICE, "assembly launch failed"));
    desc_init(p);
    if (g_autotune_on.load()) {
      const int rc2 = autotune(p, s);
      if (rc2) return bail(rc2);
    }
    *out = h;
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_assemble");
  }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Problems on general (bisection) meshes: the operator in CSR.
// ---------------------------------------------------------------------------
namespace {
int mesh_shape(const paro_mesh* m, const paro_opts_t* opts,
               std::shared_ptr<const MeshOps>* out, Layout* L) {
  if (!m) return fail(PARO_EINVAL, "NULL mesh");
  std::shared_ptr<const MeshOps> ops;
  {
    std::lock_guard<std::mutex> g(m->ops_mu);
    if (!m->ops) {
      auto built = std::make_shared<MeshOps>();
      const int rc0 = mesh_ops(m->m, built.get());
      if (rc0) return rc0;
      m->ops = built;
    }
    ops = m->ops;
  }
  *out = ops;
  int rc = check_opts(opts, ops->n);
  if (rc) return rc;
  if (opts->precision != PARO_FP64)
    return fail(PARO_EINVAL, "mesh problems are solved in PARO_FP64");
  MeshSizes ms{m->m.nv(), m->m.ne(), (int64_t)ops->inc_ptr[ops->n]};
  *L = make_layout(ops->n, (int64_t)ops->colidx.size(), opts->N + opts->m,
                   PARO_FP64, &ms);
  return PARO_OK;
}
}  // namespace

extern "C" {

int paro_mesh_query(const paro_mesh* m, const paro_opts_t* opts,
                    int64_t* n_dof, int64_t* nnz, size_t* workspace_bytes) {
  try {
    std::shared_ptr<const MeshOps> ops;
    Layout L;
    const int rc = mesh_shape(m, opts, &ops, &L);
    if (rc) return rc;
    if (n_dof) *n_dof = ops->n;
    if (nnz) *nnz = (int64_t)ops->colidx.size();
    if (workspace_bytes) *workspace_bytes = L.total;
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "host allocation failed");
  }
}

int paro_mesh_assemble(const paro_mesh* m, const double* d_V,
                       const paro_opts_t* opts, void* d_ws, size_t bytes,
                       void* stream, paro_problem** out) {
  try {
    if (!out) return fail(PARO_EINVAL, "out is NULL");
    *out = nullptr;
    std::shared_ptr<const MeshOps> opsp;
    Layout L;
    int rc = mesh_shape(m, opts, &opsp, &L);
    if (rc) return rc;
    const MeshOps& ops = *opsp;
    if (!d_V || !d_ws) return fail(PARO_EINVAL, "NULL device pointer");
    if (((uintptr_t)d_ws & 255) != 0)
      return fail(PARO_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < L.total)
      return fail(PARO_ENOMEM, "workspace %zu bytes < %zu required", bytes,
                  L.total);
    const MeshData& md = m->m;
    hipStream_t s = (hipStream_t)stream;
    paro_problem* h = new (std::nothrow) paro_problem();
    if (!h) return fail(PARO_EDEVICE, "host allocation failed");
    Problem& p = h->p;
    std::memset(&p.box, 0, sizeof p.box);
    for (int a = 0; a < 3; ++a) {
      p.box.lo[a] = md.lo[a];
      p.box.hi[a] = md.hi[a];
    }
    p.opts = *opts;
    p.mx = p.my = p.mz = 0;
    p.n = ops.n;
    p.nnz = (int64_t)ops.colidx.size();
    p.N = opts->N;
    p.Nt = opts->N + opts->m;
    p.h[0] = p.h[1] = p.h[2] = 0.0;
    p.grid = pick_grid(p.n, p.Nt);
    p.ws_bytes = bytes;
    p.last_stream = s;
    p.nv = md.nv();
    p.ne = md.ne();
    carve(p, (char*)d_ws, L);
    auto bail = [&](int code) {
      delete h;
      return code;
    };
    auto put = [&](void* dst, const void* src, size_t n) {
      return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
    };
    hipError_t he =
        hipMemsetAsync((char*)d_ws + L.vmin, 0, L.total - L.vmin, s);
    if (he == hipSuccess)
      he = put(p.Xv, md.X.data(), sizeof(double) * md.X.size());
    if (he == hipSuccess)
      he = put(p.rowptr, ops.rowptr.data(), sizeof(int32_t) * (p.n + 1));
    if (he == hipSuccess)
      he = put(p.colidx, ops.colidx.data(), sizeof(int32_t) * p.nnz);
    if (he == hipSuccess)
      he = put(p.inc_ptr, ops.inc_ptr.data(), sizeof(int32_t) * (p.n + 1));
    if (he == hipSuccess)
      he = put(p.inc, ops.inc.data(), sizeof(int32_t) * ops.inc.size());
    if (he == hipSuccess)
      he = put(p.tets, md.tets.data(), sizeof(int32_t) * md.tets.size());
    if (he == hipSuccess)
      he = put(p.dofmap, ops.dof.data(), sizeof(int32_t) * ops.dof.size());
    if (he == hipSuccess)
      he = put(p.nbr, ops.nbr.data(), sizeof(int32_t) * ops.nbr.size());
    if (he == hipSuccess)
      he = hipMemcpyAsync(p.Vv, d_V, sizeof(double) * p.nv,
                          hipMemcpyDeviceToDevice, s);
    if (he != hipSuccess)
      return bail(fail(PARO_EDEVICE, "mesh upload: %s",
                       hipGetErrorString(he)));
    if (launch_potential_range(p.Vv, p.nv, p.vmin, p.cnt + kCntMin, p.part,
                               s) != hipSuccess)
      return bail(fail(PARO_EDEVICE, "potential range launch failed"));
    double rng[3];
    he = hipMemcpyAsync(rng, p.vmin, sizeof rng, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess)
      return bail(fail(PARO_EDEVICE, "reading the potential range: %s",
                       hipGetErrorString(he)));
    if (rng[2] != 0.0)
      return bail(fail(PARO_EINVAL, "potential has %.0f non-finite values",
                       rng[2]));
    p.sigma = opts->sigma_mode == 1 ? opts->sigma
                                    : (rng[0] >= 0.0 ? 0.0 : rng[0] - 1.0);
    if (launch_mesh_assemble(p, s) != hipSuccess)
      return bail(fail(PARO_EDEVICE, "mesh assembly launch failed"));
    desc_init(p);
    *out = h;
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_mesh_assemble");
  }
}

}  // extern "C"

namespace paro {
// Step 1 of one problem; with `status`, synchronous: it receives the
// status bits after the projection (and its re-orthonormalisation retry).
int init_impl(paro_problem* h, const double* d_U0, double* d_lambda,
                     double* d_U, void* stream, int* status) {
  if (!h || !d_U0 || !d_lambda || !d_U)
    return fail(PARO_EINVAL, "NULL argument to paro_init");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  p.last_stream = s;
  HIP_OR_FAIL(hipMemsetAsync(&p.cs->status, 0, sizeof(int), s));
  Ctx c = single_ctx(p);
  Desc& d = c.tab[0];
  d.X = const_cast<double*>(d_U0);
  d.Uout = d_U;
  d.lam = d_lambda;
  d.have_old = 0;
  if (!status) return init_tables(c, s, nullptr);
  std::vector<int> st;
  const int rc = init_tables(c, s, &st);
  if (rc) return rc;
  *status = st[0];
  return PARO_OK;
}
}  // namespace paro

extern "C" {

int paro_init(paro_problem* h, const double* d_U0, double* d_lambda,
              double* d_U, void* stream) {
  return init_impl(h, d_U0, d_lambda, d_U, stream, nullptr);
}

static int step_impl(paro_problem* h, double* d_lambda, double* d_U,
                     void* stream, paro_report_t* report, bool trust) {
  try {
    if (!h || !d_lambda || !d_U)
      return fail(PARO_EINVAL, "NULL argument to paro_step");
    Problem& p = h->p;
    hipStream_t s = (hipStream_t)stream;
    p.last_stream = s;
    Ctx c = single_ctx(p);
    // The source solves run in place on d_U (x0 = u); Rayleigh-Ritz then
    // reads W from d_U and rotates it in place.
    Desc& d = c.tab[0];
    d.U0 = d.X = d.Uout = d_U;
    d.lam = d_lambda;
    d.have_old = 1;
    return step_tables(c, s, report, true, trust);
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_step");
  }
}

int paro_step(paro_problem* h, double* d_lambda, double* d_U, void* stream,
              paro_report_t* report) {
  return step_impl(h, d_lambda, d_U, stream, report, false);
}

int paro_solve(paro_problem* h, const double* d_U0, double* d_lambda,
               double* d_U, void* stream, paro_report_t* report) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  const double t0 = now_s();
  int st = 0;
  int rc = init_impl(h, d_U0, d_lambda, d_U, s, &st);
  if (rc) return rc;
  if (st & ~kStReorth) return status_to_code(st & ~kStReorth);
  paro_report_t acc{};
  acc.reorth = (st & kStReorth) ? 1 : 0;
  acc.n_dof = p.n;
  acc.nnz = p.nnz;
  acc.sigma = p.sigma;
  int code = PARO_ENOCONV;
  for (int k = 0; k < p.opts.max_steps; ++k) {
    paro_report_t r{};
    rc = step_impl(h, d_lambda, d_U, s, &r, true);  // U from the last step
    acc.steps += 1;
    acc.pcg_iters += r.pcg_iters;
    acc.refinements += r.refinements;
    acc.reorth += r.reorth;
    acc.max_dlambda = r.max_dlambda;
    acc.max_resid = r.max_resid;
    if (rc != PARO_OK && rc != PARO_ENOCONV) {
      code = rc;
      break;
    }
    if (rc == PARO_ENOCONV) {  // CG cap: keep going, report at the end
      code = rc;
      continue;
    }
    if (p.opts.lambda_tol > 0.0 && r.max_dlambda <= p.opts.lambda_tol &&
        r.max_resid <= p.opts.resid_tol) {
      code = PARO_OK;
      break;
    }
    code = PARO_ENOCONV;
  }
  acc.seconds = now_s() - t0;
  acc.status = code;
  if (report) *report = acc;
  if (code == PARO_ENOCONV)
    fail(PARO_ENOCONV, "max_steps = %d reached before the tolerances",
         p.opts.max_steps);
  return code;
}

int paro_update_potential(paro_problem* h, const double* d_V, void* stream) {
  try {
    if (!h || !d_V) return fail(PARO_EINVAL, "NULL argument");
    Problem& p = h->p;
    if (p.csr)
      return fail(PARO_EINVAL,
                  "paro_update_potential serves box problems; assemble a "
                  "mesh problem again for a new potential");
    hipStream_t s = (hipStream_t)stream;
    p.last_stream = s;
    const int64_t nv =
        (int64_t)(p.box.nx + 1) * (p.box.ny + 1) * (p.box.nz + 1);
    HIP_OR_FAIL(
        launch_potential_range(d_V, nv, p.vmin, p.cnt + kCntMin, p.part, s));
    double rng[3];
    HIP_OR_FAIL(hipMemcpyAsync(rng, p.vmin, sizeof rng, hipMemcpyDeviceToHost,
                               s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (rng[2] != 0.0)
      return fail(PARO_EINVAL, "potential has %.0f non-finite values",
                  rng[2]);
    if (p.opts.sigma_mode != 1) p.sigma = rng[0] >= 0.0 ? 0.0 : rng[0] - 1.0;
    HIP_OR_FAIL(launch_assemble(p, d_V, s));
    p.hd.sigma = p.sigma;
    p.hd.start_ready = p.hd.hu_valid = 0;  // the operator changed
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_update_potential");
  }
}

double paro_sigma(const paro_problem* h) { return h ? h->p.sigma : 0.0; }

void paro_destroy(paro_problem* h) {
  if (!h) return;
  delete h->p.timing;
  delete h->p.graphs;
  delete h;
}

size_t paro_batch_workspace_bytes(int32_t count) {
  if (count < 1) return 0;
  return batch_layout(count).total;
}

}  // extern "C"

namespace paro {
int batch_init_impl(paro_problem* const* probs, int32_t count,
                    const double* const* d_U0, double* const* d_lambda,
                    double* const* d_U, void* d_ws, size_t bytes,
                    void* stream, std::vector<int>* status) {
  try {
    if (!d_U0 || !d_lambda || !d_U) return fail(PARO_EINVAL, "NULL arrays");
    Ctx c;
    int predict[5] = {0, 0, 0, 0, 0};
    int rc = batch_ctx(c, probs, count, d_ws, bytes, predict);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
      if (!d_U0[i] || !d_lambda[i] || !d_U[i])
        return fail(PARO_EINVAL, "NULL device pointer for problem %d", i);
      probs[i]->p.last_stream = s;
      HIP_OR_FAIL(hipMemsetAsync(&probs[i]->p.cs->status, 0, sizeof(int), s));
      Desc& d = c.tab[i];
      d.X = const_cast<double*>(d_U0[i]);
      d.Uout = d_U[i];
      d.lam = d_lambda[i];
      d.have_old = 0;
    }
    return init_tables(c, s, status);
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_batch_init");
  }
}
}  // namespace paro

extern "C" {

int paro_batch_init(paro_problem* const* probs, int32_t count,
                    const double* const* d_U0, double* const* d_lambda,
                    double* const* d_U, void* d_ws, size_t bytes,
                    void* stream) {
  return paro::batch_init_impl(probs, count, d_U0, d_lambda, d_U, d_ws, bytes,
                               stream, nullptr);
}

// Batch steps keep their CG prediction between calls of one thread.
static thread_local int g_batch_predict[5] = {0, 0, 0, 0, 0};

}  // extern "C"

namespace paro {
int batch_step_impl(paro_problem* const* probs, int32_t count,
                    double* const* d_lambda, double* const* d_U, void* d_ws,
                    size_t bytes, void* stream, paro_report_t* reports,
                    bool trust) {
  try {
    if (!d_lambda || !d_U) return fail(PARO_EINVAL, "NULL arrays");
    Ctx c;
    int rc = batch_ctx(c, probs, count, d_ws, bytes, g_batch_predict);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
      if (!d_lambda[i] || !d_U[i])
        return fail(PARO_EINVAL, "NULL device pointer for problem %d", i);
      probs[i]->p.last_stream = s;
      Desc& d = c.tab[i];
      d.U0 = d.X = d.Uout = d_U[i];
      d.lam = d_lambda[i];
      d.have_old = 1;
    }
    return step_tables(c, s, reports, false, trust);
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_batch_step");
  }
}
}  // namespace paro

extern "C" {

int paro_batch_step(paro_problem* const* probs, int32_t count,
                    double* const* d_lambda, double* const* d_U, void* d_ws,
                    size_t bytes, void* stream, paro_report_t* reports) {
  return paro::batch_step_impl(probs, count, d_lambda, d_U, d_ws, bytes,
                               stream, reports, false);
}

int paro_batch_solve(paro_problem* const* probs, int32_t count,
                     const double* const* d_U0, double* const* d_lambda,
                     double* const* d_U, void* d_ws, size_t bytes,
                     void* stream, paro_report_t* reports) {
  if (!reports) return fail(PARO_EINVAL, "reports are required");
  const double t0 = now_s();
  std::vector<int> st;
  int rc = paro::batch_init_impl(probs, count, d_U0, d_lambda, d_U, d_ws,
                                 bytes, stream, &st);
  if (rc) return rc;
  std::vector<int> active;
  for (int i = 0; i < count; ++i) {
    reports[i] = paro_report_t{};
    reports[i].n_dof = probs[i]->p.n;
    reports[i].nnz = probs[i]->p.nnz;
    reports[i].sigma = probs[i]->p.sigma;
    reports[i].status = PARO_ENOCONV;
    // Start blocks that stay dependent after the re-orthonormalisation.
    reports[i].reorth = (st[i] & kStReorth) ? 1 : 0;
    if (st[i] & ~kStReorth)
      reports[i].status = status_to_code(st[i] & ~kStReorth);
    else
      active.push_back(i);
  }
  std::vector<paro_problem*> ps;
  std::vector<double*> ls, us;
  std::vector<paro_report_t> rs;
  while (!active.empty()) {
    ps.clear();
    ls.clear();
    us.clear();
    for (int i : active) {
      ps.push_back(probs[i]);
      ls.push_back(d_lambda[i]);
      us.push_back(d_U[i]);
    }
    rs.assign(active.size(), paro_report_t{});
    rc = batch_step_impl(ps.data(), (int)ps.size(), ls.data(), us.data(),
                         d_ws, bytes, stream, rs.data(), true);
    if (rc) return rc;
    std::vector<int> still;
    for (size_t k = 0; k < active.size(); ++k) {
      const int i = active[k];
      paro_report_t& a = reports[i];
      const paro_report_t& r = rs[k];
      const paro_opts_t& o = probs[i]->p.opts;
      a.steps += 1;
      a.pcg_iters += r.pcg_iters;
      a.refinements += r.refinements;
      a.reorth += r.reorth;
      a.max_dlambda = r.max_dlambda;
      a.max_resid = r.max_resid;
      bool done = false;
      if (r.status != PARO_OK && r.status != PARO_ENOCONV) {
        a.status = r.status;
        done = true;
      } else if (o.lambda_tol > 0.0 && r.max_dlambda <= o.lambda_tol &&
                 r.max_resid <= o.resid_tol) {
        a.status = PARO_OK;
        done = true;
      } else if (a.steps >= o.max_steps) {
        a.status = PARO_ENOCONV;
        done = true;
      }
      a.seconds = now_s() - t0;
      if (!done) still.push_back(i);
    }
    active.swap(still);
  }
  int first = PARO_OK;
  for (int i = 0; i < count; ++i)
    if (reports[i].status != PARO_OK) {
      first = reports[i].status;
      break;
    }
  if (first != PARO_OK)
    fail(first, "problem(s) of the batch ended with status %d", first);
  return first;
}

void paro_set_graphs(int on) { g_graphs_on.store(on ? 1 : 0); }

void paro_set_persistent(int on) { g_persistent_on.store(on ? 1 : 0); }

void paro_set_matrix_free(int on) { g_matfree_on.store(on ? 1 : 0); }

namespace {
size_t up256n(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

int paro_nonlocal_query(const paro_problem* h, int32_t k, size_t* bytes) {
  if (!h || !bytes) return fail(PARO_EINVAL, "NULL argument");
  const Problem& p = h->p;
  if (k < 0 || k > 32)
    return fail(PARO_EINVAL, "projector count must be 0..32");
  *bytes = up256n(sizeof(double) * (size_t)p.n * k) +
           up256n(sizeof(double) * (size_t)k * kNtMax) +
           up256n(sizeof(double) * (size_t)k * kNtMax * cm_tiles(p.n));
  return PARO_OK;
}

int paro_set_nonlocal(paro_problem* h, const double* d_zeta, int32_t k,
                      void* d_ws, size_t bytes, void* stream) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  if (p.csr && k != 0)
    return fail(PARO_EINVAL, "the nonlocal term serves box problems only");
  if (k == 0) {
    p.Zp = nullptr;
    p.kz = 0;
    p.zy = p.zpart = nullptr;
    p.hd.Zp = nullptr;
    p.hd.kz = 0;
    p.hd.start_ready = p.hd.hu_valid = 0;  // the operator changed
    return PARO_OK;
  }
  if (p.opts.precision != PARO_FP64)
    return fail(PARO_EINVAL, "the nonlocal term needs precision PARO_FP64");
  size_t need = 0;
  const int rc = paro_nonlocal_query(h, k, &need);
  if (rc) return rc;
  if (!d_zeta || !d_ws) return fail(PARO_EINVAL, "NULL argument");
  if (((uintptr_t)d_ws & 255) != 0)
    return fail(PARO_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(PARO_ENOMEM, "nonlocal workspace too small: %zu < %zu",
                bytes, need);
  char* base = (char*)d_ws;
  double* Z = (double*)base;
  base += up256n(sizeof(double) * (size_t)p.n * k);
  p.zy = (double*)base;
  base += up256n(sizeof(double) * (size_t)k * kNtMax);
  p.zpart = (double*)base;
  HIP_OR_FAIL(launch_nl_mass(p.hd, d_zeta, Z, k, (hipStream_t)stream));
  p.Zp = Z;
  p.kz = k;
  p.hd.Zp = p.Zp;
  p.hd.kz = k;
  p.hd.zy = p.zy;
  p.hd.zpart = p.zpart;
  p.hd.start_ready = p.hd.hu_valid = 0;  // the operator changed
  return PARO_OK;
}

int paro_set_clusters(paro_problem* h, const int32_t* sizes, int32_t count,
                      void* stream) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  if (count == 0) {
    p.clustered = false;
    p.hd.clus = nullptr;
    return PARO_OK;
  }
  if (count < 0 || count > p.Nt || !sizes)
    return fail(PARO_EINVAL, "cluster count must be 0..%d", p.Nt);
  int ids[kNtMax];
  int c = 0;
  for (int k = 0; k < count; ++k) {
    if (sizes[k] < 1 || c + sizes[k] > p.Nt)
      return fail(PARO_EINVAL, "cluster sizes must be >= 1 and sum to %d",
                  p.Nt);
    for (int j = 0; j < sizes[k]; ++j) ids[c++] = k;
  }
  if (c != p.Nt)
    return fail(PARO_EINVAL, "cluster sizes must sum to N + m = %d", p.Nt);
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(hipMemcpyAsync(p.clus, ids, sizeof(int) * p.Nt,
                             hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));  // ids is a stack array
  p.clustered = true;
  p.hd.clus = p.clus;
  return PARO_OK;
}

void paro_set_autotune(int on) { g_autotune_on.store(on ? 1 : 0); }

int paro_set_tuning(paro_problem* h, int32_t variant, int32_t blocks) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  const int vmax = p.hd.zm ? 2 : 0;
  if (variant < -1 || variant > vmax)
    return fail(PARO_EINVAL, "variant must be in [-1, %d] for this problem",
                vmax);
  if (blocks < 8 || blocks > p.hd.ns || blocks % 8)
    return fail(PARO_EINVAL, "blocks must be a multiple of 8 in [8, %d]",
                p.hd.ns);
  p.hd.cg_var = variant;
  p.hd.nb = blocks;
  return PARO_OK;
}

int paro_tuned(const paro_problem* h, int32_t* variant, int32_t* blocks) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  if (variant) *variant = h->p.hd.cg_var;
  if (blocks) *blocks = h->p.hd.nb;
  return PARO_OK;
}

int paro_set_timing(paro_problem* h, int on) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  if (!p.timing) p.timing = new (std::nothrow) Timing();
  if (!p.timing) return fail(PARO_EDEVICE, "host allocation failed");
  Timing& t = *p.timing;
  t.resolve();
  for (int k = 0; k < PARO_ST_NUM; ++k) {
    t.launches[k] = 0;
    t.ms[k] = 0.0;
  }
  unsigned long long c[2] = {0, 0};
  HIP_OR_FAIL(hipMemcpyAsync(c, &p.cs->cg_iters, sizeof c,
                             hipMemcpyDeviceToHost, p.last_stream));
  HIP_OR_FAIL(hipStreamSynchronize(p.last_stream));
  t.iters0 = c[0];
  t.cols0 = c[1];
  t.on = on != 0;
  return PARO_OK;
}

int paro_get_timing(paro_problem* h, paro_timing_t* out) {
  if (!h || !out) return fail(PARO_EINVAL, "NULL argument");
  Problem& p = h->p;
  std::memset(out, 0, sizeof *out);
  HIP_OR_FAIL(hipStreamSynchronize(p.last_stream));
  unsigned long long c[2] = {0, 0};
  HIP_OR_FAIL(hipMemcpyAsync(c, &p.cs->cg_iters, sizeof c,
                             hipMemcpyDeviceToHost, p.last_stream));
  HIP_OR_FAIL(hipStreamSynchronize(p.last_stream));
  if (p.timing) {
    p.timing->resolve();
    for (int k = 0; k < PARO_ST_NUM; ++k) {
      out->launches[k] = p.timing->launches[k];
      out->ms[k] = p.timing->ms[k];
    }
    c[0] -= p.timing->iters0;
    c[1] -= p.timing->cols0;
  }
  out->cg_iters = (int64_t)c[0];
  out->cg_col_iters = (int64_t)c[1];
  return PARO_OK;
}

int paro_export_csr(paro_problem* h, int32_t* d_rowptr, int32_t* d_col,
                    double* d_valA, double* d_valM, double* h_sigma,
                    void* stream) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  if (p.csr) {  // the operator is stored in CSR already
    const auto cp = [&](void* dst, const void* src, size_t n) {
      return dst ? hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s)
                 : hipSuccess;
    };
    HIP_OR_FAIL(cp(d_rowptr, p.rowptr, sizeof(int32_t) * (p.n + 1)));
    HIP_OR_FAIL(cp(d_col, p.colidx, sizeof(int32_t) * p.nnz));
    HIP_OR_FAIL(cp(d_valA, p.valA, sizeof(double) * p.nnz));
    HIP_OR_FAIL(cp(d_valM, p.valM, sizeof(double) * p.nnz));
  } else if (d_rowptr || d_col || d_valA || d_valM) {
    HIP_OR_FAIL(launch_csr_export(p, d_rowptr, d_col, d_valA, d_valM, s));
  }
  if (h_sigma) *h_sigma = p.sigma;
  return PARO_OK;
}

int paro_spmm(paro_problem* h, int which, const double* d_X, double* d_Y,
              int ncols, void* stream) {
  if (!h || !d_X || !d_Y) return fail(PARO_EINVAL, "NULL argument");
  if (which < 0 || which > 2) return fail(PARO_EINVAL, "which must be 0..2");
  if (ncols < 1 || ncols > kNtMax)
    return fail(PARO_EINVAL, "ncols must be 1..%d", kNtMax);
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  Ctx c = single_ctx(p);
  Desc& d = c.tab[0];
  set_cols(d, ncols);
  d.X = const_cast<double*>(d_X);
  d.Y1 = which == 1 ? nullptr : d_Y;
  d.Y2 = which == 1 ? d_Y : nullptr;
  d.s1 = which == 2 ? p.sigma : 0.0;
  int rc = upload(c, s);
  if (rc) return rc;
  HIP_OR_FAIL(launch_spmm(c.L, false, s, c.timing));
  return PARO_OK;
}

int paro_gram(paro_problem* h, const double* d_W, const double* d_Y,
              double* d_G, int ncols, void* stream) {
  if (!h || !d_W || !d_Y || !d_G) return fail(PARO_EINVAL, "NULL argument");
  if (ncols < 1 || ncols > h->p.Nt)
    return fail(PARO_EINVAL, "ncols must be 1..%d", h->p.Nt);
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  Ctx c = single_ctx(p);
  Desc& d = c.tab[0];
  set_cols(d, ncols);
  d.X = const_cast<double*>(d_W);
  d.Y1 = const_cast<double*>(d_Y);
  d.Y2 = d_G;
  int rc = upload(c, s);
  if (rc) return rc;
  HIP_OR_FAIL(launch_gram_full(c.L, s, c.timing));
  return PARO_OK;
}

int paro_gram_noalloc(const double* d_W, const double* d_Y, double* d_G,
                      int64_t n, int ncols, void* stream) {
  if (!d_W || !d_Y || !d_G) return fail(PARO_EINVAL, "NULL argument");
  if (ncols < 1 || ncols > kNtMax)
    return fail(PARO_EINVAL, "ncols must be 1..%d (the scratch holds %zu "
                "bytes: the partials of %d columns)", kNtMax, kNoAllocBytes,
                kNtMax);
  if (n < 1 || n > (int64_t)INT32_MAX)
    return fail(PARO_EINVAL, "n must be 1..%d", INT32_MAX);
  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Desc d;
  std::memset(&d, 0, sizeof d);
  d.n = n;
  set_cols(d, ncols);
  d.g0 = 0;
  // The segments of paro_gram on a problem of n rows and ncols orbitals.
  d.gnb = d.gns = std::min(pick_grid(n, ncols), kGramGrid);
  d.X = const_cast<double*>(d_W);
  d.Y1 = const_cast<double*>(d_Y);
  d.Y2 = d_G;
  d.gpart = (double*)((unsigned char*)base + kNoAllocDescBytes);
  Desc* dd = (Desc*)base;
  hipLaunchKernelGGL(store_desc_kernel, dim3(1), dim3(64), 0, s, d, dd);
  HIP_OR_FAIL(hipGetLastError());
  Launch L = make_launch(dd, &d, 1);
  HIP_OR_FAIL(launch_gram_full(L, s, nullptr));
  return PARO_OK;
}

int paro_small_geneig(const double* d_A, const double* d_B, int n,
                      double* d_theta, double* d_C, int32_t* d_info,
                      void* stream) {
  if (!d_A || !d_B || !d_theta || !d_C || !d_info)
    return fail(PARO_EINVAL, "NULL argument");
  if (n < 1 || n > kNtMax) return fail(PARO_EINVAL, "n must be 1..%d", kNtMax);
  HIP_OR_FAIL(launch_small_geneig(d_A, d_B, n, d_theta, d_C, d_info,
                                  (hipStream_t)stream));
  return PARO_OK;
}

int paro_pcg(paro_problem* h, const double* d_B, double* d_X, int ncols,
             int32_t* h_iters, void* stream) {
  try {
    if (!h || !d_B || !d_X) return fail(PARO_EINVAL, "NULL argument");
    Problem& p = h->p;
    if (ncols < 1 || ncols > p.Nt)
      return fail(PARO_EINVAL, "ncols must be 1..%d", p.Nt);
    hipStream_t s = (hipStream_t)stream;
    p.last_stream = s;
    const size_t bytes = sizeof(double) * (size_t)p.n * ncols;
    HIP_OR_FAIL(hipMemcpyAsync(p.X, d_X, bytes, hipMemcpyDeviceToDevice, s));
    Ctx c = single_ctx(p);
    forget_rotation(c);  // the CG state and H U, M U are overwritten
    Desc& d = c.tab[0];
    set_cols(d, ncols);
    d.U0 = d.X = p.X;
    d.Bin = d_B;
    d.lam = nullptr;
    const bool csr_hu = mark_csr_starts(c);
    int rc = upload(c, s);
    if (rc) return rc;
    if (csr_hu) HIP_OR_FAIL(launch_csr_dual(c.L, 2, s, c.timing));
    HIP_OR_FAIL(launch_pcg_start(c.L, s, c.timing));
    rc = solve_sources(c, s, nullptr);
    if (rc) return rc;
    HIP_OR_FAIL(hipMemcpyAsync(d_X, p.X, bytes, hipMemcpyDeviceToDevice, s));
    int st = 0;
    int iters[kNtMax];
    HIP_OR_FAIL(hipMemcpyAsync(&st, &p.cs->status, sizeof st,
                               hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipMemcpyAsync(iters, p.cs->iters, sizeof(int) * ncols,
                               hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (h_iters)
      for (int k = 0; k < ncols; ++k) h_iters[k] = iters[k];
    return status_to_code(st);
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_pcg");
  }
}

}  // extern "C"
