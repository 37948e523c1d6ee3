// C ABI of libparo: argument checking, workspace layout and the host-side
// sequencing of one ParO step (Algorithm A.1, Steps 3 and 4) and of a
// whole solve.  Every arithmetic step runs in the kernels of assemble.hip
// and solver.hip; the host only launches them and polls small flags.
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "paro_internal.h"

struct paro_problem {
  paro::Problem p;
};

namespace paro {

// Host-side event timing of kernel launches (measurement only).
struct Timing {
  bool on = false;
  struct Open {
    int stage;
    hipEvent_t a;
  };
  struct Pend {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Open> open;
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
    for (const Open& o : open) pool.push_back(o.a);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

int timing_begin(Problem& p, int stage, hipStream_t s) {
  Timing* t = p.timing;
  if (!t || !t->on) return -1;
  hipEvent_t a = t->get();
  if (!a || hipEventRecord(a, s) != hipSuccess) return -1;
  t->open.push_back({stage, a});
  return (int)t->open.size() - 1;
}

void timing_end(Problem& p, int slot, hipStream_t s) {
  Timing* t = p.timing;
  if (!t || slot < 0 || slot >= (int)t->open.size()) return;
  hipEvent_t b = t->get();
  if (b && hipEventRecord(b, s) == hipSuccess)
    t->pend.push_back({t->open[slot].stage, t->open[slot].a, b});
  else
    t->pool.push_back(t->open[slot].a);
  t->open.erase(t->open.begin() + slot);
  if (t->pend.size() > 4096) t->resolve();
}

namespace {

thread_local std::string g_err = "no error";

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
  if (o->precision == PARO_FP32_INNER &&
      (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0)))
    return fail(PARO_EINVAL, "inner_rtol must lie in (0, 1)");
  if (o->sigma_mode == 1 && !std::isfinite(o->sigma))
    return fail(PARO_EINVAL, "sigma must be finite");
  return PARO_OK;
}

void carve(Problem& p, char* base, const Layout& L) {
  auto at = [&](size_t off) { return (void*)(base + off); };
  p.rowptr = (int32_t*)at(L.rowptr);
  p.col = (int32_t*)at(L.col);
  p.valA = (double*)at(L.valA);
  p.valM = (double*)at(L.valM);
  p.valA32 = L.valA32 ? (float*)at(L.valA32) : nullptr;
  p.dinv = (double*)at(L.dinv);
  p.dinv32 = L.dinv32 ? (float*)at(L.dinv32) : nullptr;
  p.X = (double*)at(L.X);
  p.R = (double*)at(L.R);
  p.P = (double*)at(L.P);
  p.Q = (double*)at(L.Q);
  p.B = L.B ? (double*)at(L.B) : nullptr;
  p.R32 = L.R32 ? (float*)at(L.R32) : nullptr;
  p.P32 = L.P32 ? (float*)at(L.P32) : nullptr;
  p.Q32 = L.Q32 ? (float*)at(L.Q32) : nullptr;
  p.X32 = L.X32 ? (float*)at(L.X32) : nullptr;
  p.part = (double*)at(L.part);
  p.gpart = (double*)at(L.gpart);
  p.gsum = (double*)at(L.gsum);
  p.Ah = (double*)at(L.Ah);
  p.Bh = (double*)at(L.Bh);
  p.C = (double*)at(L.C);
  p.theta = (double*)at(L.theta);
  p.vmin = (double*)at(L.vmin);
  p.cs = (ColState*)at(L.cs);
  p.si = (StepInfo*)at(L.si);
  p.cnt = (unsigned*)at(L.cnt);
  p.flag = (int*)at(L.flag);
}

int pick_grid(int64_t n, int Nt) {
  const int V = (Nt % 2 == 0) ? 2 : 1;
  const int cpr = Nt / V, tr = kBlock / cpr;
  const int64_t tiles = (n + tr - 1) / tr;
  int64_t g = tiles < kGridDefault ? tiles : kGridDefault;
  g = ((g + 7) / 8) * 8;
  return (int)(g < 8 ? 8 : g);
}

// Host reads of small device values (flags, scalars, the step report).
template <typename T>
int read_back(paro_problem* h, const T* dsrc, T* out, size_t count,
              hipStream_t s) {
  (void)h;
  HIP_OR_FAIL(hipMemcpyAsync(out, dsrc, sizeof(T) * count,
                             hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  return PARO_OK;
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

// The tail of ColState read back at each poll (one copy).
struct ColTail {
  int iters[kNtMax];
  int n_active[2];
  int n_outer;
  int status;
  int maxit;
  int pad[3];
  unsigned long long cg_iters;
  unsigned long long cg_col_iters;
};
static_assert(offsetof(ColState, cg_col_iters) - offsetof(ColState, iters) ==
                  offsetof(ColTail, cg_col_iters),
              "ColTail must mirror the tail of ColState");

int read_tail(paro_problem* h, ColTail* t, hipStream_t s) {
  HIP_OR_FAIL(hipMemcpyAsync(t, &h->p.cs->iters[0], sizeof(ColTail),
                             hipMemcpyDeviceToHost, s));
  HIP_OR_FAIL(hipStreamSynchronize(s));
  return PARO_OK;
}

// Run CG iterations (FP64 or FP32) until no column is active.  The first
// batch of launches is as long as the previous solve in the same slot took,
// so that a converging solve usually needs one poll; later batches are
// short top-ups.
int run_cg(paro_problem* h, int ncols, bool fp32, hipStream_t s, int slot) {
  Problem& p = h->p;
  ColTail t;
  int rc = read_tail(h, &t, s);
  if (rc) return rc;
  if (t.n_active[0] == 0) return PARO_OK;
  const unsigned long long start = t.cg_iters;
  const int64_t cap = (int64_t)p.opts.pcg_maxit + 64;
  int pred = p.cg_predict[slot];
  int chunk = pred < 2 ? 2 : (pred > 256 ? 256 : pred);
  int par = 0;
  int64_t launched = 0;
  while (true) {
    if (launched >= cap)
      return fail(PARO_EDEVICE, "CG loop did not terminate on the device");
    for (int k = 0; k < chunk; ++k) {
      hipError_t e = fp32 ? launch_pcg32_iter(p, ncols, par, s)
                          : launch_pcg_iter(p, ncols, par, s);
      if (e != hipSuccess)
        return fail(PARO_EDEVICE, "CG launch: %s", hipGetErrorString(e));
      par ^= 1;
    }
    launched += chunk;
    rc = read_tail(h, &t, s);
    if (rc) return rc;
    if (p.timing) p.timing->resolve();
    if (t.n_active[par] == 0) break;
    chunk = (pred + 3) / 4;
    chunk = chunk < 2 ? 2 : (chunk > 16 ? 16 : chunk);
  }
  p.cg_predict[slot] = (int)(t.cg_iters - start);
  return PARO_OK;
}

// Source solves of one step, from the state prepared by a start kernel
// (X = x0, R, P, B, act[0]).  Returns the device status as a code.
int solve_sources(paro_problem* h, int ncols, hipStream_t s,
                  int64_t* refinements) {
  Problem& p = h->p;
  if (p.opts.precision == PARO_FP64) {
    int rc = run_cg(h, ncols, false, s, 0);
    if (rc) return rc;
  } else {
    for (int pass = 0;; ++pass) {
      HIP_OR_FAIL(launch_refine_residual(p, ncols, pass == 0, s));
      int no = 0;
      int rc = read_back(h, &p.cs->n_outer, &no, 1, s);
      if (rc) return rc;
      if (no == 0) break;
      if (pass > 200)
        return fail(PARO_EDEVICE, "refinement loop did not terminate");
      rc = run_cg(h, ncols, true, s, 1 + (pass < 3 ? pass : 3));
      if (rc) return rc;
      HIP_OR_FAIL(launch_refine_update(p, ncols, s));
      if (refinements) ++*refinements;
    }
  }
  return PARO_OK;
}

}  // namespace

Layout make_layout(int64_t n, int64_t nnz, int Nt, int precision) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const bool f32 = precision == PARO_FP32_INNER;
  const size_t blk = (size_t)n * Nt;
  L.rowptr = take(sizeof(int32_t) * (n + 1));
  L.col = take(sizeof(int32_t) * nnz);
  L.valA = take(sizeof(double) * nnz);
  L.valM = take(sizeof(double) * nnz);
  L.valA32 = f32 ? take(sizeof(float) * nnz) : 0;
  L.dinv = take(sizeof(double) * n);
  L.dinv32 = f32 ? take(sizeof(float) * n) : 0;
  L.X = take(sizeof(double) * blk);
  L.R = take(sizeof(double) * blk);
  L.P = take(sizeof(double) * blk);
  L.Q = take(sizeof(double) * blk);
  L.B = f32 ? take(sizeof(double) * blk) : 0;
  L.R32 = f32 ? take(sizeof(float) * blk) : 0;
  L.P32 = f32 ? take(sizeof(float) * blk) : 0;
  L.Q32 = f32 ? take(sizeof(float) * blk) : 0;
  L.X32 = f32 ? take(sizeof(float) * blk) : 0;
  L.part = take(sizeof(double) * 3 * (size_t)kGridMax * kNtMax);
  L.gpart = take(sizeof(double) * (size_t)kGramGrid * gram_tiles(Nt));
  L.gsum = take(sizeof(double) * (size_t)kGramY * gram_tiles(Nt));
  L.Ah = take(sizeof(double) * kNtMax * kNtMax);
  L.Bh = take(sizeof(double) * kNtMax * kNtMax);
  L.C = take(sizeof(double) * kNtMax * kNtMax);
  L.theta = take(sizeof(double) * kNtMax);
  L.vmin = take(sizeof(double) * 4);
  L.cs = take(sizeof(ColState));
  L.si = take(sizeof(StepInfo));
  L.cnt = take(sizeof(unsigned) * kCntNum);
  L.flag = take(sizeof(int) * 16);
  L.total = off;
  return L;
}

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
  o->inner_rtol = 1e-4;
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
        make_layout(n, z, opts->N + opts->m, opts->precision).total;
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
    const Layout L = make_layout(n, z, p.Nt, opts->precision);
    carve(p, (char*)d_ws, L);
    auto bail = [&](int code) {
      delete h;
      return code;
    };
    // Zero the small state (counters, column state, step info).
    hipError_t he = hipMemsetAsync((char*)d_ws + L.vmin, 0, L.total - L.vmin, s);
    if (he != hipSuccess)
      return bail(fail(PARO_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(he)));
    const int64_t nv = (int64_t)(box->nx + 1) * (box->ny + 1) * (box->nz + 1);
    if (launch_potential_range(d_V, nv, p.vmin, p.cnt + kCntMin, p.part, s) !=
        hipSuccess)
      return bail(fail(PARO_EDEVICE, "potential range launch failed"));
    double rng[3];
    rc = read_back(h, p.vmin, rng, 3, s);
    if (rc) return bail(rc);
    if (rng[2] != 0.0)
      return bail(fail(PARO_EINVAL, "potential has %.0f non-finite values",
                       rng[2]));
    if (opts->sigma_mode == 1)
      p.sigma = opts->sigma;
    else
      p.sigma = rng[0] >= 0.0 ? 0.0 : rng[0] - 1.0;
    if (launch_assemble(p, d_V, s) != hipSuccess)
      return bail(fail(PARO_EDEVICE, "assembly launch failed"));
    *out = h;
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_assemble");
  }
}

int paro_init(paro_problem* h, const double* d_U0, double* d_lambda,
              double* d_U, void* stream) {
  if (!h || !d_U0 || !d_lambda || !d_U)
    return fail(PARO_EINVAL, "NULL argument to paro_init");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  p.last_stream = s;
  HIP_OR_FAIL(hipMemsetAsync(&p.cs->status, 0, sizeof(int), s));
  HIP_OR_FAIL(launch_rayleigh_ritz(p, d_U0, d_lambda, d_U, p.Nt, false, s));
  return PARO_OK;
}

int paro_step(paro_problem* h, double* d_lambda, double* d_U, void* stream,
              paro_report_t* report) {
  try {
    if (!h || !d_lambda || !d_U)
      return fail(PARO_EINVAL, "NULL argument to paro_step");
    Problem& p = h->p;
    hipStream_t s = (hipStream_t)stream;
    p.last_stream = s;
    const double t0 = now_s();
    const bool f32 = p.opts.precision == PARO_FP32_INNER;
    // The source solves run in place on d_U (x0 = u); Rayleigh-Ritz then
    // reads W from d_U and rotates it in place.
    struct XGuard {
      Problem& p;
      double* saved;
      ~XGuard() { p.X = saved; }
    } guard{p, p.X};
    p.X = d_U;
    HIP_OR_FAIL(launch_pcg_start(p, d_lambda, d_U, p.Nt, f32, s));
    int64_t refinements = 0;
    int rc = solve_sources(h, p.Nt, s, &refinements);
    if (rc) return rc;
    int st = 0;
    rc = read_back(h, &p.cs->status, &st, 1, s);
    if (rc) return rc;
    if (st & (kStNonFinite | kStNotSpd)) return status_to_code(st);
    HIP_OR_FAIL(launch_rayleigh_ritz(p, p.X, d_lambda, d_U, p.Nt, true, s));
    if (report) {
      rc = read_back(h, &p.cs->status, &st, 1, s);
      if (rc) return rc;
      StepInfo si;
      rc = read_back(h, p.si, &si, 1, s);
      if (rc) return rc;
      int iters[kNtMax];
      rc = read_back(h, p.cs->iters, iters, p.Nt, s);
      if (rc) return rc;
      int64_t mx = 0;
      for (int c = 0; c < p.Nt; ++c) mx = iters[c] > mx ? iters[c] : mx;
      report->status = 0;
      report->steps = 1;
      report->pcg_iters = mx;
      report->refinements = refinements;
      report->n_dof = p.n;
      report->nnz = p.nnz;
      report->max_dlambda = si.max_dlambda;
      report->max_resid = si.max_resid;
      report->sigma = p.sigma;
      report->seconds = now_s() - t0;
      report->status = status_to_code(st);
      return report->status;
    }
    return PARO_OK;
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_step");
  }
}

int paro_solve(paro_problem* h, const double* d_U0, double* d_lambda,
               double* d_U, void* stream, paro_report_t* report) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  const double t0 = now_s();
  int rc = paro_init(h, d_U0, d_lambda, d_U, s);
  if (rc) return rc;
  int st = 0;
  rc = read_back(h, &p.cs->status, &st, 1, s);
  if (rc) return rc;
  if (st) return status_to_code(st);
  paro_report_t acc{};
  acc.n_dof = p.n;
  acc.nnz = p.nnz;
  acc.sigma = p.sigma;
  int code = PARO_ENOCONV;
  for (int k = 0; k < p.opts.max_steps; ++k) {
    paro_report_t r{};
    rc = paro_step(h, d_lambda, d_U, s, &r);
    acc.steps += 1;
    acc.pcg_iters += r.pcg_iters;
    acc.refinements += r.refinements;
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
  if (code == PARO_ENOCONV && g_err.empty())
    fail(PARO_ENOCONV, "max_steps reached");
  if (code == PARO_ENOCONV)
    fail(PARO_ENOCONV, "max_steps = %d reached before the tolerances",
         p.opts.max_steps);
  return code;
}

void paro_destroy(paro_problem* h) {
  if (!h) return;
  delete h->p.timing;
  delete h;
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
  int rc = read_back(h, &p.cs->cg_iters, c, 2, p.last_stream);
  if (rc) return rc;
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
  int rc = read_back(h, &p.cs->cg_iters, c, 2, p.last_stream);
  if (rc) return rc;
  if (p.timing) {
    p.timing->resolve();
    for (int k = 0; k < PARO_ST_NUM; ++k) {
      out->launches[k] = p.timing->launches[k];
      out->ms[k] = p.timing->ms[k];
    }
    c[0] -= p.timing->iters0;
    c[1] -= p.timing->cols0;
  }
  out->cg_iters = c[0];
  out->cg_col_iters = c[1];
  return PARO_OK;
}

int paro_export_csr(paro_problem* h, int32_t* d_rowptr, int32_t* d_col,
                    double* d_valA, double* d_valM, double* h_sigma,
                    void* stream) {
  if (!h) return fail(PARO_EINVAL, "NULL problem");
  Problem& p = h->p;
  hipStream_t s = (hipStream_t)stream;
  if (d_rowptr)
    HIP_OR_FAIL(hipMemcpyAsync(d_rowptr, p.rowptr, 4 * (p.n + 1),
                               hipMemcpyDeviceToDevice, s));
  if (d_col)
    HIP_OR_FAIL(hipMemcpyAsync(d_col, p.col, 4 * p.nnz,
                               hipMemcpyDeviceToDevice, s));
  if (d_valA)
    HIP_OR_FAIL(hipMemcpyAsync(d_valA, p.valA, 8 * p.nnz,
                               hipMemcpyDeviceToDevice, s));
  if (d_valM)
    HIP_OR_FAIL(hipMemcpyAsync(d_valM, p.valM, 8 * p.nnz,
                               hipMemcpyDeviceToDevice, s));
  if (h_sigma) *h_sigma = p.sigma;
  return PARO_OK;
}

int paro_spmm(paro_problem* h, int which, const double* d_X, double* d_Y,
              int ncols, void* stream) {
  if (!h || !d_X || !d_Y) return fail(PARO_EINVAL, "NULL argument");
  if (which < 0 || which > 2) return fail(PARO_EINVAL, "which must be 0..2");
  if (ncols < 1 || ncols > kNtMax)
    return fail(PARO_EINVAL, "ncols must be 1..%d", kNtMax);
  HIP_OR_FAIL(launch_spmm(h->p, which, d_X, d_Y, ncols, (hipStream_t)stream));
  return PARO_OK;
}

int paro_gram(paro_problem* h, const double* d_W, const double* d_Y,
              double* d_G, int ncols, void* stream) {
  if (!h || !d_W || !d_Y || !d_G) return fail(PARO_EINVAL, "NULL argument");
  if (ncols < 1 || ncols > h->p.Nt)
    return fail(PARO_EINVAL, "ncols must be 1..%d", h->p.Nt);
  HIP_OR_FAIL(
      launch_gram_full(h->p, d_W, d_Y, d_G, ncols, (hipStream_t)stream));
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
    HIP_OR_FAIL(launch_pcg_start_rhs(p, d_B, ncols,
                                     p.opts.precision == PARO_FP32_INNER, s));
    int rc = solve_sources(h, ncols, s, nullptr);
    if (rc) return rc;
    HIP_OR_FAIL(hipMemcpyAsync(d_X, p.X, bytes, hipMemcpyDeviceToDevice, s));
    int st = 0;
    rc = read_back(h, &p.cs->status, &st, 1, s);
    if (rc) return rc;
    if (h_iters) {
      int iters[kNtMax];
      rc = read_back(h, p.cs->iters, iters, ncols, s);
      if (rc) return rc;
      for (int c = 0; c < ncols; ++c) h_iters[c] = iters[c];
    }
    return status_to_code(st);
  } catch (...) {
    return fail(PARO_EDEVICE, "unexpected exception in paro_pcg");
  }
}

}  // extern "C"
