#!/usr/bin/env python
"""ParO throughput on one MI355X: orbital-updates/s on the largest
single-GPU workload, the linear eigenproblem of the 96^3 Kohn-Sham
workload's external potential (20 soft-Coulomb centres on [-14,14]^3,
857,375 dofs, N = 32 requested orbitals + 8 buffer orbitals), in FP64.

One benchmark step is one whole solve from inputs resident in HBM:
assembly of the operator, the Rayleigh-Ritz start, and ParO steps until the
requested pairs meet lambda_tol / resid_tol.  Throughput counts
n_dof * N per ParO step (requested orbitals, not the buffer).  The
eigenvalues are checked against the oracle's converged run
(tests/golden/linear_96c_lowest.txt).

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed]

Prints one JSON line (see the keys at the bottom).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
# Stopping of the linear solves: a solve ends when every requested pair
# meets LAMBDA_TOL (relative change of lambda) and RESID_TOL (relative
# residual).  The inner CG of each source problem stops one decade below
# RESID_TOL: a Ritz pair's residual cannot fall much below the relative
# residual its source solve left behind (an inner tolerance equal to
# RESID_TOL stalls the outer test), and a tighter one only adds CG
# iterations (1e-10 takes the 96^3 solve the same 492 ParO steps to the
# same eigenvalues, with 44 % more CG iterations).  Each source solve also
# stops once it has shrunk its warm start's residual (the pair's
# eigen-residual) by PCG_REDUCE: a ParO step reduces that residual by a
# few per cent at this workload's rate, so solving far beyond it is
# wasted; at 1e-2 the outer iteration takes 495 steps instead of 492.
LAMBDA_TOL, RESID_TOL = 1e-11, 1e-7
PCG_RTOL = 1e-8  # RESID_TOL / 10
PCG_REDUCE = 1e-2
GOLDEN = os.path.join(GOLDEN_DIR, "linear_96c_lowest.txt")
GOLDEN64 = os.path.join(GOLDEN_DIR, "softcoulomb_64c_lowest.txt")
GOLDEN_BATCH = os.path.join(GOLDEN_DIR, "batch64_sample_lowest.txt")
GOLDEN_SERVE = os.path.join(GOLDEN_DIR, "serve_sample_lowest.txt")
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC = {"fp64": os.path.join(PROFILES, "linear96_fp64_traffic.md"),
           "mixed": os.path.join(PROFILES, "linear96_mixed_traffic.md")}
SOLVER_SRC = os.path.join(ROOT, "paper_1405_0260_amd", "csrc", "solver.hip")
KERNEL_NAMES = {"cg_spmm": "spmm_cm_kernel", "cg_rupd": "rupd_alpha_kernel",
                "cg_pupd": "pupd_beta_kernel", "rr_spmm": "spmm_dual_kernel",
                "gram": "gram_kernel", "rotate": "rotate_kernel"}


def solver_code_sha():
    """SHA-256 of the kernel source with comments and blank lines removed
    (a comment edit does not invalidate measured counters)."""
    import hashlib
    import re
    src = open(SOLVER_SRC).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*", "", ln).rstrip() for ln in src.splitlines()]
    code = "\n".join(ln for ln in lines if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def measured_traffic(kernel, path, workload=None):
    """HBM bytes per launch of a CG kernel from a committed PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a copy of known size), or
    None when the summary is missing, lacks that kernel, covers another
    workload than `workload` (if given), or was taken on a different
    solver source than the one built now."""
    try:
        text = open(path).read()
        sha = solver_code_sha()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("solver_sha256: ", "workload: ",
                                      "traffic_bytes_per_launch[")))
    if fields.get("solver_sha256") != sha:
        return None
    if workload is not None and fields.get("workload") != workload:
        return None
    value = fields.get(f"traffic_bytes_per_launch[{kernel}]")
    return None if value is None else float(value)


def lambda_error(lam, ref):
    """max_i |l_i - r_i| / max(|r_i|, 1e-3 max|r|) over the given pairs."""
    ref = np.asarray(ref, dtype=np.float64)
    floor = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return float(np.max(np.abs(np.asarray(lam) - ref) / floor))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="arithmetic of the headline solves (the other "
                         "precision is reported beside them)")
    ap.add_argument("--nc", type=int, default=96,
                    help="cells per axis of the headline workload")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--no-other-precision", action="store_true",
                    help="skip the solves in the other precision")
    ap.add_argument("--no-64", action="store_true",
                    help="skip the 64^3 soft-Coulomb context runs")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed solves only (for rocprofv3)")
    ap.add_argument("--inner-rtol", type=float, default=1e-5,
                    help="FP32 inner CG residual reduction per refinement")
    ap.add_argument("--pcg-rtol", type=float, default=PCG_RTOL,
                    help="source solves' floor relative to ||b|| (the linear "
                         "workloads; the Kohn-Sham leg keeps 1e-7)")
    ap.add_argument("--pcg-reduce", type=float, default=PCG_REDUCE,
                    help="source solves also stop at this fraction of their "
                         "start's residual (0: to pcg-rtol only)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="with --profile-only: first copy a 256 MiB buffer "
                         "(a plain copy kernel of known size, the reference "
                         "for the HBM byte counters)")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the estimate / mark / refine-everything run")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the 24^3 harmonic latency run")
    ap.add_argument("--no-local-adaptive", action="store_true",
                    help="skip the local-refinement run on bisection meshes")
    ap.add_argument("--local-nc", type=int, default=24,
                    help="cells per axis of the local run's first mesh")
    ap.add_argument("--local-steps", type=int, default=10,
                    help="ParO iterations with an adaptive Step 2 in the "
                         "local run")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-problem uneven batch")
    ap.add_argument("--no-batch-sequential", action="store_true",
                    help="do not also solve the batch members one by one")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served request stream")
    ap.add_argument("--no-ks", action="store_true",
                    help="skip the 96^3 Kohn-Sham run")
    ap.add_argument("--no-nonlocal", action="store_true",
                    help="skip the run with a nonlocal pseudopotential term")
    ap.add_argument("--ks-nc", type=int, default=96,
                    help="cells per axis of the Kohn-Sham run")
    ap.add_argument("--ks-iters", type=int, default=3000,
                    help="outer iterations at most")
    ap.add_argument("--ks-kerker-q0", type=float, default=1.0,
                    help="Kerker screening wave number of the mixing (0: "
                         "plain linear mixing)")
    ap.add_argument("--ks-poisson-cg", action="store_true",
                    help="Hartree by Jacobi-PCG instead of the direct solve")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests per served run")
    ap.add_argument("--serve-arena-gb", type=float, default=48.0,
                    help="device arena of the server (admission budget)")
    ap.add_argument("--serve-slots", type=int, default=64,
                    help="most requests resident at once")
    ap.add_argument("--cpu-workers", type=int, default=None,
                    help="worker processes of the all-core oracle sample "
                         "(default: the usable cores, at most 16)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(stage, n, nnz, vec_bytes, mat_bytes, diag_bytes):
    """(fixed, per_column) bytes a CG kernel must move in one iteration that
    does work: one pass over each operand it reads or writes.  A launch
    with `a` active columns moves fixed + a * per_column bytes; launches
    queued after convergence return at once and move none."""
    if stage == "cg_spmm":   # read A (values + columns) + row pointers, P; write Q
        return nnz * (mat_bytes + 4) + 4 * (n + 1), 2 * n * vec_bytes
    if stage == "cg_rupd":   # read R, Q, D^-1; write R
        return n * diag_bytes, 3 * n * vec_bytes
    if stage == "cg_pupd":   # read X, P, R, D^-1; write X, P
        return n * diag_bytes, 5 * n * vec_bytes
    raise KeyError(stage)


def rr_stage_rates(td, n, nnz, nt, emitting=True):
    """Rates of the once-per-step Rayleigh-Ritz kernels from a timed solve,
    on the algorithmic bytes of each launch (FP64): the dual SpMM reads
    the matrix pair and W and writes H W and M W, z (8 + 8 + 4) + 4 (n + 1)
    + 3 n N_t 8; the Gram reads W, H W and M W, 3 n N_t 8; the rotation
    reads them and writes U and, in the library's loops, the next step's
    start state x0, r0, p0, 7 n N_t 8 (6 when it stores H U, M U).  A
    stage's time includes its finaliser (gram_final about 9 %, rotate_final
    about 2 % of the stage), and its launch count counts both kernels."""
    per = {"rr_spmm": (nnz * 20 + 4 * (n + 1) + 3 * n * nt * 8, 1),
           "gram": (3 * n * nt * 8, 2),
           "rotate": ((7 if emitting else 6) * n * nt * 8, 2)}
    out = {}
    for st, (b, kpl) in per.items():
        s_ = td["stages"].get(st)
        if not s_ or s_["ms"] <= 0 or s_["launches"] == 0:
            continue
        calls = s_["launches"] // kpl
        out[st] = {"total_ms": s_["ms"], "launches": calls,
                   "us_per_launch": 1e3 * s_["ms"] / calls,
                   "bytes_per_launch": float(b),
                   "gbs": b * calls / (s_["ms"] * 1e-3) / 1e9}
    return out


def z_march(nc):
    """Whether the library's CG SpMM marches along z on an nc^3-cell box:
    more than 2048 row tiles of 248 rows, planes of at most 256 tiles and
    at least 3 planes per range (the plane-range rule of the library)."""
    m = nc - 1
    plane = m * m
    nxy = -(-plane // 248)
    tiles = -(-plane * m // 248)
    if tiles <= 2048 or nxy * 8 > 2048:
        return False
    nzr = 8 * (-(-384 // (8 * nxy)))
    while nzr * nxy > 2048:
        nzr -= 8
    if nzr > m // 3:
        nzr = (m // 3) // 8 * 8
    return nzr >= 8


def cg_stage_rates(td, n, nnz, vec_b, nv=None):
    """Per CG kernel of one event-timed solve (timing dict td): launches,
    time and achieved GB/s on the CSR figure and on the library's own
    format (nv: vertices of the potential the matrix-free SpMM reads, or
    None for the stored stencil); also the algorithmic bytes of the whole
    CG iteration on both."""
    stages = {}
    it_bytes = 0.0
    it_own = 0.0
    for st in ("cg_spmm", "cg_rupd", "cg_pupd"):
        s = td["stages"][st]
        if s["launches"] == 0:
            continue
        fixed, per_col = algorithmic_bytes(st, n, nnz, vec_b, vec_b, vec_b)
        total = fixed * td["cg_iters"] + per_col * td["cg_col_iters"]
        fo, po = own_format_bytes(st, n, vec_b, vec_b, vec_b, nv)
        own = fo * td["cg_iters"] + po * td["cg_col_iters"]
        it_bytes += total
        it_own += own
        stages[st] = {"total_ms": s["ms"], "launches": s["launches"],
                      "us_per_launch": 1e3 * s["ms"] / s["launches"],
                      "bytes_per_launch": total / s["launches"],
                      "own_bytes_per_launch": own / s["launches"],
                      "gbs": total / (s["ms"] * 1e-3) / 1e9,
                      "own_gbs": own / (s["ms"] * 1e-3) / 1e9}
    return stages, it_bytes, it_own


def own_format_bytes(stage, n, vec_bytes, mat_bytes, diag_bytes, nv=None):
    """(fixed, per_column) bytes of the same kernels in the library's own
    format: the SpMM reads 15 stored coefficients per row (no column
    indices or row pointers), or, matrix-free (nv given), the potential at
    the nv vertices and forms the coefficients itself."""
    if stage == "cg_spmm":
        fixed = 8 * nv if nv else 15 * n * mat_bytes
        return fixed, 2 * n * vec_bytes
    return algorithmic_bytes(stage, n, 0, vec_bytes, mat_bytes, diag_bytes)


class Solver:
    """Whole solves of one workload (assembly + paro_solve) in one
    precision, with the caller-owned workspace kept across solves."""

    def __init__(self, w, prec, golden, inner_rtol, key):
        import torch
        from paper_1405_0260_amd import binding as pb
        self.pb, self.torch, self.w, self.prec = pb, torch, w, prec
        self.key = key  # the workload's label (keys its traffic summary)
        dev = torch.device("cuda:0")
        self.golden = golden
        self.box = pb.Box.cube(w.nc, w.lo, w.hi)
        self.V = torch.from_numpy(w.V).to(dev)
        self.U0 = torch.from_numpy(w.U0()).to(dev)
        self.lam = torch.zeros(w.Nt, dtype=torch.float64, device=dev)
        self.U = torch.zeros(w.n_dof, w.Nt, dtype=torch.float64, device=dev)
        self.opts = pb.default_opts(
            N=w.N, m=w.m, max_steps=4000, lambda_tol=LAMBDA_TOL,
            resid_tol=RESID_TOL, pcg_rtol=PCG_RTOL, pcg_reduce=PCG_REDUCE,
            inner_rtol=inner_rtol,
            precision=pb.PARO_FP32_INNER if prec == "mixed" else pb.PARO_FP64)
        _, self.nnz, nbytes = pb.paro_query(self.box, self.opts)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)

    def solve(self, timing=False):
        pb, torch = self.pb, self.torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob = pb.paro_assemble(self.box, self.V, self.opts,
                                workspace=self.ws)
        if timing:
            pb.paro_set_timing(prob, True)
        rep = pb.paro_solve(prob, self.U0, self.lam, self.U)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tim = pb.paro_get_timing(prob) if timing else None
        return t1 - t0, rep, prob, tim

    def run(self, steps, warmup, tag):
        w = self.w
        for k in range(warmup):
            dt, rep, _, _ = self.solve()
            log(f"[{tag}] warmup {k}: {dt:.3f} s, {rep.steps} ParO steps, "
                f"{rep.pcg_iters} CG iterations")
        self.torch.cuda.synchronize()
        times, reps = [], []
        t0 = time.perf_counter()
        for k in range(steps):
            dt, rep, _, _ = self.solve()
            times.append(dt)
            reps.append(rep)
            log(f"[{tag}] step {k}: {dt:.3f} s, {rep.steps} ParO steps, "
                f"{rep.pcg_iters} CG iterations, status {rep.status}")
        self.torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lam_host = self.lam.cpu().numpy()
        err = None
        if self.golden is not None:
            err = lambda_error(lam_host[:w.N], self.golden[:w.N])
        updates = sum(r.steps for r in reps) * w.n_dof * w.N
        last = reps[-1]
        return {
            "value": updates / wall, "wall": wall, "times": times,
            "reps": reps, "lambda_err": err, "ok": all(r.status == 0
                                                       for r in reps),
            "summary": {
                "value": updates / wall, "unit": "orbital-updates/s",
                "ms_per_solve": 1e3 * float(np.mean(times)),
                "paro_steps": last.steps, "cg_iters": last.pcg_iters,
                "refinements": last.refinements,
                "lambda_rel_err_vs_oracle_ref": err,
                "converged": all(r.status == 0 for r in reps)},
        }

    def roofline(self):
        """Roofline of the dominant kernel (the CG kernels and the
        once-per-step Rayleigh-Ritz kernels, whichever takes the most time)
        from one event-timed solve (dispatch-stamped HIP events on the
        launch stream), every such kernel's rate beside it, the whole CG
        iteration, every stage's share of kernel time and the Gram's FP64
        MFMA rate."""
        w, prec = self.w, self.prec
        n, Nt = w.n_dof, w.Nt
        _, rep_t, prob_t, tim = self.solve(timing=True)
        td = tim.as_dict()
        vec_b = 4 if prec == "mixed" else 8
        # The z-marching SpMMs are matrix-free: they read the potential.
        zm = z_march(w.nc)
        nv = (w.nc + 1) ** 3 if zm else None
        stages, it_bytes, it_own = cg_stage_rates(td, n, prob_t.nnz, vec_b,
                                                  nv)
        rr = rr_stage_rates(td, n, prob_t.nnz, Nt)
        both = dict(stages, **rr)
        dom = max(both, key=lambda k: both[k]["total_ms"])
        d = both[dom]
        kname = KERNEL_NAMES[dom]
        if dom == "cg_spmm" and zm:
            kname = "spmm_zmf_kernel"
        traffic = measured_traffic(kname, TRAFFIC[prec], self.key)
        all_ms = sum(v["ms"] for v in td["stages"].values())
        cg_ms = sum(td["stages"][k]["ms"] for k in
                    ("cg_spmm", "cg_rupd", "cg_pupd", "cg_final"))
        g = td["stages"]["gram"]
        # Two launches per Gram (MFMA tiles, then the fixed-order final).
        gram_flop = 4.0 * n * Nt * Nt * g["launches"] / 2
        return {
            "bound": "hbm", "kernel": kname,
            "achieved": round(d["gbs"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(d["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "traffic_over_algorithmic": None if traffic is None else
            round(traffic / d["bytes_per_launch"], 3),
            "bytes_per_launch": int(d["bytes_per_launch"]),
            "us_per_launch": round(d["us_per_launch"], 2),
            "launches": d["launches"],
            "active_cols_avg": round(td["cg_col_iters"] /
                                     max(1, td["cg_iters"]), 2),
            "kernels_frac": {KERNEL_NAMES[k] if k != "cg_spmm" or not zm
                             else "spmm_zmf_kernel":
                             round(v["gbs"] / HBM_PEAK_GBS, 4)
                             for k, v in both.items()},
            "cg_stage_gbs": {k: round(v["gbs"], 1) for k, v in stages.items()},
            "cg_stage_own_format_gbs": {k: round(v["own_gbs"], 1)
                                        for k, v in stages.items()},
            "cg_stage_us_per_launch": {k: round(v["us_per_launch"], 2)
                                       for k, v in stages.items()},
            "cg_iteration_gbs": round(it_bytes / (cg_ms * 1e-3) / 1e9, 1),
            "cg_iteration_frac": round(it_bytes / (cg_ms * 1e-3) / 1e9 /
                                       HBM_PEAK_GBS, 4),
            # The same on the bytes the library's own format must move
            # (matrix-free SpMM: the potential instead of a matrix).
            "cg_iteration_own_format_frac": round(
                it_own / (cg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "gram_mfma_tflops": round(gram_flop / (g["ms"] * 1e-3) / 1e12, 2)
            if g["ms"] > 0 else None,
            "gram_mfma_frac_of_fp64_peak": round(
                gram_flop / (g["ms"] * 1e-3) / 1e12 / 78.6, 4)
            if g["ms"] > 0 else None,
            "stage_ms_share": {k: round(v["ms"] / all_ms, 4)
                               for k, v in td["stages"].items()
                               if v["ms"] > 0},
        }


def main():
    args = parse()
    global PCG_RTOL, PCG_REDUCE
    PCG_RTOL, PCG_REDUCE = args.pcg_rtol, args.pcg_reduce
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} "
              "is not supported (the multi-GPU sharding is a design note, "
              "not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    w = inputs.kohn_sham_96(nc=args.nc)
    golden = np.loadtxt(GOLDEN) if (args.nc == 96 and
                                    os.path.exists(GOLDEN)) else None
    prec = args.precision
    other = "mixed" if prec == "fp64" else "fp64"

    if args.copy_probe:
        src = torch.ones(1 << 25, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    key = f"linear_{w.nc}c_N{w.N}_m{w.m}"
    head = Solver(w, prec, golden, args.inner_rtol, key)
    main_res = head.run(args.steps, args.warmup, prec)
    if args.profile_only:
        log(json.dumps({"value": main_res["value"]}))
        return
    roofline = head.roofline()
    nnz = head.nnz
    del head
    torch.cuda.empty_cache()

    other_res = None
    if not args.no_other_precision:
        s2 = Solver(w, other, golden, args.inner_rtol, key)
        r2 = s2.run(max(1, args.steps - 1), 0, other)
        other_res = dict(r2["summary"], precision=other,
                         roofline=s2.roofline())
        del s2
        torch.cuda.empty_cache()

    ctx64 = None
    if not args.no_64:
        g64 = np.loadtxt(GOLDEN64) if os.path.exists(GOLDEN64) else None
        w64 = inputs.molecule_64()
        ctx64 = {"workload": f"softcoulomb_64c_N{w64.N}_m{w64.m}",
                 "n_dof": w64.n_dof,
                 "note": "working set fits the 256 MB Infinity Cache: "
                         "its CG kernel rates are cache-assisted"}
        for p in ("fp64", "mixed"):
            s3 = Solver(w64, p, g64, args.inner_rtol, ctx64["workload"])
            r3 = s3.run(2, 1, f"64c {p}")
            ctx64[p] = dict(r3["summary"], roofline=s3.roofline())
            del s3
        torch.cuda.empty_cache()

    adaptive = None
    if not args.no_adaptive:
        adaptive = adaptive_bench(args, golden)
        torch.cuda.empty_cache()

    local = None
    if not args.no_local_adaptive:
        local = local_adaptive_bench(args, golden)
        torch.cuda.empty_cache()

    latency = None
    if not args.no_latency:
        latency = latency_bench(args)

    batch = None
    if not args.no_batch:
        batch = batch_bench(args, "mixed")

    serve = None
    if not args.no_serve:
        serve = serve_bench(args, "mixed")

    ks = None
    if not args.no_ks:
        ks = ks_bench(args, "mixed")

    nonlocal_term = None
    if not args.no_nonlocal:
        nonlocal_term = nonlocal_bench(args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_workers)

    times = np.array(main_res["times"])
    last = main_res["reps"][-1]
    out = {
        "metric": "orbital-updates/s (dofs·N per ParO step) + p50/p99 "
                  "latency, at 1e-8 rel λ error",
        "value": main_res["value"],
        "unit": "orbital-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * float(np.mean(times)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-inner/f64" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": key,
                   "potential": "20 soft-Coulomb centres, Z in 1..8, R in "
                                "[-5,5]^3 (seed 3), box [-14,14]^3",
                   "n_dof": w.n_dof, "nnz": nnz,
                   "N": w.N, "m": w.m, "precision": prec,
                   "inner_rtol": args.inner_rtol, "lambda_tol": LAMBDA_TOL,
                   "resid_tol": RESID_TOL, "pcg_rtol": PCG_RTOL,
                   "pcg_reduce": PCG_REDUCE,
                   "parallelism": "single-gpu"},
        "latency_ms": {"p50": 1e3 * float(np.percentile(times, 50)),
                       "p99": 1e3 * float(np.percentile(times, 99))},
        "paro_steps_per_solve": last.steps,
        "cg_iters_per_solve": last.pcg_iters,
        "ms_per_paro_step": 1e3 * float(np.mean(times)) / last.steps,
        "lambda_rel_err_vs_oracle_ref": main_res["lambda_err"],
        "converged": main_res["ok"],
        "other_precision": other_res,
        "softcoulomb_64c": ctx64,
        "adaptive_refine_all": adaptive,
        "adaptive_local": local,
        "harmonic_24c_latency": latency,
        "batch64": batch,
        "serve": serve,
        "kohn_sham": ks,
        "nonlocal": nonlocal_term,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def batch_bench(args, prec):
    """The 64-problem uneven batch (meshes 16^3..48^3 cells, N 2..24, half
    harmonic, half soft-Coulomb): assembly plus whole solves of all members
    through paro_batch_solve, members leaving the batch as they converge.
    Throughput counts n_dof * N per ParO step of every member."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    ws = inputs.batch_64()
    precision = pb.PARO_FP32_INNER if prec == "mixed" else pb.PARO_FP64
    opts = [pb.default_opts(N=x.N, m=x.m, max_steps=x.max_steps,
                            lambda_tol=LAMBDA_TOL, resid_tol=RESID_TOL,
                            pcg_rtol=PCG_RTOL, pcg_reduce=PCG_REDUCE,
                            inner_rtol=args.inner_rtol,
                            precision=precision)
            for x in ws]
    boxes = [pb.Box.cube(x.nc, x.lo, x.hi) for x in ws]
    Vs = [torch.from_numpy(x.V).to(dev) for x in ws]
    U0s = [torch.from_numpy(x.U0()).to(dev) for x in ws]
    lams = [torch.zeros(x.Nt, dtype=torch.float64, device=dev) for x in ws]
    Us = [torch.zeros(x.n_dof, x.Nt, dtype=torch.float64, device=dev)
          for x in ws]
    wss = [torch.empty(pb.paro_query(b, o)[2] + 256, dtype=torch.uint8,
                       device=dev) for b, o in zip(boxes, opts)]
    bt = pb.Batch(len(ws))

    def one():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        probs = [pb.paro_assemble(b, V, o, workspace=m)
                 for b, V, o, m in zip(boxes, Vs, opts, wss)]
        reps = pb.paro_batch_solve(bt, probs, U0s, lams, Us)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, reps

    one()  # warm-up
    dt, reps = one()
    steps = np.array([r.steps for r in reps])
    work = np.array([x.n_dof * x.Nt for x in ws], dtype=np.float64)
    updates = float(sum(r.steps * x.n_dof * x.N for r, x in zip(reps, ws)))
    log(f"[batch64] {dt:.3f} s, steps {steps.min()}..{steps.max()}, "
        f"{sum(r.status == 0 for r in reps)}/{len(ws)} converged")
    out = {"workload": "batch64_uneven", "members": len(ws),
           "value": updates / dt, "unit": "orbital-updates/s",
           "seconds": dt, "converged": int(sum(r.status == 0 for r in reps)),
           "paro_steps_min": int(steps.min()),
           "paro_steps_max": int(steps.max()),
           "work_weighted_occupancy": float((work * steps).sum() /
                                            (work.sum() * steps.max())),
           "n_dof_range": [int(min(x.n_dof for x in ws)),
                           int(max(x.n_dof for x in ws))]}
    errs = member_errors(GOLDEN_BATCH, {j: lams[j] for j in
                                        range(len(ws))}, ws)
    if errs:
        out["lambda_rel_err_vs_oracle_ref"] = errs
    if not args.no_batch_sequential:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        upd = 0.0
        for k in range(len(ws)):
            p = pb.paro_assemble(boxes[k], Vs[k], opts[k], workspace=wss[k])
            r = pb.paro_solve(p, U0s[k], lams[k], Us[k])
            upd += r.steps * ws[k].n_dof * ws[k].N
        torch.cuda.synchronize()
        seq = time.perf_counter() - t0
        out["sequential"] = {"value": upd / seq, "seconds": seq,
                             "batch_speedup": seq / dt}
        log(f"[batch64] one by one: {seq:.3f} s ({seq / dt:.2f}x the "
            f"batch)")
    return out


def read_member_golden(path):
    """{member index: (member name, requested eigenvalues)} from a golden
    file whose data lines read 'j name lam_1 ... lam_N'."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = line.split()
        out[int(v[0])] = (v[1], np.array([float(x) for x in v[2:]]))
    return out


def member_errors(path, lams, ws):
    """Relative lambda error of the sampled members (those with a stored
    oracle reference for the same member recipe, by name) of a batch or
    served stream."""
    ref = read_member_golden(path)
    out = {}
    for j, (name, r) in ref.items():
        if j in lams and j < len(ws) and ws[j].name == name:
            lam = lams[j]
            lam = lam.cpu().numpy() if hasattr(lam, "cpu") else lam
            out[name] = lambda_error(lam[:ws[j].N], r[:ws[j].N])
    return out


def serve_bench(args, prec):
    """The served stream: requests mixing 64^3 soft-Coulomb problems (25%)
    and uneven-batch-style problems, admitted by HBM footprint into the
    continuous-batching loop.  First a closed loop (all requests at t = 0)
    gives the saturation rate; then Poisson arrivals at 0.5x and 0.9x of
    it.  Latency runs from arrival (host arrays ready) to the eigenpairs on
    the host."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    reqs = inputs.serve_requests(args.serve_requests)
    precision = pb.PARO_FP32_INNER if prec == "mixed" else pb.PARO_FP64
    opts = [pb.default_opts(N=x.N, m=x.m, max_steps=x.max_steps,
                            lambda_tol=LAMBDA_TOL, resid_tol=RESID_TOL,
                            pcg_rtol=PCG_RTOL, pcg_reduce=PCG_REDUCE,
                            inner_rtol=args.inner_rtol,
                            precision=precision)
            for x in reqs]
    boxes = [pb.Box.cube(x.nc, x.lo, x.hi) for x in reqs]
    U0s = [x.U0() for x in reqs]
    work = [x.n_dof * x.N for x in reqs]
    arena = int(args.serve_arena_gb * (1 << 30))
    srv = pb.Server(arena, args.serve_slots)

    def run(arrive):
        """arrive: offsets (s) of each request from the start.  Returns
        (makespan, latencies, updates, reports, results)."""
        order = np.argsort(arrive, kind="stable")
        t0 = time.perf_counter()
        nxt, ids, done_at, reps, res = 0, {}, {}, {}, {}
        while len(done_at) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(order) and arrive[order[nxt]] <= now:
                j = int(order[nxt])
                ids[srv.submit(boxes[j], reqs[j].V, opts[j], U0s[j])] = j
                nxt += 1
            if len(ids) == len(done_at):   # nothing in flight
                if nxt < len(order):        # idle until the next arrival
                    time.sleep(max(0.0, arrive[order[nxt]] -
                                   (time.perf_counter() - t0)))
                continue
            done, st = srv.tick()
            t = time.perf_counter() - t0
            for rid in done:
                j = ids[rid]
                lam, U, rep = srv.result(rid)
                done_at[j] = t
                reps[j] = rep
                res[j] = lam
                if len(done_at) % 200 == 0:
                    log(f"[serve] {len(done_at)} of {len(reqs)} requests "
                        f"done at {t:.1f} s")
        makespan = time.perf_counter() - t0
        lat = np.array([done_at[j] - arrive[j] for j in range(len(reqs))])
        upd = float(sum(reps[j].steps * work[j] for j in range(len(reqs))))
        return makespan, lat, upd, reps, res

    torch.cuda.synchronize()
    span, lat, upd, reps, res = run(np.zeros(len(reqs)))
    sat = len(reqs) / span
    log(f"[serve] closed loop: {span:.2f} s for {len(reqs)} requests "
        f"({sat:.2f} req/s), p50 {np.percentile(lat, 50):.2f} s")
    out = {"workload": "served_mix", "requests": len(reqs),
           "big_requests": int(sum(x.n_dof == 250047 for x in reqs)),
           "slots": args.serve_slots, "arena_gb": args.serve_arena_gb,
           "closed_loop": {"req_per_s": sat, "value": upd / span,
                           "unit": "orbital-updates/s", "seconds": span,
                           "p50_s": float(np.percentile(lat, 50)),
                           "p99_s": float(np.percentile(lat, 99))},
           "converged": int(sum(r.status == 0 for r in reps.values()))}
    errs = member_errors(GOLDEN_SERVE, res, reqs)
    if errs:
        out["lambda_rel_err_vs_oracle_ref"] = errs
    for frac in (0.5, 0.9):
        rate = frac * sat
        arrive = inputs.arrivals(len(reqs), rate, seed=5)
        arrive = arrive - arrive[0]
        span, lat, upd, reps2, res2 = run(arrive)
        log(f"[serve] {frac}x saturation ({rate:.2f} req/s): {span:.2f} s, "
            f"p50 {np.percentile(lat, 50):.3f} s, p99 "
            f"{np.percentile(lat, 99):.3f} s")
        out[f"poisson_{frac}x"] = {
            "rate_req_per_s": rate, "value": upd / span,
            "unit": "orbital-updates/s", "seconds": span,
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "same_as_closed_loop": all(np.array_equal(res[j], res2[j])
                                       for j in res)}
    # One request alone against its result in the mix (bitwise).
    j = next(k for k, x in enumerate(reqs) if x.n_dof == 250047)
    dev = torch.device("cuda:0")
    p = pb.paro_assemble(boxes[j], torch.from_numpy(reqs[j].V).to(dev),
                         opts[j])
    lam = torch.zeros(reqs[j].Nt, dtype=torch.float64, device=dev)
    U = torch.zeros(reqs[j].n_dof, reqs[j].Nt, dtype=torch.float64,
                    device=dev)
    pb.paro_solve(p, torch.from_numpy(U0s[j]).to(dev), lam, U)
    out["alone_equals_mix"] = bool(np.array_equal(lam.cpu().numpy(), res[j]))
    srv.close()
    return out


def nonlocal_bench(args):
    """The 64^3 soft-Coulomb workload with a nonlocal pseudopotential term:
    one Gaussian projector per centre (width 1, height 0.5), FP64, solved
    to the same tolerances; reported beside the local solve's time."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    w = inputs.molecule_64()
    _, R = inputs.soft_coulomb_centres(2, 8, 6, 3.0)
    zeta = torch.from_numpy(inputs.gaussian_projectors(
        w.nc, w.lo, w.hi, R, width=1.0, height=0.5)).to(dev)
    box = pb.Box.cube(w.nc, w.lo, w.hi)
    V = torch.from_numpy(w.V).to(dev)
    U0 = torch.from_numpy(w.U0()).to(dev)
    lam = torch.zeros(w.Nt, dtype=torch.float64, device=dev)
    U = torch.zeros(w.n_dof, w.Nt, dtype=torch.float64, device=dev)
    o = pb.default_opts(N=w.N, m=w.m, max_steps=2000, lambda_tol=LAMBDA_TOL,
                        resid_tol=RESID_TOL, pcg_rtol=PCG_RTOL,
                        pcg_reduce=PCG_REDUCE, precision=pb.PARO_FP64)
    out = {}
    for name, nl in (("local", False), ("nonlocal", True)):
        times = []
        for k in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = pb.paro_assemble(box, V, o)
            if nl:
                pb.paro_set_nonlocal(p, zeta)
            rep = pb.paro_solve(p, U0, lam, U)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = min(times)
        out[name] = {"seconds": dt, "paro_steps": rep.steps,
                     "cg_iters": rep.pcg_iters, "status": rep.status,
                     "value": rep.steps * w.n_dof * w.N / dt,
                     "lambda_lowest": lam[:3].cpu().tolist()}
    log(f"[nonlocal] {out['nonlocal']['seconds']:.3f} s "
        f"({out['nonlocal']['paro_steps']} steps) vs local "
        f"{out['local']['seconds']:.3f} s ({out['local']['paro_steps']} steps)")
    out.update({"workload": f"softcoulomb_64c_N{w.N}_m{w.m}_nonlocal8",
                "projectors": int(zeta.shape[1]), "unit": "orbital-updates/s",
                "precision": "fp64"})
    return out


def ks_bench(args, prec):
    """Self-consistent Kohn-Sham around ParO on the 96^3 workload (20
    soft-Coulomb centres, N = 32 occupied orbitals, 8 buffer orbitals):
    one ParO step per outer iteration, Hartree by the direct sine-transform
    solve (--ks-poisson-cg: by Jacobi-PCG), Slater exchange, density mixing
    0.3 with the residual Kerker-filtered (q0 = 1; plain linear mixing at
    0.3 is unstable on this system), run to self-consistency.  Throughput
    counts n_dof * N per outer iteration (one ParO step each)."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    w = inputs.kohn_sham_96(nc=args.ks_nc)
    precision = pb.PARO_FP32_INNER if prec == "mixed" else pb.PARO_FP64
    o = pb.default_opts(N=w.N, m=w.m, max_steps=args.ks_iters,
                        lambda_tol=1e-10, resid_tol=1e-6, pcg_rtol=1e-7,
                        pcg_reduce=PCG_REDUCE,
                        inner_rtol=args.inner_rtol, precision=precision)
    box = pb.Box.cube(w.nc, w.lo, w.hi)
    V = torch.from_numpy(w.V).to(dev)
    U0 = torch.from_numpy(w.U0()).to(dev)
    lam = torch.zeros(w.Nt, dtype=torch.float64, device=dev)
    U = torch.zeros(w.n_dof, w.Nt, dtype=torch.float64, device=dev)
    ko = pb.ks_default_opts(max_iter=args.ks_iters, scf_tol=1e-8,
                            mixing=0.3, kerker_q0=args.ks_kerker_q0,
                            poisson_rtol=1e-10,
                            poisson_maxit=20000 if args.ks_poisson_cg else 0)
    hist = np.zeros(args.ks_iters)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = pb.paro_assemble(box, V, o)
    rep = pb.paro_ks_solve(p, V, U0, lam, U, ko, history=hist)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    updates = float(rep.iterations) * w.n_dof * w.N
    lam_h = lam.cpu().numpy()
    log(f"[kohn-sham] {dt:.2f} s, {rep.iterations} outer iterations, "
        f"residual {rep.residual:.2e}, status {rep.status}")
    return {"workload": f"kohnsham_{w.nc}c_N{w.N}_m{w.m}", "n_dof": w.n_dof,
            "value": updates / dt, "unit": "orbital-updates/s",
            "seconds": dt, "outer_iterations": rep.iterations,
            "mixing": 0.3, "kerker_q0": args.ks_kerker_q0,
            "scf_tol": 1e-8, "converged": rep.status == 0,
            "density_residual": rep.residual,
            "max_dlambda": rep.max_dlambda, "max_resid": rep.max_resid,
            "paro_cg_iters": rep.paro_pcg_iters,
            "hartree": "pcg" if args.ks_poisson_cg else "sine transform",
            "poisson_cg_iters": rep.poisson_iters,
            "lambda_lowest": lam_h[:4].tolist(),
            "homo_lumo_gap": float(lam_h[w.N] - lam_h[w.N - 1]),
            "residual_every_100": [float(x) for x in
                                   hist[1:rep.iterations:100]]}


def adaptive_bench(args, golden):
    """Step 2 with every element refined, measured: the 96^3 workload's
    potential on 48^3 cells, solved (FP64); the residual estimator and
    Doerfler marking (theta 0.5) of its pairs; the orbitals carried to the
    96^3 mesh; the 96^3 solve from them, beside the headline's solve from
    the seeded random start."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    wc, wf = inputs.kohn_sham_96(nc=48), inputs.kohn_sham_96(nc=96)
    out = {"coarse": f"linear_{wc.nc}c_N{wc.N}_m{wc.m}",
           "fine": f"linear_{wf.nc}c_N{wf.N}_m{wf.m}"}

    def solver(w):
        return Solver(w, "fp64", None, args.inner_rtol,
                      f"linear_{w.nc}c_N{w.N}_m{w.m}")

    sc = solver(wc)
    dt_c, rep_c, _, _ = sc.solve()
    out["coarse_seconds"] = dt_c
    out["coarse_paro_steps"] = rep_c.steps
    # Estimate and mark (timed apart, after a warm-up call).
    box = sc.box
    nel = pb.paro_elements(box)
    eta = torch.zeros(nel, dtype=torch.float64, device=dev)
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pb.paro_estimate(box, sc.V, sc.lam, sc.U, wc.N, eta)
        torch.cuda.synchronize()
        t_est = time.perf_counter() - t0
        t0 = time.perf_counter()
        marked, nmark = pb.paro_mark(eta, 0.5, pb.PARO_MARK_DORFLER)
        torch.cuda.synchronize()
        t_mark = time.perf_counter() - t0
    out.update({"elements": nel, "estimate_ms": 1e3 * t_est,
                "estimate_elements_per_s": nel / t_est,
                "mark_ms": 1e3 * t_mark, "marked_theta_0.5": nmark})
    sf = solver(wf)
    Uf = torch.zeros(wf.n_dof, wf.Nt, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.paro_prolong(box, sc.U, Uf)
    torch.cuda.synchronize()
    out["prolong_ms"] = 1e3 * (time.perf_counter() - t0)
    sf.U0 = Uf
    dt_f, rep_f, _, _ = sf.solve()
    lam = sf.lam.cpu().numpy()
    out.update({"fine_seconds_from_transfer": dt_f,
                "fine_paro_steps_from_transfer": rep_f.steps,
                "fine_converged": rep_f.status == 0,
                "lambda_rel_err_vs_oracle_ref":
                    lambda_error(lam[:wf.N], golden[:wf.N])
                    if golden is not None else None})
    log(f"[adaptive] 48^3 solve {dt_c:.2f} s, estimate {1e3 * t_est:.1f} ms, "
        f"mark {1e3 * t_mark:.1f} ms, 96^3 from the transfer {dt_f:.2f} s "
        f"({rep_f.steps} steps)")
    return out


def local_adaptive_bench(args, golden):
    """Algorithm 3.1 with Step 2 adaptive (Sec. 2.1 loop inside every ParO
    iteration), FP64, on bisection meshes: the 96^3 workload's 20-centre
    potential on a 24^3 Kuhn mesh of its box, solved there to the
    headline's tolerances; then iterations of estimate (GPU), Doerfler
    marking at theta 0.5 (GPU), bisection with the conforming closure
    (host), assembly of the CSR operator on the new mesh (host tables, GPU
    values), transfer of the orbitals (GPU) and one ParO step (GPU);
    finally a solve on the last mesh to the same tolerances.  Every stage is timed.  The last
    mesh's eigenvalues are set beside the uniform 96^3 oracle reference (a
    different discretisation: context, not an error)."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    dev = torch.device("cuda:0")
    w = inputs.kohn_sham_96(nc=args.local_nc)
    box = pb.Box.cube(w.nc, w.lo, w.hi)
    opts = pb.default_opts(N=w.N, m=w.m, max_steps=4000, lambda_tol=LAMBDA_TOL,
                           resid_tol=RESID_TOL, pcg_rtol=PCG_RTOL,
                           pcg_reduce=PCG_REDUCE)

    def clock():
        torch.cuda.synchronize()
        return time.perf_counter()

    def assemble(mesh):
        X = mesh.arrays()["X"]
        V = torch.from_numpy(inputs.soft_coulomb_at(X, w.Z, w.R)).to(dev)
        return pb.paro_mesh_assemble(mesh, V, opts)

    t_start = clock()
    mesh = pb.Mesh.kuhn(box)
    p = assemble(mesh)
    lam = torch.zeros(w.Nt, dtype=torch.float64, device=dev)
    U = torch.zeros(p.n, w.Nt, dtype=torch.float64, device=dev)
    rep0 = pb.paro_solve(p, torch.from_numpy(
        inputs.initial_orbitals(p.n, w.Nt, w.orbital_seed)).to(dev), lam, U)
    t_first = clock() - t_start
    dofs0 = p.n
    stages = {k: 0.0 for k in ("estimate", "mark", "refine", "assemble",
                               "transfer", "paro_step")}
    marked_total = 0
    for _ in range(args.local_steps):
        _, ne, _ = mesh.info()
        eta = torch.zeros(ne, dtype=torch.float64, device=dev)
        t0 = clock()
        pb.paro_mesh_estimate(p, lam, U, w.N, eta)
        t1 = clock()
        marked, nmark = pb.paro_mark(eta, 0.5, pb.PARO_MARK_DORFLER)
        t2 = clock()
        new = mesh.refine(marked)
        t3 = clock()
        p2 = assemble(new)
        t4 = clock()
        U2 = torch.zeros(p2.n, w.Nt, dtype=torch.float64, device=dev)
        pb.paro_mesh_prolong(mesh, new, U, U2)
        t5 = clock()
        pb.paro_step(p2, lam, U2)
        t6 = clock()
        for k, dt in zip(stages, (t1 - t0, t2 - t1, t3 - t2, t4 - t3,
                                  t5 - t4, t6 - t5)):
            stages[k] += dt
        marked_total += nmark
        mesh, p, U = new, p2, U2
    t_loop = clock()
    U0 = U.clone()
    rep = pb.paro_solve(p, U0, lam, U)
    t_end = clock()
    nv, ne, _ = mesh.info()
    lam_h = lam.cpu().numpy()
    k = max(1, args.local_steps)
    out = {"start": f"kuhn_{w.nc}c of the linear_96c_N32_m8 potential",
           "theta": 0.5, "adaptive_steps": args.local_steps,
           "first_solve_s": t_first, "first_paro_steps": rep0.steps,
           "dofs_first": dofs0, "dofs_last": p.n, "elements_last": ne,
           "marked_per_step": marked_total / k,
           "stage_ms_per_step": {s_: 1e3 * v / k for s_, v in stages.items()},
           "final_solve_s": t_end - t_loop, "final_paro_steps": rep.steps,
           "final_converged": rep.status == 0,
           "total_s": t_end - t_start,
           "lambda_first": float(lam_h[0]), "lambda_N": float(lam_h[w.N - 1])}
    if golden is not None:
        out["lambda_rel_diff_vs_uniform96_ref"] = lambda_error(
            lam_h[:w.N], golden[:w.N])
    log(f"[local-adaptive] {args.local_steps} adaptive steps: {dofs0} -> "
        f"{p.n} dofs; per step " +
        ", ".join(f"{s_} {1e3 * v / k:.1f} ms" for s_, v in stages.items()) +
        f"; final solve {t_end - t_loop:.2f} s ({rep.steps} steps)")
    return out


def latency_bench(args):
    """The harmonic-oscillator workload (24^3 cells, N = 4, FP64), whose
    working set sits in the caches: microseconds per ParO step over its 30
    steps, and its eigenvalue error after them and at convergence."""
    import torch
    from paper_1405_0260_amd import binding as pb
    from paper_1405_0260_amd import inputs

    w = inputs.harmonic_24()
    conv = np.loadtxt(os.path.join(GOLDEN_DIR, "harmonic_24c_lowest10.txt"))
    s = Solver(w, "fp64", conv, args.inner_rtol, f"harmonic_24c_N{w.N}")
    s.opts.max_steps = 30
    s.opts.lambda_tol = 0.0
    s.opts.resid_tol = 0.0
    times = []
    for k in range(6):
        dt, rep, _, _ = s.solve()
        times.append(dt)
    lam30 = s.lam.cpu().numpy()
    s.opts.max_steps = 1000
    s.opts.lambda_tol = 1e-13
    s.opts.resid_tol = 1e-9
    s.opts.pcg_rtol = 1e-10  # one decade below resid_tol, as everywhere
    dtc, repc, _, _ = s.solve()
    lamc = s.lam.cpu().numpy()
    t = float(np.median(times[1:]))
    return {"workload": "harmonic_24c_N4", "n_dof": w.n_dof,
            "paro_steps": 30, "seconds_per_solve": t,
            "us_per_paro_step": 1e6 * t / 30,
            "note": "whole solve (assembly, start, 30 steps) / 30",
            "lambda_rel_err_after_30_steps": lambda_error(lam30[:4],
                                                          conv[:4]),
            "steps_to_converge": repc.steps,
            "lambda_rel_err_converged": lambda_error(lamc[:4], conv[:4])}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(w, workers=None):
    """The oracle, as it stands, on a bounded sample of the headline
    workload: its first ParO step from the seeded start.
      * all cores: the whole step (N + m source solves and the Rayleigh-
        Ritz projection) with the oracle's worker pool for the independent
        source problems of Step 3 (one process per usable core, at most
        16) and the host BLAS threads for the projection;
      * one thread: the first source solves until ~15 s have passed and the
        projection, scaled to the whole step.
    Throughput = n_dof * N per step time.  The first step starts from
    random orbitals, so its CG solves take far more iterations than the
    average step of a solve (the CG counts are reported)."""
    from threadpoolctl import threadpool_limits

    from oracle import fem, paro as oparo

    workers = workers or min(16, usable_cores())
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    s = oparo.shift_from_potential(w.V)
    maxit = 10 * w.n_dof
    # All cores.  Step 1 (the start's Rayleigh-Ritz) is timed on its own
    # and taken out of the one-step solve.
    t0 = time.perf_counter()
    oparo.rayleigh_ritz(H, M, w.U0())
    t_start = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oparo.paro_solve(H, M, w.U0(), w.N, sigma=s, max_steps=1,
                         rtol=PCG_RTOL, maxit=maxit, workers=workers,
                         reduce=PCG_REDUCE)
    step_all = time.perf_counter() - t0 - t_start
    its_all = r.pcg_iters[0]
    # One thread.
    with threadpool_limits(limits=1):
        A = (H - s * M).tocsr()
        dinv = 1.0 / A.diagonal()
        lam, U = oparo.rayleigh_ritz(H, M, w.U0())
        MU = M @ U
        k = 0
        t0 = time.perf_counter()
        W = U.copy()
        while k < w.Nt and (time.perf_counter() - t0 < 15.0 or k < 1):
            b = (lam[k] - s) * MU[:, k]
            W[:, k], _ = oparo.jacobi_pcg(A, b, U[:, k], dinv, PCG_RTOL,
                                                maxit, reduce=PCG_REDUCE)
            k += 1
        t_solve = (time.perf_counter() - t0) / k
        t1 = time.perf_counter()
        oparo.rayleigh_ritz(H, M, W)
        t_rr = time.perf_counter() - t1
    step_one = t_solve * w.Nt + t_rr
    return {"value": w.n_dof * w.N / step_all, "unit": "orbital-updates/s",
            "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cores": usable_cores(),
            "sample": f"first ParO step of the headline workload from the "
                      f"seeded start: {w.Nt} Jacobi-PCG source solves "
                      f"({int(np.mean(its_all))} CG iterations each on "
                      f"average, {int(np.max(its_all))} at most) over "
                      f"{workers} worker processes, then the Rayleigh-Ritz "
                      f"projection; numpy/scipy",
            "seconds_per_paro_step": step_all,
            "one_thread": {
                "value": w.n_dof * w.N / step_one,
                "unit": "orbital-updates/s", "cores": 1,
                "sample": f"{k} of the same {w.Nt} source solves and the "
                          f"projection, scaled to the whole step",
                "seconds_per_paro_step": step_one}}


if __name__ == "__main__":
    main()
