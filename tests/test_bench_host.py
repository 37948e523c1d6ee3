"""Host logic of bench.py (no GPU): the algorithmic byte model of the CG
and Rayleigh-Ritz kernels, the rates derived from a timing record, the guard that ties a
committed traffic summary to the solver source it was measured on, and the
one-GPU contract of the command line."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_kernel():
    n, nnz = 1000, 14000
    # SpMM: the CSR pass (values + column indices + row pointers), then
    # read P and write Q per active column.
    assert bench.algorithmic_bytes("cg_spmm", n, nnz, 4, 4, 4) == (
        nnz * 8 + 4 * (n + 1), 2 * n * 4)
    assert bench.algorithmic_bytes("cg_spmm", n, nnz, 8, 8, 8) == (
        nnz * 12 + 4 * (n + 1), 2 * n * 8)
    # r-update: D^-1 once; R, Q read and R written per column.
    assert bench.algorithmic_bytes("cg_rupd", n, nnz, 4, 4, 4) == (
        n * 4, 3 * n * 4)
    # p-update: D^-1 once; X, P, R read and X, P written per column.
    assert bench.algorithmic_bytes("cg_pupd", n, nnz, 8, 8, 8) == (
        n * 8, 5 * n * 8)
    # The stencil format: 15 coefficients per row, no indices.
    assert bench.own_format_bytes("cg_spmm", n, 4, 4, 4) == (
        15 * n * 4, 2 * n * 4)
    # Matrix-free: the potential at the nv vertices instead.
    assert bench.own_format_bytes("cg_spmm", n, 8, 8, 8, nv=3000) == (
        3000 * 8, 2 * n * 8)
    with pytest.raises(KeyError):
        bench.algorithmic_bytes("gram", n, nnz, 8, 8, 8)


def test_stage_rates_from_a_timing_record():
    n, nnz = 2000, 28000
    td = {"cg_iters": 10, "cg_col_iters": 30,
          "stages": {"cg_spmm": {"ms": 0.5, "launches": 10},
                     "cg_rupd": {"ms": 0.25, "launches": 10},
                     "cg_pupd": {"ms": 0.0, "launches": 0}}}
    stages, it_bytes, it_own = bench.cg_stage_rates(td, n, nnz, 4)
    assert set(stages) == {"cg_spmm", "cg_rupd"}
    spmm = (nnz * 8 + 4 * (n + 1)) * 10 + 2 * n * 4 * 30
    rupd = n * 4 * 10 + 3 * n * 4 * 30
    assert it_bytes == spmm + rupd
    assert it_own == 15 * n * 4 * 10 + 2 * n * 4 * 30 + rupd
    _, _, it_mf = bench.cg_stage_rates(td, n, nnz, 4, nv=3000)
    assert it_mf == 3000 * 8 * 10 + 2 * n * 4 * 30 + rupd
    assert stages["cg_spmm"]["bytes_per_launch"] == spmm / 10
    assert abs(stages["cg_spmm"]["gbs"] - spmm / 0.5e-3 / 1e9) < 1e-9
    assert abs(stages["cg_rupd"]["us_per_launch"] - 25.0) < 1e-12


def test_rayleigh_ritz_rates_from_a_timing_record():
    """The once-per-step kernels' algorithmic bytes per launch: the dual
    SpMM reads the matrix pair (CSR figure) and W and writes H W, M W; the
    Gram reads W, H W, M W; the emitting rotation reads them and writes U
    and the next start's x0, r0, p0.  Gram and rotation stages count two
    kernels per launch (their finalisers)."""
    n, nnz, nt = 3000, 42000, 40
    td = {"stages": {"rr_spmm": {"ms": 2.0, "launches": 5},
                     "gram": {"ms": 1.0, "launches": 10},
                     "rotate": {"ms": 3.0, "launches": 10},
                     "small_eig": {"ms": 1.0, "launches": 5}}}
    rr = bench.rr_stage_rates(td, n, nnz, nt)
    assert set(rr) == {"rr_spmm", "gram", "rotate"}
    assert rr["rr_spmm"]["bytes_per_launch"] == (
        nnz * 20 + 4 * (n + 1) + 3 * n * nt * 8)
    assert rr["gram"]["bytes_per_launch"] == 3 * n * nt * 8
    assert rr["rotate"]["bytes_per_launch"] == 7 * n * nt * 8
    assert rr["gram"]["launches"] == 5 and rr["rotate"]["launches"] == 5
    assert abs(rr["rotate"]["us_per_launch"] - 600.0) < 1e-9
    assert abs(rr["rr_spmm"]["gbs"] - rr["rr_spmm"]["bytes_per_launch"] * 5
               / 2.0e-3 / 1e9) < 1e-9
    assert bench.rr_stage_rates(td, n, nnz, nt, emitting=False)[
        "rotate"]["bytes_per_launch"] == 6 * n * nt * 8


def test_z_march_rule_matches_the_library_meshes():
    # 95^3 and 81^3 rows march along z (more than 2048 tiles of 248 rows);
    # 63^3 and smaller sweep the rows.
    assert bench.z_march(96) and bench.z_march(82)
    assert not bench.z_march(64) and not bench.z_march(24)


def _summary(sha, lines):
    return "\n".join([f"solver_sha256: {sha}", ""] + lines) + "\n"


def test_traffic_summary_is_tied_to_the_source(tmp_path, monkeypatch):
    src = tmp_path / "solver.hip"
    src.write_text("int a;  // one\n\n/* block\ncomment */ int b;\n")
    monkeypatch.setattr(bench, "SOLVER_SRC", str(src))
    sha = bench.solver_code_sha()
    # Comments and blank lines do not change the fingerprint ...
    src.write_text("int a;  // two\n/* other */ int b;\n")
    assert bench.solver_code_sha() == sha
    # ... code does.
    src.write_text("int a; int b;\n")
    assert bench.solver_code_sha() != sha
    src.write_text("int a;  // one\n\n/* block\ncomment */ int b;\n")

    traffic = tmp_path / "traffic.md"
    traffic.write_text(_summary(sha, [
        "traffic_bytes_per_launch[spmm_cm_kernel]: 1234",
        "traffic_bytes_per_launch[pupd_beta_kernel]: 5678"]))
    path = str(traffic)
    assert bench.measured_traffic("spmm_cm_kernel", path) == 1234.0
    assert bench.measured_traffic("pupd_beta_kernel", path) == 5678.0
    assert bench.measured_traffic("rupd_alpha_kernel", path) is None
    # A summary names the workload it was measured on; another workload's
    # roofline gets no traffic from it.
    traffic.write_text(_summary(sha, [
        "workload: linear_96c_N32_m8",
        "traffic_bytes_per_launch[pupd_beta_kernel]: 5678"]))
    assert bench.measured_traffic("pupd_beta_kernel", path,
                                  "linear_96c_N32_m8") == 5678.0
    assert bench.measured_traffic("pupd_beta_kernel", path,
                                  "softcoulomb_64c_N16_m8") is None
    traffic.write_text(_summary("0" * 64, [
        "traffic_bytes_per_launch[spmm_cm_kernel]: 1234"]))
    assert bench.measured_traffic("spmm_cm_kernel", path) is None
    os.remove(traffic)
    assert bench.measured_traffic("spmm_cm_kernel", path) is None


def test_lambda_error_uses_the_floor():
    ref = [-2.0, 0.0, 1.0]
    assert bench.lambda_error([-2.0, 1e-6, 1.0], ref) == 1e-6 / 2e-3
    assert bench.lambda_error(ref, ref) == 0.0


def test_member_golden_format(tmp_path):
    g = tmp_path / "members.txt"
    g.write_text("# header\n3 a -1.5 -1.25\n7 b 2.5\n")
    ref = bench.read_member_golden(str(g))
    assert set(ref) == {3, 7} and ref[3][0] == "a"
    assert np.array_equal(ref[3][1], [-1.5, -1.25])

    class W:
        def __init__(self, name, N):
            self.name, self.N = name, N
    ws = [W("x", 1)] * 3 + [W("a", 2)] + [W("x", 1)] * 3 + [W("b", 1)]
    lams = {3: np.array([-1.5, -1.25, 9.0]), 7: np.array([2.5 * (1 + 1e-9)])}
    errs = bench.member_errors(str(g), lams, ws)
    assert errs["a"] == 0.0 and abs(errs["b"] - 1e-9) < 1e-15
    # A list whose member 7 is another recipe is not compared there.
    ws[7] = W("c", 1)
    assert set(bench.member_errors(str(g), lams, ws)) == {"a"}


def test_source_solve_tolerances_default_and_flags(monkeypatch):
    """The linear workloads' inner tolerances: pcg_rtol one decade below
    resid_tol and pcg_reduce 1e-2 by default; the flags override both."""
    assert bench.PCG_RTOL == pytest.approx(bench.RESID_TOL / 10)
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.pcg_rtol, a.pcg_reduce) == (bench.PCG_RTOL, bench.PCG_REDUCE)
    assert bench.PCG_REDUCE == 1e-2
    monkeypatch.setattr(sys, "argv", ["bench.py", "--pcg-reduce", "0",
                                      "--pcg-rtol", "1e-10"])
    a = bench.parse()
    assert (a.pcg_rtol, a.pcg_reduce) == (1e-10, 0.0)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
