"""ParO-level parity of the HIP path against the oracle (GPU).

Whole steps and solves through paro_init / paro_step / paro_solve, on the
workloads' seeded inputs, against the oracle's iterates and against the
plain definition of the fixed point (lowest eigenpairs of H u = l M u)."""
import os

import numpy as np
import pytest

from oracle import paro as oparo
from oracle import reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu
from paro_checks import (m_orthonormality_error, rel_lambda_err,
                         subspace_sine)

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torch():
    import torch
    return torch


def run_steps(prob, U0, steps):
    """paro_init then `steps` paro_step calls; returns the lambda history."""
    torch = _torch()
    lam = torch.zeros(prob.Nt, dtype=torch.float64, device=gu.device())
    U = torch.zeros(prob.n, prob.Nt, dtype=torch.float64, device=gu.device())
    pb.paro_init(prob, gu.to_dev(U0), lam, U)
    hist = [lam.cpu().numpy().copy()]
    reps = []
    for _ in range(steps):
        reps.append(pb.paro_step(prob, lam, U))
        hist.append(lam.cpu().numpy().copy())
    return np.array(hist), U.cpu().numpy(), reps


def test_harmonic_24_thirty_steps_match_oracle_iterates():
    """24^3 harmonic oscillator, N = 4, seeded start, 30 plain FP64 ParO
    steps: every step's Ritz values and the final subspace against the
    oracle run (same start, same CG tolerance)."""
    w = inputs.harmonic_24()
    prob = gu.workload_problem(w, pcg_rtol=1e-12)
    hist, U, reps = run_steps(prob, w.U0(), 30)
    ref_hist = np.loadtxt(os.path.join(GOLDEN,
                                       "harmonic_24c_paro30_history.txt"))
    for k in range(31):
        assert rel_lambda_err(hist[k], ref_hist[k]) < 1e-10, k
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    r = oparo.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=30,
                         rtol=1e-12)
    assert m_orthonormality_error(M, U) < 1e-12
    assert subspace_sine(M, U, r.U_all) < 1e-8
    # Distance to the converged pairs after the 30 steps (reported, and
    # bounded by the subspace-iteration rate (2.75/3.69)^60 ~ 2e-8).
    conv = np.loadtxt(os.path.join(GOLDEN, "harmonic_24c_lowest10.txt"))
    err30 = rel_lambda_err(hist[-1], conv[:4])
    gu.note(f"harmonic_24 lambda error after 30 steps: {err30:.3e}")
    assert err30 < 2e-7
    assert all(r.status == 0 for r in reps)


def test_harmonic_24_converges_to_1e8():
    w = inputs.harmonic_24()
    prob = gu.workload_problem(w, max_steps=200, lambda_tol=1e-13,
                               resid_tol=1e-9)
    lam, U, rep = gu.solve(prob, w.U0())
    conv = np.loadtxt(os.path.join(GOLDEN, "harmonic_24c_lowest10.txt"))
    assert rep.status == 0
    assert rel_lambda_err(lam[:4], conv[:4]) < 1e-8
    # The p-shell doublet is exact on this mesh.
    gu.note(f"steps {rep.steps} lambda {lam[:4]}")


def test_inexact_source_solves_match_oracle_iterates():
    """pcg_reduce (Step 3 solved inexactly: each source solve stops once it
    has shrunk its warm start's residual, the pair's eigen-residual, by
    1e-2): the 24^3 harmonic run's 30 FP64 steps against the oracle's with
    the same stopping test, step by step (Ritz values, and the largest CG
    count of each step within one of the oracle's)."""
    w = inputs.harmonic_24()
    eta = 1e-2
    prob = gu.workload_problem(w, pcg_rtol=1e-12, pcg_reduce=eta)
    hist, U, reps = run_steps(prob, w.U0(), 30)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    r = oparo.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=30,
                         rtol=1e-12, reduce=eta)
    L = np.array(r.lam_history)
    errs = [rel_lambda_err(hist[k], L[k]) for k in range(31)]
    its = [max(x) for x in r.pcg_iters]
    gu.note(f"inexact steps vs oracle: lambda rel {max(errs):.2e}; CG per "
            f"step gpu {[x.pcg_iters for x in reps][:6]} oracle {its[:6]}")
    assert max(errs) < 1e-9
    for k, rep in enumerate(reps):
        assert abs(rep.pcg_iters - its[k]) <= 1, (k, rep.pcg_iters, its[k])
    assert m_orthonormality_error(M, U) < 1e-12
    assert subspace_sine(M, U, r.U_all) < 1e-7


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_inexact_source_solves_converge_to_dense_pairs(precision):
    """With pcg_reduce the fixed point is unchanged: a solve of the 12^3
    soft-Coulomb case (N = 6, m = 4) still reaches the lowest eigenpairs
    of the dense pencil, in both precisions (mixed: the FP64 refinement
    stops at the same max(rtol ||b||, pcg_reduce ||r0||))."""
    w = make_case(kind="sc", nc=12, N=6, m=4)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    prob = gu.workload_problem(w, precision=precision, max_steps=3000,
                               lambda_tol=1e-13, resid_tol=1e-9,
                               pcg_rtol=1e-10, pcg_reduce=1e-2)
    lam, U, rep = gu.solve(prob, w.U0())
    assert rep.status == 0, rep.as_dict()
    ref, Uref = reference.dense_lowest(H, M, w.Nt + 1)
    assert rel_lambda_err(lam[:w.N], ref[:w.N]) < 1e-8
    assert subspace_sine(M, U[:, :w.N], Uref[:, :w.N]) < 1e-6
    exact = gu.workload_problem(w, precision=precision, max_steps=3000,
                                lambda_tol=1e-13, resid_tol=1e-9,
                                pcg_rtol=1e-10)
    _, _, rep_e = gu.solve(exact, w.U0())
    gu.note(f"pcg_reduce 1e-2: {rep.steps} steps, {rep.pcg_iters} CG; "
            f"without: {rep_e.steps} steps, {rep_e.pcg_iters} CG")
    assert rep.pcg_iters < rep_e.pcg_iters


CONVERGED_CASES = [
    ("ho_10", dict(kind="ho", nc=10, N=4, m=0)),
    ("sc_12_m4", dict(kind="sc", nc=12, N=6, m=4)),
    ("sc_11_odd", dict(kind="sc", nc=11, N=5, m=2)),
    ("ho_9_single", dict(kind="ho", nc=9, N=1, m=0)),
]


def make_case(kind, nc, N, m, seed=21):
    if kind == "ho":
        return inputs.harmonic(nc=nc, N=N, m=m, seed=seed)
    return inputs.molecule(nc=nc, N=N, m=m, seed=seed, lo=-6.0, hi=6.0)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
@pytest.mark.parametrize("name,case", CONVERGED_CASES,
                         ids=[c[0] for c in CONVERGED_CASES])
def test_converged_pairs_match_dense_eigensolution(name, case, precision):
    w = make_case(**case)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    prob = gu.workload_problem(w, precision=precision, max_steps=500,
                               lambda_tol=1e-13, resid_tol=1e-9)
    lam, U, rep = gu.solve(prob, w.U0())
    assert rep.status == 0, rep.as_dict()
    ref, Uref = reference.dense_lowest(H, M, w.Nt + 1)
    assert rel_lambda_err(lam[:w.N], ref[:w.N]) < 1e-8
    assert m_orthonormality_error(M, U) < 1e-11
    gap = (ref[w.N] - ref[w.N - 1]) / abs(ref[w.N - 1])
    assert gap > 1e-3
    assert subspace_sine(M, U[:, :w.N], Uref[:, :w.N]) < 1e-6
    if precision == pb.PARO_FP32_INNER:
        assert rep.refinements >= rep.steps


def test_noncubic_box_converges_to_dense_eigensolution():
    ncs, lo, hi = (7, 9, 8), (-5.0, -6.0, -5.5), (5.0, 6.0, 5.5)
    X = inputs.vertex_coords(ncs, lo, hi)
    V = 0.5 * np.sum((X * np.array([1.0, 0.7, 1.3])) ** 2, axis=1)
    H, M, s = gu.oracle_matrices(ncs, lo, hi, V)
    prob = gu.assemble(ncs, lo, hi, V, N=3, m=2, max_steps=400,
                       lambda_tol=1e-13, resid_tol=1e-9)
    n = prob.n
    U0 = inputs.initial_orbitals(n, 5, 9)
    lam, U, rep = gu.solve(prob, U0)
    ref, Uref = reference.dense_lowest(H, M, 6)
    assert rep.status == 0
    assert rel_lambda_err(lam[:3], ref[:3]) < 1e-8
    assert subspace_sine(M, U[:, :3], Uref[:, :3]) < 1e-6


def test_step_is_deterministic_and_pure():
    """Same (lambda, U) in, bitwise the same out; a step from a copy of the
    state equals the step from the original (checkpoint / resume)."""
    torch = _torch()
    w = inputs.molecule(nc=12, N=6, m=2, lo=-6.0, hi=6.0)
    prob = gu.workload_problem(w)
    lam = torch.zeros(prob.Nt, dtype=torch.float64, device=gu.device())
    U = torch.zeros(prob.n, prob.Nt, dtype=torch.float64, device=gu.device())
    pb.paro_init(prob, gu.to_dev(w.U0()), lam, U)
    for _ in range(3):
        pb.paro_step(prob, lam, U)
    lam2, U2 = lam.clone(), U.clone()
    pb.paro_step(prob, lam, U)
    pb.paro_step(prob, lam2, U2)
    torch.cuda.synchronize()
    assert torch.equal(lam, lam2) and torch.equal(U, U2)


def test_exact_eigenpairs_are_a_fixed_point():
    w = inputs.molecule(nc=10, N=4, m=1, lo=-6.0, hi=6.0)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    ref, Uref = reference.dense_lowest(H, M, 5)
    torch = _torch()
    prob = gu.workload_problem(w, pcg_rtol=1e-12)
    lam = gu.to_dev(ref)
    U = gu.to_dev(Uref)
    rep = pb.paro_step(prob, lam, U)
    assert rep.pcg_iters <= 2
    assert rel_lambda_err(lam.cpu().numpy(), ref) < 1e-12
    assert subspace_sine(M, U.cpu().numpy()[:, :4], Uref[:, :4]) < 1e-9


def test_ritz_values_are_upper_bounds_every_step():
    w = inputs.molecule(nc=10, N=4, m=2, lo=-6.0, hi=6.0)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    ref, _ = reference.dense_lowest(H, M, 6)
    prob = gu.workload_problem(w)
    hist, _, _ = run_steps(prob, w.U0(), 12)
    for h in hist:
        assert np.all(h - ref >= -1e-11 * np.max(np.abs(ref)))


def test_minimal_mesh_single_dof():
    """2 cells per axis: one interior vertex, N = 1: lambda = H/M."""
    w = inputs.harmonic(nc=2, N=1, m=0, seed=3)
    H, M, s = gu.oracle_matrices(2, w.lo, w.hi, w.V)
    prob = gu.workload_problem(w, max_steps=3)
    lam, U, rep = gu.solve(prob, np.ones((1, 1)))
    assert abs(lam[0] - H[0, 0] / M[0, 0]) < 1e-14 * abs(lam[0])
    assert abs(U[0, 0] - 1.0 / np.sqrt(M[0, 0])) < 1e-14 / np.sqrt(M[0, 0])


def test_max_columns():
    w = inputs.molecule(nc=8, N=60, m=4, lo=-6.0, hi=6.0)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    prob = gu.workload_problem(w, max_steps=3)
    hist, U, _ = run_steps(prob, w.U0(), 3)
    r = oparo.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=3)
    for k in range(4):
        assert rel_lambda_err(hist[k][:60], r.lam_history[k][:60]) < 1e-9
    assert m_orthonormality_error(M, U) < 1e-10


def test_errors_are_reported():
    torch = _torch()
    w = inputs.harmonic(nc=6, N=2, m=0)
    # Non-finite potential.
    V = w.V.copy()
    V[5] = np.nan
    with pytest.raises(pb.ParoError) as e:
        gu.assemble(w.nc, w.lo, w.hi, V, N=2)
    assert e.value.code == pb.PARO_EINVAL
    # Workspace too small.
    ws = torch.empty(1024, dtype=torch.uint8, device=gu.device())
    with pytest.raises(pb.ParoError) as e:
        pb.paro_assemble(gu.box_of(6, -6, 6), gu.to_dev(w.V),
                         pb.default_opts(N=2), workspace=ws)
    assert e.value.code == pb.PARO_ENOMEM
    # Shift above the spectrum: H - sM negative definite, CG breaks down.
    prob = gu.assemble(w.nc, w.lo, w.hi, w.V, N=2, sigma_mode=1, sigma=500.0)
    lam = torch.zeros(2, dtype=torch.float64, device=gu.device())
    U = torch.zeros(prob.n, 2, dtype=torch.float64, device=gu.device())
    pb.paro_init(prob, gu.to_dev(w.U0()), lam, U)
    with pytest.raises(pb.ParoError) as e:
        pb.paro_step(prob, lam, U)
    assert e.value.code == pb.PARO_ENOTSPD
    # Linearly dependent start: W^T M W singular.
    prob = gu.assemble(w.nc, w.lo, w.hi, w.V, N=2)
    U0 = w.U0()
    U0[:, 1] = U0[:, 0]
    with pytest.raises(pb.ParoError) as e:
        pb.paro_solve(prob, gu.to_dev(U0), lam, U)
    assert e.value.code == pb.PARO_ESINGULAR
    # Step cap before the tolerances: ENOCONV with a filled report.
    prob = gu.assemble(w.nc, w.lo, w.hi, w.V, N=2, max_steps=1,
                       lambda_tol=1e-15, resid_tol=1e-15)
    rep = pb.paro_solve(prob, gu.to_dev(w.U0()), lam, U)
    assert rep.status == pb.PARO_ENOCONV and rep.steps == 1
    assert rep.pcg_iters > 0 and np.isfinite(rep.max_resid)
    # CG cap.
    prob = gu.assemble(w.nc, w.lo, w.hi, w.V, N=2, pcg_maxit=2,
                       pcg_rtol=1e-14)
    pb.paro_init(prob, gu.to_dev(w.U0()), lam, U)
    rep = pb.paro_step(prob, lam, U)
    assert rep.status == pb.PARO_ENOCONV


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_solve_loop_matches_public_steps(precision):
    """paro_solve's steps take M u and H u from the previous rotation
    instead of applying the operators; public paro_step calls apply them.
    Both must give the same iterates up to rounding, step for step."""
    w = inputs.molecule(nc=14, N=6, m=2, lo=-6.0, hi=6.0)
    steps = 12
    # lambda_tol = 0: paro_solve runs exactly max_steps steps.
    prob_a = gu.workload_problem(w, precision=precision, max_steps=steps,
                                 lambda_tol=0.0, pcg_rtol=1e-11)
    lam_a, U_a, rep_a = gu.solve(prob_a, w.U0())
    assert rep_a.steps == steps
    prob_b = gu.workload_problem(w, precision=precision, pcg_rtol=1e-11)
    hist, U_b, reps = run_steps(prob_b, w.U0(), steps)
    lam_b = hist[-1]
    # The two starts differ by rounding; the source solves (to 1e-11)
    # carry that into W at the solve tolerance, which bounds the change.
    scale = np.max(np.abs(lam_b))
    assert np.max(np.abs(lam_a - lam_b)) <= 1e-9 * scale
    assert np.max(np.abs(U_a - U_b)) <= 1e-6 * np.max(np.abs(U_b))


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_step_reports_match_oracle_stopping_measures(precision):
    """The per-step stopping measures (Algorithm A.1 stopping reading) that
    paro_solve, the batch solve and the server act on: for the 24^3
    harmonic run, every step's reported max_i dlambda_i and max_i rho_i
    (i <= N) against the oracle's, computed from its lambda and residual
    histories of the same 30 steps from the same start."""
    w = inputs.harmonic_24()
    prob = gu.workload_problem(w, pcg_rtol=1e-12, precision=precision)
    hist, _, reps = run_steps(prob, w.U0(), 30)
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    r = oparo.paro_solve(H, M, w.U0(), w.N, V_nodal=w.V, max_steps=30,
                         rtol=1e-12)
    L = np.array(r.lam_history)
    dl = np.max(np.abs(L[1:, :w.N] - L[:-1, :w.N])
                / np.stack([oparo.scale_floor(x) for x in L[1:]])[:, :w.N],
                axis=1)
    rho = np.array([x[:w.N].max() for x in r.resid_history[1:]])
    g_dl = np.array([x.max_dlambda for x in reps])
    g_rho = np.array([x.max_resid for x in reps])
    e_dl = np.max(np.abs(g_dl - dl) / dl)
    e_rho = np.max(np.abs(g_rho - rho) / rho)
    gu.note(f"step reports vs oracle: dlambda rel {e_dl:.2e} "
            f"(last {g_dl[-1]:.3e}), rho rel {e_rho:.2e} "
            f"(last {g_rho[-1]:.3e})")
    assert e_dl < 1e-6 and e_rho < 1e-6


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_softcoulomb_64_matches_golden_and_spans_the_eigenspace(precision):
    """The 64^3 soft-Coulomb workload (N = 16, m = 8) solved to tight
    tolerances: lambda against the stored shift-invert eigenvalues, and the
    subspace angle to the exact 16-dimensional eigenspace bounded with the
    oracle's matrices: sin theta <= ||R||_{M^-1} / (lambda_17 - lambda_16)
    (Davis-Kahan), R = H U - M U Lambda over the requested pairs."""
    w = inputs.molecule_64()
    prob = gu.workload_problem(w, precision=precision, max_steps=3000,
                               lambda_tol=1e-13, resid_tol=1e-9,
                               pcg_rtol=1e-12)
    lam, U, rep = gu.solve(prob, w.U0())
    assert rep.status == 0, rep.as_dict()
    golden = np.loadtxt(os.path.join(GOLDEN, "softcoulomb_64c_lowest.txt"))
    N = w.N
    assert rel_lambda_err(lam[:N], golden[:N]) < 1e-10
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    assert m_orthonormality_error(M, U) < 1e-11
    R = H @ U[:, :N] - (M @ U[:, :N]) * lam[None, :N]
    dinv = 1.0 / M.diagonal()
    norm2 = 0.0
    for c in range(N):
        y, _ = oparo.jacobi_pcg(M, R[:, c], np.zeros(R.shape[0]), dinv,
                                1e-12, 2000)
        norm2 += float(R[:, c] @ y)
    sin_bound = np.sqrt(norm2) / (golden[N] - lam[N - 1])
    gu.note(f"64^3 subspace: sin theta <= {sin_bound:.2e}, gap "
            f"{golden[N] - golden[N - 1]:.3e}")
    assert sin_bound < 1e-6


def test_linear_96_fp64_matches_the_oracle_run():
    """The headline workload: the 96^3 linear problem of the 20-centre
    potential, solved in FP64, against the oracle's converged ParO run."""
    w = inputs.kohn_sham_96()
    prob = gu.workload_problem(w, precision=pb.PARO_FP64, max_steps=4000,
                               lambda_tol=1e-11, resid_tol=1e-7)
    lam, _, rep = gu.solve(prob, w.U0())
    assert rep.status == 0, rep.as_dict()
    golden = np.loadtxt(os.path.join(GOLDEN, "linear_96c_lowest.txt"))
    err = rel_lambda_err(lam[:w.N], golden[:w.N])
    gu.note(f"96^3 lambda error vs oracle {err:.2e} after {rep.steps} steps")
    assert err < 1e-10
