"""Recovery of a nearly dependent Rayleigh-Ritz basis (GPU).

When the Cholesky factorisation of W^T M W fails, the library
re-orthonormalises W once by a shifted Cholesky-QR pass and projects
again; columns dependent to rounding level (a duplicate, a zero column)
still give PARO_ESINGULAR.  Checked against the plain definition: the
lowest eigenpairs of H u = l M u (dense eigh of the oracle's matrices),
Ritz values as upper bounds, M-orthonormality, and bitwise agreement of
the batch members that needed no retry with their runs alone."""
import numpy as np
import pytest

from oracle import reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu
from paro_checks import m_orthonormality_error, rel_lambda_err, subspace_sine

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _nearly_dependent(U0, delta, seed=1):
    """Column 1 := column 0 + a random vector of relative size delta."""
    U = U0.copy()
    r = np.random.default_rng(seed).standard_normal(U.shape[0])
    U[:, 1] = U[:, 0] + delta * np.linalg.norm(U[:, 0]) / np.linalg.norm(r) * r
    return U


def _outputs(prob):
    torch = _torch()
    lam = torch.zeros(prob.Nt, dtype=torch.float64, device=gu.device())
    U = torch.zeros(prob.n, prob.Nt, dtype=torch.float64, device=gu.device())
    return lam, U


def _harmonic(nc=8):
    return inputs.harmonic(nc=nc, N=3, m=2, seed=5, max_steps=400)


def test_asynchronous_init_leaves_the_failed_projection():
    """paro_init (no report, no retry) on a nearly dependent start: the
    factorisation fails and the orbitals come back unrotated (C = I),
    which is the state the retry starts from."""
    w = _harmonic()
    U0 = _nearly_dependent(w.U0(), 1e-9)
    prob = gu.workload_problem(w)
    lam, U = _outputs(prob)
    gu.note("init on a nearly dependent start")
    pb.paro_init(prob, gu.to_dev(U0), lam, U)
    assert np.array_equal(U.cpu().numpy(), U0)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
@pytest.mark.parametrize("nc", [8, 14])
def test_nearly_dependent_start_is_repaired(nc, precision):
    w = _harmonic(nc)
    U0 = _nearly_dependent(w.U0(), 1e-9)
    prob = gu.workload_problem(w, precision=precision, max_steps=400,
                               lambda_tol=1e-13, resid_tol=1e-9)
    gu.note(f"solve from a nearly dependent start, nc {nc}, "
            f"precision {precision}")
    lam, U, rep = gu.solve(prob, U0)
    assert rep.status == pb.PARO_OK, rep.as_dict()
    assert rep.reorth == 1
    H, M, _ = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    ref, Uref = reference.dense_lowest(H, M, w.Nt + 1)
    assert rel_lambda_err(lam[:w.N], ref[:w.N]) < 1e-9
    assert m_orthonormality_error(M, U) < 1e-11
    assert subspace_sine(M, U[:, :1], Uref[:, :1]) < 1e-6


def test_a_good_start_is_not_retried():
    w = _harmonic()
    prob = gu.workload_problem(w, max_steps=400, lambda_tol=1e-13,
                               resid_tol=1e-9)
    lam, U, rep = gu.solve(prob, w.U0())
    assert rep.status == pb.PARO_OK and rep.reorth == 0


@pytest.mark.parametrize("nc", [6, 14])
@pytest.mark.parametrize("kind", ["duplicate", "zero"])
def test_dependent_start_stays_singular(nc, kind):
    w = _harmonic(nc)
    U0 = w.U0()
    U0[:, 1] = U0[:, 0] if kind == "duplicate" else 0.0
    prob = gu.workload_problem(w)
    lam, U = _outputs(prob)
    gu.note(f"dependent start ({kind}), nc {nc}")
    with pytest.raises(pb.ParoError) as e:
        pb.paro_solve(prob, gu.to_dev(U0), lam, U)
    assert e.value.code == pb.PARO_ESINGULAR


def test_step_on_nearly_dependent_orbitals_is_repaired():
    """A public step from orbitals whose columns 0 and 1 nearly coincide
    (equal lambda): the source solutions are nearly dependent, the step's
    projection is redone on the re-orthonormalised basis, and its Ritz
    values are upper bounds of the eigenvalues (Poincare), with u_0, an
    eigenvector, kept exactly."""
    torch = _torch()
    w = _harmonic()
    H, M, _ = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    ref, _ = reference.dense_lowest(H, M, w.Nt)
    prob = gu.workload_problem(w, max_steps=400, lambda_tol=1e-13,
                               resid_tol=1e-10)
    lam_c, U_c, rep = gu.solve(prob, w.U0())
    assert rep.status == pb.PARO_OK
    U1 = _nearly_dependent(U_c, 1e-9, seed=2)
    lam1 = lam_c.copy()
    lam1[1] = lam1[0]
    lam, U = gu.to_dev(lam1), gu.to_dev(U1)
    gu.note("step from nearly dependent orbitals")
    r = pb.paro_step(prob, lam, U)
    assert r.status == pb.PARO_OK, r.as_dict()
    assert r.reorth == 1
    lam_n, U_n = lam.cpu().numpy(), U.cpu().numpy()
    assert np.all(np.isfinite(lam_n)) and np.all(np.diff(lam_n) >= 0)
    assert np.all(lam_n - ref >= -1e-11 * np.max(np.abs(ref)))
    assert abs(lam_n[0] - ref[0]) < 1e-9 * abs(ref[0])
    assert m_orthonormality_error(M, U_n) < 1e-6
    torch.cuda.synchronize()


def test_batch_retries_only_the_dependent_member():
    """A batch with one nearly dependent start: that member is repaired;
    the others are bitwise what they are alone (the retry runs on a table
    of the failing members only, with their own block counts)."""
    torch = _torch()
    ws = [_harmonic(8),
          inputs.molecule(nc=10, N=4, m=2, lo=-6.0, hi=6.0, seed=22,
                          pot_seed=23, max_steps=300),
          inputs.harmonic(nc=12, N=2, m=3, seed=24, max_steps=300)]
    starts = [w.U0() for w in ws]
    starts[1] = _nearly_dependent(starts[1], 1e-9, seed=3)
    probs = [gu.workload_problem(w, max_steps=w.max_steps, lambda_tol=1e-12,
                                 resid_tol=1e-9) for w in ws]
    batch = pb.Batch(len(probs))
    lams = [torch.zeros(p.Nt, dtype=torch.float64, device=gu.device())
            for p in probs]
    Us = [torch.zeros(p.n, p.Nt, dtype=torch.float64, device=gu.device())
          for p in probs]
    gu.note("batch with one nearly dependent member")
    reps = pb.paro_batch_solve(batch, probs, [gu.to_dev(u) for u in starts],
                               lams, Us)
    torch.cuda.synchronize()
    for k, (w, p, r) in enumerate(zip(ws, probs, reps)):
        assert r.status == pb.PARO_OK, (k, r.as_dict())
        assert r.reorth == (1 if k == 1 else 0), k
        lam_b, U_b = lams[k].cpu().numpy(), Us[k].cpu().numpy()
        lam_a, U_a, rep_a = gu.solve(p, starts[k])
        assert rep_a.reorth == r.reorth
        assert np.array_equal(lam_a, lam_b) and np.array_equal(U_a, U_b), k
        H, M, _ = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
        ref, _ = reference.dense_lowest(H, M, w.Nt)
        assert rel_lambda_err(lam_b[:w.N], ref[:w.N]) < 1e-8, k
        assert m_orthonormality_error(M, U_b) < 1e-11, k


def test_server_repairs_or_rejects_dependent_starts():
    """Served requests: a nearly dependent start is repaired, a duplicated
    column is retired with PARO_ESINGULAR, and a good request alongside
    is bitwise its paro_solve result."""
    ws = [_harmonic(8), _harmonic(8),
          inputs.molecule(nc=10, N=4, m=2, lo=-6.0, hi=6.0, seed=22,
                          pot_seed=23, max_steps=300)]
    starts = [_nearly_dependent(ws[0].U0(), 1e-9), ws[1].U0(), ws[2].U0()]
    starts[1][:, 2] = starts[1][:, 0]

    def opts(w):
        return pb.default_opts(N=w.N, m=w.m, max_steps=w.max_steps,
                               lambda_tol=1e-12, resid_tol=1e-9)

    srv = pb.Server(1 << 28, 8)
    ids = {srv.submit(gu.box_of(w.nc, w.lo, w.hi), w.V, opts(w), u): k
           for k, (w, u) in enumerate(zip(ws, starts))}
    gu.note("serving dependent and good starts")
    res = {}
    for _ in range(2000):
        done, st = srv.tick()
        for rid in done:
            res[ids[rid]] = srv.result(rid)
        if len(res) == len(ws):
            break
    srv.close()
    assert len(res) == len(ws)
    assert res[0][2].status == pb.PARO_OK and res[0][2].reorth == 1
    assert res[1][2].status == pb.PARO_ESINGULAR
    assert res[2][2].status == pb.PARO_OK and res[2][2].reorth == 0
    w = ws[2]
    p = pb.paro_assemble(gu.box_of(w.nc, w.lo, w.hi), gu.to_dev(w.V), opts(w))
    lam_a, U_a, _ = gu.solve(p, starts[2])
    assert np.array_equal(res[2][0], lam_a) and np.array_equal(res[2][1], U_a)
