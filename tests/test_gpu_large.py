"""Source solves on a mesh large enough that the CG SpMM groups its tiles
into segments: 81^3 = 531,441 rows is more than 2048 tiles of 248 rows, so
the tiles form 8 slabs of 268 (the last one 267) and each of the 1024
p.q partials covers every 128th tile of a slab, two or three tiles (the
path the 96^3 workload takes).  Checked against the oracle's matrix: the FP64 residual of the
result, and for FP64 the iteration count of the oracle's own Jacobi-PCG
on each column (any error in an iterate changes it)."""
import numpy as np
import pytest

from oracle import paro as oparo
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu

NC = 82  # 81^3 interior dofs
NCOLS = 4


@pytest.fixture(scope="module")
def large_case():
    w = inputs.harmonic(nc=NC, N=NCOLS)
    assert w.n_dof > 2048 * 248
    H, M, s = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    A = (H - s * M).tocsr()
    rng = np.random.default_rng(11)
    B = rng.standard_normal((w.n_dof, NCOLS))
    X0 = rng.standard_normal((w.n_dof, NCOLS)) * 0.01
    return w, A, B, X0


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_pcg_with_segmented_spmm_partials(large_case, precision):
    w, A, B, X0 = large_case
    gu.note(f"large pcg: n = {w.n_dof}, ncols = {NCOLS}, "
            f"precision = {precision}")
    prob = gu.workload_problem(w, precision=precision, pcg_rtol=1e-12)
    Xd = gu.to_dev(X0)
    its = pb.paro_pcg(prob, gu.to_dev(B), Xd)
    X = Xd.cpu().numpy()
    res = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.max(res) <= 1.01e-12, res
    if precision == pb.PARO_FP64:
        dinv = 1.0 / A.diagonal()
        for c in range(NCOLS):
            _, k = oparo.jacobi_pcg(A, B[:, c], X0[:, c], dinv, 1e-12, 10000)
            assert abs(its[c] - k) <= 1, (c, its[c], k)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_batch_with_segmented_member_matches_alone(precision):
    """A batch of the 81^3 problem (slab segments) and a 12^3 one (one tile
    per segment): the launch takes the segmented SpMM for both, the small
    problem alone takes the single-tile instantiation.  Two ParO steps,
    bitwise equal to the members stepped alone."""
    import torch
    ws = [inputs.harmonic(nc=NC, N=2, m=2, seed=31, max_steps=50),
          inputs.harmonic(nc=12, N=2, m=2, seed=32, max_steps=50)]
    gu.note(f"large batch: n = {[w.n_dof for w in ws]}, "
            f"precision = {precision}")
    probs = [gu.workload_problem(w, precision=precision, pcg_rtol=1e-10)
             for w in ws]
    U0s = [gu.to_dev(w.U0()) for w in ws]

    def outs():
        return ([torch.zeros(p.Nt, dtype=torch.float64, device=gu.device())
                 for p in probs],
                [torch.zeros(p.n, p.Nt, dtype=torch.float64,
                             device=gu.device()) for p in probs])

    batch = pb.Batch(len(probs))
    lams, Us = outs()
    pb.paro_batch_init(batch, probs, U0s, lams, Us)
    lams1, Us1 = outs()
    for p, U0, l1, U1 in zip(probs, U0s, lams1, Us1):
        pb.paro_init(p, U0, l1, U1)
    for step in range(2):
        reps = pb.paro_batch_step(batch, probs, lams, Us)
        for k, p in enumerate(probs):
            r1 = pb.paro_step(p, lams1[k], Us1[k])
            assert reps[k].status == r1.status == pb.PARO_OK, (step, k)
            assert reps[k].pcg_iters == r1.pcg_iters, (step, k)
        torch.cuda.synchronize()
        for k in range(len(probs)):
            assert torch.equal(lams[k], lams1[k]), (step, k)
            assert torch.equal(Us[k], Us1[k]), (step, k)
