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
