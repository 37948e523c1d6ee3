"""A ParO step from the exact discrete eigenpairs (dense oracle solve) with
a loose source-solve tolerance: the start residual of every source problem
is already below pcg_rtol ||b||, so no column enters CG and no refinement
pass runs (the mixed path's first pass ends on the CG loop's own poll).
The step is then the Rayleigh-Ritz projection of U itself, the same
arithmetic in both precisions: the two results agree bitwise and keep the
oracle's eigenvalues."""
import numpy as np
import pytest

from oracle import reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_step_from_exact_eigenpairs_skips_the_source_solves():
    import torch
    w = inputs.harmonic(nc=12, N=2, m=2, seed=41)
    H, M, _ = gu.oracle_matrices(w.nc, w.lo, w.hi, w.V)
    lam_ref, U_ref = reference.dense_lowest(H, M, w.Nt)
    res = np.linalg.norm(H @ U_ref - (M @ U_ref) * lam_ref, axis=0)
    assert np.max(res / np.linalg.norm((M @ U_ref) * lam_ref, axis=0)) < 1e-9
    out = {}
    for precision in (pb.PARO_FP64, pb.PARO_FP32_INNER):
        gu.note(f"converged step, precision {precision}")
        prob = gu.workload_problem(w, precision=precision, pcg_rtol=1e-3)
        lam = gu.to_dev(lam_ref.copy())
        U = gu.to_dev(U_ref.copy())
        rep = pb.paro_step(prob, lam, U)
        torch.cuda.synchronize()
        assert rep.status == pb.PARO_OK, rep.as_dict()
        assert rep.pcg_iters == 0, rep.as_dict()
        assert rep.refinements == 0, rep.as_dict()
        out[precision] = (lam.cpu().numpy(), U.cpu().numpy())
    lam64, U64 = out[pb.PARO_FP64]
    lam32, U32 = out[pb.PARO_FP32_INNER]
    assert np.array_equal(lam64, lam32)
    assert np.array_equal(U64, U32)
    assert np.max(np.abs(lam64 - lam_ref) / np.abs(lam_ref)) < 1e-12
