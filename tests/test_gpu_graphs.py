"""CG chunks as captured HIP graphs (paro_set_graphs) against kernel-by-
kernel launches (GPU): the same kernels with the same arguments, so every
result must agree bit for bit, including after a change of the launch
shape that keeps the table (a nonlocal term added, its projector count
changed), which must capture new graphs instead of replaying old ones."""
import numpy as np
import pytest

from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def _case():
    return inputs.molecule(nc=12, N=5, m=3, lo=-6.0, hi=6.0, pot_seed=81,
                           seed=82, centres=3, zmax=3, spread=2.0)


def _with_graphs(on, fn):
    pb.paro_set_graphs(on)
    try:
        return fn()
    finally:
        pb.paro_set_graphs(False)


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_graph_solves_equal_kernel_launches(precision):
    w = _case()
    gu.note(f"graphs vs kernels, precision {precision}")

    def run():
        p = gu.workload_problem(w, precision=precision, max_steps=60,
                                lambda_tol=1e-12, resid_tol=1e-8)
        return gu.solve(p, w.U0())

    l0, U0, r0 = _with_graphs(False, run)
    l1, U1, r1 = _with_graphs(True, run)
    assert r0.steps == r1.steps and r0.pcg_iters == r1.pcg_iters
    assert np.array_equal(l0, l1) and np.array_equal(U0, U1)


def test_graphs_follow_a_change_of_nonlocal_projectors():
    import torch
    w = _case()
    _, R = inputs.soft_coulomb_centres(81, 3, 3, 2.0)
    R8 = np.concatenate([R, R + 0.7, R - 0.9])[:8]
    z2 = inputs.gaussian_projectors(w.nc, w.lo, w.hi, R[:2], width=1.2,
                                    height=0.8)
    z8 = inputs.gaussian_projectors(w.nc, w.lo, w.hi, R8, width=1.0,
                                    height=0.5)
    gu.note("graphs across nonlocal projector changes")

    def run():
        p = gu.workload_problem(w, precision=pb.PARO_FP64, pcg_rtol=1e-11)
        lam = torch.zeros(w.Nt, dtype=torch.float64, device=gu.device())
        U = torch.zeros(w.n_dof, w.Nt, dtype=torch.float64,
                        device=gu.device())
        pb.paro_init(p, gu.to_dev(w.U0()), lam, U)
        hist = []
        for zeta in (None, z2, z8, None):
            if zeta is not None:
                pb.paro_set_nonlocal(p, gu.to_dev(zeta))
            else:
                pb.paro_set_nonlocal(p, None)
            for _ in range(3):
                pb.paro_step(p, lam, U)
                hist.append(lam.cpu().numpy().copy())
        return np.array(hist), U.cpu().numpy()

    h0, U0 = _with_graphs(False, run)
    h1, U1 = _with_graphs(True, run)
    assert np.array_equal(h0, h1) and np.array_equal(U0, U1)
    # The projectors did change the iteration.
    assert not np.allclose(h0[2], h0[5])
