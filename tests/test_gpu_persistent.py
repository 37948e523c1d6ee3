"""Persistent CG (GPU): all CG iterations of a call in one cooperative
launch must give bitwise the results of the kernel-by-kernel path, for one
problem and for an uneven batch, in both precisions."""
import numpy as np
import pytest

from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def _solve_both(run):
    pb.paro_set_persistent(False)
    try:
        ref = run()
        pb.paro_set_persistent(True)
        got = run()
    finally:
        pb.paro_set_persistent(False)
    return ref, got


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_single_problem_matches_kernel_by_kernel(precision):
    w = inputs.molecule(nc=24, N=8, m=4, lo=-8.0, hi=8.0, pot_seed=61,
                        seed=62)
    gu.note(f"persistent CG, one problem, precision {precision}")
    p = gu.workload_problem(w, precision=precision, max_steps=80)

    def run():
        lam, U, rep = gu.solve(p, w.U0())
        return lam, U, rep.steps, rep.pcg_iters, rep.refinements

    ref, got = _solve_both(run)
    assert got[2:] == ref[2:]
    assert np.array_equal(got[0], ref[0])
    assert np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_batch_matches_kernel_by_kernel(precision):
    import torch
    ws = [
        inputs.harmonic(nc=12, N=4, m=6, seed=21, max_steps=120),
        inputs.molecule(nc=10, N=4, m=2, lo=-6.0, hi=6.0, seed=22,
                        pot_seed=23, max_steps=120),
        inputs.harmonic(nc=14, N=1, m=4, seed=24, max_steps=120),
        inputs.molecule(nc=16, N=6, m=5, lo=-8.0, hi=8.0, seed=25,
                        pot_seed=26, max_steps=120),
    ]
    gu.note(f"persistent CG, batch of {len(ws)}, precision {precision}")
    probs = [gu.workload_problem(w, max_steps=w.max_steps, lambda_tol=1e-12,
                                 resid_tol=1e-9, pcg_rtol=1e-10,
                                 precision=precision) for w in ws]
    U0s = [gu.to_dev(w.U0()) for w in ws]

    def run():
        batch = pb.Batch(len(probs))
        lams = [torch.zeros(p.Nt, dtype=torch.float64, device=gu.device())
                for p in probs]
        Us = [torch.zeros(p.n, p.Nt, dtype=torch.float64,
                          device=gu.device()) for p in probs]
        reps = pb.paro_batch_solve(batch, probs, U0s, lams, Us)
        torch.cuda.synchronize()
        return ([x.cpu().numpy() for x in lams], [x.cpu().numpy() for x in Us],
                [(r.status, r.steps, r.pcg_iters) for r in reps])

    ref, got = _solve_both(run)
    assert got[2] == ref[2]
    for a, b in zip(ref[0], got[0]):
        assert np.array_equal(a, b)
    for a, b in zip(ref[1], got[1]):
        assert np.array_equal(a, b)
