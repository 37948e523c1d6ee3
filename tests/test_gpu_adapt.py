"""Step 2 on the GPU (uniform Kuhn mesh) against the oracle (GPU).

Inputs come from the oracle or the seeded generators, never from the HIP
path: the estimator is compared on the oracle's own eigenpairs; marking on
seeded indicator values and on the oracle's indicators; the transfer with
the oracle's point-location interpolation.  The refine-everything flow
(coarse solve, transfer, fine solve) is checked against the fine mesh's
eigenvalues."""
import numpy as np
import pytest

from oracle import adapt, fem, paro as oparo, reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu

pytestmark = pytest.mark.gpu


def _molecule(nc):
    return inputs.molecule(nc=nc, N=4, m=3, lo=-6.0, hi=6.0, pot_seed=91,
                           seed=92, centres=3, zmax=4, spread=2.0)


@pytest.mark.parametrize("ncs", [(8, 8, 8), (7, 9, 6)])
def test_estimator_matches_oracle(ncs):
    import torch
    lo, hi = (-6.0, -5.0, -7.0), (6.0, 5.5, 6.0)
    X = inputs.vertex_coords(ncs, lo, hi)
    V = -2.0 / np.sqrt(np.sum(X * X, axis=1) + 0.3) + 0.05 * X[:, 0]
    m = adapt.from_kuhn(ncs, lo, hi)
    H, M = fem.hamiltonian(m.fem_mesh(), V)
    lam, U = reference.dense_lowest(H, M, 5)
    N = 3
    ref = adapt.estimator(m, V, lam[:N], U[:, :N])
    box = gu.box_of(ncs, lo, hi)
    eta = torch.zeros(pb.paro_elements(box), dtype=torch.float64,
                      device=gu.device())
    gu.note(f"estimator {ncs}")
    pb.paro_estimate(box, gu.to_dev(V), gu.to_dev(lam), gu.to_dev(U), N, eta)
    got = eta.cpu().numpy()
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13 * ref.max())


@pytest.mark.parametrize("theta", [0.3, 0.6, 0.95])
def test_doerfler_marking_matches_oracle(theta):
    rng = np.random.default_rng(17)
    eta = rng.random(100003) ** 4
    M = adapt.dorfler_mark(eta, theta)
    got, cnt = pb.paro_mark(gu.to_dev(eta), theta, pb.PARO_MARK_DORFLER)
    got = np.nonzero(got.cpu().numpy())[0]
    gu.note(f"doerfler theta {theta}: {cnt} of {eta.size}")
    assert cnt == len(got) == len(M)
    assert np.array_equal(got, M)


def test_doerfler_marking_with_ties_is_a_smallest_valid_set():
    """Many equal indicators (a symmetric field): the smallest size is
    unique, the set need not be; the GPU's set has that size, reaches theta
    and consists of the largest values (ties by lowest index)."""
    eta = np.repeat([0.5, 0.25, 0.125, 0.0625], [7, 40, 300, 2000])
    np.random.default_rng(3).shuffle(eta)
    theta = 0.5
    M = adapt.dorfler_mark(eta, theta)
    got, cnt = pb.paro_mark(gu.to_dev(eta), theta, pb.PARO_MARK_DORFLER)
    got = got.cpu().numpy().astype(bool)
    assert got.sum() == cnt == len(M)
    assert np.sum(eta[got] ** 2) >= theta * np.sum(eta ** 2)
    assert eta[got].min() >= eta[~got].max()
    t = eta[got].min()
    ties = np.nonzero(eta == t)[0]
    assert np.array_equal(got[ties], np.arange(ties.size) <
                          got[ties].sum())


def test_maximum_marking_matches_oracle():
    rng = np.random.default_rng(19)
    eta = rng.random(50001)
    eta[[5, 77]] = eta.max()
    for theta in (0.5, 0.9, 1.0):
        got, cnt = pb.paro_mark(gu.to_dev(eta), theta, pb.PARO_MARK_MAXIMUM)
        got = np.nonzero(got.cpu().numpy())[0]
        assert np.array_equal(got, adapt.maximum_mark(eta, theta))
        assert cnt == got.size


def test_marking_of_oracle_indicators():
    w = _molecule(8)
    m = adapt.from_kuhn(8, w.lo, w.hi)
    H, M = fem.hamiltonian(m.fem_mesh(), w.V)
    lam, U = reference.dense_lowest(H, M, w.N)
    eta = adapt.estimator(m, w.V, lam, U)
    for theta in (0.4, 0.7):
        got, _ = pb.paro_mark(gu.to_dev(eta), theta, pb.PARO_MARK_DORFLER)
        got = np.nonzero(got.cpu().numpy())[0]
        ref = adapt.dorfler_mark(eta, theta)
        assert got.size == ref.size
        e = eta[got]
        assert np.sum(e ** 2) >= theta * np.sum(eta ** 2)
        outside = np.setdiff1d(np.arange(eta.size), got)
        assert e.min() >= eta[outside].max()


@pytest.mark.parametrize("ncs", [(5, 5, 5), (4, 6, 3)])
def test_prolongation_matches_point_location(ncs):
    import torch
    lo, hi = (-1.0, -2.0, -0.5), (1.5, 2.0, 1.0)
    coarse = fem.kuhn_mesh(ncs, lo, hi)
    fine = fem.kuhn_mesh(tuple(2 * c for c in ncs), lo, hi)
    U = np.random.default_rng(23).standard_normal((coarse.n_dof, 5))
    ref = adapt.interpolate(coarse, U, fine.X[fine.dof >= 0], ncs)
    Uf = torch.zeros(fine.n_dof, 5, dtype=torch.float64, device=gu.device())
    pb.paro_prolong(gu.box_of(ncs, lo, hi), gu.to_dev(U), Uf)
    got = Uf.cpu().numpy()
    assert np.allclose(got, ref, rtol=0, atol=1e-14 * np.abs(U).max())


@pytest.mark.parametrize("precision", [pb.PARO_FP64, pb.PARO_FP32_INNER])
def test_refine_everything_and_continue(precision):
    """Solve on 10^3 cells, carry the orbitals to 20^3, solve there: the
    fine solve ends at the fine mesh's eigenvalues (sparse shift-invert)
    in fewer steps than from the seeded random start."""
    import torch
    wc, wf = _molecule(10), _molecule(20)
    pc = gu.workload_problem(wc, precision=precision, max_steps=500,
                             lambda_tol=1e-12, resid_tol=1e-9)
    lc, Uc, rc = gu.solve(pc, wc.U0())
    assert rc.status == 0
    Uf = torch.zeros(wf.n_dof, wf.Nt, dtype=torch.float64, device=gu.device())
    pb.paro_prolong(gu.box_of(wc.nc, wc.lo, wc.hi), gu.to_dev(Uc), Uf)
    pf = gu.workload_problem(wf, precision=precision, max_steps=500,
                             lambda_tol=1e-12, resid_tol=1e-9)
    lt, _, rt = gu.solve(pf, Uf.cpu().numpy())
    lr, _, rr = gu.solve(pf, wf.U0())
    gu.note(f"refine-and-continue: {rt.steps} steps from the transfer, "
            f"{rr.steps} from the random start")
    H, M, s = gu.oracle_matrices(wf.nc, wf.lo, wf.hi, wf.V)
    ref, _ = reference.sparse_lowest(H, M, wf.Nt + 2, s - 0.5)
    assert rt.status == 0
    assert np.max(np.abs(lt[:wf.N] - ref[:wf.N]) / np.abs(ref[:wf.N])) < 1e-9
    assert rt.steps < rr.steps
