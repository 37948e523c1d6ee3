"""Cluster-wise projection (GPU): the eigenvalue-separation variant of
Sec. 3 against the oracle's clustered ParO steps from the same start, and
a single cluster equal to the full projection bitwise."""
import numpy as np
import pytest

from oracle import fem, paro as oparo, reference
from paper_1405_0260_amd import binding as pb
from paper_1405_0260_amd import inputs
import gpu_util as gu
from paro_checks import subspace_sine

pytestmark = pytest.mark.gpu

SIZES = [1, 3, 6]


def start_block(nc=14):
    """Eigenvectors of the harmonic problem mixed inside each cluster and
    perturbed along higher eigenvectors (a good start per cluster)."""
    w = inputs.harmonic(nc=nc, N=4, m=6, seed=31)
    mesh = fem.kuhn_mesh(nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    lam, U = reference.dense_lowest(H, M, 16)
    rng = np.random.default_rng(7)
    W = U[:, :10].copy()
    s = 0
    for q in SIZES:
        Q, _ = np.linalg.qr(rng.standard_normal((q, q)))
        W[:, s:s + q] = W[:, s:s + q] @ Q
        s += q
    W += 0.05 * U[:, 10:16] @ rng.standard_normal((6, 10))
    return w, H, M, lam, W


def gpu_steps(w, W, steps, sizes):
    import torch
    p = gu.workload_problem(w, pcg_rtol=1e-12, precision=pb.PARO_FP64)
    lam = torch.zeros(10, dtype=torch.float64, device=gu.device())
    U = torch.zeros(w.n_dof, 10, dtype=torch.float64, device=gu.device())
    if sizes is not None:              # Step 1 projects per cluster too
        pb.paro_set_clusters(p, sizes)
    pb.paro_init(p, gu.to_dev(W), lam, U)
    hist = []
    for _ in range(steps):
        pb.paro_step(p, lam, U)
        torch.cuda.synchronize()
        hist.append(lam.cpu().numpy())
    return hist, U.cpu().numpy(), p


def test_clustered_steps_match_oracle():
    w, H, M, lam_ref, W = start_block()
    gu.note("clustered ParO steps vs oracle")
    hist, U, _ = gpu_steps(w, W, 8, SIZES)
    A = H.tocsr()
    dinv = 1.0 / A.diagonal()
    l, Uo = oparo.rayleigh_ritz_clustered(H, M, W, SIZES)   # Step 1
    for k in range(8):
        l, Uo, _ = oparo.paro_step(H, M, A, dinv, l, Uo, 0.0, 1e-12, 5000,
                                   clusters=SIZES)
        assert np.max(np.abs(hist[k] - l) / np.abs(l)) < 1e-10, k
    s = 0
    for q in SIZES:                                 # each cluster's span
        assert subspace_sine(M, U[:, s:s + q], Uo[:, s:s + q]) < 1e-7
        s += q
    # the first clusters approach the eigenpairs (rate set by the gaps)
    assert np.max(np.abs(hist[-1][:4] - lam_ref[:4]) / lam_ref[:4]) < 1e-5


def test_one_cluster_is_the_full_projection():
    w, H, M, lam_ref, W = start_block(nc=10)
    gu.note("one cluster vs full projection")
    h1, U1, _ = gpu_steps(w, W, 3, None)
    h2, U2, p = gpu_steps(w, W, 3, [10])
    for a, b in zip(h1, h2):
        assert np.array_equal(a, b)
    assert np.array_equal(U1, U2)
    with pytest.raises(pb.ParoError):
        pb.paro_set_clusters(p, [4, 4])            # does not sum to N + m
    with pytest.raises(pb.ParoError):
        pb.paro_set_clusters(p, [0, 10])
    pb.paro_set_clusters(p, [])                    # full projection again
