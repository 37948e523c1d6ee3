"""Pins of the oracle's nonlocal pseudopotential term (CPU):

* zero projectors leave the Rayleigh-Ritz step unchanged bit for bit;
* a projector equal to an M-normalised eigenvector u_1 of H moves exactly
  that eigenvalue by (u_1, u_1)^2 = 1 and leaves the others (Z^T u_k = 0);
* ParO on H + Z Z^T converges to the dense eigenpairs of that pencil."""
import numpy as np

from oracle import fem, nonlocal_ as onl, paro as oparo, reference
from paper_1405_0260_amd import inputs


def small(nc=9):
    w = inputs.molecule(nc=nc, N=3, m=3, lo=-6.0, hi=6.0, pot_seed=71,
                        seed=72, centres=3, zmax=3, spread=2.0)
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    H, M = fem.hamiltonian(mesh, w.V)
    return w, H, M


def test_zero_projectors_change_nothing():
    w, H, M = small()
    W = w.U0()
    Z = onl.projector_matrix(M, np.zeros((w.n_dof, 3)))
    t1, U1 = oparo.rayleigh_ritz(H, M, W)
    t2, U2 = oparo.rayleigh_ritz(onl.LowRankPlus(H, Z), M, W)
    assert np.array_equal(t1, t2) and np.array_equal(U1, U2)


def test_eigenvector_projector_shifts_one_eigenvalue_by_one():
    w, H, M = small()
    lam, U = reference.dense_lowest(H, M, 6)
    Z = onl.projector_matrix(M, U[:, :1])          # zeta = u_1 (M-normalised)
    Hn = onl.LowRankPlus(H, Z).dense()
    import scipy.linalg as sla
    mu = sla.eigh(Hn, M.toarray(), eigvals_only=True)[:6]
    expect = np.sort(np.concatenate([[lam[0] + 1.0], lam[1:6]]))[:6]
    assert np.allclose(mu, expect, rtol=1e-10, atol=1e-12)


def test_paro_with_nonlocal_term_converges_to_dense_pairs():
    w, H, M = small()
    zeta = inputs.gaussian_projectors(w.nc, w.lo, w.hi,
                                      inputs.soft_coulomb_centres(71, 3, 3, 2.0)[1],
                                      width=1.2, height=0.8)
    Z = onl.projector_matrix(M, zeta)
    Hn = onl.LowRankPlus(H, Z)
    s = oparo.shift_from_potential(w.V)
    An = onl.LowRankPlus((H - s * M).tocsr(), Z)
    dinv = 1.0 / An.diagonal()
    import scipy.linalg as sla
    mu = sla.eigh(Hn.dense(), M.toarray(), eigvals_only=True)[:w.Nt]
    lam, U = oparo.rayleigh_ritz(Hn, M, w.U0())
    for _ in range(250):
        lam, U, _ = oparo.paro_step(Hn, M, An, dinv, lam, U, s, 1e-12, 5000)
    assert np.max(np.abs(lam[:w.N] - mu[:w.N]) / np.abs(mu[:w.N])) < 1e-9
    # the term matters: the local problem's eigenvalues differ
    lam0, _ = reference.dense_lowest(H, M, w.N)
    assert np.max(np.abs(lam0 - mu[:w.N])) > 1e-3
