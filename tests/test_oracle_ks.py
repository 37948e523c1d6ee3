"""Pins of the oracle's Kohn-Sham pieces (CPU).

* Poisson: a manufactured solution that vanishes on the box boundary is
  recovered at O(h^2) (pins the operator, the 4 pi and the mass matrix).
* Slater exchange: equals the derivative of the homogeneous-electron-gas
  exchange energy density (pins prefactor and exponent independently).
* Density: occupancy 2 and only the N occupied columns.
* The outer loop: with mixing 0 the Hamiltonian never changes after the
  first density, so the iteration is the linear ParO on that Hamiltonian;
  and a converged run is self-consistent (its orbitals are the lowest
  eigenvectors of the Hamiltonian built from their own density).
"""
import numpy as np
import pytest

from oracle import fem, kohn_sham as ks, paro as oparo, reference
from paper_1405_0260_amd import inputs


def _poisson_error(nc, L=2.0):
    mesh = fem.kuhn_mesh(nc, 0.0, L)
    K, M, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    X = mesh.X[mesh.dof >= 0]
    exact = np.prod(np.sin(np.pi * X / L), axis=1)
    rho = 3.0 * np.pi * exact / (4.0 * L * L)
    d = mesh.dof[mesh.dof >= 0]
    vh = ks.hartree(K, M, rho[np.argsort(d)])
    return np.max(np.abs(vh - exact[np.argsort(d)]))


def test_poisson_manufactured_solution_converges_at_order_h2():
    e = [_poisson_error(nc) for nc in (8, 16, 32)]
    assert e[2] < 5e-3          # of max |V*| = 1
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4, (e, r1, r2)


def test_slater_exchange_is_derivative_of_gas_exchange_energy():
    rho = np.array([1e-4, 0.01, 0.3, 1.0, 7.5])
    energy = lambda r: -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * r ** (4.0 / 3.0)
    h = 1e-6 * rho
    deriv = (energy(rho + h) - energy(rho - h)) / (2 * h)
    assert np.allclose(ks.slater_exchange(rho), deriv, rtol=1e-8)
    assert ks.slater_exchange(np.array([0.0, -1e-20]))[0] == 0.0


def test_density_counts_two_electrons_per_occupied_orbital():
    U = np.array([[1.0, 2.0, 5.0], [0.5, -1.0, 7.0]])
    assert np.allclose(ks.density(U, 2), [2 * (1 + 4), 2 * (0.25 + 1)])


def small_molecule(nc=10, N=2, m=4):
    return inputs.molecule(nc=nc, N=N, m=m, lo=-6.0, hi=6.0, pot_seed=41,
                           seed=42, centres=2, zmax=3, spread=1.5)


def test_zero_mixing_is_linear_paro_on_the_first_hamiltonian():
    w = small_molecule()
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    r = ks.scf(mesh, w.V, w.U0(), w.N, iterations=4, mixing=0.0,
               rtol=1e-12)
    # Rebuild the first Hamiltonian from the Step-1 orbitals by hand.
    K, M, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    H0, _ = fem.hamiltonian(mesh, w.V)
    lam, U = oparo.rayleigh_ritz(H0, M, w.U0())
    rho = ks.density(U, w.N)
    V = ks.effective_potential(mesh, w.V, rho, ks.hartree(K, M, rho))
    H, _ = fem.hamiltonian(mesh, V)
    s = oparo.shift_from_potential(V)
    A = (H - s * M).tocsr()
    for k in range(4):
        lam, U, _ = oparo.paro_step(H, M, A, 1.0 / A.diagonal(), lam, U, s,
                                    1e-12, 10 * U.shape[0])
        assert np.allclose(lam, r.lam_history[k + 1], rtol=1e-11, atol=0)


def test_converged_scf_is_self_consistent():
    w = small_molecule()
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    r = ks.scf(mesh, w.V, w.U0(), w.N, iterations=220, rtol=1e-12)
    assert r.residual_history[-1] < 1e-8, r.residual_history[-5:]
    # The last Hamiltonian was built from rho_in; its lowest eigenpairs are
    # the final Ritz pairs.
    H, M = fem.hamiltonian(mesh, r.V_eff)
    lam_ref, _ = reference.dense_lowest(H, M, w.Nt)
    assert np.allclose(r.lam[:w.N], lam_ref[:w.N], rtol=1e-10)
    # and the output density equals the input density.
    rho_out = ks.density(r.U, w.N)
    assert np.linalg.norm(rho_out - r.rho_in) / np.linalg.norm(r.rho_in) \
        < 1e-7


def _box_mesh():
    """A non-cubic box and grid, so a dof <-> vertex numbering slip (x
    fastest, (nx-1)(ny-1) per z layer) moves values to other points."""
    nc, lo, hi = (12, 10, 14), np.zeros(3), np.array([2.0, 1.6, 2.4])
    return fem.kuhn_mesh(nc, lo, hi), lo, hi


def _at_dofs(mesh, f):
    """Values of f(x) at the interior vertices, in dof order, computed from
    the vertex coordinates (not from the dof numbering formula)."""
    inner = np.nonzero(mesh.dof >= 0)[0]
    out = np.empty(inner.size)
    out[mesh.dof[inner]] = f(mesh.X[inner])
    return out


def test_effective_potential_without_density_is_the_external_potential():
    mesh, lo, hi = _box_mesh()
    V = np.random.default_rng(5).standard_normal(mesh.X.shape[0])
    n = mesh.n_dof
    out = ks.effective_potential(mesh, V, np.zeros(n), np.zeros(n))
    assert np.array_equal(out, V)


def test_effective_potential_keeps_boundary_values_and_maps_by_coordinates():
    """Sec. 2 effective potential V_ext + V_H + v_x: on boundary vertices
    rho = V_H = 0 (homogeneous Dirichlet data), so V_ext is kept bit for
    bit; at an interior vertex x the added terms are V_H(x) and
    -(3 rho(x) / pi)^(1/3), with rho and V_H looked up by the vertex."""
    mesh, lo, hi = _box_mesh()
    V = np.random.default_rng(6).standard_normal(mesh.X.shape[0])
    rho = _at_dofs(mesh, lambda X: 1.0 + X[:, 0] + 3.0 * X[:, 1] ** 2
                   + 5.0 * X[:, 2] ** 3)
    vh = _at_dofs(mesh, lambda X: np.sin(X[:, 0]) + 7.0 * X[:, 2])
    out = ks.effective_potential(mesh, V, rho, vh)
    bnd = mesh.dof < 0
    assert np.array_equal(out[bnd], V[bnd])
    X = mesh.X[~bnd]
    r = 1.0 + X[:, 0] + 3.0 * X[:, 1] ** 2 + 5.0 * X[:, 2] ** 3
    expect = V[~bnd] + np.sin(X[:, 0]) + 7.0 * X[:, 2] \
        - (3.0 * r / np.pi) ** (1.0 / 3.0)
    assert np.allclose(out[~bnd], expect, rtol=0, atol=1e-13)


def test_effective_potential_of_a_sine_density_matches_the_closed_form():
    """Manufactured Hartree term: on [0,a]x[0,b]x[0,c] the product
    V*(x) = prod sin(pi x_k / L_k) solves -Lap V* = 4 pi rho for
    rho = pi (1/a^2 + 1/b^2 + 1/c^2) V* / 4 and vanishes on the boundary,
    so V_eff - V_ext = V* - (3 rho / pi)^(1/3) at interior vertices up to
    the O(h^2) error of the P1 Poisson solve (halving h quarters it)."""
    errs = []
    for scale in (1, 2):
        nc = tuple(scale * k for k in (8, 6, 10))
        L = np.array([2.0, 1.6, 2.4])
        mesh = fem.kuhn_mesh(nc, np.zeros(3), L)
        K, M, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
        coef = np.pi * np.sum(1.0 / L ** 2) / 4.0
        vstar = lambda X: np.prod(np.sin(np.pi * X / L), axis=1)
        rho = _at_dofs(mesh, lambda X: coef * vstar(X))
        Vext = np.cos(mesh.X[:, 0]) * mesh.X[:, 1]
        out = ks.effective_potential(mesh, Vext, rho,
                                     ks.hartree(K, M, rho))
        inner = mesh.dof >= 0
        X = mesh.X[inner]
        expect = vstar(X) - np.cbrt(3.0 * coef * vstar(X) / np.pi)
        errs.append(np.max(np.abs(out[inner] - Vext[inner] - expect)))
        assert np.array_equal(out[~inner], Vext[~inner])
    assert errs[1] < 0.025
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_kerker_filter_without_screening_is_the_identity():
    mesh = fem.kuhn_mesh((5, 6, 7), 0.0, (1.0, 1.2, 1.4))
    K, _, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    e = np.random.default_rng(3).standard_normal(mesh.n_dof)
    assert np.array_equal(ks.kerker_filter(K, e, 0.0, 0.01), e)


def test_kerker_filter_scales_a_sine_mode_by_the_closed_form_factor():
    """On a uniform box grid the P1 stiffness is the 7-point operator
    sum_a c_a T_a (c_x = h_y h_z / h_x, cyclically), whose eigenvectors
    are products of discrete sines with eigenvalues
    lambda = sum_a c_a 2 (1 - cos(pi p_a / (m_a + 1))); the filter must
    multiply such a mode by lambda / (lambda + q0^2 h_x h_y h_z)."""
    nc, L = (8, 6, 10), np.array([2.0, 1.5, 3.0])
    mesh = fem.kuhn_mesh(nc, np.zeros(3), L)
    K, _, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    h = L / np.array(nc)
    c = np.array([h[1] * h[2] / h[0], h[2] * h[0] / h[1],
                  h[0] * h[1] / h[2]])
    q0 = 1.3
    for p in ((1, 1, 1), (3, 2, 7), (7, 5, 9)):
        mode = lambda X: np.prod(np.sin(np.pi * np.array(p) * X / L), axis=1)
        e = _at_dofs(mesh, mode)
        lam = sum(c[a] * 2.0 * (1.0 - np.cos(np.pi * p[a] / nc[a]))
                  for a in range(3))
        f = lam / (lam + q0 * q0 * np.prod(h))
        got = ks.kerker_filter(K, e, q0, float(np.prod(h)))
        assert np.allclose(got, f * e, rtol=0, atol=1e-12 * np.abs(e).max())


def test_kerker_mixing_reaches_the_same_fixed_point():
    """The filter only changes the path: a converged Kerker-mixed run is
    self-consistent with the same lowest eigenvalues as linear mixing."""
    w = small_molecule()
    mesh = fem.kuhn_mesh(w.nc, w.lo, w.hi)
    a = ks.scf(mesh, w.V, w.U0(), w.N, iterations=220, rtol=1e-12)
    b = ks.scf(mesh, w.V, w.U0(), w.N, iterations=220, rtol=1e-12,
               kerker_q0=0.8)
    assert b.residual_history[-1] < 1e-8, b.residual_history[-5:]
    assert np.allclose(a.lam[:w.N], b.lam[:w.N], rtol=1e-9)
