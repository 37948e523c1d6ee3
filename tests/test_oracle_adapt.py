"""Pins of the oracle's adaptive Step 2 (CPU): marking (Doerfler and
maximum strategies, against brute force over all subsets), bisection
(conformity, volume, nestedness, the halved grid after three rounds), the
P1 transfer (the coarse function itself: linear functions exact, mass and
stiffness norms unchanged, agreement with point location and barycentric
interpolation) and the residual estimator (its element term against the
element mass matrix, its jump term zero where the gradient is continuous,
O(h) decay on a smooth eigenfunction, concentration at a Coulomb-like
centre)."""
import itertools

import numpy as np
import pytest

from oracle import adapt, fem, paro as oparo, reference
from paper_1405_0260_amd import inputs


def _face_table(mesh):
    F = adapt._faces(mesh.tets).reshape(-1, 3)
    return np.unique(F, axis=0, return_counts=True)


def _on_box_boundary(mesh, faces):
    P = mesh.X[faces]                                     # (nf, 3, 3)
    lo, hi = mesh.lo, mesh.hi
    onb = np.zeros(faces.shape[0], dtype=bool)
    for a in range(3):
        onb |= np.all(np.isclose(P[:, :, a], lo[a]), axis=1)
        onb |= np.all(np.isclose(P[:, :, a], hi[a]), axis=1)
    return onb


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_doerfler_marks_a_smallest_set_reaching_theta(seed):
    rng = np.random.default_rng(seed)
    eta = rng.random(11) ** 3
    for theta in (0.2, 0.5, 0.9):
        M = adapt.dorfler_mark(eta, theta)
        total = np.sum(eta ** 2)
        assert np.sum(eta[M] ** 2) >= theta * total
        best = min(k for k in range(1, 12)
                   for S in itertools.combinations(range(11), k)
                   if np.sum(eta[list(S)] ** 2) >= theta * total)
        assert len(M) == best


def test_maximum_strategy_marks_by_definition():
    eta = np.array([0.1, 0.9, 0.45, 0.3, 0.9, 0.0])
    assert list(adapt.maximum_mark(eta, 0.5)) == [1, 2, 4]
    assert list(adapt.maximum_mark(eta, 1.0)) == [1, 4]


def test_bisection_keeps_the_mesh_conforming():
    """Random marks over several rounds: every face lies in one element
    (then on the box boundary) or in two, the volume is the box's, no
    element degenerates, and each round's elements tile their parents
    (every old vertex is kept)."""
    rng = np.random.default_rng(0)
    m = adapt.from_kuhn((4, 3, 5), (-1.0, -1.0, -1.5), (1.0, 0.5, 1.5))
    vol0 = 2.0 * 1.5 * 3.0
    ratio0 = None
    for r in range(5):
        marked = rng.choice(m.tets.shape[0], size=max(1, m.tets.shape[0] // 8),
                            replace=False)
        new = adapt.refine(m, marked)
        assert np.array_equal(new.X[:m.X.shape[0]], m.X)
        assert new.tets.shape[0] >= m.tets.shape[0] + len(marked)
        faces, cnt = _face_table(new)
        assert set(np.unique(cnt)) <= {1, 2}
        assert np.all(_on_box_boundary(new, faces[cnt == 1]))
        assert not np.any(_on_box_boundary(new, faces[cnt == 2]))
        vol, _ = fem.element_geometry(new.fem_mesh())
        assert abs(vol.sum() - vol0) < 1e-12 * vol0 and vol.min() > 0
        # Shape regularity: longest edge^3 / volume stays bounded.
        P = new.X[new.tets]
        hT = np.max([np.linalg.norm(P[:, a] - P[:, b], axis=1)
                     for a, b in itertools.combinations(range(4), 2)], axis=0)
        ratio = np.max(hT ** 3 / vol)
        ratio0 = ratio0 or ratio
        assert ratio <= 4.0 * ratio0
        m = new


def test_three_rounds_of_bisection_halve_the_grid():
    m = adapt.from_kuhn(3, -1.0, 1.0)
    for _ in range(3):
        m = adapt.refine(m, range(m.tets.shape[0]))
    fine = fem.kuhn_mesh(6, -1.0, 1.0)
    assert sorted(map(tuple, np.round(m.X, 12))) == \
        sorted(map(tuple, np.round(fine.X, 12)))
    vol, _ = fem.element_geometry(m.fem_mesh())
    assert np.allclose(vol, (2.0 / 6.0) ** 3 / 6.0, rtol=1e-12)


def test_prolongation_is_the_coarse_function():
    rng = np.random.default_rng(4)
    m = adapt.from_kuhn(4, -2.0, 2.0)
    fm = m.fem_mesh()
    U = rng.standard_normal((fm.n_dof, 3))
    new = adapt.refine(m, rng.choice(m.tets.shape[0], 40, replace=False))
    new = adapt.refine(new, rng.choice(new.tets.shape[0], 60, replace=False))
    Uf = adapt.prolong(m, new, U)
    K0, M0, _ = fem.assemble(fm, np.zeros(fm.X.shape[0]))
    nf = new.fem_mesh()
    K1, M1, _ = fem.assemble(nf, np.zeros(nf.X.shape[0]))
    # Same function: same L2 and energy inner products.
    assert np.allclose(U.T @ (M0 @ U), Uf.T @ (M1 @ Uf), rtol=1e-12,
                       atol=1e-14)
    assert np.allclose(U.T @ (K0 @ U), Uf.T @ (K1 @ Uf), rtol=1e-12,
                       atol=1e-14)
    # A linear function (at the interior vertices; the box boundary holds
    # zero) is reproduced at every interior vertex not next to the boundary.
    lin = lambda X: 0.3 + X @ np.array([1.0, -2.0, 0.5])
    Xi = m.X[m.dof >= 0]
    g = adapt.prolong(m, new, lin(Xi))[:, 0]
    Xf = new.X[new.dof >= 0]
    far = np.all(np.abs(Xf) < 2.0 - 1.0 - 1e-9, axis=1)
    assert np.allclose(g[far], lin(Xf[far]), rtol=0, atol=1e-13)


def test_interpolation_by_point_location_matches_prolongation():
    """The P1 value at a point by locating its element and its barycentric
    coordinates equals the bisection transfer at the refined vertices."""
    rng = np.random.default_rng(5)
    m = adapt.from_kuhn(3, -1.0, 1.0)
    U = rng.standard_normal((m.fem_mesh().n_dof, 2))
    new = m
    for _ in range(3):
        new = adapt.refine(new, range(new.tets.shape[0]))
    Uf = adapt.prolong(m, new, U)
    Xf = new.X[new.dof >= 0]
    pts = adapt.interpolate(fem.kuhn_mesh(3, -1.0, 1.0), U, Xf, 3)
    assert np.allclose(pts, Uf, rtol=0, atol=1e-13)


def test_estimator_element_term_equals_the_mass_form():
    """With V = c constant the element residual of u is (lambda - c) u, so
    eta_T^2(lambda) - eta_T^2(c) = h_T^2 (lambda - c)^2 u_T^T M_T u_T with
    the element mass matrix (an independent integration)."""
    rng = np.random.default_rng(6)
    m = adapt.refine(adapt.from_kuhn(3, -1.0, 1.0), [0, 5, 9])
    fm = m.fem_mesh()
    U = rng.standard_normal((fm.n_dof, 1))
    c = 1.7
    V = np.full(m.X.shape[0], c)
    e_c = adapt.estimator(m, V, [c], U)
    e_l = adapt.estimator(m, V, [c - 0.8], U)
    _, Mt, _ = fem.element_matrices(fm, V)
    full = np.zeros(m.X.shape[0])
    full[fm.dof >= 0] = U[fm.dof[fm.dof >= 0], 0]
    ut = full[m.tets]
    P = m.X[m.tets]
    hT = np.max([np.linalg.norm(P[:, a] - P[:, b], axis=1)
                 for a, b in itertools.combinations(range(4), 2)], axis=0)
    want = hT ** 2 * 0.64 * np.einsum("ta,tab,tb->t", ut, Mt, ut)
    assert np.allclose(e_l ** 2 - e_c ** 2, want, rtol=1e-10,
                       atol=1e-14 * want.max())


def test_estimator_jump_term_vanishes_where_the_gradient_is_continuous():
    """u linear at every interior vertex (zero on the boundary) and
    V = lambda: only elements whose faces touch boundary-adjacent elements
    see a gradient jump; the others have eta = 0."""
    m = adapt.refine(adapt.from_kuhn(6, -1.0, 1.0), [3, 77, 400])
    fm = m.fem_mesh()
    Xi = m.X[fm.dof >= 0]
    U = (0.5 + Xi @ np.array([1.0, 2.0, -1.0]))[:, None]
    eta = adapt.estimator(m, np.full(m.X.shape[0], 2.0), [2.0], U)
    bnd = fm.dof < 0
    touches = np.any(bnd[m.tets], axis=1)
    # Elements sharing a face with a boundary-touching element.
    faces = adapt._faces(m.tets)
    near = touches.copy()
    fset = {}
    for t in range(m.tets.shape[0]):
        for a in range(4):
            fset.setdefault(tuple(faces[t, a]), []).append(t)
    for ts in fset.values():
        if len(ts) == 2 and (touches[ts[0]] or touches[ts[1]]):
            near[ts[0]] = near[ts[1]] = True
    assert np.all(eta[~near] < 1e-12) and np.sum(~near) > 100
    # Elements at the boundary see the kink of u down to zero there.
    assert np.mean(eta[touches] > 1e-6) > 0.5


def test_estimator_decays_like_h_on_a_smooth_eigenfunction():
    etas = []
    for nc in (8, 16):
        w = inputs.harmonic(nc=nc, N=1)
        m = adapt.from_kuhn(nc, w.lo, w.hi)
        H, M = fem.hamiltonian(m.fem_mesh(), w.V)
        lam, U = reference.sparse_lowest(H, M, 1, -0.5)
        etas.append(np.linalg.norm(adapt.estimator(m, w.V, lam, U)))
    assert 1.6 < etas[0] / etas[1] < 2.5, etas


def test_adaptive_paro_refines_at_the_centre_and_converges_on_the_final_mesh():
    """A soft-Coulomb centre at the origin: after a few steps on the first
    mesh, Doerfler marking puts the new vertices near the centre (their
    median distance is a fifth of the old vertices'), every refined step
    carries the orbitals over, and with the mesh then held fixed ParO
    converges to the lowest eigenvalue of the final mesh (dense eigh)."""
    Vfun = lambda X: -3.0 / np.sqrt(np.sum(X * X, axis=1) + 0.1)
    m = adapt.from_kuhn(6, -4.0, 4.0)
    U0 = np.random.default_rng(7).standard_normal((m.fem_mesh().n_dof, 4))
    r = adapt.adaptive_paro(m, Vfun, U0, 1, steps=50, theta=0.4,
                            refine_steps=range(8, 12))
    assert r.dofs[8] == r.dofs[0] < r.dofs[9] < r.dofs[12] == r.dofs[-1]
    new = r.mesh.X[m.X.shape[0]:]
    assert np.median(np.linalg.norm(new, axis=1)) < \
        0.25 * np.median(np.linalg.norm(m.X, axis=1))
    H, M = fem.hamiltonian(r.mesh.fem_mesh(), Vfun(r.mesh.X))
    lam, _ = reference.dense_lowest(H, M, 4)
    assert abs(r.lam[0] - lam[0]) < 1e-10 * abs(lam[0])
