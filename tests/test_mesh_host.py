"""General bisection meshes, host side of the library (CPU): the uniform
Kuhn mesh against the oracle's, the library's bisection against the
oracle's (the same elements for the same marks, whatever order each side
cuts them in), conformity, volume, the halved grid after three rounds, and
the sizes of a mesh problem against a brute-force count of the pattern."""
import ctypes
import itertools

import numpy as np
import pytest

from oracle import adapt, fem
from paper_1405_0260_amd import binding as pb


def _box(nc, lo, hi):
    ncs = (nc,) * 3 if np.isscalar(nc) else tuple(nc)
    lo = (lo,) * 3 if np.isscalar(lo) else tuple(lo)
    hi = (hi,) * 3 if np.isscalar(hi) else tuple(hi)
    return pb.Box(ncs[0], ncs[1], ncs[2], (ctypes.c_double * 3)(*lo),
                  (ctypes.c_double * 3)(*hi))


def _volumes(X, tets):
    P = X[tets]
    E = P[:, 1:] - P[:, :1]
    return np.abs(np.linalg.det(E)) / 6.0


def _faces_ok(X, tets, lo, hi):
    F = np.sort(np.stack([np.delete(tets, a, axis=1) for a in range(4)],
                         axis=1).reshape(-1, 3), axis=1)
    faces, cnt = np.unique(F, axis=0, return_counts=True)
    if not set(np.unique(cnt)) <= {1, 2}:
        return False
    P = X[faces[cnt == 1]]
    onb = np.zeros(P.shape[0], dtype=bool)
    for a in range(3):
        onb |= np.all(np.isclose(P[:, :, a], lo[a]), axis=1)
        onb |= np.all(np.isclose(P[:, :, a], hi[a]), axis=1)
    return bool(np.all(onb))


@pytest.mark.parametrize("ncs", [(3, 3, 3), (2, 4, 3)])
def test_kuhn_mesh_is_the_oracles(ncs):
    lo, hi = (-1.0, -2.0, 0.5), (1.5, 2.0, 2.0)
    m = pb.Mesh.kuhn(_box(ncs, lo, hi))
    a = m.arrays()
    o = fem.kuhn_mesh(ncs, lo, hi)
    assert np.array_equal(a["X"], o.X)
    assert np.array_equal(a["tets"], o.tets)
    assert np.array_equal(a["dof"], o.dof)
    assert np.all(a["tags"] == 3) and np.all(a["parents"] == -1)
    assert m.info() == (o.X.shape[0], o.tets.shape[0], int((o.dof >= 0).sum()))


def _ordered_elements(X, tets, tags):
    """Elements as (ordered corner coordinates, tag): the bisection state
    of every element, independent of the order elements are listed in."""
    return {(tuple(tuple(X[v]) for v in t), int(k))
            for t, k in zip(tets, tags)}


def _ball_marks(X, tets, centre, radius):
    """Elements whose centroid lies in the ball: marks that do not depend
    on how either side numbers its elements."""
    c = X[tets].mean(axis=1)
    return (np.linalg.norm(c - centre, axis=1) < radius).astype(np.uint8)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bisection_matches_the_oracle(seed):
    """Marks in a random ball over four rounds, each side refining its own
    mesh: the same vertices (bitwise coordinates, each with the same
    parents) and the same elements, each with the same corner order and
    tag.  The two sides may list elements in different orders (the closure
    visits the elements around an edge in an order of its own)."""
    rng = np.random.default_rng(seed)
    ncs, lo, hi = (3, 2, 4), (-1.0, -1.0, -1.5), (1.0, 0.5, 1.5)
    lib_m = pb.Mesh.kuhn(_box(ncs, lo, hi))
    ora_m = adapt.from_kuhn(ncs, lo, hi)
    for _ in range(4):
        centre = rng.uniform(lo, hi)
        radius = rng.uniform(0.3, 0.8)
        a = lib_m.arrays()
        ora_m = adapt.refine(ora_m, np.nonzero(
            _ball_marks(ora_m.X, ora_m.tets, centre, radius))[0])
        lib_m = lib_m.refine(_ball_marks(a["X"], a["tets"], centre, radius))
        a = lib_m.arrays()
        assert a["X"].shape == ora_m.X.shape
        assert sorted(map(tuple, a["X"])) == sorted(map(tuple, ora_m.X))
        lib_par = {tuple(a["X"][v]): tuple(sorted(map(tuple, a["X"][p])))
                   for v, p in enumerate(a["parents"]) if p[0] >= 0}
        ora_par = {tuple(ora_m.X[v]):
                   tuple(sorted(map(tuple, ora_m.X[p])))
                   for v, p in enumerate(ora_m.parents) if p[0] >= 0}
        assert lib_par == ora_par
        assert _ordered_elements(a["X"], a["tets"], a["tags"]) == \
            _ordered_elements(ora_m.X, ora_m.tets, ora_m.tags)


def test_refined_mesh_is_conforming_and_fills_the_box():
    rng = np.random.default_rng(5)
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 2.0, 0.5])
    m = pb.Mesh.kuhn(_box((4, 5, 3), lo, hi))
    vol0 = np.prod(hi - lo)
    for _ in range(5):
        _, ne, _ = m.info()
        marked = rng.random(ne) < 0.1
        m = m.refine(marked)
        a = m.arrays()
        vol = _volumes(a["X"], a["tets"])
        assert vol.min() > 0 and abs(vol.sum() - vol0) < 1e-12 * vol0
        assert _faces_ok(a["X"], a["tets"], lo, hi)
        # Every new vertex is the midpoint of its parents.
        new = np.nonzero(a["parents"][:, 0] >= 0)[0]
        p = a["parents"][new]
        assert np.array_equal(a["X"][new], 0.5 * (a["X"][p[:, 0]] +
                                                   a["X"][p[:, 1]]))
        assert np.all(p < new[:, None])


def test_three_rounds_of_refining_everything_halve_the_grid():
    m = pb.Mesh.kuhn(_box(2, -1.0, 1.0))
    for _ in range(3):
        _, ne, _ = m.info()
        m = m.refine(np.ones(ne, dtype=np.uint8))
    a = m.arrays()
    fine = fem.kuhn_mesh(4, -1.0, 1.0)
    assert sorted(map(tuple, a["X"])) == sorted(map(tuple, fine.X))
    assert np.allclose(_volumes(a["X"], a["tets"]), (2.0 / 4) ** 3 / 6.0,
                       rtol=1e-12)


def test_mesh_from_arrays_round_trip_and_checks():
    o = adapt.refine(adapt.from_kuhn(2, -1.0, 1.0), [0, 3, 7])
    box = _box(2, -1.0, 1.0)
    m = pb.Mesh.from_arrays(box, o.X, o.tets, o.tags, o.parents)
    a = m.arrays()
    assert np.array_equal(a["X"], o.X) and np.array_equal(a["tets"], o.tets)
    assert np.array_equal(a["dof"], o.dof)
    bad = o.tets.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(pb.ParoError) as e:
        pb.Mesh.from_arrays(box, o.X, bad, o.tags, o.parents)
    assert e.value.code == pb.PARO_EINVAL
    with pytest.raises(pb.ParoError):
        pb.Mesh.from_arrays(box, o.X, o.tets, o.tags * 0, o.parents)
    badp = o.parents.copy()
    badp[-1] = [badp.shape[0] - 1, 0]  # a parent not older than the vertex
    with pytest.raises(pb.ParoError):
        pb.Mesh.from_arrays(box, o.X, o.tets, o.tags, badp)


def test_problem_sizes_match_a_brute_force_pattern():
    o = adapt.refine(adapt.refine(adapt.from_kuhn(3, -2.0, 2.0),
                                  [1, 20, 40, 77]), [5, 9, 100])
    m = pb.Mesh.from_arrays(_box(3, -2.0, 2.0), o.X, o.tets, o.tags,
                            o.parents)
    dof = o.dof
    pairs = set()
    for t in o.tets:
        for a, b in itertools.product(t, t):
            if dof[a] >= 0 and dof[b] >= 0:
                pairs.add((dof[a], dof[b]))
    n, nnz, ws = pb.paro_mesh_query(m, pb.default_opts(N=2, m=1))
    assert n == int((dof >= 0).sum()) and nnz == len(pairs) and ws > 0
    with pytest.raises(pb.ParoError):
        pb.paro_mesh_query(m, pb.default_opts(N=2, m=1,
                                              precision=pb.PARO_FP32_INNER))
