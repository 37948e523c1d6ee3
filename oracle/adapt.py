"""Adaptive finite element Step 2 of the ParO iteration (oracle).

Test infrastructure only (see oracle/__init__.py).

Follows Sec. 2 (adaptive finite element approximation): the loop
Solve -> Estimate -> Mark -> Refine, the Doerfler strategy (eq.
(dorfler-strategy)), the maximum strategy (eq. (maximum-strategy)) and
refinement by shape-regular bisection; and Step 2 of Algorithm 3.1 (a new
mesh T_{n+1} built from (lambda^(n), u^(n)), on which Step 3 then solves
with the orbitals u^(n) carried over).

Readings (the paper cites these rather than defining them):
  * Estimator.  The residual-type indicator of P1 eigenpairs of
    -1/2 Lap u + V u = lambda u, summed over the N requested orbitals:
        eta_T^2 = sum_i  h_T^2 ||lambda_i u_i - V_h u_i||^2_{L2(T)}
                       + 1/2 sum_{F in faces(T), F interior}
                             h_F ||[1/2 grad u_i . n_F]||^2_{L2(F)},
    h_T the longest edge of T, h_F the longest edge of F, [.] the jump
    across F (the P1 functions have no second derivatives inside T, and
    each interior face is shared by two elements, hence the 1/2).
  * Bisection.  Maubach's tagged bisection: an element is an ordered
    vertex list (x0, x1, x2, x3) with a tag k in {1, 2, 3}; it is cut at
    the midpoint z of its refinement edge (x0, xk) into
    (x0, .., x_{k-1}, z, x_{k+1}, .., x3) and (x1, .., xk, z, x_{k+1}, .., x3),
    both tagged k - 1 (3 after 1).  The Kuhn elements of the uniform box
    mesh, listed as v, v + e_p0, v + e_p0 + e_p1, v + (1,1,1), tag 3, are
    the starting elements; three rounds of bisection of every element give
    a mesh of the half-size grid's vertices whose elements are Kuhn
    elements of half the size (the sub-cubes' diagonals alternate in
    direction, unlike the uniform Kuhn mesh).  Conformity: before an element is
    cut at an edge, every element around that edge whose refinement edge
    differs is cut first (recursively), then all elements around the edge
    are cut at it together, so no hanging vertex remains.
  * Transfer.  The orbitals move to the new mesh by P1 interpolation: a
    new vertex, the midpoint of an edge (a, b), takes (u_a + u_b) / 2.
    The coarse P1 space lies in the fine one, so this is the coarse
    function itself, written in the fine basis.
  * Vertices on the box boundary carry the homogeneous Dirichlet data; the
    interior vertices, in vertex order, are the dofs.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Callable, Dict, List, Sequence, Tuple

import numpy as np

from . import fem
from . import paro as oparo


@dataclasses.dataclass
class AdaptiveMesh:
    """A bisection mesh of the box [lo, hi]: vertex coordinates, ordered
    elements with their bisection tags, and for every vertex made by
    bisection the two ends of the edge it halves (-1, -1 otherwise)."""
    lo: np.ndarray
    hi: np.ndarray
    X: np.ndarray                  # (nv, 3)
    tets: np.ndarray               # (nt, 4), ordered (x0, x1, x2, x3)
    tags: np.ndarray               # (nt,)
    parents: np.ndarray            # (nv, 2)

    @property
    def dof(self) -> np.ndarray:
        inside = np.all((self.X > self.lo + 1e-12 * (self.hi - self.lo)) &
                        (self.X < self.hi - 1e-12 * (self.hi - self.lo)),
                        axis=1)
        d = np.full(self.X.shape[0], -1, dtype=np.int64)
        d[inside] = np.arange(int(inside.sum()))
        return d

    def fem_mesh(self) -> fem.Mesh:
        """The same mesh for the oracle's assembly (fem.assemble)."""
        return fem.Mesh(None, self.lo, self.hi, None, self.X, self.tets,
                        self.dof)


def from_kuhn(nc, lo, hi) -> AdaptiveMesh:
    """The uniform Kuhn mesh as the starting bisection mesh (tag 3)."""
    m = fem.kuhn_mesh(nc, lo, hi)
    nv = m.X.shape[0]
    return AdaptiveMesh(m.lo, m.hi, m.X.copy(), m.tets.copy(),
                        np.full(m.tets.shape[0], 3, dtype=np.int64),
                        np.full((nv, 2), -1, dtype=np.int64))


# ---------------------------------------------------------------------------
# Estimate
# ---------------------------------------------------------------------------

def _quartic_tensor() -> np.ndarray:
    """Q[a,b,c,d] = int_T lambda_a lambda_b lambda_c lambda_d / |T|."""
    Q = np.zeros((4, 4, 4, 4))
    for idx in itertools.product(range(4), repeat=4):
        e = [0, 0, 0, 0]
        for a in idx:
            e[a] += 1
        Q[idx] = fem.barycentric_integral(e, 1.0)
    return Q


def _faces(tets: np.ndarray):
    """All element faces: sorted vertex triples (nt, 4, 3), the face
    opposite local vertex a at [:, a]."""
    f = np.stack([np.delete(tets, a, axis=1) for a in range(4)], axis=1)
    return np.sort(f, axis=2)


def estimator(mesh: AdaptiveMesh, V: np.ndarray, lam: Sequence[float],
              U: np.ndarray) -> np.ndarray:
    """eta_T for every element (see the module notes).  U: nodal values of
    the orbitals at the dofs (n_dof x N); V: potential at every vertex."""
    X, T = mesh.X, mesh.tets
    nt = T.shape[0]
    dof = mesh.dof
    full = np.zeros((X.shape[0], U.shape[1]))
    full[dof >= 0] = U[dof[dof >= 0]]
    vol, g = fem.element_geometry(mesh.fem_mesh())        # (nt,), (nt,4,3)
    # h_T: longest edge.
    P = X[T]
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    hT = np.max(np.stack([np.linalg.norm(P[:, a] - P[:, b], axis=1)
                          for a, b in edges], axis=1), axis=1)
    Q = _quartic_tensor()
    Vt = V[T]                                              # (nt, 4)
    eta2 = np.zeros(nt)
    # Element residual r = lambda u - V_h u.  With sum_b phi_b = 1 on T it
    # is the quadratic form sum_{a,b} R_ab phi_a phi_b,
    # R_ab = lambda (u_a + u_b) / 2 - (V_a u_b + V_b u_a) / 2, integrated
    # exactly (degree 4); R vanishes identically where V = lambda, so no
    # cancellation between separately integrated terms.
    for i, l in enumerate(lam):
        ut = full[T, i]                                    # (nt, 4)
        R = 0.5 * l * (ut[:, :, None] + ut[:, None, :]) \
            - 0.5 * (Vt[:, :, None] * ut[:, None, :]
                     + ut[:, :, None] * Vt[:, None, :])
        r2 = vol * np.einsum("abcd,tab,tcd->t", Q, R, R)
        eta2 += hT * hT * r2
    # Face jumps of 1/2 grad u . n over interior faces.
    F = _faces(T).reshape(-1, 3)                           # (4 nt, 3)
    owner = np.repeat(np.arange(nt), 4)
    order = np.lexsort((F[:, 2], F[:, 1], F[:, 0]))
    Fs, Os = F[order], owner[order]
    same = np.all(Fs[1:] == Fs[:-1], axis=1)
    i0 = np.nonzero(same)[0]
    ta, tb = Os[i0], Os[i0 + 1]
    fv = X[Fs[i0]]                                         # (nf, 3, 3)
    nrm = np.cross(fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0])
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    n_unit = nrm / (2.0 * area)[:, None]
    hF = np.max(np.stack([np.linalg.norm(fv[:, a] - fv[:, b], axis=1)
                          for a, b in ((0, 1), (0, 2), (1, 2))], axis=1),
                axis=1)
    for i in range(len(lam)):
        ut = full[T, i]
        grad = np.einsum("ta,tak->tk", ut, g)              # (nt, 3)
        jump = 0.5 * np.einsum("fk,fk->f", grad[ta] - grad[tb], n_unit)
        share = 0.5 * hF * area * jump * jump   # to each of the two
        np.add.at(eta2, ta, share)
        np.add.at(eta2, tb, share)
    return np.sqrt(eta2)


# ---------------------------------------------------------------------------
# Mark
# ---------------------------------------------------------------------------

def dorfler_mark(eta: np.ndarray, theta: float) -> np.ndarray:
    """Eq. (dorfler-strategy): a set M with sum_M eta^2 >= theta sum eta^2,
    of the smallest size: the elements in decreasing order of eta (ties by
    index) until the sum is reached.  Returns the marked indices."""
    e2 = np.asarray(eta, dtype=np.float64) ** 2
    order = np.lexsort((np.arange(e2.size), -e2))
    cum = np.cumsum(e2[order])
    k = int(np.searchsorted(cum, theta * e2.sum(), side="left")) + 1
    return np.sort(order[:min(k, e2.size)])


def maximum_mark(eta: np.ndarray, theta: float) -> np.ndarray:
    """Eq. (maximum-strategy): every element with eta >= theta max eta."""
    eta = np.asarray(eta, dtype=np.float64)
    return np.nonzero(eta >= theta * eta.max())[0]


# ---------------------------------------------------------------------------
# Refine
# ---------------------------------------------------------------------------

def refine(mesh: AdaptiveMesh, marked: Sequence[int]) -> AdaptiveMesh:
    """Bisect every marked element at least once, keeping the mesh
    conforming (see the module notes).  Returns a new mesh; the vertices of
    the old one keep their indices."""
    X = [x for x in mesh.X]
    parents = [tuple(p) for p in mesh.parents]
    tets: Dict[int, Tuple[Tuple[int, ...], int]] = {
        i: (tuple(int(v) for v in t), int(k))
        for i, (t, k) in enumerate(zip(mesh.tets, mesh.tags))}
    by_edge: Dict[Tuple[int, int], set] = {}
    mid: Dict[Tuple[int, int], int] = {}

    def key(a, b):
        return (a, b) if a < b else (b, a)

    def add(i):
        t = tets[i][0]
        for a, b in itertools.combinations(t, 2):
            by_edge.setdefault(key(a, b), set()).add(i)

    def remove(i):
        t = tets[i][0]
        for a, b in itertools.combinations(t, 2):
            by_edge[key(a, b)].discard(i)

    for i in tets:
        add(i)
    next_id = [len(tets)]

    def ref_edge(i):
        t, k = tets[i]
        return key(t[0], t[k])

    def midpoint(e):
        if e not in mid:
            a, b = e
            X.append(0.5 * (X[a] + X[b]))
            parents.append((a, b))
            mid[e] = len(X) - 1
        return mid[e]

    def cut(i):
        (t, k) = tets[i]
        z = midpoint(key(t[0], t[k]))
        c1 = t[:k] + (z,) + t[k + 1:]
        c2 = t[1:k + 1] + (z,) + t[k + 1:]
        kk = k - 1 if k > 1 else 3
        remove(i)
        del tets[i]
        for c in (c1, c2):
            j = next_id[0]
            next_id[0] += 1
            tets[j] = (c, kk)
            add(j)

    def bisect(i):
        e = ref_edge(i)
        while True:
            bad = [j for j in by_edge.get(e, ()) if ref_edge(j) != e]
            if not bad:
                break
            bisect(bad[0])
        for j in list(by_edge.get(e, ())):
            cut(j)

    for i in marked:
        if int(i) in tets:
            bisect(int(i))
    ids = sorted(tets)
    return AdaptiveMesh(mesh.lo, mesh.hi, np.array(X),
                        np.array([tets[i][0] for i in ids], dtype=np.int64),
                        np.array([tets[i][1] for i in ids], dtype=np.int64),
                        np.array(parents, dtype=np.int64))


# ---------------------------------------------------------------------------
# Transfer
# ---------------------------------------------------------------------------

def prolong(old: AdaptiveMesh, new: AdaptiveMesh,
            U: np.ndarray) -> np.ndarray:
    """P1 interpolation of dof values U (old n_dof x k) onto the refined
    mesh `new` (old vertices keep their indices; a new vertex takes the
    mean of the two ends of the edge it halves, in creation order)."""
    U = np.atleast_2d(np.asarray(U, dtype=np.float64).T).T
    od, nd = old.dof, new.dof
    full = np.zeros((new.X.shape[0], U.shape[1]))
    nold = old.X.shape[0]
    full[:nold][od >= 0] = U[od[od >= 0]]
    for v in range(nold, new.X.shape[0]):
        a, b = new.parents[v]
        full[v] = 0.5 * (full[a] + full[b])
    return full[nd >= 0]          # interior vertices in order = dof order


def interpolate(mesh: fem.Mesh, U: np.ndarray, points: np.ndarray,
                nc) -> np.ndarray:
    """Values at `points` of the P1 functions with dof values U (n_dof x k)
    on the uniform Kuhn mesh `mesh` of nc cells per axis: the element that
    contains a point (all barycentric coordinates >= -1e-12, found among
    the six of its grid cell) and its barycentric coordinates."""
    U = np.atleast_2d(np.asarray(U, dtype=np.float64).T).T
    ncs = np.broadcast_to(np.asarray(nc), (3,))
    full = np.zeros((mesh.X.shape[0], U.shape[1]))
    full[mesh.dof >= 0] = U[mesh.dof[mesh.dof >= 0]]
    h = (mesh.hi - mesh.lo) / ncs
    cell = np.clip(np.floor((points - mesh.lo) / h).astype(np.int64), 0,
                   ncs - 1)
    cid = cell[:, 0] + ncs[0] * (cell[:, 1] + ncs[1] * cell[:, 2])
    ncell = int(np.prod(ncs))
    out = np.zeros((points.shape[0], U.shape[1]))
    # fem.kuhn_mesh lists the six elements of cell c at c + q * ncell.
    for q in range(6):
        T = mesh.tets[cid + q * ncell]                    # (np, 4)
        P = mesh.X[T]
        E = np.transpose(P[:, 1:] - P[:, :1], (0, 2, 1))  # columns x_a - x_0
        lam = np.linalg.solve(E, (points - P[:, 0])[:, :, None])[:, :, 0]
        bary = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam],
                              axis=1)
        inside = np.all(bary >= -1e-12, axis=1)
        val = np.einsum("pa,pak->pk", bary, full[T])
        out[inside] = val[inside]
    return out


# ---------------------------------------------------------------------------
# Algorithm 3.1 with Step 2 adaptive (linear eigenproblem)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class AdaptiveResult:
    mesh: AdaptiveMesh
    lam: np.ndarray
    U: np.ndarray
    dofs: List[int]
    lam_history: List[np.ndarray]


def adaptive_paro(mesh: AdaptiveMesh, Vfun: Callable[[np.ndarray], np.ndarray],
                  U0: np.ndarray, N: int, steps: int, theta: float = 0.5,
                  strategy: str = "dorfler", refine_steps=None,
                  rtol: float = 1e-12) -> AdaptiveResult:
    """ParO with Step 2 adaptive: Step 1 (Rayleigh-Ritz of U0 on the first
    mesh), then per step: estimate on the current pairs, mark (Doerfler or
    maximum, parameter theta), refine, carry the orbitals over, and take
    Steps 3 and 4 on the new mesh.  refine_steps: the steps that adapt the
    mesh (None: every step); the others keep it."""
    V = Vfun(mesh.X)
    H, M = fem.hamiltonian(mesh.fem_mesh(), V)
    lam, U = oparo.rayleigh_ritz(H, M, np.asarray(U0, dtype=np.float64))
    dofs, hist = [U.shape[0]], [lam.copy()]
    for step in range(steps):
        if refine_steps is None or step in refine_steps:
            eta = estimator(mesh, V, lam[:N], U[:, :N])
            marked = (dorfler_mark(eta, theta) if strategy == "dorfler"
                      else maximum_mark(eta, theta))
            new = refine(mesh, marked)
            U = prolong(mesh, new, U)
            mesh = new
            V = Vfun(mesh.X)
            H, M = fem.hamiltonian(mesh.fem_mesh(), V)
        s = oparo.shift_from_potential(V)
        A = (H - s * M).tocsr()
        lam, U, _ = oparo.paro_step(H, M, A, 1.0 / A.diagonal(), lam, U, s,
                                    rtol, 10 * U.shape[0])
        dofs.append(U.shape[0])
        hist.append(lam.copy())
    return AdaptiveResult(mesh, lam, U, dofs, hist)
