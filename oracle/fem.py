"""P1 finite elements on a uniform Kuhn-tetrahedral mesh of a box (oracle).

Test infrastructure only (see oracle/__init__.py).

Follows the finite-element setting of the paper:
  * Sec. 2 (preliminaries): conforming, shape-regular tetrahedral meshes and
    the space S^{h,1}_0 of continuous piecewise-linear functions vanishing on
    the boundary (the H^1_0 trace condition).
  * eq. (eq-operator-A) with a fixed potential, equivalently the appendix's
    a(u, v) = int A grad u . grad v + c u v with A = I/2 and c = V:
        a(w, v) = 1/2 (grad w, grad v) + (V w, v).
  * (., .) is the L2 inner product, so the "B" of A u = lambda B u is the
    consistent mass matrix.

Mesh: nc cubes per axis, each split into the six Kuhn tetrahedra that share
the cube's main diagonal from corner (0,0,0) to (1,1,1); for a permutation
p of the axes, the tetrahedron is v, v + e_p0, v + e_p0 + e_p1, v + (1,1,1).
All cubes use the same diagonal direction, so the mesh is conforming.

Potential: the nodal (P1) interpolant V_h of V, integrated exactly against
products of hat functions.  Exact integration of barycentric monomials over
a tetrahedron T:  int_T prod_a lambda_a^{k_a} = |T| 3! prod_a k_a! /
(sum_a k_a + 3)!.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Mesh:
    nc: tuple            # cells per axis (nx, ny, nz)
    lo: np.ndarray       # (3,)
    hi: np.ndarray       # (3,)
    h: np.ndarray        # (3,) cell sizes
    X: np.ndarray        # (nv, 3) vertex coordinates, x fastest
    tets: np.ndarray     # (nt, 4) vertex indices
    dof: np.ndarray      # (nv,) interior dof number or -1 on the boundary

    @property
    def n_dof(self) -> int:
        return int((self.dof >= 0).sum())


def kuhn_mesh(nc, lo, hi) -> Mesh:
    """Uniform Kuhn mesh of the box [lo, hi] with nc cubes per axis (nc an
    int or (nx, ny, nz); lo, hi scalars or 3-vectors).

    Interior dofs are the vertices with index 1..n_a-1 on every axis a,
    numbered x fastest: d = (i-1) + (nx-1) ((j-1) + (ny-1) (k-1)).
    """
    ncs = (nc, nc, nc) if np.isscalar(nc) else tuple(int(c) for c in nc)
    lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (3,)).copy()
    hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (3,)).copy()
    h = (hi - lo) / np.array(ncs, dtype=np.float64)
    nvx, nvy, nvz = (c + 1 for c in ncs)
    kk, jj, ii = np.meshgrid(np.arange(nvz), np.arange(nvy), np.arange(nvx),
                             indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    X = np.stack([lo[0] + h[0] * ii, lo[1] + h[1] * jj, lo[2] + h[2] * kk],
                 axis=1)

    def vid(i, j, k):
        return i + nvx * (j + nvy * k)

    ck, cj, ci = np.meshgrid(np.arange(ncs[2]), np.arange(ncs[1]),
                             np.arange(ncs[0]), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for p in itertools.permutations(range(3)):
        a = np.zeros(3, dtype=np.int64)
        b = unit[p[0]]
        c = unit[p[0]] + unit[p[1]]
        d = np.ones(3, dtype=np.int64)
        verts = [vid(ci + o[0], cj + o[1], ck + o[2]) for o in (a, b, c, d)]
        tets.append(np.stack(verts, axis=1))
    tets = np.concatenate(tets, axis=0)

    mx, my = ncs[0] - 1, ncs[1] - 1
    interior = (ii >= 1) & (ii <= ncs[0] - 1) & (jj >= 1) & (jj <= ncs[1] - 1) \
        & (kk >= 1) & (kk <= ncs[2] - 1)
    dof = np.full(X.shape[0], -1, dtype=np.int64)
    dof[interior] = (ii[interior] - 1) + mx * ((jj[interior] - 1)
                                               + my * (kk[interior] - 1))
    return Mesh(ncs, lo, hi, h, X, tets, dof)


def barycentric_integral(exponents, volume):
    """int_T prod_a lambda_a^{k_a} dx over a tetrahedron of given volume."""
    num = 6.0 * np.prod([math.factorial(k) for k in exponents])
    return volume * num / math.factorial(sum(exponents) + 3)


def element_geometry(mesh: Mesh):
    """Volumes |T| and barycentric gradients grad lambda_a (nt, 4, 3)."""
    P = mesh.X[mesh.tets]                       # (nt, 4, 3)
    E = P[:, 1:, :] - P[:, :1, :]               # rows: x_a - x_0, a = 1..3
    vol = np.abs(np.linalg.det(E)) / 6.0
    # x - x_0 = E^T lambda_{1..3}  =>  grad lambda_a = column a of E^{-1}.
    Einv = np.linalg.inv(E)                     # (nt, 3, 3)
    g = np.transpose(Einv, (0, 2, 1))           # g[:, a-1, :] = grad lambda_a
    g0 = -g.sum(axis=1, keepdims=True)
    return vol, np.concatenate([g0, g], axis=1)


def element_matrices(mesh: Mesh, V: np.ndarray):
    """Local stiffness, mass and potential-mass matrices, each (nt, 4, 4).

    K_T[a,b]  = int_T grad lambda_a . grad lambda_b
    M_T[a,b]  = int_T lambda_a lambda_b
    MV_T[a,b] = int_T V_h lambda_a lambda_b = sum_c V_c int lambda_a
                lambda_b lambda_c   (V_h = sum_c V_c lambda_c on T)
    """
    vol, g = element_geometry(mesh)
    K = vol[:, None, None] * np.einsum("tak,tbk->tab", g, g)
    two = np.zeros((4, 4))
    three = np.zeros((4, 4, 4))
    for a in range(4):
        for b in range(4):
            e = [0, 0, 0, 0]
            e[a] += 1
            e[b] += 1
            two[a, b] = barycentric_integral(e, 1.0)
            for c in range(4):
                e3 = list(e)
                e3[c] += 1
                three[a, b, c] = barycentric_integral(e3, 1.0)
    M = vol[:, None, None] * two[None]
    Vt = V[mesh.tets]                            # (nt, 4)
    MV = vol[:, None, None] * np.einsum("abc,tc->tab", three, Vt)
    return K, M, MV


def _scatter(mesh: Mesh, local: np.ndarray) -> sp.csr_matrix:
    """Sum element matrices into the interior x interior global matrix."""
    d = mesh.dof[mesh.tets]                      # (nt, 4)
    rows = np.repeat(d[:, :, None], 4, axis=2)
    cols = np.repeat(d[:, None, :], 4, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    n = mesh.n_dof
    A = sp.coo_matrix((local[keep], (rows[keep], cols[keep])), shape=(n, n))
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def assemble(mesh: Mesh, V: np.ndarray):
    """Global stiffness K, mass M and potential mass M_V (interior dofs).

    The Hamiltonian of the linear ParO problem is H = K/2 + M_V
    (eq. (eq-operator-A) with the potential held fixed)."""
    K, M, MV = element_matrices(mesh, np.asarray(V, dtype=np.float64))
    return _scatter(mesh, K), _scatter(mesh, M), _scatter(mesh, MV)


def hamiltonian(mesh: Mesh, V: np.ndarray):
    """(H, M) with H = K/2 + M_V."""
    K, M, MV = assemble(mesh, V)
    return (0.5 * K + MV).tocsr(), M
