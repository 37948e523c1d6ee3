"""Nonlocal pseudopotential term as a rank-k Galerkin operator (oracle).

Test infrastructure only (see oracle/__init__.py).

Follows the pseudopotential model of Sec. 2: V_nl u = sum_j (u, zeta_j)
zeta_j with projector functions zeta_j.  With each zeta_j taken as its P1
interpolant on the interior vertices (zero on the boundary), the Galerkin
matrix of V_nl is Z Z^T with Z = M zeta (n x k): entry (a, b) is
sum_j (phi_a, zeta_j)(zeta_j, phi_b).  The Hamiltonian of the source
problems and of the projection becomes H + Z Z^T; the Jacobi
preconditioner keeps the local diagonal (a reading: the paper does not
name a preconditioner).
"""
from __future__ import annotations

import numpy as np


def projector_matrix(M, zeta: np.ndarray) -> np.ndarray:
    """Z = M zeta: column j holds (phi_a, zeta_j) for every basis function."""
    return np.asarray(M @ np.asarray(zeta, dtype=np.float64))


class LowRankPlus:
    """S + Z Z^T applied as S @ x + Z (Z^T x) (never formed densely)."""

    def __init__(self, S, Z: np.ndarray):
        self.S = S
        self.Z = np.asarray(Z, dtype=np.float64)
        self.shape = S.shape

    def __matmul__(self, x):
        return self.S @ x + self.Z @ (self.Z.T @ x)

    def diagonal(self):
        """The local part's diagonal (the preconditioner's)."""
        return self.S.diagonal()

    def dense(self) -> np.ndarray:
        return self.S.toarray() + self.Z @ self.Z.T
