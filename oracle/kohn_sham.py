"""Self-consistent Kohn-Sham iteration around ParO (oracle).

Test infrastructure only (see oracle/__init__.py).

Follows Sec. 2 (the Kohn-Sham equation, eq. (eq-ks), its weak form
(weak-ks) and the form a(U; w, v) of eq. (eq-operator-A)) and Algorithm
3.1 (one ParO step per outer iteration, the Hamiltonian built from the
current density), with these readings:

  * The Hartree potential solves the Poisson equation -Lap V_H = 4 pi rho
    (Sec. 2) with V_H = 0 on the box boundary; its weak P1 form is
    K V_H = 4 pi M rho on the interior dofs (the 1/2 in front of the
    Hartree integral of eq. (eq-ks) is not used: the Poisson form has none).
  * Each orbital holds two electrons (spin-unpolarised, N occupied
    orbitals): rho = 2 sum_{i <= N} u_i^2, taken at the vertices (the P1
    interpolant of the density), zero on the boundary.
  * Exchange-correlation: the local-density Slater exchange
    v_x(rho) = -(3 rho / pi)^(1/3), the derivative of the exchange energy
    density -(3/4)(3/pi)^(1/3) rho^(4/3) of the homogeneous electron gas.
  * The Hamiltonian of a step is built from the mixed input density
    rho_in and used for both Step 3 and Step 4; linear mixing
    rho_in <- (1 - beta) rho_in + beta rho_out, beta = 0.3, or (the paper
    names no mixing scheme) Kerker-preconditioned mixing
    rho_in <- rho_in + beta (K + q0^2 vol I)^{-1} K (rho_out - rho_in),
    with K the P1 stiffness matrix and vol the cell volume: the grid form
    of Kerker's factor q^2 / (q^2 + q0^2), which damps the long-wavelength
    part of the residual.
  * Outer iteration n: rho_out = density of U^(n); rho_in = rho_out at
    n = 0, else the mixture; V_eff = V_ext + V_H(rho_in) + v_x(rho_in) at
    the vertices; one ParO step with H(V_eff) and its shift.  The density
    residual of iteration n is ||rho_out^(n) - rho_in^(n-1)||_2 /
    ||rho_in^(n-1)||_2.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse.linalg as spla

from . import fem
from . import paro as oparo


def density(U: np.ndarray, N: int, occupancy: float = 2.0) -> np.ndarray:
    """Nodal density on the interior dofs: occupancy * sum_{i<=N} u_i^2."""
    return occupancy * np.sum(np.asarray(U)[:, :N] ** 2, axis=1)


def hartree(K, M, rho: np.ndarray) -> np.ndarray:
    """P1 Hartree potential on the interior dofs: K V_H = 4 pi M rho
    (homogeneous Dirichlet data), solved directly."""
    return spla.spsolve(K.tocsc(), 4.0 * np.pi * (M @ rho))


def slater_exchange(rho: np.ndarray) -> np.ndarray:
    """Local-density Slater exchange potential -(3 rho / pi)^(1/3)."""
    return -np.cbrt(3.0 * np.maximum(rho, 0.0) / np.pi)


def kerker_filter(K, e: np.ndarray, q0: float, vol: float) -> np.ndarray:
    """(K + q0^2 vol I)^{-1} K e (q0 = 0: e itself), solved directly."""
    if q0 == 0.0:
        return np.array(e, dtype=np.float64, copy=True)
    import scipy.sparse as sp
    A = (K + (q0 * q0 * vol) * sp.identity(K.shape[0], format="csr")).tocsc()
    return spla.spsolve(A, K @ e)


def effective_potential(mesh: fem.Mesh, V_ext: np.ndarray, rho: np.ndarray,
                        vh: np.ndarray) -> np.ndarray:
    """V_ext + V_H + v_x at every vertex (rho = V_H = 0 on the boundary)."""
    V = np.array(V_ext, dtype=np.float64, copy=True)
    inner = mesh.dof >= 0
    d = mesh.dof[inner]
    V[inner] += vh[d] + slater_exchange(rho[d])
    return V


@dataclass
class SCFResult:
    lam: np.ndarray                 # final Ritz values (N + m)
    U: np.ndarray                   # final orbitals (n x (N + m))
    rho_in: np.ndarray              # last mixed density
    lam_history: List[np.ndarray]   # after Step 1 and after every step
    residual_history: List[float]   # density residual per iteration
    sigma_history: List[float]
    V_eff: np.ndarray               # potential of the last step


def scf(mesh: fem.Mesh, V_ext: np.ndarray, U0: np.ndarray, N: int,
        iterations: int, mixing: float = 0.3, rtol: float = 1e-10,
        maxit=None, kerker_q0: float = 0.0) -> SCFResult:
    """`iterations` outer iterations of ParO with Kohn-Sham updates.

    Step 1: Rayleigh-Ritz of U0 with the bare Hamiltonian H(V_ext).
    kerker_q0 > 0 filters the density residual before mixing
    (kerker_filter); 0 is plain linear mixing."""
    K, M, _ = fem.assemble(mesh, np.zeros(mesh.X.shape[0]))
    H0, _ = fem.hamiltonian(mesh, V_ext)
    lam, U = oparo.rayleigh_ritz(H0, M, np.asarray(U0, dtype=np.float64))
    n = U.shape[0]
    if maxit is None:
        maxit = 10 * n
    lam_hist, res_hist, sig_hist = [lam.copy()], [], []
    rho_in = None
    V = np.asarray(V_ext, dtype=np.float64)
    for it in range(iterations):
        rho_out = density(U, N)
        if rho_in is None:
            rho_in = rho_out
        else:
            res_hist.append(float(np.linalg.norm(rho_out - rho_in) /
                                  np.linalg.norm(rho_in)))
            if kerker_q0 > 0.0:
                vol = float(np.prod(mesh.h))
                rho_in = rho_in + mixing * kerker_filter(
                    K, rho_out - rho_in, kerker_q0, vol)
            else:
                rho_in = (1.0 - mixing) * rho_in + mixing * rho_out
        vh = hartree(K, M, rho_in)
        V = effective_potential(mesh, V_ext, rho_in, vh)
        H, _ = fem.hamiltonian(mesh, V)
        sigma = oparo.shift_from_potential(V)
        A = (H - sigma * M).tocsr()
        dinv = 1.0 / A.diagonal()
        lam, U, _ = oparo.paro_step(H, M, A, dinv, lam, U, sigma, rtol, maxit)
        lam_hist.append(lam.copy())
        sig_hist.append(sigma)
    return SCFResult(lam, U, rho_in, lam_hist, res_hist, sig_hist, V)
