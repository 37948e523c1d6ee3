"""Parallel orbital-updating iteration for a linear eigenproblem (oracle).

Test infrastructure only (see oracle/__init__.py).

Follows Algorithm A.1 of the appendix (ParO for a linear elliptic
eigenproblem), with the buffer orbitals of Algorithm 3.2 and with Step 2
(mesh adaptation) taken as the identity, so V_{n+1} = V_h is fixed:

  Step 1  initial pairs (lambda_i^(0), u_i^(0)), orthonormal in L2.
  Step 3  for each i independently: a(u_i^(n+1/2), v) = lambda_i^(n) (u_i^(n), v)
          for all v, i.e. the source problem H w_i = lambda_i M u_i.
  Step 4  Rayleigh-Ritz on span{u_i^(n+1/2)}: a(u, v) = lambda (u, v) for all v
          in the span, with ||u||_0 = 1, giving (lambda_i^(n+1), u_i^(n+1)).

Readings where the paper is silent (each is listed with its reason in the
design notes):
  * Shift.  The appendix assumes c >= 0, so H is positive definite.  For a
    potential with negative values the source problem is solved in the
    equivalent shifted form (H - s M) w_i = (lambda_i - s) M u_i with
    s = min_nodes V_h - 1, which keeps the matrix positive definite; s = 0
    when V_h >= 0, which is the paper's literal Step 3.  The fixed point is
    unchanged (the exact eigenpairs still reproduce themselves).
  * Initial data.  The seeded orbitals are replaced by the Ritz pairs of
    their span, which are L2-orthonormal as Step 1 requires and supply
    lambda^(0), which the paper leaves to the user.
  * Source solver.  The paper does not name one: each source problem is
    solved by Jacobi-preconditioned conjugate gradients, started from
    x0 = u_i^(n), until ||r||_2 <= rtol ||b||_2, or, with reduce > 0, until
    ||r||_2 <= max(rtol ||b||_2, reduce ||r_0||_2) (an inexact Step 3: the
    start's residual b - A u_i is minus the pair's eigen-residual
    H u_i - lambda_i M u_i, and the solve shrinks it by the factor reduce).
  * Stopping.  The paper runs a fixed number of iterations.  Here the loop
    stops after max_steps, or once every requested pair has a relative
    eigenvalue change <= lambda_tol and relative residual <= resid_tol.
"""
from __future__ import annotations

import dataclasses
import multiprocessing
from typing import List, Optional

import numpy as np
import scipy.linalg as sla


class NotSPD(RuntimeError):
    """CG met p^T A p <= 0: the source-problem matrix is not SPD."""


class NoConvergence(RuntimeError):
    """CG hit its iteration cap before the tolerance."""


def shift_from_potential(V_nodal: np.ndarray) -> float:
    """Shift s: 0 when V_h >= 0 (the unshifted Step 3), else min V_h - 1.

    The Rayleigh quotient of H = K/2 + M_V is at least min V_h because the
    kinetic term is nonnegative and int V_h u^2 >= min V_h int u^2, so
    H - s M is positive definite for s < min V_h."""
    vmin = float(np.min(V_nodal))
    return 0.0 if vmin >= 0.0 else vmin - 1.0


def jacobi_pcg(A, b, x0, dinv, rtol, maxit, reduce=0.0):
    """Jacobi-preconditioned CG for A x = b (one source problem, Step 3).

    Stops when ||r||_2 <= max(rtol ||b||_2, reduce ||r_0||_2), r_0 = b - A x0,
    checked before every iteration (so zero iterations are taken if x0
    already satisfies it).  Returns the solution and the number of
    iterations."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.linalg.norm(b))
    stop = max(rtol * bnorm, reduce * float(np.linalg.norm(r)))
    it = 0
    while float(np.linalg.norm(r)) > stop:
        if it >= maxit:
            raise NoConvergence(f"PCG: {it} iterations, "
                                f"|r|/|b| = {np.linalg.norm(r) / bnorm:.3e}")
        q = A @ p
        pq = float(p @ q)
        if not pq > 0.0:
            raise NotSPD(f"PCG breakdown: p^T A p = {pq}")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        z = dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        it += 1
    return x, it


def rayleigh_ritz(H, M, W):
    """Step 4: the Galerkin eigenproblem of H u = lambda M u on span W.

    Solves (W^T H W) c = theta (W^T M W) c; eigh returns theta ascending and
    C with C^T (W^T M W) C = I, so the Ritz vectors W C are L2-orthonormal
    (||u||_0 = 1 as Step 4 requires)."""
    HW = H @ W
    MW = M @ W
    Ah = W.T @ HW
    Bh = W.T @ MW
    Ah = 0.5 * (Ah + Ah.T)
    Bh = 0.5 * (Bh + Bh.T)
    theta, C = sla.eigh(Ah, Bh)
    return theta, W @ C


def rayleigh_ritz_clustered(H, M, W, sizes):
    """Step 4 cluster by cluster (the eigenvalue-separation variant of
    Sec. 3): the columns of W form consecutive clusters of the given sizes,
    and each cluster's span gets its own Galerkin eigenproblem, so the
    small problems cost sum q_i^3 instead of (sum q_i)^3.  Within a cluster
    the Ritz values ascend; clusters keep their order."""
    assert sum(sizes) == W.shape[1] and min(sizes) >= 1
    theta = np.empty(W.shape[1])
    U = np.empty_like(W)
    s = 0
    for q in sizes:
        th, Uc = rayleigh_ritz(H, M, W[:, s:s + q])
        theta[s:s + q] = th
        U[:, s:s + q] = Uc
        s += q
    return theta, U


def scale_floor(lam: np.ndarray) -> np.ndarray:
    """Denominator for relative eigenvalue measures: max(|l_i|, 1e-3 max|l|)."""
    return np.maximum(np.abs(lam), 1e-3 * np.max(np.abs(lam)))


def residuals(H, M, lam, U):
    """rho_i = ||H u_i - l_i M u_i||_2 / (max(|l_i|, 1e-3 max|l|) ||M u_i||_2)."""
    MU = M @ U
    R = H @ U - MU * lam[None, :]
    return np.linalg.norm(R, axis=0) / (scale_floor(lam)
                                        * np.linalg.norm(MU, axis=0))


@dataclasses.dataclass
class ParOResult:
    lam: np.ndarray              # requested eigenvalues (N,)
    U: np.ndarray                # requested orbitals (n, N), M-orthonormal
    lam_all: np.ndarray          # all N + m Ritz values of the last step
    U_all: np.ndarray
    sigma: float
    steps: int
    converged: bool
    lam_history: List[np.ndarray]
    resid_history: List[np.ndarray]
    pcg_iters: List[List[int]]


# Operator of the source problems seen by the worker processes of
# paro_solve(workers=k); set before the pool forks, read-only afterwards.
_POOL_OPERATOR = {}


def _pool_start():
    # One BLAS thread per worker: the workers already fill the cores, and a
    # BLAS thread pool inherited across fork() can stall.
    from threadpoolctl import threadpool_limits
    _POOL_OPERATOR["limits"] = threadpool_limits(limits=1)


def _pool_solve(job):
    b, x0 = job
    op = _POOL_OPERATOR
    return jacobi_pcg(op["A"], b, x0, op["dinv"], op["rtol"], op["maxit"],
                      op["reduce"])


def paro_step(H, M, A, dinv, lam, U, sigma, rtol, maxit, clusters=None,
              pool=None, reduce=0.0):
    """One ParO iteration (Steps 3 and 4) from (lam, U); returns the new
    pairs and the PCG iteration count of each source problem.  With
    `clusters` (sizes of consecutive column groups) Step 4 projects each
    cluster separately (rayleigh_ritz_clustered).  With `pool` (from
    paro_solve(workers=k)) the independent source problems of Step 3 are
    spread over worker processes, which the paper names as the method's
    parallelism; each is the same jacobi_pcg call as in the serial loop.
    `reduce`: the inexact stopping test of jacobi_pcg."""
    MU = M @ U
    W = np.empty_like(U)
    jobs = [((lam[i] - sigma) * MU[:, i], U[:, i]) for i in range(U.shape[1])]
    if pool is None:                         # Step 3: independent problems
        out = [jacobi_pcg(A, b, x0, dinv, rtol, maxit, reduce)
               for b, x0 in jobs]
    else:
        out = pool.map(_pool_solve, jobs, chunksize=1)
    its = []
    for i, (w, k) in enumerate(out):
        W[:, i] = w
        its.append(k)
    if clusters:                             # Step 4
        lam_new, U_new = rayleigh_ritz_clustered(H, M, W, clusters)
    else:
        lam_new, U_new = rayleigh_ritz(H, M, W)
    return lam_new, U_new, its


def paro_solve(H, M, U0, N, sigma: Optional[float] = None, V_nodal=None,
               max_steps=100, lambda_tol=0.0, resid_tol=0.0, rtol=1e-10,
               maxit=None, callback=None, workers=None,
               reduce=0.0) -> ParOResult:
    """Run ParO from the orbitals U0 (n x (N + m)).

    sigma: the shift (None -> shift_from_potential(V_nodal)).
    Stops after max_steps, or earlier when lambda_tol > 0 and every
    requested pair satisfies both tolerances.  workers: number of processes
    for the source problems of Step 3 (None: solved one after another);
    the iterates are the same either way.  reduce: the source solves'
    inexact stopping test (jacobi_pcg)."""
    if sigma is None:
        sigma = shift_from_potential(V_nodal)
    n = H.shape[0]
    if maxit is None:
        maxit = 10 * n
    A = (H - sigma * M).tocsr()
    dinv = 1.0 / A.diagonal()
    lam, U = rayleigh_ritz(H, M, np.asarray(U0, dtype=np.float64))  # Step 1
    lam_hist = [lam.copy()]
    res_hist = [residuals(H, M, lam, U)[:N]]
    pcg_hist = []
    pool = None
    if workers:
        _POOL_OPERATOR.update(A=A, dinv=dinv, rtol=rtol, maxit=maxit,
                              reduce=reduce)
        pool = multiprocessing.get_context("fork").Pool(workers,
                                                        _pool_start)
    try:
        lam, U, steps, converged = _iterate(
            H, M, A, dinv, lam, U, sigma, rtol, maxit, N, max_steps,
            lambda_tol, resid_tol, callback, pool, lam_hist, res_hist,
            pcg_hist, reduce)
    finally:
        if pool is not None:
            pool.close()
            pool.join()
            _POOL_OPERATOR.clear()
    return ParOResult(lam[:N].copy(), U[:, :N].copy(), lam, U, sigma, steps,
                      converged, lam_hist, res_hist, pcg_hist)


def _iterate(H, M, A, dinv, lam, U, sigma, rtol, maxit, N, max_steps,
             lambda_tol, resid_tol, callback, pool, lam_hist, res_hist,
             pcg_hist, reduce=0.0):
    """The ParO loop of paro_solve (Steps 3-4 repeated, stopping test)."""
    converged = False
    steps = 0
    for step in range(max_steps):
        lam_new, U, its = paro_step(H, M, A, dinv, lam, U, sigma, rtol, maxit,
                                    pool=pool, reduce=reduce)
        dl = np.abs(lam_new - lam) / scale_floor(lam_new)
        lam = lam_new
        rho = residuals(H, M, lam, U)
        lam_hist.append(lam.copy())
        res_hist.append(rho[:N])
        pcg_hist.append(its)
        steps = step + 1
        if callback is not None:
            callback(steps, lam, U)
        if lambda_tol > 0 and np.max(dl[:N]) <= lambda_tol \
                and np.max(rho[:N]) <= resid_tol:
            converged = True
            break
    return lam, U, steps, converged
