"""Comparison measures shared by the tests (no method arithmetic)."""
import numpy as np


def rel_lambda_err(lam, ref):
    """max_i |l_i - r_i| / max(|r_i|, 1e-3 max|r|)."""
    lam = np.asarray(lam, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return float(np.max(np.abs(lam - ref) / floor))


def subspace_sine(M, U, Uref):
    """Largest principal-angle sine between span U and span Uref in the M
    inner product (both M-orthonormal): sqrt(lambda_max(E^T M E)) with
    E = U - Uref (Uref^T M U)."""
    MU = M @ U
    E = U - Uref @ (Uref.T @ MU)
    G = E.T @ (M @ E)
    G = 0.5 * (G + G.T)
    return float(np.sqrt(max(np.max(np.linalg.eigvalsh(G)), 0.0)))


def m_orthonormality_error(M, U):
    G = U.T @ (M @ U)
    return float(np.max(np.abs(G - np.eye(G.shape[0]))))


def closed_prefix(lam_ref, N, rel_gap=1e-3):
    """Largest k <= N with a relative gap >= rel_gap between lam_ref[k-1]
    and lam_ref[k] (needs len(lam_ref) > N)."""
    for k in range(N, 0, -1):
        gap = (lam_ref[k] - lam_ref[k - 1]) / max(abs(lam_ref[k - 1]), 1e-12)
        if gap >= rel_gap:
            return k
    return 0
