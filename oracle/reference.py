"""Plain definition of the ParO fixed point (oracle).

Test infrastructure only (see oracle/__init__.py).

With the mesh held fixed, the pairs ParO converges to are the lowest N
eigenpairs of the discrete eigenproblem a(u_h, v) = lambda_h (u_h, v) for
all v in V_h (appendix, eq. (fem-eigen)), i.e. H u = lambda M u.  Written
out with library eigensolvers.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def dense_lowest(H, M, k):
    """Lowest k pairs of H u = lambda M u by a dense generalised eigh."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    Md = M.toarray() if hasattr(M, "toarray") else np.asarray(M)
    lam, U = sla.eigh(Hd, Md, subset_by_index=[0, k - 1])
    return lam, U


def sparse_lowest(H, M, k, sigma):
    """Lowest k pairs by shift-invert Lanczos about sigma < lambda_1."""
    lam, U = spla.eigsh(H.tocsc(), k=k, M=M.tocsc(), sigma=sigma,
                        which="LM", tol=1e-13)
    order = np.argsort(lam)
    lam, U = lam[order], U[:, order]
    # M-normalise (eigsh returns M-orthonormal vectors up to rounding).
    U = U / np.sqrt(np.einsum("ij,ij->j", U, M @ U))[None, :]
    return lam, U
