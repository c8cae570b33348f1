"""Oracle: critical hopping parameter, plain FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3 fixes kappa_c as the kappa at which the real part of A's smallest eigenvalue vanishes.
With A = I - kappa H the eigenvectors of A do not depend on kappa and lambda(A) = 1 - kappa
lambda(H), so kappa_c = 1 / max_j Re lambda_j(H).  The rightmost eigenvalues of H come from
ARPACK (scipy.sparse.linalg.eigs, which='LR'), or from dense eigvals on tiny lattices.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs

from .wilson import dense_hopping, hopping


def kappa_c(U, lat, nev=3, tol=1e-12, ncv=None):
    """Returns (kappa_c, rightmost eigenvalues sorted by Re descending, eigen-residual of the
    first, i.e. ||H v - lambda v|| / ||v||)."""
    n = lat.n

    def mv(v):
        return hopping(U, v, lat).reshape(-1)

    H = LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    vals, vecs = eigs(H, k=nev, which="LR", tol=tol, ncv=ncv or max(2 * nev + 1, 40),
                      maxiter=100000)
    order = np.argsort(-vals.real)
    vals = vals[order]
    v = vecs[:, order[0]]
    res = np.linalg.norm(mv(v) - vals[0] * v) / np.linalg.norm(v)
    return 1.0 / vals[0].real, vals, res


def kappa_c_dense(U, lat):
    """Dense-eigenvalue kappa_c for tiny lattices."""
    ev = np.linalg.eigvals(dense_hopping(U, lat))
    return 1.0 / ev.real.max(), ev
