"""Oracle: gradient of L = Re(eta^H A^{-1} b) with respect to the links and the source.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper computes no gradient; this serves the differentiable-solve extension.  With
x = A^{-1} b and lambda = A^{-H} eta (an adjoint solve; gamma5-hermiticity, Sec. 1, gives
A^{-H} = gamma5 A(-mu)^{-1} gamma5):

    dL = Re(lambda^H db) - Re(lambda^H dA x),   dA = -kappa dH.

Only two terms of H hold the link U_mu(y): the forward hop out of y and the backward hop out of
y + mu.  With the complex-gradient convention dL = Re sum conj(G) dU,

    G_mu(y) = kappa * sum_spin [ lambda(y) ((1 - gamma_mu) x(y+mu))^H + x(y) ((1 + gamma_mu) lambda(y+mu))^H ]

and grad_b = lambda.  The su(3) force for U -> exp(i theta T_a) U, T_a = lambda_a / 2 (Gell-Mann),
is dL/dtheta_a = Re( i tr[T_a U G^H] ).
"""
from __future__ import annotations

import numpy as np

from .wilson import GAMMA, I4


def gell_mann():
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


T_GEN = gell_mann() / 2.0


def link_gradient(U, lat, kappa, lam, x):
    """Complex gradient G (shape (4, V, 3, 3)) for one or more right-hand sides
    (lam, x of shape (V,4,3) or (nrhs,V,4,3); contributions are summed)."""
    lam = np.asarray(lam).reshape(-1, lat.V, 4, 3)
    x = np.asarray(x).reshape(-1, lat.V, 4, 3)
    G = np.zeros((4, lat.V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        f = lat.fwd[mu]
        for lj, xj in zip(lam, x):
            a = np.einsum("st,xtc->xsc", I4 - GAMMA[mu], xj[f])
            z = np.einsum("st,xtc->xsc", I4 + GAMMA[mu], lj[f])
            G[mu] += np.einsum("xsa,xsb->xab", lj, np.conj(a))
            G[mu] += np.einsum("xsa,xsb->xab", xj, np.conj(z))
    return kappa * G


def su3_force(U, G):
    """Coefficients F[mu, y, a] = Re(i tr[T_a U G^H]), shape (4, V, 8)."""
    UGh = np.einsum("mxab,mxcb->mxac", U, np.conj(G))
    return np.real(1j * np.einsum("aij,mxji->mxa", T_GEN, UGh))
