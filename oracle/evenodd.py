"""Oracle: the even-odd reduced (Schur complement) system, plain NumPy FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3 and Sec. 4 solve the even-odd preconditioned system.  H only couples sites of opposite
parity ((x+y+z+t) mod 2), so in parity blocks the operator of ``oracle.wilson`` reads

    A(mu) = [[ D,            -kappa H_eo ],      D = I + i*mu*gamma5  (site-diagonal)
             [ -kappa H_oe,   D          ]]

and eliminating the odd half gives the Schur complement on the even sites

    Ahat(mu) = D - kappa^2 H_eo D^{-1} H_oe,        D^{-1} = (I - i*mu*gamma5) / (1 + mu^2).

A x = b is then solved as  Ahat x_e = bhat,  bhat = b_e + kappa H_eo D^{-1} b_o,
x_o = D^{-1} (b_o + kappa H_oe x_e).  The adjoint: Ahat(mu)^dagger = gamma5 Ahat(-mu) gamma5 (the
hop H^dagger and D(-mu) in place of H and D(mu)), with the same elimination for A^dagger x = b.

Readings (the paper names the preconditioning but not its form): the asymmetric Schur complement
on the even sites with D = I + i*mu*gamma5 (the twisted term added literally, as in the full
operator); one application of Ahat is one matrix-vector product.

Half vectors hold the even (or odd) sites in lexicographic order, 12 complex numbers per site,
V/2 sites: for even Lx this is the order of lex >> 1.
"""
from __future__ import annotations

import numpy as np

from .wilson import gamma5, hopping, hopping_sites


def parity_sites(lat, parity):
    """Lexicographic indices of the sites of one parity, in increasing order."""
    return np.nonzero(lat.parity == parity)[0]


def embed(lat, half, parity):
    """Full (V,4,3) vector equal to ``half`` on the sites of ``parity`` and zero elsewhere."""
    out = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    out[parity_sites(lat, parity)] = np.asarray(half, dtype=np.complex128).reshape(-1, 4, 3)
    return out


def restrict(lat, full, parity):
    """The sites of ``parity`` of a full vector, as a flat half vector."""
    return np.asarray(full, dtype=np.complex128).reshape(lat.V, 4, 3)[
        parity_sites(lat, parity)].reshape(-1)


def _diag(x, mu, inverse):
    """D x = x + i mu gamma5 x, or D^{-1} x = (x - i mu gamma5 x) / (1 + mu^2), on (n,4,3) sites."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1, 4, 3)
    g5x = gamma5(x, x.shape[0])
    if inverse:
        return (x - 1j * mu * g5x) / (1.0 + mu * mu)
    return x + 1j * mu * g5x


def _hop_half(U, lat, half, parity_in, dagger):
    """H (or H^dagger) applied to a half vector of parity ``parity_in``; returns the half vector
    of the other parity."""
    full = hopping(U, embed(lat, half, parity_in), lat, dagger)
    return restrict(lat, full, 1 - parity_in)


def schur_apply(U, lat, kappa, xe, mu=0.0, dagger=False):
    """Ahat(mu) x_e (``dagger``: Ahat(mu)^dagger x_e) on a flat even half vector."""
    m = -mu if dagger else mu
    t = _hop_half(U, lat, xe, 0, dagger)                 # H_oe x_e
    t = _diag(t, m, inverse=True).reshape(-1)            # D^{-1} H_oe x_e
    u = _hop_half(U, lat, t, 1, dagger)                  # H_eo D^{-1} H_oe x_e
    return (_diag(xe, m, inverse=False).reshape(-1) - kappa * kappa * u)


def schur_operator(U, lat, kappa, mu=0.0, dagger=False):
    """Closure x_e -> Ahat x_e on flat half vectors of length 6 V."""
    def A(x):
        return schur_apply(U, lat, kappa, x, mu, dagger)
    return A


def schur_source(U, lat, kappa, b, mu=0.0, dagger=False):
    """bhat = b_e + kappa H_eo D^{-1} b_o for a full right-hand side b; returns the even half."""
    m = -mu if dagger else mu
    bo = _diag(restrict(lat, b, 1), m, inverse=True).reshape(-1)
    return restrict(lat, b, 0) + kappa * _hop_half(U, lat, bo, 1, dagger)


def schur_reconstruct(U, lat, kappa, xe, b, mu=0.0, dagger=False):
    """The full solution: x_e given, x_o = D^{-1} (b_o + kappa H_oe x_e).  Returns (V,4,3)."""
    m = -mu if dagger else mu
    xo = restrict(lat, b, 1) + kappa * _hop_half(U, lat, xe, 0, dagger)
    xo = _diag(xo, m, inverse=True).reshape(-1)
    return embed(lat, xe, 0) + embed(lat, xo, 1)


def schur_apply_sites(U, lat, kappa, xe, sites, mu=0.0, dagger=False):
    """(Ahat x_e)(x) at a list of even lexicographic sites only (for large lattices): the odd
    neighbours' D^{-1} (H x_e), then the hop of those back to the sites.  Returns
    (len(sites), 4, 3)."""
    sites = np.asarray(sites, dtype=np.int64)
    if np.any(lat.parity[sites] != 0):
        raise ValueError("sites must be even")
    m = -mu if dagger else mu
    full = embed(lat, xe, 0)
    nbr = np.unique(np.concatenate([lat.fwd[d][sites] for d in range(4)] +
                                   [lat.bwd[d][sites] for d in range(4)]))
    t = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    t[nbr] = _diag(hopping_sites(U, full, lat, nbr, dagger), m, inverse=True)
    u = hopping_sites(U, t, lat, sites, dagger)
    return _diag(full[sites], m, inverse=False) - kappa * kappa * u


def gamma5_half(x):
    """gamma5 on a flat half vector."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1, 4, 3)
    return gamma5(x, x.shape[0]).reshape(-1)
