"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the benchmark.

This module only *draws* inputs: gauge links, sources, gauge transformations and random
directions.  It holds none of the solver or operator arithmetic, so that the CPU oracle and
the HIP library can both be fed from it without sharing any computation.

Conventions (identical on both sides of the boundary):

* lattice extents ``L = (Lx, Ly, Lz, Lt)``; lexicographic site index
  ``lex = x + Lx*(y + Ly*(z + Lz*t))``; ``V = Lx*Ly*Lz*Lt``.
* gauge field: complex128 array ``U[mu, lex, a, b]`` of shape ``(4, V, 3, 3)``; ``U[mu, x]`` is the
  SU(3) link from site ``x`` to ``x + mu``.
* spinor field: complex128 array of shape ``(nrhs, V, 4, 3)`` (spin, colour), i.e. element index
  ``12*lex + 3*spin + colour`` inside one right-hand side.

The paper's quenched beta=6.0 configurations are not available; links are drawn as
``exp(i*c*Q)`` with ``Q`` a traceless Hermitian matrix built from Gaussian entries, with ``c``
setting how far the field is from the free (unit) field.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gauge_field", "unit_field", "z2_sources", "gaussian_sources",
    "point_source", "gauge_transform", "su3_directions", "random_spinors",
]


def volume(L):
    L = tuple(int(v) for v in L)
    if len(L) != 4:
        raise ValueError("lattice needs four extents")
    return L[0] * L[1] * L[2] * L[3]


def _expi_hermitian(Q, c):
    """exp(i c Q) for a stack of Hermitian 3x3 matrices via their eigendecomposition."""
    q, W = np.linalg.eigh(Q)
    ph = np.exp(1j * c * q)
    return np.einsum("...ab,...b,...cb->...ac", W, ph, W.conj())


def _traceless_hermitian(rng, shape):
    G = rng.standard_normal(shape + (2, 3, 3))
    Z = G[..., 0, :, :] + 1j * G[..., 1, :, :]
    H = 0.5 * (Z + np.conj(np.swapaxes(Z, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    return H - tr[..., None, None] * np.eye(3)


def gauge_field(L, c, seed):
    """SU(3) links U_mu(x) = exp(i c Q_mu(x)), Q traceless Hermitian with Gaussian entries.

    Draw order: one standard-normal array of shape (V, 4, 2, 3, 3) from PCG64(seed), sites in
    lexicographic order with mu the minor index, axis 2 = (real, imaginary).
    Returns complex128 (4, V, 3, 3).
    """
    V = volume(L)
    rng = np.random.default_rng(seed)
    Q = _traceless_hermitian(rng, (V, 4))
    U = _expi_hermitian(Q, float(c))
    return np.ascontiguousarray(np.transpose(U, (1, 0, 2, 3)))


def unit_field(L):
    V = volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def z2_sources(L, nrhs, seed):
    """Z2 noise: every complex entry is +1 or -1 (imaginary part 0). Shape (nrhs, V, 4, 3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    n = 12 * V
    out = np.empty((nrhs, V, 4, 3), dtype=np.complex128)
    for j in range(nrhs):
        out[j] = (2 * rng.integers(0, 2, n) - 1).astype(np.float64).reshape(V, 4, 3)
    return out


def gaussian_sources(L, nrhs, seed):
    """Complex Gaussian: real and imaginary parts each N(0, 1). Shape (nrhs, V, 4, 3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nrhs, V, 4, 3))
    im = rng.standard_normal((nrhs, V, 4, 3))
    return re + 1j * im


random_spinors = gaussian_sources


def point_source(L, site=0, spin=0, colour=0):
    """Unit point source; default site (0,0,0,0), spin 0, colour 0. Shape (1, V, 4, 3)."""
    V = volume(L)
    out = np.zeros((1, V, 4, 3), dtype=np.complex128)
    out[0, site, spin, colour] = 1.0
    return out


def gauge_transform(L, seed):
    """Random SU(3) matrix per site (same recipe as the links with c = pi). Shape (V, 3, 3)."""
    V = volume(L)
    rng = np.random.default_rng(seed)
    Q = _traceless_hermitian(rng, (V,))
    return _expi_hermitian(Q, np.pi)


def su3_directions(nd, seed):
    """Random su(3) directions: nd draws of (site-independent) coefficient vectors c in R^8,
    normalised to unit length, plus a site and direction index drawn from the same stream by
    the caller.  Returns float64 (nd, 8)."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((nd, 8))
    return c / np.linalg.norm(c, axis=1, keepdims=True)
