"""Oracle: lattice geometry and the Wilson / twisted-mass Wilson matrix, plain NumPy FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Operator (Sec. 1: the Wilson matrix A_W with gamma5 A_W gamma5 = A_W^dagger; Sec. 3: kappa
near kappa_c; Sec. 4, action equation: twisted mass term i*mu*gamma5):

    (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]
    A(mu)      = I - kappa*H + i*mu*gamma5
    A(mu)^dagger = gamma5 A(-mu) gamma5

Readings where the paper is silent: chiral (DeGrand-Rossi) gamma basis, (1 - gamma) on the
forward hop, periodic boundaries in all four directions, the twisted term added literally as
i*mu*gamma5 to I - kappa*H, and the full (not even-odd reduced) operator.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------- gamma matrices
def gamma_matrices():
    """Chiral (DeGrand-Rossi) basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1, 2, 3
    (directions x, y, z), gamma_4 = [[0, 1], [1, 0]] (direction t), gamma5 = g1 g2 g3 g4.
    Returns (list of four 4x4 matrices indexed by mu = 0..3, gamma5)."""
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    Z = np.zeros((2, 2), dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    gam = [np.block([[Z, -1j * s], [1j * s, Z]]) for s in (s1, s2, s3)]
    gam.append(np.block([[Z, I2], [I2, Z]]))
    g5 = gam[0] @ gam[1] @ gam[2] @ gam[3]
    return gam, g5


GAMMA, GAMMA5 = gamma_matrices()
I4 = np.eye(4, dtype=np.complex128)


# --------------------------------------------------------------------------- geometry
class Lattice:
    """Periodic 4-d lattice with lexicographic sites lex = x + Lx*(y + Ly*(z + Lz*t)).

    Tables (int64 here; the HIP side produces int32 and the tests compare values):

    * ``coords[lex]``     -- (x, y, z, t)
    * ``fwd[mu][lex]``    -- lex index of x + mu (periodic)
    * ``bwd[mu][lex]``    -- lex index of x - mu
    * ``parity[lex]``     -- (x + y + z + t) mod 2
    * ``eo_of_lex[lex]``  -- even-odd index parity*V/2 + (lex >> 1)   (a bijection for even Lx)
    * ``lex_of_eo[eo]``   -- the inverse permutation

    With ``tile`` = (T0, T1, T2, T3) (each even and dividing the extent) the even-odd order is
    blocked into tiles: eo = parity*V/2 + tile_index*(T0*T1*T2*T3/2) + (in_tile_lex >> 1), where
    tile_index is the lexicographic index of (x//T0, y//T1, z//T2, t//T3) over the tile grid and
    in_tile_lex that of (x%T0, y%T1, z%T2, t%T3) inside the tile.  One tile covering the whole
    lattice gives the plain order.  (A storage order only: the operator does not depend on it.)
    """

    def __init__(self, L, tile=None):
        L = tuple(int(v) for v in L)
        if len(L) != 4 or any(v < 1 for v in L):
            raise ValueError("need four positive extents")
        if tile is not None:
            tile = tuple(int(v) for v in tile)
            if len(tile) != 4 or any(t < 2 or t % 2 or l % t for t, l in zip(tile, L)):
                raise ValueError("tile extents must be even and divide the lattice extents")
        self.L = L
        self.tile = tile
        self.V = L[0] * L[1] * L[2] * L[3]
        lex = np.arange(self.V)
        x = lex % L[0]
        y = (lex // L[0]) % L[1]
        z = (lex // (L[0] * L[1])) % L[2]
        t = lex // (L[0] * L[1] * L[2])
        self.coords = np.stack([x, y, z, t], axis=1)
        self.fwd = np.empty((4, self.V), dtype=np.int64)
        self.bwd = np.empty((4, self.V), dtype=np.int64)
        for mu in range(4):
            cp = self.coords.copy()
            cp[:, mu] = (cp[:, mu] + 1) % L[mu]
            self.fwd[mu] = self.lex(cp)
            cm = self.coords.copy()
            cm[:, mu] = (cm[:, mu] - 1) % L[mu]
            self.bwd[mu] = self.lex(cm)
        self.parity = self.coords.sum(axis=1) % 2
        if tile is not None:
            T = np.array(tile)
            NT = np.array(L) // T
            tc = self.coords // T
            ic = self.coords % T
            tile_index = tc[:, 0] + NT[0] * (tc[:, 1] + NT[1] * (tc[:, 2] + NT[2] * tc[:, 3]))
            in_tile_lex = ic[:, 0] + T[0] * (ic[:, 1] + T[1] * (ic[:, 2] + T[2] * ic[:, 3]))
            half = int(np.prod(T)) // 2
            self.eo_of_lex = self.parity * (self.V // 2) + tile_index * half + (in_tile_lex >> 1)
            self.lex_of_eo = np.empty(self.V, dtype=np.int64)
            self.lex_of_eo[self.eo_of_lex] = lex
        elif L[0] % 2 == 0:
            self.eo_of_lex = self.parity * (self.V // 2) + (lex >> 1)
            self.lex_of_eo = np.empty(self.V, dtype=np.int64)
            self.lex_of_eo[self.eo_of_lex] = lex
        else:
            self.eo_of_lex = self.lex_of_eo = None

    def lex(self, c):
        L = self.L
        return c[:, 0] + L[0] * (c[:, 1] + L[1] * (c[:, 2] + L[2] * c[:, 3]))

    @property
    def n(self):
        return 12 * self.V


# --------------------------------------------------------------------------- operator
def _as_sites(psi, V):
    return np.asarray(psi, dtype=np.complex128).reshape(V, 4, 3)


def hopping(U, psi, lat, dagger=False):
    """(H psi)(x) with full 4x4 spin projectors.  ``dagger`` applies H^dagger, which swaps the
    spin projectors of the two hops (gamma_mu Hermitian).  psi: any shape reshapeable to (V,4,3);
    returns (V,4,3)."""
    V = lat.V
    p = _as_sites(psi, V)
    out = np.zeros((V, 4, 3), dtype=np.complex128)
    for mu in range(4):
        Pf = I4 - GAMMA[mu]
        Pb = I4 + GAMMA[mu]
        if dagger:
            Pf, Pb = Pb, Pf
        # forward hop: U_mu(x) psi(x + mu)
        t = np.einsum("xab,xsb->xsa", U[mu], p[lat.fwd[mu]])
        out += np.einsum("st,xta->xsa", Pf, t)
        # backward hop: U_mu(x - mu)^dagger psi(x - mu)
        Ub = U[mu][lat.bwd[mu]]
        t = np.einsum("xba,xsb->xsa", np.conj(Ub), p[lat.bwd[mu]])
        out += np.einsum("st,xta->xsa", Pb, t)
    return out


def gamma5(psi, V):
    return np.einsum("st,xta->xsa", GAMMA5, _as_sites(psi, V))


def apply_A(U, psi, lat, kappa, mu=0.0, dagger=False):
    """A(mu) psi = psi - kappa H psi + i mu gamma5 psi; with ``dagger`` A(mu)^dagger psi
    = psi - kappa H^dagger psi - i mu gamma5 psi.  Returns the same shape as psi (flattened
    per right-hand side if psi is 1-d)."""
    V = lat.V
    shape = np.shape(psi)
    p = _as_sites(psi, V)
    m = -mu if dagger else mu
    out = p - kappa * hopping(U, p, lat, dagger) + 1j * m * gamma5(p, V)
    return out.reshape(shape)


def apply_A_multi(U, psis, lat, kappa, mu=0.0, dagger=False):
    """Apply to a stack of right-hand sides, shape (nrhs, V, 4, 3)."""
    return np.stack([apply_A(U, p, lat, kappa, mu, dagger) for p in psis])


def operator(U, lat, kappa, mu=0.0, dagger=False):
    """Closure x -> A x on flat complex vectors of length 12 V."""
    def A(x):
        return apply_A(U, x.reshape(lat.V, 4, 3), lat, kappa, mu, dagger).reshape(-1)
    return A


def dense_matrix(U, lat, kappa, mu=0.0, dagger=False):
    """Dense n x n matrix by applying A to unit vectors (tiny lattices only)."""
    n = lat.n
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = apply_A(U, e, lat, kappa, mu, dagger)
        e[j] = 0.0
    return M


def dense_hopping(U, lat):
    n = lat.n
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = hopping(U, e, lat).reshape(-1)
        e[j] = 0.0
    return M


def gamma5_flat(x, V):
    return gamma5(x.reshape(V, 4, 3), V).reshape(-1)


# --------------------------------------------------------------------------- sampled apply
def hopping_sites(U, psi, lat, sites, dagger=False):
    """(H psi)(x) (``dagger``: H^dagger) at a list of lexicographic sites only.
    Returns (len(sites), 4, 3)."""
    p = _as_sites(psi, lat.V)
    sites = np.asarray(sites, dtype=np.int64)
    acc = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for mu_ in range(4):
        Pf = I4 - GAMMA[mu_]
        Pb = I4 + GAMMA[mu_]
        if dagger:
            Pf, Pb = Pb, Pf
        f = lat.fwd[mu_][sites]
        b = lat.bwd[mu_][sites]
        t = np.einsum("xab,xsb->xsa", U[mu_][sites], p[f])
        acc += np.einsum("st,xta->xsa", Pf, t)
        t = np.einsum("xba,xsb->xsa", np.conj(U[mu_][b]), p[b])
        acc += np.einsum("st,xta->xsa", Pb, t)
    return acc


def apply_A_sites(U, psi, lat, kappa, sites, mu=0.0, dagger=False):
    """(A psi)(x) at a list of lexicographic sites only: lets large-lattice GPU outputs be
    checked one site at a time.  Returns (len(sites), 4, 3)."""
    p = _as_sites(psi, lat.V)
    sites = np.asarray(sites, dtype=np.int64)
    acc = hopping_sites(U, p, lat, sites, dagger)
    m = -mu if dagger else mu
    ps = p[sites]
    return ps - kappa * acc + 1j * m * np.einsum("st,xta->xsa", GAMMA5, ps)
