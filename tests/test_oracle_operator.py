"""Pins of the oracle's lattice geometry and Wilson operator against closed forms and exact
invariants (CPU only).

Each test would fail under a plausible mistake in ``oracle.wilson``: a dropped hop (free-field
spectrum), a wrong hop sign or projector (plane-wave symbol), a link on the wrong site
(gauge covariance), a missing dagger (gamma5-hermiticity), a wrong neighbour table
(translation covariance, bipartiteness).
"""
import numpy as np
import pytest

import synth
from oracle import wilson as W


def _rnd(L, seed, nrhs=None):
    s = synth.gaussian_sources(L, 1 if nrhs is None else nrhs, seed)
    return s[0] if nrhs is None else s


def test_clifford_algebra_and_gamma5():
    g, g5 = W.GAMMA, W.GAMMA5
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.array_equal(ac, 2.0 * (mu == nu) * np.eye(4))
    # chiral basis: gamma5 diagonal with chirality (+,+,-,-)
    assert np.array_equal(g5, np.diag([1, 1, -1, -1]).astype(complex))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 8), (2, 2, 2, 2)])
def test_geometry_tables(L):
    lat = W.Lattice(L)
    V = lat.V
    for mu in range(4):
        assert np.array_equal(lat.fwd[mu][lat.bwd[mu]], np.arange(V))
        # neighbours differ by one unit in direction mu only (periodic)
        d = (lat.coords[lat.fwd[mu]] - lat.coords) % np.array(L)
        e = np.zeros(4, dtype=int)
        e[mu] = 1 % L[mu]
        assert np.all(d == e)
    assert np.array_equal(np.sort(lat.eo_of_lex), np.arange(V))
    assert np.array_equal(lat.eo_of_lex[lat.lex_of_eo], np.arange(V))
    even = lat.parity == 0
    assert np.all(lat.eo_of_lex[even] < V // 2) and np.all(lat.eo_of_lex[~even] >= V // 2)
    # with all extents even, every neighbour of an even site is odd (bipartite lattice)
    if all(l % 2 == 0 for l in L) and min(L) > 2:
        for mu in range(4):
            assert np.all(lat.parity[lat.fwd[mu]] != lat.parity)


@pytest.mark.parametrize("L,T", [((8, 4, 4, 8), (4, 2, 2, 4)), ((24, 12, 4, 8), (8, 4, 4, 4)),
                                 ((6, 4, 2, 10), (2, 2, 2, 2)), ((6, 10, 4, 2), (6, 10, 4, 2))])
def test_blocked_even_odd_order(L, T):
    """The tiled even-odd storage order: a bijection that keeps the parity halves, fills each
    tile's half-range with exactly that tile's sites of that parity in in-tile lex order, and
    reduces to parity*V/2 + (lex >> 1) when one tile covers the lattice."""
    lat = W.Lattice(L, tile=T)
    V = lat.V
    h = int(np.prod(T)) // 2
    assert np.array_equal(np.sort(lat.eo_of_lex), np.arange(V))
    assert np.array_equal(lat.eo_of_lex[lat.lex_of_eo], np.arange(V))
    even = lat.parity == 0
    assert np.all(lat.eo_of_lex[even] < V // 2) and np.all(lat.eo_of_lex[~even] >= V // 2)
    # the sites stored in one tile's half-range: same parity, same tile, a box of extents T
    c = lat.coords[lat.lex_of_eo]
    for start in range(0, V, h):
        box = c[start:start + h]
        assert np.all(box // np.array(T) == box[0] // np.array(T))
        assert len(np.unique(lat.parity[lat.lex_of_eo[start:start + h]])) == 1
        lexs = lat.lex_of_eo[start:start + h]
        assert np.all(np.diff(lexs) > 0)  # in-tile lex order is lattice lex order within a box
    plain = W.Lattice(L)
    single = W.Lattice(L, tile=L)
    assert np.array_equal(single.eo_of_lex, plain.eo_of_lex)
    with pytest.raises(ValueError):
        W.Lattice(L, tile=(3, 2, 2, 2))


def _free_symbol(p, kappa):
    g = W.GAMMA
    return (np.eye(4) * (1 - 2 * kappa * np.cos(p).sum())
            + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4)))


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_free_field_dense_spectrum(L):
    """Unit links: lambda(p) = 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), each sign with
    multiplicity 6 (spin 2 x colour 3), p_mu = 2 pi n_mu / L_mu."""
    kappa = 0.11
    lat = W.Lattice(L)
    A = W.dense_matrix(synth.unit_field(L), lat, kappa)
    ev = np.linalg.eigvals(A)
    expect = []
    for n in np.ndindex(*L):
        p = 2 * np.pi * np.array(n) / np.array(L)
        a = 1 - 2 * kappa * np.cos(p).sum()
        s = 2 * kappa * np.sqrt((np.sin(p) ** 2).sum())
        expect += [a + 1j * s] * 6 + [a - 1j * s] * 6
    expect = np.array(expect)
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    assert np.allclose(ev[key(ev)], expect[key(expect)], atol=1e-13)


def test_free_field_plane_wave_symbol():
    """A (e^{ipx} chi) = e^{ipx} A(p) chi with A(p) = 1 - 2k sum cos p + 2ik sum gamma sin p,
    and the same with the twisted term and with the dagger."""
    L = (4, 6, 4, 8)
    lat = W.Lattice(L)
    U = synth.unit_field(L)
    rng = np.random.default_rng(7)
    kappa, mu = 0.13, 0.05
    for _ in range(4):
        n = rng.integers(0, 8, 4) % np.array(L)
        p = 2 * np.pi * n / np.array(L)
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * lat.coords @ p)
        psi = phase[:, None, None] * chi[None]
        Ap = _free_symbol(p, kappa) + 1j * mu * W.GAMMA5
        out = W.apply_A(U, psi, lat, kappa, mu)
        assert np.allclose(out, phase[:, None, None] * (Ap @ chi)[None], atol=1e-13)
        outd = W.apply_A(U, psi, lat, kappa, mu, dagger=True)
        assert np.allclose(outd, phase[:, None, None] * (Ap.conj().T @ chi)[None], atol=1e-13)


def _g5(psi):
    return np.einsum("st,xta->xsa", W.GAMMA5, psi)


@pytest.mark.parametrize("mu", [0.0, 0.07])
def test_gamma5_hermiticity_and_dagger(mu):
    L = (4, 4, 4, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 11)
    phi, psi = _rnd(L, 1), _rnd(L, 2)
    k = 0.137
    # <phi, A psi> = <A^dagger phi, psi>
    lhs = np.vdot(phi, W.apply_A(U, psi, lat, k, mu))
    rhs = np.vdot(W.apply_A(U, phi, lat, k, mu, dagger=True), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # A(mu)^dagger = gamma5 A(-mu) gamma5, checked through inner products
    g = np.vdot(phi, _g5(W.apply_A(U, _g5(psi), lat, k, -mu)))
    d = np.vdot(phi, W.apply_A(U, psi, lat, k, mu, dagger=True))
    assert abs(g - d) <= 1e-13 * abs(g)
    # ... while A itself is not Hermitian, so the dagger is not a no-op
    assert abs(np.vdot(phi, W.apply_A(U, psi, lat, k, mu)) - g) > 1e-6 * abs(g)


def test_gauge_covariance():
    L = (4, 4, 2, 6)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 12)
    G = synth.gauge_transform(L, 13)
    UG = np.einsum("xab,mxbc,mxdc->mxad", G, U, np.conj(G[lat.fwd]))
    psi = _rnd(L, 3)
    Gpsi = np.einsum("xab,xsb->xsa", G, psi)
    lhs = W.apply_A(UG, Gpsi, lat, 0.12, 0.03)
    rhs = np.einsum("xab,xsb->xsa", G, W.apply_A(U, psi, lat, 0.12, 0.03))
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_translation_covariance():
    L = (4, 4, 4, 6)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 14)
    psi = _rnd(L, 4)
    shift = np.array([1, 3, 2, 5])
    dst = lat.lex((lat.coords + shift) % np.array(L))
    Us = np.empty_like(U)
    Us[:, dst] = U
    ps = np.empty_like(psi)
    ps[dst] = psi
    out = W.apply_A(U, psi, lat, 0.12)
    outs = W.apply_A(Us, ps, lat, 0.12)
    assert np.allclose(outs[dst], out, atol=1e-14, rtol=0)


def test_bipartite_and_norm_bound():
    L = (4, 4, 4, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 15)
    psi = _rnd(L, 5)
    eps = (1 - 2 * lat.parity)[:, None, None]
    H = W.hopping(U, psi, lat)
    assert np.allclose(eps * W.hopping(U, eps * psi, lat), -H, atol=1e-14, rtol=0)
    assert np.linalg.norm(H) <= 8 * np.linalg.norm(psi)


def test_twisted_mass_norm_identity():
    """||A(mu) psi||^2 = ||A(0) psi||^2 + mu^2 ||psi||^2 because gamma5 A(0) is Hermitian."""
    L = (4, 4, 4, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 16)
    psi = _rnd(L, 6)
    mu = 0.173
    a = np.linalg.norm(W.apply_A(U, psi, lat, 0.13, mu)) ** 2
    b = np.linalg.norm(W.apply_A(U, psi, lat, 0.13, 0.0)) ** 2 + mu ** 2 * np.linalg.norm(psi) ** 2
    assert abs(a - b) <= 1e-13 * b


def test_left_eigenvectors_are_gamma5_right():
    """gamma5 v is an eigenvector of A^dagger for the same eigenvalue (so a left eigenvector of
    A for its conjugate); the spectrum is closed under conjugation."""
    L = (2, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 17)
    A = W.dense_matrix(U, lat, 0.15)
    ev, R = np.linalg.eig(A)
    G5 = np.kron(np.eye(lat.V), np.kron(W.GAMMA5, np.eye(3)))
    for j in range(0, 192, 17):
        v = G5 @ R[:, j]
        assert np.linalg.norm(A.conj().T @ v - ev[j] * v) <= 1e-12 * np.linalg.norm(v)
        assert np.min(np.abs(ev - np.conj(ev[j]))) <= 1e-12


def test_sampled_apply_matches_full():
    L = (4, 2, 4, 6)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 18)
    psi = _rnd(L, 7)
    full = W.apply_A(U, psi, lat, 0.12, 0.02, dagger=True)
    sites = np.array([0, 5, 17, lat.V - 1])
    part = W.apply_A_sites(U, psi, lat, 0.12, sites, 0.02, dagger=True)
    assert np.array_equal(part, full[sites])


def test_generator_links_are_su3():
    U = synth.gauge_field((4, 2, 2, 2), 0.6, 19)
    eye = np.einsum("mxab,mxcb->mxac", U, np.conj(U))
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # third row = conj(row0 x row1): the identity 12-real link storage relies on
    r2 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.abs(r2 - U[..., 2, :]).max() < 1e-14
