"""Pins of the oracle's even-odd reduced system (``oracle.evenodd``) against the full operator,
closed forms and dense linear algebra (CPU only).

Each test would fail under a plausible mistake in the Schur complement: a wrong sign or power of
kappa, D in place of D^{-1} (or a dropped 1/(1+mu^2)), the twisted term's sign in the adjoint,
a parity mix-up in the half vectors, a wrong source (bhat) or reconstruction (x_o).
"""
import numpy as np
import pytest

import synth
from oracle import evenodd as EO
from oracle import solvers as S
from oracle import wilson as W


def _field(L, seed):
    return synth.gauge_field(L, 0.5, seed)


def _gauss(L, seed):
    return synth.gaussian_sources(L, 1, seed)[0]


def _dinv(mu):
    """(I - i mu gamma5) / (1 + mu^2) as a 4x4 spin matrix, written out from gamma5."""
    return (np.eye(4) - 1j * mu * W.GAMMA5) / (1.0 + mu * mu)


@pytest.mark.parametrize("L", [(4, 4, 2, 2), (2, 4, 4, 6)])
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_complement_is_the_even_block_of_the_full_operator(L, mu, dagger):
    """With x_o = kappa D^{-1} H_oe x_e (the odd rows of A x = 0), A x is Ahat x_e on the even
    sites and zero on the odd ones; built here from the full operator and the parity mask only."""
    lat = W.Lattice(L)
    U = _field(L, 11)
    kappa = 0.13
    m = -mu if dagger else mu
    even = lat.parity == 0
    xe = _gauss(L, 12)[even]                                   # (V/2, 4, 3), lex order
    xf = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    xf[even] = xe
    h = W.hopping(U, xf, lat, dagger)
    xf[~even] = kappa * np.einsum("st,xta->xsa", _dinv(m), h[~even])
    ax = W.apply_A(U, xf, lat, kappa, mu, dagger)
    assert np.max(np.abs(ax[~even])) < 1e-13 * np.max(np.abs(ax[even]))
    got = EO.schur_apply(U, lat, kappa, xe.reshape(-1), mu, dagger).reshape(-1, 4, 3)
    assert np.allclose(got, ax[even], rtol=0, atol=1e-13 * np.max(np.abs(ax)))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 2, 4, 8)])
@pytest.mark.parametrize("mu,dagger", [(0.0, False), (0.25, False), (0.25, True)])
def test_free_field_plane_wave_symbol(L, mu, dagger):
    """Unit links: an even-site plane wave e^{ipx} chi is mapped to e^{ipx} Ahat(p) chi with
    Ahat(p) = D - kappa^2 H(p) D^{-1} H(p), H(p) = sum_mu [(1-gamma_mu) e^{ip_mu} +
    (1+gamma_mu) e^{-ip_mu}] (dagger: the projectors swap and mu -> -mu)."""
    lat = W.Lattice(L)
    U = synth.unit_field(L)
    kappa = 0.11
    rng = np.random.default_rng(5)
    even = lat.parity == 0
    m = -mu if dagger else mu
    for _ in range(3):
        n = rng.integers(0, np.array(L))
        p = 2 * np.pi * n / np.array(L)
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        ph = np.exp(1j * (lat.coords @ p))
        psi_e = (ph[:, None, None] * chi[None])[even]
        Hp = np.zeros((4, 4), dtype=np.complex128)
        for mu_ in range(4):
            f, b = np.eye(4) - W.GAMMA[mu_], np.eye(4) + W.GAMMA[mu_]
            if dagger:
                f, b = b, f
            Hp += f * np.exp(1j * p[mu_]) + b * np.exp(-1j * p[mu_])
        D = np.eye(4) + 1j * m * W.GAMMA5
        sym = D - kappa * kappa * Hp @ _dinv(m) @ Hp
        want = ph[even][:, None, None] * (sym @ chi)[None]
        got = EO.schur_apply(U, lat, kappa, psi_e.reshape(-1), mu, dagger).reshape(-1, 4, 3)
        assert np.allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mu,dagger", [(0.0, False), (0.2, False), (0.2, True)])
def test_dense_solve_through_the_schur_complement(mu, dagger):
    """x from Ahat x_e = bhat and the reconstruction equals the dense solution of A x = b."""
    L = (2, 2, 2, 4)
    lat = W.Lattice(L)
    U = _field(L, 21)
    kappa = 0.12
    b = _gauss(L, 22)
    Ad = W.dense_matrix(U, lat, kappa, mu, dagger)
    x_ref = np.linalg.solve(Ad, b.reshape(-1))
    nh = lat.n // 2
    Sd = np.empty((nh, nh), dtype=np.complex128)
    e = np.zeros(nh, dtype=np.complex128)
    for j in range(nh):
        e[j] = 1.0
        Sd[:, j] = EO.schur_apply(U, lat, kappa, e, mu, dagger)
        e[j] = 0.0
    xe = np.linalg.solve(Sd, EO.schur_source(U, lat, kappa, b, mu, dagger))
    x = EO.schur_reconstruct(U, lat, kappa, xe, b, mu, dagger).reshape(-1)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    # and the full residual of the reconstructed solution
    r = b.reshape(-1) - W.apply_A(U, x, lat, kappa, mu, dagger)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("mu", [0.0, 0.15])
def test_gamma5_hermiticity(mu):
    """Ahat(mu)^dagger = gamma5 Ahat(-mu) gamma5, and <phi, Ahat^dagger psi> = <Ahat phi, psi>."""
    L = (4, 2, 2, 4)
    lat = W.Lattice(L)
    U = _field(L, 31)
    kappa = 0.14
    even = lat.parity == 0
    phi = _gauss(L, 32)[even].reshape(-1)
    psi = _gauss(L, 33)[even].reshape(-1)
    ad = EO.schur_apply(U, lat, kappa, psi, mu, dagger=True)
    g5 = EO.gamma5_half
    assert np.allclose(ad, g5(EO.schur_apply(U, lat, kappa, g5(psi), -mu)), rtol=0, atol=1e-13)
    lhs = np.vdot(phi, ad)
    rhs = np.vdot(EO.schur_apply(U, lat, kappa, phi, mu), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_deflated_solve_of_the_reduced_system_solves_the_full_one():
    """GMRES-DR on Ahat, then D-BiCGStab on Ahat with gamma5 V as left vectors: the reconstructed
    x meets the tolerance on the full system (odd rows are exact by construction)."""
    L = (4, 4, 4, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 101)
    kappa, mu = 0.15, 0.0
    A = EO.schur_operator(U, lat, kappa, mu)
    b1 = synth.point_source(L)[0]
    x1, V, th, info = S.gmresdr(A, EO.schur_source(U, lat, kappa, b1), 20, 6, tol=1e-10)
    assert info["status"] == S.OK
    assert np.allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-12)
    b = synth.z2_sources(L, 1, 1101)[0]
    bh = EO.schur_source(U, lat, kappa, b)
    xe, inf2 = S.dbicgstab(A, bh, V, EO.gamma5_half, tol=1e-10)
    assert inf2["status"] == S.OK
    x = EO.schur_reconstruct(U, lat, kappa, xe, b).reshape(-1)
    r = b.reshape(-1) - W.apply_A(U, x, lat, kappa)
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(bh)


def test_sampled_sites_equal_the_whole_field():
    """The one-site-at-a-time Schur apply (for full-size GPU checks) agrees with the pinned
    whole-field one."""
    L = (4, 4, 2, 6)
    lat = W.Lattice(L)
    U = _field(L, 41)
    xe = _gauss(L, 42)[lat.parity == 0].reshape(-1)
    ev = np.nonzero(lat.parity == 0)[0]
    pick = np.array([0, 5, 17, 40, len(ev) - 1])
    for mu, dagger in [(0.0, False), (0.2, True)]:
        whole = EO.schur_apply(U, lat, 0.13, xe, mu, dagger).reshape(-1, 4, 3)
        got = EO.schur_apply_sites(U, lat, 0.13, xe, ev[pick], mu, dagger)
        assert np.array_equal(got, whole[pick])
