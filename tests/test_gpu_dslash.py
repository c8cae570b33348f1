"""GPU parity of the geometry tables and the Wilson / twisted-mass operator apply against the
oracle, element by element, plus invariants checked on the GPU's own output."""
import numpy as np
import pytest

import synth
from oracle import wilson as W
from gpuhelp import dev, host, relerr

pytestmark = pytest.mark.gpu

# sizes spanning several 256-site tiles with a ragged last tile, and the 2^4 degenerate case
LATS = [(4, 4, 4, 4), (6, 4, 2, 10), (2, 2, 2, 2), (8, 6, 4, 6)]


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 10), (24, 24, 24, 48)])
def test_geometry_tables_bit_exact(gpu_lib, L):
    lex, nbr = gpu_lib.geometry(L)
    lat = W.Lattice(L, tile=gpu_lib.site_tile(L))
    assert np.array_equal(host(lex), lat.lex_of_eo)
    nb = host(nbr)
    k = 0
    for mu in range(4):
        for tab in (lat.fwd[mu], lat.bwd[mu]):
            assert np.array_equal(nb[k], lat.eo_of_lex[tab[lat.lex_of_eo]])
            k += 1


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("mu", [0.0, 0.037])
def test_apply_fp64_matches_oracle(gpu_lib, L, dagger, mu):
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 201)
    psi = synth.gaussian_sources(L, 3, 202)
    kappa = 0.1337
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), kappa, mu, dagger, "fp64"))
    ref = W.apply_A_multi(U, psi, lat, kappa, mu, dagger)
    assert relerr(out, ref) <= 1e-14


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_fp32_matches_oracle(gpu_lib, L, dagger):
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 203)
    psi = synth.gaussian_sources(L, 2, 204)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.125, 0.02, dagger, "mixed"))
    ref = W.apply_A_multi(U, psi, lat, 0.125, 0.02, dagger)
    # FP32 arithmetic with 12-real links: a few ulps of float per term
    assert relerr(out, ref) <= 2e-6


@pytest.mark.parametrize("L", LATS + [(8, 8, 4, 12), (16, 8, 12, 8)])
@pytest.mark.parametrize("shape", [("0", "1"), ("0", "2"), ("0", "0"), ("1", "1"), ("1", "0"),
                                   ("2", "1"), ("4", "0"), ("0", "1", "1"), ("0", "0", "1"),
                                   ("0", "2", "2"), ("0", "1", "2"), ("0", "1", "0", "1"),
                                   ("0", "1", "3"), ("0", "0", "3")])
def test_every_fp32_launch_shape_matches_oracle(gpu_lib, monkeypatch, L, shape):
    """Each FP32 launch shape: rhs per thread 1/2/4 with rhs grouping, and the LDS-staged tile
    kernel (nb 0) with 1, 2 or all rhs per block in each tile order (lexicographic; eight x/y/z
    regions; regions with rhs chunks outermost; eight z/t regions); 5 rhs leave a ragged last chunk, and the tile
    grids include odd and unit tile counts, whose regions are uneven or empty, and tiles smaller
    than 4^4."""
    monkeypatch.setenv("DBQ_DS_NB", shape[0])
    monkeypatch.setenv("DBQ_DS_RG", shape[1])
    if len(shape) > 2:
        monkeypatch.setenv("DBQ_TILE_ORDER", shape[2])
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 208)
    psi = synth.gaussian_sources(L, 5, 209)
    for dagger, mu in ((False, 0.0), (True, 0.031)):
        out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.127, mu, dagger, "mixed"))
        ref = W.apply_A_multi(U, psi, lat, 0.127, mu, dagger)
        assert relerr(out, ref) <= 2e-6


def test_gpu_output_is_gamma5_hermitian_and_gauge_covariant(gpu_lib):
    L = (4, 4, 4, 6)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 205)
    phi, psi = synth.gaussian_sources(L, 2, 206)
    k, mu = 0.14, 0.03
    Ad_phi = host(gpu_lib.wilson_apply(L, dev(U), dev(phi), k, mu, True))
    A_psi = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), k, mu, False))
    a, b = np.vdot(phi, A_psi), np.vdot(Ad_phi, psi)
    assert abs(a - b) <= 1e-13 * abs(a)
    G = synth.gauge_transform(L, 207)
    UG = np.einsum("xab,mxbc,mxdc->mxad", G, U, np.conj(G[lat.fwd]))
    Gpsi = np.einsum("xab,xsb->xsa", G, psi)
    lhs = host(gpu_lib.wilson_apply(L, dev(UG), dev(Gpsi), k, mu))
    rhs = np.einsum("xab,xsb->xsa", G, A_psi)
    assert relerr(lhs, rhs) <= 1e-13


def test_free_field_plane_wave_on_gpu(gpu_lib):
    L = (8, 4, 6, 4)
    lat = W.Lattice(L)
    U = synth.unit_field(L)
    p = 2 * np.pi * np.array([3, 1, 2, 3]) / np.array(L)
    chi = np.arange(12).reshape(4, 3) * (0.3 - 0.1j) + 1.0
    ph = np.exp(1j * lat.coords @ p)
    psi = ph[:, None, None] * chi[None]
    k = 0.11
    Ap = (np.eye(4) * (1 - 2 * k * np.cos(p).sum())
          + 2j * k * sum(W.GAMMA[m] * np.sin(p[m]) for m in range(4)))
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), k))
    assert relerr(out, ph[:, None, None] * (Ap @ chi)[None]) <= 1e-14


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("mixed", 2e-6)])
def test_full_size_24x48_sampled_sites(gpu_lib, prec, tol):
    """24^3 x 48 (the twisted-mass lattice): every site computed on the GPU, 512 sampled sites
    recomputed by the oracle one by one."""
    L = (24, 24, 24, 48)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 105)
    psi = synth.z2_sources(L, 1, 1105)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.13, 0.005, False, prec))[0]
    sites = np.random.default_rng(5).choice(lat.V, 512, replace=False)
    ref = W.apply_A_sites(U, psi[0], lat, 0.13, sites, 0.005)
    assert relerr(out[sites], ref) <= tol


@pytest.mark.parametrize("dagger", [False, True])
def test_full_size_16x16x16x16_batch_of_12_sampled_sites(gpu_lib, dagger):
    """The benchmark's operator launch: 16^4, 12 Z2 sources in one FP32 call in the tuned launch
    shape; 256 sampled sites of every source recomputed by the oracle."""
    L = (16, 16, 16, 16)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 102)
    psi = synth.z2_sources(L, 12, 1102)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.2074870, 0.0, dagger, "mixed"))
    sites = np.random.default_rng(6).choice(lat.V, 256, replace=False)
    for j in range(12):
        ref = W.apply_A_sites(U, psi[j], lat, 0.2074870, sites, 0.0, dagger)
        assert relerr(out[j][sites], ref) <= 2e-6


_BIG = {}


def _big_batch():
    """24^3 x 48 field and 12 Z2 sources (host and device), built once for the module."""
    if not _BIG:
        L = (24, 24, 24, 48)
        U = synth.gauge_field(L, 0.6, 105)
        psi = synth.z2_sources(L, 12, 1105)
        _BIG.update(L=L, lat=W.Lattice(L), U=U, psi=psi, Ud=dev(U), psid=dev(psi))
    return _BIG


@pytest.mark.parametrize("order", [None, "0", "1", "2", "3"])
def test_full_size_24x48_batch_of_12_sampled_sites(gpu_lib, monkeypatch, order):
    """The HBM-sized operator launch: 24^3 x 48 with 12 Z2 sources in one FP32 call, in the tuned
    launch shape (None) and as the LDS tile kernel with 4 rhs per block in each tile order; 128
    sampled sites of every source recomputed by the oracle one by one."""
    if order is not None:
        monkeypatch.setenv("DBQ_DS_NB", "0")
        monkeypatch.setenv("DBQ_DS_RG", "4")
        monkeypatch.setenv("DBQ_TILE_ORDER", order)
    d = _big_batch()
    out = gpu_lib.wilson_apply(d["L"], d["Ud"], d["psid"], 0.13, 0.005, False, "mixed")
    sites = np.random.default_rng(11).choice(d["lat"].V, 128, replace=False)
    got = host(out[:, sites])
    del out
    for j in range(12):
        ref = W.apply_A_sites(d["U"], d["psi"][j], d["lat"], 0.13, sites, 0.005)
        assert relerr(got[j], ref) <= 2e-6, j


def test_rejects_bad_shapes_before_launch(gpu_lib):
    import torch
    L = (4, 4, 4, 4)
    U = dev(synth.unit_field(L))
    with pytest.raises(ValueError):
        gpu_lib.wilson_apply(L, U, torch.zeros(100, dtype=torch.complex128, device="cuda"), 0.1)
    with pytest.raises(ValueError):
        gpu_lib.wilson_apply((4, 4, 4, 6), U, dev(synth.z2_sources((4, 4, 4, 6), 1, 1)), 0.1)
