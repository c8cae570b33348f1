"""GPU parity of the even-odd reduced system (Schur complement on the even sites): the operator
apply (FP64, FP32, dagger, twisted mass, batches), GMRES-DR and D-BiCGStab on it (FP64, mixed,
batched, uneven, adjoint), the shift projection, against ``oracle.evenodd``."""
import numpy as np
import pytest

import synth
from oracle import evenodd as EO
from oracle import solvers as S
from oracle import wilson as W
from gpuhelp import dev, host, projector_distance, relerr, same_eigenvalues

pytestmark = pytest.mark.gpu

LATS = [(4, 4, 4, 4), (6, 4, 2, 8), (8, 8, 4, 12), (2, 4, 6, 4)]


def _even(lat, v):
    return np.asarray(v).reshape(lat.V, 4, 3)[lat.parity == 0].reshape(-1)


def _odd(lat, v):
    return np.asarray(v).reshape(lat.V, 4, 3)[lat.parity == 1]


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("mu,dagger", [(0.0, False), (0.2, False), (0.2, True)])
def test_schur_apply_fp64_matches_oracle(gpu_lib, L, mu, dagger):
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 7)
    psi = synth.gaussian_sources(L, 3, 8)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.13, mu, dagger, "fp64", schur=True))
    for j in range(3):
        want = EO.schur_apply(U, lat, 0.13, _even(lat, psi[j]), mu, dagger)
        assert relerr(_even(lat, out[j]), want) <= 1e-13
        assert np.all(_odd(lat, out[j]) == 0)


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("nrhs", [1, 5])
def test_schur_apply_fp32_matches_oracle(gpu_lib, L, nrhs):
    """FP32 with 12-real links: two hops in single precision, rounding ~1e-7 relative."""
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 17)
    psi = synth.gaussian_sources(L, nrhs, 18)
    for dagger in (False, True):
        out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.13, 0.05, dagger, "mixed",
                                        schur=True))
        for j in range(nrhs):
            want = EO.schur_apply(U, lat, 0.13, _even(lat, psi[j]), 0.05, dagger)
            assert relerr(_even(lat, out[j]), want) <= 2e-6
            assert np.all(_odd(lat, out[j]) == 0)


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("shape", [("0", "1"), ("0", "2"), ("0", "0"), ("1", "1"), ("1", "0"),
                                   ("2", "0"), ("2", "2"), ("0", "1", "1"), ("0", "0", "1"),
                                   ("0", "2", "2"), ("0", "1", "3")])
def test_every_schur_fp32_launch_shape_matches_oracle(gpu_lib, monkeypatch, L, shape):
    """Each FP32 launch shape of the half-lattice kernels: the LDS-staged tile kernel (nb 0) with
    1, 2 or all rhs per block in each tile order, and 1 or 2 rhs per thread; 5 rhs leave a
    ragged last chunk."""
    monkeypatch.setenv("DBQ_DS_NB", shape[0])
    monkeypatch.setenv("DBQ_DS_RG", shape[1])
    if len(shape) > 2:
        monkeypatch.setenv("DBQ_TILE_ORDER", shape[2])
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 218)
    psi = synth.gaussian_sources(L, 5, 219)
    for dagger, mu in ((False, 0.0), (True, 0.031)):
        out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.127, mu, dagger, "mixed",
                                        schur=True))
        for j in range(5):
            want = EO.schur_apply(U, lat, 0.127, _even(lat, psi[j]), mu, dagger)
            assert relerr(_even(lat, out[j]), want) <= 2e-6
            assert np.all(_odd(lat, out[j]) == 0)


def test_schur_apply_full_size_16x16x16x16_batch_of_12_sampled_sites(gpu_lib):
    """16^4, 12 Z2 sources in one FP32 launch pair (the benchmark's shape), checked at 64 sampled
    even sites per source against the oracle's one-site apply."""
    L = (16, 16, 16, 16)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 102)
    psi = synth.z2_sources(L, 12, 1102)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.2075, 0.0, False, "mixed",
                                    schur=True)).reshape(12, lat.V, 4, 3)
    ev = np.nonzero(lat.parity == 0)[0]
    rng = np.random.default_rng(3)
    for j in (0, 5, 11):
        pick = np.sort(rng.choice(ev, 64, replace=False))
        pick[0] = ev[0]
        pick[-1] = ev[-1]
        xe = _even(lat, psi[j])
        want = EO.schur_apply_sites(U, lat, 0.2075, xe, pick)
        assert relerr(out[j][pick], want) <= 2e-6


# ----------------------------------------------------------------------------- solvers
C = dict(L=(4, 4, 4, 4), c=0.6, seed=101, kappa=0.15)


def _setup(L=C["L"], c=C["c"], seed=C["seed"]):
    lat = W.Lattice(L)
    U = synth.gauge_field(L, c, seed)
    return lat, U


def _true_rel(U, lat, kappa, mu, x, b, dagger=False):
    r = b.reshape(-1) - W.apply_A(U, x.reshape(-1), lat, kappa, mu, dagger)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_schur_gmresdr_matches_oracle(gpu_lib):
    """GMRES-DR(20,6) on Ahat from the point source: full solution to the tolerance, the oracle's
    cycle count, harmonic Ritz values of Ahat and the same deflation space; V zero on odd sites."""
    L = C["L"]
    lat, U = _setup()
    kappa = C["kappa"]
    b = synth.point_source(L)
    x, V, th, st = gpu_lib.gmresdr_first_rhs(L, dev(U), dev(b), kappa, 20, 6, tol=1e-10,
                                             schur=True)
    A = EO.schur_operator(U, lat, kappa)
    bh = EO.schur_source(U, lat, kappa, b[0])
    nb = np.linalg.norm(b)
    xo, Vo, tho, io = S.gmresdr(A, bh, 20, 6, tol=1e-10 * nb / np.linalg.norm(bh))
    assert st["status"] == 0 and io["status"] == 0
    assert st["matvecs"] == 20 + 14 * (st["iterations"] - 1)
    assert abs(st["iterations"] - io["cycles"]) <= 1
    assert _true_rel(U, lat, kappa, 0.0, host(x), b) <= 1.0001e-10
    assert st["rel_true_resid"] <= 1.0001e-10
    Vg = host(V).reshape(len(th), lat.V, 4, 3)
    assert np.all(Vg[:, lat.parity == 1] == 0)
    Vg = Vg[:, lat.parity == 0].reshape(len(th), -1).T
    assert np.allclose(Vg.conj().T @ Vg, np.eye(Vg.shape[1]), atol=1e-12)
    if st["iterations"] == io["cycles"]:
        assert len(th) == len(tho)
        assert same_eigenvalues(th, tho, rtol=1e-6, atol=1e-9)
        assert projector_distance(Vg, Vo) <= 1e-6


@pytest.mark.parametrize("prec,shape", [("fp64", None), ("mixed", None), ("mixed", ("0", "1")),
                                         ("mixed", ("0", "0")), ("mixed", ("2", "0"))])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_dbicgstab_batched_matches_oracle(gpu_lib, monkeypatch, prec, shape, dagger):
    """D-BiCGStab(6) on Ahat for 3 Z2 sources in one call (FP32 launch shapes forced or tuned):
    every full solution meets 1e-8 on A x = b (or A^dagger x = b), and agrees with the oracle's
    deflated solve of the same reduced system to the conditioning of the tolerance."""
    if shape is not None:
        monkeypatch.setenv("DBQ_DS_NB", shape[0])
        monkeypatch.setenv("DBQ_DS_RG", shape[1])
    L = C["L"]
    lat, U = _setup()
    kappa = C["kappa"]
    _, V, th, _ = gpu_lib.gmresdr_first_rhs(L, dev(U), dev(synth.point_source(L)), kappa, 20, 6,
                                            tol=1e-10, schur=True)
    B = synth.z2_sources(L, 3, 1101)
    X, sts, status = gpu_lib.dbicgstab_solve(
        [dict(L=L, links=dev(U), kappa=kappa, B=dev(B), V=V, schur=True)], tol=1e-8, prec=prec,
        dagger=dagger)
    assert status == 0
    Xh = host(X[0])
    Vh = host(V).reshape(V.shape[0], lat.V, 4, 3)[:, lat.parity == 0].reshape(V.shape[0], -1).T
    A = EO.schur_operator(U, lat, kappa, dagger=dagger)
    for j in range(3):
        assert sts[j]["status"] == 0
        rel = _true_rel(U, lat, kappa, 0.0, Xh[j], B[j], dagger)
        assert rel <= 1.05e-8, rel
        assert abs(sts[j]["rel_true_resid"] - rel) <= 1e-3 * rel
        bh = EO.schur_source(U, lat, kappa, B[j], dagger=dagger)
        xe, info = S.dbicgstab(A, bh, Vh, EO.gamma5_half, tol=1e-12, dagger=dagger)
        xo = EO.schur_reconstruct(U, lat, kappa, xe, B[j], dagger=dagger).reshape(-1)
        assert np.linalg.norm(Xh[j].reshape(-1) - xo) <= 1e-5 * np.linalg.norm(xo)


def test_schur_uneven_batch_equals_separate_solves(gpu_lib):
    """Two lattices of different size and a twisted mass in one reduced-system call: each
    solution meets the tolerance on its full system."""
    probs = []
    for L, seed, mu in [((4, 4, 4, 4), 31, 0.0), ((6, 4, 4, 8), 32, 0.05)]:
        lat = W.Lattice(L)
        U = synth.gauge_field(L, 0.5, seed)
        B = synth.z2_sources(L, 2, seed + 1000)
        probs.append((L, lat, U, B, mu))
    X, sts, status = gpu_lib.dbicgstab_solve(
        [dict(L=L, links=dev(U), kappa=0.12, mu=mu, B=dev(B), V=None, schur=True)
         for L, lat, U, B, mu in probs], tol=1e-8, prec="mixed")
    assert status == 0
    for (L, lat, U, B, mu), x in zip(probs, X):
        for j in range(2):
            assert _true_rel(U, lat, 0.12, mu, host(x)[j], B[j]) <= 1.05e-8


def test_schur_project_shifts_matches_oracle(gpu_lib):
    """MR projection over two previous twisted-mass solutions on the reduced system of the new
    shift: the same minimal residual norm as the oracle's projection of that system."""
    L = (4, 4, 4, 4)
    lat, U = _setup(L, 0.5, 51)
    kappa = 0.12
    b = synth.z2_sources(L, 1, 52)
    Q = []
    for mu in (0.04, 0.03):
        X, _, st = gpu_lib.dbicgstab_solve(
            [dict(L=L, links=dev(U), kappa=kappa, mu=mu, B=dev(b), V=None, schur=True)],
            tol=1e-10, prec="fp64")
        assert st == 0
        Q.append(host(X[0])[0])
    Q = np.stack(Q)[None]
    mu_new = 0.02
    X0, rb, ra = gpu_lib.project_shifts(L, dev(U), kappa, mu_new, dev(Q), dev(b), schur=True)
    A = EO.schur_operator(U, lat, kappa, mu_new)
    bh = EO.schur_source(U, lat, kappa, b[0], mu_new)
    Qe = np.stack([_even(lat, q) for q in Q[0]], axis=1)
    xe, r_new, info = S.mr_project(A, Qe, bh)
    assert abs(rb[0] - np.linalg.norm(bh)) <= 1e-12 * np.linalg.norm(bh)
    assert abs(ra[0] - info["rnorm_after"]) <= 1e-9 * info["rnorm_before"]
    assert ra[0] < rb[0]
    # the minimiser need not be unique (nearby shifts' solutions are nearly collinear), its
    # residual is: the returned x0 has the reported reduced residual, and its odd sites are the
    # reconstruction from its even ones
    xg = host(X0)[0].reshape(lat.V, 4, 3)
    xge = _even(lat, xg)
    assert abs(np.linalg.norm(bh - A(xge)) - ra[0]) <= 1e-9 * rb[0]
    want = EO.schur_reconstruct(U, lat, kappa, xge, b[0], mu_new)
    assert relerr(xg, want) <= 1e-12


def test_link_force_rejects_the_reduced_operator(gpu_lib):
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 61)
    x = synth.gaussian_sources(L, 1, 62)
    from paper_0710_1988_amd import _abi
    import ctypes
    h = gpu_lib._ctx(dev(U).device)
    Ud = dev(U)
    op = gpu_lib._operator(L, Ud, 0.12, 0.0, True)
    xd = dev(x)
    F = dev(np.zeros((4, 64 * 4, 8)))
    st = _abi.load().link_force(h, ctypes.byref(op), xd.data_ptr(), xd.data_ptr(), 1, 0,
                                F.data_ptr())
    assert st == -1


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 2e-6)])
def test_schur_apply_full_size_24x48_sampled_sites(gpu_lib, prec, tol):
    """24^3 x 48 (the twisted-mass lattice), twisted mass and the dagger: every even site computed
    on the GPU, 256 sampled even sites (first and last included) recomputed by the oracle."""
    L = (24, 24, 24, 48)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 105)
    psi = synth.z2_sources(L, 1, 1105)
    out = host(gpu_lib.wilson_apply(L, dev(U), dev(psi), 0.2089, 0.003, True, prec,
                                    schur=True))[0]
    ev = np.nonzero(lat.parity == 0)[0]
    pick = np.sort(np.random.default_rng(6).choice(ev, 256, replace=False))
    pick[0], pick[-1] = ev[0], ev[-1]
    want = EO.schur_apply_sites(U, lat, 0.2089, _even(lat, psi[0]), pick, 0.003, True)
    assert relerr(out[pick], want) <= tol
    assert np.all(_odd(lat, out) == 0)
