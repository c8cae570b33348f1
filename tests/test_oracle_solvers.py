"""Pins of the oracle's solvers, kappa_c and gradient against dense linear algebra, closed forms,
exact invariants and the paper's printed counts (CPU only)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import force as F
from oracle import kappa as K
from oracle import solvers as S
from oracle import wilson as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mvp_counts.json")


def _setup(L, c, seed, kappa, mu=0.0):
    lat = W.Lattice(L)
    U = synth.gauge_field(L, c, seed)
    return lat, U, W.operator(U, lat, kappa, mu)


# ----------------------------------------------------------------------------- paper's counts
def test_paper_counting_conventions():
    """Tables 1-3: every BiCGStab / D-BiCGStab count is even (two MVPs per iteration) and every
    GMRES-DR count has the form m + (m-k)(cycles-1) for an integer number of cycles >= 1
    (convergence tested once per cycle) -- the conventions the oracle's counts follow."""
    g = json.load(open(GOLDEN))
    for tab in ("table1_16x16x16x16", "table2_20x20x20x32"):
        for row in g[tab]["rows"]:
            _, m, k, gd, l1, l2, l3, bi = row
            for v in (l1, l2, l3, bi):
                if v is not None:
                    assert v % 2 == 0
            if gd != "F":
                assert (gd - m) % (m - k) == 0 and gd >= m
    t3 = g["table3_twisted_mass_20x20x20x32"]
    m, k = t3["m"], t3["k"]
    cols = np.array([r[3:] for r in t3["rows"]])
    assert list(cols.sum(axis=0)) == t3["totals"]
    for v in cols[:, 0]:   # x0 = 0 column: plain GMRES-DR(40,10) runs
        assert (v - m) % (m - k) == 0


# ----------------------------------------------------------------------------- BiCGStab
def test_bicgstab_matches_dense_solve():
    L = (2, 2, 2, 4)
    lat, U, A = _setup(L, 0.6, 31, 0.17, 0.01)
    M = W.dense_matrix(U, lat, 0.17, 0.01)
    b = synth.z2_sources(L, 1, 32)[0].reshape(-1)
    x, info = S.bicgstab(A, b, tol=1e-12)
    xe = np.linalg.solve(M, b)
    assert info["status"] == S.OK
    assert np.linalg.norm(x - xe) <= 1e-12 * np.linalg.cond(M) * np.linalg.norm(xe)
    assert info["matvecs"] == 2 * info["iterations"] + 1   # + the confirming true residual


def test_point_source_breakdown_is_exact():
    """With rhat = r0 = point source the second rho vanishes exactly on L >= 3: the diagonal of
    H^2 is zero since (1 - gamma)(1 + gamma) = 0 kills every back-and-forth hop."""
    L = (4, 4, 4, 4)
    lat, U, A = _setup(L, 0.3, 101, 0.15)
    for c in range(12):
        e = np.zeros(lat.n, dtype=complex)
        e[c] = 1.0
        HH = W.hopping(U, W.hopping(U, e, lat), lat).reshape(-1)
        assert HH[c] == 0.0
    b = synth.point_source(L)[0].reshape(-1)
    x, info = S.bicgstab(A, b, tol=1e-8, max_restarts=0)
    assert info["status"] == S.EBREAKDOWN and info["iterations"] == 1
    x, info = S.bicgstab(A, b, tol=1e-8)
    assert info["status"] == S.OK and info["restarts"] >= 1


def test_bicgstab_max_mv_reports_not_converged():
    L = (4, 4, 4, 4)
    lat, U, A = _setup(L, 0.3, 101, 0.15)
    b = synth.z2_sources(L, 1, 1101)[0].reshape(-1)
    x, info = S.bicgstab(A, b, tol=1e-8, max_mv=10)
    assert info["status"] == S.NOT_CONVERGED and info["matvecs"] >= 10


# ----------------------------------------------------------------------------- GMRES-DR
def test_gmresdr_c1_invariants():
    """4^4, links exp(0.3 i Q) seed 101, kappa 0.15, point source, GMRES-DR(20,6), 1e-8."""
    L = (4, 4, 4, 4)
    lat, U, A = _setup(L, 0.3, 101, 0.15)
    b = synth.point_source(L)[0].reshape(-1)
    x, V, th, info = S.gmresdr(A, b, 20, 6, tol=1e-8, return_basis=True)
    assert info["status"] == S.OK
    assert info["matvecs"] == 20 + 14 * (info["cycles"] - 1)
    assert np.linalg.norm(b - A(x)) <= 1.0001e-8 * np.linalg.norm(b)
    Vb, Hb = info["Vbasis"], info["Hbar"]
    AV = np.stack([A(Vb[:, j]) for j in range(20)], axis=1)
    assert np.linalg.norm(AV - Vb @ Hb) <= 1e-12
    assert np.allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-13)
    assert np.all(np.diff(np.abs(th)) >= -1e-15)


def test_gmresdr_free_field_distinct_closed_form_eigenvalues():
    """Unit links, kappa 0.12 on 4^4: a single-start Krylov space sees one vector per eigenspace,
    so the harmonic Ritz values converge to distinct closed-form eigenvalues nearest 0:
    1-8k, 1-6k +- 2ik, 1-4k."""
    L = (4, 4, 4, 4)
    lat = W.Lattice(L)
    k = 0.12
    A = W.operator(synth.unit_field(L), lat, k)
    b = synth.point_source(L)[0].reshape(-1)
    x, V, th, info = S.gmresdr(A, b, 20, 6, tol=1e-12)
    expect = [1 - 8 * k, 1 - 6 * k + 2j * k, 1 - 6 * k - 2j * k, 1 - 4 * k]
    for e in expect:
        assert np.min(np.abs(th - e)) <= 1e-8


def test_gmresdr_harmonic_ritz_values_match_dense_spectrum():
    L = (2, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 21)
    kc, _ = K.kappa_c_dense(U, lat)
    A = W.operator(U, lat, 0.98 * kc)
    ev = np.linalg.eigvals(W.dense_matrix(U, lat, 0.98 * kc))
    b = synth.z2_sources(L, 1, 5)[0].reshape(-1)
    x, V, th, info = S.gmresdr(A, b, 30, 8, tol=1e-13)
    assert info["k_out"] == 8
    for t in th:
        assert np.min(np.abs(ev - t)) <= 1e-6 * abs(t)
    # and they are the 8 eigenvalues nearest the origin
    assert np.max(np.abs(th)) <= np.sort(np.abs(ev))[8] + 1e-9


def test_conjugate_closure_rule():
    th = np.array([0.1 + 0.02j, 0.1 - 0.02j, 0.2 + 0.05j, 0.2 - 0.05j, 0.3])
    o = S.smallest_order(th)
    ts = th[o]
    assert S.conjugate_closed_k(ts, 2) == 2
    assert S.conjugate_closed_k(ts, 3) == 2
    assert S.conjugate_closed_k(ts, 4) == 4
    assert S.conjugate_closed_k(np.array([0.1, 0.1000001, 0.3]), 1) == 1


# ----------------------------------------------------------------------------- D-BiCGStab
def _exact_vectors(M, k):
    ev, R = np.linalg.eig(M)
    o = S.smallest_order(ev)
    return ev[o], R[:, o]


def test_dbicgstab_with_exact_eigenvectors():
    """Exact right eigenvectors (conjugate-closed set) with left vectors gamma5 V: U^H A V is
    well conditioned, the deflated residual is left-orthogonal (gamma5 V)^H r = 0, and the
    solution agrees with the dense solve."""
    L = (4, 4, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 22)
    kc, _ = K.kappa_c_dense(U, lat)
    kap = 0.995 * kc
    M = W.dense_matrix(U, lat, kap)
    A = W.operator(U, lat, kap)
    ev, R = _exact_vectors(M, 8)
    k = S.conjugate_closed_k(ev, 8)
    Vq, _ = np.linalg.qr(R[:, :k])
    g5 = lambda v: W.gamma5_flat(v, lat.V)
    b = synth.z2_sources(L, 1, 23)[0].reshape(-1)
    x, info = S.dbicgstab(A, b, Vq, g5, tol=1e-11)
    assert info["status"] == S.OK
    assert info["cond"] < 1e3
    assert info["left_proj"] <= 1e-13
    xe = np.linalg.solve(M, b)
    assert np.linalg.norm(x - xe) <= 1e-11 * np.linalg.cond(M) * np.linalg.norm(xe)
    x0, i0 = S.bicgstab(A, b, tol=1e-11)
    assert info["iterations"] < i0["iterations"]


def test_split_conjugate_pair_makes_projection_singular():
    L = (4, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 24)
    M = W.dense_matrix(U, lat, 0.17)
    ev, R = _exact_vectors(M, 6)
    # find a complex eigenvalue whose partner comes right after it
    starts, i = [], 0
    while i < len(ev) - 1:
        if abs(ev[i].imag) > 1e-6 and abs(ev[i] - np.conj(ev[i + 1])) < 1e-9:
            starts.append(i)
            i += 2
        else:
            i += 1
    j = next(i for i in starts if i >= 2)
    G5 = np.kron(np.eye(lat.V), np.kron(W.GAMMA5, np.eye(3)))
    def cond_of(cols):
        V, _ = np.linalg.qr(R[:, cols])
        return np.linalg.cond((G5 @ V).conj().T @ M @ V)
    assert cond_of(list(range(j + 1))) > 1e10           # partner missing
    assert cond_of(list(range(j + 2))) < 1e6            # pair closed


def test_dbicgstab_adjoint_roles_swap():
    """A^dagger x = b solved with right vectors gamma5 V and left vectors V agrees with the dense
    solve of the adjoint system."""
    L = (4, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 25)
    M = W.dense_matrix(U, lat, 0.16, 0.02)
    Ad = W.operator(U, lat, 0.16, 0.02, dagger=True)
    ev, R = _exact_vectors(M, 6)
    k = S.conjugate_closed_k(ev, 6)
    V, _ = np.linalg.qr(R[:, :k])
    g5 = lambda v: W.gamma5_flat(v, lat.V)
    b = synth.gaussian_sources(L, 1, 26)[0].reshape(-1)
    x, info = S.dbicgstab(Ad, b, V, g5, tol=1e-12, dagger=True)
    xe = np.linalg.solve(M.conj().T, b)
    assert info["status"] == S.OK
    assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)


# ----------------------------------------------------------------------------- MR projection
def test_gmresdr_from_nonzero_x0_matches_dense_solve():
    """GMRES-DR started from x0 != 0 (as in the Sec. 4 shift sequence) solves A x = b, not a
    problem with the sign of r0 flipped: the solution matches a dense solve to the conditioning
    of the tolerance; the initial residual costs one product, so matvecs = 1 + m + (m-k)(c-1).
    From x0 = x* + 1e-3 e the start sits near the solution: fewer cycles than from zero reach
    x* (a flipped r0 = A x0 - b would land at 2 x0 - x*, an error of 2e-3 ||e||)."""
    L = (2, 2, 2, 4)
    lat, U, A = _setup(L, 0.6, 41, 0.16, 0.02)
    M = W.dense_matrix(U, lat, 0.16, 0.02)
    b = synth.z2_sources(L, 1, 42)[0].reshape(-1)
    xe = np.linalg.solve(M, b)
    cond = np.linalg.cond(M)
    x0 = synth.gaussian_sources(L, 1, 43)[0].reshape(-1)
    x, V, th, info = S.gmresdr(A, b, 12, 4, tol=1e-10, x0=x0)
    assert info["status"] == S.OK
    assert info["matvecs"] == 1 + 12 + 8 * (info["cycles"] - 1)
    assert np.linalg.norm(x - xe) <= 1e-10 * cond * np.linalg.norm(xe)
    assert np.linalg.norm(b - M @ x) <= 1.0001e-10 * np.linalg.norm(b)
    e = synth.gaussian_sources(L, 1, 44)[0].reshape(-1)
    xs = xe + 1e-3 * e / np.linalg.norm(e) * np.linalg.norm(xe)
    x, _, _, info = S.gmresdr(A, b, 12, 4, tol=1e-8, x0=xs)
    _, _, _, info0 = S.gmresdr(A, b, 12, 4, tol=1e-8)
    assert info["status"] == S.OK and info["cycles"] < info0["cycles"]
    assert info["matvecs"] == 1 + 12 + 8 * (info["cycles"] - 1)
    assert np.linalg.norm(x - xe) <= 1e-8 * cond * np.linalg.norm(xe)


def test_mr_projection_from_nonzero_x0_matches_lstsq():
    """The Sec. 4 projection from x0 != 0: d minimises ||(b - A x0) - A Q d|| (checked against
    lstsq on the dense matrix), x = x0 + Q d, the returned residual is b - A x, the reported
    initial norm is ||b - A x0||, and the products are 1 (for r0) + nq."""
    L = (4, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 27)
    b = synth.z2_sources(L, 1, 28)[0].reshape(-1)
    mus = [0.05, 0.03, 0.02]
    Q = np.stack([np.linalg.solve(W.dense_matrix(U, lat, 0.15, m), b) for m in mus], axis=1)
    Mn = W.dense_matrix(U, lat, 0.15, 0.01)
    A = W.operator(U, lat, 0.15, 0.01)
    x0 = 0.5 * Q[:, -1] + 0.1 * synth.gaussian_sources(L, 1, 29)[0].reshape(-1)
    x, r, info = S.mr_project(A, Q, b, x0=x0)
    r0 = b - Mn @ x0
    d_ls = np.linalg.lstsq(Mn @ Q, r0, rcond=None)[0]
    assert info["matvecs"] == 1 + 3
    assert abs(info["rnorm_before"] - np.linalg.norm(r0)) <= 1e-12 * np.linalg.norm(r0)
    assert np.linalg.norm(info["d"] - d_ls) <= 1e-8 * np.linalg.norm(d_ls)
    assert np.linalg.norm(x - (x0 + Q @ d_ls)) <= 1e-8 * np.linalg.norm(x)
    assert np.linalg.norm(r - (b - Mn @ x)) <= 1e-11 * np.linalg.norm(b)
    assert info["rnorm_after"] <= info["rnorm_before"]
    # starting from x0 gives the residual of the best x in x0 + span(Q), which is at most the
    # residual of the projection from zero over span(Q) when x0 lies in span(Q)
    x0q = Q @ np.array([0.2, -0.1, 0.7])
    _, r_q, _ = S.mr_project(A, Q, b, x0=x0q)
    _, r_z, _ = S.mr_project(A, Q, b)
    assert abs(np.linalg.norm(r_q) - np.linalg.norm(r_z)) <= 1e-10 * np.linalg.norm(b)


def test_mr_projection_minimises_residual():
    L = (4, 2, 2, 2)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 27)
    b = synth.z2_sources(L, 1, 28)[0].reshape(-1)
    mus = [0.05, 0.03, 0.02]
    Q = np.stack([np.linalg.solve(W.dense_matrix(U, lat, 0.15, m), b) for m in mus], axis=1)
    Mn = W.dense_matrix(U, lat, 0.15, 0.01)
    A = W.operator(U, lat, 0.15, 0.01)
    x, r, info = S.mr_project(A, Q, b)
    Wm = Mn @ Q
    d_ls = np.linalg.lstsq(Wm, b, rcond=None)[0]
    assert np.linalg.norm(r - (b - Wm @ d_ls)) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(Wm.conj().T @ r) <= 1e-10 * np.linalg.norm(b)
    assert info["rnorm_after"] <= info["rnorm_before"]
    assert np.linalg.norm(b - Mn @ x - r) <= 1e-11 * np.linalg.norm(b)
    # the paper's normal equations give the same minimiser here (well-conditioned W)
    d_ne = np.linalg.solve(Wm.conj().T @ Wm, Wm.conj().T @ b)
    assert np.linalg.norm(d_ne - info["d"]) <= 1e-6 * np.linalg.norm(d_ne)


# ----------------------------------------------------------------------------- kappa_c
def test_kappa_c_free_field_is_one_eighth():
    L = (4, 4, 4, 4)
    kc, vals, res = K.kappa_c(synth.unit_field(L), W.Lattice(L))
    assert abs(kc - 0.125) <= 1e-12 and res <= 1e-10


def test_kappa_c_matches_dense_eigenvalues():
    L = (2, 2, 2, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.6, 29)
    kd, ev = K.kappa_c_dense(U, lat)
    ka, vals, res = K.kappa_c(U, lat)
    assert abs(kd - ka) <= 1e-12 * kd and res <= 1e-10
    # spectrum of H symmetric under lambda -> -lambda (bipartite lattice)
    assert max(np.min(np.abs(ev + e)) for e in ev) <= 1e-10


# ----------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("mu", [0.0, 0.04])
def test_link_force_matches_finite_differences(mu):
    """L(theta) = Re(eta^H A(U(theta))^{-1} b), U_mu(y) -> exp(i theta T_a) U_mu(y): central
    differences with dense solves against F[mu, y, a] = Re(i tr[T_a U G^H])."""
    L = (2, 2, 2, 4)
    lat = W.Lattice(L)
    U = synth.gauge_field(L, 0.5, 30)
    kap = 0.15
    b = synth.z2_sources(L, 1, 31)[0]
    eta = synth.gaussian_sources(L, 1, 32)[0]
    M = W.dense_matrix(U, lat, kap, mu)
    x = np.linalg.solve(M, b.reshape(-1)).reshape(lat.V, 4, 3)
    lam = np.linalg.solve(M.conj().T, eta.reshape(-1)).reshape(lat.V, 4, 3)
    G = F.link_gradient(U, lat, kap, lam, x)
    Fo = F.su3_force(U, G)
    rng = np.random.default_rng(33)
    h = 1e-5
    for _ in range(5):
        m_, y, a = rng.integers(0, 4), rng.integers(0, lat.V), rng.integers(0, 8)
        vals = []
        for s in (+1, -1):
            Up = U.copy()
            q, Wv = np.linalg.eigh(F.T_GEN[a])
            Up[m_, y] = (Wv * np.exp(1j * s * h * q)) @ Wv.conj().T @ U[m_, y]
            Mp = W.dense_matrix(Up, lat, kap, mu)
            vals.append(np.real(np.vdot(eta.reshape(-1), np.linalg.solve(Mp, b.reshape(-1)))))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - Fo[m_, y, a]) <= 1e-6 * max(1.0, abs(fd))
    # grad_b = lambda = A^{-H} eta, and A^{-H} = gamma5 A(-mu)^{-1} gamma5
    M5 = W.dense_matrix(U, lat, kap, -mu)
    g5 = lambda v: W.gamma5_flat(v, lat.V)
    lam2 = g5(np.linalg.solve(M5, g5(eta.reshape(-1))))
    assert np.allclose(lam2, lam.reshape(-1), atol=1e-11)


# ----------------------------------------------------------------------------- GMRES-Proj
def test_gmres_proj_first_cycle_is_the_krylov_minimal_residual():
    """Without eigenvectors one GMRES(m) cycle from x0 = 0 gives the minimal residual over the
    Krylov space span{b, Ab, ..., A^{m-1} b}, here by least squares on the explicit power basis."""
    L = (2, 2, 2, 4)
    lat, U, A = _setup(L, 0.6, 41, 0.12)
    b = synth.gaussian_sources(L, 1, 42)[0].reshape(-1)
    m = 5
    x, info = S.gmres_proj(A, b, np.zeros((b.size, 0), complex), m, tol=1e-30, max_mv=m)
    K = [b]
    for _ in range(m - 1):
        K.append(A(K[-1]))
    K = np.stack(K, axis=1)
    AK = np.stack([A(K[:, i]) for i in range(m)], axis=1)
    y = np.linalg.lstsq(AK, b, rcond=None)[0]
    r_ref = b - AK @ y
    assert info["matvecs"] == m and info["cycles"] == 1
    assert abs(np.linalg.norm(b - A(x)) - np.linalg.norm(r_ref)) <= 1e-10 * np.linalg.norm(b)
    assert abs(info["rel_resid"] - np.linalg.norm(r_ref) / np.linalg.norm(b)) <= 1e-10


def test_gmres_proj_projection_is_exact_on_the_range_of_AV():
    """If b lies in span(A V) the first minimal-residual projection solves the system outright."""
    L = (2, 2, 2, 4)
    lat, U, A = _setup(L, 0.6, 43, 0.12)
    n = lat.n
    rng = np.random.default_rng(44)
    V = np.linalg.qr(rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4)))[0]
    c = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    b = np.stack([A(V[:, i]) for i in range(4)], axis=1) @ c
    x, info = S.gmres_proj(A, b, V, 10, tol=1e-12)
    assert info["status"] == S.OK and info["matvecs"] == 0 and info["cycles"] == 0
    assert np.linalg.norm(x - V @ c) <= 1e-12 * np.linalg.norm(V @ c)


def test_gmres_proj_matches_dense_solve_and_beats_plain_restarted_gmres():
    """With GMRES-DR eigenvectors of the small eigenvalues, GMRES(m)-Proj(k) converges to the
    dense solution in fewer products than GMRES(m) without projection."""
    L = (4, 4, 4, 4)
    lat, U, A = _setup(L, 0.3, 101, 0.139)   # near kappa_c = 0.140
    b1 = synth.point_source(L)[0].reshape(-1)
    _, V, _, _ = S.gmresdr(A, b1, 20, 6, tol=1e-10)
    b = synth.z2_sources(L, 1, 1101)[0].reshape(-1)
    x, info = S.gmres_proj(A, b, V, 20, tol=1e-10)
    x0, info0 = S.gmres_proj(A, b, np.zeros((b.size, 0), complex), 20, tol=1e-10)
    assert info["status"] == S.OK and info0["status"] == S.OK
    assert np.linalg.norm(b - A(x)) <= 1.001e-10 * np.linalg.norm(b)
    assert info["matvecs"] < info0["matvecs"]
    assert info["matvecs"] % 20 == 0 and info["setup_matvecs"] == V.shape[1]
    assert np.linalg.norm(x - x0) <= 1e-8 * np.linalg.norm(x0)
