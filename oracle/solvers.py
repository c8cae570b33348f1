"""Oracle: Krylov solvers of the method, plain NumPy FP64 complex.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``bicgstab``    -- BiCGStab (van der Vorst), the non-restarted method of Sec. 1 / Sec. 2 that
                     the paper deflates; 2 matrix-vector products (MVPs) per iteration.
* ``gmresdr``     -- GMRES-DR(m,k) (Sec. 1: GMRES with deflated restarting, which keeps k
                     approximate eigenvectors of small eigenvalues through every restart and
                     returns them with the solution of the first right-hand side).
* ``dbicgstab``   -- D-BiCGStab(k), Sec. 2: solve U^H A V y = U^H r0 with left vectors
                     U = gamma5 V (Sec. 1), set x0 += V y, then run BiCGStab.
* ``mr_project``  -- Sec. 4: minimal-residual projection of a new shift's initial residual over the
                     solutions Q of previous shifts, x0 += Q d with d minimising ||r0 - A Q d||.
* ``gmres_proj``  -- GMRES(m)-Proj(k), the comparison method of Sec. 1 and Sec. 3: cycles of
                     restarted GMRES(m) alternating with a minimal-residual projection over the
                     right eigenvectors V from GMRES-DR.

All functions take the operator as a callable on flat complex128 vectors.  Statuses:
OK = 0, NOT_CONVERGED = 1 (the paper's "F"), EBREAKDOWN = -2, ESINGULAR = -3.

Readings where the paper is silent (each listed with its reason in the design notes):
relative residual ||b - A x|| / ||b||; GMRES-DR orthogonalises with classical Gram-Schmidt
applied twice and tests convergence once per cycle, which makes its MVP count
m + (m-k)(cycles-1), the form every GMRES-DR entry of Tables 1-3 has; the k kept vectors are
the harmonic Ritz vectors of smallest |theta|; the returned k is reduced by one when the k-th and
(k+1)-th values form a complex-conjugate pair (gamma5-hermiticity makes the spectrum symmetric under
conjugation and a split pair makes U^H A V singular); BiCGStab restarts with rhat <- r on
breakdown.
"""
from __future__ import annotations

import numpy as np

OK, NOT_CONVERGED, EBREAKDOWN, ESINGULAR = 0, 1, -2, -3


def _norm(v):
    return float(np.linalg.norm(v))


# --------------------------------------------------------------------------- BiCGStab
def bicgstab(A, b, x0=None, tol=1e-8, max_mv=20000, bnorm=None, max_restarts=10,
             mv_start=0, history=False):
    """Complex BiCGStab from initial guess x0 with shadow vector rhat = r0.

    Iteration (inner product <a,b> = a^H b):
        rho = <rhat, r>; beta = (rho/rho_prev)(alpha/omega); p = r + beta (p - omega v)
        v = A p; alpha = rho / <rhat, v>; s = r - alpha v; t = A s
        omega = <t, s>/<t, t>; x += alpha p + omega s; r = s - omega t
    Convergence when ||r|| <= tol ||b||, confirmed with the true residual b - A x (counted as an
    MVP); if the confirmation fails the recursion continues from the true residual.
    Breakdown (|rho| <= 1e-14 ||rhat|| ||r||, or omega = 0) restarts with rhat <- r, p = v = 0.
    Returns (x, info) with info = dict(status, matvecs, iterations, restarts, rel_true_resid,
    history).
    """
    b = np.asarray(b, dtype=np.complex128)
    bn = _norm(b) if bnorm is None else bnorm
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    mv = mv_start
    if x0 is not None and np.any(x0 != 0):
        r = b - A(x)
        mv += 1
    else:
        r = b.copy()
    hist = [_norm(r) / bn] if history else None
    if bn == 0.0:
        return x, dict(status=OK, matvecs=mv, iterations=0, restarts=0, rel_true_resid=0.0,
                       history=hist)
    if _norm(r) <= tol * bn:
        return x, dict(status=OK, matvecs=mv, iterations=0, restarts=0,
                       rel_true_resid=_norm(r) / bn, history=hist)
    rhat = r.copy()
    rho_prev = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    iters = restarts = 0
    status = NOT_CONVERGED
    while mv < max_mv:
        rho = np.vdot(rhat, r)
        if abs(rho) <= 1e-14 * _norm(rhat) * _norm(r):
            restarts += 1
            if restarts > max_restarts:
                status = EBREAKDOWN
                break
            rhat = r.copy()
            rho_prev = alpha = omega = 1.0 + 0j
            v[:] = 0
            p[:] = 0
            rho = np.vdot(rhat, r)
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        t = A(s)
        mv += 2
        iters += 1
        tt = np.vdot(t, t).real
        if tt == 0.0:
            # s = 0: x + alpha p is exact
            x = x + alpha * p
            r = s
            omega = 0.0
        else:
            omega = np.vdot(t, s) / tt
            x = x + alpha * p + omega * s
            r = s - omega * t
        rho_prev = rho
        rn = _norm(r)
        if history:
            hist.append(rn / bn)
        if rn <= tol * bn:
            rt = b - A(x)
            mv += 1
            if _norm(rt) <= tol * bn:
                status = OK
                break
            r = rt
        if omega == 0.0:
            # omega = 0 breakdown: the next rho test restarts with rhat <- r
            restarts += 1
            if restarts > max_restarts:
                status = EBREAKDOWN
                break
            rhat = r.copy()
            rho_prev = alpha = omega = 1.0 + 0j
            v[:] = 0
            p[:] = 0
    rel = _norm(b - A(x)) / bn
    return x, dict(status=status, matvecs=mv, iterations=iters, restarts=restarts,
                   rel_true_resid=rel, history=hist)


# --------------------------------------------------------------------------- small dense helpers
def _orthonormalize_columns(P):
    """Orthonormal basis of the column span, column by column (Gram-Schmidt applied twice)."""
    Q = np.zeros_like(P)
    for j in range(P.shape[1]):
        w = P[:, j].copy()
        for _ in range(2):
            if j:
                w = w - Q[:, :j] @ (Q[:, :j].conj().T @ w)
        Q[:, j] = w / _norm(w)
    return Q


def harmonic_ritz(Hbar):
    """Harmonic Ritz pairs of the (m+1) x m matrix Hbar: eigenpairs of
    H_m + |h_{m+1,m}|^2 f e_m^T with f = H_m^{-H} e_m (H_m = first m rows of Hbar).
    Returns (theta, G) with G's columns the (unnormalised) eigenvectors in C^m."""
    m = Hbar.shape[1]
    Hm = Hbar[:m, :m]
    em = np.zeros(m, dtype=np.complex128)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.conj().T, em)
    h = Hbar[m, m - 1]
    G = Hm.copy()
    G[:, -1] += abs(h) ** 2 * f
    theta, vecs = np.linalg.eig(G)
    return theta, vecs


def smallest_order(theta):
    """Indices sorting theta by |theta| ascending, ties broken by (Re, Im)."""
    return np.lexsort((theta.imag, theta.real, np.abs(theta)))


def conjugate_closed_k(theta_sorted, k, rtol=1e-3):
    """Reduce k by one when the k-th and (k+1)-th values (in sorted order) are an approximate
    complex-conjugate pair with non-real theta_k."""
    if k <= 0 or k >= len(theta_sorted):
        return k
    a, b = theta_sorted[k - 1], theta_sorted[k]
    scale = abs(a)
    if abs(a.imag) > rtol * scale and abs(a - np.conj(b)) <= rtol * scale:
        return k - 1
    return k


# --------------------------------------------------------------------------- GMRES-DR
def gmresdr(A, b, m, k, tol=1e-8, max_mv=20000, x0=None, return_basis=False):
    """GMRES-DR(m,k), complex.

    Cycle: Arnoldi A V_m = V_{m+1} Hbar_m (classical Gram-Schmidt twice), least squares
    d = argmin ||c - Hbar d||, x += V_m d, rho = c - Hbar d; converged when ||rho|| <= tol ||b||.
    Restart: harmonic Ritz vectors g_1..g_k of smallest |theta|, orthonormalised, padded with a
    zero row, then rho appended and orthonormalised -> P_{k+1}; Hbar_k = P_{k+1}^H Hbar_m P_k,
    V_{k+1} = V_{m+1} P_{k+1}, c = P_{k+1}^H rho; Arnoldi continues from column k+1.
    Returns (x, V, theta, info) where V (n x k_out) is orthonormal and spans the harmonic Ritz
    vectors of the final cycle, theta their values (sorted by |theta|), and info =
    dict(status, matvecs, cycles, k_out, rel_resid, theta_all) plus, with ``return_basis``, the
    final cycle's Arnoldi basis V_{m+1} and Hbar_m (for checking A V_m = V_{m+1} Hbar_m).
    """
    if not (0 < k < m):
        raise ValueError("need 0 < k < m")
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    bn = _norm(b)
    mv = 0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if x0 is not None and np.any(x0 != 0):
        r = b - A(x)
        mv += 1
    else:
        r = b.copy()
    Vb = np.zeros((n, m + 1), dtype=np.complex128)
    Hb = np.zeros((m + 1, m), dtype=np.complex128)
    beta = _norm(r)
    Vb[:, 0] = r / beta
    c = np.zeros(m + 1, dtype=np.complex128)
    c[0] = beta
    j0 = 0
    cycles = 0
    status = NOT_CONVERGED
    while True:
        for j in range(j0, m):
            w = A(Vb[:, j])
            mv += 1
            Vj = Vb[:, :j + 1]
            h = Vj.conj().T @ w
            w = w - Vj @ h
            h2 = Vj.conj().T @ w
            w = w - Vj @ h2
            Hb[:j + 1, j] = h + h2
            hn = _norm(w)
            Hb[j + 1, j] = hn
            Vb[:, j + 1] = w / hn
        cycles += 1
        d = np.linalg.lstsq(Hb, c, rcond=None)[0]
        x = x + Vb[:, :m] @ d
        rho = c - Hb @ d
        rn = _norm(rho)
        if rn <= tol * bn:
            status = OK
            break
        if mv >= max_mv:
            break
        theta, G = harmonic_ritz(Hb)
        order = smallest_order(theta)
        Pk = _orthonormalize_columns(G[:, order[:k]])
        P = np.zeros((m + 1, k + 1), dtype=np.complex128)
        P[:m, :k] = Pk
        w = rho.copy()
        for _ in range(2):
            w = w - P[:, :k] @ (P[:, :k].conj().T @ w)
        P[:, k] = w / _norm(w)
        Hnew = P.conj().T @ Hb @ P[:m, :k]
        Vb[:, :k + 1] = Vb @ P
        Vb[:, k + 1:] = 0
        c = np.zeros(m + 1, dtype=np.complex128)
        c[:k + 1] = P.conj().T @ rho
        Hb[:] = 0
        Hb[:k + 1, :k] = Hnew
        j0 = k
    # eigenvector output from the last cycle
    theta, G = harmonic_ritz(Hb)
    order = smallest_order(theta)
    ts = theta[order]
    k_out = conjugate_closed_k(ts, k)
    Pk = _orthonormalize_columns(G[:, order[:k_out]])
    Vout = Vb[:, :m] @ Pk
    info = dict(status=status, matvecs=mv, cycles=cycles, k_out=k_out, rel_resid=rn / bn,
                theta_all=ts)
    if return_basis:
        info.update(Vbasis=Vb, Hbar=Hb)
    return x, Vout, ts[:k_out], info


# --------------------------------------------------------------------------- D-BiCGStab
def deflation_matrix(A, V, left):
    """M = left^H A V (k MVPs) and W = A V."""
    W = np.stack([A(V[:, i]) for i in range(V.shape[1])], axis=1)
    return left.conj().T @ W, W


def dbicgstab(A, b, V, g5, tol=1e-8, max_mv=20000, x0=None, dagger=False, cond_max=1e12):
    """D-BiCGStab(k), Sec. 2.

    Right vectors V, left vectors U = gamma5 V (Sec. 1: gamma5 A gamma5 = A^dagger).  For the
    adjoint system (``dagger``: ``A`` must then apply A^dagger) the roles swap: right vectors
    gamma5 V, left vectors V.  Steps: r0 = b - A x0; solve (U^H A V) y = U^H r0; x = x0 + V y;
    r = b - A x (one MVP); BiCGStab from x with rhat = r.
    ``g5`` maps a flat vector to gamma5 times it.  Returns (x, info); info adds setup_matvecs,
    cond and the deflated residual's left-projection norm |U^H r| / ||r||.
    """
    b = np.asarray(b, dtype=np.complex128)
    k = V.shape[1]
    G5V = np.stack([g5(V[:, i]) for i in range(k)], axis=1)
    right, left = (G5V, V) if dagger else (V, G5V)
    M, _ = deflation_matrix(A, right, left)
    cond = np.linalg.cond(M)
    if not np.isfinite(cond) or cond > cond_max:
        return np.zeros_like(b), dict(status=ESINGULAR, cond=cond, matvecs=0, iterations=0,
                                      restarts=0, setup_matvecs=k, rel_true_resid=np.nan)
    mv = 0
    if x0 is not None and np.any(x0 != 0):
        x = np.array(x0, dtype=np.complex128)
        r0 = b - A(x)
        mv += 1
    else:
        x = np.zeros_like(b)
        r0 = b
    y = np.linalg.solve(M, left.conj().T @ r0)
    x = x + right @ y
    r = b - A(x)
    mv += 1
    proj = _norm(left.conj().T @ r) / max(_norm(r), 1e-300)
    x, info = bicgstab(A, b, x0=x, tol=tol, max_mv=max_mv, mv_start=mv - 1)
    info.update(setup_matvecs=k, cond=cond, left_proj=proj)
    return x, info


# --------------------------------------------------------------------------- GMRES-Proj
def gmres_proj(A, b, V, m, tol=1e-8, max_mv=20000, x0=None):
    """GMRES(m)-Proj(k) (Sec. 1; compared with D-BiCGStab in Sec. 3): for a later right-hand side,
    alternate a minimal-residual projection over the right eigenvectors V (n x k) -- x += V d,
    d = argmin ||r - A V d|| -- with one cycle of GMRES(m) (Arnoldi with classical Gram-Schmidt
    twice from r, x += V_m y with y = argmin ||beta e_1 - Hbar y||, r = V_{m+1}(beta e_1 - Hbar y)).
    Convergence ||r|| <= tol ||b|| is tested after each projection and each cycle.  W = A V (k
    products) is setup, reported apart from ``matvecs``.  Returns (x, info) with info =
    dict(status, matvecs, cycles, setup_matvecs, rel_resid, resid_history)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    bn = _norm(b)
    k = V.shape[1]
    mv = 0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if x0 is not None and np.any(x0 != 0):
        r = b - A(x)
        mv += 1
    else:
        r = b.copy()
    W = np.stack([A(V[:, i]) for i in range(k)], axis=1) if k else np.zeros((n, 0), complex)
    hist = [_norm(r)]
    cycles = 0
    status = NOT_CONVERGED
    while True:
        if k:
            d = np.linalg.lstsq(W, r, rcond=None)[0]
            x = x + V @ d
            r = r - W @ d
        rn = _norm(r)
        hist.append(rn)
        if rn <= tol * bn:
            status = OK
            break
        if mv >= max_mv:
            break
        Vb = np.zeros((n, m + 1), dtype=np.complex128)
        Hb = np.zeros((m + 1, m), dtype=np.complex128)
        beta = rn
        Vb[:, 0] = r / beta
        for j in range(m):
            w = A(Vb[:, j])
            mv += 1
            Vj = Vb[:, :j + 1]
            h = Vj.conj().T @ w
            w = w - Vj @ h
            h2 = Vj.conj().T @ w
            w = w - Vj @ h2
            Hb[:j + 1, j] = h + h2
            hn = _norm(w)
            Hb[j + 1, j] = hn
            Vb[:, j + 1] = w / hn
        c = np.zeros(m + 1, dtype=np.complex128)
        c[0] = beta
        y = np.linalg.lstsq(Hb, c, rcond=None)[0]
        x = x + Vb[:, :m] @ y
        r = Vb @ (c - Hb @ y)
        cycles += 1
        rn = _norm(r)
        hist.append(rn)
        if rn <= tol * bn:
            status = OK
            break
        if mv >= max_mv:
            break
    return x, dict(status=status, matvecs=mv, cycles=cycles, setup_matvecs=k,
                   rel_resid=_norm(r) / bn, resid_history=hist)


# --------------------------------------------------------------------------- MR projection
def mr_project(A, Q, b, x0=None):
    """Sec. 4: x0 += Q d with d = argmin ||r0 - A Q d|| (the paper's normal equations
    Q^H A^H A Q d = Q^H A^H r0 have this minimiser; the oracle solves the least-squares
    problem with a Householder QR of W = A Q, which avoids squaring cond(W)).
    Returns (x_new, r_new, info) with info = dict(rnorm_before, rnorm_after, matvecs, d)."""
    b = np.asarray(b, dtype=np.complex128)
    mv = 0
    if x0 is not None and np.any(x0 != 0):
        x = np.array(x0, dtype=np.complex128)
        r0 = b - A(x)
        mv += 1
    else:
        x = np.zeros_like(b)
        r0 = b.copy()
    W = np.stack([A(Q[:, j]) for j in range(Q.shape[1])], axis=1)
    mv += Q.shape[1]
    Qw, R = np.linalg.qr(W)
    d = np.linalg.solve(R, Qw.conj().T @ r0)
    x = x + Q @ d
    r_new = r0 - W @ d
    return x, r_new, dict(rnorm_before=_norm(r0), rnorm_after=_norm(r_new), matvecs=mv, d=d)
