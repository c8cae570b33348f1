"""Deflated BiCGStab for Wilson and twisted-mass fermion systems on MI355X.

Thin PyTorch binding of the HIP library libdbq.so (C ABI in include/dbq.h): argument checks and
marshalling only; every step of the solvers runs in the library's gfx950 kernels.  There is no CPU
fallback -- importing works without a GPU (for the host-side geometry and ABI checks), but every
compute call needs the library and a GPU and raises otherwise.

Field conventions (see dbq.h): links complex128 (4, V, 3, 3) with links[mu, x] = U_mu(x); spinors
complex128 (nrhs, V, 4, 3); lattice extents L = (Lx, Ly, Lz, Lt), all even; lexicographic sites
lex = x + Lx*(y + Ly*(z + Lz*t)).  Operator A(mu) = I - kappa*H + i*mu*gamma5.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import DBQ_FP64, DBQ_MIXED, Stats, Operator

__all__ = ["DbqError", "wilson_apply", "gmresdr_first_rhs", "dbicgstab_solve", "project_shifts",
           "link_force", "kappa_critical", "geometry", "geometry_host", "site_tile", "set_timing",
           "kernel_time", "reset_timing", "version", "library_path", "DeflatedSolve",
           "tile_schedule_host", "stream_probe"]


class DbqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_abi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def library_path():
    return _abi.LIB_PATH


def version():
    return _abi.load().dbq_version().decode()


# ----------------------------------------------------------------------------- context
_CTX = {}


def _torch():
    import torch
    return torch


def _ctx(device):
    torch = _torch()
    lib = _abi.load()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _CTX.get(idx)
    if h is None:
        h = ctypes.c_void_p()
        with torch.cuda.device(idx):
            st = lib.dbq_create(ctypes.byref(h), None)
        if st != 0:
            raise DbqError(st, "dbq_create failed")
        _CTX[idx] = h
    stream = torch.cuda.current_stream(idx).cuda_stream
    lib.dbq_set_stream(h, ctypes.c_void_p(stream))
    return h


def _check(st, h, ok=(0, 1)):
    if st not in ok:
        raise DbqError(st, _abi.load().dbq_last_error(h).decode())
    return st


# ----------------------------------------------------------------------------- argument checks
def _lattice(L):
    L = tuple(int(v) for v in L)
    if len(L) != 4 or any(v < 2 or v % 2 for v in L):
        raise ValueError(f"lattice extents must be four even integers >= 2, got {L}")
    V = L[0] * L[1] * L[2] * L[3]
    return L, V


def _dev_tensor(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    return t.contiguous()


def _links(U, V):
    U = _dev_tensor(U, "links")
    if tuple(U.shape) != (4, V, 3, 3):
        raise ValueError(f"links must have shape (4, {V}, 3, 3), got {tuple(U.shape)}")
    return U


def _spinors(x, V, name):
    x = _dev_tensor(x, name)
    if x.numel() % (12 * V) != 0 or x.numel() == 0:
        raise ValueError(f"{name} must hold a whole number of spinor fields of {12 * V} elements")
    return x.reshape(-1, V, 4, 3)


def _operator(L, U, kappa, mu, schur=False):
    op = Operator()
    for i in range(4):
        op.L[i] = L[i]
    op.links = ctypes.c_void_p(U.data_ptr())
    op.kappa = float(kappa)
    op.mu = float(mu)
    op.schur = 1 if schur else 0
    op.pad = 0
    return op


def _prec(prec):
    if prec in ("fp64", DBQ_FP64):
        return DBQ_FP64
    if prec in ("mixed", "fp32", DBQ_MIXED):
        return DBQ_MIXED
    raise ValueError(f"precision must be 'fp64' or 'mixed', got {prec!r}")


# ----------------------------------------------------------------------------- entry points
def wilson_apply(L, links, psi, kappa, mu=0.0, dagger=False, prec="fp64", schur=False):
    """A(mu) psi (or A(mu)^dagger psi) for one or many right-hand sides; returns psi's shape.
    With ``schur`` the even-odd reduced operator: out_e = Ahat psi_e, out_o = 0."""
    torch = _torch()
    L, V = _lattice(L)
    U = _links(links, V)
    p = _spinors(psi, V, "psi")
    if p.device != U.device:
        raise ValueError("psi and links must be on the same device")
    out = torch.empty_like(p)
    h = _ctx(U.device)
    op = _operator(L, U, kappa, mu, schur)
    st = _abi.load().wilson_apply(h, ctypes.byref(op), p.data_ptr(), out.data_ptr(), p.shape[0],
                                  int(bool(dagger)), _prec(prec))
    _check(st, h, ok=(0,))
    return out.reshape(psi.shape)


def gmresdr_first_rhs(L, links, b, kappa, m, k, mu=0.0, tol=1e-8, max_mv=20000, x0=None,
                      schur=False):
    """GMRES-DR(m,k) on one right-hand side.  Returns (x, V, theta, stats): x like b, V complex128
    (k_out, V, 4, 3) holding the orthonormal columns of the n x k_out eigenvector basis, theta a
    numpy complex array of the k_out harmonic Ritz values, stats a dict.  With ``schur`` the
    iteration runs on the even-odd reduced operator (V: its eigenvectors on the even sites, zero
    on the odd ones) and x is still the full solution."""
    torch = _torch()
    L, Vol = _lattice(L)
    U = _links(links, Vol)
    bb = _spinors(b, Vol, "b")
    if bb.shape[0] != 1:
        raise ValueError("gmresdr_first_rhs takes one right-hand side")
    if not (2 <= int(k) < int(m) <= 128):
        raise ValueError("need 2 <= k < m <= 128")
    x = torch.zeros_like(bb) if x0 is None else _spinors(x0, Vol, "x0").clone()
    if x.shape != bb.shape:
        raise ValueError("x0 must match b")
    Vout = torch.empty((int(k), Vol, 4, 3), dtype=torch.complex128, device=U.device)
    theta = (ctypes.c_double * (2 * int(k)))()
    kout = ctypes.c_int32(0)
    stats = Stats()
    h = _ctx(U.device)
    op = _operator(L, U, kappa, mu, schur)
    st = _abi.load().gmresdr_first_rhs(h, ctypes.byref(op), bb.data_ptr(), x.data_ptr(), int(m),
                                       int(k), float(tol), int(max_mv), Vout.data_ptr(), theta,
                                       ctypes.byref(kout), ctypes.byref(stats))
    _check(st, h)
    ko = kout.value
    th = np.array(theta[:2 * ko]).reshape(ko, 2)
    return x.reshape(b.shape), Vout[:ko], th[:, 0] + 1j * th[:, 1], stats.as_dict()


def dbicgstab_solve(problems, tol=1e-8, max_mv=20000, prec="mixed", dagger=False):
    """D-BiCGStab(k) over a batch of (possibly different-size) lattices in one call.

    problems: list (1..8) of dicts with keys L, links, kappa, mu (default 0), B (nrhs, V, 4, 3),
    V (k, V, 4, 3) deflation vectors or None, X0 (like B) or None, schur (default False: the
    even-odd reduced operator, the same for every problem; V then from
    ``gmresdr_first_rhs(..., schur=True)``).
    Returns (X list, per-rhs stats list, overall status)."""
    torch = _torch()
    if not (1 <= len(problems) <= 8):
        raise ValueError("between 1 and 8 problems per call")
    n = len(problems)
    ops = (Operator * n)()
    Vp = (ctypes.c_void_p * n)()
    kk = (ctypes.c_int32 * n)()
    Bp = (ctypes.c_void_p * n)()
    Xp = (ctypes.c_void_p * n)()
    nr = (ctypes.c_int32 * n)()
    keep, Xs = [], []
    dev = None
    for i, pr in enumerate(problems):
        L, Vol = _lattice(pr["L"])
        U = _links(pr["links"], Vol)
        dev = U.device if dev is None else dev
        if U.device != dev:
            raise ValueError("all problems must be on one device")
        B = _spinors(pr["B"], Vol, "B")
        X0 = pr.get("X0")
        X = torch.zeros_like(B) if X0 is None else _spinors(X0, Vol, "X0").clone()
        if X.shape != B.shape:
            raise ValueError("X0 must match B")
        Vd = pr.get("V")
        if Vd is not None:
            Vd = _spinors(Vd, Vol, "V")
            if Vd.shape[0] > 128:
                raise ValueError("at most 128 deflation vectors")
            Vp[i] = Vd.data_ptr()
            kk[i] = Vd.shape[0]
        else:
            Vp[i] = None
            kk[i] = 0
        for t in (B, X) + ((Vd,) if Vd is not None else ()):
            if t.device != dev:
                raise ValueError("all tensors must be on the links' device")
        ops[i] = _operator(L, U, pr["kappa"], pr.get("mu", 0.0), pr.get("schur", False))
        Bp[i] = B.data_ptr()
        Xp[i] = X.data_ptr()
        nr[i] = B.shape[0]
        keep += [U, B, Vd]
        Xs.append(X)
    NR = sum(nr)
    stats = (Stats * NR)()
    h = _ctx(dev)
    st = _abi.load().dbicgstab_solve(h, ops, n, Vp, kk, Bp, Xp, nr, float(tol), int(max_mv),
                                     _prec(prec), int(bool(dagger)), stats)
    _check(st, h, ok=(0, 1, -2))
    out = [X.reshape(pr["B"].shape) for X, pr in zip(Xs, problems)]
    return out, [s.as_dict() for s in stats], st


def project_shifts(L, links, kappa, mu, Q, B, X0=None, schur=False):
    """Minimal-residual projection over previous solutions: Q (nrhs, nq, V, 4, 3), B (nrhs, V, 4, 3).
    Returns (X0_new, rnorm_before (nrhs,), rnorm_after (nrhs,)).  With ``schur`` on the even-odd
    reduced system (X0_new full, its odd sites reconstructed)."""
    torch = _torch()
    L, Vol = _lattice(L)
    U = _links(links, Vol)
    Bt = _spinors(B, Vol, "B")
    nrhs = Bt.shape[0]
    Qt = _dev_tensor(Q, "Q")
    if Qt.numel() % (nrhs * 12 * Vol) != 0:
        raise ValueError("Q must have shape (nrhs, nq, V, 4, 3)")
    nq = Qt.numel() // (nrhs * 12 * Vol)
    if not (1 <= nq <= 32):
        raise ValueError("nq must be in 1..32")
    X = torch.zeros_like(Bt) if X0 is None else _spinors(X0, Vol, "X0").clone()
    if X.shape != Bt.shape:
        raise ValueError("X0 must match B")
    rn = (ctypes.c_double * (2 * nrhs))()
    h = _ctx(U.device)
    op = _operator(L, U, kappa, mu, schur)
    st = _abi.load().project_shifts(h, ctypes.byref(op), Qt.data_ptr(), nq, Bt.data_ptr(),
                                    X.data_ptr(), nrhs, rn)
    _check(st, h, ok=(0,))
    r = np.array(rn[:]).reshape(nrhs, 2)
    return X.reshape(B.shape), r[:, 0], r[:, 1]


def gmres_proj_solve(L, links, kappa, B, V=None, m=20, mu=0.0, tol=1e-8, max_mv=20000, X0=None,
                     schur=False):
    """GMRES(m)-Proj(k) for later right-hand sides B (nrhs, V, 4, 3) with the eigenvectors V
    (k, V, 4, 3) of ``gmresdr_first_rhs`` (None: plain restarted GMRES(m)); FP64.
    Returns (X, per-rhs stats list, overall status)."""
    torch = _torch()
    L, Vol = _lattice(L)
    U = _links(links, Vol)
    Bt = _spinors(B, Vol, "B")
    X = torch.zeros_like(Bt) if X0 is None else _spinors(X0, Vol, "X0").clone()
    if X.shape != Bt.shape:
        raise ValueError("X0 must match B")
    if not (2 <= int(m) <= 128):
        raise ValueError("m must be in 2..128")
    if V is not None:
        Vd = _spinors(V, Vol, "V")
        if Vd.shape[0] > 128:
            raise ValueError("at most 128 eigenvectors")
        vp, k = Vd.data_ptr(), Vd.shape[0]
    else:
        Vd, vp, k = None, None, 0
    for t in (Bt, X) + ((Vd,) if Vd is not None else ()):
        if t.device != U.device:
            raise ValueError("all tensors must be on the links' device")
    nrhs = Bt.shape[0]
    stats = (Stats * nrhs)()
    h = _ctx(U.device)
    op = _operator(L, U, kappa, mu, schur)
    st = _abi.load().gmres_proj_solve(h, ctypes.byref(op), vp, int(k), Bt.data_ptr(), X.data_ptr(),
                                      nrhs, int(m), float(tol), int(max_mv), stats)
    _check(st, h, ok=(0, 1))
    return X.reshape(B.shape), [s.as_dict() for s in stats], st


def link_force(L, links, kappa, lam, x, kind="su3"):
    """kind 'su3': real (4, V, 8) derivatives along U -> exp(i theta T_a) U;
    kind 'complex': complex (4, V, 3, 3) gradient G with dL = Re sum conj(G) dU."""
    torch = _torch()
    L, Vol = _lattice(L)
    U = _links(links, Vol)
    lt = _spinors(lam, Vol, "lambda")
    xt = _spinors(x, Vol, "x")
    if lt.shape != xt.shape:
        raise ValueError("lambda and x must have the same shape")
    if kind == "su3":
        F = torch.empty((4, Vol, 8), dtype=torch.float64, device=U.device)
        kd = 0
    elif kind == "complex":
        F = torch.empty((4, Vol, 3, 3), dtype=torch.complex128, device=U.device)
        kd = 1
    else:
        raise ValueError("kind must be 'su3' or 'complex'")
    h = _ctx(U.device)
    op = _operator(L, U, kappa, 0.0)
    st = _abi.load().link_force(h, ctypes.byref(op), lt.data_ptr(), xt.data_ptr(), lt.shape[0],
                                kd, F.data_ptr())
    _check(st, h, ok=(0,))
    return F


def kappa_critical(L, links, m=48, k=16, tol=1e-10, max_mv=200000, nritz=0):
    """kappa_c = 1 / max Re lambda(H).  Returns (kappa_c, lambda (complex), eigen-residual, status),
    and with nritz > 0 also the final cycle's nritz Ritz values of largest real part (a list of
    complex, decreasing real part, the first being lambda)."""
    L, Vol = _lattice(L)
    U = _links(links, Vol)
    Larr = (ctypes.c_int32 * 4)(*L)
    kc = ctypes.c_double(0)
    lam = (ctypes.c_double * 2)()
    res = ctypes.c_double(0)
    h = _ctx(U.device)
    lib = _abi.load()
    if nritz > 0:
        rz = (ctypes.c_double * (2 * int(nritz)))()
        st = lib.kappa_critical_ritz(h, Larr, ctypes.c_void_p(U.data_ptr()), int(m), int(k),
                                     float(tol), int(max_mv), ctypes.byref(kc), lam,
                                     ctypes.byref(res), int(nritz), rz)
    else:
        st = lib.kappa_critical(h, Larr, ctypes.c_void_p(U.data_ptr()), int(m), int(k),
                                float(tol), int(max_mv), ctypes.byref(kc), lam, ctypes.byref(res))
    _check(st, h)
    out = (kc.value, complex(lam[0], lam[1]), res.value, st)
    if nritz > 0:
        out = out + ([complex(rz[2 * i], rz[2 * i + 1]) for i in range(int(nritz))],)
    return out


def geometry(L, device=None):
    """GPU-built even-odd tables (lex_of_eo (V,), nbr (8, V)) as int32 tensors."""
    torch = _torch()
    L, V = _lattice(L)
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    lex = torch.empty(V, dtype=torch.int32, device=dev)
    nbr = torch.empty((8, V), dtype=torch.int32, device=dev)
    h = _ctx(dev)
    Larr = (ctypes.c_int32 * 4)(*L)
    st = _abi.load().dbq_geometry(h, Larr, lex.data_ptr(), nbr.data_ptr())
    _check(st, h, ok=(0,))
    return lex, nbr


def geometry_host(L):
    """The same tables computed by the library's host code (no GPU needed), as numpy int32."""
    L, V = _lattice(L)
    lex = np.empty(V, dtype=np.int32)
    nbr = np.empty((8, V), dtype=np.int32)
    Larr = (ctypes.c_int32 * 4)(*L)
    PI = ctypes.POINTER(ctypes.c_int32)
    st = _abi.load().dbq_geometry_host(Larr, lex.ctypes.data_as(PI), nbr.ctypes.data_as(PI))
    if st != 0:
        raise DbqError(st, "dbq_geometry_host failed")
    return lex, nbr


def site_tile(L):
    """Tile extents (T0, T1, T2, T3) of the library's internal site order for extents L."""
    L, V = _lattice(L)
    T = (ctypes.c_int32 * 4)()
    st = _abi.load().dbq_site_tile((ctypes.c_int32 * 4)(*L), T)
    if st != 0:
        raise DbqError(st, "dbq_site_tile failed")
    return tuple(int(v) for v in T)


def tile_schedule_host(L, nchunks, order):
    """(tile, chunk) visited by each logical block of an LDS-tile Dslash launch with ``nchunks``
    chunks of right-hand sides in tile order ``order`` (0 to 3), as numpy int32 arrays."""
    L, V = _lattice(L)
    T = site_tile(L)
    nt = (L[0] // T[0]) * (L[1] // T[1]) * (L[2] // T[2]) * (L[3] // T[3])
    tile = np.empty(nt * int(nchunks), dtype=np.int32)
    chunk = np.empty(nt * int(nchunks), dtype=np.int32)
    PI = ctypes.POINTER(ctypes.c_int32)
    st = _abi.load().dbq_tile_schedule_host((ctypes.c_int32 * 4)(*L), int(nchunks), int(order),
                                            tile.ctypes.data_as(PI), chunk.ctypes.data_as(PI))
    if st != 0:
        raise DbqError(st, "dbq_tile_schedule_host failed")
    return tile, chunk


def stream_probe(src, dst, kind=0, reps=10):
    """Average milliseconds of the library's hand-written streaming kernel over ``src``/``dst``
    (device tensors of equal byte size): kind 0 copy, 1 read (dst receives per-block sums),
    2 fill dst."""
    torch = _torch()
    if not (isinstance(dst, torch.Tensor) and dst.is_cuda and dst.is_contiguous()):
        raise ValueError("dst must be a contiguous GPU tensor")
    nbytes = dst.numel() * dst.element_size()
    if kind != 2:
        if not (isinstance(src, torch.Tensor) and src.is_cuda and src.is_contiguous()):
            raise ValueError("src must be a contiguous GPU tensor")
        nbytes = src.numel() * src.element_size()
        if kind == 0 and dst.numel() * dst.element_size() < nbytes:
            raise ValueError("dst smaller than src")
        if kind == 1 and dst.numel() * dst.element_size() < 4 * 2048:
            raise ValueError("dst must hold one float per block (8 KiB)")
    h = _ctx(dst.device)
    ms = ctypes.c_double(0)
    sp = ctypes.c_void_p(src.data_ptr() if kind != 2 else 0)
    _check(_abi.load().dbq_stream_probe(h, sp, ctypes.c_void_p(dst.data_ptr()), int(nbytes),
                                        int(kind), int(reps), ctypes.byref(ms)), h, ok=(0,))
    return ms.value


def set_timing(on, device=None):
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _ctx(dev)
    # on: False/0 off, True/1 every launch, N > 1 every N-th launch of each kernel class
    _check(_abi.load().dbq_set_timing(h, int(on)), h, ok=(0,))


def reset_timing(device=None):
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _ctx(dev)
    _check(_abi.load().dbq_reset_timing(h), h, ok=(0,))


def kernel_time(kind, device=None):
    """(total ms, launches, algorithmic bytes) of the timed launches of one kernel class: 0 Dslash
    FP64, 1 Dslash FP32, 2 the FP32 BiCGStab update step."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _ctx(dev)
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    by = ctypes.c_double(0)
    _check(_abi.load().dbq_kernel_time(h, int(kind), ctypes.byref(ms), ctypes.byref(n),
                                       ctypes.byref(by)), h, ok=(0,))
    return ms.value, n.value, by.value


from .autograd import DeflatedSolve  # noqa: E402
