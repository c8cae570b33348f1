"""Helpers shared by the GPU parity tests: move seeded synthetic inputs to the device and back."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def projector_distance(V1, V2):
    """|| P1 - P2 ||_2 for the orthogonal projectors onto span(V1), span(V2) (columns)."""
    Q1, _ = np.linalg.qr(V1)
    Q2, _ = np.linalg.qr(V2)
    s = np.linalg.svd(Q1.conj().T @ Q2, compute_uv=False)
    s = np.clip(s, 0, 1)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2))) if len(s) else 0.0


def same_eigenvalues(a, b, rtol=1e-6, atol=1e-9):
    """a and b hold the same values up to the tolerance, in any order: the pairing that
    minimises the total distance matches every value within rtol |b| + atol.  (Members of a
    complex-conjugate pair share modulus and real part, so their order in a sorted list is
    decided by rounding.)"""
    from scipy.optimize import linear_sum_assignment
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    if a.shape != b.shape:
        return False
    d = np.abs(a[:, None] - b[None, :])
    i, j = linear_sum_assignment(d)
    return bool(np.all(d[i, j] <= rtol * np.abs(b[j]) + atol))

