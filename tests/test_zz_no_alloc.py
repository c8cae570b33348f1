"""The allocation-free operator apply (wilson_apply_noalloc, C ABI) against wilson_apply.

Both calls go through ctypes on device buffers the test allocates; the entry point under test
uses only the library's static scratch array.  Two calls in a row, the second on a smaller input,
check that the shared scratch is reused correctly, in FP64 and in FP32 (12-real links), for
A and A^dagger; an input beyond the scratch is rejected with DBQ_EINVAL before any launch."""
import ctypes

import numpy as np
import pytest

import synth
from gpuhelp import dev, host, relerr

pytestmark = pytest.mark.gpu


def _noalloc(gpu_lib, L, U, psi, kappa, mu, dagger, prec):
    import torch
    from paper_0710_1988_amd import _abi
    lib = _abi.load()
    out = torch.empty_like(psi)
    h = gpu_lib._ctx(U.device)
    op = gpu_lib._operator(L, U, kappa, mu, False)
    st = lib.wilson_apply_noalloc(h, ctypes.byref(op), ctypes.c_void_p(psi.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), int(psi.shape[0]),
                                  int(dagger), gpu_lib._prec(prec))
    torch.cuda.synchronize()
    return st, out


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-14), ("mixed", 2e-6)])
@pytest.mark.parametrize("dagger", [False, True])
def test_noalloc_apply_matches_wilson_apply_twice(gpu_lib, prec, tol, dagger):
    for L, nrhs, seed in (((8, 8, 8, 8), 3, 31), ((4, 4, 4, 6), 2, 32)):
        U = dev(synth.gauge_field(L, 0.6, seed))
        psi = dev(synth.gaussian_sources(L, nrhs, seed + 100))
        st, out = _noalloc(gpu_lib, L, U, psi, 0.131, 0.017, dagger, prec)
        assert st == 0, gpu_lib._abi.load().dbq_last_error(gpu_lib._ctx(U.device)).decode()
        ref = gpu_lib.wilson_apply(L, U, psi, 0.131, 0.017, dagger, prec)
        assert relerr(host(out), host(ref)) <= tol, (L, nrhs)


def test_noalloc_apply_rejects_inputs_beyond_its_scratch(gpu_lib):
    L = (16, 16, 16, 16)
    U = dev(synth.unit_field(L))
    psi = dev(np.zeros((2, 16 ** 4, 4, 3), complex))
    st, _ = _noalloc(gpu_lib, L, U, psi, 0.1, 0.0, False, "fp64")
    assert st == gpu_lib._abi.DBQ_EINVAL
