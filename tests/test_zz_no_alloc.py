"""The allocation-free factorisation (spike_factor_scratch: the library's own
per-GPU scratch array as the workspace) against spike_factor with a
caller-allocated workspace, through the C ABI: two calls in a row on one
GPU, the second with a smaller system, each solved (N and T) and compared
bitwise with the workspace path and against the oracle's bars."""
import ctypes

import numpy as np
import pytest

from gpu_util import check
from paper_1811_03559_amd import inputs, spike

pytestmark = pytest.mark.gpu


def _solve(fac, F, trans):
    import torch
    B = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B, trans=trans)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def test_scratch_factor_matches_workspace_factor_twice():
    import torch
    assert spike.lib().spike_scratch_capacity() == 64 << 20
    cases = [(60000, 16, 16, 4), (9001, 5, 3, 2)]      # the second smaller
    for n, k, p, nrhs in cases:
        opts = dict(p=p, nrhs_max=4)
        assert spike.workspace_size(n, k, k, **opts) <= spike.lib().spike_scratch_capacity()
        ab = inputs.band_dominant(n, k, k, inputs.rng_for(7700 + n), diag_mult=1.05, diag_add=0.0)
        F = inputs.rhs(n, nrhs, inputs.rng_for(7800 + n))
        dab = torch.from_numpy(ab).cuda()
        ref = spike.Factorization(dab, k, k, **opts)
        sc = spike.Factorization(dab, k, k, workspace="scratch", **opts)
        assert sc.ws is None
        for trans in (False, True):
            X_ref = _solve(ref, F, trans)
            X = _solve(sc, F, trans)
            assert np.array_equal(X, X_ref), (n, trans)
            check(ab, k, k, F, X, trans=trans, pivot=False)
        assert sc.info()["info"] == 0
        sc.close()
        ref.close()


def test_scratch_factor_rejects_systems_beyond_its_capacity():
    import torch
    L = spike.lib()
    n, k, p = 400000, 16, 64
    o = spike.make_opts(p=p)
    need = spike.workspace_size(n, k, k, p=p)
    assert need > L.spike_scratch_capacity()
    dab = torch.zeros((n, 2 * k + 1), dtype=torch.float64, device="cuda")
    h = ctypes.c_void_p()
    assert L.spike_factor_scratch(n, k, k, ctypes.c_void_p(dab.data_ptr()), 2 * k + 1, ctypes.byref(o), None,
                                  ctypes.byref(h)) == -7
    assert h.value is None
