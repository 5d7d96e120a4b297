"""GPU parity of the batched factorisation (spike_factor_batch): systems of
one kernel configuration share every launch of the factor stage; each must
give, bitwise, the factorisation of the same system factored alone (same
kernels, same arithmetic per workgroup), and the oracle's solution."""
import numpy as np
import pytest

from gpu_util import check
from paper_1811_03559_amd import inputs

pytestmark = pytest.mark.gpu


def _solve(fac, F, trans=False):
    import torch
    B = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B, trans=trans)
    torch.cuda.synchronize()
    return B.cpu().numpy()


@pytest.mark.parametrize("k", [4, 16, 64, 160])
def test_factor_batch_equals_single_factorisations(k):
    import torch
    from paper_1811_03559_amd import spike
    sizes = [(3000 + 977 * i) * max(1, k // 32) for i in range(5)] + [2 * k + 5]   # the last one: p = 1
    systems, abs_ = [], []
    for i, n in enumerate(sizes):
        ab = inputs.band_dominant(n, k, k, inputs.rng_for(9700 + 13 * k + i), diag_mult=1.05, diag_add=0.0)
        abs_.append(ab)
        systems.append((torch.from_numpy(ab).cuda(), k, k))
    facs = spike.factor_batch(systems, nrhs_max=8)
    for (dab, _, _), ab, f in zip(systems, abs_, facs):
        n = ab.shape[0]
        F = inputs.rhs(n, 2, inputs.rng_for(n))
        X = _solve(f, F)
        Xt = _solve(f, F, trans=True)
        alone = spike.Factorization(dab, k, k, nrhs_max=8)
        assert np.array_equal(X, _solve(alone, F)), (k, n)
        assert np.array_equal(Xt, _solve(alone, F, trans=True)), (k, n)
        assert f.info()["info"] == 0
        check(ab, k, k, F, X, pivot=False)
        check(ab, k, k, F, Xt, trans=True, pivot=False)
        alone.close()
        f.close()


def test_factor_batch_mixed_configurations():
    """Different bandwidths form separate batches within one call; pivoting
    systems are factored one by one."""
    import torch
    from paper_1811_03559_amd import spike
    specs = [(20000, 8, False), (15000, 8, False), (12000, 24, False), (9000, 24, False), (8000, 8, True)]
    systems, abs_ = [], []
    for i, (n, k, _) in enumerate(specs):
        ab = inputs.band_dominant(n, k, k, inputs.rng_for(9800 + i), diag_mult=1.05, diag_add=0.0)
        abs_.append(ab)
        systems.append((torch.from_numpy(ab).cuda(), k, k))
    # one batch per option set (the binding applies opts to all): FP64 ...
    facs = spike.factor_batch(systems[:4], nrhs_max=4)
    # ... and pivoting for the last system
    facs_p = spike.factor_batch([systems[4]], nrhs_max=4, pivot=True)
    for (dab, k, _), ab, f in zip(systems[:4], abs_[:4], facs):
        F = inputs.rhs(ab.shape[0], 3, inputs.rng_for(ab.shape[0] + 1))
        X = _solve(f, F)
        alone = spike.Factorization(dab, k, k, nrhs_max=4)
        assert np.array_equal(X, _solve(alone, F))
        check(ab, k, k, F, X, pivot=False)
        alone.close()
        f.close()
    F = inputs.rhs(abs_[4].shape[0], 2, inputs.rng_for(9899))
    check(abs_[4], 8, 8, F, _solve(facs_p[0], F), pivot=True)
    facs_p[0].close()


def test_factor_batch_zero_pivot_is_per_system():
    import torch
    from paper_1811_03559_amd import spike
    k = 8
    a = inputs.band_dominant(6000, k, k, inputs.rng_for(9900), diag_mult=1.05, diag_add=0.0)
    b = inputs.band_dominant(7000, k, k, inputs.rng_for(9901), diag_mult=1.05, diag_add=0.0)
    b[:, k] = 0.0                # zero diagonal: the non-pivoting LU meets a zero pivot
    facs = spike.factor_batch([(torch.from_numpy(a).cuda(), k, k), (torch.from_numpy(b).cuda(), k, k)],
                              boost_tau=0.0)
    assert facs[0].info()["info"] == 0
    assert facs[1].info()["info"] > 0
    F = inputs.rhs(6000, 1, inputs.rng_for(9902))
    check(a, k, k, F, _solve(facs[0], F), pivot=False)
    for f in facs:
        f.close()
