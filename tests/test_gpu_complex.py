"""Complex banded systems (spike_zfactor / spike_zsolve: the real 2 x 2-block
embedding on the SPIKE path) against the complex oracle (plain complex
banded elimination), for A, A^T and A^H, pivoting or not, FP64 and FP32
factors with FP64 refinement."""
import numpy as np
import pytest

import oracle
from paper_1811_03559_amd import inputs, spike

pytestmark = pytest.mark.gpu


def zdense(ab, kl, ku):
    n = ab.shape[0]
    A = np.zeros((n, n), dtype=complex)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = ab[j, ku + i - j]
    return A


def zrun(ab, kl, ku, F, trans, **opts):
    import torch
    fac = spike.ZFactorization(torch.from_numpy(ab).cuda(), kl, ku, **opts)
    B = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B, trans=trans)
    torch.cuda.synchronize()
    X = B.cpu().numpy()
    info = fac.info()
    fac.close()
    return X, info


def zcheck(ab, kl, ku, F, X, trans, kappa, X_true=None):
    Xo = oracle.zgbsv(ab, kl, ku, F, pivot=True, trans=trans)
    rr = oracle.zrelres(ab, kl, ku, X, F, trans=trans)
    agree = oracle.fwd_err(X, Xo)
    assert np.all(np.isfinite(X))
    assert rr <= 1e-13, rr
    assert agree <= 1e-11 * max(kappa, 1.0), (agree, kappa)
    if X_true is not None:
        assert oracle.fwd_err(X, X_true) <= 1e-11 * max(kappa, 1.0)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("kl,ku", [(1, 1), (2, 5), (4, 4), (0, 3)])
@pytest.mark.parametrize("trans", ["N", "T", "C"])
@pytest.mark.parametrize("pivot", [False, True])
def test_complex_grid(p, kl, ku, trans, pivot):
    n = 37 * p + 11
    ab = inputs.zband_dominant(n, kl, ku, inputs.rng_for(5100 + 97 * p + 13 * kl + ku), diag_add=1.0)
    X_true = inputs.zrhs(n, 3, inputs.rng_for(5200 + p))
    F = oracle.zgbmv(ab, kl, ku, X_true, trans=trans)
    X, info = zrun(ab, kl, ku, F, trans, p=p, pivot=pivot)
    assert info["info"] == 0
    zcheck(ab, kl, ku, F, X, trans, np.linalg.cond(zdense(ab, kl, ku), 1), X_true)


@pytest.mark.parametrize("trans", ["N", "T", "C"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_complex_wide_band(trans, precision):
    """k = 64 (the embedding has 129 sub- and superdiagonals: the MFMA block
    LU and tile engine at a window of 9 tiles), 4 partitions; FP32 factors
    refine to the bar in FP64."""
    n, k, p = 2400, 64, 4
    ab = inputs.zband_dominant(n, k, k, inputs.rng_for(5300), diag_mult_range=(1.01, 1.5))
    X_true = inputs.zrhs(n, 2, inputs.rng_for(5301))
    F = oracle.zgbmv(ab, k, k, X_true, trans=trans)
    X, info = zrun(ab, k, k, F, trans, p=p, precision=precision)
    assert info["info"] == 0
    if precision == "mixed":
        assert 1 <= info["refine_iters"] <= 6 and info["berr"] <= 1e-13, info
    zcheck(ab, k, k, F, X, trans, np.linalg.cond(zdense(ab, k, k), 1), X_true)


def test_complex_not_dominant_pivoting():
    """No diagonal dominance: pivoting factors of the embedding, two
    partitions, against the oracle's complex partial pivoting."""
    n, k = 900, 6
    ab = inputs.zband_dominant(n, k, k, inputs.rng_for(5400), diag_mult=0.0, diag_add=0.3)
    F = inputs.zrhs(n, 2, inputs.rng_for(5401))
    for trans in ("N", "T", "C"):
        X, info = zrun(ab, k, k, F, trans, p=2, pivot=True)
        assert info["info"] == 0
        zcheck(ab, k, k, F, X, trans, np.linalg.cond(zdense(ab, k, k), 1))


def test_complex_zero_pivot_info_and_untouched_b():
    """A zero complex diagonal entry with boosting off: info names the real
    row 2j + 1 of the embedding (complex row j + 1), and B is untouched."""
    n, k, p = 400, 2, 4
    ab = inputs.zband_dominant(n, k, k, inputs.rng_for(5500), diag_add=1.0)
    j = 100                                   # first row of partition 1 of the 800-row embedding
    ab[j, k] = 0.0
    F = inputs.zrhs(n, 1, inputs.rng_for(5501))
    X, info = zrun(ab, k, k, F, "N", p=p, boost_tau=0.0)
    assert info["info"] == 2 * j + 1 and (info["info"] + 1) // 2 == j + 1, info
    assert np.array_equal(X, F)


def test_complex_real_matrix_matches_real_solver():
    """A complex band with zero imaginary parts and a complex right-hand side
    solves like two real systems: the same as the real solver on the real
    and imaginary parts (to rounding)."""
    import torch
    n, k, p = 3000, 5, 5
    ar = inputs.band_dominant(n, k, k, inputs.rng_for(5600), diag_add=1.0)
    F = inputs.zrhs(n, 1, inputs.rng_for(5601))
    Xz, _ = zrun(ar.astype(complex), k, k, F, "N", p=p)
    fac = spike.Factorization(torch.from_numpy(ar).cuda(), k, k, p=p)
    B = torch.from_numpy(np.stack([F.real[0], F.imag[0]])).cuda()
    fac.solve_(B)
    Xr = B.cpu().numpy()
    fac.close()
    assert oracle.fwd_err(Xz, Xr[0] + 1j * Xr[1]) <= 1e-13
