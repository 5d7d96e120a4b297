"""GPU checks of the C-ABI's numerical-status contract: a singular interface
system reports info = n + j (j the 1-based merge between partitions j and
j+1), a zero pivot reports its global row, and a solve on a failed
factorisation leaves dB bitwise untouched, refined or not."""
import numpy as np
import pytest

from gpu_util import run
from paper_1811_03559_amd import inputs

pytestmark = pytest.mark.gpu


def singular_interface_band(copies=1):
    """p = 2 blocks of the identity (nonsingular leaves) coupled so that the
    whole matrix is singular: A(m-1, m) = A(m, m-1) = 1 makes rows m-1 and m
    equal.  By det(E_J) = det(A_J) / (det A_L det A_R) (S_J = diag(A_i)^{-1}
    A_J with S^[l] = D^[l] S^[l+1]) the interface system is singular, and
    its Schur complement 1 - W_t V_b = 1 - 1 * 1 is exactly zero in floating
    point.  kl = ku = 1, n = 4 * copies, partitions of 2 * copies rows."""
    n = 4 * copies
    m = n // 2
    A = np.eye(n)
    A[m - 1, m] = 1.0
    A[m, m - 1] = 1.0
    ab = np.zeros((n, 3))
    for j in range(n):
        for i in range(max(0, j - 1), min(n, j + 2)):
            ab[j, 1 + i - j] = A[i, j]
    return ab, A


@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("copies", [1, 8])
def test_singular_interface_reports_info_and_leaves_b(pivot, trans, copies):
    ab, A = singular_interface_band(copies)
    n = ab.shape[0]
    assert abs(np.linalg.det(A)) == 0.0
    m = n // 2
    assert abs(np.linalg.det(A[:m, :m])) == 1.0 and abs(np.linalg.det(A[m:, m:])) == 1.0
    F = inputs.rhs(n, 2, inputs.rng_for(3))
    X, info, _ = run(ab, 1, 1, F, trans=trans, p=2, pivot=pivot)
    assert info["info"] == n + 1, info
    assert np.array_equal(X, F)


@pytest.mark.parametrize("mode", ["pivot_refine", "noboost_refine", "mixed_noboost"])
@pytest.mark.parametrize("trans", [False, True])
def test_failed_factorisation_refined_solve_leaves_b(mode, trans):
    """A zero pivot that stops the factorisation (non-pivoting without
    boosting, FP64 or FP32) or a zero pivot column under partial pivoting
    (an all-zero column): with refinement on, the solve still leaves dB
    bitwise equal to F and info reports the row."""
    n, k, p = 400, 3, 4
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(5))
    s = 100                               # first row of partition 1
    if mode == "pivot_refine":
        ab[s, :] = 0.0                    # column s of A is zero: singular for any pivoting
        opts = dict(pivot=True, max_refine=3)
    elif mode == "noboost_refine":
        ab[s, k] = 0.0                    # A(s, s) = 0, leading pivot of partition 1
        opts = dict(pivot=False, boost_tau=0.0, max_refine=3)
    else:
        ab[s, k] = 0.0
        opts = dict(pivot=False, boost_tau=0.0, precision="mixed")
    F = inputs.rhs(n, 3, inputs.rng_for(6))
    X, info, _ = run(ab, k, k, F, trans=trans, p=p, **opts)
    assert info["info"] == s + 1, info
    assert np.array_equal(X, F)
    assert info["refine_iters"] == 0

