"""Pins for the FP64 oracle against things other than itself: LAPACK (via
numpy/scipy), closed-form inverses of Toeplitz tridiagonal matrices, dense
reconstruction of the pivoted factors, the exact 1-norm condition number, and
the paper's load-balancing closed forms and table."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1811_03559_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_from_band(ab, kl, ku):
    n = ab.shape[0]
    A = np.zeros((n, n))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = ab[j, ku + i - j]
    return A


def band_from_dense(A, kl, ku):
    n = A.shape[0]
    ab = np.zeros((n, kl + ku + 1))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            ab[j, ku + i - j] = A[i, j]
    return ab


def rand_band(n, kl, ku, seed, dominant):
    rng = inputs.rng_for(seed)
    if dominant:
        return inputs.band_dominant(n, kl, ku, rng, diag_mult=1.0, diag_add=1.0)
    return inputs.band_gaussian_rowscaled(n, kl, ku, rng, log10_range=(0.0, 0.0))


# ---------------------------------------------------------------- products

@pytest.mark.parametrize("kl,ku", [(0, 0), (1, 2), (3, 1), (5, 5)])
@pytest.mark.parametrize("trans", [False, True])
def test_gbmv_matches_dense_product(kl, ku, trans):
    n = 37
    ab = rand_band(n, kl, ku, 11 + kl + 7 * ku, dominant=False)
    A = dense_from_band(ab, kl, ku)
    X = inputs.rhs(n, 3, inputs.rng_for(5))
    Y = oracle.gbmv(ab, kl, ku, X, trans=trans)
    ref = (A.T if trans else A) @ X.T
    np.testing.assert_allclose(Y, ref.T, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- solves vs LAPACK

CASES = [(kl, ku) for kl in range(0, 6) for ku in range(0, 6) if (kl + ku) % 2 == 0 or kl == 5]


@pytest.mark.parametrize("kl,ku", CASES)
@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
def test_solve_matches_lapack_dense(kl, ku, pivot, trans):
    n = 48
    ab = rand_band(n, kl, ku, 100 + 10 * kl + ku, dominant=not pivot)
    A = dense_from_band(ab, kl, ku)
    F = inputs.rhs(n, 2, inputs.rng_for(7))
    X = oracle.gbsv(ab, kl, ku, F, pivot=pivot, trans=trans)
    ref = np.linalg.solve(A.T if trans else A, F.T).T
    kappa = np.linalg.cond(A, 1)
    assert oracle.fwd_err(X, ref) <= 1e-14 * kappa * n


@pytest.mark.parametrize("kl,ku", [(8, 8), (3, 11), (13, 2)])
def test_solve_matches_scipy_gbsv(kl, ku):
    n = 3000
    # far from diagonally dominant (diagonal = a tenth of the row sum): rows get exchanged
    ab = inputs.band_dominant(n, kl, ku, inputs.rng_for(7 + kl), diag_mult=0.1)
    F = inputs.rhs(n, 3, inputs.rng_for(8))
    X = oracle.gbsv(ab, kl, ku, F, pivot=True)
    _, _, ipiv = oracle.gbtrf(ab, kl, ku, pivot=True)
    assert np.count_nonzero(ipiv != np.arange(n)) > n // 10
    # scipy wants the band as (kl+ku+1, n) with the same row convention
    ref = sla.solve_banded((kl, ku), ab.T.copy(), F.T.copy()).T
    kappa = oracle.cond1(ab, kl, ku)
    assert oracle.fwd_err(X, ref) <= 1e-14 * kappa


def test_pivoting_needed_case():
    """A zero leading entry: the non-pivoting elimination reports info=1, the
    pivoting one solves it exactly as LAPACK does."""
    A = np.array([[0.0, 2.0, 0.0], [1.0, 1.0, 3.0], [0.0, 4.0, 1.0]])
    ab = band_from_dense(A, 1, 1)
    F = np.array([[2.0, 5.0, 5.0]])
    with pytest.raises(ZeroDivisionError):
        oracle.gbsv(ab, 1, 1, F, pivot=False)
    X = oracle.gbsv(ab, 1, 1, F, pivot=True)
    np.testing.assert_allclose(X[0], np.linalg.solve(A, F[0]), rtol=1e-15)


def test_degenerate_sizes():
    # n = 1
    ab = np.array([[4.0]])
    np.testing.assert_allclose(oracle.gbsv(ab, 0, 0, np.array([[2.0]])), [[0.5]])
    # diagonal matrix: X = F / d exactly
    d = np.arange(1.0, 11.0)
    X = oracle.gbsv(d[:, None], 0, 0, np.ones((1, 10)))
    np.testing.assert_array_equal(X[0], 1.0 / d)
    # band wider than the matrix
    ab = rand_band(6, 8, 8, 3, dominant=True)
    A = dense_from_band(ab, 8, 8)
    F = inputs.rhs(6, 1, inputs.rng_for(1))
    np.testing.assert_allclose(oracle.gbsv(ab, 8, 8, F), np.linalg.solve(A, F.T).T, rtol=1e-12)


# ---------------------------------------------------------------- closed forms

def usmani_inverse(m, b, a, c):
    """Inverse of the Toeplitz tridiagonal tridiag(b, a, c) of order m (b on the
    sub-diagonal, c on the super-diagonal), Usmani (1994)."""
    dt = np.result_type(a, b, c, float)    # complex entries give a complex inverse
    theta = np.zeros(m + 2, dtype=dt)
    theta[0], theta_m1 = 1.0, 0.0          # theta_0 = 1, theta_{-1} = 0
    theta[1] = a * theta[0] - b * c * theta_m1
    for i in range(2, m + 1):
        theta[i] = a * theta[i - 1] - b * c * theta[i - 2]
    phi = np.zeros(m + 3, dtype=dt)        # phi_{m+1} = 1, phi_{m+2} = 0
    phi[m + 1], phi[m + 2] = 1.0, 0.0
    for i in range(m, 0, -1):
        phi[i] = a * phi[i + 1] - b * c * phi[i + 2]

    def th(i):
        return theta_m1 if i == -1 else theta[i]

    T = np.zeros((m, m), dtype=dt)
    for i in range(1, m + 1):
        for j in range(1, m + 1):
            if i <= j:
                T[i - 1, j - 1] = (-1) ** (i + j) * c ** (j - i) * th(i - 1) * phi[j + 1] / theta[m]
            else:
                T[i - 1, j - 1] = (-1) ** (i + j) * b ** (i - j) * th(j - 1) * phi[i + 1] / theta[m]
    return T


@pytest.mark.parametrize("b,a,c", [(-1.0, 3.0, 0.5), (0.7, -2.5, 1.1), (1.0, 4.0, 1.0)])
@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
def test_toeplitz_tridiagonal_closed_form(b, a, c, pivot, trans):
    m = 40
    ab = np.zeros((m, 3))
    ab[:, 0], ab[:, 1], ab[:, 2] = c, a, b      # ku=1: slot 0 super, 1 diag, 2 sub
    ab[0, 0] = 0.0
    ab[m - 1, 2] = 0.0
    Tinv = usmani_inverse(m, b, a, c)
    X = oracle.gbsv(ab, 1, 1, np.eye(m), pivot=pivot, trans=trans)   # rows = columns of inverse
    ref = Tinv.T if trans else Tinv
    np.testing.assert_allclose(X.T, ref, rtol=1e-12, atol=1e-14)


def test_second_difference_closed_form():
    """tridiag(-1, 2, -1): (T^{-1})_{ij} = min(i,j) (m+1-max(i,j)) / (m+1)."""
    m = 50
    ab = np.zeros((m, 3))
    ab[:, 0], ab[:, 1], ab[:, 2] = -1.0, 2.0, -1.0
    ab[0, 0] = ab[m - 1, 2] = 0.0
    X = oracle.gbsv(ab, 1, 1, np.eye(m), pivot=False)
    i = np.arange(1, m + 1)[:, None]
    j = np.arange(1, m + 1)[None, :]
    ref = np.minimum(i, j) * (m + 1 - np.maximum(i, j)) / (m + 1)
    np.testing.assert_allclose(X, ref, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- manufactured solutions

@pytest.mark.parametrize("pivot", [False, True])
def test_manufactured_solution_cfg0_recipe(pivot):
    ab, kl, ku, X_true = inputs.cfg0()
    F = oracle.gbmv(ab, kl, ku, X_true)
    X = oracle.gbsv(ab, kl, ku, F, pivot=pivot)
    kappa = oracle.cond1(ab, kl, ku)
    assert kappa < 100
    assert oracle.fwd_err(X, X_true) <= 1e-11 * kappa
    assert oracle.relres(ab, kl, ku, X, F) <= 1e-15


def test_manufactured_solution_rowscaled_pivoting():
    n, k = 2000, 6
    rng = inputs.rng_for(42)
    ab = inputs.band_gaussian_rowscaled(n, k, k, rng)
    X_true = inputs.rhs(n, 2, rng)
    F = oracle.gbmv(ab, k, k, X_true)
    X = oracle.gbsv(ab, k, k, F, pivot=True)
    kappa = oracle.cond1(ab, k, k)
    assert kappa > 1e6                       # ill-conditioned on purpose
    assert oracle.fwd_err(X, X_true) <= 1e-11 * kappa
    assert oracle.relres(ab, k, k, X, F) <= 1e-13


# ---------------------------------------------------------------- pivoting invariants

@pytest.mark.parametrize("kl,ku", [(1, 1), (2, 3), (4, 1), (3, 3)])
def test_pivot_invariants_and_reconstruction(kl, ku):
    """0 <= ipiv_j - j <= kl (a row moves at most kl places), U has at most
    kl+ku superdiagonals, and replaying the interchanges and multipliers
    reconstructs A."""
    n = 30
    ab = rand_band(n, kl, ku, 300 + kl * 7 + ku, dominant=False)
    A = dense_from_band(ab, kl, ku)
    info, w, ipiv = oracle.gbtrf(ab, kl, ku, pivot=True)
    assert info == 0
    j = np.arange(n)
    assert np.all(ipiv >= j) and np.all(ipiv - j <= kl)
    uw = kl + ku
    U = np.zeros((n, n))
    Lcols = np.zeros((n, n))
    for c in range(n):
        for r in range(max(0, c - uw), c + 1):
            U[r, c] = w[c, uw + r - c]
        for r in range(c + 1, min(n, c + kl + 1)):
            Lcols[r, c] = w[c, uw + r - c]
    # A = P_0 L_0 P_1 L_1 ... P_{n-1} L_{n-1} U with the elementary factors
    M = U.copy()
    for c in range(n - 1, -1, -1):
        Lc = np.eye(n)
        Lc[:, c] += Lcols[:, c]
        M = Lc @ M
        P = np.eye(n)
        P[[c, ipiv[c]]] = P[[ipiv[c], c]]
        M = P @ M
    np.testing.assert_allclose(M, A, rtol=1e-12, atol=1e-12)


def test_nonpivot_factor_is_plain_lu():
    n, kl, ku = 25, 3, 2
    ab = rand_band(n, kl, ku, 9, dominant=True)
    A = dense_from_band(ab, kl, ku)
    info, w, _ = oracle.gbtrf(ab, kl, ku, pivot=False)
    assert info == 0
    L = np.eye(n)
    U = np.zeros((n, n))
    for c in range(n):
        for r in range(max(0, c - ku), c + 1):
            U[r, c] = w[c, ku + r - c]
        for r in range(c + 1, min(n, c + kl + 1)):
            L[r, c] = w[c, ku + r - c]
    np.testing.assert_allclose(L @ U, A, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- norms, residual, condition

def test_norms_and_relres_against_dense():
    n, kl, ku = 40, 4, 2
    ab = rand_band(n, kl, ku, 77, dominant=False)
    A = dense_from_band(ab, kl, ku)
    assert oracle.gbnorm(ab, kl, ku, "inf") == pytest.approx(np.abs(A).sum(axis=1).max(), rel=1e-15)
    assert oracle.gbnorm(ab, kl, ku, "one") == pytest.approx(np.abs(A).sum(axis=0).max(), rel=1e-15)
    X = inputs.rhs(n, 2, inputs.rng_for(3))
    F = inputs.rhs(n, 2, inputs.rng_for(4))
    R = F.T - A @ X.T
    ref = max(np.abs(R[:, c]).max() / (np.abs(A).sum(axis=1).max() * np.abs(X[c]).max())
              for c in range(2))
    assert oracle.relres(ab, kl, ku, X, F) == pytest.approx(ref, rel=1e-12)
    Rt = F.T - A.T @ X.T
    ref_t = max(np.abs(Rt[:, c]).max() / (np.abs(A).sum(axis=0).max() * np.abs(X[c]).max())
                for c in range(2))
    assert oracle.relres(ab, kl, ku, X, F, trans=True) == pytest.approx(ref_t, rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_condition_estimate_against_exact(seed):
    n, k = 60, 3
    ab = inputs.band_gaussian_rowscaled(n, k, k, inputs.rng_for(seed), log10_range=(-2, 2))
    A = dense_from_band(ab, k, k)
    exact = np.linalg.norm(A, 1) * np.linalg.norm(np.linalg.inv(A), 1)
    est = oracle.cond1(ab, k, k)
    assert est <= exact * (1 + 1e-10)
    assert est >= exact / 3.0


# ---------------------------------------------------------------- load-balancing closed forms

def test_r13_limits():
    for K in (0.5, 4.0 / 3.0, 2.0):
        assert oracle.r13(K, 0.0) == pytest.approx(1.0 + 1.5 * K, rel=1e-15)   # eq. ratiof (x2)
        assert oracle.r13(K, 1e9) == pytest.approx(2.0, rel=1e-6)              # eq. ratios
    # the paper's factor-optimal ratios for its machine: R13 = 3, R12 = 1.5 at K = 4/3
    assert oracle.r13(4.0 / 3.0, 0.0) == pytest.approx(3.0, rel=1e-15)


def test_r13_reproduces_paper_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "tab_ratios.txt"))
            if l.strip() and not l.startswith("#")]
    for nrhs, r13_paper, r12_paper in rows:
        r = oracle.r13(4.0 / 3.0, float(nrhs) / 160.0)
        assert abs(r - float(r13_paper)) <= 0.11
        assert abs(r / 2 - float(r12_paper)) <= 0.06


# ---------------------------------------------------------------- one factorisation, two solves

@pytest.mark.parametrize("kl,ku", [(0, 0), (2, 5), (5, 2), (4, 4)])
@pytest.mark.parametrize("pivot", [False, True])
def test_gbsv_nt_matches_separate_solves_and_dense(kl, ku, pivot):
    """orc_gbsv_nt (the CPU-baseline routine: one factorisation, then the A and
    A^T solves) returns bitwise what two separate orc_gbsv calls return, and
    both solutions agree with dense LAPACK solves of A and A^T."""
    n = 53
    ab = rand_band(n, kl, ku, 400 + 10 * kl + ku, dominant=not pivot)
    A = dense_from_band(ab, kl, ku)
    F = inputs.rhs(n, 3, inputs.rng_for(17))
    X, Xt = oracle.gbsv_nt(ab, kl, ku, F, pivot=pivot)
    np.testing.assert_array_equal(X, oracle.gbsv(ab, kl, ku, F, pivot=pivot))
    np.testing.assert_array_equal(Xt, oracle.gbsv(ab, kl, ku, F, pivot=pivot, trans=True))
    kappa = np.linalg.cond(A, 1)
    assert oracle.fwd_err(X, np.linalg.solve(A, F.T).T) <= 1e-14 * kappa * n
    assert oracle.fwd_err(Xt, np.linalg.solve(A.T, F.T).T) <= 1e-14 * kappa * n
    # off the diagonal A is not symmetric, so the two solutions differ: a
    # routine that returned the same solve for both would fail here
    if kl + ku > 0:
        assert oracle.fwd_err(X, Xt) > 1e-6


def test_gbsv_nt_degenerate():
    """n = 0 is a no-op; a zero pivot is reported and leaves both right-hand
    sides untouched."""
    X, Xt = oracle.gbsv_nt(np.zeros((0, 3)), 1, 1, np.zeros((2, 0)))
    assert X.shape == (2, 0) and Xt.shape == (2, 0)
    ab = band_from_dense(np.diag([1.0, 0.0, 2.0]), 1, 1)
    with pytest.raises(ZeroDivisionError):
        oracle.gbsv_nt(ab, 1, 1, np.ones((1, 3)), pivot=False)


# ---------------------------------------------------------------- transpose via explicit A^T

def transpose_band(ab, kl, ku):
    """Band storage of A^T (kl and ku swapped), built entry by entry."""
    n = ab.shape[0]
    at = np.zeros((n, kl + ku + 1))
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            # A(i, j) becomes A^T(j, i), stored in column i with ku' = kl
            at[i, kl + j - i] = ab[j, ku + i - j]
    return at


@pytest.mark.parametrize("kl,ku", [(1, 1), (2, 5), (5, 2), (0, 3), (3, 0), (6, 6)])
@pytest.mark.parametrize("pivot", [False, True])
def test_transpose_solve_against_explicit_transpose(kl, ku, pivot):
    """The transpose solve (U^T then L^T with the interchanges undone) equals
    a fresh factorisation of A^T, stored as a band with kl and ku swapped,
    followed by the plain non-transpose solve."""
    n = 211
    ab = rand_band(n, kl, ku, 900 + 10 * kl + ku, dominant=not pivot)
    at = transpose_band(ab, kl, ku)
    np.testing.assert_array_equal(dense_from_band(at, ku, kl), dense_from_band(ab, kl, ku).T)
    F = inputs.rhs(n, 2, inputs.rng_for(23))
    Xt = oracle.gbsv(ab, kl, ku, F, pivot=pivot, trans=True)
    Xe = oracle.gbsv(at, ku, kl, F, pivot=pivot)
    kappa = oracle.cond1(ab, kl, ku)
    assert oracle.fwd_err(Xt, Xe) <= 1e-14 * kappa * n
    assert oracle.relres(ab, kl, ku, Xt, F, trans=True) <= 1e-14
    assert oracle.relres(at, ku, kl, Xe, F) <= 1e-14


def test_singular_coupling_makes_elimination_meet_a_zero_pivot():
    """Two identity blocks coupled by A(m-1, m) = A(m, m-1) = 1 (rows m-1 and
    m equal): the leaves are nonsingular but A is not, and partial-pivoting
    elimination meets an exactly zero pivot (the matrix the GPU contract test
    uses for a singular interface system)."""
    for copies in (1, 8):
        n = 4 * copies
        m = n // 2
        A = np.eye(n)
        A[m - 1, m] = A[m, m - 1] = 1.0
        ab = band_from_dense(A, 1, 1)
        for pivot in (False, True):
            with pytest.raises(ZeroDivisionError):
                oracle.gbsv(ab, 1, 1, np.ones((1, n)), pivot=pivot)


@pytest.mark.parametrize("kl,ku", [(0, 2), (3, 3), (5, 1)])
@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
def test_gbtrf_then_gbtrs_is_gbsv(kl, ku, pivot, trans):
    """Factor once (orc_gbtrf) and solve with the stored factors (orc_gbtrs):
    bitwise the one-call solve, and the dense solution to rounding."""
    n = 77
    ab = rand_band(n, kl, ku, 50 + kl + 3 * ku, dominant=not pivot)
    F = inputs.rhs(n, 2, inputs.rng_for(51))
    info, w, ipiv = oracle.gbtrf(ab, kl, ku, pivot=pivot)
    assert info == 0
    X = oracle.gbtrs(w, ipiv, kl, ku, F, pivot=pivot, trans=trans)
    np.testing.assert_array_equal(X, oracle.gbsv(ab, kl, ku, F, pivot=pivot, trans=trans))
    A = dense_from_band(ab, kl, ku)
    ref = np.linalg.solve(A.T if trans else A, F.T).T
    assert oracle.fwd_err(X, ref) <= 1e-14 * np.linalg.cond(A, 1) * n


# ---------------------------------------------------------------- complex bands

def zdense_from_band(ab, kl, ku):
    n = ab.shape[0]
    A = np.zeros((n, n), dtype=complex)
    for j in range(n):
        for i in range(max(0, j - ku), min(n, j + kl + 1)):
            A[i, j] = ab[j, ku + i - j]
    return A


def zrand_band(n, kl, ku, seed, dominant):
    rng = inputs.rng_for(seed)
    if dominant:
        return inputs.zband_dominant(n, kl, ku, rng, diag_mult=1.0, diag_add=1.0)
    return inputs.zband_dominant(n, kl, ku, rng, diag_mult=0.0, diag_add=0.3)   # no dominance


@pytest.mark.parametrize("kl,ku", [(0, 0), (1, 2), (3, 1), (4, 4)])
@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", ["N", "T", "C"])
def test_zgbsv_matches_dense_complex_solve(kl, ku, pivot, trans):
    n = 41
    ab = zrand_band(n, kl, ku, 300 + 10 * kl + ku, dominant=not pivot)
    A = zdense_from_band(ab, kl, ku)
    op = {"N": A, "T": A.T, "C": A.conj().T}[trans]
    F = inputs.zrhs(n, 2, inputs.rng_for(13))
    X = oracle.zgbsv(ab, kl, ku, F, pivot=pivot, trans=trans)
    ref = np.linalg.solve(op, F.T).T
    kappa = np.linalg.cond(A, 1)
    assert oracle.fwd_err(X, ref) <= 1e-14 * kappa * n
    np.testing.assert_allclose(oracle.zgbmv(ab, kl, ku, X, trans=trans), F, atol=1e-10 * np.abs(F).max())
    assert oracle.zrelres(ab, kl, ku, X, F, trans=trans) <= 1e-14


@pytest.mark.parametrize("trans", ["N", "T", "C"])
def test_zgbmv_and_zrelres_against_dense(trans):
    n, kl, ku = 37, 3, 2
    ab = zrand_band(n, kl, ku, 77, dominant=True)
    A = zdense_from_band(ab, kl, ku)
    op = {"N": A, "T": A.T, "C": A.conj().T}[trans]
    X = inputs.zrhs(n, 3, inputs.rng_for(78))
    np.testing.assert_allclose(oracle.zgbmv(ab, kl, ku, X, trans=trans), (op @ X.T).T, rtol=1e-13, atol=1e-13)
    F = (op @ X.T).T + 1e-3 * inputs.zrhs(n, 3, inputs.rng_for(79))
    r = F - (op @ X.T).T
    rel = max(np.abs(r[c]).max() / (np.abs(op).sum(axis=1).max() * np.abs(X[c]).max()) for c in range(3))
    assert abs(oracle.zrelres(ab, kl, ku, X, F, trans=trans) - rel) <= 1e-12 * rel


@pytest.mark.parametrize("trans", ["N", "T", "C"])
def test_zgbsv_complex_toeplitz_closed_form(trans):
    """Usmani's inverse holds over the complex numbers: tridiag(b, a, c) with
    complex entries, the oracle's solution against it."""
    m = 30
    b, a, c = 0.7 - 0.4j, 3.0 + 1.5j, -0.5 + 0.9j
    Tinv = usmani_inverse(m, b, a, c)
    ab = np.zeros((m, 3), dtype=complex)
    ab[:, 0], ab[:, 1], ab[:, 2] = c, a, b        # ku = kl = 1: A(j-1, j) = c, A(j+1, j) = b
    ab[0, 0] = 0
    ab[-1, 2] = 0
    F = inputs.zrhs(m, 2, inputs.rng_for(80))
    op_inv = {"N": Tinv, "T": Tinv.T, "C": Tinv.conj().T}[trans]
    X = oracle.zgbsv(ab, 1, 1, F, pivot=False, trans=trans)
    np.testing.assert_allclose(X, (op_inv @ F.T).T, rtol=1e-12, atol=1e-12)
