"""CPU replay of the workgroup kernel path under AddressSanitizer.

The partial-pivoting leaf kernels (factor with tips, D stage, retrieval, Z
sweeps, transposed D stage), the generic interface-merge kernels and the
transpose G-tip kernel are compiled for the host (tests/hostemu) and run with
every workgroup as 256 host threads.  Every workspace region and every
dynamic LDS buffer is its own allocation of the size the planner reserves,
so an index outside its region stops the run.  The results must match the
oracle to the GPU parity bars.

The first cases are the exact inputs of the pivoting two-partition wide-band
GPU parity cases (kl = ku = 200 and 160, NB = 16 panels, dense L panel tiles,
the reversed-frame last partition)."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1811_03559_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "hostemu"))
import replay  # noqa: E402


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return replay.build(str(tmp_path_factory.mktemp("hostemu")))


def _wide_band_case(k, p, nrhs=5):
    # the inputs of test_gpu_parity.test_wide_band(k, p)
    n = p * (2 * k + 37) + 3
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(9000 + k + p), diag_mult=1.05, diag_add=0.0)
    F = inputs.rhs(n, nrhs, inputs.rng_for(k * p))
    return ab, k, k, F


def _check(ab, kl, ku, F, X, trans):
    Xo = oracle.gbsv(ab, kl, ku, F, pivot=True, trans=trans)
    kappa = oracle.cond1(ab, kl, ku)
    assert oracle.relres(ab, kl, ku, X, F, trans=trans) <= 1e-13
    assert oracle.fwd_err(X, Xo) <= 1e-11 * max(kappa, 1.0)


@pytest.mark.parametrize("k", [200, 160])
@pytest.mark.parametrize("trans", [False, True])
def test_pivoting_two_partition_wide_band(exe, k, trans):
    ab, kl, ku, F = _wide_band_case(k, 2)
    info, X = replay.run(exe, ab, kl, ku, F, p=2, pivot=True, trans=trans)
    assert info == 0
    _check(ab, kl, ku, F, X, trans)


@pytest.mark.parametrize("n,kl,ku,p,mult", [(600, 8, 8, 3, 0.3), (900, 5, 2, 5, 0.5), (700, 40, 17, 2, 0.2)])
@pytest.mark.parametrize("trans", [False, True])
def test_pivoting_with_row_swaps(exe, n, kl, ku, p, mult, trans):
    """Not diagonally dominant: rows are exchanged inside every panel, and the
    L panel tiles hold multipliers below the band."""
    ab = inputs.band_dominant(n, kl, ku, inputs.rng_for(n + kl), diag_mult=mult)
    _, _, ipiv = oracle.gbtrf(ab, kl, ku, pivot=True)
    assert np.count_nonzero(ipiv != np.arange(n)) > 0
    F = inputs.rhs(n, 3, inputs.rng_for(n))
    info, X = replay.run(exe, ab, kl, ku, F, p=p, pivot=True, trans=trans)
    assert info == 0
    _check(ab, kl, ku, F, X, trans)


@pytest.mark.parametrize("trans", [False, True])
def test_non_pivoting_generic_path(exe, trans):
    """The non-pivoting workgroup kernels (the path of bandwidths beyond the
    MFMA engines), with unequal bands and several partitions."""
    n, kl, ku, p = 1500, 12, 5, 6
    ab = inputs.band_dominant(n, kl, ku, inputs.rng_for(77))
    F = inputs.rhs(n, 2, inputs.rng_for(78))
    info, X = replay.run(exe, ab, kl, ku, F, p=p, pivot=False, trans=trans)
    assert info == 0
    _check(ab, kl, ku, F, X, trans)


@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_sweep_counts_match_paper_table(exe, pivot, trans, nrhs):
    """Table tab:sweeps of section "Optimizing per-partition costs": the
    factorisation does no full sweep on the first and last partitions and 3 on
    a middle one, the solve 2 and 4 (the transpose solve the same, as the
    transpose section states); counted by the workgroup kernels themselves."""
    import sweep_table
    n, kl, ku, p = 1200, 6, 4, 5
    ab = inputs.band_dominant(n, kl, ku, inputs.rng_for(91))
    F = inputs.rhs(n, nrhs, inputs.rng_for(92))
    info, X, cnt = replay.run(exe, ab, kl, ku, F, p=p, pivot=pivot, trans=trans, sweeps=True)
    assert info == 0
    _check(ab, kl, ku, F, X, trans)
    counts = sweep_table.from_array(cnt)
    sweep_table.check(counts, p, stages=("factor", "solve_t" if trans else "solve"))
    assert counts[("solve" if trans else "solve_t", "middle", True)] == 0
    # the truncated sweeps of the first and last partitions are there too
    assert counts[("factor", "first", False)] == 2 and counts[("factor", "last", False)] == 2


def test_sweep_table_is_the_papers():
    """The golden file holds the paper's values (a mistyped table would make
    the counter test above compare against the wrong numbers)."""
    import sweep_table
    assert sweep_table.table() == {"first_last": (0, 2), "middle": (3, 4)}


@pytest.mark.parametrize("pivot", [False, True])
@pytest.mark.parametrize("trans", [False, True])
def test_paper_tree_ratio_sizing(exe, pivot, trans):
    """The paper layout (p = 2^m + r: 11 = 8 + 3, leaves 1..6 the halves of
    the two-thread partitions, merged first) with explicit (R12, R13) sizes
    off the R12 = R13 / 2 line, on the workgroup kernels: the transposed
    level-1 merge included, and the sweep counters give the table's counts
    for every leaf."""
    import sweep_table
    n, k, p = 11 * 260 + 7, 12, 11
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(9600 + k), diag_mult=1.05, diag_add=0.0)
    F = inputs.rhs(n, 2, inputs.rng_for(9601))
    info, X, sw = replay.run(exe, ab, k, k, F, p=p, pivot=pivot, trans=trans, sweeps=True, tree="paper",
                             ratios=(1.2, 2.0))
    assert info == 0
    _check(ab, k, k, F, X, trans)
    sweep_table.check(sweep_table.from_array(sw), p,
                      stages=("factor", "solve_t" if trans else "solve"))


# ---- the diagonal-tile LU of the block LU (row-per-lane, DPP row broadcasts)

@pytest.fixture(scope="module")
def tile_exe(tmp_path_factory):
    return replay.build_tile_lu(str(tmp_path_factory.mktemp("hostemu_lu")))


def _plain_lu(A, boost, mrem):
    """LU without interchanges, written out step by step: at step t the pivot
    A(t, t) (raised by `boost` in magnitude when below it, for t < mrem), the
    multipliers below it and the rank-1 update of the trailing block."""
    a = np.array(A, dtype=np.float64)
    nb = 0
    for t in range(16):
        piv = a[t, t]
        if boost > 0 and t < mrem and abs(piv) < boost:
            piv = piv + boost if piv >= 0 else piv - boost
            nb += 1
        a[t, t] = piv
        for r in range(t + 1, 16):
            a[r, t] = a[r, t] / piv
            a[r, t + 1:] -= a[r, t] * a[t, t + 1:]
    return a, nb


def _tiles(rng, count, dominant):
    A = rng.standard_normal((count, 16, 16))
    if dominant:
        A += np.eye(16) * rng.uniform(4.0, 8.0, (count, 1, 1))
    return A


@pytest.mark.parametrize("dominant", [True, False])
def test_tile_lu_factors_and_inverses(tile_exe, dominant):
    rng = np.random.default_rng(11 + dominant)
    A = _tiles(rng, 12, dominant)
    lu, li, ui, nb = replay.run_tile_lu(tile_exe, A, 0.0, 16)
    assert (nb == 0).all()
    for i in range(len(A)):
        ref, _ = _plain_lu(A[i], 0.0, 16)
        L = np.tril(lu[i], -1) + np.eye(16)
        U = np.triu(lu[i])
        grow = max(1.0, np.abs(ref).max())
        assert np.abs(lu[i] - ref).max() <= 1e-12 * grow
        assert np.abs(L @ U - A[i]).max() <= 1e-13 * np.abs(A[i]).max() * grow
        # the inverses, against the identity
        assert np.abs(li[i] @ L - np.eye(16)).max() <= 1e-12 * max(1.0, np.abs(li[i]).max())
        assert np.abs(ui[i] @ U - np.eye(16)).max() <= 1e-12 * max(1.0, np.abs(ui[i]).max() * np.abs(U).max())
        assert np.allclose(np.triu(li[i], 1), 0.0) and np.allclose(np.tril(ui[i], -1), 0.0)
        assert np.allclose(np.diag(li[i]), 1.0)


def test_tile_lu_boosting_and_padding(tile_exe):
    rng = np.random.default_rng(5)
    A = _tiles(rng, 10, False) * 0.3
    boost = 0.5
    for mrem in (16, 9, 1):
        B = A.copy()
        if mrem < 16:   # rows and columns past the order are the identity
            B[:, mrem:, :] = 0.0
            B[:, :, mrem:] = 0.0
            B[:, mrem:, mrem:] = np.eye(16 - mrem)
        lu, li, ui, nb = replay.run_tile_lu(tile_exe, B, boost, mrem)
        for i in range(len(B)):
            ref, rnb = _plain_lu(B[i], boost, mrem)
            assert nb[i] == rnb
            assert np.abs(lu[i] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
            piv = np.diag(lu[i])[:mrem]
            assert (np.abs(piv) >= boost * (1 - 1e-15)).all()
            U = np.triu(lu[i])
            assert np.abs(ui[i] @ U - np.eye(16)).max() <= 1e-11 * max(1.0, np.abs(ui[i]).max() * np.abs(U).max())


def test_tile_lu_zero_pivot_stays_finite(tile_exe):
    A = np.eye(16)[None].copy()
    A[0, 5, 5] = 0.0
    lu, li, ui, nb = replay.run_tile_lu(tile_exe, A, 0.0, 16)
    assert lu[0, 5, 5] == 0.0
    assert np.isfinite(lu).all() and np.isfinite(li).all() and np.isfinite(ui).all()
    assert (ui[0, 5] == 0.0).all()   # the reciprocal of a zero pivot is taken as zero


def test_tile_lu_single_precision(tile_exe):
    rng = np.random.default_rng(21)
    A = _tiles(rng, 6, True).astype(np.float32).astype(np.float64)
    lu, li, ui, nb = replay.run_tile_lu(tile_exe, A, 0.0, 16, fp32=True)
    for i in range(len(A)):
        L = np.tril(lu[i], -1) + np.eye(16)
        U = np.triu(lu[i])
        assert np.abs(L @ U - A[i]).max() <= 2e-6 * np.abs(A[i]).max()
        assert np.abs(li[i] @ L - np.eye(16)).max() <= 2e-6
        assert np.abs(ui[i] @ U - np.eye(16)).max() <= 2e-6
