"""GPU parity of the paper's merge-tree layout: p = 2^m + r leaves, where the
halves of the r two-thread partitions (placed from the second partition on)
merge first and a complete binary tree runs over the 2^m nodes left.  Every
tree gives the same X up to rounding, so the bars are those of the balanced
tree: relative residual <= 1e-13 and agreement with the oracle's solution to
1e-11 * kappa_1, for both operations, with and without pivoting, on the MFMA
tile engine's bandwidths, in FP32+refinement and inside a batch."""
import numpy as np
import pytest

import oracle
from gpu_util import check, run
from paper_1811_03559_amd import inputs, spike

pytestmark = pytest.mark.gpu


def dd_band(n, kl, ku, seed, mult=1.0, add=1.0):
    return inputs.band_dominant(n, kl, ku, inputs.rng_for(seed), diag_mult=mult, diag_add=add)


@pytest.mark.parametrize("p", [5, 6, 12, 13, 17])
@pytest.mark.parametrize("kl,ku", [(2, 5), (4, 4), (0, 3)])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("pivot", [False, True])
def test_paper_tree_grid(p, kl, ku, trans, pivot):
    n = 37 * p + 11
    ab = dd_band(n, kl, ku, 7700 + 97 * p + 13 * kl + ku)
    F = inputs.rhs(n, 3, inputs.rng_for(31 + p))
    X, info, plan = run(ab, kl, ku, F, trans=trans, p=p, pivot=pivot, tree="paper")
    assert info["info"] == 0 and plan["p"] == p
    check(ab, kl, ku, F, X, trans=trans, pivot=pivot)


@pytest.mark.parametrize("k", [64, 160])
@pytest.mark.parametrize("p", [6, 12])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("pivot", [False, True])
def test_paper_tree_wide_band(k, p, trans, pivot):
    n = p * (2 * k + 37) + 3
    ab = dd_band(n, k, k, 9100 + k + p, mult=1.05, add=0.0)
    F = inputs.rhs(n, 5, inputs.rng_for(k * p + 1))
    X, info, _ = run(ab, k, k, F, trans=trans, p=p, pivot=pivot, tree="paper")
    assert info["info"] == 0
    check(ab, k, k, F, X, trans=trans, pivot=pivot)


@pytest.mark.parametrize("trans", [False, True])
def test_paper_tree_mixed_precision(trans):
    n, k, p = 20000, 16, 6
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(inputs.seed_for(3)), diag_mult_range=(1.01, 1.5))
    X_true = inputs.rhs(n, 3, inputs.rng_for(4))
    F = oracle.gbmv(ab, k, k, X_true, trans=trans)
    X, info, _ = run(ab, k, k, F, trans=trans, p=p, precision="mixed", tree="paper")
    assert 1 <= info["refine_iters"] <= 6, info
    assert 0 <= info["berr"] <= 1e-13, info
    check(ab, k, k, F, X, trans=trans, pivot=False, X_true=X_true)


@pytest.mark.parametrize("p", [11, 21])
@pytest.mark.parametrize("r12,r13", [(1.2, 2.0), (0.8, 3.0)])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("k", [4, 40])
def test_paper_tree_ratio_sizing(p, r12, r13, trans, k):
    """The paper layout with explicit (R12, R13) partition sizes, R12 off the
    R13 / 2 line so the halves of the two-thread partitions (which merge
    first, also in the transpose solve) differ in size from the
    single-thread partitions."""
    n = p * (3 * k + 90) + 7
    ab = dd_band(n, k, k, 9300 + p + k, mult=1.05, add=0.0)
    F = inputs.rhs(n, 2, inputs.rng_for(9400 + p))
    opts = dict(p=p, tree="paper", sizing="ratios", r12=r12, r13=r13)
    X, info, plan = run(ab, k, k, F, trans=trans, **opts)
    assert info["info"] == 0 and plan["p"] == p
    sz = spike.plan_query(n, k, k, **opts)["sizes"]
    assert abs(sz[1] - sz[-2]) > 2
    check(ab, k, k, F, X, trans=trans, pivot=False)


@pytest.mark.parametrize("k", [8, 40])
def test_paper_tree_sweep_counts(k):
    """Table tab:sweeps for the paper layout: the halves of a two-thread
    partition (leaves 1 .. 2r) each run the middle partition's 3 factor and
    4 solve sweeps, so together they do the table's 3 and 4 sweeps over
    the two-thread partition's rows, as the SPIKE 2x2 kernel does; the
    transpose solve too."""
    import torch
    import sweep_table
    from paper_1811_03559_amd import spike
    p = 11                                   # 2^3 + 3: leaves 1..6 two-thread halves
    n = p * (5 * k + 90) + 5
    ab = dd_band(n, k, k, 9500 + k, mult=1.05, add=0.0)
    F = inputs.rhs(n, 2, inputs.rng_for(9501))
    dab = torch.from_numpy(ab).cuda()
    with spike.sweep_counting():
        fac = spike.Factorization(dab, k, k, p=p, tree="paper", sizing="ratios", r12=1.2, r13=2.0)
    B = torch.from_numpy(F.copy()).cuda()
    Bt = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B)
    fac.solve_(Bt, trans=True)
    torch.cuda.synchronize()
    counts = fac.sweep_counts()
    fac.close()
    sweep_table.check(counts, p)
    check(ab, k, k, F, B.cpu().numpy(), pivot=False)
    check(ab, k, k, F, Bt.cpu().numpy(), trans=True, pivot=False)


def test_batch_mixing_trees_equals_individual_solves_bitwise():
    import torch
    from paper_1811_03559_amd import spike
    systems = [(3000, 8, 6, "paper", False), (4000, 16, 5, "balanced", True),
               (5200, 8, 13, "paper", True), (2600, 4, 7, "balanced", False),
               (6000, 16, 17, "paper", False)]
    facs, Fs, abs_, alone = [], [], [], []
    for i, (n, k, p, tree, trans) in enumerate(systems):
        ab = dd_band(n, k, k, 7900 + i, mult=1.05, add=0.0)
        F = inputs.rhs(n, 2, inputs.rng_for(7950 + i))
        fac = spike.Factorization(torch.from_numpy(ab).cuda(), k, k, p=p, tree=tree)
        B = torch.from_numpy(F.copy()).cuda()
        fac.solve_(B, trans=trans)
        facs.append(fac), Fs.append(F), abs_.append(ab), alone.append(B)
    Bs = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    spike.solve_batch(facs, Bs, trans=[s[4] for s in systems])
    torch.cuda.synchronize()
    for (n, k, p, tree, trans), ab, F, B0, B1, fac in zip(systems, abs_, Fs, alone, Bs, facs):
        X1 = B1.cpu().numpy()
        assert np.array_equal(B0.cpu().numpy(), X1), (p, tree)
        check(ab, k, k, F, X1, trans=trans, pivot=False)
        fac.close()
