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
from paper_1811_03559_amd import inputs

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
