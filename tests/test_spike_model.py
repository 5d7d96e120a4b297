"""Identities of the SPIKE decomposition checked on tiny dense matrices with
the NumPy stage model (CPU only), plus the merge-tree and reduced-system
shape counts of the recursive reduced system."""
import math

import numpy as np
import pytest

from paper_1811_03559_amd import inputs
from spike_model import Model, merge_tree, tree_from_spans
from test_oracle import dense_from_band


def dd_matrix(n, kl, ku, seed):
    ab = inputs.band_dominant(n, kl, ku, inputs.rng_for(seed), diag_mult=1.0, diag_add=1.0)
    return ab, dense_from_band(ab, kl, ku)


def sizes_for(n, p):
    base, rem = divmod(n, p)
    return [base + (1 if i >= p - rem else 0) for i in range(p)]


@pytest.mark.parametrize("p", list(range(1, 18)))
def test_merge_tree_shape(p):
    merges, levels = merge_tree(p)
    assert len(merges) == p - 1                          # one interface system per interface
    assert levels == (0 if p == 1 else math.ceil(math.log2(p)))
    assert sorted(J["mif"] for J in merges) == list(range(p - 1))


@pytest.mark.parametrize("p", [2, 3, 4, 5, 7, 8, 13])
@pytest.mark.parametrize("kl,ku", [(1, 1), (2, 3), (3, 2), (4, 4), (0, 2), (2, 0)])
def test_model_solves_match_dense(p, kl, ku):
    n = 16 * p + 5
    _, A = dd_matrix(n, kl, ku, 1000 + 31 * p + 7 * kl + ku)
    F = inputs.rhs(n, 3, inputs.rng_for(9)).T
    M = Model(A, sizes_for(n, p), kl, ku)
    np.testing.assert_allclose(M.solve(F), np.linalg.solve(A, F), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(M.solve_t(F), np.linalg.solve(A.T, F), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("p", [5, 6, 9, 12, 14])
@pytest.mark.parametrize("kl,ku", [(2, 3), (4, 4), (0, 2)])
def test_model_solves_match_dense_over_the_planners_paper_tree(p, kl, ku):
    """The merge tree the host planner builds for the paper's 2^m + r layout
    (host query, no device) is a valid merge order for the SPIKE algebra:
    every merge joins two nodes that exist, and the solves it gives match
    dense solves."""
    from paper_1811_03559_amd import spike
    n = 16 * p + 5
    _, A = dd_matrix(n, kl, ku, 2000 + 31 * p + 7 * kl + ku)
    F = inputs.rhs(n, 3, inputs.rng_for(19)).T
    sizes = spike.plan_query(n, kl, ku, p=p, tree="paper")["sizes"]
    tree = tree_from_spans(p, spike.plan_tree(n, kl, ku, p=p, tree="paper"))
    assert tree[0] != merge_tree(p)[0]                   # not the balanced tree
    M = Model(A, sizes, kl, ku, tree=tree)
    np.testing.assert_allclose(M.solve(F), np.linalg.solve(A, F), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(M.solve_t(F), np.linalg.solve(A.T, F), rtol=1e-10, atol=1e-12)


def test_paper_four_partition_merge_formulas():
    """p = 4: the level-1 merge of partitions 1,2 gives V^[2] with
    V^[2]_1t = -V^[1]_1t V^[2]_2t and V^[2]_2b = V^[1]_2b - W^[1]_2b V^[2]_1b,
    and of partitions 3,4 gives W^[2]_3t = W^[1]_3t - V^[1]_3t W^[2]_4t and
    W^[2]_4b = -W^[1]_4b W^[2]_3b, with the interface solves of eqs.
    RED_SYS_RECB/RED_SYS_W.  Checked against spikes of the merged dense blocks."""
    n, kl, ku, p = 80, 3, 3, 4
    _, A = dd_matrix(n, kl, ku, 77)
    sizes = sizes_for(n, p)
    M = Model(A, sizes, kl, ku)
    s = M.starts
    # merged node of leaves 0,1 = node p + 0; of leaves 2,3 = node p + 2
    A12 = A[0:s[2], 0:s[2]]
    V2 = np.linalg.solve(A12, A[0:s[2], s[2]:s[2] + ku])
    np.testing.assert_allclose(M.tips[p + 0]["Vb"], V2[-kl:], rtol=1e-10, atol=1e-13)
    A34 = A[s[2]:n, s[2]:n]
    W2 = np.linalg.solve(A34, A[s[2]:n, s[2] - kl:s[2]])
    np.testing.assert_allclose(M.tips[p + 2]["Wt"], W2[:ku], rtol=1e-10, atol=1e-13)
    # interface coefficients are the merged spikes at the interface rows
    f = M.fac[0]
    np.testing.assert_allclose(f["beta"], V2[s[1]:s[1] + ku], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(f["alpha"], V2[s[1] - kl:s[1]], rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_interface_determinant_identity(p):
    """det(E_J) = det(S) = det(A_J) / (det(A_L) det(A_R)) for every merge."""
    n, kl, ku = 12 * p, 2, 2
    _, A = dd_matrix(n, kl, ku, 500 + p)
    sizes = sizes_for(n, p)
    M = Model(A, sizes, kl, ku)
    s = list(M.starts) + [n]

    def rng(a, b):
        return s[a], s[b + 1]

    spans = {i: (i, i) for i in range(p)}
    for J in M.merges:
        a, b = J["a"], J["b"]
        la, lb = spans[J["left"]]
        ra, rb = spans[J["right"]]
        spans[p + J["mif"]] = (a, b)
        dJ = np.linalg.slogdet(A[slice(*rng(a, b)), slice(*rng(a, b))])
        dL = np.linalg.slogdet(A[slice(*rng(la, lb)), slice(*rng(la, lb))])
        dR = np.linalg.slogdet(A[slice(*rng(ra, rb)), slice(*rng(ra, rb))])
        dS = np.linalg.slogdet(M.fac[J["mif"]]["S"])
        assert dS[0] * dL[0] * dR[0] == dJ[0]
        assert dS[1] + dL[1] + dR[1] == pytest.approx(dJ[1], abs=1e-9)


def test_reduced_system_size_and_interface_values():
    """The reduced unknowns are the (kl+ku)(p-1) interface rows; the model's
    interface values equal the exact solution there."""
    n, kl, ku, p = 90, 2, 3, 5
    _, A = dd_matrix(n, kl, ku, 4242)
    M = Model(A, sizes_for(n, p), kl, ku)
    F = inputs.rhs(n, 1, inputs.rng_for(3)).T
    X = np.linalg.solve(A, F)
    M.solve(F)
    total = 0
    for mi, (xb, xt) in M.last_x.items():
        s1 = M.starts[mi + 1]
        np.testing.assert_allclose(xb, X[s1 - kl:s1], rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(xt, X[s1:s1 + ku], rtol=1e-10, atol=1e-12)
        total += xb.shape[0] + xt.shape[0]
    assert total == (kl + ku) * (p - 1)


def test_transpose_s_stage_identity():
    """Transpose S stage: rows of Y outside the tips equal F there (Y~ = F~),
    i.e. D^T X = Y with X = A^{-T} F."""
    n, kl, ku, p = 60, 2, 2, 3
    _, A = dd_matrix(n, kl, ku, 8)
    M = Model(A, sizes_for(n, p), kl, ku)
    F = inputs.rhs(n, 2, inputs.rng_for(5)).T
    X = np.linalg.solve(A.T, F)
    for i in range(p):
        s, m = M.starts[i], M.sizes[i]
        Y = M.block(i).T @ X[s:s + m]
        lo = ku if i > 0 else 0
        hi = m - kl if i < p - 1 else m
        np.testing.assert_allclose(Y[lo:hi], F[s + lo:s + hi], rtol=1e-10, atol=1e-12)
