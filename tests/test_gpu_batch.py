"""Batched solves and captured solve graphs (the batching row of the hot
path).  A batched solve must give, bitwise, what each system gives alone;
every replay of a captured graph must give, bitwise, the eager result."""
import numpy as np
import pytest

import oracle
from gpu_util import check
from paper_1811_03559_amd import inputs

pytestmark = pytest.mark.gpu

# (n, k, p, nrhs, trans, options): uneven sizes, bandwidths, partition counts,
# both operations, one FP32+refinement and one pivoting system (solved one
# by one inside the batch), one single-partition system.
SYSTEMS = [
    (3000, 8, 5, 1, False, {}),
    (5000, 16, 8, 3, True, {}),
    (2500, 8, 3, 2, False, {}),
    (4000, 16, 7, 1, False, {}),
    (1800, 4, 1, 1, True, {}),
    (6000, 32, 9, 4, False, {}),
    (3500, 16, 4, 1, True, {"precision": "mixed"}),
    (3000, 12, 3, 2, False, {"pivot": True}),
    (4200, 16, 6, 1, True, {}),
]


def _systems():
    import torch
    from paper_1811_03559_amd import spike
    out = []
    for i, (n, k, p, nrhs, trans, opts) in enumerate(SYSTEMS):
        ab = inputs.band_dominant(n, k, k, inputs.rng_for(5100 + i), diag_mult=1.05, diag_add=0.0)
        F = inputs.rhs(n, nrhs, inputs.rng_for(5200 + i))
        fac = spike.Factorization(torch.from_numpy(ab).cuda(), k, k, p=p, **opts)
        out.append((ab, k, F, trans, fac))
    return out


def test_batch_equals_individual_solves_bitwise():
    import torch
    from paper_1811_03559_amd import spike
    sysl = _systems()
    alone = []
    for ab, k, F, trans, fac in sysl:
        B = torch.from_numpy(F.copy()).cuda()
        fac.solve_(B, trans=trans)
        alone.append(B)
    Bs = [torch.from_numpy(F.copy()).cuda() for _, _, F, _, _ in sysl]
    spike.solve_batch([s[4] for s in sysl], Bs, trans=[s[3] for s in sysl])
    torch.cuda.synchronize()
    for (ab, k, F, trans, fac), B0, B1 in zip(sysl, alone, Bs):
        X0, X1 = B0.cpu().numpy(), B1.cpu().numpy()
        assert np.array_equal(X0, X1)
        check(ab, k, k, F, X1, trans=trans, pivot=False)
    for s in sysl:
        s[4].close()


def test_batch_of_more_systems_than_one_launch_holds():
    import torch
    from paper_1811_03559_amd import spike
    n, k = 1200, 4
    facs, Fs, abs_ = [], [], []
    for i in range(40):
        ab = inputs.band_dominant(n + 7 * i, k, k, inputs.rng_for(5300 + i))
        abs_.append(ab)
        facs.append(spike.Factorization(torch.from_numpy(ab).cuda(), k, k, p=2 + i % 5))
        Fs.append(inputs.rhs(n + 7 * i, 1, inputs.rng_for(5400 + i)))
    Bs = [torch.from_numpy(F.copy()).cuda() for F in Fs]
    spike.solve_batch(facs, Bs, trans=[i % 2 == 1 for i in range(40)])
    torch.cuda.synchronize()
    for i, (ab, F, B) in enumerate(zip(abs_, Fs, Bs)):
        check(ab, k, k, F, B.cpu().numpy(), trans=i % 2 == 1, pivot=False)
        facs[i].close()


def test_batch_argument_errors():
    import ctypes
    from paper_1811_03559_amd import spike
    L = spike.lib()
    assert L.spike_solve_batch(None, None, None, None, None, -1, None) == -6
    assert L.spike_solve_batch(None, None, None, None, None, 0, None) == 0
    assert L.spike_solve_batch(None, None, None, None, None, 1, None) == -1
    bad = (ctypes.c_void_p * 1)(12345)
    nr = (ctypes.c_int32 * 1)(1)
    assert L.spike_solve_batch(bad, nr, None, None, None, 1, None) == -3


@pytest.mark.parametrize("trans", [False, True])
def test_graph_replays_match_eager(trans):
    import torch
    from paper_1811_03559_amd import spike
    n, k, p = 20000, 16, 8
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(5500), diag_mult=1.05, diag_add=0.0)
    F = inputs.rhs(n, 1, inputs.rng_for(5501))
    dF = torch.from_numpy(F).cuda()
    fac = spike.Factorization(torch.from_numpy(ab).cuda(), k, k, p=p)
    B = dF.clone()
    fac.solve_(B, trans=trans)
    torch.cuda.synchronize()
    eager = B.cpu().numpy()
    check(ab, k, k, F, eager, trans=trans, pivot=False)
    Bg = dF.clone()
    torch.cuda.synchronize()
    g = spike.SolveGraph(fac, Bg, trans=trans)
    for _ in range(3):
        Bg.copy_(dF)                  # eager work between the replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(Bg.cpu().numpy(), eager)
    g.close()
    fac.close()


def test_graph_of_a_batch_replays_match_eager():
    import torch
    from paper_1811_03559_amd import spike
    sysl = [s for s in _systems() if not s[4].opts.precision]   # refinement is not capturable
    Fs = [torch.from_numpy(s[2].copy()).cuda() for s in sysl]
    eager = [F.clone() for F in Fs]
    spike.solve_batch([s[4] for s in sysl], eager, trans=[s[3] for s in sysl])
    torch.cuda.synchronize()
    Bs = [F.clone() for F in Fs]
    torch.cuda.synchronize()
    g = spike.SolveGraph([s[4] for s in sysl], Bs, trans=[s[3] for s in sysl])
    for _ in range(3):
        for B, F in zip(Bs, Fs):
            B.copy_(F)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for B, E in zip(Bs, eager):
            assert np.array_equal(B.cpu().numpy(), E.cpu().numpy())
    g.close()
    for s in sysl:
        s[4].close()


def test_autotune_returns_a_working_plan():
    import torch
    from paper_1811_03559_amd import spike
    n, k = 60000, 16
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(5600), diag_mult=1.05, diag_add=0.0)
    dab = torch.from_numpy(ab).cuda()
    spike.tune_cache_clear()
    opts, res = spike.autotune(dab, k, k, nrhs=2)
    assert res["candidates"] >= 2 and res["K"] > 0, res
    assert not res["cached"]
    assert res["factor_ms"] > 0 and res["solve_ms"] > 0, res
    F = inputs.rhs(n, 2, inputs.rng_for(5601))
    fac = spike.Factorization(dab, k, k, **opts)
    B = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B)
    torch.cuda.synchronize()
    check(ab, k, k, F, B.cpu().numpy(), pivot=False)
    fac.close()


def test_autotune_cache_reuses_and_reloads(tmp_path):
    """A second autotune of the same shape (n, kl, ku, log2 nrhs, precision,
    pivot) comes from the cache with the same options; after clearing, the
    file written by tune_cache_save restores it; a new shape is tuned."""
    import torch
    from paper_1811_03559_amd import spike
    n, k = 40000, 8
    ab = inputs.band_dominant(n, k, k, inputs.rng_for(5700), diag_mult=1.05, diag_add=0.0)
    dab = torch.from_numpy(ab).cuda()
    spike.tune_cache_clear()
    o1, r1 = spike.autotune(dab, k, k, nrhs=3)
    assert not r1["cached"] and spike.tune_cache_size() == 1
    o2, r2 = spike.autotune(dab, k, k, nrhs=2)   # same log2 bucket
    assert r2["cached"] and o2["p"] == o1["p"] and o2["tree"] == o1["tree"] and o2["sizing"] == o1["sizing"]
    assert r2["factor_ms"] == r1["factor_ms"]
    path = tmp_path / "cache.txt"
    spike.tune_cache_save(path)
    spike.tune_cache_clear()
    spike.tune_cache_load(path)
    o3, r3 = spike.autotune(dab, k, k, nrhs=3)
    assert r3["cached"] and o3["p"] == o1["p"] and o3["tree"] == o1["tree"]
    o4, r4 = spike.autotune(dab, k, k, nrhs=16)   # another bucket
    assert not r4["cached"] and spike.tune_cache_size() == 2
    F = inputs.rhs(n, 3, inputs.rng_for(5701))
    fac = spike.Factorization(dab, k, k, **o3)
    B = torch.from_numpy(F.copy()).cuda()
    fac.solve_(B)
    torch.cuda.synchronize()
    check(ab, k, k, F, B.cpu().numpy(), pivot=False)
    fac.close()
    spike.tune_cache_clear()
