"""Helpers shared by the GPU tests: run the HIP solver through the C ABI on
numpy inputs and measure it against the oracle."""
import numpy as np

import oracle
from paper_1811_03559_amd import spike


def run(ab, kl, ku, F, trans=False, opts_factor=None, solves=None, **opts):
    """Factor ``ab`` and solve op(A) X = F on the GPU.  Returns (X, info, plan)."""
    import torch
    dev = torch.device("cuda:0")
    dab = torch.from_numpy(np.ascontiguousarray(ab)).to(dev)
    fac = spike.Factorization(dab, kl, ku, **opts)
    B = torch.from_numpy(np.ascontiguousarray(F)).to(dev)
    fac.solve_(B, trans=trans)
    torch.cuda.synchronize()
    X = B.cpu().numpy()
    info = fac.info()
    plan = fac.plan()
    fac.close()
    return X, info, plan


def check(ab, kl, ku, F, X, trans=False, pivot=True, relres_bar=1e-13, fwd_factor=1e-11,
          kappa=None, X_true=None):
    """Relative residual, forward error vs the oracle's solution (and vs X_true
    when given).  Returns the metrics; asserts the bars."""
    Xo = oracle.gbsv(ab, kl, ku, F, pivot=pivot, trans=trans)
    rr = oracle.relres(ab, kl, ku, X, F, trans=trans)
    agree = oracle.fwd_err(X, Xo)
    if kappa is None:
        kappa = oracle.cond1(ab, kl, ku) if ab.shape[0] <= 20000 else 1.0
    out = {"relres": rr, "agree": agree, "kappa": kappa}
    assert np.all(np.isfinite(X)), "non-finite result"
    assert rr <= relres_bar, out
    assert agree <= fwd_factor * max(kappa, 1.0), out
    if X_true is not None:
        fe = oracle.fwd_err(X, X_true)
        out["fwd"] = fe
        assert fe <= fwd_factor * max(kappa, 1.0), out
    return out
