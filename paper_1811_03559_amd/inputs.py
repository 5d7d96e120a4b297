"""Seeded synthetic inputs for the banded solver (shared by tests and the
benchmark).  This module only draws random numbers and assembles band arrays;
it holds none of the solver's arithmetic.

Band arrays are numpy arrays of shape ``(n, ldab)`` in C order, i.e. LAPACK
column-major band storage with ``ab[j, ku + i - j] = A(i, j)`` (entries that
fall outside the matrix are zero).  Right-hand sides are ``(nrhs, n)`` C-order
arrays, i.e. column-major ``n x nrhs``.

Every generator takes a numpy ``Generator(PCG64(seed))`` and fills, in this
order: the band entries (column-major), then the diagonal scalings, then the
row scalings.  ``seed_for(cfg, replicate)`` gives the seed convention
``1811035590 + 100*cfg + replicate``.

The matrices follow the paper's synthetic workloads (it uses randomly filled
dense bands with a prescribed degree of diagonal dominance, plus non-dominant
ill-conditioned bands for the pivoting study); there is no public dataset.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 1811035590


def seed_for(cfg: int, replicate: int = 0) -> int:
    return SEED_BASE + 100 * cfg + replicate


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _mask_outside(ab: np.ndarray, kl: int, ku: int) -> None:
    """Zero the storage slots that correspond to rows outside [0, n)."""
    n = ab.shape[0]
    for d in range(-ku, kl + 1):            # d = i - j, slot ku + d
        s = ku + d
        if d < 0:                            # rows i = j + d < 0 for j < -d
            ab[: min(n, -d), s] = 0.0
        elif d > 0:                          # rows i = j + d >= n for j >= n - d
            ab[max(0, n - d):, s] = 0.0


def offdiag_abs_rowsum(ab: np.ndarray, kl: int, ku: int) -> np.ndarray:
    """Sum over j != i inside the band of |A(i, j)|, for every row i."""
    n = ab.shape[0]
    out = np.zeros(n, dtype=np.float64)
    for d in range(-ku, kl + 1):             # A(i, i - d) at ab[i - d, ku + d]
        if d == 0:
            continue
        lo, hi = max(0, d), min(n, n + d)
        if hi > lo:
            out[lo:hi] += np.abs(ab[lo - d:hi - d, ku + d])
    return out


def set_diag(ab: np.ndarray, ku: int, diag: np.ndarray) -> None:
    ab[:, ku] = diag


def band_dominant(n: int, kl: int, ku: int, rng: np.random.Generator, *,
                  diag_mult=1.0, diag_add=0.0, diag_mult_range=None,
                  ldab: int | None = None) -> np.ndarray:
    """Off-diagonals iid U[-1, 1]; diagonal = (off-diagonal row abs-sum) *
    mult + add, with mult fixed or drawn per row from U[lo, hi]."""
    ldab = ldab or (kl + ku + 1)
    ab = rng.uniform(-1.0, 1.0, size=(n, ldab))
    if ldab > kl + ku + 1:
        ab[:, kl + ku + 1:] = 0.0
    _mask_outside(ab, kl, ku)
    rs = offdiag_abs_rowsum(ab, kl, ku)
    if diag_mult_range is not None:
        mult = rng.uniform(diag_mult_range[0], diag_mult_range[1], size=n)
    else:
        mult = diag_mult
    set_diag(ab, ku, rs * mult + diag_add)
    return ab


def band_gaussian_rowscaled(n: int, kl: int, ku: int, rng: np.random.Generator, *,
                            log10_range=(-4.0, 4.0), ldab: int | None = None) -> np.ndarray:
    """Band entries (diagonal included) iid N(0, 1), no dominance; then row i
    is scaled by 10**u_i with u_i ~ U[lo, hi].  Ill-conditioned on purpose."""
    ldab = ldab or (kl + ku + 1)
    ab = rng.standard_normal(size=(n, ldab))
    if ldab > kl + ku + 1:
        ab[:, kl + ku + 1:] = 0.0
    _mask_outside(ab, kl, ku)
    u = rng.uniform(log10_range[0], log10_range[1], size=n)
    scale = 10.0 ** u
    for d in range(-ku, kl + 1):             # A(i, i - d) at ab[i - d, ku + d]
        lo, hi = max(0, d), min(n, n + d)
        if hi > lo:
            ab[lo - d:hi - d, ku + d] *= scale[lo:hi]
    return ab


def band_paper_dd(n: int, kl: int, ku: int, rng: np.random.Generator, dd: float) -> np.ndarray:
    """The paper's test family: band filled uniformly on (-1, 1), then the
    diagonal set to DD times the off-diagonal absolute column sum (reading of
    the degree of diagonal dominance with absolute values)."""
    ab = rng.uniform(-1.0, 1.0, size=(n, kl + ku + 1))
    _mask_outside(ab, kl, ku)
    colsum = np.abs(ab).sum(axis=1) - np.abs(ab[:, ku])
    set_diag(ab, ku, dd * colsum)
    return ab


def zband_dominant(n: int, kl: int, ku: int, rng: np.random.Generator, *, diag_mult=1.05, diag_add=0.0,
                   diag_mult_range=None) -> np.ndarray:
    """Complex band: off-diagonal real and imaginary parts iid U[-1, 1]; the
    diagonal has modulus (off-diagonal row sum of moduli) * mult + add and a
    phase drawn from U[0, 2 pi).  complex128 array (n, kl + ku + 1) in the
    real band's layout (ab[j, ku + i - j] = A(i, j))."""
    ab = rng.uniform(-1.0, 1.0, size=(n, kl + ku + 1)) + 1j * rng.uniform(-1.0, 1.0, size=(n, kl + ku + 1))
    mask = np.ones((n, kl + ku + 1))
    _mask_outside(mask, kl, ku)
    ab *= mask
    rs = np.zeros(n)
    for d in range(-ku, kl + 1):            # A(i, i - d) at ab[i - d, ku + d]
        if d == 0:
            continue
        lo, hi = max(0, d), min(n, n + d)
        if hi > lo:
            rs[lo:hi] += np.abs(ab[lo - d:hi - d, ku + d])
    mult = rng.uniform(diag_mult_range[0], diag_mult_range[1], size=n) if diag_mult_range else diag_mult
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n)
    ab[:, ku] = (rs * mult + diag_add) * np.exp(1j * phase)
    return ab


def zrhs(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """Complex right-hand sides, real and imaginary parts N(0, 1): (nrhs, n)."""
    return rng.standard_normal(size=(nrhs, n)) + 1j * rng.standard_normal(size=(nrhs, n))


def rhs(n: int, nrhs: int, rng: np.random.Generator) -> np.ndarray:
    """X_true (or a right-hand side) ~ N(0, 1), shape (nrhs, n)."""
    return rng.standard_normal(size=(nrhs, n))


# Recipes of the benchmark/test configurations ------------------------------------

def cfg0(seed=None):
    """n=4096, kl=ku=4, nrhs=1; diagonal = row abs-sum + 1."""
    rng = rng_for(seed if seed is not None else seed_for(0))
    ab = band_dominant(4096, 4, 4, rng, diag_mult=1.0, diag_add=1.0)
    return ab, 4, 4, rhs(4096, 1, rng)


def cfg1(n=1_000_000, k=160, nrhs=1, seed=None):
    """Dense band, off-diagonals U[-1,1], diagonal = row abs-sum * 1.05."""
    rng = rng_for(seed if seed is not None else seed_for(1))
    ab = band_dominant(n, k, k, rng, diag_mult=1.05)
    return ab, k, k, rhs(n, nrhs, rng)


def cfg2(n=500_000, k=64, nrhs=16, seed=None):
    """N(0,1) band with row scales 10^U[-4,4]: needs pivoting."""
    rng = rng_for(seed if seed is not None else seed_for(2))
    ab = band_gaussian_rowscaled(n, k, k, rng)
    return ab, k, k, rhs(n, nrhs, rng)


def cfg3(n=1_000_000, k=128, nrhs=32, seed=None):
    """Diagonal = row abs-sum * U[1.01, 1.5] (mixed-precision workload)."""
    rng = rng_for(seed if seed is not None else seed_for(3))
    ab = band_dominant(n, k, k, rng, diag_mult_range=(1.01, 1.5))
    return ab, k, k, rhs(n, nrhs, rng)


def cfg4_requests(nreq=1024, seed=None, pool_per_bucket=4):
    """Request table of the serving stream: n = round(2^U[12, 20]) per pooled
    matrix, k in {2, 8, 32, 128}, nrhs in {1, 4, 16, 64}, 30% transpose, 50%
    re-solving a uniformly chosen earlier matrix id, 80% dominant (cfg1
    recipe) / 20% pivoting-class (cfg2 recipe) matrices, FP64 or FP32 with
    FP64 refinement half and half for the dominant class (the pivoting class
    is FP64 only).  Matrices come from a pool of `pool_per_bucket` per
    (class, k) bucket; every new id factors a pool matrix afresh.

    Returns (pool, reqs): pool[(cls, k)] = list of (n, seed); reqs = list of
    dicts with id, cls, k, member, nrhs, trans, precision, rhs_seed."""
    rng = rng_for(seed if seed is not None else seed_for(4))
    ks = (2, 8, 32, 128)
    pool = {}
    for cls in ("dom", "piv"):
        for k in ks:
            pool[(cls, k)] = [(int(round(2.0 ** rng.uniform(12.0, 20.0))), int(rng.integers(1 << 31)))
                              for _ in range(pool_per_bucket)]
    ids = []
    reqs = []
    for i in range(nreq):
        if ids and rng.random() < 0.5:
            base = ids[int(rng.integers(len(ids)))]
            r = dict(base)
        else:
            cls = "piv" if rng.random() < 0.2 else "dom"
            k = ks[int(rng.integers(4))]
            prec = "mixed" if cls == "dom" and rng.random() < 0.5 else "fp64"
            r = {"id": len(ids), "cls": cls, "k": k, "member": int(rng.integers(pool_per_bucket)),
                 "precision": prec}
            ids.append(dict(r))
        r["nrhs"] = (1, 4, 16, 64)[int(rng.integers(4))]
        r["trans"] = bool(rng.random() < 0.3)
        r["rhs_seed"] = int(rng.integers(1 << 31))
        reqs.append(r)
    return pool, reqs


def cfg4_matrix(cls, k, n, seed):
    """One pooled matrix of the serving stream (cfg1 or cfg2 recipe)."""
    rng = rng_for(seed)
    if cls == "piv":
        return band_gaussian_rowscaled(n, k, k, rng)
    return band_dominant(n, k, k, rng, diag_mult=1.05)
