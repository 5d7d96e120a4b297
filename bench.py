#!/usr/bin/env python3
"""Benchmark of the MI355X recursive SPIKE solver.

Workload: the paper's headline problem size, n = 1,000,000, kl = ku = 160
(bandwidth 321), FP64, dense band with off-diagonals U[-1,1] and diagonal =
row abs-sum * 1.05, p = 256 partitions, nrhs = 1, synthetic and seeded.

One step is one pass of the whole hot path on a fresh system:
  factorisation (block LU/UL, spike tips, recursive reduced-system factors)
  + solve A X = F (D stage, reduced solve, retrieval)
  + solve A^T X = F (transpose S stage, transposed reduced solve, transpose D stage).
`value` is steps per second (solves/s).  Inputs are resident in HBM before
the timed region.

Prints one JSON line (rank 0, one GPU).  Extra fields: `roofline` for the
kernel that takes the most time in a step, `cpu_baseline` (the FP64 oracle
on one host core at the full size, factorisation and solves timed apart,
with the host's CPU model and core count) and `detail` (per-kernel and
per-phase times, solve GB/s, nrhs = 64 solves, residuals, agreement with the
oracle's solutions, and the other workloads: the small n = 4096 system,
partition counts and sizings, pivoting, mixed precision, serving).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HBM GB/s + solves/s, n=1M k=160 FP64; mixed-prec speedup; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def band_matvec(ab, kl, ku, x, trans=False):
    """numpy banded product (bench-side residual check only)."""
    n = ab.shape[0]
    y = np.zeros_like(x)
    for d in range(-ku, kl + 1):            # A(i, i-d) at ab[i-d, ku+d]
        lo, hi = max(0, d), min(n, n + d)
        if hi <= lo:
            continue
        a = ab[lo - d:hi - d, ku + d]
        if not trans:
            y[lo:hi] += a * x[lo - d:hi - d]
        else:
            y[lo - d:hi - d] += a * x[lo:hi]
    return y


def relres(ab, kl, ku, X, F, trans=False):
    A_inf = np.abs(ab).sum(axis=1).max() if trans else None
    if not trans:
        rows = np.zeros(ab.shape[0])
        for d in range(-ku, kl + 1):
            n = ab.shape[0]
            lo, hi = max(0, d), min(n, n + d)
            if hi > lo:
                rows[lo:hi] += np.abs(ab[lo - d:hi - d, ku + d])
        A_inf = rows.max()
    r = F - band_matvec(ab, kl, ku, X, trans)
    return float(np.abs(r).max() / (A_inf * np.abs(X).max()))


def merge_tree(p):
    """Leaf ranges (a, b) of every merge: adjacent nodes are paired left to
    right at each level, an odd last node is carried up unchanged."""
    nodes = [(i, i) for i in range(p)]
    out = []
    while len(nodes) > 1:
        nxt = []
        for j in range(0, len(nodes) - 1, 2):
            a, b = nodes[j][0], nodes[j + 1][1]
            out.append((a, b))
            nxt.append((a, b))
        if len(nodes) % 2:
            nxt.append(nodes[-1])
        nodes = nxt
    return out


def step_work(sizes, k, nrhs):
    """Algorithmic work of the kernels of one step (kl = ku = k, FP64,
    non-pivoting, the MFMA tile path of the factor and the solve).

    Factor:
      k_flu          block LU/UL of every partition: 2 m k^2 flops; reads the
                     band and writes the factors (2 x 8 (2k+1) m bytes);
      k_ftip_v       truncated spike sweeps: the bottom k x k block of
                     L^{-1}[0; B^] per middle partition (k^3), and for the
                     first/last partition a truncated L and U sweep (2 k^3);
      k_ftip_w       W spike L-sweep, 2 m k^2 per middle partition;
      k_ftip_u       [V W] U-sweep, 4 m k^2 per middle partition;
      merges         per merge J: Schur complement S = I - Wt Vb (2k^3,
                     k_mgemm; with Dm = -Wt Wb another 2k^3 when J has a left
                     neighbour), LU of S (2/3 k^3, k_mlu), beta/delta
                     (triangular solves 2k^3 each in k_mtrsm), alpha/gamma
                     (products 2k^3 each in k_mgemm), merged tips 2k^3 each
                     (k_mgemm), none at the root.
    Solve (bytes; nrhs = 1 is bandwidth bound): a full sweep streams half the
    band (k+1 of the 2k+1 diagonals, 8 bytes each); per solve the middle
    partitions make 4 full sweeps and first/last 2 (the paper's sweep table),
    split 2/2 and 1/1 between the two partition kernels of a solve
    (k_fdstage/k_fretrieve, transpose k_fzsweep/k_fdtstage), each of which
    also reads and writes the right-hand side once (16 bytes per row and
    column)."""
    p = len(sizes)
    n = sum(sizes)
    mid = sum(sizes[1:-1]) if p > 2 else 0
    ends = n - mid
    band_half = 8.0 * (k + 1)
    k3 = float(k) ** 3
    f_lu = f_trsm = f_gemm = 0.0
    for a, b in merge_tree(p):
        nv, nw = b < p - 1, a > 0
        f_lu += (2.0 / 3.0) * k3
        f_gemm += 2 * k3 * (1 + nw)
        f_trsm += 2 * k3 * (nv + nw)
        f_gemm += 2 * k3 * (nv + nw)
        if not (a == 0 and b == p - 1):
            f_gemm += 2 * k3 * ((nv and nw) * 2 + nv + nw)
    sweep = (2 * mid + ends) * band_half + 16.0 * n * nrhs
    w = {
        "k_flu": {"flops": 2.0 * n * k * k, "bytes": 2 * 8.0 * (2 * k + 1) * n, "engine": "mfma"},
        "k_ftip_v": {"flops": k3 * max(p - 2, 0) + 4 * k3, "engine": "mfma"},
        "k_ftip_w": {"flops": 2.0 * mid * k * k, "engine": "mfma"},
        "k_ftip_u": {"flops": 4.0 * mid * k * k, "engine": "mfma"},
        "k_mgemm": {"flops": f_gemm, "engine": "mfma"},
        "k_mlu": {"flops": f_lu, "engine": "alu"},   # pivot search and rank-1 steps on the VALU
        "k_mtrsm": {"flops": f_trsm, "engine": "mfma"},
        "k_fdstage": {"bytes": sweep},
        "k_fretrieve": {"bytes": sweep},
        "k_fzsweep": {"bytes": sweep},
        "k_fdtstage": {"bytes": sweep},
    }
    return w


def calib_copy(gib=1.0, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_read": n * 8, "calib_copy_bytes_written": n * 8,
                      "reps": reps}), flush=True)


def kernel_source_digest():
    """SHA-256 over the library's device-code sources: the HIP translation
    units and headers (names and bytes, sorted); the host-only planner, API,
    server and profiler units (.cpp) compile to no kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1811_03559_amd", "csrc")
    for f in sorted(f for f in os.listdir(d) if f.endswith((".hip", ".hpp"))):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    no record for this workload or the kernel sources changed since it was
    taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh).get(workload)
    if not rec or rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    t = rec["per_dispatch"].get(kernel)
    return None if t is None else t["read_bytes"] + t["write_bytes"]


def roofline(name, work, timing, workload):
    """Roofline entry of one kernel: algorithmic work per step over its time
    per step (HIP events around every launch; for a kernel launched once a
    step this is the work per launch over the average launch time).  A kernel
    with both flops and bytes is placed against the engine its dense
    contraction runs on."""
    traffic = measured_traffic(name, workload)
    if work is None:
        return {"kernel": name, "bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": None, "traffic": traffic}
    t_step = timing["ms_per_step"] / 1000.0
    if "flops" in work:
        ach = work["flops"] / t_step / 1e12
        out = {"kernel": name, "bound": work.get("engine", "alu"), "achieved": ach,
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
               "traffic": traffic, "work_per_step": work["flops"]}
        if "bytes" in work:
            out["hbm_gbs"] = work["bytes"] / t_step / 1e9
            out["hbm_frac"] = out["hbm_gbs"] / HBM_PEAK_GBS
        return out
    ach = work["bytes"] / t_step / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "work_per_step": work["bytes"]}


def host_cpu():
    """Model name and core counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count()}


def cpu_baseline(ab, kl, ku, F):
    """The oracle (plain FP64 banded GE, non-pivoting LU) on one host core at
    the full headline size: one factorisation, then A X = F and A^T X = F,
    timed apart."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    info, w, ipiv = oracle.gbtrf(ab, kl, ku, pivot=False)
    t1 = time.perf_counter()
    X = oracle.gbtrs(w, ipiv, kl, ku, F, pivot=False)
    t2 = time.perf_counter()
    Xt = oracle.gbtrs(w, ipiv, kl, ku, F, pivot=False, trans=True)
    t3 = time.perf_counter()
    del w
    total = t3 - t0
    return {"value": 1.0 / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": ("the full step at n=%d, kl=ku=%d, nrhs=1 (FP64 banded GE without pivoting: one "
                       "factorisation, then A X = F and A^T X = F), single thread" % (ab.shape[0], kl)),
            "factor_s": t1 - t0, "solve_s": t2 - t1, "solve_t_s": t3 - t2, "info": info,
            "host": host_cpu(), "_x": (X, Xt)}


def _ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def _timed(fn, reps=1):
    """Median device time (ms) of fn() over `reps` runs, HIP events on the
    current stream (the stream the library launches on)."""
    import torch
    ts = []
    for _ in range(reps):
        e0, e1 = _ev(), _ev()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def fwd_err(X, Xt):
    return float(np.abs(X - Xt).max() / np.abs(Xt).max())


def inputs_rhs64(n):
    from paper_1811_03559_amd import inputs
    return inputs.rhs(n, 64, inputs.rng_for(inputs.seed_for(1, 1)))


def bench_cfg0(reps=20):
    """The small configuration (n = 4096, kl = ku = 4, p = 3, nrhs = 1):
    latency-bound, so factor and solve times in microseconds."""
    import torch
    import oracle
    from paper_1811_03559_amd import inputs, spike
    ab, kl, ku, Xt = inputs.cfg0()
    F = oracle.gbmv(ab, kl, ku, Xt)
    dab = torch.from_numpy(ab).cuda()
    dF = torch.from_numpy(F).cuda()
    ws = torch.empty(spike.workspace_size(ab.shape[0], kl, ku, p=3), dtype=torch.uint8, device="cuda")
    holder = {}

    def fac():
        if "f" in holder:
            holder["f"].close()
        holder["f"] = spike.Factorization(dab, kl, ku, p=3, workspace=ws)
    fac()
    torch.cuda.synchronize()
    t_f = _timed(fac, reps)
    B = dF.clone()
    t_n = _timed(lambda: (B.copy_(dF), holder["f"].solve_(B)), reps)
    t_t = _timed(lambda: (B.copy_(dF), holder["f"].solve_(B, trans=True)), reps)
    B.copy_(dF)
    holder["f"].solve_(B)
    X = B.cpu().numpy()
    out = {"n": ab.shape[0], "kl": kl, "ku": ku, "p": 3, "factor_us": t_f * 1e3, "solve_us": t_n * 1e3,
           "solve_t_us": t_t * 1e3, "relres": oracle.relres(ab, kl, ku, X, F),
           "vs_oracle": oracle.fwd_err(X, oracle.gbsv(ab, kl, ku, F, pivot=False))}
    holder["f"].close()
    return out


def bench_p_sweep(dab, ab, k, F, ps=(250, 500)):
    """Factor and N/T solve times of the headline system at other partition
    counts (equal sizes; balanced merge tree and the paper's 2^m + r layout)
    and with R13 sizing at p = 256, 250 and 500; nrhs = 1 N and T, and
    nrhs = 64 N."""
    import torch
    from paper_1811_03559_amd import spike
    out = {}
    dF = torch.from_numpy(F).cuda()
    cases = [(pp, "equal", "balanced") for pp in ps] + [(pp, "equal", "paper") for pp in ps]
    cases += [(pp, "r13", "balanced") for pp in (256,) + tuple(ps)]
    F64 = torch.from_numpy(inputs_rhs64(F.shape[1])).cuda()
    for p, sizing, tree in cases:
        opts = dict(p=p, sizing=sizing, nrhs_hint=1, tree=tree, nrhs_max=64)
        holder = {}

        def fac():
            holder["f"] = spike.Factorization(dab, k, k, **opts)
        t_f = _timed(fac)
        f = holder["f"]
        B, Bt = dF.clone(), dF.clone()
        t_n = _timed(lambda: f.solve_(B))
        t_t = _timed(lambda: f.solve_(Bt, trans=True))
        B64 = F64.clone()
        t_64 = _timed(lambda: f.solve_(B64))
        out["p%d_%s%s" % (p, sizing, "_paper_tree" if tree == "paper" else "")] = {
            "levels": spike.plan_query(ab.shape[0], k, k, **opts)["levels"],
            "factor_ms": t_f, "solve_ms": t_n, "solve_t_ms": t_t, "solve_ms_nrhs64": t_64,
            "step_ms": t_f + t_n + t_t,
            "sizes_first_mid": spike.plan_query(ab.shape[0], k, k, **opts)["sizes"][:2],
            "relres_n": relres(ab, k, k, B.cpu().numpy()[0], F[0]),
            "relres_t": relres(ab, k, k, Bt.cpu().numpy()[0], F[0], trans=True)}
        f.close()
    return out


def bench_ratio_grid(dab, ab, k, p=192, nrhss=(80, 160, 320), r12s=(0.5, 0.75, 1.0, 1.25, 1.5),
                     r13s=(1.0, 1.5, 2.0, 2.5, 3.0)):
    """The partition-ratio experiment on the GPU: factor and solve times of
    the headline band over an (R12, R13) grid of partition sizes, with the
    paper's thread layout at p = 192 = 128 + 64 (64 two-thread partitions
    split in two leaves, 62 single-thread inner partitions, first and last),
    for nrhs = 80, 160 and 320 (nrhs / k = 1/2, 1, 2).  K is measured as the
    paper prescribes (solve time over factor time at nrhs = k, equal
    sizes) and the model's compromise ratios R13 (eq. R13_calculation) and
    R12 = R13 / 2 are timed beside the grid."""
    import torch
    from paper_1811_03559_amd import spike
    n = ab.shape[0]
    nmax = max(nrhss)
    Fbig = torch.randn((nmax, n), dtype=torch.float64, device=dab.device,
                       generator=torch.Generator(device=dab.device).manual_seed(1811))
    base = dict(p=p, tree="paper", nrhs_max=nmax)

    def measure(opts):
        holder = {}

        def fac():
            holder["f"] = spike.Factorization(dab, k, k, **opts)
        t_f = _timed(fac)
        f = holder["f"]
        res = {"factor_ms": t_f}
        for r in nrhss:
            B = Fbig[:r].clone()
            res["solve_ms_nrhs%d" % r] = _timed(lambda: f.solve_(B))
        f.close()
        return res

    eq = measure(dict(base, sizing="equal"))
    K = eq["solve_ms_nrhs%d" % k] / eq["factor_ms"] if ("solve_ms_nrhs%d" % k) in eq else None
    grid = []
    for r12 in r12s:
        for r13 in r13s:
            try:
                m = measure(dict(base, sizing="ratios", r12=r12, r13=r13))
            except spike.SpikeError as e:
                m = {"error": e.code}
            m.update({"r12": r12, "r13": r13})
            grid.append(m)
    model = {}
    if K:
        for r in nrhss:
            R13 = (1.0 + 1.5 * K + 2.0 * K * r / k) / (1.0 + K * r / k)
            m = measure(dict(base, sizing="ratios", r12=R13 / 2, r13=R13))
            model["nrhs%d" % r] = {"r12": R13 / 2, "r13": R13, "factor_ms": m["factor_ms"],
                                   "solve_ms": m["solve_ms_nrhs%d" % r]}
    best = {}
    for r in nrhss:
        ok = [g for g in grid if "error" not in g]
        for what, key in (("factor", lambda g: g["factor_ms"]),
                          ("solve", lambda g: g["solve_ms_nrhs%d" % r]),
                          ("combined", lambda g: g["factor_ms"] + g["solve_ms_nrhs%d" % r])):
            g = min(ok, key=key)
            best["nrhs%d_%s" % (r, what)] = {"r12": g["r12"], "r13": g["r13"], "ms": key(g)}
    return {"p": p, "tree": "paper", "K": K, "equal_sizes": eq, "grid": grid, "model_ratios": model,
            "best": best}


def bench_pivoting(n=500_000, k=64, nrhs=16, ps=(2, 3, 256)):
    """Pivoting SPIKE next to non-pivoting SPIKE (with boosting) on the
    ill-conditioned N(0,1) row-scaled band: errors against the manufactured
    solution, residuals, FP64 refinement of the pivoting factors (<= 3
    steps), the boosted non-pivoting factors used as a preconditioner for
    FP64 refinement (<= 10 steps), and both factorisations as right
    preconditioners of GMRES(30) (<= 150 Arnoldi steps; `refine_iters`
    then counts the Arnoldi steps and `berr` is GMRES's final backward
    error)."""
    import torch
    from paper_1811_03559_amd import inputs, spike
    ab, kl, ku, Xtrue = inputs.cfg2(n=n, k=k, nrhs=nrhs)
    F = np.stack([band_matvec(ab, kl, ku, Xtrue[j]) for j in range(nrhs)])
    dab = torch.from_numpy(ab).cuda()
    dF = torch.from_numpy(F).cuda()
    import oracle
    t0 = time.perf_counter()
    kappa = oracle.cond1(ab, kl, ku)
    out = {"n": n, "k": k, "nrhs": nrhs, "oracle_kappa1": kappa, "oracle_kappa1_s": time.perf_counter() - t0}
    for p in ps:
        row = {}
        for label, opts in (("pivoting", dict(pivot=True)), ("non_pivoting", dict(pivot=False)),
                            ("pivoting_refined", dict(pivot=True, max_refine=3)),
                            ("boosted_refined", dict(pivot=False, max_refine=10)),
                            ("pivoting_gmres", dict(pivot=True)), ("boosted_gmres", dict(pivot=False))):
            holder = {}

            def fac():
                holder["f"] = spike.Factorization(dab, kl, ku, p=p, nrhs_max=nrhs, **opts)
            t_f = _timed(fac)
            f = holder["f"]
            B = dF.clone()
            gm = {}
            if label.endswith("gmres"):
                t_s = _timed(lambda: gm.update(f.solve_gmres_(B, restart=30, max_iters=150)))
            else:
                t_s = _timed(lambda: f.solve_(B))
            X = B.cpu().numpy()
            info = f.info()
            if gm:
                info["refine_iters"] = gm["iters"]
                info["berr"] = gm["berr"]
            row[label] = {"factor_ms": t_f, "solve_ms": t_s,
                          "relres": max(relres(ab, kl, ku, X[j], F[j]) for j in range(0, nrhs, 5)),
                          "fwd_err": fwd_err(X, Xtrue), "n_boosts": info["n_boosts"],
                          "refine_iters": info["refine_iters"], "berr": info["berr"], "info": info["info"]}
            f.close()
        out["p%d" % p] = row
    return out


def bench_complex(n=500_000, k=80, nrhs=1, p=256):
    """A complex band of half the headline order with half its bandwidth
    (its real embedding is n = 10^6 with 161 sub- and superdiagonals, the
    headline's size), diagonally dominant, FP64 and FP32 factors with
    refinement: factorisation and A, A^T, A^H solves, residuals from the
    complex oracle's product."""
    import torch
    import oracle
    from paper_1811_03559_amd import inputs, spike
    rng = inputs.rng_for(inputs.seed_for(5))
    ab = inputs.zband_dominant(n, k, k, rng, diag_mult=1.05)
    Xt = inputs.zrhs(n, nrhs, rng)
    out = {"n": n, "k": k, "nrhs": nrhs, "p": p}
    dab = torch.from_numpy(ab).cuda()
    for label, opts in (("fp64", {}), ("mixed", dict(precision="mixed"))):
        holder = {}

        def fac():
            holder["f"] = spike.ZFactorization(dab, k, k, p=p, nrhs_max=max(nrhs, 1), **opts)
        t_f = _timed(fac)
        f = holder["f"]
        row = {"factor_ms": t_f}
        for trans in ("N", "T", "C"):
            F = oracle.zgbmv(ab, k, k, Xt, trans=trans)
            dF = torch.from_numpy(F).cuda()
            B = dF.clone()
            row["solve_%s_ms" % trans] = _timed(lambda: (B.copy_(dF), f.solve_(B, trans=trans)))
            X = B.cpu().numpy()
            row["relres_%s" % trans] = oracle.zrelres(ab, k, k, X, F, trans=trans)
            row["fwd_err_%s" % trans] = fwd_err(X, Xt)
        row["info"] = f.info()
        f.close()
        out[label] = row
    return out


def bench_mixed(n=1_000_000, k=128, nrhs=32, p=256):
    """FP32 block factors and tips with FP64 reduced system, residual and
    refinement, against plain FP64, both to a backward error of 1e-13."""
    import torch
    from paper_1811_03559_amd import inputs, spike
    ab, kl, ku, F = inputs.cfg3(n=n, k=k, nrhs=nrhs)
    dab = torch.from_numpy(ab).cuda()
    dF = torch.from_numpy(F).cuda()
    out = {"n": n, "k": k, "nrhs": nrhs, "p": p}
    for label, opts in (("fp64", {}), ("mixed", dict(precision="mixed"))):
        res = []
        for _ in range(3):
            holder = {}

            def fac():
                holder["f"] = spike.Factorization(dab, kl, ku, p=p, nrhs_max=nrhs, **opts)
            t_f = _timed(fac)
            f = holder["f"]
            B = dF.clone()
            t_s = _timed(lambda: f.solve_(B))
            res.append((t_f + t_s, t_f, t_s, f, B))
        res.sort(key=lambda r: r[0])
        t, t_f, t_s, f, B = res[1]
        X = B.cpu().numpy()
        info = f.info()
        out[label] = {"total_ms": t, "factor_ms": t_f, "solve_ms": t_s,
                      "relres": max(relres(ab, kl, ku, X[j], F[j]) for j in range(0, nrhs, 8)),
                      "refine_iters": info["refine_iters"], "berr": info["berr"]}
        for r in res:
            r[3].close()
    out["speedup"] = out["fp64"]["total_ms"] / out["mixed"]["total_ms"]
    out["factor_speedup"] = out["fp64"]["factor_ms"] / out["mixed"]["factor_ms"]
    return out


def bench_serving(nreq=1024, budget_gib=64, pool_per_bucket=4, seed=None):
    """Serving stream: a burst (all requests at t = 0) gives the saturated
    throughput; Poisson arrivals at 0.5x and 0.9x of it give the latency
    under load.  Latency is submission (= arrival) to observed completion."""
    import torch
    from paper_1811_03559_amd import inputs, spike
    pool, reqs = inputs.cfg4_requests(nreq, seed, pool_per_bucket)
    t_gen = time.perf_counter()
    mats = {}
    for (cls, k), members in pool.items():
        for j, (n, sd) in enumerate(members):
            ab = inputs.cfg4_matrix(cls, k, n, sd)
            mats[(cls, k, j)] = (ab, torch.from_numpy(ab).cuda())
    t_gen = time.perf_counter() - t_gen
    torch.cuda.synchronize()
    # every request with n <= 2^16 and one in 20 of the rest is checked
    chk_rng = np.random.default_rng(7)
    check = [pool[(r["cls"], r["k"])][r["member"]][0] <= (1 << 16) or chk_rng.random() < 0.05
             for r in reqs]

    def run(rate):
        srv = spike.Server(hbm_budget=budget_gib << 30, max_inflight=64, streams=4, batch_window=32)
        arr = np.random.default_rng(11)
        Bs, Fs, tickets = [], {}, []
        gen = torch.Generator(device="cuda")
        for i, r in enumerate(reqs):
            n = pool[(r["cls"], r["k"])][r["member"]][0]
            gen.manual_seed(r["rhs_seed"])
            B = torch.randn(r["nrhs"], n, dtype=torch.float64, device="cuda", generator=gen)
            if check[i]:
                Fs[i] = B[:2].cpu().numpy()
            Bs.append(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_next = t0
        for i, r in enumerate(reqs):
            if rate:
                t_next += arr.exponential(1.0 / rate)
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            ab, dab = mats[(r["cls"], r["k"], r["member"])]
            tickets.append(srv.submit(r["id"], dab, r["k"], r["k"], Bs[i], trans=r["trans"],
                                      pivot=r["cls"] == "piv", precision=r["precision"],
                                      nrhs_max=64))
        sts = [srv.wait(t) for t in tickets]
        t1 = time.perf_counter()
        st = srv.stats()
        srv.close()
        import oracle
        worst = {"dom_fp64": 0.0, "dom_mixed": 0.0, "piv": 0.0}
        lat = {"dom_fp64": [], "dom_mixed": [], "piv": []}
        for i, r in enumerate(reqs):
            key = "piv" if r["cls"] == "piv" else "dom_" + r["precision"]
            if sts[i]["state"] == 2:
                lat[key].append(sts[i]["latency_s"])
            if not check[i] or sts[i]["state"] != 2:
                continue
            ab = mats[(r["cls"], r["k"], r["member"])][0]
            X = Bs[i][:2].cpu().numpy()
            e = max(oracle.relres(ab, r["k"], r["k"], X[j], Fs[i][j], trans=r["trans"])
                    for j in range(min(2, r["nrhs"])))
            worst[key] = max(worst[key], e)
        by_class = {c: {"requests": len(v), "p50_ms": float(np.percentile(v, 50)) * 1e3 if v else None,
                        "p99_ms": float(np.percentile(v, 99)) * 1e3 if v else None} for c, v in lat.items()}
        print("[bench] serving rate=%s: %d done in %.2f s" % (rate, st["completed"], t1 - t0),
              file=sys.stderr, flush=True)
        return {"requests": len(reqs), "failed": st["failed"], "completed": st["completed"],
                "wall_s": t1 - t0, "solves_per_s": st["solves_per_s"],
                "p50_ms": st["p50_s"] * 1e3, "p99_ms": st["p99_s"] * 1e3, "max_ms": st["max_s"] * 1e3,
                "factorizations": st["factorizations"], "evictions": st["evictions"],
                "hbm_high_water_gib": st["hbm_high_water"] / 2.0 ** 30,
                "checked": int(sum(check)), "max_relres": worst, "by_class": by_class}

    burst = run(None)
    theta = burst["solves_per_s"]
    out = {"pool_matrices": len(mats), "generation_s": t_gen, "budget_gib": budget_gib,
           "burst": burst,
           "poisson_0.5": run(0.5 * theta), "poisson_0.9": run(0.9 * theta)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--k", type=int, default=160)
    ap.add_argument("--p", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-detail", action="store_true",
                    help="skip every detail section (phase times and the other workloads)")
    ap.add_argument("--sections", default="psweep,ratios,pivoting,mixed,complex,serving",
                    help="detail sections: psweep, ratios, pivoting, mixed, complex, serving")
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
        return

    import torch
    from paper_1811_03559_amd import inputs, spike

    t_start = time.perf_counter()
    dev = torch.device("cuda:0")
    n, k, p = args.n, args.k, args.p
    t_gen = time.perf_counter()
    ab, kl, ku, F = inputs.cfg1(n=n, k=k, nrhs=1)
    F64 = inputs.rhs(n, 64, inputs.rng_for(inputs.seed_for(1, 1)))
    t_gen = time.perf_counter() - t_gen
    dab = torch.from_numpy(ab).to(dev)
    dF = torch.from_numpy(F).to(dev)
    dF64 = torch.from_numpy(F64).to(dev)
    B = torch.empty_like(dF)
    Bt = torch.empty_like(dF)
    opts = dict(p=p, nrhs_max=64)
    ws = torch.empty(spike.workspace_size(n, kl, ku, **opts), dtype=torch.uint8, device=dev)
    plan = spike.plan_query(n, kl, ku, **opts)

    def step():
        fac = spike.Factorization(dab, kl, ku, workspace=ws, **opts)
        B.copy_(dF)
        fac.solve_(B)
        Bt.copy_(dF)
        fac.solve_(Bt, trans=True)
        fac.close()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel times of untimed steps (every launch bracketed by events), to
    # find the dominant kernel; the timed steps then carry the events of that
    # kernel only, so that the other launches run without event overhead
    nprof = max(1, min(args.steps, 3))
    spike.profile_only(None)
    spike.profile_enable(True)
    for _ in range(nprof):
        step()
    torch.cuda.synchronize()
    prof = spike.profile_report()
    spike.profile_enable(False)
    kernels = {name: {"calls": c, "avg_ms": ms / max(c, 1), "ms_per_step": ms / nprof}
               for name, (c, ms) in prof.items()}
    dom = max(kernels, key=lambda nm: kernels[nm]["ms_per_step"])
    spike.profile_only(dom)
    spike.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_prof = spike.profile_report()
    spike.profile_enable(False)
    spike.profile_only(None)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    c_dom, ms_dom = dom_prof[dom]
    kernels[dom].update({"calls_timed": c_dom, "avg_ms": ms_dom / max(c_dom, 1),
                         "ms_per_step": ms_dom / args.steps})

    # roofline of the kernel with the largest share of a step
    work = step_work(plan["sizes"], k, 1)
    workload = "spike_step_n%d_k%d_p%d" % (n, k, p)
    for name, kt in kernels.items():
        if name in work:
            r = roofline(name, work[name], kt, workload)
            kt.update({x: r[x] for x in ("bound", "achieved", "unit", "frac", "traffic")})
            if "hbm_gbs" in r:
                kt["hbm_gbs"], kt["hbm_frac"] = r["hbm_gbs"], r["hbm_frac"]
    roof = roofline(dom, work.get(dom), kernels[dom], workload)
    detail = {"kernels": kernels, "generation_s": t_gen}
    if not args.no_detail:
        # phase times, checked results, solve bandwidth, nrhs = 64
        fac = spike.Factorization(dab, kl, ku, workspace=ws, **opts)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
        ev[0].record()
        fac.close()
        fac = spike.Factorization(dab, kl, ku, workspace=ws, **opts)
        ev[1].record()
        B.copy_(dF)
        ev[2].record()
        fac.solve_(B)
        ev[3].record()
        Bt.copy_(dF)
        ev[4].record()
        fac.solve_(Bt, trans=True)
        ev[5].record()
        B64 = dF64.clone()
        ev[6].record()
        fac.solve_(B64)
        ev[7].record()
        torch.cuda.synchronize()
        t_fac = ev[0].elapsed_time(ev[1])
        t_sn = ev[2].elapsed_time(ev[3])
        t_st = ev[4].elapsed_time(ev[5])
        t_s64 = ev[6].elapsed_time(ev[7])
        solve_bytes = 2 * work["k_fdstage"]["bytes"]
        X = B.cpu().numpy()[0]
        Xt = Bt.cpu().numpy()[0]
        X64 = B64.cpu().numpy()
        detail.update({
            "factor_ms": t_fac, "solve_ms_nrhs1": t_sn, "solve_t_ms_nrhs1": t_st,
            "solve_ms_nrhs64": t_s64,
            "solve_hbm_gbs_nrhs1": solve_bytes / (t_sn / 1e3) / 1e9,
            "solve_t_hbm_gbs_nrhs1": solve_bytes / (t_st / 1e3) / 1e9,
            "resident_solves_per_s_nrhs1": 1000.0 / t_sn,
            "relres_n": relres(ab, kl, ku, X, F[0]),
            "relres_t": relres(ab, kl, ku, Xt, F[0], trans=True),
            "relres_n_nrhs64_col0": relres(ab, kl, ku, X64[0], F64[0]),
            "info": fac.info(),
        })
        fac.close()
        secs = set(args.sections.split(",")) if args.sections else set()
        del B64
        def note(msg):
            print("[bench] %s (%.1f s)" % (msg, time.perf_counter() - t_start), file=sys.stderr, flush=True)
        note("cfg0")
        detail["cfg0"] = bench_cfg0()
        if "psweep" in secs:
            note("p sweep")
            detail["p_sweep"] = bench_p_sweep(dab, ab, k, F)
        del dF64, ws
        torch.cuda.empty_cache()
        if "ratios" in secs:
            note("partition ratio grid")
            detail["ratio_grid"] = bench_ratio_grid(dab, ab, k)
        del dab, dF
        torch.cuda.empty_cache()
        if "pivoting" in secs:
            note("pivoting")
            detail["pivoting"] = bench_pivoting()
            torch.cuda.empty_cache()
        if "mixed" in secs:
            note("mixed precision")
            detail["mixed_precision"] = bench_mixed()
            torch.cuda.empty_cache()
        if "complex" in secs:
            note("complex")
            detail["complex"] = bench_complex()
            torch.cuda.empty_cache()
        if "serving" in secs:
            note("serving")
            detail["serving"] = bench_serving(args.serve_requests)
            torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": 1000.0 / ms_per_step, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded PCG64 band, diagonal = row abs-sum * 1.05)",
        "config": {"workload": "recursive SPIKE factor + solve + transpose solve, FP64, n=%d, "
                               "kl=ku=%d, nrhs=1, p=%d" % (n, k, p),
                   "n": n, "kl": kl, "ku": ku, "nrhs": 1, "p": p, "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, one core, full size) (%.1f s)" % (time.perf_counter() - t_start),
              file=sys.stderr, flush=True)
        cb = cpu_baseline(ab, kl, ku, F)
        Xo, Xot = cb.pop("_x")
        out["cpu_baseline"] = cb
        # the GPU step's solutions against the oracle's, element by element
        if "relres_n" in detail:
            detail["vs_oracle_n"] = fwd_err(X, Xo[0])
            detail["vs_oracle_t"] = fwd_err(Xt, Xot[0])
    out["detail"] = detail
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
