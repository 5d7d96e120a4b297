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
on the host, a bounded sample scaled to the full size) and `detail`
(per-phase times, solve GB/s, nrhs = 64 solves, residuals).
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


def step_work(sizes, k, nrhs, fast_tips):
    """Algorithmic work of the kernels of one step (kl = ku = k).

    Factor:
      k_leaf_factor  block LU, 2 m k^2 flops per partition (plus, without the
                     tile-engine tips, the spike sweeps: W L-sweep 2 m k^2 and
                     [V W] U-sweep 4 m k^2 per middle partition);
      k_ftip_w       W spike L-sweep, 2 m k^2 per middle partition;
      k_ftip_u       [V W] U-sweep, 4 m k^2 per middle partition;
      k_merge_factor per merge: Schur complement S = I - W_t V_b (2k^3), LU of
                     S (2/3 k^3), alpha/beta (2k^3 sweeps + 2k^3 product) when
                     the node has a right neighbour, gamma/delta (6k^3) when it
                     has a left one, merged tips 2k^3 each (not at the root).
    Solve (bytes, nrhs = 1 is bandwidth bound): each full sweep streams half
    the band (k+1 of the 2k+1 diagonals, 8 bytes each); per solve the middle
    partitions make 4 full sweeps and first/last 2 (the paper's sweep table),
    split 2/2 and 1/1 between the two partition kernels of a solve, each of
    which also reads and writes the right-hand side once (16 bytes a row per
    column)."""
    p = len(sizes)
    n = sum(sizes)
    mid = sum(sizes[1:-1]) if p > 2 else 0
    ends = n - mid
    band_half = 8.0 * (k + 1)
    k3 = float(k) ** 3
    mflops = 0.0
    for a, b in merge_tree(p):
        nv, nw = b < p - 1, a > 0
        f = 2 * k3 + (2.0 / 3.0) * k3
        if nv:
            f += 4 * k3
        if nw:
            f += 6 * k3
        if not (a == 0 and b == p - 1):
            f += 2 * k3 * ((nv and nw) * 2 + nv + nw)
        mflops += f
    sweep = (2 * mid + ends) * band_half + 16.0 * n * nrhs
    w = {
        "k_leaf_factor": {"flops": 2.0 * n * k * k + (0.0 if fast_tips else 6.0 * mid * k * k)},
        "k_merge_factor": {"flops": mflops},
        "k_leaf_dstage": {"bytes": sweep},
        "k_leaf_retrieve": {"bytes": sweep},
        "k_leaf_zsweep": {"bytes": sweep},
        "k_leaf_dtstage": {"bytes": sweep},
    }
    if fast_tips:
        w["k_ftip_w"] = {"flops": 2.0 * mid * k * k, "engine": "mfma"}
        w["k_ftip_u"] = {"flops": 4.0 * mid * k * k, "engine": "mfma"}
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
    """SHA-256 over the library's kernel sources (names and bytes, sorted)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1811_03559_amd", "csrc")
    for f in sorted(os.listdir(d)):
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


def roofline(name, work, timing, steps, workload):
    """Roofline entry of one kernel: algorithmic work per launch over its
    average launch time (launches of one step may differ in size, so the
    per-step work over the per-step time is used; for one launch a step the
    two agree)."""
    traffic = measured_traffic(name, workload)
    if work is None:
        return {"kernel": name, "bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": None, "traffic": traffic}
    t_step = timing["ms_per_step"] / 1000.0
    if "flops" in work:
        ach = work["flops"] / t_step / 1e12
        return {"kernel": name, "bound": work.get("engine", "alu"), "achieved": ach,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "traffic": traffic, "work_per_step": work["flops"]}
    ach = work["bytes"] / t_step / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "work_per_step": work["bytes"]}


def cpu_baseline(k, n_full, n_sample=150_000):
    import oracle
    from paper_1811_03559_amd import inputs
    ab, kl, ku, F = inputs.cfg1(n=n_sample, k=k, nrhs=1)
    oracle.build()
    t0 = time.perf_counter()
    oracle.gbsv_nt(ab, kl, ku, F, pivot=False)
    dt = time.perf_counter() - t0
    t_full = dt * n_full / n_sample          # banded GE cost is linear in n
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": ("FP64 banded GE (non-pivoting LU, one factorisation, then A X = F and "
                       "A^T X = F), single thread, on the first %d rows' recipe (n=%d, k=%d, nrhs=1): "
                       "%.2f s, scaled linearly to n=%d" % (n_sample, n_sample, k, dt, n_full)),
            "sample_seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--k", type=int, default=160)
    ap.add_argument("--p", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-detail", action="store_true")
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
    spike.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = spike.profile_report()
    spike.profile_enable(False)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps

    # roofline of the kernel with the largest share of a step
    fast_tips = k <= 256 and p >= 3          # non-pivoting FP64: tile-engine spike tips
    work = step_work(plan["sizes"], k, 1, fast_tips)
    kernels = {name: {"calls": c, "avg_ms": ms / max(c, 1), "ms_per_step": ms / args.steps}
               for name, (c, ms) in prof.items()}
    dom = max(kernels, key=lambda nm: kernels[nm]["ms_per_step"])
    roof = roofline(dom, work.get(dom), kernels[dom], args.steps,
                    "spike_step_n%d_k%d_p%d" % (n, k, p))
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
        solve_bytes = 2 * work["k_leaf_dstage"]["bytes"]
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
        out["cpu_baseline"] = cpu_baseline(k, n)
    out["detail"] = detail
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
