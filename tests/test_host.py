"""Host-side checks that need no GPU: the C ABI library loads and exports
every symbol its header declares, and the planner's partition sizes, merge
tree and reduced-system shape match the paper's closed forms."""
import math

import pytest

import oracle
from paper_1811_03559_amd import spike


def test_library_exports_every_header_symbol():
    names = spike.header_symbols()
    assert {"spike_factor", "spike_solve", "spike_solve_transpose", "spike_workspace_size",
            "spike_info", "spike_destroy"} <= set(names)
    L = spike.lib()
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 7, 8, 13, 250, 256, 500])
def test_plan_tree_shape(p):
    kl = ku = 4
    info = spike.plan_query(100_000, kl, ku, p=p)
    assert info["p"] == p
    assert info["merges"] == p - 1                         # p-1 interface solves
    assert info["levels"] == (0 if p == 1 else math.ceil(math.log2(p)))
    assert info["reduced_size"] == (kl + ku) * (p - 1)     # 2k(p-1) unknowns
    assert sum(info["sizes"]) == 100_000


def _paper_admissible(t):
    """The flexible partitioning section's distribution of threads:
    t = 2^m + r threads, with 2^m <= t <= 2^(m+1) - 2 (the first and last
    partitions keep one thread),
    so 7 threads are used as 6 and 15 as 14; one thread is plain LU."""
    m = int(math.floor(math.log2(t)))
    return t == 1 or 2 ** m <= t <= 2 ** (m + 1) - 2


@pytest.mark.parametrize("p", range(1, 65))
def test_paper_tree_admits_exactly_the_paper_thread_counts(p):
    n = 600 * 64
    if _paper_admissible(p):
        info = spike.plan_query(n, 4, 4, p=p, tree="paper")
        assert info["p"] == p and info["merges"] == p - 1
        assert info["levels"] == (0 if p == 1 else math.ceil(math.log2(p)))
    else:
        with pytest.raises(spike.SpikeError) as e:
            spike.plan_query(n, 4, 4, p=p, tree="paper")
        assert e.value.code == -4
        assert spike.plan_query(n, 4, 4, p=p)["p"] == p      # the balanced tree takes any p


@pytest.mark.parametrize("t,used", [(7, 6), (15, 14), (6, 6), (3, 2)])
def test_paper_tree_lowers_the_planners_count(t, used):
    # kl = ku = 4: the planner's own count is n / 512
    assert spike.plan_query(512 * t, 4, 4)["p"] == t
    assert spike.plan_query(512 * t, 4, 4, tree="paper")["p"] == used


@pytest.mark.parametrize("p", [2, 4, 5, 6, 12, 13, 14, 17, 250, 256, 500])
def test_paper_tree_layout(p):
    """Level 1 merges the halves of the r two-thread partitions, which sit at
    the paper's partitions 2, 3, ..., r+1 (leaf pairs (1,2), (3,4), ... from
    0); every later level pairs all 2^m remaining nodes with none carried."""
    n, k = 1_000_000, 160
    m2 = 2 ** int(math.floor(math.log2(p)))
    r = p - m2
    tree = spike.plan_tree(n, k, k, p=p, tree="paper")
    assert len(tree) == p - 1
    assert sorted(m for _, _, m, _ in tree) == list(range(p - 1))
    lvl1 = [J for J in tree if J[0] == 1]
    if r:
        assert lvl1 == [(1, 2 * j - 1, 2 * j - 1, 2 * j) for j in range(1, r + 1)]
    nodes = [(0, 0)] + [(2 * j - 1, 2 * j) for j in range(1, r + 1)] + [(i, i) for i in range(2 * r + 1, p)]
    if not r:
        nodes = [(i, i) for i in range(p)]
    assert len(nodes) == m2
    first = 2 if r else 1
    for level in range(first, max(J[0] for J in tree) + 1):
        got = [(a, m, b) for lv, a, m, b in tree if lv == level]
        want = [(nodes[i][0], nodes[i][1], nodes[i + 1][1]) for i in range(0, len(nodes), 2)]
        assert got == want, level
        nodes = [(nodes[i][0], nodes[i + 1][1]) for i in range(0, len(nodes), 2)]
    assert nodes == [(0, p - 1)]
    # the paper's R12 = R13 / 2 gives every half of a two-thread partition
    # the single-thread size n3, so both trees size the partitions alike
    for sizing in ("equal", "r13"):
        a = spike.plan_query(n, k, k, p=p, sizing=sizing, nrhs_hint=1)["sizes"]
        b = spike.plan_query(n, k, k, p=p, sizing=sizing, nrhs_hint=1, tree="paper")["sizes"]
        assert a == b


def test_unknown_tree_is_an_error():
    import ctypes
    o = spike.make_opts()
    o.tree = 2
    info = spike.PlanInfo()
    assert spike.lib().spike_plan_query(1000, 2, 2, ctypes.byref(o), ctypes.byref(info), None) == -4


def test_cfg0_equal_sizes():
    info = spike.plan_query(4096, 4, 4, p=3)
    assert info["sizes"] == [1365, 1365, 1366]
    assert info["reduced_size"] == 16


@pytest.mark.parametrize("nrhs,K", [(1, 1.0), (80, 4.0 / 3.0), (160, 4.0 / 3.0), (320, 2.0)])
def test_r13_sizing_matches_closed_form(nrhs, K):
    n, k, p = 1_000_000, 160, 16
    info = spike.plan_query(n, k, k, p=p, sizing="r13", K=K, nrhs_hint=nrhs)
    R13 = oracle.r13(K, nrhs / k)
    n1 = n * R13 / (2 * R13 + p - 2)
    n3 = n / (2 * R13 + p - 2)
    sz = info["sizes"]
    assert sum(sz) == n
    assert sz[0] == sz[-1] == math.floor(n1)
    assert all(abs(s - n3) <= 1 + p for s in sz[1:-1])
    assert sz[0] / sz[1] == pytest.approx(R13, rel=1e-3)


@pytest.mark.parametrize("p,tree,x", [(11, "paper", 3), (21, "paper", 5), (16, "paper", 0),
                                       (11, "balanced", 0), (24, "balanced", 0)])
@pytest.mark.parametrize("r12,r13", [(1.2, 2.0), (1.0, 2.0), (1.5, 1.0), (0.6, 3.0)])
def test_explicit_ratio_sizing_matches_closed_form(p, tree, x, r12, r13):
    """Sizing from explicit R12 = n1/n2 and R13 = n1/n3 (the load-balancing
    section's partition-size equations): x two-thread partitions (the paper
    layout's r = p - 2^m, each split in two leaves of n2 / 2), y = p - 2 - 2x
    single-thread inner partitions."""
    n, k = 1_000_003, 40
    sz = spike.plan_query(n, k, k, p=p, sizing="ratios", r12=r12, r13=r13, tree=tree)["sizes"]
    y = p - 2 - 2 * x
    den = 2 * r12 * r13 + x * r13 + y * r12
    n1, n2, n3 = n * r12 * r13 / den, n * r13 / den, n * r12 / den
    assert len(sz) == p and sum(sz) == n
    assert 2 * n1 + x * n2 + y * n3 == pytest.approx(n, rel=1e-12)
    assert sz[0] == sz[-1] == math.floor(n1)
    for i in range(1, 2 * x + 1):
        assert abs(sz[i] - n2 / 2) <= 3, (i, sz[i], n2 / 2)
    for i in range(2 * x + 1, p - 1):
        assert abs(sz[i] - n3) <= 3, (i, sz[i], n3)
    assert sz[0] / sz[-2 if y else 1] == pytest.approx(r13 if y else 2 * r12, rel=1e-4)
    if x:
        assert (sz[1] + sz[2]) == pytest.approx(n1 / r12, abs=6)


def test_ratio_sizing_with_half_r13_equals_model_sizing():
    """R12 = R13 / 2 (the paper's choice n2 = 2 n3) given explicitly sizes
    the partitions as the model sizing does with the same R13, for both
    layouts."""
    n, k, p, K, nrhs = 1_000_000, 160, 12, 4.0 / 3.0, 80
    R13 = oracle.r13(K, nrhs / k)
    for tree in ("balanced", "paper"):
        a = spike.plan_query(n, k, k, p=p, sizing="r13", K=K, nrhs_hint=nrhs, tree=tree)["sizes"]
        b = spike.plan_query(n, k, k, p=p, sizing="ratios", r12=R13 / 2, r13=R13, tree=tree)["sizes"]
        assert max(abs(u - v) for u, v in zip(a, b)) <= 1, tree


def test_ratio_sizing_rejects_nonpositive_ratios():
    for r12, r13 in ((0.0, 2.0), (1.0, 0.0), (-1.0, 2.0), (float("nan"), 2.0)):
        with pytest.raises(spike.SpikeError) as e:
            spike.plan_query(100_000, 4, 4, p=6, sizing="ratios", r12=r12, r13=r13)
        assert e.value.code == -4
    # ratios so skewed that a partition falls below kl + ku rows
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(10_000, 40, 40, p=6, sizing="ratios", r12=1.0, r13=1000.0)
    assert e.value.code == -4


def test_argument_errors():
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(-1, 2, 2)
    assert e.value.code == -1
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(100, -1, 2)
    assert e.value.code == -2
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(100, 2, -3)
    assert e.value.code == -3
    # infeasible p: partitions smaller than kl + ku
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(100, 30, 30, p=5)
    assert e.value.code == -4
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(10, 1, 1, p=11)
    assert e.value.code == -4


def test_workspace_grows_with_problem():
    a = spike.workspace_size(10_000, 4, 4, p=4)
    b = spike.workspace_size(20_000, 4, 4, p=4)
    c = spike.workspace_size(20_000, 8, 8, p=4)
    d = spike.workspace_size(20_000, 8, 8, p=4, pivot=True)
    assert a < b < c < d
    assert spike.workspace_size(0, 3, 3) > 0


# ctypes mirrors of the header's structs, checked field by field against what
# a C compiler lays out (gcc on the header itself).
_STRUCTS = [("spike_opts", "Opts"), ("spike_status", "Status"), ("spike_plan_info", "PlanInfo"),
            ("spike_kernel_time", "KernelTime"), ("spike_tune_result", "TuneResult"),
            ("spike_server_opts", "ServerOpts"), ("spike_request", "Request"),
            ("spike_request_status", "RequestStatus"), ("spike_server_report", "ServerReport"),
            ("spike_krylov_opts", "KrylovOpts"), ("spike_krylov_result", "KrylovResult")]


def test_ctypes_structs_match_the_c_layout(tmp_path):
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "spike.h"', "int main(void) {"]
    for cname, pyname in _STRUCTS:
        cls = getattr(spike, pyname)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, pyname in _STRUCTS:
        cls = getattr(spike, pyname)
        assert int(out["%s size" % cname]) == __import__("ctypes").sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_server_argument_errors_need_no_device():
    import ctypes
    L = spike.lib()
    o = spike.ServerOpts()
    L.spike_server_default_opts(ctypes.byref(o))
    assert o.hbm_budget == 16 << 30 and o.max_inflight == 64 and o.streams == 4 and o.batch_window == 32
    bad = spike.ServerOpts(hbm_budget=1 << 20, max_inflight=0, streams=1, batch_window=1)
    s = ctypes.c_void_p()
    assert L.spike_server_create(ctypes.byref(bad), ctypes.byref(s)) == -1
    bad = spike.ServerOpts(hbm_budget=1 << 20, max_inflight=4, streams=17, batch_window=1)
    assert L.spike_server_create(ctypes.byref(bad), ctypes.byref(s)) == -1
    assert L.spike_server_create(None, None) == -2
    # the caller provides the device pool: a missing or misaligned one is refused
    # before anything touches a device
    assert o.dpool is None
    assert L.spike_server_create(ctypes.byref(o), ctypes.byref(s)) == -1
    odd = spike.ServerOpts(hbm_budget=1 << 20, max_inflight=4, streams=1, batch_window=1, dpool=0x1008)
    assert L.spike_server_create(ctypes.byref(odd), ctypes.byref(s)) == -1
    st = spike.RequestStatus()
    rep = spike.ServerReport()
    t = ctypes.c_int64()
    assert L.spike_server_submit(None, None, ctypes.byref(t)) == -1
    assert L.spike_server_poll(None, 1, ctypes.byref(st)) == -1
    assert L.spike_server_wait(None, 1, ctypes.byref(st)) == -1
    assert L.spike_server_release(None, 1) == -1
    assert L.spike_server_drain(None) == -1
    assert L.spike_server_stats(None, ctypes.byref(rep)) == -1
    assert L.spike_server_destroy(None) == -1


def test_binding_rejects_bad_tensors_before_any_library_call(monkeypatch):
    """Every binding entry point that hands tensor pointers to the library
    refuses float32, host-resident and transposed (non-contiguous) tensors with
    ValueError before it calls into the library."""
    import types
    import torch

    calls = []

    class Trap:
        def __getattr__(self, name):
            calls.append(name)
            raise AssertionError("library called: " + name)

    monkeypatch.setattr(spike, "lib", lambda: Trap())
    n, kl, ku = 40, 2, 3
    good_ab = torch.zeros((n, kl + ku + 1), dtype=torch.float64)
    bad_bands = [good_ab.float(), good_ab,                       # float32; host (no CUDA here)
                 torch.zeros((kl + ku + 1, n), dtype=torch.float64).t()]   # transposed view
    for ab in bad_bands:
        with pytest.raises(ValueError):
            spike.Factorization(ab, kl, ku)
        with pytest.raises(ValueError):
            spike.autotune(ab, kl, ku)
        srv = spike.Server.__new__(spike.Server)
        with pytest.raises(ValueError):
            srv.submit(1, ab, kl, ku, torch.zeros((1, n), dtype=torch.float64))
    # right-hand sides: a fake factorisation that fails if its handle is read
    fac = types.SimpleNamespace(n=n)
    bad_rhs = [torch.zeros((2, n), dtype=torch.float32), torch.zeros((2, n), dtype=torch.float64),
               torch.zeros((n, 2), dtype=torch.float64).t(), torch.zeros((2, n + 1), dtype=torch.float64)]
    for B in bad_rhs:
        with pytest.raises(ValueError):
            spike.solve_batch([fac], [B])
        with pytest.raises(ValueError):
            spike.Factorization.solve_(fac, B)
        with pytest.raises(ValueError):
            spike._check_rhs(B, n)
    assert calls == []


def test_factor_argument_errors_need_no_device():
    """spike_factor validates its arguments on the host, in argument order,
    before it touches the device: -5 for ldab < kl + ku + 1, -7 for a NULL or
    misaligned workspace, -8 for a workspace smaller than the planner's size,
    -10 for a NULL handle pointer (the device pointers below are never
    dereferenced)."""
    import ctypes
    L = spike.lib()
    n, kl, ku = 1000, 3, 2
    o = spike.make_opts(p=4)
    need = spike.workspace_size(n, kl, ku, p=4)
    fake_ab = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)             # 256-byte aligned
    h = ctypes.c_void_p()
    f = L.spike_factor
    assert f(-1, kl, ku, fake_ab, 6, ctypes.byref(o), ws, need, None, ctypes.byref(h)) == -1
    assert f(n, -1, ku, fake_ab, 6, ctypes.byref(o), ws, need, None, ctypes.byref(h)) == -2
    assert f(n, kl, -1, fake_ab, 6, ctypes.byref(o), ws, need, None, ctypes.byref(h)) == -3
    assert f(n, kl, ku, None, 6, ctypes.byref(o), ws, need, None, ctypes.byref(h)) == -4
    assert f(n, kl, ku, fake_ab, kl + ku, ctypes.byref(o), ws, need, None, ctypes.byref(h)) == -5
    bad = spike.make_opts(p=n + 1)
    assert f(n, kl, ku, fake_ab, 6, ctypes.byref(bad), ws, need, None, ctypes.byref(h)) == -6
    assert f(n, kl, ku, fake_ab, 6, ctypes.byref(o), None, need, None, ctypes.byref(h)) == -7
    assert f(n, kl, ku, fake_ab, 6, ctypes.byref(o), ctypes.c_void_p(0x200008), need, None,
             ctypes.byref(h)) == -7
    assert f(n, kl, ku, fake_ab, 6, ctypes.byref(o), ws, need - 1, None, ctypes.byref(h)) == -8
    assert f(n, kl, ku, fake_ab, 6, ctypes.byref(o), ws, need, None, None) == -10
    assert h.value is None
    # solves and queries on an invalid handle
    assert L.spike_solve(None, 1, fake_ab, n, None) == -1
    assert L.spike_solve_transpose(None, 1, fake_ab, n, None) == -1
    st = spike.Status()
    assert L.spike_info(None, ctypes.byref(st)) == -1
    assert L.spike_destroy(None) == -1


def test_pivoting_limited_to_32_column_panels():
    """The planner refuses partial pivoting where the leaf kernels would need
    16-column panels (FP64, kl = ku > 160), and accepts it up to 160 and for
    every non-pivoting bandwidth the engines serve."""
    n = 50000
    assert spike.plan_query(n, 160, 160, p=8, pivot=True)["p"] == 8
    assert spike.plan_query(n, 200, 200, p=8)["p"] == 8
    with pytest.raises(spike.SpikeError) as e:
        spike.plan_query(n, 200, 200, p=8, pivot=True)
    assert e.value.code == -4
    # FP32 factors halve the LDS per element: 32-column panels still fit
    assert spike.plan_query(n, 200, 200, p=8, pivot=True, precision="mixed")["p"] == 8


def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache's text format: load merges entries, save writes them
    back (the same 16 fields), a malformed line is refused after the good
    lines before it, a missing file is an error."""
    spike.tune_cache_clear()
    assert spike.tune_cache_size() == 0
    src = tmp_path / "tune.txt"
    src.write_text("# n kl ku log2_nrhs precision pivot p sizing tree K nrhs_hint r12 r13 f_ms s_ms cand\n"
                   "1000000 160 160 0 0 0 256 0 0 0 1 0 0 13.5 5.25 6\n"
                   "500000 64 64 4 0 1 250 1 1 0.75 16 0 0 40 15 7\n")
    spike.tune_cache_load(src)
    assert spike.tune_cache_size() == 2
    out = tmp_path / "out.txt"
    spike.tune_cache_save(out)
    rows = sorted(line.split() for line in out.read_text().splitlines())
    assert len(rows) == 2 and all(len(r) == 16 for r in rows)
    by_n = {r[0]: r for r in rows}
    assert by_n["1000000"][6:9] == ["256", "0", "0"] and float(by_n["1000000"][13]) == 13.5
    assert by_n["500000"][4:9] == ["0", "1", "250", "1", "1"] and float(by_n["500000"][9]) == 0.75
    spike.tune_cache_clear()
    spike.tune_cache_load(out)
    assert spike.tune_cache_size() == 2
    bad = tmp_path / "bad.txt"
    bad.write_text("1000 4 4 0 0 0 3 0 0 0 1 0 0 1 1 1\n1000 4 4 0 0 0 3 7 0 0 1 0 0 1 1 1\n")
    spike.tune_cache_clear()
    with pytest.raises(spike.SpikeError) as e:
        spike.tune_cache_load(bad)
    assert e.value.code == -3
    assert spike.tune_cache_size() == 1
    with pytest.raises(spike.SpikeError) as e:
        spike.tune_cache_load(tmp_path / "missing.txt")
    assert e.value.code == -2
    spike.tune_cache_clear()


def test_profile_only_name_length():
    assert spike.lib().spike_profile_only(b"x" * 48) == -1
    spike.profile_only("k_flu")
    spike.profile_only(None)


def test_factor_batch_argument_errors():
    """spike_factor_batch checks every system before anything is launched."""
    import ctypes
    L = spike.lib()
    I64, I32, P, SZ = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    out = (P * 2)()

    def call(count, n=(1000, 2000), kl=(4, 4), ku=(4, 4), ldab=(9, 9), wb=(1 << 40, 1 << 40),
             dab=(256, 256), dw=(256, 512)):
        return L.spike_factor_batch(count, (I64 * 2)(*n), (I32 * 2)(*kl), (I32 * 2)(*ku), (P * 2)(*dab),
                                    (I64 * 2)(*ldab), None, (P * 2)(*dw), (SZ * 2)(*wb), None, out)
    assert L.spike_factor_batch(-1, None, None, None, None, None, None, None, None, None, None) == -11
    assert L.spike_factor_batch(0, None, None, None, None, None, None, None, None, None, None) == 0
    assert L.spike_factor_batch(2, None, None, None, None, None, None, None, None, None, None) == -12
    assert call(2, n=(1000, -5)) == -1
    assert call(2, kl=(4, -1)) == -2
    assert call(2, ldab=(9, 8)) == -5
    assert call(2, dw=(256, 100)) == -7
    assert call(2, wb=(1 << 40, 16)) == -8
    assert call(2, dab=(256, 0)) == -4
