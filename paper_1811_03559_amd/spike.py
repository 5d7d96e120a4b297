"""ctypes binding of ``libspike.so`` (the C ABI in ``include/spike.h``).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch provides device memory and the current stream.  If the library is
missing, every call raises: there is no fallback path.

Layouts: a band is a float64 tensor of shape ``(n, ldab)`` (C order), i.e.
LAPACK column-major band storage with ``ab[j, ku + i - j] = A(i, j)``.  A
right-hand-side block is a float64 tensor of shape ``(nrhs, n)`` (C order),
i.e. column-major ``n x nrhs`` with ``ldb = n``.
"""
from __future__ import annotations

import ctypes
import math
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspike.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "spike.h")

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_dbl = ctypes.c_double
_c_size = ctypes.c_size_t
_c_p = ctypes.c_void_p


class Opts(ctypes.Structure):
    _fields_ = [("p", _c_i32), ("pivot", _c_i32), ("precision", _c_i32), ("sizing", _c_i32),
                ("K", _c_dbl), ("nrhs_hint", _c_i32), ("nrhs_max", _c_i32),
                ("boost_tau", _c_dbl), ("max_refine", _c_i32), ("refine_tol", _c_dbl),
                ("tree", _c_i32), ("r12", _c_dbl), ("r13", _c_dbl)]


class Status(ctypes.Structure):
    _fields_ = [("info", _c_i64), ("n_boosts", _c_i32), ("refine_iters", _c_i32),
                ("min_abs_pivot", _c_dbl), ("berr", _c_dbl)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("p", _c_i32), ("levels", _c_i32), ("merges", _c_i32),
                ("reduced_size", _c_i64), ("workspace_bytes", _c_size)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("calls", _c_i32), ("total_ms", _c_dbl)]


class TuneResult(ctypes.Structure):
    _fields_ = [("opts", Opts), ("factor_ms", _c_dbl), ("solve_ms", _c_dbl), ("K", _c_dbl),
                ("candidates", _c_i32), ("cached", _c_i32)]


class KrylovOpts(ctypes.Structure):
    _fields_ = [("restart", _c_i32), ("max_iters", _c_i32), ("tol", _c_dbl)]


class KrylovResult(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("restarts", _c_i32), ("converged", _c_i32), ("berr", _c_dbl)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", _c_size), ("max_inflight", _c_i32), ("streams", _c_i32),
                ("batch_window", _c_i32), ("dpool", _c_p)]


class Request(ctypes.Structure):
    _fields_ = [("matrix_id", _c_i64), ("n", _c_i64), ("kl", _c_i32), ("ku", _c_i32), ("dAB", _c_p),
                ("ldab", _c_i64), ("opts", Opts), ("nrhs", _c_i32), ("dB", _c_p), ("ldb", _c_i64),
                ("trans", _c_i32)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("state", _c_i32), ("error", _c_i32), ("info", _c_i64), ("latency_s", _c_dbl)]


class ServerReport(ctypes.Structure):
    _fields_ = [("completed", _c_i64), ("failed", _c_i64), ("factorizations", _c_i64),
                ("evictions", _c_i64), ("resident", _c_i64), ("hbm_used", _c_size),
                ("hbm_high_water", _c_size), ("p50_s", _c_dbl), ("p99_s", _c_dbl), ("max_s", _c_dbl),
                ("solves_per_s", _c_dbl)]


class SpikeError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s returned %d" % (fn, code))
        self.code = code


_lock = threading.Lock()
_lib = None


def lib():
    """Load libspike.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libspike.so not built; run paper_1811_03559_amd.build.build()")
            L = ctypes.CDLL(LIB_PATH)
            L.spike_default_opts.restype = None
            L.spike_default_opts.argtypes = [ctypes.POINTER(Opts)]
            L.spike_plan_query.restype = ctypes.c_int
            L.spike_plan_query.argtypes = [_c_i64, _c_i32, _c_i32, ctypes.POINTER(Opts),
                                           ctypes.POINTER(PlanInfo), ctypes.POINTER(_c_i64)]
            L.spike_plan_tree.restype = ctypes.c_int
            L.spike_plan_tree.argtypes = [_c_i64, _c_i32, _c_i32, ctypes.POINTER(Opts),
                                          ctypes.POINTER(_c_i32)]
            L.spike_workspace_size.restype = ctypes.c_int
            L.spike_workspace_size.argtypes = [_c_i64, _c_i32, _c_i32, ctypes.POINTER(Opts),
                                               ctypes.POINTER(_c_size)]
            L.spike_factor.restype = ctypes.c_int
            L.spike_factor.argtypes = [_c_i64, _c_i32, _c_i32, _c_p, _c_i64, ctypes.POINTER(Opts),
                                       _c_p, _c_size, _c_p, ctypes.POINTER(_c_p)]
            L.spike_solve.restype = ctypes.c_int
            L.spike_solve.argtypes = [_c_p, _c_i32, _c_p, _c_i64, _c_p]
            L.spike_solve_transpose.restype = ctypes.c_int
            L.spike_solve_transpose.argtypes = [_c_p, _c_i32, _c_p, _c_i64, _c_p]
            L.spike_info.restype = ctypes.c_int
            L.spike_info.argtypes = [_c_p, ctypes.POINTER(Status)]
            L.spike_handle_plan.restype = ctypes.c_int
            L.spike_handle_plan.argtypes = [_c_p, ctypes.POINTER(PlanInfo)]
            L.spike_destroy.restype = ctypes.c_int
            L.spike_destroy.argtypes = [_c_p]
            L.spike_factor_batch.restype = ctypes.c_int
            L.spike_factor_batch.argtypes = [_c_i32, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]
            L.spike_solve_batch.restype = ctypes.c_int
            L.spike_solve_batch.argtypes = [_c_p, _c_p, _c_p, _c_p, _c_p, _c_i32, _c_p]
            L.spike_graph_capture_batch.restype = ctypes.c_int
            L.spike_graph_capture_batch.argtypes = [_c_p, _c_p, _c_p, _c_p, _c_p, _c_i32, _c_p,
                                                    ctypes.POINTER(_c_p)]
            L.spike_graph_capture_solve.restype = ctypes.c_int
            L.spike_graph_capture_solve.argtypes = [_c_p, _c_i32, _c_p, _c_i64, _c_i32, _c_p,
                                                    ctypes.POINTER(_c_p)]
            L.spike_graph_launch.restype = ctypes.c_int
            L.spike_graph_launch.argtypes = [_c_p, _c_p]
            L.spike_graph_destroy.restype = ctypes.c_int
            L.spike_graph_destroy.argtypes = [_c_p]
            L.spike_server_default_opts.restype = None
            L.spike_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
            L.spike_server_create.restype = ctypes.c_int
            L.spike_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_c_p)]
            L.spike_server_submit.restype = ctypes.c_int
            L.spike_server_submit.argtypes = [_c_p, ctypes.POINTER(Request), ctypes.POINTER(_c_i64)]
            for fn in ("spike_server_poll", "spike_server_wait"):
                getattr(L, fn).restype = ctypes.c_int
                getattr(L, fn).argtypes = [_c_p, _c_i64, ctypes.POINTER(RequestStatus)]
            L.spike_server_release.restype = ctypes.c_int
            L.spike_server_release.argtypes = [_c_p, _c_i64]
            L.spike_server_drain.restype = ctypes.c_int
            L.spike_server_drain.argtypes = [_c_p]
            L.spike_server_stats.restype = ctypes.c_int
            L.spike_server_stats.argtypes = [_c_p, ctypes.POINTER(ServerReport)]
            L.spike_server_destroy.restype = ctypes.c_int
            L.spike_server_destroy.argtypes = [_c_p]
            L.spike_autotune_workspace_size.restype = ctypes.c_int
            L.spike_autotune_workspace_size.argtypes = [_c_i64, _c_i32, _c_i32, ctypes.POINTER(Opts),
                                                        ctypes.POINTER(_c_size)]
            L.spike_autotune.restype = ctypes.c_int
            L.spike_autotune.argtypes = [_c_i64, _c_i32, _c_i32, _c_p, _c_i64, _c_i32, ctypes.POINTER(Opts),
                                         _c_p, _c_size, _c_p, _c_i64, _c_p, ctypes.POINTER(TuneResult)]
            L.spike_zworkspace_size.restype = ctypes.c_int
            L.spike_zworkspace_size.argtypes = [_c_i64, _c_i32, _c_i32, ctypes.POINTER(Opts), ctypes.POINTER(_c_size)]
            L.spike_zfactor.restype = ctypes.c_int
            L.spike_zfactor.argtypes = [_c_i64, _c_i32, _c_i32, _c_p, _c_i64, ctypes.POINTER(Opts), _c_p, _c_size,
                                        _c_p, ctypes.POINTER(_c_p)]
            L.spike_zsolve.restype = ctypes.c_int
            L.spike_zsolve.argtypes = [_c_p, _c_i32, _c_p, _c_i64, _c_i32, _c_p]
            L.spike_krylov_default_opts.restype = None
            L.spike_krylov_default_opts.argtypes = [ctypes.POINTER(KrylovOpts)]
            L.spike_krylov_workspace_size.restype = ctypes.c_int
            L.spike_krylov_workspace_size.argtypes = [_c_p, _c_i32, ctypes.POINTER(KrylovOpts),
                                                      ctypes.POINTER(_c_size)]
            L.spike_solve_gmres.restype = ctypes.c_int
            L.spike_solve_gmres.argtypes = [_c_p, _c_i32, _c_p, _c_i64, _c_i32, ctypes.POINTER(KrylovOpts), _c_p,
                                            _c_size, _c_p, ctypes.POINTER(KrylovResult)]
            L.spike_scratch_capacity.restype = _c_size
            L.spike_scratch_capacity.argtypes = []
            L.spike_factor_scratch.restype = ctypes.c_int
            L.spike_factor_scratch.argtypes = [_c_i64, _c_i32, _c_i32, _c_p, _c_i64, ctypes.POINTER(Opts), _c_p,
                                               ctypes.POINTER(_c_p)]
            L.spike_sweep_counting.restype = ctypes.c_int
            L.spike_sweep_counting.argtypes = [ctypes.c_int]
            L.spike_sweep_counts.restype = ctypes.c_int
            L.spike_sweep_counts.argtypes = [_c_p, ctypes.POINTER(ctypes.c_uint64)]
            L.spike_profile_enable.restype = ctypes.c_int
            L.spike_profile_enable.argtypes = [ctypes.c_int]
            L.spike_profile_only.restype = ctypes.c_int
            L.spike_profile_only.argtypes = [ctypes.c_char_p]
            L.spike_tune_cache_clear.restype = ctypes.c_int
            L.spike_tune_cache_clear.argtypes = []
            L.spike_tune_cache_size.restype = ctypes.c_int
            L.spike_tune_cache_size.argtypes = []
            L.spike_tune_cache_save.restype = ctypes.c_int
            L.spike_tune_cache_save.argtypes = [ctypes.c_char_p]
            L.spike_tune_cache_load.restype = ctypes.c_int
            L.spike_tune_cache_load.argtypes = [ctypes.c_char_p]
            L.spike_profile_report.restype = ctypes.c_int
            L.spike_profile_report.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int)]
            _lib = L
    return _lib


def header_symbols():
    """Names the public header declares with SPIKE_API."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"SPIKE_API\s+[\w\s\*]+?\b(spike_\w+)\s*\(", txt)))


def profile_enable(on=True):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    rc = lib().spike_profile_enable(1 if on else 0)
    if rc != 0:
        raise SpikeError("spike_profile_enable", rc)


def profile_only(name=None):
    """Bracket only the launches of kernel `name` (None: every kernel) from
    the next profile_enable(True) on (spike_profile_only)."""
    rc = lib().spike_profile_only(name.encode() if name else None)
    if rc != 0:
        raise SpikeError("spike_profile_only", rc)


def profile_report():
    """{kernel name: (launches, summed milliseconds)} of the recorded launches."""
    cap = 64
    buf = (KernelTime * cap)()
    cnt = ctypes.c_int()
    rc = lib().spike_profile_report(buf, cap, ctypes.byref(cnt))
    if rc != 0:
        raise SpikeError("spike_profile_report", rc)
    return {buf[i].name.decode(): (buf[i].calls, buf[i].total_ms) for i in range(min(cnt.value, cap))}


def make_opts(p=0, pivot=False, precision="fp64", sizing="equal", K=0.0, nrhs_hint=0,
              nrhs_max=64, boost_tau=-1.0, max_refine=-1, refine_tol=1e-13,
              tree="balanced", r12=0.0, r13=0.0) -> Opts:
    """spike_opts from keyword options (the header documents each field):
    precision "fp64" | "mixed", sizing "equal" | "r13" (ratios from K and
    nrhs_hint) | "ratios" (the explicit r12 = n1/n2 and r13 = n1/n3), tree
    "balanced" | "paper" (the 2^m + r layout, which rejects other p)."""
    o = Opts()
    lib().spike_default_opts(ctypes.byref(o))
    o.p = int(p)
    o.pivot = 1 if pivot else 0
    o.precision = {"fp64": 0, "mixed": 1, 0: 0, 1: 1}[precision]
    o.sizing = {"equal": 0, "r13": 1, "ratios": 2, 0: 0, 1: 1, 2: 2}[sizing]
    o.K = float(K)
    o.nrhs_hint = int(nrhs_hint)
    o.nrhs_max = int(nrhs_max)
    o.boost_tau = float(boost_tau)
    o.max_refine = int(max_refine)
    o.refine_tol = float(refine_tol)
    o.tree = {"balanced": 0, "paper": 1, 0: 0, 1: 1}[tree]
    o.r12 = float(r12)
    o.r13 = float(r13)
    return o


def plan_query(n, kl, ku, **opts):
    """Host-only planner query: dict with p, levels, merges, reduced_size,
    workspace_bytes and the partition sizes."""
    o = make_opts(**opts)
    info = PlanInfo()
    cap = max(int(opts.get("p", 0) or 0), 4096)
    sizes = (_c_i64 * cap)()
    rc = lib().spike_plan_query(int(n), int(kl), int(ku), ctypes.byref(o), ctypes.byref(info), sizes)
    if rc != 0:
        raise SpikeError("spike_plan_query", rc)
    return {"p": info.p, "levels": info.levels, "merges": info.merges,
            "reduced_size": info.reduced_size, "workspace_bytes": info.workspace_bytes,
            "sizes": [sizes[i] for i in range(info.p)]}


def plan_tree(n, kl, ku, **opts):
    """Host-only query of the merge tree: a list of (level, a, m, b) per
    interface system in launch order; the merged node spans leaves a..b and
    its children a..m and m+1..b."""
    o = make_opts(**opts)
    p = plan_query(n, kl, ku, **opts)["p"]
    buf = (_c_i32 * max(1, 4 * (p - 1)))()
    rc = lib().spike_plan_tree(int(n), int(kl), int(ku), ctypes.byref(o), buf)
    if rc != 0:
        raise SpikeError("spike_plan_tree", rc)
    return [tuple(buf[4 * d:4 * d + 4]) for d in range(p - 1)]


def workspace_size(n, kl, ku, **opts) -> int:
    o = make_opts(**opts)
    out = _c_size()
    rc = lib().spike_workspace_size(int(n), int(kl), int(ku), ctypes.byref(o), ctypes.byref(out))
    if rc != 0:
        raise SpikeError("spike_workspace_size", rc)
    return out.value


def _check_band(ab, kl, ku):
    """A band handed to the library: a contiguous float64 CUDA tensor of shape
    (n, ldab) with ldab >= kl + ku + 1 (checked before any library call)."""
    import torch
    if not isinstance(ab, torch.Tensor) or ab.dtype != torch.float64 or not ab.is_cuda \
            or ab.dim() != 2 or not ab.is_contiguous():
        raise ValueError("band must be a contiguous 2-D float64 CUDA tensor (n, ldab)")
    if int(ab.shape[1]) < int(kl) + int(ku) + 1:
        raise ValueError("band has ldab = %d < kl + ku + 1" % int(ab.shape[1]))


def _check_rhs(B, n):
    """A right-hand side handed to the library: a float64 CUDA tensor of shape
    (nrhs, n) or (n,) with unit column stride.  Returns the 2-D view."""
    import torch
    if not isinstance(B, torch.Tensor) or B.dtype != torch.float64 or not B.is_cuda:
        raise ValueError("B must be a float64 CUDA tensor")
    if B.dim() == 1:
        B = B.view(1, -1)
    if B.dim() != 2 or B.shape[1] != n or (B.shape[1] > 1 and B.stride(1) != 1) \
            or (B.shape[0] > 1 and B.stride(0) < max(n, 1)):
        raise ValueError("B must have shape (nrhs, n) with unit column stride")
    return B


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Factorization:
    """A SPIKE factorisation resident in a device workspace.

    ``ab``: float64 CUDA tensor (n, ldab), LAPACK band storage.  The tensor is
    kept referenced (mixed precision reads it for residuals).  ``workspace``:
    a uint8 CUDA tensor, None (one is allocated), or "scratch": the library's
    own per-GPU scratch array (spike_factor_scratch, no allocation; a later
    "scratch" factorisation on the same GPU overwrites this one)."""

    def __init__(self, ab, kl, ku, *, stream=None, workspace=None, **opts):
        import torch
        _check_band(ab, kl, ku)
        self.n, self.ldab = int(ab.shape[0]), int(ab.shape[1])
        self.kl, self.ku = int(kl), int(ku)
        self.opts = make_opts(**opts)
        self.nrhs_max = self.opts.nrhs_max
        need = workspace_size(self.n, kl, ku, **opts)
        if isinstance(workspace, str):
            if workspace != "scratch":
                raise ValueError("workspace must be a tensor, None or 'scratch'")
            self.ab, self.ws, self.device = ab, None, ab.device
            h = ctypes.c_void_p()
            rc = lib().spike_factor_scratch(self.n, self.kl, self.ku, ctypes.c_void_p(ab.data_ptr()), self.ldab,
                                            ctypes.byref(self.opts), _stream_handle(stream), ctypes.byref(h))
            if rc != 0:
                raise SpikeError("spike_factor_scratch", rc)
            self.h = h
            return
        if workspace is None:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=ab.device)
        if workspace.numel() < need:
            raise ValueError("workspace too small")
        self.ab = ab
        self.ws = workspace
        self.device = ab.device
        h = ctypes.c_void_p()
        rc = lib().spike_factor(self.n, self.kl, self.ku, ctypes.c_void_p(ab.data_ptr()), self.ldab,
                                ctypes.byref(self.opts), ctypes.c_void_p(workspace.data_ptr()),
                                workspace.numel(), _stream_handle(stream), ctypes.byref(h))
        if rc != 0:
            raise SpikeError("spike_factor", rc)
        self.h = h

    def solve_(self, B, *, trans=False, stream=None):
        """In-place solve on B ((nrhs, n) float64 CUDA tensor, C order)."""
        B = _check_rhs(B, self.n)
        ldb = B.stride(0) if B.shape[0] > 1 else max(self.n, 1)
        fn = lib().spike_solve_transpose if trans else lib().spike_solve
        rc = fn(self.h, int(B.shape[0]), ctypes.c_void_p(B.data_ptr()), int(ldb), _stream_handle(stream))
        if rc != 0:
            raise SpikeError("spike_solve_transpose" if trans else "spike_solve", rc)
        return B

    def solve_gmres_(self, B, *, trans=False, restart=30, max_iters=300, tol=1e-13, stream=None):
        """In-place GMRES solve of op(A) X = B with this factorisation as the
        right preconditioner (spike_solve_gmres; blocks until done).  Returns
        a dict with iters, restarts, converged and berr; raises SpikeError
        with code 1 when the factorisation failed (B untouched)."""
        import torch
        B = _check_rhs(B, self.n)
        ldb = B.stride(0) if B.shape[0] > 1 else max(self.n, 1)
        o = KrylovOpts(int(restart), int(max_iters), float(tol))
        need = _c_size()
        rc = lib().spike_krylov_workspace_size(self.h, int(B.shape[0]), ctypes.byref(o), ctypes.byref(need))
        if rc != 0:
            raise SpikeError("spike_krylov_workspace_size", rc)
        ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device=B.device)
        res = KrylovResult()
        rc = lib().spike_solve_gmres(self.h, int(B.shape[0]), ctypes.c_void_p(B.data_ptr()), int(ldb),
                                     1 if trans else 0, ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel(), _stream_handle(stream), ctypes.byref(res))
        if rc != 0:
            raise SpikeError("spike_solve_gmres", rc)
        return {"iters": res.iters, "restarts": res.restarts, "converged": bool(res.converged),
                "berr": res.berr}

    def info(self):
        st = Status()
        rc = lib().spike_info(self.h, ctypes.byref(st))
        if rc != 0:
            raise SpikeError("spike_info", rc)
        return {"info": st.info, "n_boosts": st.n_boosts, "refine_iters": st.refine_iters,
                "min_abs_pivot": st.min_abs_pivot, "berr": st.berr}

    def sweep_counts(self):
        """The handle's instrumented sweep counters (it must have been made
        inside ``sweep_counting()``): a dict keyed by (stage, partition type,
        full) with stage in ("factor", "solve", "solve_t"), type in ("single",
        "first", "middle", "last") and full True for sweeps over all of a
        partition's rows."""
        buf = (ctypes.c_uint64 * 24)()
        rc = lib().spike_sweep_counts(self.h, buf)
        if rc != 0:
            raise SpikeError("spike_sweep_counts", rc)
        out = {}
        for si, stage in enumerate(("factor", "solve", "solve_t")):
            for ti, typ in enumerate(("single", "first", "middle", "last")):
                for full in (0, 1):
                    out[(stage, typ, bool(full))] = int(buf[(si * 4 + ti) * 2 + full])
        return out

    def plan(self):
        info = PlanInfo()
        rc = lib().spike_handle_plan(self.h, ctypes.byref(info))
        if rc != 0:
            raise SpikeError("spike_handle_plan", rc)
        return {"p": info.p, "levels": info.levels, "merges": info.merges,
                "reduced_size": info.reduced_size, "workspace_bytes": info.workspace_bytes}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().spike_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class sweep_counting:
    """Context manager: factorisations made inside it count their triangular
    sweeps on the device (spike_sweep_counting)."""

    def __enter__(self):
        lib().spike_sweep_counting(1)
        return self

    def __exit__(self, *exc):
        lib().spike_sweep_counting(0)
        return False


class ZFactorization(Factorization):
    """A complex band's SPIKE factorisation (spike_zfactor: the real
    embedding with 2 x 2 blocks [[Re a, -Im a], [Im a, Re a]], factored on
    the real path).  ``ab``: complex128 CUDA tensor (n, ldab), the real
    band's layout; options as Factorization, for the 2n-row embedding."""

    _TRANS = {"N": 0, "T": 1, "C": 2, False: 0, True: 1}

    def __init__(self, ab, kl, ku, *, stream=None, workspace=None, **opts):
        import torch
        if not isinstance(ab, torch.Tensor) or ab.dtype != torch.complex128 or not ab.is_cuda \
                or ab.dim() != 2 or not ab.is_contiguous():
            raise ValueError("band must be a contiguous 2-D complex128 CUDA tensor (n, ldab)")
        if int(ab.shape[1]) < int(kl) + int(ku) + 1:
            raise ValueError("band has ldab < kl + ku + 1")
        self.n, self.ldab = int(ab.shape[0]), int(ab.shape[1])
        self.kl, self.ku = int(kl), int(ku)
        self.opts = make_opts(**opts)
        self.nrhs_max = self.opts.nrhs_max
        need = _c_size()
        rc = lib().spike_zworkspace_size(self.n, self.kl, self.ku, ctypes.byref(self.opts), ctypes.byref(need))
        if rc != 0:
            raise SpikeError("spike_zworkspace_size", rc)
        if workspace is None:
            workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=ab.device)
        if workspace.numel() < need.value:
            raise ValueError("workspace too small")
        self.ab, self.ws, self.device = ab, workspace, ab.device
        h = ctypes.c_void_p()
        rc = lib().spike_zfactor(self.n, self.kl, self.ku, ctypes.c_void_p(ab.data_ptr()), self.ldab,
                                 ctypes.byref(self.opts), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel(), _stream_handle(stream), ctypes.byref(h))
        if rc != 0:
            raise SpikeError("spike_zfactor", rc)
        self.h = h

    def solve_(self, B, *, trans="N", stream=None):
        """In-place solve of op(A) Z = B, B a complex128 CUDA tensor (nrhs, n)
        or (n,) with unit column stride; trans "N", "T" (A^T) or "C" (A^H)."""
        import torch
        if not isinstance(B, torch.Tensor) or B.dtype != torch.complex128 or not B.is_cuda:
            raise ValueError("B must be a complex128 CUDA tensor")
        if B.dim() == 1:
            B = B.view(1, -1)
        if B.dim() != 2 or B.shape[1] != self.n or (self.n > 1 and B.stride(1) != 1) \
                or (B.shape[0] > 1 and B.stride(0) < max(self.n, 1)):
            raise ValueError("B must have shape (nrhs, n) with unit column stride")
        ldb = B.stride(0) if B.shape[0] > 1 else max(self.n, 1)
        rc = lib().spike_zsolve(self.h, int(B.shape[0]), ctypes.c_void_p(B.data_ptr()), int(ldb),
                                self._TRANS[trans], _stream_handle(stream))
        if rc != 0:
            raise SpikeError("spike_zsolve", rc)
        return B

    def solve_gmres_(self, *a, **kw):
        raise NotImplementedError("GMRES runs on real systems")


def levels_for(p: int) -> int:
    return 0 if p <= 1 else math.ceil(math.log2(p))


def _batch_arrays(facs, Bs, trans):
    """ctypes arrays for the batched entry points (B tensors: (nrhs, n), C order)."""
    cnt = len(facs)
    if len(Bs) != cnt:
        raise ValueError("one right-hand side per factorisation")
    if isinstance(trans, bool):
        trans = [trans] * cnt
    for f, B in zip(facs, Bs):
        _check_rhs(B, f.n)
    hs = (_c_p * cnt)(*[f.h.value for f in facs])
    nr = (_c_i32 * cnt)()
    bp = (_c_p * cnt)()
    ld = (_c_i64 * cnt)()
    tr = (_c_i32 * cnt)(*[1 if t else 0 for t in trans])
    for i, (f, B) in enumerate(zip(facs, Bs)):
        B = _check_rhs(B, f.n)
        nr[i] = int(B.shape[0])
        bp[i] = B.data_ptr()
        ld[i] = B.stride(0) if B.shape[0] > 1 else max(f.n, 1)
    return cnt, hs, nr, bp, ld, tr


def factor_batch(systems, stream=None, **opts):
    """Factor several banded systems with batched launches
    (spike_factor_batch).  ``systems``: a list of (ab, kl, ku) with ab a
    float64 CUDA band tensor; ``opts`` apply to every system.  Returns one
    Factorization per system, each with its own workspace."""
    import torch
    cnt = len(systems)
    facs = []
    for ab, kl, ku in systems:
        _check_band(ab, kl, ku)
        f = Factorization.__new__(Factorization)
        f.n, f.ldab = int(ab.shape[0]), int(ab.shape[1])
        f.kl, f.ku = int(kl), int(ku)
        f.opts = make_opts(**opts)
        f.nrhs_max = f.opts.nrhs_max
        f.ab, f.device = ab, ab.device
        f.ws = torch.empty(max(workspace_size(f.n, kl, ku, **opts), 256), dtype=torch.uint8, device=ab.device)
        f.h = None
        facs.append(f)
    n = (_c_i64 * cnt)(*[f.n for f in facs])
    kl = (_c_i32 * cnt)(*[f.kl for f in facs])
    ku = (_c_i32 * cnt)(*[f.ku for f in facs])
    ap = (_c_p * cnt)(*[f.ab.data_ptr() for f in facs])
    ld = (_c_i64 * cnt)(*[f.ldab for f in facs])
    op = (Opts * cnt)(*[f.opts for f in facs])
    wp = (_c_p * cnt)(*[f.ws.data_ptr() for f in facs])
    wb = (_c_size * cnt)(*[f.ws.numel() for f in facs])
    hs = (_c_p * cnt)()
    rc = lib().spike_factor_batch(cnt, n, kl, ku, ap, ld, op, wp, wb, _stream_handle(stream), hs)
    if rc != 0:
        raise SpikeError("spike_factor_batch", rc)
    for f, h in zip(facs, hs):
        f.h = ctypes.c_void_p(h)
    return facs


def solve_batch(facs, Bs, trans=False, stream=None):
    """In-place solves of several factorisations, phases batched across
    systems (spike_solve_batch).  ``trans``: bool or one bool per system."""
    cnt, hs, nr, bp, ld, tr = _batch_arrays(facs, Bs, trans)
    rc = lib().spike_solve_batch(hs, nr, bp, ld, tr, cnt, _stream_handle(stream))
    if rc != 0:
        raise SpikeError("spike_solve_batch", rc)
    return Bs


class SolveGraph:
    """The solve stage of one or more factorisations captured into a HIP
    graph on ``stream`` (a torch.cuda.Stream other than the default), to be
    replayed with launch()."""

    def __init__(self, facs, Bs, trans=False, stream=None):
        import torch
        if not isinstance(facs, (list, tuple)):
            facs, Bs = [facs], [Bs]
        self.facs, self.Bs = list(facs), list(Bs)   # keep them alive with the graph
        self.stream = stream if stream is not None else torch.cuda.Stream()
        cnt, hs, nr, bp, ld, tr = _batch_arrays(self.facs, self.Bs, trans)
        g = _c_p()
        rc = lib().spike_graph_capture_batch(hs, nr, bp, ld, tr, cnt, ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(g))
        if rc != 0:
            raise SpikeError("spike_graph_capture_batch", rc)
        self.g = g

    def launch(self, stream=None):
        rc = lib().spike_graph_launch(self.g, _stream_handle(stream))
        if rc != 0:
            raise SpikeError("spike_graph_launch", rc)

    def close(self):
        if getattr(self, "g", None) is not None and self.g.value:
            lib().spike_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ab, kl, ku, nrhs=1, stream=None, **base):
    """Pick p and the partition sizing for this matrix and nrhs by timing
    candidate plans (spike_autotune).  Returns (opts dict, result dict)."""
    import torch
    _check_band(ab, kl, ku)
    n, ldab = int(ab.shape[0]), int(ab.shape[1])
    o = make_opts(**base)
    need = _c_size()
    rc = lib().spike_autotune_workspace_size(n, int(kl), int(ku), ctypes.byref(o), ctypes.byref(need))
    if rc != 0:
        raise SpikeError("spike_autotune_workspace_size", rc)
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device=ab.device)
    B = torch.zeros((int(nrhs), n), dtype=torch.float64, device=ab.device)
    res = TuneResult()
    rc = lib().spike_autotune(n, int(kl), int(ku), ctypes.c_void_p(ab.data_ptr()), ldab, int(nrhs),
                              ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              ctypes.c_void_p(B.data_ptr()), n, _stream_handle(stream), ctypes.byref(res))
    if rc != 0:
        raise SpikeError("spike_autotune", rc)
    r = res.opts
    opts = {"p": r.p, "pivot": bool(r.pivot), "precision": "mixed" if r.precision else "fp64",
            "sizing": ("equal", "r13", "ratios")[r.sizing], "r12": r.r12, "r13": r.r13,
            "K": r.K, "nrhs_hint": r.nrhs_hint,
            "nrhs_max": r.nrhs_max, "tree": "paper" if r.tree else "balanced"}
    return opts, {"factor_ms": res.factor_ms, "solve_ms": res.solve_ms, "K": res.K,
                  "candidates": res.candidates, "cached": bool(res.cached)}


def tune_cache_clear():
    lib().spike_tune_cache_clear()


def tune_cache_size():
    return int(lib().spike_tune_cache_size())


def tune_cache_save(path):
    rc = lib().spike_tune_cache_save(str(path).encode())
    if rc != 0:
        raise SpikeError("spike_tune_cache_save", rc)


def tune_cache_load(path):
    rc = lib().spike_tune_cache_load(str(path).encode())
    if rc != 0:
        raise SpikeError("spike_tune_cache_load", rc)


class Server:
    """Serving runtime (spike_server_*): queued banded solves with resident
    factorisations, HBM-budgeted admission and continuous batching.  Tensors
    handed to submit() are kept referenced until release()."""

    def __init__(self, hbm_budget=16 << 30, max_inflight=64, streams=4, batch_window=32, device=None):
        import torch
        o = ServerOpts()
        lib().spike_server_default_opts(ctypes.byref(o))
        o.hbm_budget, o.max_inflight, o.streams, o.batch_window = int(hbm_budget), int(max_inflight), \
            int(streams), int(batch_window)
        # the device pool the server carves workspaces from (the library
        # allocates no device memory); kept referenced until close()
        self._pool = torch.empty(max(int(hbm_budget), 4096), dtype=torch.uint8,
                                 device=device if device is not None else torch.device("cuda"))
        o.dpool = self._pool.data_ptr()
        s = _c_p()
        rc = lib().spike_server_create(ctypes.byref(o), ctypes.byref(s))
        if rc != 0:
            raise SpikeError("spike_server_create", rc)
        self.s = s
        self._keep = {}

    def submit(self, matrix_id, ab, kl, ku, B, trans=False, **opts):
        """Queue op(A) X = B for matrix ``matrix_id`` (band tensor ``ab``,
        (n, ldab)); B: (nrhs, n) float64 CUDA tensor, solved in place."""
        _check_band(ab, kl, ku)
        n = int(ab.shape[0])
        B = _check_rhs(B, n)
        r = Request()
        r.matrix_id, r.n, r.kl, r.ku = int(matrix_id), n, int(kl), int(ku)
        r.dAB, r.ldab = ab.data_ptr(), int(ab.shape[1])
        r.opts = make_opts(**opts)
        r.nrhs, r.dB = int(B.shape[0]), B.data_ptr()
        r.ldb = B.stride(0) if B.shape[0] > 1 else n
        r.trans = 1 if trans else 0
        t = _c_i64()
        rc = lib().spike_server_submit(self.s, ctypes.byref(r), ctypes.byref(t))
        if rc != 0:
            raise SpikeError("spike_server_submit", rc)
        self._keep[t.value] = (ab, B)
        return t.value

    @staticmethod
    def _st(st):
        return {"state": st.state, "error": st.error, "info": st.info, "latency_s": st.latency_s}

    def poll(self, ticket):
        st = RequestStatus()
        rc = lib().spike_server_poll(self.s, int(ticket), ctypes.byref(st))
        if rc != 0:
            raise SpikeError("spike_server_poll", rc)
        return self._st(st)

    def wait(self, ticket):
        st = RequestStatus()
        rc = lib().spike_server_wait(self.s, int(ticket), ctypes.byref(st))
        if rc != 0:
            raise SpikeError("spike_server_wait", rc)
        return self._st(st)

    def release(self, ticket):
        rc = lib().spike_server_release(self.s, int(ticket))
        if rc != 0:
            raise SpikeError("spike_server_release", rc)
        self._keep.pop(int(ticket), None)

    def drain(self):
        rc = lib().spike_server_drain(self.s)
        if rc != 0:
            raise SpikeError("spike_server_drain", rc)

    def stats(self):
        r = ServerReport()
        rc = lib().spike_server_stats(self.s, ctypes.byref(r))
        if rc != 0:
            raise SpikeError("spike_server_stats", rc)
        return {f: getattr(r, f) for f, _ in ServerReport._fields_}

    def close(self):
        if getattr(self, "s", None) is not None and self.s.value:
            lib().spike_server_destroy(self.s)
            self.s = None
            self._keep.clear()
            self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

