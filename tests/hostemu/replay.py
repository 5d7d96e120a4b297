"""Build and run the CPU replay of the workgroup kernel path (emu_main.cpp).

The kernel headers are copied with the few rewrites a host compiler needs
(LDS declarations become per-workgroup buffers of the stand-in runtime,
address-space qualifiers are dropped, vector types take the host compiler's
spelling), then compiled with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer together with the host
planner."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1811_03559_amd", "csrc")
HEADERS = ["spike_device.hpp", "spike_kernels.hpp", "spike_tile.hpp", "spike_launch.hpp", "spike_profile.hpp",
           "spike_types.hpp", "spike_plan.hpp", "spike_plan.cpp", "spike_rowlu.hpp"]


def _rewrite(text: str) -> str:
    text = re.sub(r"extern\s+__shared__\s+__align__\(16\)\s+unsigned char smem_raw\[\];",
                  "unsigned char* smem_raw = ::emu::cur_block()->lds;", text)
    text = text.replace("__shared__", "static")
    text = re.sub(r"__attribute__\(\(address_space\(\d\)\)\)", "", text)
    text = re.sub(r"typedef (\w+) (\w+) __attribute__\(\(ext_vector_type\((\d+)\)\)\);",
                  r"typedef \1 \2 __attribute__((vector_size(\3 * sizeof(\1))));", text)
    text = text.replace('asm volatile("" : "+v"(x));', "")
    return text


def _sources(work: str) -> str:
    """The rewritten kernel headers under work/p/csrc; returns that folder."""
    src = os.path.join(work, "p", "csrc")
    os.makedirs(src, exist_ok=True)
    os.makedirs(os.path.join(work, "include"), exist_ok=True)
    shutil.copy(os.path.join(ROOT, "include", "spike.h"), os.path.join(work, "include", "spike.h"))
    for h in HEADERS:
        with open(os.path.join(CSRC, h)) as f:
            t = f.read()
        with open(os.path.join(src, h), "w") as f:
            f.write(_rewrite(t))
    return src


def _compile(work: str, main: str, extra: list[str], name: str) -> str:
    src = _sources(work)
    exe = os.path.join(work, name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
           "-I", HERE, "-I", src, os.path.join(HERE, main), os.path.join(HERE, "emu_runtime.cpp"),
           *[os.path.join(src, e) for e in extra], "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def build(workdir: str | None = None) -> str:
    """Compile the replay; returns the executable's path."""
    work = workdir or tempfile.mkdtemp(prefix="spike_hostemu_")
    return _compile(work, "emu_main.cpp", ["spike_plan.cpp"], "emu_main")


def build_tile_lu(workdir: str | None = None) -> str:
    """Compile the replay of the diagonal-tile LU of the block LU (the
    row-per-lane routines of spike_rowlu.hpp, one wavefront); returns the
    executable's path."""
    work = workdir or tempfile.mkdtemp(prefix="spike_hostemu_lu_")
    return _compile(work, "tile_lu_main.cpp", [], "tile_lu_main")


def run_tile_lu(exe: str, tiles: np.ndarray, boost: float, mrem: int, fp32: bool = False):
    """Factor each 16 x 16 tile of `tiles` (count x 16 x 16) as the block LU's
    panel does: returns (L\\U, L^{-1}, U^{-1}, boosted pivot counts), the
    matrices row-major like the tiles."""
    tiles = np.ascontiguousarray(tiles, dtype=np.float64).reshape(-1, 16, 16)
    work = tempfile.mkdtemp(prefix="spike_hostemu_lu_run_")
    fin, fout = os.path.join(work, "in.bin"), os.path.join(work, "out.bin")
    with open(fin, "wb") as f:
        np.array([tiles.shape[0], mrem, int(fp32)], dtype=np.int64).tofile(f)
        np.array([boost], dtype=np.float64).tofile(f)
        tiles.tofile(f)
    subprocess.run([exe, fin, fout], check=True, capture_output=True, text=True, timeout=300)
    cnt = tiles.shape[0]
    raw = np.fromfile(fout, dtype=np.float64, count=cnt * 768).reshape(cnt, 3, 16, 16)
    nb = np.fromfile(fout, dtype=np.int64, offset=cnt * 768 * 8, count=cnt)
    shutil.rmtree(work, ignore_errors=True)
    return raw[:, 0], raw[:, 1], raw[:, 2], nb


def run(exe: str, ab: np.ndarray, kl: int, ku: int, F: np.ndarray, p: int, pivot: bool, trans: bool,
        timeout: float = 600.0, sweeps: bool = False, tree: str = "balanced", ratios=None):
    """Factor and solve on the CPU replay.  ab: (n, kl+ku+1) band rows in the
    binding's layout; F: (nrhs, n); tree "balanced" | "paper"; ratios None
    (equal sizes) or (R12, R13).  Returns (info, X with F's shape), or
    (info, X, sweep counters) with sweeps=True."""
    n = ab.shape[0]
    F = np.atleast_2d(F)
    nrhs = F.shape[0]
    work = tempfile.mkdtemp(prefix="spike_hostemu_run_")
    fin, fout = os.path.join(work, "in.bin"), os.path.join(work, "out.bin")
    with open(fin, "wb") as f:
        np.array([n, kl, ku, p, int(pivot), nrhs, int(trans), {"balanced": 0, "paper": 1}[tree],
                  0 if ratios is None else 2], dtype=np.int64).tofile(f)
        np.array(ratios if ratios is not None else (0.0, 0.0), dtype=np.float64).tofile(f)
        np.ascontiguousarray(ab, dtype=np.float64).tofile(f)
        np.ascontiguousarray(F, dtype=np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout, env=env)
    if res.returncode != 0:
        raise RuntimeError("replay failed (rc %d):\n%s" % (res.returncode, (res.stdout + res.stderr)[-6000:]))
    out = np.fromfile(fout, dtype=np.float64)
    info = int(out[:1].view(np.int64)[0])
    shutil.rmtree(work, ignore_errors=True)
    X = out[1:1 + n * nrhs].reshape(nrhs, n)
    if sweeps:
        return info, X, out[1 + n * nrhs:].view(np.uint64).astype(np.int64)
    return info, X
