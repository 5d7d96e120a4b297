"""Build the gfx950 shared library ``libspike.so`` in-tree with hipcc.

The kernel templates are instantiated in separate translation units (one per
panel width and precision for the partition kernels, one per panel width for
the interface kernels) that compile in parallel, then link into one library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspike.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("SPIKE_OFFLOAD_ARCH", "gfx950")
NBS = (8, 16, 32)
HTS = (1, 2, 4, 8, 10, 16)

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-fvisibility=hidden",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    env = os.environ.get("HIPCC")
    if env:
        return env
    return "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"


def units() -> list[tuple[str, str, list[str]]]:
    """(object name, source, extra flags) for every translation unit."""
    u = []
    for t in ("double", "float"):
        for nb in NBS:
            u.append((f"leaf_{t}_{nb}.o", "spike_inst.hip",
                      ["-DSPIKE_INST_LEAF", f"-DSPIKE_T={t}", f"-DSPIKE_NB={nb}"]))
    for nb in NBS:
        u.append((f"merge_{nb}.o", "spike_inst.hip", ["-DSPIKE_INST_MERGE", f"-DSPIKE_NB={nb}"]))
    for t in ("double", "float"):
        for ht in HTS:
            u.append((f"fast_{t}_{ht}.o", "spike_inst.hip",
                      ["-DSPIKE_INST_FAST", f"-DSPIKE_T={t}", f"-DSPIKE_HT={ht}"]))
    for ht in HTS:
        u.append((f"mfast_{ht}.o", "spike_inst.hip", ["-DSPIKE_INST_MFAST", f"-DSPIKE_HT={ht}"]))
    u.append(("common.o", "spike_inst.hip", ["-DSPIKE_INST_COMMON"]))
    for src in ("spike_dispatch.hip", "spike_refine.hip", "spike_krylov.hip", "spike_complex.hip", "spike_scratch.hip", "spike_plan.cpp", "spike_api.cpp",
                "spike_profile.cpp", "spike_server.cpp"):
        u.append((src.rsplit(".", 1)[0] + ".o", src, []))
    return u


def _compile(item):
    obj, src, extra = item
    out = os.path.join(OBJ, obj)
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return obj, res.returncode, res.stdout + res.stderr, cmd


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit (always) and link libspike.so."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, rc, log, cmd in ex.map(_compile, units()):
            if verbose:
                print("compiled", obj, flush=True)
            if rc != 0:
                sys.stderr.write(" ".join(cmd) + "\n" + log)
                raise RuntimeError("hipcc failed on " + obj)
            objs.append(os.path.join(OBJ, obj))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
        raise RuntimeError("link of libspike.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
