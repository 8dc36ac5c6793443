"""Build libhme.so for gfx950: generate the process headers, compile every HIP
translation unit with hipcc (in parallel), link in-tree.

    python -m paper_2507_21039_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhme.so")
ARCH = "gfx950"

# -packed-fp32-ops keeps the compiler from emitting packed FP32 VALU instructions.
HIPFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-variable",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
_KERNEL_DEPS = ["me2_kernels.h", "colour_mfma.h", "helas.h", "process.h"]
_PROCS = ("eemumu", "ggtt", "ggttg", "ggttgg", "ggttggg", "uuee", "uueeg", "uueegg", "uueeggg")
# g g -> t tbar g g g runs as pieces, one generated translation unit each
PIECES = {"ggttggg": 12}
# processes also built in the Feynman-diagram gauge
_FD = ("ggttg", "ggttgg")
SOURCES = ["hme.cpp", "server.hip", "rambo.hip"] + [f"proc_{p}.hip" for p in _PROCS] + [
    f"proc_{p}_fd.hip" for p in _FD] + [
    f"procs/{p}_c{c}.hip" for p, n in PIECES.items() for c in range(n)]
DEPS = {
    "hme.cpp": _KERNEL_DEPS + ["params.h", "../../include/hme.h"],
    "server.hip": ["../../include/hme.h"],
    "rambo.hip": ["../../include/hme.h"],
    **{f"proc_{p}.hip": _KERNEL_DEPS + [f"procs/{p}.h"] for p in _PROCS},
    **{f"proc_{p}_fd.hip": _KERNEL_DEPS + [f"procs/{p}_fd.h"] for p in _FD},
    **{f"procs/{p}_c{c}.hip": _KERNEL_DEPS + ["piece_kernels.h", "colour_blocked.h", f"procs/{p}.h", f"procs/{p}_c{c}.h"]
       for p, n in PIECES.items() for c in range(n)},
}
DEPS["proc_ggttggg.hip"] = DEPS["proc_ggttggg.hip"] + ["piece_kernels.h", "colour_blocked.h", "procs/ggttggg_chunks.h"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.exists(c) or c == "hipcc"):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool, force: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    deps = [os.path.join(CSRC, d) for d in [src] + DEPS[src]] + [os.path.abspath(__file__)]
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in deps):
        return obj
    cmd = [hipcc(), *HIPFLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None, force: bool = True) -> str:
    """Generate the process headers and compile; force=False reuses objects newer than their sources."""
    from .gen.__main__ import PROCESSES, generate
    infos = generate(os.path.join(CSRC, "procs"))
    for p, n in PIECES.items():
        if infos[p]["nchunk"] != n or PROCESSES[p]["pieces"] != n:
            raise RuntimeError(f"{p}: generator makes {infos[p]['nchunk']} pieces, build expects {n}")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, force), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--incremental" not in sys.argv))
