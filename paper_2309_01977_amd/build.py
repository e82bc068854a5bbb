"""Build the gfx950 HIP library in-tree with hipcc.

    python -m paper_2309_01977_amd.build [-v]

Compiles the host/C-ABI translation units (projector library, server) and
one translation unit per blur-radius class (spect_kmc.hip with -DSPECT_KMC=0,4,...,32) in parallel,
then links paper_2309_01977_amd/_lib/libspect_hip.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libspect_hip.so")
ARCH = "gfx950"
KMC_CLASSES = (0, 4, 8, 12, 16, 20, 24, 28, 32)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions stay off
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc, fl = hipcc(), common_flags()
    units = [(os.path.join(CSRC, "spect.hip"), os.path.join(OBJ_DIR, "spect.o"), []),
             (os.path.join(CSRC, "spect_server.hip"), os.path.join(OBJ_DIR, "spect_server.o"), [])]
    for k in KMC_CLASSES:
        units.append((os.path.join(CSRC, "spect_kmc.hip"), os.path.join(OBJ_DIR, f"spect_kmc{k}.o"),
                      [f"-DSPECT_KMC={k}"]))
    cmds = [[cc] + fl + extra + ["-c", src, "-o", obj] for src, obj, extra in units]
    n = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=n) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in units], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
