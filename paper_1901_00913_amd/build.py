"""Build libsfista.so (HIP, gfx950) in place next to this file.

    python -m paper_1901_00913_amd.build

Compiles every HIP source under csrc/ with hipcc for gfx950 and links one
shared library exporting the C ABI of include/sfista.h.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfista.so")
SOURCES = ["sfista.hip", "kron.hip", "diff.hip", "fft.hip"]
ARCH = os.environ.get("SFISTA_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++20", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def _clean(text: str) -> str:
    return "\n".join(ln for ln in text.splitlines() if "packed-fp32-ops" not in ln)


def build(verbose: bool = False) -> str:
    """Compiles the sources to objects in parallel, then links the library."""
    objdir = tempfile.mkdtemp(prefix="sfista_build_")
    try:
        procs = []
        for src in SOURCES:
            obj = os.path.join(objdir, src + ".o")
            cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src),
                                             "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                                     text=True)))
        failed = []
        for src, _, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                failed.append(f"{src} ({pr.returncode}):\n{_clean(out)}")
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}"] + [o for _, o, _ in procs] + ["-o", tmp]
        res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed ({res.returncode}):\n{_clean(res.stdout)}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
