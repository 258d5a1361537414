"""Compile the HIP sources into the C-ABI shared library librs.so (gfx950)."""

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librs.so")
SOURCES = ["rs_api.hip", "rs_build.hip", "rs_render.hip", "rs_mesh.hip", "rs_loss.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=on", "-munsafe-fp-atomics",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, extra=(), out=None):
    """Compile every source to an object in parallel, then link librs.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    target = out or LIB
    flags = [f for f in HIPCC_FLAGS if f != "-shared"] + list(extra)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="rs_build_") as tmpdir:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc] + flags + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            return obj, subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        log = []
        for _, r in results:
            log += [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
        if any(r.returncode != 0 for _, r in results):
            raise RuntimeError("hipcc failed:\n" + "\n".join(log))
        tmp = target + ".tmp"
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for o, _ in results] + ["-o", tmp]
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
        if verbose and log:
            print("\n".join(log))
        os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
