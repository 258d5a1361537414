"""The FP64 oracle's C sources built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only), with the oracle's pins run
against that build in a child process. CPU only."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "oracle", f) for f in ("rs_oracle.c", "rs_oracle_bvh.c", "rs_oracle_mesh.c")]
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_bvh_pins.py", "tests/test_oracle_ploc_pins.py",
        "tests/test_oracle_paper_pins.py"]


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-Wall", "-o", lib] + SRCS + ["-lm"])
    asan = subprocess.check_output([gcc, "-print-file-name=libasan.so"], text=True).strip()
    pre = os.environ.get("LD_PRELOAD")
    env = dict(os.environ, RS_ORACLE_LIB=lib, OMP_NUM_THREADS="4",
               LD_PRELOAD=asan + (":" + pre if pre else ""),  # the ASan runtime must come first
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child loads the sanitized build, with the ASan runtime mapped
    probe = subprocess.run([sys.executable, "-c", "from oracle import oracle as O; import sys; O.lib(); "
                            "print(O.lib()._name); print(any('libasan' in l for l in open('/proc/self/maps')))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert probe.stdout.split() == [lib, "True"], probe.stdout
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m",
                        "not gpu and not slow"] + PINS, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=850)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
