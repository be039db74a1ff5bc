"""The oracle's pins, run again against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (CPU only, g++).

The instrumented library is built in a temporary folder and loaded by a child pytest
process through TTORACLE_LIB, with the ASan runtime preloaded (the Python interpreter
itself is not instrumented, so leak checking is off).  Any out-of-bounds access,
use-after-free or undefined behaviour in the oracle aborts the child.  The two large
Table 2 FDM rank pins are left out (minutes under the sanitizers); every other oracle
pin runs.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    if not shutil.which("g++") or rt is None:
        pytest.skip("g++ with the AddressSanitizer runtime is not available")
    lib = tmp_path / "libttoracle_asan.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "ttoracle.cpp")], check=True)
    env = dict(os.environ, LD_PRELOAD=rt, TTORACLE_LIB=str(lib),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = ["tests/test_oracle_sparse.py", "tests/test_oracle_rounding.py", "tests/test_oracle_eval.py",
             "tests/test_oracle_snap.py", "tests/test_oracle_mpo.py", "tests/test_oracle_knife_edge.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-k", "not (fdm_mpo_ranks_table2 and random)", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0, "oracle pins failed or a sanitizer aborted"
    assert "passed" in r.stdout
