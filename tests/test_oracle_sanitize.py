"""The FP64 oracle under host AddressSanitizer + UndefinedBehaviorSanitizer.

``oracle/selftest.c`` drives every exported routine of ``oracle/svo.c`` on
degenerate and ragged sizes with hostile inputs (empty pixels of every kind,
motion off the image or non-finite, zero-length histories, a-trous steps
larger than the image).  Built with ``-fsanitize=address,undefined
-fno-sanitize-recover=all``, any out-of-bounds access, leak or undefined
operation ends the run with a non-zero status.  Host code only; no GPU.
"""

import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("make") is None,
                    reason="needs gcc and make")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "svo_selftest")
    b = subprocess.run(["make", "-s", "-C", ORACLE, f"SELFTEST={exe}", exe],
                       capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    last = r.stdout.strip().splitlines()[-1]
    assert last.startswith("selftest ok ")
    assert int(last.split()[-1]) > 10000
