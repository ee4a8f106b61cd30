"""The host-only code of the library (work plans of the contraction and
Hessian passes, the SPD inverse of the preconditioner: tk_host.cpp), built
with the address and undefined-behaviour sanitizers and checked by
tests/host/host_check.cpp.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2003_10482_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_code_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_check")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-I", CSRC, os.path.join(HERE, "host", "host_check.cpp"), os.path.join(CSRC, "tk_host.cpp"),
               "-o", exe]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        # the sanitizer runtime need not come first in the process's library list
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert run.returncode == 0 and run.stdout.strip().endswith("ok"), (run.stdout[-3000:], run.stderr[-3000:])
